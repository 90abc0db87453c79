// Backward of a submanifold sparse convolution layer (chain rule on the forward definition).
//   dZ = dY * [Y > 0] (ReLU'(0) = 0) or dY;
//   dX = conv(dZ, W'), W'_k = (W_{26-k})^T: the rulebook is symmetric (R_{26-k} is R_k with the
//        roles of input and output swapped), so the data gradient is a forward convolution;
//   dW_k = sum_{(i,r) in R_k} X[i]^T dZ[r]: per-offset reduced outer products over the CSR
//        pair list, cut into a fixed number of slices per offset and reduced in a fixed order;
//   db = sum_r dZ[r], from per-row-block partial sums written while dZ is formed.
// Every float32 reduction adds short plain partial sums into a Neumaier-compensated total, and
// all reduction orders are fixed, so gradients are bit-identical run to run.
#include "bwd_layout.hpp"

namespace npvs {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;


struct Comp {  // Neumaier-compensated float sum
  float s, c;
  __device__ __forceinline__ void add(float y) {
    float t = s + y;
    c += (__builtin_fabsf(s) >= __builtin_fabsf(y)) ? (s - t) + y : (y - t) + s;
    s = t;
  }
  __device__ __forceinline__ float value() const { return s + c; }
};

__device__ __forceinline__ float load_as_f32(const float *p, int64_t i) { return p[i]; }
__device__ __forceinline__ float load_as_f32(const uint16_t *p, int64_t i) { return bf16_to_f32(p[i]); }

constexpr int kDbBlocks = kBwdDbBlocks;  // row blocks of the bias-gradient partial sums (one layer)

// dZ in float32 (for wgrad; nullable) and, for the BF16 path, a bfloat16 copy (MFMA operand),
// plus the bias-gradient partial of this block's rows: blockIdx.x = partial row, blockIdx.y = a
// window of 64 columns (one window when C <= 64), 256 threads.  With vec (C % 4 == 0 and 16-byte
// aligned rows) a thread owns 4 adjacent columns, else one; the threads of a row group cover the
// window of one row, the row groups stride over the block's rows and are combined in LDS in a
// fixed order.
__device__ __forceinline__ void load4(const float *p, int64_t e, float *v) {
  const f32x4_t x = *reinterpret_cast<const f32x4_t *>(p + e);
  v[0] = x[0], v[1] = x[1], v[2] = x[2], v[3] = x[3];
}
__device__ __forceinline__ void load4(const uint16_t *p, int64_t e, float *v) {
  const uint2 x = *reinterpret_cast<const uint2 *>(p + e);
  v[0] = bf16_to_f32((uint16_t)x.x), v[1] = bf16_to_f32((uint16_t)(x.x >> 16));
  v[2] = bf16_to_f32((uint16_t)x.y), v[3] = bf16_to_f32((uint16_t)(x.y >> 16));
}

template <typename T>
__global__ __launch_bounds__(256) void relu_grad_kernel(const T *__restrict__ Y, const float *__restrict__ dY,
                                                         const npvs_counts *__restrict__ counts, int C, int relu,
                                                         int vec, float *__restrict__ dZ32, uint16_t *__restrict__ dZ16,
                                                         float *__restrict__ dbpart) {
  __shared__ float red[256 * 4];
  const int64_t n = counts->n_sites;
  const int64_t r0 = n * blockIdx.x / gridDim.x, r1 = n * (blockIdx.x + 1) / gridDim.x;
  const int c0 = 64 * blockIdx.y, Cw = C - c0 < 64 ? C - c0 : 64;
  const int V = vec ? 4 : 1, TPR = Cw / V, RG = 256 / TPR;
  const int cg = threadIdx.x % TPR, rg = threadIdx.x / TPR;
  Comp a[4] = {{0.0f, 0.0f}, {0.0f, 0.0f}, {0.0f, 0.0f}, {0.0f, 0.0f}};
  if (rg < RG) {
    if (vec) {
      for (int64_t r = r0 + rg; r < r1; r += RG) {
        const int64_t e = r * C + c0 + 4 * cg;
        float g[4], y[4];
        load4(dY, e, g);
        if (relu) {
          load4(Y, e, y);
#pragma unroll
          for (int i = 0; i < 4; ++i) g[i] = y[i] > 0.0f ? g[i] : 0.0f;
        }
        f32x4_t o;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          o[i] = g[i];
          a[i].add(g[i]);
        }
        if (dZ32) *reinterpret_cast<f32x4_t *>(dZ32 + e) = o;
        if (dZ16) {
          uint2 h;
          h.x = (uint32_t)f32_to_bf16(g[0]) | ((uint32_t)f32_to_bf16(g[1]) << 16);
          h.y = (uint32_t)f32_to_bf16(g[2]) | ((uint32_t)f32_to_bf16(g[3]) << 16);
          *reinterpret_cast<uint2 *>(dZ16 + e) = h;
        }
      }
    } else {
      for (int64_t r = r0 + rg; r < r1; r += RG) {
        const int64_t e = r * C + c0 + cg;
        float g = dY[e];
        if (relu && !(load_as_f32(Y, e) > 0.0f)) g = 0.0f;
        if (dZ32) dZ32[e] = g;
        if (dZ16) dZ16[e] = f32_to_bf16(g);
        a[0].add(g);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) red[threadIdx.x * 4 + i] = a[i].value();
  __syncthreads();
  if (threadIdx.x < Cw) {
    const int c = threadIdx.x, g0 = c / V, comp = c % V;
    Comp t{0.0f, 0.0f};
    for (int g = 0; g < RG; ++g) t.add(red[(g * TPR + g0) * 4 + comp]);
    dbpart[(int64_t)blockIdx.x * C + c0 + c] = t.value();
  }
}

constexpr int kMaxWgradLayers = NPVS_MAX_WGRAD_LAYERS;  // layers of one batched weight-gradient launch
constexpr int kWgSlices = 16;  // slices of each offset's pair list (at most; fewer for wide layers)
constexpr int kWgBatchBlocks = 512;  // workgroups resident at once (72 KB of LDS each: two per compute unit)
constexpr size_t kWgPartBudget = size_t(8) << 20;  // bytes of float32 slice partials aimed at

// Slices per offset: 16 while the float32 partials of every slice stay within the budget (every
// layer of at most 64 x 64 channels), fewer for wider layers, at least one.
int wg_slices(int cin, int cout) {
  const size_t per = sizeof(float) * 27 * (size_t)cin * cout;
  const size_t s = kWgPartBudget / per;
  return s < 1 ? 1 : s > (size_t)kWgSlices ? kWgSlices : (int)s;
}
constexpr int kWgPairs = 32;   // pairs staged per step (vector path)
constexpr int kWgEPT = 16;     // dW entries per thread per pass (vector path)

// Vector FP32 path: grid (S slices, K offsets, output windows of 64 channels), 256 threads.
// Partial dW of offset k over slice s for the outputs o0 .. o0 + 63.  A pair member of -1 (the
// pair lists of the strided layers) reads as a zero row.
template <typename T>
__global__ __launch_bounds__(256) void wgrad_partial_kernel(const T *__restrict__ X, int cin,
                                                             const float *__restrict__ dZ, int cout,
                                                             const int32_t *__restrict__ rb_off,
                                                             const int32_t *__restrict__ pairs,
                                                             float *__restrict__ part) {
  __shared__ __align__(16) float Xs[kWgPairs][64];
  __shared__ float Gs[kWgPairs][64];
  __shared__ int in_s[2][kWgPairs], out_s[2][kWgPairs];  // pair indices of steps t (slot t % 2)
  const int k = blockIdx.y, s = blockIdx.x, S = gridDim.x, tid = threadIdx.x;
  const int o0 = 64 * blockIdx.z, ow = cout - o0 < 64 ? cout - o0 : 64;
  const int64_t pk0 = rb_off[k], pk = (int64_t)rb_off[k + 1] - pk0;
  const int64_t p0 = pk0 + pk * s / S, p1 = pk0 + pk * (s + 1) / S;
  const int nsteps = (int)((p1 - p0 + kWgPairs - 1) / kWgPairs);
  const int cw = (256 * kWgEPT) / ow < 64 ? (256 * kWgEPT) / ow : 64;  // channels of X per pass
  // the dW entries of this thread: with a full 64 x 64 window, channels 16 (tid / 64) + j of
  // output tid % 64 (the channels read as four broadcast float4 per pair); otherwise (c, o) of
  // e = tid + 256 j
  const bool block = ow == 64 && cin % 64 == 0;
  const int bc0 = 16 * (tid >> 6), bo = tid & 63;
  for (int cbase = 0; cbase < cin; cbase += cw) {
    const int cn = cin - cbase < cw ? cin - cbase : cw;
    const int e_pass = cn * ow;
    Comp acc[kWgEPT];
#pragma unroll
    for (int j = 0; j < kWgEPT; ++j) acc[j] = Comp{0.0f, 0.0f};
    // Step t stages pairs [p0 + 32 t, ..) in LDS.  The pair indices of step t + 2 are loaded
    // into registers during step t and the rows of step t + 1 too, so a step waits for memory
    // only where its products are shorter than a load.  Products and additions keep the order
    // (step, pair).
    auto pair_idx = [&](int t, int &vi, int &vo) {
      const int64_t pb = p0 + (int64_t)t * kWgPairs;
      const bool ok = tid < kWgPairs && t < nsteps && pb + tid < p1;
      vi = ok ? pairs[2 * (pb + tid)] : -1;
      vo = ok ? pairs[2 * (pb + tid) + 1] : -1;
    };
    float xr[8], gr[8];
    auto load_rows = [&](int t) {  // through the indices of step t in LDS
      const int *is = in_s[t & 1], *os = out_s[t & 1];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = tid + 256 * u, p = e >> 6, c = e & 63, ii = is[p], io = os[p];
        xr[u] = (c < cn && ii >= 0) ? load_as_f32(X, (int64_t)ii * cin + cbase + c) : 0.0f;
        gr[u] = (c < ow && io >= 0) ? dZ[(int64_t)io * cout + o0 + c] : 0.0f;
      }
    };
    auto store_rows = [&]() {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = tid + 256 * u;
        Xs[e >> 6][e & 63] = xr[u];
        Gs[e >> 6][e & 63] = gr[u];
      }
    };
    __syncthreads();  // the previous pass is done with the LDS
    if (tid < kWgPairs) {
      int vi, vo;
      pair_idx(0, vi, vo);
      in_s[0][tid] = vi;
      out_s[0][tid] = vo;
      pair_idx(1, vi, vo);
      in_s[1][tid] = vi;
      out_s[1][tid] = vo;
    }
    __syncthreads();
    if (nsteps > 0) {
      load_rows(0);
      store_rows();
    }
    __syncthreads();
    for (int t = 0; t < nsteps; ++t) {
      const int m = p1 - (p0 + (int64_t)t * kWgPairs) < kWgPairs ? (int)(p1 - (p0 + (int64_t)t * kWgPairs)) : kWgPairs;
      int ni = -1, no = -1;
      pair_idx(t + 2, ni, no);
      if (t + 1 < nsteps) load_rows(t + 1);
      if (block) {  // cn = 64: every entry is in range
        float v[kWgEPT];
#pragma unroll
        for (int j = 0; j < kWgEPT; ++j) v[j] = 0.0f;
        for (int p = 0; p < m; ++p) {
          const float g = Gs[p][bo];
#pragma unroll
          for (int q = 0; q < kWgEPT / 4; ++q) {
            const float4 x = *reinterpret_cast<const float4 *>(&Xs[p][bc0 + 4 * q]);
            v[4 * q] = fmaf(x.x, g, v[4 * q]);
            v[4 * q + 1] = fmaf(x.y, g, v[4 * q + 1]);
            v[4 * q + 2] = fmaf(x.z, g, v[4 * q + 2]);
            v[4 * q + 3] = fmaf(x.w, g, v[4 * q + 3]);
          }
        }
#pragma unroll
        for (int j = 0; j < kWgEPT; ++j) acc[j].add(v[j]);
      } else {
#pragma unroll
        for (int j = 0; j < kWgEPT; ++j) {
          const int e = tid + 256 * j;
          if (e < e_pass) {
            const int c = e / ow, o = e - c * ow;
            float v = 0.0f;
            for (int p = 0; p < m; ++p) v = fmaf(Xs[p][c], Gs[p][o], v);
            acc[j].add(v);
          }
        }
      }
      __syncthreads();  // the products of step t are done with Xs, Gs and the indices of slot t % 2
      if (t + 1 < nsteps) store_rows();
      if (tid < kWgPairs) {
        in_s[t & 1][tid] = ni;
        out_s[t & 1][tid] = no;
      }
      __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < kWgEPT; ++j) {
      const int e = tid + 256 * j;
      const int c = block ? bc0 + j : e / ow, o = block ? bo : e - (e / ow) * ow;
      if (block || e < e_pass) part[((int64_t)(k * S + s) * cin + cbase + c) * cout + o0 + o] = acc[j].value();
    }
  }
}

// BF16 path on MFMA.  256 threads = 4 waves; a workgroup computes the window of at most 64 x 64
// entries (input channels c0 .., outputs o0 ..) that its window index selects (one window when
// cin, cout <= 64), over the pairs of its slice (sliced form, grid (S, K, windows)) or of its
// range of the whole pair list (balanced form, see wgrad_bf16_kernel).
// dW_k[c][o] = sum_p X[in_p][c] dZ[out_p][o] is a [cin x P] x [P x cout] product with the pair
// index as the contraction.  128 pairs at a time are staged into LDS transposed (channel-major,
// XT[c][p], GT[o][p]) so that both MFMA operands of v_mfma_f32_32x32x16_bf16 are one 16-byte
// LDS read per lane; wave w computes the 32 x 32 block (mb, nb) = (w / OB, w % OB):
//   A (32 x 16): lane l gives XT[mb*32 + l%32][kk + 8(l/32) + j]
//   B (16 x 32): lane l gives GT[nb*32 + l%32][kk + 8(l/32) + j]
//   D: entry r of lane l is dW[mb*32 + 8(r/4) + 4(l/32) + r%4][nb*32 + l%32]
// A staging task is 4 consecutive pairs x 8 channels of X or dZ (at most 2 per thread; the 8
// tasks of one pair quad sit in adjacent lanes).  The pair
// indices are fetched two chunks ahead and the rows of the next chunk are loaded while the
// current chunk's products run, then stored into the other LDS buffer.  Each chunk's product
// starts from zero and is added into a compensated total.
constexpr int kWgChunk = 128;
constexpr int kMaxWgOffsets = 27;  // offsets of one pair list (27 for 3^3 layers, 8 for strided ones)
constexpr int kWgPitch = kWgChunk + 16;  // bf16 elements per LDS row (padding spreads banks)
constexpr int kWgQuads = kWgChunk / 4;

// LDS position of pair p of staged row `row` (a channel): the 16-byte blocks of 8 pairs are
// permuted within the row by XOR with (row / 8) % 8 and with bit 2 of the row.  The row pitch
// (72 dwords) puts row r on 16-byte bank group (2 r + block) % 8.  A staging store writes 4 pairs
// of rows 8 cc + j for 8 channel groups cc at once: without the swizzle all 8 on one bank group,
// with it (row / 8 differs) on 8 different ones.  An MFMA operand read has 8 lanes read rows
// 8 g .. 8 g + 7 at one block: 2 r alone puts rows i and i + 4 on the same group, and bit 2
// separates them.  A block stays 16 bytes and aligned, so an operand is one 16-byte read.
__device__ __forceinline__ int wg_lds_pos(int row, int p) {
  return row * kWgPitch + ((((p >> 3) ^ (row >> 3) ^ ((row >> 2) & 1)) & 15) << 3) + (p & 7);
}

struct WgTask {
  int pq, cc;  // pair quad, 8-channel group within X (isx) or dZ
  bool isx, valid;
};

// Loads are unconditional (a missing pair reads pair pb, a missing row reads row 0; both exist
// whenever the chunk does) so that the wait before a chunk's use only covers that chunk's loads.
__device__ __forceinline__ void wg_indices(const int32_t *__restrict__ pairs, int64_t pb, int m, const WgTask &t,
                                           int *r) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int p = 4 * t.pq + i;
    const bool ok = t.valid && p < m;
    const int v = pairs[2 * (pb + (ok ? p : 0)) + (t.isx ? 0 : 1)];
    r[i] = ok ? v : -1;
  }
}

__device__ __forceinline__ void wg_gather(const uint16_t *__restrict__ X, int cin, const uint16_t *__restrict__ G,
                                          int cout, const WgTask &t, const int *r, uint4 *v) {
  const uint16_t *src = t.isx ? X : G;
  const int C = t.isx ? cin : cout;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const bool ok = r[i] >= 0;
    const uint4 x = *reinterpret_cast<const uint4 *>(src + (ok ? (int64_t)r[i] * C + 8 * t.cc : 0));
    const uint32_t m = ok ? ~0u : 0u;  // a mask, not a select of the loaded value: no branch around the load
    v[i] = make_uint4(x.x & m, x.y & m, x.z & m, x.w & m);
  }
}

__device__ __forceinline__ uint32_t word_of(const uint4 &v, int w) {
  return w == 0 ? v.x : w == 1 ? v.y : w == 2 ? v.z : v.w;
}

// Channel j of the 4 staged rows as two packed dwords (rows 0,1 and rows 2,3): one byte permute
// per dword picks the same 16-bit half of two source words (0x05040100: low halves, 0x07060302:
// high halves).
__device__ __forceinline__ void wg_store(uint16_t *XT, uint16_t *GT, const WgTask &t, const uint4 *v) {
  if (!t.valid) return;
  uint16_t *dst = t.isx ? XT : GT;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const uint32_t sel = (j & 1) ? 0x07060302u : 0x05040100u;
    const uint2 pk2 = make_uint2(__builtin_amdgcn_perm(word_of(v[1], j >> 1), word_of(v[0], j >> 1), sel),
                                 __builtin_amdgcn_perm(word_of(v[3], j >> 1), word_of(v[2], j >> 1), sel));
    *reinterpret_cast<uint2 *>(dst + wg_lds_pos(8 * t.cc + j, 4 * t.pq)) = pk2;
  }
}

// The layers of one weight-gradient launch (one rulebook): layer i owns the windows
// blockIdx.z in [z0, next layer's z0).
struct WgLayer {
  const uint16_t *X, *dZ;
  float *part;
  int cin, cout, z0;
};
struct WgBatch {
  int n;
  WgLayer L[kMaxWgradLayers];
};

// A chunk: pairs [pb, pb + m) of offset k; `last` when it ends the workgroup's part of offset k
// (the partial sum of that offset is then written out).
struct WgChunk {
  int pb, m, k;
  bool last;
};

// Sliced form (G = 0): grid (S, K, windows); workgroup (s, k) takes slice s of offset k's pairs
// and writes partial slot k S + s.  Balanced form (G > 0): grid (G, 1, windows); with P pairs in
// the whole list of the K offsets and L = ceil(P / G), workgroup g takes pairs [g L, (g + 1) L)
// (clipped to P), so every workgroup has the same number of pairs whatever their spread over
// the offsets, and writes the partial of each offset k its range meets to slot g + k.  The pair
// list is ordered by offset, so a later workgroup only meets the same or later offsets: no two
// (g, k) written share a slot, and the slots number at most G + K - 1.  The workgroups that
// meet offset k (pairs [a, b)) are g = a / L .. (b - 1) / L, which is how the reduction finds
// them.
__global__ __launch_bounds__(256) void wgrad_bf16_kernel(const WgBatch B, const int32_t *__restrict__ rb_off,
                                                          const int32_t *__restrict__ pairs, int G, int K) {
  // two staging buffers: chunk ch is read from buffer ch & 1 while chunk ch + 1 is written to the
  // other one, so one barrier per chunk orders both
  __shared__ __attribute__((aligned(16))) uint16_t XT[2][64 * kWgPitch];
  __shared__ __attribute__((aligned(16))) uint16_t GT[2][64 * kWgPitch];
  __shared__ int offs[kMaxWgOffsets + 1];
  int li = 0;
  for (int i = 1; i < B.n; ++i) li = (int)blockIdx.z >= B.L[i].z0 ? i : li;
  const uint16_t *__restrict__ X = B.L[li].X;
  const uint16_t *__restrict__ dZ16 = B.L[li].dZ;
  float *__restrict__ part = B.L[li].part;
  const int cin = B.L[li].cin, cout = B.L[li].cout, z = (int)blockIdx.z - B.L[li].z0;
  const int s = blockIdx.x, S = gridDim.x, tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index, uniform (scalar)
  const int otiles = (cout + 63) / 64;
  const int c0 = 64 * (z / otiles), o0 = 64 * (z % otiles);
  const int cw = cin - c0 < 64 ? cin - c0 : 64, ow = cout - o0 < 64 ? cout - o0 : 64;  // window size
  if (tid <= K) offs[tid] = rb_off[tid];
  __syncthreads();
  // this workgroup's pairs [pA, pB) and the offset of its first pair
  int pA, pB, k0;
  if (G > 0) {
    const int64_t P = offs[K] - offs[0], L = (P + G - 1) / G;
    const int64_t a = (int64_t)s * L, b = a + L;
    pA = offs[0] + (int)(a < P ? a : P);
    pB = offs[0] + (int)(b < P ? b : P);
    k0 = 0;
    while (k0 + 1 < K && offs[k0 + 1] <= pA) ++k0;
  } else {
    k0 = blockIdx.y;
    const int64_t pk = offs[k0 + 1] - offs[k0];
    pA = offs[k0] + (int)(pk * s / S);
    pB = offs[k0] + (int)(pk * (s + 1) / S);
  }
  // chunks in order: at most kWgChunk pairs, never across an offset boundary
  auto next_chunk = [&](int &p, int &k) {
    const int end = pB < offs[k + 1] ? pB : offs[k + 1];
    const int m = end - p < kWgChunk ? end - p : kWgChunk;
    const WgChunk c{p, m, k, p + m == end};
    p += m;
    if (c.last)
      while (k + 1 < K && offs[k + 1] <= p) ++k;  // past the end of offset k (and empty offsets)
    return c;
  };
  int nch = 0;
  {
    int p = pA, k = k0;
    while (p < pB) {
      next_chunk(p, k);
      ++nch;
    }
  }
  // 32 x 32 blocks of the window: wave wv computes block (wv / OB, wv % OB) when wv < nblk
  const int CB = (cw + 31) / 32, OB = (ow + 31) / 32, nblk = CB * OB;
  const int cin8 = (cw + 7) / 8, cout8 = (ow + 7) / 8;
  // rows are read from the window's first channel on; the row pitch stays cin / cout
  const uint16_t *Xw = X + c0, *Gw = dZ16 + o0;
  // tasks of X first, then of dZ; the channel group runs fastest, so the lanes of one load
  // instruction cover whole 128-byte rows (8 lanes per row) instead of 16 bytes of 64 rows
  WgTask task[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int t = tid + 256 * u, nx = cin8 * kWgQuads;
    task[u].isx = t < nx;
    const int tt = task[u].isx ? t : t - nx, c8 = task[u].isx ? cin8 : cout8;
    task[u].cc = tt % c8;
    task[u].pq = tt / c8;
    task[u].valid = t < (cin8 + cout8) * kWgQuads;
  }
  // channel rows past cin / cout (up to the 16-row MFMA block) stay zero; the others are written
  // by every chunk
  for (int e = cw * kWgPitch / 2 + tid; e < CB * 32 * kWgPitch / 2; e += 256) {
    reinterpret_cast<uint32_t *>(XT[0])[e] = 0;
    reinterpret_cast<uint32_t *>(XT[1])[e] = 0;
  }
  for (int e = ow * kWgPitch / 2 + tid; e < OB * 32 * kWgPitch / 2; e += 256) {
    reinterpret_cast<uint32_t *>(GT[0])[e] = 0;
    reinterpret_cast<uint32_t *>(GT[1])[e] = 0;
  }
  Comp tot[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) tot[r] = Comp{0.0f, 0.0f};
  // the partial of offset k goes to slot k S + s (sliced) or s + k (balanced, s = g); entry r of
  // lane l is dW[mb 32 + 8 (r / 4) + 4 (l / 32) + r % 4][nb 32 + l % 32]
  auto write_partial = [&](int k, const Comp(&t)[16], bool zero) {
    const int64_t slot = G > 0 ? (int64_t)s + k : (int64_t)k * S + s;
    if (wv < nblk) {
      const int mb = wv / OB, nb = wv % OB;
      const int o = nb * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int c = mb * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (c < cw && o < ow) part[(slot * cin + c0 + c) * cout + o0 + o] = zero ? 0.0f : t[r].value();
      }
    }
  };
  // an empty slice of the sliced form still writes its (zero) slot, which the reduction reads;
  // the balanced form's reduction reads only the slots of ranges that meet an offset
  if (nch == 0) {
    if (G == 0) write_partial(k0, tot, true);
    return;
  }
  // chunk descriptors: q0 = chunk ch, q1 = ch + 1, q2 = ch + 2; the prefetches past the last
  // chunk re-read the last chunk (no branch around a load)
  int gp = pA, gk = k0;
  WgChunk q0 = next_chunk(gp, gk);
  WgChunk q1 = nch > 1 ? next_chunk(gp, gk) : q0;
  WgChunk q2 = nch > 2 ? next_chunk(gp, gk) : q1;
  int rn[2][4];
  {
    uint4 v[2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      wg_indices(pairs, q0.pb, q0.m, task[u], rn[u]);
      wg_gather(Xw, cin, Gw, cout, task[u], rn[u], v[u]);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      wg_indices(pairs, q1.pb, q1.m, task[u], rn[u]);
      wg_store(XT[0], GT[0], task[u], v[u]);
    }
  }
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int cur = ch & 1;
    uint4 v[2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u) wg_gather(Xw, cin, Gw, cout, task[u], rn[u], v[u]);  // chunk ch + 1
#pragma unroll
    for (int u = 0; u < 2; ++u) wg_indices(pairs, q2.pb, q2.m, task[u], rn[u]);
    f32x16_t acc = {};
    {
      // a wave past nblk computes on in-range rows and is discarded at the store, so the
      // products need no branch
      const int mb = wv / OB < 1 ? wv / OB : 1, nb = wv % OB;
#pragma unroll
      for (int kk = 0; kk < kWgChunk; kk += 16) {
        const bf16x8_t a =
            *reinterpret_cast<const bf16x8_t *>(XT[cur] + wg_lds_pos(mb * 32 + (lane & 31), kk + 8 * (lane >> 5)));
        const bf16x8_t b =
            *reinterpret_cast<const bf16x8_t *>(GT[cur] + wg_lds_pos(nb * 32 + (lane & 31), kk + 8 * (lane >> 5)));
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) tot[r].add(acc[r]);
    if (q0.last) {  // the end of this workgroup's part of offset q0.k
      write_partial(q0.k, tot, false);
#pragma unroll
      for (int r = 0; r < 16; ++r) tot[r] = Comp{0.0f, 0.0f};
    }
    q0 = q1;
    q1 = q2;
    if (ch + 3 < nch) q2 = next_chunk(gp, gk);
    // the other buffer was last read in chunk ch - 1, before the barrier that ended it
#pragma unroll
    for (int u = 0; u < 2; ++u) wg_store(XT[cur ^ 1], GT[cur ^ 1], task[u], v[u]);
    __syncthreads();
  }
}

// The final reductions of the layers of one launch: layer i owns the blocks [b0, next layer's b0):
// nbw blocks for dW, then one per 4 bias channels.
struct RdLayer {
  const float *wpart, *dbpart;
  float *dW, *db;
  int cin, cout, nbw, b0, S;  // S: slices per offset of this layer's partials (sliced form)
};
struct RdBatch {
  int n;
  RdLayer L[kMaxWgradLayers];
};

// Per layer: blocks [0, nbw) reduce dW (K offsets) over the slices (grid-stride, one entry per
// thread); each block after them reduces db over the nparts partial rows for 4 channels, one wave
// per channel: lane l adds partials l, l + 64, ..., then a fixed butterfly adds the 64 lane totals;
// lane 0 writes.  G > 0: the partials are those of the balanced weight-gradient form with G
// workgroups per window over the pair list rb_off (see wgrad_bf16_kernel), added in the order of g.
__global__ __launch_bounds__(256) void grad_reduce_kernel(const RdBatch B, int nparts, int K, int G,
                                                           const int32_t *__restrict__ rb_off) {
  int li = 0;
  for (int i = 1; i < B.n; ++i) li = (int)blockIdx.x >= B.L[i].b0 ? i : li;
  const float *__restrict__ wpart = B.L[li].wpart;
  const float *__restrict__ dbpart = B.L[li].dbpart;
  float *__restrict__ dW = B.L[li].dW;
  float *__restrict__ db = B.L[li].db;
  const int cin = B.L[li].cin, cout = B.L[li].cout, nbw = B.L[li].nbw, S = B.L[li].S;
  const int bx = (int)blockIdx.x - B.L[li].b0;
  if (bx < nbw && G > 0) {  // nbw = K blocks_per_offset: block bx reduces 256 entries of one offset
    const int64_t E = (int64_t)cin * cout;
    const int per_k = (int)((E + 255) / 256), k = bx / per_k;
    const int64_t ce = (int64_t)(bx - k * per_k) * 256 + threadIdx.x;
    const int off0 = rb_off[0];
    const int64_t P = rb_off[K] - off0;
    const int a = rb_off[k] - off0, b = rb_off[k + 1] - off0;
    Comp t{0.0f, 0.0f};
    if (a < b && ce < E) {
      const uint32_t L = (uint32_t)((P + G - 1) / G);
      const int g0 = (int)((uint32_t)a / L), g1 = (int)((uint32_t)(b - 1) / L);
      const float *src = wpart + (int64_t)k * E + ce;  // slot g + k of this entry: src[g E]
      for (int g = g0; g <= g1; g += 4) {  // four slots loaded before any is added, in order of g
        float v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = g + i <= g1 ? src[(int64_t)(g + i) * E] : 0.0f;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (g + i <= g1) t.add(v[i]);
      }
    }
    if (ce < E) dW[(int64_t)k * E + ce] = t.value();
    return;
  }
  if (bx < nbw) {
    const int64_t E = (int64_t)cin * cout;
    for (int64_t e = (int64_t)bx * blockDim.x + threadIdx.x; e < K * E; e += (int64_t)nbw * blockDim.x) {
      Comp a{0.0f, 0.0f};
      const int64_t k = e / E, ce = e % E;
      if (S == kWgSlices) {  // the usual count, unrolled so that the loads are issued together
#pragma unroll
        for (int s = 0; s < kWgSlices; ++s) a.add(wpart[(k * kWgSlices + s) * E + ce]);
      } else {
        for (int s = 0; s < S; ++s) a.add(wpart[(k * S + s) * E + ce]);
      }
      dW[e] = a.value();
    }
    return;
  }
  const int o = (bx - nbw) * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (o >= cout) return;  // whole waves leave together
  Comp a{0.0f, 0.0f};
  for (int s = lane; s < nparts; s += 64) a.add(dbpart[s * cout + o]);
  float t = a.value();
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off, 64);
  if (lane == 0) db[o] = t;
}

npvs_status bwd_form_dz(int32_t dtype, const void *Y, const float *dY, const npvs_counts *counts, int32_t C,
                        int32_t relu, float *dZ32, uint16_t *dZ16, float *dbpart, hipStream_t s) {
  const int vec = C % 4 == 0 && (reinterpret_cast<uintptr_t>(dY) & 15) == 0 &&
                  (!relu || (reinterpret_cast<uintptr_t>(Y) & (dtype == NPVS_F32 ? 15 : 7)) == 0);
  const dim3 gz(kDbBlocks, (C + 63) / 64);
  if (dtype == NPVS_F32)
    relu_grad_kernel<float><<<gz, 256, 0, s>>>((const float *)Y, dY, counts, C, relu, vec, dZ32, nullptr, dbpart);
  else
    relu_grad_kernel<uint16_t><<<gz, 256, 0, s>>>((const uint16_t *)Y, dY, counts, C, relu, vec, nullptr, dZ16,
                                                   dbpart);
  return check_hip(hipGetLastError(), "backward: dZ");
}

npvs_status bwd_wgrad(int32_t dtype, const void *X, int32_t cin, const void *dZ, int32_t cout, int32_t K,
                      const int32_t *rb_off, const int32_t *pairs, int S, float *wpart, hipStream_t s) {
  if (dtype == NPVS_F32)
    wgrad_partial_kernel<float><<<dim3(S, K, (cout + 63) / 64), 256, 0, s>>>(
        (const float *)X, cin, (const float *)dZ, cout, rb_off, pairs, wpart);
  else {
    WgBatch B{};
    B.n = 1;
    B.L[0] = WgLayer{(const uint16_t *)X, (const uint16_t *)dZ, wpart, cin, cout, 0};
    wgrad_bf16_kernel<<<dim3(S, K, ((cin + 63) / 64) * ((cout + 63) / 64)), 256, 0, s>>>(B, rb_off, pairs, 0, K);
  }
  return check_hip(hipGetLastError(), "backward: weight gradient");
}

static int reduce_blocks(int32_t K, int32_t cin, int32_t cout) {
  return stride_grid((int64_t)K * cin * cout, 256, 2048);
}

npvs_status bwd_reduce(const float *wpart, const float *dbpart, int nparts, int32_t K, int S, int32_t cin,
                       int32_t cout, float *dW, float *db, hipStream_t s) {
  const int nbw = reduce_blocks(K, cin, cout);
  RdBatch B{};
  B.n = 1;
  B.L[0] = RdLayer{wpart, dbpart, dW, db, cin, cout, nbw, 0, S};
  grad_reduce_kernel<<<nbw + (cout + 3) / 4, 256, 0, s>>>(B, nparts, K, 0, nullptr);
  return check_hip(hipGetLastError(), "backward: reductions");
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace: float32 dZ (FP32 path), bfloat16 dZ (BF16 path), the slice partials of dW, the bias
// partials, and the split-input partials of the data gradient (BF16 layers with 1024+ outputs,
// whose data gradient reads that many channels).
static void bwd_ws_layout(int32_t cin, int32_t cout, int32_t cap, int32_t dtype, size_t *o_dz32, size_t *o_dz16,
                          size_t *o_wp, size_t *o_dbp, size_t *o_dx, size_t *dx_bytes, size_t *bytes) {
  size_t o = 0;
  *o_dz32 = o;
  if (dtype == NPVS_F32) o += align256(sizeof(float) * (size_t)cap * cout);
  *o_dz16 = o;
  if (dtype == NPVS_BF16) o += align256(sizeof(uint16_t) * (size_t)cap * cout);
  *o_wp = o;
  o += align256(sizeof(float) * 27 * wg_slices(cin, cout) * (size_t)cin * cout);
  *o_dbp = o;
  o += align256(sizeof(float) * kDbBlocks * (size_t)cout);
  *o_dx = o;
  *dx_bytes = conv_fwd_ws_bytes(cout, cin, cap, dtype);
  o += align256(*dx_bytes);
  *bytes = o;
}

void bwd_ws_dz_parts(int32_t cin, int32_t cout, int32_t cap, size_t *o_dz16, size_t *o_dbpart, size_t *bytes) {
  size_t a, c, e, f;
  bwd_ws_layout(cin, cout, cap, NPVS_BF16, &a, o_dz16, &c, o_dbpart, &e, &f, bytes);
}

}  // namespace npvs

using namespace npvs;

extern "C" npvs_status npvs_conv_bwd_workspace_size(int32_t cin, int32_t cout, int32_t cap_sites, int32_t dtype,
                                                    size_t *bytes) {
  if (!bytes || cin < 1 || cout < 1 || cap_sites < 1)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_conv_bwd_workspace_size: bad arguments");
  size_t a, b, c, d, e, f;
  bwd_ws_layout(cin, cout, cap_sites, dtype, &a, &b, &c, &d, &e, &f, bytes);
  return NPVS_OK;
}

// One event per thread and device orders a second stream after the first.  Re-recording it is
// safe: a wait takes the state the event had when the wait was enqueued.
static npvs_status fork_event(hipEvent_t *ev) {
  constexpr int kMaxDevices = 64;
  thread_local hipEvent_t events[kMaxDevices] = {};
  int dev = 0;
  npvs_status st = check_hip(hipGetDevice(&dev), "backward stream join");
  if (st != NPVS_OK) return st;
  if (dev < 0 || dev >= kMaxDevices) return fail(NPVS_ERR_UNSUPPORTED, "backward stream join: device index");
  if (!events[dev]) {
    st = check_hip(hipEventCreateWithFlags(&events[dev], hipEventDisableTiming), "backward stream join");
    if (st != NPVS_OK) return st;
  }
  *ev = events[dev];
  return NPVS_OK;
}

// s2 waits for the work enqueued so far on s (no-op when they are the same stream).
static npvs_status join_after(hipStream_t s, hipStream_t s2) {
  if (s2 == s) return NPVS_OK;
  hipEvent_t ev;
  npvs_status st = fork_event(&ev);
  if (st == NPVS_OK) st = check_hip(hipEventRecord(ev, s), "backward stream join");
  if (st == NPVS_OK) st = check_hip(hipStreamWaitEvent(s2, ev, 0), "backward stream join");
  return st;
}

// dZ and the bias partials on s; the data gradient on s; the weight gradient on s2 and the
// reductions on s3 (s2 first waits for the dZ of s, s3 for the weight gradient of s2; equal
// streams need no wait).
static npvs_status conv_bwd(const void *X, int32_t cin, const void *Wt, int32_t cout, const void *Y, const float *dY,
                            const int32_t *nbr, const int32_t *rb_off, const int32_t *rb_pairs,
                            const npvs_counts *counts, int32_t cap_sites, int32_t dtype, int32_t relu, float *dX,
                            float *dW, float *db, void *ws, size_t ws_bytes, hipStream_t s, hipStream_t s2,
                            hipStream_t s3) {
  if (!X || !dY || !nbr || !rb_off || !rb_pairs || !counts || !ws || (relu && !Y) || (dX && !Wt))
    return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_bwd: null pointer");
  if (!dW != !db) return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_bwd: dW and db must both be given or both null");
  if (cin < 1 || cout < 1 || cap_sites < 1) return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_bwd: bad sizes");
  if (dtype != NPVS_F32 && dtype != NPVS_BF16)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_bwd: dtype must be NPVS_F32 or NPVS_BF16");
  if (dtype == NPVS_BF16 && (cin % 8 || cout % 8))
    return fail(NPVS_ERR_UNSUPPORTED, "npvs_sparse_conv_bwd: BF16 needs cin % 8 == 0 and cout % 8 == 0");
  size_t o32, o16, owp, odb, odx, dx_bytes, need;
  bwd_ws_layout(cin, cout, cap_sites, dtype, &o32, &o16, &owp, &odb, &odx, &dx_bytes, &need);
  if (ws_bytes < need) return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_bwd: workspace too small");
  char *w = static_cast<char *>(ws);
  // the FP32 path keeps dZ in float32, the BF16 path in bfloat16 only (both of its products read it)
  float *dZ32 = dtype == NPVS_F32 ? reinterpret_cast<float *>(w + o32) : nullptr;
  uint16_t *dZ16 = dtype == NPVS_BF16 ? reinterpret_cast<uint16_t *>(w + o16) : nullptr;
  float *wpart = reinterpret_cast<float *>(w + owp);
  float *dbpart = reinterpret_cast<float *>(w + odb);
  npvs_status st = bwd_form_dz(dtype, Y, dY, counts, cout, relu, dZ32, dZ16, dbpart, s);
  if (st != NPVS_OK) return st;
  if (dW) st = join_after(s, s2);
  if (st != NPVS_OK) return st;
  if (dX) {
    st = conv_fwd_dispatch(dtype == NPVS_F32 ? (const void *)dZ32 : (const void *)dZ16, cout, Wt, nullptr, cin, nbr,
                           counts, cap_sites, dtype, 0, 1, dX, s, kDefaultConvVariant, dx_bytes ? w + odx : nullptr,
                           dx_bytes);
    if (st != NPVS_OK) return st;
  }
  if (!dW) return NPVS_OK;  // dZ and the bias partials stay in ws for npvs_sparse_conv_wgrad
  const int S = wg_slices(cin, cout);
  st = bwd_wgrad(dtype, X, cin, dtype == NPVS_F32 ? (const void *)dZ32 : (const void *)dZ16, cout, 27, rb_off,
                 rb_pairs, S, wpart, s2);
  if (st == NPVS_OK) st = join_after(s2, s3);
  if (st != NPVS_OK) return st;
  return bwd_reduce(wpart, dbpart, kDbBlocks, 27, S, cin, cout, dW, db, s3);
}


extern "C" npvs_status npvs_sparse_conv_bwd(const void *X, int32_t cin, const void *Wt, int32_t cout, const void *Y,
                                           const float *dY, const int32_t *nbr, const int32_t *rb_off,
                                           const int32_t *rb_pairs, const npvs_counts *counts, int32_t cap_sites,
                                           int32_t dtype, int32_t relu, float *dX, float *dW, float *db, void *ws,
                                           size_t ws_bytes, void *stream, void *wgrad_stream, void *reduce_stream) {
  const hipStream_t s = as_stream(stream);
  const hipStream_t s2 = wgrad_stream ? as_stream(wgrad_stream) : s;
  const hipStream_t s3 = reduce_stream ? as_stream(reduce_stream) : s2;
  return conv_bwd(X, cin, Wt, cout, Y, dY, nbr, rb_off, rb_pairs, counts, cap_sites, dtype, relu, dX, dW, db, ws,
                  ws_bytes, s, s2, s3);
}

extern "C" npvs_status npvs_sparse_conv_wgrad(int32_t n_layers, const npvs_wgrad_layer *layers,
                                             const int32_t *rb_off, const int32_t *rb_pairs, int32_t cap_sites,
                                             int32_t dtype, int32_t slices, void *stream) {
  if (!layers || !rb_off || !rb_pairs) return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_wgrad: null pointer");
  if (n_layers < 1 || n_layers > NPVS_MAX_WGRAD_LAYERS || cap_sites < 1 || slices < 0)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_wgrad: bad sizes");
  if (dtype != NPVS_F32 && dtype != NPVS_BF16)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_wgrad: dtype must be NPVS_F32 or NPVS_BF16");
  int S = kWgSlices, windows = 0;
  for (int i = 0; i < n_layers; ++i) {
    const npvs_wgrad_layer &l = layers[i];
    if (!l.X || !l.ws || !l.dW || !l.db) return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_wgrad: null pointer");
    if (l.cin < 1 || l.cout < 1) return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_wgrad: bad sizes");
    if (dtype == NPVS_BF16 && (l.cin % 8 || l.cout % 8))
      return fail(NPVS_ERR_UNSUPPORTED, "npvs_sparse_conv_wgrad: BF16 needs cin % 8 == 0 and cout % 8 == 0");
    size_t a, b, c, d, e, f, need;
    bwd_ws_layout(l.cin, l.cout, cap_sites, dtype, &a, &b, &c, &d, &e, &f, &need);
    if (l.ws_bytes < need) return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_wgrad: workspace too small");
    const int sl = wg_slices(l.cin, l.cout);
    S = sl < S ? sl : S;
    windows += ((l.cin + 63) / 64) * ((l.cout + 63) / 64);
  }
  // BF16 with slices = 0: the balanced form, at most kWgBatchBlocks workgroups in all so that they
  // run in one round, and at most as many per window as the partial slots allow (G + 26 slots of
  // the 27 S the workspace holds); otherwise the sliced form with `slices` slices per offset
  int G = 0;
  if (slices > 0) {
    S = slices < S ? slices : S;
  } else if (dtype == NPVS_BF16) {
    const int want = kWgBatchBlocks / windows, cap = 27 * S - 26;
    G = want < cap ? want : cap;
    G = G < 1 ? 1 : G;
  }
  const hipStream_t s = as_stream(stream);
  WgBatch W{};
  RdBatch R{};
  W.n = R.n = n_layers;
  int z0 = 0, b0 = 0;
  for (int i = 0; i < n_layers; ++i) {
    const npvs_wgrad_layer &l = layers[i];
    size_t o32, o16, owp, odb, odx, dxb, need;
    bwd_ws_layout(l.cin, l.cout, cap_sites, dtype, &o32, &o16, &owp, &odb, &odx, &dxb, &need);
    char *w = static_cast<char *>(l.ws);
    float *wpart = reinterpret_cast<float *>(w + owp);
    const float *dbpart = reinterpret_cast<const float *>(w + odb);
    // FP32: one launch per layer (the FP32 kernel's grid is per layer), each with the layer's own
    // slice count (or `slices` when smaller)
    int Sl = S;
    if (dtype == NPVS_F32) {
      Sl = wg_slices(l.cin, l.cout);
      Sl = slices > 0 && slices < Sl ? slices : Sl;
      const npvs_status st = bwd_wgrad(dtype, l.X, l.cin, w + o32, l.cout, 27, rb_off, rb_pairs, Sl, wpart, s);
      if (st != NPVS_OK) return st;
    }
    W.L[i] = WgLayer{(const uint16_t *)l.X, reinterpret_cast<const uint16_t *>(w + o16), wpart, l.cin, l.cout, z0};
    z0 += ((l.cin + 63) / 64) * ((l.cout + 63) / 64);
    const int nbw = G > 0 ? 27 * (int)(((int64_t)l.cin * l.cout + 255) / 256) : reduce_blocks(27, l.cin, l.cout);
    R.L[i] = RdLayer{wpart, dbpart, l.dW, l.db, l.cin, l.cout, nbw, b0, Sl};
    b0 += nbw + (l.cout + 3) / 4;
  }
  if (dtype == NPVS_BF16) {
    const dim3 grid = G > 0 ? dim3(G, 1, z0) : dim3(S, 27, z0);
    wgrad_bf16_kernel<<<grid, 256, 0, s>>>(W, rb_off, rb_pairs, G, 27);
    const npvs_status st = check_hip(hipGetLastError(), "npvs_sparse_conv_wgrad: weight gradient");
    if (st != NPVS_OK) return st;
  }
  grad_reduce_kernel<<<b0, 256, 0, s>>>(R, kDbBlocks, 27, G, rb_off);
  return check_hip(hipGetLastError(), "npvs_sparse_conv_wgrad: reductions");
}

extern "C" npvs_status npvs_sparse_conv_dgrad_relu(const void *Wt, int32_t cin, int32_t cout, const void *M,
                                                  int32_t cin_below, const int32_t *nbr, const npvs_counts *counts,
                                                  int32_t cap_sites, const void *ws, size_t ws_bytes,
                                                  void *ws_below, size_t ws_below_bytes, void *stream) {
  if (!Wt || !nbr || !counts || !ws || !ws_below)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_dgrad_relu: null pointer");
  if (cin < 1 || cout < 1 || cin_below < 1 || cap_sites < 1)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_dgrad_relu: bad sizes");
  if (ws == ws_below) return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_dgrad_relu: ws and ws_below must differ");
  if (cin > 64 || cout > 64 || cin % 8 || cout % 8 || cin_below % 8)
    return fail(NPVS_ERR_UNSUPPORTED,
                "npvs_sparse_conv_dgrad_relu: needs cin, cout <= 64 and cin, cout, cin_below multiples of 8");
  size_t a, o16, c, d, e, f, need;
  bwd_ws_layout(cin, cout, cap_sites, NPVS_BF16, &a, &o16, &c, &d, &e, &f, &need);
  if (ws_bytes < need) return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_dgrad_relu: workspace too small");
  size_t b16, bdb;
  bwd_ws_layout(cin_below, cin, cap_sites, NPVS_BF16, &a, &b16, &c, &bdb, &e, &f, &need);
  if (ws_below_bytes < need)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_dgrad_relu: workspace of the layer below too small");
  const uint16_t *dZ = reinterpret_cast<const uint16_t *>(static_cast<const char *>(ws) + o16);
  char *wb = static_cast<char *>(ws_below);
  return dgrad_relu_fused(dZ, cout, Wt, cin, nbr, counts, cap_sites, static_cast<const uint16_t *>(M),
                          reinterpret_cast<uint16_t *>(wb + b16), reinterpret_cast<float *>(wb + bdb),
                          as_stream(stream));
}
