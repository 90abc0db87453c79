// Pieces of the two-level sparse U-Net backbone (Sec. 3.3 adopts an encoder/decoder; the
// supplement's network settings give its shapes: down ratio 2, embedding and encoder channels
// 64, decoder channels 96).  Level 0 holds the active blocks of interleave factor d, level 1
// those of factor 2d, which are exactly the 2x2x2 groups of level-0 blocks with an active member.
//   * level maps: children[k][c] (level-0 row of child k of level-1 row c, or -1) and
//     parent[f] = 8 * (level-1 row) + k for level-0 row f, k = ((bz&1)*2 + (by&1))*2 + (bx&1);
//   * strided convolution (kernel 2, stride 2): Y1[c] = b + sum_k X0[children[k][c]] W_k;
//   * its inverse on the same blocks: Y0[f] = b + X1[parent row of f] W_{k(f)};
//   * the skip connection's channel concatenation Y[r] = [A[r] | B[r]].
// Weights of the two strided layers are [8][cin][cout], packed like the submanifold ones.
#include "npvs_common.hpp"

namespace npvs {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;

// Per-grid geometry of both levels (the full batch descriptors would not fit a kernel argument).
struct LevelDesc {
  int32_t n;
  int32_t Bx[NPVS_MAX_GRIDS], By[NPVS_MAX_GRIDS];      // level-0 blocks
  int32_t off0[NPVS_MAX_GRIDS], off1[NPVS_MAX_GRIDS];  // first global key per level
};

__device__ __forceinline__ int level_grid(const int32_t *off, int n, int32_t key) {
  int b = 0;
  while (b + 1 < n && key >= off[b + 1]) ++b;
  return b;
}

// One thread per level-1 row (its 8 children, looked up in the level-0 block table) and per
// level-0 row (its parent, looked up in the level-1 table); rows past the counts get -1.
__global__ __launch_bounds__(256) void level_maps_kernel(LevelDesc L, const npvs_counts *__restrict__ c0,
                                                         const int32_t *__restrict__ keys0,
                                                         const int32_t *__restrict__ row0, int cap0,
                                                         const npvs_counts *__restrict__ c1,
                                                         const int32_t *__restrict__ keys1,
                                                         const int32_t *__restrict__ row1, int cap1,
                                                         int32_t *__restrict__ children, int32_t *__restrict__ parent) {
  const int n0 = c0->n_sites, n1 = c1->n_sites;
  const int64_t total = (int64_t)cap1 + cap0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    if (i < cap1) {
      const int r = (int)i;
      if (r >= n1) {
#pragma unroll
        for (int k = 0; k < 8; ++k) children[(int64_t)k * cap1 + r] = -1;
        continue;
      }
      const int32_t key = keys1[r];
      const int b = level_grid(L.off1, L.n, key);
      const int Bx = L.Bx[b], By = L.By[b], Cx = Bx >> 1, Cy = By >> 1;
      const int32_t l = key - L.off1[b];
      const int cx = l % Cx, cy = (l / Cx) % Cy, cz = l / (Cx * Cy);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int fx = 2 * cx + (k & 1), fy = 2 * cy + ((k >> 1) & 1), fz = 2 * cz + (k >> 2);
        children[(int64_t)k * cap1 + r] = row0[L.off0[b] + (fz * By + fy) * Bx + fx];
      }
    } else {
      const int f = (int)(i - cap1);
      if (f >= n0) {
        parent[f] = -1;
        continue;
      }
      const int32_t key = keys0[f];
      const int b = level_grid(L.off0, L.n, key);
      const int Bx = L.Bx[b], By = L.By[b], Cx = Bx >> 1, Cy = By >> 1;
      const int32_t l = key - L.off0[b];
      const int bx = l % Bx, by = (l / Bx) % By, bz = l / (Bx * By);
      const int32_t r1 = row1[L.off1[b] + ((bz >> 1) * Cy + (by >> 1)) * Cx + (bx >> 1)];
      const int k = ((bz & 1) * 2 + (by & 1)) * 2 + (bx & 1);
      parent[f] = r1 >= 0 ? r1 * 8 + k : -1;
    }
  }
}

// ------------------------------------------------------------------------------------------
// Packing of K-offset weights [K][cin][cout]: the F32 layout is the weight itself; the BF16
// layout is that of the submanifold kernels, Wp[k][nb][kb][lane][j] = W[k][kb*32 + 8(lane/16) + j]
// [nb*16 + lane%16] (zero outside cin x cout).
// ------------------------------------------------------------------------------------------
// With transpose the packed weight is P_k = W_k^T ([K][cout][cin]: the data gradient of the
// strided layers), else P = W.
__global__ void pack_k_kernel(const float *__restrict__ W, int K, int cin, int cout, int transpose, int dtype,
                              void *__restrict__ P) {
  const int CI = transpose ? cout : cin, CO = transpose ? cin : cout;
  const int KB = (CI + 31) / 32, NB = (CO + 15) / 16;
  const int64_t total = dtype == NPVS_F32 ? (int64_t)K * CI * CO : (int64_t)K * NB * KB * 512;
  auto src = [&](int k, int c, int o) {  // P[k][c][o]
    return transpose ? W[((int64_t)k * cin + o) * cout + c] : W[((int64_t)k * cin + c) * cout + o];
  };
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    if (dtype == NPVS_F32) {
      const int o = (int)(e % CO), c = (int)((e / CO) % CI), k = (int)(e / ((int64_t)CO * CI));
      static_cast<float *>(P)[e] = src(k, c, o);
      continue;
    }
    const int j = e & 7, lane = (e >> 3) & 63;
    const int64_t frag = e >> 9;
    const int kb = frag % KB, nb = (frag / KB) % NB, k = (int)(frag / ((int64_t)KB * NB));
    const int c = kb * 32 + 8 * (lane >> 4) + j, o = nb * 16 + (lane & 15);
    const float v = (c < CI && o < CO) ? src(k, c, o) : 0.0f;
    static_cast<uint16_t *>(P)[e] = f32_to_bf16(v);
  }
}

// ------------------------------------------------------------------------------------------
// Strided convolution and its inverse, BF16 on MFMA (v_mfma_f32_16x16x32_bf16, FP32
// accumulation), computed as D = W^T X^T like the submanifold kernels: a wave owns 16 output
// rows, lane l's B operand is 8 input channels of the row of lane l%16, and its accumulator
// holds 4 consecutive output channels of that row.  Output channel blocks are taken four at a
// time.  Down: each of the 8 offsets gathers the row's child (zeros for a missing child).  Up:
// the parent row is gathered once per channel chunk and enters only the product of the row's
// own offset (the other offsets see zeros), so one pass over the 8 weight blocks serves rows of
// every offset.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ uint4 row8(const uint16_t *__restrict__ X, int cin, int idx, int c0) {
  const bool ok = idx >= 0 && c0 < cin;  // cin % 8 == 0: a chunk of 8 is wholly in or out
  const uint4 v = *reinterpret_cast<const uint4 *>(X + (ok ? (int64_t)idx * cin + c0 : 0));
  const uint32_t m = ok ? ~0u : 0u;  // a mask, not a branch around the load
  return make_uint4(v.x & m, v.y & m, v.z & m, v.w & m);
}

__device__ __forceinline__ bf16x8_t as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8_t, v); }

template <bool UP>
__global__ __launch_bounds__(256) void strided_bf16_kernel(const uint16_t *__restrict__ X, int cin,
                                                           const bf16x8_t *__restrict__ Wp,
                                                           const float *__restrict__ bias, int cout,
                                                           const int32_t *__restrict__ map,
                                                           const npvs_counts *__restrict__ counts, int cap, int relu,
                                                           int out_f32, void *__restrict__ Y) {
  const int n = counts->n_sites;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int KB = (cin + 31) / 32, NB = (cout + 15) / 16, csub = 8 * (lane >> 4);
  const int ntiles = (n + 15) / 16;
  for (int tile = blockIdx.x * 4 + wv; tile < ntiles; tile += gridDim.x * 4) {
    const int r = tile * 16 + (lane & 15);
    int idx[8];
    int prow = -1, kf = -1;
    if constexpr (UP) {
      const int m = r < n ? map[r] : -1;
      prow = m >= 0 ? m >> 3 : -1;
      kf = m >= 0 ? m & 7 : -1;
    } else {
#pragma unroll
      for (int k = 0; k < 8; ++k) idx[k] = r < n ? map[(int64_t)k * cap + r] : -1;
    }
    for (int ng = 0; ng < NB; ng += 4) {
      f32x4_t acc[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[j] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
      for (int kb = 0; kb < KB; ++kb) {
        uint4 up = make_uint4(0u, 0u, 0u, 0u);
        if constexpr (UP) up = row8(X, cin, prow, kb * 32 + csub);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          uint4 v;
          if constexpr (UP) {
            const uint32_t m = kf == k ? ~0u : 0u;
            v = make_uint4(up.x & m, up.y & m, up.z & m, up.w & m);
          } else {
            v = row8(X, cin, idx[k], kb * 32 + csub);
          }
          const bf16x8_t b = as_bf16x8(v);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            // blocks past NB compute on a valid fragment and are not stored (no branch around
            // the products)
            const int nb = ng + j < NB ? ng + j : NB - 1;
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Wp[((int64_t)(k * NB + nb) * KB + kb) * 64 + lane], b,
                                                             acc[j], 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int o = (ng + j) * 16 + 4 * (lane >> 4);
        if (ng + j >= NB || r >= n || o >= cout) continue;
        float v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          v[i] = acc[j][i] + (bias ? bias[o + i] : 0.0f);
          if (relu && v[i] < 0.0f) v[i] = 0.0f;
        }
        if (out_f32) {
          *reinterpret_cast<f32x4_t *>(static_cast<float *>(Y) + (int64_t)r * cout + o) = f32x4_t{v[0], v[1], v[2], v[3]};
        } else {
          uint2 h;
          h.x = (uint32_t)f32_to_bf16(v[0]) | ((uint32_t)f32_to_bf16(v[1]) << 16);
          h.y = (uint32_t)f32_to_bf16(v[2]) | ((uint32_t)f32_to_bf16(v[3]) << 16);
          *reinterpret_cast<uint2 *>(static_cast<uint16_t *>(Y) + (int64_t)r * cout + o) = h;
        }
      }
    }
  }
}

// FP32 (vector FMA): one thread per output entry, channels summed in order.
template <bool UP>
__global__ __launch_bounds__(256) void strided_f32_kernel(const float *__restrict__ X, int cin,
                                                          const float *__restrict__ P, const float *__restrict__ bias,
                                                          int cout, const int32_t *__restrict__ map,
                                                          const npvs_counts *__restrict__ counts, int cap, int relu,
                                                          float *__restrict__ Y) {
  const int64_t total = (int64_t)counts->n_sites * cout;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / cout), o = (int)(e % cout);
    float acc = 0.0f;
    if constexpr (UP) {
      const int m = map[r];
      if (m >= 0) {
        const float *x = X + (int64_t)(m >> 3) * cin;
        const float *w = P + (int64_t)(m & 7) * cin * cout + o;
        for (int c = 0; c < cin; ++c) acc = fmaf(x[c], w[(int64_t)c * cout], acc);
      }
    } else {
      for (int k = 0; k < 8; ++k) {
        const int i = map[(int64_t)k * cap + r];
        if (i < 0) continue;
        const float *x = X + (int64_t)i * cin;
        const float *w = P + (int64_t)k * cin * cout + o;
        for (int c = 0; c < cin; ++c) acc = fmaf(x[c], w[(int64_t)c * cout], acc);
      }
    }
    const float v = acc + (bias ? bias[o] : 0.0f);
    Y[e] = (relu && v < 0.0f) ? 0.0f : v;
  }
}

// Channel concatenation, 16 bytes per thread step.
__global__ __launch_bounds__(256) void concat_kernel(const uint4 *__restrict__ A, int qa, const uint4 *__restrict__ B,
                                                     int qb, const npvs_counts *__restrict__ counts,
                                                     uint4 *__restrict__ Y) {
  const int q = qa + qb;
  const int64_t total = (int64_t)counts->n_sites * q;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / q;
    const int j = (int)(e % q);
    Y[e] = j < qa ? A[r * qa + j] : B[r * qb + (j - qa)];
  }
}

// Pair lists of the strided layers' weight gradients, one CSR segment per child index k over the
// coarse rows c < n1: (children[k][c], c) for the strided convolution (input level 0, output level
// 1), (c, children[k][c]) for its inverse.  A missing child (-1) stays in the list and reads as a
// zero row.  rb_off[k] = k n1.
__global__ __launch_bounds__(256) void strided_pairs_kernel(const int32_t *__restrict__ children,
                                                            const npvs_counts *__restrict__ counts1, int cap1, int up,
                                                            int32_t *__restrict__ rb_off,
                                                            int32_t *__restrict__ pairs) {
  const int n1 = counts1->n_sites;
  if (blockIdx.x == 0 && threadIdx.x <= 8) rb_off[threadIdx.x] = (int32_t)threadIdx.x * n1;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < 8LL * n1; e += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(e / n1), c = (int)(e % n1);
    const int32_t m = children[(int64_t)k * cap1 + c];
    pairs[2 * e] = up ? c : m;
    pairs[2 * e + 1] = up ? m : c;
  }
}

// Gradient of the channel concatenation Y = [A | B]: dA[r] = dY[r][0, ca), dB[r] = dY[r][ca,
// ca + cb) + add[r] (add nullable: the skip's gradient from its other consumer), float32, four
// channels per thread step.
__global__ __launch_bounds__(256) void concat_bwd_kernel(const f32x4_t *__restrict__ dY, int qa, int qb,
                                                         const f32x4_t *__restrict__ add,
                                                         const npvs_counts *__restrict__ counts,
                                                         f32x4_t *__restrict__ dA, f32x4_t *__restrict__ dB) {
  const int q = qa + qb;
  const int64_t total = (int64_t)counts->n_sites * q;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / q;
    const int j = (int)(e % q);
    if (j < qa) {
      if (dA) dA[r * qa + j] = dY[e];
    } else if (dB) {
      const int64_t i = r * qb + (j - qa);
      dB[i] = add ? dY[e] + add[i] : dY[e];
    }
  }
}

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace of the strided backward: dZ [cap_out][cout] (float32 or bfloat16), the pair list
// [8 cap1][2], rb_off [9], the weight-gradient slice partials and the bias partials.
static void strided_bwd_layout(int32_t cin, int32_t cout, int32_t cap_in, int32_t cap_out, int32_t up, int32_t dtype,
                               size_t *o_pairs, size_t *o_off, size_t *o_wp, size_t *o_dbp, size_t *bytes) {
  const size_t cap1 = up ? cap_in : cap_out;
  size_t o = al256((dtype == NPVS_F32 ? 4 : 2) * (size_t)cap_out * cout);
  *o_pairs = o;
  o += al256(sizeof(int32_t) * 2 * 8 * cap1);
  *o_off = o;
  o += al256(sizeof(int32_t) * 9);
  *o_wp = o;
  o += al256(sizeof(float) * 8 * wg_slices(cin, cout) * (size_t)cin * cout);
  *o_dbp = o;
  o += al256(sizeof(float) * kBwdDbBlocks * (size_t)cout);
  *bytes = o;
}

}  // namespace npvs

using namespace npvs;

extern "C" npvs_status npvs_level_maps(int32_t n_grids, const npvs_dims *dims, int32_t d, const npvs_counts *counts0,
                                      const int32_t *site_keys0, const int32_t *block_row0, int32_t cap0,
                                      const npvs_counts *counts1, const int32_t *site_keys1,
                                      const int32_t *block_row1, int32_t cap1, int32_t *children, int32_t *parent,
                                      void *stream) {
  if (!counts0 || !site_keys0 || !block_row0 || !counts1 || !site_keys1 || !block_row1 || !children || !parent)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_level_maps: null pointer");
  if (cap0 < 1 || cap1 < 1) return fail(NPVS_ERR_INVALID_ARG, "npvs_level_maps: capacities must be >= 1");
  Batch B0, B1;
  npvs_status st = make_batch(n_grids, dims, d, nullptr, &B0);
  if (st != NPVS_OK) return st;
  if (d > 16) return fail(NPVS_ERR_INVALID_ARG, "npvs_level_maps: 2d must be at most 32");
  st = make_batch(n_grids, dims, 2 * d, nullptr, &B1);  // extents must be multiples of 2d
  if (st != NPVS_OK) return st;
  LevelDesc L = {};
  L.n = n_grids;
  for (int b = 0; b < n_grids; ++b) {
    L.Bx[b] = B0.g[b].Bx;
    L.By[b] = B0.g[b].By;
    L.off0[b] = B0.g[b].key_off;
    L.off1[b] = B1.g[b].key_off;
  }
  level_maps_kernel<<<stride_grid((int64_t)cap0 + cap1, 256, 1024), 256, 0, as_stream(stream)>>>(
      L, counts0, site_keys0, block_row0, cap0, counts1, site_keys1, block_row1, cap1, children, parent);
  return check_hip(hipGetLastError(), "npvs_level_maps");
}

extern "C" size_t npvs_packed_weight_bytes_k(int32_t K, int32_t cin, int32_t cout, int32_t dtype) {
  if (K < 1 || cin < 1 || cout < 1) return 0;
  if (dtype == NPVS_F32) return sizeof(float) * (size_t)K * cin * cout;
  if (dtype == NPVS_BF16) return (size_t)K * ((cout + 15) / 16) * ((cin + 31) / 32) * 1024;
  return 0;
}

extern "C" npvs_status npvs_pack_weights_k(const float *W, int32_t K, int32_t cin, int32_t cout, int32_t transpose,
                                          int32_t dtype, void *Wp, void *stream) {
  if (!W || !Wp) return fail(NPVS_ERR_INVALID_ARG, "npvs_pack_weights_k: null pointer");
  if (K < 1 || cin < 1 || cout < 1) return fail(NPVS_ERR_INVALID_ARG, "npvs_pack_weights_k: bad sizes");
  if (dtype != NPVS_F32 && dtype != NPVS_BF16)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_pack_weights_k: dtype must be NPVS_F32 or NPVS_BF16");
  const int64_t elems = (int64_t)npvs_packed_weight_bytes_k(K, transpose ? cout : cin, transpose ? cin : cout, dtype) /
                        (dtype == NPVS_F32 ? 4 : 2);
  pack_k_kernel<<<stride_grid(elems, 256, 1024), 256, 0, as_stream(stream)>>>(W, K, cin, cout, transpose ? 1 : 0,
                                                                              dtype, Wp);
  return check_hip(hipGetLastError(), "npvs_pack_weights_k");
}


extern "C" npvs_status npvs_strided_conv_fwd(const void *X, int32_t cin, const void *Wp, const float *bias,
                                            int32_t cout, const int32_t *map, int32_t up,
                                            const npvs_counts *counts_out, int32_t cap_out, int32_t dtype,
                                            int32_t relu, int32_t out_f32, void *Y, void *stream) {
  if (!X || !Wp || !map || !counts_out || !Y) return fail(NPVS_ERR_INVALID_ARG, "npvs_strided_conv_fwd: null pointer");
  if (cin < 1 || cout < 1 || cap_out < 1) return fail(NPVS_ERR_INVALID_ARG, "npvs_strided_conv_fwd: bad sizes");
  if (X == Y) return fail(NPVS_ERR_INVALID_ARG, "npvs_strided_conv_fwd: X and Y must not alias");
  hipStream_t s = as_stream(stream);
  if (dtype == NPVS_F32) {
    const int G = stride_grid((int64_t)cap_out * cout, 256, 4096);
    if (up)
      strided_f32_kernel<true><<<G, 256, 0, s>>>((const float *)X, cin, (const float *)Wp, bias, cout, map,
                                                 counts_out, cap_out, relu, (float *)Y);
    else
      strided_f32_kernel<false><<<G, 256, 0, s>>>((const float *)X, cin, (const float *)Wp, bias, cout, map,
                                                  counts_out, cap_out, relu, (float *)Y);
  } else if (dtype == NPVS_BF16) {
    if (cin % 8 || cout % 8)
      return fail(NPVS_ERR_UNSUPPORTED, "npvs_strided_conv_fwd: BF16 needs cin % 8 == 0 and cout % 8 == 0");
    const int G = stride_grid(((int64_t)cap_out + 15) / 16, 4, 2048);
    if (up)
      strided_bf16_kernel<true><<<G, 256, 0, s>>>((const uint16_t *)X, cin, (const bf16x8_t *)Wp, bias, cout, map,
                                                  counts_out, cap_out, relu, out_f32, Y);
    else
      strided_bf16_kernel<false><<<G, 256, 0, s>>>((const uint16_t *)X, cin, (const bf16x8_t *)Wp, bias, cout, map,
                                                   counts_out, cap_out, relu, out_f32, Y);
  } else {
    return fail(NPVS_ERR_INVALID_ARG, "npvs_strided_conv_fwd: dtype must be NPVS_F32 or NPVS_BF16");
  }
  return check_hip(hipGetLastError(), "npvs_strided_conv_fwd");
}

extern "C" npvs_status npvs_concat_channels(const void *A, int32_t ca, const void *B, int32_t cb, int32_t elem_bytes,
                                           const npvs_counts *counts, int32_t cap, void *Y, void *stream) {
  if (!A || !B || !counts || !Y) return fail(NPVS_ERR_INVALID_ARG, "npvs_concat_channels: null pointer");
  if (ca < 1 || cb < 1 || cap < 1 || (elem_bytes != 2 && elem_bytes != 4))
    return fail(NPVS_ERR_INVALID_ARG, "npvs_concat_channels: bad sizes");
  if ((ca * elem_bytes) % 16 || (cb * elem_bytes) % 16)
    return fail(NPVS_ERR_UNSUPPORTED, "npvs_concat_channels: rows of A and B must be multiples of 16 bytes");
  const int qa = ca * elem_bytes / 16, qb = cb * elem_bytes / 16;
  concat_kernel<<<stride_grid((int64_t)cap * (qa + qb), 256, 4096), 256, 0, as_stream(stream)>>>(
      (const uint4 *)A, qa, (const uint4 *)B, qb, counts, (uint4 *)Y);
  return check_hip(hipGetLastError(), "npvs_concat_channels");
}

extern "C" npvs_status npvs_concat_channels_bwd(const float *dY, int32_t ca, int32_t cb, const float *add_b,
                                               const npvs_counts *counts, int32_t cap, float *dA, float *dB,
                                               void *stream) {
  if (!dY || !counts || (!dA && !dB)) return fail(NPVS_ERR_INVALID_ARG, "npvs_concat_channels_bwd: null pointer");
  if (ca < 1 || cb < 1 || cap < 1) return fail(NPVS_ERR_INVALID_ARG, "npvs_concat_channels_bwd: bad sizes");
  if (ca % 4 || cb % 4) return fail(NPVS_ERR_UNSUPPORTED, "npvs_concat_channels_bwd: ca and cb must be multiples of 4");
  const uintptr_t any = reinterpret_cast<uintptr_t>(dY) | reinterpret_cast<uintptr_t>(add_b) |
                        reinterpret_cast<uintptr_t>(dA) | reinterpret_cast<uintptr_t>(dB);
  if (any & 15) return fail(NPVS_ERR_INVALID_ARG, "npvs_concat_channels_bwd: buffers must be 16-byte aligned");
  const int qa = ca / 4, qb = cb / 4;
  concat_bwd_kernel<<<stride_grid((int64_t)cap * (qa + qb), 256, 4096), 256, 0, as_stream(stream)>>>(
      (const f32x4_t *)dY, qa, qb, (const f32x4_t *)add_b, counts, (f32x4_t *)dA, (f32x4_t *)dB);
  return check_hip(hipGetLastError(), "npvs_concat_channels_bwd");
}

extern "C" npvs_status npvs_strided_bwd_workspace_size(int32_t cin, int32_t cout, int32_t cap_in, int32_t cap_out,
                                                      int32_t up, int32_t dtype, size_t *bytes) {
  if (!bytes || cin < 1 || cout < 1 || cap_in < 1 || cap_out < 1)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_strided_bwd_workspace_size: bad arguments");
  size_t a, b, c, d;
  strided_bwd_layout(cin, cout, cap_in, cap_out, up, dtype, &a, &b, &c, &d, bytes);
  return NPVS_OK;
}

extern "C" npvs_status npvs_strided_conv_bwd(const void *X, int32_t cin, const void *Wt, int32_t cout, const void *Y,
                                            const float *dY, const int32_t *children, const int32_t *parent,
                                            int32_t up, const npvs_counts *counts_in, int32_t cap_in,
                                            const npvs_counts *counts_out, int32_t cap_out, int32_t dtype,
                                            int32_t relu, float *dX, float *dW, float *db, void *ws, size_t ws_bytes,
                                            void *stream) {
  if (!X || !dY || !children || !parent || !counts_in || !counts_out || !dW || !db || !ws || (relu && !Y) ||
      (dX && !Wt))
    return fail(NPVS_ERR_INVALID_ARG, "npvs_strided_conv_bwd: null pointer");
  if (cin < 1 || cout < 1 || cap_in < 1 || cap_out < 1)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_strided_conv_bwd: bad sizes");
  if (dtype != NPVS_F32 && dtype != NPVS_BF16)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_strided_conv_bwd: dtype must be NPVS_F32 or NPVS_BF16");
  if (dtype == NPVS_BF16 && (cin % 8 || cout % 8))
    return fail(NPVS_ERR_UNSUPPORTED, "npvs_strided_conv_bwd: BF16 needs cin % 8 == 0 and cout % 8 == 0");
  size_t o_pairs, o_off, o_wp, o_dbp, need;
  strided_bwd_layout(cin, cout, cap_in, cap_out, up, dtype, &o_pairs, &o_off, &o_wp, &o_dbp, &need);
  if (ws_bytes < need) return fail(NPVS_ERR_INVALID_ARG, "npvs_strided_conv_bwd: workspace too small");
  char *w = static_cast<char *>(ws);
  void *dZ = w;
  int32_t *pairs = reinterpret_cast<int32_t *>(w + o_pairs), *rb_off = reinterpret_cast<int32_t *>(w + o_off);
  float *wpart = reinterpret_cast<float *>(w + o_wp), *dbpart = reinterpret_cast<float *>(w + o_dbp);
  const hipStream_t s = as_stream(stream);
  npvs_status st = bwd_form_dz(dtype, Y, dY, counts_out, cout, relu, dtype == NPVS_F32 ? (float *)dZ : nullptr,
                               dtype == NPVS_BF16 ? (uint16_t *)dZ : nullptr, dbpart, s);
  if (st != NPVS_OK) return st;
  if (dX) {  // the data gradient is the opposite strided layer with the transposed weights
    st = npvs_strided_conv_fwd(dZ, cout, Wt, nullptr, cin, up ? children : parent, up ? 0 : 1, counts_in, cap_in,
                               dtype, 0, 1, dX, stream);
    if (st != NPVS_OK) return st;
  }
  const int cap1 = up ? cap_in : cap_out;
  strided_pairs_kernel<<<stride_grid(8LL * cap1, 256, 1024), 256, 0, s>>>(children, up ? counts_in : counts_out, cap1,
                                                                         up ? 1 : 0, rb_off, pairs);
  st = check_hip(hipGetLastError(), "npvs_strided_conv_bwd");
  if (st != NPVS_OK) return st;
  const int S = wg_slices(cin, cout);
  st = bwd_wgrad(dtype, X, cin, dZ, cout, 8, rb_off, pairs, S, wpart, s);
  if (st != NPVS_OK) return st;
  return bwd_reduce(wpart, dbpart, kBwdDbBlocks, 8, S, cin, cout, dW, db, s);
}
