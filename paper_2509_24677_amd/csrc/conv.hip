// Submanifold sparse 3x3x3 convolution, forward (Sec. 2.3, 3.3):
//   Y[r][o] = act(b[o] + sum_k sum_c X[nbr[k][r]][c] W[k][c][o])
// Output-stationary gather-GEMM: a tile of output rows loops over the 27 offsets, gathers the
// neighbour rows of each offset and multiplies them by W_k.  Each offset really is a dense
// [rows x Cin] x [Cin x Cout] contraction, so the BF16 path runs it on MFMA.
#include "conv_common.hpp"

namespace npvs {

// ------------------------------------------------------------------------------------------
// Weight packing.  P is the conv weight a kernel reads, [27][CI][CO]:
//   plain: P[k][c][o] = W[k][c][o]            (CI = cin,  CO = cout)
//   flip : P[k][c][o] = W[26-k][o][c]         (CI = cout, CO = cin; the data-gradient weight)
// F32 layout: P itself.  BF16 layout: MFMA A-operand fragments of P^T for
// v_mfma_f32_16x16x32_bf16, Wp[k][nb][kb][lane][j] = P[k][kb*32 + 8*(lane/16) + j][nb*16 + lane%16]
// (zero outside CI x CO), so each lane loads its 8 values with one 16-byte load.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ float packed_src(const float *W, int cin, int cout, int flip, int k, int c, int o) {
  return flip ? W[((int64_t)(26 - k) * cin + o) * cout + c] : W[((int64_t)k * cin + c) * cout + o];
}

__global__ void pack_f32_kernel(const float *__restrict__ W, int cin, int cout, int flip, float *__restrict__ P) {
  const int CI = flip ? cout : cin, CO = flip ? cin : cout;
  const int64_t total = 27LL * CI * CO;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int o = e % CO, c = (e / CO) % CI, k = e / ((int64_t)CO * CI);
    P[e] = packed_src(W, cin, cout, flip, k, c, o);
  }
}

__device__ __forceinline__ void pack_bf16_entry(const float *__restrict__ W, int cin, int cout, int flip,
                                                uint16_t *__restrict__ P, int64_t e) {
  const int CI = flip ? cout : cin, CO = flip ? cin : cout;
  const int KB = (CI + 31) / 32, NB = (CO + 15) / 16;
  int j = e & 7, lane = (e >> 3) & 63;
  int64_t f = e >> 9;  // fragment index (k, nb, kb)
  int kb = f % KB, nb = (f / KB) % NB, k = f / ((int64_t)KB * NB);
  int c = kb * 32 + 8 * (lane >> 4) + j, o = nb * 16 + (lane & 15);
  float v = (c < CI && o < CO) ? packed_src(W, cin, cout, flip, k, c, o) : 0.0f;
  P[e] = f32_to_bf16(v);
}

// The buffer holds npvs_packed_weight_bytes() bytes, sized for the larger orientation; entries
// past this orientation's fragments are zero, so the whole buffer is defined.
__global__ void pack_bf16_kernel(const float *__restrict__ W, int cin, int cout, int flip, int64_t buf_elems,
                                 uint16_t *__restrict__ P) {
  const int CI = flip ? cout : cin, CO = flip ? cin : cout;
  const int64_t total = 27LL * ((CO + 15) / 16) * ((CI + 31) / 32) * 64 * 8;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < buf_elems; e += (int64_t)gridDim.x * blockDim.x) {
    if (e < total) pack_bf16_entry(W, cin, cout, flip, P, e);
    else P[e] = 0;
  }
}

// Batched packing: blockIdx.y selects the entry; each entry is grid-strided over blockIdx.x.
struct PackBatch {
  npvs_pack_desc d[NPVS_MAX_PACK];
  int64_t elems[NPVS_MAX_PACK];  // buffer entries (npvs_packed_weight_bytes / element size)
};

__global__ void pack_batch_kernel(PackBatch PB, int dtype) {
  const npvs_pack_desc &D = PB.d[blockIdx.y];
  const int flip = D.flip_transpose ? 1 : 0;
  const int CI = flip ? D.cout : D.cin, CO = flip ? D.cin : D.cout;
  const int64_t total = dtype == NPVS_F32 ? 27LL * CI * CO : 27LL * ((CO + 15) / 16) * ((CI + 31) / 32) * 64 * 8;
  const int64_t buf = PB.elems[blockIdx.y];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < buf; e += (int64_t)gridDim.x * blockDim.x) {
    if (e >= total) {
      static_cast<uint16_t *>(D.Wp)[e] = 0;  // only the BF16 layout has a tail
    } else if (dtype == NPVS_F32) {
      const int o = e % CO, c = (e / CO) % CI, k = e / ((int64_t)CO * CI);
      static_cast<float *>(D.Wp)[e] = packed_src(D.W, D.cin, D.cout, flip, k, c, o);
    } else {
      pack_bf16_entry(D.W, D.cin, D.cout, flip, static_cast<uint16_t *>(D.Wp), e);
    }
  }
}

// ------------------------------------------------------------------------------------------
// Plain FP32 path (vector FMA).  Workgroup of 256 = 4 waves; a tile of 32 output rows; blockIdx.y
// selects 64 output channels; lane = output channel, each wave owns 8 rows.  A tile is a
// sequence of steps (offset k, 64-channel input chunk c0): the step's 32 gathered rows and its
// 64 x 64 weight block go through LDS, every lane reading the rows as broadcasts and its weight
// column without conflicts.  The loads of step s + 1 are issued into registers before the
// products of step s, and the neighbour indices of offset k + 2 when offset k begins, so a step
// waits for memory only when its products are shorter than a load.  The products run in the
// order (offset, channel) for every output, so the result does not depend on the launch shape.
// ------------------------------------------------------------------------------------------
constexpr int kF32Rows = 32;

__global__ __launch_bounds__(256) void conv_fwd_f32_kernel(const float *__restrict__ X, int cin,
                                                            const float *__restrict__ P,
                                                            const float *__restrict__ bias, int cout,
                                                            const int32_t *__restrict__ nbr,
                                                            const npvs_counts *__restrict__ counts, int cap, int relu,
                                                            float *__restrict__ Y) {
  __shared__ __align__(16) float Xs[kF32Rows][64];
  __shared__ __align__(16) float Ws[64][64];
  __shared__ int idx_s[2][kF32Rows];  // neighbour indices of offsets k (slot k % 2)
  const int32_t n = counts->n_sites;
  const int ntiles = (n + kF32Rows - 1) / kF32Rows;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index, uniform (scalar)
  const int cg = 64 * blockIdx.y, o = cg + lane;
  const int CB = (cin + 63) / 64, S = 27 * CB;  // steps per tile
  for (int j = 0;; ++j) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x, ntiles, j);
    if (tile < 0) break;
    const int row0 = tile * kF32Rows;
    auto idx_load = [&](int k) {
      return tid < kF32Rows && row0 + tid < n ? nbr[(int64_t)k * cap + row0 + tid] : -1;
    };
    float xr[8], wr[16];
    auto load_step = [&](int s) {  // step s's rows (through the indices in LDS) and weights
      const int k = s / CB, c0 = (s - k * CB) * 64;
      const int *ids = idx_s[k & 1];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = tid + 256 * u, r = e >> 6, c = c0 + (e & 63), src = ids[r];
        xr[u] = src >= 0 && c < cin ? X[(int64_t)src * cin + c] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = tid + 256 * u, c = c0 + (e >> 6), oo = cg + (e & 63);
        wr[u] = c < cin && oo < cout ? P[((int64_t)k * cin + c) * cout + oo] : 0.0f;
      }
    };
    auto store_step = [&]() {
#pragma unroll
      for (int u = 0; u < 8; ++u) Xs[(tid + 256 * u) >> 6][tid & 63] = xr[u];
#pragma unroll
      for (int u = 0; u < 16; ++u) Ws[(tid + 256 * u) >> 6][tid & 63] = wr[u];
    };
    if (tid < kF32Rows) {
      idx_s[0][tid] = idx_load(0);
      idx_s[1][tid] = idx_load(1);
    }
    __syncthreads();
    load_step(0);
    store_step();
    __syncthreads();
    float acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = 0.0f;
    int ni = -1;  // indices of offset k + 2, loaded when offset k begins
    for (int s = 0; s < S; ++s) {
      const int k = s / CB, cb = s - k * CB, c0 = cb * 64;
      if (cb == 0 && k + 2 < 27) ni = idx_load(k + 2);
      if (s + 1 < S) load_step(s + 1);
      const int cn = ((cin - c0 < 64 ? cin - c0 : 64) + 3) & ~3;  // entries past cin are zero
      for (int c = 0; c < cn; c += 4) {
        const float w0 = Ws[c][lane], w1 = Ws[c + 1][lane], w2 = Ws[c + 2][lane], w3 = Ws[c + 3][lane];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const float4 xv = *reinterpret_cast<const float4 *>(&Xs[wv * 8 + i][c]);
          acc[i] = fmaf(xv.x, w0, acc[i]);
          acc[i] = fmaf(xv.y, w1, acc[i]);
          acc[i] = fmaf(xv.z, w2, acc[i]);
          acc[i] = fmaf(xv.w, w3, acc[i]);
        }
      }
      __syncthreads();  // the products of step s are done with Xs and Ws
      if (s + 1 < S) store_step();
      // offset k's indices were last read by the loads of its last step, issued during step s
      if (cb == CB - 1 && k + 2 < 27 && tid < kF32Rows) idx_s[k & 1][tid] = ni;
      __syncthreads();
    }
    if (o < cout) {
      const float bo = bias ? bias[o] : 0.0f;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int r = row0 + wv * 8 + i;
        if (r < n) {
          const float v = acc[i] + bo;
          Y[(int64_t)r * cout + o] = (relu && v < 0.0f) ? 0.0f : v;
        }
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// BF16 path on MFMA (v_mfma_f32_16x16x32_bf16, FP32 accumulation).
// The product is computed transposed, D = W^T X^T, so that a lane's accumulator holds four
// consecutive output channels of one row (a single 8- or 16-byte store):
//   A (16 x 32) = W^T block: lane l gives W[kb*32 + 8(l/16) + j][nb*16 + l%16]   (packed, one load)
//   B (32 x 16) = X^T block: lane l gives X[row0 + l%16][kb*32 + 8(l/16) + j]    (gathered row, one load)
//   D (16 x 16): lane l holds Y[row0 + l%16][nb*16 + 4(l/16) + i], i = 0..3
// A wave owns MB x 16 rows and all NB x 16 output channels.  The KSPLIT waves of a workgroup
// take consecutive slices of 27 / KSPLIT offsets of the same rows.  A wave loads the neighbour
// indices of all its offsets at once, then loads the row and weight fragments of offset q + 1
// while the MFMAs of offset q run; offsets where none of its rows has a neighbour are skipped.
// The partial sums of the waves are added in LDS in wave order (deterministic) and every wave
// finishes some of the 16 x 16 output blocks (bias, ReLU, rounding, store).
// ------------------------------------------------------------------------------------------
// 8 channels [c, c + 8) of row i of X, or zero when i < 0 or c >= cin.  The load itself is
// unconditional (a missing row reads row 0, which exists whenever a tile does, and the value is
// discarded), so the loads of a stage are the same on every path and the wait before the MFMAs
// of a stage only covers that stage's loads, not the ones prefetched after it.
template <int KB, int NB, int MB, int KSPLIT>
__global__ __launch_bounds__(64 * KSPLIT) void conv_fwd_bf16_kernel(const uint16_t *__restrict__ X, int cin,
                                                                     const bf16x8_t *__restrict__ Wp,
                                                                     const float *__restrict__ bias, int cout,
                                                                     const int32_t *__restrict__ nbr,
                                                                     const npvs_counts *__restrict__ counts, int cap,
                                                                     int relu, int out_f32, void *__restrict__ Y) {
  constexpr int ROWS = 16 * MB;
  constexpr int KPER = 27 / KSPLIT;
  constexpr int NBLK = MB * NB;
  constexpr int S = KPER * KB;  // stages: (offset, 32-channel chunk)
  constexpr int PD = S < 4 ? S : 4;  // stages in flight
  static_assert(KPER * KSPLIT == 27, "KSPLIT must divide 27");
  __shared__ f32x4_t red[KSPLIT > 1 ? KSPLIT * NBLK * 64 : 1];
  const int32_t n = counts->n_sites;
  const int ntiles = (n + ROWS - 1) / ROWS;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave index, uniform (scalar)
  const int kbeg = wv * KPER;
  const int csub = 8 * (lane >> 4);
  for (int j = 0;; ++j) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x, ntiles, j);
    if (tile < 0) break;
    const int row0 = tile * ROWS;
    const bf16x8_t *W = Wp + opaque_zero();
    int idx[KPER][MB];
#pragma unroll
    for (int q = 0; q < KPER; ++q)
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) idx[q][mb] = nbr_index(nbr, cap, kbeg + q, row0 + mb * 16 + (lane & 15), n);
    bool act[KPER];
#pragma unroll
    for (int q = 0; q < KPER; ++q) {
      bool a = false;
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) a = a || idx[q][mb] >= 0;
      act[q] = __any(a);
    }
    f32x4_t acc[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
    bf16x8_t bx[PD][MB], aw[PD][NB];
#pragma unroll
    for (int st = -(PD - 1); st < S; ++st) {
      const int ld = st + PD - 1;  // stage whose loads are issued now
      if (ld < S) {  // compile-time after unrolling; loads are issued even for skipped offsets
        const int q = ld / KB, kb = ld % KB, slot = ld % PD;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) bx[slot][mb] = gather8(X, cin, idx[q][mb], kb * 32 + csub);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) aw[slot][nb] = W[(((int64_t)(kbeg + q) * NB + nb) * KB + kb) * 64 + lane];
      }
      if (st >= 0 && act[st / KB]) {
        const int slot = st % PD;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw[slot][nb], bx[slot][mb], acc[mb][nb], 0, 0, 0);
      }
    }
    if constexpr (KSPLIT == 1) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          conv_bf16_epilogue<NB>(acc[mb][nb], row0 + mb * 16 + (lane & 15), n, nb * 16 + 4 * (lane >> 4), cout, bias,
                                 relu, out_f32, Y);
    } else {
      __syncthreads();  // the previous tile's readers are done with red
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) red[(wv * NBLK + mb * NB + nb) * 64 + lane] = acc[mb][nb];
      __syncthreads();
      for (int blk = wv; blk < NBLK; blk += KSPLIT) {
        f32x4_t sum = red[blk * 64 + lane];
        for (int w = 1; w < KSPLIT; ++w) sum += red[(w * NBLK + blk) * 64 + lane];
        const int mb = blk / NB, nb = blk % NB;
        conv_bf16_epilogue<NB>(sum, row0 + mb * 16 + (lane & 15), n, nb * 16 + 4 * (lane >> 4), cout, bias, relu,
                               out_f32, Y);
      }
    }
  }
}

// Shared-weight variant: the RG waves of a workgroup own different rows (16 MB each) and all 27
// offsets; each offset's packed weights are staged once per workgroup into a double-buffered LDS
// slot (loaded into registers one offset ahead, stored after the current offset's MFMAs), so the
// L2 reads of weights drop by a factor of RG.  The neighbour rows are gathered straight from
// global memory one offset ahead as in the split kernel.
// ------------------------------------------------------------------------------------------
// BF16 path for any channel counts (cin % 8 == 0, cout % 8 == 0), used for the shapes the tuned
// kernels above do not cover, e.g. the wide first and last layers of interleave factors 8 and 16
// (Cin or Cout = d^3 = 512 or 4096).  Workgroup = 9 waves over the same MB x 16 rows, wave w owning
// offsets 3w .. 3w + 2; blockIdx.y selects 64 output channels (4 MFMA output blocks).  The
// (offset, 32-channel chunk) stages are walked with a runtime chunk count and 4 stages in flight;
// loads past the last stage re-read it and are masked to zero, and offsets with no neighbour
// gather zeros, so every MFMA is unconditional (no branch around an accumulator).  The 9 partial
// sums are added in LDS in wave order, as in the split kernel.
// ------------------------------------------------------------------------------------------
template <int MB>
__global__ __launch_bounds__(576) void conv_fwd_bf16_wide_kernel(const uint16_t *__restrict__ X, int cin,
                                                                  const bf16x8_t *__restrict__ Wp,
                                                                  const float *__restrict__ bias, int cout,
                                                                  const int32_t *__restrict__ nbr,
                                                                  const npvs_counts *__restrict__ counts, int cap,
                                                                  int relu, int out_f32, void *__restrict__ Y,
                                                                  float *__restrict__ part) {
  constexpr int KSPLIT = 9, KPER = 3, ROWS = 16 * MB, NBLK = MB * 4, PD = 4;
  __shared__ f32x4_t red[KSPLIT * NBLK * 64];
  const int32_t n = counts->n_sites;
  const int ntiles = (n + ROWS - 1) / ROWS;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave index, uniform (scalar)
  const int kbeg = wv * KPER, csub = 8 * (lane >> 4);
  const int KB = (cin + 31) / 32, NBT = (cout + 15) / 16, nb0 = 4 * blockIdx.y;
  // input-channel split (gridDim.z > 1 only with `part`): this workgroup's 32-channel chunks
  const int KBZ = (KB + gridDim.z - 1) / gridDim.z, kb_lo = blockIdx.z * KBZ;
  const int nkb = KB - kb_lo < KBZ ? KB - kb_lo : KBZ;
  const int S = KPER * nkb;  // stages of this wave
  for (int j = 0;; ++j) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x, ntiles, j);
    if (tile < 0) break;
    const int row0 = tile * ROWS;
    const bf16x8_t *W = Wp + opaque_zero();
    int idx[KPER][MB];
#pragma unroll
    for (int q = 0; q < KPER; ++q)
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) idx[q][mb] = nbr_index(nbr, cap, kbeg + q, row0 + mb * 16 + (lane & 15), n);
    f32x4_t acc[MB][4];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) acc[mb][nb] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
    bf16x8_t bx[PD][MB], aw[PD][4];
    // operands of stage st (clamped to the last one; zero rows past the end)
    auto load = [&](int st, int slot) {
      const bool live = st < S;
      st = live ? st : S - 1;
      const int q = st / nkb, kb = kb_lo + st - q * nkb;
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const int i = q == 0 ? idx[0][mb] : q == 1 ? idx[1][mb] : idx[2][mb];
        bx[slot][mb] = gather8(X, cin, live ? i : -1, kb * 32 + csub);
      }
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        const int g = nb0 + nb < NBT ? nb0 + nb : NBT - 1;  // blocks past cout: any valid fragment
        aw[slot][nb] = W[(((int64_t)(kbeg + q) * NBT + g) * KB + kb) * 64 + lane];
      }
    };
#pragma unroll
    for (int p = 0; p < PD; ++p) load(p, p);
    for (int g = 0; g < S; g += PD) {
#pragma unroll
      for (int p = 0; p < PD; ++p) {
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw[p][nb], bx[p][mb], acc[mb][nb], 0, 0, 0);
        load(g + p + PD, p);
      }
    }
    __syncthreads();  // the previous tile's readers are done with red
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) red[(wv * NBLK + mb * 4 + nb) * 64 + lane] = acc[mb][nb];
    __syncthreads();
    for (int blk = wv; blk < NBLK; blk += KSPLIT) {
      f32x4_t sum = red[blk * 64 + lane];
      for (int w = 1; w < KSPLIT; ++w) sum += red[(w * NBLK + blk) * 64 + lane];
      const int mb = blk / 4, nb = blk % 4;
      const int r = row0 + mb * 16 + (lane & 15), o = (nb0 + nb) * 16 + 4 * (lane >> 4);
      if (part) {  // raw partial sum of this channel range; the finishing kernel adds the ranges
        if (r < n && o < cout) *reinterpret_cast<f32x4_t *>(part + ((int64_t)blockIdx.z * cap + r) * cout + o) = sum;
      } else {
        conv_bf16_epilogue<4>(sum, r, n, o, cout, bias, relu, out_f32, Y);
      }
    }
  }
}

// Sum of the channel-range partials in range order, then bias, ReLU and rounding: one thread per
// 4 outputs of an active row.
__global__ __launch_bounds__(256) void conv_splitk_finish_kernel(const float *__restrict__ part, int KZ, int cap,
                                                                  const float *__restrict__ bias, int cout,
                                                                  const npvs_counts *__restrict__ counts, int relu,
                                                                  int out_f32, void *__restrict__ Y) {
  const int64_t q = cout / 4, total = (int64_t)counts->n_sites * q;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / q), o = (int)(e % q) * 4;
    f32x4_t sum = *reinterpret_cast<const f32x4_t *>(part + (int64_t)r * cout + o);
    for (int z = 1; z < KZ; ++z) sum += *reinterpret_cast<const f32x4_t *>(part + ((int64_t)z * cap + r) * cout + o);
    conv_bf16_epilogue<4>(sum, r, r + 1, o, cout, bias, relu, out_f32, Y);
  }
}

// ------------------------------------------------------------------------------------------
// BF16 path, weight-stationary, for inputs of at most 96 channels and any number of outputs.
// Workgroup = 9 waves over the same MB x 16 rows, wave w owning offsets 3w .. 3w + 2;
// blockIdx.y selects 16 NBW output channels (NBW MFMA output blocks).  A wave loads the weight
// fragments of its 3 offsets x KB chunks x NBW output blocks once and keeps them in registers
// while the workgroup walks its row tiles; the neighbour indices of the tile after next are
// loaded during the current tile.  The 9 partial sums are added in LDS in wave order.
// ------------------------------------------------------------------------------------------
// NBW: output blocks of 16 channels per workgroup (2, 4, or 1 for 4 or 5 input chunks).  With
// two blocks the rows of the next tile are gathered into a second buffer while the current
// tile's products run; with one or four (whose weights leave no registers for a second buffer)
// they are gathered into the same buffer as soon as the products have issued, ahead of the
// reduction and the epilogue.
// With FUSE (the data gradient of a layer, feeding the backward of the layer below): the result
// is masked by M > 0 (the ReLU' of the layer below, whose output M is; no mask when M is null),
// rounded to bf16 into Y, and each epilogue wave keeps per-lane running sums of its masked values
// over the tiles its workgroup walks; at the end a fixed butterfly adds the 16 rows of each
// column and workgroup b writes row b of the bias partial table dbp[kBwdDbBlocks][cout] (rows
// past the grid are written as zeros), so the layer below's bias gradient is a fixed-order sum
// over that table.  Needs one column group (cout <= 16 NBW) and MB = 1.
template <int KB, int MB, int NBW, bool FUSE>
__device__ __forceinline__ void wsta_body(const uint16_t *__restrict__ X, int cin, const bf16x8_t *__restrict__ Wp,
                                          const float *__restrict__ bias, int cout, const int32_t *__restrict__ nbr,
                                          const npvs_counts *__restrict__ counts, int cap, int relu, int out_f32,
                                          void *__restrict__ Y, const uint16_t *__restrict__ M,
                                          float *__restrict__ dbp) {
  constexpr int KSPLIT = 9, KPER = 3, ROWS = 16 * MB, NBLK = MB * NBW;
  constexpr bool PF = NBW == 2;  // rows of the next tile prefetched (the registers of 4 blocks' weights leave no room)
  static_assert(!FUSE || MB == 1, "the fused data gradient keeps one column block per epilogue wave");
  __shared__ f32x4_t red[KSPLIT * NBLK * 64];
  const int32_t n = counts->n_sites;
  const int ntiles = (n + ROWS - 1) / ROWS;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave index, uniform (scalar)
  const int kbeg = wv * KPER, csub = 8 * (lane >> 4);
  const int NBT = (cout + 15) / 16, nb0 = NBW * blockIdx.y;
  bf16x8_t aw[KPER][KB][NBW];
#pragma unroll
  for (int q = 0; q < KPER; ++q)
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int nb = 0; nb < NBW; ++nb) {
        const int g = nb0 + nb < NBT ? nb0 + nb : NBT - 1;  // blocks past cout: any valid fragment
        aw[q][kb][nb] = Wp[(((int64_t)(kbeg + q) * NBT + g) * KB + kb) * 64 + lane];
      }
  float da[4] = {0.0f, 0.0f, 0.0f, 0.0f};  // FUSE: this lane's running column sums
  auto write_db_parts = [&]() {
    if (wv >= NBLK) return;
#pragma unroll
    for (int off = 1; off < 16; off <<= 1)
#pragma unroll
      for (int i = 0; i < 4; ++i) da[i] += __shfl_xor(da[i], off, 64);
    const int o = (nb0 + wv) * 16 + 4 * (lane >> 4);
    if ((lane & 15) == 0 && o < cout)
      for (int row = blockIdx.x; row < kBwdDbBlocks; row += gridDim.x)
        *reinterpret_cast<f32x4_t *>(dbp + (int64_t)row * cout + o) =
            row == (int)blockIdx.x ? f32x4_t{da[0], da[1], da[2], da[3]} : f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
  };
  int tile = xcd_tile(blockIdx.x, gridDim.x, ntiles, 0);
  if (tile < 0) {  // whole workgroup: tile depends on blockIdx only
    if constexpr (FUSE) write_db_parts();
    return;
  }
  // Loads retire in order, so a value used right after its load makes every load issued before
  // it wait too.  The neighbour indices are therefore loaded raw (rows past the last site read
  // the last site's entry) and judged only when their rows are gathered, and a gathered row is
  // loaded raw (a missing neighbour loads row 0) with its mask kept beside it, applied only where
  // the products read the row; the bias of the epilogue is loaded once, before the tiles.
  // (A missing tile re-reads the indices of the last valid one.)
  auto indices = [&](int t, int (&ix)[KPER][MB]) {
#pragma unroll
    for (int q = 0; q < KPER; ++q)
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const int r = t * ROWS + mb * 16 + (lane & 15);
        ix[q][mb] = nbr[(int64_t)(kbeg + q) * cap + (r < n ? r : n - 1)];
      }
  };
  // rows of tile t, whose raw indices ix holds; bit q MB + mb of m marks a row that exists
  auto rows = [&](const int (&ix)[KPER][MB], int t, uint4 (&b)[KPER][KB][MB], uint32_t &m) {
    m = 0u;
#pragma unroll
    for (int q = 0; q < KPER; ++q)
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const bool ok = t * ROWS + mb * 16 + (lane & 15) < n && ix[q][mb] >= 0;
        m |= (ok ? 1u : 0u) << (q * MB + mb);
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          const int c = kb * 32 + csub;
          b[q][kb][mb] = *reinterpret_cast<const uint4 *>(X + (ok && c < cin ? (int64_t)ix[q][mb] * cin + c : 0));
        }
      }
  };
  auto masked = [&](const uint4 &v, uint32_t m, int bit, int kb) {
    const uint32_t mm = ((m >> bit) & 1u) && kb * 32 + csub < cin ? ~0u : 0u;
    return make_uint4(v.x & mm, v.y & mm, v.z & mm, v.w & mm);
  };
  // with a second buffer, rows are masked when they become the current tile's (a whole tile after
  // their loads were issued), so the current buffer needs no mask word
  auto mask_all = [&](const uint4 (&src)[KPER][KB][MB], uint32_t m, uint4 (&dst)[KPER][KB][MB]) {
#pragma unroll
    for (int q = 0; q < KPER; ++q)
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) dst[q][kb][mb] = masked(src[q][kb][mb], m, q * MB + mb, kb);
  };
  // the epilogue block of this wave (at most one: NBLK <= KSPLIT) and its bias, loaded once
  // (except with two 16-row blocks and a second row buffer, whose registers leave no room: there
  // the epilogue loads it, after this tile's loads and before the next tile's are needed)
  constexpr bool BIAS_ONCE = !(PF && MB == 2);
  float bv[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  if constexpr (BIAS_ONCE && !FUSE) {
    const int o = (nb0 + wv % NBW) * 16 + 4 * (lane >> 4);
    if (bias && wv < NBLK && o < cout)
#pragma unroll
      for (int i = 0; i < 4; ++i) bv[i] = bias[o + i];
  }
  int ix[KPER][MB];
  uint4 bx[KPER][KB][MB];
  uint32_t bm;
  indices(tile, ix);
  rows(ix, tile, bx, bm);
  if constexpr (PF) mask_all(bx, bm, bx);
  int t1 = xcd_tile(blockIdx.x, gridDim.x, ntiles, 1);
  indices(t1 >= 0 ? t1 : tile, ix);
  for (int j = 0; tile >= 0; ++j) {
    const int t2 = xcd_tile(blockIdx.x, gridDim.x, ntiles, j + 2);
    // FUSE: the epilogue waves fetch this tile's mask before the next tile's rows are issued, so
    // waiting for it does not wait for them
    uint2 mk = {0u, 0u};
    if constexpr (FUSE) {
      const int r = tile * ROWS + (lane & 15), o = (nb0 + wv) * 16 + 4 * (lane >> 4);
      if (M && wv < NBLK && r < n && o < cout) mk = *reinterpret_cast<const uint2 *>(M + (int64_t)r * cout + o);
    }
    uint4 bn[KPER][KB][MB];
    uint32_t bnm;
    if constexpr (PF) {
      rows(ix, t1 >= 0 ? t1 : tile, bn, bnm);              // tile j + 1 (or a repeat)
      indices(t2 >= 0 ? t2 : (t1 >= 0 ? t1 : tile), ix);  // tile j + 2 (or a repeat)
    }
    f32x4_t acc[MB][NBW];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NBW; ++nb) acc[mb][nb] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int q = 0; q < KPER; ++q)
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb)
#pragma unroll
          for (int mb = 0; mb < MB; ++mb) {
            const uint4 row = PF ? bx[q][kb][mb] : masked(bx[q][kb][mb], bm, q * MB + mb, kb);
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw[q][kb][nb], __builtin_bit_cast(bf16x8_t, row),
                                                                  acc[mb][nb], 0, 0, 0);
          }
    if constexpr (!PF) {
      // without a second row buffer, the next tile's rows go into this tile's registers as soon
      // as the products have taken them, their latency hidden by the reduction and the epilogue
      rows(ix, t1 >= 0 ? t1 : tile, bx, bm);               // tile j + 1 (or a repeat)
      indices(t2 >= 0 ? t2 : (t1 >= 0 ? t1 : tile), ix);  // tile j + 2 (or a repeat)
    }
    __syncthreads();  // the previous tile's readers are done with red
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NBW; ++nb) red[(wv * NBLK + mb * NBW + nb) * 64 + lane] = acc[mb][nb];
    __syncthreads();
    const int row0 = tile * ROWS;
    for (int blk = wv; blk < NBLK; blk += KSPLIT) {
      f32x4_t sum = red[blk * 64 + lane];
#pragma unroll 4  // with the next tile's rows in flight, a full unroll would spill
      for (int w = 1; w < KSPLIT; ++w) sum += red[(w * NBLK + blk) * 64 + lane];
      const int mb = blk / NBW, nb = blk % NBW;
      const int r = row0 + mb * 16 + (lane & 15), o = (nb0 + nb) * 16 + 4 * (lane >> 4);
      if constexpr (FUSE) {
        if (r < n && o < cout) {
          float g[4] = {sum[0], sum[1], sum[2], sum[3]};
          if (M) {
            const uint16_t mv[4] = {(uint16_t)mk.x, (uint16_t)(mk.x >> 16), (uint16_t)mk.y, (uint16_t)(mk.y >> 16)};
#pragma unroll
            for (int i = 0; i < 4; ++i) g[i] = bf16_to_f32(mv[i]) > 0.0f ? g[i] : 0.0f;
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) da[i] += g[i];
          uint2 h;
          h.x = (uint32_t)f32_to_bf16(g[0]) | ((uint32_t)f32_to_bf16(g[1]) << 16);
          h.y = (uint32_t)f32_to_bf16(g[2]) | ((uint32_t)f32_to_bf16(g[3]) << 16);
          *reinterpret_cast<uint2 *>(static_cast<uint16_t *>(Y) + (int64_t)r * cout + o) = h;
        }
      } else if constexpr (BIAS_ONCE) {
        conv_bf16_epilogue_bias(sum, r, n, o, cout, bv, relu, out_f32, Y);
      } else {
        conv_bf16_epilogue<4>(sum, r, n, o, cout, bias, relu, out_f32, Y);
      }
    }
    if constexpr (PF) {
      mask_all(bn, bnm, bx);
    }
    tile = t1;
    t1 = t2;
  }
  if constexpr (FUSE) write_db_parts();
}

template <int KB, int MB, int NBW = 2>
__global__ __launch_bounds__(576) void conv_fwd_bf16_wsta_kernel(const uint16_t *__restrict__ X, int cin,
                                                                  const bf16x8_t *__restrict__ Wp,
                                                                  const float *__restrict__ bias, int cout,
                                                                  const int32_t *__restrict__ nbr,
                                                                  const npvs_counts *__restrict__ counts, int cap,
                                                                  int relu, int out_f32, void *__restrict__ Y) {
  wsta_body<KB, MB, NBW, false>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, nullptr, nullptr);
}

// The weight-stationary layer (at most 64 outputs, 16-row tiles) with its cross-wave reduction
// taken off the product waves.  Nine product waves hold the weights of three offsets each and,
// per tile, write their partial products to one of two LDS tables; three reducer waves sum a
// table (partials 0 .. 8 in order, as the single-role kernel does) and apply the epilogue while
// the product waves go on to the next tile.  One barrier per tile: a table is rewritten two
// tiles later, after a barrier that every reducer reaches only once it has read the table.  The
// twelve waves fill three per SIMD at up to 168 registers, as many as the nine-wave kernel's
// register budget allows on the busiest SIMD.
template <int KB>
__global__ __launch_bounds__(768) void conv_fwd_bf16_wsred_kernel(const uint16_t *__restrict__ X, int cin,
                                                                  const bf16x8_t *__restrict__ Wp,
                                                                  const float *__restrict__ bias, int cout,
                                                                  const int32_t *__restrict__ nbr,
                                                                  const npvs_counts *__restrict__ counts, int cap,
                                                                  int relu, int out_f32, void *__restrict__ Y) {
  constexpr int KSPLIT = 9, KPER = 3, ROWS = 16, NBLK = 4, NRED = 3;
  __shared__ f32x4_t red[2][KSPLIT * NBLK * 64];
  const int32_t n = counts->n_sites;
  const int ntiles = (n + ROWS - 1) / ROWS;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave index, uniform (scalar)
  const bool prod = wv < KSPLIT;                                     // a product wave (else a reducer)
  const int kbeg = (prod ? wv : 0) * KPER, csub = 8 * (lane >> 4);
  const int NBT = (cout + 15) / 16;
  int tile = xcd_tile(blockIdx.x, gridDim.x, ntiles, 0);
  if (tile < 0) return;  // whole workgroup: tile depends on blockIdx only
  bf16x8_t aw[KPER][KB][NBLK];
  if (prod)
#pragma unroll
    for (int q = 0; q < KPER; ++q)
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int nb = 0; nb < NBLK; ++nb) {
          const int g = nb < NBT ? nb : NBT - 1;  // blocks past cout: any valid fragment
          aw[q][kb][nb] = Wp[(((int64_t)(kbeg + q) * NBT + g) * KB + kb) * 64 + lane];
        }
  // as in the single-role kernel: indices and rows loaded raw, rows masked where the products
  // read them (loads retire in order, so nothing loaded is used right after its load)
  auto indices = [&](int t, int (&ix)[KPER]) {
#pragma unroll
    for (int q = 0; q < KPER; ++q) {
      const int r = t * ROWS + (lane & 15);
      ix[q] = nbr[(int64_t)(kbeg + q) * cap + (r < n ? r : n - 1)];
    }
  };
  auto rows = [&](const int (&ix)[KPER], int t, uint4 (&b)[KPER][KB], uint32_t &m) {
    m = 0u;
#pragma unroll
    for (int q = 0; q < KPER; ++q) {
      const bool ok = t * ROWS + (lane & 15) < n && ix[q] >= 0;
      m |= (ok ? 1u : 0u) << q;
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const int c = kb * 32 + csub;
        b[q][kb] = *reinterpret_cast<const uint4 *>(X + (ok && c < cin ? (int64_t)ix[q] * cin + c : 0));
      }
    }
  };
  // a reducer's blocks: wv - 9 and wv - 6 (the second only for wave 9); their bias, loaded once
  float bv[2][4] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
  if (!prod && bias)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int blk = wv - KSPLIT + NRED * h, o = blk * 16 + 4 * (lane >> 4);
      if (blk < NBLK && o < cout)
#pragma unroll
        for (int i = 0; i < 4; ++i) bv[h][i] = bias[o + i];
    }
  // The two roles walk the same tiles in their own loops, one barrier per tile each (the role is
  // uniform over a wave, so every wave of the workgroup meets every barrier); in the reducers'
  // loop no product registers are live, so a reducer loads all nine partials of its blocks at once.
  int t1 = xcd_tile(blockIdx.x, gridDim.x, ntiles, 1);
  if (prod) {
    int ix[KPER];
    uint4 bx[KPER][KB];
    uint32_t bm = 0u;
    indices(tile, ix);
    rows(ix, tile, bx, bm);
    indices(t1 >= 0 ? t1 : tile, ix);
    for (int j = 0; tile >= 0; ++j) {
      const int t2 = xcd_tile(blockIdx.x, gridDim.x, ntiles, j + 2);
      f32x4_t *tab = red[j & 1];
      f32x4_t acc[NBLK];
#pragma unroll
      for (int nb = 0; nb < NBLK; ++nb) acc[nb] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int q = 0; q < KPER; ++q)
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          const uint32_t mm = ((bm >> q) & 1u) && kb * 32 + csub < cin ? ~0u : 0u;
          const uint4 v = bx[q][kb];
          const uint4 row = make_uint4(v.x & mm, v.y & mm, v.z & mm, v.w & mm);
#pragma unroll
          for (int nb = 0; nb < NBLK; ++nb)
            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw[q][kb][nb], __builtin_bit_cast(bf16x8_t, row),
                                                              acc[nb], 0, 0, 0);
        }
      // the next tile's rows go into this tile's registers as soon as the products have taken
      // them; their latency is covered by the table writes, the barrier and the wait there for
      // the waves of the busiest SIMD
      rows(ix, t1 >= 0 ? t1 : tile, bx, bm);               // tile j + 1 (or a repeat)
      indices(t2 >= 0 ? t2 : (t1 >= 0 ? t1 : tile), ix);  // tile j + 2 (or a repeat)
#pragma unroll
      for (int nb = 0; nb < NBLK; ++nb) tab[(wv * NBLK + nb) * 64 + lane] = acc[nb];
      __syncthreads();  // table j % 2 is complete
      tile = t1;
      t1 = t2;
    }
  } else {
    const int blk0 = wv - KSPLIT, blk1 = blk0 + NRED;  // blk1 < NBLK for wave 9 only
    for (int j = 0; tile >= 0; ++j) {
      const int t2 = xcd_tile(blockIdx.x, gridDim.x, ntiles, j + 2);
      const f32x4_t *tab = red[j & 1];
      __syncthreads();  // table j % 2 is complete; this wave is done with table (j - 1) % 2
      f32x4_t p0[KSPLIT], p1[KSPLIT];
#pragma unroll
      for (int w = 0; w < KSPLIT; ++w) {
        p0[w] = tab[(w * NBLK + blk0) * 64 + lane];
        if (blk1 < NBLK) p1[w] = tab[(w * NBLK + blk1) * 64 + lane];
      }
      const int r = tile * ROWS + (lane & 15);
      f32x4_t sum = p0[0];
#pragma unroll
      for (int w = 1; w < KSPLIT; ++w) sum += p0[w];
      conv_bf16_epilogue_bias(sum, r, n, blk0 * 16 + 4 * (lane >> 4), cout, bv[0], relu, out_f32, Y);
      if (blk1 < NBLK) {
        sum = p1[0];
#pragma unroll
        for (int w = 1; w < KSPLIT; ++w) sum += p1[w];
        conv_bf16_epilogue_bias(sum, r, n, blk1 * 16 + 4 * (lane >> 4), cout, bv[1], relu, out_f32, Y);
      }
      tile = t1;
      t1 = t2;
    }
  }
}

// The data gradient of a BF16 layer with the ReLU' of the layer below fused in: dZ_below =
// bf16(conv(dZ, W') masked by M > 0) and the bias partial table dbp (see wsta_body).
template <int KB>
__global__ __launch_bounds__(576) void dgrad_relu_bf16_wsta_kernel(const uint16_t *__restrict__ dZ, int cin,
                                                                    const bf16x8_t *__restrict__ Wt, int cout,
                                                                    const int32_t *__restrict__ nbr,
                                                                    const npvs_counts *__restrict__ counts, int cap,
                                                                    uint16_t *__restrict__ dZ_below,
                                                                    const uint16_t *__restrict__ M,
                                                                    float *__restrict__ dbp) {
  wsta_body<KB, 1, 4, true>(dZ, cin, Wt, nullptr, cout, nbr, counts, cap, 0, 0, dZ_below, M, dbp);
}

template <int KB, int NB, int MB, int RG>
__global__ __launch_bounds__(64 * RG) void conv_fwd_bf16_lds_kernel(const uint16_t *__restrict__ X, int cin,
                                                                     const bf16x8_t *__restrict__ Wp,
                                                                     const float *__restrict__ bias, int cout,
                                                                     const int32_t *__restrict__ nbr,
                                                                     const npvs_counts *__restrict__ counts, int cap,
                                                                     int relu, int out_f32, void *__restrict__ Y) {
  constexpr int ROWS = 16 * MB * RG;
  constexpr int FR = NB * KB;              // weight fragments of one offset (64 lanes x 16 bytes each)
  constexpr int WPT = (FR + RG - 1) / RG;  // fragments each thread stages per offset (some idle)
  constexpr int NS = 4;                    // LDS weight slots: offset o lives in slot o % NS
  // Offset o's weights are loaded into registers at step o - 4, stored to LDS at step o - 2 and
  // read at step o; its rows are gathered at step o - 3.  One barrier ends every step, which
  // orders each slot's store after the last read of the offset it held (step o - 4) and before
  // its first read.
  __shared__ bf16x8_t Ws[NS][FR * 64];
  const int32_t n = counts->n_sites;
  const int ntiles = (n + ROWS - 1) / ROWS;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index, uniform (scalar)
  const int csub = 8 * (lane >> 4);
  for (int j = 0;; ++j) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x, ntiles, j);
    if (tile < 0) break;
    const int row0 = tile * ROWS + wv * 16 * MB;
    const bf16x8_t *W = Wp + opaque_zero();
    int idx[27][MB];
#pragma unroll
    for (int q = 0; q < 27; ++q)
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) idx[q][mb] = nbr_index(nbr, cap, q, row0 + mb * 16 + (lane & 15), n);
    f32x4_t acc[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
    bf16x8_t wreg[2][WPT], bx[4][MB][KB];
    auto wload = [&](int o, bf16x8_t (&w)[WPT]) {
#pragma unroll
      for (int i = 0; i < WPT; ++i)
        if (FR % RG == 0 || tid + i * 64 * RG < FR * 64) w[i] = W[(int64_t)o * FR * 64 + tid + i * 64 * RG];
    };
    auto wstore = [&](int slot, const bf16x8_t (&w)[WPT]) {
#pragma unroll
      for (int i = 0; i < WPT; ++i)
        if (FR % RG == 0 || tid + i * 64 * RG < FR * 64) Ws[slot][tid + i * 64 * RG] = w[i];
    };
    auto gather = [&](int o, bf16x8_t (&b)[MB][KB]) {
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) b[mb][kb] = gather8(X, cin, idx[o][mb], kb * 32 + csub);
    };
    // prologue: offsets 0 and 1 in LDS, 2 and 3 in registers, rows of offsets 0-2
    {
      bf16x8_t w0[WPT], w1[WPT];
      wload(0, w0);
      wload(1, w1);
      wload(2, wreg[0]);
      wload(3, wreg[1]);
      gather(0, bx[0]);
      gather(1, bx[1]);
      gather(2, bx[2]);
      wstore(0, w0);
      wstore(1, w1);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 27; ++k) {
      if (k + 2 < 27) wstore((k + 2) % NS, wreg[k % 2]);  // offset k + 2 (loaded at step k - 2)
      if (k + 4 < 27) wload(k + 4, wreg[k % 2]);
      if (k + 3 < 27) gather(k + 3, bx[(k + 3) % 4]);
      // offsets without any neighbour in this wave gather zeros: no branch around the products
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const bf16x8_t aw = Ws[k % NS][(nb * KB + kb) * 64 + lane];
#pragma unroll
          for (int mb = 0; mb < MB; ++mb)
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw, bx[k % 4][mb][kb], acc[mb][nb], 0, 0, 0);
        }
      __syncthreads();
    }
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        conv_bf16_epilogue<NB>(acc[mb][nb], row0 + mb * 16 + (lane & 15), n, nb * 16 + 4 * (lane >> 4), cout, bias,
                               relu, out_f32, Y);
  }
}

template <int KB, int NB, int MB, int RG>
static void launch_bf16_lds(const void *X, int cin, const void *Wp, const float *bias, int cout, const int32_t *nbr,
                            const npvs_counts *counts, int cap, int relu, int out_f32, void *Y, hipStream_t s) {
  int G = stride_grid(cap, 16 * MB * RG, 4096);
  G = (G + 7) & ~7;
  conv_fwd_bf16_lds_kernel<KB, NB, MB, RG><<<G, 64 * RG, 0, s>>>(
      (const uint16_t *)X, cin, (const bf16x8_t *)Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y);
}

// Tile shapes.  Split kernel (MB, KSPLIT) = (rows per wave / 16, waves sharing the 27 offsets of a
// tile): variant 0 (1, 9), 1 (2, 1), 2 (1, 3), 3 (2, 3), 4 (1, 1), 5 (2, 9).  Shared-weight kernel
// (MB, RG) = (rows per wave / 16, waves per workgroup): 6 (1, 4), 7 (1, 2), 8 (2, 2), 9 (1, 8),
// 10 (2, 4), 11 (2, 8).  Larger row blocks read each staged weight fragment for more rows (less
// weight traffic per row) and suit large batches; small ones keep more waves busy on one frame.
// Weight-stationary kernel (inputs of at most 64 channels): 12 (16-row tiles), 13 (32-row tiles).
// Inputs wider than 64 channels use only the 9-way split (a long unrolled offset loop would not
// fit the registers, nor a double-buffered offset of weights the LDS).
// kDefaultConvVariant is used by npvs_sparse_conv_fwd; the autotuner can pick another per layer.

template <int KB, int NB, int MB, int KSPLIT>
static void launch_bf16(const void *X, int cin, const void *Wp, const float *bias, int cout, const int32_t *nbr,
                        const npvs_counts *counts, int cap, int relu, int out_f32, void *Y, hipStream_t s) {
  const int rows = 16 * MB;
  int G = stride_grid(cap, rows, 4096);
  G = (G + 7) & ~7;
  conv_fwd_bf16_kernel<KB, NB, MB, KSPLIT><<<G, 64 * KSPLIT, 0, s>>>(
      (const uint16_t *)X, cin, (const bf16x8_t *)Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y);
}

template <int KB, int MB, int NBW = 2>
static void launch_bf16_wsta(const void *X, int cin, const void *Wp, const float *bias, int cout, const int32_t *nbr,
                             const npvs_counts *counts, int cap, int relu, int out_f32, void *Y, hipStream_t s) {
  // as many workgroups as fit on the chip at once (9-wave workgroups: two per compute unit with
  // one input chunk, one with two or more chunks or 32-row tiles), spread over the output groups;
  // each walks several row tiles
  const int groups = (cout + 16 * NBW - 1) / (16 * NBW);
  int G = (KB == 1 && MB == 1 && NBW <= 2 ? 512 : 256) / groups;
  G = G < 8 ? 8 : G & ~7;  // a multiple of 8 (one per XCD), rounded down so that all fit at once
  const int most = stride_grid(cap, 16 * MB, 4096);
  if (G > most) G = (most + 7) & ~7;
  conv_fwd_bf16_wsta_kernel<KB, MB, NBW><<<dim3(G, groups), 576, 0, s>>>(
      (const uint16_t *)X, cin, (const bf16x8_t *)Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y);
}

npvs_status dgrad_relu_fused(const uint16_t *dZ, int cin, const void *Wt, int cout, const int32_t *nbr,
                             const npvs_counts *counts, int cap, const uint16_t *M, uint16_t *dZ_below, float *dbp,
                             hipStream_t s) {
  if (cin > 64 || cin % 8 || cout > 64 || cout % 4)
    return fail(NPVS_ERR_UNSUPPORTED, "data gradient with fused ReLU': unsupported channel counts");
  // the grid of the default forward shape (one column group); at most kBwdDbBlocks workgroups,
  // one bias partial row each
  int G = 256;
  const int most = stride_grid(cap, 16, 4096);
  if (G > most) G = (most + 7) & ~7;
  G = G > kBwdDbBlocks ? kBwdDbBlocks : G;
  const bf16x8_t *W = (const bf16x8_t *)Wt;
  if (cin <= 32)
    dgrad_relu_bf16_wsta_kernel<1><<<dim3(G, 1), 576, 0, s>>>(dZ, cin, W, cout, nbr, counts, cap, dZ_below, M, dbp);
  else
    dgrad_relu_bf16_wsta_kernel<2><<<dim3(G, 1), 576, 0, s>>>(dZ, cin, W, cout, nbr, counts, cap, dZ_below, M, dbp);
  return check_hip(hipGetLastError(), "data gradient with fused ReLU'");
}

template <int MB>
static void launch_bf16_wide(const void *X, int cin, const void *Wp, const float *bias, int cout, const int32_t *nbr,
                             const npvs_counts *counts, int cap, int relu, int out_f32, void *Y, hipStream_t s,
                             int KZ, float *part) {
  int G = stride_grid(cap, 16 * MB, 4096);
  G = (G + 7) & ~7;
  const dim3 grid(G, (cout + 63) / 64, part ? KZ : 1);
  conv_fwd_bf16_wide_kernel<MB><<<grid, 576, 0, s>>>((const uint16_t *)X, cin, (const bf16x8_t *)Wp, bias, cout, nbr,
                                                      counts, cap, relu, out_f32, Y, part);
  if (part)
    conv_splitk_finish_kernel<<<stride_grid((int64_t)cap * (cout / 4), 256, 4096), 256, 0, s>>>(
        part, KZ, cap, bias, cout, counts, relu, out_f32, Y);
}

template <int KB, int NB>
static void launch_bf16_variant(int v, const void *X, int cin, const void *Wp, const float *bias, int cout,
                                const int32_t *nbr, const npvs_counts *counts, int cap, int relu, int out_f32, void *Y,
                                hipStream_t s) {
  if constexpr (KB > 2) {
    if (v == 5)
      launch_bf16<KB, NB, 2, 9>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s);
    else
      launch_bf16<KB, NB, 1, 9>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s);
  } else {
    switch (v) {
      case 0: launch_bf16<KB, NB, 1, 9>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s); break;
      case 1: launch_bf16<KB, NB, 2, 1>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s); break;
      case 2: launch_bf16<KB, NB, 1, 3>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s); break;
      case 3: launch_bf16<KB, NB, 2, 3>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s); break;
      case 4: launch_bf16<KB, NB, 1, 1>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s); break;
      case 5: launch_bf16<KB, NB, 2, 9>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s); break;
      case 6: launch_bf16_lds<KB, NB, 1, 4>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s); break;
      case 7: launch_bf16_lds<KB, NB, 1, 2>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s); break;
      case 8: launch_bf16_lds<KB, NB, 2, 2>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s); break;
      case 9: launch_bf16_lds<KB, NB, 1, 8>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s); break;
      case 10: launch_bf16_lds<KB, NB, 2, 4>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s); break;
      default: launch_bf16_lds<KB, NB, 2, 8>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s); break;
    }
  }
}

}  // namespace npvs

using namespace npvs;

extern "C" size_t npvs_packed_weight_bytes(int32_t cin, int32_t cout, int32_t dtype) {
  if (cin < 1 || cout < 1) return 0;
  if (dtype == NPVS_F32) return sizeof(float) * 27 * (size_t)cin * cout;
  if (dtype == NPVS_BF16) {
    size_t a = 27 * (size_t)((cout + 15) / 16) * ((cin + 31) / 32) * 1024;
    size_t b = 27 * (size_t)((cin + 15) / 16) * ((cout + 31) / 32) * 1024;
    return a > b ? a : b;
  }
  return 0;
}

extern "C" npvs_status npvs_pack_weights(const float *W, int32_t cin, int32_t cout, int32_t dtype,
                                        int32_t flip_transpose, void *Wp, void *stream) {
  if (!W || !Wp) return fail(NPVS_ERR_INVALID_ARG, "npvs_pack_weights: null pointer");
  if (cin < 1 || cout < 1) return fail(NPVS_ERR_INVALID_ARG, "npvs_pack_weights: channels must be >= 1");
  hipStream_t s = as_stream(stream);
  if (dtype == NPVS_F32) {
    pack_f32_kernel<<<stride_grid(27LL * cin * cout, 256, 1024), 256, 0, s>>>(W, cin, cout, flip_transpose ? 1 : 0,
                                                                             (float *)Wp);
  } else if (dtype == NPVS_BF16) {
    const int64_t buf = (int64_t)npvs_packed_weight_bytes(cin, cout, dtype) / 2;
    pack_bf16_kernel<<<stride_grid(buf, 256, 1024), 256, 0, s>>>(W, cin, cout, flip_transpose ? 1 : 0, buf,
                                                                  (uint16_t *)Wp);
  } else {
    return fail(NPVS_ERR_INVALID_ARG, "npvs_pack_weights: dtype must be NPVS_F32 or NPVS_BF16");
  }
  return check_hip(hipGetLastError(), "npvs_pack_weights");
}

extern "C" npvs_status npvs_pack_weights_batch(int32_t n, const npvs_pack_desc *descs, int32_t dtype, void *stream) {
  if (n < 0 || n > NPVS_MAX_PACK) return fail(NPVS_ERR_INVALID_ARG, "npvs_pack_weights_batch: n out of range");
  if (n == 0) return NPVS_OK;
  if (!descs) return fail(NPVS_ERR_INVALID_ARG, "npvs_pack_weights_batch: null descriptors");
  if (dtype != NPVS_F32 && dtype != NPVS_BF16)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_pack_weights_batch: dtype must be NPVS_F32 or NPVS_BF16");
  PackBatch PB = {};
  size_t most = 0;
  for (int i = 0; i < n; ++i) {
    const npvs_pack_desc &D = descs[i];
    if (!D.W || !D.Wp) return fail(NPVS_ERR_INVALID_ARG, "npvs_pack_weights_batch: null pointer");
    if (D.cin < 1 || D.cout < 1) return fail(NPVS_ERR_INVALID_ARG, "npvs_pack_weights_batch: channels must be >= 1");
    PB.d[i] = D;
    const size_t e = npvs_packed_weight_bytes(D.cin, D.cout, dtype) / (dtype == NPVS_F32 ? 4 : 2);
    PB.elems[i] = (int64_t)e;
    most = e > most ? e : most;
  }
  dim3 grid(stride_grid((int64_t)most, 256, 256), n);
  pack_batch_kernel<<<grid, 256, 0, as_stream(stream)>>>(PB, dtype);
  return check_hip(hipGetLastError(), "npvs_pack_weights_batch");
}

namespace npvs {
// Dispatch of the BF16 kernel on (ceil(cin/32), ceil(cout/16)); MB = 2 rows blocks per wave,
// offsets split three ways.
// Input-channel split of the general BF16 kernel: 1, or a divisor-friendly count for 1024+ input
// channels (8 chunks of 32 channels per split at least, at most 16 splits).
int splitk_factor(int32_t cin, int32_t cout, int32_t dtype) {
  const int KB = (cin + 31) / 32;
  if (dtype != NPVS_BF16 || KB < 32 || cin % 8 || cout % 8) return 1;
  const int kz = KB / 8;
  return kz > 16 ? 16 : kz;
}

size_t conv_fwd_ws_bytes(int32_t cin, int32_t cout, int32_t cap, int32_t dtype) {
  const int kz = splitk_factor(cin, cout, dtype);
  return kz > 1 ? sizeof(float) * (size_t)kz * cap * cout : 0;
}

npvs_status conv_fwd_dispatch(const void *X, int32_t cin, const void *Wp, const float *bias, int32_t cout,
                              const int32_t *nbr, const npvs_counts *counts, int32_t cap, int32_t dtype, int32_t relu,
                              int32_t out_f32, void *Y, hipStream_t s, int variant, void *ws, size_t ws_bytes) {
  if (dtype == NPVS_F32) {
    const int groups = (cout + 63) / 64;
    int G = stride_grid(cap, kF32Rows, 2048);
    const int most = 8192 / groups;  // workgroups over all output groups, at most about 8192
    if (G > most) G = most;
    G = G < 8 ? 8 : (G + 7) & ~7;
    conv_fwd_f32_kernel<<<dim3(G, groups), 256, 0, s>>>((const float *)X, cin, (const float *)Wp, bias, cout, nbr,
                                                         counts, cap, relu, (float *)Y);
    return check_hip(hipGetLastError(), "npvs_sparse_conv_fwd");
  }
  if (cin % 8 || cout % 8)
    return fail(NPVS_ERR_UNSUPPORTED, "npvs_sparse_conv_fwd: BF16 needs cin % 8 == 0 and cout % 8 == 0");
  const int KB = (cin + 31) / 32, NB = (cout + 15) / 16;
  if (variant == 15) {  // variant 14 with dedicated reducer waves: at most 64 inputs and outputs
    if (KB <= 2 && NB <= 4) {
      int G = 256;
      const int most = stride_grid(cap, 16, 4096);
      if (G > most) G = (most + 7) & ~7;
      if (KB == 1)
        conv_fwd_bf16_wsred_kernel<1><<<dim3(G, 1), 768, 0, s>>>((const uint16_t *)X, cin, (const bf16x8_t *)Wp,
                                                                 bias, cout, nbr, counts, cap, relu, out_f32, Y);
      else
        conv_fwd_bf16_wsred_kernel<2><<<dim3(G, 1), 768, 0, s>>>((const uint16_t *)X, cin, (const bf16x8_t *)Wp,
                                                                 bias, cout, nbr, counts, cap, relu, out_f32, Y);
      return check_hip(hipGetLastError(), "npvs_sparse_conv_fwd");
    }
    variant = 14;
  }
  if (variant == 14 && KB <= 2 && NB <= 4) {  // weight-stationary, all (at most 64) outputs per workgroup
    if (KB == 1) launch_bf16_wsta<1, 1, 4>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s);
    else launch_bf16_wsta<2, 1, 4>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s);
    return check_hip(hipGetLastError(), "npvs_sparse_conv_fwd");
  }
  if (variant == 14) variant = 12;  // more than 64 outputs: 32 per workgroup
  if ((variant == 12 || variant == 13) && KB <= 2) {  // weight-stationary tiles
    if (KB == 1) {
      if (variant == 12) launch_bf16_wsta<1, 1>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s);
      else launch_bf16_wsta<1, 2>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s);
    } else {
      if (variant == 12) launch_bf16_wsta<2, 1>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s);
      else launch_bf16_wsta<2, 2>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s);
    }
    return check_hip(hipGetLastError(), "npvs_sparse_conv_fwd");
  }
#define NPVS_BF16_CASE(kb, nb)                                                                           \
  if (KB == kb && NB == nb) {                                                                            \
    launch_bf16_variant<kb, nb>(variant, X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s); \
    return check_hip(hipGetLastError(), "npvs_sparse_conv_fwd");                                         \
  }
  NPVS_BF16_CASE(1, 1)
  NPVS_BF16_CASE(1, 2)
  NPVS_BF16_CASE(1, 3)
  NPVS_BF16_CASE(1, 4)
  NPVS_BF16_CASE(2, 1)
  NPVS_BF16_CASE(2, 2)
  NPVS_BF16_CASE(2, 3)
  NPVS_BF16_CASE(2, 4)
  NPVS_BF16_CASE(16, 4)
#undef NPVS_BF16_CASE
  // any other shape: up to 64 input channels (e.g. the wide last layer of d = 8 or 16) the
  // weight-stationary kernel, else the general one (variants 5 and 13 pick 32-row tiles)
  if (KB <= 2) {
    const bool wide_rows = variant == 5 || variant == 13;
    if (KB == 1) {
      if (wide_rows) launch_bf16_wsta<1, 2>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s);
      else launch_bf16_wsta<1, 1>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s);
    } else {
      if (wide_rows) launch_bf16_wsta<2, 2>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s);
      else launch_bf16_wsta<2, 1>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s);
    }
    return check_hip(hipGetLastError(), "npvs_sparse_conv_fwd");
  }
  // 65 to 160 input channels (the U-Net decoder: 160 -> 96, 96 -> 96, 96 -> 64): the
  // weight-stationary kernel, since the general kernel re-reads every offset's weights for each
  // 16-row tile; 3 input chunks with two output blocks per workgroup (168 VGPRs), 4 or 5 with one
  if (KB <= 5 && variant != 5) {
    if (KB == 3) launch_bf16_wsta<3, 1>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s);
    else if (KB == 4) launch_bf16_wsta<4, 1, 1>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s);
    else launch_bf16_wsta<5, 1, 1>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s);
    return check_hip(hipGetLastError(), "npvs_sparse_conv_fwd");
  }
  // wide inputs: split the channel chunks over workgroups when the caller gave a workspace
  const int KZ = splitk_factor(cin, cout, dtype);
  float *part = (KZ > 1 && ws && ws_bytes >= conv_fwd_ws_bytes(cin, cout, cap, dtype)) ? (float *)ws : nullptr;
  if (variant == 5 || variant == 13)
    launch_bf16_wide<2>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s, KZ, part);
  else
    launch_bf16_wide<1>(X, cin, Wp, bias, cout, nbr, counts, cap, relu, out_f32, Y, s, KZ, part);
  return check_hip(hipGetLastError(), "npvs_sparse_conv_fwd");
}
}  // namespace npvs

extern "C" npvs_status npvs_conv_fwd_workspace_size(int32_t cin, int32_t cout, int32_t cap_sites, int32_t dtype,
                                                    size_t *bytes) {
  if (!bytes || cin < 1 || cout < 1 || cap_sites < 1)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_conv_fwd_workspace_size: bad arguments");
  *bytes = conv_fwd_ws_bytes(cin, cout, cap_sites, dtype);
  return NPVS_OK;
}

extern "C" npvs_status npvs_sparse_conv_fwd(const void *X, int32_t cin, const void *Wp, const float *bias,
                                           int32_t cout, const int32_t *nbr, const npvs_counts *counts,
                                           int32_t cap_sites, int32_t dtype, int32_t relu, int32_t out_f32,
                                           int32_t variant, void *Y, void *ws, size_t ws_bytes, void *stream) {
  if (!X || !Wp || !nbr || !counts || !Y) return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_fwd: null pointer");
  if (cin < 1 || cout < 1 || cap_sites < 1) return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_fwd: bad sizes");
  if (dtype != NPVS_F32 && dtype != NPVS_BF16)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_fwd: dtype must be NPVS_F32 or NPVS_BF16");
  if (X == Y) return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_fwd: X and Y must not alias");
  if (variant == -1) variant = kDefaultConvVariant;
  if (variant < 0 || variant >= NPVS_CONV_VARIANTS)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_fwd: variant out of range");
  const size_t need = conv_fwd_ws_bytes(cin, cout, cap_sites, dtype);
  if (ws && ws_bytes < need) return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_fwd: workspace too small");
  return conv_fwd_dispatch(X, cin, Wp, bias, cout, nbr, counts, cap_sites, dtype, relu, out_f32, Y,
                           as_stream(stream), variant, ws, ws ? ws_bytes : 0);
}
