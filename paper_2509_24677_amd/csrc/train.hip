// Training loss over the froxels of each grid's active blocks and Adam.
//   Sec. 3.3: repulsive visibility loss L_rv = L_attr + L_rep with L_rep = FP/GTP; the
//   attraction term is read as 1 - TP/GTP = FN/GTP (printed literally it would reward missed
//   geometry); combined as L = lambda * T + (1 - lambda) * L_rv, with T = BCE in place of Dice
//   (the weight alpha of the Dice term is unstated) or T = the weighted Dice term
//   1 - 2 TP / (2 TP + alpha FN + (1 - alpha) FP), alpha on the missed ground truth.
//   Soft counts use p = sigmoid(l): TP = sum y p, FN = sum y (1-p), FP = sum (1-y) p, GTP = sum y.
// Three launches: per-(grid, slice) compensated partial sums, one workgroup that finishes the
// sums in a fixed order and writes the statistics and gradient coefficients, and the
// elementwise gradient dL/dl = c0_b (p - y) + p (1 - p) (y ? cy_b : cn_b).
#include <cmath>

#include "bwd_layout.hpp"

namespace npvs {

struct Comp {
  float s, c;
  __device__ __forceinline__ void add(float y) {
    float t = s + y;
    c += (__builtin_fabsf(s) >= __builtin_fabsf(y)) ? (s - t) + y : (y - t) + s;
    s = t;
  }
  __device__ __forceinline__ void merge(const Comp &o) {
    add(o.s);
    c += o.c;
  }
};

constexpr int kLossSlices = 512;
constexpr int kLossQ = 5;  // BCE sum, TP, FN, FP, GTP
constexpr int kLossBatch = 8;  // elements per thread loaded together

__device__ __forceinline__ float sigmoidf_(float l) { return 1.0f / (1.0f + expf(-l)); }

// grid (kLossSlices, n_grids), 256 threads
__global__ __launch_bounds__(256) void loss_partial_kernel(const float *__restrict__ logits,
                                                            const uint8_t *__restrict__ labels, int C,
                                                            const int32_t *__restrict__ grid_rows,
                                                            float *__restrict__ part, uint32_t *__restrict__ ticket) {
  __shared__ Comp red[kLossQ][256];
  const int b = blockIdx.y, s = blockIdx.x, tid = threadIdx.x;
  if (b == 0 && s == 0 && tid == 0) *ticket = 0u;  // for the finishing kernel that follows
  const int64_t e0 = (int64_t)grid_rows[b] * C, e1 = (int64_t)grid_rows[b + 1] * C;
  const int64_t m = e1 - e0;
  const int64_t a0 = e0 + m * s / kLossSlices, a1 = e0 + m * (s + 1) / kLossSlices;
  Comp q[kLossQ];
#pragma unroll
  for (int i = 0; i < kLossQ; ++i) q[i] = Comp{0.0f, 0.0f};
  // kLossBatch elements per thread are loaded before any is used (a value used right after its
  // load would make each element wait for memory in turn); they are added in the same order.
  for (int64_t eb = a0 + tid; eb < a1; eb += 256 * kLossBatch) {
    float lv[kLossBatch];
    uint8_t yv[kLossBatch];
#pragma unroll
    for (int u = 0; u < kLossBatch; ++u) {
      const int64_t e = eb + 256 * u;
      lv[u] = e < a1 ? logits[e] : 0.0f;
      yv[u] = e < a1 ? labels[e] : 0;
    }
#pragma unroll
    for (int u = 0; u < kLossBatch; ++u) {
      if (eb + 256 * u >= a1) break;
      const float l = lv[u];
      const float y = yv[u] ? 1.0f : 0.0f;
      const float p = sigmoidf_(l);
      const float sp = fmaxf(l, 0.0f) + log1pf(expf(-__builtin_fabsf(l)));
      q[0].add(sp - y * l);
      q[1].add(y * p);
      q[2].add(y * (1.0f - p));
      q[3].add((1.0f - y) * p);
      q[4].add(y);
    }
  }
#pragma unroll
  for (int i = 0; i < kLossQ; ++i) red[i][tid] = q[i];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {  // fixed-shape tree
    if (tid < w)
#pragma unroll
      for (int i = 0; i < kLossQ; ++i) red[i][tid].merge(red[i][tid + w]);
    __syncthreads();
  }
  if (tid < kLossQ) part[((int64_t)b * kLossSlices + s) * kLossQ + tid] = red[tid][0].s + red[tid][0].c;
}

// One workgroup per grid: thread s takes slice s's partial sums, a fixed-shape tree adds them,
// thread 0 writes the grid's statistics and gradient coefficients coef[b] = {c0_b, cy_b, cn_b}.
// One block per grid finishes that grid's sums (fixed tree); the last block to finish, found with
// a ticket taken after a device-scope fence, writes the batch mean (grids in order).
__global__ __launch_bounds__(kLossSlices) void loss_final_kernel(const float *__restrict__ part,
                                                                 const int32_t *__restrict__ grid_rows, int n_grids,
                                                                 int C, float lambda, int term, float alpha,
                                                                 float *__restrict__ stats, float *__restrict__ coef,
                                                                 uint32_t *__restrict__ ticket) {
  __shared__ Comp red[kLossQ][kLossSlices];
  __shared__ bool last;
  const int b = blockIdx.x, s = threadIdx.x;
#pragma unroll
  for (int i = 0; i < kLossQ; ++i) red[i][s] = Comp{part[((int64_t)b * kLossSlices + s) * kLossQ + i], 0.0f};
  __syncthreads();
  for (int w = kLossSlices / 2; w > 0; w >>= 1) {
    if (s < w)
#pragma unroll
      for (int i = 0; i < kLossQ; ++i) red[i][s].merge(red[i][s + w]);
    __syncthreads();
  }
  if (s == 0) {
    const float m = (float)((int64_t)(grid_rows[b + 1] - grid_rows[b]) * C);
    const float bce_sum = red[0][0].s + red[0][0].c, tp = red[1][0].s + red[1][0].c, fn = red[2][0].s + red[2][0].c,
                fp = red[3][0].s + red[3][0].c, gtp = red[4][0].s + red[4][0].c;
    const float g = gtp > 1.0f ? gtp : 1.0f;
    const float lrv = fn / g + fp / g;
    const float crv = (1.0f - lambda) / (g * n_grids);  // L_rv: d/dp = (1 - 2y) / GTP
    float first, c0, cy, cn;
    if (term == NPVS_LOSS_DICE) {
      // quotient rule on 1 - 2TP/den: d(2TP)/dp = 2y, d(den)/dp = 2y - alpha y + (1 - alpha)(1 - y)
      const float den = 2.0f * tp + alpha * fn + (1.0f - alpha) * fp;
      const float kd = lambda / n_grids;
      first = den > 0.0f ? 1.0f - 2.0f * tp / den : 0.0f;
      c0 = 0.0f;
      cy = (den > 0.0f ? kd * (-2.0f / den + 2.0f * tp * (2.0f - alpha) / (den * den)) : 0.0f) - crv;
      cn = (den > 0.0f ? kd * (2.0f * tp * (1.0f - alpha) / (den * den)) : 0.0f) + crv;
    } else {
      first = m > 0.0f ? bce_sum / m : 0.0f;
      c0 = m > 0.0f ? lambda / (m * n_grids) : 0.0f;
      cy = -crv;
      cn = crv;
    }
    const float v[8] = {lambda * first + (1.0f - lambda) * lrv, first, lrv, tp, fn, fp, gtp, m};
    for (int i = 0; i < 8; ++i) stats[b * 8 + i] = v[i];
    coef[3 * b] = c0;
    coef[3 * b + 1] = cy;
    coef[3 * b + 2] = cn;
    __threadfence();  // this grid's stats are visible before its ticket
    last = atomicAdd(ticket, 1u) == (uint32_t)(n_grids - 1);
  }
  __syncthreads();
  if (last && s < 8) {
    __threadfence();  // every grid's stats are visible to the last block
    float t = 0.0f;
    for (int gb = 0; gb < n_grids; ++gb) t += __builtin_nontemporal_load(stats + gb * 8 + s);
    stats[n_grids * 8 + s] = t / n_grids;
  }
}

// dL/dl of one element of grid b (both gradient kernels evaluate it with this one function, with
// no multiply-add contraction, so that both round every operation the same way)
__device__ __forceinline__ float loss_grad_value(float l, uint8_t lab, const float *__restrict__ coef, int b) {
#pragma clang fp contract(off)
  const float y = lab ? 1.0f : 0.0f;
  const float p = sigmoidf_(l);
  return coef[3 * b] * (p - y) + p * (1.0f - p) * (lab ? coef[3 * b + 1] : coef[3 * b + 2]);
}

__global__ __launch_bounds__(256) void loss_grad_kernel(const float *__restrict__ logits,
                                                         const uint8_t *__restrict__ labels, int C,
                                                         const int32_t *__restrict__ grid_rows, int n_grids,
                                                         const npvs_counts *__restrict__ counts,
                                                         const float *__restrict__ coef, float *__restrict__ dl) {
  const int64_t total = (int64_t)counts->n_sites * C;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = (int32_t)(e / C);
    int b = 0;
    while (b + 1 < n_grids && r >= grid_rows[b + 1]) ++b;
    dl[e] = loss_grad_value(logits[e], labels[e], coef, b);
  }
}

// The gradient formed as the top layer's dZ (no ReLU on the logits): bf16 dZ16 [cap][C], the bias
// partial table dbpart[kBwdDbBlocks][C] and, when dl is given, the float32 gradient too.  The
// blocks, the row ranges, the four columns per thread and the fixed-order sums are those of the
// backward's own dZ pass (backward.hip) on that gradient, so both form the same values.  grid
// (kBwdDbBlocks, ceil(C / 64)), 256 threads; C % 4 == 0 and 16-byte aligned rows.
__global__ __launch_bounds__(256) void loss_dz_kernel(const float *__restrict__ logits,
                                                       const uint8_t *__restrict__ labels, int C,
                                                       const int32_t *__restrict__ grid_rows, int n_grids,
                                                       const npvs_counts *__restrict__ counts,
                                                       const float *__restrict__ coef, float *__restrict__ dl,
                                                       uint16_t *__restrict__ dZ16, float *__restrict__ dbpart) {
  __shared__ float red[256 * 4];
  const int64_t n = counts->n_sites;
  const int64_t r0 = n * blockIdx.x / gridDim.x, r1 = n * (blockIdx.x + 1) / gridDim.x;
  const int c0 = 64 * blockIdx.y, Cw = C - c0 < 64 ? C - c0 : 64;
  const int TPR = Cw / 4, RG = 256 / TPR;
  const int cg = threadIdx.x % TPR, rg = threadIdx.x / TPR;
  Comp a[4] = {{0.0f, 0.0f}, {0.0f, 0.0f}, {0.0f, 0.0f}, {0.0f, 0.0f}};
  if (rg < RG) {
    for (int64_t r = r0 + rg; r < r1; r += RG) {
      int b = 0;
      while (b + 1 < n_grids && r >= grid_rows[b + 1]) ++b;
      const int64_t e = r * C + c0 + 4 * cg;
      const float4 lv = *reinterpret_cast<const float4 *>(logits + e);
      const uint32_t yv = *reinterpret_cast<const uint32_t *>(labels + e);
      float g[4] = {loss_grad_value(lv.x, (uint8_t)yv, coef, b), loss_grad_value(lv.y, (uint8_t)(yv >> 8), coef, b),
                    loss_grad_value(lv.z, (uint8_t)(yv >> 16), coef, b),
                    loss_grad_value(lv.w, (uint8_t)(yv >> 24), coef, b)};
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i].add(g[i]);
      if (dl) *reinterpret_cast<float4 *>(dl + e) = make_float4(g[0], g[1], g[2], g[3]);
      uint2 h;
      h.x = (uint32_t)f32_to_bf16(g[0]) | ((uint32_t)f32_to_bf16(g[1]) << 16);
      h.y = (uint32_t)f32_to_bf16(g[2]) | ((uint32_t)f32_to_bf16(g[3]) << 16);
      *reinterpret_cast<uint2 *>(dZ16 + e) = h;
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) red[threadIdx.x * 4 + i] = a[i].s + a[i].c;
  __syncthreads();
  if (threadIdx.x < Cw) {
    const int c = threadIdx.x, g0 = c / 4, comp = c % 4;
    Comp t{0.0f, 0.0f};
    for (int g = 0; g < RG; ++g) t.add(red[(g * TPR + g0) * 4 + comp]);
    dbpart[(int64_t)blockIdx.x * C + c0 + c] = t.s + t.c;
  }
}

// Adam over the flat parameter buffer with the updated weights written straight into their
// packed forms (the forward packing and the flipped-transpose packing of the data gradient), so
// no separate packing pass follows the optimizer step.  Layer l's weight W[27][cin][cout] sits at
// flat offset off; its entry (k, c, o) is P[k][c][o] of the forward packing and P'[26-k][o][c]
// of the flipped one (CI x CO = cout x cin).  BF16 packing: fragment entry
// ((k NB + o / 16) KB + c / 32) 512 + (o % 16 + 16 ((c % 32) / 8)) 8 + c % 8, NB = ceil(CO / 16),
// KB = ceil(CI / 32), rounded to nearest even; FP32: [k][c][o].  Padding entries keep the zeros
// of the first packing.
struct AdamPack {
  int32_t n;
  npvs_adam_pack_desc L[NPVS_MAX_ADAM_PACK];
};

__device__ __forceinline__ int64_t packed_index(int k, int c, int o, int CI, int CO, int dtype) {
  if (dtype == NPVS_F32) return ((int64_t)k * CI + c) * CO + o;
  const int KB = (CI + 31) / 32, NB = (CO + 15) / 16;
  return (((int64_t)k * NB + o / 16) * KB + c / 32) * 512 + ((o & 15) + 16 * ((c & 31) >> 3)) * 8 + (c & 7);
}

__device__ __forceinline__ void store_packed(void *P, int64_t e, float w, int dtype) {
  if (dtype == NPVS_F32)
    static_cast<float *>(P)[e] = w;
  else
    static_cast<uint16_t *>(P)[e] = f32_to_bf16(w);
}

__global__ __launch_bounds__(256) void adam_pack_kernel(float *__restrict__ p, const float *__restrict__ g,
                                                         float *__restrict__ m, float *__restrict__ v, int64_t n,
                                                         float lr, float b1, float b2, float eps, float wd,
                                                         const npvs_adam_step *__restrict__ coef, AdamPack AP,
                                                         int dtype) {
  const float c1 = coef->c1, c2 = coef->c2;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i] + wd * p[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float w = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = w;
    for (int l = 0; l < AP.n; ++l) {
      const npvs_adam_pack_desc &D = AP.L[l];
      const int64_t e64 = i - D.off;
      if (e64 < 0 || e64 >= 27LL * D.cin * D.cout) continue;
      // 32-bit index arithmetic (27 cin cout < 2^31, checked by the host): a 64-bit division
      // is a long instruction sequence on the GPU
      const uint32_t e = (uint32_t)e64, co = (uint32_t)D.cout, ci = (uint32_t)D.cin;
      const uint32_t eo = e / co;
      const int o = (int)(e - eo * co), c = (int)(eo % ci), k = (int)(eo / ci);
      store_packed(D.Wp, packed_index(k, c, o, D.cin, D.cout, dtype), w, dtype);
      store_packed(D.Wt, packed_index(26 - k, o, c, D.cout, D.cin, dtype), w, dtype);
      break;
    }
  }
}

__global__ void adam_step_kernel(npvs_adam_step *st, float b1, float b2) {
  const int64_t t = st->t + 1;
  st->t = t;
  st->c1 = 1.0f - (float)pow((double)b1, (double)t);
  st->c2 = 1.0f - (float)pow((double)b2, (double)t);
}

}  // namespace npvs

using namespace npvs;

extern "C" npvs_status npvs_loss_workspace_size(int32_t n_grids, size_t *bytes) {
  if (!bytes || n_grids < 1 || n_grids > NPVS_MAX_GRIDS)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_loss_workspace_size: bad arguments");
  *bytes = sizeof(float) * ((size_t)n_grids * kLossSlices * kLossQ + 3 * (size_t)n_grids) + 256;
  return NPVS_OK;
}

extern "C" npvs_status npvs_loss(const float *logits, const uint8_t *labels, int32_t C, const int32_t *grid_rows,
                                int32_t n_grids, const npvs_counts *counts, int32_t cap_sites, float lambda,
                                int32_t term, float alpha, float *stats, float *dlogits, void *dz_ws,
                                size_t dz_ws_bytes, int32_t dz_cin, void *ws, size_t ws_bytes, void *stream) {
  if (!logits || !labels || !grid_rows || !counts || !stats || !ws)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_loss: null pointer");
  if (C < 1 || n_grids < 1 || n_grids > NPVS_MAX_GRIDS || cap_sites < 1)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_loss: bad sizes");
  size_t need;
  npvs_loss_workspace_size(n_grids, &need);
  if (ws_bytes < need) return fail(NPVS_ERR_INVALID_ARG, "npvs_loss: workspace too small");
  float *part = static_cast<float *>(ws);
  if (term != NPVS_LOSS_BCE && term != NPVS_LOSS_DICE)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_loss: term must be NPVS_LOSS_BCE or NPVS_LOSS_DICE");
  float *coef = part + (size_t)n_grids * kLossSlices * kLossQ;
  uint32_t *ticket = reinterpret_cast<uint32_t *>(coef + 3 * (size_t)n_grids);
  size_t o_dz = 0, o_db = 0;
  if (dz_ws) {
    size_t need_dz;
    if (C % 8 || dz_cin < 1 || dz_cin % 8)
      return fail(NPVS_ERR_UNSUPPORTED, "npvs_loss: dZ into a backward workspace needs C and dz_cin multiples of 8");
    if ((reinterpret_cast<uintptr_t>(logits) & 15) || (reinterpret_cast<uintptr_t>(labels) & 3) ||
        (dlogits && (reinterpret_cast<uintptr_t>(dlogits) & 15)))
      return fail(NPVS_ERR_UNSUPPORTED, "npvs_loss: dZ into a backward workspace needs aligned rows");
    bwd_ws_dz_parts(dz_cin, C, cap_sites, &o_dz, &o_db, &need_dz);
    if (dz_ws_bytes < need_dz) return fail(NPVS_ERR_INVALID_ARG, "npvs_loss: dZ workspace too small");
  }
  hipStream_t s = as_stream(stream);
  loss_partial_kernel<<<dim3(kLossSlices, n_grids), 256, 0, s>>>(logits, labels, C, grid_rows, part, ticket);
  loss_final_kernel<<<n_grids, kLossSlices, 0, s>>>(part, grid_rows, n_grids, C, lambda, term, alpha, stats, coef,
                                                    ticket);
  if (dz_ws) {
    char *w = static_cast<char *>(dz_ws);
    loss_dz_kernel<<<dim3(kBwdDbBlocks, (C + 63) / 64), 256, 0, s>>>(
        logits, labels, C, grid_rows, n_grids, counts, coef, dlogits, reinterpret_cast<uint16_t *>(w + o_dz),
        reinterpret_cast<float *>(w + o_db));
  } else if (dlogits) {
    loss_grad_kernel<<<stride_grid((int64_t)cap_sites * C, 256, 4096), 256, 0, s>>>(logits, labels, C, grid_rows,
                                                                                   n_grids, counts, coef, dlogits);
  }
  return check_hip(hipGetLastError(), "npvs_loss");
}

extern "C" npvs_status npvs_adam(float *p, const float *g, float *m, float *v, int64_t n, npvs_adam_step *step,
                                float lr, float beta1, float beta2, float eps, float weight_decay, int32_t n_layers,
                                const npvs_adam_pack_desc *layers, int32_t dtype, void *stream) {
  if (!p || !g || !m || !v || !step || n < 0 || (n_layers && !layers))
    return fail(NPVS_ERR_INVALID_ARG, "npvs_adam: bad arguments");
  if (n_layers < 0 || n_layers > NPVS_MAX_ADAM_PACK)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_adam: 0 to NPVS_MAX_ADAM_PACK layers");
  if (dtype != NPVS_F32 && dtype != NPVS_BF16)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_adam: dtype must be NPVS_F32 or NPVS_BF16");
  AdamPack AP = {};
  AP.n = n_layers;
  for (int l = 0; l < n_layers; ++l) {
    const npvs_adam_pack_desc &D = layers[l];
    if (!D.Wp || !D.Wt || D.cin < 1 || D.cout < 1 || D.off < 0 || D.off + 27LL * D.cin * D.cout > n)
      return fail(NPVS_ERR_INVALID_ARG, "npvs_adam: layer outside the parameter buffer");
    if (27LL * D.cin * D.cout > 0x7fffffffLL)
      return fail(NPVS_ERR_UNSUPPORTED, "npvs_adam: a layer of 2^31 or more weights");
    for (int q = 0; q < l; ++q) {
      const npvs_adam_pack_desc &E = layers[q];
      if (D.off < E.off + 27LL * E.cin * E.cout && E.off < D.off + 27LL * D.cin * D.cout)
        return fail(NPVS_ERR_INVALID_ARG, "npvs_adam: overlapping layers");
    }
    AP.L[l] = D;
  }
  hipStream_t s = as_stream(stream);
  adam_step_kernel<<<1, 1, 0, s>>>(step, beta1, beta2);
  if (n > 0)
    adam_pack_kernel<<<stride_grid(n, 256, 2048), 256, 0, s>>>(p, g, m, v, n, lr, beta1, beta2, eps, weight_decay,
                                                               step, AP, dtype);
  return check_hip(hipGetLastError(), "npvs_adam");
}
