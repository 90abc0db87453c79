// Backward of a submanifold sparse convolution layer (chain rule on the forward definition).
//   dZ = dY * [Y > 0] (ReLU'(0) = 0) or dY;
//   dX = conv(dZ, W'), W'_k = (W_{26-k})^T: the rulebook is symmetric (R_{26-k} is R_k with the
//        roles of input and output swapped), so the data gradient is a forward convolution;
//   dW_k = sum_{(i,r) in R_k} X[i]^T dZ[r]: per-offset reduced outer products over the CSR
//        pair list, cut into a fixed number of slices per offset, reduced in a fixed order;
//   db = sum_r dZ[r].
// Every float32 reduction adds short plain partial sums into a Neumaier-compensated total, and
// all reduction orders are fixed, so gradients are bit-identical run to run.
#include "npvs_common.hpp"

namespace npvs {

npvs_status conv_fwd_dispatch(const void *X, int32_t cin, const void *Wp, const float *bias, int32_t cout,
                              const int32_t *nbr, const npvs_counts *counts, int32_t cap, int32_t dtype, int32_t relu,
                              int32_t out_f32, void *Y, hipStream_t s, int variant);

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

// dZ in float32 (for wgrad/db) and, for the BF16 path, a bfloat16 copy (dgrad input).
template <typename T>
__global__ __launch_bounds__(256) void relu_grad_kernel(const T *__restrict__ Y, const float *__restrict__ dY,
                                                         const npvs_counts *__restrict__ counts, int C, int relu,
                                                         float *__restrict__ dZ32, uint16_t *__restrict__ dZ16) {
  const int64_t total = (int64_t)counts->n_sites * C;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    float g = dY[e];
    if (relu && !(load_as_f32(Y, e) > 0.0f)) g = 0.0f;
    dZ32[e] = g;
    if (dZ16) dZ16[e] = f32_to_bf16(g);
  }
}

constexpr int kWgSlices = 16;  // slices of each offset's pair list
constexpr int kWgPairs = 32;   // pairs staged per step
constexpr int kWgEPT = 16;     // dW entries per thread per pass

// grid (kWgSlices, 27), 256 threads.  Partial dW of offset k over slice s of its pairs.
template <typename T>
__global__ __launch_bounds__(256) void wgrad_partial_kernel(const T *__restrict__ X, int cin,
                                                             const float *__restrict__ dZ, int cout,
                                                             const int32_t *__restrict__ rb_off,
                                                             const int32_t *__restrict__ pairs,
                                                             float *__restrict__ part) {
  __shared__ float Xs[kWgPairs][65];
  __shared__ float Gs[kWgPairs][64];
  __shared__ int in_s[kWgPairs], out_s[kWgPairs];
  const int k = blockIdx.y, s = blockIdx.x, tid = threadIdx.x;
  const int64_t pk0 = rb_off[k], pk = (int64_t)rb_off[k + 1] - pk0;
  const int64_t p0 = pk0 + pk * s / kWgSlices, p1 = pk0 + pk * (s + 1) / kWgSlices;
  const int E = cin * cout;
  const int cw = (256 * kWgEPT) / cout < 64 ? (256 * kWgEPT) / cout : 64;  // channels of X per pass
  for (int cbase = 0; cbase < cin; cbase += cw) {
    const int cn = cin - cbase < cw ? cin - cbase : cw;
    const int e_pass = cn * cout;
    Comp acc[kWgEPT];
#pragma unroll
    for (int j = 0; j < kWgEPT; ++j) acc[j] = Comp{0.0f, 0.0f};
    for (int64_t pb = p0; pb < p1; pb += kWgPairs) {
      const int m = p1 - pb < kWgPairs ? (int)(p1 - pb) : kWgPairs;
      __syncthreads();
      if (tid < kWgPairs) {
        in_s[tid] = tid < m ? pairs[2 * (pb + tid)] : -1;
        out_s[tid] = tid < m ? pairs[2 * (pb + tid) + 1] : -1;
      }
      __syncthreads();
      for (int e = tid; e < kWgPairs * 64; e += 256) {
        int p = e >> 6, c = e & 63;
        Xs[p][c] = (p < m && c < cn) ? load_as_f32(X, (int64_t)in_s[p] * cin + cbase + c) : 0.0f;
        Gs[p][c] = (p < m && c < cout) ? dZ[(int64_t)out_s[p] * cout + c] : 0.0f;
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < kWgEPT; ++j) {
        const int e = tid + 256 * j;
        if (e < e_pass) {
          const int c = e / cout, o = e % cout;
          float t = 0.0f;
          for (int p = 0; p < m; ++p) t = fmaf(Xs[p][c], Gs[p][o], t);
          acc[j].add(t);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kWgEPT; ++j) {
      const int e = tid + 256 * j;
      if (e < e_pass) {
        const int c = e / cout, o = e % cout;
        part[((int64_t)(k * kWgSlices + s) * cin + cbase + c) * cout + o] = acc[j].value();
      }
    }
  }
  (void)E;
}

constexpr int kDbSlices = 64;

// grid kDbSlices: column sums of dZ over a slice of rows.
__global__ __launch_bounds__(256) void db_partial_kernel(const float *__restrict__ dZ, int cout,
                                                          const npvs_counts *__restrict__ counts,
                                                          float *__restrict__ part) {
  const int64_t n = counts->n_sites;
  const int64_t r0 = n * blockIdx.x / kDbSlices, r1 = n * (blockIdx.x + 1) / kDbSlices;
  for (int o = threadIdx.x; o < cout; o += blockDim.x) {
    Comp a{0.0f, 0.0f};
    for (int64_t r = r0; r < r1; r += 32) {
      float t = 0.0f;
      int64_t re = r + 32 < r1 ? r + 32 : r1;
      for (int64_t q = r; q < re; ++q) t += dZ[q * cout + o];
      a.add(t);
    }
    part[blockIdx.x * cout + o] = a.value();
  }
}

__global__ __launch_bounds__(256) void grad_reduce_kernel(const float *__restrict__ wpart,
                                                           const float *__restrict__ dbpart, int cin, int cout,
                                                           float *__restrict__ dW, float *__restrict__ db) {
  const int64_t E = (int64_t)cin * cout;
  const int64_t total = 27 * E + cout;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    Comp a{0.0f, 0.0f};
    if (e < 27 * E) {
      int64_t k = e / E, ce = e % E;
      for (int s = 0; s < kWgSlices; ++s) a.add(wpart[(k * kWgSlices + s) * E + ce]);
      dW[e] = a.value();
    } else {
      int o = (int)(e - 27 * E);
      for (int s = 0; s < kDbSlices; ++s) a.add(dbpart[s * cout + o]);
      db[o] = a.value();
    }
  }
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static void bwd_ws_layout(int32_t cin, int32_t cout, int32_t cap, int32_t dtype, size_t *o_dz32, size_t *o_dz16,
                          size_t *o_wp, size_t *o_dbp, size_t *bytes) {
  size_t o = 0;
  *o_dz32 = o;
  o += align256(sizeof(float) * (size_t)cap * cout);
  *o_dz16 = o;
  if (dtype == NPVS_BF16) o += align256(sizeof(uint16_t) * (size_t)cap * cout);
  *o_wp = o;
  o += align256(sizeof(float) * 27 * kWgSlices * (size_t)cin * cout);
  *o_dbp = o;
  o += align256(sizeof(float) * kDbSlices * (size_t)cout);
  *bytes = o;
}

}  // namespace npvs

using namespace npvs;

extern "C" npvs_status npvs_conv_bwd_workspace_size(int32_t cin, int32_t cout, int32_t cap_sites, int32_t dtype,
                                                    size_t *bytes) {
  if (!bytes || cin < 1 || cout < 1 || cap_sites < 1)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_conv_bwd_workspace_size: bad arguments");
  size_t a, b, c, d;
  bwd_ws_layout(cin, cout, cap_sites, dtype, &a, &b, &c, &d, bytes);
  return NPVS_OK;
}

extern "C" npvs_status npvs_sparse_conv_bwd(const void *X, int32_t cin, const void *Wt, int32_t cout, const void *Y,
                                           const float *dY, const int32_t *nbr, const int32_t *rb_off,
                                           const int32_t *rb_pairs, const npvs_counts *counts, int32_t cap_sites,
                                           int32_t dtype, int32_t relu, float *dX, float *dW, float *db, void *ws,
                                           size_t ws_bytes, void *stream) {
  if (!X || !dY || !nbr || !rb_off || !rb_pairs || !counts || !dW || !db || !ws || (relu && !Y) || (dX && !Wt))
    return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_bwd: null pointer");
  if (cin < 1 || cout < 1 || cap_sites < 1) return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_bwd: bad sizes");
  if (cout > 64) return fail(NPVS_ERR_UNSUPPORTED, "npvs_sparse_conv_bwd: cout > 64");
  if (dtype != NPVS_F32 && dtype != NPVS_BF16)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_bwd: dtype must be NPVS_F32 or NPVS_BF16");
  size_t o32, o16, owp, odb, need;
  bwd_ws_layout(cin, cout, cap_sites, dtype, &o32, &o16, &owp, &odb, &need);
  if (ws_bytes < need) return fail(NPVS_ERR_INVALID_ARG, "npvs_sparse_conv_bwd: workspace too small");
  char *w = static_cast<char *>(ws);
  float *dZ32 = reinterpret_cast<float *>(w + o32);
  uint16_t *dZ16 = dtype == NPVS_BF16 ? reinterpret_cast<uint16_t *>(w + o16) : nullptr;
  float *wpart = reinterpret_cast<float *>(w + owp);
  float *dbpart = reinterpret_cast<float *>(w + odb);
  hipStream_t s = as_stream(stream);
  const int g_el = stride_grid((int64_t)cap_sites * cout, 256, 4096);
  if (dtype == NPVS_F32)
    relu_grad_kernel<float><<<g_el, 256, 0, s>>>((const float *)Y, dY, counts, cout, relu, dZ32, nullptr);
  else
    relu_grad_kernel<uint16_t><<<g_el, 256, 0, s>>>((const uint16_t *)Y, dY, counts, cout, relu, dZ32, dZ16);
  npvs_status st = check_hip(hipGetLastError(), "npvs_sparse_conv_bwd");
  if (st != NPVS_OK) return st;
  if (dX) {
    st = conv_fwd_dispatch(dtype == NPVS_F32 ? (const void *)dZ32 : (const void *)dZ16, cout, Wt, nullptr, cin, nbr,
                           counts, cap_sites, dtype, 0, 1, dX, s, 0);
    if (st != NPVS_OK) return st;
  }
  dim3 gw(kWgSlices, 27);
  if (dtype == NPVS_F32)
    wgrad_partial_kernel<float><<<gw, 256, 0, s>>>((const float *)X, cin, dZ32, cout, rb_off, rb_pairs, wpart);
  else
    wgrad_partial_kernel<uint16_t><<<gw, 256, 0, s>>>((const uint16_t *)X, cin, dZ32, cout, rb_off, rb_pairs, wpart);
  db_partial_kernel<<<kDbSlices, 256, 0, s>>>(dZ32, cout, counts, dbpart);
  grad_reduce_kernel<<<stride_grid(27LL * cin * cout + cout, 256, 2048), 256, 0, s>>>(wpart, dbpart, cin, cout, dW, db);
  return check_hip(hipGetLastError(), "npvs_sparse_conv_bwd");
}
