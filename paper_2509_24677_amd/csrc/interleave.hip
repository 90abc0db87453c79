// Interleave g_d, its inverse, the sparse interleave onto active sites and the fused
// de-interleave + threshold (Sec. 3.1, Sec. 3.3).  All are pure index permutations bounded by
// HBM bandwidth: each thread moves one contiguous run so that either the loads or the stores
// of a wave are contiguous.
#include "npvs_common.hpp"

namespace npvs {

// Dense g_d through LDS (d >= 2; g_1 is the identity and a plain copy).  For one (bz, by) the
// output [Bx][d^3] is one contiguous run and the input is d^2 contiguous row segments
// (z = bz d + oz, y = by d + oy, row r = oz d + oy).  A workgroup takes Kx consecutive blocks of
// one (bz, by) and R of their rows: it reads the R row segments of Kx d elements (coalesced
// along x, V elements per lane) into an LDS tile [R][P] (row pitch P = Kx d + V keeps the
// strided reads of the other side off a single bank), then writes the Kx R d outputs in output
// order, V per lane, element (bx, r, ox) from tile[r][bx d + ox].  The inverse reads and writes
// the other way round.  Kx and R are powers of two, so every index is a shift or a mask; the
// last chunk of a row of blocks leaves its columns beyond the grid idle.  One tile holds 16 KiB:
// R = d^2 and Kx = min(16 KiB / d^3 elements, Bx rounded up to a power of two) while a block
// fits, else Kx = 1 and R = 16 KiB / d elements.
constexpr int kDenseTileBytes = 16384;
constexpr int kDenseSmemBytes = 24576;  // tile + row padding (at most R V elements)

struct DenseShape {
  int ld, lkx, lr;    // log2 of d, Kx, R
  int chunks, rchunks, pitch;
};

template <int B> struct VecOf;
template <> struct VecOf<16> { using type = uint4; };
template <> struct VecOf<8> { using type = uint2; };
template <> struct VecOf<4> { using type = uint32_t; };
template <> struct VecOf<2> { using type = uint16_t; };
template <> struct VecOf<1> { using type = uint8_t; };

template <typename T, int V>
__global__ __launch_bounds__(256) void dense_interleave_kernel(const T *__restrict__ in, T *__restrict__ out, int nx,
                                                                int ny, int nz, DenseShape t, int inverse) {
  using Vec = typename VecOf<V * sizeof(T)>::type;
  union Pack {
    Vec v;
    T e[V];
  };
  __shared__ __align__(16) unsigned char smem[kDenseSmemBytes];
  T *tile = reinterpret_cast<T *>(smem);
  const int ld = t.ld, d = 1 << ld, P = t.pitch;
  const int Bx = nx >> ld, By = ny >> ld, Bz = nz >> ld;
  const int lcols = t.lkx + ld, lrd = t.lr + ld;  // log2 of Kx d (tile columns) and R d (outputs per block)
  const int64_t items = (int64_t)Bz * By * t.chunks * t.rchunks;
  for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const int rc = it % t.rchunks;
    const int64_t rest = it / t.rchunks;
    const int ch = rest % t.chunks;
    const int64_t byz = rest / t.chunks;
    const int by = byz % By, bz = byz / By;
    const int bx0 = ch << t.lkx, kx = min(1 << t.lkx, Bx - bx0), W = kx << ld, r0 = rc << t.lr;
    // source row r of the tile: z = bz d + (r0 + r) / d, y = by d + (r0 + r) % d, x from bx0 d
    const int64_t src0 = ((int64_t)(bz << ld) * ny + (by << ld)) * nx + ((int64_t)bx0 << ld);
    const int64_t dst0 = (((int64_t)(bz * By + by) * Bx + bx0) << (3 * ld)) + ((int64_t)r0 << ld);
    const int nrow = (1 << (t.lr + lcols)) / V, nout = (1 << (t.lkx + lrd)) / V;
    if (!inverse) {
      for (int q = threadIdx.x; q < nrow; q += 256) {
        const int e = q * V, r = e >> lcols, x = e & ((1 << lcols) - 1);
        if (x >= W) continue;
        const int rr = r0 + r;
        *reinterpret_cast<Vec *>(tile + r * P + x) =
            *reinterpret_cast<const Vec *>(in + src0 + ((int64_t)(rr >> ld) * ny + (rr & (d - 1))) * nx + x);
      }
      __syncthreads();
      for (int q = threadIdx.x; q < nout; q += 256) {
        const int o = q * V, bxl = o >> lrd, rem = o & ((1 << lrd) - 1);
        if (bxl >= kx) continue;
        Pack u;
#pragma unroll
        for (int j = 0; j < V; ++j) u.e[j] = tile[((rem + j) >> ld) * P + (bxl << ld) + ((rem + j) & (d - 1))];
        *reinterpret_cast<Vec *>(out + dst0 + ((int64_t)bxl << (3 * ld)) + rem) = u.v;
      }
    } else {
      for (int q = threadIdx.x; q < nout; q += 256) {
        const int o = q * V, bxl = o >> lrd, rem = o & ((1 << lrd) - 1);
        if (bxl >= kx) continue;
        Pack u;
        u.v = *reinterpret_cast<const Vec *>(in + dst0 + ((int64_t)bxl << (3 * ld)) + rem);
#pragma unroll
        for (int j = 0; j < V; ++j) tile[((rem + j) >> ld) * P + (bxl << ld) + ((rem + j) & (d - 1))] = u.e[j];
      }
      __syncthreads();
      for (int q = threadIdx.x; q < nrow; q += 256) {
        const int e = q * V, r = e >> lcols, x = e & ((1 << lcols) - 1);
        if (x >= W) continue;
        const int rr = r0 + r;
        *reinterpret_cast<Vec *>(out + src0 + ((int64_t)(rr >> ld) * ny + (rr & (d - 1))) * nx + x) =
            *reinterpret_cast<const Vec *>(tile + r * P + x);
      }
    }
    __syncthreads();  // the tile is refilled by the next item
  }
}

static int ilog2(int v) {
  int l = 0;
  while ((1 << (l + 1)) <= v) ++l;
  return l;
}

// Tile shape for Bx blocks along x at interleave factor d >= 2, elements of esize bytes moved V
// at a time.
static DenseShape dense_shape(int Bx, int d, int esize, int V) {
  DenseShape t;
  const int tile = kDenseTileBytes / esize, d2 = d * d, d3 = d2 * d;
  int kx = 1, r = d2;
  if (d3 <= tile) {
    while (kx < Bx && kx * 2 * d3 <= tile) kx *= 2;
  } else {
    r = tile / d;
  }
  t.ld = ilog2(d);
  t.lkx = ilog2(kx);
  t.lr = ilog2(r);
  t.chunks = (Bx + kx - 1) / kx;
  t.rchunks = d2 / r;
  t.pitch = kx * d + V;
  return t;
}

template <typename T>
static void launch_dense(const void *in, void *out, const npvs_dims &g, int d, int inverse, hipStream_t s) {
  // 16-byte lanes (8 for single bytes, whose rows are only known to be multiples of 8 long) when
  // both buffers allow it
  constexpr int VV = sizeof(T) == 1 ? 8 : 16 / (int)sizeof(T);
  const bool vec = ((uintptr_t)in % (VV * sizeof(T))) == 0 && ((uintptr_t)out % (VV * sizeof(T))) == 0;
  const DenseShape t = dense_shape(g.nx / d, d, sizeof(T), vec ? VV : 1);
  const int64_t items = (int64_t)(g.ny / d) * (g.nz / d) * t.chunks * t.rchunks;
  const int grid = stride_grid(items, 1, 16384);
  if (vec)
    dense_interleave_kernel<T, VV><<<grid, 256, 0, s>>>((const T *)in, (T *)out, g.nx, g.ny, g.nz, t, inverse);
  else
    dense_interleave_kernel<T, 1><<<grid, 256, 0, s>>>((const T *)in, (T *)out, g.nx, g.ny, g.nz, t, inverse);
}

// Sparse interleave of packed bits onto active sites: one thread per (site, oz, oy) run of d
// channels.
template <typename T>
__device__ __forceinline__ T one_zero(int bit);
template <>
__device__ __forceinline__ float one_zero<float>(int bit) { return bit ? 1.0f : 0.0f; }
template <>
__device__ __forceinline__ uint16_t one_zero<uint16_t>(int bit) { return bit ? (uint16_t)0x3f80 : (uint16_t)0; }
template <>
__device__ __forceinline__ uint8_t one_zero<uint8_t>(int bit) { return (uint8_t)bit; }

// Row r of X is [stride] elements: the d^3 values, then zeros up to the stride (the padding a
// BF16 layer of fewer than 8 input channels reads as channels of zero).
// With X2, a second bit grid of the same shape, bits2, is gathered in the same pass into the
// uint8 rows X2 [cap][d^3] (the labels of a training step, beside its input).
template <typename T>
__global__ __launch_bounds__(256) void gather_bits_kernel(Batch B, const uint8_t *__restrict__ bits,
                                                           const int32_t *__restrict__ site_keys,
                                                           const npvs_counts *__restrict__ counts, T *__restrict__ X,
                                                           int stride, const uint8_t *__restrict__ bits2,
                                                           uint8_t *__restrict__ X2) {
  const int d = B.d;
  const int32_t n = counts->n_sites;
  const int64_t runs = (int64_t)n * d * d;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < runs; t += (int64_t)gridDim.x * blockDim.x) {
    int oy = t % d, oz = (t / d) % d;
    int32_t r = (int32_t)(t / ((int64_t)d * d));
    int32_t key = site_keys[r];
    const GridDesc &g = B.g[grid_of_key(B, key)];
    int32_t l = key - g.key_off;
    int bx = l % g.Bx, by = (l / g.Bx) % g.By, bz = l / (g.Bx * g.By);
    const int64_t row_off = g.occ_off + ((int64_t)(bz * d + oz) * g.ny + (by * d + oy)) * (g.nx >> 3);
    const uint8_t *row = bits + row_off;
    T *dst = X + (int64_t)r * stride + (oz * d + oy) * d;
    const int x0 = bx * d;
    for (int ox = 0; ox < d; ++ox) {
      int x = x0 + ox;
      dst[ox] = one_zero<T>((row[x >> 3] >> (x & 7)) & 1);
    }
    if (X2) {
      const uint8_t *row2 = bits2 + row_off;
      uint8_t *dst2 = X2 + (int64_t)r * d * d * d + (oz * d + oy) * d;
      for (int ox = 0; ox < d; ++ox) {
        int x = x0 + ox;
        dst2[ox] = (row2[x >> 3] >> (x & 7)) & 1;
      }
    }
    if (oy == d - 1 && oz == d - 1)  // the row's last run also clears its padding
      for (int c = d * d * d; c < stride; ++c) X[(int64_t)r * stride + c] = one_zero<T>(0);
  }
}

// De-interleave + threshold + pack: one thread per packed output byte (8 froxels along x).  The
// byte's froxels lie in 8/d consecutive blocks (d <= 8) or in one block (d >= 8); each block's
// row is looked up once and its logits of this (y, z) line are contiguous in Y.
__global__ __launch_bounds__(256) void deinterleave_threshold_kernel(Batch B, int64_t total_bytes,
                                                                      const float *__restrict__ Y, int C,
                                                                      const int32_t *__restrict__ block_row,
                                                                      const uint8_t *__restrict__ occ,
                                                                      uint8_t *__restrict__ pvs,
                                                                      float *__restrict__ logits) {
  const int d = B.d;  // C: elements per row of Y (d^3, or more for a padded row)
  const float ninf = -__builtin_huge_valf();
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total_bytes;
       t += (int64_t)gridDim.x * blockDim.x) {
    const uint8_t gbits = occ[t];
    if (!logits && !gbits) {  // no occupied froxel in this byte: no PVS bit either
      pvs[t] = 0;
      continue;
    }
    int b = 0;
    while (b + 1 < B.n && t >= B.g[b + 1].occ_off) ++b;
    const GridDesc &g = B.g[b];
    // 32-bit index arithmetic: a grid holds at most 1024^3 / 8 bytes
    const uint32_t l = (uint32_t)(t - g.occ_off), rb = (uint32_t)g.nx >> 3, ny = (uint32_t)g.ny;
    const uint32_t ly = l / rb;
    const int xb = (int)(l - ly * rb);
    const int y = (int)(ly % ny);
    const int z = (int)(ly / ny);
    const int key_yz = g.key_off + ((z / d) * g.By + (y / d)) * g.Bx;
    const int cyz = ((z % d) * d + (y % d)) * d;
    float lv[8];
    if (d == 4 && (C & 3) == 0) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int32_t row = block_row[key_yz + xb * 2 + j];
        float4 v = row >= 0 ? *reinterpret_cast<const float4 *>(Y + (int64_t)row * C + cyz)
                            : make_float4(ninf, ninf, ninf, ninf);
        lv[4 * j] = v.x;
        lv[4 * j + 1] = v.y;
        lv[4 * j + 2] = v.z;
        lv[4 * j + 3] = v.w;
      }
    } else if (d < 8) {
      for (int j = 0; j < 8 / d; ++j) {
        const int32_t row = block_row[key_yz + (xb * 8) / d + j];
        for (int ox = 0; ox < d; ++ox) lv[j * d + ox] = row >= 0 ? Y[(int64_t)row * C + cyz + ox] : ninf;
      }
    } else {
      const int32_t row = block_row[key_yz + (xb * 8) / d];
      const int off = (xb * 8) % d;
#pragma unroll
      for (int i = 0; i < 8; ++i) lv[i] = row >= 0 ? Y[(int64_t)row * C + cyz + off + i] : ninf;
    }
    uint8_t out = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) out |= (uint8_t)(((lv[i] >= 0.0f) && ((gbits >> i) & 1)) << i);
    pvs[t] = out;
    if (logits) {
      float4 *dst = reinterpret_cast<float4 *>(logits + g.dense_off + (((int64_t)z * g.ny + y) * g.nx + xb * 8));
      dst[0] = make_float4(lv[0], lv[1], lv[2], lv[3]);
      dst[1] = make_float4(lv[4], lv[5], lv[6], lv[7]);
    }
  }
}

}  // namespace npvs

using namespace npvs;

static npvs_status dense_perm(const void *in, npvs_dims g, int32_t d, int32_t esize, void *out, void *stream,
                              int inverse, const char *name) {
  if (!in || !out) return fail(NPVS_ERR_INVALID_ARG, std::string(name) + ": null pointer");
  Batch B;
  npvs_status st = make_batch(1, &g, d, nullptr, &B);
  if (st != NPVS_OK) return st;
  hipStream_t s = as_stream(stream);
  if (esize != 1 && esize != 2 && esize != 4 && esize != 8)
    return fail(NPVS_ERR_INVALID_ARG, std::string(name) + ": elem_bytes must be 1, 2, 4 or 8");
  if (d == 1)  // g_1 is the identity
    return check_hip(hipMemcpyAsync(out, in, (size_t)g.nx * g.ny * g.nz * esize, hipMemcpyDeviceToDevice, s), name);
  switch (esize) {
    case 1: launch_dense<uint8_t>(in, out, g, d, inverse, s); break;
    case 2: launch_dense<uint16_t>(in, out, g, d, inverse, s); break;
    case 4: launch_dense<uint32_t>(in, out, g, d, inverse, s); break;
    default: launch_dense<uint64_t>(in, out, g, d, inverse, s); break;
  }
  return check_hip(hipGetLastError(), name);
}

extern "C" npvs_status npvs_interleave(const void *in, npvs_dims g, int32_t d, int32_t elem_bytes, void *out,
                                      void *stream) {
  return dense_perm(in, g, d, elem_bytes, out, stream, 0, "npvs_interleave");
}

extern "C" npvs_status npvs_deinterleave(const void *in, npvs_dims g, int32_t d, int32_t elem_bytes, void *out,
                                        void *stream) {
  return dense_perm(in, g, d, elem_bytes, out, stream, 1, "npvs_deinterleave");
}

extern "C" npvs_status npvs_gather_input(const uint8_t *bits, int32_t n_grids, const npvs_dims *dims, int32_t d,
                                        const int32_t *site_keys, const npvs_counts *counts, int32_t cap_sites,
                                        int32_t dtype, int32_t row_stride, void *X, const uint8_t *bits2,
                                        uint8_t *X2, void *stream) {
  if (!bits || !site_keys || !counts || !X) return fail(NPVS_ERR_INVALID_ARG, "npvs_gather_input: null pointer");
  if (!bits2 != !X2) return fail(NPVS_ERR_INVALID_ARG, "npvs_gather_input: bits2 and X2 must both be given or both null");
  Batch B;
  npvs_status st = make_batch(n_grids, dims, d, nullptr, &B);
  if (st != NPVS_OK) return st;
  if (cap_sites < 1) return fail(NPVS_ERR_INVALID_ARG, "npvs_gather_input: cap_sites < 1");
  const int C = d * d * d, stride = row_stride ? row_stride : C;
  if (stride < C) return fail(NPVS_ERR_INVALID_ARG, "npvs_gather_input: row_stride below d^3");
  int grid = stride_grid((int64_t)cap_sites * d * d, 256, 4096);
  hipStream_t s = as_stream(stream);
  switch (dtype) {
    case NPVS_F32:
      gather_bits_kernel<float><<<grid, 256, 0, s>>>(B, bits, site_keys, counts, (float *)X, stride, bits2, X2);
      break;
    case NPVS_BF16:
      gather_bits_kernel<uint16_t><<<grid, 256, 0, s>>>(B, bits, site_keys, counts, (uint16_t *)X, stride, bits2, X2);
      break;
    case NPVS_U8:
      gather_bits_kernel<uint8_t><<<grid, 256, 0, s>>>(B, bits, site_keys, counts, (uint8_t *)X, stride, bits2, X2);
      break;
    default: return fail(NPVS_ERR_INVALID_ARG, "npvs_gather_input: dtype must be NPVS_F32, NPVS_BF16 or NPVS_U8");
  }
  return check_hip(hipGetLastError(), "npvs_gather_input");
}

extern "C" npvs_status npvs_deinterleave_threshold(const float *Y, int32_t y_stride, const int32_t *block_row,
                                                   const uint8_t *occ_bits, int32_t n_grids, const npvs_dims *dims,
                                                   int32_t d, uint8_t *pvs_bits, float *logits, void *stream) {
  if (!Y || !block_row || !occ_bits || !pvs_bits)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_deinterleave_threshold: null pointer");
  Batch B;
  npvs_status st = make_batch(n_grids, dims, d, nullptr, &B);
  if (st != NPVS_OK) return st;
  int64_t total = 0;
  for (int b = 0; b < n_grids; ++b) total += (int64_t)dims[b].nz * dims[b].ny * (dims[b].nx / 8);
  const int C = d * d * d, stride = y_stride ? y_stride : C;
  if (stride < C) return fail(NPVS_ERR_INVALID_ARG, "npvs_deinterleave_threshold: y_stride below d^3");
  int grid = stride_grid(total, 256, 8192);
  deinterleave_threshold_kernel<<<grid, 256, 0, as_stream(stream)>>>(B, total, Y, stride, block_row, occ_bits,
                                                                      pvs_bits, logits);
  return check_hip(hipGetLastError(), "npvs_deinterleave_threshold");
}
