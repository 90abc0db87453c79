// Shared device/host helpers of the gfx950 NeuralPVS library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/neuralpvs.h"

namespace npvs {

// ------------------------------------------------------------------------------------------
// Batch descriptor passed to kernels by value.
// ------------------------------------------------------------------------------------------
struct GridDesc {
  int32_t nx, ny, nz;     // froxels
  int32_t Bx, By, Bz;     // blocks of the interleave factor d
  int64_t occ_off;        // byte offset of the packed grid
  int64_t dense_off;      // element offset of a dense per-froxel array (logits)
  int32_t key_off;        // global key of block 0
  int32_t tile_off;       // first froxelization tile
  int64_t tri_off;        // first triangle
  int32_t tri_n;          // triangles
  int32_t tiles_x, tiles_y, tiles_z;
};

struct Batch {
  int32_t n;              // grids
  int32_t d;              // interleave factor
  int32_t total_blocks;
  int32_t total_tiles;
  GridDesc g[NPVS_MAX_GRIDS];
};

// Grid of a global block key (linear scan: at most NPVS_MAX_GRIDS grids).
__device__ __forceinline__ int grid_of_key(const Batch &B, int32_t key) {
  int b = 0;
  while (b + 1 < B.n && key >= B.g[b + 1].key_off) ++b;
  return b;
}

// ------------------------------------------------------------------------------------------
// bfloat16: raw uint16 bit patterns.  float -> bf16 rounds to nearest, ties to even (IEEE
// round-to-nearest applied to the upper 16 bits); NaN stays a quiet NaN.
// ------------------------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__host__ __device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __builtin_bit_cast(float, (uint32_t)h << 16);
}

// ------------------------------------------------------------------------------------------
// Host-side error reporting.
// ------------------------------------------------------------------------------------------
void set_error(const std::string &msg);
npvs_status fail(npvs_status code, const std::string &msg);
npvs_status check_hip(hipError_t e, const char *what);

// Fills a Batch from host dims; returns NPVS_OK or an argument error.
npvs_status make_batch(int32_t n_grids, const npvs_dims *dims, int32_t d, const int64_t *n_tris, Batch *out);

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Grid size for grid-stride kernels whose work count is only known on the device: enough
// workgroups to fill every compute unit several times, never more than the work needs.
inline int stride_grid(int64_t max_items, int per_block, int cap = 4096) {
  int64_t b = (max_items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

constexpr int kFroxTileX = 32;  // froxels per tile along x (one 32-froxel word)
constexpr int kFroxTileY = 8;
constexpr int kFroxTileZ = 8;
constexpr int kFroxTileCap = 2048;  // triangle slots per tile before the tile falls back to a full scan

// Tile shape of the BF16 convolution used when no autotuned choice is given (see conv.hip).
constexpr int kDefaultConvVariant = NPVS_DEFAULT_CONV_VARIANT;

// One convolution layer on `s` (conv.hip).  ws (nullable): workspace of conv_fwd_ws_bytes() bytes
// that lets wide BF16 inputs split their channels over several workgroups.
npvs_status conv_fwd_dispatch(const void *X, int32_t cin, const void *Wp, const float *bias, int32_t cout,
                              const int32_t *nbr, const npvs_counts *counts, int32_t cap, int32_t dtype, int32_t relu,
                              int32_t out_f32, void *Y, hipStream_t s, int variant, void *ws, size_t ws_bytes);
size_t conv_fwd_ws_bytes(int32_t cin, int32_t cout, int32_t cap, int32_t dtype);

// Backward building blocks shared by the submanifold and the strided layers (backward.hip), all
// enqueued on `s`:
//   bwd_form_dz: dZ = dY [Y > 0] (or dY) for the rows counts->n_sites, as float32 (dZ32, FP32
//     path) or bfloat16 (dZ16, BF16 path), plus the bias partials dbpart[kBwdDbBlocks][C];
//   bwd_wgrad: slice partials wpart[K][S][cin][cout] of dW_k = sum over the pairs (i, r) of
//     offset k (CSR rb_off[K + 1], pairs[][2]; a member of -1 reads as a zero row) of X[i]^T dZ[r];
//   bwd_reduce: dW = the slice partials summed in a fixed order, db = the bias partials summed.
constexpr int kBwdDbBlocks = 256;
int wg_slices(int cin, int cout);  // slices per offset of the weight-gradient partials
npvs_status bwd_form_dz(int32_t dtype, const void *Y, const float *dY, const npvs_counts *counts, int32_t C,
                        int32_t relu, float *dZ32, uint16_t *dZ16, float *dbpart, hipStream_t s);
npvs_status bwd_wgrad(int32_t dtype, const void *X, int32_t cin, const void *dZ, int32_t cout, int32_t K,
                      const int32_t *rb_off, const int32_t *pairs, int S, float *wpart, hipStream_t s);
npvs_status bwd_reduce(const float *wpart, const float *dbpart, int nparts, int32_t K, int S, int32_t cin,
                       int32_t cout, float *dW, float *db, hipStream_t s);
// The data gradient of a BF16 layer (dZ [cap][cin] of this layer -> [cap][cout] of the layer
// below, weights packed as for the data gradient) with the layer below's ReLU' fused in
// (conv.hip): dZ_below = bf16(result masked by M > 0; M null: no mask) and that layer's bias
// partials dbp[kBwdDbBlocks][cout].  cin <= 64 (multiple of 8), cout <= 64 (multiple of 4).
npvs_status dgrad_relu_fused(const uint16_t *dZ, int cin, const void *Wt, int cout, const int32_t *nbr,
                             const npvs_counts *counts, int cap, const uint16_t *M, uint16_t *dZ_below, float *dbp,
                             hipStream_t s);

}  // namespace npvs
