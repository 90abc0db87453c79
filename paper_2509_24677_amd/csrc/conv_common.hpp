// Device helpers shared by the BF16 convolution kernels (conv.hip, stack.hip).
#pragma once

#include "npvs_common.hpp"

namespace npvs {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;

// ------------------------------------------------------------------------------------------
// XCD-aware tile order: workgroup i runs on XCD (i % 8); the tiles of a layer are cut into 8
// contiguous ranges, one per XCD, so neighbouring rows (which gather overlapping inputs) share
// that XCD's L2.  Returns the j-th tile of workgroup i, or -1.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ int xcd_tile(int i, int G, int ntiles, int j) {
  const int per = (ntiles + 7) >> 3;  // tiles per XCD
  const int slot = (i >> 3) + j * (G >> 3);
  if (slot >= per) return -1;
  int t = (i & 7) * per + slot;
  return t < ntiles ? t : -1;
}

__device__ __forceinline__ bf16x8_t gather8(const uint16_t *__restrict__ X, int cin, int i, int c) {
  const bool ok = i >= 0 && c < cin;
  const uint4 v = *reinterpret_cast<const uint4 *>(X + (ok ? (int64_t)i * cin + c : 0));
  const uint32_t m = ok ? ~0u : 0u;  // a mask, not a select of the loaded value: no branch around the load
  return __builtin_bit_cast(bf16x8_t, make_uint4(v.x & m, v.y & m, v.z & m, v.w & m));
}

// Zero as a value the compiler cannot see through, taken once per tile and added to the weight
// index: the weight loads then stay inside the tile loop instead of being hoisted out of it into
// registers for all tiles (which would cost the occupancy the gather latency needs), and the
// pointer keeps its global address space.  The empty asm emits no instruction.
__device__ __forceinline__ int opaque_zero() {
  int z = 0;
  asm volatile("" : "+s"(z));
  return z;
}

// Neighbour index of row r for offset k, or -1 past the last site (unconditional load of a row
// that exists: r is clamped to n - 1).
__device__ __forceinline__ int nbr_index(const int32_t *__restrict__ nbr, int cap, int k, int r, int n) {
  const int v = nbr[(int64_t)k * cap + (r < n ? r : n - 1)];
  return r < n ? v : -1;
}

// Bias (4 values, already loaded) + optional ReLU, stored as float32 or bfloat16.
__device__ __forceinline__ void conv_bf16_epilogue_bias(const f32x4_t &acc, int r, int n, int o, int cout,
                                                        const float (&bv)[4], int relu, int out_f32, void *Y) {
  if (r >= n || o >= cout) return;
  float v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float t = acc[i] + bv[i];
    v[i] = (relu && t < 0.0f) ? 0.0f : t;
  }
  if (out_f32) {
    *reinterpret_cast<float4 *>(static_cast<float *>(Y) + (int64_t)r * cout + o) = make_float4(v[0], v[1], v[2], v[3]);
  } else {
    uint2 p;
    p.x = (uint32_t)f32_to_bf16(v[0]) | ((uint32_t)f32_to_bf16(v[1]) << 16);
    p.y = (uint32_t)f32_to_bf16(v[2]) | ((uint32_t)f32_to_bf16(v[3]) << 16);
    *reinterpret_cast<uint2 *>(static_cast<uint16_t *>(Y) + (int64_t)r * cout + o) = p;
  }
}

template <int NB>
__device__ __forceinline__ void conv_bf16_epilogue(const f32x4_t &acc, int r, int n, int o, int cout,
                                                   const float *__restrict__ bias, int relu, int out_f32, void *Y) {
  if (r >= n || o >= cout) return;
  float v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float t = acc[i] + (bias ? bias[o + i] : 0.0f);
    v[i] = (relu && t < 0.0f) ? 0.0f : t;
  }
  if (out_f32) {
    *reinterpret_cast<float4 *>(static_cast<float *>(Y) + (int64_t)r * cout + o) = make_float4(v[0], v[1], v[2], v[3]);
  } else {
    uint2 p;
    p.x = (uint32_t)f32_to_bf16(v[0]) | ((uint32_t)f32_to_bf16(v[1]) << 16);
    p.y = (uint32_t)f32_to_bf16(v[2]) | ((uint32_t)f32_to_bf16(v[3]) << 16);
    *reinterpret_cast<uint2 *>(static_cast<uint16_t *>(Y) + (int64_t)r * cout + o) = p;
  }
}

}  // namespace npvs
