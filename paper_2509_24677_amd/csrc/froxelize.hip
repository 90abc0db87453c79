// Froxelization of grid-space triangles into packed occupancy bits (Sec. 3.2, Fig. 2(b)).
//
// G(x) = 1 iff a triangle meets the closed froxel x.  Vertices are quantized to 1/256 froxel
// (round half to even) and overlap is decided by the separating-axis theorem in exact integer
// arithmetic, so the result does not depend on triangle order or on the schedule.
//
// Three launches:
//   1. zero the per-tile triangle counters;
//   2. one thread per triangle: quantize, clip the froxel range, append the triangle to the
//      list of every tile (128 x 8 x 8 froxels) its range meets;
//   3. one workgroup per tile, one thread per 32-froxel word: stream the tile's triangles
//      through LDS (per-triangle axis constants computed once per tile), test the word's
//      froxels, write the word once.  No atomics touch the output.
// A tile whose list overflowed scans every triangle of its grid instead (same result).
#include "npvs_common.hpp"

namespace npvs {

struct TriRec {
  int32_t q[9];     // fixed-point vertices v0, v1, v2 (x, y, z)
  int16_t lo[3];    // clipped froxel range; lo > hi when empty or ignored
  int16_t hi[3];
};
static_assert(sizeof(TriRec) == 48, "record layout");

constexpr int kChunk = 128;  // triangles staged in LDS at a time

__global__ void frox_zero_kernel(int32_t *p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

__device__ __forceinline__ int tri_grid(const Batch &B, int64_t t) {
  int b = 0;
  while (b + 1 < B.n && t >= B.g[b + 1].tri_off) ++b;
  return b;
}

__global__ __launch_bounds__(256) void frox_bin_kernel(const float *__restrict__ tris, Batch B, int64_t total,
                                                        TriRec *__restrict__ recs, int32_t *__restrict__ tile_count,
                                                        int32_t *__restrict__ tile_list) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const GridDesc &g = B.g[tri_grid(B, t)];
  TriRec r;
  bool ok = true;
  int32_t mn[3], mx[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) { mn[a] = 0x7fffffff; mx[a] = -0x7fffffff; }
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float x = tris[t * 9 + v * 3 + a];
      // finite and |x| < 1024 (NaN fails the comparison)
      ok = ok && (__builtin_fabsf(x) < (float)NPVS_MAX_DIM);
      int32_t q = ok ? (int32_t)__builtin_rintf(x * 256.0f) : 0;  // exact scaling, then round half to even
      r.q[v * 3 + a] = q;
      mn[a] = q < mn[a] ? q : mn[a];
      mx[a] = q > mx[a] ? q : mx[a];
    }
  int32_t dims[3] = {g.nx, g.ny, g.nz};
  int32_t lo[3], hi[3];
  bool empty = !ok;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    // closed cells [256 i, 256 i + 256] meeting [mn, mx]: i in [floor((mn-1)/256), floor(mx/256)]
    lo[a] = (mn[a] - 1) >> 8;
    hi[a] = mx[a] >> 8;
    lo[a] = lo[a] < 0 ? 0 : lo[a];
    hi[a] = hi[a] > dims[a] - 1 ? dims[a] - 1 : hi[a];
    empty = empty || lo[a] > hi[a];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r.lo[a] = (int16_t)(empty ? 1 : lo[a]);
    r.hi[a] = (int16_t)(empty ? 0 : hi[a]);
  }
  recs[t] = r;
  if (empty) return;
  int tx0 = lo[0] / kFroxTileX, tx1 = hi[0] / kFroxTileX;
  int ty0 = lo[1] / kFroxTileY, ty1 = hi[1] / kFroxTileY;
  int tz0 = lo[2] / kFroxTileZ, tz1 = hi[2] / kFroxTileZ;
  for (int tz = tz0; tz <= tz1; ++tz)
    for (int ty = ty0; ty <= ty1; ++ty)
      for (int tx = tx0; tx <= tx1; ++tx) {
        int tile = g.tile_off + (tz * g.tiles_y + ty) * g.tiles_x + tx;
        int slot = atomicAdd(&tile_count[tile], 1);
        if (slot < kFroxTileCap) tile_list[(int64_t)tile * kFroxTileCap + slot] = (int32_t)t;
      }
}

// Per-triangle constants of the exact overlap test, staged in LDS.  For an axis a the closed
// froxel I = (i, j, k) meets the triangle along a iff L <= a . I <= H, where
//   L = ceil((min_v a.q_v - 256 sum_c max(0, a_c)) / 256),  H = floor((max_v a.q_v - 256 sum_c min(0, a_c)) / 256)
// (the box [256 I, 256 I + 256] projects onto [256 a.I + R-, 256 a.I + R+]).  The axes are the
// triangle normal and the nine cross products of the edges with the box axes; the box normals
// are the clipped froxel range.  A zero axis gives L = H = 0 = a.I and never separates.
struct SetupLds {
  int32_t lo[3][kChunk], hi[3][kChunk];
  int32_t e[3][3][kChunk];           // edge i, component c
  int32_t L[3][3][kChunk], H[3][3][kChunk];  // edge i x box axis j
  int64_t n[3][kChunk];
  int64_t nL[kChunk], nH[kChunk];
};

__device__ __forceinline__ void axis_bounds(int64_t a0, int64_t a1, int64_t a2, const int32_t *q, int64_t &L,
                                            int64_t &H) {
  int64_t p0 = a0 * q[0] + a1 * q[1] + a2 * q[2];
  int64_t p1 = a0 * q[3] + a1 * q[4] + a2 * q[5];
  int64_t p2 = a0 * q[6] + a1 * q[7] + a2 * q[8];
  int64_t pmin = p0 < p1 ? p0 : p1, pmax = p0 > p1 ? p0 : p1;
  pmin = p2 < pmin ? p2 : pmin;
  pmax = p2 > pmax ? p2 : pmax;
  int64_t rp = 256 * ((a0 > 0 ? a0 : 0) + (a1 > 0 ? a1 : 0) + (a2 > 0 ? a2 : 0));
  int64_t rm = 256 * ((a0 < 0 ? a0 : 0) + (a1 < 0 ? a1 : 0) + (a2 < 0 ? a2 : 0));
  L = (pmin - rp + 255) >> 8;  // ceil division by 256 (arithmetic shift floors)
  H = (pmax - rm) >> 8;
}

__device__ void setup_triangle(SetupLds &S, int j, const TriRec &r) {
  const int32_t *q = r.q;
  int64_t e[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      e[i][c] = (int64_t)q[((i + 1) % 3) * 3 + c] - q[i * 3 + c];
      S.e[i][c][j] = (int32_t)e[i][c];
    }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    S.lo[a][j] = r.lo[a];
    S.hi[a][j] = r.hi[a];
  }
  int64_t n0 = e[0][1] * e[1][2] - e[0][2] * e[1][1];
  int64_t n1 = e[0][2] * e[1][0] - e[0][0] * e[1][2];
  int64_t n2 = e[0][0] * e[1][1] - e[0][1] * e[1][0];
  S.n[0][j] = n0;
  S.n[1][j] = n1;
  S.n[2][j] = n2;
  int64_t L, H;
  axis_bounds(n0, n1, n2, q, L, H);
  S.nL[j] = L;
  S.nH[j] = H;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    // e x x = (0, e_z, -e_y), e x y = (-e_z, 0, e_x), e x z = (e_y, -e_x, 0)
    axis_bounds(0, e[i][2], -e[i][1], q, L, H);
    S.L[i][0][j] = (int32_t)L;
    S.H[i][0][j] = (int32_t)H;
    axis_bounds(-e[i][2], 0, e[i][0], q, L, H);
    S.L[i][1][j] = (int32_t)L;
    S.H[i][1][j] = (int32_t)H;
    axis_bounds(e[i][1], -e[i][0], 0, q, L, H);
    S.L[i][2][j] = (int32_t)L;
    S.H[i][2][j] = (int32_t)H;
  }
}

__global__ __launch_bounds__(256) void frox_tile_kernel(Batch B, const TriRec *__restrict__ recs,
                                                         const int32_t *__restrict__ tile_count,
                                                         const int32_t *__restrict__ tile_list,
                                                         uint8_t *__restrict__ occ) {
  __shared__ SetupLds S;
  const int tile = blockIdx.x;
  int b = 0;
  while (b + 1 < B.n && tile >= B.g[b + 1].tile_off) ++b;
  const GridDesc &g = B.g[b];
  int lt = tile - g.tile_off;
  int tx = lt % g.tiles_x, ty = (lt / g.tiles_x) % g.tiles_y, tz = lt / (g.tiles_x * g.tiles_y);
  const int tid = threadIdx.x;
  const int x0 = tx * kFroxTileX + (tid & 3) * 32;
  const int y = ty * kFroxTileY + ((tid >> 2) & 7);
  const int z = tz * kFroxTileZ + (tid >> 5);
  const bool in_grid = x0 < g.nx && y < g.ny && z < g.nz;
  const int xe = (x0 + 31 < g.nx - 1 ? x0 + 31 : g.nx - 1);
  uint32_t word = 0;

  const int cnt = tile_count[tile];
  const bool listed = cnt <= kFroxTileCap;
  const int items = listed ? cnt : g.tri_n;
  for (int base = 0; base < items; base += kChunk) {
    __syncthreads();
    if (tid < kChunk && base + tid < items) {
      int64_t t = listed ? (int64_t)tile_list[(int64_t)tile * kFroxTileCap + base + tid] : g.tri_off + base + tid;
      setup_triangle(S, tid, recs[t]);
    }
    __syncthreads();
    const int m = items - base < kChunk ? items - base : kChunk;
    if (!in_grid) continue;
    for (int j = 0; j < m; ++j) {
      if (y < S.lo[1][j] || y > S.hi[1][j] || z < S.lo[2][j] || z > S.hi[2][j]) continue;
      int ia = S.lo[0][j] > x0 ? S.lo[0][j] : x0;
      int ib = S.hi[0][j] < xe ? S.hi[0][j] : xe;
      if (ia > ib) continue;
      // edge x x-axis tests do not depend on x: test once for the row
      bool row_ok = true;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        int32_t s = S.e[i][2][j] * y - S.e[i][1][j] * z;
        row_ok = row_ok && s >= S.L[i][0][j] && s <= S.H[i][0][j];
      }
      if (!row_ok) continue;
      int32_t sy[3], sz[3], dy[3], dz[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        dy[i] = -S.e[i][2][j];  // x-component of e x y-axis
        dz[i] = S.e[i][1][j];   // x-component of e x z-axis
        sy[i] = dy[i] * ia + S.e[i][0][j] * z;
        sz[i] = dz[i] * ia - S.e[i][0][j] * y;
      }
      int64_t nx_ = S.n[0][j];
      int64_t sn = nx_ * ia + S.n[1][j] * (int64_t)y + S.n[2][j] * (int64_t)z;
      const int64_t nL = S.nL[j], nH = S.nH[j];
      for (int i = ia; i <= ib; ++i) {
        bool hit = sn >= nL && sn <= nH;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          hit = hit && sy[e] >= S.L[e][1][j] && sy[e] <= S.H[e][1][j];
          hit = hit && sz[e] >= S.L[e][2][j] && sz[e] <= S.H[e][2][j];
          sy[e] += dy[e];
          sz[e] += dz[e];
        }
        sn += nx_;
        word |= (uint32_t)hit << (i - x0);
      }
    }
  }
  if (!in_grid) return;
  const int64_t row_bytes = g.nx / 8;
  uint8_t *dst = occ + g.occ_off + ((int64_t)z * g.ny + y) * row_bytes + x0 / 8;
  if (x0 + 32 <= g.nx && (row_bytes & 3) == 0 && (g.occ_off & 3) == 0) {
    *reinterpret_cast<uint32_t *>(dst) = word;
  } else {
    for (int k = 0; k < 4 && x0 + 8 * k < g.nx; ++k) dst[k] = (uint8_t)(word >> (8 * k));
  }
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static void frox_ws_layout(const Batch &B, int64_t total_tris, size_t *off_count, size_t *off_list,
                           size_t *off_recs, size_t *bytes) {
  size_t o = 0;
  *off_count = o;
  o += align256(sizeof(int32_t) * (size_t)B.total_tiles);
  *off_list = o;
  o += align256(sizeof(int32_t) * (size_t)B.total_tiles * kFroxTileCap);
  *off_recs = o;
  o += align256(sizeof(TriRec) * (size_t)(total_tris > 0 ? total_tris : 1));
  *bytes = o;
}

}  // namespace npvs

using namespace npvs;

extern "C" npvs_status npvs_froxelize_workspace_size(int32_t n_grids, const npvs_dims *dims, const int64_t *n_tris,
                                                     size_t *bytes) {
  if (!bytes || !n_tris) return fail(NPVS_ERR_INVALID_ARG, "npvs_froxelize_workspace_size: null pointer");
  Batch B;
  npvs_status st = make_batch(n_grids, dims, 1, n_tris, &B);
  if (st != NPVS_OK) return st;
  int64_t total = 0;
  for (int b = 0; b < n_grids; ++b) total += n_tris[b];
  size_t a, c, r;
  frox_ws_layout(B, total, &a, &c, &r, bytes);
  return NPVS_OK;
}

extern "C" npvs_status npvs_froxelize(const float *tris, const int64_t *n_tris, int32_t n_grids, const npvs_dims *dims,
                                      uint8_t *occ_bits, void *ws, size_t ws_bytes, void *stream) {
  if (!n_tris || !occ_bits || !ws) return fail(NPVS_ERR_INVALID_ARG, "npvs_froxelize: null pointer");
  Batch B;
  npvs_status st = make_batch(n_grids, dims, 1, n_tris, &B);
  if (st != NPVS_OK) return st;
  int64_t total = 0;
  for (int b = 0; b < n_grids; ++b) total += n_tris[b];
  if (total > 0 && !tris) return fail(NPVS_ERR_INVALID_ARG, "npvs_froxelize: null triangles");
  if (total > INT32_MAX) return fail(NPVS_ERR_INVALID_ARG, "npvs_froxelize: too many triangles");
  size_t oc, ol, orr, need;
  frox_ws_layout(B, total, &oc, &ol, &orr, &need);
  if (ws_bytes < need) return fail(NPVS_ERR_INVALID_ARG, "npvs_froxelize: workspace too small");
  char *w = static_cast<char *>(ws);
  int32_t *cnt = reinterpret_cast<int32_t *>(w + oc);
  int32_t *lst = reinterpret_cast<int32_t *>(w + ol);
  TriRec *recs = reinterpret_cast<TriRec *>(w + orr);
  hipStream_t s = as_stream(stream);
  frox_zero_kernel<<<stride_grid(B.total_tiles, 256, 1024), 256, 0, s>>>(cnt, B.total_tiles);
  if (total > 0)
    frox_bin_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(tris, B, total, recs, cnt, lst);
  frox_tile_kernel<<<B.total_tiles, 256, 0, s>>>(B, recs, cnt, lst, occ_bits);
  return check_hip(hipGetLastError(), "npvs_froxelize");
}
