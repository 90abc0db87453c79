// Froxelization of grid-space triangles into packed occupancy bits (Sec. 3.2, Fig. 2(b)).
//
// G(x) = 1 iff a triangle meets the closed froxel x.  Vertices are quantized to 1/256 froxel
// (round half to even) and overlap is decided by the separating-axis theorem in exact integer
// arithmetic, so the result does not depend on triangle order or on the schedule.
//
// Three launches:
//   1. zero: the per-tile triangle counters (and the ignored-triangle count) and, on the parts
//      path, the output words;
//   2. bin: one thread per triangle quantizes it, clips its froxel range, computes the constants
//      of its separating-axis test once, and appends it to the list of every tile (32 x 8 x 8
//      froxels) the range meets; a workgroup counts its appends per tile in LDS first, so each
//      (workgroup, tile) pair makes one global counter update, and each chunk of 64 slots of a
//      tile's list is entered in a chunk list by the workgroup whose appends start it;
//   3. parts (every grid's x extent a multiple of 32): workgroups take chunks from the list, test
//      their triangles row by row, OR the hits into 64 words in LDS and each non-zero word into
//      the output with one atomic; otherwise one workgroup per tile tests all of the tile's
//      triangles and writes each of its words once.
// A tile whose list overflowed (more than 2048 triangles) scans all triangles of its grid.
#include <algorithm>

#include "npvs_common.hpp"

namespace npvs {

// Constants of one triangle's overlap test.  For an axis a the closed froxel I = (i, j, k) meets
// the triangle along a iff L <= a . I <= H.  The axes are the triangle normal n and the nine
// cross products of the edges e_i with the box axes (e x x = (0, e_z, -e_y), e x y = (-e_z, 0, e_x),
// e x z = (e_y, -e_x, 0)); the box normals are the clipped froxel range.  With |v| < 2048 the
// fixed-point coordinates are below 2^19 and edges below 2^20, so an edge-axis projection of a
// froxel index (below 1024 per axis) is below 2 * 2^20 * 1023 < 2^31 in magnitude and fits int32.
// The bounds L, H themselves can exceed that range; they are computed in int64 and clamped to
// [INT32_MIN, INT32_MAX], which keeps every comparison with an in-range projection unchanged.
struct TriSetup {
  int64_t n[3];          // normal (fixed-point cross product of two edges)
  int64_t nL, nH;        // normal-axis bounds
  int32_t e[3][3];       // edges e_i = v_{i+1} - v_i
  int32_t L[3][3];       // [edge][box axis]
  int32_t H[3][3];
  int16_t lo[3], hi[3];  // clipped froxel range; lo > hi when empty or ignored
};
static_assert(sizeof(TriSetup) % 16 == 0, "setup record is loaded as 16-byte words");

constexpr int kTileWords = (kFroxTileX / 32) * kFroxTileY * kFroxTileZ;  // 64
constexpr int kPartTris = 64;  // triangles of a chunk of the parts path
static_assert(kFroxTileX == 32 && kTileWords == 64, "one 32-froxel word per tile row");

// Zeroes the tile counters with the chunk count and, for the parts path, the output words.
__global__ void frox_zero_kernel(int32_t *p, int n, int32_t *n_ignored, uint32_t *occ_words, int64_t n_words) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_words; i += (int64_t)gridDim.x * blockDim.x)
    occ_words[i] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0 && n_ignored) *n_ignored = 0;
}

__device__ __forceinline__ int tri_grid(const Batch &B, int64_t t) {
  int b = 0;
  while (b + 1 < B.n && t >= B.g[b + 1].tri_off) ++b;
  return b;
}

// L = ceil((min_v a.q_v - 256 sum_c max(0, a_c)) / 256), H = floor((max_v a.q_v - 256 sum_c min(0, a_c)) / 256):
// the box [256 I, 256 I + 256] projects onto [256 a.I + R-, 256 a.I + R+].  A zero axis gives
// L = H = 0 = a . I and never separates.
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

__device__ __forceinline__ int32_t clamp_i32(int64_t v) {
  return v < (int64_t)INT32_MIN ? INT32_MIN : v > (int64_t)INT32_MAX ? INT32_MAX : (int32_t)v;
}

__device__ __forceinline__ void make_setup(const int32_t *q, TriSetup &S) {
  int32_t e[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      e[i][c] = q[((i + 1) % 3) * 3 + c] - q[i * 3 + c];
      S.e[i][c] = e[i][c];
    }
  S.n[0] = (int64_t)e[0][1] * e[1][2] - (int64_t)e[0][2] * e[1][1];
  S.n[1] = (int64_t)e[0][2] * e[1][0] - (int64_t)e[0][0] * e[1][2];
  S.n[2] = (int64_t)e[0][0] * e[1][1] - (int64_t)e[0][1] * e[1][0];
  axis_bounds(S.n[0], S.n[1], S.n[2], q, S.nL, S.nH);
  int64_t L, H;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    axis_bounds(0, e[i][2], -e[i][1], q, L, H);
    S.L[i][0] = clamp_i32(L);
    S.H[i][0] = clamp_i32(H);
    axis_bounds(-e[i][2], 0, e[i][0], q, L, H);
    S.L[i][1] = clamp_i32(L);
    S.H[i][1] = clamp_i32(H);
    axis_bounds(e[i][1], -e[i][0], 0, q, L, H);
    S.L[i][2] = clamp_i32(L);
    S.H[i][2] = clamp_i32(H);
  }
}

// Fixed-point vertices (rint(256 v), round half to even) and the clipped closed-froxel range of
// triangle t; true when the triangle is ignored (a coordinate not finite or |v| >= 2048; then
// *bad is set) or its range misses the grid.
__device__ __forceinline__ bool quantize_tri(const float *__restrict__ tris, int64_t t, const GridDesc &g,
                                             int32_t *q, int32_t *lo, int32_t *hi, bool *bad = nullptr) {
  bool ok = true;
  int32_t mn[3], mx[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    mn[a] = 0x7fffffff;
    mx[a] = -0x7fffffff;
  }
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float x = tris[t * 9 + v * 3 + a];
      ok = ok && (__builtin_fabsf(x) < (float)NPVS_COORD_LIMIT);  // finite and |x| < 2048 (NaN fails)
      int32_t qq = ok ? (int32_t)__builtin_rintf(x * 256.0f) : 0;  // exact scaling, round half to even
      q[v * 3 + a] = qq;
      mn[a] = qq < mn[a] ? qq : mn[a];
      mx[a] = qq > mx[a] ? qq : mx[a];
    }
  if (bad) *bad = !ok;
  const int32_t dims[3] = {g.nx, g.ny, g.nz};
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
  return empty;
}

// LDS table of the tiles one workgroup appends to (open addressing on the tile index).
constexpr int kBinSlots = 512;
constexpr int kBinKeep = 8;  // (triangle, tile) appends a thread remembers; more go straight to memory

// Chunk list entries: tile * 64 + c, c < kListedChunks a chunk of 64 listed triangles, c >=
// kListedChunks the (c - kListedChunks)-th of kListedChunks ranges of an overflowed tile's grid.
constexpr int kListedChunks = kFroxTileCap / kPartTris;  // 32
constexpr int kChunkCodes = 2 * kListedChunks;

// The chunk entries that the appends of slots [base, base + k) of a tile start: a chunk c begins
// at slot 64 c (listed slots only); the range holding slot kFroxTileCap (the first that does not
// fit) starts the tile's overflow ranges.
__device__ __forceinline__ int chunks_started(int base, int k) {
  const int end = min(base + k, kFroxTileCap);
  const int first = (base + kPartTris - 1) / kPartTris;
  const int listed = end > base ? max(0, (end - 1) / kPartTris - first + 1) : 0;
  const bool ovf = base <= kFroxTileCap && base + k > kFroxTileCap;
  return listed + (ovf ? kListedChunks : 0);
}
__device__ __forceinline__ void write_chunks(int tile, int base, int k, int32_t *__restrict__ chunks, int pos) {
  const int end = min(base + k, kFroxTileCap);
  for (int c = (base + kPartTris - 1) / kPartTris; c * kPartTris < end; ++c) chunks[pos++] = tile * kChunkCodes + c;
  if (base <= kFroxTileCap && base + k > kFroxTileCap)
    for (int c = 0; c < kListedChunks; ++c) chunks[pos++] = tile * kChunkCodes + kListedChunks + c;
}

__global__ __launch_bounds__(256) void frox_bin_kernel(const float *__restrict__ tris, Batch B, int64_t total,
                                                        TriSetup *__restrict__ recs, int32_t *__restrict__ tile_count,
                                                        int32_t *__restrict__ tile_list, int32_t *__restrict__ n_ignored,
                                                        int32_t *__restrict__ n_chunks, int32_t *__restrict__ chunks) {
  __shared__ int htile[kBinSlots];
  __shared__ int hcount[kBinSlots];
  __shared__ int hbase[kBinSlots];
  for (int i = threadIdx.x; i < kBinSlots; i += blockDim.x) {
    htile[i] = -1;
    hcount[i] = 0;
  }
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int ntl = 0, tx0 = 0, ty0 = 0, tz0 = 0, ntx = 1, nty = 1, toff = 0, tys = 1, txs = 1;
  bool bad = false;
  if (t < total) {
    const GridDesc &g = B.g[tri_grid(B, t)];
    TriSetup S = {};
    int32_t q[9], lo[3], hi[3];
    const bool empty = quantize_tri(tris, t, g, q, lo, hi, &bad);
    if (!empty) make_setup(q, S);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      S.lo[a] = (int16_t)(empty ? 1 : lo[a]);
      S.hi[a] = (int16_t)(empty ? 0 : hi[a]);
    }
    recs[t] = S;
    if (!empty) {
      tx0 = lo[0] / kFroxTileX;
      ty0 = lo[1] / kFroxTileY;
      tz0 = lo[2] / kFroxTileZ;
      ntx = hi[0] / kFroxTileX - tx0 + 1;
      nty = hi[1] / kFroxTileY - ty0 + 1;
      const int ntz = hi[2] / kFroxTileZ - tz0 + 1;
      ntl = ntx * nty * ntz;
      toff = g.tile_off;
      txs = g.tiles_x;
      tys = g.tiles_y;
    }
  }
  // ignored triangles: one counter update per wave that has any
  const uint64_t badm = __ballot(bad);
  if (n_ignored && badm && (threadIdx.x & 63) == 0) atomicAdd(n_ignored, (int)__popcll(badm));
  __syncthreads();  // the table is initialized
  // Appends are counted per workgroup first: each (triangle, tile) takes a local slot from the
  // tile's entry in the LDS table, then one global counter update per (workgroup, tile) reserves
  // the entry's range.  Consecutive triangles mostly share tiles, so a tile that hundreds of
  // triangles meet sees a few global updates instead of hundreds.  An append that finds no free
  // table entry, or a thread's appends past kBinKeep, take a global slot directly.
  auto tile_of = [&](int j) {
    const int ix = j % ntx, iy = (j / ntx) % nty, iz = j / (ntx * nty);
    return toff + ((tz0 + iz) * tys + (ty0 + iy)) * txs + (tx0 + ix);
  };
  auto append = [&](int tile, int slot) {
    if (slot < kFroxTileCap) tile_list[(int64_t)tile * kFroxTileCap + slot] = (int32_t)t;
  };
  // an append that reserved its slot alone lists the chunks it starts itself
  auto direct = [&](int tile) {
    const int slot = atomicAdd(&tile_count[tile], 1);
    append(tile, slot);
    if (chunks) {
      const int k = chunks_started(slot, 1);
      if (k) write_chunks(tile, slot, 1, chunks, atomicAdd(n_chunks, k));
    }
  };
  int kslot[kBinKeep], kent[kBinKeep];
#pragma unroll
  for (int j = 0; j < kBinKeep; ++j) {
    kent[j] = -1;
    kslot[j] = 0;
    if (j < ntl) {
      const int tile = tile_of(j);
      int h = (int)(((uint32_t)tile * 2654435761u) >> 23) & (kBinSlots - 1);
      for (int probe = 0; probe < kBinSlots; ++probe, h = (h + 1) & (kBinSlots - 1)) {
        const int cur = atomicCAS(&htile[h], -1, tile);
        if (cur == -1 || cur == tile) {
          kent[j] = h;
          kslot[j] = atomicAdd(&hcount[h], 1);
          break;
        }
      }
      if (kent[j] < 0) direct(tile);  // table full
    }
  }
  for (int j = kBinKeep; j < ntl; ++j) direct(tile_of(j));  // large triangles: the rest directly
  __syncthreads();
  // one counter update per table entry, then the chunks the workgroup's ranges start: one update
  // of the chunk count for the whole workgroup
  __shared__ int wsum[4];
  __shared__ int cbase;
  int nch[kBinSlots / 256] = {};
#pragma unroll
  for (int u = 0; u < kBinSlots / 256; ++u) {
    const int i = threadIdx.x + 256 * u;
    if (htile[i] >= 0) {
      hbase[i] = atomicAdd(&tile_count[htile[i]], hcount[i]);
      if (chunks) nch[u] = chunks_started(hbase[i], hcount[i]);
    }
  }
  if (chunks) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int mine = 0;
#pragma unroll
    for (int u = 0; u < kBinSlots / 256; ++u) mine += nch[u];
    int x = mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int pre = 0, tot = 0;
    for (int k = 0; k < 4; ++k) {
      pre += k < w ? wsum[k] : 0;
      tot += wsum[k];
    }
    if (threadIdx.x == 0) cbase = tot ? atomicAdd(n_chunks, tot) : 0;
    __syncthreads();
    int pos = cbase + pre + x - mine;
#pragma unroll
    for (int u = 0; u < kBinSlots / 256; ++u) {
      const int i = threadIdx.x + 256 * u;
      if (nch[u]) {
        write_chunks(htile[i], hbase[i], hcount[i], chunks, pos);
        pos += nch[u];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kBinKeep; ++j)
    if (kent[j] >= 0) append(htile[kent[j]], hbase[kent[j]] + kslot[j]);
}

// Froxels x in [xa, xb] of row (y, z) that the triangle meets, as bits x - X0 of a 32-bit word.
__device__ __forceinline__ uint32_t frox_row(const TriSetup &S, int xa, int xb, int y, int z, int X0) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {  // the edge x x-axis tests do not depend on x
    const int32_t s = S.e[i][2] * y - S.e[i][1] * z;
    if (s < S.L[i][0] || s > S.H[i][0]) return 0u;
  }
  int32_t sy[3], sz[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    sy[i] = -S.e[i][2] * xa + S.e[i][0] * z;
    sz[i] = S.e[i][1] * xa - S.e[i][0] * y;
  }
  int64_t sn = S.n[0] * xa + S.n[1] * y + S.n[2] * z;
  uint32_t m = 0;
  for (int x = xa; x <= xb; ++x) {
    bool hit = sn >= S.nL && sn <= S.nH;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      hit = hit && sy[i] >= S.L[i][1] && sy[i] <= S.H[i][1] && sz[i] >= S.L[i][2] && sz[i] <= S.H[i][2];
      sy[i] -= S.e[i][2];
      sz[i] += S.e[i][1];
    }
    sn += S.n[0];
    m |= (uint32_t)hit << (x - X0);
  }
  return m;
}

// Culling against a PVS.  A workgroup takes 256 triangles: each thread quantizes one and stages
// its overlap constants in LDS, a scan of the rows (y, z) each range covers gives a flat list of
// (triangle, row) items, and each thread tests one row at a time: the PVS word(s) of the row
// first, the exact overlap test only where a visible froxel lies in the range.  A hit sets the
// triangle's flag in LDS (a plain store of 1), and rows of flagged triangles are skipped.
__global__ __launch_bounds__(256) void visible_tris_kernel(const float *__restrict__ tris, Batch B, int64_t total,
                                                            const uint8_t *__restrict__ pvs,
                                                            uint8_t *__restrict__ visible) {
  __shared__ TriSetup srec[256];
  __shared__ int row0[257];
  __shared__ int wsum[4];
  __shared__ int gidx[256];
  __shared__ uint32_t flag[256];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int64_t base = (int64_t)blockIdx.x * 256; base < total; base += (int64_t)gridDim.x * 256) {
    const int64_t t = base + tid;
    int rows = 0;
    flag[tid] = 0;
    if (t < total) {
      const int b = tri_grid(B, t);
      int32_t q[9], lo[3], hi[3];
      TriSetup S = {};
      const bool empty = quantize_tri(tris, t, B.g[b], q, lo, hi);
      if (!empty) make_setup(q, S);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        S.lo[a] = (int16_t)(empty ? 1 : lo[a]);
        S.hi[a] = (int16_t)(empty ? 0 : hi[a]);
      }
      srec[tid] = S;
      gidx[tid] = b;
      if (!empty) rows = (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1);
    }
    int x = rows;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();  // also orders the previous chunk's reads before these writes
    int pre = 0;
    for (int k = 0; k < w; ++k) pre += wsum[k];
    row0[tid] = pre + x - rows;
    if (tid == 255) row0[256] = pre + x;
    __syncthreads();
    const int R = row0[256];
    const int n = total - base < 256 ? (int)(total - base) : 256;
    for (int r = tid; r < R; r += 256) {
      int lo = 0, hi = n - 1;  // last staged triangle whose rows start at or before r
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (row0[mid] <= r) lo = mid;
        else hi = mid - 1;
      }
      if (flag[lo]) continue;  // already visible
      const TriSetup &S = srec[lo];
      const GridDesc &g = B.g[gidx[lo]];
      const int rr = r - row0[lo], ny = S.hi[1] - S.lo[1] + 1;
      const int y = S.lo[1] + rr % ny, z = S.lo[2] + rr / ny;
      const uint8_t *row = pvs + g.occ_off + ((int64_t)z * g.ny + y) * (g.nx >> 3);
      for (int X0 = S.lo[0] & ~31; X0 <= S.hi[0]; X0 += 32) {
        const int xa = S.lo[0] > X0 ? S.lo[0] : X0, xb = S.hi[0] < X0 + 31 ? S.hi[0] : X0 + 31;
        uint32_t m = 0;  // PVS bits of froxels X0 .. X0 + 31 (bytes past the row read as 0)
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (X0 + 8 * k < g.nx) m |= (uint32_t)row[(X0 >> 3) + k] << (8 * k);
        m &= (xb - X0 == 31 ? ~0u : ((2u << (xb - X0)) - 1u)) & ~((1u << (xa - X0)) - 1u);
        if (m && (frox_row(S, xa, xb, y, z, X0) & m)) {
          flag[lo] = 1u;
          break;
        }
      }
    }
    __syncthreads();
    if (t < total) visible[t] = flag[tid] ? 1 : 0;
    __syncthreads();  // flags and staging are rewritten by the next chunk
  }
}

// One thread per object: OR of its triangles' flags.
__global__ __launch_bounds__(256) void visible_objects_kernel(const uint8_t *__restrict__ vis_tris,
                                                               const int64_t *__restrict__ obj_off, int64_t n_obj,
                                                               uint8_t *__restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_obj; i += (int64_t)gridDim.x * blockDim.x) {
    uint8_t v = 0;
    for (int64_t t = obj_off[i]; t < obj_off[i + 1] && !v; ++t) v = vis_tris[t];
    out[i] = v;
  }
}

__device__ __forceinline__ const GridDesc &tile_grid(const Batch &B, int tile) {
  int b = 0;
  while (b + 1 < B.n && tile >= B.g[b + 1].tile_off) ++b;
  return B.g[b];
}

__device__ __forceinline__ void tile_origin(const GridDesc &g, int tile, int &X0, int &Y0, int &Z0) {
  const int lt = tile - g.tile_off;
  X0 = (lt % g.tiles_x) * kFroxTileX;
  Y0 = ((lt / g.tiles_x) % g.tiles_y) * kFroxTileY;
  Z0 = (lt / (g.tiles_x * g.tiles_y)) * kFroxTileZ;
}

// Grid-stride over the chunk list, 256 threads per chunk: 64 of a tile's listed triangles, or
// (a tile whose list overflowed) one of kListedChunks ranges of its grid's triangles, 64 at a
// time; the listed chunks of an overflowed tile have nothing left to do.  A chunk's setup records
// go to LDS, a scan of the number of tile rows (y, z) each triangle covers gives a flat list of
// (triangle, row) items, and each thread tests the froxels of one row at a time (a short binary
// search over 64 row offsets finds an item's triangle).  Hits are OR-ed into the workgroup's
// 64-word mask in LDS and each non-zero word into the output (zeroed beforehand) with one atomic,
// so a tile that hundreds of triangles meet is spread over many workgroups.  Requires every
// grid's x extent to be a multiple of 32 (whole aligned words).
__global__ __launch_bounds__(256) void frox_part_kernel(Batch B, const TriSetup *__restrict__ recs,
                                                         const int32_t *__restrict__ tile_count,
                                                         const int32_t *__restrict__ tile_list,
                                                         const int32_t *__restrict__ n_chunks,
                                                         const int32_t *__restrict__ chunks,
                                                         uint8_t *__restrict__ occ) {
  __shared__ TriSetup srec[kPartTris];
  __shared__ int row0[kPartTris + 1];  // exclusive scan of the rows of the staged triangles
  __shared__ uint32_t mask[kTileWords];
  const int tid = threadIdx.x, lane = tid & 63;
  const int nc = *n_chunks;
  for (int ci = blockIdx.x; ci < nc; ci += gridDim.x) {
    const int code = chunks[ci];
    const int tile = code / kChunkCodes, c = code % kChunkCodes;
    const int cnt = tile_count[tile];
    const GridDesc &g = tile_grid(B, tile);
    const bool listed = cnt <= kFroxTileCap;
    if (listed != (c < kListedChunks)) continue;  // uniform: an overflowed tile's listed chunk
    int i0, i1;
    if (listed) {
      i0 = c * kPartTris;
      i1 = min(cnt, i0 + kPartTris);
    } else {
      const int per = (g.tri_n + kListedChunks - 1) / kListedChunks;
      i0 = (c - kListedChunks) * per;
      i1 = min(g.tri_n, i0 + per);
    }
    int X0, Y0, Z0;
    tile_origin(g, tile, X0, Y0, Z0);
    if (tid < kTileWords) mask[tid] = 0;
    for (int c0 = i0; c0 < i1; c0 += kPartTris) {
      const int n = min(kPartTris, i1 - c0);
      if (tid < 64) {  // wave 0 stages the triangles and scans their rows
        int rows = 0;
        if (lane < n) {
          const int64_t t = listed ? (int64_t)tile_list[(int64_t)tile * kFroxTileCap + c0 + lane] : g.tri_off + c0 + lane;
          const TriSetup S = recs[t];
          srec[lane] = S;
          const int xa = S.lo[0] > X0 ? S.lo[0] : X0, xb = S.hi[0] < X0 + 31 ? S.hi[0] : X0 + 31;
          const int ya = S.lo[1] > Y0 ? S.lo[1] : Y0, yb = S.hi[1] < Y0 + 7 ? S.hi[1] : Y0 + 7;
          const int za = S.lo[2] > Z0 ? S.lo[2] : Z0, zb = S.hi[2] < Z0 + 7 ? S.hi[2] : Z0 + 7;
          if (xa <= xb && ya <= yb && za <= zb) rows = (yb - ya + 1) * (zb - za + 1);
        }
        int x = rows;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const int y = __shfl_up(x, o, 64);
          if (lane >= o) x += y;
        }
        row0[lane] = x - rows;
        if (lane == 63) row0[kPartTris] = x;
      }
      __syncthreads();
      const int R = row0[kPartTris];
      for (int r = tid; r < R; r += 256) {
        int lo = 0, hi = n - 1;  // last staged triangle whose rows start at or before r
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (row0[mid] <= r) lo = mid;
          else hi = mid - 1;
        }
        const TriSetup &S = srec[lo];
        const int xa = S.lo[0] > X0 ? S.lo[0] : X0, xb = S.hi[0] < X0 + 31 ? S.hi[0] : X0 + 31;
        const int ya = S.lo[1] > Y0 ? S.lo[1] : Y0, yb = S.hi[1] < Y0 + 7 ? S.hi[1] : Y0 + 7;
        const int za = S.lo[2] > Z0 ? S.lo[2] : Z0;
        const int rr = r - row0[lo], ny = yb - ya + 1;
        const int y = ya + rr % ny, z = za + rr / ny;
        const uint32_t m = frox_row(S, xa, xb, y, z, X0);
        if (m) atomicOr(mask + (z - Z0) * 8 + (y - Y0), m);
      }
      __syncthreads();  // srec and row0 are rewritten by the next chunk; the mask is complete
    }
    if (tid < kTileWords) {
      const uint32_t word = mask[tid];
      const int y = Y0 + (tid & 7), z = Z0 + (tid >> 3);
      if (word && y < g.ny && z < g.nz)
        atomicOr(reinterpret_cast<uint32_t *>(occ + g.occ_off + ((int64_t)z * g.ny + y) * (g.nx / 8) + X0 / 8), word);
    }
    __syncthreads();  // the mask is cleared for the next chunk only after it has been read
  }
}

// One workgroup of 256 threads per tile: all of the tile's triangles, 256 at a time.  Their
// setup records go to LDS, a scan of the number of tile rows (y, z) each one covers gives a flat
// list of (triangle, row) items, and each thread tests the froxels of one row at a time, so a
// triangle that covers the whole tile costs 64 short rows spread over the workgroup rather than
// one long loop on one lane.  Hits are OR-ed into the tile's 64-word mask in LDS, and the tile's
// words are stored once at the end.  A tile whose list overflowed scans every triangle of its grid.
__global__ __launch_bounds__(256) void frox_tile_kernel(Batch B, const TriSetup *__restrict__ recs,
                                                         const int32_t *__restrict__ tile_count,
                                                         const int32_t *__restrict__ tile_list,
                                                         uint8_t *__restrict__ occ) {
  __shared__ TriSetup srec[256];
  __shared__ int row0[257];  // exclusive scan of the rows of the staged triangles
  __shared__ int wsum[4];
  __shared__ uint32_t mask[kTileWords];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int tile = blockIdx.x;
  const GridDesc &g = tile_grid(B, tile);
  const int cnt = tile_count[tile];
  const bool listed = cnt <= kFroxTileCap;
  const int items = listed ? cnt : g.tri_n;
  int X0, Y0, Z0;
  tile_origin(g, tile, X0, Y0, Z0);
  if (tid < kTileWords) mask[tid] = 0;
  for (int c0 = 0; c0 < items; c0 += 256) {
    const int i = c0 + tid;
    int rows = 0;
    if (i < items) {
      const int64_t t = listed ? (int64_t)tile_list[(int64_t)tile * kFroxTileCap + i] : g.tri_off + i;
      const TriSetup S = recs[t];
      srec[tid] = S;
      const int xa = S.lo[0] > X0 ? S.lo[0] : X0, xb = S.hi[0] < X0 + 31 ? S.hi[0] : X0 + 31;
      const int ya = S.lo[1] > Y0 ? S.lo[1] : Y0, yb = S.hi[1] < Y0 + 7 ? S.hi[1] : Y0 + 7;
      const int za = S.lo[2] > Z0 ? S.lo[2] : Z0, zb = S.hi[2] < Z0 + 7 ? S.hi[2] : Z0 + 7;
      if (xa <= xb && ya <= yb && za <= zb) rows = (yb - ya + 1) * (zb - za + 1);
    }
    int x = rows;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();  // also orders the previous chunk's reads of srec / row0 before these writes
    int pre = 0;
    for (int k = 0; k < w; ++k) pre += wsum[k];
    row0[tid] = pre + x - rows;
    if (tid == 255) row0[256] = pre + x;
    __syncthreads();
    const int R = row0[256];
    const int n = items - c0 < 256 ? items - c0 : 256;
    for (int r = tid; r < R; r += 256) {
      int lo = 0, hi = n - 1;  // last staged triangle whose rows start at or before r
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (row0[mid] <= r) lo = mid;
        else hi = mid - 1;
      }
      const TriSetup &S = srec[lo];
      const int xa = S.lo[0] > X0 ? S.lo[0] : X0, xb = S.hi[0] < X0 + 31 ? S.hi[0] : X0 + 31;
      const int ya = S.lo[1] > Y0 ? S.lo[1] : Y0, yb = S.hi[1] < Y0 + 7 ? S.hi[1] : Y0 + 7;
      const int za = S.lo[2] > Z0 ? S.lo[2] : Z0;
      const int rr = r - row0[lo], ny = yb - ya + 1;
      const int y = ya + rr % ny, z = za + rr / ny;
      const uint32_t m = frox_row(S, xa, xb, y, z, X0);
      if (m) atomicOr(mask + (z - Z0) * 8 + (y - Y0), m);
    }
    __syncthreads();  // srec and row0 are rewritten by the next chunk; the mask is complete
  }
  if (tid >= kTileWords) return;
  const uint32_t word = mask[tid];
  const int y = Y0 + (tid & 7), z = Z0 + (tid >> 3);
  if (y >= g.ny || z >= g.nz) return;
  const int64_t row_bytes = g.nx / 8;
  uint8_t *dst = occ + g.occ_off + ((int64_t)z * g.ny + y) * row_bytes + X0 / 8;
  if (X0 + 32 <= g.nx && (row_bytes & 3) == 0 && (g.occ_off & 3) == 0) {
    *reinterpret_cast<uint32_t *>(dst) = word;
  } else {
    for (int k = 0; k < 4 && X0 + 8 * k < g.nx; ++k) dst[k] = (uint8_t)(word >> (8 * k));
  }
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static void frox_ws_layout(const Batch &B, int64_t total_tris, size_t *off_count, size_t *off_list,
                           size_t *off_recs, size_t *bytes) {
  size_t o = 0;
  *off_count = o;  // tile counters, the chunk count, the chunk list
  o += align256(sizeof(int32_t) * ((size_t)B.total_tiles + 1 + (size_t)B.total_tiles * kChunkCodes));
  *off_list = o;
  o += align256(sizeof(int32_t) * (size_t)B.total_tiles * kFroxTileCap);
  *off_recs = o;
  o += align256(sizeof(TriSetup) * (size_t)(total_tris > 0 ? total_tris : 1));
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
                                      uint8_t *occ_bits, int32_t *n_ignored, void *ws, size_t ws_bytes, void *stream) {
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
  TriSetup *recs = reinterpret_cast<TriSetup *>(w + orr);
  hipStream_t s = as_stream(stream);
  // the parts path ORs whole aligned 32-froxel words into the output: every grid's x extent a
  // multiple of 32 (then every grid's bytes start on a 4-byte boundary too) and an aligned output
  bool parts = total > 0 && (reinterpret_cast<uintptr_t>(occ_bits) & 3) == 0;
  int64_t total_bytes = 0;
  for (int b = 0; b < n_grids; ++b) {
    parts = parts && dims[b].nx % 32 == 0;
    total_bytes += (int64_t)dims[b].nz * dims[b].ny * (dims[b].nx / 8);
  }
  const int64_t n_words = parts ? total_bytes / 4 : 0;
  int32_t *n_chunks = cnt + B.total_tiles, *chunks = n_chunks + 1;
  frox_zero_kernel<<<stride_grid(std::max<int64_t>(B.total_tiles + 1, n_words), 256, 1024), 256, 0, s>>>(
      cnt, B.total_tiles + 1, n_ignored, reinterpret_cast<uint32_t *>(occ_bits), n_words);
  if (total > 0)
    frox_bin_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(tris, B, total, recs, cnt, lst, n_ignored,
                                                                     parts ? n_chunks : nullptr,
                                                                     parts ? chunks : nullptr);
  if (parts)
    frox_part_kernel<<<stride_grid((int64_t)B.total_tiles * kChunkCodes, 1, 4096), 256, 0, s>>>(B, recs, cnt, lst,
                                                                                              n_chunks, chunks, occ_bits);
  else
    frox_tile_kernel<<<B.total_tiles, 256, 0, s>>>(B, recs, cnt, lst, occ_bits);
  return check_hip(hipGetLastError(), "npvs_froxelize");
}

extern "C" npvs_status npvs_visible_triangles(const float *tris, const int64_t *n_tris, int32_t n_grids,
                                              const npvs_dims *dims, const uint8_t *pvs_bits, uint8_t *visible,
                                              void *stream) {
  if (!n_tris || !pvs_bits) return fail(NPVS_ERR_INVALID_ARG, "npvs_visible_triangles: null pointer");
  Batch B;
  npvs_status st = make_batch(n_grids, dims, 1, n_tris, &B);
  if (st != NPVS_OK) return st;
  int64_t total = 0;
  for (int b = 0; b < n_grids; ++b) total += n_tris[b];
  if (total == 0) return NPVS_OK;
  if (!tris || !visible) return fail(NPVS_ERR_INVALID_ARG, "npvs_visible_triangles: null triangles or output");
  visible_tris_kernel<<<stride_grid(total, 256, 4096), 256, 0, as_stream(stream)>>>(tris, B, total, pvs_bits,
                                                                                      visible);
  return check_hip(hipGetLastError(), "npvs_visible_triangles");
}

extern "C" npvs_status npvs_visible_objects(const uint8_t *vis_tris, const int64_t *obj_off, int64_t n_objects,
                                            uint8_t *visible, void *stream) {
  if (n_objects < 0) return fail(NPVS_ERR_INVALID_ARG, "npvs_visible_objects: n_objects < 0");
  if (n_objects == 0) return NPVS_OK;
  if (!vis_tris || !obj_off || !visible) return fail(NPVS_ERR_INVALID_ARG, "npvs_visible_objects: null pointer");
  visible_objects_kernel<<<stride_grid(n_objects, 256, 4096), 256, 0, as_stream(stream)>>>(vis_tris, obj_off,
                                                                                           n_objects, visible);
  return check_hip(hipGetLastError(), "npvs_visible_objects");
}
