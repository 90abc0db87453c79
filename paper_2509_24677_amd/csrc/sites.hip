// Active sites and the submanifold rulebook (Sec. 2.3: sparse tensors store only sites with
// geometry and the submanifold kernel is centred on active sites only).
//
// The site lookup table is direct-indexed: block_row[global key] = row or -1.  On a GPU with
// 288 GB of HBM a table of 4 bytes per block (512 KB for a 64 x 64 x 32 block grid) is a
// perfect hash: one load per probe, no collisions, and it stays resident in L2.
//
// Rows are numbered by ascending global key through a two-pass compaction (per-workgroup
// counts, then every workgroup adds the counts of the workgroups before it and scans its own
// flags), so the numbering is canonical and identical run to run.
#include <mutex>
#include <string>

#include "npvs_common.hpp"

namespace npvs {

// Exclusive scan of one int per thread over a 256-thread workgroup (4 waves of 64).
__device__ __forceinline__ int block_exclusive_scan(int v, int *total) {
  __shared__ int wsum[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  __syncthreads();
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int pre = 0;
  for (int i = 0; i < w; ++i) pre += wsum[i];
  *total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
  return pre + x - v;
}

__device__ __forceinline__ int block_sum(int v) {
  int t;
  block_exclusive_scan(v, &t);
  return t;
}

// Each thread tests BPT consecutive blocks (global keys).  When every grid has nx % 32 == 0 the
// BPT = 32 / d blocks of a thread share one 32-froxel span of their rows, so the thread ORs d*d
// dword loads and splits the word into block flags; otherwise BPT = 4 and each block is tested
// byte by byte.
__device__ __forceinline__ int block_active(const Batch &B, const uint8_t *__restrict__ occ, int32_t gb) {
  if (gb >= B.total_blocks) return 0;
  const GridDesc &g = B.g[grid_of_key(B, gb)];
  const int d = B.d;
  int32_t l = gb - g.key_off;
  int bx = l % g.Bx, by = (l / g.Bx) % g.By, bz = l / (g.Bx * g.By);
  const int64_t row_bytes = g.nx >> 3;
  const int x0 = bx * d, x1 = x0 + d - 1;
  const uint8_t *base = occ + g.occ_off;
  int any = 0;
  for (int oz = 0; oz < d; ++oz)
    for (int oy = 0; oy < d; ++oy) {
      const uint8_t *row = base + ((int64_t)(bz * d + oz) * g.ny + (by * d + oy)) * row_bytes;
      for (int xb = x0 >> 3; xb <= (x1 >> 3); ++xb) {
        int lo = xb * 8 > x0 ? 0 : x0 - xb * 8;
        int hi = xb * 8 + 7 < x1 ? 7 : x1 - xb * 8;
        unsigned mask = ((2u << hi) - 1u) & ~((1u << lo) - 1u);
        any |= row[xb] & mask;
      }
    }
  return any != 0;
}

// Bit i of the result = activity of block gb0 + i, i < bpt.
__device__ __forceinline__ uint32_t thread_flags(const Batch &B, const uint8_t *__restrict__ occ, int32_t gb0,
                                                 int bpt, int fast) {
  if (gb0 >= B.total_blocks) return 0u;
  if (!fast) {
    uint32_t f = 0;
    for (int i = 0; i < bpt; ++i) f |= (uint32_t)block_active(B, occ, gb0 + i) << i;
    return f;
  }
  const GridDesc &g = B.g[grid_of_key(B, gb0)];
  const int d = B.d;
  const int32_t l = gb0 - g.key_off;
  const int bx = l % g.Bx, by = (l / g.Bx) % g.By, bz = l / (g.Bx * g.By);
  const int64_t row_words = g.nx >> 5;
  const uint32_t *base = reinterpret_cast<const uint32_t *>(occ + g.occ_off) + (bx * d >> 5);
  uint32_t w = 0;
  for (int oz = 0; oz < d; ++oz)
    for (int oy = 0; oy < d; ++oy) w |= base[((int64_t)(bz * d + oz) * g.ny + (by * d + oy)) * row_words];
  if (d == 32) return w != 0u;
  const uint32_t m = (1u << d) - 1u;
  uint32_t f = 0;
  for (int i = 0; i < bpt; ++i) f |= (uint32_t)(((w >> (i * d)) & m) != 0u) << i;
  return f;
}

__global__ __launch_bounds__(256) void sites_count_kernel(Batch B, const uint8_t *__restrict__ occ, int bpt, int fast,
                                                           int32_t *__restrict__ wg_counts) {
  const int32_t gb0 = (blockIdx.x * 256 + threadIdx.x) * bpt;
  int t = block_sum(__popc(thread_flags(B, occ, gb0, bpt, fast)));
  if (threadIdx.x == 0) wg_counts[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void sites_write_kernel(Batch B, const uint8_t *__restrict__ occ, int bpt, int fast,
                                                           const int32_t *__restrict__ wg_counts, int32_t cap,
                                                           npvs_counts *__restrict__ counts,
                                                           int32_t *__restrict__ site_keys,
                                                           int32_t *__restrict__ block_row,
                                                           int32_t *__restrict__ grid_rows) {
  // rows before this workgroup
  int part = 0;
  for (int i = threadIdx.x; i < (int)blockIdx.x; i += 256) part += wg_counts[i];
  const int prefix = block_sum(part);
  const int32_t gb0 = (blockIdx.x * 256 + threadIdx.x) * bpt;
  const uint32_t f = thread_flags(B, occ, gb0, bpt, fast);
  int wg_total;
  int pos = prefix + block_exclusive_scan(__popc(f), &wg_total);
  for (int i = 0; i < bpt; ++i) {
    const int32_t gb = gb0 + i;
    if (gb >= B.total_blocks) break;
    const int b = grid_of_key(B, gb);
    if (gb == B.g[b].key_off) grid_rows[b] = pos < cap ? pos : cap;
    const int fi = (f >> i) & 1;
    if (fi && pos < cap) {
      site_keys[pos] = gb;
      block_row[gb] = pos;
    } else {
      block_row[gb] = -1;
    }
    pos += fi;
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    const int total = prefix + wg_total;
    const int stored = total < cap ? total : cap;
    counts->n_sites = stored;
    counts->n_sites_needed = total;
    counts->n_pairs = 0;
    grid_rows[B.n] = stored;
  }
}

// Neighbour of row r through offset k, or -1.
__device__ __forceinline__ int32_t neighbor_row(const Batch &B, const int32_t *__restrict__ site_keys,
                                                const int32_t *__restrict__ block_row, int32_t r, int k) {
  int32_t key = site_keys[r];
  const GridDesc &g = B.g[grid_of_key(B, key)];
  int32_t l = key - g.key_off;
  int bx = l % g.Bx + (k % 3 - 1);
  int by = (l / g.Bx) % g.By + ((k / 3) % 3 - 1);
  int bz = l / (g.Bx * g.By) + (k / 9 - 1);
  if (bx < 0 || by < 0 || bz < 0 || bx >= g.Bx || by >= g.By || bz >= g.Bz) return -1;
  return block_row[g.key_off + (bz * g.By + by) * g.Bx + bx];
}

constexpr int kRowsPerChunk = 1024;

// grid (chunks, 27): neighbour map for offset k = blockIdx.y, and per-chunk pair counts.
__global__ __launch_bounds__(256) void rulebook_nbr_kernel(Batch B, const int32_t *__restrict__ site_keys,
                                                            const int32_t *__restrict__ block_row,
                                                            const npvs_counts *__restrict__ counts, int32_t cap,
                                                            int32_t *__restrict__ nbr,
                                                            int32_t *__restrict__ chunk_counts, int32_t n_chunks) {
  const int k = blockIdx.y;
  const int32_t n = counts->n_sites;
  const int used_chunks = (n + kRowsPerChunk - 1) / kRowsPerChunk;
  for (int ch = blockIdx.x; ch < used_chunks; ch += gridDim.x) {
    int c = 0;
    for (int i = 0; i < 4; ++i) {
      int32_t r = ch * kRowsPerChunk + i * 256 + threadIdx.x;
      if (r < n) {
        int32_t v = neighbor_row(B, site_keys, block_row, r, k);
        nbr[(int64_t)k * cap + r] = v;
        c += v >= 0;
      }
    }
    if (chunk_counts) {
      int t = block_sum(c);
      if (threadIdx.x == 0) chunk_counts[k * n_chunks + ch] = t;
    }
  }
}

// Pair lists (CSR by offset): the pairs of offset k and chunk ch start after every pair of the
// (offset, chunk) items before it in offset-major order; each workgroup adds those items' counts
// itself (27 x 10 at most for a city frame), so no separate scan launch is needed.  The workgroup
// of each offset's first chunk writes rb_off[k], that of the last item rb_off[27] and the count.
__global__ __launch_bounds__(256) void rulebook_pairs_kernel(npvs_counts *__restrict__ counts, int32_t cap,
                                                              const int32_t *__restrict__ nbr,
                                                              const int32_t *__restrict__ chunk_counts,
                                                              int32_t n_chunks, int32_t *__restrict__ rb_off,
                                                              int32_t *__restrict__ pairs) {
  const int k = blockIdx.y;
  const int32_t n = counts->n_sites;
  const int used = (n + kRowsPerChunk - 1) / kRowsPerChunk;
  if (used == 0) {
    if (blockIdx.x == 0 && k == 0 && threadIdx.x < 28) {
      rb_off[threadIdx.x] = 0;
      if (threadIdx.x == 0) counts->n_pairs = 0;
    }
    return;
  }
  for (int ch = blockIdx.x; ch < used; ch += gridDim.x) {
    // pairs before this item: chunks of the offsets before k, then the chunks of k before ch
    const int before = k * used + ch;
    int part = 0;
    for (int i = threadIdx.x; i < before; i += 256) part += chunk_counts[(i / used) * n_chunks + i % used];
    const int base = block_sum(part);
    // 4 consecutive rows per thread keep the output ascending in row order
    int32_t r0 = ch * kRowsPerChunk + threadIdx.x * 4;
    int32_t v[4];
    int c = 0;
    for (int i = 0; i < 4; ++i) {
      v[i] = r0 + i < n ? nbr[(int64_t)k * cap + r0 + i] : -1;
      c += v[i] >= 0;
    }
    int tot;
    int pos = base + block_exclusive_scan(c, &tot);
    if (threadIdx.x == 0) {
      if (ch == 0) rb_off[k] = base;
      if (k == 26 && ch == used - 1) {
        rb_off[27] = base + tot;
        counts->n_pairs = base + tot;
      }
    }
    for (int i = 0; i < 4; ++i)
      if (v[i] >= 0) {
        pairs[2 * (int64_t)pos] = v[i];
        pairs[2 * (int64_t)pos + 1] = r0 + i;
        ++pos;
      }
    __syncthreads();
  }
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Blocks per thread of the site kernels and whether the 32-froxel span path applies.
static void sites_shape(const Batch &B, int *bpt, int *fast) {
  bool all32 = B.d <= 32;
  for (int b = 0; b < B.n; ++b) all32 = all32 && (B.g[b].nx % 32 == 0);
  *fast = all32 ? 1 : 0;
  *bpt = all32 ? 32 / B.d : 4;
}

static void rb_ws_layout(const Batch &B, int32_t cap, size_t *o_wg, size_t *o_cc, size_t *bytes, int *n_wg,
                         int *n_chunks) {
  int bpt, fast;
  sites_shape(B, &bpt, &fast);
  *n_wg = (B.total_blocks + 256 * bpt - 1) / (256 * bpt);
  *n_chunks = (cap + kRowsPerChunk - 1) / kRowsPerChunk;
  size_t o = 0;
  *o_wg = o;
  o += align256(sizeof(int32_t) * (size_t)(*n_wg > 0 ? *n_wg : 1));
  *o_cc = o;
  o += align256(sizeof(int32_t) * 27 * (size_t)(*n_chunks > 0 ? *n_chunks : 1));
  *bytes = o;
}

}  // namespace npvs

using namespace npvs;

extern "C" npvs_status npvs_rulebook_workspace_size(int32_t n_grids, const npvs_dims *dims, int32_t d,
                                                    int32_t cap_sites, size_t *bytes) {
  if (!bytes) return fail(NPVS_ERR_INVALID_ARG, "npvs_rulebook_workspace_size: null pointer");
  Batch B;
  npvs_status st = make_batch(n_grids, dims, d, nullptr, &B);
  if (st != NPVS_OK) return st;
  if (cap_sites < 1) return fail(NPVS_ERR_INVALID_ARG, "npvs_rulebook_workspace_size: cap_sites < 1");
  size_t a, b;
  int nw, nc;
  rb_ws_layout(B, cap_sites, &a, &b, bytes, &nw, &nc);
  return NPVS_OK;
}

// The rulebook build proper; `ws` is caller memory (npvs_build_rulebook) or this file's scratch
// array (npvs_build_rulebook_noalloc).  Every workspace word is written before it is read.
static npvs_status build_rulebook_impl(const char *fn, const uint8_t *occ_bits, int32_t n_grids,
                                       const npvs_dims *dims, int32_t d, int32_t cap_sites, npvs_counts *counts,
                                       int32_t *site_keys, int32_t *block_row, int32_t *grid_rows, int32_t *nbr,
                                       int32_t *rb_off, int32_t *rb_pairs, void *ws, size_t ws_bytes,
                                       void *stream) {
  if (!occ_bits || !counts || !site_keys || !block_row || !grid_rows || !nbr || !ws)
    return fail(NPVS_ERR_INVALID_ARG, std::string(fn) + ": null pointer");
  if ((rb_off == nullptr) != (rb_pairs == nullptr))
    return fail(NPVS_ERR_INVALID_ARG, std::string(fn) + ": give both rb_off and rb_pairs or neither");
  Batch B;
  npvs_status st = make_batch(n_grids, dims, d, nullptr, &B);
  if (st != NPVS_OK) return st;
  if (cap_sites < 1) return fail(NPVS_ERR_INVALID_ARG, std::string(fn) + ": cap_sites < 1");
  if ((int64_t)cap_sites * 27 > INT32_MAX) return fail(NPVS_ERR_INVALID_ARG, std::string(fn) + ": cap_sites too large");
  size_t o_wg, o_cc, need;
  int n_wg, n_chunks;
  rb_ws_layout(B, cap_sites, &o_wg, &o_cc, &need, &n_wg, &n_chunks);
  if (ws_bytes < need)
    return fail(NPVS_ERR_INVALID_ARG, std::string(fn) + ": workspace too small (" + std::to_string(need) +
                                          " bytes needed, " + std::to_string(ws_bytes) + " given)");
  char *w = static_cast<char *>(ws);
  int32_t *wg_counts = reinterpret_cast<int32_t *>(w + o_wg);
  int32_t *chunk_counts = reinterpret_cast<int32_t *>(w + o_cc);
  hipStream_t s = as_stream(stream);
  int bpt, fast;
  sites_shape(B, &bpt, &fast);
  sites_count_kernel<<<n_wg, 256, 0, s>>>(B, occ_bits, bpt, fast, wg_counts);
  sites_write_kernel<<<n_wg, 256, 0, s>>>(B, occ_bits, bpt, fast, wg_counts, cap_sites, counts, site_keys, block_row,
                                          grid_rows);
  dim3 g(stride_grid(cap_sites, kRowsPerChunk, 512), 27);
  rulebook_nbr_kernel<<<g, 256, 0, s>>>(B, site_keys, block_row, counts, cap_sites, nbr,
                                        rb_off ? chunk_counts : nullptr, n_chunks);
  if (rb_off) rulebook_pairs_kernel<<<g, 256, 0, s>>>(counts, cap_sites, nbr, chunk_counts, n_chunks, rb_off, rb_pairs);
  return check_hip(hipGetLastError(), fn);
}

extern "C" npvs_status npvs_build_rulebook(const uint8_t *occ_bits, int32_t n_grids, const npvs_dims *dims, int32_t d,
                                           int32_t cap_sites, npvs_counts *counts, int32_t *site_keys,
                                           int32_t *block_row, int32_t *grid_rows, int32_t *nbr, int32_t *rb_off,
                                           int32_t *rb_pairs, void *ws, size_t ws_bytes, void *stream) {
  return build_rulebook_impl("npvs_build_rulebook", occ_bits, n_grids, dims, d, cap_sites, counts, site_keys,
                             block_row, grid_rows, nbr, rb_off, rb_pairs, ws, ws_bytes, stream);
}

// ---------------------------------------------------------------------------------------------
// The same build without caller workspace: the workspace is this file-scope device array, one
// copy per GPU, held until the process ends.  In host code `scratch` names a host-side stand-in,
// not device memory: its device address is taken once per device with hipGetSymbolAddress and
// only that address is ever handed to a kernel.  Calls that overlap on one GPU share the array
// and race; nothing in it needs to start at zero.
static __device__ __align__(256) unsigned char scratch[NPVS_RULEBOOK_SCRATCH_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxScratchDevices] = {};

npvs_status scratch_address(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return check_hip(e, "npvs_build_rulebook_noalloc: hipGetDevice");
  if (dev < 0 || dev >= kMaxScratchDevices)
    return fail(NPVS_ERR_UNSUPPORTED, "npvs_build_rulebook_noalloc: device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return check_hip(e, "npvs_build_rulebook_noalloc: hipGetSymbolAddress");
    if (!p) return fail(NPVS_ERR_HIP, "npvs_build_rulebook_noalloc: hipGetSymbolAddress gave a null address");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return NPVS_OK;
}
}  // namespace

extern "C" npvs_status npvs_build_rulebook_noalloc(const uint8_t *occ_bits, int32_t n_grids, const npvs_dims *dims,
                                                   int32_t d, int32_t cap_sites, npvs_counts *counts,
                                                   int32_t *site_keys, int32_t *block_row, int32_t *grid_rows,
                                                   int32_t *nbr, int32_t *rb_off, int32_t *rb_pairs, void *stream) {
  // sizes first: an oversized request is refused before anything touches the device
  Batch B;
  npvs_status st = make_batch(n_grids, dims, d, nullptr, &B);
  if (st != NPVS_OK) return st;
  if (cap_sites < 1) return fail(NPVS_ERR_INVALID_ARG, "npvs_build_rulebook_noalloc: cap_sites < 1");
  size_t o_wg, o_cc, need;
  int n_wg, n_chunks;
  rb_ws_layout(B, cap_sites, &o_wg, &o_cc, &need, &n_wg, &n_chunks);
  if (need > NPVS_RULEBOOK_SCRATCH_BYTES)
    return fail(NPVS_ERR_CAPACITY, "npvs_build_rulebook_noalloc: this batch needs " + std::to_string(need) +
                                       " bytes of workspace, beyond the " +
                                       std::to_string((size_t)NPVS_RULEBOOK_SCRATCH_BYTES) +
                                       "-byte scratch; use npvs_build_rulebook with a workspace");
  void *ws = nullptr;
  st = scratch_address(&ws);
  if (st != NPVS_OK) return st;
  return build_rulebook_impl("npvs_build_rulebook_noalloc", occ_bits, n_grids, dims, d, cap_sites, counts,
                             site_keys, block_row, grid_rows, nbr, rb_off, rb_pairs, ws,
                             NPVS_RULEBOOK_SCRATCH_BYTES, stream);
}
