// World-space front end (Sec. 3.2): the frustum of a viewcell and the froxelization of
// world-space triangles into its froxels, with linear depth slices (the depth scaling the
// supplement's implementation notes use).
//
// Eye coordinates (x, y, z) = ((p - eye).right, (p - eye).up, (p - eye).forward).  Froxel
// (i, j, k) of an nx x ny x nz grid is the closed set with z in [zn + k s, zn + (k+1) s]
// (s = (zf - zn) / nz), x / z in [tx (2i/nx - 1), tx (2(i+1)/nx - 1)] and y / z likewise with ty.
// The map (X, Y, Q) = (x/z, y/z, 1/z) is projective on z > 0: a triangle clipped to z >= zn maps
// to a convex polygon and every froxel to an axis-aligned box.  The froxels of row (j, k) form
// the slab Y in [Y_j, Y_j+1], Q in [Q_k+1, Q_k] cut at the X boundaries, so the froxels the
// polygon meets in that row are exactly those whose closed X interval meets the X extent of the
// polygon clipped to the slab.  All geometry is in float64 on the device.
//
// Three launches: one thread per triangle (transform, near clip, map, froxel index box, number
// of (j, k) rows, and each workgroup's total), a scan of the row counts (each workgroup adds the
// totals before it), and one thread per (triangle, row) that clips the polygon to its slab and
// ORs the covered 32-froxel words.
#include <cmath>

#include "npvs_common.hpp"

namespace npvs {

struct WorldTri {  // the mapped polygon (at most 4 vertices after the near clip) and its box
  double P[4][3];
  int32_t n;
  int32_t i0, i1, j0, j1, k0, k1;
  int32_t pad;
};

struct ViewK {  // the view as the kernels take it
  double eye[3], right[3], up[3], fwd[3];
  double tx, ty, zn, zf;
};

__device__ __forceinline__ double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

__device__ __forceinline__ int clampi(double v, int hi) { return (int)(v < 0.0 ? 0.0 : (v > (double)hi ? (double)hi : v)); }

// One thread per triangle (grid ceil(T / 256)); each workgroup also writes its rows' total.
__global__ __launch_bounds__(256) void world_setup_kernel(const float *__restrict__ tris, int64_t T, ViewK V, int nx,
                                                          int ny, int nz, WorldTri *__restrict__ rec,
                                                          int32_t *__restrict__ rows, int64_t *__restrict__ wg_rows) {
  __shared__ int64_t red[256];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t my_rows = 0;
  if (t < T) {
    double e[3][3];
    bool finite = true;
    for (int v = 0; v < 3; ++v) {
      double d[3];
      for (int c = 0; c < 3; ++c) d[c] = (double)tris[(t * 3 + v) * 3 + c] - V.eye[c];
      e[v][0] = dot3(d, V.right);
      e[v][1] = dot3(d, V.up);
      e[v][2] = dot3(d, V.fwd);
      for (int c = 0; c < 3; ++c) finite = finite && __builtin_isfinite(e[v][c]);
    }
    WorldTri R = {};
    if (finite) {
      // keep z >= zn: each edge contributes its start if kept and its crossing if it crosses
      double q[4][3];
      int n = 0;
      for (int a = 0; a < 3; ++a) {
        const double *P = e[a], *Q = e[(a + 1) % 3];
        const double dp = P[2] - V.zn, dq = Q[2] - V.zn;
        if (dp >= 0.0) {
          q[n][0] = P[0], q[n][1] = P[1], q[n][2] = P[2];
          ++n;
        }
        if ((dp >= 0.0) != (dq >= 0.0)) {
          const double u = dp / (dp - dq);
          for (int c = 0; c < 3; ++c) q[n][c] = P[c] + u * (Q[c] - P[c]);
          ++n;
        }
      }
      if (n >= 3) {
        double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
        for (int a = 0; a < n; ++a) {
          R.P[a][0] = q[a][0] / q[a][2];
          R.P[a][1] = q[a][1] / q[a][2];
          R.P[a][2] = 1.0 / q[a][2];
          for (int c = 0; c < 3; ++c) {
            mn[c] = fmin(mn[c], R.P[a][c]);
            mx[c] = fmax(mx[c], R.P[a][c]);
          }
        }
        // froxel index box: froxel n spans [n, n + 1] in grid units and meets [a, b] iff
        // ceil(a) - 1 <= n <= floor(b) (closed); boxes wholly outside the grid are dropped
        const double s = (V.zf - V.zn) / nz;
        const double fi0 = ceil((mn[0] / V.tx + 1.0) * 0.5 * nx) - 1.0, fi1 = floor((mx[0] / V.tx + 1.0) * 0.5 * nx);
        const double fj0 = ceil((mn[1] / V.ty + 1.0) * 0.5 * ny) - 1.0, fj1 = floor((mx[1] / V.ty + 1.0) * 0.5 * ny);
        const double fk0 = ceil((1.0 / mx[2] - V.zn) / s) - 1.0, fk1 = floor((1.0 / mn[2] - V.zn) / s);
        if (fi1 >= 0.0 && fi0 <= nx - 1 && fj1 >= 0.0 && fj0 <= ny - 1 && fk1 >= 0.0 && fk0 <= nz - 1) {
          R.n = n;
          R.i0 = clampi(fi0, nx - 1), R.i1 = clampi(fi1, nx - 1);
          R.j0 = clampi(fj0, ny - 1), R.j1 = clampi(fj1, ny - 1);
          R.k0 = clampi(fk0, nz - 1), R.k1 = clampi(fk1, nz - 1);
        }
      }
    }
    rec[t] = R;
    my_rows = R.n ? (int64_t)(R.j1 - R.j0 + 1) * (R.k1 - R.k0 + 1) : 0;
    rows[t] = (int32_t)my_rows;
  }
  red[threadIdx.x] = my_rows;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) wg_rows[blockIdx.x] = red[0];
}

// Exclusive scan of rows[0, T) into off[0, T] (off[T] = total), one workgroup per 256 triangles:
// the workgroup adds the totals of the workgroups before it, then scans its own counts.
__global__ __launch_bounds__(256) void world_scan_kernel(const int32_t *__restrict__ rows,
                                                         const int64_t *__restrict__ wg_rows, int64_t T,
                                                         int64_t *__restrict__ off) {
  __shared__ int64_t sh[256];
  const int tid = threadIdx.x;
  int64_t carry = 0;
  for (int i = tid; i < (int)blockIdx.x; i += 256) carry += wg_rows[i];
  sh[tid] = carry;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) sh[tid] += sh[tid + w];
    __syncthreads();
  }
  carry = sh[0];
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * 256 + tid;
  const int64_t v = t < T ? rows[t] : 0;
  sh[tid] = v;
  __syncthreads();
  for (int d = 1; d < 256; d <<= 1) {  // inclusive Hillis-Steele scan
    const int64_t u = tid >= d ? sh[tid - d] : 0;
    __syncthreads();
    sh[tid] += u;
    __syncthreads();
  }
  if (t < T) off[t] = carry + sh[tid] - v;
  if (t == T - 1) off[T] = carry + sh[tid];
}

// Streaming Sutherland-Hodgman clip of a convex polygon by four planes (the row's slab), each
// stage keeping only its first and previous vertex and passing what it emits to the next stage;
// the last stage records the X extent.  No vertex arrays, so everything stays in registers.
struct V3 {
  double x, y, z;
};

struct ClipStage {
  V3 f, p;
  bool has;
};

struct SlabClip {  // stages 0, 1 cut Y at b0 (keep above) and b1 (keep below); 2, 3 cut Q likewise
  ClipStage s0, s1, s2, s3;
  double b0, b1, b2, b3;
  double xmin, xmax;

  template <int S>
  __device__ __forceinline__ ClipStage &stage() {
    if constexpr (S == 0) return s0;
    else if constexpr (S == 1) return s1;
    else if constexpr (S == 2) return s2;
    else return s3;
  }
  template <int S>
  __device__ __forceinline__ double side(V3 v) const {
    if constexpr (S == 0) return v.y - b0;
    else if constexpr (S == 1) return b1 - v.y;
    else if constexpr (S == 2) return v.z - b2;
    else return b3 - v.z;
  }
  template <int S>
  __device__ __forceinline__ void edge(V3 P, V3 Q) {  // stage S edge P -> Q
    const double dp = side<S>(P), dq = side<S>(Q);
    if ((dp >= 0.0) != (dq >= 0.0)) {
      const double u = dp / (dp - dq);
      push<S + 1>(V3{P.x + u * (Q.x - P.x), P.y + u * (Q.y - P.y), P.z + u * (Q.z - P.z)});
    }
    if (dq >= 0.0) push<S + 1>(Q);
  }
  template <int S>
  __device__ __forceinline__ void push(V3 v) {
    if constexpr (S == 4) {
      xmin = fmin(xmin, v.x);
      xmax = fmax(xmax, v.x);
    } else {
      ClipStage &c = stage<S>();
      if (!c.has) {
        c.has = true;
        c.f = v;
      } else {
        edge<S>(c.p, v);
      }
      c.p = v;
    }
  }
  template <int S>
  __device__ __forceinline__ void finish() {  // close stage S's polygon, then the next stage's
    if constexpr (S < 4) {
      if (stage<S>().has) edge<S>(stage<S>().p, stage<S>().f);
      finish<S + 1>();
    }
  }
};

__global__ __launch_bounds__(256) void world_rows_kernel(const WorldTri *__restrict__ rec, const int64_t *__restrict__ off,
                                                         int64_t T, ViewK V, int nx, int ny, int nz,
                                                         uint32_t *__restrict__ occ_words) {
  const int64_t total = off[T];
  const double s = (V.zf - V.zn) / nz;
  for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total; it += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = T - 1;  // the last triangle whose first row is <= it
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (off[mid] <= it) lo = mid;
      else hi = mid - 1;
    }
    const WorldTri &R = rec[lo];
    const int64_t r = it - off[lo];
    const int nj = R.j1 - R.j0 + 1;
    const int j = R.j0 + (int)(r % nj), k = R.k0 + (int)(r / nj);
    SlabClip C;
    C.s0.has = C.s1.has = C.s2.has = C.s3.has = false;
    C.b0 = V.ty * (2.0 * j / ny - 1.0);
    C.b1 = V.ty * (2.0 * (j + 1) / ny - 1.0);
    C.b2 = 1.0 / (V.zn + (k + 1) * s);
    C.b3 = 1.0 / (V.zn + k * s);
    C.xmin = 1e300, C.xmax = -1e300;
    C.push<0>(V3{R.P[0][0], R.P[0][1], R.P[0][2]});
    C.push<0>(V3{R.P[1][0], R.P[1][1], R.P[1][2]});
    C.push<0>(V3{R.P[2][0], R.P[2][1], R.P[2][2]});
    if (R.n > 3) C.push<0>(V3{R.P[3][0], R.P[3][1], R.P[3][2]});
    C.finish<0>();
    if (C.xmin > C.xmax) continue;  // nothing of the polygon in this row's slab
    const double xmin = C.xmin, xmax = C.xmax;
    // froxel i spans [i, i + 1] in u = (X / tx + 1) nx / 2 and meets [umin, umax] iff
    // ceil(umin) - 1 <= i <= floor(umax)
    const double umin = (xmin / V.tx + 1.0) * 0.5 * nx, umax = (xmax / V.tx + 1.0) * 0.5 * nx;
    const double fa = ceil(umin) - 1.0, fb = floor(umax);
    if (fb < 0.0 || fa > nx - 1) continue;
    const int ia = fa < 0.0 ? 0 : (int)fa, ib = fb > nx - 1 ? nx - 1 : (int)fb;
    uint32_t *row = occ_words + ((int64_t)k * ny + j) * (nx >> 5);
    for (int w = ia >> 5; w <= (ib >> 5); ++w) {
      const int b0 = ia > 32 * w ? ia - 32 * w : 0, b1 = ib < 32 * w + 31 ? ib - 32 * w : 31;
      const uint32_t mask = (b1 == 31 ? ~0u : ((1u << (b1 + 1)) - 1u)) & ~((1u << b0) - 1u);
      atomicOr(row + w, mask);
    }
  }
}

__global__ void world_zero_kernel(uint32_t *__restrict__ w, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) w[i] = 0u;
}

static size_t align256w(size_t x) { return (x + 255) & ~(size_t)255; }

static void world_ws_layout(int64_t T, size_t *o_rec, size_t *o_rows, size_t *o_off, size_t *o_wg, size_t *bytes) {
  size_t o = 0;
  *o_rec = o;
  o += align256w(sizeof(WorldTri) * (size_t)(T > 0 ? T : 1));
  *o_rows = o;
  o += align256w(sizeof(int32_t) * (size_t)(T > 0 ? T : 1));
  *o_off = o;
  o += align256w(sizeof(int64_t) * (size_t)(T + 1));
  *o_wg = o;
  o += align256w(sizeof(int64_t) * (size_t)((T + 255) / 256 + 1));
  *bytes = o;
}

}  // namespace npvs

using namespace npvs;

extern "C" npvs_status npvs_viewcell_frustum(const double *c, const double *forward, const double *up, double fov_y,
                                            double aspect, double r, double beta, double z_near, double z_far,
                                            npvs_view *out) {
  if (!c || !forward || !up || !out) return fail(NPVS_ERR_INVALID_ARG, "npvs_viewcell_frustum: null pointer");
  if (!(fov_y > 0.0) || !(fov_y + 2.0 * beta < 3.14159265358979) || !(aspect > 0.0) || !(r >= 0.0) ||
      !(beta >= 0.0) || !(z_near > 0.0) || !(z_far > z_near))
    return fail(NPVS_ERR_INVALID_ARG, "npvs_viewcell_frustum: bad camera parameters");
  double f[3] = {forward[0], forward[1], forward[2]};
  const double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  if (!(fl > 0.0)) return fail(NPVS_ERR_INVALID_ARG, "npvs_viewcell_frustum: zero forward vector");
  for (double &x : f) x /= fl;
  // right = up x forward, then the up vector orthogonal to both
  double rt[3] = {up[1] * f[2] - up[2] * f[1], up[2] * f[0] - up[0] * f[2], up[0] * f[1] - up[1] * f[0]};
  const double rl = std::sqrt(rt[0] * rt[0] + rt[1] * rt[1] + rt[2] * rt[2]);
  if (!(rl > 1e-12 * std::sqrt(up[0] * up[0] + up[1] * up[1] + up[2] * up[2])))
    return fail(NPVS_ERR_INVALID_ARG, "npvs_viewcell_frustum: up is parallel to forward");
  for (double &x : rt) x /= rl;
  const double u[3] = {f[1] * rt[2] - f[2] * rt[1], f[2] * rt[0] - f[0] * rt[2], f[0] * rt[1] - f[1] * rt[0]};
  const double back = r / std::tan(fov_y / 2.0);  // the apex sits this far behind the camera
  for (int i = 0; i < 3; ++i) {
    out->eye[i] = c[i] - back * f[i];
    out->right[i] = rt[i];
    out->up[i] = u[i];
    out->forward[i] = f[i];
  }
  out->tan_half_y = std::tan((fov_y + 2.0 * beta) / 2.0);
  out->tan_half_x = aspect * out->tan_half_y;
  out->z_near = z_near;
  out->z_far = z_far;
  return NPVS_OK;
}

extern "C" npvs_status npvs_froxelize_view_workspace_size(int64_t n_tris, size_t *bytes) {
  if (!bytes || n_tris < 0) return fail(NPVS_ERR_INVALID_ARG, "npvs_froxelize_view_workspace_size: bad arguments");
  size_t a, b, c, d;
  world_ws_layout(n_tris, &a, &b, &c, &d, bytes);
  return NPVS_OK;
}

extern "C" npvs_status npvs_froxelize_view(const float *tris, int64_t n_tris, const npvs_view *view, npvs_dims g,
                                          uint8_t *occ_bits, void *ws, size_t ws_bytes, void *stream) {
  if (!view || !occ_bits || !ws || (n_tris > 0 && !tris)) return fail(NPVS_ERR_INVALID_ARG, "npvs_froxelize_view: null pointer");
  if (n_tris < 0 || n_tris > INT32_MAX) return fail(NPVS_ERR_INVALID_ARG, "npvs_froxelize_view: bad triangle count");
  if (g.nx < 32 || g.nx % 32 || g.ny < 1 || g.nz < 1 || g.nx > NPVS_MAX_DIM || g.ny > NPVS_MAX_DIM || g.nz > NPVS_MAX_DIM)
    return fail(NPVS_ERR_INVALID_ARG, "npvs_froxelize_view: nx must be a multiple of 32, extents in [1, 1024]");
  if ((reinterpret_cast<uintptr_t>(occ_bits) & 3))
    return fail(NPVS_ERR_INVALID_ARG, "npvs_froxelize_view: occ_bits must be 4-byte aligned");
  if (!(view->z_near > 0.0) || !(view->z_far > view->z_near) || !(view->tan_half_x > 0.0) || !(view->tan_half_y > 0.0))
    return fail(NPVS_ERR_INVALID_ARG, "npvs_froxelize_view: bad view");
  size_t o_rec, o_rows, o_off, o_wg, need;
  world_ws_layout(n_tris, &o_rec, &o_rows, &o_off, &o_wg, &need);
  if (ws_bytes < need) return fail(NPVS_ERR_INVALID_ARG, "npvs_froxelize_view: workspace too small");
  char *w = static_cast<char *>(ws);
  WorldTri *rec = reinterpret_cast<WorldTri *>(w + o_rec);
  int32_t *rows = reinterpret_cast<int32_t *>(w + o_rows);
  int64_t *off = reinterpret_cast<int64_t *>(w + o_off);
  int64_t *wg_rows = reinterpret_cast<int64_t *>(w + o_wg);
  ViewK V;
  for (int i = 0; i < 3; ++i) {
    V.eye[i] = view->eye[i];
    V.right[i] = view->right[i];
    V.up[i] = view->up[i];
    V.fwd[i] = view->forward[i];
  }
  V.tx = view->tan_half_x, V.ty = view->tan_half_y, V.zn = view->z_near, V.zf = view->z_far;
  hipStream_t s = as_stream(stream);
  const int64_t words = (int64_t)g.nz * g.ny * (g.nx / 32);
  world_zero_kernel<<<stride_grid(words, 256, 4096), 256, 0, s>>>(reinterpret_cast<uint32_t *>(occ_bits), words);
  if (n_tris > 0) {
    const int nwg = (int)((n_tris + 255) / 256);
    world_setup_kernel<<<nwg, 256, 0, s>>>(tris, n_tris, V, g.nx, g.ny, g.nz, rec, rows, wg_rows);
    world_scan_kernel<<<nwg, 256, 0, s>>>(rows, wg_rows, n_tris, off);
    world_rows_kernel<<<4096, 256, 0, s>>>(rec, off, n_tris, V, g.nx, g.ny, g.nz,
                                          reinterpret_cast<uint32_t *>(occ_bits));
  }
  return check_hip(hipGetLastError(), "npvs_froxelize_view");
}
