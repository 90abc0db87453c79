/*
 * NeuralPVS CPU oracle.  TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU implementation of what the visibility network's forward
 * path computes (froxelize -> interleave -> submanifold sparse 3x3x3 convolutions ->
 * deinterleave -> threshold), plus the loss, its gradient, the convolution backward, Adam and a
 * ray-march visibility labeller.  Floating point is FP64; froxel overlap is exact integer
 * arithmetic.  It shares no code with the HIP library: only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it.
 *
 * Conventions (the paper writes the domain 1-based and leaves memory order open):
 *   froxel (x, y, z) 0-based, x fastest; packed grid uint8 [nz][ny][nx/8], bit (x & 7) of byte
 *   x >> 3 (LSB = lowest x); block (bx, by, bz) of d^3 froxels, key = (bz*By + by)*Bx + bx;
 *   channel c = (oz*d + oy)*d + ox; conv offset k = (dz+1)*9 + (dy+1)*3 + (dx+1) and
 *   Y[p] += X[p + delta_k] W_k (cross-correlation).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define FX 256 /* fixed-point scale: 1/256 froxel */
/* Representation bound of the exact overlap test: |v| < 2048 froxels with 8 fractional bits gives
 * fixed-point coordinates below 2^19, so every separating-axis projection is a sum of three
 * products below 2^61 and fits int64.  It bounds how large a triangle can be, not where the grid
 * is: a triangle that reaches far outside the grid still marks every froxel it meets. */
#define COORD_LIMIT 2048.0

static int64_t floordiv(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) q--;
  return q;
}
static int64_t min3(int64_t a, int64_t b, int64_t c) { int64_t m = a < b ? a : b; return m < c ? m : c; }
static int64_t max3(int64_t a, int64_t b, int64_t c) { int64_t m = a > b ? a : b; return m > c ? m : c; }

/* ------------------------------------------------------------------------------------------
 * Froxelization (Sec. 3.2, pre-processing; Fig. 2(b)): G(x) = 1 iff some triangle overlaps
 * froxel x.  The paper rasterizes "conservatively"; the exact reading used here is
 * closed-box / triangle intersection, decided by the separating-axis theorem on vertices
 * quantized to 1/256 froxel with round-half-to-even.  All predicates are exact in int64.
 * ------------------------------------------------------------------------------------------ */

/* Quantize one triangle.  Returns 0 when a coordinate is non-finite or |v| >= 2048 froxels
 * (such triangles are ignored, and counted by oracle_froxelize). */
int oracle_quantize_tri(const float *t, int64_t q[3][3]) {
  for (int v = 0; v < 3; ++v)
    for (int a = 0; a < 3; ++a) {
      double x = (double)t[v * 3 + a];
      if (!isfinite(x) || fabs(x) >= COORD_LIMIT) return 0;
      q[v][a] = (int64_t)rint(x * FX); /* default rounding mode: nearest, ties to even */
    }
  return 1;
}

/* Projection interval of the closed box [lo, hi] (per-axis fixed-point bounds) onto axis a. */
static void box_interval(const int64_t a[3], const int64_t lo[3], const int64_t hi[3],
                         int64_t *bmin, int64_t *bmax) {
  int64_t mn = 0, mx = 0;
  for (int c = 0; c < 3; ++c) {
    int64_t p = a[c] * lo[c], r = a[c] * hi[c];
    mn += p < r ? p : r;
    mx += p < r ? r : p;
  }
  *bmin = mn;
  *bmax = mx;
}

/* 1 iff the axis a separates the triangle from the box (a zero axis never separates). */
static int separates(const int64_t a[3], int64_t q[3][3], const int64_t lo[3], const int64_t hi[3]) {
  if (a[0] == 0 && a[1] == 0 && a[2] == 0) return 0;
  int64_t p[3];
  for (int v = 0; v < 3; ++v) p[v] = a[0] * q[v][0] + a[1] * q[v][1] + a[2] * q[v][2];
  int64_t bmin, bmax;
  box_interval(a, lo, hi, &bmin, &bmax);
  return max3(p[0], p[1], p[2]) < bmin || min3(p[0], p[1], p[2]) > bmax;
}

/* Closed box [lo, hi] (fixed point) meets the triangle q?  13 candidate axes: the 3 box face
 * normals, the triangle normal and the 9 cross products of triangle edges with box axes. */
int oracle_tri_box_overlap(int64_t q[3][3], const int64_t lo[3], const int64_t hi[3]) {
  static const int64_t unit[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int j = 0; j < 3; ++j)
    if (separates(unit[j], q, lo, hi)) return 0;
  int64_t e[3][3];
  for (int i = 0; i < 3; ++i)
    for (int c = 0; c < 3; ++c) e[i][c] = q[(i + 1) % 3][c] - q[i][c];
  int64_t n[3] = {e[0][1] * e[1][2] - e[0][2] * e[1][1], e[0][2] * e[1][0] - e[0][0] * e[1][2],
                  e[0][0] * e[1][1] - e[0][1] * e[1][0]};
  if (separates(n, q, lo, hi)) return 0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const int64_t *u = unit[j];
      int64_t a[3] = {e[i][1] * u[2] - e[i][2] * u[1], e[i][2] * u[0] - e[i][0] * u[2],
                      e[i][0] * u[1] - e[i][1] * u[0]};
      if (separates(a, q, lo, hi)) return 0;
    }
  return 1;
}

/* Froxel index range [*i0, *i1] whose closed cells [256 i, 256 i + 256] meet [mn, mx], clipped
 * to [0, n-1].  Empty when *i0 > *i1. */
static void cell_range(int64_t mn, int64_t mx, int n, int64_t *i0, int64_t *i1) {
  int64_t a = floordiv(mn - 1, FX), b = floordiv(mx, FX);
  if (a < 0) a = 0;
  if (b > n - 1) b = n - 1;
  *i0 = a;
  *i1 = b;
}

/* occ: uint8 [nz][ny][nx/8], fully overwritten.  Returns the number of ignored triangles. */
int64_t oracle_froxelize(const float *tris, int64_t T, int nx, int ny, int nz, uint8_t *occ) {
  size_t row = (size_t)nx / 8;
  memset(occ, 0, row * (size_t)ny * (size_t)nz);
  int64_t ignored = 0;
  for (int64_t t = 0; t < T; ++t) {
    int64_t q[3][3];
    if (!oracle_quantize_tri(tris + 9 * t, q)) { ignored++; continue; }
    int64_t r0[3], r1[3];
    int dims[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a)
      cell_range(min3(q[0][a], q[1][a], q[2][a]), max3(q[0][a], q[1][a], q[2][a]), dims[a], &r0[a], &r1[a]);
    for (int64_t k = r0[2]; k <= r1[2]; ++k)
      for (int64_t j = r0[1]; j <= r1[1]; ++j)
        for (int64_t i = r0[0]; i <= r1[0]; ++i) {
          int64_t lo[3] = {FX * i, FX * j, FX * k}, hi[3] = {FX * i + FX, FX * j + FX, FX * k + FX};
          if (oracle_tri_box_overlap(q, lo, hi))
            occ[((size_t)k * ny + (size_t)j) * row + (size_t)(i >> 3)] |= (uint8_t)(1u << (i & 7));
        }
  }
  return ignored;
}

static int get_bit(const uint8_t *g, int nx, int ny, int x, int y, int z) {
  return (g[((size_t)z * ny + y) * (nx / 8) + (x >> 3)] >> (x & 7)) & 1;
}

/* ------------------------------------------------------------------------------------------
 * Active sites (Sec. 2.3: sparse tensors store only sites that contain geometry; Sec. 5.2: an
 * empty region costs no memory).  A block is active iff one of its
 * d^3 froxels is occupied; rows are numbered in ascending key order.
 * ------------------------------------------------------------------------------------------ */
int32_t oracle_active_sites(const uint8_t *occ, int nx, int ny, int nz, int d, int32_t *keys) {
  int Bx = nx / d, By = ny / d, Bz = nz / d;
  int32_t n = 0;
  for (int bz = 0; bz < Bz; ++bz)
    for (int by = 0; by < By; ++by)
      for (int bx = 0; bx < Bx; ++bx) {
        int any = 0;
        for (int oz = 0; oz < d && !any; ++oz)
          for (int oy = 0; oy < d && !any; ++oy)
            for (int ox = 0; ox < d && !any; ++ox)
              any = get_bit(occ, nx, ny, bx * d + ox, by * d + oy, bz * d + oz);
        if (any) keys[n++] = (bz * By + by) * Bx + bx;
      }
  return n;
}

/* ------------------------------------------------------------------------------------------
 * Interleave g_d and its inverse (Sec. 3.3, "3D volume-preserving interleaving"): the grid is
 * cut into d x d x d blocks and each block is stacked into a d^3 feature vector.
 *   dense:  out[bz][by][bx][c] = in[bz d + oz][by d + oy][bx d + ox],  c = (oz d + oy) d + ox
 * ------------------------------------------------------------------------------------------ */
void oracle_interleave(const void *in, int nx, int ny, int nz, int d, int esize, void *out) {
  const char *s = (const char *)in;
  char *t = (char *)out;
  int Bx = nx / d, By = ny / d, Bz = nz / d, C = d * d * d;
  for (int bz = 0; bz < Bz; ++bz)
    for (int by = 0; by < By; ++by)
      for (int bx = 0; bx < Bx; ++bx)
        for (int oz = 0; oz < d; ++oz)
          for (int oy = 0; oy < d; ++oy)
            for (int ox = 0; ox < d; ++ox) {
              size_t src = ((size_t)(bz * d + oz) * ny + (size_t)(by * d + oy)) * nx + (size_t)(bx * d + ox);
              size_t dst = (((size_t)bz * By + by) * Bx + bx) * C + (size_t)((oz * d + oy) * d + ox);
              memcpy(t + dst * esize, s + src * esize, (size_t)esize);
            }
}

void oracle_deinterleave(const void *in, int nx, int ny, int nz, int d, int esize, void *out) {
  const char *s = (const char *)in;
  char *t = (char *)out;
  int Bx = nx / d, By = ny / d, Bz = nz / d, C = d * d * d;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int bx = x / d, by = y / d, bz = z / d, c = ((z % d) * d + (y % d)) * d + (x % d);
        size_t src = (((size_t)bz * By + by) * Bx + bx) * C + (size_t)c;
        size_t dst = ((size_t)z * ny + y) * nx + x;
        memcpy(t + dst * esize, s + src * esize, (size_t)esize);
      }
}

/* Sparse interleave: X[r][c] = G at froxel (bx d + ox, by d + oy, bz d + oz) of site r. */
void oracle_gather_sites(const uint8_t *occ, int nx, int ny, int nz, int d, int32_t n,
                         const int32_t *keys, double *X) {
  (void)nz;
  int Bx = nx / d, By = ny / d, C = d * d * d;
  for (int32_t r = 0; r < n; ++r) {
    int bx = keys[r] % Bx, by = (keys[r] / Bx) % By, bz = keys[r] / (Bx * By);
    for (int oz = 0; oz < d; ++oz)
      for (int oy = 0; oy < d; ++oy)
        for (int ox = 0; ox < d; ++ox)
          X[(size_t)r * C + (oz * d + oy) * d + ox] = get_bit(occ, nx, ny, bx * d + ox, by * d + oy, bz * d + oz);
  }
}

/* ------------------------------------------------------------------------------------------
 * Rulebook of a submanifold 3x3x3 convolution (Sec. 2.3; Graham et al.: the kernel is centred
 * only on active sites, so the output active set equals the input active set).  For each
 * offset k and each output row r in ascending order, if p_r + delta_k is an active site i,
 * the pair (i, r) is appended.  rb_off[28] is the CSR offset array.  Returns the pair count.
 * ------------------------------------------------------------------------------------------ */
int64_t oracle_rulebook(const int32_t *keys, int32_t n, int Bx, int By, int Bz, int32_t *rb_off,
                        int32_t *pairs) {
  int64_t B = (int64_t)Bx * By * Bz;
  int32_t *row_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)B);
  for (int64_t b = 0; b < B; ++b) row_of[b] = -1;
  for (int32_t r = 0; r < n; ++r) row_of[keys[r]] = r;
  int64_t np = 0;
  for (int k = 0; k < 27; ++k) {
    rb_off[k] = (int32_t)np;
    int dz = k / 9 - 1, dy = (k / 3) % 3 - 1, dx = k % 3 - 1;
    for (int32_t r = 0; r < n; ++r) {
      int bx = keys[r] % Bx + dx, by = (keys[r] / Bx) % By + dy, bz = keys[r] / (Bx * By) + dz;
      if (bx < 0 || by < 0 || bz < 0 || bx >= Bx || by >= By || bz >= Bz) continue;
      int32_t i = row_of[((int64_t)bz * By + by) * Bx + bx];
      if (i < 0) continue;
      pairs[2 * np] = i;
      pairs[2 * np + 1] = r;
      np++;
    }
  }
  rb_off[27] = (int32_t)np;
  free(row_of);
  return np;
}

/* ------------------------------------------------------------------------------------------
 * Submanifold sparse convolution, FP64, straight from the definition:
 *   Y[r][o] = b[o] + sum_k sum_{(i,r) in R_k} sum_c X[i][c] W[k][c][o],  then max(0, .) if relu.
 * ------------------------------------------------------------------------------------------ */
void oracle_subm_conv(const double *X, int32_t n, int cin, const double *W, const double *b, int cout,
                      const int32_t *rb_off, const int32_t *pairs, int relu, double *Y) {
  for (int32_t r = 0; r < n; ++r)
    for (int o = 0; o < cout; ++o) Y[(size_t)r * cout + o] = b ? b[o] : 0.0;
  for (int k = 0; k < 27; ++k)
    for (int32_t p = rb_off[k]; p < rb_off[k + 1]; ++p) {
      int32_t i = pairs[2 * p], r = pairs[2 * p + 1];
      for (int c = 0; c < cin; ++c) {
        double x = X[(size_t)i * cin + c];
        for (int o = 0; o < cout; ++o) Y[(size_t)r * cout + o] += x * W[((size_t)k * cin + c) * cout + o];
      }
    }
  if (relu)
    for (size_t t = 0; t < (size_t)n * cout; ++t) Y[t] = Y[t] > 0.0 ? Y[t] : 0.0;
}

/* Second, independent form of the same layer: a dense zero-padded 3x3x3 cross-correlation on
 * the whole block grid, bias and ReLU, after which every inactive site is set to zero.
 * in: [Bz][By][Bx][cin], active: [Bz][By][Bx] (0/1), out: [Bz][By][Bx][cout]. */
void oracle_masked_dense_conv(const double *in, const uint8_t *active, int Bx, int By, int Bz, int cin,
                              const double *W, const double *b, int cout, int relu, double *out) {
  for (int z = 0; z < Bz; ++z)
    for (int y = 0; y < By; ++y)
      for (int x = 0; x < Bx; ++x) {
        double *o_ = out + (((size_t)z * By + y) * Bx + x) * cout;
        for (int o = 0; o < cout; ++o) o_[o] = b ? b[o] : 0.0;
        for (int k = 0; k < 27; ++k) {
          int zz = z + k / 9 - 1, yy = y + (k / 3) % 3 - 1, xx = x + k % 3 - 1;
          if (zz < 0 || yy < 0 || xx < 0 || zz >= Bz || yy >= By || xx >= Bx) continue;
          const double *i_ = in + (((size_t)zz * By + yy) * Bx + xx) * cin;
          for (int c = 0; c < cin; ++c)
            for (int o = 0; o < cout; ++o) o_[o] += i_[c] * W[((size_t)k * cin + c) * cout + o];
        }
        for (int o = 0; o < cout; ++o) {
          if (relu && o_[o] < 0.0) o_[o] = 0.0;
          if (!active[((size_t)z * By + y) * Bx + x]) o_[o] = 0.0;
        }
      }
}

/* ------------------------------------------------------------------------------------------
 * De-interleave and threshold (Sec. 3.1: V = 1[f(G) >= tau], tau = 0.5; Sec. 3.3: g_d^-1).
 * The threshold sigma(l) >= 0.5 is taken as l >= 0.  Froxels of inactive blocks have no logit
 * (-inf, V = 0).  The output is masked by G because the visible set lies inside the occupied
 * set (Sec. 3.2).  logits: optional dense [nz][ny][nx]; pvs: packed like occ.
 * ------------------------------------------------------------------------------------------ */
void oracle_deinterleave_threshold(const double *Y, int32_t n, const int32_t *keys, const uint8_t *occ,
                                   int nx, int ny, int nz, int d, double *logits, uint8_t *pvs) {
  int Bx = nx / d, By = ny / d, Bz = nz / d, C = d * d * d;
  int64_t B = (int64_t)Bx * By * Bz;
  int32_t *row_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)B);
  for (int64_t b = 0; b < B; ++b) row_of[b] = -1;
  for (int32_t r = 0; r < n; ++r) row_of[keys[r]] = r;
  memset(pvs, 0, (size_t)nx / 8 * ny * nz);
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int32_t r = row_of[((int64_t)(z / d) * By + (y / d)) * Bx + (x / d)];
        double l = -INFINITY;
        if (r >= 0) l = Y[(size_t)r * C + ((z % d) * d + (y % d)) * d + (x % d)];
        if (logits) logits[((size_t)z * ny + y) * nx + x] = l;
        if (r >= 0 && l >= 0.0 && get_bit(occ, nx, ny, x, y, z))
          pvs[((size_t)z * ny + y) * (nx / 8) + (x >> 3)] |= (uint8_t)(1u << (x & 7));
      }
  free(row_of);
}

/* ------------------------------------------------------------------------------------------
 * Training loss over the froxels of the active blocks of one grid (Sec. 3.3 "Repulsive
 * visibility loss" and the combined loss, with BCE in place of the Dice term):
 *   p = sigma(l);  BCE = mean(softplus(l) - y l);  soft TP = sum y p,  FN = sum y (1 - p),
 *   FP = sum (1 - y) p,  GTP = sum y;  L_rv = FN / max(GTP,1) + FP / max(GTP,1);
 *   L = lambda BCE + (1 - lambda) L_rv.
 * The attraction term is read as 1 - TP/GTP (= FN/GTP): printed literally it would reward
 * missed geometry.  out[7] = {L, BCE, L_rv, TP, FN, FP, GTP}; grad (optional) = dL/dl.
 * ------------------------------------------------------------------------------------------ */
void oracle_loss(const double *l, const uint8_t *y, int64_t m, double lambda, double *out, double *grad) {
  double bce = 0, tp = 0, fn = 0, fp = 0, gtp = 0;
  for (int64_t t = 0; t < m; ++t) {
    double p = 1.0 / (1.0 + exp(-l[t]));
    double sp = (l[t] > 0 ? l[t] : 0.0) + log1p(exp(-fabs(l[t])));
    bce += sp - y[t] * l[t];
    tp += y[t] * p;
    fn += y[t] * (1.0 - p);
    fp += (1 - y[t]) * p;
    gtp += y[t];
  }
  double g = gtp > 1.0 ? gtp : 1.0;
  double mean_bce = m > 0 ? bce / (double)m : 0.0;
  double lrv = fn / g + fp / g;
  out[0] = lambda * mean_bce + (1.0 - lambda) * lrv;
  out[1] = mean_bce;
  out[2] = lrv;
  out[3] = tp;
  out[4] = fn;
  out[5] = fp;
  out[6] = gtp;
  if (grad)
    for (int64_t t = 0; t < m; ++t) {
      double p = 1.0 / (1.0 + exp(-l[t]));
      /* d/dl of FN/g is -y p(1-p)/g; of FP/g is (1-y) p(1-p)/g */
      grad[t] = lambda * (p - y[t]) / (double)m + (1.0 - lambda) * p * (1.0 - p) * (1.0 - 2.0 * y[t]) / g;
    }
}

/* ------------------------------------------------------------------------------------------
 * The paper's combined loss with its weighted Dice term (Sec. 3.3):
 *   L = lambda * L_dice + (1 - lambda) * L_rv,
 *   L_dice = 1 - 2 TP / (2 TP + alpha * A + (1 - alpha) * B),
 * where A and B are the terms the printed formulas call FP and FN: A = sum y (1-p) (ground-truth
 * froxels the prediction misses) and B = sum (1-y) p, so that alpha weighs the missed froxels,
 * as the text says.  L_rv as in oracle_loss (FN = A, FP = B in the words' sense).  Soft counts
 * with p = sigmoid(l).  out: L, L_dice, L_rv, TP, FN, FP, GTP; grad = dL/dl (nullable).
 * ------------------------------------------------------------------------------------------ */
void oracle_loss_dice(const double *l, const uint8_t *y, int64_t m, double lambda, double alpha, double *out,
                      double *grad) {
  double tp = 0, fn = 0, fp = 0, gtp = 0;
  for (int64_t t = 0; t < m; ++t) {
    double p = 1.0 / (1.0 + exp(-l[t]));
    tp += y[t] * p;
    fn += y[t] * (1.0 - p);
    fp += (1 - y[t]) * p;
    gtp += y[t];
  }
  double g = gtp > 1.0 ? gtp : 1.0;
  double den = 2.0 * tp + alpha * fn + (1.0 - alpha) * fp;
  double dice = den > 0.0 ? 1.0 - 2.0 * tp / den : 0.0;
  double lrv = fn / g + fp / g;
  out[0] = lambda * dice + (1.0 - lambda) * lrv;
  out[1] = dice;
  out[2] = lrv;
  out[3] = tp;
  out[4] = fn;
  out[5] = fp;
  out[6] = gtp;
  if (grad)
    for (int64_t t = 0; t < m; ++t) {
      double p = 1.0 / (1.0 + exp(-l[t]));
      double yt = y[t];
      /* quotient rule: d(2TP)/dp = 2y, d(den)/dp = 2y - alpha y + (1 - alpha)(1 - y) */
      double ddice = den > 0.0 ? -(2.0 * yt * den - 2.0 * tp * (2.0 * yt - alpha * yt + (1.0 - alpha) * (1.0 - yt))) /
                                     (den * den)
                               : 0.0;
      double drv = (1.0 - 2.0 * yt) / g;
      grad[t] = (lambda * ddice + (1.0 - lambda) * drv) * p * (1.0 - p);
    }
}

/* ------------------------------------------------------------------------------------------
 * Backward of one submanifold layer, FP64, by the chain rule on the forward definition:
 *   dZ = dY * [Y > 0] (ReLU'(0) = 0) when relu, else dY;
 *   dX[i] += sum_k sum_{(i,r) in R_k} dZ[r] W_k^T;  dW_k = sum_{(i,r)} X[i]^T dZ[r];  db = sum_r dZ[r].
 * Y is the layer's output after activation.  dX, dW, db are overwritten (dX may be NULL).
 * ------------------------------------------------------------------------------------------ */
void oracle_subm_conv_bwd(const double *X, int32_t n, int cin, const double *W, int cout, const int32_t *rb_off,
                          const int32_t *pairs, const double *Y, const double *dY, int relu, double *dX,
                          double *dW, double *db) {
  double *dZ = (double *)malloc(sizeof(double) * (size_t)n * cout + 1);
  for (size_t t = 0; t < (size_t)n * cout; ++t) dZ[t] = (relu && !(Y[t] > 0.0)) ? 0.0 : dY[t];
  if (dX) memset(dX, 0, sizeof(double) * (size_t)n * cin);
  memset(dW, 0, sizeof(double) * 27 * (size_t)cin * cout);
  for (int o = 0; o < cout; ++o) db[o] = 0.0;
  for (int32_t r = 0; r < n; ++r)
    for (int o = 0; o < cout; ++o) db[o] += dZ[(size_t)r * cout + o];
  for (int k = 0; k < 27; ++k)
    for (int32_t p = rb_off[k]; p < rb_off[k + 1]; ++p) {
      int32_t i = pairs[2 * p], r = pairs[2 * p + 1];
      for (int c = 0; c < cin; ++c)
        for (int o = 0; o < cout; ++o) {
          double g = dZ[(size_t)r * cout + o];
          dW[((size_t)k * cin + c) * cout + o] += X[(size_t)i * cin + c] * g;
          if (dX) dX[(size_t)i * cin + c] += g * W[((size_t)k * cin + c) * cout + o];
        }
    }
  free(dZ);
}

/* ------------------------------------------------------------------------------------------
 * Adam (Kingma & Ba), one step t >= 1, on FP64 copies; weight decay is added to the gradient
 * (the decay rate of 1e-10 that the paper lists with the learning rate, read as weight decay).
 * ------------------------------------------------------------------------------------------ */
void oracle_adam(double *p, const double *g, double *m, double *v, int64_t count, int64_t t, double lr,
                 double b1, double b2, double eps, double wd) {
  double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
  for (int64_t i = 0; i < count; ++i) {
    double gi = g[i] + wd * p[i];
    m[i] = b1 * m[i] + (1.0 - b1) * gi;
    v[i] = b2 * v[i] + (1.0 - b2) * gi * gi;
    p[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
  }
}

/* ------------------------------------------------------------------------------------------
 * Ray-march visibility labeller (Sec. 3.2: the ground-truth PVS is obtained by dense sampling of
 * the viewcell; every viewpoint renders a depth buffer whose fragments mark froxels).
 * Reading for grid space: rays go from each viewpoint c_m to an s x s raster of target points
 * per froxel face on every face of the grid box except z = 0; they walk the grid with a 3D DDA
 * (Amanatides & Woo; on equal crossing times x steps first, then y, then z).  In each occupied
 * froxel the ray is intersected with the triangles overlapping that froxel (Moller-Trumbore,
 * FP64); the first hit inside the froxel's ray segment marks the froxel and ends the ray.
 * ------------------------------------------------------------------------------------------ */
typedef struct {
  int nx, ny, nz;
  const int64_t *cell_off; /* CSR over froxels */
  const int32_t *cell_tri;
  const double *tri; /* [T][3][3] FP64 copies of the float vertices */
  uint8_t *lab;
} lab_ctx;

static int ray_tri(const double o[3], const double dir[3], const double *t, double *s_out) {
  double e1[3], e2[3], pv[3], tv[3], qv[3];
  for (int a = 0; a < 3; ++a) { e1[a] = t[3 + a] - t[a]; e2[a] = t[6 + a] - t[a]; }
  pv[0] = dir[1] * e2[2] - dir[2] * e2[1];
  pv[1] = dir[2] * e2[0] - dir[0] * e2[2];
  pv[2] = dir[0] * e2[1] - dir[1] * e2[0];
  double det = e1[0] * pv[0] + e1[1] * pv[1] + e1[2] * pv[2];
  if (det == 0.0) return 0;
  double inv = 1.0 / det;
  for (int a = 0; a < 3; ++a) tv[a] = o[a] - t[a];
  double u = (tv[0] * pv[0] + tv[1] * pv[1] + tv[2] * pv[2]) * inv;
  if (u < 0.0 || u > 1.0) return 0;
  qv[0] = tv[1] * e1[2] - tv[2] * e1[1];
  qv[1] = tv[2] * e1[0] - tv[0] * e1[2];
  qv[2] = tv[0] * e1[1] - tv[1] * e1[0];
  double v = (dir[0] * qv[0] + dir[1] * qv[1] + dir[2] * qv[2]) * inv;
  if (v < 0.0 || u + v > 1.0) return 0;
  *s_out = (e2[0] * qv[0] + e2[1] * qv[1] + e2[2] * qv[2]) * inv;
  return 1;
}

static void march(const lab_ctx *L, const double o[3], const double target[3]) {
  double dir[3] = {target[0] - o[0], target[1] - o[1], target[2] - o[2]};
  double hi[3] = {L->nx, L->ny, L->nz};
  double s0 = 0.0, s1 = 1.0;
  for (int a = 0; a < 3; ++a) { /* slab clip of the segment o + s dir, s in [0,1], to the grid box */
    if (dir[a] == 0.0) {
      if (o[a] < 0.0 || o[a] > hi[a]) return;
      continue;
    }
    double ta = (0.0 - o[a]) / dir[a], tb = (hi[a] - o[a]) / dir[a];
    if (ta > tb) { double tmp = ta; ta = tb; tb = tmp; }
    if (ta > s0) s0 = ta;
    if (tb < s1) s1 = tb;
  }
  if (s0 > s1) return;
  int dims[3] = {L->nx, L->ny, L->nz};
  int cell[3], step[3];
  double tmax[3], tdel[3];
  double sm = s0 + 1e-9 * (s1 - s0); /* the cell the ray is in just after entering the box */
  for (int a = 0; a < 3; ++a) {
    double p = o[a] + sm * dir[a];
    int c = (int)floor(p);
    if (c < 0) c = 0;
    if (c > dims[a] - 1) c = dims[a] - 1;
    cell[a] = c;
    if (dir[a] > 0) { step[a] = 1; tmax[a] = (c + 1 - o[a]) / dir[a]; tdel[a] = 1.0 / dir[a]; }
    else if (dir[a] < 0) { step[a] = -1; tmax[a] = (c - o[a]) / dir[a]; tdel[a] = -1.0 / dir[a]; }
    else { step[a] = 0; tmax[a] = INFINITY; tdel[a] = INFINITY; }
  }
  double s_in = s0;
  for (;;) {
    int ax = 0;
    if (tmax[1] < tmax[ax]) ax = 1;
    if (tmax[2] < tmax[ax]) ax = 2;
    double s_out = tmax[ax] < s1 ? tmax[ax] : s1;
    size_t cid = ((size_t)cell[2] * L->ny + cell[1]) * L->nx + cell[0];
    for (int64_t e = L->cell_off[cid]; e < L->cell_off[cid + 1]; ++e) {
      double s;
      if (ray_tri(o, dir, L->tri + 9 * (size_t)L->cell_tri[e], &s) && s >= s_in && s <= s_out) {
        L->lab[((size_t)cell[2] * L->ny + cell[1]) * (L->nx / 8) + (cell[0] >> 3)] |= (uint8_t)(1u << (cell[0] & 7));
        return;
      }
    }
    if (tmax[ax] >= s1) return;
    cell[ax] += step[ax];
    if (cell[ax] < 0 || cell[ax] >= dims[ax]) return;
    s_in = tmax[ax];
    tmax[ax] += tdel[ax];
  }
}

/* views: [M][3] viewpoints.  lab: packed like occ, overwritten.  Returns rays cast. */
int64_t oracle_label_raymarch(const float *tris, int64_t T, int nx, int ny, int nz, const double *views, int M,
                              int s_r, uint8_t *lab) {
  size_t N = (size_t)nx * ny * nz;
  int64_t *cnt = (int64_t *)calloc(N + 1, sizeof(int64_t));
  double *tri = (double *)malloc(sizeof(double) * 9 * (size_t)(T > 0 ? T : 1));
  for (int64_t t = 0; t < 9 * T; ++t) tri[t] = (double)tris[t];
  /* two passes over the exact overlap: count, then fill the per-froxel triangle lists */
  for (int pass = 0; pass < 2; ++pass) {
    int64_t *fill = NULL;
    int32_t *lst = NULL;
    if (pass == 1) {
      for (size_t c = 0; c < N; ++c) cnt[c + 1] += cnt[c];
      fill = (int64_t *)calloc(N, sizeof(int64_t));
      lst = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cnt[N] > 0 ? cnt[N] : 1));
    }
    for (int64_t t = 0; t < T; ++t) {
      int64_t q[3][3];
      if (!oracle_quantize_tri(tris + 9 * t, q)) continue;
      int64_t r0[3], r1[3];
      int dims[3] = {nx, ny, nz};
      for (int a = 0; a < 3; ++a)
        cell_range(min3(q[0][a], q[1][a], q[2][a]), max3(q[0][a], q[1][a], q[2][a]), dims[a], &r0[a], &r1[a]);
      for (int64_t k = r0[2]; k <= r1[2]; ++k)
        for (int64_t j = r0[1]; j <= r1[1]; ++j)
          for (int64_t i = r0[0]; i <= r1[0]; ++i) {
            int64_t lo[3] = {FX * i, FX * j, FX * k}, hi[3] = {FX * i + FX, FX * j + FX, FX * k + FX};
            if (!oracle_tri_box_overlap(q, lo, hi)) continue;
            size_t c = ((size_t)k * ny + j) * nx + i;
            if (pass == 0) cnt[c + 1]++;
            else lst[cnt[c] + fill[c]++] = (int32_t)t;
          }
    }
    if (pass == 1) {
      lab_ctx L = {nx, ny, nz, cnt, lst, tri, lab};
      memset(lab, 0, (size_t)nx / 8 * ny * nz);
      int64_t rays = 0;
      for (int m = 0; m < M; ++m) {
        const double *o = views + 3 * m;
        double tg[3];
        /* far face z = nz */
        for (int j = 0; j < ny * s_r; ++j)
          for (int i = 0; i < nx * s_r; ++i) {
            tg[0] = (i + 0.5) / s_r; tg[1] = (j + 0.5) / s_r; tg[2] = nz;
            march(&L, o, tg); rays++;
          }
        /* side faces x = 0, x = nx */
        for (int side = 0; side < 2; ++side)
          for (int k = 0; k < nz * s_r; ++k)
            for (int j = 0; j < ny * s_r; ++j) {
              tg[0] = side ? nx : 0.0; tg[1] = (j + 0.5) / s_r; tg[2] = (k + 0.5) / s_r;
              march(&L, o, tg); rays++;
            }
        /* faces y = 0, y = ny */
        for (int side = 0; side < 2; ++side)
          for (int k = 0; k < nz * s_r; ++k)
            for (int i = 0; i < nx * s_r; ++i) {
              tg[0] = (i + 0.5) / s_r; tg[1] = side ? ny : 0.0; tg[2] = (k + 0.5) / s_r;
              march(&L, o, tg); rays++;
            }
      }
      free(fill);
      free(lst);
      free(cnt);
      free(tri);
      return rays;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------------------------
 * World-space froxelization of the viewcell frustum (Sec. 3.2; linear depth slices, Suppl. A.1).
 * Camera: apex e, orthonormal right / up / forward (r, u, f); eye coordinates
 * (x, y, z) = ((p-e).r, (p-e).u, (p-e).f).  Froxel (i, j, k) of an Nx x Ny x Nz grid is the set of
 * points with z in [zn + k s, zn + (k+1) s] (s = (zf - zn) / Nz), x / z in
 * [tx (2i/Nx - 1), tx (2(i+1)/Nx - 1)] and y / z likewise with ty.  G(i, j, k) = 1 iff a
 * triangle meets that closed set.  Under (X, Y, Q) = (x/z, y/z, 1/z), a projective map on z > 0,
 * triangles stay triangles and each froxel becomes an axis-aligned box, so the test is: clip the
 * triangle at the near plane z = zn, map the pieces, and clip each against the six planes of the
 * box (non-empty result = overlap).  `margin` moves every box plane outward by margin times the
 * box's extent along that axis (negative: inward), for tests that need the robustly inside and
 * robustly outside sets.  occ is packed like the grid-space froxelization.
 * ------------------------------------------------------------------------------------------ */
static int clip_poly(double (*in)[3], int n, int axis, double bound, int keep_above, double (*out)[3]) {
  int m = 0;
  for (int a = 0; a < n; ++a) {
    const double *P = in[a], *R = in[(a + 1) % n];
    double dp = keep_above ? P[axis] - bound : bound - P[axis];
    double dr = keep_above ? R[axis] - bound : bound - R[axis];
    if (dp >= 0) {
      out[m][0] = P[0], out[m][1] = P[1], out[m][2] = P[2];
      ++m;
    }
    if ((dp >= 0) != (dr >= 0)) {
      double t = dp / (dp - dr);
      for (int c = 0; c < 3; ++c) out[m][c] = P[c] + t * (R[c] - P[c]);
      ++m;
    }
  }
  return m;
}

int64_t oracle_froxelize_view(const float *tris, int64_t T, const double *eye, const double *right, const double *up,
                              const double *fwd, double tx, double ty, double zn, double zf, int nx, int ny, int nz,
                              double margin, uint8_t *occ) {
  memset(occ, 0, (size_t)nz * ny * (nx / 8));
  const double s = (zf - zn) / nz;
  int64_t marked = 0;
  for (int64_t t = 0; t < T; ++t) {
    double poly[16][3], tmp[16][3];
    for (int v = 0; v < 3; ++v) {
      double d[3];
      for (int c = 0; c < 3; ++c) d[c] = (double)tris[(t * 3 + v) * 3 + c] - eye[c];
      poly[v][0] = d[0] * right[0] + d[1] * right[1] + d[2] * right[2];
      poly[v][1] = d[0] * up[0] + d[1] * up[1] + d[2] * up[2];
      poly[v][2] = d[0] * fwd[0] + d[1] * fwd[1] + d[2] * fwd[2];
    }
    int finite = 1;
    for (int v = 0; v < 3; ++v)
      for (int c = 0; c < 3; ++c) finite &= isfinite(poly[v][c]) != 0;
    if (!finite) continue;
    int n = clip_poly(poly, 3, 2, zn, 1, tmp); /* keep z >= zn */
    if (n < 3) continue;
    double P[16][3];
    for (int a = 0; a < n; ++a) {
      P[a][0] = tmp[a][0] / tmp[a][2];
      P[a][1] = tmp[a][1] / tmp[a][2];
      P[a][2] = 1.0 / tmp[a][2];
    }
    /* froxels outside the index range of the mapped polygon (one froxel of slack) cannot meet it */
    double mn[3] = {P[0][0], P[0][1], P[0][2]}, mx[3] = {P[0][0], P[0][1], P[0][2]};
    for (int a = 1; a < n; ++a)
      for (int c = 0; c < 3; ++c) {
        mn[c] = P[a][c] < mn[c] ? P[a][c] : mn[c];
        mx[c] = P[a][c] > mx[c] ? P[a][c] : mx[c];
      }
#define CLAMPI(v, hi) ((int)((v) < 0.0 ? 0.0 : ((v) > (double)(hi) ? (double)(hi) : (v))))
    const int i0 = CLAMPI(floor((mn[0] / tx + 1.0) * 0.5 * nx) - 1.0, nx - 1);
    const int i1 = CLAMPI(floor((mx[0] / tx + 1.0) * 0.5 * nx) + 1.0, nx - 1);
    const int j0 = CLAMPI(floor((mn[1] / ty + 1.0) * 0.5 * ny) - 1.0, ny - 1);
    const int j1 = CLAMPI(floor((mx[1] / ty + 1.0) * 0.5 * ny) + 1.0, ny - 1);
    const int k0 = CLAMPI(floor((1.0 / mx[2] - zn) / s) - 1.0, nz - 1);
    const int k1 = CLAMPI(floor((1.0 / mn[2] - zn) / s) + 1.0, nz - 1);
#undef CLAMPI
    for (int k = k0; k <= k1; ++k) {
      const double qlo = 1.0 / (zn + (k + 1) * s), qhi = 1.0 / (zn + k * s);
      for (int j = j0; j <= j1; ++j) {
        const double ylo = ty * (2.0 * j / ny - 1.0), yhi = ty * (2.0 * (j + 1) / ny - 1.0);
        for (int i = i0; i <= i1; ++i) {
          const double xlo = tx * (2.0 * i / nx - 1.0), xhi = tx * (2.0 * (i + 1) / nx - 1.0);
          const double lo[3] = {xlo - margin * (xhi - xlo), ylo - margin * (yhi - ylo), qlo - margin * (qhi - qlo)};
          const double hi[3] = {xhi + margin * (xhi - xlo), yhi + margin * (yhi - ylo), qhi + margin * (qhi - qlo)};
          double A[16][3], B[16][3];
          int m = n;
          for (int a = 0; a < n; ++a) A[a][0] = P[a][0], A[a][1] = P[a][1], A[a][2] = P[a][2];
          for (int ax = 0; ax < 3 && m > 0; ++ax) {
            m = clip_poly(A, m, ax, lo[ax], 1, B);
            if (m == 0) break;
            m = clip_poly(B, m, ax, hi[ax], 0, A);
          }
          if (m > 0) {
            uint8_t *w = occ + ((size_t)k * ny + j) * (nx / 8) + (i >> 3);
            if (!(*w & (1u << (i & 7)))) ++marked;
            *w |= (uint8_t)(1u << (i & 7));
          }
        }
      }
    }
  }
  return marked;
}
