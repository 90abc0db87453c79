/*
 * neuralpvs.h — C ABI of the MI355X (gfx950) NeuralPVS hot-path library.
 *
 * The library computes the forward pass of the visibility network of NeuralPVS (arXiv
 * 2509.24677): the scene triangles are froxelized into a binary occupancy grid G (Sec. 3.2),
 * G is interleaved by g_d (Sec. 3.3), a stack of submanifold sparse 3x3x3 convolutions runs on
 * the interleaved sites (Sec. 2.3, 3.3), and the result is de-interleaved by g_d^-1 and
 * thresholded into the potentially visible set V = 1[f(G) >= tau] (Sec. 3.1), so that
 * V = g_d^-1(f(g_d(G))).  It also provides the hand-written backward, the training loss (the
 * repulsive visibility loss of Sec. 3.3 combined with BCE) and Adam.
 *
 * Conventions shared by every call:
 *  - Pointers marked (device) are HIP device pointers owned by the caller; the library never
 *    frees them.  Pointers marked (host) are read during the call only.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Every call only
 *    enqueues work on it and returns; nothing synchronizes with the host unless stated.
 *  - Argument errors are detected on the host before anything is enqueued and return
 *    NPVS_ERR_INVALID_ARG; launch failures return NPVS_ERR_HIP.  npvs_last_error() gives the
 *    message of the calling thread's last failure.
 *  - Froxels are (x, y, z), 0-based, x fastest (the paper writes the domain 1-based).  A grid
 *    of nx*ny*nz froxels is packed as uint8 [nz][ny][nx/8], bit (x & 7) of byte (x >> 3) is
 *    froxel x (least significant bit = lowest x), as the paper packs eight consecutive
 *    x-froxels per byte.
 *  - Interleave factor d: block (bx, by, bz) holds froxels [bx*d, bx*d+d) x ...; its key is
 *    (bz*By + by)*Bx + bx with (Bx, By, Bz) = (nx/d, ny/d, nz/d); its channel vector stacks the
 *    froxels as c = (oz*d + oy)*d + ox.
 *  - A batch of grids is laid out back to back: grid b's packed bits start at byte
 *    sum_{b'<b} nz*ny*nx/8 and its block keys are offset by sum_{b'<b} Bx*By*Bz ("global
 *    keys").  Active sites (rows) are numbered in ascending global key.
 *  - Convolution offset k = (dz+1)*9 + (dy+1)*3 + (dx+1), dz,dy,dx in {-1,0,1}; a layer is
 *    the cross-correlation Y[p] = b + sum_k X[p + delta_k] W_k over active sites p only.
 *  - Weights are float32 [27][cin][cout] (masters) and are packed once per layer into the
 *    layout a convolution kernel reads (npvs_pack_weights).  Bias is always float32.
 *  - bf16 values are raw uint16 bit patterns rounded to nearest even from float32.
 */
#ifndef NEURALPVS_H
#define NEURALPVS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t npvs_status;
#define NPVS_OK 0
#define NPVS_ERR_INVALID_ARG (-1)
#define NPVS_ERR_CAPACITY (-2)
#define NPVS_ERR_HIP (-3)
#define NPVS_ERR_UNSUPPORTED (-4)

/* element types */
#define NPVS_F32 0
#define NPVS_BF16 1
#define NPVS_U8 2

/* limits */
#define NPVS_MAX_GRIDS 32        /* grids per batch */
#define NPVS_MAX_DIM 1024        /* froxels per axis */
#define NPVS_COORD_LIMIT 2048    /* triangles with a coordinate |v| >= 2048 (grid units) are ignored */
#define NPVS_MAX_WGRAD_LAYERS 16 /* layers of one npvs_sparse_conv_wgrad call */

typedef struct {
  int32_t nx, ny, nz; /* froxels; nx % 8 == 0 and every extent divisible by d */
} npvs_dims;

/* Device-side counters written by npvs_build_rulebook and read by later calls, so that no
 * call needs the host to know the number of active sites. */
typedef struct {
  int32_t n_sites;        /* active sites stored (min of found and cap_sites) */
  int32_t n_sites_needed; /* active sites found; > cap_sites means the capacity overflowed */
  int32_t n_pairs;        /* rulebook pairs stored (when the CSR form is requested) */
  int32_t n_tris_ignored; /* triangles the plan's froxelization ignored (npvs_froxelize's n_ignored);
                             npvs_build_rulebook does not write it */
} npvs_counts;

const char *npvs_version(void);
/* 16 hex digits identifying the sources the library was built from (SHA-256 over the HIP
   sources, this header and the compile flags); static string, never freed. */
const char *npvs_source_hash(void);
const char *npvs_last_error(void);

/* Total blocks of a batch (sum of Bx*By*Bz) and total packed bytes (sum of nz*ny*nx/8). */
npvs_status npvs_batch_sizes(int32_t n_grids, const npvs_dims *dims /*host*/, int32_t d, int64_t *total_blocks,
                             int64_t *total_bytes);

/* ---------------------------------------------------------------------------------------------
 * Froxelization (Sec. 3.2; Fig. 2(b)): G(x) = 1 iff a triangle meets the closed froxel x.
 * Vertices are in grid units (one froxel = 1), quantized to 1/256 froxel with round half to
 * even, and tested exactly (integer separating-axis test).  A triangle may reach outside the grid
 * (it marks the froxels it meets); one with a non-finite coordinate or |coordinate| >= 2048
 * (NPVS_COORD_LIMIT, the range in which the fixed-point test is exact in 64-bit integers) is
 * ignored and counted.
 *   tris      (device) float32 [sum T_b][3][3], grid b's triangles after those of grids < b
 *   n_tris    (host)   int64 [n_grids] triangle counts
 *   occ_bits  (device) packed grids of the batch, fully overwritten
 *   n_ignored (device, nullable) int32, overwritten with the number of ignored triangles
 *   ws        (device) workspace of npvs_froxelize_workspace_size() bytes
 * ------------------------------------------------------------------------------------------- */
npvs_status npvs_froxelize_workspace_size(int32_t n_grids, const npvs_dims *dims, const int64_t *n_tris,
                                          size_t *bytes);
npvs_status npvs_froxelize(const float *tris, const int64_t *n_tris, int32_t n_grids, const npvs_dims *dims,
                           uint8_t *occ_bits, int32_t *n_ignored, void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Active sites and rulebook of the submanifold convolution (Sec. 2.3: the kernel is centred
 * only on active sites; sparse tensors store only sites with geometry).  A block is active iff
 * one of its d^3 froxels is occupied.
 *   counts     (device) npvs_counts, written
 *   site_keys  (device) int32 [cap_sites] global key of each row, ascending
 *   block_row  (device) int32 [total_blocks] row of each block or -1 (the site lookup table)
 *   grid_rows  (device) int32 [n_grids + 1] first row of each grid, grid_rows[n_grids] = n_sites
 *   nbr        (device) int32 [27][cap_sites] nbr[k][r] = row at p_r + delta_k, or -1
 *   rb_off     (device, nullable) int32 [28] CSR offsets of the per-offset pair lists
 *   rb_pairs   (device, nullable) int32 [27*cap_sites][2] (in_row, out_row), ascending out_row
 *              within each offset; both rb_off and rb_pairs or neither
 *   ws         (device) workspace of npvs_rulebook_workspace_size() bytes
 * Rows beyond cap_sites are dropped (their blocks read as inactive) and counts->n_sites_needed
 * tells the required capacity; cap_sites = total_blocks never overflows.
 * ------------------------------------------------------------------------------------------- */
npvs_status npvs_rulebook_workspace_size(int32_t n_grids, const npvs_dims *dims, int32_t d, int32_t cap_sites,
                                         size_t *bytes);
npvs_status npvs_build_rulebook(const uint8_t *occ_bits, int32_t n_grids, const npvs_dims *dims, int32_t d,
                                int32_t cap_sites, npvs_counts *counts, int32_t *site_keys, int32_t *block_row,
                                int32_t *grid_rows, int32_t *nbr, int32_t *rb_off, int32_t *rb_pairs, void *ws,
                                size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------------------------
 * npvs_build_rulebook without caller workspace, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation): the same
 * arguments and results as npvs_build_rulebook except ws / ws_bytes.  Its workspace is a static
 * device array of NPVS_RULEBOOK_SCRATCH_BYTES (1 MiB) inside the library, one per GPU, held until
 * the process ends; the call allocates nothing (no hipMalloc, no library allocation).  A batch
 * whose workspace (npvs_rulebook_workspace_size) exceeds it is refused with NPVS_ERR_CAPACITY
 * before anything is enqueued (1 MiB covers 32 grids of 256x256x128 froxels at d = 4; a
 * 1024^3 grid at d = 4 needs about 1.7 MiB and is refused).  Calls that overlap on one GPU share that array and race: order
 * them on one stream.  Outputs are the caller's, as for npvs_build_rulebook.
 * ------------------------------------------------------------------------------------------- */
#define NPVS_RULEBOOK_SCRATCH_BYTES (1u << 20)
npvs_status npvs_build_rulebook_noalloc(const uint8_t *occ_bits, int32_t n_grids, const npvs_dims *dims, int32_t d,
                                        int32_t cap_sites, npvs_counts *counts, int32_t *site_keys,
                                        int32_t *block_row, int32_t *grid_rows, int32_t *nbr, int32_t *rb_off,
                                        int32_t *rb_pairs, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Interleave g_d and its inverse (Sec. 3.3): pure index permutations of a dense grid,
 *   out[bz][by][bx][c] = in[bz d + oz][by d + oy][bx d + ox],  c = (oz d + oy) d + ox,
 * for any element size (1, 2, 4 or 8 bytes).  in/out (device), not aliased.
 * ------------------------------------------------------------------------------------------- */
npvs_status npvs_interleave(const void *in, npvs_dims g, int32_t d, int32_t elem_bytes, void *out, void *stream);
npvs_status npvs_deinterleave(const void *in, npvs_dims g, int32_t d, int32_t elem_bytes, void *out, void *stream);

/* ---------------------------------------------------------------------------------------------
 * World-space front end (Sec. 3.2): the frustum F of a viewcell and the froxelization of
 * world-space triangles into F's froxels with linear depth slices.
 *
 * npvs_viewcell_frustum (host): a camera at c looking along `forward` (up hint `up`, not parallel
 *   to it) with vertical field of view fov_y radians and aspect ratio `aspect` may move
 *   laterally by up to r and turn by up to beta; F has its apex r / tan(fov_y / 2) behind c on the
 *   view axis and the field of view fov_y + 2 beta.  Writes the apex, the orthonormal basis
 *   (right = up x forward, up, forward), the half-angle tangents and the depth range.
 * npvs_froxelize_view: eye coordinates (x, y, z) = ((p - eye).right, (p - eye).up,
 *   (p - eye).forward); froxel (i, j, k) of grid g is the closed set with z in
 *   [z_near + k s, z_near + (k+1) s] (s = (z_far - z_near) / nz), x / z in
 *   [tx (2i/nx - 1), tx (2(i+1)/nx - 1)], y / z likewise with ty; G = 1 iff a triangle meets it
 *   (decided in float64: triangles clipped at z = z_near, mapped to (x/z, y/z, 1/z) where froxels
 *   are boxes; each row (j, k) of froxels is the slab y/z in its Y interval, 1/z in its Q
 *   interval, and the triangle's polygon clipped to that slab marks the froxels its X extent
 *   meets).  tris (device) float32 [T][3][3] in world units; view (host); occ_bits (device,
 *   4-byte aligned) packed as the grid-space froxelization, fully overwritten; nx a multiple of
 *   32; triangles with a non-finite coordinate are ignored.
 *   ws: npvs_froxelize_view_workspace_size(T) bytes.
 * ------------------------------------------------------------------------------------------- */
typedef struct {
  double eye[3], right[3], up[3], forward[3];
  double tan_half_x, tan_half_y;
  double z_near, z_far;
} npvs_view;
npvs_status npvs_viewcell_frustum(const double *c, const double *forward, const double *up, double fov_y,
                                  double aspect, double r, double beta, double z_near, double z_far, npvs_view *out);
npvs_status npvs_froxelize_view_workspace_size(int64_t n_tris, size_t *bytes);
npvs_status npvs_froxelize_view(const float *tris, int64_t n_tris, const npvs_view *view, npvs_dims g,
                                uint8_t *occ_bits, void *ws, size_t ws_bytes, void *stream);

/* Sparse interleave of a packed bit grid onto the active sites:
 *   X[r][c] = bit of froxel (bx d + ox, by d + oy, bz d + oz) of site r, as 0/1 in `dtype`
 *   (NPVS_F32, NPVS_BF16 or NPVS_U8).  X (device) [cap_sites][row_stride], row_stride = 0 meaning
 *   d^3; elements d^3 .. row_stride - 1 of a row are written as 0 (the input channels a BF16
 *   layer with fewer than 8 real ones reads, e.g. d = 1); rows >= n_sites untouched.
 * Used for the network input (bits = G) and for training labels.  bits2 / X2 (device, both or
 * neither): a second bit grid of the same grids, gathered in the same pass into uint8 rows
 * X2 [cap_sites][d^3] (a training step's labels beside its input: one launch instead of two). */
npvs_status npvs_gather_input(const uint8_t *bits, int32_t n_grids, const npvs_dims *dims, int32_t d,
                              const int32_t *site_keys, const npvs_counts *counts, int32_t cap_sites, int32_t dtype,
                              int32_t row_stride, void *X, const uint8_t *bits2, uint8_t *X2, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Weight packing.  W (device) float32 [27][cin][cout] -> Wp (device) of
 * npvs_packed_weight_bytes() bytes in the layout of `dtype`'s convolution kernel.
 * flip_transpose = 1 packs W'_k = (W_{26-k})^T, a [27][cout][cin] weight: the data gradient of
 * a submanifold layer is the same convolution run with W' (the rulebook is symmetric).
 * The size serves both orientations (for BF16 the larger one); the whole buffer is written,
 * entries past the orientation's own layout as zero.
 * ------------------------------------------------------------------------------------------- */
size_t npvs_packed_weight_bytes(int32_t cin, int32_t cout, int32_t dtype);
npvs_status npvs_pack_weights(const float *W, int32_t cin, int32_t cout, int32_t dtype, int32_t flip_transpose,
                              void *Wp, void *stream);

/* Several packings in one launch (a training step re-packs every layer, in both orientations,
 * after each optimizer update).  descs (host) [n]: each entry is one npvs_pack_weights call with
 * the same meaning of its fields; all entries use `dtype`.  At most NPVS_MAX_PACK entries; the
 * outputs must not overlap each other or any W. */
#define NPVS_MAX_PACK 64
typedef struct {
  const float *W;  /* (device) float32 [27][cin][cout] */
  void *Wp;        /* (device) npvs_packed_weight_bytes(cin, cout, dtype) bytes */
  int32_t cin, cout, flip_transpose, reserved;
} npvs_pack_desc;
npvs_status npvs_pack_weights_batch(int32_t n, const npvs_pack_desc *descs, int32_t dtype, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Submanifold sparse 3x3x3 convolution, forward (Sec. 2.3, 3.3):
 *   Y[r][o] = act(bias[o] + sum_k sum_c X[nbr[k][r]][c] W[k][c][o]),  act = ReLU if relu.
 * dtype NPVS_F32: X, Y float32, vector FMA.  dtype NPVS_BF16: X bfloat16, products on MFMA
 * with float32 accumulation, bias and ReLU in float32; Y is bfloat16, or float32 when
 * out_f32 = 1 (the logits of the last layer).
 *   X (device) [cap_sites][cin]; Wp packed weights; bias (device, nullable) float32 [cout];
 *   nbr, counts from npvs_build_rulebook; Y (device) [cap_sites][cout], rows >= n_sites untouched.
 * BF16 requires cin % 8 == 0 and cout % 8 == 0 (NPVS_ERR_UNSUPPORTED otherwise).
 * variant: the BF16 tile shape in [0, NPVS_CONV_VARIANTS), or -1 for NPVS_DEFAULT_CONV_VARIANT.
 *   Variants 0-5 split a tile's 27 offsets over several waves, (rows per wave, waves) = 0 (16, 9),
 *   1 (32, 1), 2 (16, 3), 3 (32, 3), 4 (16, 1), 5 (32, 9); variants 6-11 give each wave its own
 *   rows and all offsets and share each offset's weights through LDS, (rows per wave, waves) =
 *   6 (16, 4), 7 (16, 2), 8 (32, 2), 9 (16, 8), 10 (32, 4), 11 (32, 8); variants 12 and 13 (inputs
 *   of at most 64 channels) keep each wave's weights in registers while a workgroup walks several
 *   row tiles of 16 or 32 rows (32 outputs per workgroup); variant 14 is variant 12 with every
 *   output block (at most 64 outputs) in one workgroup, so a gathered row serves all outputs (more
 *   than 64 outputs: variant 12); variant 15 is variant 14 with three more waves that only sum
 *   the other waves' partial products and store the tile, while those go on to the next tile
 *   (at most 64 inputs and outputs; other shapes take variant 14).  Channel counts no tuned shape covers use a general kernel
 *   (variants 5 and 13 select its 32-row tiles), except 65 to 160 inputs, which take the
 *   weight-stationary kernel with 16-row tiles unless variant 5 is asked for.  All variants give
 *   results within float32 rounding of each other; each one is deterministic.  Ignored by the
 *   FP32 path.
 * ws (device, nullable): scratch of npvs_conv_fwd_workspace_size() bytes.  BF16 layers with 1024
 *   or more input channels (the first layer of interleave factor 16, cin = 4096) then split their
 *   input channels over several workgroups and add the partial sums in a fixed order (within
 *   float32 rounding of the unsplit kernel, deterministic); without it (or when the size is 0)
 *   the unsplit kernel runs.  A non-null ws of fewer bytes than needed is an argument error.
 * ------------------------------------------------------------------------------------------- */
#define NPVS_CONV_VARIANTS 16
#define NPVS_DEFAULT_CONV_VARIANT 15 /* the tile shape of variant -1 (the data gradient: variant 14's) */
npvs_status npvs_conv_fwd_workspace_size(int32_t cin, int32_t cout, int32_t cap_sites, int32_t dtype, size_t *bytes);
npvs_status npvs_sparse_conv_fwd(const void *X, int32_t cin, const void *Wp, const float *bias, int32_t cout,
                                 const int32_t *nbr, const npvs_counts *counts, int32_t cap_sites, int32_t dtype,
                                 int32_t relu, int32_t out_f32, int32_t variant, void *Y, void *ws, size_t ws_bytes,
                                 void *stream);

/* ---------------------------------------------------------------------------------------------
 * Backward of one submanifold layer (chain rule on the forward definition):
 *   dZ = dY * [Y > 0] when relu (ReLU'(0) = 0), else dY;
 *   dX[i] = sum_k sum_{(i,r) in R_k} dZ[r] W_k^T           (nullable dX: skipped)
 *   dW[k] = sum_{(i,r) in R_k} X[i]^T dZ[r],   db = sum_r dZ[r]   (float32, overwritten)
 *   X (device) layer input [cap][cin] in `dtype`; Y (device, used when relu) layer output
 *   [cap][cout] in `dtype`; dY (device) float32 [cap][cout]; Wt = npvs_pack_weights(W, ...,
 *   flip_transpose = 1); rb_off/rb_pairs: CSR rulebook.  dX is float32 [cap][cin].
 *   Reductions are deterministic (fixed order, compensated float32 sums).
 *   ws (device) workspace of npvs_conv_bwd_workspace_size() bytes.
 *   Any channel counts (BF16: multiples of 8, NPVS_ERR_UNSUPPORTED otherwise), e.g. the 512- and
 *   4096-channel first and last layers of interleave factors 8 and 16: dW is computed in windows
 *   of 64 x 64 channels, and the data gradient of a BF16 layer with 1024+ outputs splits its input
 *   channels over several workgroups (the workspace size covers it).
 * ------------------------------------------------------------------------------------------- */
/* dW and db both null: the weight gradient is not computed here; dZ and the bias partials stay in
 * ws for a later npvs_sparse_conv_wgrad (one non-null and one null is an argument error).
 * Streams: dZ and the bias partials are formed on `stream`, and the data gradient dX runs there.
 * wgrad_stream (nullable: `stream`) waits for dZ and computes the weight-gradient slices, so they
 * overlap the data-gradient chain of the layers below; reduce_stream (nullable: wgrad_stream)
 * waits for those and adds the slices and the bias partials into dW and db, so that the next
 * layer's weight gradient does not wait for this layer's reductions.  Until the caller makes
 * `stream` wait for the side streams, dW, db, X and ws are in use by them (do not read dW / db
 * or reuse ws or X before that).  All streams may be under capture (the waits are graph
 * dependencies). */
npvs_status npvs_conv_bwd_workspace_size(int32_t cin, int32_t cout, int32_t cap_sites, int32_t dtype, size_t *bytes);
npvs_status npvs_sparse_conv_bwd(const void *X, int32_t cin, const void *Wt, int32_t cout, const void *Y,
                                 const float *dY, const int32_t *nbr, const int32_t *rb_off, const int32_t *rb_pairs,
                                 const npvs_counts *counts, int32_t cap_sites, int32_t dtype, int32_t relu, float *dX,
                                 float *dW, float *db, void *ws, size_t ws_bytes, void *stream, void *wgrad_stream,
                                 void *reduce_stream);

/* ---------------------------------------------------------------------------------------------
 * The data gradient of a BF16 layer fused with the ReLU' of the layer below it (the chain rule
 * through two consecutive layers of the stack): from this layer's dZ [cap][cout], held by its
 * backward workspace ws (npvs_sparse_conv_bwd with dW = db = NULL, or an earlier call of this
 * function with ws as ws_below), computes dX = sum_k sum_{(i,r) in R_k} dZ[r] W_k^T and writes
 * the layer below's dZ_below = bf16(dX * [M > 0]) and its bias partials into ws_below, the
 * workspace of the layer below (cin_below -> cin channels), exactly as npvs_sparse_conv_bwd of
 * that layer with dY = dX and relu = 1 would form them (the same bfloat16 values; the bias
 * partials in another grouping), so its data gradient can follow with this function again and
 * its weight gradient with npvs_sparse_conv_wgrad.
 *   Wt = npvs_pack_weights(W, ..., flip_transpose = 1) of this layer (cin -> cout); M (device,
 *   nullable: no mask) the layer below's output = this layer's input X, bfloat16 [cap][cin].
 *   cin, cout <= 64 and multiples of 8; cin_below a multiple of 8 (NPVS_ERR_UNSUPPORTED
 *   otherwise).  ws and ws_below must differ.
 * Why: it removes the elementwise dZ pass (a launch-bound kernel) between the data gradients of
 * a stack of narrow layers.
 * ------------------------------------------------------------------------------------------- */
npvs_status npvs_sparse_conv_dgrad_relu(const void *Wt, int32_t cin, int32_t cout, const void *M, int32_t cin_below,
                                        const int32_t *nbr, const npvs_counts *counts, int32_t cap_sites,
                                        const void *ws, size_t ws_bytes, void *ws_below, size_t ws_below_bytes,
                                        void *stream);

/* ---------------------------------------------------------------------------------------------
 * Weight and bias gradients of several layers of one rulebook (the dW / db of the backward
 * above), in one weight-gradient launch and one reduction launch for all of them:
 *   layers (host) array of n_layers (1 .. NPVS_MAX_WGRAD_LAYERS) descriptors, read during the
 *   call: X (device) the layer input [cap][cin] in `dtype`; ws (device) the workspace that an
 *   npvs_sparse_conv_bwd call of that layer with dW = db = NULL left its dZ and bias partials in
 *   (same cin, cout, cap_sites, dtype; its slice partials are overwritten here); dW / db (device)
 *   float32 [27][cin][cout] / [cout], overwritten.
 *   rb_off / rb_pairs: the CSR rulebook of those backward calls.
 *   slices > 0: each offset's pair list is cut into that many slices (at most the single-layer
 *   count, which is used when larger), and the results equal npvs_sparse_conv_bwd's dW / db
 *   computed with the same slice count bit for bit (the single-layer call uses 16 slices for
 *   layers of at most 64 x 64 channels).  slices = 0 (BF16): the whole pair list of the 27
 *   offsets is cut into equal ranges, one per workgroup (as many as run at once), so that an
 *   offset with more pairs (the centre one pairs every site with itself) does not make its
 *   workgroups the last to finish; the sums are the same up to float32 regrouping.  The FP32
 *   path takes one weight-gradient launch per layer, each with that layer's single-layer slice
 *   count (or `slices` when smaller), and one reduction launch.
 * Why: a layer's weight gradient is a short latency-bound kernel; issued one layer at a time it
 * forms a serial chain behind the data gradients of the layers below, whereas all layers at once
 * fill the chip and pay the launch and memory round trips once (Sec. 3.3 trains the stack end to
 * end; the gradients themselves are those of the layer backward above).
 * ------------------------------------------------------------------------------------------- */
typedef struct {
  const void *X;
  int32_t cin, cout;
  void *ws;
  size_t ws_bytes;
  float *dW, *db;
} npvs_wgrad_layer;
npvs_status npvs_sparse_conv_wgrad(int32_t n_layers, const npvs_wgrad_layer *layers, const int32_t *rb_off,
                                   const int32_t *rb_pairs, int32_t cap_sites, int32_t dtype, int32_t slices,
                                   void *stream);

/* ---------------------------------------------------------------------------------------------
 * Two-level sparse U-Net pieces (Sec. 3.3 adopts an encoder/decoder backbone; the supplement's
 * network settings give a down ratio of 2 and 64 / 96 channels).  Level 0 is the rulebook of
 * interleave factor d, level 1 that of factor 2d (npvs_build_rulebook with 2d): its blocks are
 * the 2x2x2 groups of level-0 blocks that contain an active one.
 *
 * npvs_level_maps: children (device) int32 [8][cap1]: children[k][c] = level-0 row of child k
 *   = ((bz&1)*2 + (by&1))*2 + (bx&1) of level-1 row c, or -1; parent (device) int32 [cap0]:
 *   8 * (level-1 row) + k for level-0 row f.  Entries past the counts are -1.  The level-0 and
 *   level-1 site_keys / block_row / counts are those written by npvs_build_rulebook at d and 2d
 *   for the same grids (extents multiples of 2d, d <= 16).
 * npvs_packed_weight_bytes_k / npvs_pack_weights_k: float32 [K][cin][cout] weights of K offsets
 *   packed like npvs_pack_weights (no flip) with transpose = 0; with transpose = 1 the packing of
 *   the per-offset transposes W_k^T ([K][cout][cin], npvs_packed_weight_bytes_k(K, cout, cin,
 *   dtype) bytes), the weight of the data gradient.  The strided layers use K = 8.
 * npvs_strided_conv_fwd: up = 0, the convolution with kernel 2 and stride 2 (level 0 -> 1):
 *     Y[c] = act(b + sum_k X[children[k][c]] W_k), map = children, counts_out / cap_out of level 1;
 *   up = 1, its transposed convolution on the same blocks (level 1 -> 0):
 *     Y[f] = act(b + X[parent[f] / 8] W_{parent[f] % 8}), map = parent, counts_out / cap_out of
 *     level 0.
 *   X [cap_in][cin] and Y [cap_out][cout] in `dtype` (with BF16, Y is float32 when out_f32;
 *   cin, cout multiples of 8); Wp from npvs_pack_weights_k(K = 8); bias nullable; rows past the
 *   output count untouched.
 * npvs_concat_channels: Y[r] = [A[r] | B[r]] for r < n_sites, A [cap][ca], B [cap][cb],
 *   Y [cap][ca + cb], elements of elem_bytes (2 or 4) bytes, rows of A and B multiples of 16
 *   bytes; rows past n_sites untouched.
 * ------------------------------------------------------------------------------------------- */
npvs_status npvs_level_maps(int32_t n_grids, const npvs_dims *dims, int32_t d, const npvs_counts *counts0,
                            const int32_t *site_keys0, const int32_t *block_row0, int32_t cap0,
                            const npvs_counts *counts1, const int32_t *site_keys1, const int32_t *block_row1,
                            int32_t cap1, int32_t *children, int32_t *parent, void *stream);
size_t npvs_packed_weight_bytes_k(int32_t K, int32_t cin, int32_t cout, int32_t dtype);
npvs_status npvs_pack_weights_k(const float *W, int32_t K, int32_t cin, int32_t cout, int32_t transpose,
                                int32_t dtype, void *Wp, void *stream);
npvs_status npvs_strided_conv_fwd(const void *X, int32_t cin, const void *Wp, const float *bias, int32_t cout,
                                  const int32_t *map, int32_t up, const npvs_counts *counts_out, int32_t cap_out,
                                  int32_t dtype, int32_t relu, int32_t out_f32, void *Y, void *stream);
npvs_status npvs_concat_channels(const void *A, int32_t ca, const void *B, int32_t cb, int32_t elem_bytes,
                                 const npvs_counts *counts, int32_t cap, void *Y, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Backward of the U-Net's strided layers and skip concatenation (chain rule on the forward
 * definitions above; the paper trains its encoder/decoder backbone, Sec. 3.3, 4.2):
 * npvs_strided_conv_bwd: dZ = dY [Y > 0] when relu (ReLU'(0) = 0), else dY; for the strided
 *   convolution (up = 0: X level 0, Y level 1) dX0[child k of c] = dZ[c] W_k^T and
 *   dW_k = sum_c X0[child k of c]^T dZ[c]; for its inverse (up = 1: X level 1, Y level 0)
 *   dX1[c] = sum over the children f of c of dZ[f] W_{k(f)}^T and dW_k = sum over the level-0
 *   rows f with child index k of X1[parent f]^T dZ[f]; db = sum of dZ over the output rows.
 *   X (device) [cap_in][cin] and Y [cap_out][cout] in `dtype`; dY float32 [cap_out][cout];
 *   children / parent from npvs_level_maps; counts_in / counts_out the input and output level's
 *   counts; Wt = npvs_pack_weights_k(W, 8, cin, cout, transpose = 1, ...) (nullable when dX is);
 *   dX (nullable) float32 [cap_in][cin], dW float32 [8][cin][cout], db float32 [cout], all
 *   overwritten (rows of dX past the input count untouched).  ws (device) scratch of
 *   npvs_strided_bwd_workspace_size() bytes.  Deterministic (fixed reduction orders).  BF16:
 *   products on MFMA from bfloat16 dZ, cin and cout multiples of 8.
 * npvs_concat_channels_bwd: for r < n_sites, dA[r] = dY[r][0, ca) and dB[r] = dY[r][ca, ca + cb)
 *   (+ add_b[r] when add_b is given: the gradient the second part receives from elsewhere);
 *   float32, dA or dB nullable (not both), ca and cb multiples of 4, 16-byte aligned buffers.
 * ------------------------------------------------------------------------------------------- */
npvs_status npvs_strided_bwd_workspace_size(int32_t cin, int32_t cout, int32_t cap_in, int32_t cap_out, int32_t up,
                                            int32_t dtype, size_t *bytes);
npvs_status npvs_strided_conv_bwd(const void *X, int32_t cin, const void *Wt, int32_t cout, const void *Y,
                                  const float *dY, const int32_t *children, const int32_t *parent, int32_t up,
                                  const npvs_counts *counts_in, int32_t cap_in, const npvs_counts *counts_out,
                                  int32_t cap_out, int32_t dtype, int32_t relu, float *dX, float *dW, float *db,
                                  void *ws, size_t ws_bytes, void *stream);
npvs_status npvs_concat_channels_bwd(const float *dY, int32_t ca, int32_t cb, const float *add_b,
                                     const npvs_counts *counts, int32_t cap, float *dA, float *dB, void *stream);

/* ---------------------------------------------------------------------------------------------
 * De-interleave and threshold (Sec. 3.1 V = 1[f(G) >= tau] with tau = 0.5, read as logit >= 0;
 * Sec. 3.3 g_d^-1; Sec. 3.2 the visible set lies inside the occupied set, so V is masked by G):
 *   V(x) = [L(x) >= 0] and G(x),  L(x) = Y[row(block(x))][c(x)], -inf for inactive blocks.
 *   Y (device) float32 [cap][y_stride] (y_stride = 0 meaning d^3; a padded row, as the BF16 last
 *   layer of d = 1 writes, has its d^3 logits first); pvs_bits (device) packed like occ_bits, fully
 *   overwritten; logits (device, nullable) float32 dense [sum nz*ny*nx], grid after grid, fully
 *   overwritten.
 * ------------------------------------------------------------------------------------------- */
npvs_status npvs_deinterleave_threshold(const float *Y, int32_t y_stride, const int32_t *block_row,
                                        const uint8_t *occ_bits, int32_t n_grids, const npvs_dims *dims, int32_t d,
                                        uint8_t *pvs_bits, float *logits, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Culling against the PVS (the pipeline discards primitives whose froxels are all invisible,
 * Fig. 3; Sec. 5.6: the froxelized temporal bounding volume of a moving object is tested
 * against the froxelized PVS and the object is pruned when none of its froxels is visible).
 *   visible[t] = 1 iff some froxel that triangle t overlaps (the exact test of npvs_froxelize:
 *   closed froxels, 1/256 fixed point) has its bit set in pvs_bits, else 0; ignored triangles
 *   (|coordinate| >= 2048 or not finite) are 0.  tris, n_tris, n_grids, dims as for
 *   npvs_froxelize; pvs_bits (device) packed like occ_bits; visible (device) uint8 [total].
 * npvs_visible_objects: visible[i] = OR of vis_tris[obj_off[i] .. obj_off[i + 1] - 1];
 *   obj_off (device) int64 [n_objects + 1], non-decreasing, within vis_tris.
 * ------------------------------------------------------------------------------------------- */
npvs_status npvs_visible_triangles(const float *tris, const int64_t *n_tris, int32_t n_grids, const npvs_dims *dims,
                                   const uint8_t *pvs_bits, uint8_t *visible, void *stream);
npvs_status npvs_visible_objects(const uint8_t *vis_tris, const int64_t *obj_off, int64_t n_objects,
                                 uint8_t *visible, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Training loss per grid over the froxels of its active blocks (Sec. 3.3: repulsive visibility
 * loss L_rv = L_attr + L_rep with L_attr read as FN/GTP, L_rep = FP/GTP, combined with weight
 * lambda with a term T):
 *   p = sigmoid(l); TP = sum y p; FN = sum y (1-p); FP = sum (1-y) p; GTP = sum y;
 *   L = lambda T + (1-lambda)(FN + FP)/max(GTP, 1), with
 *   term = NPVS_LOSS_BCE:  T = BCE = mean(softplus(l) - y l) (alpha unused), or
 *   term = NPVS_LOSS_DICE: T = L_dice = 1 - 2 TP / (2 TP + alpha FN + (1-alpha) FP), the paper's
 *     weighted Dice term (alpha weighs the missed ground-truth froxels, as the text of Sec. 3.3
 *     says; the printed formulas name that term FP).
 * The batch loss is the mean over grids.
 *   logits (device) float32 [cap][C]; labels (device) uint8 [cap][C] 0/1; grid_rows from the
 *   rulebook; stats (device) float32 [n_grids + 1][8] = {L, T, L_rv, TP, FN, FP, GTP, m} per
 *   grid, row n_grids = batch mean; dlogits (device, nullable) float32 [cap][C] = dL_batch/dl,
 *   rows >= n_sites untouched.
 *   dz_ws (device, nullable): the BF16 backward workspace of the network's last layer (dz_cin ->
 *   C channels, npvs_conv_bwd_workspace_size bytes, dz_ws_bytes): the gradient is also written
 *   there as that layer's dZ (bfloat16; the last layer has no ReLU) and bias partials, exactly
 *   the values npvs_sparse_conv_bwd of that layer with dY = dlogits and dW = db = NULL forms, so
 *   that call can be skipped (its data gradient follows with npvs_sparse_conv_dgrad_relu, its
 *   weight gradient with npvs_sparse_conv_wgrad).  Needs C and dz_cin multiples of 8 and
 *   16-byte aligned logits / dlogits rows (NPVS_ERR_UNSUPPORTED otherwise).
 *   ws: npvs_loss_workspace_size() bytes.
 * ------------------------------------------------------------------------------------------- */
#define NPVS_LOSS_BCE 0
#define NPVS_LOSS_DICE 1
npvs_status npvs_loss_workspace_size(int32_t n_grids, size_t *bytes);
npvs_status npvs_loss(const float *logits, const uint8_t *labels, int32_t C, const int32_t *grid_rows,
                      int32_t n_grids, const npvs_counts *counts, int32_t cap_sites, float lambda, int32_t term,
                      float alpha, float *stats, float *dlogits, void *dz_ws, size_t dz_ws_bytes, int32_t dz_cin,
                      void *ws, size_t ws_bytes, void *stream);

/* Adam (Kingma & Ba) on float32 masters, with weight decay added to the gradient (read from the
 * decay rate the paper lists with the learning rate); p, g, m, v (device) float32 [n].  The step
 * counter lives on the device, so that a captured training step replays with the right bias
 * correction: `step` (device) is advanced on the stream first (t += 1, c1 = 1 - beta1^t,
 * c2 = 1 - beta2^t, each rounded from double to float), then the update uses its c1, c2 (start
 * from t = 0; a caller that counts on the host writes t - 1 before the call).
 * Each listed layer's updated weights are also written into its two packings in the same pass:
 * Wp = npvs_pack_weights(W, ..., flip_transpose = 0) and Wt = the flip_transpose = 1 packing
 * (forward and data gradient), both of npvs_packed_weight_bytes(cin, cout, dtype) bytes and
 * packed once before (their padding entries are not rewritten).  Layer l's weight [27][cin][cout]
 * is p[off, off + 27 cin cout); layers must not overlap; at most NPVS_MAX_ADAM_PACK layers (none
 * is fine), each of fewer than 2^31 weights (NPVS_ERR_UNSUPPORTED otherwise).  The result
 * equals the plain update followed by the two packings. */
typedef struct {
  int64_t t;
  float c1, c2;
} npvs_adam_step;
#define NPVS_MAX_ADAM_PACK 32
typedef struct {
  int64_t off;       /* first entry of the layer's weight in p */
  int32_t cin, cout;
  void *Wp, *Wt;     /* (device) the forward and the flipped-transpose packing */
} npvs_adam_pack_desc;
npvs_status npvs_adam(float *p, const float *g, float *m, float *v, int64_t n, npvs_adam_step *step, float lr,
                      float beta1, float beta2, float eps, float weight_decay, int32_t n_layers,
                      const npvs_adam_pack_desc *layers, int32_t dtype, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Whole forward pass V = threshold(g_d^-1(f(g_d(froxelize(tris))))) through a library-owned
 * plan that holds the workspace, the site table, the activations and the packed weights of a
 * fixed batch shape and network.  channels[0] must be d^3 and channels[n_layers] must be d^3;
 * ReLU follows every layer but the last.
 * ------------------------------------------------------------------------------------------- */
typedef struct npvs_plan npvs_plan;

npvs_status npvs_plan_create(int32_t n_grids, const npvs_dims *dims, const int64_t *n_tris, int32_t d,
                             int32_t n_layers, const int32_t *channels, int32_t dtype, npvs_plan **plan);
npvs_status npvs_plan_destroy(npvs_plan *plan);
/* W (device) float32 [27][cin][cout], b (device, nullable) float32 [cout] of layer `layer`. */
npvs_status npvs_plan_set_weights(npvs_plan *plan, int32_t layer, const float *W, const float *b, void *stream);
/* tris as in npvs_froxelize.  occ_bits (nullable) receives G; logits (nullable) as in
 * npvs_deinterleave_threshold; pvs_bits (device) receives V. */
npvs_status npvs_pvs_forward(npvs_plan *plan, const float *tris, uint8_t *occ_bits, uint8_t *pvs_bits, float *logits,
                             void *stream);
/* Capture one npvs_pvs_forward with these buffers into a HIP graph owned by the plan, then
 * replay it with npvs_plan_replay (one launch for the whole pass). */
npvs_status npvs_plan_capture(npvs_plan *plan, const float *tris, uint8_t *occ_bits, uint8_t *pvs_bits, float *logits,
                              void *stream);
npvs_status npvs_plan_replay(npvs_plan *plan, void *stream);
/* Autotuner: runs the pass once on `tris`, then times every BF16 tile shape (`reps` launches
 * each, HIP events on `stream`) for each distinct layer shape on the real rulebook and keeps the
 * fastest for later passes and captures (the default shape stays unless another is faster by
 * more than 3 %).  Synchronizes `stream`.  variants (host, nullable)
 * receives the chosen variant of each layer. */
npvs_status npvs_plan_autotune(npvs_plan *plan, const float *tris, int32_t reps, int32_t *variants, void *stream);
/* Synchronizes `stream` and copies the plan's npvs_counts to host memory; returns
 * NPVS_ERR_CAPACITY if the site capacity overflowed (it cannot with the plan's capacity). */
npvs_status npvs_plan_counts(npvs_plan *plan, npvs_counts *host_counts, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* NEURALPVS_H */
