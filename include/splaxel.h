/*
 * splaxel.h -- C ABI of libsplaxel.so, the MI355X (gfx950) hot path of
 * pixel-level distributed 3D Gaussian splatting (Splaxel, arXiv 2606.18588).
 *
 * One GPU renders the Gaussians of each convex cell (one GPU's partition in
 * the paper) into a *partial pixel* buffer (premultiplied colour C^m and
 * residual transmittance T^m, Eq. 3-4), composes the K partial buffers front
 * to back per pixel (Eq. 5) and back-propagates through the composition and
 * each local render (Eq. 6-7).  The paper's cross-GPU pixel exchange is
 * replaced by K buffers resident in HBM.
 *
 * Conventions for every call:
 *   - Array arguments are DEVICE pointers owned by the caller unless a
 *     comment says "host".  The library never allocates device memory; the
 *     caller provides workspaces sized by the *_workspace_size queries (one
 *     exception: the static scratch array of sx_render_backward_noalloc).
 *   - All work is enqueued on `stream` (a hipStream_t; NULL = the default
 *     stream) and is asynchronous unless a comment says the call
 *     synchronises.
 *   - Return value: SX_OK (0) or a negative sx_status.  Argument errors are
 *     detected on the host before anything is enqueued (SX_EINVAL);
 *     launch/runtime failures map to SX_EDEVICE.  No C++ exception or abort
 *     crosses the ABI; sx_last_error_string() describes the last failure of
 *     the calling thread.
 *   - Layouts are row-major; pixel (x, y) has index y*W + x and its centre
 *     at (x + 0.5, y + 0.5).  FP32 throughout unless stated.
 *   - Device arrays start on 16-byte boundaries (the kernels use vector
 *     loads; hipMalloc and torch allocations qualify).
 *   - Calls on distinct streams with distinct buffers are independent; the
 *     library holds no mutable global state.
 */
#ifndef SPLAXEL_H
#define SPLAXEL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sx_status;
#define SX_OK 0
#define SX_EINVAL (-1)      /* null/inconsistent argument, unsupported size */
#define SX_ECAPACITY (-2)   /* instance count exceeds the caller's capacity */
#define SX_EDEVICE (-3)     /* HIP launch or runtime error                  */
#define SX_EUNSUPPORTED (-4)

typedef void* sx_stream; /* hipStream_t */

/* Pinhole camera: x_cam = R x_world + t, OpenCV axes (x right, y down,
 * z forward); R row-major. */
typedef struct sx_camera {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height;
  float znear; /* Gaussians whose mean has camera z <= znear are culled */
} sx_camera;

/* Rendering constants.  tile_w*tile_h pixels form one work item; supported
 * shapes: 16x16, 32x8, 8x32, 32x16, 16x32, 8x8. */
typedef struct sx_params {
  int32_t tile_w, tile_h;
  int32_t sh_degree; /* 0..3 */
  int32_t flags;     /* SX_FLAG_* */
  float alpha_min;   /* pairs with alpha < alpha_min are skipped (1/255)  */
  float alpha_max;   /* alpha = min(alpha_max, o exp(-q/2)) (0.99)        */
  float t_min;       /* stop after the blend that takes T below it (1e-4);
                        also the saturation threshold of the composition  */
  float eps2d;       /* added to the diagonal of the 2D covariance (0.3)  */
  float bg[3];       /* background colour composed behind the last cell   */
  float fov_guard;   /* frustum cull by the mean: a Gaussian is culled when
                        its mean projects farther from the principal point
                        than fov_guard times the image's half-extent on that
                        side (1.3); 0 disables the lateral test            */
} sx_params;

/* treat (cell, pixel) pairs behind a saturated prefix as the identity in
 * the same frame (otherwise they are only marked inactive for the next
 * render of the view) */
#define SX_FLAG_SAME_FRAME_CULL 1

/* Gaussian parameters of one cell, SoA FP32, device pointers:
 *   means[n*3], log_scales[n*3], quats[n*4] (w,x,y,z, need not be unit),
 *   opacity_logits[n], sh[n*(D+1)^2*3] (coefficient l*l+l+m, channel
 *   fastest).  The parametrisation is the paper's background section:
 *   Sigma = R(q) S S^T R(q)^T, S = diag(exp(log_scales)),
 *   o = sigmoid(logit), colour = max(0, sum_lm k_lm Y_lm(dir) + 0.5). */
typedef struct sx_gaussians {
  int64_t n;
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* opacity_logits;
  const float* sh;
} sx_gaussians;

/* Per-Gaussian projection written by sx_preprocess (caller-allocated):
 *   rec[n*12]   float record: mean2d - (cx, cy) (2), conic a, b, c of the
 *               inverse 2D covariance (3), opacity, rgb (3), camera depth,
 *               then the pixel box [x0, x1] x [y0, y1] of the exact
 *               alpha >= alpha_min footprint as two uint32 words
 *               x0 | (x1 - x0) << 16 and y0 | (y1 - y0) << 16 (the
 *               render walks an entry only for the pixel rectangles its
 *               box meets).  Valid only where n_tiles > 0.
 *   rect[n*4]   uint16 tile rectangle [x0, y0, x1, y1) of the exact
 *               alpha >= alpha_min footprint.
 *   n_tiles[n]  tiles touched; 0 = culled.
 *   block_sums[sx_preprocess_blocks(n)*2]  per-block (visible, instances)
 *               partial sums consumed by sx_sort. */
typedef struct sx_projected {
  float* rec;
  uint16_t* rect;
  uint32_t* n_tiles;
  uint32_t* block_sums;
  /* optional per-ray cross-boundary filter of this cell's render and its
   * backward (sx_cross_filter); xf NULL = off.  Only sx_render_partial,
   * sx_render_backward(_stages) and sx_backward apply it; the batched
   * multi-view calls reject it.
   *   xf       [n] filter bits written by sx_cross_filter
   *   omega    the K geometric maps of the view (sx_visibility layout)
   *   cell     this cell's index in 0..n_cells-1
   *   n_cells  K, 1..16 */
  const uint32_t* xf;
  const uint32_t* omega;
  int32_t cell, n_cells;
} sx_projected;

/* Axis-aligned convex cell (one GPU's partition); bounds may be +-inf. */
typedef struct sx_cell {
  float lo[3];
  float hi[3];
} sx_cell;

/* Parameter gradients of one cell, same layouts as sx_gaussians. */
typedef struct sx_grads {
  float* means;
  float* log_scales;
  float* quats;
  float* opacity_logits;
  float* sh;
} sx_grads;

const char* sx_last_error_string(void);
const char* sx_version(void);

/* ------------------------------------------------------------------ a1 --
 * Projection of one cell's Gaussians for one camera (paper, background:
 * projection step; Eq. 1 footprint).  Per Gaussian: cull by mean depth,
 * Sigma2D = J W Sigma W^T J^T + eps2d I (EWA), conic = Sigma2D^-1, mean2d,
 * depth, SH colour, opacity, exact alpha >= alpha_min footprint, tiles
 * touched.  Computed in FP64, stored in FP32.
 * Errors: SX_EINVAL for null pointers, n < 0, n >= 2^31, sh_degree > 3,
 * unsupported tile shape, or width/height outside 1..16384. */
int64_t sx_preprocess_blocks(int64_t n);
sx_status sx_preprocess(const sx_gaussians* g, const sx_camera* cam,
                        const sx_params* p, sx_projected* out,
                        sx_stream stream);

/* ------------------------------------------------------------- a2-a4 --
 * Depth sort (paper, background: sorting step): the result of a stable
 * sort of the 64-bit keys  key = tile_id << 32 | bits(float32 depth)  with
 * ties by Gaussian index.  The visible Gaussians' instances are binned by
 * tile (a count pass, a scan and a write pass), then every tile's list is
 * sorted by (depth bits, index) in LDS.
 * Outputs: vals[i] = Gaussian index of the i-th instance, optionally
 * keys[i], and tile_ranges[t] = [start, end) per tile (tile_id = ty *
 * tiles_x + tx; an empty tile has start == end), tiles * 2 uint32.
 *   capacity   instances the caller allocated in keys/vals.
 *   ws         workspace of sx_sort_workspace_size(n, capacity, tiles_x,
 *              tiles_y) for this view's tile grid.
 *   h_counts   HOST uint64[2] or NULL.  If non-NULL the call synchronises
 *              the stream once after counting, writes {visible,
 *              instances} and returns SX_ECAPACITY (with nothing sorted)
 *              when instances > capacity.  If NULL the call is fully
 *              asynchronous; an overflow writes no instance (every tile
 *              range is empty) and raises a flag read by sx_sort_counts().
 * The workspace begins with uint64 {visible, instances, overflow, error}
 * (32 bytes, valid once the call's work has completed), so a caller may
 * also copy them to pinned host memory asynchronously (error is reserved
 * and left 0: no step of the sort waits on another workgroup).
 * keys may be NULL. */
/* Bytes of the sort workspace for n Gaussians, `capacity` instances and a
 * tiles_x x tiles_y grid: about 20 bytes per Gaussian (the compacted
 * visible list), 16 bytes per instance (the per-tile lists and their merge
 * buffer) and 8 bytes per tile. */
sx_status sx_sort_workspace_size(int64_t n, int64_t capacity,
                                 int32_t tiles_x, int32_t tiles_y,
                                 size_t* bytes);
sx_status sx_sort(const sx_projected* proj, int64_t n, const sx_camera* cam,
                  const sx_params* p, int64_t capacity, uint64_t* keys,
                  uint32_t* vals, uint32_t* tile_ranges, void* ws,
                  size_t ws_bytes, uint64_t* h_counts, sx_stream stream);
/* Reads the four count words of a sort workspace into HOST uint64[4]:
 * {visible, instances, overflow, error}; synchronises the stream.
 * overflow != 0: the instances exceeded the capacity (nothing was binned:
 * every tile range is empty); error != 0 means the list must not be used
 * (reserved: the current sort always leaves it 0). */
sx_status sx_sort_counts(const void* ws, int64_t n, uint64_t* h_out,
                         sx_stream stream);

/* ------------------------------------------------------------------ a5 --
 * Partial render of one cell (Eq. 1-4): per pixel, front to back over its
 * tile's list, alpha = min(alpha_max, o exp(-q/2)); skip alpha < alpha_min;
 * C += c alpha T, D += z alpha T, T *= 1 - alpha; stop after T < t_min.
 *   mask       active bits, bit (y*W+x) of uint32 words, NULL = all.
 *              Inactive pixels output the identity (C=0, T=1).
 *   partial    [H*W*4] out: (C_r, C_g, C_b, T) per pixel.
 *   depth      [H*W] out or NULL: D = sum z alpha T.
 *   last       [H*W] out: 1 + position (within the tile list) of the last
 *              blended pair, 0 if none; needed by the backward.
 *   nblend     [H*W] out or NULL: number of blended pairs. */
sx_status sx_render_partial(const sx_projected* proj, const uint32_t* vals,
                            const uint32_t* tile_ranges, const sx_camera* cam,
                            const sx_params* p, const uint32_t* mask,
                            float* partial, float* depth, uint32_t* last,
                            uint32_t* nblend, sx_stream stream);

/* KD-tree partition of n Gaussians into K convex cells by their means (the
 * paper's partition strategy): recursive binary splits, each along the axis
 * on which the node's means have the largest extent, at the quantile that
 * gives the two halves their share of cells (the median for K a power of
 * two); means < split go left.  Cells are numbered depth first, left
 * before right; the boxes are disjoint half-open boxes that cover space
 * (outermost bounds infinite).  HOST arrays: means [n*3], cells [K] (out),
 * cell_of [n] (out).  K in 1..16.  Runs on the host; allocates host memory
 * only. */
sx_status sx_kd_partition(int64_t n, const float* means, int32_t K, sx_cell* cells,
                          int32_t* cell_of);

/* Load monitoring and repartitioning (the paper's appendix, implementation
 * details: the imbalance ratio N_max / mean(N) - 1 of the cells' Gaussian
 * counts is checked during training and the cells are repartitioned when it
 * exceeds 20%; on one GPU the all-to-all redistribution is a move of rows
 * between cell buffers).
 * sx_imbalance: ratio of HOST counts[K] (K in 1..16, at least one
 *   Gaussian) into *ratio.  Host code.
 * sx_repartition_plan: for HOST cell_of[n] (the new cell of every Gaussian,
 *   indexed over the old cells laid end to end, e.g. from sx_kd_partition
 *   of all their means), writes HOST dst_index[n] (each Gaussian's row in
 *   its new cell: its rank among that cell's Gaussians, in the old order)
 *   and counts[K] (the new cell sizes).  Host code.
 * sx_move_rows: moves rows of row_floats floats (one parameter array, or an
 *   optimiser state of the same layout) from K_src source buffers (HOST
 *   array of device pointers, src_counts[K_src] rows each, laid end to end
 *   in that order) to K_dst destination buffers (HOST array of device
 *   pointers, each sized for its new count): row g goes to row dst_index[g]
 *   of buffer dst_cell[g] (DEVICE int32 [n] each, n = sum of src_counts).
 *   Destinations must not overlap sources.  Asynchronous on `stream`. */
sx_status sx_imbalance(int32_t K, const int64_t* counts, double* ratio);
sx_status sx_repartition_plan(int64_t n, const int32_t* cell_of, int32_t K, int32_t* dst_index,
                              int64_t* counts);
sx_status sx_move_rows(int32_t row_floats, int32_t K_src, const int64_t* src_counts,
                       const float* const* src, int32_t K_dst, float* const* dst,
                       const int32_t* dst_cell, const int32_t* dst_index, sx_stream stream);

/* Geometric visibility of K cell boxes for one view (redundancy reduction
 * section, spatial part): the part of a box inside the view frustum is
 * convex, and its projection onto the image is the set of pixels whose
 * centre ray meets it (between the near plane and infinity).  Writes masks
 * [K * ceil(H*W/32)] uint32 words, cell-major, bit (m, p) = 1 where cell m
 * is visible at pixel p, in the layout of sx_composite's saturation masks:
 * initialising those masks with this map restricts every render and
 * composition of the view to the cells' visible regions.  cells: HOST array
 * of K boxes (bounds may be infinite), K in 1..16. */
sx_status sx_visibility(int32_t K, const sx_cell* cells, const sx_camera* cam,
                        uint32_t* masks, sx_stream stream);

/* Pixels per cell of K mask rows of `words` uint32 words each (the layout
 * of sx_visibility): counts[m] (device, K uint32) = set bits of row m.  The
 * cells with a non-empty geometric map are a view's participants, the set
 * the paper's view bucketing (Sec. 4.4, GetParticipants) schedules by. */
sx_status sx_mask_counts(int32_t K, const uint32_t* masks, int64_t words, uint32_t* counts,
                         sx_stream stream);

/* Per-ray cross-boundary filter (appendix, implementation details:
 * cross-boundary Gaussians).  A Gaussian assigned to cell k by its mean
 * whose spatial support reaches into cell s is removed from the ray of
 * pixel p when its depth lies in the overlapped depth interval of k and s
 * and p lies in both cells' visibility maps, so that the composition of
 * the two partials does not interleave their Gaussians.  Readings: support
 * = the axis-aligned box mean +- 3 sqrt(Sigma_aa); depth = camera z of the
 * mean (the record's depth); overlapped interval = intersection of the
 * camera-z ranges of the two boxes.
 * Writes xf[i] (device, [n]): bit s set when Gaussian i is visible in the
 * view (n_tiles > 0 after sx_preprocess), s != cell, its support box meets
 * box s and its depth is in the interval of (cell, s).  proj must hold the
 * preprocess output of this view; cells: HOST array of K boxes (K in
 * 1..16), cell in 0..K-1.  To apply the filter, set proj->xf, omega, cell
 * and n_cells for the render and backward calls. */
sx_status sx_cross_filter(const sx_gaussians* g, const sx_projected* proj, int32_t K,
                          const sx_cell* cells, int32_t cell, const sx_camera* cam,
                          uint32_t* xf, sx_stream stream);

/* ------------------------------------------------------------------ a6 --
 * Composition of K partial buffers (Eq. 5).  Per pixel the cells are
 * ordered by the ray's entry parameter into their box, max(0, t_near)
 * (ties by cell index); C = sum_j P_j C_j, P_{j+1} = P_j T_j; output
 * (C + P_{K+1} bg, P_{K+1}).  Saturation (redundancy reduction): when
 * P_j < t_min the bit of (cell m_j, pixel) is cleared in masks for the
 * next render of the view (and, with SX_FLAG_SAME_FRAME_CULL, the cell is
 * skipped now).
 *   partials  HOST array of K device pointers to [H*W*4] buffers.
 *   cells     HOST array of K boxes.
 *   out       [H*W*4] (rgb, T).
 *   masks     [K * ceil(H*W/32)] uint32 words, cell-major, or NULL; bits
 *             are only cleared, so the caller initialises them (all ones
 *             = every pair active).
 * K in 1..16. */
sx_status sx_composite(int32_t K, const float* const* partials,
                       const sx_cell* cells, const sx_camera* cam,
                       const sx_params* p, float* out, uint32_t* masks,
                       sx_stream stream);

/* Composition with the saturation state carried between renders of a view
 * and its speculative re-evaluation (appendix, experimental analysis:
 * saturation stability during training), so that pairs pruned by
 * saturation come back when the transmittance in front of them recovers.
 * Same order, output and K range as sx_composite; per pixel, with P the
 * incoming transmittance of the cells rendered now:
 *   - a pair whose masks bit is set (rendered now) keeps it while
 *     P >= t_min; otherwise the bit is cleared and budget[m*H*W + p] =
 *     P (1 - T_m), its transmittance consumption;
 *   - a pair whose bit is clear and whose box the ray meets (omega bit set,
 *     or omega NULL) is re-activated, in entry order, while the residual
 *     R = P - S reaches t_min and R >= its budget (S: budgets of the pairs
 *     re-activated before it on this ray); the first that fails ends the
 *     scan for the pixel;
 *   - other pairs are cleared.
 *   masks   [K * ceil(H*W/32)] words, read and rewritten (bits past H*W
 *           cleared); partials of cleared pairs must be the identity
 *           (0, 0, 0, 1), as sx_render writes them.
 *   omega   the geometric map of sx_visibility, same layout, or NULL.
 *   budget  [K * H * W] floats owned by the caller, zero-initialised once
 *           per view and kept with its masks: read for pairs pruned in an
 *           earlier render, written for pairs pruned now.
 * A pair cleared by other means (sx_composite, sx_visibility, the caller)
 * is tested with whatever budget the buffer holds for it (zero after
 * initialisation). */
sx_status sx_composite_reeval(int32_t K, const float* const* partials,
                              const sx_cell* cells, const sx_camera* cam,
                              const sx_params* p, float* out, uint32_t* masks,
                              const uint32_t* omega, float* budget, sx_stream stream);

/* L1 loss of the composed image (the RGB term of the paper's loss):
 * dout[H*W*4] = (sign(rgb - target) / (3HW), 0); loss_sum (device float,
 * may be NULL) receives += the mean absolute error.  target [H*W*3]. */
sx_status sx_l1_loss(const float* out, const float* target, int32_t width,
                     int32_t height, float* dout, float* loss_sum,
                     sx_stream stream);

/* The composition (Eq. 5, as sx_composite with its clearing rule), the L1
 * loss of the composed image (the RGB term of the paper's loss) and the
 * composition backward of that loss (Eq. 6-7; as
 * sx_l1_loss followed by sx_composite_backward) in one pass over the
 * pixels; the results are bit-identical to the three calls.
 *   target [H*W*3]; out [H*W*4]; masks as sx_composite (or NULL);
 *   loss_sum (device float, may be NULL) receives += the mean absolute
 *   error; dpartials HOST array of K device pointers to [H*W*4] buffers
 *   receiving dL/d(C^m, T^m). */
sx_status sx_composite_l1(int32_t K, const float* const* partials, const sx_cell* cells,
                          const sx_camera* cam, const sx_params* p, const float* target,
                          float* out, uint32_t* masks, float* loss_sum,
                          float* const* dpartials, sx_stream stream);

/* ------------------------------------------------------------- a7-a9 --
 * Backward through the composition and every cell's render and
 * projection (Eq. 6-7).  For cell m at pixel p with order position j:
 * dC^m = P_j G, dT^m = P_j (G . B_{j+1} + g_T U_j) with B the colour behind
 * the cell (background included) and U_j the transmittance behind it; then
 * a reverse walk of the cell's blended pairs gives per-Gaussian gradients of
 * mean2d, conic, opacity, colour and depth, chained to the parameters.
 * Per cell (sx_cell_state, device pointers):
 *   g, proj, vals, ranges, sort_ws, capacity
 *                                   the cell's inputs, sort outputs and the
 *                                   sort workspace/capacity they came from
 *   partial, last, mask             its forward outputs / mask (mask NULL =
 *                                   all active)
 *   grads                           parameter gradients: rows of Gaussians
 *                                   visible in this view are written
 *                                   (or accumulated with SX_BWD_ACCUMULATE);
 *                                   other rows are untouched
 *   g2d_ws                          [n*12] scratch (screen-space grads)
 *   dpartial_ws                     [H*W*4] scratch (dL/d(C^m, T^m))
 *   bwd_ws                          sx_backward_workspace_size bytes
 * The render backward uses no global atomics: every (Gaussian, tile) pair
 * stores its partial gradient row at the instance's own slot of bwd_ws and
 * a balanced per-Gaussian reduction sums the valid slots.
 * dout [H*W*4]: dL/d(rgb, T) of the composed image.
 * cells: HOST array of K boxes (same order as the forward). */
#define SX_BWD_ACCUMULATE 1
typedef struct sx_cell_state {
  const sx_gaussians* g;
  const sx_projected* proj;
  const uint32_t* vals;
  const uint32_t* ranges;
  const void* sort_ws;
  int64_t capacity;
  const float* partial;
  const uint32_t* last;
  const uint32_t* mask;
  const sx_grads* grads;
  float* g2d_ws;
  float* dpartial_ws;
  void* bwd_ws;
} sx_cell_state;

sx_status sx_backward_workspace_size(int64_t capacity, int64_t tiles_total,
                                     size_t* bytes);

sx_status sx_backward(int32_t K, const sx_cell_state* cells,
                      const sx_cell* boxes, const sx_camera* cam,
                      const sx_params* p, const float* dout, int32_t flags,
                      sx_stream stream);

/* Stages of sx_backward, exposed for testing and for callers that
 * schedule them themselves. */
sx_status sx_composite_backward(int32_t K, const float* const* partials,
                                const sx_cell* cells, const sx_camera* cam,
                                const sx_params* p, const uint32_t* masks,
                                const float* dout, float* const* dpartials,
                                sx_stream stream);
/* writes screen-space gradients of the Gaussians visible in the view:
 * g2d[i*12 + 0..9] = d(mean2d x, y, conic a, b, c, opacity, r, g, b,
 * depth); sort_ws/capacity are those of the sx_sort call that produced
 * vals and tile_ranges, bwd_ws has sx_backward_workspace_size bytes */
sx_status sx_render_backward(const sx_projected* proj, const uint32_t* vals,
                             const uint32_t* tile_ranges, const void* sort_ws,
                             int64_t n, int64_t capacity, void* bwd_ws,
                             const sx_camera* cam,
                             const sx_params* p, const uint32_t* mask,
                             const float* partial, const uint32_t* last,
                             const float* dpartial, const float* ddepth,
                             float* g2d, sx_stream stream);
/* The three stages of sx_render_backward, for callers that schedule or time
 * them separately; stages is a mask of SX_RB_* bits and the stages must run
 * in this order on one stream with the same arguments:
 *   SX_RB_PREPARE  entries each tile's reverse walk visits (the largest
 *                  `last` over its pixels);
 *   SX_RB_WALK     the reverse walk (Eq. 6-7): one gradient row per
 *                  (Gaussian, tile) instance in bwd_ws, at the instance's
 *                  place in its Gaussian's tile rectangle (zeros for the
 *                  entries no pixel reached);
 *   SX_RB_REDUCE   each visible Gaussian's contiguous rows summed into g2d.
 * sx_render_backward is this call with SX_RB_ALL. */
#define SX_RB_PREPARE 1
#define SX_RB_WALK 2
#define SX_RB_REDUCE 4
#define SX_RB_ALL 7
sx_status sx_render_backward_stages(const sx_projected* proj, const uint32_t* vals,
                                    const uint32_t* tile_ranges, const void* sort_ws,
                                    int64_t n, int64_t capacity, void* bwd_ws,
                                    const sx_camera* cam, const sx_params* p,
                                    const uint32_t* mask, const float* partial,
                                    const uint32_t* last, const float* dpartial,
                                    const float* ddepth, float* g2d, int32_t stages,
                                    sx_stream stream);
/* sx_render_backward for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same arguments and results (the same kernels) without
 * bwd_ws.  Its scratch, the per-tile visited counts and one 40-byte
 * gradient row per instance (sx_backward_workspace_size(capacity, tiles)
 * bytes), is a static device array of SX_NOALLOC_SCRATCH_BYTES that every
 * device the library runs on holds until the process ends (64 MiB: about
 * 1.6M instances at 1080p with 16x16 tiles).  A capacity whose scratch does
 * not fit returns SX_EINVAL before anything is enqueued.  Calls no
 * allocator.  All calls on one device share the array: calls that overlap
 * in time on one device (on different streams, or from different threads)
 * race and must be ordered by the caller.  No part of the array needs
 * clearing between calls (each call writes every row and count it reads). */
#define SX_NOALLOC_SCRATCH_BYTES (64ull << 20)
sx_status sx_render_backward_noalloc(const sx_projected* proj, const uint32_t* vals,
                                     const uint32_t* tile_ranges, const void* sort_ws,
                                     int64_t n, int64_t capacity, const sx_camera* cam,
                                     const sx_params* p, const uint32_t* mask,
                                     const float* partial, const uint32_t* last,
                                     const float* dpartial, const float* ddepth, float* g2d,
                                     sx_stream stream);
/* sort_ws/capacity: the sort of this view (its list of visible Gaussians
 * drives the launch). */
sx_status sx_preprocess_backward(const sx_gaussians* g, const sx_camera* cam,
                                 const sx_params* p, const sx_projected* proj,
                                 const void* sort_ws, int64_t capacity,
                                 const float* g2d,
                                 const sx_grads* grads, int32_t flags,
                                 sx_stream stream);

/* ----------------------------------------------------------------- a10 --
 * Adam (the paper's optimiser is unnamed; textbook Adam with bias
 * correction) over n FP32 elements: m = b1 m + (1-b1) g,
 * v = b2 v + (1-b2) g^2, param -= lr (m / (1-b1^t)) / (sqrt(v/(1-b2^t)) +
 * eps). */
sx_status sx_adam(int64_t n, float* param, const float* grad, float* m,
                  float* v, int32_t step, float lr, float beta1, float beta2,
                  float eps, sx_stream stream);

/* Fill n uint32 words with a value (kernel, safe inside graph capture). */
sx_status sx_fill_u32(uint32_t* ptr, int64_t n, uint32_t value,
                      sx_stream stream);

/* ----------------------------------------------------------------- a11 --
 * Batched views.  The paper spreads the views of a training batch over
 * GPUs and groups views whose participant cells do not overlap (Sec. 4.4,
 * view bucketing); on one GPU the views of a batch share the device, so the
 * batched calls below run the per-view stages of up to SX_MAX_VIEWS items in
 * one launch each: workgroup b takes the b-th (item, tile) work unit, the
 * items' tile grids laid end to end, each in raster order.  An item is one
 * view of one cell; the items of a render or render-backward launch may
 * belong to different cells (each carries its cell's projection, sort and,
 * for the backward, Gaussian count), which is how a bucket of views with
 * disjoint participant cells runs in one launch.  Results are
 * bit-identical to the per-view calls (every work item owns its pixels;
 * the per-Gaussian gradient rows of each item are reduced separately). */
#define SX_MAX_VIEWS 16

/* One view of a batched call.  Every pointer refers to that view's buffers
 * exactly as the matching per-view call takes them (sizes follow cam). */
typedef struct sx_view {
  sx_camera cam;
  sx_projected proj;           /* sx_preprocess(_multi) output          */
  const uint32_t* vals;        /* sx_sort output                        */
  const uint32_t* tile_ranges; /* sx_sort output                        */
  const void* sort_ws;         /* this view's sort workspace            */
  int64_t capacity;            /* its instance capacity                 */
  const uint32_t* mask;        /* optional active-pixel bits, or NULL   */
  float* partial;              /* [H*W*4] (C, T)                        */
  float* depth;                /* optional [H*W], or NULL               */
  uint32_t* last;              /* [H*W]                                 */
  uint32_t* nblend;            /* optional [H*W], or NULL               */
  const float* dpartial;       /* backward: [H*W*4] upstream gradient   */
  float* g2d;                  /* backward: [n*12] screen gradients     */
  void* bwd_ws;                /* backward: sx_backward_workspace_size  */
  int64_t n;                   /* backward: Gaussians of this item's
                                  cell, or 0 for the call's n           */
} sx_view;

/* Preprocess of one cell's Gaussians for V views in one launch (Eq. 1
 * projection and SH colour per view).  outs[v] is laid out as for
 * sx_preprocess with cams[v]; host arrays cams[V], outs[V]. */
sx_status sx_preprocess_multi(const sx_gaussians* g, int32_t V,
                              const sx_camera* cams, const sx_params* p,
                              sx_projected* outs, sx_stream stream);

/* Workspace of the batched launches: bytes for V views with cams[V] (the
 * current launches need only a small block; callers size it with this query
 * so the layout can change without an interface change). */
sx_status sx_multi_workspace_size(int32_t V, const sx_camera* cams,
                                  const sx_params* p, size_t* bytes);

/* Partial render (Eq. 3-4) of V views in one launch (one workgroup per
 * (view, tile)); each view needs proj, vals, tile_ranges, mask, partial,
 * depth, last, nblend.
 * views: host array [V]; ws: device workspace (contents scratch). */
sx_status sx_render_multi(int32_t V, const sx_view* views,
                          const sx_params* p, void* ws, size_t ws_bytes,
                          sx_stream stream);

/* Render backward (Eq. 6-7 through each item's local render) of V items in
 * one launch, then each item's per-Gaussian reduction into views[v].g2d;
 * each item needs every member; an item's cell has views[v].n Gaussians,
 * or n when that member is 0.
 * Follow with sx_preprocess_backward_multi (or sx_preprocess_backward per
 * view) to sum the views' parameter gradients. */
sx_status sx_render_backward_multi(int32_t V, const sx_view* views, int64_t n,
                                   const sx_params* p, void* ws,
                                   size_t ws_bytes, sx_stream stream);

/* Parameter gradients (chain of the projection, Eq. 1, and of the SH
 * colour) summed over V views of the Gaussians g; each view needs cam,
 * proj.n_tiles (its sx_preprocess output), sort_ws/capacity (its sx_sort)
 * and g2d (its sx_render_backward output).  Per Gaussian the views'
 * contributions are added in view order: the result equals
 * sx_preprocess_backward called per view with SX_BWD_ACCUMULATE on the same
 * grads, bit for bit.  flags: SX_BWD_ACCUMULATE adds to grads (rows of
 * Gaussians no view sees are left untouched); without it grads are
 * overwritten with the sum (zero rows for Gaussians no view sees).
 * views: host array [V], V in 1..SX_MAX_VIEWS. */
sx_status sx_preprocess_backward_multi(const sx_gaussians* g, int32_t V,
                                       const sx_view* views, const sx_params* p,
                                       const sx_grads* grads, int32_t flags,
                                       sx_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* SPLAXEL_H */
