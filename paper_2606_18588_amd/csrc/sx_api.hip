// Host side of the C ABI declared in include/splaxel.h: argument
// validation, conversion of the camera/parameters to kernel form, and
// mapping of HIP errors to sx_status.  Nothing here allocates device memory.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "sx_internal.h"

namespace {
thread_local std::string g_err;

sx_status fail(sx_status code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
sx_status fail(sx_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

sx_status dev(hipError_t e, const char* where) {
  if (e == hipSuccess) return SX_OK;
  return fail(SX_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

sx_status check_cam(const sx_camera* c) {
  if (!c) return fail(SX_EINVAL, "camera is NULL");
  if (c->width < 1 || c->height < 1 || c->width > 16384 || c->height > 16384)
    return fail(SX_EINVAL, "image size %dx%d outside 1..16384", c->width, c->height);
  if (!(c->fx > 0.f) || !(c->fy > 0.f)) return fail(SX_EINVAL, "focal lengths must be > 0");
  if (!(c->znear > 0.f)) return fail(SX_EINVAL, "znear must be > 0");
  return SX_OK;
}

sx_status check_params(const sx_params* p) {
  if (!p) return fail(SX_EINVAL, "params is NULL");
  if (!sx::tile_shape_supported(p->tile_w, p->tile_h))
    return fail(SX_EINVAL, "unsupported tile shape %dx%d", p->tile_w, p->tile_h);
  if (p->sh_degree < 0 || p->sh_degree > 3)
    return fail(SX_EINVAL, "sh_degree %d outside 0..3", p->sh_degree);
  if (!(p->alpha_min > 0.f) || !(p->alpha_max > p->alpha_min) || !(p->alpha_max < 1.f))
    return fail(SX_EINVAL, "need 0 < alpha_min < alpha_max < 1");
  if (!(p->t_min >= 0.f) || !(p->eps2d >= 0.f)) return fail(SX_EINVAL, "t_min, eps2d must be >= 0");
  if (!(p->fov_guard >= 0.f && p->fov_guard <= 1e6f)) return fail(SX_EINVAL, "fov_guard must be in [0, 1e6]");
  return SX_OK;
}

sx_status check_gauss(const sx_gaussians* g) {
  if (!g) return fail(SX_EINVAL, "gaussians is NULL");
  if (g->n < 0 || g->n >= (int64_t(1) << 31)) return fail(SX_EINVAL, "n=%lld out of range", (long long)g->n);
  if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->sh))
    return fail(SX_EINVAL, "null Gaussian parameter array");
  return SX_OK;
}

int64_t tiles_of(const sx_camera* c, const sx_params* p) {
  return (int64_t)((c->width + p->tile_w - 1) / p->tile_w) * ((c->height + p->tile_h - 1) / p->tile_h);
}

#define SX_TRY(expr)                 \
  do {                               \
    sx_status _s = (expr);           \
    if (_s != SX_OK) return _s;      \
  } while (0)
}  // namespace

namespace sx {
DCam make_dcam(const sx_camera& c) {
  DCam d;
  for (int i = 0; i < 9; ++i) d.R[i] = c.R[i];
  for (int i = 0; i < 3; ++i) d.t[i] = c.t[i];
  d.fx = c.fx, d.fy = c.fy, d.cx = c.cx, d.cy = c.cy, d.znear = c.znear;
  for (int j = 0; j < 3; ++j)
    d.C[j] = -(d.R[0 * 3 + j] * d.t[0] + d.R[1 * 3 + j] * d.t[1] + d.R[2 * 3 + j] * d.t[2]);
  d.W = c.width, d.H = c.height;
  return d;
}

KParams make_kparams(const sx_params& p, const sx_camera& c) {
  KParams k;
  k.tile_w = p.tile_w, k.tile_h = p.tile_h;
  k.tiles_x = (c.width + p.tile_w - 1) / p.tile_w;
  k.tiles_y = (c.height + p.tile_h - 1) / p.tile_h;
  k.sh_degree = p.sh_degree, k.flags = p.flags;
  k.alpha_min = p.alpha_min, k.alpha_max = p.alpha_max, k.t_min = p.t_min;
  k.eps2d = p.eps2d, k.alpha_min_d = p.alpha_min, k.fov_guard = p.fov_guard;
  for (int i = 0; i < 3; ++i) k.bg[i] = p.bg[i];
  return k;
}
}  // namespace sx

extern "C" {

const char* sx_last_error_string(void) { return g_err.c_str(); }
const char* sx_version(void) { return "splaxel-mi355x 0.1 (gfx950)"; }

int64_t sx_preprocess_blocks(int64_t n) { return n <= 0 ? 1 : (n + sx::kPreBlock - 1) / sx::kPreBlock; }

sx_status sx_preprocess(const sx_gaussians* g, const sx_camera* cam,
                        const sx_params* p, sx_projected* out,
                        sx_stream stream) {
  SX_TRY(check_gauss(g));
  SX_TRY(check_cam(cam));
  SX_TRY(check_params(p));
  if (!out || (g->n > 0 && (!out->rec || !out->rect || !out->n_tiles || !out->block_sums)))
    return fail(SX_EINVAL, "null projected output array");
  const int64_t tiles_x = (cam->width + p->tile_w - 1) / p->tile_w;
  const int64_t tiles_y = (cam->height + p->tile_h - 1) / p->tile_h;
  if (tiles_x > 65535 || tiles_y > 65535) return fail(SX_EINVAL, "tile grid too large for uint16 rects");
  return dev(sx::launch_preprocess(*g, sx::make_dcam(*cam), sx::make_kparams(*p, *cam), *out,
                                   (hipStream_t)stream),
             "sx_preprocess");
}

sx_status sx_sort_workspace_size(int64_t n, int64_t capacity, int32_t tiles_x, int32_t tiles_y,
                                 size_t* bytes) {
  if (!bytes) return fail(SX_EINVAL, "bytes is NULL");
  if (n < 0 || capacity < 0 || tiles_x < 1 || tiles_y < 1) return fail(SX_EINVAL, "negative size");
  if (capacity >= (int64_t(1) << 31)) return fail(SX_EINVAL, "capacity must be < 2^31");
  *bytes = sx::sort_layout(n, capacity, tiles_x, tiles_y).total;
  return SX_OK;
}

sx_status sx_sort(const sx_projected* proj, int64_t n, const sx_camera* cam,
                  const sx_params* p, int64_t capacity, uint64_t* keys,
                  uint32_t* vals, uint32_t* tile_ranges, void* ws,
                  size_t ws_bytes, uint64_t* h_counts, sx_stream stream) {
  SX_TRY(check_cam(cam));
  SX_TRY(check_params(p));
  if (!proj || (n > 0 && (!proj->rec || !proj->rect || !proj->n_tiles || !proj->block_sums)))
    return fail(SX_EINVAL, "null projected array");
  if (n > 0 && (reinterpret_cast<uintptr_t>(proj->block_sums) & 7))
    return fail(SX_EINVAL, "block_sums is not 8-byte aligned");
  if (n < 0 || n >= (int64_t(1) << 31)) return fail(SX_EINVAL, "n out of range");
  if (capacity < 0 || capacity >= (int64_t(1) << 31)) return fail(SX_EINVAL, "capacity must be in [0, 2^31)");
  if (!vals && capacity > 0) return fail(SX_EINVAL, "vals is NULL");
  if (!tile_ranges || !ws) return fail(SX_EINVAL, "tile_ranges/ws is NULL");
  const int64_t tiles = tiles_of(cam, p);
  const sx::KParams kp = sx::make_kparams(*p, *cam);
  const size_t need = sx::sort_layout(n, capacity, kp.tiles_x, kp.tiles_y).total;
  if (ws_bytes < need) return fail(SX_EINVAL, "workspace %zu bytes < required %zu", ws_bytes, need);
  bool over = false;
  hipError_t e = sx::launch_sort(*proj, n, sx::make_kparams(*p, *cam), capacity, tiles, keys, vals,
                                 tile_ranges, static_cast<char*>(ws), h_counts, &over,
                                 (hipStream_t)stream);
  SX_TRY(dev(e, "sx_sort"));
  if (over)
    return fail(SX_ECAPACITY, "instances %llu exceed capacity %lld",
                (unsigned long long)h_counts[1], (long long)capacity);
  return SX_OK;
}

sx_status sx_sort_counts(const void* ws, int64_t n, uint64_t* h_out, sx_stream stream) {
  (void)n;
  if (!ws || !h_out) return fail(SX_EINVAL, "null argument");
  const size_t off = sx::sort_layout(0, 0, 1, 1).counts;
  hipError_t e = hipMemcpyAsync(h_out, static_cast<const char*>(ws) + off, 4 * sizeof(uint64_t),
                                hipMemcpyDeviceToHost, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  return dev(e, "sx_sort_counts");
}

// The optional cross-boundary filter fields of a projection.
static sx_status check_filter(const sx_projected* proj) {
  if (!proj->xf) return SX_OK;
  if (!proj->omega) return fail(SX_EINVAL, "cross-boundary filter without visibility maps");
  if (proj->n_cells < 1 || proj->n_cells > sx::kMaxCells || proj->cell < 0 ||
      proj->cell >= proj->n_cells)
    return fail(SX_EINVAL, "cross-boundary filter: cell %d of %d", proj->cell, proj->n_cells);
  return SX_OK;
}

sx_status sx_render_partial(const sx_projected* proj, const uint32_t* vals,
                            const uint32_t* tile_ranges, const sx_camera* cam,
                            const sx_params* p, const uint32_t* mask,
                            float* partial, float* depth, uint32_t* last,
                            uint32_t* nblend, sx_stream stream) {
  SX_TRY(check_cam(cam));
  SX_TRY(check_params(p));
  if (!proj || !proj->rec || !tile_ranges || !partial || !last)
    return fail(SX_EINVAL, "null argument");
  SX_TRY(check_filter(proj));
  return dev(sx::launch_render(*proj, vals, tile_ranges, sx::make_dcam(*cam),
                               sx::make_kparams(*p, *cam), mask, partial, depth, last, nblend,
                               (hipStream_t)stream),
             "sx_render_partial");
}

static sx_status check_cells(int32_t K, const void* partials, const sx_cell* cells) {
  if (K < 1 || K > sx::kMaxCells) return fail(SX_EINVAL, "K=%d outside 1..%d", K, sx::kMaxCells);
  if (!partials || !cells) return fail(SX_EINVAL, "null partials/cells");
  for (int m = 0; m < K; ++m)
    for (int j = 0; j < 3; ++j)
      if (std::isnan(cells[m].lo[j]) || std::isnan(cells[m].hi[j]) || cells[m].lo[j] > cells[m].hi[j])
        return fail(SX_EINVAL, "cell %d has an empty or NaN box", m);
  return SX_OK;
}

sx_status sx_kd_partition(int64_t n, const float* means, int32_t K, sx_cell* cells,
                          int32_t* cell_of) {
  if (n < 0 || n >= (int64_t(1) << 31)) return fail(SX_EINVAL, "n out of range");
  if (K < 1 || K > sx::kMaxCells) return fail(SX_EINVAL, "K=%d outside 1..%d", K, sx::kMaxCells);
  if (!cells || (n > 0 && (!means || !cell_of))) return fail(SX_EINVAL, "null argument");
  for (int64_t i = 0; i < n * 3; ++i)
    if (!std::isfinite(means[i])) return fail(SX_EINVAL, "mean %lld is not finite", (long long)(i / 3));
  float lo[sx::kMaxCells * 3], hi[sx::kMaxCells * 3];
  sx::kd_partition(n, means, K, lo, hi, cell_of);
  for (int m = 0; m < K; ++m)
    for (int j = 0; j < 3; ++j) cells[m].lo[j] = lo[m * 3 + j], cells[m].hi[j] = hi[m * 3 + j];
  return SX_OK;
}

sx_status sx_imbalance(int32_t K, const int64_t* counts, double* ratio) {
  if (K < 1 || K > sx::kMaxCells) return fail(SX_EINVAL, "K=%d outside 1..%d", K, sx::kMaxCells);
  if (!counts || !ratio) return fail(SX_EINVAL, "null argument");
  int64_t mx = 0, tot = 0;
  for (int k = 0; k < K; ++k) {
    if (counts[k] < 0) return fail(SX_EINVAL, "negative count in cell %d", k);
    mx = std::max(mx, counts[k]);
    tot += counts[k];
  }
  if (tot == 0) return fail(SX_EINVAL, "no Gaussians");
  *ratio = (double)mx * K / (double)tot - 1.0;
  return SX_OK;
}

sx_status sx_repartition_plan(int64_t n, const int32_t* cell_of, int32_t K, int32_t* dst_index,
                              int64_t* counts) {
  if (n < 0 || n >= (int64_t(1) << 31)) return fail(SX_EINVAL, "n out of range");
  if (K < 1 || K > sx::kMaxCells) return fail(SX_EINVAL, "K=%d outside 1..%d", K, sx::kMaxCells);
  if (!counts || (n > 0 && (!cell_of || !dst_index))) return fail(SX_EINVAL, "null argument");
  for (int64_t g = 0; g < n; ++g)
    if (cell_of[g] < 0 || cell_of[g] >= K)
      return fail(SX_EINVAL, "cell_of[%lld] = %d outside 0..%d", (long long)g, cell_of[g], K - 1);
  sx::repartition_plan(n, cell_of, K, dst_index, counts);
  return SX_OK;
}

sx_status sx_move_rows(int32_t row_floats, int32_t K_src, const int64_t* src_counts,
                       const float* const* src, int32_t K_dst, float* const* dst,
                       const int32_t* dst_cell, const int32_t* dst_index, sx_stream stream) {
  if (row_floats < 1 || row_floats > 4096) return fail(SX_EINVAL, "row_floats=%d", row_floats);
  if (K_src < 1 || K_src > sx::kMaxCells || K_dst < 1 || K_dst > sx::kMaxCells)
    return fail(SX_EINVAL, "cell counts %d, %d outside 1..%d", K_src, K_dst, sx::kMaxCells);
  if (!src_counts || !src || !dst) return fail(SX_EINVAL, "null argument");
  int64_t off[sx::kMaxCells + 1];
  off[0] = 0;
  for (int c = 0; c < K_src; ++c) {
    if (src_counts[c] < 0) return fail(SX_EINVAL, "negative count in source cell %d", c);
    if (src_counts[c] > 0 && !src[c]) return fail(SX_EINVAL, "source cell %d is NULL", c);
    off[c + 1] = off[c] + src_counts[c];
  }
  if (off[K_src] >= (int64_t(1) << 31)) return fail(SX_EINVAL, "too many rows");
  if (off[K_src] > 0 && (!dst_cell || !dst_index)) return fail(SX_EINVAL, "null mapping");
  for (int c = 0; c < K_dst; ++c)
    if (!dst[c]) return fail(SX_EINVAL, "destination cell %d is NULL", c);
  return dev(sx::launch_move_rows(off[K_src], row_floats, K_src, off, src, K_dst, dst, dst_cell,
                                  dst_index, (hipStream_t)stream),
             "sx_move_rows");
}

sx_status sx_mask_counts(int32_t K, const uint32_t* masks, int64_t words, uint32_t* counts,
                         sx_stream stream) {
  if (K < 1 || K > sx::kMaxCells) return fail(SX_EINVAL, "K=%d outside 1..%d", K, sx::kMaxCells);
  if (words < 0) return fail(SX_EINVAL, "words < 0");
  if (!counts || (words > 0 && !masks)) return fail(SX_EINVAL, "null argument");
  return dev(sx::launch_mask_counts(K, masks, words, counts, (hipStream_t)stream), "sx_mask_counts");
}

sx_status sx_visibility(int32_t K, const sx_cell* cells, const sx_camera* cam, uint32_t* masks,
                        sx_stream stream) {
  SX_TRY(check_cam(cam));
  if (K < 1 || K > sx::kMaxCells) return fail(SX_EINVAL, "K=%d outside 1..%d", K, sx::kMaxCells);
  if (!cells || !masks) return fail(SX_EINVAL, "null argument");
  for (int m = 0; m < K; ++m)
    for (int j = 0; j < 3; ++j)
      if (!(cells[m].lo[j] <= cells[m].hi[j])) return fail(SX_EINVAL, "cell %d: lo > hi or NaN", m);
  return dev(sx::launch_visibility(K, cells, sx::make_dcam(*cam), masks, (hipStream_t)stream),
             "sx_visibility");
}

sx_status sx_cross_filter(const sx_gaussians* g, const sx_projected* proj, int32_t K,
                          const sx_cell* cells, int32_t cell, const sx_camera* cam,
                          uint32_t* xf, sx_stream stream) {
  SX_TRY(check_cam(cam));
  if (!g || !proj || !cells || !xf) return fail(SX_EINVAL, "null argument");
  if (g->n < 0 || g->n >= (int64_t(1) << 31)) return fail(SX_EINVAL, "n out of range");
  if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !proj->rec || !proj->n_tiles))
    return fail(SX_EINVAL, "null argument");
  if (K < 1 || K > sx::kMaxCells) return fail(SX_EINVAL, "K=%d outside 1..%d", K, sx::kMaxCells);
  if (cell < 0 || cell >= K) return fail(SX_EINVAL, "cell %d outside 0..%d", cell, K - 1);
  for (int m = 0; m < K; ++m)
    for (int j = 0; j < 3; ++j)
      if (!(cells[m].lo[j] <= cells[m].hi[j])) return fail(SX_EINVAL, "cell %d: lo > hi or NaN", m);
  return dev(sx::launch_cross_filter(*g, *proj, K, cells, cell, sx::make_dcam(*cam), xf,
                                     (hipStream_t)stream),
             "sx_cross_filter");
}

sx_status sx_composite(int32_t K, const float* const* partials,
                       const sx_cell* cells, const sx_camera* cam,
                       const sx_params* p, float* out, uint32_t* masks,
                       sx_stream stream) {
  SX_TRY(check_cam(cam));
  SX_TRY(check_params(p));
  SX_TRY(check_cells(K, partials, cells));
  if (!out) return fail(SX_EINVAL, "out is NULL");
  for (int m = 0; m < K; ++m)
    if (!partials[m]) return fail(SX_EINVAL, "partial %d is NULL", m);
  return dev(sx::launch_composite(K, partials, cells, sx::make_dcam(*cam), sx::make_kparams(*p, *cam),
                                  out, masks, nullptr, nullptr, (hipStream_t)stream),
             "sx_composite");
}

sx_status sx_composite_reeval(int32_t K, const float* const* partials,
                              const sx_cell* cells, const sx_camera* cam,
                              const sx_params* p, float* out, uint32_t* masks,
                              const uint32_t* omega, float* budget, sx_stream stream) {
  SX_TRY(check_cam(cam));
  SX_TRY(check_params(p));
  SX_TRY(check_cells(K, partials, cells));
  if (!out || !masks || !budget) return fail(SX_EINVAL, "out, masks and budget are required");
  for (int m = 0; m < K; ++m)
    if (!partials[m]) return fail(SX_EINVAL, "partial %d is NULL", m);
  return dev(sx::launch_composite(K, partials, cells, sx::make_dcam(*cam), sx::make_kparams(*p, *cam),
                                  out, masks, omega, budget, (hipStream_t)stream),
             "sx_composite_reeval");
}

sx_status sx_composite_l1(int32_t K, const float* const* partials, const sx_cell* cells,
                          const sx_camera* cam, const sx_params* p, const float* target,
                          float* out, uint32_t* masks, float* loss_sum,
                          float* const* dpartials, sx_stream stream) {
  SX_TRY(check_cam(cam));
  SX_TRY(check_params(p));
  SX_TRY(check_cells(K, partials, cells));
  if (!target || !out || !dpartials) return fail(SX_EINVAL, "null argument");
  for (int m = 0; m < K; ++m)
    if (!partials[m] || !dpartials[m]) return fail(SX_EINVAL, "null buffer for cell %d", m);
  return dev(sx::launch_composite_l1(K, partials, cells, sx::make_dcam(*cam),
                                     sx::make_kparams(*p, *cam), target, out, masks, loss_sum,
                                     dpartials, (hipStream_t)stream),
             "sx_composite_l1");
}

sx_status sx_l1_loss(const float* out, const float* target, int32_t width,
                     int32_t height, float* dout, float* loss_sum, sx_stream stream) {
  if (!out || !target || !dout) return fail(SX_EINVAL, "null argument");
  if (width < 1 || height < 1) return fail(SX_EINVAL, "bad image size");
  return dev(sx::launch_l1(out, target, width, height, dout, loss_sum, (hipStream_t)stream),
             "sx_l1_loss");
}

sx_status sx_composite_backward(int32_t K, const float* const* partials,
                                const sx_cell* cells, const sx_camera* cam,
                                const sx_params* p, const uint32_t* masks,
                                const float* dout, float* const* dpartials,
                                sx_stream stream) {
  (void)masks;
  SX_TRY(check_cam(cam));
  SX_TRY(check_params(p));
  SX_TRY(check_cells(K, partials, cells));
  if (!dout || !dpartials) return fail(SX_EINVAL, "null argument");
  for (int m = 0; m < K; ++m)
    if (!partials[m] || !dpartials[m]) return fail(SX_EINVAL, "null buffer for cell %d", m);
  return dev(sx::launch_composite_backward(K, partials, cells, sx::make_dcam(*cam),
                                           sx::make_kparams(*p, *cam), dout, dpartials,
                                           (hipStream_t)stream),
             "sx_composite_backward");
}

sx_status sx_backward_workspace_size(int64_t capacity, int64_t tiles_total, size_t* bytes) {
  if (!bytes) return fail(SX_EINVAL, "bytes is NULL");
  if (capacity < 0 || capacity >= (int64_t(1) << 31) || tiles_total < 1)
    return fail(SX_EINVAL, "bad size");
  *bytes = sx::bwd_layout(capacity, tiles_total).total;
  return SX_OK;
}

sx_status sx_render_backward_stages(const sx_projected* proj, const uint32_t* vals,
                                    const uint32_t* tile_ranges, const void* sort_ws,
                                    int64_t n, int64_t capacity, void* bwd_ws,
                                    const sx_camera* cam, const sx_params* p,
                                    const uint32_t* mask, const float* partial,
                                    const uint32_t* last, const float* dpartial,
                                    const float* ddepth, float* g2d, int32_t stages,
                                    sx_stream stream) {
  SX_TRY(check_cam(cam));
  SX_TRY(check_params(p));
  if (!proj || !proj->rec || !proj->n_tiles || !proj->rect || !tile_ranges || !sort_ws || !bwd_ws ||
      !partial || !last || !dpartial || !g2d)
    return fail(SX_EINVAL, "null argument");
  if (n < 0 || capacity < 0 || capacity >= (int64_t(1) << 31)) return fail(SX_EINVAL, "bad n/capacity");
  if (stages & ~SX_RB_ALL) return fail(SX_EINVAL, "unknown stage bits 0x%x", stages);
  SX_TRY(check_filter(proj));
  const sx::KParams kp = sx::make_kparams(*p, *cam);
  return dev(sx::launch_render_backward(*proj, vals, tile_ranges, sx::sort_view(sort_ws, n, capacity, kp.tiles_x, kp.tiles_y),
                                        n, capacity, sx::make_dcam(*cam), kp, mask,
                                        partial, last, dpartial, ddepth, g2d, static_cast<char*>(bwd_ws),
                                        stages, (hipStream_t)stream),
             "sx_render_backward");
}

// Scratch of sx_render_backward_noalloc: the per-tile visited counts and
// the per-instance gradient rows of the render backward, in one static
// device array instead of a caller workspace.  Each device holds its own
// copy (allocated when the code object is loaded, held until the process
// ends); host code only ever uses the per-device address that
// hipGetSymbolAddress returns for it, never the array's name.
static __device__ __align__(256) unsigned char scratch[SX_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch`, looked up once per device.
sx_status scratch_address(void** out) {
  int dev_id = 0;
  hipError_t e = hipGetDevice(&dev_id);
  if (e != hipSuccess) return dev(e, "hipGetDevice");
  if (dev_id < 0 || dev_id >= kMaxDevices) return fail(SX_EUNSUPPORTED, "device %d", dev_id);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev_id]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return dev(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(SX_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev_id] = p;
  }
  *out = g_scratch_ptr[dev_id];
  return SX_OK;
}
}  // namespace

sx_status sx_render_backward(const sx_projected* proj, const uint32_t* vals,
                             const uint32_t* tile_ranges, const void* sort_ws,
                             int64_t n, int64_t capacity, void* bwd_ws,
                             const sx_camera* cam, const sx_params* p,
                             const uint32_t* mask, const float* partial,
                             const uint32_t* last, const float* dpartial,
                             const float* ddepth, float* g2d, sx_stream stream) {
  return sx_render_backward_stages(proj, vals, tile_ranges, sort_ws, n, capacity, bwd_ws, cam, p,
                                   mask, partial, last, dpartial, ddepth, g2d, SX_RB_ALL, stream);
}

sx_status sx_render_backward_noalloc(const sx_projected* proj, const uint32_t* vals,
                                     const uint32_t* tile_ranges, const void* sort_ws,
                                     int64_t n, int64_t capacity, const sx_camera* cam,
                                     const sx_params* p, const uint32_t* mask,
                                     const float* partial, const uint32_t* last,
                                     const float* dpartial, const float* ddepth, float* g2d,
                                     sx_stream stream) {
  SX_TRY(check_cam(cam));
  SX_TRY(check_params(p));
  if (capacity < 0 || capacity >= (int64_t(1) << 31)) return fail(SX_EINVAL, "bad capacity");
  const sx::KParams kp = sx::make_kparams(*p, *cam);
  const size_t need = sx::bwd_layout(capacity, (int64_t)kp.tiles_x * kp.tiles_y).total;
  if (need > (size_t)SX_NOALLOC_SCRATCH_BYTES)
    return fail(SX_EINVAL,
                "sx_render_backward_noalloc: capacity %lld on a %dx%d tile grid needs %zu scratch "
                "bytes, more than the static %llu",
                (long long)capacity, kp.tiles_x, kp.tiles_y, need,
                (unsigned long long)SX_NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  SX_TRY(scratch_address(&ws));
  return sx_render_backward_stages(proj, vals, tile_ranges, sort_ws, n, capacity, ws, cam, p, mask,
                                   partial, last, dpartial, ddepth, g2d, SX_RB_ALL, stream);
}

sx_status sx_preprocess_backward(const sx_gaussians* g, const sx_camera* cam,
                                 const sx_params* p, const sx_projected* proj,
                                 const void* sort_ws, int64_t capacity,
                                 const float* g2d, const sx_grads* grads,
                                 int32_t flags, sx_stream stream) {
  SX_TRY(check_gauss(g));
  SX_TRY(check_cam(cam));
  SX_TRY(check_params(p));
  if (!proj || !proj->n_tiles || !sort_ws || !g2d || !grads) return fail(SX_EINVAL, "null argument");
  if (capacity < 0 || capacity >= (int64_t(1) << 31)) return fail(SX_EINVAL, "bad capacity");
  if (g->n > 0 && (!grads->means || !grads->log_scales || !grads->quats || !grads->opacity_logits || !grads->sh))
    return fail(SX_EINVAL, "null gradient array");
  const sx::KParams kp = sx::make_kparams(*p, *cam);
  return dev(sx::launch_preprocess_backward(*g, sx::make_dcam(*cam), kp, *proj,
                                            sx::sort_view(sort_ws, g->n, capacity, kp.tiles_x, kp.tiles_y), g2d, *grads,
                                            (flags & SX_BWD_ACCUMULATE) != 0, (hipStream_t)stream),
             "sx_preprocess_backward");
}


sx_status sx_backward(int32_t K, const sx_cell_state* cells, const sx_cell* boxes,
                      const sx_camera* cam, const sx_params* p, const float* dout,
                      int32_t flags, sx_stream stream) {
  SX_TRY(check_cam(cam));
  SX_TRY(check_params(p));
  if (K < 1 || K > sx::kMaxCells) return fail(SX_EINVAL, "K=%d outside 1..%d", K, sx::kMaxCells);
  if (!cells || !boxes || !dout) return fail(SX_EINVAL, "null argument");
  const float* parts[sx::kMaxCells];
  float* dparts[sx::kMaxCells];
  for (int m = 0; m < K; ++m) {
    const sx_cell_state& c = cells[m];
    if (!c.g || !c.proj || !c.ranges || !c.sort_ws || !c.partial || !c.last || !c.grads || !c.g2d_ws ||
        !c.dpartial_ws || !c.bwd_ws)
      return fail(SX_EINVAL, "cell %d has a null member", m);
    SX_TRY(check_gauss(c.g));
    parts[m] = c.partial;
    dparts[m] = c.dpartial_ws;
  }
  SX_TRY(sx_composite_backward(K, parts, boxes, cam, p, nullptr, dout, dparts, stream));
  for (int m = 0; m < K; ++m) {
    const sx_cell_state& c = cells[m];
    SX_TRY(sx_render_backward(c.proj, c.vals, c.ranges, c.sort_ws, c.g->n, c.capacity, c.bwd_ws, cam, p,
                              c.mask, c.partial, c.last, c.dpartial_ws, nullptr, c.g2d_ws, stream));
    SX_TRY(sx_preprocess_backward(c.g, cam, p, c.proj, c.sort_ws, c.capacity, c.g2d_ws, c.grads, flags,
                                  stream));
  }
  return SX_OK;
}

static_assert(SX_MAX_VIEWS == sx::kMaxViews, "view limit");

// ------------------------------------------------------------ batched views
static sx_status check_views(int32_t V, const sx_view* views, const sx_params* p, bool backward) {
  if (V < 1 || V > sx::kMaxViews) return fail(SX_EINVAL, "V=%d outside 1..%d", V, sx::kMaxViews);
  if (!views) return fail(SX_EINVAL, "views is NULL");
  SX_TRY(check_params(p));
  for (int v = 0; v < V; ++v) {
    const sx_view& w = views[v];
    SX_TRY(check_cam(&w.cam));
    if (tiles_of(&w.cam, p) >= (int64_t(1) << 24)) return fail(SX_EINVAL, "view %d has too many tiles", v);
    if (!w.proj.rec || !w.tile_ranges || !w.partial || !w.last)
      return fail(SX_EINVAL, "view %d: null forward buffer", v);
    if (w.capacity < 0 || w.capacity >= (int64_t(1) << 31)) return fail(SX_EINVAL, "view %d: bad capacity", v);
    if (backward && (!w.proj.rect || !w.proj.n_tiles || !w.sort_ws || !w.dpartial || !w.g2d || !w.bwd_ws))
      return fail(SX_EINVAL, "view %d: null backward buffer", v);
    if (w.proj.xf) return fail(SX_EINVAL, "view %d: the batched renders apply no cross-boundary filter", v);
  }
  return SX_OK;
}

static void to_multi(int32_t V, const sx_view* views, const sx_params* p, sx::MultiView* mv) {
  for (int v = 0; v < V; ++v) {
    const sx_view& w = views[v];
    sx::MultiView& m = mv[v];
    m.cam = sx::make_dcam(w.cam);
    const sx::KParams k = sx::make_kparams(*p, w.cam);
    m.tiles_x = k.tiles_x, m.tiles_y = k.tiles_y;
    m.proj = w.proj;
    m.vals = w.vals, m.ranges = w.tile_ranges, m.mask = w.mask;
    m.partial = w.partial, m.depth = w.depth, m.last = w.last, m.nblend = w.nblend;
    m.sort_ws = w.sort_ws, m.capacity = w.capacity;
    m.dpartial = w.dpartial, m.g2d = w.g2d, m.bwd_ws = w.bwd_ws;
    m.n = w.n;
  }
}

static size_t multi_ws_need(int32_t V, const sx_camera* cams, int stride, const sx_params* p) {
  int64_t items = 0;
  for (int v = 0; v < V; ++v)
    items += tiles_of(reinterpret_cast<const sx_camera*>(reinterpret_cast<const char*>(cams) + (size_t)v * stride), p);
  return sx::multi_workspace_bytes(items);
}

sx_status sx_preprocess_multi(const sx_gaussians* g, int32_t V, const sx_camera* cams,
                              const sx_params* p, sx_projected* outs, sx_stream stream) {
  SX_TRY(check_gauss(g));
  SX_TRY(check_params(p));
  if (V < 1 || V > sx::kMaxViews) return fail(SX_EINVAL, "V=%d outside 1..%d", V, sx::kMaxViews);
  if (!cams || !outs) return fail(SX_EINVAL, "null cams/outs");
  for (int v = 0; v < V; ++v) {
    SX_TRY(check_cam(&cams[v]));
    const int64_t tx = (cams[v].width + p->tile_w - 1) / p->tile_w;
    const int64_t ty = (cams[v].height + p->tile_h - 1) / p->tile_h;
    if (tx > 65535 || ty > 65535) return fail(SX_EINVAL, "tile grid too large for uint16 rects");
    if (g->n > 0 && (!outs[v].rec || !outs[v].rect || !outs[v].n_tiles || !outs[v].block_sums))
      return fail(SX_EINVAL, "view %d: null projected output array", v);
  }
  return dev(sx::launch_preprocess_multi(*g, V, cams, sx::make_kparams(*p, cams[0]), outs,
                                         (hipStream_t)stream),
             "sx_preprocess_multi");
}

sx_status sx_multi_workspace_size(int32_t V, const sx_camera* cams, const sx_params* p,
                                  size_t* bytes) {
  if (!bytes || !cams) return fail(SX_EINVAL, "null argument");
  SX_TRY(check_params(p));
  if (V < 1 || V > sx::kMaxViews) return fail(SX_EINVAL, "V=%d outside 1..%d", V, sx::kMaxViews);
  for (int v = 0; v < V; ++v) SX_TRY(check_cam(&cams[v]));
  *bytes = multi_ws_need(V, cams, sizeof(sx_camera), p);
  return SX_OK;
}

sx_status sx_render_multi(int32_t V, const sx_view* views, const sx_params* p, void* ws,
                          size_t ws_bytes, sx_stream stream) {
  SX_TRY(check_views(V, views, p, false));
  if (!ws) return fail(SX_EINVAL, "ws is NULL");
  const size_t need = multi_ws_need(V, &views[0].cam, sizeof(sx_view), p);
  if (ws_bytes < need) return fail(SX_EINVAL, "workspace %zu bytes < required %zu", ws_bytes, need);
  sx::MultiView mv[sx::kMaxViews];
  to_multi(V, views, p, mv);
  return dev(sx::launch_render_multi(V, mv, sx::make_kparams(*p, views[0].cam), static_cast<char*>(ws),
                                     (hipStream_t)stream),
             "sx_render_multi");
}

sx_status sx_render_backward_multi(int32_t V, const sx_view* views, int64_t n, const sx_params* p,
                                   void* ws, size_t ws_bytes, sx_stream stream) {
  SX_TRY(check_views(V, views, p, true));
  if (!ws) return fail(SX_EINVAL, "ws is NULL");
  if (n < 0 || n >= (int64_t(1) << 31)) return fail(SX_EINVAL, "n out of range");
  const size_t need = multi_ws_need(V, &views[0].cam, sizeof(sx_view), p);
  if (ws_bytes < need) return fail(SX_EINVAL, "workspace %zu bytes < required %zu", ws_bytes, need);
  sx::MultiView mv[sx::kMaxViews];
  to_multi(V, views, p, mv);
  for (int v = 0; v < V; ++v) {
    if (mv[v].n < 0 || mv[v].n >= (int64_t(1) << 31)) return fail(SX_EINVAL, "view %d: n out of range", v);
    if (mv[v].n == 0) mv[v].n = n;
  }
  const sx::KParams kp = sx::make_kparams(*p, views[0].cam);
  SX_TRY(dev(sx::launch_render_backward_multi(V, mv, kp, static_cast<char*>(ws), (hipStream_t)stream),
             "sx_render_backward_multi"));
  for (int v = 0; v < V; ++v)
    SX_TRY(dev(sx::launch_grad_reduce_view(mv[v], kp, (hipStream_t)stream), "sx_render_backward_multi"));
  return SX_OK;
}

sx_status sx_preprocess_backward_multi(const sx_gaussians* g, int32_t V, const sx_view* views,
                                       const sx_params* p, const sx_grads* grads, int32_t flags,
                                       sx_stream stream) {
  SX_TRY(check_gauss(g));
  SX_TRY(check_params(p));
  if (V < 1 || V > sx::kMaxViews) return fail(SX_EINVAL, "V=%d outside 1..%d", V, sx::kMaxViews);
  if (!views || !grads) return fail(SX_EINVAL, "null argument");
  if (g->n > 0 && (!grads->means || !grads->log_scales || !grads->quats || !grads->opacity_logits || !grads->sh))
    return fail(SX_EINVAL, "null gradient array");
  sx::DCam cams[sx::kMaxViews];
  sx_projected projs[sx::kMaxViews];
  sx::SortView svs[sx::kMaxViews];
  const float* g2d[sx::kMaxViews];
  for (int v = 0; v < V; ++v) {
    const sx_view& w = views[v];
    SX_TRY(check_cam(&w.cam));
    if (g->n > 0 && (!w.proj.n_tiles || !w.g2d || !w.sort_ws))
      return fail(SX_EINVAL, "view %d: null n_tiles/g2d/sort_ws", v);
    if (w.capacity < 0 || w.capacity >= (int64_t(1) << 31)) return fail(SX_EINVAL, "view %d: bad capacity", v);
    const sx::KParams kv = sx::make_kparams(*p, w.cam);
    cams[v] = sx::make_dcam(w.cam);
    projs[v] = w.proj;
    svs[v] = sx::sort_view(w.sort_ws, g->n, w.capacity, kv.tiles_x, kv.tiles_y);
    g2d[v] = w.g2d;
  }
  return dev(sx::launch_preprocess_backward_multi(*g, V, cams, projs, svs, g2d,
                                                  sx::make_kparams(*p, views[0].cam), *grads,
                                                  (flags & SX_BWD_ACCUMULATE) != 0,
                                                  (hipStream_t)stream),
             "sx_preprocess_backward_multi");
}

sx_status sx_adam(int64_t n, float* param, const float* grad, float* m, float* v,
                  int32_t step, float lr, float beta1, float beta2, float eps,
                  sx_stream stream) {
  if (n < 0) return fail(SX_EINVAL, "n < 0");
  if (n > 0 && (!param || !grad || !m || !v)) return fail(SX_EINVAL, "null argument");
  if (step < 1) return fail(SX_EINVAL, "step must be >= 1");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f)) return fail(SX_EINVAL, "betas in [0,1)");
  const float bc1 = (float)(1.0 - std::pow((double)beta1, (double)step));
  const float bc2 = (float)(1.0 - std::pow((double)beta2, (double)step));
  return dev(sx::launch_adam(n, param, grad, m, v, lr, beta1, beta2, eps, bc1, bc2, (hipStream_t)stream),
             "sx_adam");
}

sx_status sx_fill_u32(uint32_t* ptr, int64_t n, uint32_t value, sx_stream stream) {
  if (n < 0 || (n > 0 && !ptr)) return fail(SX_EINVAL, "bad fill arguments");
  return dev(sx::launch_fill(ptr, n, value, (hipStream_t)stream), "sx_fill_u32");
}

}  // extern "C"
