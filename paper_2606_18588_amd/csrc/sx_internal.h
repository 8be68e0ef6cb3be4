// Internal declarations shared by the HIP translation units of libsplaxel.
// Device helpers live here; the public C ABI is include/splaxel.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "splaxel.h"

namespace sx {

constexpr int kRecFloats = 12;   // per-Gaussian render record (48 B)
constexpr int kG2dFloats = 12;   // per-Gaussian screen-space gradient row
constexpr int kPreBlock = 256;   // Gaussians per preprocess block
constexpr int kMaxCells = 16;
constexpr int kMaxViews = 16;  // views per batched launch
constexpr float kLog2e = 1.4426950408889634f;

// Camera in double (exact widening of the caller's float values) plus the
// camera centre -R^T t, used by the FP64 projection kernels.
struct DCam {
  double R[9];
  double t[3];
  double fx, fy, cx, cy, znear;
  double C[3];
  int32_t W, H;
};

struct KParams {
  int32_t tile_w, tile_h, tiles_x, tiles_y, sh_degree, flags;
  float alpha_min, alpha_max, t_min;
  double eps2d, alpha_min_d, fov_guard;
  float bg[3];
};

DCam make_dcam(const sx_camera& c);
KParams make_kparams(const sx_params& p, const sx_camera& c);

// ---------------------------------------------------------------------------
// sort workspace layout (byte offsets), shared by the size query and sx_sort
struct SortLayout {
  size_t counts;       // uint64[4]: visible, instances, overflow, error
  size_t vis_off;      // uint32[nb]   exclusive visible offsets per block
  size_t inst_off;     // uint32[nb]   exclusive instance offsets per block
  size_t ioff;         // uint32[n]    first instance of each visible Gaussian
  size_t scan_part;    // uint64[tiles][2] per-tile (visible, instance) sums
  size_t vidx;         // uint32[n]    visible Gaussians in index order
  size_t vrect;        // ushort4[n]   their tile rectangles (same order)
  size_t vkey;         // uint32[n]    their depth bits (same order)
  size_t tcount;       // uint32[tiles] instances per tile (cleared by the
                       // first kernel of every call)
  size_t cursor;       // uint32[tiles] next free slot of each tile's list
  size_t order;        // uint32[tiles] tiles by descending list length
  size_t pairs[2];     // uint64[cap] per-tile lists of depth bits << 32 | index
                       // (the binning's output; [1] is the merge buffer of
                       // tiles longer than one LDS chunk)
  size_t total;
  int64_t nb;
};
SortLayout sort_layout(int64_t n, int64_t capacity, int64_t tiles_x, int64_t tiles_y);

// backward workspace.  Each tile's walk visits a prefix of its list (the
// entries up to the last one any of its pixels reached); the visited entries
// of all tiles get consecutive gradient rows, tile by tile, and (Gaussian,
// row) pairs that are sorted by Gaussian to sum each Gaussian's rows.
constexpr int kRowFloats = 10;  // d(mean2d x, y, conic a, b, c, opacity, r, g, b, depth)
struct BwdLayout {
  size_t nv;        // uint32[tiles] entries visited per tile
  size_t rows;      // float[cap][kRowFloats]: one gradient row per (Gaussian, tile)
                    // instance, Gaussian-major (see SortView::ioff)
  size_t total;
};
BwdLayout bwd_layout(int64_t capacity, int64_t tiles_total);

// what the backward needs from a cell's sort workspace
struct SortView {
  const uint64_t* counts;
  const uint32_t* vidx;   // the visible Gaussians in index order
  const uint32_t* ioff;   // [n] first instance of each visible Gaussian, index order
  const uint32_t* order;  // [tiles] tiles by descending list length (the walk's order)
};
SortView sort_view(const void* ws, int64_t n, int64_t capacity, int64_t tiles_x, int64_t tiles_y);

// ---------------------------------------------------------------------------
// device helpers

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Sum of unsigned integers over a 64-lane wavefront with DPP: quad
// permutations and row rotations give every lane its 16-lane row's sum,
// then row broadcasts carry rows 0-2 into row 3; the total ends up in lane
// 63 (exact).
__device__ __forceinline__ uint32_t wave_sum_u32_to_lane63(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);
  v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);
  v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x124, 0xF, 0xF, false);
  v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);
  return v;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  for (int o = 32; o >= 1; o >>= 1) {
    uint32_t w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

// Real orthonormal SH (Condon-Shortley phase) as homogeneous polynomials of
// the unit direction (x, y, z); the constants are the normalisations
// sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) times sqrt2 for m != 0, folded with the
// polynomial coefficients of P_l^m.
struct SHC {
  static constexpr double c0 = 0.28209479177387814;   // 1/(2 sqrt(pi))
  static constexpr double c1 = 0.48860251190291992;   // sqrt(3/(4 pi))
  static constexpr double c2a = 1.0925484305920792;   // sqrt(15/(4 pi))
  static constexpr double c2b = 0.31539156525252005;  // sqrt(5/(16 pi))
  static constexpr double c2c = 0.54627421529603959;  // sqrt(15/(16 pi))
  static constexpr double c3a = 0.59004358992664352;  // sqrt(35/(32 pi))
  static constexpr double c3b = 2.8906114426405538;   // sqrt(105/(4 pi))
  static constexpr double c3c = 0.45704579946446572;  // sqrt(21/(32 pi))
  static constexpr double c3d = 0.37317633259011546;  // sqrt(7/(16 pi))
  static constexpr double c3e = 1.4453057213202769;   // sqrt(105/(16 pi))
};

__device__ __forceinline__ void sh_basis(int deg, double x, double y, double z,
                                         double* Y) {
  Y[0] = SHC::c0;
  if (deg < 1) return;
  Y[1] = -SHC::c1 * y;
  Y[2] = SHC::c1 * z;
  Y[3] = -SHC::c1 * x;
  if (deg < 2) return;
  const double xx = x * x, yy = y * y, zz = z * z;
  Y[4] = SHC::c2a * x * y;
  Y[5] = -SHC::c2a * y * z;
  Y[6] = SHC::c2b * (2.0 * zz - xx - yy);
  Y[7] = -SHC::c2a * x * z;
  Y[8] = SHC::c2c * (xx - yy);
  if (deg < 3) return;
  Y[9] = -SHC::c3a * y * (3.0 * xx - yy);
  Y[10] = SHC::c3b * x * y * z;
  Y[11] = -SHC::c3c * y * (4.0 * zz - xx - yy);
  Y[12] = SHC::c3d * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
  Y[13] = -SHC::c3c * x * (4.0 * zz - xx - yy);
  Y[14] = SHC::c3e * z * (xx - yy);
  Y[15] = -SHC::c3a * x * (xx - 3.0 * yy);
}

// gradient of each polynomial above with respect to (x, y, z): dY[k*3+c]
template <typename T>
__device__ __forceinline__ void sh_basis_grad(int deg, T x, T y, T z, T* dY) {
  for (int k = 0; k < 3; ++k) dY[k] = T(0.0);
  if (deg < 1) return;
  dY[3 + 0] = T(0.0), dY[3 + 1] = (T)-SHC::c1, dY[3 + 2] = T(0.0);
  dY[6 + 0] = T(0.0), dY[6 + 1] = T(0.0), dY[6 + 2] = (T)SHC::c1;
  dY[9 + 0] = (T)-SHC::c1, dY[9 + 1] = T(0.0), dY[9 + 2] = T(0.0);
  if (deg < 2) return;
  const T a = (T)SHC::c2a, b = (T)SHC::c2b, c = (T)SHC::c2c;
  dY[12 + 0] = a * y, dY[12 + 1] = a * x, dY[12 + 2] = T(0.0);
  dY[15 + 0] = T(0.0), dY[15 + 1] = -a * z, dY[15 + 2] = -a * y;
  dY[18 + 0] = -T(2.0) * b * x, dY[18 + 1] = -T(2.0) * b * y, dY[18 + 2] = T(4.0) * b * z;
  dY[21 + 0] = -a * z, dY[21 + 1] = T(0.0), dY[21 + 2] = -a * x;
  dY[24 + 0] = T(2.0) * c * x, dY[24 + 1] = -T(2.0) * c * y, dY[24 + 2] = T(0.0);
  if (deg < 3) return;
  const T e = (T)-SHC::c3a, f = (T)SHC::c3b, g = (T)-SHC::c3c, h = (T)SHC::c3d,
          k = (T)SHC::c3e;
  const T xx = x * x, yy = y * y, zz = z * z;
  // e (3 x^2 y - y^3)
  dY[27 + 0] = T(6.0) * e * x * y, dY[27 + 1] = e * (T(3.0) * xx - T(3.0) * yy), dY[27 + 2] = T(0.0);
  // f x y z
  dY[30 + 0] = f * y * z, dY[30 + 1] = f * x * z, dY[30 + 2] = f * x * y;
  // g (4 y z^2 - x^2 y - y^3)
  dY[33 + 0] = -T(2.0) * g * x * y, dY[33 + 1] = g * (T(4.0) * zz - xx - T(3.0) * yy),
          dY[33 + 2] = T(8.0) * g * y * z;
  // h (2 z^3 - 3 x^2 z - 3 y^2 z)
  dY[36 + 0] = -T(6.0) * h * x * z, dY[36 + 1] = -T(6.0) * h * y * z,
          dY[36 + 2] = h * (T(6.0) * zz - T(3.0) * xx - T(3.0) * yy);
  // g (4 x z^2 - x^3 - x y^2)
  dY[39 + 0] = g * (T(4.0) * zz - T(3.0) * xx - yy), dY[39 + 1] = -T(2.0) * g * x * y,
          dY[39 + 2] = T(8.0) * g * x * z;
  // k (x^2 z - y^2 z)
  dY[42 + 0] = T(2.0) * k * x * z, dY[42 + 1] = -T(2.0) * k * y * z, dY[42 + 2] = k * (xx - yy);
  // e (x^3 - 3 x y^2)
  dY[45 + 0] = e * (T(3.0) * xx - T(3.0) * yy), dY[45 + 1] = -T(6.0) * e * x * y, dY[45 + 2] = T(0.0);
}

// Rotation matrix of a unit quaternion (w, x, y, z), row-major.
__device__ __forceinline__ void quat_rot(double w, double x, double y,
                                         double z, double* R) {
  R[0] = 1.0 - 2.0 * (y * y + z * z);
  R[1] = 2.0 * (x * y - w * z);
  R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);
  R[4] = 1.0 - 2.0 * (x * x + z * z);
  R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);
  R[7] = 2.0 * (y * z + w * x);
  R[8] = 1.0 - 2.0 * (x * x + y * y);
}


// Per-pixel alpha of one Gaussian (Eq. 1 with the clamp): the forward and
// the backward kernels call this same function so their decisions agree
// bit for bit.
struct AlphaEval {
  float G;      // exp(-q/2)
  float alpha;  // min(alpha_max, o G)
  bool clamped;
};
// (a, b2, c): the conic times kConicToExp2, so that the form below is
// -q/2 in base 2, with b doubled (b2 = b + b, exact) when the record is
// staged rather than at every evaluation
constexpr float kConicToExp2 = -0.5f * kLog2e;
__device__ __forceinline__ AlphaEval eval_alpha(float dx, float dy, float a,
                                                float b2, float c, float o,
                                                float alpha_max) {
  const float t = fmaf(b2, dy, a * dx);        // a dx + 2 b dy
  const float e = fmaf(t, dx, (c * dy) * dy);  // a dx^2 + 2 b dx dy + c dy^2
  AlphaEval r;
  r.G = __builtin_amdgcn_exp2f(e);
  const float araw = o * r.G;
  r.clamped = araw > alpha_max;
  r.alpha = fminf(araw, alpha_max);
  return r;
}

}  // namespace sx

// host-side launchers (defined in the .hip files)
namespace sx {
hipError_t launch_preprocess(const sx_gaussians& g, const DCam& cam,
                             const KParams& p, const sx_projected& out,
                             hipStream_t st);
struct SortView;
hipError_t launch_preprocess_multi(const sx_gaussians& g, int V, const sx_camera* cams,
                                   const KParams& p, const sx_projected* outs, hipStream_t st);
hipError_t launch_preprocess_backward_multi(const sx_gaussians& g, int V, const DCam* cams,
                                            const sx_projected* projs, const SortView* svs,
                                            const float* const* g2d, const KParams& p,
                                            const sx_grads& gr, bool accumulate, hipStream_t st);
hipError_t launch_preprocess_backward(const sx_gaussians& g, const DCam& cam,
                                      const KParams& p,
                                      const sx_projected& proj, const SortView& sv,
                                      const float* g2d, const sx_grads& gr,
                                      bool accumulate, hipStream_t st);
hipError_t launch_sort(const sx_projected& proj, int64_t n, const KParams& p,
                       int64_t capacity, int64_t tiles_total, uint64_t* keys,
                       uint32_t* vals, uint32_t* ranges, char* ws,
                       uint64_t* h_counts, bool* over_capacity,
                       hipStream_t st);
hipError_t launch_render(const sx_projected& proj, const uint32_t* vals,
                         const uint32_t* ranges, const DCam& cam,
                         const KParams& p, const uint32_t* mask,
                         float* partial, float* depth, uint32_t* last,
                         uint32_t* nblend, hipStream_t st);
hipError_t launch_render_backward(const sx_projected& proj,
                                  const uint32_t* vals, const uint32_t* ranges,
                                  const SortView& sv, int64_t n, int64_t capacity,
                                  const DCam& cam, const KParams& p,
                                  const uint32_t* mask, const float* partial,
                                  const uint32_t* last, const float* dpartial,
                                  const float* ddepth, float* g2d, char* bws, int stages,
                                  hipStream_t st);
// one view of a batched call, in kernel-ready form
struct MultiView {
  DCam cam;
  int tiles_x, tiles_y;
  sx_projected proj;
  const uint32_t* vals;
  const uint32_t* ranges;
  const uint32_t* mask;
  float* partial;
  float* depth;
  uint32_t* last;
  uint32_t* nblend;
  const void* sort_ws;
  int64_t capacity;
  const float* dpartial;
  float* g2d;
  void* bwd_ws;
  int64_t n;  // Gaussians of the item's cell
};
size_t multi_workspace_bytes(int64_t items);
hipError_t launch_render_multi(int V, const MultiView* mv, const KParams& p, char* ws,
                               hipStream_t st);
hipError_t launch_render_backward_multi(int V, const MultiView* mv, const KParams& p,
                                        char* ws, hipStream_t st);
hipError_t launch_grad_reduce_view(const MultiView& v, const KParams& p, hipStream_t st);
// host: KD-tree partition of n means [n*3] into K boxes lo/hi [K*3], cell_of [n]
void kd_partition(int64_t n, const float* means, int K, float* lo, float* hi, int32_t* cell_of);
void repartition_plan(int64_t n, const int32_t* cell_of, int K, int32_t* dst_index,
                      int64_t* counts);
hipError_t launch_move_rows(int64_t n, int row_floats, int k_src, const int64_t* src_off,
                            const float* const* src, int k_dst, float* const* dst,
                            const int32_t* dst_cell, const int32_t* dst_index, hipStream_t st);
hipError_t launch_mask_counts(int K, const uint32_t* masks, int64_t words, uint32_t* counts,
                              hipStream_t st);
hipError_t launch_visibility(int K, const sx_cell* cells, const DCam& cam, uint32_t* masks,
                             hipStream_t st);
hipError_t launch_cross_filter(const sx_gaussians& g, const sx_projected& proj, int K,
                               const sx_cell* cells, int cell, const DCam& cam, uint32_t* xf,
                               hipStream_t st);
hipError_t launch_composite_l1(int K, const float* const* partials, const sx_cell* cells,
                               const DCam& cam, const KParams& p, const float* target,
                               float* out, uint32_t* masks, float* loss,
                               float* const* dpartials, hipStream_t st);
// budget non-NULL selects the re-evaluating form (masks then required)
hipError_t launch_composite(int K, const float* const* partials,
                            const sx_cell* cells, const DCam& cam,
                            const KParams& p, float* out, uint32_t* masks,
                            const uint32_t* omega, float* budget, hipStream_t st);
hipError_t launch_composite_backward(int K, const float* const* partials,
                                     const sx_cell* cells, const DCam& cam,
                                     const KParams& p, const float* dout,
                                     float* const* dpartials, hipStream_t st);
hipError_t launch_l1(const float* out, const float* target, int W, int H,
                     float* dout, float* loss, hipStream_t st);
hipError_t launch_adam(int64_t n, float* param, const float* grad, float* m,
                       float* v, float lr, float b1, float b2, float eps,
                       float bc1, float bc2, hipStream_t st);
hipError_t launch_fill(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);
bool tile_shape_supported(int tw, int th);
}  // namespace sx
