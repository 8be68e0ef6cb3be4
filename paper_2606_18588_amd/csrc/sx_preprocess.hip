// Projection of Gaussians to screen space and its backward (paper,
// background: projection step; Eq. 1 footprint; chain of the
// parametrisation Sigma = R S S^T R^T).
//
// One thread per Gaussian.  The arithmetic is FP64 (cheap on CDNA4: the
// kernel is bound by HBM reads of the parameters), rounded once to FP32 for
// the render record, so depths, footprints and tile counts are reproducible
// to the last bit.  A Gaussian culled by its mean depth costs one 12-byte
// read and a 4-byte write; only visible ones read rotation, scale, opacity
// and SH coefficients.
#include <cmath>

#include "sx_internal.h"

namespace sx {

struct PreArgs {
  int64_t n;
  const float* __restrict__ means;
  const float* __restrict__ log_scales;
  const float* __restrict__ quats;
  const float* __restrict__ logits;
  const float* __restrict__ sh;
  DCam cam;
  KParams p;
  struct {
    float R[9], t[3], fx, fy, cx, cy, znear, logit_min, tau_max, eps2d;
  } cull;
  float* __restrict__ rec;
  uint16_t* __restrict__ rect;
  uint32_t* __restrict__ n_tiles;
  uint32_t* __restrict__ block_sums;
};

// Screen-space quantities of one Gaussian, double precision.
struct Proj64 {
  double t[3];       // camera-space mean
  double Rq[9];      // rotation of the normalised quaternion
  double qh[4], qn;  // normalised quaternion and the input norm
  double s[3];       // scales
  double M[9];       // W Sigma W^T
  double J[6];
  double cov[3];     // dilated 2D covariance xx, xy, yy
  double conic[3];
  double o;
  double dir[3], dist;
};

// One Gaussian's geometric parameters, read with independent loads issued
// together (one memory round trip instead of one per culling test).
struct GIn {
  float m[3], ls[3], q[4], logit;
};
__device__ __forceinline__ GIn load_gin(const float* __restrict__ means,
                                        const float* __restrict__ log_scales,
                                        const float* __restrict__ quats,
                                        const float* __restrict__ logits, int64_t i) {
  GIn r;
#pragma unroll
  for (int k = 0; k < 3; ++k) r.m[k] = means[i * 3 + k], r.ls[k] = log_scales[i * 3 + k];
  const float4 q = reinterpret_cast<const float4*>(quats)[i];
  r.q[0] = q.x, r.q[1] = q.y, r.q[2] = q.z, r.q[3] = q.w;
  r.logit = logits[i];
  return r;
}

// Camera transform, culling and the EWA covariance.  Returns false when the
// Gaussian is culled (mean behind znear, zero quaternion, singular 2D
// covariance).
__device__ __forceinline__ bool project_geometry(const GIn& gi, const DCam& cam, double eps2d,
                                                 Proj64& g) {
  const double mx = gi.m[0], my = gi.m[1], mz = gi.m[2];
  for (int r = 0; r < 3; ++r)
    g.t[r] = cam.R[r * 3 + 0] * mx + cam.R[r * 3 + 1] * my + cam.R[r * 3 + 2] * mz + cam.t[r];
  if (!(g.t[2] > cam.znear)) return false;
  const double qw = gi.q[0], qx = gi.q[1], qy = gi.q[2], qz = gi.q[3];
  g.qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  if (g.qn < 1e-12) return false;
  g.qh[0] = qw / g.qn, g.qh[1] = qx / g.qn, g.qh[2] = qy / g.qn, g.qh[3] = qz / g.qn;
  quat_rot(g.qh[0], g.qh[1], g.qh[2], g.qh[3], g.Rq);
  double s2[3];
  for (int k = 0; k < 3; ++k) {
    g.s[k] = exp((double)gi.ls[k]);
    s2[k] = g.s[k] * g.s[k];
  }
  double Sig[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double v = 0;
      for (int k = 0; k < 3; ++k) v += g.Rq[r * 3 + k] * s2[k] * g.Rq[c * 3 + k];
      Sig[r * 3 + c] = v;
    }
  double WS[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double v = 0;
      for (int k = 0; k < 3; ++k) v += cam.R[r * 3 + k] * Sig[k * 3 + c];
      WS[r * 3 + c] = v;
    }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double v = 0;
      for (int k = 0; k < 3; ++k) v += WS[r * 3 + k] * cam.R[c * 3 + k];
      g.M[r * 3 + c] = v;
    }
  const double z = g.t[2];
  g.J[0] = cam.fx / z, g.J[1] = 0.0, g.J[2] = -cam.fx * g.t[0] / (z * z);
  g.J[3] = 0.0, g.J[4] = cam.fy / z, g.J[5] = -cam.fy * g.t[1] / (z * z);
  double JM[6];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c) {
      double v = 0;
      for (int k = 0; k < 3; ++k) v += g.J[r * 3 + k] * g.M[k * 3 + c];
      JM[r * 3 + c] = v;
    }
  double S2[4];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) {
      double v = 0;
      for (int k = 0; k < 3; ++k) v += JM[r * 3 + k] * g.J[c * 3 + k];
      S2[r * 2 + c] = v;
    }
  g.cov[0] = S2[0] + eps2d;
  g.cov[1] = 0.5 * (S2[1] + S2[2]);
  g.cov[2] = S2[3] + eps2d;
  const double det = g.cov[0] * g.cov[2] - g.cov[1] * g.cov[1];
  if (!(det > 0.0)) return false;
  g.conic[0] = g.cov[2] / det;
  g.conic[1] = -g.cov[1] / det;
  g.conic[2] = g.cov[0] / det;
  const double dv[3] = {mx - cam.C[0], my - cam.C[1], mz - cam.C[2]};
  g.dist = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
  for (int k = 0; k < 3; ++k) g.dir[k] = dv[k] / g.dist;
  return true;
}

// Cheap conservative test run by every Gaussian before the FP64 projection:
// mean depth, opacity, and whether the footprint can reach the image.  For
// any direction u, u^T Sigma2D u <= s_max^2 |J|_F^2 + eps2d, and
// tau <= 2 ln(1/alpha_min), so the half-extent of the alpha >= alpha_min
// footprint is at most E = sqrt(tau_max (s_max^2 |J|_F^2 + eps2d)); a mean
// projected farther than E outside the image cannot touch a pixel.  The test
// runs in FP32 with margins far above its rounding error (it only has to
// never drop a Gaussian the exact FP64 test in project_one would keep).
__device__ __forceinline__ bool maybe_visible(const PreArgs& a, int64_t i) {
  // the mean decides most culls (depth, and the guarded field of view that
  // project_one applies to the mean), so only the Gaussians that pass it
  // read their opacity and scales
  const float mx = a.means[i * 3 + 0], my = a.means[i * 3 + 1], mz = a.means[i * 3 + 2];
  const float* R = a.cull.R;
  const float p6 = R[6] * mx, p7 = R[7] * my, p8 = R[8] * mz;
  const float tz = p6 + p7 + p8 + a.cull.t[2];
  const float zslack = 1e-5f * (fabsf(p6) + fabsf(p7) + fabsf(p8) + fabsf(a.cull.t[2])) + 1e-6f;
  if (tz + zslack <= a.cull.znear) return false;
  const float tzc = fmaxf(tz, a.cull.znear * 0.5f);
  const float p0 = R[0] * mx, p1 = R[1] * my, p2 = R[2] * mz;
  const float p3 = R[3] * mx, p4 = R[4] * my, p5 = R[5] * mz;
  const float tx = p0 + p1 + p2 + a.cull.t[0];
  const float ty = p3 + p4 + p5 + a.cull.t[1];
  const float iz = 1.f / tzc;
  const float gd = (float)a.p.fov_guard;
  if (gd > 0.f) {
    // FP32 image of the FP64 test, widened far beyond its rounding error
    // (relative, and the absolute error of tx, ty scaled to pixels)
    const float qx = a.cull.fx * tx * iz, qy = a.cull.fy * ty * iz;
    const float ex = 1e-5f * (fabsf(p0) + fabsf(p1) + fabsf(p2) + fabsf(a.cull.t[0]));
    const float ey = 1e-5f * (fabsf(p3) + fabsf(p4) + fabsf(p5) + fabsf(a.cull.t[1]));
    const float mgx = 1e-4f * (fabsf(qx) + gd * (float)a.cam.W) + a.cull.fx * iz * ex + 1.f;
    const float mgy = 1e-4f * (fabsf(qy) + gd * (float)a.cam.H) + a.cull.fy * iz * ey + 1.f;
    if (qx < -gd * a.cull.cx - mgx || qx > gd * ((float)a.cam.W - a.cull.cx) + mgx) return false;
    if (qy < -gd * a.cull.cy - mgy || qy > gd * ((float)a.cam.H - a.cull.cy) + mgy) return false;
  }
  const float lgt = a.logits[i];
  if (lgt < a.cull.logit_min) return false;
  const float ls = fmaxf(fmaxf(a.log_scales[i * 3 + 0], a.log_scales[i * 3 + 1]),
                         a.log_scales[i * 3 + 2]);
  const float s2 = __expf(2.f * ls);
  const float jx = a.cull.fx * iz, jy = a.cull.fy * iz;
  const float jf = jx * jx * (1.f + tx * tx * iz * iz) + jy * jy * (1.f + ty * ty * iz * iz);
  const float E = sqrtf(a.cull.tau_max * (s2 * jf + a.cull.eps2d)) * 1.01f + 2.f;
  const float ux = a.cull.fx * tx * iz + a.cull.cx, uy = a.cull.fy * ty * iz + a.cull.cy;
  const float mxs = E + 1e-4f * fabsf(ux), mys = E + 1e-4f * fabsf(uy);
  if (ux + mxs < 0.f || ux - mxs > (float)a.cam.W) return false;
  if (uy + mys < 0.f || uy - mys > (float)a.cam.H) return false;
  return true;
}

template <int D>
__device__ __forceinline__ uint32_t project_one(const PreArgs& a, int64_t i) {
  const GIn gi = load_gin(a.means, a.log_scales, a.quats, a.logits, i);
  Proj64 g;
  if (!project_geometry(gi, a.cam, a.p.eps2d, g)) return 0;
  const double z = g.t[2];
  const double mx2 = a.cam.fx * g.t[0] / z, my2 = a.cam.fy * g.t[1] / z;
  // frustum cull by the mean: its offset from the principal point must lie
  // within the image's half-extents on each side, widened by fov_guard
  const double gd = a.p.fov_guard;
  if (gd > 0.0 && (mx2 < -(gd * a.cam.cx) || mx2 > gd * ((double)a.cam.W - a.cam.cx) ||
                   my2 < -(gd * a.cam.cy) || my2 > gd * ((double)a.cam.H - a.cam.cy)))
    return 0;
  const double mux = mx2 + a.cam.cx, muy = my2 + a.cam.cy;
  const double o = 1.0 / (1.0 + exp(-(double)gi.logit));
  if (o < a.p.alpha_min_d) return 0;
  // exact footprint of alpha >= alpha_min: q <= tau with tau = 2 ln(o/alpha_min)
  const double tau = 2.0 * log(o / a.p.alpha_min_d);
  const double ex = sqrt(tau * g.cov[0]), ey = sqrt(tau * g.cov[2]);
  double x0 = ceil(mux - ex - 0.5), x1 = floor(mux + ex - 0.5);
  double y0 = ceil(muy - ey - 0.5), y1 = floor(muy + ey - 0.5);
  x0 = fmin(fmax(x0, 0.0), (double)a.cam.W);
  y0 = fmin(fmax(y0, 0.0), (double)a.cam.H);
  x1 = fmin(fmax(x1, -1.0), (double)a.cam.W - 1);
  y1 = fmin(fmax(y1, -1.0), (double)a.cam.H - 1);
  if (!(x0 <= x1 && y0 <= y1)) return 0;
  const int tx0 = (int)x0 / a.p.tile_w, tx1 = (int)x1 / a.p.tile_w;
  const int ty0 = (int)y0 / a.p.tile_h, ty1 = (int)y1 / a.p.tile_h;
  // colour: max(0, sum_lm k_lm Y_lm(dir) + 0.5)
  constexpr int nc = (D + 1) * (D + 1);
  double Y[16];
  sh_basis(D, g.dir[0], g.dir[1], g.dir[2], Y);
  const float* __restrict__ shp = a.sh + (size_t)i * nc * 3;
  double col[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < nc; ++k) {
    col[0] += (double)shp[k * 3 + 0] * Y[k];
    col[1] += (double)shp[k * 3 + 1] * Y[k];
    col[2] += (double)shp[k * 3 + 2] * Y[k];
  }
  float* r = a.rec + (size_t)i * kRecFloats;
  float4 r0, r1, r2;
  r0.x = (float)mx2, r0.y = (float)my2, r0.z = (float)g.conic[0], r0.w = (float)g.conic[1];
  r1.x = (float)g.conic[2], r1.y = (float)o;
  r1.z = (float)fmax(col[0] + 0.5, 0.0), r1.w = (float)fmax(col[1] + 0.5, 0.0);
  r2.x = (float)fmax(col[2] + 0.5, 0.0), r2.y = (float)z;
  // pixel box of the footprint (inside the image, so 16-bit coordinates)
  r2.z = __uint_as_float((uint32_t)x0 | ((uint32_t)(x1 - x0) << 16));
  r2.w = __uint_as_float((uint32_t)y0 | ((uint32_t)(y1 - y0) << 16));
  reinterpret_cast<float4*>(r)[0] = r0;
  reinterpret_cast<float4*>(r)[1] = r1;
  reinterpret_cast<float4*>(r)[2] = r2;
  ushort4 rc;
  rc.x = (uint16_t)tx0, rc.y = (uint16_t)ty0, rc.z = (uint16_t)(tx1 + 1), rc.w = (uint16_t)(ty1 + 1);
  reinterpret_cast<ushort4*>(a.rect)[i] = rc;
  return (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
}

// Block-level compaction: lanes whose Gaussian may be visible are packed to
// the front of the block, so the FP64 projection runs in full wavefronts
// even when only a few percent of the scene is in view.
template <int D>
__device__ __forceinline__ void preprocess_block(const PreArgs& a, int64_t blk) {
  __shared__ uint32_t s_cand[kPreBlock];
  __shared__ uint32_t s_w[kPreBlock / 64];
  __shared__ uint32_t sv[kPreBlock / 64], sc[kPreBlock / 64];
  const int64_t i = blk * kPreBlock + threadIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  bool cand = false;
  if (i < a.n) {
    cand = maybe_visible(a, i);
    if (!cand) a.n_tiles[i] = 0;
  }
  const uint64_t bal = __ballot(cand);
  if (lane == 0) s_w[w] = (uint32_t)__popcll(bal);
  __syncthreads();
  uint32_t pre = 0, ncand = 0;
  for (int k = 0; k < kPreBlock / 64; ++k) {
    if (k < w) pre += s_w[k];
    ncand += s_w[k];
  }
  // most blocks of a large scene lie wholly outside the view: no FP64 work
  // and zero sums (ncand is the same in every thread, so the whole block
  // leaves here and no barrier below is left waiting)
  if (ncand == 0) {
    if (threadIdx.x == 0) {
      a.block_sums[2 * (size_t)blk + 0] = 0;
      a.block_sums[2 * (size_t)blk + 1] = 0;
    }
    return;
  }
  if (cand) s_cand[pre + __popcll(bal & ((1ull << lane) - 1))] = threadIdx.x;
  __syncthreads();
  uint32_t cnt = 0;
  if (threadIdx.x < ncand) {
    const int64_t ii = blk * kPreBlock + s_cand[threadIdx.x];
    cnt = project_one<D>(a, ii);
    a.n_tiles[ii] = cnt;
  }
  const uint32_t vis = (uint32_t)__popcll(__ballot(cnt > 0));
  cnt = __builtin_amdgcn_readlane(wave_sum_u32_to_lane63(cnt), 63);
  if (lane == 0) sv[w] = vis, sc[w] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t a0 = 0, a1 = 0;
    for (int k = 0; k < kPreBlock / 64; ++k) a0 += sv[k], a1 += sc[k];
    a.block_sums[2 * (size_t)blk + 0] = a0;
    a.block_sums[2 * (size_t)blk + 1] = a1;
  }
}

template <int D>
__global__ __launch_bounds__(kPreBlock) void k_preprocess(PreArgs a) {
  preprocess_block<D>(a, blockIdx.x);
}

// Several views in one launch: each workgroup takes one block of Gaussians
// and projects it for every view in turn, so the block's parameters come
// from HBM once and from the caches for the other views.
struct PreView {
  float R[9], t[3];
  float fx, fy, cx, cy, znear;
  int W, H, tiles_x, tiles_y;
  float* rec;
  uint16_t* rect;
  uint32_t* n_tiles;
  uint32_t* block_sums;
};
struct PreMultiArgs {
  int64_t n;
  int V;
  const float* __restrict__ means;
  const float* __restrict__ log_scales;
  const float* __restrict__ quats;
  const float* __restrict__ logits;
  const float* __restrict__ sh;
  KParams p;  // tiles_x / tiles_y are per view
  float logit_min, tau_max;
  PreView v[kMaxViews];
};

template <int D>
__device__ __forceinline__ void preprocess_view(const PreMultiArgs& m, int v, int64_t blk) {
  const PreView& pv = m.v[v];
  PreArgs a;
  a.n = m.n;
  a.means = m.means, a.log_scales = m.log_scales, a.quats = m.quats;
  a.logits = m.logits, a.sh = m.sh;
  for (int k = 0; k < 9; ++k) a.cam.R[k] = pv.R[k];
  for (int k = 0; k < 3; ++k) a.cam.t[k] = pv.t[k];
  a.cam.fx = pv.fx, a.cam.fy = pv.fy, a.cam.cx = pv.cx, a.cam.cy = pv.cy, a.cam.znear = pv.znear;
  for (int j = 0; j < 3; ++j)
    a.cam.C[j] = -(a.cam.R[0 * 3 + j] * a.cam.t[0] + a.cam.R[1 * 3 + j] * a.cam.t[1] +
                   a.cam.R[2 * 3 + j] * a.cam.t[2]);
  a.cam.W = pv.W, a.cam.H = pv.H;
  a.p = m.p;
  a.p.tiles_x = pv.tiles_x, a.p.tiles_y = pv.tiles_y;
  for (int k = 0; k < 9; ++k) a.cull.R[k] = pv.R[k];
  for (int k = 0; k < 3; ++k) a.cull.t[k] = pv.t[k];
  a.cull.fx = pv.fx, a.cull.fy = pv.fy, a.cull.cx = pv.cx, a.cull.cy = pv.cy;
  a.cull.znear = pv.znear;
  a.cull.logit_min = m.logit_min, a.cull.tau_max = m.tau_max, a.cull.eps2d = (float)m.p.eps2d;
  a.rec = pv.rec, a.rect = pv.rect, a.n_tiles = pv.n_tiles, a.block_sums = pv.block_sums;
  preprocess_block<D>(a, blk);
}

template <int D>
__global__ __launch_bounds__(kPreBlock) void k_preprocess_multi(PreMultiArgs m) {
  for (int v = 0; v < m.V; ++v) {
    preprocess_view<D>(m, v, blockIdx.x);
    __syncthreads();  // the next view reuses the block's LDS
  }
}

hipError_t launch_preprocess_multi(const sx_gaussians& g, int V, const sx_camera* cams,
                                   const KParams& p, const sx_projected* outs, hipStream_t st) {
  if (g.n == 0 || V == 0) return hipSuccess;
  PreMultiArgs m;
  m.n = g.n;
  m.V = V;
  m.means = g.means, m.log_scales = g.log_scales, m.quats = g.quats;
  m.logits = g.opacity_logits, m.sh = g.sh;
  m.p = p;
  m.logit_min = (float)(std::log(p.alpha_min_d / (1.0 - p.alpha_min_d)) - 1e-3);
  m.tau_max = (float)(2.0 * std::log(1.0 / p.alpha_min_d));
  for (int v = 0; v < V; ++v) {
    const sx_camera& c = cams[v];
    PreView& pv = m.v[v];
    for (int k = 0; k < 9; ++k) pv.R[k] = c.R[k];
    for (int k = 0; k < 3; ++k) pv.t[k] = c.t[k];
    pv.fx = c.fx, pv.fy = c.fy, pv.cx = c.cx, pv.cy = c.cy, pv.znear = c.znear;
    pv.W = c.width, pv.H = c.height;
    pv.tiles_x = (c.width + p.tile_w - 1) / p.tile_w;
    pv.tiles_y = (c.height + p.tile_h - 1) / p.tile_h;
    pv.rec = outs[v].rec, pv.rect = outs[v].rect, pv.n_tiles = outs[v].n_tiles;
    pv.block_sums = outs[v].block_sums;
  }
  const dim3 grid((unsigned)((g.n + kPreBlock - 1) / kPreBlock));
  switch (p.sh_degree) {
    case 0: hipLaunchKernelGGL(k_preprocess_multi<0>, grid, dim3(kPreBlock), 0, st, m); break;
    case 1: hipLaunchKernelGGL(k_preprocess_multi<1>, grid, dim3(kPreBlock), 0, st, m); break;
    case 2: hipLaunchKernelGGL(k_preprocess_multi<2>, grid, dim3(kPreBlock), 0, st, m); break;
    default: hipLaunchKernelGGL(k_preprocess_multi<3>, grid, dim3(kPreBlock), 0, st, m); break;
  }
  return hipGetLastError();
}

hipError_t launch_preprocess(const sx_gaussians& g, const DCam& cam,
                             const KParams& p, const sx_projected& out,
                             hipStream_t st) {
  if (g.n == 0) return hipSuccess;
  PreArgs a;
  a.n = g.n;
  a.means = g.means, a.log_scales = g.log_scales, a.quats = g.quats;
  a.logits = g.opacity_logits, a.sh = g.sh;
  a.cam = cam, a.p = p;
  for (int k = 0; k < 9; ++k) a.cull.R[k] = (float)cam.R[k];
  for (int k = 0; k < 3; ++k) a.cull.t[k] = (float)cam.t[k];
  a.cull.fx = (float)cam.fx, a.cull.fy = (float)cam.fy;
  a.cull.cx = (float)cam.cx, a.cull.cy = (float)cam.cy;
  a.cull.znear = (float)cam.znear;
  // o < alpha_min  <=>  logit < ln(alpha_min / (1 - alpha_min)); keep a margin
  a.cull.logit_min = (float)(std::log(p.alpha_min_d / (1.0 - p.alpha_min_d)) - 1e-3);
  a.cull.tau_max = (float)(2.0 * std::log(1.0 / p.alpha_min_d));
  a.cull.eps2d = (float)p.eps2d;
  a.rec = out.rec, a.rect = out.rect, a.n_tiles = out.n_tiles;
  a.block_sums = out.block_sums;
  const int64_t blocks = (g.n + kPreBlock - 1) / kPreBlock;
  switch (p.sh_degree) {
    case 0: hipLaunchKernelGGL(k_preprocess<0>, dim3((unsigned)blocks), dim3(kPreBlock), 0, st, a); break;
    case 1: hipLaunchKernelGGL(k_preprocess<1>, dim3((unsigned)blocks), dim3(kPreBlock), 0, st, a); break;
    case 2: hipLaunchKernelGGL(k_preprocess<2>, dim3((unsigned)blocks), dim3(kPreBlock), 0, st, a); break;
    default: hipLaunchKernelGGL(k_preprocess<3>, dim3((unsigned)blocks), dim3(kPreBlock), 0, st, a); break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- backward
struct PreBwdArgs {
  int64_t n;
  const float* __restrict__ means;
  const float* __restrict__ log_scales;
  const float* __restrict__ quats;
  const float* __restrict__ logits;
  const float* __restrict__ sh;
  const uint32_t* __restrict__ n_tiles;
  const uint32_t* __restrict__ vis;  // compacted visible Gaussians
  const uint64_t* vis_count;
  const float* __restrict__ g2d;
  DCam cam;
  KParams p;
  float* gmeans;
  float* glog_scales;
  float* gquats;
  float* glogits;
  float* gsh;
  int accumulate;
};

__device__ __forceinline__ void put(float* p, double v, bool acc) {
  if (acc)
    *p += (float)v;
  else
    *p = (float)v;
}

// Chain of screen-space gradients (mean2d, conic, opacity, colour, depth)
// to the parameters: conic -> 2D covariance (G_S = -A Gc A), -> (J, M)
// (dM = J^T G_S J, dJ = 2 G_S J M), M -> Sigma (W^T dM W), Sigma = L L^T
// with L = R(q) S (dL = 2 dSigma L) -> log-scales and the quaternion; the
// mean through mean2d, J(t), depth and the SH view direction.
template <int D>
__device__ __forceinline__ void backward_one(const PreBwdArgs& a, int64_t i, bool acc) {
  const GIn gi = load_gin(a.means, a.log_scales, a.quats, a.logits, i);
  Proj64 g;
  if (!project_geometry(gi, a.cam, a.p.eps2d, g)) return;
  const float* gr = a.g2d + (size_t)i * kG2dFloats;
  const float4 g0 = reinterpret_cast<const float4*>(gr)[0];
  const float4 g1 = reinterpret_cast<const float4*>(gr)[1];
  const float2 g2 = reinterpret_cast<const float2*>(gr)[4];
  const double gmx = g0.x, gmy = g0.y, ga = g0.z, gb = g0.w, gc = g1.x, gop = g1.y;
  const double gcol[3] = {g1.z, g1.w, g2.x};
  const double gz = g2.y;
  constexpr int nc = (D + 1) * (D + 1);
  constexpr int nf = nc * 3;
  // colour -> SH coefficients and direction.  The clamp decision uses the
  // forward's FP64 sum; the direction gradient runs in FP32.  Rows of nf
  // floats are moved as float4 where nf is a multiple of 4 (SH1, SH3).
  double Y[16];
  sh_basis(D, g.dir[0], g.dir[1], g.dir[2], Y);
  float dY[48];
  sh_basis_grad<float>(D, (float)g.dir[0], (float)g.dir[1], (float)g.dir[2], dY);
  float sh[nf];
  const float* __restrict__ shp = a.sh + (size_t)i * nf;
  if constexpr (nf % 4 == 0) {
#pragma unroll
    for (int j = 0; j < nf / 4; ++j) {
      const float4 q = reinterpret_cast<const float4*>(shp)[j];
      sh[4 * j] = q.x, sh[4 * j + 1] = q.y, sh[4 * j + 2] = q.z, sh[4 * j + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < nf; ++j) sh[j] = shp[j];
  }
  float gcv[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < nc; ++k) v += (double)sh[k * 3 + ch] * Y[k];
    gcv[ch] = v + 0.5 > 0.0 ? (float)gcol[ch] : 0.f;
  }
  float gdf[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < nc; ++k)
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const float w = gcv[ch] * sh[k * 3 + ch];
      gdf[0] += w * dY[k * 3 + 0];
      gdf[1] += w * dY[k * 3 + 1];
      gdf[2] += w * dY[k * 3 + 2];
    }
  float* gshp = a.gsh + (size_t)i * nf;
  auto gsh_at = [&](int j) { return (float)((double)gcv[j % 3] * Y[j / 3]); };
  if constexpr (nf % 4 == 0) {
#pragma unroll
    for (int j = 0; j < nf / 4; ++j) {
      float4 q = make_float4(gsh_at(4 * j), gsh_at(4 * j + 1), gsh_at(4 * j + 2), gsh_at(4 * j + 3));
      if (acc) {
        const float4 o = reinterpret_cast<const float4*>(gshp)[j];
        q.x += o.x, q.y += o.y, q.z += o.z, q.w += o.w;
      }
      reinterpret_cast<float4*>(gshp)[j] = q;
    }
  } else {
#pragma unroll
    for (int j = 0; j < nf; ++j) put(&gshp[j], (double)gsh_at(j), acc);
  }
  const double gdir[3] = {gdf[0], gdf[1], gdf[2]};
  double gmu[3];
  {
    const double dd = gdir[0] * g.dir[0] + gdir[1] * g.dir[1] + gdir[2] * g.dir[2];
    for (int k = 0; k < 3; ++k) gmu[k] = (gdir[k] - dd * g.dir[k]) / g.dist;
  }
  // opacity through the sigmoid
  const double o = 1.0 / (1.0 + exp(-(double)gi.logit));
  put(&a.glogits[i], gop * o * (1.0 - o), acc);
  // conic -> covariance
  const double A[4] = {g.conic[0], g.conic[1], g.conic[1], g.conic[2]};
  const double Gc[4] = {ga, 0.5 * gb, 0.5 * gb, gc};
  double T1[4], GS[4];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) T1[r * 2 + c] = A[r * 2 + 0] * Gc[0 * 2 + c] + A[r * 2 + 1] * Gc[1 * 2 + c];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) GS[r * 2 + c] = -(T1[r * 2 + 0] * A[0 * 2 + c] + T1[r * 2 + 1] * A[1 * 2 + c]);
  double dM[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double v = 0;
      for (int u = 0; u < 2; ++u)
        for (int w = 0; w < 2; ++w) v += g.J[u * 3 + r] * GS[u * 2 + w] * g.J[w * 3 + c];
      dM[r * 3 + c] = v;
    }
  double GJ[6], dJ[6];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c) GJ[r * 3 + c] = GS[r * 2 + 0] * g.J[0 * 3 + c] + GS[r * 2 + 1] * g.J[1 * 3 + c];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c) {
      double v = 0;
      for (int k = 0; k < 3; ++k) v += GJ[r * 3 + k] * g.M[k * 3 + c];
      dJ[r * 3 + c] = 2.0 * v;
    }
  const double* W = a.cam.R;
  double Tm[9], dS[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double v = 0;
      for (int k = 0; k < 3; ++k) v += W[k * 3 + r] * dM[k * 3 + c];
      Tm[r * 3 + c] = v;
    }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double v = 0;
      for (int k = 0; k < 3; ++k) v += Tm[r * 3 + k] * W[k * 3 + c];
      dS[r * 3 + c] = v;
    }
  // dL = 2 dSigma L, L = Rq diag(s)
  double dLm[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double v = 0;
      for (int k = 0; k < 3; ++k) v += dS[r * 3 + k] * g.Rq[k * 3 + c] * g.s[c];
      dLm[r * 3 + c] = 2.0 * v;
    }
  for (int k = 0; k < 3; ++k) {
    double v = 0;
    for (int r = 0; r < 3; ++r) v += dLm[r * 3 + k] * g.Rq[r * 3 + k];
    put(&a.glog_scales[i * 3 + k], v * g.s[k], acc);
  }
  double dR[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) dR[r * 3 + c] = dLm[r * 3 + c] * g.s[c];
  const double w = g.qh[0], x = g.qh[1], y = g.qh[2], zq = g.qh[3];
  double dq[4];
  dq[0] = 2.0 * (-zq * dR[1] + y * dR[2] + zq * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
  dq[1] = 2.0 * (y * dR[1] + zq * dR[2] + y * dR[3] - 2.0 * x * dR[4] - w * dR[5] + zq * dR[6] +
                 w * dR[7] - 2.0 * x * dR[8]);
  dq[2] = 2.0 * (-2.0 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + zq * dR[5] - w * dR[6] +
                 zq * dR[7] - 2.0 * y * dR[8]);
  dq[3] = 2.0 * (-2.0 * zq * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.0 * zq * dR[4] +
                 y * dR[5] + x * dR[6] + y * dR[7]);
  {
    const double dd = dq[0] * g.qh[0] + dq[1] * g.qh[1] + dq[2] * g.qh[2] + dq[3] * g.qh[3];
    for (int k = 0; k < 4; ++k) put(&a.gquats[i * 4 + k], (dq[k] - dd * g.qh[k]) / g.qn, acc);
  }
  // mean: mean2d, J(t), depth; then world = W^T dt (+ SH direction term)
  const double z = g.t[2], fx = a.cam.fx, fy = a.cam.fy;
  const double tx = g.t[0], ty = g.t[1];
  double dt[3];
  dt[0] = gmx * fx / z + dJ[2] * (-fx / (z * z));
  dt[1] = gmy * fy / z + dJ[5] * (-fy / (z * z));
  dt[2] = gmx * (-fx * tx / (z * z)) + gmy * (-fy * ty / (z * z)) + dJ[0] * (-fx / (z * z)) +
          dJ[2] * (2.0 * fx * tx / (z * z * z)) + dJ[4] * (-fy / (z * z)) +
          dJ[5] * (2.0 * fy * ty / (z * z * z)) + gz;
  for (int k = 0; k < 3; ++k)
    put(&a.gmeans[i * 3 + k],
             W[0 * 3 + k] * dt[0] + W[1 * 3 + k] * dt[1] + W[2 * 3 + k] * dt[2] + gmu[k], acc);
}

// One lane per visible Gaussian, taken from the sort's compacted list in
// index order, so the FP64 chain runs in full wavefronts and neighbouring
// lanes read and write neighbouring parameter rows.  The grid is capped
// (kPreBwdGrid workgroups, each striding over the list): the visible count
// is known on the device only, and a grid sized for every Gaussian would
// send thousands of workgroups that find nothing to do through the few
// slots this kernel's register footprint leaves per CU (two workgroups),
// each holding its slot for a memory round trip.
constexpr unsigned kPreBwdGrid = 1024;
template <int D, bool ACC>
__global__ __launch_bounds__(kPreBlock) void k_preprocess_backward(PreBwdArgs a) {
  const uint64_t nv = a.vis_count[0];
  for (uint64_t i = (uint64_t)blockIdx.x * kPreBlock + threadIdx.x; i < nv;
       i += (uint64_t)gridDim.x * kPreBlock) {
    const uint32_t g = a.vis[i];
    if (a.n_tiles[g] != 0) backward_one<D>(a, (int64_t)g, ACC);
  }
}

hipError_t launch_preprocess_backward(const sx_gaussians& g, const DCam& cam,
                                      const KParams& p,
                                      const sx_projected& proj, const SortView& sv,
                                      const float* g2d, const sx_grads& gr,
                                      bool accumulate, hipStream_t st) {
  if (g.n == 0) return hipSuccess;
  PreBwdArgs a;
  a.vis = sv.vidx;
  a.vis_count = sv.counts;
  a.n = g.n;
  a.means = g.means, a.log_scales = g.log_scales, a.quats = g.quats;
  a.logits = g.opacity_logits, a.sh = g.sh;
  a.n_tiles = proj.n_tiles;
  a.g2d = g2d;
  a.cam = cam, a.p = p;
  a.gmeans = gr.means, a.glog_scales = gr.log_scales, a.gquats = gr.quats;
  a.glogits = gr.opacity_logits, a.gsh = gr.sh;
  a.accumulate = accumulate ? 1 : 0;
  const int64_t blocks = (g.n + kPreBlock - 1) / kPreBlock;
  const dim3 grid((unsigned)(blocks < kPreBwdGrid ? blocks : kPreBwdGrid));
#define SX_PB(D)                                                                               \
  do {                                                                                         \
    if (accumulate)                                                                            \
      hipLaunchKernelGGL((k_preprocess_backward<D, true>), grid, dim3(kPreBlock), 0, st, a);   \
    else                                                                                       \
      hipLaunchKernelGGL((k_preprocess_backward<D, false>), grid, dim3(kPreBlock), 0, st, a);  \
  } while (0)
  switch (p.sh_degree) {
    case 0: SX_PB(0); break;
    case 1: SX_PB(1); break;
    case 2: SX_PB(2); break;
    default: SX_PB(3); break;
  }
#undef SX_PB
  return hipGetLastError();
}

// Several views of one set of Gaussians: the per-view kernel once per view,
// in view order, accumulating, so each Gaussian receives its views'
// contributions in that order (the same sums as one accumulating call per
// view).  Without accumulation the gradients are cleared first.  (One
// launch that looped over the views inside each workgroup, to read the
// parameters once, measured slower: per view only the lanes of Gaussians
// that view sees were busy between workgroup barriers.)
hipError_t launch_preprocess_backward_multi(const sx_gaussians& g, int V, const DCam* cams,
                                            const sx_projected* projs, const SortView* svs,
                                            const float* const* g2d, const KParams& p,
                                            const sx_grads& gr, bool accumulate, hipStream_t st) {
  if (g.n == 0 || V == 0) return hipSuccess;
  hipError_t e = hipSuccess;
  if (!accumulate) {
    const int nf = (p.sh_degree + 1) * (p.sh_degree + 1) * 3;
    if ((e = launch_fill(reinterpret_cast<uint32_t*>(gr.means), g.n * 3, 0, st))) return e;
    if ((e = launch_fill(reinterpret_cast<uint32_t*>(gr.log_scales), g.n * 3, 0, st))) return e;
    if ((e = launch_fill(reinterpret_cast<uint32_t*>(gr.quats), g.n * 4, 0, st))) return e;
    if ((e = launch_fill(reinterpret_cast<uint32_t*>(gr.opacity_logits), g.n, 0, st))) return e;
    if ((e = launch_fill(reinterpret_cast<uint32_t*>(gr.sh), g.n * nf, 0, st))) return e;
  }
  for (int v = 0; v < V; ++v)
    if ((e = launch_preprocess_backward(g, cams[v], p, projs[v], svs[v], g2d[v], gr, true, st)))
      return e;
  return hipSuccess;
}

}  // namespace sx

namespace sx {

// ------------------------------------------------- cross-boundary filter --
// Bits of the per-ray cross-boundary filter of one cell's Gaussians for one
// view (appendix, implementation details: cross-boundary Gaussians).  Bit s
// of xf[i] is set when Gaussian i is visible, its 3-sigma support box,
// mean +- 3 sqrt(Sigma_aa), meets box s (s != cell) and its camera depth
// lies in [dlo[s], dhi[s]], the overlap of the camera-z ranges of box s and
// of the cell's own box (computed on the host).  The render removes the
// Gaussian from the rays whose pixel lies in the visibility maps of both.
struct XFArgs {
  const float* __restrict__ means;
  const float* __restrict__ log_scales;
  const float4* __restrict__ quats;
  const float* __restrict__ rec;
  const uint32_t* __restrict__ n_tiles;
  int64_t n;
  int K, cell;
  float lo[kMaxCells][3], hi[kMaxCells][3];
  float dlo[kMaxCells], dhi[kMaxCells];
  uint32_t* __restrict__ xf;
};

__global__ __launch_bounds__(256) void k_cross_filter(XFArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.n) return;
  uint32_t bits = 0;
  if (a.n_tiles[i] != 0) {
    const float4 q4 = a.quats[i];
    const float qn = sqrtf(q4.x * q4.x + q4.y * q4.y + q4.z * q4.z + q4.w * q4.w);
    const float w = q4.x / qn, x = q4.y / qn, y = q4.z / qn, z = q4.w / qn;
    const float R[9] = {1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y),
                        2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x),
                        2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)};
    float s[3], mu[3], h[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) s[b] = expf(a.log_scales[3 * i + b]), mu[b] = a.means[3 * i + b];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      float v = 0.f;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const float e = R[3 * r + b] * s[b];
        v = fmaf(e, e, v);
      }
      h[r] = 3.f * sqrtf(v);
    }
    const float d = a.rec[(size_t)i * kRecFloats + 9];
    for (int c = 0; c < a.K; ++c) {
      if (c == a.cell) continue;
      bool meets = d >= a.dlo[c] && d <= a.dhi[c];
#pragma unroll
      for (int r = 0; r < 3; ++r)
        meets = meets && mu[r] - h[r] < a.hi[c][r] && mu[r] + h[r] > a.lo[c][r];
      bits |= meets ? 1u << c : 0u;
    }
  }
  a.xf[i] = bits;
}

hipError_t launch_cross_filter(const sx_gaussians& g, const sx_projected& proj, int K,
                               const sx_cell* cells, int cell, const DCam& cam, uint32_t* xf,
                               hipStream_t st) {
  XFArgs a;
  a.means = g.means;
  a.log_scales = g.log_scales;
  a.quats = reinterpret_cast<const float4*>(g.quats);
  a.rec = proj.rec;
  a.n_tiles = proj.n_tiles;
  a.n = g.n;
  a.K = K, a.cell = cell;
  // camera-z range of each box: z = R[2] . x + t[2] is linear over the box
  double zlo[kMaxCells], zhi[kMaxCells];
  for (int m = 0; m < K; ++m) {
    double lo = cam.t[2], hi = cam.t[2];
    for (int j = 0; j < 3; ++j) {
      a.lo[m][j] = cells[m].lo[j], a.hi[m][j] = cells[m].hi[j];
      const double r = cam.R[6 + j];
      if (r == 0.0) continue;
      const double u = r * (double)cells[m].lo[j], v = r * (double)cells[m].hi[j];
      lo += u < v ? u : v;
      hi += u < v ? v : u;
    }
    zlo[m] = lo, zhi[m] = hi;
  }
  for (int m = 0; m < K; ++m) {
    a.dlo[m] = (float)(zlo[m] > zlo[cell] ? zlo[m] : zlo[cell]);
    a.dhi[m] = (float)(zhi[m] < zhi[cell] ? zhi[m] : zhi[cell]);
  }
  a.xf = xf;
  if (g.n > 0)
    hipLaunchKernelGGL(k_cross_filter, dim3((unsigned)((g.n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace sx
