// Partial render of one cell (Eq. 1-4) and its backward (Eq. 6-7, the part
// local to one cell).
//
// One workgroup per screen tile, one lane per pixel.  Every lane of a tile
// walks the same depth-sorted list, so the Gaussian index and its 48-byte
// record are wavefront-uniform: they are fetched with scalar loads into
// SGPRs and feed the VALU directly as scalar operands.  No LDS staging and
// no workgroup barrier is needed; each wavefront leaves the list as soon as
// a ballot says all its pixels are saturated (T < t_min) or masked.
//
// Workgroups are dispatched round-robin over the 8 XCDs of the chip; the
// block -> tile map gives every XCD a contiguous band of tiles so that
// neighbouring tiles, which share most of their Gaussians, share an L2.
#include "sx_internal.h"

namespace sx {

struct RenderArgs {
  const float* __restrict__ rec;
  const uint32_t* __restrict__ vals;
  const uint2* __restrict__ ranges;
  const uint32_t* __restrict__ mask;
  int W, H, tiles_x, tiles_y;
  float cx, cy;
  float alpha_min, alpha_max, t_min;
  float4* __restrict__ partial;
  float* __restrict__ depth;
  uint32_t* __restrict__ last;
  uint32_t* __restrict__ nblend;
};

__device__ __forceinline__ int xcd_tile(int b, int ntile) {
  const int per = (ntile + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}

template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void k_render(RenderArgs a) {
  const int ntile = a.tiles_x * a.tiles_y;
  const int tile = xcd_tile(blockIdx.x, ntile);
  if (tile >= ntile) return;
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const int lx = threadIdx.x % TW, ly = threadIdx.x / TW;
  const int px = tx * TW + lx, py = ty * TH + ly;
  const bool inside = px < a.W && py < a.H;
  const uint32_t pix = (uint32_t)py * a.W + px;
  bool active = inside;
  if (active && a.mask) active = (a.mask[pix >> 5] >> (pix & 31)) & 1u;
  const float fx = (float)px + 0.5f - a.cx, fy = (float)py + 0.5f - a.cy;
  const uint2 rg = a.ranges[tile];
  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f;
  uint32_t lst = 0, nb = 0;
  bool done = !active;
  for (uint32_t j = rg.x; j < rg.y; ++j) {
    if (__ballot(!done) == 0) break;
    const uint32_t g = a.vals[j];
    const float4* r = reinterpret_cast<const float4*>(a.rec + (size_t)g * kRecFloats);
    const float4 r0 = r[0], r1 = r[1], r2 = r[2];
    const AlphaEval ae = eval_alpha(fx - r0.x, fy - r0.y, r0.z, r0.w, r1.x, r1.y, a.alpha_max);
    if (!done && ae.alpha >= a.alpha_min) {
      const float w = ae.alpha * T;
      C0 = fmaf(r1.z, w, C0);
      C1 = fmaf(r1.w, w, C1);
      C2 = fmaf(r2.x, w, C2);
      D = fmaf(r2.y, w, D);
      T = T * (1.f - ae.alpha);
      ++nb;
      lst = j - rg.x + 1;
      if (T < a.t_min) done = true;
    }
  }
  if (inside) {
    a.partial[pix] = make_float4(C0, C1, C2, T);
    a.last[pix] = lst;
    if (a.depth) a.depth[pix] = D;
    if (a.nblend) a.nblend[pix] = nb;
  }
}

struct RenderBwdArgs {
  const float* __restrict__ rec;
  const uint32_t* __restrict__ vals;
  const uint2* __restrict__ ranges;
  const uint32_t* __restrict__ mask;
  int W, H, tiles_x, tiles_y;
  float cx, cy;
  float alpha_min, alpha_max;
  const float4* __restrict__ partial;
  const uint32_t* __restrict__ last;
  const float4* __restrict__ dpartial;
  const float* __restrict__ ddepth;
  float* g2d;
};

// Reverse walk of each pixel's blended pairs.  With R the colour behind pair
// i (normalised by T_{i+1}), T_final the partial transmittance and
// (G, g_T, g_D) the gradients of (C^m, T^m, D^m):
//   dc_i = alpha_i T_i G,   dz_i = alpha_i T_i g_D,
//   dalpha_i = T_i [G.(c_i - R) + g_D (z_i - RD)] - g_T T_final / (1 - alpha_i)
// then alpha = o exp(-q/2) gives do = dalpha exp(-q/2), dq = -alpha/2 dalpha
// (zero when alpha was clamped), and q gives the mean2d and conic terms.
// Gradients are summed over the wavefront (DPP) and added with one atomic
// per (Gaussian, wavefront, field).
template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void k_render_bwd(RenderBwdArgs a) {
  const int ntile = a.tiles_x * a.tiles_y;
  const int tile = xcd_tile(blockIdx.x, ntile);
  if (tile >= ntile) return;
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const int lx = threadIdx.x % TW, ly = threadIdx.x / TW;
  const int px = tx * TW + lx, py = ty * TH + ly;
  const bool inside = px < a.W && py < a.H;
  const uint32_t pix = inside ? (uint32_t)py * a.W + px : 0u;
  bool active = inside;
  if (active && a.mask) active = (a.mask[pix >> 5] >> (pix & 31)) & 1u;
  const float fx = (float)px + 0.5f - a.cx, fy = (float)py + 0.5f - a.cy;
  const uint2 rg = a.ranges[tile];
  float Tfin = 1.f;
  float4 gC = make_float4(0.f, 0.f, 0.f, 0.f);
  float gD = 0.f;
  uint32_t my_last = 0;
  if (active) {
    Tfin = a.partial[pix].w;
    gC = a.dpartial[pix];
    if (a.ddepth) gD = a.ddepth[pix];
    my_last = a.last[pix];
  }
  const uint32_t wave_last = wave_max_u32(my_last);
  const bool lane63 = (threadIdx.x & 63) == 63;
  float T = Tfin, R0 = 0.f, R1 = 0.f, R2 = 0.f, RD = 0.f;
  for (int k = (int)wave_last - 1; k >= 0; --k) {
    const uint32_t j = rg.x + (uint32_t)k;
    const uint32_t g = a.vals[j];
    const float4* r = reinterpret_cast<const float4*>(a.rec + (size_t)g * kRecFloats);
    const float4 r0 = r[0], r1 = r[1], r2 = r[2];
    const float dx = fx - r0.x, dy = fy - r0.y;
    const AlphaEval ae = eval_alpha(dx, dy, r0.z, r0.w, r1.x, r1.y, a.alpha_max);
    const bool contrib = (uint32_t)k < my_last && ae.alpha >= a.alpha_min;
    if (__ballot(contrib) == 0) continue;
    float v[10];
#pragma unroll
    for (int m = 0; m < 10; ++m) v[m] = 0.f;
    if (contrib) {
      const float om = 1.f - ae.alpha;
      const float rom = 1.f / om;
      const float Ti = T * rom;
      const float w = ae.alpha * Ti;
      v[6] = w * gC.x;
      v[7] = w * gC.y;
      v[8] = w * gC.z;
      v[9] = w * gD;
      float da = gC.x * (r1.z - R0) + gC.y * (r1.w - R1) + gC.z * (r2.x - R2) + gD * (r2.y - RD);
      da = Ti * da - gC.w * (Tfin * rom);
      R0 = fmaf(r1.z, ae.alpha, om * R0);
      R1 = fmaf(r1.w, ae.alpha, om * R1);
      R2 = fmaf(r2.x, ae.alpha, om * R2);
      RD = fmaf(r2.y, ae.alpha, om * RD);
      T = Ti;
      if (!ae.clamped) {
        v[5] = da * ae.G;
        const float dq = -0.5f * ae.alpha * da;
        v[0] = -2.f * dq * (r0.z * dx + r0.w * dy);
        v[1] = -2.f * dq * (r0.w * dx + r1.x * dy);
        v[2] = dq * dx * dx;
        v[3] = 2.f * dq * dx * dy;
        v[4] = dq * dy * dy;
      }
    }
    float* dst = a.g2d + (size_t)g * kG2dFloats;
#pragma unroll
    for (int m = 0; m < 10; ++m) {
      const float s = wave_sum_to_lane63(v[m]);
      if (lane63) unsafeAtomicAdd(dst + m, s);
    }
  }
}

__global__ __launch_bounds__(256) void k_zero_g2d(const uint32_t* __restrict__ n_tiles, int64_t n,
                                                  float* __restrict__ g2d) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n || n_tiles[i] == 0) return;
  float4* d = reinterpret_cast<float4*>(g2d + (size_t)i * kG2dFloats);
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
  d[0] = z, d[1] = z, d[2] = z;
}

bool tile_shape_supported(int tw, int th) {
  return (tw == 16 && th == 16) || (tw == 32 && th == 8) || (tw == 8 && th == 32) ||
         (tw == 32 && th == 16) || (tw == 16 && th == 32) || (tw == 8 && th == 8);
}

template <int TW, int TH>
static void launch_fwd_t(const RenderArgs& a, hipStream_t st) {
  const int ntile = a.tiles_x * a.tiles_y;
  const int grid = ((ntile + 7) >> 3) * 8;
  hipLaunchKernelGGL((k_render<TW, TH>), dim3(grid), dim3(TW * TH), 0, st, a);
}
template <int TW, int TH>
static void launch_bwd_t(const RenderBwdArgs& a, hipStream_t st) {
  const int ntile = a.tiles_x * a.tiles_y;
  const int grid = ((ntile + 7) >> 3) * 8;
  hipLaunchKernelGGL((k_render_bwd<TW, TH>), dim3(grid), dim3(TW * TH), 0, st, a);
}

#define SX_DISPATCH_TILE(tw, th, FN, ARGS, ST)           \
  do {                                                   \
    if (tw == 16 && th == 16) FN<16, 16>(ARGS, ST);      \
    else if (tw == 32 && th == 8) FN<32, 8>(ARGS, ST);   \
    else if (tw == 8 && th == 32) FN<8, 32>(ARGS, ST);   \
    else if (tw == 32 && th == 16) FN<32, 16>(ARGS, ST); \
    else if (tw == 16 && th == 32) FN<16, 32>(ARGS, ST); \
    else FN<8, 8>(ARGS, ST);                             \
  } while (0)

hipError_t launch_render(const sx_projected& proj, const uint32_t* vals,
                         const uint32_t* ranges, const DCam& cam,
                         const KParams& p, const uint32_t* mask,
                         float* partial, float* depth, uint32_t* last,
                         uint32_t* nblend, hipStream_t st) {
  RenderArgs a;
  a.rec = proj.rec;
  a.vals = vals;
  a.ranges = reinterpret_cast<const uint2*>(ranges);
  a.mask = mask;
  a.W = cam.W, a.H = cam.H, a.tiles_x = p.tiles_x, a.tiles_y = p.tiles_y;
  a.cx = (float)cam.cx, a.cy = (float)cam.cy;
  a.alpha_min = p.alpha_min, a.alpha_max = p.alpha_max, a.t_min = p.t_min;
  a.partial = reinterpret_cast<float4*>(partial);
  a.depth = depth, a.last = last, a.nblend = nblend;
  SX_DISPATCH_TILE(p.tile_w, p.tile_h, launch_fwd_t, a, st);
  return hipGetLastError();
}

hipError_t launch_render_backward(const sx_projected& proj,
                                  const uint32_t* vals, const uint32_t* ranges,
                                  int64_t n, const DCam& cam, const KParams& p,
                                  const uint32_t* mask, const float* partial,
                                  const uint32_t* last, const float* dpartial,
                                  const float* ddepth, float* g2d,
                                  hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(k_zero_g2d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       proj.n_tiles, n, g2d);
  RenderBwdArgs a;
  a.rec = proj.rec;
  a.vals = vals;
  a.ranges = reinterpret_cast<const uint2*>(ranges);
  a.mask = mask;
  a.W = cam.W, a.H = cam.H, a.tiles_x = p.tiles_x, a.tiles_y = p.tiles_y;
  a.cx = (float)cam.cx, a.cy = (float)cam.cy;
  a.alpha_min = p.alpha_min, a.alpha_max = p.alpha_max;
  a.partial = reinterpret_cast<const float4*>(partial);
  a.last = last;
  a.dpartial = reinterpret_cast<const float4*>(dpartial);
  a.ddepth = ddepth;
  a.g2d = g2d;
  SX_DISPATCH_TILE(p.tile_w, p.tile_h, launch_bwd_t, a, st);
  return hipGetLastError();
}

}  // namespace sx
