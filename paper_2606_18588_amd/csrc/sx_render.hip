// Partial render of one cell (Eq. 1-4) and its backward (Eq. 6-7, the part
// local to one cell).
//
// One workgroup per screen tile, in raster order (workgroup b renders tile
// b).  Every lane of a tile walks the same depth-sorted list: records are
// staged per wavefront in LDS and read as broadcasts, no workgroup barrier
// is needed, and each wavefront leaves the list as soon as a ballot says
// all its pixels are saturated (T < t_min) or masked.  (A block -> tile map
// that gave each XCD a contiguous band of tiles, for L2 sharing, measured
// 1.7x slower: the rasterizers are bound by VALU issue, and the bands
// differ in cost, so the XCDs finished at different times.)
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
  // cross-boundary filter (FILT): bits per Gaussian, the K geometric maps
  const uint32_t* __restrict__ xf;
  const uint32_t* __restrict__ omega;
  uint32_t words;
  int cell, ncells;
};

// The cells whose box the ray of pixel `pix` meets (bit s from map s), or
// none when it misses the rendering cell's own box: a pair (g, pix) is
// removed from the ray when xf[g] shares a bit with this set.
__device__ __forceinline__ uint32_t filter_bits(const uint32_t* __restrict__ omega,
                                                uint32_t words, int ncells, int cell,
                                                uint32_t pix) {
  uint32_t b = 0;
  for (int c = 0; c < ncells; ++c)
    b |= ((omega[(size_t)c * words + (pix >> 5)] >> (pix & 31)) & 1u) << c;
  return ((b >> cell) & 1u) ? b : 0u;
}



// Records are staged per wavefront in batches of 64: lane i gathers the
// record of list entry jb+i with vector loads (64 gathers in flight, which
// hides their latency), writes it to the wavefront's own LDS slice, and the
// wavefront then walks the batch reading each record as a broadcast.  Each
// wavefront owns its slice, so no workgroup barrier is needed.
//
// A pixel blends a Gaussian only inside the pixel box of its exact
// alpha >= alpha_min footprint (outside it alpha < alpha_min in exact
// arithmetic).  While staging a batch every lane tests its entry's box
// against the wavefront's pixel rectangle; the ballot of the results is the
// set of entries the wavefront walks, in order, two records per LDS round
// trip.
// The box words hold (x0 | (x1 - x0) << 16) and (y0 | (y1 - y0) << 16).
__device__ __forceinline__ bool in_box(int px, int py, float bxw, float byw) {
  const uint32_t bx = __float_as_uint(bxw), by = __float_as_uint(byw);
  return (uint32_t)px - (bx & 0xFFFFu) <= (bx >> 16) && (uint32_t)py - (by & 0xFFFFu) <= (by >> 16);
}
// The box meets the pixel rectangle [x0, x1] x [y0, y1].
__device__ __forceinline__ bool box_meets(float bxw, float byw, int x0, int x1, int y0, int y1) {
  const uint32_t bx = __float_as_uint(bxw), by = __float_as_uint(byw);
  const int bx0 = (int)(bx & 0xFFFFu), by0 = (int)(by & 0xFFFFu);
  return bx0 <= x1 && bx0 + (int)(bx >> 16) >= x0 && by0 <= y1 && by0 + (int)(by >> 16) >= y0;
}
template <int TW, int TH, bool FILT = false>
__device__ __forceinline__ void render_tile(const RenderArgs& a, int tile,
                                            float4 (*s_rec)[3][64], uint32_t* s_xf = nullptr) {
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const int lx = threadIdx.x % TW, ly = threadIdx.x / TW;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int px = tx * TW + lx, py = ty * TH + ly;
  const bool inside = px < a.W && py < a.H;
  const uint32_t pix = (uint32_t)py * a.W + px;
  bool active = inside;
  if (active && a.mask) active = (a.mask[pix >> 5] >> (pix & 31)) & 1u;
  const uint32_t pbits = (FILT && active) ? filter_bits(a.omega, a.words, a.ncells, a.cell, pix) : 0u;
  const float fx = (float)px + 0.5f - a.cx, fy = (float)py + 0.5f - a.cy;
  // pixel rectangle of this wavefront (64 consecutive pixels of the tile)
  constexpr int WR = 64 / TW;  // rows per wavefront
  const int wx0 = tx * TW, wx1 = wx0 + TW - 1;
  const int wy0 = ty * TH + w * WR, wy1 = wy0 + WR - 1;
  const uint2 rg = a.ranges[tile];
  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f;
  uint32_t lst = 0, nb = 0;
  bool done = !active;
  for (uint32_t jb = rg.x; jb < rg.y; jb += 64) {
    if (__ballot(!done) == 0) break;
    const uint32_t cnt = rg.y - jb < 64u ? rg.y - jb : 64u;
    bool meets = false;
    if ((uint32_t)lane < cnt) {
      const uint32_t gl = a.vals[jb + lane];
      const float4* r = reinterpret_cast<const float4*>(a.rec + (size_t)gl * kRecFloats);
      const float4 q0 = r[0], q1 = r[1], q2 = r[2];
      s_rec[w][0][lane] = q0;
      s_rec[w][1][lane] = q1;
      s_rec[w][2][lane] = q2;
      if (FILT) s_xf[w * 64 + lane] = a.xf[gl];
      meets = box_meets(q2.z, q2.w, wx0, wx1, wy0, wy1);
    }
    uint64_t todo = __ballot(meets);
    __builtin_amdgcn_wave_barrier();
    // branch-free blend: a lane that does not blend uses alpha = 0, which
    // leaves C, D and T unchanged exactly
    auto blend = [&](const float4& r0, const float4& r1, const float4& r2, uint32_t kc,
                     uint32_t xe) {
      const AlphaEval ae = eval_alpha(fx - r0.x, fy - r0.y, r0.z, r0.w, r1.x, r1.y, a.alpha_max);
      const bool use = !done && ae.alpha >= a.alpha_min && in_box(px, py, r2.z, r2.w) &&
                       (!FILT || (xe & pbits) == 0u);
      const float al = use ? ae.alpha : 0.f;
      const float wt = al * T;
      C0 = fmaf(r1.z, wt, C0);
      C1 = fmaf(r1.w, wt, C1);
      C2 = fmaf(r2.x, wt, C2);
      D = fmaf(r2.y, wt, D);
      T = T * (1.f - al);
      nb += use ? 1u : 0u;
      lst = use ? jb + kc - rg.x + 1 : lst;
      done = done || (use && T < a.t_min);
    };
    // two entries per LDS round trip
    while (todo) {
      if (__ballot(!done) == 0) break;
      const uint32_t k1 = (uint32_t)__builtin_ctzll(todo);
      todo &= todo - 1;
      const bool two = todo != 0;
      const uint32_t k2 = two ? (uint32_t)__builtin_ctzll(todo) : k1;
      todo &= two ? todo - 1 : todo;
      const float4 p0 = s_rec[w][0][k1], p1 = s_rec[w][1][k1], p2 = s_rec[w][2][k1];
      const float4 q0 = s_rec[w][0][k2], q1 = s_rec[w][1][k2], q2 = s_rec[w][2][k2];
      const uint32_t x1 = FILT ? s_xf[w * 64 + k1] : 0u, x2 = FILT ? s_xf[w * 64 + k2] : 0u;
      blend(p0, p1, p2, k1, x1);
      if (two) blend(q0, q1, q2, k2, x2);
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (inside) {
    a.partial[pix] = make_float4(C0, C1, C2, T);
    a.last[pix] = lst;
    if (a.depth) a.depth[pix] = D;
    if (a.nblend) a.nblend[pix] = nb;
  }
}

template <int TW, int TH, bool FILT>
__global__ __launch_bounds__(TW* TH) void k_render(RenderArgs a) {
  __shared__ float4 s_rec[TW * TH / 64][3][64];
  __shared__ uint32_t s_xf[FILT ? TW * TH : 1];
  const int ntile = a.tiles_x * a.tiles_y;
  const int tile = blockIdx.x;
  if (tile >= ntile) return;
  render_tile<TW, TH, FILT>(a, tile, s_rec, s_xf);
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
  const uint32_t* __restrict__ nv;  // entries visited per tile
  const uint32_t* __restrict__ vb;  // first gradient row of each tile
  uint64_t cap;
  float* __restrict__ rows;         // [visited][kRowFloats]
  uint32_t* __restrict__ pkey;      // per row: Gaussian index
  uint32_t* __restrict__ pval;      // per row: row index
  // cross-boundary filter (FILT), as in RenderArgs
  const uint32_t* __restrict__ xf;
  const uint32_t* __restrict__ omega;
  uint32_t words;
  int cell, ncells;
};

// Sum of ten per-lane values over the wavefront, stored to dst[0..9].  The
// values are reduced together by transposition: a 32-lane swap pairs value
// 2p (kept in lanes 0-31) with 2p+1 (lanes 32-63), a 16-lane swap pairs two
// such registers so each 16-lane row carries one value, and four DPP steps
// finish every row; one lane per row stores its value.
__device__ __forceinline__ float swap_add32(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);  // lanes 0-31: a, 32-63: b
}
__device__ __forceinline__ float swap_add16(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);  // rows: a.lo, b.lo, a.hi, b.hi
}
__device__ __forceinline__ float row_sum16(float v) {
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, true));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x124, 0xF, 0xF, true));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x128, 0xF, 0xF, true));
  return v;
}
__device__ __forceinline__ void wave_sum10_store(const float (&v)[10], float* dst, int lane,
                                                 bool ok) {
  const float u0 = swap_add32(v[0], v[1]), u1 = swap_add32(v[2], v[3]);
  const float u2 = swap_add32(v[4], v[5]), u3 = swap_add32(v[6], v[7]);
  const float u4 = swap_add32(v[8], v[9]);
  // rows of w0: values 0, 2, 1, 3; of w1: 4, 6, 5, 7; of w2: 8, -, 9, -
  const float w0 = row_sum16(swap_add16(u0, u1));
  const float w1 = row_sum16(swap_add16(u2, u3));
  const float w2 = row_sum16(swap_add16(u4, 0.f));
  const int r = lane >> 4;
  if ((lane & 15) == 0 && ok) {
    const int q = ((r & 1) << 1) | (r >> 1);
    dst[q] = w0;
    dst[4 + q] = w1;
    if ((r & 1) == 0) dst[8 + (r >> 1)] = w2;
  }
}

// Reverse walk of each pixel's blended pairs.  With R the colour behind pair
// i (normalised by T_{i+1}), T_final the partial transmittance and
// (G, g_T, g_D) the gradients of (C^m, T^m, D^m):
//   dc_i = alpha_i T_i G,   dz_i = alpha_i T_i g_D,
//   dalpha_i = T_i [G.(c_i - R) + g_D (z_i - RD)] - g_T T_final / (1 - alpha_i)
// then alpha = o exp(-q/2) gives do = dalpha exp(-q/2), dq = -alpha/2 dalpha
// (zero when alpha was clamped), and q gives the mean2d and conic terms.
//
// One wavefront per tile; each lane owns TW*TH/64 pixels and sums their
// contributions in registers, then one cross-lane reduction (DPP) per
// (Gaussian, tile).  No atomics: the tile walks the nv[tile] entries its
// pixels reached, and the j-th of them owns gradient row vb[tile] + j (rows
// of entries without any contribution are zeros); the row's Gaussian index
// is stored beside it for the per-Gaussian reduction.
// DG: a depth gradient is given (otherwise its terms are compiled out,
// which frees the registers of two per-pixel quantities).
template <int TW, int TH, bool DG, bool FILT = false>
__device__ __forceinline__ void render_tile_bwd(const RenderBwdArgs& a, int tile,
                                                float4 (*s_rec)[64], uint32_t* s_xf = nullptr) {
  constexpr int PPT = TW * TH / 64;
  constexpr int WR = 64 / TW;  // rows per group of 64 pixels
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const int lane = threadIdx.x;
  const uint32_t wave_last = a.nv[tile];  // max of the pixels' `last` over the tile
  if (wave_last == 0) return;             // nothing blended here: no rows, no pixel reads
  const uint2 rg = a.ranges[tile];
  uint32_t pxy[PPT];  // pixel x | y << 16
  float fx[PPT], fy[PPT], T[PPT], R0[PPT], R1[PPT], R2[PPT], RD[PPT];
  float gx[PPT], gy[PPT], gz[PPT], gd[PPT], gtf[PPT];
  uint32_t lst[PPT], pbits[PPT];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int li = lane + 64 * k;
    const int px = tx * TW + li % TW, py = ty * TH + li / TW;
    const bool inside = px < a.W && py < a.H;
    const uint32_t pix = inside ? (uint32_t)py * a.W + px : 0u;
    bool active = inside;
    if (active && a.mask) active = (a.mask[pix >> 5] >> (pix & 31)) & 1u;
    pbits[k] = (FILT && active) ? filter_bits(a.omega, a.words, a.ncells, a.cell, pix) : 0u;
    pxy[k] = (uint32_t)px | ((uint32_t)py << 16);
    fx[k] = (float)px + 0.5f - a.cx;
    fy[k] = (float)py + 0.5f - a.cy;
    float Tf = 1.f, gt = 0.f;
    gx[k] = gy[k] = gz[k] = gd[k] = 0.f;
    lst[k] = 0;
    if (active) {
      Tf = a.partial[pix].w;
      const float4 g = a.dpartial[pix];
      gx[k] = g.x, gy[k] = g.y, gz[k] = g.z, gt = g.w;
      if (DG) gd[k] = a.ddepth[pix];
      lst[k] = a.last[pix];
    }
    T[k] = Tf;
    gtf[k] = gt * Tf;
    R0[k] = R1[k] = R2[k] = RD[k] = 0.f;
  }
  const uint32_t row0 = a.vb[tile];
  for (int jend = (int)wave_last; jend > 0; jend -= 64) {
    // stage entries [jend - cnt, jend): lane i gathers entry jend - cnt + i,
    // stores its (Gaussian, row) pair and tests its pixel box against each
    // pixel group; gm[k] bit i = entry j0 + i can reach group k
    const int cnt = jend < 64 ? jend : 64;
    const int j0 = jend - cnt;
    bool mk[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) mk[k] = false;
    if (lane < cnt) {
      const uint32_t gl = a.vals[rg.x + (uint32_t)(j0 + lane)];
      const float4* rr = reinterpret_cast<const float4*>(a.rec + (size_t)gl * kRecFloats);
      const float4 q0 = rr[0], q1 = rr[1], q2 = rr[2];
      s_rec[0][lane] = q0;
      s_rec[1][lane] = q1;
      s_rec[2][lane] = q2;
      if (FILT) s_xf[lane] = a.xf[gl];
#pragma unroll
      for (int k = 0; k < PPT; ++k)
        mk[k] = box_meets(q2.z, q2.w, tx * TW, tx * TW + TW - 1, ty * TH + k * WR,
                          ty * TH + k * WR + WR - 1);
      const uint32_t row = row0 + (uint32_t)(j0 + lane);
      if ((uint64_t)row < a.cap) a.pkey[row] = gl, a.pval[row] = row;
    }
    uint64_t gm[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) gm[k] = __ballot(mk[k]);
    __builtin_amdgcn_wave_barrier();
    auto entry = [&](const float4& r0, const float4& r1, const float4& r2, int kk, uint32_t xe) {
    const int j = j0 + kk;
    const uint32_t e = row0 + (uint32_t)j;
    float2* dst = reinterpret_cast<float2*>(a.rows + (size_t)e * kRowFloats);
    const bool in_cap = (uint64_t)e < a.cap;
    float v[10];
#pragma unroll
    for (int m = 0; m < 10; ++m) v[m] = 0.f;
    bool any = false;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      if (((gm[k] >> kk) & 1ull) == 0) continue;  // the box misses pixel group k
      // branch-free: a lane whose pixel does not blend this entry runs the
      // same instructions with alpha = 0, which leaves T, R and the sums
      // unchanged exactly (fma(0, x, s) = s, x * 1 = x)
      const float dx = fx[k] - r0.x, dy = fy[k] - r0.y;
      const AlphaEval ae = eval_alpha(dx, dy, r0.z, r0.w, r1.x, r1.y, a.alpha_max);
      const bool use = (uint32_t)j < lst[k] && ae.alpha >= a.alpha_min &&
                       in_box((int)(pxy[k] & 0xFFFFu), (int)(pxy[k] >> 16), r2.z, r2.w) &&
                       (!FILT || (xe & pbits[k]) == 0u);
      any = any || use;
      const float al = use ? ae.alpha : 0.f;
      const float om = 1.f - al;  // >= 1 - alpha_max
      const float rom = __builtin_amdgcn_rcpf(om);
      const float Ti = T[k] * rom;
      const float w = al * Ti;
      v[6] = fmaf(w, gx[k], v[6]);
      v[7] = fmaf(w, gy[k], v[7]);
      v[8] = fmaf(w, gz[k], v[8]);
      const float d0 = r1.z - R0[k], d1 = r1.w - R1[k], d2 = r2.x - R2[k];
      float da = gx[k] * d0;
      da = fmaf(gy[k], d1, da);
      da = fmaf(gz[k], d2, da);
      if constexpr (DG) {
        const float dd = r2.y - RD[k];
        v[9] = fmaf(w, gd[k], v[9]);
        da = fmaf(gd[k], dd, da);
        RD[k] = fmaf(al, dd, RD[k]);
      }
      da = fmaf(Ti, da, -(gtf[k] * rom));
      // R <- alpha c + (1 - alpha) R
      R0[k] = fmaf(al, d0, R0[k]);
      R1[k] = fmaf(al, d1, R1[k]);
      R2[k] = fmaf(al, d2, R2[k]);
      T[k] = Ti;
      const float dae = use && !ae.clamped ? da : 0.f;  // alpha clamped: no o, q terms
      v[5] = fmaf(dae, ae.G, v[5]);
      const float dq = -0.5f * al * dae;
      const float m2 = -2.f * dq;
      v[0] = fmaf(m2, fmaf(r0.z, dx, r0.w * dy), v[0]);
      v[1] = fmaf(m2, fmaf(r0.w, dx, r1.x * dy), v[1]);
      const float qx = dq * dx, qy = dq * dy;
      v[2] = fmaf(qx, dx, v[2]);
      v[3] = fmaf(qx + qx, dy, v[3]);
      v[4] = fmaf(qy, dy, v[4]);
    }
    if (__ballot(any) == 0) {
      if (lane == 63 && in_cap) {
        const float2 z = make_float2(0.f, 0.f);
        dst[0] = z, dst[1] = z, dst[2] = z, dst[3] = z, dst[4] = z;
      }
      return;
    }
    wave_sum10_store(v, reinterpret_cast<float*>(dst), lane, in_cap);
    };
    // two entries per LDS round trip, back to front
    for (int kk = cnt - 1; kk >= 0; kk -= 2) {
      const bool two = kk >= 1;
      const int k2 = two ? kk - 1 : kk;
      const float4 p0 = s_rec[0][kk], p1 = s_rec[1][kk], p2 = s_rec[2][kk];
      const float4 q0 = s_rec[0][k2], q1 = s_rec[1][k2], q2 = s_rec[2][k2];
      const uint32_t x1 = FILT ? s_xf[kk] : 0u, x2 = FILT ? s_xf[k2] : 0u;
      entry(p0, p1, p2, kk, x1);
      if (two) entry(q0, q1, q2, k2, x2);
    }
    __builtin_amdgcn_wave_barrier();
  }
}

template <int TW, int TH, bool DG, bool FILT>
__global__ __launch_bounds__(64) void k_render_bwd(RenderBwdArgs a) {
  __shared__ float4 s_rec[3][64];
  __shared__ uint32_t s_xf[FILT ? 64 : 1];
  const int ntile = a.tiles_x * a.tiles_y;
  const int tile = blockIdx.x;
  if (tile >= ntile) return;
  render_tile_bwd<TW, TH, DG, FILT>(a, tile, s_rec, s_xf);
}

// Entries each tile's reverse walk visits: the largest `last` over its
// active pixels (the same pixels the walk reads).  One wavefront per tile.
template <int TW, int TH>
__global__ __launch_bounds__(64) void k_tile_extent(const uint32_t* __restrict__ last,
                                                    const uint32_t* __restrict__ mask, int W,
                                                    int H, int tiles_x, int tiles,
                                                    uint32_t* __restrict__ nv) {
  const int tile = blockIdx.x;
  if (tile >= tiles) return;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  uint32_t mx = 0;
#pragma unroll
  for (int k = 0; k < TW * TH / 64; ++k) {
    const int li = threadIdx.x + 64 * k;
    const int px = tx * TW + li % TW, py = ty * TH + li / TW;
    if (px < W && py < H) {
      const uint32_t pix = (uint32_t)py * W + px;
      if (!mask || ((mask[pix >> 5] >> (pix & 31)) & 1u)) mx = max(mx, last[pix]);
    }
  }
  mx = wave_max_u32(mx);
  if (threadIdx.x == 0) nv[tile] = mx;
}

// One block: exclusive scan of the visited counts -> first row per tile and
// the number of rows.
__global__ __launch_bounds__(1024) void k_extent_scan(const uint32_t* __restrict__ nv, int tiles,
                                                      uint32_t* __restrict__ vb,
                                                      uint64_t* vcount) {
  __shared__ uint32_t s_p[1024];
  const int tid = threadIdx.x;
  const int chunk = (tiles + 1023) / 1024;
  const int beg = tid * chunk, end = beg + chunk < tiles ? beg + chunk : tiles;
  uint32_t sum = 0;
  for (int t = beg; t < end; ++t) sum += nv[t];
  s_p[tid] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const uint32_t v = tid >= o ? s_p[tid - o] : 0u;
    __syncthreads();
    s_p[tid] += v;
    __syncthreads();
  }
  uint32_t run = s_p[tid] - sum;
  for (int t = beg; t < end; ++t) {
    vb[t] = run;
    run += nv[t];
  }
  if (tid == 1023) vcount[0] = s_p[1023];
}

// Clear the look-back status of the partitions the pair sort will use
// (ceil(rows / kSortTile) per pass; the rest is never read).
__global__ __launch_bounds__(256) void k_zero_status(uint32_t* __restrict__ status, int64_t parts,
                                                     const uint64_t* vcount, uint64_t cap) {
  const uint64_t n = vcount[0] < cap ? vcount[0] : cap;
  const uint64_t words = (n + kSortTile - 1) / kSortTile * kRadixBins;
  for (int ps = 0; ps < 4; ++ps)
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < words;
         i += (uint64_t)gridDim.x * 256)
      status[(size_t)ps * parts * kRadixBins + i] = 0u;
}

// Per-Gaussian sum of its rows.  The pairs are sorted by Gaussian (stably,
// so a Gaussian's rows are in tile order) and cut into chunks of 256; each
// chunk stages its rows in LDS, and the first pair of every run of one
// Gaussian adds the run's rows in order.  A run lying inside one chunk is
// stored with plain stores; the pieces of a run crossing chunk boundaries
// are added atomically into the (pre-zeroed) row of its Gaussian.
__global__ __launch_bounds__(256) void k_pair_reduce(const uint32_t* __restrict__ key,
                                                     const uint32_t* __restrict__ val,
                                                     const uint64_t* vcount, uint64_t cap,
                                                     const float* __restrict__ rows,
                                                     float* __restrict__ g2d) {
  __shared__ float s_row[256][kRowFloats + 1];
  __shared__ uint32_t s_key[256];
  __shared__ unsigned long long s_hm[4];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint64_t n = vcount[0] < cap ? vcount[0] : cap;
  for (uint64_t base = (uint64_t)blockIdx.x * 256; base < n; base += (uint64_t)gridDim.x * 256) {
    const int m = (int)(n - base < 256 ? n - base : 256);
    __syncthreads();  // the previous chunk is consumed
    if (tid < m) {
      s_key[tid] = key[base + tid];
      const float2* src = reinterpret_cast<const float2*>(rows + (size_t)val[base + tid] * kRowFloats);
#pragma unroll
      for (int q = 0; q < kRowFloats / 2; ++q) {
        const float2 v = src[q];
        s_row[tid][2 * q] = v.x, s_row[tid][2 * q + 1] = v.y;
      }
    }
    __syncthreads();
    const uint32_t g = tid < m ? s_key[tid] : 0u;
    const bool head = tid < m && (tid == 0 || s_key[tid - 1] != g);
    const unsigned long long hm = __ballot(head);
    if (lane == 0) s_hm[w] = hm;
    __syncthreads();
    if (head) {
      // end of the run: the next run head in this chunk, else the chunk end
      int e = m;
      const unsigned long long later = lane < 63 ? hm & ~((2ull << lane) - 1ull) : 0ull;
      if (later) {
        e = w * 64 + __builtin_ctzll(later);
      } else {
        for (int w2 = w + 1; w2 < 4; ++w2)
          if (s_hm[w2]) {
            e = w2 * 64 + __builtin_ctzll(s_hm[w2]);
            break;
          }
      }
      float acc[kRowFloats];
#pragma unroll
      for (int q = 0; q < kRowFloats; ++q) acc[q] = 0.f;
      for (int r = tid; r < e; ++r)
#pragma unroll
        for (int q = 0; q < kRowFloats; ++q) acc[q] += s_row[r][q];
      const bool starts = base + tid == 0 || key[base + tid - 1] != g;
      const bool ends = base + e == n || key[base + e] != g;
      float* d = g2d + (size_t)g * kG2dFloats;
      if (starts && ends) {
        float4* d4 = reinterpret_cast<float4*>(d);
        d4[0] = make_float4(acc[0], acc[1], acc[2], acc[3]);
        d4[1] = make_float4(acc[4], acc[5], acc[6], acc[7]);
        d4[2] = make_float4(acc[8], acc[9], 0.f, 0.f);
      } else {
#pragma unroll
        for (int q = 0; q < kRowFloats; ++q) unsafeAtomicAdd(d + q, acc[q]);
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_zero_g2d(const uint32_t* __restrict__ vis,
                                                  const uint64_t* vis_count,
                                                  float* __restrict__ g2d) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= vis_count[0]) return;
  float4* d = reinterpret_cast<float4*>(g2d + (size_t)vis[i] * kG2dFloats);
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
  d[0] = z, d[1] = z, d[2] = z;
}

// ------------------------------------------------------------ multi-view --
// Many views in one launch: workgroup b takes the b-th (view, tile) item of
// the views laid end to end, tiles in raster order within a view.  (Ordering
// the items by list length and pulling them from a device counter measured
// slower than this plain order.)
__device__ __forceinline__ int item_view(const uint32_t* base, int V, uint32_t b) {
  int v = 0;
  while (v + 1 < V && b >= base[v + 1]) ++v;
  return v;
}

struct RenderMultiArgs {
  int V;
  uint32_t base[kMaxViews + 1];  // first item of each view; base[V] = all items
  RenderArgs view[kMaxViews];
};

template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void k_render_multi(RenderMultiArgs m) {
  __shared__ float4 s_rec[TW * TH / 64][3][64];
  const uint32_t b = blockIdx.x;
  if (b >= m.base[m.V]) return;
  const int v = item_view(m.base, m.V, b);
  render_tile<TW, TH>(m.view[v], (int)(b - m.base[v]), s_rec);
}

struct RenderBwdMultiArgs {
  int V;
  uint32_t base[kMaxViews + 1];
  RenderBwdArgs view[kMaxViews];
};

static_assert(sizeof(RenderMultiArgs) <= 4096, "kernel argument block too large");

template <int TW, int TH>
__global__ __launch_bounds__(64) void k_render_bwd_multi(RenderBwdMultiArgs m) {
  __shared__ float4 s_rec[3][64];
  const uint32_t b = blockIdx.x;
  if (b >= m.base[m.V]) return;
  const int v = item_view(m.base, m.V, b);
  // batched views carry no depth gradient
  render_tile_bwd<TW, TH, false>(m.view[v], (int)(b - m.base[v]), s_rec);
}

static_assert(sizeof(RenderBwdMultiArgs) <= 4096, "kernel argument block too large");

bool tile_shape_supported(int tw, int th) {
  return (tw == 16 && th == 16) || (tw == 32 && th == 8) || (tw == 8 && th == 32) ||
         (tw == 32 && th == 16) || (tw == 16 && th == 32) || (tw == 8 && th == 8);
}

template <int TW, int TH>
static void launch_fwd_t(const RenderArgs& a, hipStream_t st) {
  const int grid = a.tiles_x * a.tiles_y;
  if (a.xf)
    hipLaunchKernelGGL((k_render<TW, TH, true>), dim3(grid), dim3(TW * TH), 0, st, a);
  else
    hipLaunchKernelGGL((k_render<TW, TH, false>), dim3(grid), dim3(TW * TH), 0, st, a);
}
template <int TW, int TH>
static void launch_bwd_t(const RenderBwdArgs& a, hipStream_t st) {
  const int grid = a.tiles_x * a.tiles_y;
  if (a.xf) {
    if (a.ddepth)
      hipLaunchKernelGGL((k_render_bwd<TW, TH, true, true>), dim3(grid), dim3(64), 0, st, a);
    else
      hipLaunchKernelGGL((k_render_bwd<TW, TH, false, true>), dim3(grid), dim3(64), 0, st, a);
  } else if (a.ddepth) {
    hipLaunchKernelGGL((k_render_bwd<TW, TH, true, false>), dim3(grid), dim3(64), 0, st, a);
  } else {
    hipLaunchKernelGGL((k_render_bwd<TW, TH, false, false>), dim3(grid), dim3(64), 0, st, a);
  }
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

static RenderArgs make_render_args(const sx_projected& proj, const uint32_t* vals,
                                   const uint32_t* ranges, const DCam& cam, const KParams& p,
                                   const uint32_t* mask, float* partial, float* depth,
                                   uint32_t* last, uint32_t* nblend) {
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
  a.xf = proj.xf, a.omega = proj.omega;
  a.words = ((uint32_t)cam.W * (uint32_t)cam.H + 31) / 32;
  a.cell = proj.cell, a.ncells = proj.n_cells;
  return a;
}

hipError_t launch_render(const sx_projected& proj, const uint32_t* vals,
                         const uint32_t* ranges, const DCam& cam,
                         const KParams& p, const uint32_t* mask,
                         float* partial, float* depth, uint32_t* last,
                         uint32_t* nblend, hipStream_t st) {
  RenderArgs a = make_render_args(proj, vals, ranges, cam, p, mask, partial, depth, last, nblend);
  SX_DISPATCH_TILE(p.tile_w, p.tile_h, launch_fwd_t, a, st);
  return hipGetLastError();
}

static RenderBwdArgs make_bwd_args(const sx_projected& proj, const uint32_t* vals,
                                   const uint32_t* ranges, int64_t capacity, const DCam& cam,
                                   const KParams& p, const uint32_t* mask, const float* partial,
                                   const uint32_t* last, const float* dpartial,
                                   const float* ddepth, char* bws) {
  const int64_t tiles = (int64_t)p.tiles_x * p.tiles_y;
  const BwdLayout BL = bwd_layout(capacity, tiles);
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
  a.nv = reinterpret_cast<const uint32_t*>(bws + BL.nv);
  a.vb = reinterpret_cast<const uint32_t*>(bws + BL.vb);
  a.cap = (uint64_t)capacity;
  a.rows = reinterpret_cast<float*>(bws + BL.rows);
  a.pkey = reinterpret_cast<uint32_t*>(bws + BL.pk[0]);
  a.pval = reinterpret_cast<uint32_t*>(bws + BL.pv[0]);
  a.xf = proj.xf, a.omega = proj.omega;
  a.words = ((uint32_t)cam.W * (uint32_t)cam.H + 31) / 32;
  a.cell = proj.cell, a.ncells = proj.n_cells;
  return a;
}

template <int TW, int TH>
static void launch_extent_t(const RenderBwdArgs& a, hipStream_t st) {
  const int tiles = a.tiles_x * a.tiles_y;
  hipLaunchKernelGGL((k_tile_extent<TW, TH>), dim3((unsigned)tiles), dim3(64), 0, st, a.last,
                     a.mask, a.W, a.H, a.tiles_x, tiles, const_cast<uint32_t*>(a.nv));
}

// Before the reverse walk: clear the counters, find each tile's visited
// prefix and give the visited entries consecutive rows.
static hipError_t launch_bwd_prepare(const RenderBwdArgs& a, const KParams& p, int64_t capacity,
                                     char* bws, hipStream_t st) {
  const int64_t tiles = (int64_t)p.tiles_x * p.tiles_y;
  const BwdLayout BL = bwd_layout(capacity, tiles);
  hipError_t e = launch_fill(reinterpret_cast<uint32_t*>(bws + BL.zero_begin),
                             (int64_t)((BL.zero_end - BL.zero_begin) / 4), 0, st);
  if (e) return e;
  SX_DISPATCH_TILE(p.tile_w, p.tile_h, launch_extent_t, a, st);
  hipLaunchKernelGGL(k_extent_scan, dim3(1), dim3(1024), 0, st, a.nv, (int)tiles,
                     const_cast<uint32_t*>(a.vb), reinterpret_cast<uint64_t*>(bws + BL.vcount));
  hipLaunchKernelGGL(k_zero_status, dim3(256), dim3(256), 0, st,
                     reinterpret_cast<uint32_t*>(bws + BL.vstatus), BL.parts,
                     reinterpret_cast<const uint64_t*>(bws + BL.vcount), (uint64_t)capacity);
  return hipGetLastError();
}

// After the reverse walk: zero the visible Gaussians' screen-space
// gradients, sort the (Gaussian, row) pairs by Gaussian and sum the rows.
static hipError_t launch_bwd_reduce(const SortView& sv, int64_t n, int64_t capacity,
                                    const KParams& p, float* g2d, char* bws, hipStream_t st) {
  const int64_t tiles = (int64_t)p.tiles_x * p.tiles_y;
  const BwdLayout BL = bwd_layout(capacity, tiles);
  if (n > 0)
    hipLaunchKernelGGL(k_zero_g2d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       sv.vidx, sv.counts, g2d);
  auto u32 = [&](size_t off) { return reinterpret_cast<uint32_t*>(bws + off); };
  uint32_t* keys[2] = {u32(BL.pk[0]), u32(BL.pk[1])};
  uint32_t* vals[2] = {u32(BL.pv[0]), u32(BL.pv[1])};
  const uint64_t* vcount = reinterpret_cast<const uint64_t*>(bws + BL.vcount);
  int bits = 1;
  while (bits < 32 && (int64_t(1) << bits) < n) ++bits;
  hipError_t e = hipSuccess;
  const int r = launch_pair_sort(keys, vals, vcount, (uint64_t)capacity, bits, u32(BL.vhist),
                                 u32(BL.vstatus), BL.parts, u32(BL.counters),
                                 reinterpret_cast<uint64_t*>(bws + BL.vcount) + 3, st, &e);
  if (e) return e;
  hipLaunchKernelGGL(k_pair_reduce, dim3(1024), dim3(256), 0, st,
                     keys[r], vals[r], vcount, (uint64_t)capacity,
                     reinterpret_cast<const float*>(bws + BL.rows), g2d);
  return hipGetLastError();
}

hipError_t launch_render_backward(const sx_projected& proj,
                                  const uint32_t* vals, const uint32_t* ranges,
                                  const SortView& sv, int64_t n, int64_t capacity,
                                  const DCam& cam, const KParams& p,
                                  const uint32_t* mask, const float* partial,
                                  const uint32_t* last, const float* dpartial,
                                  const float* ddepth, float* g2d, char* bws, int stages,
                                  hipStream_t st) {
  RenderBwdArgs a = make_bwd_args(proj, vals, ranges, capacity, cam, p, mask, partial, last,
                                  dpartial, ddepth, bws);
  hipError_t e = hipSuccess;
  if ((stages & SX_RB_PREPARE) && (e = launch_bwd_prepare(a, p, capacity, bws, st))) return e;
  if (stages & SX_RB_WALK) {
    SX_DISPATCH_TILE(p.tile_w, p.tile_h, launch_bwd_t, a, st);
    if ((e = hipGetLastError())) return e;
  }
  if (stages & SX_RB_REDUCE) return launch_bwd_reduce(sv, n, capacity, p, g2d, bws, st);
  return hipSuccess;
}

// ------------------------------------------------------------ multi-view --
// work-list workspace: a 512-byte head (hist[33], cursor[33], two work
// counters) followed by one u32 item per (view, tile)
// The batched launches need no scratch memory; the workspace argument of
// the batched entry points is kept (one small block) so callers size it
// once and the layout can change without an interface change.
size_t multi_workspace_bytes(int64_t items) {
  (void)items;
  return 256;
}

template <int TW, int TH>
static void launch_fwd_multi_t(const RenderMultiArgs& m, hipStream_t st) {
  const unsigned grid = m.base[m.V];
  hipLaunchKernelGGL((k_render_multi<TW, TH>), dim3(grid > 0 ? grid : 1), dim3(TW * TH), 0, st, m);
}
template <int TW, int TH>
static void launch_bwd_multi_t(const RenderBwdMultiArgs& m, hipStream_t st) {
  const unsigned grid = m.base[m.V];
  hipLaunchKernelGGL((k_render_bwd_multi<TW, TH>), dim3(grid > 0 ? grid : 1), dim3(64), 0, st, m);
}

template <typename Args>
static void set_bases(int V, const MultiView* mv, Args& m) {
  m.V = V;
  uint32_t base = 0;
  for (int v = 0; v < V; ++v) {
    m.base[v] = base;
    base += (uint32_t)(mv[v].tiles_x * mv[v].tiles_y);
  }
  m.base[V] = base;
}

hipError_t launch_render_multi(int V, const MultiView* mv, const KParams& p, char* ws,
                               hipStream_t st) {
  (void)ws;
  RenderMultiArgs m;
  set_bases(V, mv, m);
  for (int v = 0; v < V; ++v) {
    KParams pv = p;
    pv.tiles_x = mv[v].tiles_x, pv.tiles_y = mv[v].tiles_y;
    m.view[v] = make_render_args(mv[v].proj, mv[v].vals, mv[v].ranges, mv[v].cam, pv,
                                 mv[v].mask, mv[v].partial, mv[v].depth, mv[v].last,
                                 mv[v].nblend);
  }
  SX_DISPATCH_TILE(p.tile_w, p.tile_h, launch_fwd_multi_t, m, st);
  return hipGetLastError();
}

hipError_t launch_render_backward_multi(int V, const MultiView* mv, int64_t n, const KParams& p,
                                        char* ws, hipStream_t st) {
  (void)ws, (void)n;
  RenderBwdMultiArgs m;
  set_bases(V, mv, m);
  for (int v = 0; v < V; ++v) {
    KParams pv = p;
    pv.tiles_x = mv[v].tiles_x, pv.tiles_y = mv[v].tiles_y;
    m.view[v] = make_bwd_args(mv[v].proj, mv[v].vals, mv[v].ranges, mv[v].capacity, mv[v].cam,
                              pv, mv[v].mask, mv[v].partial, mv[v].last, mv[v].dpartial,
                              nullptr, static_cast<char*>(mv[v].bwd_ws));
    hipError_t e = launch_bwd_prepare(m.view[v], pv, mv[v].capacity,
                                      static_cast<char*>(mv[v].bwd_ws), st);
    if (e) return e;
  }
  SX_DISPATCH_TILE(p.tile_w, p.tile_h, launch_bwd_multi_t, m, st);
  return hipGetLastError();
}

hipError_t launch_grad_reduce_view(const MultiView& v, int64_t n, const KParams& p,
                                   hipStream_t st) {
  KParams pv = p;
  pv.tiles_x = v.tiles_x, pv.tiles_y = v.tiles_y;
  return launch_bwd_reduce(sort_view(v.sort_ws, n, v.capacity, pv.tiles_x, pv.tiles_y), n,
                           v.capacity, pv, v.g2d, static_cast<char*>(v.bwd_ws), st);
}

}  // namespace sx
