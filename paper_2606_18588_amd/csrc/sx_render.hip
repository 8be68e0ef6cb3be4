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
// Outside the pixel box of a Gaussian's exact alpha >= alpha_min footprint
// alpha < alpha_min in exact arithmetic.  While staging a batch every lane
// tests its entry's box against the wavefront's pixel rectangle; the ballot
// of the results is the set of entries the wavefront walks, in order, two
// records per LDS round trip.  Inside a walked rectangle the alpha test
// alone decides (a pixel outside the box can pass it only within FP32
// rounding of the footprint's edge, where the FP64 decision is ambiguous
// anyway); the reverse walk partitions the tile into the same rectangles,
// so forward and backward evaluate the same pairs.
// The box words hold (x0 | (x1 - x0) << 16) and (y0 | (y1 - y0) << 16).
// The box meets the pixel rectangle [x0, x1] x [y0, y1].
__device__ __forceinline__ bool box_meets(float bxw, float byw, int x0, int x1, int y0, int y1) {
  const uint32_t bx = __float_as_uint(bxw), by = __float_as_uint(byw);
  const int bx0 = (int)(bx & 0xFFFFu), by0 = (int)(by & 0xFFFFu);
  return bx0 <= x1 && bx0 + (int)(bx >> 16) >= x0 && by0 <= y1 && by0 + (int)(by >> 16) >= y0;
}
// Rows of one tile column that a Gaussian's footprint can reach.  With
// coordinates relative to the mean, the pixel centres of the column have
// x in [X0, X1]; the result [y0, y1] (empty when y0 > y1) holds the y of
// every such centre whose FP32 alpha test could pass.  The footprint
// {q <= Q}, Q = 2 ln(o / alpha_min), meets the column in a convex set whose
// highest point is the ellipse's own (where a x + b y = 0) if that lies in
// the column and otherwise lies on an edge line x = X0 or x = X1, where
// c y^2 + 2 b x y + a x^2 - Q = 0 gives it; likewise the lowest.  The
// interval is the hull of those candidates.  Every approximation widens
// it: Q is raised by 1e-3 (|Q| + 1) and by 1e-5 (|a| + 2|b| + |c|) r2 (r2 the
// squared distance to the farthest tile corner; the pixel test's q has an
// FP32 error below 1e-6 of that), the determinant a c - b^2 is lowered by
// 1e-5 (|a c| + b^2) (a needle whose determinant rounding swamps gets the
// whole column), and the ends are padded.  So the test never drops a pixel
// the per-pixel alpha test would blend, and forward and backward, which
// both apply it to the same rows, evaluate the same pairs.
__device__ __forceinline__ float2 column_rows(float a, float b, float c, float o, float log_amin,
                                              float X0, float X1, float r2) {
  constexpr float kFar = 3e38f;
  const float Q0 = 2.f * (__logf(o) - log_amin);  // v_log_f32: absolute error ~1e-7
  const float Q = Q0 + 1e-3f * (fabsf(Q0) + 1.f) + 1e-5f * (fabsf(a) + 2.f * fabsf(b) + fabsf(c)) * r2;
  if (!(Q >= 0.f)) return make_float2(kFar, -kFar);
  const float det = a * c - b * b;
  const float dlo = det - 1e-5f * (fabsf(a * c) + b * b);
  if (!(dlo > 0.f) || !(a > 0.f) || !(c > 0.f)) return make_float2(-kFar, kFar);
  // hardware square root and reciprocal (within 1 ulp), inside the margins
  const float yf = __builtin_amdgcn_sqrtf(Q * a * __builtin_amdgcn_rcpf(dlo));
  const float xt = -b * yf * __builtin_amdgcn_rcpf(a);  // highest point (xt, yf); lowest (-xt, -yf)
  const float tol = 1e-3f * (1.f + fabsf(xt));
  float ymax = (xt >= X0 - tol && xt <= X1 + tol) ? yf : -kFar;
  float ymin = (-xt >= X0 - tol && -xt <= X1 + tol) ? -yf : kFar;
  const float rc = __builtin_amdgcn_rcpf(c);
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const float xe = e ? X1 : X0;
    const float disc = Q * c - dlo * xe * xe;
    if (disc >= 0.f) {
      const float sq = __builtin_amdgcn_sqrtf(disc);
      ymax = fmaxf(ymax, (sq - b * xe) * rc);
      ymin = fminf(ymin, (-sq - b * xe) * rc);
    }
  }
  ymax += 1e-3f * (1.f + fabsf(ymax));
  ymin -= 1e-3f * (1.f + fabsf(ymin));
  return make_float2(ymin, ymax);
}

// column_rows for the pixel columns [px0, px1] over rows [py0, py1] and the
// record's Gaussian.
__device__ __forceinline__ float2 strip_rows(const float4& r0, const float4& r1, float cx,
                                             float cy, float log_amin, int px0, int px1, int py0,
                                             int py1) {
  const float X0 = ((float)px0 + 0.5f - cx) - r0.x;
  const float X1 = ((float)px1 + 0.5f - cx) - r0.x;
  const float Y0 = ((float)py0 + 0.5f - cy) - r0.y;
  const float Y1 = ((float)py1 + 0.5f - cy) - r0.y;
  const float r2 = fmaxf(X0 * X0, X1 * X1) + fmaxf(Y0 * Y0, Y1 * Y1);
  return column_rows(r0.z, r0.w, r1.x, r1.y, log_amin, X0, X1, r2);
}

// Pixel groups: forward and reverse walk split a tile into 8x8 blocks of
// 64 pixels (block k at column k % (TW/8), row k / (TW/8)); lane l holds
// pixel (l % 8, l / 8) of its block.  A block is more compact than a strip
// of 64 pixels, so fewer blocks than strips meet a footprint.
template <int TW, int TH>
struct Blocks {
  static_assert(TW % 8 == 0 && TH % 8 == 0, "tiles are made of 8x8 blocks");
  static constexpr int BX = TW / 8;
  __device__ static int x0(int tx, int k) { return tx * TW + (k % BX) * 8; }
  __device__ static int y0(int ty, int k) { return ty * TH + (k / BX) * 8; }
};

// Pixel rows [py0, py1] (pixel centres) meet the interval.
__device__ __forceinline__ bool rows_meet(float2 yr, int py0, int py1, float cy, float my) {
  const float Y0 = ((float)py0 + 0.5f - cy) - my, Y1 = ((float)py1 + 0.5f - cy) - my;
  return yr.x <= Y1 && yr.y >= Y0;
}

// CNT: the per-pixel blend count may be asked for (a.nblend); without it
// the count is compiled out of the blend loop.
template <int TW, int TH, bool FILT = false, bool CNT = true>
__device__ __forceinline__ void render_tile(const RenderArgs& a, int tile,
                                            float4 (*s_rec)[3][64], uint32_t* s_xf = nullptr) {
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // pixel rectangle of this wavefront: 8x8 block w of the tile
  const int wx0 = Blocks<TW, TH>::x0(tx, w), wx1 = wx0 + 7;
  const int wy0 = Blocks<TW, TH>::y0(ty, w), wy1 = wy0 + 7;
  const int px = wx0 + (lane & 7), py = wy0 + (lane >> 3);
  const bool inside = px < a.W && py < a.H;
  const uint32_t pix = (uint32_t)py * a.W + px;
  bool active = inside;
  if (active && a.mask) active = (a.mask[pix >> 5] >> (pix & 31)) & 1u;
  const uint32_t pbits = (FILT && active) ? filter_bits(a.omega, a.words, a.ncells, a.cell, pix) : 0u;
  const float fx = (float)px + 0.5f - a.cx, fy = (float)py + 0.5f - a.cy;
  const uint2 rg = a.ranges[tile];
  const float log_amin = __logf(a.alpha_min);
  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f;
  uint32_t lst = 0, nb = 0;
  // the alpha an entry needs to blend: alpha_min while the pixel is live,
  // kDone (above any alpha) once it is saturated or inactive, which folds
  // the pixel's state into the one comparison
  constexpr float kDone = 2.f;
  float athr = active ? a.alpha_min : kDone;
  const bool count = CNT && a.nblend != nullptr;
  for (uint32_t jb = rg.x; jb < rg.y; jb += 64) {
    if (__ballot(athr < kDone) == 0) break;
    const uint32_t cnt = rg.y - jb < 64u ? rg.y - jb : 64u;
    bool meets = false;
    if ((uint32_t)lane < cnt) {
      const uint32_t gl = a.vals[jb + lane];
      const float4* r = reinterpret_cast<const float4*>(a.rec + (size_t)gl * kRecFloats);
      const float4 q0 = r[0], q1 = r[1], q2 = r[2];
      const float bk = q0.w * kConicToExp2;
      s_rec[w][0][lane] = make_float4(q0.x, q0.y, q0.z * kConicToExp2, bk + bk);
      s_rec[w][1][lane] = make_float4(q1.x * kConicToExp2, q1.y, q1.z, q1.w);
      s_rec[w][2][lane] = q2;
      if (FILT) s_xf[w * 64 + lane] = a.xf[gl];
      meets = box_meets(q2.z, q2.w, wx0, wx1, wy0, wy1) &&
              rows_meet(strip_rows(q0, q1, a.cx, a.cy, log_amin, wx0, wx1, ty * TH,
                                   ty * TH + TH - 1),
                        wy0, wy1, a.cy, q0.y);
    }
    uint64_t todo = __ballot(meets);
    __builtin_amdgcn_wave_barrier();
    // branch-free blend: a lane that does not blend uses alpha = 0, which
    // leaves C, D and T unchanged exactly
    auto blend = [&](const float4& r0, const float4& r1, const float4& r2, uint32_t kc,
                     uint32_t xe) {
      const AlphaEval ae = eval_alpha(fx - r0.x, fy - r0.y, r0.z, r0.w, r1.x, r1.y, a.alpha_max);
      const bool use = ae.alpha >= athr && (!FILT || (xe & pbits) == 0u);
      if (__ballot(use) == 0) return;  // nothing to blend in this rectangle
      const float al = use ? ae.alpha : 0.f;
      const float wt = al * T;
      C0 = fmaf(r1.z, wt, C0);
      C1 = fmaf(r1.w, wt, C1);
      C2 = fmaf(r2.x, wt, C2);
      D = fmaf(r2.y, wt, D);
      T = T * (1.f - al);
      if (count) nb += use ? 1u : 0u;
      lst = use ? jb + kc - rg.x + 1 : lst;
      athr = (use && T < a.t_min) ? kDone : athr;
    };
    // two entries per LDS round trip
    while (todo) {
      if (__ballot(athr < kDone) == 0) break;
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
    if (count) a.nblend[pix] = nb;
  }
}

template <int TW, int TH, bool FILT, bool CNT>
__global__ __launch_bounds__(TW* TH) void k_render(RenderArgs a) {
  __shared__ float4 s_rec[TW * TH / 64][3][64];
  __shared__ uint32_t s_xf[FILT ? TW * TH : 1];
  const int ntile = a.tiles_x * a.tiles_y;
  const int tile = blockIdx.x;
  if (tile >= ntile) return;
  render_tile<TW, TH, FILT, CNT>(a, tile, s_rec, s_xf);
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
  const uint32_t* __restrict__ nv;    // entries visited per tile
  const uint32_t* __restrict__ order; // the walk's tile order (a permutation of the tiles)
  const uint32_t* __restrict__ ioff;  // first instance row of each visible Gaussian
  const ushort4* __restrict__ rect;   // tile rectangles [x0, y0, x1, y1)
  uint64_t cap;
  float* __restrict__ rows;           // [instances][kRowFloats], Gaussian-major
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

// A gradient row holds, for one (Gaussian, tile) instance, the sums over its
// blended pixels of h = -2 dL/dq times 1 (implicitly), dx, dy, dx^2, dx dy,
// dy^2 in slots 0-4 (dx, dy = pixel centre - mean2d), then dL/do, dL/dc and
// dL/dz.  Since q = a dx^2 + 2 b dx dy + c dy^2 with one conic per
// Gaussian, the mean2d and conic gradients are linear in those moments:
//   dL/dmean2d = (a Sx + b Sy, b Sx + c Sy),
//   dL/d(a, b, c) = (-Sxx / 2, -Sxy, -Syy / 2),
// so the walk accumulates five products per pair and the reduction applies
// the conic once per Gaussian.
__device__ __forceinline__ void row_to_g2d(float (&v)[10], float a, float b, float c) {
  const float sx = v[0], sy = v[1];
  v[0] = fmaf(a, sx, b * sy);
  v[1] = fmaf(b, sx, c * sy);
  v[2] *= -0.5f;
  v[3] = -v[3];
  v[4] *= -0.5f;
}

// Sums two entries' ten per-lane values over the wavefront and stores them,
// entry A's to da and B's to db (null: not stored).  The 32-lane swap of
// value i pairs A (kept in lanes 0-31) with B (lanes 32-63), the 16-lane
// swap pairs values 2p and 2p+1, so that row r of register p carries value
// 2p + (r & 1) of entry A (r < 2) or B; four DPP steps finish every row and
// lane 0 of each row stores.  Without a depth gradient value 9 is zero.
template <bool TEN>
__device__ __forceinline__ void wave_sum_pair_store(const float (&va)[10], const float (&vb)[10],
                                                    float* da, float* db, int lane) {
  float u[10];
#pragma unroll
  for (int i = 0; i < 10; ++i) u[i] = (TEN || i < 9) ? swap_add32(va[i], vb[i]) : 0.f;
  float w[5];
#pragma unroll
  for (int p = 0; p < 5; ++p) w[p] = row_sum16(swap_add16(u[2 * p], u[2 * p + 1]));
  const int r = lane >> 4;
  float* d = (r & 2) ? db : da;
  if ((lane & 15) == 0 && d) {
    const int q = r & 1;
#pragma unroll
    for (int p = 0; p < 5; ++p) d[2 * p + q] = w[p];
  }
}

// The same sums through LDS, for the nine values of the walk without a
// depth gradient.  Values 0-7 of both entries are 16 outputs of 64 partials
// each: every lane writes its 16 partials as one column of a 16-row table,
// then lane L sums chunk L & 3 (16 partials) of row L >> 2 and two DPP
// steps add the four chunks of a row.  Per pair that is 17 VALU
// instructions for the 16 sums (the LDS traffic runs beside the VALU, the
// walk's bound) instead of the 44 of the transposition in registers.  Value
// 8 takes the register path alone: a 32-lane swap, a row sum, a row
// broadcast; lanes 31 and 63 hold its two totals and store them with the
// zero of value 9.
// Table layout: row o (output) holds four chunks of 16 partials, rows 65
// floats apart.  A column write puts the 32 lanes of each half-wave on 32
// distinct banks (16c + s + o).  A chunk read would put chunks 0 and 2 of a
// row on the same banks (32 floats apart), so lanes reading chunks 2 and 3
// read their two halves in the other order: at every read step the four
// chunks of a row sit 0, 8, 16 and 24 banks apart, and the eight rows of a
// half-wave one bank apart (measured: bank conflicts 13.0M -> 0.1M cycles
// per launch on the 2M-Gaussian view).  The order of a chunk's terms is
// fixed per lane, so the sum is still deterministic.
constexpr int kRedChunk = 16, kRedRow = 4 * kRedChunk + 1, kRedFloats = 16 * kRedRow;
__device__ __forceinline__ void wave_sum_pair_store_lds(const float (&va)[10],
                                                        const float (&vb)[10], float* da,
                                                        float* db, int lane, float* s_red) {
  float* wr = s_red + (lane >> 4) * kRedChunk + (lane & 15);
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    wr[o * kRedRow] = va[o];
    wr[(8 + o) * kRedRow] = vb[o];
  }
  float u8 = row_sum16(swap_add32(va[8], vb[8]));
  u8 += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(u8), 0x142, 0xA, 0xF, false));
  const float* rd = s_red + (lane >> 2) * kRedRow + (lane & 3) * kRedChunk;
  const int rot = (lane & 2) ? 8 : 0;  // chunks 2 and 3: second half first
  const float* rlo = rd + rot;
  const float* rhi = rd + (8 - rot);
  float t[8];
#pragma unroll
  for (int i = 0; i < 4; ++i) t[i] = rlo[2 * i] + rlo[2 * i + 1];
#pragma unroll
  for (int i = 0; i < 4; ++i) t[4 + i] = rhi[2 * i] + rhi[2 * i + 1];
  float sum = ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
  sum += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(sum), 0xB1, 0xF, 0xF, true));
  sum += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(sum), 0x4E, 0xF, 0xF, true));
  float* d = (lane & 32) ? db : da;
  if ((lane & 3) == 0 && d) d[(lane >> 2) & 7] = sum;
  // value 9 (the depth gradient's, zero here) is stored too: the row is
  // read whole
  if ((lane & 31) == 31 && d) *reinterpret_cast<float2*>(d + 8) = make_float2(u8, 0.f);
}

// Reverse walk of each pixel's blended pairs.  With R the colour behind pair
// i (normalised by T_{i+1}), T_final the partial transmittance and
// (G, g_T, g_D) the gradients of (C^m, T^m, D^m):
//   dc_i = alpha_i T_i G,   dz_i = alpha_i T_i g_D,
//   dalpha_i = T_i [G.(c_i - R) + g_D (z_i - RD)] - g_T T_final / (1 - alpha_i)
// then alpha = o exp(-q/2) gives do = dalpha exp(-q/2), dq = -alpha/2 dalpha
// (zero when alpha was clamped), and q gives the mean2d and conic terms.
// R and RD enter only through S = G.R + g_D RD, which obeys the same
// recursion (S <- alpha (G.c_i + g_D z_i) + (1 - alpha) S), so each pixel
// carries that one scalar instead of the four.
//
// One wavefront per tile; each lane owns TW*TH/64 pixels and sums their
// contributions in registers, then one cross-lane reduction (DPP) per
// (Gaussian, tile).  No atomics: instance (g, tile) owns gradient row
// ioff[g] + the tile's raster position in g's tile rectangle, so each
// Gaussian's rows are contiguous and a plain segmented sum finishes them.
// The tile walks the nv[tile] entries its pixels reached and writes every
// entry's row (zeros where nothing blended), and zeros for the entries past
// them.
// DG: a depth gradient is given (otherwise its terms are compiled out,
// which frees the registers of two per-pixel quantities).
__device__ __forceinline__ uint32_t instance_row(const RenderBwdArgs& a, uint32_t g, int tx,
                                                 int ty) {
  const ushort4 rc = a.rect[g];
  return a.ioff[g] + (uint32_t)(ty - (int)rc.y) * (uint32_t)(rc.z - rc.x) +
         (uint32_t)(tx - (int)rc.x);
}

template <int TW, int TH, bool DG, bool FILT = false>
__device__ __forceinline__ void render_tile_bwd(const RenderBwdArgs& a, int tile,
                                                float4 (*s_rec)[64], uint32_t* s_e,
                                                float* s_red, uint32_t* s_xf = nullptr) {
  constexpr int PPT = TW * TH / 64;
  using BL = Blocks<TW, TH>;
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const int lane = threadIdx.x;
  const uint32_t wave_last = a.nv[tile];  // max of the pixels' `last` over the tile
  const uint2 rg = a.ranges[tile];
  // rows of the entries no pixel reached are zero
  for (uint32_t j = wave_last + (uint32_t)lane; j < rg.y - rg.x; j += 64) {
    const uint32_t e = instance_row(a, a.vals[rg.x + j], tx, ty);
    if ((uint64_t)e < a.cap) {
      float2* d = reinterpret_cast<float2*>(a.rows + (size_t)e * kRowFloats);
      const float2 z = make_float2(0.f, 0.f);
      d[0] = z, d[1] = z, d[2] = z, d[3] = z, d[4] = z;
    }
  }
  if (wave_last == 0) return;  // nothing blended here: no pixel reads
  const float log_amin = __logf(a.alpha_min);
  float fx[PPT], fy[PPT], T[PPT], S[PPT];
  float gx[PPT], gy[PPT], gz[PPT], gd[PPT], gtf[PPT];
  uint32_t lst[PPT], pbits[PPT];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int px = BL::x0(tx, k) + (lane & 7), py = BL::y0(ty, k) + (lane >> 3);
    const bool inside = px < a.W && py < a.H;
    const uint32_t pix = inside ? (uint32_t)py * a.W + px : 0u;
    bool active = inside;
    if (active && a.mask) active = (a.mask[pix >> 5] >> (pix & 31)) & 1u;
    pbits[k] = (FILT && active) ? filter_bits(a.omega, a.words, a.ncells, a.cell, pix) : 0u;
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
    S[k] = 0.f;
  }
  // per pixel group, the entries any of its pixels reached
  uint32_t gmax[PPT];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    uint32_t m = lst[k];
    for (int o = 32; o >= 1; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o, 64));
    gmax[k] = __builtin_amdgcn_readfirstlane(m);
  }
  for (int jend = (int)wave_last; jend > 0; jend -= 64) {
    // stage entries [jend - cnt, jend): lane i gathers entry jend - cnt + i,
    // stores its record and gradient row and tests its pixel box against
    // each pixel group; gm[k] bit i = entry j0 + i can reach group k and
    // some pixel of the group reached the entry
    const int cnt = jend < 64 ? jend : 64;
    const int j0 = jend - cnt;
    bool mk[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) mk[k] = false;
    if (lane < cnt) {
      const uint32_t gl = a.vals[rg.x + (uint32_t)(j0 + lane)];
      const float4* rr = reinterpret_cast<const float4*>(a.rec + (size_t)gl * kRecFloats);
      const float4 q0 = rr[0], q1 = rr[1], q2 = rr[2];
      const float bk = q0.w * kConicToExp2;
      s_rec[0][lane] = make_float4(q0.x, q0.y, q0.z * kConicToExp2, bk + bk);
      s_rec[1][lane] = make_float4(q1.x * kConicToExp2, q1.y, q1.z, q1.w);
      s_rec[2][lane] = q2;
      if (FILT) s_xf[lane] = a.xf[gl];
      // the rows of each block column the footprint reaches (the same
      // interval the forward computes for its blocks of that column)
      float2 yr[BL::BX];
#pragma unroll
      for (int c = 0; c < BL::BX; ++c) {
        const int x0 = BL::x0(tx, c);
        yr[c] = strip_rows(q0, q1, a.cx, a.cy, log_amin, x0, x0 + 7, ty * TH, ty * TH + TH - 1);
      }
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        const int x0 = BL::x0(tx, k), y0 = BL::y0(ty, k);
        mk[k] = (uint32_t)(j0 + lane) < gmax[k] && box_meets(q2.z, q2.w, x0, x0 + 7, y0, y0 + 7) &&
                rows_meet(yr[k % BL::BX], y0, y0 + 7, a.cy, q0.y);
      }
      s_e[lane] = instance_row(a, gl, tx, ty);
    }
    uint64_t gm[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) gm[k] = __ballot(mk[k]);
    __builtin_amdgcn_wave_barrier();
    // one entry's contributions, summed per lane into v; false when no
    // pixel of the tile blends it
    auto entry = [&](const float4& r0, const float4& r1, const float4& r2, int kk, uint32_t xe,
                     float (&v)[10]) -> bool {
    const int j = j0 + kk;
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
                       (!FILT || (xe & pbits[k]) == 0u);
      // no pixel of the group blends: the chain below would change nothing
      if (__ballot(use) == 0) continue;
      any = true;
      const float al = use ? ae.alpha : 0.f;
      const float om = 1.f - al;  // >= 1 - alpha_max
      const float rom = __builtin_amdgcn_rcpf(om);
      const float Ti = T[k] * rom;
      const float w = al * Ti;
      v[6] = fmaf(w, gx[k], v[6]);
      v[7] = fmaf(w, gy[k], v[7]);
      v[8] = fmaf(w, gz[k], v[8]);
      float gc = fmaf(gz[k], r2.x, fmaf(gy[k], r1.w, gx[k] * r1.z));  // G.c_i (+ g_D z_i)
      if constexpr (DG) {
        v[9] = fmaf(w, gd[k], v[9]);
        gc = fmaf(gd[k], r2.y, gc);
      }
      const float dS = gc - S[k];
      const float da = fmaf(Ti, dS, -(gtf[k] * rom));
      S[k] = fmaf(al, dS, S[k]);
      T[k] = Ti;
      const float dae = use && !ae.clamped ? da : 0.f;  // alpha clamped: no o, q terms
      v[5] = fmaf(dae, ae.G, v[5]);
      // h = -2 dL/dq; the row keeps the moments of h (see row_to_g2d)
      const float h = al * dae;
      const float hx = h * dx, hy = h * dy;
      v[0] += hx;
      v[1] += hy;
      v[2] = fmaf(hx, dx, v[2]);
      v[3] = fmaf(hx, dy, v[3]);
      v[4] = fmaf(hy, dy, v[4]);
    }
    return any;
    };
    // two entries per LDS round trip, back to front; their rows are summed
    // over the wavefront together
    for (int kk = cnt - 1; kk >= 0; kk -= 2) {
      const bool two = kk >= 1;
      const int k2 = two ? kk - 1 : kk;
      const float4 p0 = s_rec[0][kk], p1 = s_rec[1][kk], p2 = s_rec[2][kk];
      const float4 q0 = s_rec[0][k2], q1 = s_rec[1][k2], q2 = s_rec[2][k2];
      const uint32_t x1 = FILT ? s_xf[kk] : 0u, x2 = FILT ? s_xf[k2] : 0u;
      const uint32_t e1 = s_e[kk], e2 = s_e[k2];
      float va[10], vb[10];
      bool any = entry(p0, p1, p2, kk, x1, va);
      if (two) {
        const bool anyb = entry(q0, q1, q2, k2, x2, vb);
        any = any || anyb;
      } else {
#pragma unroll
        for (int m = 0; m < 10; ++m) vb[m] = 0.f;
      }
      float* da = (uint64_t)e1 < a.cap ? a.rows + (size_t)e1 * kRowFloats : nullptr;
      float* db = two && (uint64_t)e2 < a.cap ? a.rows + (size_t)e2 * kRowFloats : nullptr;
      if (any) {
        if constexpr (DG)
          wave_sum_pair_store<true>(va, vb, da, db, lane);
        else
          wave_sum_pair_store_lds(va, vb, da, db, lane, s_red);
      } else {
        // nothing blended either entry: zero rows
        float* d = lane == 63 ? da : lane == 62 ? db : nullptr;
        if (d) {
          float2* d2 = reinterpret_cast<float2*>(d);
          const float2 z = make_float2(0.f, 0.f);
          d2[0] = z, d2[1] = z, d2[2] = z, d2[3] = z, d2[4] = z;
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

template <int TW, int TH, bool DG, bool FILT>
__global__ __launch_bounds__(64) void k_render_bwd(RenderBwdArgs a) {
  __shared__ float4 s_rec[3][64];
  __shared__ uint32_t s_e[64];
  __shared__ float s_red[DG ? 1 : kRedFloats];
  __shared__ uint32_t s_xf[FILT ? 64 : 1];
  const int ntile = a.tiles_x * a.tiles_y;
  if ((int)blockIdx.x >= ntile) return;
  // the sort's order (a permutation of the tiles; its n = 0 call writes
  // none, and then no tile has an entry)
  const uint32_t tile = a.order[blockIdx.x];
  if (tile >= (uint32_t)ntile) return;
  render_tile_bwd<TW, TH, DG, FILT>(a, (int)tile, s_rec, s_e, s_red, s_xf);
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

// Per-Gaussian sum of its instance rows, which are contiguous (rows
// ioff[g] .. ioff[g] + n_tiles[g]), into g2d[g]; every visible Gaussian's
// row is written, so nothing is cleared first.  Four lanes share a
// Gaussian with up to kQuadRows rows: lane q of the quad sums rows q, q + 4,
// ... (the quad reads consecutive rows together) and two DPP steps add the
// quad's four sums, so a lane's chain of dependent loads is a quarter as
// long; the wavefront shares the rows of each Gaussian with more (strided,
// then one cross-lane sum).
constexpr uint32_t kQuadRows = 64;

__global__ __launch_bounds__(256) void k_slot_reduce(const uint32_t* __restrict__ vidx,
                                                     const uint64_t* counts,
                                                     const uint32_t* __restrict__ ioff,
                                                     const uint32_t* __restrict__ n_tiles,
                                                     const float* __restrict__ rows, uint64_t cap,
                                                     const float* __restrict__ rec,
                                                     float* __restrict__ g2d) {
  const int lane = threadIdx.x & 63, q = lane & 3;
  const uint64_t nvis = counts[0];
  // t0: the wavefront's first thread; its 16 quads take visible Gaussians
  // t0 / 4 .. t0 / 4 + 15 (a uniform loop, so every lane of a quad runs
  // the DPP steps)
  for (uint64_t t0 = (uint64_t)blockIdx.x * 256 + (threadIdx.x & ~63u); t0 / 4 < nvis;
       t0 += (uint64_t)gridDim.x * 256) {
    const uint64_t i = (t0 + (uint64_t)lane) >> 2;
    uint32_t g = 0, base = 0, cnt = 0;
    if (i < nvis) {
      g = vidx[i];
      base = ioff[g];
      cnt = n_tiles[g];
      // rows past the buffer (an instance overflow) are not read
      const uint64_t end = (uint64_t)base + cnt;
      cnt = end <= cap ? cnt : (uint32_t)(base < cap ? cap - base : 0);
    }
    const bool wide = cnt > kQuadRows;
    float acc[kRowFloats];
#pragma unroll
    for (int m = 0; m < kRowFloats; ++m) acc[m] = 0.f;
    if (!wide) {
      for (uint32_t r = (uint32_t)q; r < cnt; r += 4) {
        const float2* src = reinterpret_cast<const float2*>(rows + (size_t)(base + r) * kRowFloats);
#pragma unroll
        for (int m = 0; m < kRowFloats / 2; ++m) {
          const float2 v = src[m];
          acc[2 * m] += v.x, acc[2 * m + 1] += v.y;
        }
      }
    }
#pragma unroll
    for (int m = 0; m < kRowFloats; ++m) {
      float x = acc[m];
      x += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, true));
      x += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x4E, 0xF, 0xF, true));
      acc[m] = x;
    }
    if (i < nvis && q == 0 && !wide) {
      const float* cg = rec + (size_t)g * kRecFloats;
      row_to_g2d(acc, cg[2], cg[3], cg[4]);
      float4* d = reinterpret_cast<float4*>(g2d + (size_t)g * kG2dFloats);
      d[0] = make_float4(acc[0], acc[1], acc[2], acc[3]);
      d[1] = make_float4(acc[4], acc[5], acc[6], acc[7]);
      d[2] = make_float4(acc[8], acc[9], 0.f, 0.f);
    }
    // the wide Gaussians, one at a time over the whole wavefront (the four
    // lanes of its quad agree on it; its first lane is taken)
    for (uint64_t wm = __ballot(i < nvis && q == 0 && wide); wm; wm &= wm - 1) {
      const int l = __builtin_ctzll(wm);
      const uint32_t gw = __shfl(g, l, 64), bw = __shfl(base, l, 64), cw = __shfl(cnt, l, 64);
      float v[kRowFloats];
#pragma unroll
      for (int m = 0; m < kRowFloats; ++m) v[m] = 0.f;
      for (uint32_t r = (uint32_t)lane; r < cw; r += 64) {
        const float2* src = reinterpret_cast<const float2*>(rows + (size_t)(bw + r) * kRowFloats);
#pragma unroll
        for (int m = 0; m < kRowFloats / 2; ++m) {
          const float2 x = src[m];
          v[2 * m] += x.x, v[2 * m + 1] += x.y;
        }
      }
      // linear in the row sums, so applied to each lane's part before the
      // cross-lane sum
      const float* cg = rec + (size_t)gw * kRecFloats;
      row_to_g2d(v, cg[2], cg[3], cg[4]);
      float* d = g2d + (size_t)gw * kG2dFloats;
      wave_sum10_store(v, d, lane, true);
      if (lane == 0) d[10] = 0.f, d[11] = 0.f;
    }
  }
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
  __shared__ uint32_t s_e[64];
  __shared__ float s_red[kRedFloats];
  const uint32_t b = blockIdx.x;
  if (b >= m.base[m.V]) return;
  const int v = item_view(m.base, m.V, b);
  // batched views carry no depth gradient
  render_tile_bwd<TW, TH, false>(m.view[v], (int)(b - m.base[v]), s_rec, s_e, s_red);
}

static_assert(sizeof(RenderBwdMultiArgs) <= 4096, "kernel argument block too large");

bool tile_shape_supported(int tw, int th) {
  return (tw == 16 && th == 16) || (tw == 32 && th == 8) || (tw == 8 && th == 32) ||
         (tw == 32 && th == 16) || (tw == 16 && th == 32) || (tw == 8 && th == 8);
}

template <int TW, int TH>
static void launch_fwd_t(const RenderArgs& a, hipStream_t st) {
  const int grid = a.tiles_x * a.tiles_y;
  if (a.xf && a.nblend)
    hipLaunchKernelGGL((k_render<TW, TH, true, true>), dim3(grid), dim3(TW * TH), 0, st, a);
  else if (a.xf)
    hipLaunchKernelGGL((k_render<TW, TH, true, false>), dim3(grid), dim3(TW * TH), 0, st, a);
  else if (a.nblend)
    hipLaunchKernelGGL((k_render<TW, TH, false, true>), dim3(grid), dim3(TW * TH), 0, st, a);
  else
    hipLaunchKernelGGL((k_render<TW, TH, false, false>), dim3(grid), dim3(TW * TH), 0, st, a);
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
                                   const uint32_t* ranges, const SortView& sv, int64_t capacity,
                                   const DCam& cam, const KParams& p, const uint32_t* mask,
                                   const float* partial, const uint32_t* last,
                                   const float* dpartial, const float* ddepth, char* bws) {
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
  a.order = sv.order;
  a.ioff = sv.ioff;
  a.rect = reinterpret_cast<const ushort4*>(proj.rect);
  a.cap = (uint64_t)capacity;
  a.rows = reinterpret_cast<float*>(bws + BL.rows);
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

// Before the reverse walk: each tile's visited prefix.
static hipError_t launch_bwd_prepare(const RenderBwdArgs& a, const KParams& p, hipStream_t st) {
  SX_DISPATCH_TILE(p.tile_w, p.tile_h, launch_extent_t, a, st);
  return hipGetLastError();
}

// After the reverse walk: every visible Gaussian's screen-space gradient,
// the sum of its contiguous instance rows.
static hipError_t launch_bwd_reduce(const sx_projected& proj, const SortView& sv, int64_t n,
                                    int64_t capacity, const KParams& p, float* g2d, char* bws,
                                    hipStream_t st) {
  const int64_t tiles = (int64_t)p.tiles_x * p.tiles_y;
  const BwdLayout BL = bwd_layout(capacity, tiles);
  if (n > 0) {
    const int64_t blocks = (4 * n + 255) / 256;  // four lanes per Gaussian
    hipLaunchKernelGGL(k_slot_reduce, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256),
                       0, st, sv.vidx, sv.counts, sv.ioff, proj.n_tiles,
                       reinterpret_cast<const float*>(bws + BL.rows), (uint64_t)capacity,
                       proj.rec, g2d);
  }
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
  RenderBwdArgs a = make_bwd_args(proj, vals, ranges, sv, capacity, cam, p, mask, partial, last,
                                  dpartial, ddepth, bws);
  hipError_t e = hipSuccess;
  if ((stages & SX_RB_PREPARE) && (e = launch_bwd_prepare(a, p, st))) return e;
  if (stages & SX_RB_WALK) {
    SX_DISPATCH_TILE(p.tile_w, p.tile_h, launch_bwd_t, a, st);
    if ((e = hipGetLastError())) return e;
  }
  if (stages & SX_RB_REDUCE) return launch_bwd_reduce(proj, sv, n, capacity, p, g2d, bws, st);
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

hipError_t launch_render_backward_multi(int V, const MultiView* mv, const KParams& p,
                                        char* ws, hipStream_t st) {
  (void)ws;
  RenderBwdMultiArgs m;
  set_bases(V, mv, m);
  for (int v = 0; v < V; ++v) {
    KParams pv = p;
    pv.tiles_x = mv[v].tiles_x, pv.tiles_y = mv[v].tiles_y;
    const SortView sv = sort_view(mv[v].sort_ws, mv[v].n, mv[v].capacity, pv.tiles_x, pv.tiles_y);
    m.view[v] = make_bwd_args(mv[v].proj, mv[v].vals, mv[v].ranges, sv, mv[v].capacity,
                              mv[v].cam, pv, mv[v].mask, mv[v].partial, mv[v].last,
                              mv[v].dpartial, nullptr, static_cast<char*>(mv[v].bwd_ws));
    hipError_t e = launch_bwd_prepare(m.view[v], pv, st);
    if (e) return e;
  }
  SX_DISPATCH_TILE(p.tile_w, p.tile_h, launch_bwd_multi_t, m, st);
  return hipGetLastError();
}

hipError_t launch_grad_reduce_view(const MultiView& v, const KParams& p, hipStream_t st) {
  KParams pv = p;
  pv.tiles_x = v.tiles_x, pv.tiles_y = v.tiles_y;
  return launch_bwd_reduce(v.proj, sort_view(v.sort_ws, v.n, v.capacity, pv.tiles_x, pv.tiles_y),
                           v.n, v.capacity, pv, v.g2d, static_cast<char*>(v.bwd_ws), st);
}

}  // namespace sx
