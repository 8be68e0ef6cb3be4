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

// Records are staged per wavefront in batches of 64: lane i gathers the
// record of list entry jb+i with vector loads (64 gathers in flight, which
// hides their latency), writes it to the wavefront's own LDS slice, and the
// wavefront then walks the batch reading each record as a broadcast.  Each
// wavefront owns its slice, so no workgroup barrier is needed.
template <int TW, int TH>
__device__ __forceinline__ void render_tile(const RenderArgs& a, int tile,
                                            float4 (*s_rec)[3][64]) {
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const int lx = threadIdx.x % TW, ly = threadIdx.x / TW;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
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
  for (uint32_t jb = rg.x; jb < rg.y; jb += 64) {
    if (__ballot(!done) == 0) break;
    const uint32_t cnt = rg.y - jb < 64u ? rg.y - jb : 64u;
    if ((uint32_t)lane < cnt) {
      const float4* r = reinterpret_cast<const float4*>(a.rec + (size_t)a.vals[jb + lane] * kRecFloats);
      s_rec[w][0][lane] = r[0];
      s_rec[w][1][lane] = r[1];
      s_rec[w][2][lane] = r[2];
    }
    __builtin_amdgcn_wave_barrier();
    for (uint32_t k = 0; k < cnt; ++k) {
      if (__ballot(!done) == 0) break;
      const float4 r0 = s_rec[w][0][k], r1 = s_rec[w][1][k], r2 = s_rec[w][2][k];
      const AlphaEval ae = eval_alpha(fx - r0.x, fy - r0.y, r0.z, r0.w, r1.x, r1.y, a.alpha_max);
      if (!done && ae.alpha >= a.alpha_min) {
        const float wt = ae.alpha * T;
        C0 = fmaf(r1.z, wt, C0);
        C1 = fmaf(r1.w, wt, C1);
        C2 = fmaf(r2.x, wt, C2);
        D = fmaf(r2.y, wt, D);
        T = T * (1.f - ae.alpha);
        ++nb;
        lst = jb + k - rg.x + 1;
        if (T < a.t_min) done = true;
      }
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

template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void k_render(RenderArgs a) {
  __shared__ float4 s_rec[TW * TH / 64][3][64];
  const int ntile = a.tiles_x * a.tiles_y;
  const int tile = xcd_tile(blockIdx.x, ntile);
  if (tile >= ntile) return;
  render_tile<TW, TH>(a, tile, s_rec);
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
  const uint16_t* __restrict__ rect;
  const uint32_t* __restrict__ goffs;
  uint64_t cap;
  float* __restrict__ gpart;
  uint64_t* __restrict__ last_key;
};

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
// (Gaussian, tile).  No atomics: the tile's partial gradient row is stored
// at the instance's position in emission order, e = (first instance of the
// Gaussian) + (row-major index of the tile within its rectangle), a slot no
// other tile writes; rows of visited entries without any contribution are
// stored as zeros.  The tile records the sort key of the last entry it
// visited, which tells the per-Gaussian reduction which slots are valid.
template <int TW, int TH>
__device__ __forceinline__ void render_tile_bwd(const RenderBwdArgs& a, int tile,
                                                float4 (*s_rec)[64], uint32_t* s_e) {
  constexpr int PPT = TW * TH / 64;
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const int lane = threadIdx.x;
  const uint2 rg = a.ranges[tile];
  float fx[PPT], fy[PPT], T[PPT], R0[PPT], R1[PPT], R2[PPT], RD[PPT];
  float gx[PPT], gy[PPT], gz[PPT], gt[PPT], gd[PPT], Tf[PPT];
  uint32_t lst[PPT];
  uint32_t mx = 0;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int li = lane + 64 * k;
    const int px = tx * TW + li % TW, py = ty * TH + li / TW;
    const bool inside = px < a.W && py < a.H;
    const uint32_t pix = inside ? (uint32_t)py * a.W + px : 0u;
    bool active = inside;
    if (active && a.mask) active = (a.mask[pix >> 5] >> (pix & 31)) & 1u;
    fx[k] = (float)px + 0.5f - a.cx;
    fy[k] = (float)py + 0.5f - a.cy;
    Tf[k] = 1.f, gx[k] = gy[k] = gz[k] = gt[k] = gd[k] = 0.f;
    lst[k] = 0;
    if (active) {
      Tf[k] = a.partial[pix].w;
      const float4 g = a.dpartial[pix];
      gx[k] = g.x, gy[k] = g.y, gz[k] = g.z, gt[k] = g.w;
      if (a.ddepth) gd[k] = a.ddepth[pix];
      lst[k] = a.last[pix];
    }
    T[k] = Tf[k];
    R0[k] = R1[k] = R2[k] = RD[k] = 0.f;
    mx = lst[k] > mx ? lst[k] : mx;
  }
  const uint32_t wave_last = wave_max_u32(mx);
  if (lane == 0) {
    uint64_t key = 0;
    if (wave_last > 0) {
      const uint32_t gl = a.vals[rg.x + wave_last - 1];
      key = ((uint64_t)__float_as_uint(a.rec[(size_t)gl * kRecFloats + 9]) << 32) | gl;
    }
    a.last_key[tile] = key;
  }
  for (int jend = (int)wave_last; jend > 0; jend -= 64) {
    // stage entries [jend - cnt, jend): lane i gathers entry jend - cnt + i
    // and its gradient slot e = (first instance of the Gaussian) + (index of
    // this tile in the Gaussian's rectangle, row-major)
    const int cnt = jend < 64 ? jend : 64;
    const int j0 = jend - cnt;
    if (lane < cnt) {
      const uint32_t gl = a.vals[rg.x + (uint32_t)(j0 + lane)];
      const float4* rr = reinterpret_cast<const float4*>(a.rec + (size_t)gl * kRecFloats);
      s_rec[0][lane] = rr[0];
      s_rec[1][lane] = rr[1];
      s_rec[2][lane] = rr[2];
      const ushort4 rc = reinterpret_cast<const ushort4*>(a.rect)[gl];
      s_e[lane] = a.goffs[gl] + ((uint32_t)ty - rc.y) * ((uint32_t)rc.z - rc.x) + ((uint32_t)tx - rc.x);
    }
    __builtin_amdgcn_wave_barrier();
  for (int kk = cnt - 1; kk >= 0; --kk) {
    const int j = j0 + kk;
    const float4 r0 = s_rec[0][kk], r1 = s_rec[1][kk], r2 = s_rec[2][kk];
    const uint32_t e = s_e[kk];
    float4* dst = reinterpret_cast<float4*>(a.gpart + (size_t)e * kG2dFloats);
    const bool in_cap = (uint64_t)e < a.cap;
    float v[10];
#pragma unroll
    for (int m = 0; m < 10; ++m) v[m] = 0.f;
    bool any = false;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const float dx = fx[k] - r0.x, dy = fy[k] - r0.y;
      const AlphaEval ae = eval_alpha(dx, dy, r0.z, r0.w, r1.x, r1.y, a.alpha_max);
      if ((uint32_t)j < lst[k] && ae.alpha >= a.alpha_min) {
        any = true;
        const float om = 1.f - ae.alpha;
        const float rom = 1.f / om;
        const float Ti = T[k] * rom;
        const float w = ae.alpha * Ti;
        v[6] += w * gx[k];
        v[7] += w * gy[k];
        v[8] += w * gz[k];
        v[9] += w * gd[k];
        float da = gx[k] * (r1.z - R0[k]) + gy[k] * (r1.w - R1[k]) + gz[k] * (r2.x - R2[k]) +
                   gd[k] * (r2.y - RD[k]);
        da = Ti * da - gt[k] * (Tf[k] * rom);
        R0[k] = fmaf(r1.z, ae.alpha, om * R0[k]);
        R1[k] = fmaf(r1.w, ae.alpha, om * R1[k]);
        R2[k] = fmaf(r2.x, ae.alpha, om * R2[k]);
        RD[k] = fmaf(r2.y, ae.alpha, om * RD[k]);
        T[k] = Ti;
        if (!ae.clamped) {
          v[5] += da * ae.G;
          const float dq = -0.5f * ae.alpha * da;
          v[0] += -2.f * dq * (r0.z * dx + r0.w * dy);
          v[1] += -2.f * dq * (r0.w * dx + r1.x * dy);
          v[2] += dq * dx * dx;
          v[3] += 2.f * dq * dx * dy;
          v[4] += dq * dy * dy;
        }
      }
    }
    if (__ballot(any) == 0) {
      if (lane == 63 && in_cap) {
        const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
        dst[0] = z, dst[1] = z, dst[2] = z;
      }
      continue;
    }
    float sum[10];
#pragma unroll
    for (int m = 0; m < 10; ++m) sum[m] = wave_sum_to_lane63(v[m]);
    if (lane == 63 && in_cap) {
      dst[0] = make_float4(sum[0], sum[1], sum[2], sum[3]);
      dst[1] = make_float4(sum[4], sum[5], sum[6], sum[7]);
      dst[2] = make_float4(sum[8], sum[9], 0.f, 0.f);
    }
  }
    __builtin_amdgcn_wave_barrier();
  }
}

template <int TW, int TH>
__global__ __launch_bounds__(64) void k_render_bwd(RenderBwdArgs a) {
  __shared__ float4 s_rec[3][64];
  __shared__ uint32_t s_e[64];
  const int ntile = a.tiles_x * a.tiles_y;
  const int tile = xcd_tile(blockIdx.x, ntile);
  if (tile >= ntile) return;
  render_tile_bwd<TW, TH>(a, tile, s_rec, s_e);
}

// Per-Gaussian sum of the partial gradient rows.  Balanced like the
// emission: every block owns instances [c0, c0 + kEmitChunk) in emission
// order, where each Gaussian's instances are contiguous.  An instance's row
// is valid iff its tile visited it, i.e. (depth bits, index) of the
// Gaussian <= the tile's last visited key.  Sums are formed in LDS; a
// Gaussian lying wholly inside the chunk is stored with plain stores, one
// that straddles a chunk boundary is added atomically into its
// (pre-zeroed) row, so atomics occur at most twice per chunk.
struct ReduceArgs {
  const uint32_t* __restrict__ didx;
  const uint32_t* __restrict__ offs;
  const uint32_t* __restrict__ chunk_first;
  const uint64_t* counts;
  const uint16_t* __restrict__ rect;
  const uint32_t* __restrict__ n_tiles;
  const float* __restrict__ rec;
  const float* __restrict__ gpart;
  const uint64_t* __restrict__ last_key;
  int tiles_x, tiles;
  uint64_t cap;
  float* __restrict__ g2d;
};

__global__ __launch_bounds__(256) void k_grad_reduce(ReduceArgs a) {
  __shared__ uint32_t s_off[257], s_end[256], s_g[256], s_x0[256], s_y0[256], s_w[256];
  __shared__ unsigned long long s_key[256];
  __shared__ float s_acc[256 * 10];
  __shared__ uint32_t s_lohi[2];
  extern __shared__ uint32_t s_ldep[];  // per tile: depth bits of the last visited entry
  const int tid = threadIdx.x;
  if (a.counts[2] != 0) return;
  const bool staged = a.tiles <= kReduceLdsTiles;
  if (staged)
    for (int t = tid; t < a.tiles; t += 256) s_ldep[t] = (uint32_t)(a.last_key[t] >> 32);
  const uint64_t ninst = a.counts[1] < a.cap ? a.counts[1] : a.cap;
  const uint64_t nvis = a.counts[0];
  const uint64_t c0 = (uint64_t)blockIdx.x * kEmitChunk;
  if (c0 >= ninst) return;
  const uint64_t c1 = c0 + kEmitChunk < ninst ? c0 + kEmitChunk : ninst;
  if (tid == 0) chunk_bounds(a.chunk_first, a.offs, nvis, ninst, c0, c1, s_lohi);
  __syncthreads();
  const uint32_t slo = s_lohi[0], shi = s_lohi[1];
  for (uint32_t w0 = slo; w0 <= shi; w0 += 256) {
    const uint32_t wn = (shi - w0 + 1) < 256u ? (shi - w0 + 1) : 256u;
    if ((uint32_t)tid < wn) {
      const uint32_t sidx = w0 + tid;
      const uint32_t g = a.didx[sidx];
      const ushort4 rc = reinterpret_cast<const ushort4*>(a.rect)[g];
      s_off[tid] = a.offs[sidx];
      s_end[tid] = a.offs[sidx] + a.n_tiles[g];
      s_g[tid] = g;
      s_x0[tid] = rc.x, s_y0[tid] = rc.y, s_w[tid] = (uint32_t)rc.z - rc.x;
      s_key[tid] = ((unsigned long long)__float_as_uint(a.rec[(size_t)g * kRecFloats + 9]) << 32) | g;
#pragma unroll
      for (int m = 0; m < 10; ++m) s_acc[tid * 10 + m] = 0.f;
    }
    if (tid == 0) {
      const uint64_t e = (uint64_t)w0 + wn < nvis ? (uint64_t)a.offs[w0 + wn] : ninst;
      s_off[wn] = (uint32_t)(e < c1 ? e : c1);
    }
    __syncthreads();
    const uint64_t k0 = (uint64_t)s_off[0] > c0 ? (uint64_t)s_off[0] : c0;
    const uint64_t k1 = s_off[wn];
    // runs of consecutive slots per thread: sums stay in registers while the
    // run stays on one Gaussian and go to LDS when it moves on
    const uint32_t run = ((uint32_t)(k1 - k0) + 255) / 256;
    uint64_t k = k0 + (uint64_t)tid * run;
    const uint64_t kend = k + run < k1 ? k + run : k1;
    if (k < kend) {
      int j = 0, hi = (int)wn - 1;
      while (j < hi) {
        const int mid = (j + hi + 1) >> 1;
        if (s_off[mid] <= k) j = mid; else hi = mid - 1;
      }
      uint32_t wj = s_w[j];
      const uint32_t r = (uint32_t)(k - s_off[j]);
      uint32_t ty = r / wj, tx = r - ty * wj;
      float acc[10];
#pragma unroll
      for (int m = 0; m < 10; ++m) acc[m] = 0.f;
      bool dirty = false;
      for (; k < kend; ++k) {
        if (k == s_off[j + 1]) {
          if (dirty) {
#pragma unroll
            for (int m = 0; m < 10; ++m) atomicAdd(s_acc + j * 10 + m, acc[m]), acc[m] = 0.f;
            dirty = false;
          }
          ++j;
          wj = s_w[j], tx = 0, ty = 0;
        }
        const uint32_t tile = (s_y0[j] + ty) * (uint32_t)a.tiles_x + s_x0[j] + tx;
        bool visited;
        if (staged) {
          const uint32_t dg = (uint32_t)(s_key[j] >> 32), dt = s_ldep[tile];
          visited = dg < dt || (dg == dt && s_key[j] <= a.last_key[tile]);
        } else {
          visited = s_key[j] <= a.last_key[tile];
        }
        if (visited) {
          const float4* src = reinterpret_cast<const float4*>(a.gpart + (size_t)k * kG2dFloats);
          const float4 p0 = src[0], p1 = src[1], p2 = src[2];
          acc[0] += p0.x, acc[1] += p0.y, acc[2] += p0.z, acc[3] += p0.w, acc[4] += p1.x;
          acc[5] += p1.y, acc[6] += p1.z, acc[7] += p1.w, acc[8] += p2.x, acc[9] += p2.y;
          dirty = true;
        }
        if (++tx == wj) tx = 0, ++ty;
      }
      if (dirty) {
#pragma unroll
        for (int m = 0; m < 10; ++m) atomicAdd(s_acc + j * 10 + m, acc[m]);
      }
    }
    __syncthreads();
    if ((uint32_t)tid < wn) {
      float* dst = a.g2d + (size_t)s_g[tid] * kG2dFloats;
      const bool interior = s_off[tid] >= c0 && s_end[tid] <= c1;
      if (interior) {
#pragma unroll
        for (int m = 0; m < 10; ++m) dst[m] = s_acc[tid * 10 + m];
      } else {
#pragma unroll
        for (int m = 0; m < 10; ++m) unsafeAtomicAdd(dst + m, s_acc[tid * 10 + m]);
      }
    }
    __syncthreads();
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
// Many views in one persistent launch: the (view, tile) work items of all
// views are ordered by descending cost class (bit length of the tile's list
// length) and workgroups take items from a global counter until none is
// left, so large and small views share the GPU with no per-view tail.
struct WorkArgs {
  int V;
  uint32_t base[kMaxViews + 1];  // first work item of each view
  const uint2* ranges[kMaxViews];
  uint32_t* hist;    // [32] items per cost class
  uint32_t* cursor;  // [32]
  uint32_t* items;   // [n] (view << 24) | tile
};

__device__ __forceinline__ int work_view(const WorkArgs& w, uint32_t item) {
  int v = 0;
  while (v + 1 < w.V && item >= w.base[v + 1]) ++v;
  return v;
}

__device__ __forceinline__ int cost_class(uint2 r) {
  const uint32_t c = r.y - r.x;
  return c == 0 ? 0 : 32 - __clz(c);
}

__global__ __launch_bounds__(256) void k_work_hist(WorkArgs w) {
  __shared__ uint32_t h[33];
  if (threadIdx.x < 33) h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t item = blockIdx.x * 256 + threadIdx.x;
  if (item < w.base[w.V]) {
    const int v = work_view(w, item);
    atomicAdd(&h[cost_class(w.ranges[v][item - w.base[v]])], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 33 && h[threadIdx.x]) atomicAdd(&w.hist[threadIdx.x], h[threadIdx.x]);
}

__global__ __launch_bounds__(256) void k_work_scatter(WorkArgs w) {
  __shared__ uint32_t h[33], start[33], mine[33];
  if (threadIdx.x < 33) h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t item = blockIdx.x * 256 + threadIdx.x;
  int cls = -1, v = 0;
  uint32_t rank = 0;
  if (item < w.base[w.V]) {
    v = work_view(w, item);
    cls = cost_class(w.ranges[v][item - w.base[v]]);
    rank = atomicAdd(&h[cls], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 33) {
    // classes are laid out from the most expensive down
    uint32_t s0 = 0;
    for (int c = 32; c > (int)threadIdx.x; --c) s0 += w.hist[c];
    start[threadIdx.x] = s0;
    mine[threadIdx.x] = h[threadIdx.x] ? atomicAdd(&w.cursor[threadIdx.x], h[threadIdx.x]) : 0u;
  }
  __syncthreads();
  if (cls >= 0)
    w.items[start[cls] + mine[cls] + rank] = ((uint32_t)v << 24) | (item - w.base[v]);
}

static_assert(sizeof(WorkArgs) <= 1024, "work-list arguments");

struct RenderMultiArgs {
  int V;
  uint32_t n_items;
  const uint32_t* __restrict__ items;
  uint32_t* counter;
  RenderArgs view[kMaxViews];
};

template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void k_render_multi(RenderMultiArgs m) {
  __shared__ float4 s_rec[TW * TH / 64][3][64];
  __shared__ uint32_t s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(m.counter, 1u);
    __syncthreads();
    const uint32_t it = s_item;
    __syncthreads();
    if (it >= m.n_items) break;
    const uint32_t code = m.items[it];
    render_tile<TW, TH>(m.view[code >> 24], (int)(code & 0xFFFFFF), s_rec);
  }
}

struct RenderBwdMultiArgs {
  int V;
  uint32_t n_items;
  const uint32_t* __restrict__ items;
  uint32_t* counter;
  RenderBwdArgs view[kMaxViews];
};

static_assert(sizeof(RenderMultiArgs) <= 4096, "kernel argument block too large");

template <int TW, int TH>
__global__ __launch_bounds__(64) void k_render_bwd_multi(RenderBwdMultiArgs m) {
  __shared__ float4 s_rec[3][64];
  __shared__ uint32_t s_e[64];
  for (;;) {
    uint32_t it = 0;
    if (threadIdx.x == 0) it = atomicAdd(m.counter, 1u);
    it = __shfl(it, 0, 64);
    if (it >= m.n_items) break;
    const uint32_t code = m.items[it];
    render_tile_bwd<TW, TH>(m.view[code >> 24], (int)(code & 0xFFFFFF), s_rec, s_e);
  }
}

static_assert(sizeof(RenderBwdMultiArgs) <= 4096, "kernel argument block too large");

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
  hipLaunchKernelGGL((k_render_bwd<TW, TH>), dim3(grid), dim3(64), 0, st, a);
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
  return a;
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
  a.rect = proj.rect;
  a.goffs = sv.goffs;
  a.cap = (uint64_t)capacity;
  a.gpart = reinterpret_cast<float*>(bws + BL.gpart);
  a.last_key = reinterpret_cast<uint64_t*>(bws + BL.last_key);
  return a;
}

// zero the visible rows of g2d, then sum each Gaussian's valid partial rows
static hipError_t launch_grad_reduce(const sx_projected& proj, const SortView& sv, int64_t n,
                                     int64_t capacity, const KParams& p, float* g2d, char* bws,
                                     hipStream_t st) {
  const int64_t tiles = (int64_t)p.tiles_x * p.tiles_y;
  const BwdLayout BL = bwd_layout(capacity, tiles);
  if (n > 0)
    hipLaunchKernelGGL(k_zero_g2d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       sv.didx, sv.counts, g2d);
  ReduceArgs r;
  r.didx = sv.didx, r.offs = sv.offs, r.counts = sv.counts, r.chunk_first = sv.chunk_first;
  r.rect = proj.rect, r.n_tiles = proj.n_tiles, r.rec = proj.rec;
  r.gpart = reinterpret_cast<const float*>(bws + BL.gpart);
  r.last_key = reinterpret_cast<const uint64_t*>(bws + BL.last_key);
  r.tiles_x = p.tiles_x;
  r.tiles = (int)tiles;
  r.cap = (uint64_t)capacity;
  r.g2d = g2d;
  const int64_t rb = (capacity + kEmitChunk - 1) / kEmitChunk;
  const size_t lds = tiles <= kReduceLdsTiles ? (size_t)tiles * 4 : 0;
  hipLaunchKernelGGL(k_grad_reduce, dim3((unsigned)(rb > 0 ? rb : 1)), dim3(256), lds, st, r);
  return hipGetLastError();
}

hipError_t launch_render_backward(const sx_projected& proj,
                                  const uint32_t* vals, const uint32_t* ranges,
                                  const SortView& sv, int64_t n, int64_t capacity,
                                  const DCam& cam, const KParams& p,
                                  const uint32_t* mask, const float* partial,
                                  const uint32_t* last, const float* dpartial,
                                  const float* ddepth, float* g2d, char* bws,
                                  hipStream_t st) {
  RenderBwdArgs a = make_bwd_args(proj, vals, ranges, sv, capacity, cam, p, mask, partial, last,
                                  dpartial, ddepth, bws);
  SX_DISPATCH_TILE(p.tile_w, p.tile_h, launch_bwd_t, a, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_grad_reduce(proj, sv, n, capacity, p, g2d, bws, st);
}

// ------------------------------------------------------------ multi-view --
// work-list workspace: a 512-byte head (hist[33], cursor[33], two work
// counters) followed by one u32 item per (view, tile)
constexpr int kWorkHeadWords = 128;
size_t multi_workspace_bytes(int64_t items) {
  return kWorkHeadWords * 4 + (size_t)(items > 0 ? items : 1) * 4;
}

static hipError_t build_worklist(int V, const MultiView* mv, const KParams& p, char* ws,
                                 WorkArgs& w, hipStream_t st) {
  uint32_t* head = reinterpret_cast<uint32_t*>(ws);
  w.V = V;
  uint32_t base = 0;
  for (int v = 0; v < V; ++v) {
    w.base[v] = base;
    w.ranges[v] = reinterpret_cast<const uint2*>(mv[v].ranges);
    base += (uint32_t)(mv[v].tiles_x * mv[v].tiles_y);
  }
  w.base[V] = base;
  w.hist = head;
  w.cursor = head + 33;
  w.items = reinterpret_cast<uint32_t*>(ws + kWorkHeadWords * 4);
  hipError_t e = launch_fill(head, kWorkHeadWords, 0, st);  // hist, cursor, work counters
  if (e) return e;
  const unsigned nb = (base + 255) / 256;
  hipLaunchKernelGGL(k_work_hist, dim3(nb > 0 ? nb : 1), dim3(256), 0, st, w);
  hipLaunchKernelGGL(k_work_scatter, dim3(nb > 0 ? nb : 1), dim3(256), 0, st, w);
  return hipGetLastError();
}

template <int TW, int TH>
static void launch_fwd_multi_t(const RenderMultiArgs& m, hipStream_t st) {
  const unsigned grid = m.n_items < 2048u ? m.n_items : 2048u;
  hipLaunchKernelGGL((k_render_multi<TW, TH>), dim3(grid > 0 ? grid : 1), dim3(TW * TH), 0, st, m);
}
template <int TW, int TH>
static void launch_bwd_multi_t(const RenderBwdMultiArgs& m, hipStream_t st) {
  const unsigned grid = m.n_items < 5120u ? m.n_items : 5120u;
  hipLaunchKernelGGL((k_render_bwd_multi<TW, TH>), dim3(grid > 0 ? grid : 1), dim3(64), 0, st, m);
}

hipError_t launch_render_multi(int V, const MultiView* mv, const KParams& p, char* ws,
                               hipStream_t st) {
  WorkArgs w;
  hipError_t e = build_worklist(V, mv, p, ws, w, st);
  if (e) return e;
  RenderMultiArgs m;
  m.V = V;
  m.n_items = w.base[V];
  m.items = w.items;
  m.counter = w.hist + 66;
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
  WorkArgs w;
  hipError_t e = build_worklist(V, mv, p, ws, w, st);
  if (e) return e;
  RenderBwdMultiArgs m;
  m.V = V;
  m.n_items = w.base[V];
  m.items = w.items;
  m.counter = w.hist + 67;
  for (int v = 0; v < V; ++v) {
    KParams pv = p;
    pv.tiles_x = mv[v].tiles_x, pv.tiles_y = mv[v].tiles_y;
    const int64_t tiles = (int64_t)pv.tiles_x * pv.tiles_y;
    m.view[v] = make_bwd_args(mv[v].proj, mv[v].vals, mv[v].ranges,
                              sort_view(mv[v].sort_ws, n, mv[v].capacity, pv.tiles_x, pv.tiles_y), mv[v].capacity,
                              mv[v].cam, pv, mv[v].mask, mv[v].partial, mv[v].last,
                              mv[v].dpartial, nullptr, static_cast<char*>(mv[v].bwd_ws));
  }
  SX_DISPATCH_TILE(p.tile_w, p.tile_h, launch_bwd_multi_t, m, st);
  return hipGetLastError();
}

hipError_t launch_grad_reduce_view(const MultiView& v, int64_t n, const KParams& p,
                                   hipStream_t st) {
  KParams pv = p;
  pv.tiles_x = v.tiles_x, pv.tiles_y = v.tiles_y;
  const int64_t tiles = (int64_t)pv.tiles_x * pv.tiles_y;
  return launch_grad_reduce(v.proj, sort_view(v.sort_ws, n, v.capacity, pv.tiles_x, pv.tiles_y), n, v.capacity,
                            pv, v.g2d, static_cast<char*>(v.bwd_ws), st);
}

}  // namespace sx
