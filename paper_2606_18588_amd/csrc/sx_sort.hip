// Depth sort of the instance list (paper, background: sorting step).
//
// The result equals a stable sort of 64-bit keys
//     key = tile_id << 32 | bits(float32 depth)
// over instances emitted in Gaussian-index order, i.e. the order
// (tile, depth bits, Gaussian index).  Because the 32 depth bits are the same
// for every instance of a Gaussian, the LSD radix sort is split in two:
//   1. the low (depth) digits are applied to the compacted list of visible
//      Gaussians *before* duplication (4 passes over ~N_vis elements);
//   2. instances are emitted in that depth order, so only the tile digits
//      remain, sorted stably over the duplicated list (ceil(bits/8) passes,
//      e.g. 2 for a 1080p frame's 8160 tiles).
// Per-tile instance counts come from a 2D difference grid of the Gaussians'
// tile rectangles (four atomics per visible Gaussian, then a 2D prefix sum),
// which yields the tile ranges and the tile-digit histograms without reading
// the instance list.  Instances are emitted by blocks that each own a fixed
// chunk of the output (balanced however many tiles a Gaussian covers).
// Each pass is a single "onesweep" kernel: per-partition digit ranking with
// wavefront ballots (wave64 match), a decoupled look-back across partitions
// for the global offsets, and an LDS reorder so that global writes are
// coalesced runs.  Partitions take their index from an atomic counter, so a
// partition only ever waits on partitions that are already running, and
// every wait is bounded (a spin limit raises an error flag instead of
// hanging).
#include "sx_internal.h"

namespace sx {

namespace {

constexpr uint32_t kFlagAgg = 1u << 30;
constexpr uint32_t kFlagIncl = 2u << 30;
constexpr uint32_t kValMask = (1u << 30) - 1;
constexpr uint64_t kEFlagAgg = 1ull << 62;
constexpr uint64_t kEFlagIncl = 2ull << 62;
constexpr uint64_t kEValMask = (1ull << 62) - 1;
constexpr int kSpinLimit = 1 << 20;

__device__ __forceinline__ uint32_t ld_acq(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_acq64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive scan of one uint32 per thread over a 256-thread block.
__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t v, uint32_t* s4,
                                                       uint32_t* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s4[w] = x;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
  for (int k = 0; k < 4; ++k) {
    if (k < w) pre += s4[k];
    tot += s4[k];
  }
  __syncthreads();
  if (total) *total = tot;
  return pre + x - v;
}

}  // namespace

SortLayout sort_layout(int64_t n, int64_t cap, int64_t tiles_total) {
  SortLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  L.nb = (n + kPreBlock - 1) / kPreBlock;
  L.dparts = (n + kSortTile - 1) / kSortTile;
  L.tparts = (cap + kSortTile - 1) / kSortTile;
  L.eparts = (n + kScanTile - 1) / kScanTile;
  if (L.dparts < 1) L.dparts = 1;
  if (L.tparts < 1) L.tparts = 1;
  if (L.eparts < 1) L.eparts = 1;
  L.zero_begin = off;
  L.counts = take(4 * sizeof(uint64_t));
  L.dhist = take(4 * kRadixBins * 4);
  L.thist = take(3 * kRadixBins * 4);
  L.counters = take(16 * 4);
  L.dstatus = take((size_t)4 * L.dparts * kRadixBins * 4);
  L.tstatus = take((size_t)3 * L.tparts * kRadixBins * 4);
  L.estatus = take((size_t)L.eparts * 8);
  L.diff = take((size_t)(2 * tiles_total + 2) * 4);
  L.zero_end = off;
  L.diffparts = take((size_t)kDiffParts * (2 * tiles_total + 2) * 4);
  L.offs = take((size_t)(n > 0 ? n : 1) * 4);
  L.goffs = take((size_t)(n > 0 ? n : 1) * 4);
  L.chunk_first = take((size_t)((cap + kEmitChunk - 1) / kEmitChunk + 2) * 4);
  L.vis_off = take((size_t)(L.nb > 0 ? L.nb : 1) * 4);
  for (int k = 0; k < 2; ++k) L.dkey[k] = take((size_t)(n > 0 ? n : 1) * 4);
  for (int k = 0; k < 2; ++k) L.didx[k] = take((size_t)(n > 0 ? n : 1) * 4);
  for (int k = 0; k < 2; ++k) L.tkey[k] = take((size_t)(cap > 0 ? cap : 1) * 4);
  for (int k = 0; k < 2; ++k) L.tval[k] = take((size_t)(cap > 0 ? cap : 1) * 4);
  L.total = off;
  return L;
}

BwdLayout bwd_layout(int64_t cap, int64_t tiles_total) {
  BwdLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  L.gpart = take((size_t)(cap > 0 ? cap : 1) * kG2dFloats * 4);
  L.last_key = take((size_t)(tiles_total > 0 ? tiles_total : 1) * 8);
  L.total = off;
  return L;
}

SortView sort_view(const void* ws, int64_t n, int64_t capacity, int64_t tiles_total) {
  const SortLayout L = sort_layout(n, capacity, tiles_total);
  const char* b = static_cast<const char*>(ws);
  SortView v;
  v.counts = reinterpret_cast<const uint64_t*>(b + L.counts);
  v.didx = reinterpret_cast<const uint32_t*>(b + L.didx[0]);
  v.offs = reinterpret_cast<const uint32_t*>(b + L.offs);
  v.goffs = reinterpret_cast<const uint32_t*>(b + L.goffs);
  v.chunk_first = reinterpret_cast<const uint32_t*>(b + L.chunk_first);
  return v;
}

// ------------------------------------------------------------- counting --
// One block: exclusive scan of the per-preprocess-block visible counts and
// the total instance count.
__global__ __launch_bounds__(1024) void k_scan_blocks(const uint32_t* __restrict__ bsum,
                                                      int64_t nb, uint32_t* __restrict__ vis_off,
                                                      uint64_t* counts, int64_t cap) {
  __shared__ uint32_t sw[16];
  __shared__ unsigned long long si[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t chunk = (nb + 1023) / 1024;
  const int64_t beg = tid * chunk, end = beg + chunk < nb ? beg + chunk : nb;
  uint32_t sv = 0;
  unsigned long long sinst = 0;
  for (int64_t k = beg; k < end; ++k) {
    sv += bsum[2 * k];
    sinst += bsum[2 * k + 1];
  }
  uint32_t x = sv;
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  unsigned long long r = sinst;
  for (int o = 32; o >= 1; o >>= 1) r += __shfl_xor(r, o, 64);
  if (lane == 63) sw[w] = x;
  if (lane == 0) si[w] = r;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
  unsigned long long itot = 0;
  for (int k = 0; k < 16; ++k) {
    if (k < w) pre += sw[k];
    tot += sw[k];
    itot += si[k];
  }
  uint32_t run = pre + x - sv;
  for (int64_t k = beg; k < end; ++k) {
    vis_off[k] = run;
    run += bsum[2 * k];
  }
  if (tid == 0) {
    counts[0] = tot;
    counts[1] = itot;
    counts[2] = itot > (unsigned long long)cap ? 1ull : 0ull;
  }
}

// Compacted (depth bits, Gaussian index) list of visible Gaussians in index
// order.
// Also adds each visible Gaussian's tile rectangle to the 2D difference grid
// diff[(tiles_y+1) x (tiles_x+1)]: +1 at (x0,y0) and (x1,y1), -1 at (x1,y0)
// and (x0,y1); its 2D prefix sum is the number of instances per tile.
__global__ __launch_bounds__(kPreBlock) void k_compact(const uint32_t* __restrict__ n_tiles,
                                                       const float* __restrict__ rec,
                                                       const uint16_t* __restrict__ rect, int64_t n,
                                                       const uint32_t* __restrict__ vis_off,
                                                       uint32_t* __restrict__ dkey,
                                                       uint32_t* __restrict__ didx,
                                                       int* __restrict__ diff, int gw,
                                                       int use_global_diff) {
  __shared__ uint32_t sw[kPreBlock / 64];
  const int64_t i = (int64_t)blockIdx.x * kPreBlock + threadIdx.x;
  const bool v = i < n && n_tiles[i] > 0;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t b = __ballot(v);
  const uint32_t rank = __popcll(b & ((1ull << lane) - 1));
  if (lane == 0) sw[w] = __popcll(b);
  __syncthreads();
  uint32_t pre = 0;
  for (int k = 0; k < w; ++k) pre += sw[k];
  if (v) {
    const uint32_t pos = vis_off[blockIdx.x] + pre + rank;
    dkey[pos] = __float_as_uint(rec[(size_t)i * kRecFloats + 9]);
    didx[pos] = (uint32_t)i;
    if (use_global_diff) {
      const ushort4 rc = reinterpret_cast<const ushort4*>(rect)[i];
      atomicAdd(&diff[rc.y * gw + rc.x], 1);
      atomicAdd(&diff[rc.y * gw + rc.z], -1);
      atomicAdd(&diff[rc.w * gw + rc.x], -1);
      atomicAdd(&diff[rc.w * gw + rc.z], 1);
    }
  }
}

// Difference grid without global atomics (used when the grid fits in LDS):
// each of kDiffParts blocks accumulates a contiguous share of the visible
// Gaussians into an LDS copy of the grid and stores it to its own slot;
// k_tile_counts adds the slots.
__global__ __launch_bounds__(1024) void k_tile_diff(const uint32_t* __restrict__ didx,
                                                    const uint16_t* __restrict__ rect,
                                                    const uint64_t* counts, int gw, int cells,
                                                    int* __restrict__ parts) {
  extern __shared__ int s_grid[];
  for (int c = threadIdx.x; c < cells; c += 1024) s_grid[c] = 0;
  __syncthreads();
  const uint64_t nvis = counts[0];
  const uint64_t per = (nvis + gridDim.x - 1) / gridDim.x;
  const uint64_t beg = (uint64_t)blockIdx.x * per;
  const uint64_t end = beg + per < nvis ? beg + per : nvis;
  for (uint64_t i = beg + threadIdx.x; i < end; i += 1024) {
    const ushort4 rc = reinterpret_cast<const ushort4*>(rect)[didx[i]];
    atomicAdd(&s_grid[rc.y * gw + rc.x], 1);
    atomicAdd(&s_grid[rc.y * gw + rc.z], -1);
    atomicAdd(&s_grid[rc.w * gw + rc.x], -1);
    atomicAdd(&s_grid[rc.w * gw + rc.z], 1);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < cells; c += 1024) parts[(size_t)blockIdx.x * cells + c] = s_grid[c];
}

// Sum of the per-block difference grids (one lane per grid cell).
__global__ __launch_bounds__(256) void k_diff_sum(const int* __restrict__ parts, int nparts,
                                                  int cells, int* __restrict__ diff) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= cells) return;
  int acc = 0;
#pragma unroll 8
  for (int b = 0; b < nparts; ++b) acc += parts[(size_t)b * cells + c];
  diff[c] = acc;
}

// One block: per-tile instance counts from the difference grid, tile ranges
// [start, end) by an exclusive scan in tile order, and the histograms of the
// tile digits used by the radix passes.  If the instance count overflowed
// the caller's capacity every range is left empty.
__global__ __launch_bounds__(1024) void k_tile_counts(int* __restrict__ diff, int tiles_x,
                                                      int tiles_y, const uint64_t* counts,
                                                      uint32_t* __restrict__ ranges,
                                                      uint32_t* __restrict__ thist, int npass,
                                                      int sh0, int b0, int sh1, int b1, int sh2,
                                                      int b2) {
  __shared__ uint32_t h[3][kRadixBins];
  __shared__ uint32_t s_part[1024];
  const int tid = threadIdx.x;
  const int gw = tiles_x + 1, gh = tiles_y;  // the last grid row is never summed
  const int lane = tid & 63, w = tid >> 6;
  for (int k = tid; k < 3 * kRadixBins; k += 1024) (&h[0][0])[k] = 0;

  // row prefix sums: one wavefront per row, 64 columns at a time
  for (int r = w; r < gh; r += 16) {
    int carry = 0;
    for (int c0 = 0; c0 < gw; c0 += 64) {
      const int c = c0 + lane;
      int x = c < gw ? diff[r * gw + c] : 0;
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
      }
      if (c < gw) diff[r * gw + c] = x + carry;
      carry += __shfl(x, 63, 64);
    }
  }
  __syncthreads();
  // column prefix sums: one lane per column, eight rows in flight
  for (int c = tid; c < gw; c += 1024) {
    int acc = 0;
    for (int r0 = 0; r0 < gh; r0 += 8) {
      int v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = r0 + k < gh ? diff[(r0 + k) * gw + c] : 0;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        acc += v[k];
        if (r0 + k < gh) diff[(r0 + k) * gw + c] = acc;
      }
    }
  }
  __syncthreads();
  const bool over = counts[2] != 0;
  const int T = tiles_x * tiles_y;
  const int chunk = (T + 1023) / 1024;
  const int beg = tid * chunk, end = beg + chunk < T ? beg + chunk : T;
  uint32_t sum = 0;
  for (int t = beg; t < end; ++t) sum += (uint32_t)diff[(t / tiles_x) * gw + (t % tiles_x)];
  s_part[tid] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const uint32_t v = tid >= o ? s_part[tid - o] : 0u;
    __syncthreads();
    s_part[tid] += v;
    __syncthreads();
  }
  uint32_t run = s_part[tid] - sum;
  const int shs[3] = {sh0, sh1, sh2}, bs[3] = {b0, b1, b2};
  for (int t = beg; t < end; ++t) {
    const uint32_t c = (uint32_t)diff[(t / tiles_x) * gw + (t % tiles_x)];
    ranges[2 * (size_t)t] = over ? 0u : run;
    ranges[2 * (size_t)t + 1] = over ? 0u : run + c;
    run += c;
    if (c)
      for (int p = 0; p < npass; ++p) atomicAdd(&h[p][(t >> shs[p]) & ((1 << bs[p]) - 1)], c);
  }
  __syncthreads();
  for (int k = tid; k < npass * kRadixBins; k += 1024) thist[k] = over ? 0u : (&h[0][0])[k];
}

// Exclusive scan of the tile counts of the depth-sorted visible Gaussians
// (single pass, decoupled look-back over partitions of kScanTile).
__global__ __launch_bounds__(kSortBlock) void k_offsets(const uint32_t* __restrict__ didx,
                                                        const uint32_t* __restrict__ n_tiles,
                                                        const uint64_t* counts,
                                                        uint32_t* __restrict__ offs,
                                                        uint32_t* __restrict__ goffs,
                                                        uint32_t* __restrict__ chunk_first,
                                                        uint64_t cap,
                                                        uint64_t* status, uint32_t* part_counter,
                                                        uint64_t* err) {
  __shared__ uint32_t s_scan[4];
  __shared__ uint32_t s_part;
  __shared__ unsigned long long s_base;
  const int tid = threadIdx.x;
  if (tid == 0) s_part = atomicAdd(part_counter, 1u);
  __syncthreads();
  const uint32_t part = s_part;
  const uint64_t nvis = counts[0];
  const uint64_t base_s = (uint64_t)part * kScanTile;
  if (base_s >= nvis) return;
  constexpr int IT = kScanTile / kSortBlock;
  uint32_t c[IT], gi[IT];
  uint32_t tsum = 0;
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const uint64_t sidx = base_s + (uint64_t)tid * IT + k;
    gi[k] = sidx < nvis ? didx[sidx] : 0u;
    c[k] = sidx < nvis ? n_tiles[gi[k]] : 0u;
    tsum += c[k];
  }
  uint32_t total;
  const uint32_t pre = block_excl_scan256(tsum, s_scan, &total);
  if (tid == 0) {
    uint64_t excl = 0;
    if (part == 0) {
      st_rel64(&status[0], kEFlagIncl | total);
    } else {
      st_rel64(&status[part], kEFlagAgg | total);
      int64_t j = (int64_t)part - 1;
      int spins = 0;
      while (j >= 0) {
        const uint64_t st = ld_acq64(&status[j]);
        if ((st & ~kEValMask) == 0) {
          if (++spins > kSpinLimit) {
            atomicOr((unsigned long long*)err, 1ull);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        excl += st & kEValMask;
        if ((st & kEFlagIncl) != 0) break;
        --j;
      }
      st_rel64(&status[part], kEFlagIncl | (excl + total));
    }
    s_base = excl;
  }
  __syncthreads();
  uint32_t run = (uint32_t)s_base + pre;
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const uint64_t sidx = base_s + (uint64_t)tid * IT + k;
    if (sidx < nvis) {
      offs[sidx] = run;
      goffs[gi[k]] = run;
      // this Gaussian owns the first slot of every chunk that starts inside
      // its instance range
      uint64_t cb = ((uint64_t)run + kEmitChunk - 1) / kEmitChunk;
      const uint64_t ce = (uint64_t)run + c[k];
      for (; cb * kEmitChunk < ce && cb * kEmitChunk < cap; ++cb) chunk_first[cb] = (uint32_t)sidx;
    }
    run += c[k];
  }
}

// Global digit histograms of the depth keys for all four passes.
__global__ __launch_bounds__(kSortBlock) void k_hist_depth(const uint32_t* __restrict__ keys,
                                                           const uint64_t* counts,
                                                           uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[4][kRadixBins];
  for (int k = threadIdx.x; k < 4 * kRadixBins; k += kSortBlock) (&h[0][0])[k] = 0;
  __syncthreads();
  const uint64_t n = counts[0];
  const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
  for (int it = 0; it < kSortItems; ++it) {
    const uint64_t i = base + (uint64_t)it * kSortBlock + threadIdx.x;
    if (i < n) {
      const uint32_t k = keys[i];
      atomicAdd(&h[0][k & 255], 1u);
      atomicAdd(&h[1][(k >> 8) & 255], 1u);
      atomicAdd(&h[2][(k >> 16) & 255], 1u);
      atomicAdd(&h[3][(k >> 24) & 255], 1u);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < 4 * kRadixBins; k += kSortBlock) {
    const uint32_t c = (&h[0][0])[k];
    if (c) atomicAdd(&hist[k], c);
  }
}

// ------------------------------------------------------------- onesweep --
// Instance emission in depth order: a Gaussian's tiles, row-major over its
// rectangle, occupy slots [offs[s], offs[s] + n_tiles) of the emission order.
struct EmitArgs {
  const uint32_t* __restrict__ didx;  // depth-sorted visible Gaussians
  const uint32_t* __restrict__ offs;  // exclusive instance offsets
  const uint32_t* __restrict__ chunk_first;  // owner of each chunk's first slot
  const uint64_t* counts;
  const uint16_t* __restrict__ rect;
  int tiles_x;
  uint32_t tile_base;
  uint64_t cap;
  uint32_t* __restrict__ tkey;
  uint32_t* __restrict__ tval;
};

// Enumerate emission slots [c0, c1) as (tile id, Gaussian index) pairs into
// out_key/out_val[k - c0]: find the depth-sorted Gaussians covering the
// slots by binary search over the offsets, stage windows of 256 of them in
// LDS, and map each slot to its Gaussian and tile.  Called by every thread
// of a 256-thread block.
__device__ __forceinline__ void emit_range(const EmitArgs& a, uint64_t c0, uint64_t c1,
                                           uint32_t* out_key, uint32_t* out_val,
                                           uint32_t* s_off, uint32_t* s_g, uint32_t* s_x0,
                                           uint32_t* s_y0, uint32_t* s_w, uint32_t* s_lohi) {
  const int tid = threadIdx.x;
  const uint64_t nvis = a.counts[0];
  const uint64_t ninst = a.counts[1];
  if (tid == 0) chunk_bounds(a.chunk_first, a.offs, nvis, ninst, c0, c1, s_lohi);
  __syncthreads();
  const uint32_t slo = s_lohi[0], shi = s_lohi[1];
  for (uint32_t w0 = slo; w0 <= shi; w0 += kSortBlock) {
    const uint32_t wn = (shi - w0 + 1) < (uint32_t)kSortBlock ? (shi - w0 + 1) : (uint32_t)kSortBlock;
    if ((uint32_t)tid < wn) {
      const uint32_t sidx = w0 + tid;
      const uint32_t g = a.didx[sidx];
      const ushort4 rc = reinterpret_cast<const ushort4*>(a.rect)[g];
      s_off[tid] = a.offs[sidx];
      s_g[tid] = g;
      s_x0[tid] = rc.x, s_y0[tid] = rc.y, s_w[tid] = (uint32_t)rc.z - rc.x;
    }
    if (tid == 0) {
      const uint64_t e = (uint64_t)w0 + wn < nvis ? (uint64_t)a.offs[w0 + wn] : ninst;
      s_off[wn] = (uint32_t)(e < c1 ? e : c1);
    }
    __syncthreads();
    const uint64_t k0 = (uint64_t)s_off[0] > c0 ? (uint64_t)s_off[0] : c0;
    const uint64_t k1 = s_off[wn];
    // each thread takes a run of consecutive slots (odd length, so the LDS
    // writes of a wavefront fall in distinct banks); one search and one
    // division per run, then the tile index advances row-major
    const uint32_t run = ((uint32_t)(k1 - k0) + kSortBlock - 1) / kSortBlock | 1u;
    uint64_t k = k0 + (uint64_t)tid * run;
    const uint64_t kend = k + run < k1 ? k + run : k1;
    if (k < kend) {
      int j = 0, hi = (int)wn - 1;  // largest j with s_off[j] <= k
      while (j < hi) {
        const int mid = (j + hi + 1) >> 1;
        if (s_off[mid] <= k) j = mid; else hi = mid - 1;
      }
      uint32_t wj = s_w[j];
      const uint32_t r = (uint32_t)(k - s_off[j]);
      uint32_t ty = r / wj, tx = r - ty * wj;
      for (; k < kend; ++k) {
        if (k == s_off[j + 1]) {
          ++j;
          wj = s_w[j], tx = 0, ty = 0;
        }
        out_key[k - c0] = a.tile_base + (s_y0[j] + ty) * (uint32_t)a.tiles_x + s_x0[j] + tx;
        out_val[k - c0] = s_g[j];
        if (++tx == wj) tx = 0, ++ty;
      }
    }
    __syncthreads();
  }
}
struct SweepArgs {
  const uint32_t* __restrict__ keys_in;
  const uint32_t* __restrict__ vals_in;
  uint32_t* __restrict__ keys_out;
  uint32_t* __restrict__ vals_out;
  const uint64_t* count;
  uint64_t cap;
  const uint64_t* skip;  // if non-null and *skip != 0, the pass sorts nothing
  int shift, bits;
  const uint32_t* __restrict__ hist;
  uint32_t* status;
  uint32_t* part_counter;
  uint64_t* err;
  uint64_t* __restrict__ keys64_out;  // final tile pass: tile<<32 | depth bits
  const float* __restrict__ rec;
};

// FROM_EMIT: the pass reads no input array; each partition enumerates its
// kSortTile emission slots itself (fusing the emission into the first tile
// pass).
template <bool FROM_EMIT>
__global__ __launch_bounds__(kSortBlock) void k_onesweep(SweepArgs a, EmitArgs em) {
  __shared__ uint32_t s_keys[kSortTile];
  __shared__ uint32_t s_vals[kSortTile];
  // per-wave digit counters, then destinations and local offsets; the emit
  // staging arrays of the fused pass live in the same words before ranking
  __shared__ uint32_t s_aux[6 * kRadixBins + 8];
  uint32_t(*s_wh)[kRadixBins] = reinterpret_cast<uint32_t(*)[kRadixBins]>(s_aux);
  uint32_t* s_dst = s_aux + 4 * kRadixBins;
  uint32_t* s_loc = s_aux + 5 * kRadixBins;
  __shared__ uint32_t s_scan[4];
  __shared__ uint32_t s_part;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  uint64_t n64 = *a.count;
  if (n64 > a.cap) n64 = a.cap;
  if (a.skip && *a.skip != 0) n64 = 0;
  const uint32_t n = (uint32_t)n64;
  if (tid == 0) s_part = atomicAdd(a.part_counter, 1u);
  __syncthreads();
  const uint32_t part = s_part;
  const uint64_t base = (uint64_t)part * kSortTile;
  if (base >= n) return;
  const uint32_t tile_n = (n - base) < (uint64_t)kSortTile ? (uint32_t)(n - base) : (uint32_t)kSortTile;
  const uint32_t dmask = (1u << a.bits) - 1u;
  if (FROM_EMIT)  // ends with a barrier, after which the staging words are free
    emit_range(em, base, base + tile_n, s_keys, s_vals, s_aux, s_aux + 257, s_aux + 513,
               s_aux + 769, s_aux + 1025, s_aux + 1281);
  for (int k = tid; k < 4 * kRadixBins; k += kSortBlock) s_aux[k] = 0;
  __syncthreads();

  uint32_t k[kSortItems], v[kSortItems], rk[kSortItems], dg[kSortItems];
  if (FROM_EMIT) {
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
      const uint32_t idx = (uint32_t)w * (kSortTile / 4) + it * 64 + lane;
      const bool valid = idx < tile_n;
      k[it] = valid ? s_keys[idx] : 0u;
      v[it] = valid ? s_vals[idx] : 0u;
    }
  } else {
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
      const uint32_t idx = (uint32_t)w * (kSortTile / 4) + it * 64 + lane;
      const bool valid = idx < tile_n;
      k[it] = valid ? a.keys_in[base + idx] : 0u;
      v[it] = valid ? a.vals_in[base + idx] : 0u;
    }
  }
  const uint64_t lt_mask = (1ull << lane) - 1ull;
#pragma unroll
  for (int it = 0; it < kSortItems; ++it) {
    const uint32_t idx = (uint32_t)w * (kSortTile / 4) + it * 64 + lane;
    const bool valid = idx < tile_n;
    const uint32_t d = (k[it] >> a.shift) & dmask;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < a.bits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const uint64_t lower = peers & lt_mask;
    uint32_t pre = 0;
    if (valid) pre = s_wh[w][d];
    if (valid && lower == 0) s_wh[w][d] = pre + (uint32_t)__popcll(peers);
    rk[it] = pre + (uint32_t)__popcll(lower);
    dg[it] = valid ? d : 0xFFFFFFFFu;
  }
  __syncthreads();
  // per digit: wave offsets, block total, block-local offsets
  const uint32_t d = tid;
  const uint32_t c0 = s_wh[0][d], c1 = s_wh[1][d], c2 = s_wh[2][d], c3 = s_wh[3][d];
  const uint32_t tot = c0 + c1 + c2 + c3;
  if (part == 0)
    st_rel(&a.status[d], kFlagIncl | tot);
  else
    st_rel(&a.status[(size_t)part * kRadixBins + d], kFlagAgg | tot);
  __syncthreads();
  s_wh[0][d] = 0, s_wh[1][d] = c0, s_wh[2][d] = c0 + c1, s_wh[3][d] = c0 + c1 + c2;
  const uint32_t loc = block_excl_scan256(tot, s_scan, nullptr);
  const uint32_t gex = block_excl_scan256(a.hist[d], s_scan, nullptr);
  s_loc[d] = loc;
  // decoupled look-back over earlier partitions for this digit
  uint32_t excl = 0;
  if (part > 0) {
    int64_t j = (int64_t)part - 1;
    int spins = 0;
    while (j >= 0) {
      const uint32_t s = ld_acq(&a.status[(size_t)j * kRadixBins + d]);
      if ((s & ~kValMask) == 0) {
        if (++spins > kSpinLimit) {
          atomicOr((unsigned long long*)a.err, 1ull);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      excl += s & kValMask;
      if ((s & kFlagIncl) != 0) break;
      --j;
    }
    st_rel(&a.status[(size_t)part * kRadixBins + d], kFlagIncl | ((excl + tot) & kValMask));
  }
  s_dst[d] = gex + excl - loc;
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kSortItems; ++it) {
    if (dg[it] != 0xFFFFFFFFu) {
      const uint32_t pos = s_loc[dg[it]] + s_wh[w][dg[it]] + rk[it];
      if (pos < (uint32_t)kSortTile) {
        s_keys[pos] = k[it];
        s_vals[pos] = v[it];
      }
    }
  }
  __syncthreads();
  for (uint32_t i = tid; i < tile_n; i += kSortBlock) {
    const uint32_t key = s_keys[i];
    const uint32_t val = s_vals[i];
    const uint32_t o = s_dst[(key >> a.shift) & dmask] + i;
    if (o >= n) continue;  // only reachable if the counts were inconsistent
    if (a.keys_out) a.keys_out[o] = key;
    a.vals_out[o] = val;
    if (a.keys64_out)
      a.keys64_out[o] = ((uint64_t)key << 32) | __float_as_uint(a.rec[(size_t)val * kRecFloats + 9]);
  }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
  const uint64_t stride = (uint64_t)gridDim.x * 256 * 4;
  for (uint64_t i = ((uint64_t)blockIdx.x * 256 + threadIdx.x) * 4; i < n; i += stride) {
    if (i + 4 <= n && ((reinterpret_cast<uintptr_t>(p + i) & 15) == 0)) {
      *reinterpret_cast<uint4*>(p + i) = make_uint4(v, v, v, v);
    } else {
      for (uint64_t j = i; j < i + 4 && j < n; ++j) p[j] = v;
    }
  }
}

hipError_t launch_fill(uint32_t* p, int64_t n, uint32_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n / 4 + 255) / 256 + 1;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, (uint64_t)n, v);
  return hipGetLastError();
}

static int bit_width(uint64_t v) {
  int b = 0;
  while ((1ull << b) < v) ++b;
  return b < 1 ? 1 : b;
}

hipError_t launch_sort(const sx_projected& proj, int64_t n, const KParams& p,
                       int64_t capacity, int64_t tiles_total, uint64_t* keys,
                       uint32_t* vals, uint32_t* ranges, char* ws,
                       uint64_t* h_counts, bool* over_capacity,
                       hipStream_t st) {
  *over_capacity = false;
  const SortLayout L = sort_layout(n, capacity, tiles_total);
  hipError_t e;
  auto u32 = [&](size_t off) { return reinterpret_cast<uint32_t*>(ws + off); };
  uint64_t* counts = reinterpret_cast<uint64_t*>(ws + L.counts);
  if ((e = launch_fill(u32(L.zero_begin), (int64_t)((L.zero_end - L.zero_begin) / 4), 0, st))) return e;
  if (n == 0) {
    if ((e = launch_fill(ranges, tiles_total * 2, 0, st))) return e;
    if (h_counts) h_counts[0] = h_counts[1] = 0;
    return hipSuccess;
  }
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, proj.block_sums, (int64_t)L.nb,
                     u32(L.vis_off), counts, (int64_t)capacity);
  if ((e = hipGetLastError())) return e;
  if (h_counts) {
    uint64_t c[2];
    if ((e = hipMemcpyAsync(c, counts, sizeof(c), hipMemcpyDeviceToHost, st))) return e;
    if ((e = hipStreamSynchronize(st))) return e;
    h_counts[0] = c[0];
    h_counts[1] = c[1];
    if (c[1] > (uint64_t)capacity) {
      *over_capacity = true;
      return hipSuccess;
    }
  }
  const int gw = p.tiles_x + 1;
  const int cells = gw * (p.tiles_y + 1);
  const bool lds_diff = cells <= kDiffMaxCells;
  int* diff = reinterpret_cast<int*>(ws + L.diff);
  int* dparts = reinterpret_cast<int*>(ws + L.diffparts);
  hipLaunchKernelGGL(k_compact, dim3((unsigned)L.nb), dim3(kPreBlock), 0, st, proj.n_tiles,
                     proj.rec, proj.rect, n, u32(L.vis_off), u32(L.dkey[0]), u32(L.didx[0]),
                     diff, gw, lds_diff ? 0 : 1);
  if (lds_diff) {
    hipLaunchKernelGGL(k_tile_diff, dim3(kDiffParts), dim3(1024), (size_t)cells * 4, st,
                       u32(L.didx[0]), proj.rect, counts, gw, cells, dparts);
    hipLaunchKernelGGL(k_diff_sum, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, st,
                       (const int*)dparts, kDiffParts, cells, diff);
  }
  // tile digits: ceil(bits/8) balanced passes
  const int tbits = bit_width((uint64_t)tiles_total);
  const int npass = (tbits + 7) / 8;
  int shs[3] = {0, 0, 0}, bs[3] = {1, 1, 1};
  {
    int sh = 0;
    for (int k = 0; k < npass; ++k) {
      bs[k] = tbits / npass + (k < tbits % npass ? 1 : 0);
      shs[k] = sh;
      sh += bs[k];
    }
  }
  hipLaunchKernelGGL(k_tile_counts, dim3(1), dim3(1024), 0, st, diff, p.tiles_x, p.tiles_y,
                     counts, ranges, u32(L.thist), npass, shs[0], bs[0], shs[1], bs[1], shs[2],
                     bs[2]);
  hipLaunchKernelGGL(k_hist_depth, dim3((unsigned)L.dparts), dim3(kSortBlock), 0, st,
                     u32(L.dkey[0]), counts, u32(L.dhist));
  uint32_t* counters = u32(L.counters);
  uint64_t* err = counts + 3;
  // depth digits: bits 0..30 (depth > 0, sign bit clear) in 8,8,8,7
  for (int ps = 0; ps < 4; ++ps) {
    SweepArgs a{};
    a.keys_in = u32(L.dkey[ps & 1]);
    a.vals_in = u32(L.didx[ps & 1]);
    a.keys_out = u32(L.dkey[(ps + 1) & 1]);
    a.vals_out = u32(L.didx[(ps + 1) & 1]);
    a.count = counts;
    a.cap = (uint64_t)n;
    a.skip = nullptr;
    a.shift = 8 * ps;
    a.bits = ps == 3 ? 7 : 8;
    a.hist = u32(L.dhist) + ps * kRadixBins;
    a.status = u32(L.dstatus) + (size_t)ps * L.dparts * kRadixBins;
    a.part_counter = counters + ps;
    a.err = err;
    hipLaunchKernelGGL(k_onesweep<false>, dim3((unsigned)L.dparts), dim3(kSortBlock), 0, st, a,
                       EmitArgs{});
  }
  hipLaunchKernelGGL(k_offsets, dim3((unsigned)L.eparts), dim3(kSortBlock), 0, st,
                     u32(L.didx[0]), proj.n_tiles, counts, u32(L.offs), u32(L.goffs),
                     u32(L.chunk_first), (uint64_t)capacity,
                     reinterpret_cast<uint64_t*>(ws + L.estatus), counters + 4, err);
  EmitArgs em{};
  em.didx = u32(L.didx[0]);
  em.offs = u32(L.offs);
  em.chunk_first = u32(L.chunk_first);
  em.counts = counts;
  em.rect = proj.rect;
  em.tiles_x = p.tiles_x;
  em.tile_base = 0;
  for (int ps = 0; ps < npass; ++ps) {
    const bool last = ps == npass - 1;
    SweepArgs a{};
    a.keys_in = u32(L.tkey[ps & 1]);
    a.vals_in = u32(L.tval[ps & 1]);
    a.keys_out = last ? nullptr : u32(L.tkey[(ps + 1) & 1]);
    a.vals_out = last ? vals : u32(L.tval[(ps + 1) & 1]);
    a.count = counts + 1;
    a.cap = (uint64_t)capacity;
    a.skip = counts + 2;
    a.shift = shs[ps];
    a.bits = bs[ps];
    a.hist = u32(L.thist) + ps * kRadixBins;
    a.status = u32(L.tstatus) + (size_t)ps * L.tparts * kRadixBins;
    a.part_counter = counters + 5 + ps;
    a.err = err;
    a.keys64_out = last ? keys : nullptr;
    a.rec = proj.rec;
    if (ps == 0)
      hipLaunchKernelGGL(k_onesweep<true>, dim3((unsigned)L.tparts), dim3(kSortBlock), 0, st, a, em);
    else
      hipLaunchKernelGGL(k_onesweep<false>, dim3((unsigned)L.tparts), dim3(kSortBlock), 0, st, a,
                         em);
  }
  return hipGetLastError();
}

}  // namespace sx
