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

SortLayout sort_layout(int64_t n, int64_t cap) {
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
  L.eparts = (n + kSortBlock - 1) / kSortBlock;
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
  L.zero_end = off;
  L.vis_off = take((size_t)(L.nb > 0 ? L.nb : 1) * 4);
  for (int k = 0; k < 2; ++k) L.dkey[k] = take((size_t)(n > 0 ? n : 1) * 4);
  for (int k = 0; k < 2; ++k) L.didx[k] = take((size_t)(n > 0 ? n : 1) * 4);
  for (int k = 0; k < 2; ++k) L.tkey[k] = take((size_t)(cap > 0 ? cap : 1) * 4);
  for (int k = 0; k < 2; ++k) L.tval[k] = take((size_t)(cap > 0 ? cap : 1) * 4);
  L.tsorted = take((size_t)(cap > 0 ? cap : 1) * 4);
  L.total = off;
  return L;
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
__global__ __launch_bounds__(kPreBlock) void k_compact(const uint32_t* __restrict__ n_tiles,
                                                       const float* __restrict__ rec, int64_t n,
                                                       const uint32_t* __restrict__ vis_off,
                                                       uint32_t* __restrict__ dkey,
                                                       uint32_t* __restrict__ didx) {
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
struct SweepArgs {
  const uint32_t* __restrict__ keys_in;
  const uint32_t* __restrict__ vals_in;
  uint32_t* __restrict__ keys_out;
  uint32_t* __restrict__ vals_out;
  const uint64_t* count;
  uint64_t cap;
  int shift, bits;
  const uint32_t* __restrict__ hist;
  uint32_t* status;
  uint32_t* part_counter;
  uint64_t* err;
  uint64_t* __restrict__ keys64_out;  // final tile pass: tile<<32 | depth bits
  const float* __restrict__ rec;
};

__global__ __launch_bounds__(kSortBlock) void k_onesweep(SweepArgs a) {
  __shared__ uint32_t s_keys[kSortTile];
  __shared__ uint32_t s_vals[kSortTile];
  __shared__ uint32_t s_wh[4][kRadixBins];
  __shared__ uint32_t s_dst[kRadixBins];
  __shared__ uint32_t s_loc[kRadixBins];
  __shared__ uint32_t s_scan[4];
  __shared__ uint32_t s_part;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  uint64_t n64 = *a.count;
  if (n64 > a.cap) n64 = a.cap;
  const uint32_t n = (uint32_t)n64;
  if (tid == 0) s_part = atomicAdd(a.part_counter, 1u);
  for (int k = tid; k < 4 * kRadixBins; k += kSortBlock) (&s_wh[0][0])[k] = 0;
  __syncthreads();
  const uint32_t part = s_part;
  const uint64_t base = (uint64_t)part * kSortTile;
  if (base >= n) return;
  const uint32_t tile_n = (n - base) < (uint64_t)kSortTile ? (uint32_t)(n - base) : (uint32_t)kSortTile;
  const uint32_t dmask = (1u << a.bits) - 1u;

  uint32_t k[kSortItems], v[kSortItems], rk[kSortItems], dg[kSortItems];
#pragma unroll
  for (int it = 0; it < kSortItems; ++it) {
    const uint32_t idx = (uint32_t)w * (kSortTile / 4) + it * 64 + lane;
    const bool valid = idx < tile_n;
    k[it] = valid ? a.keys_in[base + idx] : 0u;
    v[it] = valid ? a.vals_in[base + idx] : 0u;
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

// ----------------------------------------------------------------- emit --
struct EmitArgs {
  const uint32_t* __restrict__ didx;  // depth-sorted visible Gaussians
  const uint64_t* counts;
  const uint32_t* __restrict__ n_tiles;
  const uint16_t* __restrict__ rect;
  int tiles_x;
  uint32_t tile_base;
  uint64_t cap;
  uint32_t* __restrict__ tkey;
  uint32_t* __restrict__ tval;
  uint32_t* __restrict__ thist;  // [3][256]
  int npass;
  int shift[3], bits[3];
  uint64_t* status;
  uint32_t* part_counter;
  uint64_t* err;
};

__global__ __launch_bounds__(kSortBlock) void k_emit(EmitArgs a) {
  __shared__ uint32_t s_off[kSortBlock + 1];
  __shared__ uint32_t s_g[kSortBlock];
  __shared__ uint32_t s_x0[kSortBlock], s_y0[kSortBlock], s_w[kSortBlock];
  __shared__ uint32_t s_h[3][kRadixBins];
  __shared__ uint32_t s_scan[4];
  __shared__ uint32_t s_part;
  __shared__ unsigned long long s_base;
  const int tid = threadIdx.x;
  if (tid == 0) s_part = atomicAdd(a.part_counter, 1u);
  for (int k = tid; k < 3 * kRadixBins; k += kSortBlock) (&s_h[0][0])[k] = 0;
  __syncthreads();
  const uint32_t part = s_part;
  const uint64_t nvis = a.counts[0];
  const uint64_t s = (uint64_t)part * kSortBlock + tid;
  if ((uint64_t)part * kSortBlock >= nvis) return;
  uint32_t g = 0, cnt = 0, x0 = 0, y0 = 0, wd = 1;
  if (s < nvis) {
    g = a.didx[s];
    cnt = a.n_tiles[g];
    const ushort4 rc = reinterpret_cast<const ushort4*>(a.rect)[g];
    x0 = rc.x, y0 = rc.y, wd = (uint32_t)rc.z - rc.x;
  }
  uint32_t total;
  const uint32_t off = block_excl_scan256(cnt, s_scan, &total);
  s_off[tid] = off, s_g[tid] = g, s_x0[tid] = x0, s_y0[tid] = y0, s_w[tid] = wd;
  if (tid == 0) {
    s_off[kSortBlock] = total;
    uint64_t excl = 0;
    if (part == 0) {
      st_rel64(&a.status[0], kEFlagIncl | total);
    } else {
      st_rel64(&a.status[part], kEFlagAgg | total);
      int64_t j = (int64_t)part - 1;
      int spins = 0;
      while (j >= 0) {
        const uint64_t st = ld_acq64(&a.status[j]);
        if ((st & ~kEValMask) == 0) {
          if (++spins > kSpinLimit) {
            atomicOr((unsigned long long*)a.err, 1ull);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        excl += st & kEValMask;
        if ((st & kEFlagIncl) != 0) break;
        --j;
      }
      st_rel64(&a.status[part], kEFlagIncl | (excl + total));
    }
    s_base = excl;
  }
  __syncthreads();
  const uint64_t base = s_base;
  for (uint32_t k = tid; k < total; k += kSortBlock) {
    int lo = 0, hi = kSortBlock - 1;  // largest j with s_off[j] <= k
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_off[mid] <= k)
        lo = mid;
      else
        hi = mid - 1;
    }
    const uint32_t r = k - s_off[lo];
    const uint32_t wj = s_w[lo];
    const uint32_t ty = r / wj, tx = r - ty * wj;
    const uint32_t tile = a.tile_base + (s_y0[lo] + ty) * (uint32_t)a.tiles_x + s_x0[lo] + tx;
    const uint64_t pos = base + k;
    if (pos < a.cap) {
      a.tkey[pos] = tile;
      a.tval[pos] = s_g[lo];
      for (int p = 0; p < a.npass; ++p)
        atomicAdd(&s_h[p][(tile >> a.shift[p]) & ((1u << a.bits[p]) - 1u)], 1u);
    }
  }
  __syncthreads();
  for (int k = tid; k < a.npass * kRadixBins; k += kSortBlock) {
    const uint32_t c = (&s_h[0][0])[k];
    if (c) atomicAdd(&a.thist[k], c);
  }
}

// --------------------------------------------------------------- ranges --
__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ tiles,
                                                const uint64_t* counts, uint64_t cap,
                                                uint32_t tiles_total,
                                                uint32_t* __restrict__ ranges) {
  uint64_t n = counts[1];
  if (n > cap) n = cap;
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint32_t t = tiles[i];
  if (t >= tiles_total) return;
  if (i == 0 || tiles[i - 1] != t) ranges[2 * (size_t)t] = (uint32_t)i;
  if (i + 1 == n || tiles[i + 1] != t) ranges[2 * (size_t)t + 1] = (uint32_t)(i + 1);
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
  const SortLayout L = sort_layout(n, capacity);
  hipError_t e;
  auto u32 = [&](size_t off) { return reinterpret_cast<uint32_t*>(ws + off); };
  uint64_t* counts = reinterpret_cast<uint64_t*>(ws + L.counts);
  if ((e = launch_fill(u32(L.zero_begin), (int64_t)((L.zero_end - L.zero_begin) / 4), 0, st))) return e;
  if ((e = launch_fill(ranges, tiles_total * 2, 0, st))) return e;
  if (n == 0) {
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
  hipLaunchKernelGGL(k_compact, dim3((unsigned)L.nb), dim3(kPreBlock), 0, st, proj.n_tiles,
                     proj.rec, n, u32(L.vis_off), u32(L.dkey[0]), u32(L.didx[0]));
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
    a.shift = 8 * ps;
    a.bits = ps == 3 ? 7 : 8;
    a.hist = u32(L.dhist) + ps * kRadixBins;
    a.status = u32(L.dstatus) + (size_t)ps * L.dparts * kRadixBins;
    a.part_counter = counters + ps;
    a.err = err;
    hipLaunchKernelGGL(k_onesweep, dim3((unsigned)L.dparts), dim3(kSortBlock), 0, st, a);
  }
  // tile digits
  const int tbits = bit_width((uint64_t)tiles_total);
  const int npass = (tbits + 7) / 8;
  EmitArgs em{};
  em.didx = u32(L.didx[0]);
  em.counts = counts;
  em.n_tiles = proj.n_tiles;
  em.rect = proj.rect;
  em.tiles_x = p.tiles_x;
  em.tile_base = 0;
  em.cap = (uint64_t)capacity;
  em.tkey = u32(L.tkey[0]);
  em.tval = u32(L.tval[0]);
  em.thist = u32(L.thist);
  em.npass = npass;
  {
    int sh = 0;
    for (int k = 0; k < npass; ++k) {
      const int b = tbits / npass + (k < tbits % npass ? 1 : 0);
      em.shift[k] = sh;
      em.bits[k] = b;
      sh += b;
    }
  }
  em.status = reinterpret_cast<uint64_t*>(ws + L.estatus);
  em.part_counter = counters + 4;
  em.err = err;
  hipLaunchKernelGGL(k_emit, dim3((unsigned)L.eparts), dim3(kSortBlock), 0, st, em);
  for (int ps = 0; ps < npass; ++ps) {
    const bool last = ps == npass - 1;
    SweepArgs a{};
    a.keys_in = u32(L.tkey[ps & 1]);
    a.vals_in = u32(L.tval[ps & 1]);
    a.keys_out = last ? u32(L.tsorted) : u32(L.tkey[(ps + 1) & 1]);
    a.vals_out = last ? vals : u32(L.tval[(ps + 1) & 1]);
    a.count = counts + 1;
    a.cap = (uint64_t)capacity;
    a.shift = em.shift[ps];
    a.bits = em.bits[ps];
    a.hist = u32(L.thist) + ps * kRadixBins;
    a.status = u32(L.tstatus) + (size_t)ps * L.tparts * kRadixBins;
    a.part_counter = counters + 5 + ps;
    a.err = err;
    a.keys64_out = last ? keys : nullptr;
    a.rec = proj.rec;
    hipLaunchKernelGGL(k_onesweep, dim3((unsigned)L.tparts), dim3(kSortBlock), 0, st, a);
  }
  const int64_t rb = (capacity + 255) / 256;
  hipLaunchKernelGGL(k_ranges, dim3((unsigned)(rb > 0 ? rb : 1)), dim3(256), 0, st,
                     u32(L.tsorted), counts, (uint64_t)capacity, (uint32_t)tiles_total, ranges);
  return hipGetLastError();
}

}  // namespace sx
