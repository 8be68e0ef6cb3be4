// Depth sort of the instance list (paper, background: sorting step).
//
// The result equals a stable sort of 64-bit keys
//     key = tile_id << 32 | bits(float32 depth)
// over instances emitted in Gaussian-index order, i.e. the order
// (tile, depth bits, Gaussian index).  It is built in two phases:
//   1. the depth digits are radix sorted on the compacted list of visible
//      Gaussians before duplication (4 LSD passes over ~N_vis elements, one
//      "onesweep" kernel each: wave64 ballot ranking, decoupled look-back
//      with bounded waits, LDS reorder for coalesced writes);
//   2. the depth-ordered list is split by tile through a hierarchy of bins
//      (bins of 4^L x 4^L tiles, each bin having 4 x 4 child bins): the
//      list of a bin is cut into segments, and for every segment each of 16
//      wavefronts ballot-filters the entries whose tile rectangle meets its
//      child bin.  A count pass and an exclusive scan give every (segment,
//      child) its output offset, and a write pass stores the entries in
//      order, so each child's list stays depth-ordered and every store is a
//      contiguous run of a wavefront.  The last level's bins are single
//      tiles; their lists are the instance values and the scan gives the
//      tile ranges.
// No step uses atomics on the output; every wait is bounded (a spin limit
// raises an error flag instead of hanging).
#include "sx_internal.h"

namespace sx {

namespace {

constexpr uint32_t kFlagAgg = 1u << 30;
constexpr uint32_t kFlagIncl = 2u << 30;
constexpr uint32_t kValMask = (1u << 30) - 1;
constexpr int kSpinLimit = 1 << 20;
constexpr int kLookback = 8;  // predecessor statuses read per look-back round trip
constexpr int kScanItems = 4;  // preprocess blocks per thread in the count scan
constexpr int kScanTile = 256 * kScanItems;

// Look-back status words: the flag and the count share one 32-bit word, so
// a reader that sees the flag sees its count, and no other memory is
// published through the word (the scattered keys are read by the next
// launch).  Device-scope atomic loads and stores without ordering suffice,
// and they avoid the cache write-back and invalidation an acquire or
// release at device scope costs on a multi-XCD GPU.
__device__ __forceinline__ uint32_t ld_status(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_status(uint32_t* p, uint32_t v) {
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

SortLayout sort_layout(int64_t n, int64_t cap, int64_t tiles_x, int64_t tiles_y) {
  SortLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  L.nb = (n + kPreBlock - 1) / kPreBlock;
  L.dparts = (n + kSortTile - 1) / kSortTile;
  if (L.dparts < 1) L.dparts = 1;
  L.zero_begin = off;
  L.counts = take(4 * sizeof(uint64_t));  // offset 0: part of the ABI
  L.dhist = take(4 * kRadixBins * 4);
  L.counters = take(16 * 4);
  L.dstatus = take((size_t)4 * L.dparts * kRadixBins * 4);
  // binning: levels of 4x4 bins until one bin covers the grid; per level,
  // the children's entry totals (accumulated by the count pass)
  const int64_t big = tiles_x > tiles_y ? tiles_x : tiles_y;
  int levels = 1;
  while ((int64_t(1) << (2 * levels)) < big) ++levels;
  L.bl_levels = levels;
  int64_t tot_words = 0;
  for (int lev = 0; lev < levels; ++lev) {
    const int64_t side = int64_t(1) << (2 * lev);
    tot_words += ((tiles_x + side - 1) / side) * ((tiles_y + side - 1) / side);
  }
  L.bl_tot = take((size_t)tot_words * 4);
  L.zero_end = off;
  L.vis_off = take((size_t)(L.nb > 0 ? L.nb : 1) * 4);
  L.inst_off = take((size_t)(L.nb > 0 ? L.nb : 1) * 4);
  L.ioff = take((size_t)(n > 0 ? n : 1) * 4);
  L.scan_part = take((size_t)((L.nb + kScanTile - 1) / kScanTile + 1) * 16);
  for (int k = 0; k < 2; ++k) L.dkey[k] = take((size_t)(n > 0 ? n : 1) * 4);
  for (int k = 0; k < 2; ++k) L.didx[k] = take((size_t)(n > 0 ? n : 1) * 4);
  L.vidx = take((size_t)(n > 0 ? n : 1) * 4);
  // every entry of an inner level is a (Gaussian, bin) pair with at least
  // one instance in the bin, so an inner list never exceeds the instance count
  const int64_t bins = ((tiles_x + 3) / 4) * ((tiles_y + 3) / 4);
  const size_t list_bytes = (size_t)(cap > 0 ? cap : 1) * 4;
  L.bl_list[1] = levels >= 2 ? take(list_bytes) : off;  // level 1 writes list[1]
  L.bl_list[0] = levels >= 3 ? take(list_bytes) : off;
  for (int k = 0; k < 2; ++k) L.bl_bins[k] = take((size_t)(bins + 1) * 8);
  for (int k = 0; k < 2; ++k) L.bl_seg[k] = take((size_t)(bins + 2) * 4);
  L.bl_cnt = take((size_t)(cap / kBinSeg + bins + 2) * 16 * 4);
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
  const size_t c = (size_t)(cap > 0 ? cap : 1);
  const size_t t = (size_t)(tiles_total > 0 ? tiles_total : 1);
  L.nv = take(t * 4);
  L.rows = take(c * kRowFloats * 4);
  L.total = off;
  return L;
}

SortView sort_view(const void* ws, int64_t n, int64_t capacity, int64_t tiles_x, int64_t tiles_y) {
  const SortLayout L = sort_layout(n, capacity, tiles_x, tiles_y);
  const char* b = static_cast<const char*>(ws);
  SortView v;
  v.counts = reinterpret_cast<const uint64_t*>(b + L.counts);
  v.didx = reinterpret_cast<const uint32_t*>(b + L.didx[0]);
  v.vidx = reinterpret_cast<const uint32_t*>(b + L.vidx);
  v.ioff = reinterpret_cast<const uint32_t*>(b + L.ioff);
  return v;
}

// ------------------------------------------------------------- counting --
// Exclusive scan of the per-preprocess-block visible counts and the total
// instance count, in two launches over tiles of kScanTile blocks: per-tile
// sums, then every tile adds the sums of the tiles before it.
__device__ __forceinline__ uint64_t block_sum256_u64(uint64_t v, unsigned long long* s4) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if (lane == 0) s4[w] = v;
  __syncthreads();
  return s4[0] + s4[1] + s4[2] + s4[3];
}

__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t* __restrict__ bsum, int64_t nb,
                                                     uint64_t* __restrict__ part) {
  __shared__ unsigned long long s4[4];
  const int64_t b0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint64_t sv = 0, si = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j)
    if (b0 + j < nb) {
      sv += bsum[2 * (b0 + j)];
      si += bsum[2 * (b0 + j) + 1];
    }
  sv = block_sum256_u64(sv, s4);
  si = block_sum256_u64(si, s4);
  if (threadIdx.x == 0) part[2 * blockIdx.x] = sv, part[2 * blockIdx.x + 1] = si;
}

__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t* __restrict__ bsum, int64_t nb,
                                                    const uint64_t* __restrict__ part,
                                                    uint32_t* __restrict__ vis_off,
                                                    uint32_t* __restrict__ inst_off,
                                                    uint64_t* counts, int64_t cap,
                                                    uint2* __restrict__ root_bin,
                                                    uint32_t* __restrict__ root_seg) {
  __shared__ unsigned long long s4[4];
  __shared__ uint32_t s_scan[4];
  const bool last = blockIdx.x == gridDim.x - 1;
  // visible and instance sums of the earlier tiles; the last tile also
  // sums the instances of all tiles
  uint64_t pv = 0, pib = 0, pi = 0;
  for (uint32_t k = threadIdx.x; k < (last ? gridDim.x : blockIdx.x); k += 256) {
    if (k < blockIdx.x) pv += part[2 * k], pib += part[2 * k + 1];
    pi += part[2 * k + 1];
  }
  pv = block_sum256_u64(pv, s4);
  pib = block_sum256_u64(pib, s4);
  if (last) pi = block_sum256_u64(pi, s4);
  const int64_t b0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems], iv[kScanItems];
  uint32_t tsum = 0, isum = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = b0 + j < nb ? bsum[2 * (b0 + j)] : 0u;
    iv[j] = b0 + j < nb ? bsum[2 * (b0 + j) + 1] : 0u;
    tsum += v[j];
    isum += iv[j];
  }
  uint32_t total;
  uint32_t run = (uint32_t)pv + block_excl_scan256(tsum, s_scan, &total);
  // instance offsets: exact while the instances fit the 2^31 capacity bound
  uint32_t irun = (uint32_t)pib + block_excl_scan256(isum, s_scan, nullptr);
#pragma unroll
  for (int j = 0; j < kScanItems; ++j)
    if (b0 + j < nb) {
      vis_off[b0 + j] = run;
      inst_off[b0 + j] = irun;
      run += v[j];
      irun += iv[j];
    }
  if (last && threadIdx.x == 0) {
    const bool over = pi > (uint64_t)cap;
    counts[0] = pv + total;
    counts[1] = pi;
    counts[2] = over ? 1ull : 0ull;
    // the root of the binning: one bin holding every visible Gaussian in
    // depth order (none when the instances overflow the buffer)
    const uint32_t nvis = over ? 0u : (uint32_t)(pv + total);
    root_bin[0] = make_uint2(0u, nvis);
    root_seg[0] = 0;
    root_seg[1] = (nvis + kBinSeg - 1) / kBinSeg;
  }
}

// Compacted (depth bits, Gaussian index) list of visible Gaussians in index
// order.  The index list stays untouched by the depth passes (the first one
// reads it): the backward walks the visible Gaussians in this order, where
// neighbouring lanes read neighbouring parameter rows.
// Also gives every visible Gaussian the offset of its first (Gaussian, tile)
// instance in index order, ioff[i]: the backward stores the gradient row of
// instance (i, tile) at ioff[i] + the tile's raster position in i's tile
// rectangle, so that each Gaussian's rows are contiguous.
__global__ __launch_bounds__(kPreBlock) void k_compact(const uint32_t* __restrict__ n_tiles,
                                                       const float* __restrict__ rec, int64_t n,
                                                       const uint32_t* __restrict__ vis_off,
                                                       const uint32_t* __restrict__ inst_off,
                                                       uint32_t* __restrict__ dkey,
                                                       uint32_t* __restrict__ didx,
                                                       uint32_t* __restrict__ ioff) {
  static_assert(kPreBlock == 256, "the instance scan is a 256-lane block scan");
  __shared__ uint32_t sw[kPreBlock / 64];
  __shared__ uint32_t s_scan[4];
  const int64_t i = (int64_t)blockIdx.x * kPreBlock + threadIdx.x;
  const uint32_t nt = i < n ? n_tiles[i] : 0u;
  const bool v = nt > 0;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t b = __ballot(v);
  const uint32_t rank = __popcll(b & ((1ull << lane) - 1));
  if (lane == 0) sw[w] = __popcll(b);
  const uint32_t iex = block_excl_scan256(nt, s_scan, nullptr);  // synchronises
  uint32_t pre = 0;
  for (int k = 0; k < w; ++k) pre += sw[k];
  if (v) {
    const uint32_t pos = vis_off[blockIdx.x] + pre + rank;
    dkey[pos] = __float_as_uint(rec[(size_t)i * kRecFloats + 9]);
    didx[pos] = (uint32_t)i;
    ioff[i] = inst_off[blockIdx.x] + iex;
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
  // reduce-then-scan form: status holds, digit-major with row length
  // pstride, each partition's first output position per digit (no look-back)
  int offsets;
  uint32_t pstride;
};

// Reduce-then-scan form of a pass, used when there are many partitions (a
// look-back chain grows with the partition count): every partition's digit
// counts, then per digit a scan over the partitions, then the scatter of
// k_onesweep with those positions.
__device__ __forceinline__ uint32_t sweep_n(const SweepArgs& a) {
  uint64_t n64 = *a.count;
  if (n64 > a.cap) n64 = a.cap;
  return (uint32_t)n64;
}

__global__ __launch_bounds__(kSortBlock) void k_part_hist(SweepArgs a) {
  __shared__ uint32_t h[kRadixBins];
  const uint32_t n = sweep_n(a);
  const uint32_t parts = (n + kSortTile - 1) / kSortTile;
  const uint32_t dmask = (1u << a.bits) - 1u;
  for (uint32_t part = blockIdx.x; part < parts; part += gridDim.x) {
    __syncthreads();
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)part * kSortTile;
    for (uint32_t i = threadIdx.x; i < (uint32_t)kSortTile; i += kSortBlock)
      if (base + i < n) atomicAdd(&h[(a.keys_in[base + i] >> a.shift) & dmask], 1u);
    __syncthreads();
    a.status[(size_t)threadIdx.x * a.pstride + part] = h[threadIdx.x];
  }
}

// One block per digit: the digit's global start (the counts of smaller
// digits) plus an exclusive scan of its per-partition counts.
__global__ __launch_bounds__(kSortBlock) void k_part_scan(SweepArgs a) {
  __shared__ uint32_t s4[4];
  __shared__ uint32_t s_tot;
  const uint32_t n = sweep_n(a);
  const uint32_t parts = (n + kSortTile - 1) / kSortTile;
  const uint32_t d = blockIdx.x;
  uint32_t gtot;
  const uint32_t gex = block_excl_scan256(a.hist[threadIdx.x], s4, &gtot);
  if (threadIdx.x == d) s_tot = gex;
  __syncthreads();
  uint32_t run = s_tot;
  uint32_t* row = a.status + (size_t)d * a.pstride;
  for (uint32_t p0 = 0; p0 < parts; p0 += kSortBlock) {
    const uint32_t p = p0 + threadIdx.x;
    const uint32_t c = p < parts ? row[p] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan256(c, s4, &tot);
    if (p < parts) row[p] = run + ex;
    run += tot;
  }
}

// One stable LSD pass over `bits` digits at `shift` of the keys.  Blocks
// take partitions from an atomic counter until none is left, so a partition
// only waits (in the look-back) on partitions that running blocks hold.
__global__ __launch_bounds__(kSortBlock) void k_onesweep(SweepArgs a) {
  __shared__ uint32_t s_keys[kSortTile];
  __shared__ uint32_t s_vals[kSortTile];
  // per-wave digit counters, then destinations and local offsets
  __shared__ uint32_t s_aux[6 * kRadixBins + 8];
  uint32_t(*s_wh)[kRadixBins] = reinterpret_cast<uint32_t(*)[kRadixBins]>(s_aux);
  uint32_t* s_dst = s_aux + 4 * kRadixBins;
  uint32_t* s_loc = s_aux + 5 * kRadixBins;
  __shared__ uint32_t s_scan[4];
  __shared__ uint32_t s_part;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint32_t n = sweep_n(a);
  for (;;) {
  __syncthreads();  // the previous partition is fully written out
  if (tid == 0) s_part = atomicAdd(a.part_counter, 1u);
  __syncthreads();
  const uint32_t part = s_part;
  const uint64_t base = (uint64_t)part * kSortTile;
  if (base >= n) return;
  const uint32_t tile_n = (n - base) < (uint64_t)kSortTile ? (uint32_t)(n - base) : (uint32_t)kSortTile;
  const uint32_t dmask = (1u << a.bits) - 1u;
  for (int k = tid; k < 4 * kRadixBins; k += kSortBlock) s_aux[k] = 0;
  __syncthreads();

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
  if (!a.offsets) {
    if (part == 0)
      st_status(&a.status[d], kFlagIncl | tot);
    else
      st_status(&a.status[(size_t)part * kRadixBins + d], kFlagAgg | tot);
  }
  __syncthreads();
  s_wh[0][d] = 0, s_wh[1][d] = c0, s_wh[2][d] = c0 + c1, s_wh[3][d] = c0 + c1 + c2;
  const uint32_t loc = block_excl_scan256(tot, s_scan, nullptr);
  const uint32_t gex =
      a.offsets ? a.status[(size_t)d * a.pstride + part] : block_excl_scan256(a.hist[d], s_scan, nullptr);
  s_loc[d] = loc;
  // decoupled look-back over earlier partitions for this digit, reading a
  // window of kLookback predecessors per round trip: their sum is taken down
  // to the nearest inclusive prefix; a predecessor not yet published ends
  // the window and is waited for (bounded spin)
  uint32_t excl = 0;
  if (!a.offsets && part > 0) {
    int64_t j = (int64_t)part - 1;
    int spins = 0;
    while (j >= 0) {
      uint32_t st[kLookback];
#pragma unroll
      for (int q = 0; q < kLookback; ++q)
        st[q] = j - q >= 0 ? ld_status(&a.status[(size_t)(j - q) * kRadixBins + d]) : kFlagIncl;
      bool stop = false;
      int used = 0;
#pragma unroll
      for (int q = 0; q < kLookback; ++q) {
        if (stop) continue;
        if ((st[q] & ~kValMask) == 0) {  // not published yet: wait on it
          stop = true;
          continue;
        }
        excl += st[q] & kValMask;
        ++used;
        if ((st[q] & kFlagIncl) != 0) {
          stop = true;
          j = -1;  // done
        }
      }
      if (j < 0) break;
      j -= used;
      if (used == 0) {
        if (++spins > kSpinLimit) {
          atomicOr((unsigned long long*)a.err, 1ull);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    st_status(&a.status[(size_t)part * kRadixBins + d], kFlagIncl | ((excl + tot) & kValMask));
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
    a.keys_out[o] = key;
    a.vals_out[o] = val;
  }
  }
}

// ------------------------------------------------------------ binning --
// One level of the tile hierarchy: parents are bins of 4*side x 4*side
// tiles (grid pgx x pgy, lists in `in`), children bins of side x side
// (grid cgx x cgy).  Child (cx, cy) belongs to parent (cx/4, cy/4) at slot
// (cy%4)*4 + cx%4.  Parent lists are cut into segments of kBinSeg entries;
// pseg[p] is the first segment of parent p and pseg[nparents] the total.
struct BinLevel {
  const uint32_t* __restrict__ in;
  const uint2* __restrict__ pbins;   // (start, length) per parent
  const uint32_t* __restrict__ pseg;
  int pgx, pgy, cgx, cgy, side, tiles_x, tiles_y;
  const uint16_t* __restrict__ rect;
  const uint64_t* counts;
  uint32_t* __restrict__ cnt;   // [segments][16]
  uint32_t* __restrict__ tot;   // [children], zeroed before the count pass
  uint2* __restrict__ cbins;    // (start, length) per child (inner levels)
  uint32_t* __restrict__ cseg;  // segment starts of the children (inner levels)
  uint32_t* __restrict__ out;   // child lists; the instance values at the last level
  uint32_t* __restrict__ ranges;  // last level: [tiles][2]
  uint64_t* __restrict__ keys;    // last level, optional
  const float* __restrict__ rec;
  int last;
  int inline_scan;  // few children: the write pass scans the totals itself
};

// Segment `sg`: its parent, first entry and entry count.
__device__ __forceinline__ int bin_segment(const BinLevel& a, uint32_t sg, uint32_t* lo,
                                           uint32_t* m) {
  int l = 0, h = a.pgx * a.pgy - 1;  // largest p with pseg[p] <= sg
  while (l < h) {
    const int mid = (l + h + 1) >> 1;
    if (a.pseg[mid] <= sg) l = mid; else h = mid - 1;
  }
  const uint2 pb = a.pbins[l];
  const uint32_t off = (sg - a.pseg[l]) * (uint32_t)kBinSeg;
  *lo = pb.x + off;
  const uint32_t rest = pb.y - off;
  *m = rest < (uint32_t)kBinSeg ? rest : (uint32_t)kBinSeg;
  return l;
}

// Tile region of the child bin of parent p at slot w; false if outside.
__device__ __forceinline__ bool bin_child(const BinLevel& a, int p, int w, int* c, int* rx0,
                                          int* rx1, int* ry0, int* ry1) {
  const int cx = (p % a.pgx) * 4 + (w & 3), cy = (p / a.pgx) * 4 + (w >> 2);
  if (cx >= a.cgx || cy >= a.cgy) return false;
  *c = cy * a.cgx + cx;
  *rx0 = cx * a.side, *ry0 = cy * a.side;
  *rx1 = min(*rx0 + a.side, a.tiles_x), *ry1 = min(*ry0 + a.side, a.tiles_y);
  return true;
}

// Stage one segment (Gaussian ids and tile rectangles) in LDS.
__device__ __forceinline__ void bin_stage(const BinLevel& a, uint32_t lo, uint32_t m,
                                          uint32_t* s_g, ushort4* s_rc) {
  __syncthreads();  // the previous segment is consumed
  for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
    const uint32_t g = a.in[lo + i];
    s_g[i] = g;
    s_rc[i] = reinterpret_cast<const ushort4*>(a.rect)[g];
  }
  __syncthreads();
}

__device__ __forceinline__ bool meets(ushort4 rc, int rx0, int rx1, int ry0, int ry1) {
  return (int)rc.x < rx1 && rx0 < (int)rc.z && (int)rc.y < ry1 && ry0 < (int)rc.w;
}

// Count pass: entries of each (segment, child).
__global__ __launch_bounds__(1024) void k_bin_count(BinLevel a) {
  __shared__ uint32_t s_g[kBinSeg];
  __shared__ ushort4 s_rc[kBinSeg];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t nseg = a.pseg[a.pgx * a.pgy];
  for (uint32_t sg = blockIdx.x; sg < nseg; sg += gridDim.x) {
    uint32_t lo, m;
    const int p = bin_segment(a, sg, &lo, &m);
    bin_stage(a, lo, m, s_g, s_rc);
    int c = 0, rx0, rx1, ry0, ry1;
    uint32_t n = 0;
    if (bin_child(a, p, w, &c, &rx0, &rx1, &ry0, &ry1))
      for (uint32_t j = lane; j < (m + 63) / 64 * 64; j += 64) {
        const bool hit = j < m && meets(s_rc[j < m ? j : 0], rx0, rx1, ry0, ry1);
        n += (uint32_t)__popcll(__ballot(hit));
      }
    if (lane == 0) {
      a.cnt[(size_t)sg * 16 + w] = n;
      if (n) atomicAdd(&a.tot[c], n);  // integer sum: the order does not matter
    }
  }
}

// One block: exclusive scan of the children's totals (their list starts;
// tile ranges at the last level) and, for inner levels, of their segment
// counts.
__device__ __forceinline__ void bin_scan(const BinLevel& a, uint32_t* s_a, uint32_t* s_b) {
  const int tid = threadIdx.x;
  const int C = a.cgx * a.cgy;
  const int chunk = (C + 1023) / 1024;
  const int beg = tid * chunk, end = beg + chunk < C ? beg + chunk : C;
  uint32_t sa = 0, sb = 0;
  for (int c = beg; c < end; ++c) {
    const uint32_t t = a.tot[c];
    sa += t;
    sb += (t + kBinSeg - 1) / kBinSeg;
  }
  s_a[tid] = sa, s_b[tid] = sb;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const uint32_t va = tid >= o ? s_a[tid - o] : 0u, vb = tid >= o ? s_b[tid - o] : 0u;
    __syncthreads();
    s_a[tid] += va, s_b[tid] += vb;
    __syncthreads();
  }
  uint32_t ra = s_a[tid] - sa, rb = s_b[tid] - sb;
  for (int c = beg; c < end; ++c) {
    const uint32_t t = a.tot[c];
    if (a.last) {
      a.ranges[2 * (size_t)c] = ra;
      a.ranges[2 * (size_t)c + 1] = ra + t;
    } else {
      a.cbins[c] = make_uint2(ra, t);
      a.cseg[c] = rb;
    }
    ra += t;
    rb += (t + kBinSeg - 1) / kBinSeg;
  }
  if (!a.last && tid == 1023) a.cseg[C] = s_b[1023];
}

// The same scan for up to kScanLds children: the totals are read once,
// coalesced, into LDS, and scanned with wavefront shuffles and one
// cross-wavefront step instead of a barrier per Hillis-Steele round.
constexpr int kScanLds = 8192;

__device__ __forceinline__ void bin_scan_lds(const BinLevel& a, uint32_t* s_t) {
  __shared__ uint32_t s_wa[16], s_wb[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int C = a.cgx * a.cgy;
  for (int c = tid; c < C; c += 1024) s_t[c] = a.tot[c];
  __syncthreads();
  constexpr int chunk = kScanLds / 1024;
  const int beg = tid * chunk, end = beg + chunk < C ? beg + chunk : C;
  uint32_t sa = 0, sb = 0;
  for (int c = beg; c < end; ++c) {
    const uint32_t t = s_t[c];
    sa += t;
    sb += (t + kBinSeg - 1) / kBinSeg;
  }
  uint32_t xa = sa, xb = sb;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t ya = __shfl_up(xa, o, 64), yb = __shfl_up(xb, o, 64);
    if (lane >= o) xa += ya, xb += yb;
  }
  if (lane == 63) s_wa[w] = xa, s_wb[w] = xb;
  __syncthreads();
  uint32_t pa = 0, pb = 0, tb = 0;
  for (int k = 0; k < 16; ++k) {
    if (k < w) pa += s_wa[k], pb += s_wb[k];
    tb += s_wb[k];
  }
  uint32_t ra = pa + xa - sa, rb = pb + xb - sb;
  for (int c = beg; c < end; ++c) {
    const uint32_t t = s_t[c];
    if (a.last) {
      a.ranges[2 * (size_t)c] = ra;
      a.ranges[2 * (size_t)c + 1] = ra + t;
    } else {
      a.cbins[c] = make_uint2(ra, t);
      a.cseg[c] = rb;
    }
    ra += t;
    rb += (t + kBinSeg - 1) / kBinSeg;
  }
  if (!a.last && tid == 0) a.cseg[C] = tb;
}

__global__ __launch_bounds__(1024) void k_bin_scan(BinLevel a) {
  if (a.cgx * a.cgy <= kScanLds) {
    __shared__ uint32_t s_t[kScanLds];
    bin_scan_lds(a, s_t);
    return;
  }
  __shared__ uint32_t s_a[1024], s_b[1024];
  bin_scan(a, s_a, s_b);
}

// Write pass: every wavefront appends the entries of its child in order.
// With inline_scan (at most kInlineChildren children) there is no scan
// launch: each wavefront sums the totals of the children before its own,
// and workgroup 0 also writes the scan's outputs for the next level.
constexpr int kInlineChildren = 1024;

__global__ __launch_bounds__(1024) void k_bin_write(BinLevel a) {
  __shared__ uint32_t s_g[kBinSeg];
  __shared__ ushort4 s_rc[kBinSeg];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (a.inline_scan && blockIdx.x == 0) {
    __shared__ uint32_t s_a[1024], s_b[1024];
    bin_scan(a, s_a, s_b);
  }
  const uint32_t nseg = a.pseg[a.pgx * a.pgy];
  const uint64_t lt = (1ull << lane) - 1ull;
  for (uint32_t sg = blockIdx.x; sg < nseg; sg += gridDim.x) {
    uint32_t lo, m;
    const int p = bin_segment(a, sg, &lo, &m);
    bin_stage(a, lo, m, s_g, s_rc);
    int c, rx0, rx1, ry0, ry1;
    if (!bin_child(a, p, w, &c, &rx0, &rx1, &ry0, &ry1)) continue;
    // start of this (segment, child): the child's start plus the entries
    // the parent's earlier segments gave it
    uint32_t base = 0;
    for (uint32_t q = a.pseg[p] + lane; q < sg; q += 64) base += a.cnt[(size_t)q * 16 + w];
    for (int o = 32; o >= 1; o >>= 1) base += __shfl_xor(base, o, 64);
    if (a.inline_scan) {
      uint32_t start = 0;
      for (int q = lane; q < c; q += 64) start += a.tot[q];
      for (int o = 32; o >= 1; o >>= 1) start += __shfl_xor(start, o, 64);
      base += start;
    } else {
      base += a.last ? a.ranges[2 * (size_t)c] : a.cbins[c].x;
    }
    const uint64_t zkey = (uint64_t)c << 32;
    for (uint32_t j = lane; j < (m + 63) / 64 * 64; j += 64) {
      const bool hit = j < m && meets(s_rc[j < m ? j : 0], rx0, rx1, ry0, ry1);
      const uint64_t b = __ballot(hit);
      if (hit) {
        const uint32_t pos = base + (uint32_t)__popcll(b & lt);
        const uint32_t g = s_g[j];
        a.out[pos] = g;
        if (a.keys) a.keys[pos] = zkey | __float_as_uint(a.rec[(size_t)g * kRecFloats + 9]);
      }
      base += (uint32_t)__popcll(b);
    }
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

// One pass over at most `parts` partitions: with few partitions the
// look-back form, otherwise reduce-then-scan (status must then hold
// parts * kRadixBins words, which the look-back form needs as well).
constexpr uint32_t kLookbackParts = 512;
static void launch_pass(SweepArgs a, uint32_t parts, hipStream_t st) {
  const unsigned grid = parts < 1024u ? parts : 1024u;
  if (parts > kLookbackParts) {
    a.offsets = 1;
    a.pstride = parts;
    hipLaunchKernelGGL(k_part_hist, dim3(parts < 2048u ? parts : 2048u), dim3(kSortBlock), 0, st, a);
    hipLaunchKernelGGL(k_part_scan, dim3(kRadixBins), dim3(kSortBlock), 0, st, a);
  }
  hipLaunchKernelGGL(k_onesweep, dim3(grid > 0 ? grid : 1), dim3(kSortBlock), 0, st, a);
}


hipError_t launch_sort(const sx_projected& proj, int64_t n, const KParams& p,
                       int64_t capacity, int64_t tiles_total, uint64_t* keys,
                       uint32_t* vals, uint32_t* ranges, char* ws,
                       uint64_t* h_counts, bool* over_capacity,
                       hipStream_t st) {
  *over_capacity = false;
  const SortLayout L = sort_layout(n, capacity, p.tiles_x, p.tiles_y);
  hipError_t e;
  auto u32 = [&](size_t off) { return reinterpret_cast<uint32_t*>(ws + off); };
  uint64_t* counts = reinterpret_cast<uint64_t*>(ws + L.counts);
  if ((e = launch_fill(u32(L.zero_begin), (int64_t)((L.zero_end - L.zero_begin) / 4), 0, st))) return e;
  if (n == 0) {
    if ((e = launch_fill(ranges, tiles_total * 2, 0, st))) return e;
    if (h_counts) h_counts[0] = h_counts[1] = 0;
    return hipSuccess;
  }
  {
    const unsigned tiles = (unsigned)((L.nb + kScanTile - 1) / kScanTile);
    uint64_t* part = reinterpret_cast<uint64_t*>(ws + L.scan_part);
    hipLaunchKernelGGL(k_scan_reduce, dim3(tiles), dim3(256), 0, st, proj.block_sums,
                       (int64_t)L.nb, part);
    hipLaunchKernelGGL(k_scan_apply, dim3(tiles), dim3(256), 0, st, proj.block_sums,
                       (int64_t)L.nb, part, u32(L.vis_off), u32(L.inst_off), counts,
                       (int64_t)capacity,
                       reinterpret_cast<uint2*>(ws + L.bl_bins[0]), u32(L.bl_seg[0]));
  }
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
  // phase 1: depth digits (bits 0..30; depth > 0, sign bit clear) in 8,8,8,7
  hipLaunchKernelGGL(k_compact, dim3((unsigned)L.nb), dim3(kPreBlock), 0, st, proj.n_tiles,
                     proj.rec, n, u32(L.vis_off), u32(L.inst_off), u32(L.dkey[0]), u32(L.vidx),
                     u32(L.ioff));
  hipLaunchKernelGGL(k_hist_depth, dim3((unsigned)L.dparts), dim3(kSortBlock), 0, st,
                     u32(L.dkey[0]), counts, u32(L.dhist));
  uint32_t* counters = u32(L.counters);
  uint64_t* err = counts + 3;
  for (int ps = 0; ps < 4; ++ps) {
    SweepArgs a{};
    a.keys_in = u32(L.dkey[ps & 1]);
    a.vals_in = ps == 0 ? u32(L.vidx) : u32(L.didx[ps & 1]);
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
    launch_pass(a, (uint32_t)L.dparts, st);
  }
  // phase 2: split the depth-ordered list by tile, level by level
  uint2* bins[2] = {reinterpret_cast<uint2*>(ws + L.bl_bins[0]),
                    reinterpret_cast<uint2*>(ws + L.bl_bins[1])};
  uint32_t* seg[2] = {u32(L.bl_seg[0]), u32(L.bl_seg[1])};
  uint32_t* lists[2] = {u32(L.bl_list[0]), u32(L.bl_list[1])};
  // (the root bin, bins[0] and seg[0], was written with the visible count)
  int64_t tot_off[32];
  for (int lev = 0, o = 0; lev < L.bl_levels; ++lev) {
    const int side = 1 << (2 * lev);
    tot_off[lev] = o;
    o += ((p.tiles_x + side - 1) / side) * ((p.tiles_y + side - 1) / side);
  }
  const uint32_t* in = u32(L.didx[0]);
  int cur = 0;
  for (int lev = L.bl_levels - 1; lev >= 0; --lev) {
    const int side = 1 << (2 * lev);
    BinLevel a{};
    a.in = in;
    a.pbins = bins[cur];
    a.pseg = seg[cur];
    a.cgx = (p.tiles_x + side - 1) / side;
    a.cgy = (p.tiles_y + side - 1) / side;
    a.pgx = (a.cgx + 3) / 4;
    a.pgy = (a.cgy + 3) / 4;
    a.side = side;
    a.tiles_x = p.tiles_x, a.tiles_y = p.tiles_y;
    a.rect = proj.rect;
    a.counts = counts;
    a.cnt = u32(L.bl_cnt);
    a.tot = u32(L.bl_tot) + tot_off[lev];
    a.cbins = bins[cur ^ 1];
    a.cseg = seg[cur ^ 1];
    a.last = lev == 0;
    a.out = a.last ? vals : lists[lev & 1];
    a.ranges = ranges;
    a.keys = a.last ? keys : nullptr;
    a.rec = proj.rec;
    const int64_t nparents = (int64_t)a.pgx * a.pgy;
    const int64_t segs_max = capacity / kBinSeg + nparents + 1;
    const unsigned grid = (unsigned)(segs_max < 4096 ? segs_max : 4096);
    a.inline_scan = a.cgx * a.cgy <= kInlineChildren;
    hipLaunchKernelGGL(k_bin_count, dim3(grid), dim3(1024), 0, st, a);
    if (!a.inline_scan) hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, st, a);
    hipLaunchKernelGGL(k_bin_write, dim3(grid), dim3(1024), 0, st, a);
    in = a.out;
    cur ^= 1;
  }
  return hipGetLastError();
}

}  // namespace sx
