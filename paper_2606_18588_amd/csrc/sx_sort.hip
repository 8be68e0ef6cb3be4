// Depth sort of the instance list (paper, background: sorting step).
//
// The result equals a stable sort of 64-bit keys
//     key = tile_id << 32 | bits(float32 depth)
// over instances emitted in Gaussian-index order, i.e. the order
// (tile, depth bits, Gaussian index).  It is built in two phases:
//   1. the compacted visible Gaussians are binned by tile: a count pass,
//      one scan (the tile ranges) and a write pass that stores each
//      instance's (depth bits, index) pair at a free slot of its tile's
//      list, in no particular order;
//   2. every tile's list is sorted by (depth bits, index) by one workgroup
//      in LDS: a rank count for lists of up to 256 entries, a bitonic
//      network up to 2048, and sorted 2048-entry chunks merged through LDS
//      windows beyond that.  The pairs are unique, so the result does not
//      depend on the order phase 1 left.
// No step waits on another workgroup.
#include <algorithm>

#include "sx_internal.h"

namespace sx {

namespace {

constexpr int kScanItems = 4;  // preprocess blocks per thread in the count scan
constexpr int kScanTile = 256 * kScanItems;
constexpr int kTsThreads = 256;  // threads of the per-tile sort
constexpr int kTsRank = 256;     // longest list sorted by rank counting
constexpr int kTsChunk = 2048;   // longest list sorted in LDS at once (16 KB: the
                                 // LDS of 10 workgroups fits a CU, more than its
                                 // wave slots hold)
constexpr int kTsWin = 1024;     // merge window per run

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
  L.counts = take(4 * sizeof(uint64_t));  // offset 0: part of the ABI
  const size_t tiles = (size_t)(tiles_x * tiles_y > 0 ? tiles_x * tiles_y : 1);
  L.tcount = take(tiles * 4);
  L.cursor = take(tiles * 4);
  L.order = take(tiles * 4);
  L.vis_off = take((size_t)(L.nb > 0 ? L.nb : 1) * 4);
  L.inst_off = take((size_t)(L.nb > 0 ? L.nb : 1) * 4);
  L.ioff = take((size_t)(n > 0 ? n : 1) * 4);
  L.scan_part = take((size_t)((L.nb + kScanTile - 1) / kScanTile + 1) * 16);
  L.vidx = take((size_t)(n > 0 ? n : 1) * 4);
  L.vrect = take((size_t)(n > 0 ? n : 1) * 8);
  L.vkey = take((size_t)(n > 0 ? n : 1) * 4);
  for (int k = 0; k < 2; ++k) L.pairs[k] = take((size_t)(cap > 0 ? cap : 1) * 8);
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
  v.vidx = reinterpret_cast<const uint32_t*>(b + L.vidx);
  v.ioff = reinterpret_cast<const uint32_t*>(b + L.ioff);
  v.order = reinterpret_cast<const uint32_t*>(b + L.order);
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
                                                     uint64_t* __restrict__ part,
                                                     uint32_t* __restrict__ tot, int64_t tot_words,
                                                     uint64_t* counts) {
  __shared__ unsigned long long s4[4];
  // the first kernel of the call also clears what later kernels accumulate
  // into: the binning's tile counts and the reserved error word
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < tot_words;
       k += (int64_t)gridDim.x * 256)
    tot[k] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) counts[3] = 0;
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
                                                    uint64_t* counts, int64_t cap) {
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
    counts[2] = over ? 1ull : 0ull;  // the binning then writes nothing
  }
}

// The same scan in one workgroup (one launch instead of two) for scenes of
// at most kOneScan preprocess blocks: the block sums are loaded coalesced
// into LDS, each of 1024 threads adds up kOneScan / 1024 consecutive
// blocks, and one block-wide scan of those sums gives every offset.  It
// also clears the tile counts and the reserved error word.
constexpr int kOneScan = 8192;

__global__ __launch_bounds__(1024) void k_scan_one(const uint2* __restrict__ bsum, int64_t nb,
                                                   uint32_t* __restrict__ vis_off,
                                                   uint32_t* __restrict__ inst_off,
                                                   uint64_t* counts, int64_t cap,
                                                   uint32_t* __restrict__ tcount, int64_t tiles) {
  __shared__ uint16_t s_vis[kOneScan];  // a block has at most kPreBlock visible
  __shared__ uint32_t s_ins[kOneScan];
  __shared__ unsigned long long s_v[16], s_i[16];
  constexpr int per = kOneScan / 1024;
  static_assert(kPreBlock <= 65535, "visible counts fit 16 bits");
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int64_t k = tid; k < tiles; k += 1024) tcount[k] = 0;
  for (int j = tid; j < kOneScan; j += 1024) {
    const uint2 b = j < nb ? bsum[j] : make_uint2(0u, 0u);  // (visible, instances)
    s_vis[j] = (uint16_t)b.x;
    s_ins[j] = b.y;
  }
  __syncthreads();
  uint32_t sv = 0;
  unsigned long long si = 0;
#pragma unroll
  for (int k = 0; k < per; ++k) sv += s_vis[tid * per + k], si += s_ins[tid * per + k];
  uint32_t xv = sv;
  unsigned long long xi = si;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t yv = __shfl_up(xv, o, 64);
    const unsigned long long yi = __shfl_up(xi, o, 64);
    if (lane >= o) xv += yv, xi += yi;
  }
  if (lane == 63) s_v[w] = xv, s_i[w] = xi;
  __syncthreads();
  unsigned long long pv = xv - sv, pi = xi - si, tv = 0, ti = 0;
  for (int k = 0; k < 16; ++k) {
    if (k < w) pv += s_v[k], pi += s_i[k];
    tv += s_v[k], ti += s_i[k];
  }
#pragma unroll
  for (int k = 0; k < per; ++k) {
    const int64_t j = (int64_t)tid * per + k;
    if (j < nb) {
      vis_off[j] = (uint32_t)pv;
      inst_off[j] = (uint32_t)pi;  // exact within the 2^31 capacity bound
    }
    pv += s_vis[j], pi += s_ins[j];
  }
  if (tid == 0) {
    counts[0] = tv;
    counts[1] = ti;
    counts[2] = ti > (unsigned long long)cap ? 1ull : 0ull;  // the binning then writes nothing
    counts[3] = 0;
  }
}

// Compacted list of the visible Gaussians in index order: the input of the
// tile binning, and the order in which the backward walks the visible
// Gaussians (neighbouring lanes read neighbouring parameter rows).
// Also gives every visible Gaussian the offset of its first (Gaussian, tile)
// instance in index order, ioff[i]: the backward stores the gradient row of
// instance (i, tile) at ioff[i] + the tile's raster position in i's tile
// rectangle, so that each Gaussian's rows are contiguous.
__global__ __launch_bounds__(kPreBlock) void k_compact(const uint32_t* __restrict__ n_tiles,
                                                       const float* __restrict__ rec,
                                                       const uint16_t* __restrict__ rect,
                                                       int64_t n,
                                                       const uint32_t* __restrict__ vis_off,
                                                       const uint32_t* __restrict__ inst_off,
                                                       uint32_t* __restrict__ vidx,
                                                       ushort4* __restrict__ vrect,
                                                       uint32_t* __restrict__ vkey,
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
    vidx[pos] = (uint32_t)i;
    vrect[pos] = reinterpret_cast<const ushort4*>(rect)[i];
    vkey[pos] = __float_as_uint(rec[(size_t)i * kRecFloats + 9]);
    ioff[i] = inst_off[blockIdx.x] + iex;
  }
}

// ------------------------------------------------------------ binning --
// Every visible Gaussian's instances go to the lists of the tiles its
// rectangle covers: a count pass gives each tile's length, one scan its
// range, and a write pass stores (depth bits << 32 | index) at the tile's
// next free slot.  The order inside a tile's list is whatever the slots
// were taken in; the tile sort below makes it (depth bits, index).
//
// Each workgroup takes a contiguous run of the compacted visible list (the
// Gaussians are stored in Morton order, so a run covers few tiles), in
// chunks of kBinChunk Gaussians.  A chunk's instances are numbered through
// a block scan of the rectangle areas and dealt to the threads in turn
// (thread q takes instances q, q + kBinThreads, ...; a binary search over
// the chunk's instance starts in LDS names the Gaussian), so a Gaussian
// covering hundreds of tiles does not serialise one thread.  Counts and
// slots are aggregated in an LDS counter per tile, so that a tile sees one
// device atomic per workgroup that reaches it (grids of more than
// kLdsTiles tiles in windows of that many).
constexpr int kBinThreads = 512;
constexpr int kBinChunk = 2048;
constexpr int kBinPer = kBinChunk / kBinThreads;
constexpr int kLdsTiles = 8192;  // 32 KB of LDS counters

struct TileBin {
  const ushort4* __restrict__ vrect;  // tile rectangle per compacted position
  const uint32_t* __restrict__ vkey;  // depth bits per compacted position
  const uint32_t* __restrict__ vidx;  // Gaussian index per compacted position
  const uint64_t* counts;             // [0] visible, [2] overflow
  int tiles_x, tiles;
  uint32_t* __restrict__ tcount;  // [tiles] instances per tile (cleared by the
                                  // first kernel of the call)
  uint32_t* __restrict__ cursor;  // [tiles] next free slot (set by the scan)
  uint64_t* __restrict__ pairs;   // per-tile lists
  uint64_t cap;                   // entries of pairs
};

struct BinLds {
  uint32_t start[kBinChunk + 1];  // exclusive scan of the chunk's areas
  ushort4 rc[kBinChunk];
  uint32_t scan[kBinThreads / 64];
};

// The run of compacted positions [*b0, *b1) of this workgroup (empty when
// the instances overflowed the buffer: nothing is binned).
__device__ __forceinline__ void bin_run(const TileBin& a, uint64_t* b0, uint64_t* b1) {
  const uint64_t nvis = a.counts[2] ? 0ull : a.counts[0];
  const uint64_t per = (nvis + gridDim.x - 1) / gridDim.x;
  *b0 = (uint64_t)blockIdx.x * per;
  *b1 = *b0 + per < nvis ? *b0 + per : nvis;
}

// Calls f(compacted position, tile) for every instance of the run.
template <typename F>
__device__ __forceinline__ void bin_each(const TileBin& a, uint64_t b0, uint64_t b1, BinLds& L,
                                         F f) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (uint64_t c0 = b0; c0 < b1; c0 += kBinChunk) {
    const int m = b1 - c0 < (uint64_t)kBinChunk ? (int)(b1 - c0) : kBinChunk;
    // areas of the thread's kBinPer consecutive Gaussians, block scan
    ushort4 rc[kBinPer];
    uint32_t ar[kBinPer], sum = 0;
#pragma unroll
    for (int k = 0; k < kBinPer; ++k) {
      const int j = tid * kBinPer + k;
      rc[k] = j < m ? a.vrect[c0 + j] : make_ushort4(0, 0, 0, 0);
      ar[k] = (uint32_t)(rc[k].z - rc[k].x) * (uint32_t)(rc[k].w - rc[k].y);
      sum += ar[k];
    }
    uint32_t x = sum;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    __syncthreads();  // every thread is done with the previous chunk's arrays
#pragma unroll
    for (int k = 0; k < kBinPer; ++k)
      if (tid * kBinPer + k < m) L.rc[tid * kBinPer + k] = rc[k];
    if (lane == 63) L.scan[w] = x;
    __syncthreads();
    uint32_t run = x - sum, total = 0;
    for (int k = 0; k < kBinThreads / 64; ++k) {
      if (k < w) run += L.scan[k];
      total += L.scan[k];
    }
#pragma unroll
    for (int k = 0; k < kBinPer; ++k) {
      L.start[tid * kBinPer + k] = run;
      run += ar[k];
    }
    if (tid == 0) L.start[kBinChunk] = total;
    __syncthreads();
    for (uint32_t q = tid; q < total; q += kBinThreads) {
      int lo = 0, hi = m - 1;  // last Gaussian whose start <= q
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L.start[mid] <= q) lo = mid; else hi = mid - 1;
      }
      const ushort4 g = L.rc[lo];
      const uint32_t r = q - L.start[lo], wd = (uint32_t)(g.z - g.x);
      const uint32_t ry = r / wd;
      const int t = (int)(g.y + ry) * a.tiles_x + (int)(g.x + (r - ry * wd));
      if ((unsigned)t < (unsigned)a.tiles) f(c0 + (uint64_t)lo, t);  // always, by construction
    }
  }
}

// Both passes aggregate in LDS over windows of kLdsTiles tiles: a grid
// wider than one window is taken window by window, each enumerating the
// run's instances again and keeping those of its window.
__global__ __launch_bounds__(kBinThreads) void k_tile_count(TileBin a) {
  __shared__ BinLds L;
  __shared__ uint32_t s_h[kLdsTiles];
  uint64_t b0, b1;
  bin_run(a, &b0, &b1);
  if (b0 >= b1) return;  // the same for the whole workgroup
  for (int w0 = 0; w0 < a.tiles; w0 += kLdsTiles) {
    const int wn = a.tiles - w0 < kLdsTiles ? a.tiles - w0 : kLdsTiles;
    __syncthreads();  // the previous window's counters are flushed
    for (int t = threadIdx.x; t < wn; t += kBinThreads) s_h[t] = 0;
    bin_each(a, b0, b1, L, [&](uint64_t, int t) {
      if ((unsigned)(t - w0) < (unsigned)wn) atomicAdd(&s_h[t - w0], 1u);
    });
    __syncthreads();
    for (int t = threadIdx.x; t < wn; t += kBinThreads) {
      const uint32_t c = s_h[t];
      if (c) atomicAdd(&a.tcount[w0 + t], c);  // integer sums: any order
    }
  }
}

// One workgroup: exclusive scan of the tile counts into the tile ranges
// [start, end) and the write pass's cursors (= start), through LDS in
// chunks of kScanChunk tiles with a running carry; then the tiles in
// descending order of list length (buckets of 4 entries, any order within
// a bucket), the order in which the reverse walk takes them: the long
// tiles start early and the wave slots drain evenly at the end (the order
// changes no result: each tile's rows depend on that tile alone).
constexpr int kScanChunk = 8192;
constexpr int kOrderBuckets = 256;

__global__ __launch_bounds__(1024) void k_tile_scan(const uint32_t* __restrict__ tcount,
                                                    int tiles, uint32_t* __restrict__ ranges,
                                                    uint32_t* __restrict__ cursor,
                                                    uint32_t* __restrict__ order) {
  __shared__ uint32_t s_t[kScanChunk];
  __shared__ uint32_t s_w[16];
  __shared__ uint32_t s_c[kOrderBuckets];
  constexpr int per = kScanChunk / 1024;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  uint32_t carry = 0;
  for (int c0 = 0; c0 < tiles; c0 += kScanChunk) {
    const int m = tiles - c0 < kScanChunk ? tiles - c0 : kScanChunk;
    for (int t = tid; t < kScanChunk; t += 1024) s_t[t] = t < m ? tcount[c0 + t] : 0u;
    __syncthreads();
    uint32_t v[per], sum = 0;
#pragma unroll
    for (int k = 0; k < per; ++k) v[k] = s_t[tid * per + k], sum += v[k];
    uint32_t x = sum;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    uint32_t run = carry + x - sum, total = 0;
    for (int k = 0; k < 16; ++k) {
      if (k < w) run += s_w[k];
      total += s_w[k];
    }
#pragma unroll
    for (int k = 0; k < per; ++k) s_t[tid * per + k] = run, run += v[k];
    __syncthreads();
    for (int t = tid; t < m; t += 1024) {
      const uint32_t st = s_t[t];
      ranges[2 * (size_t)(c0 + t)] = st;
      ranges[2 * (size_t)(c0 + t) + 1] = st + tcount[c0 + t];
      cursor[c0 + t] = st;
    }
    carry += total;
    __syncthreads();
  }
  auto bucket = [&](int t) {
    const uint32_t b = tcount[t] >> 2;
    return kOrderBuckets - 1 - (int)(b < (uint32_t)kOrderBuckets - 1 ? b : kOrderBuckets - 1);
  };
  if (tid < kOrderBuckets) s_c[tid] = 0;
  __syncthreads();
  for (int t = tid; t < tiles; t += 1024) atomicAdd(&s_c[bucket(t)], 1u);
  __syncthreads();
  if (tid < 64) {  // exclusive scan of the bucket sizes, 4 per lane
    constexpr int bp = kOrderBuckets / 64;
    uint32_t v[bp], sum = 0;
#pragma unroll
    for (int k = 0; k < bp; ++k) v[k] = s_c[tid * bp + k], sum += v[k];
    uint32_t x = sum;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (tid >= o) x += y;
    }
    uint32_t run = x - sum;
#pragma unroll
    for (int k = 0; k < bp; ++k) s_c[tid * bp + k] = run, run += v[k];
  }
  __syncthreads();
  for (int t = tid; t < tiles; t += 1024) order[atomicAdd(&s_c[bucket(t)], 1u)] = (uint32_t)t;
}

__global__ __launch_bounds__(kBinThreads) void k_tile_write(TileBin a) {
  __shared__ BinLds L;
  __shared__ uint32_t s_h[kLdsTiles];
  uint64_t b0, b1;
  bin_run(a, &b0, &b1);
  if (b0 >= b1) return;
  auto key = [&](uint64_t i) { return (uint64_t)a.vkey[i] << 32 | a.vidx[i]; };
  for (int w0 = 0; w0 < a.tiles; w0 += kLdsTiles) {
    const int wn = a.tiles - w0 < kLdsTiles ? a.tiles - w0 : kLdsTiles;
    auto in_window = [&](int t) { return (unsigned)(t - w0) < (unsigned)wn; };
    // count again, reserve each tile's slots with one device atomic, then
    // hand them out from LDS
    __syncthreads();  // the previous window's slots are handed out
    for (int t = threadIdx.x; t < wn; t += kBinThreads) s_h[t] = 0;
    bin_each(a, b0, b1, L, [&](uint64_t, int t) {
      if (in_window(t)) atomicAdd(&s_h[t - w0], 1u);
    });
    __syncthreads();
    for (int t = threadIdx.x; t < wn; t += kBinThreads) {
      const uint32_t c = s_h[t];
      if (c) s_h[t] = atomicAdd(&a.cursor[w0 + t], c);
    }
    __syncthreads();
    bin_each(a, b0, b1, L, [&](uint64_t i, int t) {
      if (!in_window(t)) return;
      const uint32_t pos = atomicAdd(&s_h[t - w0], 1u);
      if (pos < a.cap) a.pairs[pos] = key(i);  // always, the slots being reserved
    });
  }
}

// ------------------------------------------------------------ tile sort --
// Every tile's list of (depth bits << 32 | Gaussian index) keys, in index
// order after the binning, sorted ascending by one workgroup; the keys are
// unique, so the order is (depth bits, index) whatever the method.

// Bitonic network over np (a power of two <= kTsChunk) keys in LDS.
__device__ __forceinline__ void ts_bitonic(uint64_t* s, uint32_t np) {
  const uint32_t tid = threadIdx.x;
  for (uint32_t k = 2; k <= np; k <<= 1)
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = tid; i < np / 2; i += kTsThreads) {
        const uint32_t x = ((i & ~(j - 1)) << 1) | (i & (j - 1)), y = x + j;
        const uint64_t u = s[x], v = s[y];
        if ((u > v) == ((x & k) == 0)) s[x] = v, s[y] = u;
      }
      __syncthreads();
    }
}

// Outputs of one list position: the instance value and, if asked, the
// 64-bit key tile << 32 | depth bits.
__device__ __forceinline__ void ts_out(uint32_t* vals, uint64_t* keys, uint32_t pos,
                                       uint32_t tile, uint64_t k) {
  vals[pos] = (uint32_t)k;
  if (keys) keys[pos] = (uint64_t)tile << 32 | (k >> 32);
}

// Merge-path split of the first d outputs of merging a[0..na) and b[0..nb)
// (ascending, unique): how many come from a.
__device__ __forceinline__ uint32_t ts_split(const uint64_t* a, uint32_t na, const uint64_t* b,
                                             uint32_t nb, uint32_t d) {
  uint32_t lo = d > nb ? d - nb : 0u, hi = d < na ? d : na;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (a[mid] < b[d - 1 - mid]) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(kTsThreads) void k_tile_sort(const uint32_t* __restrict__ ranges,
                                                          uint64_t* __restrict__ pa,
                                                          uint64_t* __restrict__ pb,
                                                          uint32_t* __restrict__ vals,
                                                          uint64_t* __restrict__ keys) {
  __shared__ uint64_t s_k[kTsChunk];
  const uint32_t tile = blockIdx.x, tid = threadIdx.x;
  const uint32_t s0 = ranges[2 * (size_t)tile], L = ranges[2 * (size_t)tile + 1] - s0;
  if (L == 0) return;
  if (L <= (uint32_t)kTsRank) {
    // rank counting: each key's position is the number of smaller keys
    uint64_t k = 0;
    if (tid < L) k = s_k[tid] = pa[s0 + tid];
    __syncthreads();
    if (tid < L) {
      uint32_t r = 0;
      for (uint32_t j = 0; j < L; ++j) r += s_k[j] < k ? 1u : 0u;
      ts_out(vals, keys, s0 + r, tile, k);
    }
    return;
  }
  if (L <= (uint32_t)kTsChunk) {
    uint32_t np = 512;
    while (np < L) np <<= 1;
    for (uint32_t i = tid; i < np; i += kTsThreads) s_k[i] = i < L ? pa[s0 + i] : ~0ull;
    __syncthreads();
    ts_bitonic(s_k, np);
    for (uint32_t i = tid; i < L; i += kTsThreads) ts_out(vals, keys, s0 + i, tile, s_k[i]);
    return;
  }
  // long list: sorted chunks of kTsChunk keys (in place in pa), then merge
  // passes of doubling run width between pa and pb, each merge streamed
  // through LDS windows of kTsWin keys per run
  uint64_t* src = pa + s0;
  uint64_t* dst = pb + s0;
  for (uint32_t c0 = 0; c0 < L; c0 += kTsChunk) {
    const uint32_t m = L - c0 < (uint32_t)kTsChunk ? L - c0 : (uint32_t)kTsChunk;
    __syncthreads();
    for (uint32_t i = tid; i < (uint32_t)kTsChunk; i += kTsThreads) s_k[i] = i < m ? src[c0 + i] : ~0ull;
    __syncthreads();
    ts_bitonic(s_k, kTsChunk);
    for (uint32_t i = tid; i < m; i += kTsThreads) src[c0 + i] = s_k[i];
  }
  uint64_t* sa = s_k;
  uint64_t* sb = s_k + kTsWin;
  constexpr uint32_t kPer = kTsWin / kTsThreads;  // outputs per thread per window
  for (uint32_t w = kTsChunk; w < L; w <<= 1) {
    for (uint32_t lo = 0; lo < L; lo += 2 * w) {
      const uint32_t la = L - lo < w ? L - lo : w;
      const uint32_t lb = L - lo - la < w ? L - lo - la : w;
      const uint64_t* A = src + lo;
      const uint64_t* Bv = src + lo + la;
      uint32_t ia = 0, ib = 0, o = 0;
      while (o < la + lb) {
        const uint32_t na = la - ia < (uint32_t)kTsWin ? la - ia : (uint32_t)kTsWin;
        const uint32_t nb = lb - ib < (uint32_t)kTsWin ? lb - ib : (uint32_t)kTsWin;
        __syncthreads();  // the previous window is consumed
        for (uint32_t i = tid; i < (uint32_t)kTsWin; i += kTsThreads) {
          sa[i] = i < na ? A[ia + i] : ~0ull;
          sb[i] = i < nb ? Bv[ib + i] : ~0ull;
        }
        __syncthreads();
        // the window's outputs are the `win` smallest remaining keys, all
        // within the loaded prefixes of both runs
        const uint32_t left = la + lb - o;
        const uint32_t win = left < (uint32_t)kTsWin ? left : (uint32_t)kTsWin;
        const uint32_t d0 = tid * kPer < win ? tid * kPer : win;
        uint32_t i = ts_split(sa, na, sb, nb, d0), j = d0 - i;
        for (uint32_t q = 0; q < kPer && d0 + q < win; ++q) {
          const bool take_a = j >= nb || (i < na && sa[i] < sb[j]);
          dst[lo + o + d0 + q] = take_a ? sa[i] : sb[j];
          if (take_a) ++i; else ++j;
        }
        const uint32_t ea = ts_split(sa, na, sb, nb, win);
        ia += ea;
        ib += win - ea;
        o += win;
      }
    }
    uint64_t* t = src;
    src = dst;
    dst = t;
    __syncthreads();  // this pass's outputs are written before the next reads them
  }
  __syncthreads();
  for (uint32_t i = tid; i < L; i += kTsThreads) ts_out(vals, keys, s0 + i, tile, src[i]);
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
  if (n == 0) {
    // no instance: zero counts, empty ranges and the tile order
    if ((e = launch_fill(u32(L.counts), 8, 0, st))) return e;
    if ((e = launch_fill(u32(L.tcount), tiles_total, 0, st))) return e;
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, st, u32(L.tcount), (int)tiles_total,
                       ranges, u32(L.cursor), u32(L.order));
    if (h_counts) h_counts[0] = h_counts[1] = 0;
    return hipGetLastError();
  }
  if (L.nb <= kOneScan) {
    hipLaunchKernelGGL(k_scan_one, dim3(1), dim3(1024), 0, st,
                       reinterpret_cast<const uint2*>(proj.block_sums), (int64_t)L.nb,
                       u32(L.vis_off), u32(L.inst_off), counts, (int64_t)capacity,
                       u32(L.tcount), tiles_total);
  } else {
    const unsigned tiles = (unsigned)((L.nb + kScanTile - 1) / kScanTile);
    uint64_t* part = reinterpret_cast<uint64_t*>(ws + L.scan_part);
    hipLaunchKernelGGL(k_scan_reduce, dim3(tiles), dim3(256), 0, st, proj.block_sums,
                       (int64_t)L.nb, part, u32(L.tcount), tiles_total, counts);
    hipLaunchKernelGGL(k_scan_apply, dim3(tiles), dim3(256), 0, st, proj.block_sums,
                       (int64_t)L.nb, part, u32(L.vis_off), u32(L.inst_off), counts,
                       (int64_t)capacity);
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
  hipLaunchKernelGGL(k_compact, dim3((unsigned)L.nb), dim3(kPreBlock), 0, st, proj.n_tiles,
                     proj.rec, proj.rect, n, u32(L.vis_off), u32(L.inst_off), u32(L.vidx),
                     reinterpret_cast<ushort4*>(ws + L.vrect), u32(L.vkey), u32(L.ioff));
  // phase 1: the instances into their tiles' lists
  {
    TileBin a{};
    a.vrect = reinterpret_cast<const ushort4*>(ws + L.vrect);
    a.vkey = u32(L.vkey);
    a.vidx = u32(L.vidx);
    a.counts = counts;
    a.tiles_x = p.tiles_x;
    a.tiles = (int)tiles_total;
    a.tcount = u32(L.tcount);
    a.cursor = u32(L.cursor);
    a.pairs = reinterpret_cast<uint64_t*>(ws + L.pairs[0]);
    a.cap = (uint64_t)(capacity > 0 ? capacity : 1);
    int64_t blocks = n / 4096;
    blocks = blocks < 1 ? 1 : blocks > 512 ? 512 : blocks;
    hipLaunchKernelGGL(k_tile_count, dim3((unsigned)blocks), dim3(kBinThreads), 0, st, a);
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, st, a.tcount, a.tiles, ranges,
                       a.cursor, u32(L.order));
    hipLaunchKernelGGL(k_tile_write, dim3((unsigned)blocks), dim3(kBinThreads), 0, st, a);
  }
  uint64_t* pairs[2] = {reinterpret_cast<uint64_t*>(ws + L.pairs[0]),
                        reinterpret_cast<uint64_t*>(ws + L.pairs[1])};
  // phase 2: each tile's list by (depth bits, index)
  hipLaunchKernelGGL(k_tile_sort, dim3((unsigned)tiles_total), dim3(kTsThreads), 0, st, ranges,
                     pairs[0], pairs[1], vals, keys);
  return hipGetLastError();
}

}  // namespace sx
