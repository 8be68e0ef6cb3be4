// Depth sort of the instance list (paper, background: sorting step).
//
// The result equals a stable sort of 64-bit keys
//     key = tile_id << 32 | bits(float32 depth)
// over instances emitted in Gaussian-index order, i.e. the order
// (tile, depth bits, Gaussian index).  It is built in two phases:
//   1. the list of visible Gaussians, in index order, is split by tile
//      through a hierarchy of bins (bins of 4^L x 4^L tiles, each bin having
//      4 x 4 child bins): the list of a bin is cut into segments, and for
//      every segment each of 16 wavefronts ballot-filters the entries whose
//      tile rectangle meets its child bin.  A count pass and an exclusive
//      scan give every (segment, child) its output offset, and a write pass
//      stores the entries in order, so each child's list keeps the index
//      order and every store is a contiguous run of a wavefront.  The last
//      level's bins are single tiles: their lists hold (depth bits, index)
//      pairs and the scan gives the tile ranges;
//   2. every tile's list is sorted by (depth bits, index) by one workgroup
//      in LDS: a rank count for lists of up to 256 entries, a bitonic
//      network up to 2048, and sorted 2048-entry chunks merged through LDS
//      windows beyond that.
// No step uses atomics on the output, and no step waits on another
// workgroup.
#include <algorithm>

#include "sx_internal.h"

namespace sx {

namespace {

constexpr int kScanItems = 4;  // preprocess blocks per thread in the count scan
constexpr int kScanTile = 256 * kScanItems;
constexpr int kRootFan = 4;      // child bins per axis of the root's split
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
  // binning: levels of 4x4 bins until one bin covers the grid; per level,
  // the children's entry totals (accumulated by the count pass)
  const int64_t big = tiles_x > tiles_y ? tiles_x : tiles_y;
  // the root (kRootFan) over levels of fan 4 covers kRootFan * 4^(levels - 1) tiles
  int levels = 1;
  while ((int64_t(kRootFan) << (2 * (levels - 1))) < big) ++levels;
  L.bl_levels = levels;
  int64_t tot_words = 0;
  for (int lev = 0; lev < levels; ++lev) {
    const int64_t side = int64_t(1) << (2 * lev);
    tot_words += ((tiles_x + side - 1) / side) * ((tiles_y + side - 1) / side);
  }
  L.bl_tot = take((size_t)tot_words * 4);
  L.tot_words = tot_words;
  L.vis_off = take((size_t)(L.nb > 0 ? L.nb : 1) * 4);
  L.inst_off = take((size_t)(L.nb > 0 ? L.nb : 1) * 4);
  L.ioff = take((size_t)(n > 0 ? n : 1) * 4);
  L.scan_part = take((size_t)((L.nb + kScanTile - 1) / kScanTile + 1) * 16);
  L.vidx = take((size_t)(n > 0 ? n : 1) * 4);
  L.vrect = take((size_t)(n > 0 ? n : 1) * 8);
  L.vkey = take((size_t)(n > 0 ? n : 1) * 4);
  // every entry of an inner level is a (Gaussian, bin) pair with at least
  // one instance in the bin, so an inner list never exceeds the instance count
  const int64_t bins = ((tiles_x + 3) / 4) * ((tiles_y + 3) / 4);
  const size_t list_bytes = (size_t)(cap > 0 ? cap : 1) * 4;
  L.bl_list[1] = levels >= 2 ? take(list_bytes) : off;  // level 1 writes list[1]
  L.bl_list[0] = levels >= 3 ? take(list_bytes) : off;
  for (int k = 0; k < 2; ++k) L.bl_bins[k] = take((size_t)(bins + 1) * 8);
  for (int k = 0; k < 2; ++k) L.bl_seg[k] = take((size_t)(bins + 2) * 4);
  {
    // (segment, child) counts: 256 per segment of the root, 16 below
    const size_t segs = (size_t)(cap / kBinSeg) + 2;
    const size_t words = std::max(segs * 256, (segs + (size_t)bins) * 16);
    L.bl_cnt = take(words * 4);
  }
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
  // into: the binning's child totals and the reserved error word
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
// One level of the tile hierarchy: parents are bins of fan*side x fan*side
// tiles (grid pgx x pgy, lists in `in`), children bins of side x side
// (grid cgx x cgy).  Child (cx, cy) belongs to parent (cx/fan, cy/fan) at
// slot (cy%fan)*fan + cx%fan; a wavefront takes fan*fan/16 slots.  The
// root level has one parent and fan kRootFan, the levels below fan 4 (a
// root of fan 16, a row of 16 slots per wavefront, measured slower: its
// wavefronts scan the segment once per slot).  Parent lists are cut into
// segments of kBinSeg entries; pseg[p] is the first segment of parent p and
// pseg[nparents] the total.
struct BinLevel {
  const uint32_t* __restrict__ in;  // positions in the compacted visible list
  const uint2* __restrict__ pbins;   // (start, length) per parent
  const uint32_t* __restrict__ pseg;
  int pgx, pgy, cgx, cgy, side, tiles_x, tiles_y;
  int fan;    // children per parent along each axis (4 or 16)
  int cpw;    // children per wavefront: fan * fan / 16
  const ushort4* __restrict__ vrect;  // tile rectangle per compacted position
  const uint32_t* __restrict__ vkey;  // depth bits per compacted position
  const uint32_t* __restrict__ vidx;  // Gaussian index per compacted position
  const uint64_t* counts;
  uint32_t* __restrict__ cnt;   // [segments][fan * fan]
  uint32_t* __restrict__ tot;   // [children], zeroed before the count pass
  uint2* __restrict__ cbins;    // (start, length) per child (inner levels)
  uint32_t* __restrict__ cseg;  // segment starts of the children (inner levels)
  uint32_t* __restrict__ out;     // child lists of the inner levels
  uint32_t* __restrict__ ranges;  // last level: [tiles][2]
  uint64_t* __restrict__ pairs;   // last level: depth bits << 32 | index per instance
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

// Tile region of the child bin of parent p at slot `slot`; false if outside.
__device__ __forceinline__ bool bin_child(const BinLevel& a, int p, int slot, int* c, int* rx0,
                                          int* rx1, int* ry0, int* ry1) {
  const int cx = (p % a.pgx) * a.fan + slot % a.fan, cy = (p / a.pgx) * a.fan + slot / a.fan;
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
    const uint32_t g = a.in ? a.in[lo + i] : lo + i;  // the root list is 0, 1, ...
    s_g[i] = g;
    s_rc[i] = a.vrect[g];
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
    const int nslot = a.fan * a.fan;
    for (int k = 0; k < a.cpw; ++k) {
      const int slot = w * a.cpw + k;
      int c = 0, rx0, rx1, ry0, ry1;
      uint32_t n = 0;
      if (bin_child(a, p, slot, &c, &rx0, &rx1, &ry0, &ry1))
        for (uint32_t j = lane; j < (m + 63) / 64 * 64; j += 64) {
          const bool hit = j < m && meets(s_rc[j < m ? j : 0], rx0, rx1, ry0, ry1);
          n += (uint32_t)__popcll(__ballot(hit));
        }
      if (lane == 0) {
        a.cnt[(size_t)sg * nslot + slot] = n;
        if (n) atomicAdd(&a.tot[c], n);  // integer sum: the order does not matter
      }
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
    const int nslot = a.fan * a.fan;
    for (int k = 0; k < a.cpw; ++k) {
    const int slot = w * a.cpw + k;
    int c, rx0, rx1, ry0, ry1;
    if (!bin_child(a, p, slot, &c, &rx0, &rx1, &ry0, &ry1)) continue;
    // start of this (segment, child): the child's start plus the entries
    // the parent's earlier segments gave it
    uint32_t base = 0;
    for (uint32_t q = a.pseg[p] + lane; q < sg; q += 64) base += a.cnt[(size_t)q * nslot + slot];
    for (int o = 32; o >= 1; o >>= 1) base += __shfl_xor(base, o, 64);
    if (a.inline_scan) {
      uint32_t start = 0;
      for (int q = lane; q < c; q += 64) start += a.tot[q];
      for (int o = 32; o >= 1; o >>= 1) start += __shfl_xor(start, o, 64);
      base += start;
    } else {
      base += a.last ? a.ranges[2 * (size_t)c] : a.cbins[c].x;
    }
    for (uint32_t j = lane; j < (m + 63) / 64 * 64; j += 64) {
      const bool hit = j < m && meets(s_rc[j < m ? j : 0], rx0, rx1, ry0, ry1);
      const uint64_t b = __ballot(hit);
      if (hit) {
        const uint32_t pos = base + (uint32_t)__popcll(b & lt);
        const uint32_t g = s_g[j];
        if (a.last)
          a.pairs[pos] = (uint64_t)a.vkey[g] << 32 | a.vidx[g];
        else
          a.out[pos] = g;
      }
      base += (uint32_t)__popcll(b);
    }
    }
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
    if ((e = launch_fill(u32(L.counts), 8, 0, st))) return e;
    if ((e = launch_fill(ranges, tiles_total * 2, 0, st))) return e;
    if (h_counts) h_counts[0] = h_counts[1] = 0;
    return hipSuccess;
  }
  {
    const unsigned tiles = (unsigned)((L.nb + kScanTile - 1) / kScanTile);
    uint64_t* part = reinterpret_cast<uint64_t*>(ws + L.scan_part);
    hipLaunchKernelGGL(k_scan_reduce, dim3(tiles), dim3(256), 0, st, proj.block_sums,
                       (int64_t)L.nb, part, u32(L.bl_tot), L.tot_words, counts);
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
  hipLaunchKernelGGL(k_compact, dim3((unsigned)L.nb), dim3(kPreBlock), 0, st, proj.n_tiles,
                     proj.rec, proj.rect, n, u32(L.vis_off), u32(L.inst_off), u32(L.vidx),
                     reinterpret_cast<ushort4*>(ws + L.vrect), u32(L.vkey), u32(L.ioff));
  // phase 1: split the index-ordered list of visible Gaussians by tile,
  // level by level
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
  const uint32_t* in = nullptr;  // the root bin lists compacted positions 0, 1, ...
  uint64_t* pairs[2] = {reinterpret_cast<uint64_t*>(ws + L.pairs[0]),
                        reinterpret_cast<uint64_t*>(ws + L.pairs[1])};
  int cur = 0;
  for (int lev = L.bl_levels - 1; lev >= 0; --lev) {
    const int side = 1 << (2 * lev);
    BinLevel a{};
    a.in = in;
    a.pbins = bins[cur];
    a.pseg = seg[cur];
    a.cgx = (p.tiles_x + side - 1) / side;
    a.cgy = (p.tiles_y + side - 1) / side;
    a.fan = lev == L.bl_levels - 1 ? kRootFan : 4;  // the root: one parent
    a.cpw = a.fan * a.fan / 16;
    a.pgx = (a.cgx + a.fan - 1) / a.fan;
    a.pgy = (a.cgy + a.fan - 1) / a.fan;
    a.side = side;
    a.tiles_x = p.tiles_x, a.tiles_y = p.tiles_y;
    a.vrect = reinterpret_cast<const ushort4*>(ws + L.vrect);
    a.vkey = u32(L.vkey);
    a.vidx = u32(L.vidx);
    a.counts = counts;
    a.cnt = u32(L.bl_cnt);
    a.tot = u32(L.bl_tot) + tot_off[lev];
    a.cbins = bins[cur ^ 1];
    a.cseg = seg[cur ^ 1];
    a.last = lev == 0;
    a.out = a.last ? nullptr : lists[lev & 1];
    a.ranges = ranges;
    a.pairs = a.last ? pairs[0] : nullptr;
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
  // phase 2: each tile's list by (depth bits, index)
  hipLaunchKernelGGL(k_tile_sort, dim3((unsigned)tiles_total), dim3(kTsThreads), 0, st, ranges,
                     pairs[0], pairs[1], vals, keys);
  return hipGetLastError();
}

}  // namespace sx
