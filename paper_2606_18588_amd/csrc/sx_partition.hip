// KD-tree partition of a scene's Gaussians into K convex cells by their
// means (paper: partition strategy of the evaluation's robustness study):
// recursive binary splits, each along the axis on which the node's means
// have the largest extent, at the quantile of the means that gives the two
// halves their share of cells (the median when K is a power of two).  The
// boxes are disjoint and cover space (the outermost bounds are infinite),
// so the composition's per-ray order is exact for them.  Host code, plus
// the device move of a repartition's rows.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "sx_internal.h"

namespace sx {
namespace {

struct Box {
  float lo[3], hi[3];
};

void split(const float* means, std::vector<int64_t>& idx, int64_t b, int64_t e, int K, Box box,
           int first_cell, float* lo, float* hi, int32_t* cell_of, std::vector<float>& key) {
  if (K == 1 || e - b == 0) {
    // a leaf (an empty node keeps its box and takes all its cells' slots)
    for (int c = 0; c < K; ++c)
      for (int j = 0; j < 3; ++j) {
        lo[(first_cell + c) * 3 + j] = box.lo[j];
        hi[(first_cell + c) * 3 + j] = c == 0 ? box.hi[j] : box.lo[j];
      }
    for (int64_t i = b; i < e; ++i) cell_of[idx[i]] = first_cell;
    return;
  }
  // axis of the largest extent of the node's means (ties: lowest axis)
  float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = b; i < e; ++i)
    for (int j = 0; j < 3; ++j) {
      const float v = means[idx[i] * 3 + j];
      mn[j] = std::min(mn[j], v), mx[j] = std::max(mx[j], v);
    }
  int ax = 0;
  for (int j = 1; j < 3; ++j)
    if (mx[j] - mn[j] > mx[ax] - mn[ax]) ax = j;
  // split value: the q-th smallest mean on that axis, q = n * K_left / K
  const int kl = K / 2;
  const int64_t n = e - b;
  const int64_t q = n * kl / K;
  key.resize((size_t)n);
  for (int64_t i = 0; i < n; ++i) key[(size_t)i] = means[idx[b + i] * 3 + ax];
  std::nth_element(key.begin(), key.begin() + q, key.end());
  const float s = key[(size_t)q];
  // left: mean < s, right: mean >= s (stable, so the order is reproducible)
  const auto mid = std::stable_partition(idx.begin() + b, idx.begin() + e,
                                         [&](int64_t i) { return means[i * 3 + ax] < s; });
  const int64_t m = mid - idx.begin();
  Box bl = box, br = box;
  bl.hi[ax] = s, br.lo[ax] = s;
  split(means, idx, b, m, kl, bl, first_cell, lo, hi, cell_of, key);
  split(means, idx, m, e, K - kl, br, first_cell + kl, lo, hi, cell_of, key);
}

}  // namespace

// Destination of every Gaussian of a repartition: dst_index[g] is g's rank
// among the Gaussians of its new cell cell_of[g], in the order of g (so each
// new cell keeps the relative order of its Gaussians); counts[k] the new
// cell sizes.
void repartition_plan(int64_t n, const int32_t* cell_of, int K, int32_t* dst_index,
                      int64_t* counts) {
  for (int k = 0; k < K; ++k) counts[k] = 0;
  for (int64_t g = 0; g < n; ++g) dst_index[g] = (int32_t)counts[cell_of[g]]++;
}

// Row moves of a repartition: row g (global index over the source cells
// laid end to end) of every array goes to row dst_index[g] of new cell
// dst_cell[g].  One thread per (row, float4 or float).
struct MoveArgs {
  const float* src[kMaxCells];
  float* dst[kMaxCells];
  int64_t src_off[kMaxCells + 1];  // first global row of each source cell
  int k_src;
  int row_floats;
  int64_t n;
  const int32_t* dst_cell;
  const int32_t* dst_index;
};

__global__ __launch_bounds__(256) void k_move_rows(MoveArgs a) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t g = t / a.row_floats;
  const int f = (int)(t - g * a.row_floats);
  if (g >= a.n) return;
  int c = 0;
  while (c + 1 < a.k_src && a.src_off[c + 1] <= g) ++c;
  const int64_t i = g - a.src_off[c];
  a.dst[a.dst_cell[g]][(int64_t)a.dst_index[g] * a.row_floats + f] =
      a.src[c][i * a.row_floats + f];
}

hipError_t launch_move_rows(int64_t n, int row_floats, int k_src, const int64_t* src_off,
                            const float* const* src, int k_dst, float* const* dst,
                            const int32_t* dst_cell, const int32_t* dst_index, hipStream_t st) {
  if (n == 0) return hipSuccess;
  MoveArgs a{};
  for (int c = 0; c < k_src; ++c) a.src[c] = src[c];
  for (int c = 0; c <= k_src; ++c) a.src_off[c] = src_off[c];
  for (int c = 0; c < k_dst; ++c) a.dst[c] = dst[c];
  a.k_src = k_src;
  a.row_floats = row_floats;
  a.n = n;
  a.dst_cell = dst_cell;
  a.dst_index = dst_index;
  const int64_t threads = n * row_floats;
  hipLaunchKernelGGL(k_move_rows, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

void kd_partition(int64_t n, const float* means, int K, float* lo, float* hi, int32_t* cell_of) {
  std::vector<int64_t> idx((size_t)n);
  for (int64_t i = 0; i < n; ++i) idx[(size_t)i] = i;
  std::vector<float> key;
  Box root;
  for (int j = 0; j < 3; ++j) root.lo[j] = -INFINITY, root.hi[j] = INFINITY;
  split(means, idx, 0, n, K, root, 0, lo, hi, cell_of, key);
}

}  // namespace sx
