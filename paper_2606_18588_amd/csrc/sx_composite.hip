// Composition of K partial-pixel buffers (Eq. 5) with the transmittance
// saturation test of the redundancy reduction, its backward (Eq. 6-7 at the
// level of partial pixels), the L1 loss of the composed image and Adam.
//
// All of these are HBM-bound streams: one lane per pixel (or per parameter),
// 16-byte (rgb, T) loads and stores, no LDS.  The saturation masks are
// updated without atomics: a wavefront covers 64 consecutive pixels, i.e.
// exactly two 32-bit mask words, which it rewrites from one ballot.
#include "sx_internal.h"

namespace sx {

struct CompArgs {
  int K;
  const float4* part[kMaxCells];
  float lo[kMaxCells][3];
  float hi[kMaxCells][3];
  float O[3];   // camera centre
  float Rm[9];  // world->camera rotation
  float fx, fy, cx, cy;
  int W, H;
  float t_min;
  float bg[3];
  int same_frame;
  // forward
  float4* out;
  uint32_t* masks;
  uint32_t words;
  const uint32_t* omega;  // re-evaluation: boxes the pixel rays meet (NULL = all)
  float* budget;          // re-evaluation: [K][H*W] stale consumption of pruned pairs
  // backward
  const float4* dout;
  float4* dpart[kMaxCells];
};

// Ray entry parameter into a box, max(0, t_near) of the slab test; an axis
// the ray runs parallel to imposes no entry constraint.
__device__ __forceinline__ float entry_key(const float O[3], const float d[3],
                                           const float lo[3], const float hi[3]) {
  float tn = -INFINITY;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    if (d[j] == 0.f) continue;
    const float t1 = (lo[j] - O[j]) / d[j], t2 = (hi[j] - O[j]) / d[j];
    tn = fmaxf(tn, fminf(t1, t2));
  }
  return fmaxf(tn, 0.f);
}

// Position of every cell in the per-pixel front-to-back order (ties by cell
// index), computed by counting without dynamic register indexing.
template <int KM>
__device__ __forceinline__ void cell_ranks(const CompArgs& a, int px, int py,
                                           int rank[KM]) {
  const float u = ((float)px + 0.5f - a.cx) / a.fx;
  const float v = ((float)py + 0.5f - a.cy) / a.fy;
  float d[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) d[j] = a.Rm[0 * 3 + j] * u + a.Rm[1 * 3 + j] * v + a.Rm[2 * 3 + j];
  float key[KM];
#pragma unroll
  for (int m = 0; m < KM; ++m) key[m] = m < a.K ? entry_key(a.O, d, a.lo[m], a.hi[m]) : INFINITY;
#pragma unroll
  for (int m = 0; m < KM; ++m) {
    int r = 0;
#pragma unroll
    for (int q = 0; q < KM; ++q)
      r += (q < a.K) && (key[q] < key[m] || (key[q] == key[m] && q < m));
    rank[m] = r;
  }
}

// RE = false: the saturation test only clears mask bits.  RE = true: the
// masks are the per-pair state carried between renders of the view and are
// rewritten whole: a rendered pair stays set while its incoming
// transmittance P reaches t_min, and is pruned otherwise with its
// consumption P (1 - T) kept as its budget; a pruned pair whose box the ray
// meets is re-activated while the residual R = P - S (S: budgets of the
// pairs re-activated before it on the ray) reaches t_min and covers its
// budget, the first that fails ending the scan (appendix, experimental
// analysis: speculative re-evaluation of saturation).
template <int KM, bool RE>
__global__ __launch_bounds__(256) void k_composite(CompArgs a) {
  const uint32_t HW = (uint32_t)a.W * a.H;
  const uint32_t p = blockIdx.x * 256 + threadIdx.x;
  const bool inside = p < HW;
  const uint32_t pp = inside ? p : 0u;
  const int px = (int)(pp % a.W), py = (int)(pp / a.W);
  int rank[KM];
  cell_ranks<KM>(a, px, py, rank);
  float4 cm[KM];
#pragma unroll
  for (int m = 0; m < KM; ++m)
    cm[m] = (inside && m < a.K) ? a.part[m][pp] : make_float4(0.f, 0.f, 0.f, 1.f);
  // RE: bit m of `on` = pair rendered now, of `vis` = the ray meets box m
  uint32_t on = ~0u, vis = ~0u;
  if (RE) {
    const uint32_t wi = pp >> 5, bi = pp & 31;
    on = 0;
#pragma unroll
    for (int m = 0; m < KM; ++m)
      if (m < a.K) on |= ((a.masks[(size_t)m * a.words + wi] >> bi) & 1u) << m;
    if (a.omega) {
      vis = 0;
#pragma unroll
      for (int m = 0; m < KM; ++m)
        if (m < a.K) vis |= ((a.omega[(size_t)m * a.words + wi] >> bi) & 1u) << m;
    }
  }
  float P = 1.f, c0 = 0.f, c1 = 0.f, c2 = 0.f, S = 0.f;
  bool scanning = true;
  bool act[KM];
#pragma unroll
  for (int j = 0; j < KM; ++j) {
#pragma unroll
    for (int m = 0; m < KM; ++m) {
      if (m < a.K && rank[m] == j) {
        if (!RE || ((on >> m) & 1u)) {
          act[m] = P >= a.t_min;
          if (RE && !act[m] && inside) a.budget[(size_t)m * HW + p] = P * (1.f - cm[m].w);
          if (act[m] || !a.same_frame) {
            c0 = fmaf(P, cm[m].x, c0);
            c1 = fmaf(P, cm[m].y, c1);
            c2 = fmaf(P, cm[m].z, c2);
            P = P * cm[m].w;
          }
        } else if ((vis >> m) & 1u) {
          const float R = P - S;
          const float b = (scanning && inside) ? a.budget[(size_t)m * HW + p] : 0.f;
          act[m] = scanning && R >= a.t_min && R >= b;
          if (act[m]) S += b;
          scanning = act[m];
        } else {
          act[m] = false;
        }
      }
    }
  }
  if (inside) a.out[p] = make_float4(c0 + P * a.bg[0], c1 + P * a.bg[1], c2 + P * a.bg[2], P);
  if (a.masks) {
    const int lane = threadIdx.x & 63;
    const uint32_t w0 = (p - lane) >> 5;
#pragma unroll
    for (int m = 0; m < KM; ++m) {
      if (m >= a.K) break;
      // RE rewrites the words (bits past the image cleared); otherwise the
      // pairs that stay active are kept
      const uint64_t keep = __ballot(RE ? (inside && act[m]) : (!inside || act[m]));
      if (lane == 0 || lane == 32) {
        const uint32_t w = w0 + (lane >> 5);
        if (w < a.words) {
          uint32_t* word = a.masks + (size_t)m * a.words + w;
          if (RE)
            *word = (uint32_t)(keep >> lane);
          else
            *word &= (uint32_t)(keep >> lane);
        }
      }
    }
  }
}

// dC_m = P_j G, dT_m = P_j (G . B_{j+1} + g_T U_j), walking the order back
// to front with B the colour behind (background first) and U the product of
// transmittances behind.
template <int KM>
__global__ __launch_bounds__(256) void k_composite_bwd(CompArgs a) {
  const uint32_t HW = (uint32_t)a.W * a.H;
  const uint32_t p = blockIdx.x * 256 + threadIdx.x;
  if (p >= HW) return;
  const int px = (int)(p % a.W), py = (int)(p / a.W);
  int rank[KM];
  cell_ranks<KM>(a, px, py, rank);
  float4 cm[KM];
#pragma unroll
  for (int m = 0; m < KM; ++m) cm[m] = m < a.K ? a.part[m][p] : make_float4(0.f, 0.f, 0.f, 1.f);
  float Pin[KM];
  bool use[KM];
  float P = 1.f;
#pragma unroll
  for (int j = 0; j < KM; ++j) {
#pragma unroll
    for (int m = 0; m < KM; ++m) {
      if (m < a.K && rank[m] == j) {
        Pin[m] = P;
        use[m] = !(a.same_frame && P < a.t_min);
        if (use[m]) P = P * cm[m].w;
      }
    }
  }
  const float4 G = a.dout[p];
  float B0 = a.bg[0], B1 = a.bg[1], B2 = a.bg[2], U = 1.f;
#pragma unroll
  for (int j = KM - 1; j >= 0; --j) {
#pragma unroll
    for (int m = 0; m < KM; ++m) {
      if (m < a.K && rank[m] == j) {
        float4 o = make_float4(0.f, 0.f, 0.f, 0.f);
        if (use[m]) {
          const float Pj = Pin[m];
          o.x = Pj * G.x, o.y = Pj * G.y, o.z = Pj * G.z;
          o.w = Pj * (G.x * B0 + G.y * B1 + G.z * B2 + G.w * U);
          B0 = fmaf(cm[m].w, B0, cm[m].x);
          B1 = fmaf(cm[m].w, B1, cm[m].y);
          B2 = fmaf(cm[m].w, B2, cm[m].z);
          U = U * cm[m].w;
        }
        a.dpart[m][p] = o;
      }
    }
  }
}

// Composition, L1 loss and composition backward in one pass per pixel: the
// same arithmetic as k_composite (clearing rule), k_l1 and k_composite_bwd
// in that order, so the results are bit-identical to the three launches,
// without writing and re-reading dL/d(rgb) or re-reading the partials.
template <int KM>
__global__ __launch_bounds__(256) void k_composite_l1(CompArgs a, const float* __restrict__ target,
                                                      float inv_n, float* loss) {
  const uint32_t HW = (uint32_t)a.W * a.H;
  const uint32_t p = blockIdx.x * 256 + threadIdx.x;
  const bool inside = p < HW;
  const uint32_t pp = inside ? p : 0u;
  const int px = (int)(pp % a.W), py = (int)(pp / a.W);
  int rank[KM];
  cell_ranks<KM>(a, px, py, rank);
  float4 cm[KM];
#pragma unroll
  for (int m = 0; m < KM; ++m)
    cm[m] = (inside && m < a.K) ? a.part[m][pp] : make_float4(0.f, 0.f, 0.f, 1.f);
  float P = 1.f, c0 = 0.f, c1 = 0.f, c2 = 0.f;
  bool act[KM], use[KM];
  float Pin[KM];
#pragma unroll
  for (int j = 0; j < KM; ++j) {
#pragma unroll
    for (int m = 0; m < KM; ++m) {
      if (m < a.K && rank[m] == j) {
        Pin[m] = P;
        act[m] = P >= a.t_min;
        use[m] = act[m] || !a.same_frame;
        if (use[m]) {
          c0 = fmaf(P, cm[m].x, c0);
          c1 = fmaf(P, cm[m].y, c1);
          c2 = fmaf(P, cm[m].z, c2);
          P = P * cm[m].w;
        }
      }
    }
  }
  const float4 o = make_float4(c0 + P * a.bg[0], c1 + P * a.bg[1], c2 + P * a.bg[2], P);
  if (inside) a.out[p] = o;
  if (a.masks) {
    const int lane = threadIdx.x & 63;
    const uint32_t w0 = (p - lane) >> 5;
#pragma unroll
    for (int m = 0; m < KM; ++m) {
      if (m >= a.K) break;
      const uint64_t keep = __ballot(!inside || act[m]);
      if (lane == 0 || lane == 32) {
        const uint32_t w = w0 + (lane >> 5);
        if (w < a.words) a.masks[(size_t)m * a.words + w] &= (uint32_t)(keep >> lane);
      }
    }
  }
  // L1: dL/d(rgb) = sign(rgb - target) / (3HW), dL/dT = 0
  float l = 0.f;
  float4 G = make_float4(0.f, 0.f, 0.f, 0.f);
  if (inside) {
    const float d0 = o.x - target[3 * (size_t)p + 0];
    const float d1 = o.y - target[3 * (size_t)p + 1];
    const float d2 = o.z - target[3 * (size_t)p + 2];
    auto sgn = [](float x) { return x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f); };
    G = make_float4(sgn(d0) * inv_n, sgn(d1) * inv_n, sgn(d2) * inv_n, 0.f);
    l = (fabsf(d0) + fabsf(d1) + fabsf(d2)) * inv_n;
  }
  if (loss) {
    for (int off = 32; off >= 1; off >>= 1) l += __shfl_xor(l, off, 64);
    if ((threadIdx.x & 63) == 0) unsafeAtomicAdd(loss, l);
  }
  if (!inside) return;
  float B0 = a.bg[0], B1 = a.bg[1], B2 = a.bg[2], U = 1.f;
#pragma unroll
  for (int j = KM - 1; j >= 0; --j) {
#pragma unroll
    for (int m = 0; m < KM; ++m) {
      if (m < a.K && rank[m] == j) {
        float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
        if (use[m]) {
          const float Pj = Pin[m];
          q.x = Pj * G.x, q.y = Pj * G.y, q.z = Pj * G.z;
          q.w = Pj * (G.x * B0 + G.y * B1 + G.z * B2 + G.w * U);
          B0 = fmaf(cm[m].w, B0, cm[m].x);
          B1 = fmaf(cm[m].w, B1, cm[m].y);
          B2 = fmaf(cm[m].w, B2, cm[m].z);
          U = U * cm[m].w;
        }
        a.dpart[m][p] = q;
      }
    }
  }
}

static CompArgs comp_args(int K, const float* const* partials, const sx_cell* cells,
                          const DCam& cam, const KParams& p) {
  CompArgs a{};
  a.K = K;
  for (int m = 0; m < K; ++m) {
    a.part[m] = reinterpret_cast<const float4*>(partials[m]);
    for (int j = 0; j < 3; ++j) a.lo[m][j] = cells[m].lo[j], a.hi[m][j] = cells[m].hi[j];
  }
  for (int j = 0; j < 3; ++j) a.O[j] = (float)cam.C[j];
  for (int j = 0; j < 9; ++j) a.Rm[j] = (float)cam.R[j];
  a.fx = (float)cam.fx, a.fy = (float)cam.fy, a.cx = (float)cam.cx, a.cy = (float)cam.cy;
  a.W = cam.W, a.H = cam.H;
  a.t_min = p.t_min;
  for (int j = 0; j < 3; ++j) a.bg[j] = p.bg[j];
  a.same_frame = (p.flags & SX_FLAG_SAME_FRAME_CULL) ? 1 : 0;
  return a;
}

// ---------------------------------------------------- geometric visibility
// Visible-pixel maps of the cell boxes (redundancy reduction, spatial part):
// the part of a box inside the view frustum is convex and projects onto the
// pixels whose centre ray meets it.  The ray point C + s d has camera depth
// s, so the ray meets (box within the frustum) iff the box's slab interval
// cut below by the near plane is not empty.  FP64 throughout, with the same
// operations in the same order as the oracle, so the maps agree bit for
// bit.  One lane per pixel; a wavefront covers two mask words and writes
// them from one ballot.
struct VisArgs {
  int K;
  double lo[kMaxCells][3], hi[kMaxCells][3];
  DCam cam;
  uint32_t* masks;
  uint32_t words;
};

__device__ __forceinline__ bool ray_meets_box(const DCam& c, int px, int py, const double lo[3],
                                              const double hi[3]) {
  const double u = ((double)px + 0.5 - c.cx) / c.fx, v = ((double)py + 0.5 - c.cy) / c.fy;
  double d[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) d[j] = c.R[0 * 3 + j] * u + c.R[1 * 3 + j] * v + c.R[2 * 3 + j] * 1.0;
  double s_in = c.znear, s_out = INFINITY;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    if (d[j] == 0.0) {
      if (c.C[j] < lo[j] || c.C[j] > hi[j]) return false;
      continue;
    }
    const double t1 = (lo[j] - c.C[j]) / d[j], t2 = (hi[j] - c.C[j]) / d[j];
    s_in = fmax(s_in, fmin(t1, t2));
    s_out = fmin(s_out, fmax(t1, t2));
  }
  return s_in <= s_out;
}

__global__ __launch_bounds__(256) void k_visibility(VisArgs a) {
  const uint32_t HW = (uint32_t)a.cam.W * a.cam.H;
  const uint32_t p = blockIdx.x * 256 + threadIdx.x;
  const bool inside = p < HW;
  const uint32_t pp = inside ? p : 0u;
  const int px = (int)(pp % a.cam.W), py = (int)(pp / a.cam.W);
  const int lane = threadIdx.x & 63;
  const uint32_t w0 = (p - lane) >> 5;
  for (int m = 0; m < a.K; ++m) {
    const bool vis = inside && ray_meets_box(a.cam, px, py, a.lo[m], a.hi[m]);
    const uint64_t b = __ballot(vis);
    if (lane == 0 || lane == 32) {
      const uint32_t w = w0 + (lane >> 5);
      if (w < a.words) a.masks[(size_t)m * a.words + w] = (uint32_t)(b >> lane);
    }
  }
}

hipError_t launch_visibility(int K, const sx_cell* cells, const DCam& cam, uint32_t* masks,
                             hipStream_t st) {
  VisArgs a;
  a.K = K;
  for (int m = 0; m < K; ++m)
    for (int j = 0; j < 3; ++j) a.lo[m][j] = cells[m].lo[j], a.hi[m][j] = cells[m].hi[j];
  a.cam = cam;
  a.masks = masks;
  const uint64_t HW = (uint64_t)cam.W * cam.H;
  a.words = (uint32_t)((HW + 31) / 32);
  hipLaunchKernelGGL(k_visibility, dim3((unsigned)((HW + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

// Set bits per row of K mask rows of `words` words (a cell's visible pixels
// in a geometric map): one row per grid row, a wavefront sum per block and
// one integer atomic per block (the order of the integer sums is free).
__global__ __launch_bounds__(256) void k_mask_counts(const uint32_t* __restrict__ masks,
                                                     int64_t words, uint32_t* counts) {
  const int m = blockIdx.y;
  uint32_t c = 0;
  for (int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x; w < words;
       w += (int64_t)gridDim.x * 256)
    c += __popc(masks[(int64_t)m * words + w]);
  for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(&counts[m], c);
}

hipError_t launch_mask_counts(int K, const uint32_t* masks, int64_t words, uint32_t* counts,
                              hipStream_t st) {
  hipError_t e = launch_fill(counts, K, 0, st);
  if (e != hipSuccess || words == 0) return e;
  int64_t bx = (words + 255) / 256;
  if (bx > 256) bx = 256;
  hipLaunchKernelGGL(k_mask_counts, dim3((unsigned)bx, (unsigned)K), dim3(256), 0, st, masks,
                     words, counts);
  return hipGetLastError();
}

template <bool RE>
static void launch_comp_k(int K, dim3 grid, const CompArgs& a, hipStream_t st) {
  if (K <= 1)
    hipLaunchKernelGGL((k_composite<1, RE>), grid, dim3(256), 0, st, a);
  else if (K <= 2)
    hipLaunchKernelGGL((k_composite<2, RE>), grid, dim3(256), 0, st, a);
  else if (K <= 4)
    hipLaunchKernelGGL((k_composite<4, RE>), grid, dim3(256), 0, st, a);
  else if (K <= 8)
    hipLaunchKernelGGL((k_composite<8, RE>), grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_composite<16, RE>), grid, dim3(256), 0, st, a);
}

hipError_t launch_composite(int K, const float* const* partials,
                            const sx_cell* cells, const DCam& cam,
                            const KParams& p, float* out, uint32_t* masks,
                            const uint32_t* omega, float* budget, hipStream_t st) {
  CompArgs a = comp_args(K, partials, cells, cam, p);
  a.out = reinterpret_cast<float4*>(out);
  a.masks = masks;
  a.omega = omega;
  a.budget = budget;
  const uint32_t HW = (uint32_t)cam.W * cam.H;
  a.words = (HW + 31) / 32;
  const dim3 grid((HW + 255) / 256);
  if (budget)
    launch_comp_k<true>(K, grid, a, st);
  else
    launch_comp_k<false>(K, grid, a, st);
  return hipGetLastError();
}

hipError_t launch_composite_backward(int K, const float* const* partials,
                                     const sx_cell* cells, const DCam& cam,
                                     const KParams& p, const float* dout,
                                     float* const* dpartials, hipStream_t st) {
  CompArgs a = comp_args(K, partials, cells, cam, p);
  a.dout = reinterpret_cast<const float4*>(dout);
  for (int m = 0; m < K; ++m) a.dpart[m] = reinterpret_cast<float4*>(dpartials[m]);
  const uint32_t HW = (uint32_t)cam.W * cam.H;
  const dim3 grid((HW + 255) / 256);
  if (K <= 1)
    hipLaunchKernelGGL(k_composite_bwd<1>, grid, dim3(256), 0, st, a);
  else if (K <= 2)
    hipLaunchKernelGGL(k_composite_bwd<2>, grid, dim3(256), 0, st, a);
  else if (K <= 4)
    hipLaunchKernelGGL(k_composite_bwd<4>, grid, dim3(256), 0, st, a);
  else if (K <= 8)
    hipLaunchKernelGGL(k_composite_bwd<8>, grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(k_composite_bwd<16>, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_composite_l1(int K, const float* const* partials, const sx_cell* cells,
                               const DCam& cam, const KParams& p, const float* target,
                               float* out, uint32_t* masks, float* loss,
                               float* const* dpartials, hipStream_t st) {
  CompArgs a = comp_args(K, partials, cells, cam, p);
  a.out = reinterpret_cast<float4*>(out);
  a.masks = masks;
  const uint32_t HW = (uint32_t)cam.W * cam.H;
  a.words = (HW + 31) / 32;
  for (int m = 0; m < K; ++m) a.dpart[m] = reinterpret_cast<float4*>(dpartials[m]);
  const float inv_n = 1.f / (3.f * (float)HW);
  const dim3 grid((HW + 255) / 256);
  if (K <= 1)
    hipLaunchKernelGGL(k_composite_l1<1>, grid, dim3(256), 0, st, a, target, inv_n, loss);
  else if (K <= 2)
    hipLaunchKernelGGL(k_composite_l1<2>, grid, dim3(256), 0, st, a, target, inv_n, loss);
  else if (K <= 4)
    hipLaunchKernelGGL(k_composite_l1<4>, grid, dim3(256), 0, st, a, target, inv_n, loss);
  else if (K <= 8)
    hipLaunchKernelGGL(k_composite_l1<8>, grid, dim3(256), 0, st, a, target, inv_n, loss);
  else
    hipLaunchKernelGGL(k_composite_l1<16>, grid, dim3(256), 0, st, a, target, inv_n, loss);
  return hipGetLastError();
}

// ----------------------------------------------------------------- loss --
__global__ __launch_bounds__(256) void k_l1(const float4* __restrict__ out,
                                            const float* __restrict__ target, uint32_t HW,
                                            float inv_n, float4* __restrict__ dout,
                                            float* loss) {
  const uint32_t p = blockIdx.x * 256 + threadIdx.x;
  float l = 0.f;
  if (p < HW) {
    const float4 o = out[p];
    const float d0 = o.x - target[3 * (size_t)p + 0];
    const float d1 = o.y - target[3 * (size_t)p + 1];
    const float d2 = o.z - target[3 * (size_t)p + 2];
    auto sgn = [](float x) { return x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f); };
    dout[p] = make_float4(sgn(d0) * inv_n, sgn(d1) * inv_n, sgn(d2) * inv_n, 0.f);
    l = (fabsf(d0) + fabsf(d1) + fabsf(d2)) * inv_n;
  }
  if (loss) {
    for (int o = 32; o >= 1; o >>= 1) l += __shfl_xor(l, o, 64);
    if ((threadIdx.x & 63) == 0) unsafeAtomicAdd(loss, l);
  }
}

hipError_t launch_l1(const float* out, const float* target, int W, int H,
                     float* dout, float* loss, hipStream_t st) {
  const uint32_t HW = (uint32_t)W * H;
  hipLaunchKernelGGL(k_l1, dim3((HW + 255) / 256), dim3(256), 0, st,
                     reinterpret_cast<const float4*>(out), target, HW, 1.f / (3.f * (float)HW),
                     reinterpret_cast<float4*>(dout), loss);
  return hipGetLastError();
}

// ----------------------------------------------------------------- Adam --
__device__ __forceinline__ void adam1(float& p, float g, float& m, float& v, float lr, float b1,
                                      float b2, float eps, float bc1, float bc2) {
  m = b1 * m + (1.f - b1) * g;
  v = b2 * v + (1.f - b2) * g * g;
  const float mh = m / bc1, vh = v / bc2;
  p = p - lr * mh / (sqrtf(vh) + eps);
}

__global__ __launch_bounds__(256) void k_adam(int64_t n, float* __restrict__ param,
                                              const float* __restrict__ grad, float* __restrict__ m,
                                              float* __restrict__ v, float lr, float b1, float b2,
                                              float eps, float bc1, float bc2, int vec) {
  if (!vec) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride)
      adam1(param[i], grad[i], m[i], v[i], lr, b1, b2, eps, bc1, bc2);
    return;
  }
  const int64_t n4 = n / 4;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += stride) {
    float4 P = reinterpret_cast<float4*>(param)[i];
    const float4 G = reinterpret_cast<const float4*>(grad)[i];
    float4 M = reinterpret_cast<float4*>(m)[i];
    float4 V = reinterpret_cast<float4*>(v)[i];
    adam1(P.x, G.x, M.x, V.x, lr, b1, b2, eps, bc1, bc2);
    adam1(P.y, G.y, M.y, V.y, lr, b1, b2, eps, bc1, bc2);
    adam1(P.z, G.z, M.z, V.z, lr, b1, b2, eps, bc1, bc2);
    adam1(P.w, G.w, M.w, V.w, lr, b1, b2, eps, bc1, bc2);
    reinterpret_cast<float4*>(param)[i] = P;
    reinterpret_cast<float4*>(m)[i] = M;
    reinterpret_cast<float4*>(v)[i] = V;
  }
  if (blockIdx.x == 0 && threadIdx.x < (n & 3)) {
    const int64_t i = n4 * 4 + threadIdx.x;
    adam1(param[i], grad[i], m[i], v[i], lr, b1, b2, eps, bc1, bc2);
  }
}

hipError_t launch_adam(int64_t n, float* param, const float* grad, float* m,
                       float* v, float lr, float b1, float b2, float eps,
                       float bc1, float bc2, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n / 4 + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 16384) blocks = 16384;
  const uintptr_t al = reinterpret_cast<uintptr_t>(param) | reinterpret_cast<uintptr_t>(grad) |
                       reinterpret_cast<uintptr_t>(m) | reinterpret_cast<uintptr_t>(v);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0, st, n, param, grad, m, v, lr,
                     b1, b2, eps, bc1, bc2, (al & 15) == 0 ? 1 : 0);
  return hipGetLastError();
}

}  // namespace sx
