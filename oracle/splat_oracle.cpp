// FP64 CPU oracle for pixel-level Gaussian splatting.
//
// TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
// call this library; it exists so that tests, the smoke check and the CPU
// baseline leg of the benchmark can compare the HIP path against a plain,
// slow, obviously correct implementation written from the paper:
//
//   * Gaussian parametrisation Sigma = R S S^T R^T and EWA projection
//     Sigma2D = J W Sigma W^T J^T            (paper, background: projection)
//   * per-pixel alpha  o * exp(-1/2 d^T Sigma2D^-1 d)   (Eq. 1)
//   * front-to-back blending C = sum c_i alpha_i T_i   (Eq. 2)
//   * per-cell partial colour / transmittance / depth  (Eq. 3-4)
//   * composition of partials in ray order             (Eq. 5)
//   * gradients through the composition                (Eq. 6-7)
//   * transmittance-saturation masks (redundancy reduction, saturation part)
//     and their speculative re-evaluation (appendix, saturation stability)
//   * geometric visibility of cell boxes (redundancy reduction, spatial part)
//   * per-ray cross-boundary filter (appendix, cross-boundary Gaussians)
//
// Everything is computed in double precision from the caller's inputs.  The
// per-pixel list is "every Gaussian whose footprint can reach the pixel",
// ordered by (float32(depth) bits, index); the "binned" mode gathers those
// Gaussians through exact-extent tile bins and must agree bit-for-bit with
// the "brute" mode that scans every Gaussian for every pixel.
//
// Where the paper is silent the following readings are used (all parameters
// below are caller-supplied):
//   alpha = min(alpha_max, o*exp(-q/2)); a pair is skipped iff alpha <
//   alpha_min; after each blend the walk stops once T < t_min ("blend, then
//   stop"); Sigma2D gets eps2d*I added; culling by mean depth z <= znear, by
//   a mean that projects outside the field of view widened by the guard
//   factor fov_guard (0 = no lateral test), by degenerate covariance, by
//   o < alpha_min and by an empty footprint; colour
//   is the orthonormal real spherical-harmonic expansion plus 0.5, clamped at
//   0; the partial depth is D = sum z_i alpha_i T_i; cells are ordered per
//   pixel by the ray's entry parameter into their box (max(0, t_near)), ties
//   by cell index.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

constexpr int LMAX = 3;
constexpr double PI = 3.14159265358979323846;

struct Cam {
  double R[9];
  double t[3];
  double fx, fy, cx, cy, znear;
  int32_t width, height;
};

struct Params {
  int32_t tile_w, tile_h, sh_degree, same_frame_cull;
  double alpha_min, alpha_max, t_min, eps2d;
  double bg[3];
  double delta_q;  // extra absolute half-width of the alpha-threshold band
  double fov_guard;  // field-of-view cull: half-extents scaled by this (0 = off)
};

// Per-Gaussian projected record, all double.
struct Proj {
  uint8_t valid;
  double depth;        // camera-space z
  double tc[3];        // camera-space position
  double mean2d[2];
  double cov2d[3];     // xx, xy, yy (dilated)
  double conic[3];     // a, b, c of Sigma2D^-1
  double opacity;
  double rgb[3];
  uint8_t rgb_pos[3];  // pre-clamp value > 0
  double tau;          // 2 ln(o / alpha_min)
  int32_t pix[4];      // inclusive pixel rect x0,y0,x1,y1
  int32_t tile[4];     // inclusive tile rect
  int64_t n_tiles;
  float zf;            // float32(depth): the sort key
  double zerr;         // bound on the rounding error of depth (0 if exact)
  double dirv[3];      // unit view direction used for SH
  double dist;         // |mu - camera centre|
};

// ---------------------------------------------------------------- SH ------
// Real orthonormal spherical harmonics with the Condon-Shortley phase,
//   Y_l^0 = K_l^0 P_l^0(cos th),
//   Y_l^m = sqrt2 K_l^m P_l^m(cos th) cos(m ph),    m > 0
//   Y_l^-m = sqrt2 K_l^m P_l^m(cos th) sin(m ph),   m > 0
// with K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).  Written as polynomials in
// the unit direction (x, y, z): P_l^m(z) sin^m(th) e^{i m ph} =
// (-1)^m P_l^(m)(z) (x + i y)^m, where P_l^(m) is the m-th derivative of the
// Legendre polynomial, whose coefficients come from Bonnet's recursion.
struct SHTables {
  double leg[LMAX + 2][LMAX + 2];  // leg[l][k]: coefficient of z^k in P_l
  double K[LMAX + 1][LMAX + 1];
  SHTables() {
    std::memset(leg, 0, sizeof(leg));
    leg[0][0] = 1.0;
    leg[1][1] = 1.0;
    for (int n = 1; n < LMAX + 1; ++n)  // (n+1) P_{n+1} = (2n+1) z P_n - n P_{n-1}
      for (int k = 0; k <= n + 1; ++k) {
        double v = 0.0;
        if (k >= 1) v += (2 * n + 1) * leg[n][k - 1];
        v -= n * leg[n - 1][k];
        leg[n + 1][k] = v / (n + 1);
      }
    for (int l = 0; l <= LMAX; ++l)
      for (int m = 0; m <= l; ++m) {
        double r = 1.0;  // (l-m)!/(l+m)!
        for (int i = l - m + 1; i <= l + m; ++i) r /= i;
        K[l][m] = std::sqrt((2 * l + 1) / (4.0 * PI) * r);
      }
  }
  // j-th derivative of P_l evaluated at z
  double dleg(int l, int j, double z) const {
    double s = 0.0;
    for (int k = LMAX + 1; k >= j; --k) {
      double c = leg[l][k];
      for (int i = 0; i < j; ++i) c *= (k - i);
      s = s * z + c;
    }
    // the loop above evaluates sum_k c_k z^(k-j) in Horner form
    return s;
  }
};

const SHTables& sh_tables() {
  static SHTables t;
  return t;
}

// (x + i y)^m as (re, im)
static void cpow(double x, double y, int m, double* re, double* im) {
  double a = 1.0, b = 0.0;
  for (int i = 0; i < m; ++i) {
    double na = a * x - b * y, nb = a * y + b * x;
    a = na;
    b = nb;
  }
  *re = a;
  *im = b;
}

// Y[(l*l+l+m)] and, if grad != nullptr, the gradient of the polynomial
// extension with respect to (x, y, z).
static void sh_eval(int degree, const double d[3], double* Y, double* grad) {
  const SHTables& T = sh_tables();
  const double x = d[0], y = d[1], z = d[2];
  for (int l = 0; l <= degree; ++l) {
    for (int m = -l; m <= l; ++m) {
      const int am = m < 0 ? -m : m;
      const double N = (am == 0 ? 1.0 : std::sqrt(2.0)) * T.K[l][am] *
                       ((am & 1) ? -1.0 : 1.0);
      const double P = T.dleg(l, am, z);
      const double dP = T.dleg(l, am + 1, z);
      double re, im, re1 = 0.0, im1 = 0.0;
      cpow(x, y, am, &re, &im);
      if (am >= 1) cpow(x, y, am - 1, &re1, &im1);
      const int idx = l * l + l + m;
      if (m >= 0) {
        Y[idx] = N * P * re;
        if (grad) {
          grad[idx * 3 + 0] = N * P * am * re1;
          grad[idx * 3 + 1] = -N * P * am * im1;
          grad[idx * 3 + 2] = N * dP * re;
        }
      } else {
        Y[idx] = N * P * im;
        if (grad) {
          grad[idx * 3 + 0] = N * P * am * im1;
          grad[idx * 3 + 1] = N * P * am * re1;
          grad[idx * 3 + 2] = N * dP * im;
        }
      }
    }
  }
}

// ------------------------------------------------------------ geometry ----
static void quat_to_rot(const double q[4], double R[9]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z);
  R[1] = 2 * (x * y - w * z);
  R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);
  R[4] = 1 - 2 * (x * x + z * z);
  R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);
  R[7] = 2 * (y * z + w * x);
  R[8] = 1 - 2 * (x * x + y * y);
}

static void matmul3(const double* A, const double* B, double* C) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += A[i * 3 + k] * B[k * 3 + j];
      C[i * 3 + j] = s;
    }
}
static void transpose3(const double* A, double* B) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) B[j * 3 + i] = A[i * 3 + j];
}

static void cam_center(const Cam& c, double C[3]) {
  for (int j = 0; j < 3; ++j)
    C[j] = -(c.R[0 * 3 + j] * c.t[0] + c.R[1 * 3 + j] * c.t[1] +
             c.R[2 * 3 + j] * c.t[2]);
}

struct Gauss {  // one Gaussian's raw parameters, double
  double mu[3], ls[3], q[4], logit;
  const double* sh;  // (D+1)^2 * 3
};

static void preprocess_one(const Gauss& g, const Cam& cam, const Params& P,
                           Proj& o) {
  std::memset(&o, 0, sizeof(Proj));
  o.valid = 0;
  // camera transform, cull by mean depth
  double t[3];
  for (int i = 0; i < 3; ++i)
    t[i] = cam.R[i * 3 + 0] * g.mu[0] + cam.R[i * 3 + 1] * g.mu[1] +
           cam.R[i * 3 + 2] * g.mu[2] + cam.t[i];
  o.tc[0] = t[0];
  o.tc[1] = t[1];
  o.tc[2] = t[2];
  {
    // products of two floats are exact in double; the three additions can
    // each round.  Exact when every partial sum is representable.
    const double p0 = cam.R[6] * g.mu[0], p1 = cam.R[7] * g.mu[1], p2 = cam.R[8] * g.mu[2];
    const double mag = std::fabs(p0) + std::fabs(p1) + std::fabs(p2) + std::fabs(cam.t[2]);
    const double s1 = p0 + p1, s2 = s1 + p2, s3 = s2 + cam.t[2];
    const bool exact = (s1 - p0 == p1) && (s2 - s1 == p2) && (s3 - s2 == cam.t[2]);
    o.zerr = exact ? 0.0 : std::ldexp(mag, -50);
  }
  o.depth = t[2];
  o.zf = (float)t[2];
  if (!(t[2] > cam.znear)) return;
  // frustum cull by the mean (background, projection step): the mean's
  // offset from the principal point, fx*x/z and fy*y/z in pixels, must lie
  // within the image's half-extents on each side, scaled by fov_guard
  if (P.fov_guard > 0.0) {
    const double ux = cam.fx * t[0] / t[2], uy = cam.fy * t[1] / t[2];
    if (ux < -(P.fov_guard * cam.cx) || ux > P.fov_guard * ((double)cam.width - cam.cx) ||
        uy < -(P.fov_guard * cam.cy) || uy > P.fov_guard * ((double)cam.height - cam.cy))
      return;
  }
  double qn = std::sqrt(g.q[0] * g.q[0] + g.q[1] * g.q[1] + g.q[2] * g.q[2] +
                        g.q[3] * g.q[3]);
  if (qn < 1e-12) return;
  double qh[4] = {g.q[0] / qn, g.q[1] / qn, g.q[2] / qn, g.q[3] / qn};
  double Rq[9];
  quat_to_rot(qh, Rq);
  double s2[3];
  for (int k = 0; k < 3; ++k) {
    double s = std::exp(g.ls[k]);
    s2[k] = s * s;
  }
  double Sig[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double v = 0;
      for (int k = 0; k < 3; ++k) v += Rq[i * 3 + k] * s2[k] * Rq[j * 3 + k];
      Sig[i * 3 + j] = v;
    }
  double WT[9], tmp[9], M[9];
  transpose3(cam.R, WT);
  matmul3(cam.R, Sig, tmp);
  matmul3(tmp, WT, M);
  const double z = t[2];
  double J[6] = {cam.fx / z, 0.0, -cam.fx * t[0] / (z * z),
                 0.0, cam.fy / z, -cam.fy * t[1] / (z * z)};
  double JM[6];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) {
      double v = 0;
      for (int k = 0; k < 3; ++k) v += J[i * 3 + k] * M[k * 3 + j];
      JM[i * 3 + j] = v;
    }
  double S2[4];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      double v = 0;
      for (int k = 0; k < 3; ++k) v += JM[i * 3 + k] * J[j * 3 + k];
      S2[i * 2 + j] = v;
    }
  const double cxx = S2[0] + P.eps2d, cxy = 0.5 * (S2[1] + S2[2]),
               cyy = S2[3] + P.eps2d;
  o.cov2d[0] = cxx;
  o.cov2d[1] = cxy;
  o.cov2d[2] = cyy;
  const double det = cxx * cyy - cxy * cxy;
  if (!(det > 0.0)) return;
  o.conic[0] = cyy / det;
  o.conic[1] = -cxy / det;
  o.conic[2] = cxx / det;
  o.mean2d[0] = cam.fx * t[0] / z + cam.cx;
  o.mean2d[1] = cam.fy * t[1] / z + cam.cy;
  o.opacity = 1.0 / (1.0 + std::exp(-g.logit));
  if (o.opacity < P.alpha_min) return;
  o.tau = 2.0 * std::log(o.opacity / P.alpha_min);
  const double ex = std::sqrt(o.tau * cxx), ey = std::sqrt(o.tau * cyy);
  auto clampd = [](double v, double lo, double hi) {
    return v < lo ? lo : (v > hi ? hi : v);
  };
  double x0 = std::ceil(o.mean2d[0] - ex - 0.5);
  double x1 = std::floor(o.mean2d[0] + ex - 0.5);
  double y0 = std::ceil(o.mean2d[1] - ey - 0.5);
  double y1 = std::floor(o.mean2d[1] + ey - 0.5);
  x0 = clampd(x0, 0.0, (double)cam.width);
  y0 = clampd(y0, 0.0, (double)cam.height);
  x1 = clampd(x1, -1.0, (double)cam.width - 1);
  y1 = clampd(y1, -1.0, (double)cam.height - 1);
  if (!(x0 <= x1 && y0 <= y1)) return;
  o.pix[0] = (int32_t)x0;
  o.pix[1] = (int32_t)y0;
  o.pix[2] = (int32_t)x1;
  o.pix[3] = (int32_t)y1;
  o.tile[0] = o.pix[0] / P.tile_w;
  o.tile[1] = o.pix[1] / P.tile_h;
  o.tile[2] = o.pix[2] / P.tile_w;
  o.tile[3] = o.pix[3] / P.tile_h;
  o.n_tiles = (int64_t)(o.tile[2] - o.tile[0] + 1) * (o.tile[3] - o.tile[1] + 1);
  // colour from the view direction
  double C[3];
  cam_center(cam, C);
  double dv[3] = {g.mu[0] - C[0], g.mu[1] - C[1], g.mu[2] - C[2]};
  double dn = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
  o.dist = dn;
  for (int k = 0; k < 3; ++k) o.dirv[k] = dv[k] / dn;
  const int nc = (P.sh_degree + 1) * (P.sh_degree + 1);
  double Y[(LMAX + 1) * (LMAX + 1)];
  sh_eval(P.sh_degree, o.dirv, Y, nullptr);
  for (int ch = 0; ch < 3; ++ch) {
    double v = 0.0;
    for (int i = 0; i < nc; ++i) v += g.sh[i * 3 + ch] * Y[i];
    v += 0.5;
    o.rgb_pos[ch] = v > 0.0;
    o.rgb[ch] = v > 0.0 ? v : 0.0;
  }
  o.valid = 1;
}

// -------------------------------------------------------------- scene ----
struct SceneIn {
  int64_t n;
  const double *means, *log_scales, *quats, *logits, *sh;
};

static Gauss gauss_at(const SceneIn& s, int64_t i, int nc) {
  Gauss g;
  for (int k = 0; k < 3; ++k) {
    g.mu[k] = s.means[i * 3 + k];
    g.ls[k] = s.log_scales[i * 3 + k];
  }
  for (int k = 0; k < 4; ++k) g.q[k] = s.quats[i * 4 + k];
  g.logit = s.logits[i];
  g.sh = s.sh + (size_t)i * nc * 3;
  return g;
}

static std::vector<Proj> preprocess_all(const SceneIn& s, const Cam& cam,
                                        const Params& P) {
  std::vector<Proj> pr((size_t)s.n);
  const int nc = (P.sh_degree + 1) * (P.sh_degree + 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < s.n; ++i) preprocess_one(gauss_at(s, i, nc), cam, P, pr[i]);
  return pr;
}

static inline uint32_t fbits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return u;
}

// Gaussian order on a ray: (float32 depth bits, index); depth > znear > 0 so
// the IEEE bit pattern orders like the value.
static inline bool ray_less(const std::vector<Proj>& pr, int64_t a, int64_t b) {
  uint32_t ka = fbits(pr[a].zf), kb = fbits(pr[b].zf);
  return ka < kb || (ka == kb && a < b);
}

struct Bins {
  int tiles_x = 0, tiles_y = 0;
  std::vector<std::vector<int64_t>> lists;  // per tile, sorted ray order
};

static Bins make_bins(const std::vector<Proj>& pr, const Cam& cam,
                      const Params& P) {
  Bins b;
  b.tiles_x = (cam.width + P.tile_w - 1) / P.tile_w;
  b.tiles_y = (cam.height + P.tile_h - 1) / P.tile_h;
  b.lists.assign((size_t)b.tiles_x * b.tiles_y, {});
  for (int64_t i = 0; i < (int64_t)pr.size(); ++i) {
    const Proj& p = pr[i];
    if (!p.valid) continue;
    for (int ty = p.tile[1]; ty <= p.tile[3]; ++ty)
      for (int tx = p.tile[0]; tx <= p.tile[2]; ++tx)
        b.lists[(size_t)ty * b.tiles_x + tx].push_back(i);
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t t = 0; t < (int64_t)b.lists.size(); ++t)
    std::sort(b.lists[t].begin(), b.lists[t].end(),
              [&](int64_t a, int64_t c) { return ray_less(pr, a, c); });
  return b;
}

static std::vector<int64_t> brute_list(const std::vector<Proj>& pr) {
  std::vector<int64_t> all;
  for (int64_t i = 0; i < (int64_t)pr.size(); ++i)
    if (pr[i].valid) all.push_back(i);
  std::sort(all.begin(), all.end(),
            [&](int64_t a, int64_t c) { return ray_less(pr, a, c); });
  return all;
}

// flag bits (ambiguity of the FP32 path against this FP64 reference)
enum : uint8_t {
  FLAG_ALPHA_BAND = 1,   // a pair's q lies within rounding reach of tau
  FLAG_TERMINATE = 2,    // transmittance within 1e-3 relative of t_min
  FLAG_DEPTH_ROUND = 4,  // float32(depth) rounding could go either way
  FLAG_ORDER = 8,        // two cell entry keys within 1e-6 relative
  FLAG_CLAMP = 16,       // alpha within 1e-6 relative of the alpha_max clamp
  FLAG_VISIBILITY = 32,  // a cell box's geometric visibility within rounding of flipping
  FLAG_SATURATION = 64,  // a saturation or re-activation test within 1e-3 relative
                         // of its threshold
  FLAG_CROSS = 128,      // a cross-boundary filter decision within rounding reach
};

// Per-ray cross-boundary filter of one cell's render (appendix,
// implementation details: cross-boundary Gaussians): pair (g, pixel) is
// dropped when xf[g] & pbits != 0, pbits being the cells whose box the
// pixel's ray meets (zero where it misses the rendering cell's own box);
// xamb[g] marks the bits whose decision is within rounding reach.
struct XFilter {
  const uint32_t* xf;
  const uint32_t* xamb;
  uint32_t pbits;
};

struct Blend {  // one blended pair on a pixel's ray
  int64_t g;
  double alpha, gval, Ti, dx, dy;
  bool clamped;
};

// float32(depth) could round the other way if the depth computed in double
// elsewhere (different summation order) differs by its rounding error `err`
// and the value sits that close to a float32 rounding midpoint.  A value
// exactly on a midpoint is not ambiguous when the double computation was
// exact (both sides then round ties-to-even alike); `err` is zero then.
static inline bool depth_round_ambiguous(double z, double err) {
  if (err == 0.0) return false;
  float f = (float)z;
  double lo = (double)std::nextafter(f, -INFINITY), hi = (double)std::nextafter(f, INFINITY);
  double m1 = 0.5 * (lo + (double)f), m2 = 0.5 * ((double)f + hi);
  return std::fabs(z - m1) <= err || std::fabs(z - m2) <= err;
}

// Walk one pixel's ordered list (Eq. 1-4).  Returns the blended pairs and
// accumulates C, T, D, flags.
template <class List>
static void walk_pixel(const std::vector<Proj>& pr, const List& list, int px,
                       int py, const Cam& cam, const Params& P, double C[3],
                       double* Tout, double* Dout, int* nblend, uint8_t* flags,
                       std::vector<Blend>* blends, const XFilter* xfil = nullptr) {
  double T = 1.0, D = 0.0;
  C[0] = C[1] = C[2] = 0.0;
  int nb = 0;
  uint8_t fl = 0;
  const double x = px + 0.5, y = py + 0.5;
  for (int64_t g : list) {
    const Proj& p = pr[g];
    const double dx = x - p.mean2d[0], dy = y - p.mean2d[1];
    const double a = p.conic[0], b = p.conic[1], c = p.conic[2];
    const double q = a * dx * dx + 2.0 * b * dx * dy + c * dy * dy;
    // rounding reach of the FP32 evaluation of q (conic, mean and the
    // arithmetic are each rounded once to float) plus the caller's margin
    const double qa = std::fabs(a) * dx * dx + 2.0 * std::fabs(b * dx * dy) +
                      std::fabs(c) * dy * dy;
    const double gx = std::fabs(a * dx + b * dy), gy = std::fabs(b * dx + c * dy);
    const double mc = std::max(std::fabs(p.mean2d[0] - cam.cx),
                               std::fabs(p.mean2d[1] - cam.cy)) + 2.0;
    const double dmu = std::ldexp(mc, -23);
    const double band = 4.0 * (2e-6 * (1.0 + qa) + 2.0 * (gx + gy) * dmu) + P.delta_q;
    if (std::fabs(q - p.tau) <= band) fl |= FLAG_ALPHA_BAND;
    const double gval = std::exp(-0.5 * q);
    const double araw = p.opacity * gval;
    const bool clamped = araw > P.alpha_max;
    const double alpha = clamped ? P.alpha_max : araw;
    if (alpha < P.alpha_min) continue;
    if (xfil) {
      if (xfil->xamb[g] & xfil->pbits) fl |= FLAG_CROSS;
      if (xfil->xf[g] & xfil->pbits) continue;  // removed from this ray
    }
    if (std::fabs(araw - P.alpha_max) <= 1e-6 * P.alpha_max) fl |= FLAG_CLAMP;
    if (depth_round_ambiguous(p.depth, p.zerr)) fl |= FLAG_DEPTH_ROUND;
    if (blends) blends->push_back({g, alpha, gval, T, dx, dy, clamped});
    const double w = alpha * T;
    for (int k = 0; k < 3; ++k) C[k] += p.rgb[k] * w;
    D += p.depth * w;
    T *= (1.0 - alpha);
    ++nb;
    if (std::fabs(T - P.t_min) <= 1e-3 * P.t_min) fl |= FLAG_TERMINATE;
    if (T < P.t_min) break;
  }
  *Tout = T;
  *Dout = D;
  *nblend = nb;
  *flags |= fl;
}

// ------------------------------------------------------------ composite --
static double entry_key(const Cam& cam, int px, int py, const double lo[3],
                        const double hi[3]) {
  double O[3];
  cam_center(cam, O);
  const double u = (px + 0.5 - cam.cx) / cam.fx, v = (py + 0.5 - cam.cy) / cam.fy;
  double d[3];
  for (int j = 0; j < 3; ++j)
    d[j] = cam.R[0 * 3 + j] * u + cam.R[1 * 3 + j] * v + cam.R[2 * 3 + j] * 1.0;
  double tn = -INFINITY;
  for (int j = 0; j < 3; ++j) {
    if (d[j] == 0.0) continue;  // parallel to the slab: no entry constraint
    const double t1 = (lo[j] - O[j]) / d[j], t2 = (hi[j] - O[j]) / d[j];
    const double tm = std::min(t1, t2);
    if (tm > tn) tn = tm;
  }
  return tn > 0.0 ? tn : 0.0;
}

// Geometric visibility of a cell box (redundancy reduction section,
// spatial part): the part of the box inside the view frustum is convex, and
// its projection onto the image is the set of pixels whose centre ray meets
// it.  With the camera-space depth of the ray point C + s d equal to s, the
// ray meets (box within the frustum) iff the slab interval [s_in, s_out] of
// the box, cut below by the near plane (s >= znear), is not empty.  An axis
// the ray runs parallel to keeps the whole ray if the centre lies in that
// slab and removes it otherwise.  `margin` returns how far the decision is
// from flipping: s_out - max(s_in, znear).
static bool ray_meets_box(const Cam& cam, int px, int py, const double lo[3], const double hi[3],
                          double* margin) {
  double O[3];
  cam_center(cam, O);
  const double u = (px + 0.5 - cam.cx) / cam.fx, v = (py + 0.5 - cam.cy) / cam.fy;
  double d[3];
  for (int j = 0; j < 3; ++j)
    d[j] = cam.R[0 * 3 + j] * u + cam.R[1 * 3 + j] * v + cam.R[2 * 3 + j] * 1.0;
  double s_in = cam.znear, s_out = INFINITY;
  for (int j = 0; j < 3; ++j) {
    if (d[j] == 0.0) {
      if (O[j] < lo[j] || O[j] > hi[j]) {
        *margin = -INFINITY;
        return false;
      }
      continue;
    }
    const double t1 = (lo[j] - O[j]) / d[j], t2 = (hi[j] - O[j]) / d[j];
    s_in = std::max(s_in, std::min(t1, t2));
    s_out = std::min(s_out, std::max(t1, t2));
  }
  *margin = s_out - s_in;
  return s_in <= s_out;
}

}  // namespace

// =================================================================== C ABI
extern "C" {

// Per-Gaussian preprocess (double outputs).  Arrays are length n (x k).
int or_preprocess(int64_t n, const double* means, const double* log_scales,
                  const double* quats, const double* logits, const double* sh,
                  const Cam* cam, const Params* P, uint8_t* valid,
                  double* depth, double* tcam, double* mean2d, double* cov2d,
                  double* conic, double* opacity, double* rgb,
                  uint8_t* rgb_pos, double* tau, int32_t* pix_rect,
                  int32_t* tile_rect, int64_t* n_tiles) {
  SceneIn s{n, means, log_scales, quats, logits, sh};
  std::vector<Proj> pr = preprocess_all(s, *cam, *P);
  for (int64_t i = 0; i < n; ++i) {
    const Proj& p = pr[i];
    valid[i] = p.valid;
    depth[i] = p.depth;
    for (int k = 0; k < 3; ++k) {
      tcam[i * 3 + k] = p.tc[k];
      cov2d[i * 3 + k] = p.cov2d[k];
      conic[i * 3 + k] = p.conic[k];
      rgb[i * 3 + k] = p.rgb[k];
      rgb_pos[i * 3 + k] = p.rgb_pos[k];
    }
    mean2d[i * 2 + 0] = p.mean2d[0];
    mean2d[i * 2 + 1] = p.mean2d[1];
    opacity[i] = p.opacity;
    tau[i] = p.tau;
    for (int k = 0; k < 4; ++k) {
      pix_rect[i * 4 + k] = p.valid ? p.pix[k] : 0;
      tile_rect[i * 4 + k] = p.valid ? p.tile[k] : 0;
    }
    n_tiles[i] = p.valid ? p.n_tiles : 0;
  }
  return 0;
}

// Real SH basis values [n, (D+1)^2] and gradients [n, (D+1)^2, 3] of the
// polynomial extension at the given directions.
int or_sh_eval(int degree, int64_t n, const double* dirs, double* Y,
               double* grad) {
  const int nc = (degree + 1) * (degree + 1);
  for (int64_t i = 0; i < n; ++i)
    sh_eval(degree, dirs + i * 3, Y + i * nc, grad ? grad + i * nc * 3 : nullptr);
  return 0;
}

// Sorted (key, value) instance list: key = tile_id << 32 | bits(float32 z),
// value = Gaussian index, ordered by (key, index); tile ranges [start, end).
// Returns the instance count; keys/vals may be null to query it.
int64_t or_sort_keys(int64_t n, const double* means, const double* log_scales,
                     const double* quats, const double* logits, const double* sh,
                     const Cam* cam, const Params* P, uint64_t* keys,
                     uint32_t* vals, uint32_t* ranges) {
  SceneIn s{n, means, log_scales, quats, logits, sh};
  std::vector<Proj> pr = preprocess_all(s, *cam, *P);
  Bins b = make_bins(pr, *cam, *P);
  int64_t off = 0;
  for (size_t t = 0; t < b.lists.size(); ++t) {
    if (ranges) ranges[2 * t] = (uint32_t)off;
    for (int64_t g : b.lists[t]) {
      if (keys) keys[off] = ((uint64_t)t << 32) | fbits(pr[g].zf);
      if (vals) vals[off] = (uint32_t)g;
      ++off;
    }
    if (ranges) ranges[2 * t + 1] = (uint32_t)off;
  }
  return off;
}

// Partial render of one cell (Eq. 3-4).  mode 0 = brute (every Gaussian for
// every pixel), 1 = binned.  mask: per-pixel byte, 0 = inactive (output
// C=0, T=1, D=0), may be null.  Outputs per pixel: C[3], T, D, number of
// blended pairs, ambiguity flags (OR-ed into `flags`).
int or_render(int64_t n, const double* means, const double* log_scales,
              const double* quats, const double* logits, const double* sh,
              const Cam* cam, const Params* P, int mode, const uint8_t* mask,
              double* C, double* T, double* D, int32_t* nblend,
              uint8_t* flags, const uint32_t* xf, const uint32_t* xamb,
              const uint32_t* pixbits) {
  SceneIn s{n, means, log_scales, quats, logits, sh};
  std::vector<Proj> pr = preprocess_all(s, *cam, *P);
  const int W = cam->width, H = cam->height;
  if (mode == 0) {
    std::vector<int64_t> all = brute_list(pr);
#pragma omp parallel for schedule(dynamic, 1)
    for (int py = 0; py < H; ++py)
      for (int px = 0; px < W; ++px) {
        const int64_t p = (int64_t)py * W + px;
        if (mask && !mask[p]) {
          C[p * 3] = C[p * 3 + 1] = C[p * 3 + 2] = 0;
          T[p] = 1;
          D[p] = 0;
          nblend[p] = 0;
          continue;
        }
        const XFilter xfl{xf, xamb, pixbits ? pixbits[p] : 0u};
        walk_pixel(pr, all, px, py, *cam, *P, C + p * 3, T + p, D + p,
                   nblend + p, flags + p, nullptr, xf ? &xfl : nullptr);
      }
  } else {
    Bins b = make_bins(pr, *cam, *P);
#pragma omp parallel for schedule(dynamic, 1)
    for (int py = 0; py < H; ++py)
      for (int px = 0; px < W; ++px) {
        const int64_t p = (int64_t)py * W + px;
        if (mask && !mask[p]) {
          C[p * 3] = C[p * 3 + 1] = C[p * 3 + 2] = 0;
          T[p] = 1;
          D[p] = 0;
          nblend[p] = 0;
          continue;
        }
        const auto& list = b.lists[(size_t)(py / P->tile_h) * b.tiles_x + px / P->tile_w];
        const XFilter xfl{xf, xamb, pixbits ? pixbits[p] : 0u};
        walk_pixel(pr, list, px, py, *cam, *P, C + p * 3, T + p, D + p,
                   nblend + p, flags + p, nullptr, xf ? &xfl : nullptr);
      }
  }
  return 0;
}

// Composition of K partial buffers in per-pixel ray order (Eq. 5) with the
// saturation test: a cell whose incoming transmittance P_j is below t_min is
// marked inactive in mask_out (for the next render of this view); with
// same_frame_cull it is also treated as the identity now.
//   Cparts [K][H*W*3], Tparts [K][H*W], lo/hi [K][3]
//   out_rgb [H*W*3] = sum_j P_j C_j + P_{K+1} bg, out_T [H*W] = P_{K+1}
//   order [H*W*K] cell indices front to back; mask_out [K][H*W] bytes
int or_composite(int K, const double* Cparts, const double* Tparts,
                 const double* lo, const double* hi, const Cam* cam,
                 const Params* P, double* out_rgb, double* out_T,
                 int32_t* order, uint8_t* mask_out, uint8_t* flags) {
  const int W = cam->width, H = cam->height;
  const int64_t HW = (int64_t)W * H;
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < HW; ++p) {
    const int px = (int)(p % W), py = (int)(p / W);
    std::vector<std::pair<double, int>> ks(K);
    for (int m = 0; m < K; ++m)
      ks[m] = {entry_key(*cam, px, py, lo + m * 3, hi + m * 3), m};
    std::stable_sort(ks.begin(), ks.end(),
                     [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
                       return a.first < b.first;
                     });
    // an order within rounding reach of a tie matters only between two
    // cells that both contribute here: a cell with C = 0 and T = 1 commutes
    // with any other in Eq. 5
    auto contributes = [&](int m) {
      const double* cm = Cparts + ((int64_t)m * HW + p) * 3;
      return cm[0] != 0.0 || cm[1] != 0.0 || cm[2] != 0.0 || Tparts[(int64_t)m * HW + p] != 1.0;
    };
    for (int j = 0; j + 1 < K; ++j)
      for (int j2 = j + 1; j2 < K; ++j2) {
        const double a = ks[j].first, b = ks[j2].first;
        if (!(a == 0.0 && b == 0.0) &&
            std::fabs(b - a) <= 1e-6 * std::max(std::fabs(a), std::fabs(b)) &&
            contributes(ks[j].second) && contributes(ks[j2].second))
          if (flags) flags[p] |= FLAG_ORDER;
      }
    double Pj = 1.0, c[3] = {0, 0, 0};
    for (int j = 0; j < K; ++j) {
      const int m = ks[j].second;
      if (order) order[p * K + j] = m;
      bool active = true;
      if (flags && std::fabs(Pj - P->t_min) <= 1e-3 * P->t_min) flags[p] |= FLAG_SATURATION;
      if (Pj < P->t_min) {
        active = false;
        if (mask_out) mask_out[(int64_t)m * HW + p] = 0;
      } else if (mask_out) {
        mask_out[(int64_t)m * HW + p] = 1;
      }
      if (!active && P->same_frame_cull) continue;
      for (int k = 0; k < 3; ++k) c[k] += Pj * Cparts[((int64_t)m * HW + p) * 3 + k];
      Pj *= Tparts[(int64_t)m * HW + p];
    }
    for (int k = 0; k < 3; ++k) out_rgb[p * 3 + k] = c[k] + Pj * P->bg[k];
    out_T[p] = Pj;
  }
  return 0;
}

// Composition with the saturation state carried from one render of a view
// to the next, and its speculative re-evaluation (appendix, experimental
// analysis: saturation stability during training).  Per pixel, in entry
// order, with P the incoming transmittance of the cells rendered now:
//   * a cell active at this pixel (mask_in bit set) is composited; if
//     P < t_min it is pruned for the next render and its transmittance
//     consumption P (1 - T_j) is kept as its budget;
//   * a pruned cell whose box the pixel's ray meets (omega set, or omega
//     null) is tested with the residual R = P - S, S being the budgets of
//     the cells re-activated before it on this ray: it is re-activated when
//     R >= t_min and R covers its whole budget, and S grows by that budget;
//     the first pruned cell that fails ends the scan for the pixel;
//   * any other cell stays inactive.
// Cells rendered with their bit cleared have C = 0, T = 1 and are skipped.
//   mask_in, omega, mask_out [K][H*W] bytes; budget [K][H*W] in/out
//   (written for pairs pruned now, read for pairs pruned before); flips
//   [H*W] counts the re-activated cells of each pixel.
int or_composite_reeval(int K, const double* Cparts, const double* Tparts,
                        const double* lo, const double* hi, const Cam* cam,
                        const Params* P, const uint8_t* mask_in, const uint8_t* omega,
                        double* budget, double* out_rgb, double* out_T,
                        uint8_t* mask_out, int32_t* flips, uint8_t* flags) {
  const int W = cam->width, H = cam->height;
  const int64_t HW = (int64_t)W * H;
  const double band = 1e-3 * P->t_min;
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < HW; ++p) {
    const int px = (int)(p % W), py = (int)(p / W);
    std::vector<std::pair<double, int>> ks(K);
    for (int m = 0; m < K; ++m)
      ks[m] = {entry_key(*cam, px, py, lo + m * 3, hi + m * 3), m};
    std::stable_sort(ks.begin(), ks.end(),
                     [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
                       return a.first < b.first;
                     });
    // an order within rounding of a tie is ambiguous for any two cells that
    // take part here (composited or tested)
    auto takes_part = [&](int m) {
      return mask_in[(int64_t)m * HW + p] || !omega || omega[(int64_t)m * HW + p];
    };
    for (int j = 0; j + 1 < K; ++j)
      for (int j2 = j + 1; j2 < K; ++j2) {
        const double a = ks[j].first, b = ks[j2].first;
        if (!(a == 0.0 && b == 0.0) &&
            std::fabs(b - a) <= 1e-6 * std::max(std::fabs(a), std::fabs(b)) &&
            takes_part(ks[j].second) && takes_part(ks[j2].second))
          flags[p] |= FLAG_ORDER;
      }
    double Pj = 1.0, S = 0.0, c[3] = {0, 0, 0};
    bool scanning = true;
    int32_t nflip = 0;
    for (int j = 0; j < K; ++j) {
      const int64_t mp = (int64_t)ks[j].second * HW + p;
      if (mask_in[mp]) {
        const double Tm = Tparts[mp];
        if (std::fabs(Pj - P->t_min) <= band) flags[p] |= FLAG_SATURATION;
        const bool active = Pj >= P->t_min;
        mask_out[mp] = active ? 1 : 0;
        if (!active) budget[mp] = Pj * (1.0 - Tm);
        if (!active && P->same_frame_cull) continue;
        for (int k = 0; k < 3; ++k) c[k] += Pj * Cparts[mp * 3 + k];
        Pj *= Tm;
      } else if (!omega || omega[mp]) {
        const double R = Pj - S, b = budget[mp];
        if (scanning &&
            (std::fabs(R - P->t_min) <= band || std::fabs(R - b) <= 1e-3 * std::max(R, b)))
          flags[p] |= FLAG_SATURATION;
        if (scanning && R >= P->t_min && R >= b) {
          mask_out[mp] = 1;
          S += b;
          ++nflip;
        } else {
          scanning = false;
          mask_out[mp] = 0;
        }
      } else {
        mask_out[mp] = 0;
      }
    }
    for (int k = 0; k < 3; ++k) out_rgb[p * 3 + k] = c[k] + Pj * P->bg[k];
    out_T[p] = Pj;
    flips[p] = nflip;
  }
  return 0;
}

// Gradient of the composition (Eq. 6-7 at the level of partial pixels):
// dC_j = P_j G ; dT_j = P_j (G . B_{j+1} + gT U_j), with B_{K+1} = bg,
// B_j = C_j + T_j B_{j+1} and U_j the product of the transmittances behind
// cell j.  `order` as produced by or_composite; `active` [K][H*W] bytes
// (null = all active) is honoured only with same_frame_cull.
int or_composite_backward(int K, const double* Cparts, const double* Tparts,
                          const int32_t* order, const uint8_t* active,
                          const Cam* cam, const Params* P, const double* dout_rgb,
                          const double* dout_T, double* dC, double* dT) {
  const int64_t HW = (int64_t)cam->width * cam->height;
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < HW; ++p) {
    std::vector<double> Pj(K + 1);
    std::vector<char> use(K);
    Pj[0] = 1.0;
    for (int j = 0; j < K; ++j) {
      const int m = order[p * K + j];
      use[j] = !(P->same_frame_cull && active && !active[(int64_t)m * HW + p]);
      Pj[j + 1] = use[j] ? Pj[j] * Tparts[(int64_t)m * HW + p] : Pj[j];
    }
    const double G[3] = {dout_rgb[p * 3], dout_rgb[p * 3 + 1], dout_rgb[p * 3 + 2]};
    const double gT = dout_T ? dout_T[p] : 0.0;
    double B[3] = {P->bg[0], P->bg[1], P->bg[2]};
    double U = 1.0;
    for (int j = K - 1; j >= 0; --j) {
      const int m = order[p * K + j];
      const int64_t e = (int64_t)m * HW + p;
      if (!use[j]) {
        for (int k = 0; k < 3; ++k) dC[e * 3 + k] = 0.0;
        dT[e] = 0.0;
        continue;
      }
      double gb = 0.0;
      for (int k = 0; k < 3; ++k) {
        dC[e * 3 + k] = Pj[j] * G[k];
        gb += G[k] * B[k];
      }
      dT[e] = Pj[j] * (gb + gT * U);
      const double Tm = Tparts[e];
      for (int k = 0; k < 3; ++k) B[k] = Cparts[e * 3 + k] + Tm * B[k];
      U *= Tm;
    }
  }
  return 0;
}

// Backward of one cell's partial render and of its preprocess.
// Inputs: the cell's Gaussians, dL/dC [H*W*3], dL/dT [H*W], dL/dD [H*W]
// (each may be null = 0), an optional per-pixel active mask.
// Outputs (accumulated with +=, caller zeroes):
//   g2d [n*10]: dmean2d(2), dconic(3), dopacity, drgb(3), ddepth  (screen)
//   gmeans [n*3], glog_scales [n*3], gquats [n*4], glogits [n], gsh [n*nc*3]
// Chain of the screen-space gradients acc [n][10] (mean2d x, y, conic a, b,
// c, opacity, rgb, depth) through the projection to the raw parameters
// (paper, background: the parametrisation Sigma = R S S^T R^T, the EWA
// projection and the SH colour), added into the parameter gradients.
static void chain_to_params(const SceneIn& s, const Cam* cam, const Params* P,
                            const std::vector<Proj>& pr, const double* acc,
                            double* gmeans, double* glog_scales, double* gquats,
                            double* glogits, double* gsh);

int or_render_backward(int64_t n, const double* means, const double* log_scales,
                       const double* quats, const double* logits, const double* sh,
                       const Cam* cam, const Params* P, const uint8_t* mask,
                       const double* dC, const double* dT, const double* dD,
                       double* g2d, double* gmeans, double* glog_scales,
                       double* gquats, double* glogits, double* gsh,
                       const uint32_t* xf, const uint32_t* pixbits, double* g2d_scale) {
  SceneIn s{n, means, log_scales, quats, logits, sh};
  std::vector<Proj> pr = preprocess_all(s, *cam, *P);
  Bins b = make_bins(pr, *cam, *P);
  const int W = cam->width, H = cam->height;
  std::vector<double> acc((size_t)n * 10, 0.0);
  // Optional first-order rounding-error scale of each screen-space gradient
  // entry of an FP32 evaluation (test tolerances only; it enters no
  // gradient), in units of the FP32 unit roundoff.  Per pixel term:
  //  - the magnitudes the term is formed from before they cancel (for
  //    d alpha: T_i (|G| (|c| + |R|) + |g_D| (|z| + |RD|)) + |g_T| T_i U);
  //  - times (N + 16 + rho): a walk that recovers T_i and carries R, RD and
  //    U over the pixel's N blended pairs is off by a few ulps per pair, and
  //    alpha computed from FP32 record fields is off by rho ulps relative,
  //    rho = (dq/u)/2 + 3 with dq the error of q from rounding the screen
  //    position (held relative to the principal point: magnitude M =
  //    max|mean2d - c| + max(W, H)/2 pixels), the conic and q's own sum;
  //  - plus the rounding of the offsets dx, dy (M ulps) in the factors of
  //    the mean and conic terms.
  std::vector<double> sacc(g2d_scale ? (size_t)n * 10 : 0, 0.0);
#pragma omp parallel
  {
    std::vector<Blend> bl;
#pragma omp for schedule(dynamic, 1)
    for (int py = 0; py < H; ++py)
      for (int px = 0; px < W; ++px) {
        const int64_t p = (int64_t)py * W + px;
        if (mask && !mask[p]) continue;
        bl.clear();
        double C[3], T, D;
        int nb;
        uint8_t fl = 0;
        const auto& list = b.lists[(size_t)(py / P->tile_h) * b.tiles_x + px / P->tile_w];
        const XFilter xfl{xf, xf, pixbits ? pixbits[p] : 0u};  // flags unused here
        walk_pixel(pr, list, px, py, *cam, *P, C, &T, &D, &nb, &fl, &bl, xf ? &xfl : nullptr);
        const double G[3] = {dC ? dC[p * 3] : 0.0, dC ? dC[p * 3 + 1] : 0.0,
                             dC ? dC[p * 3 + 2] : 0.0};
        const double gT = dT ? dT[p] : 0.0, gD = dD ? dD[p] : 0.0;
        double R[3] = {0, 0, 0}, RD = 0.0, U = 1.0;
        for (int i = (int)bl.size() - 1; i >= 0; --i) {
          const Blend& e = bl[i];
          const Proj& pj = pr[e.g];
          const double w = e.alpha * e.Ti;
          double dalpha = 0.0;
          for (int k = 0; k < 3; ++k) dalpha += G[k] * (pj.rgb[k] - R[k]);
          dalpha = e.Ti * (dalpha + gD * (pj.depth - RD)) - gT * e.Ti * U;
          double* a = &acc[(size_t)e.g * 10];
          double loc[10] = {0};
          for (int k = 0; k < 3; ++k) loc[6 + k] = w * G[k];
          loc[9] = w * gD;
          if (!e.clamped) {
            loc[5] = dalpha * e.gval;
            const double dq = dalpha * (-0.5 * e.alpha);
            const double A = pj.conic[0], Bc = pj.conic[1], Cc = pj.conic[2];
            loc[0] = dq * (-2.0) * (A * e.dx + Bc * e.dy);
            loc[1] = dq * (-2.0) * (Bc * e.dx + Cc * e.dy);
            loc[2] = dq * e.dx * e.dx;
            loc[3] = dq * 2.0 * e.dx * e.dy;
            loc[4] = dq * e.dy * e.dy;
          }
          for (int k = 0; k < 10; ++k) {
#pragma omp atomic
            a[k] += loc[k];
          }
          if (g2d_scale) {
            double sa = 0.0;
            for (int k = 0; k < 3; ++k) sa += std::fabs(G[k]) * (std::fabs(pj.rgb[k]) + std::fabs(R[k]));
            sa = e.Ti * (sa + std::fabs(gD) * (std::fabs(pj.depth) + std::fabs(RD)) +
                         std::fabs(gT) * U);
            const double A = std::fabs(pj.conic[0]), Bc = std::fabs(pj.conic[1]),
                         Cc = std::fabs(pj.conic[2]);
            const double ax = std::fabs(e.dx), ay = std::fabs(e.dy);
            const double M = std::max(std::fabs(pj.mean2d[0] - cam->cx),
                                      std::fabs(pj.mean2d[1] - cam->cy)) +
                             0.5 * std::max(W, H);
            const double qabs = A * ax * ax + 2.0 * Bc * ax * ay + Cc * ay * ay;
            const double rho =
                0.5 * (2.0 * ((A * ax + Bc * ay) + (Bc * ax + Cc * ay)) * M + 2.0 * qabs) + 3.0;
            const double f = (double)bl.size() + 16.0 + rho;
            double sl[10] = {0};
            for (int k = 0; k < 3; ++k) sl[6 + k] = f * std::fabs(w * G[k]);
            sl[9] = f * std::fabs(w * gD);
            if (!e.clamped) {
              sl[5] = f * sa * e.gval;
              const double dq = sa * 0.5 * e.alpha;
              sl[0] = dq * 2.0 * (f * (A * ax + Bc * ay) + (A + Bc) * M);
              sl[1] = dq * 2.0 * (f * (Bc * ax + Cc * ay) + (Bc + Cc) * M);
              sl[2] = dq * (f * ax * ax + 2.0 * ax * M);
              sl[3] = dq * 2.0 * (f * ax * ay + (ax + ay) * M);
              sl[4] = dq * (f * ay * ay + 2.0 * ay * M);
            }
            double* sc = &sacc[(size_t)e.g * 10];
            for (int k = 0; k < 10; ++k) {
#pragma omp atomic
              sc[k] += sl[k];
            }
          }
          for (int k = 0; k < 3; ++k) R[k] = pj.rgb[k] * e.alpha + (1.0 - e.alpha) * R[k];
          RD = pj.depth * e.alpha + (1.0 - e.alpha) * RD;
          U *= (1.0 - e.alpha);
        }
      }
  }
  if (g2d)
    for (size_t k = 0; k < acc.size(); ++k) g2d[k] += acc[k];
  if (g2d_scale)
    for (size_t k = 0; k < sacc.size(); ++k) g2d_scale[k] += sacc[k];
  chain_to_params(s, cam, P, pr, acc.data(), gmeans, glog_scales, gquats, glogits, gsh);
  return 0;
}

// The projection backward alone: screen-space gradients g2d_in [n][10] of a
// view chained to the parameters (added into the outputs).
int or_preprocess_backward(int64_t n, const double* means, const double* log_scales,
                           const double* quats, const double* logits, const double* sh,
                           const Cam* cam, const Params* P, const double* g2d_in,
                           double* gmeans, double* glog_scales, double* gquats,
                           double* glogits, double* gsh) {
  SceneIn s{n, means, log_scales, quats, logits, sh};
  std::vector<Proj> pr = preprocess_all(s, *cam, *P);
  chain_to_params(s, cam, P, pr, g2d_in, gmeans, glog_scales, gquats, glogits, gsh);
  return 0;
}

}  // extern "C"

static void chain_to_params(const SceneIn& s, const Cam* cam, const Params* P,
                            const std::vector<Proj>& pr, const double* acc,
                            double* gmeans, double* glog_scales, double* gquats,
                            double* glogits, double* gsh) {
  const int64_t n = s.n;
  const int nc = (P->sh_degree + 1) * (P->sh_degree + 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const Proj& p = pr[i];
    const double* a = &acc[(size_t)i * 10];
    if (!p.valid) continue;
    const Gauss g = gauss_at(s, i, nc);
    // colour -> SH coefficients and view direction
    double Y[(LMAX + 1) * (LMAX + 1)], dY[(LMAX + 1) * (LMAX + 1) * 3];
    sh_eval(P->sh_degree, p.dirv, Y, dY);
    double gdir[3] = {0, 0, 0};
    for (int ch = 0; ch < 3; ++ch) {
      if (!p.rgb_pos[ch]) continue;
      const double gc = a[6 + ch];
      for (int j = 0; j < nc; ++j) {
        gsh[((size_t)i * nc + j) * 3 + ch] += gc * Y[j];
        for (int k = 0; k < 3; ++k) gdir[k] += gc * g.sh[j * 3 + ch] * dY[j * 3 + k];
      }
    }
    double gmu[3];
    {
      const double dd = gdir[0] * p.dirv[0] + gdir[1] * p.dirv[1] + gdir[2] * p.dirv[2];
      for (int k = 0; k < 3; ++k) gmu[k] = (gdir[k] - dd * p.dirv[k]) / p.dist;
    }
    // opacity
    glogits[i] += a[5] * p.opacity * (1.0 - p.opacity);
    // conic -> dilated 2D covariance: G_S = -A Gc A with Gc symmetric
    const double A2[4] = {p.conic[0], p.conic[1], p.conic[1], p.conic[2]};
    const double Gc[4] = {a[2], 0.5 * a[3], 0.5 * a[3], a[4]};
    double tmp[4], GS[4];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) {
        double v = 0;
        for (int k = 0; k < 2; ++k) v += A2[r * 2 + k] * Gc[k * 2 + c];
        tmp[r * 2 + c] = v;
      }
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) {
        double v = 0;
        for (int k = 0; k < 2; ++k) v += tmp[r * 2 + k] * A2[k * 2 + c];
        GS[r * 2 + c] = -v;
      }
    // rebuild J, M, Rq, s
    const double* t = p.tc;
    const double z = t[2];
    const double J[6] = {cam->fx / z, 0.0, -cam->fx * t[0] / (z * z),
                         0.0, cam->fy / z, -cam->fy * t[1] / (z * z)};
    double qn = std::sqrt(g.q[0] * g.q[0] + g.q[1] * g.q[1] + g.q[2] * g.q[2] + g.q[3] * g.q[3]);
    double qh[4] = {g.q[0] / qn, g.q[1] / qn, g.q[2] / qn, g.q[3] / qn};
    double Rq[9];
    quat_to_rot(qh, Rq);
    double sv[3];
    for (int k = 0; k < 3; ++k) sv[k] = std::exp(g.ls[k]);
    double Sig[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double v = 0;
        for (int k = 0; k < 3; ++k) v += Rq[r * 3 + k] * sv[k] * sv[k] * Rq[c * 3 + k];
        Sig[r * 3 + c] = v;
      }
    double WT[9], tmp3[9], M[9];
    transpose3(cam->R, WT);
    matmul3(cam->R, Sig, tmp3);
    matmul3(tmp3, WT, M);
    // dM = J^T GS J ; dJ = 2 GS J M
    double dM[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double v = 0;
        for (int u = 0; u < 2; ++u)
          for (int w2 = 0; w2 < 2; ++w2) v += J[u * 3 + r] * GS[u * 2 + w2] * J[w2 * 3 + c];
        dM[r * 3 + c] = v;
      }
    double GJ[6], dJ[6];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c) {
        double v = 0;
        for (int k = 0; k < 2; ++k) v += GS[r * 2 + k] * J[k * 3 + c];
        GJ[r * 3 + c] = v;
      }
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c) {
        double v = 0;
        for (int k = 0; k < 3; ++k) v += GJ[r * 3 + k] * M[k * 3 + c];
        dJ[r * 3 + c] = 2.0 * v;
      }
    // dSigma = W^T dM W
    double dSig[9];
    matmul3(WT, dM, tmp3);
    matmul3(tmp3, cam->R, dSig);
    // Sigma = L L^T with L = Rq diag(s): dL = 2 dSigma L
    double Lm[9], dL[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) Lm[r * 3 + c] = Rq[r * 3 + c] * sv[c];
    matmul3(dSig, Lm, dL);
    for (int k = 0; k < 9; ++k) dL[k] *= 2.0;
    for (int k = 0; k < 3; ++k) {
      double v = 0;
      for (int r = 0; r < 3; ++r) v += dL[r * 3 + k] * Rq[r * 3 + k];
      glog_scales[i * 3 + k] += v * sv[k];
    }
    double dR[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) dR[r * 3 + c] = dL[r * 3 + c] * sv[c];
    const double w = qh[0], x = qh[1], y = qh[2], zq = qh[3];
    double dqh[4];
    dqh[0] = dR[1] * (-2 * zq) + dR[2] * (2 * y) + dR[3] * (2 * zq) + dR[5] * (-2 * x) +
             dR[6] * (-2 * y) + dR[7] * (2 * x);
    dqh[1] = dR[1] * (2 * y) + dR[2] * (2 * zq) + dR[3] * (2 * y) + dR[4] * (-4 * x) +
             dR[5] * (-2 * w) + dR[6] * (2 * zq) + dR[7] * (2 * w) + dR[8] * (-4 * x);
    dqh[2] = dR[0] * (-4 * y) + dR[1] * (2 * x) + dR[2] * (2 * w) + dR[3] * (2 * x) +
             dR[5] * (2 * zq) + dR[6] * (-2 * w) + dR[7] * (2 * zq) + dR[8] * (-4 * y);
    dqh[3] = dR[0] * (-4 * zq) + dR[1] * (-2 * w) + dR[2] * (2 * x) + dR[3] * (2 * w) +
             dR[4] * (-4 * zq) + dR[5] * (2 * y) + dR[6] * (2 * x) + dR[7] * (2 * y);
    {
      const double dd = dqh[0] * qh[0] + dqh[1] * qh[1] + dqh[2] * qh[2] + dqh[3] * qh[3];
      for (int k = 0; k < 4; ++k) gquats[i * 4 + k] += (dqh[k] - dd * qh[k]) / qn;
    }
    // mean: through mean2d, J(t) and depth
    double dt[3] = {0, 0, 0};
    dt[0] += a[0] * cam->fx / z;
    dt[2] += a[0] * (-cam->fx * t[0] / (z * z));
    dt[1] += a[1] * cam->fy / z;
    dt[2] += a[1] * (-cam->fy * t[1] / (z * z));
    dt[0] += dJ[2] * (-cam->fx / (z * z));
    dt[1] += dJ[5] * (-cam->fy / (z * z));
    dt[2] += dJ[0] * (-cam->fx / (z * z)) + dJ[2] * (2.0 * cam->fx * t[0] / (z * z * z)) +
             dJ[4] * (-cam->fy / (z * z)) + dJ[5] * (2.0 * cam->fy * t[1] / (z * z * z));
    dt[2] += a[9];
    for (int k = 0; k < 3; ++k) {
      double v = 0;
      for (int r = 0; r < 3; ++r) v += cam->R[r * 3 + k] * dt[r];
      gmeans[i * 3 + k] += v + gmu[k];
    }
  }
}

extern "C" {

// Visible-pixel maps of K cell boxes for one camera: vis [K][H*W] bytes
// (1 = the pixel's centre ray meets the part of the box inside the
// frustum); flags [H*W] gets FLAG_VISIBILITY where a decision lies within
// 1e-9 relative of flipping.
// Cross-boundary filter bits of one cell's Gaussians for a view (appendix,
// implementation details: cross-boundary Gaussians).  Readings: a
// Gaussian's spatial support is the axis-aligned box of its 3-sigma extent,
// mean +- 3 sqrt(Sigma_aa); its support spans cell s when that box meets
// box s (strict inequalities); its depth is the camera z of its mean; the
// overlapped depth interval of cells k and s is the intersection of the
// camera-z ranges of the two boxes (a box unbounded along an axis the depth
// varies on has an unbounded range).  Bit s of xf[i] (s != cell) is set when
// Gaussian i is visible in the view, its support spans cell s and its depth
// lies in the overlapped interval of (cell, s).  xamb[i] marks the bits
// whose comparisons lie within 1e-5 relative of flipping.
int or_cross_filter(int64_t n, const double* means, const double* log_scales,
                    const double* quats, const double* logits, const double* sh,
                    const Cam* cam, const Params* P, int K, const double* lo,
                    const double* hi, int cell, uint32_t* xf, uint32_t* xamb) {
  SceneIn s{n, means, log_scales, quats, logits, sh};
  std::vector<Proj> pr = preprocess_all(s, *cam, *P);
  // camera-z range of every box: z = R[2] . x + t[2], linear over the box
  std::vector<double> zlo(K), zhi(K);
  for (int m = 0; m < K; ++m) {
    double a = cam->t[2], b = cam->t[2];
    for (int j = 0; j < 3; ++j) {
      const double r = cam->R[6 + j];
      if (r == 0.0) continue;
      const double u = r * lo[m * 3 + j], v = r * hi[m * 3 + j];
      a += std::min(u, v);
      b += std::max(u, v);
    }
    zlo[m] = a, zhi[m] = b;
  }
  // x < y decided, and whether it is within rounding reach
  auto near = [](double x, double y, double scale) {
    return std::isfinite(y) && std::fabs(x - y) <= 1e-5 * scale;
  };
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    xf[i] = xamb[i] = 0;
    if (!pr[i].valid) continue;
    double q[4];
    double qn = 0.0;
    for (int k = 0; k < 4; ++k) qn += quats[i * 4 + k] * quats[i * 4 + k];
    qn = std::sqrt(qn);
    for (int k = 0; k < 4; ++k) q[k] = quats[i * 4 + k] / qn;
    double Rq[9];
    quat_to_rot(q, Rq);
    double h[3];
    for (int a = 0; a < 3; ++a) {
      double v = 0.0;
      for (int b = 0; b < 3; ++b) {
        const double e = Rq[a * 3 + b] * std::exp(log_scales[i * 3 + b]);
        v += e * e;
      }
      h[a] = 3.0 * std::sqrt(v);
    }
    const double* mu = means + i * 3;
    const double d = pr[i].depth;
    for (int sc = 0; sc < K; ++sc) {
      if (sc == cell) continue;
      bool meets = true, amb = false;
      for (int a = 0; a < 3; ++a) {
        const double l = mu[a] - h[a], r = mu[a] + h[a];
        const double scale = std::fabs(mu[a]) + h[a];
        meets = meets && l < hi[sc * 3 + a] && r > lo[sc * 3 + a];
        amb = amb || near(l, hi[sc * 3 + a], scale + std::fabs(hi[sc * 3 + a])) ||
              near(r, lo[sc * 3 + a], scale + std::fabs(lo[sc * 3 + a]));
      }
      const double Dlo = std::max(zlo[cell], zlo[sc]), Dhi = std::min(zhi[cell], zhi[sc]);
      const bool in = d >= Dlo && d <= Dhi;
      amb = amb || near(d, Dlo, std::fabs(d) + std::fabs(Dlo)) ||
            near(d, Dhi, std::fabs(d) + std::fabs(Dhi));
      if (meets && in) xf[i] |= 1u << sc;
      if (amb) xamb[i] |= 1u << sc;
    }
  }
  return 0;
}

int or_visibility(int K, const double* lo, const double* hi, const Cam* cam, uint8_t* vis,
                  uint8_t* flags) {
  const int W = cam->width, H = cam->height;
  const int64_t HW = (int64_t)W * H;
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < HW; ++p) {
    const int px = (int)(p % W), py = (int)(p / W);
    for (int m = 0; m < K; ++m) {
      double margin;
      const bool in = ray_meets_box(*cam, px, py, lo + m * 3, hi + m * 3, &margin);
      vis[(int64_t)m * HW + p] = in ? 1 : 0;
      if (flags && std::isfinite(margin) && std::fabs(margin) <= 1e-9 * (1.0 + std::fabs(margin)))
        flags[p] |= FLAG_VISIBILITY;
    }
  }
  return 0;
}

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

}  // extern "C"
