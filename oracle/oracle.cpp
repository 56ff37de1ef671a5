// FP64 reference renderer for Approximate Puzzlepiece Compositing (APC).
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
// call this file; it exists so that tests, the smoke check and the benchmark's
// CPU-baseline leg can compare the HIP library against a plain, slow,
// obviously-correct computation of the same method.  It shares no code,
// header or table with the HIP library.
//
// What it computes, in the paper's order (Section 3, Algs. 1-3; Section 4):
//   * rays of an orthographic or pinhole camera, and one global depth range
//     [t_near, t_far] from the bounding sphere of the whole mesh, which the
//     log-depth warp of Alg. 2 needs and which every subdomain shares;
//   * for every tet, the chord of each pixel ray by clipping against the 4
//     face planes (cell projection, tets visited in any order);
//   * pieces: each chord is cut at the points t_near + k*step of one global
//     lattice; a piece carries its mid depth, length, the scalar at the mid
//     point (barycentric interpolation), the transfer-function RGBA there and
//     its optical depth a = min(kappa*A*length, absorbance_max);
//   * pass 1 (Alg. 2, Section 4.1): per subdomain, b_j += a * z^j for
//     j = 0..m with z the warped depth; the global moments are the sum over
//     subdomains;
//   * pass 2 (Alg. 3, Section 4.2): per pixel normalise and bias the moments,
//     Cholesky-factor the Hankel matrix, then per piece solve for the kernel
//     polynomial, find its roots, weight the nodes 1/0 by depth order and eta
//     at the piece's own depth, and turn the interpolant's moment functional
//     into transmittance exp(-b0 * F); colour += T * alpha_piece * rgb per
//     subdomain, and the final image is the sum over subdomains (Alg. 1),
//     renormalised by the total opacity 1 - exp(-b0) (Section 4.3);
//   * the exact front-to-back compositing of the same pieces, which the
//     moment method approximates (reported, never a pass/fail bar).
//
// Roots: Durand-Kerner (Weierstrass) simultaneous iteration in complex FP64.
// Weights: Lagrange basis polynomials of the nodes applied to the moments.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {

struct OView {
  int32_t width, height, projection, pad;  // projection: 0 orthographic, 1 pinhole
  double eye[3], dir[3], right[3], down[3];
};

struct OScene {
  int64_t n_vertices, n_tets;
  int32_t n_sub, n_tf;
  const float* xyz;        // [V][3]
  const float* scalar;     // [V]
  const int32_t* tets;     // [T][4]
  const int32_t* tet_sub;  // [T]
  const float* tf;         // [n_tf][4]
  double s_min, s_max, kappa, amax, step;
  OView view;
  int32_t m, renormalize;
  double alpha, eta;
  double bias[8];          // b*_1..b*_m
};

struct OOut {
  const int64_t* pixels;   // pixel ids (row*W + col) to render, or null for all
  int64_t n_pixels;        // length of `pixels` (ignored when null)
  int32_t do_pass2, do_exact, n_threads, pad;
  double* moments_sub;     // [S][m+1][P] or null
  double* moments;         // [m+1][P] or null
  double* color_sub;       // [S][P][4] additive (sum T*a*rgb, sum T*a) or null
  double* color;           // [P][4] additive, summed over subdomains, or null
  double* rgba;            // [P][4] final image or null
  double* exact;           // [P][4] exact sorted compositing or null
  int64_t* pieces_sub;     // [S] piece counts or null
  int64_t n_pieces, n_chords, n_nonpd, n_rank1;
  double t_near, t_far;
  int32_t* segments;       // [2][P]: segments per pixel, subdomains met per pixel; or null
};

}  // extern "C"

namespace {

struct V3 {
  double x, y, z;
};
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline V3 from(const double* p) { return {p[0], p[1], p[2]}; }

V3 vertex(const OScene& s, int64_t v) {
  return {double(s.xyz[3 * v]), double(s.xyz[3 * v + 1]), double(s.xyz[3 * v + 2])};
}

// Camera ray of pixel (row i, column j).  Orthographic: origin on the image
// plane, one direction.  Pinhole: origin at the eye, unit direction through
// the pixel centre.
void pixel_ray(const OView& v, int64_t i, int64_t j, V3& o, V3& d) {
  double a = double(j) + 0.5, b = double(i) + 0.5;
  if (v.projection == 0) {
    o = from(v.eye) + a * from(v.right) + b * from(v.down);
    d = from(v.dir);
  } else {
    o = from(v.eye);
    a -= 0.5 * v.width;
    b -= 0.5 * v.height;
    d = from(v.dir) + a * from(v.right) + b * from(v.down);
  }
  d = (1.0 / std::sqrt(dot(d, d))) * d;
}

// Global depth range: the bounding sphere of the bounding box of all vertices.
void depth_range(const OScene& s, double& t_near, double& t_far) {
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t v = 0; v < s.n_vertices; ++v)
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], double(s.xyz[3 * v + k]));
      hi[k] = std::max(hi[k], double(s.xyz[3 * v + k]));
    }
  V3 c = {0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1]), 0.5 * (lo[2] + hi[2])};
  V3 ext = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
  double r = 0.5 * std::sqrt(dot(ext, ext));
  double dist;
  if (s.view.projection == 0) {
    V3 d = from(s.view.dir);
    d = (1.0 / std::sqrt(dot(d, d))) * d;
    dist = dot(c - from(s.view.eye), d);
  } else {
    V3 e = c - from(s.view.eye);
    dist = std::sqrt(dot(e, e));
  }
  t_near = dist - r;
  t_far = dist + r;
}

// Log-depth warp of Alg. 2 / Alg. 3: ln t rescaled so that t_near -> -1 and
// t_far -> +1, clamped to [-1, 1].
double warp(double t, double t_near, double t_far) {
  double z = 2.0 * (std::log(t) - std::log(t_near)) / (std::log(t_far) - std::log(t_near)) - 1.0;
  return std::min(1.0, std::max(-1.0, z));
}

// Ray/tet chord by clipping the ray against the 4 face planes (outward
// normals).  Returns false when the chord is empty.
bool tet_chord(const V3 p[4], V3 o, V3 d, double& t0, double& t1) {
  static const int F[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
  t0 = -1e300;
  t1 = 1e300;
  for (int f = 0; f < 4; ++f) {
    V3 a = p[F[f][0]], b = p[F[f][1]], c = p[F[f][2]];
    V3 n = cross(b - a, c - a);
    if (dot(p[f] - a, n) > 0) n = -1.0 * n;  // point away from the opposite vertex
    double num = dot(a - o, n), den = dot(d, n);
    if (den == 0.0) {
      if (num < 0.0) return false;  // parallel and outside
      continue;
    }
    double t = num / den;
    if (den < 0.0)
      t0 = std::max(t0, t);
    else
      t1 = std::min(t1, t);
  }
  return t1 > t0;
}

// Barycentric interpolation of the vertex scalars at point x.
double bary_scalar(const V3 p[4], const double sv[4], V3 x) {
  V3 e1 = p[1] - p[0], e2 = p[2] - p[0], e3 = p[3] - p[0], r = x - p[0];
  double det = dot(e1, cross(e2, e3));
  double l1 = dot(r, cross(e2, e3)) / det;
  double l2 = dot(e1, cross(r, e3)) / det;
  double l3 = dot(e1, cross(e2, r)) / det;
  return sv[0] * (1.0 - l1 - l2 - l3) + sv[1] * l1 + sv[2] * l2 + sv[3] * l3;
}

// Transfer function: linear interpolation in a table over [s_min, s_max].
void tf_lookup(const OScene& s, double sc, double rgba[4]) {
  double u = (sc - s.s_min) / (s.s_max - s.s_min) * double(s.n_tf - 1);
  u = std::min(double(s.n_tf - 1), std::max(0.0, u));
  int i0 = std::min(int(std::floor(u)), s.n_tf - 2);
  double f = u - i0;
  for (int c = 0; c < 4; ++c) rgba[c] = (1.0 - f) * s.tf[4 * i0 + c] + f * s.tf[4 * (i0 + 1) + c];
}

struct Piece {
  double tm, len, a, rgb[3];
};

// Cut chord [t0, t1] at the global lattice t_near + k*step and describe each
// piece.  `emit` is called once per piece.
template <class Emit>
void pieces_of_chord(const OScene& s, const V3 p[4], const double sv[4], V3 o, V3 d, double t0, double t1,
                     double t_near, Emit emit) {
  double k = std::floor((t0 - t_near) / s.step) + 1.0;
  double u = t0;
  while (u < t1) {
    double next = t_near + k * s.step;
    double v = next < t1 ? next : t1;
    if (v > u) {
      Piece pc;
      pc.tm = 0.5 * (u + v);
      pc.len = v - u;
      double sc = bary_scalar(p, sv, o + pc.tm * d);
      double rgba[4];
      tf_lookup(s, sc, rgba);
      pc.a = std::min(s.kappa * rgba[3] * pc.len, s.amax);
      pc.rgb[0] = rgba[0];
      pc.rgb[1] = rgba[1];
      pc.rgb[2] = rgba[2];
      emit(pc);
    }
    u = v;
    k += 1.0;
  }
}

// ---------------------------------------------------------------- reconstruction

// Real parts of the roots of sum_j c[j] x^j (degree n) by Durand-Kerner.
// Leading coefficients that are zero are dropped first (a root at infinity
// carries no weight).  Returns the number of finite roots.
int poly_roots(const double* c, int n, double* roots) {
  int deg = n;
  while (deg > 0 && c[deg] == 0.0) --deg;
  if (deg == 0) return 0;
  std::vector<double> a(deg + 1);
  for (int j = 0; j <= deg; ++j) a[j] = c[j] / c[deg];  // monic
  double bound = 0.0;
  for (int j = 0; j < deg; ++j) bound = std::max(bound, std::fabs(a[j]));
  bound += 1.0;
  typedef std::complex<double> C;
  std::vector<C> x(deg), xn(deg);
  C seed(0.4, 0.9);
  for (int i = 0; i < deg; ++i) x[i] = bound * std::pow(seed, i + 1) / std::abs(std::pow(seed, i + 1));
  auto eval = [&](C z) {
    C r = 1.0;
    for (int j = deg - 1; j >= 0; --j) r = r * z + a[j];
    return r;
  };
  for (int it = 0; it < 500; ++it) {
    double change = 0.0;
    for (int i = 0; i < deg; ++i) {
      C den = 1.0;
      for (int k = 0; k < deg; ++k)
        if (k != i) den *= (x[i] - x[k]);
      C step = eval(x[i]) / den;
      xn[i] = x[i] - step;
      change = std::max(change, std::abs(step) / (1.0 + std::abs(x[i])));
    }
    x = xn;
    if (change < 1e-15) break;
  }
  for (int i = 0; i < deg; ++i) {
    double r = x[i].real();
    for (int it = 0; it < 3; ++it) {  // real Newton polish on the original polynomial
      double p = 0.0, dp = 0.0;
      for (int j = deg; j >= 0; --j) {
        dp = dp * r + p;
        p = p * r + a[j];
      }
      if (dp == 0.0) break;
      double nr = r - p / dp;
      if (!std::isfinite(nr)) break;
      r = nr;
    }
    roots[i] = r;
  }
  return deg;
}

struct PixelSetup {
  int n;                 // m/2
  bool empty;            // b0 == 0
  bool rank1;            // absorbance concentrated at one depth (singular Hankel)
  bool nonpd;            // a non-positive pivot was floored
  double b0;
  double bp[17];         // biased normalised moments beta'_0..beta'_m
  double L[5][5];        // Cholesky factor of the Hankel matrix
};

// Per-pixel part of Alg. 3: normalise by b0, mix in the bias vector, build the
// Hankel matrix B[j][k] = beta'_{j+k} and factor B = L L^T.
PixelSetup pixel_setup(const double* b, int m, double alpha, const double* bias) {
  PixelSetup P;
  std::memset(&P, 0, sizeof(P));
  P.n = m / 2;
  P.b0 = b[0];
  if (!(b[0] > 0.0)) {
    P.empty = true;
    return P;
  }
  P.bp[0] = 1.0;
  for (int j = 1; j <= m; ++j) P.bp[j] = (1.0 - alpha) * (b[j] / b[0]) + alpha * bias[j - 1];
  int n = P.n;
  // a single depth carries all absorbance: the variance beta'_2 - beta'_1^2 vanishes
  if (P.bp[2] - P.bp[1] * P.bp[1] <= 1e-12) {
    P.rank1 = true;
    return P;
  }
  for (int j = 0; j <= n; ++j) {
    for (int k = 0; k <= j; ++k) {
      double sum = P.bp[j + k];
      for (int l = 0; l < k; ++l) sum -= P.L[j][l] * P.L[k][l];
      if (j == k) {
        if (sum <= 1e-12 * P.bp[0]) {
          P.nonpd = true;
          sum = 1e-12 * P.bp[0];
        }
        P.L[j][j] = std::sqrt(sum);
      } else {
        P.L[j][k] = sum / P.L[k][k];
      }
    }
  }
  return P;
}

// Per-sample part of Alg. 3 at warped depth zf.  Returns the fraction F of the
// pixel's absorbance attributed to depths before zf; nodes/weights (n+1 each)
// are written when non-null.
double bound_at(const PixelSetup& P, double zf, double eta, double* nodes, double* weights) {
  int n = P.n;
  if (P.rank1) {
    double z1 = P.bp[1];
    if (nodes) {
      nodes[0] = zf;
      nodes[1] = z1;
      weights[0] = 0.0;
      weights[1] = 1.0;
    }
    if (std::fabs(z1 - zf) <= 1e-5) return eta;
    return z1 < zf ? 1.0 : 0.0;
  }
  // solve B q = (1, zf, ..., zf^n) by forward and back substitution
  double rhs[5], y[5], q[5];
  rhs[0] = 1.0;
  for (int j = 1; j <= n; ++j) rhs[j] = rhs[j - 1] * zf;
  for (int j = 0; j <= n; ++j) {
    double sum = rhs[j];
    for (int k = 0; k < j; ++k) sum -= P.L[j][k] * y[k];
    y[j] = sum / P.L[j][j];
  }
  for (int j = n; j >= 0; --j) {
    double sum = y[j];
    for (int k = j + 1; k <= n; ++k) sum -= P.L[k][j] * q[k];
    q[j] = sum / P.L[j][j];
  }
  // nodes: zf and the roots of the kernel polynomial sum_j q_j x^j
  double x[5];
  x[0] = zf;
  int nr = poly_roots(q, n, x + 1);
  int nn = nr + 1;
  // weight of each node = moment functional of its Lagrange basis polynomial
  double F = 0.0;
  for (int i = 0; i < nn; ++i) {
    double coef[5] = {1.0, 0.0, 0.0, 0.0, 0.0};  // running product, ascending powers
    int deg = 0;
    for (int k = 0; k < nn; ++k) {
      if (k == i) continue;
      double inv = 1.0 / (x[i] - x[k]);
      double nc[5] = {0, 0, 0, 0, 0};
      for (int j = 0; j <= deg; ++j) {
        nc[j + 1] += coef[j] * inv;
        nc[j] -= coef[j] * x[k] * inv;
      }
      ++deg;
      std::memcpy(coef, nc, sizeof(nc));
    }
    double lam = 0.0;
    for (int j = 0; j <= deg; ++j) lam += coef[j] * P.bp[j];
    double target = (i == 0) ? eta : (x[i] < zf ? 1.0 : 0.0);
    F += target * lam;
    if (nodes) {
      nodes[i] = x[i];
      weights[i] = lam;
    }
  }
  for (int i = nn; i <= n && nodes; ++i) {
    nodes[i] = INFINITY;
    weights[i] = 0.0;
  }
  return F;
}

// ---------------------------------------------------------------- rendering

struct TetScreen {
  int32_t r0, r1, c0, c1;  // inclusive pixel row/column ranges that may be hit
};

// Conservative pixel range covered by the projection of a tet (one pixel of
// margin); the chord test decides coverage exactly.
bool project_tet(const OView& v, const V3 p[4], TetScreen& ts) {
  V3 e = from(v.eye), f = from(v.dir), r = from(v.right), dn = from(v.down);
  double fn = std::sqrt(dot(f, f));
  V3 fu = (1.0 / fn) * f;
  double rr = dot(r, r), dd = dot(dn, dn);
  double cmin = 1e300, cmax = -1e300, rmin = 1e300, rmax = -1e300;
  for (int k = 0; k < 4; ++k) {
    V3 y = p[k] - e;
    double a, b;
    if (v.projection == 0) {
      a = dot(y, r) / rr - 0.5;
      b = dot(y, dn) / dd - 0.5;
    } else {
      double depth = dot(y, fu) / fn;  // coefficient of dir
      if (depth <= 0.0) return false;
      a = dot(y, r) / (rr * depth) + 0.5 * v.width - 0.5;
      b = dot(y, dn) / (dd * depth) + 0.5 * v.height - 0.5;
    }
    cmin = std::min(cmin, a);
    cmax = std::max(cmax, a);
    rmin = std::min(rmin, b);
    rmax = std::max(rmax, b);
  }
  cmin = std::floor(cmin) - 1;
  rmin = std::floor(rmin) - 1;
  cmax = std::ceil(cmax) + 1;
  rmax = std::ceil(rmax) + 1;
  if (cmax < 0 || rmax < 0 || cmin > v.width - 1 || rmin > v.height - 1) return false;
  ts.c0 = int32_t(std::max(0.0, cmin));
  ts.r0 = int32_t(std::max(0.0, rmin));
  ts.c1 = int32_t(std::min(double(v.width - 1), cmax));
  ts.r1 = int32_t(std::min(double(v.height - 1), rmax));
  return true;
}

constexpr int TILE = 16;

struct ExactPiece {
  double tm;
  int32_t sub;
  int64_t tet;
  double a, rgb[3];
};

}  // namespace

extern "C" {

double oracle_warp(double t, double t_near, double t_far) { return warp(t, t_near, t_far); }

int oracle_chord(const double* p12, const double* o3, const double* d3, double* out2) {
  V3 p[4] = {from(p12), from(p12 + 3), from(p12 + 6), from(p12 + 9)};
  return tet_chord(p, from(o3), from(d3), out2[0], out2[1]) ? 1 : 0;
}

int oracle_roots(const double* coef, int n, double* roots) { return poly_roots(coef, n, roots); }

// Moment bound for one moment vector b[0..m] at warped depth zf.
// flags out: bit0 empty, bit1 rank1, bit2 non-PD.
double oracle_bound(const double* b, int m, double alpha, const double* bias, double eta, double zf,
                    double* nodes, double* weights, int* flags) {
  PixelSetup P = pixel_setup(b, m, alpha, bias);
  if (flags) *flags = (P.empty ? 1 : 0) | (P.rank1 ? 2 : 0) | (P.nonpd ? 4 : 0);
  if (P.empty) return 0.0;
  return bound_at(P, zf, eta, nodes, weights);
}

void oracle_depth_range(const OScene* s, double* out2) { depth_range(*s, out2[0], out2[1]); }

int oracle_render(const OScene* sp, OOut* out) {
  const OScene& s = *sp;
  const OView& v = s.view;
  const int m = s.m, S = s.n_sub, M1 = m + 1;
  if (m < 2 || m > 8 || (m & 1)) return 1;
  double t_near, t_far;
  depth_range(s, t_near, t_far);
  out->t_near = t_near;
  out->t_far = t_far;
  if (!(t_near > 0.0)) return 2;
  const int64_t W = v.width, H = v.height;
  const int64_t P = out->pixels ? out->n_pixels : W * H;
  // pixel id -> output slot
  std::vector<int64_t> slot_of(W * H, -1);
  for (int64_t q = 0; q < P; ++q) {
    int64_t pid = out->pixels ? out->pixels[q] : q;
    if (pid < 0 || pid >= W * H) return 3;
    slot_of[pid] = q;
  }
  const int64_t TW = (W + TILE - 1) / TILE, TH = (H + TILE - 1) / TILE;
  std::vector<char> tile_active(TW * TH, 0);
  for (int64_t pid = 0; pid < W * H; ++pid)
    if (slot_of[pid] >= 0) tile_active[(pid / W / TILE) * TW + (pid % W) / TILE] = 1;
  // bin tets into the active tiles their projection may touch
  std::vector<TetScreen> scr(s.n_tets);
  std::vector<char> vis(s.n_tets, 0);
  int nth = out->n_threads > 0 ? out->n_threads : 1;
#pragma omp parallel for schedule(static) num_threads(nth)
  for (int64_t t = 0; t < s.n_tets; ++t) {
    V3 p[4];
    for (int k = 0; k < 4; ++k) p[k] = vertex(s, s.tets[4 * t + k]);
    vis[t] = project_tet(v, p, scr[t]) ? 1 : 0;
  }
  std::vector<std::vector<int64_t>> bins(TW * TH);
  for (int64_t t = 0; t < s.n_tets; ++t) {
    if (!vis[t]) continue;
    const TetScreen& ts = scr[t];
    for (int64_t ty = ts.r0 / TILE; ty <= ts.r1 / TILE; ++ty)
      for (int64_t tx = ts.c0 / TILE; tx <= ts.c1 / TILE; ++tx)
        if (tile_active[ty * TW + tx]) bins[ty * TW + tx].push_back(t);
  }
  std::vector<int64_t> active;
  for (int64_t k = 0; k < TW * TH; ++k)
    if (tile_active[k]) active.push_back(k);

  std::vector<double> gmom(size_t(M1) * P, 0.0);
  std::vector<int64_t> pieces_sub(S, 0);
  int64_t n_chords = 0, n_nonpd = 0, n_rank1 = 0;

  // visit every (pixel, tet) chord of a tile's active pixels
  auto for_each_chord = [&](int64_t tile, auto&& fn) {
    int64_t ty = tile / TW, tx = tile % TW;
    for (int64_t t : bins[tile]) {
      const TetScreen& ts = scr[t];
      V3 p[4];
      double sv[4];
      for (int k = 0; k < 4; ++k) {
        p[k] = vertex(s, s.tets[4 * t + k]);
        sv[k] = s.scalar[s.tets[4 * t + k]];
      }
      int64_t r0 = std::max<int64_t>(ts.r0, ty * TILE), r1 = std::min<int64_t>(ts.r1, ty * TILE + TILE - 1);
      int64_t c0 = std::max<int64_t>(ts.c0, tx * TILE), c1 = std::min<int64_t>(ts.c1, tx * TILE + TILE - 1);
      for (int64_t i = r0; i <= r1; ++i)
        for (int64_t j = c0; j <= c1; ++j) {
          int64_t q = slot_of[i * W + j];
          if (q < 0) continue;
          V3 o, d;
          pixel_ray(v, i, j, o, d);
          double t0, t1;
          if (!tet_chord(p, o, d, t0, t1)) continue;
          fn(q, t, p, sv, o, d, t0, t1);
        }
    }
  };

  // ---- pass 1: per-subdomain moments, then their sum (Section 4.1)
#pragma omp parallel num_threads(nth) reduction(+ : n_chords)
  {
    std::vector<int64_t> my_pieces(S, 0);
    std::vector<double> local;
    std::vector<int64_t> tile_pix;
    std::vector<std::vector<std::pair<double, double>>> ivl;  // chords per (local pixel, subdomain)
#pragma omp for schedule(dynamic, 1)
    for (int64_t ai = 0; ai < int64_t(active.size()); ++ai) {
      int64_t tile = active[ai];
      int64_t ty = tile / TW, tx = tile % TW;
      tile_pix.clear();
      for (int64_t i = ty * TILE; i < std::min(H, ty * TILE + TILE); ++i)
        for (int64_t j = tx * TILE; j < std::min(W, tx * TILE + TILE); ++j)
          if (slot_of[i * W + j] >= 0) tile_pix.push_back(slot_of[i * W + j]);
      // local[q_local][sub][j]
      local.assign(size_t(TILE * TILE) * S * M1, 0.0);
      auto lidx = [&](int64_t q) {
        int64_t pid = out->pixels ? out->pixels[q] : q;
        int64_t i = pid / W - ty * TILE, j = pid % W - tx * TILE;
        return (i * TILE + j) * S * M1;
      };
      if (out->segments) ivl.assign(size_t(TILE * TILE) * S, {});
      for_each_chord(tile, [&](int64_t q, int64_t t, const V3* p, const double* sv, V3 o, V3 d, double t0,
                               double t1) {
        ++n_chords;
        int sub = s.tet_sub[t];
        double* bl = &local[lidx(q) + size_t(sub) * M1];
        if (out->segments) ivl[lidx(q) / M1 + sub].push_back({t0, t1});
        pieces_of_chord(s, p, sv, o, d, t0, t1, t_near, [&](const Piece& pc) {
          double z = warp(pc.tm, t_near, t_far);
          double zp = 1.0;
          for (int j = 0; j <= m; ++j) {
            bl[j] += pc.a * zp;  // Alg. 2: moment j gains absorbance * depth^j
            zp *= z;
          }
          ++my_pieces[sub];
        });
      });
      // segments: a pixel ray's chords in one subdomain, sorted along the ray, form one segment per run of
      // chords that meet end to start (neighbouring tets share the face); a gap starts a new segment
      if (out->segments)
        for (int64_t q : tile_pix) {
          int32_t segs = 0, met = 0;
          for (int sub = 0; sub < S; ++sub) {
            auto& c = ivl[lidx(q) / M1 + sub];
            if (c.empty()) continue;
            std::sort(c.begin(), c.end());
            ++met;
            ++segs;
            for (size_t k = 1; k < c.size(); ++k)
              if (c[k].first > c[k - 1].second + 1e-9 * (1.0 + std::fabs(c[k - 1].second))) ++segs;
          }
          out->segments[q] = segs;
          out->segments[P + q] = met;
        }
      for (int64_t q : tile_pix) {
        const double* bl = &local[lidx(q)];
        for (int j = 0; j <= m; ++j) {
          double sum = 0.0;
          for (int sub = 0; sub < S; ++sub) {
            sum += bl[sub * M1 + j];
            if (out->moments_sub) out->moments_sub[(size_t(sub) * M1 + j) * P + q] = bl[sub * M1 + j];
          }
          gmom[size_t(j) * P + q] = sum;
        }
      }
    }
#pragma omp critical
    for (int k = 0; k < S; ++k) pieces_sub[k] += my_pieces[k];
  }
  if (out->moments) std::memcpy(out->moments, gmom.data(), sizeof(double) * M1 * P);
  int64_t total_pieces = 0;
  for (int k = 0; k < S; ++k) total_pieces += pieces_sub[k];
  if (out->pieces_sub)
    for (int k = 0; k < S; ++k) out->pieces_sub[k] = pieces_sub[k];
  out->n_pieces = total_pieces;
  out->n_chords = n_chords;
  if (!out->do_pass2) return 0;

  // ---- pass 2: transmittance from the global moments, colour per subdomain (Section 4.2)
  std::vector<PixelSetup> setup(P);
#pragma omp parallel for schedule(static) num_threads(nth) reduction(+ : n_nonpd, n_rank1)
  for (int64_t q = 0; q < P; ++q) {
    double b[9];
    for (int j = 0; j <= m; ++j) b[j] = gmom[size_t(j) * P + q];
    setup[q] = pixel_setup(b, m, s.alpha, s.bias);
    n_nonpd += setup[q].nonpd ? 1 : 0;
    n_rank1 += setup[q].rank1 ? 1 : 0;
  }
  out->n_nonpd = n_nonpd;
  out->n_rank1 = n_rank1;
#pragma omp parallel num_threads(nth)
  {
    std::vector<double> local;
    std::vector<std::vector<ExactPiece>> plist;
    std::vector<int64_t> tile_pix;
#pragma omp for schedule(dynamic, 1)
    for (int64_t ai = 0; ai < int64_t(active.size()); ++ai) {
      int64_t tile = active[ai];
      int64_t ty = tile / TW, tx = tile % TW;
      tile_pix.clear();
      for (int64_t i = ty * TILE; i < std::min(H, ty * TILE + TILE); ++i)
        for (int64_t j = tx * TILE; j < std::min(W, tx * TILE + TILE); ++j)
          if (slot_of[i * W + j] >= 0) tile_pix.push_back(slot_of[i * W + j]);
      local.assign(size_t(TILE * TILE) * S * 4, 0.0);
      if (out->exact) {
        plist.assign(TILE * TILE, {});
      }
      auto lpix = [&](int64_t q) {
        int64_t pid = out->pixels ? out->pixels[q] : q;
        int64_t i = pid / W - ty * TILE, j = pid % W - tx * TILE;
        return i * TILE + j;
      };
      for_each_chord(tile, [&](int64_t q, int64_t t, const V3* p, const double* sv, V3 o, V3 d, double t0,
                               double t1) {
        const PixelSetup& ps = setup[q];
        int sub = s.tet_sub[t];
        double* cl = &local[(lpix(q) * S + sub) * 4];
        pieces_of_chord(s, p, sv, o, d, t0, t1, t_near, [&](const Piece& pc) {
          double alpha_p = -std::expm1(-pc.a);
          if (!ps.empty) {
            double z = warp(pc.tm, t_near, t_far);
            double F = bound_at(ps, z, s.eta, nullptr, nullptr);
            double T = std::exp(-ps.b0 * F);
            T = std::min(1.0, std::max(0.0, T));
            for (int c = 0; c < 3; ++c) cl[c] += T * alpha_p * pc.rgb[c];  // Alg. 1, second loop
            cl[3] += T * alpha_p;
          }
          if (out->exact) {
            ExactPiece e;
            e.tm = pc.tm;
            e.sub = sub;
            e.tet = t;
            e.a = pc.a;
            for (int c = 0; c < 3; ++c) e.rgb[c] = pc.rgb[c];
            plist[lpix(q)].push_back(e);
          }
        });
      });
      for (int64_t q : tile_pix) {
        int64_t lp = lpix(q);
        double acc[4] = {0, 0, 0, 0};
        for (int sub = 0; sub < S; ++sub) {
          const double* cl = &local[(lp * S + sub) * 4];
          for (int c = 0; c < 4; ++c) acc[c] += cl[c];
          if (out->color_sub)
            for (int c = 0; c < 4; ++c) out->color_sub[(size_t(sub) * P + q) * 4 + c] = cl[c];
        }
        if (out->color)
          for (int c = 0; c < 4; ++c) out->color[q * 4 + c] = acc[c];
        if (out->rgba) {
          double b0 = gmom[q];
          double* o4 = out->rgba + q * 4;
          if (s.renormalize) {
            double A = -std::expm1(-b0);
            double sc = acc[3] > 1e-30 ? A / acc[3] : 0.0;
            for (int c = 0; c < 3; ++c) o4[c] = acc[c] * sc;
            o4[3] = A;
          } else {
            for (int c = 0; c < 4; ++c) o4[c] = acc[c];
          }
        }
        if (out->exact) {
          auto& L = plist[lp];
          std::sort(L.begin(), L.end(), [](const ExactPiece& x, const ExactPiece& y) {
            if (x.tm != y.tm) return x.tm < y.tm;
            if (x.sub != y.sub) return x.sub < y.sub;
            return x.tet < y.tet;
          });
          double tau = 0.0, e4[4] = {0, 0, 0, 0};
          for (const ExactPiece& e : L) {
            double w = std::exp(-tau) * (-std::expm1(-e.a));
            for (int c = 0; c < 3; ++c) e4[c] += w * e.rgb[c];
            tau += e.a;
          }
          e4[3] = -std::expm1(-tau);
          for (int c = 0; c < 4; ++c) out->exact[q * 4 + c] = e4[c];
        }
      }
    }
  }
  return 0;
}

}  // extern "C"
