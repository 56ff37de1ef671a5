// Moment-bound reconstruction of transmittance (paper Alg. 3), for the GPU.
//
// Per pixel (hoisted out of the per-sample loop of Alg. 3, same result):
//   beta'_j = (1 - alpha) * b_j / b0 + alpha * bias_j,  beta'_0 = 1
//   B = Hankel(beta'_0..beta'_2n) of size (n+1)^2,  B = L L^T,  Li = L^-1
//   xlo, xhi = smallest and largest zero of the orthonormal polynomial of
//              degree n (row n of Li)
// Per sample at warped depth z:
//   P = Li * (1, z, ..., z^n)       values of the orthonormal polynomials at z
//   q = Li^T * P                    coefficients of the kernel polynomial
//                                   K(x, z) = (1, x, ..., x^n) B^-1 (1, z, ..., z^n)^T
//   x_1..x_n = roots of K(., z)     (real and simple when B is positive definite)
//   the nodes {z, x_1..x_n} carry the weights 1 / K(x_i, x_i) (Christoffel
//   numbers: the nodes are pairwise K-orthogonal, so a degree-2n quadrature on
//   them reproduces all moments exactly; the weights sum to 1)
//   F = eta / K(z, z) + sum_{x_i < z} 1 / K(x_i, x_i)
// F is the fraction of the pixel's absorbance in front of z; the caller forms
// T = clamp(exp(-b0 * F), 0, 1).  This is the same quantity as evaluating the
// 0/1/eta interpolant through the nodes against the biased moments (Alg. 3,
// the polynomial solve and dot product), reached through the Christoffel
// numbers instead of a Lagrange or Newton interpolant.
//
// The nodes other than z interlace with the zeros of the degree-n orthonormal
// polynomial: each gap between consecutive zeros, and each of the two
// unbounded ends, holds exactly one node except the gap that holds z.  So for
// z below the smallest zero no node lies in front (F = eta / K(z, z)), for z
// above the largest all do (F = 1 - (1 - eta) / K(z, z)), and only in between
// are the roots needed; the weights are summed over whichever side of z has
// fewer nodes.
//
// Roots: closed forms (quadratic; trigonometric cubic; Ferrari quartic whose
// resolvent's largest root comes from the trigonometric cubic), each root
// polished by Newton steps on the kernel polynomial.  A vanishing leading
// coefficient means one node has gone to infinity with zero weight; the
// degree is lowered instead of dividing by it.  Reciprocals use the hardware
// estimate plus Newton-Raphson steps in FP64 on the device: two, or one for
// the weights in the continuation below (measured: the same FP32 image).
//
// Gap tables (n >= 3, FP64).  Written t for the zeros of the degree-n
// orthonormal polynomial, the node sets vary smoothly with z inside each gap
// (t_k-1, t_k), and at the gap's ends they become the other zeros plus one node
// at infinity.  A pixel with many samples therefore solves the closed forms
// only at 64 depths spread over its gaps (one per lane), stores a regularised
// position of each root a sample in that gap will need, and gives each sample
// its roots by quadratic interpolation in that table followed by four Newton
// steps on the kernel polynomial.  A root that does not land in its gap, or
// whose last Newton step is not small enough for the weight to be exact to
// about 1e-12, sends the sample back to the closed forms, so the table changes
// the cost of a sample but not its result beyond rounding.
//
// Precision R is float or double; n = m/2 is 2, 3 or 4.
//
// The functions are host+device so that host-side tests can exercise the code
// the kernels run (on the host, reciprocals are IEEE divisions).
#pragma once

#include <math.h>

#include <type_traits>

#if defined(__HIPCC__)
#define APC_HD __host__ __device__ inline
// out of line on the device: called once per pixel or for rare samples, and
// inlined it would set the register budget of the loops around it
#define APC_HD_COLD __host__ __device__ __attribute__((noinline))
#else
#define APC_HD inline
#define APC_HD_COLD inline
#endif

namespace apcm {

template <class R>
struct Num;
template <>
struct Num<float> {
  static constexpr float rank1_tol = 1e-6f;    // variance below which all absorbance sits at one depth
  static constexpr float pivot_floor = 1e-9f;  // smallest admitted Cholesky pivot
  static constexpr float deg_tol = 1e-6f;      // relative size of a negligible leading coefficient
  static constexpr float far = 1e8f;           // nodes beyond this carry no weight
  static constexpr float same_depth = 1e-5f;   // single-depth branch: "at the sample's depth"
};
template <>
struct Num<double> {
  static constexpr double rank1_tol = 1e-12;
  static constexpr double pivot_floor = 1e-12;
  static constexpr double deg_tol = 1e-13;
  static constexpr double far = 1e30;
  static constexpr double same_depth = 1e-5;
};

APC_HD float m_sqrt(float x) { return sqrtf(x); }
APC_HD double m_sqrt(double x) { return sqrt(x); }
APC_HD float m_acos(float x) { return acosf(x); }
APC_HD double m_acos(double x) { return acos(x); }
APC_HD float m_cos(float x) { return cosf(x); }
APC_HD double m_cos(double x) { return cos(x); }
APC_HD float m_cbrt(float x) { return cbrtf(x); }
APC_HD double m_cbrt(double x) { return cbrt(x); }
APC_HD float m_abs(float x) { return fabsf(x); }
APC_HD double m_abs(double x) { return fabs(x); }

// 1/b for finite b != 0: hardware reciprocal estimate (refined by
// Newton-Raphson in FP64) on the device, a plain division on the host.
APC_HD float m_rcp(float b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(b);
#else
  return 1.0f / b;
#endif
}
APC_HD double m_rcp(double b) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(b);
  r = fma(fma(-b, r, 1.0), r, r);
  r = fma(fma(-b, r, 1.0), r, r);
  return r;
#else
  return 1.0 / b;
#endif
}

// 1/b for finite b != 0 with one Newton-Raphson refinement of the estimate
APC_HD double m_rcp1(double b) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(b);
  return fma(fma(-b, r, 1.0), r, r);
#else
  return 1.0 / b;
#endif
}

// 1/b to about half precision (hardware estimate on the device): enough for
// the steps of an iteration whose final step is checked
APC_HD double m_rcp_est(double b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcp(b);
#else
  return 1.0 / b;
#endif
}

template <class R>
APC_HD R m_max(R a, R b) {
  return a > b ? a : b;
}
template <class R>
APC_HD R m_min(R a, R b) {
  return a < b ? a : b;
}
template <class R>
APC_HD R m_clamp(R x, R lo, R hi) {
  return x < lo ? lo : (x > hi ? hi : x);
}
template <class R>
APC_HD bool m_finite(R x) {
  return x - x == R(0);
}

// Real roots of c0 + c1 x + c2 x^2 (numerically stable form).  Returns count.
template <class R>
APC_HD int roots2(R c0, R c1, R c2, R* x) {
  R x0 = R(0), x1 = R(0);
  int nr = 2;
  if (c2 == R(0)) {
    nr = c1 == R(0) ? 0 : 1;
    x0 = nr ? -c0 * m_rcp(c1) : R(0);
  } else {
    R disc = m_max(c1 * c1 - R(4) * c2 * c0, R(0));
    R s = m_sqrt(disc);
    R t = R(-0.5) * (c1 + (c1 < R(0) ? -s : s));
    if (t != R(0)) {  // t = 0 only for c1 = c0 = 0: double root at 0
      x0 = t * m_rcp(c2);
      x1 = c0 * m_rcp(t);
    }
  }
  x[0] = x0;
  x[1] = x1;
  return nr;
}

// Roots of the depressed cubic y^3 + p y + q, real parts when two are complex;
// y[0] is the largest when all three are real.
template <class R>
APC_HD void depressed3(R p, R q, R* y) {
  // both branches end in one store per element (stores sunk out of the
  // branches would otherwise be merged into one with a run-time address)
  const R two_pi_3 = R(2.0943951023931954923);
  R y0, y1, y2;
  if (p < R(0)) {
    R mm = m_sqrt(-p * R(1.0 / 3.0));
    R arg = m_clamp(-q * m_rcp(R(2) * mm * mm * mm), R(-1), R(1));
    R th = m_acos(arg) * R(1.0 / 3.0);
    y0 = R(2) * mm * m_cos(th);
    y1 = R(2) * mm * m_cos(th - two_pi_3);
    y2 = R(2) * mm * m_cos(th + two_pi_3);
  } else {
    R sd = m_sqrt(m_max(q * q * R(0.25) + p * p * p * R(1.0 / 27.0), R(0)));
    R u = m_cbrt(-q * R(0.5) + sd), w = m_cbrt(-q * R(0.5) - sd);
    y0 = u + w;
    y1 = R(-0.5) * (u + w);
    y2 = y1;
  }
  y[0] = y0;
  y[1] = y1;
  y[2] = y2;
}

// Roots of c0 + c1 x + c2 x^2 + c3 x^3 (c3 != 0); x[0] is the largest when all are real.
template <class R>
APC_HD int roots3(const R* c, R* x) {
  R inv = m_rcp(c[3]);
  R a = c[2] * inv, b = c[1] * inv, cc = c[0] * inv;
  R a3 = a * R(1.0 / 3.0);
  R p = b - a * a3;
  R q = cc + a3 * (R(2) * a3 * a3 - b);
  R y[3];
  depressed3(p, q, y);
#pragma unroll
  for (int i = 0; i < 3; ++i) x[i] = y[i] - a3;
  return 3;
}

// Largest real root of m^3 + p m^2 + s m + t (only that root is needed, so
// one cosine instead of three), polished by two Newton steps.
template <class R>
APC_HD R largest_root3(R p, R s, R t) {
  const R a3 = p * R(1.0 / 3.0);
  const R pp = s - p * a3;
  const R qq = t + a3 * (R(2) * a3 * a3 - s);
  R m0;
  if (pp < R(0)) {
    const R mm = m_sqrt(-pp * R(1.0 / 3.0));
    const R arg = m_clamp(-qq * m_rcp(R(2) * mm * mm * mm), R(-1), R(1));
    m0 = R(2) * mm * m_cos(m_acos(arg) * R(1.0 / 3.0)) - a3;
  } else {
    const R sd = m_sqrt(m_max(qq * qq * R(0.25) + pp * pp * pp * R(1.0 / 27.0), R(0)));
    m0 = m_cbrt(-qq * R(0.5) + sd) + m_cbrt(-qq * R(0.5) - sd) - a3;
  }
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const R f = ((m0 + p) * m0 + s) * m0 + t;
    const R df = (R(3) * m0 + R(2) * p) * m0 + s;
    if (df != R(0)) {
      const R mn = m0 - f * m_rcp(df);
      if (m_finite(mn)) m0 = mn;
    }
  }
  return m0;
}

// Roots of c0 + ... + c4 x^4 (c4 != 0) by Ferrari's resolvent.
template <class R>
APC_HD int roots4(const R* c, R* x) {
  R inv = m_rcp(c[4]);
  R a = c[3] * inv, b = c[2] * inv, cc = c[1] * inv, d = c[0] * inv;
  R a4 = a * R(0.25), a4s = a4 * a4;
  R p = b - R(6) * a4s;
  R q = cc - R(2) * b * a4 + R(8) * a4s * a4;
  R r = d - cc * a4 + b * a4s - R(3) * a4s * a4s;
  // resolvent m^3 + p m^2 + (p^2/4 - r) m - q^2/8 = 0: its largest root is >= 0
  R m0 = largest_root3(p, p * p * R(0.25) - r, -q * q * R(0.125));
  R y[4];
  if (!(m0 > R(0))) {  // biquadratic y^4 + p y^2 + r
    R w[2];
    roots2(r, p, R(1), w);
    R s0 = m_sqrt(m_max(w[0], R(0))), s1 = m_sqrt(m_max(w[1], R(0)));
    y[0] = s0;
    y[1] = -s0;
    y[2] = s1;
    y[3] = -s1;
  } else {
    R s = m_sqrt(R(2) * m0);
    R h = q * m_rcp(R(2) * s);
    R base = p * R(0.5) + m0;
    roots2(base + h, -s, R(1), y);
    roots2(base - h, s, R(1), y + 2);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) x[i] = y[i] - a4;
  return 4;
}

// The closed-form solve runs out of line (see APC_HD_COLD) with its
// coefficients and roots passed by value, which keeps them in registers
// instead of a stack frame in scratch memory.
template <int N, class R>
struct RootSet {
  R x[N];
  int n;
};
template <int N, class R>
struct PolyCoef {
  R c[N + 1];
};
template <int N, class R, int POLISH>
APC_HD int poly_roots_body(const R* q, R* x);
template <int N, class R, int POLISH>
APC_HD_COLD RootSet<N, R> poly_roots_v(PolyCoef<N, R> q) {
  RootSet<N, R> r;
#pragma unroll
  for (int i = 0; i < N; ++i) r.x[i] = R(0);
  r.n = poly_roots_body<N, R, POLISH>(q.c, r.x);
  return r;
}
// Roots of the polynomial q[0..N]; returns how many finite ones (x[0..nr)).  POLISH Newton steps on the
// full polynomial follow the closed forms: for cubics and quartics, made monic first, three give working
// precision even when the leading coefficient nearly vanishes (one suffices where the roots only start
// further Newton iterations); the quadratic formula here divides by no small coefficient, so one step.
template <int N, class R, int POLISH = (N >= 3 ? 3 : 1)>
APC_HD int poly_roots(const R* q, R* x) {
  PolyCoef<N, R> c;
#pragma unroll
  for (int j = 0; j <= N; ++j) c.c[j] = q[j];
  const RootSet<N, R> r = poly_roots_v<N, R, POLISH>(c);
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = r.x[i];
  return r.n;
}
template <int N, class R, int POLISH>
APC_HD int poly_roots_body(const R* q, R* x) {
  R cmax = R(0);
#pragma unroll
  for (int j = 0; j <= N; ++j) cmax = m_max(cmax, m_abs(q[j]));
  // degree after dropping negligible leading coefficients (unrolled: no indexed arrays)
  int deg = 0;
  bool top = true;
#pragma unroll
  for (int j = N; j >= 1; --j) {
    if (top && m_abs(q[j]) > Num<R>::deg_tol * cmax) {
      deg = j;
      top = false;
    }
  }
  int nr = 0;
  if (N >= 3 && deg == N && m_abs(q[N]) < R(1e-4) * cmax) {
    // A small leading coefficient: one root lies far out (the sample depth is near a zero of the degree-N
    // orthonormal polynomial).  Made monic, the polynomial's other coefficients would swamp the closed
    // forms; instead the far root comes from the two leading coefficients, refined by Newton on the full
    // polynomial, and is divided out from the low end (b_0 = -q_0 / r, b_j = (b_(j-1) - q_j) / r), which is
    // stable for a large root; the quotient's roots come from the closed forms one degree lower.
    R r = -q[N - 1] * m_rcp(q[N]);
#pragma unroll
    for (int it = 0; it < 3; ++it) {
      R p = q[N], dp = R(0);
#pragma unroll
      for (int j = N - 1; j >= 0; --j) {
        dp = dp * r + p;
        p = p * r + q[j];
      }
      if (dp != R(0)) {
        const R rn = r - p * m_rcp(dp);
        if (m_finite(rn)) r = rn;
      }
    }
    R b[N];
    const R ir = m_rcp(r);
    b[0] = -q[0] * ir;
#pragma unroll
    for (int j = 1; j < N; ++j) b[j] = (b[j - 1] - q[j]) * ir;
    if constexpr (N == 4) {
      nr = roots3(b, x) + 1;
    } else {
      nr = roots2(b[0], b[1], b[2], x) + 1;
    }
    x[N - 1] = r;
  } else if (deg == 1) {
    x[0] = -q[0] * m_rcp(q[1]);
    nr = 1;
  } else if (deg == 2) {
    nr = roots2(q[0], q[1], q[2], x);
  } else if (N >= 3 && deg == 3) {
    nr = roots3(q, x);
  } else if (N >= 4 && deg == 4) {
    nr = roots4(q, x);
  }
  // Newton steps on the full polynomial (fixed trip counts: no indexed arrays).  A vanishing leading
  // coefficient (one root far out) makes the monic closed forms lose digits of the other roots: one step
  // left F off by up to 1.5e-7 on rendered pixels at m = 8, three keep it within 1e-12.
#pragma unroll
  for (int i = 0; i < N; ++i) {
    if (i >= nr) continue;
    R xi = x[i];
#pragma unroll
    for (int it = 0; it < POLISH; ++it) {
      R p = q[N], dp = R(0);
#pragma unroll
      for (int j = N - 1; j >= 0; --j) {
        dp = dp * xi + p;
        p = p * xi + q[j];
      }
      if (dp != R(0)) {
        R xn = xi - p * m_rcp(dp);
        if (m_finite(xn)) xi = xn;
      }
    }
    x[i] = xi;
  }
  return nr;
}

// the name the host tests use
template <int N, class R>
APC_HD int kernel_roots(const R* q, R* x) {
  return poly_roots<N, R>(q, x);
}

// Storage of the packed inverse factor: a plain array (host tests), or a
// lane-strided slice of LDS shared by a wavefront (kernels).
template <int NL, class R>
struct ArrayStore {
  R v[NL];
  APC_HD R& operator[](int k) { return v[k]; }
  APC_HD const R& operator[](int k) const { return v[k]; }
};
template <int NL, class R, int STRIDE>
struct StridedStore {
  R* base;  // element k at base[k * STRIDE]
  APC_HD R& operator[](int k) const { return base[k * STRIDE]; }
};

// Gap-table shape for n = N: NI nodes per gap, N - 1 gaps, at most NC roots
// per sample (the side of z with fewer nodes).
template <int N>
struct Gaps {
  static constexpr int NI = N >= 3 ? 64 / (N - 1) : 2;
  static constexpr int NC = N / 2;
  static constexpr int NODES = (N - 1) * NI;
};

// Storage of one pixel's gap table: a plain array (host tests) or a slice of
// LDS shared by the wavefront (kernels).  Entry (node, c) at node * NC + c.
template <int N, class R>
struct TableArray {
  R v[Gaps<N>::NODES * Gaps<N>::NC];
  APC_HD R& at(int node, int c) { return v[node * Gaps<N>::NC + c]; }
  APC_HD const R& at(int node, int c) const { return v[node * Gaps<N>::NC + c]; }
};
template <int N, class R>
struct TablePtr {
  R* base;
  APC_HD R& at(int node, int c) const { return base[node * Gaps<N>::NC + c]; }
};

// a[i] for a run-time i: plain indexing for memory-backed accessors (the
// zeros live in LDS on the device) ...
template <int K, class A>
APC_HD auto pick(const A& a, int i) -> decltype(a[0] + 0) {
  return a[i];
}
// ... and, for a register array, a sum of masked terms, which the compiler
// cannot turn back into an indexed (scratch) access; a[] must be finite.
template <int K, class R>
APC_HD R pick_reg(const R* a, int i) {
  R r = R(0);
#pragma unroll
  for (int t = 0; t < K; ++t) r += R(i == t ? 1 : 0) * a[t];
  return r;
}

// K values held in registers, read with a run-time index as an OR of masked
// bit patterns (never an indexed register or scratch access; a constant index
// folds to the element itself).  A chain of selects between the elements is
// not enough: the compiler folds a select of two loads into one load from a
// selected address, and a run-time address into the array keeps the whole
// array, and any structure holding it, in scratch memory.
template <int K, class R>
struct RegArray {
  R v[K];
  APC_HD R operator[](int i) const {
    using U = typename std::conditional<sizeof(R) == 8, unsigned long long, unsigned>::type;
    U r = 0;
#pragma unroll
    for (int t = 0; t < K; ++t) r |= (i == t ? ~U(0) : U(0)) & __builtin_bit_cast(U, v[t]);
    return __builtin_bit_cast(R, r);
  }
};

// Per-pixel state of the bound.
template <int N, class R, class Store = ArrayStore<(N + 1) * (N + 2) / 2, R>>
struct Bound {
  static constexpr int NL = (N + 1) * (N + 2) / 2;
  R b0;
  R z1;        // single-depth branch: the depth
  R xlo, xhi;  // smallest / largest zero of the degree-N orthonormal polynomial
  Store Li;    // L^-1, packed lower triangle: row k starts at k(k+1)/2
  int mode;    // 0: no absorbance, 1: all absorbance at depth z1, 2: regular

  // b[0..2N] raw moments; bias[0..2N-1] = b*_1..b*_2N.  Returns the number of
  // Cholesky pivots that had to be floored.  With zeros != null, the N zeros
  // of the degree-N orthonormal polynomial are written there in ascending
  // order (all equal to 0 when they could not be found; xlo > xhi then).
  APC_HD int setup(const R* b, R alpha, const R* bias, R* zeros = nullptr) {
    mode = 0;
    b0 = b[0];
    z1 = R(0);
    xlo = R(1);
    xhi = R(-1);
    if (zeros) {
#pragma unroll
      for (int i = 0; i < N; ++i) zeros[i] = R(0);
    }
    if (!(b0 > R(0))) return 0;
    R bp[2 * N + 1];
    bp[0] = R(1);
    R inv0 = R(1) / b0;
#pragma unroll
    for (int j = 1; j <= 2 * N; ++j) bp[j] = (R(1) - alpha) * (b[j] * inv0) + alpha * bias[j - 1];
    if (bp[2] - bp[1] * bp[1] <= Num<R>::rank1_tol) {
      mode = 1;
      z1 = bp[1];
      return 0;
    }
    mode = 2;
    R L[N + 1][N + 1];
    int floored = 0;
#pragma unroll
    for (int j = 0; j <= N; ++j) {
#pragma unroll
      for (int k = 0; k < j; ++k) {
        R s = bp[j + k];
#pragma unroll
        for (int l = 0; l < k; ++l) s -= L[j][l] * L[k][l];
        L[j][k] = s / L[k][k];
      }
      R dd = bp[2 * j];
#pragma unroll
      for (int l = 0; l < j; ++l) dd -= L[j][l] * L[j][l];
      if (!(dd > Num<R>::pivot_floor)) {
        dd = Num<R>::pivot_floor;
        ++floored;
      }
      L[j][j] = m_sqrt(dd);
    }
    R row[N + 1];  // row N of Li: coefficients of the orthonormal polynomial of degree N
#pragma unroll
    for (int j = 0; j <= N; ++j) {
      R dj = R(1) / L[j][j];
      Li[j * (j + 1) / 2 + j] = dj;
      if (j == N) row[N] = dj;
#pragma unroll
      for (int k = 0; k < j; ++k) {
        R s = R(0);
#pragma unroll
        for (int l = k; l < j; ++l) s += L[j][l] * Li[l * (l + 1) / 2 + k];
        Li[j * (j + 1) / 2 + k] = -s * dj;
        if (j == N) row[k] = -s * dj;
      }
    }
    // its zeros lie inside (-1, 1)
    R xi[N];
#pragma unroll
    for (int i = 0; i < N; ++i) xi[i] = R(0);
    const int nz = poly_roots<N, R>(row, xi);
    if (nz < N) return floored;  // cannot happen for a positive definite factor; no shortcut
    sort_up(xi);
    xlo = xi[0];
    xhi = xi[N - 1];
    if (zeros) {
#pragma unroll
      for (int i = 0; i < N; ++i) zeros[i] = xi[i];
    }
    return floored;
  }

  // ascending order of N values (odd-even transposition: fixed compare-exchanges)
  APC_HD static void sort_up(R* x) {
#pragma unroll
    for (int pass = 0; pass < N; ++pass) {
#pragma unroll
      for (int i = pass & 1; i + 1 < N; i += 2) {
        const R a = x[i], b = x[i + 1];
        x[i] = m_min(a, b);
        x[i + 1] = m_max(a, b);
      }
    }
  }

  // P = Li (1, z, ..., z^N): the orthonormal polynomials at z
  APC_HD void values(R z, R* P) const {
#pragma unroll
    for (int k = 0; k <= N; ++k) P[k] = R(0);
    R v = R(1);
#pragma unroll
    for (int j = 0; j <= N; ++j) {
#pragma unroll
      for (int k = j; k <= N; ++k) P[k] += Li[k * (k + 1) / 2 + j] * v;
      v *= z;
    }
  }

  // q = Li^T P: power-basis coefficients of K(., z)
  APC_HD void coeffs(const R* P, R* q) const {
#pragma unroll
    for (int j = 0; j <= N; ++j) {
      R s = R(0);
#pragma unroll
      for (int k = j; k <= N; ++k) s += Li[k * (k + 1) / 2 + j] * P[k];
      q[j] = s;
    }
  }

  // K(x, x) = |Li (1, x, ..., x^N)|^2
  APC_HD R kernel_diag(R x) const {
    R P[N + 1];
    values(x, P);
    R K = R(0);
#pragma unroll
    for (int k = 0; k <= N; ++k) K += P[k] * P[k];
    return K;
  }

  // the bound from the closed-form roots of K(., z) = q
  APC_HD R closed_tail(R z, R eta, R lam0, const R* q) const {
    R x[N];
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = R(0);
    const int nr = poly_roots<N, R>(q, x);
    int below = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) below += (i < nr && x[i] < z) ? 1 : 0;
    const bool use_below = 2 * below <= nr;  // sum over the side with fewer nodes
    R S = R(0);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      if (i < nr && ((x[i] < z) == use_below) && m_abs(x[i]) < Num<R>::far) S += m_rcp(kernel_diag(x[i]));
    }
    // a node at infinity (nr < N) carries no weight, so the finite weights still sum to 1
    return use_below ? eta * lam0 + S : R(1) - (R(1) - eta) * lam0 - S;
  }

  // Fraction of the absorbance in front of warped depth z.
  APC_HD R frac_before(R z, R eta) const {
    if (mode == 1) {
      if (m_abs(z1 - z) <= Num<R>::same_depth) return eta;
      return z1 < z ? R(1) : R(0);
    }
    R P[N + 1];
    values(z, P);
    R K0 = R(0);
#pragma unroll
    for (int k = 0; k <= N; ++k) K0 += P[k] * P[k];
    const R lam0 = m_rcp(K0);
    if (z < xlo) return eta * lam0;                  // no node in front of z
    if (z > xhi) return R(1) - (R(1) - eta) * lam0;  // every other node in front of z
    R q[N + 1];
    coeffs(P, q);
    return closed_tail(z, eta, lam0, q);
  }

  // ---- gap tables (see the header comment); zs = the sorted zeros

  // For z in gap k (zs[k-1] < z < zs[k], 1 <= k <= N-1) the nodes on the side
  // of z with fewer of them: gaps 0..k-1 when 2k <= N, else gaps k+1..N.
  APC_HD static int side_count(int k) { return 2 * k <= N ? k : N - k; }
  APC_HD static int side_gap(int k, int c) { return 2 * k <= N ? c : k + 1 + c; }

  // regularised position of root r of gap j, for z in gap (lo, hi) with
  // sz = (z - lo) / (hi - z): finite and smooth in z up to both gap ends
  // (reciprocal estimates: the value only seeds a later Newton iteration)
  template <class Z>
  APC_HD static R to_table(const Z& zs, int j, R r, R sz) {
    if (j == 0) return (r - zs[0]) * sz;
    if (j == N) return (r - zs[N - 1]) * m_rcp_est(sz);
    const R a = pick<N>(zs, j - 1), b = pick<N>(zs, j);
    const R fr = (r - a) * m_rcp_est(b - a);
    return fr * m_rcp_est((R(1) - fr) * sz);
  }
  template <class Z>
  APC_HD static R from_table(const Z& zs, int j, R v, R sz, R isz) {
    if (j == 0) return zs[0] + v * isz;
    if (j == N) return zs[N - 1] + v * sz;
    const R a = pick<N>(zs, j - 1), b = pick<N>(zs, j);
    const R e = v * sz;
    return a + (b - a) * e * m_rcp_est(R(1) + e);  // a Newton start: the estimate suffices
  }

  // Table entries of node l (0 <= l < NODES): gap k = l / NI + 1, depth
  // zs[k-1] + (l % NI + 1/2) * (zs[k] - zs[k-1]) / NI.  Entries that cannot be
  // formed are +inf, which makes every sample that would use them fall back.
  template <class Z, class Tab>
  APC_HD void gap_node(const Z& zs, int l, Tab& tab) const {
    constexpr int NI = Gaps<N>::NI, NC = Gaps<N>::NC;
    const int k = l / NI + 1, i = l - (k - 1) * NI;
    const R lo = pick<N>(zs, k - 1), hi = pick<N>(zs, k);
    const R z = lo + (R(i) + R(0.5)) * (hi - lo) / R(NI);
    const R sz = (z - lo) / (hi - z);
    R P[N + 1], q[N + 1], x[N];
    values(z, P);
    coeffs(P, q);
#pragma unroll
    for (int t = 0; t < N; ++t) x[t] = R(0);
    const int nr = poly_roots<N, R, 1>(q, x);  // table entries only start Newton iterations
    sort_up(x);
    bool ok = nr == N && pick_reg<N>(x, k - 1) < z && pick_reg<N>(x, k) > z;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      R v = R(HUGE_VAL);
      if (ok && c < side_count(k)) {
        const int j = side_gap(k, c);
        const R r = pick_reg<N>(x, j < k ? j : j - 1);
        const bool in_gap = (j == 0 || r > pick<N>(zs, j - 1)) && (j == N || r < pick<N>(zs, j));
        if (in_gap) v = to_table(zs, j, r, sz);
      }
      tab.at(l, c) = v;
    }
  }

  // frac_before with the roots from the pixel's gap table.  Returns false
  // (F unset) when a root did not converge: the caller then takes
  // frac_before, the closed forms, for this sample.
  template <class Z, class Tab>
  APC_HD bool frac_before_tab(R z, R eta, const Z& zs, const Tab& tab, R& F) const {
    constexpr int NI = Gaps<N>::NI, NC = Gaps<N>::NC;
    R P[N + 1];
    values(z, P);
    R K0 = R(0);
#pragma unroll
    for (int k = 0; k <= N; ++k) K0 += P[k] * P[k];
    const R lam0 = m_rcp(K0);
    if (z < xlo) {
      F = eta * lam0;
      return true;
    }
    if (z > xhi) {
      F = R(1) - (R(1) - eta) * lam0;
      return true;
    }
    R q[N + 1];
    coeffs(P, q);
    int k = 0;
#pragma unroll
    for (int t = 0; t < N; ++t) k += zs[t] < z ? 1 : 0;
    bool ok = k >= 1 && k <= N - 1;
    const int kk = ok ? k : 1;
    const R lo = pick<N>(zs, kk - 1), hi = pick<N>(zs, kk);
    // the interpolation coordinates only shape the Newton start: reciprocal estimates suffice
    const R sz = (z - lo) * m_rcp_est(hi - z), isz = (hi - z) * m_rcp_est(z - lo);
    const R u = (z - lo) * R(NI) * m_rcp_est(hi - lo) - R(0.5);
    int i = int(floor(u + R(0.5)));
    i = i < 1 ? 1 : (i > NI - 2 ? NI - 2 : i);
    const R w = u - R(i);
    const int node = (kk - 1) * NI + i;
    const int nn = side_count(kk);
    R S = R(0);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (c < nn) {
        const int j = side_gap(kk, c);
        const R v0 = tab.at(node - 1, c), v1 = tab.at(node, c), v2 = tab.at(node + 1, c);
        const R v = v1 + R(0.5) * w * (v2 - v0) + R(0.5) * w * w * (v2 - R(2) * v1 + v0);
        R x = from_table(zs, j, v, sz, isz);
        R d = R(0);
#pragma unroll
        for (int it = 0; it < 4; ++it) {
          R p = q[N], dp = R(0);
#pragma unroll
          for (int t = N - 1; t >= 0; --t) {
            dp = dp * x + p;
            p = p * x + q[t];
          }
          d = p * m_rcp_est(dp);
          x -= d;
        }
        const R blo = j == 0 ? -R(HUGE_VAL) : pick<N>(zs, j - 1);
        const R bhi = j == N ? R(HUGE_VAL) : pick<N>(zs, j);
        const R lam = m_rcp(kernel_diag(x));
        const R ad = m_abs(d);
        // converged: a small last step, or (outer gaps, where K grows away
        // from the zeros) a weight too small for the step to matter -- from an
        // iterate that has settled (a step small against its distance to the
        // gap's edge; one running off to infinity has a tiny weight too)
        const R edge = j == 0 ? bhi : blo;
        const bool conv = ad <= R(1e-7) * m_max(R(1), m_abs(x)) ||
                          ((j == 0 || j == N) && lam * ad <= R(1e-12) * m_abs(x - edge) &&
                           ad <= R(1e-3) * m_abs(x - edge));
        ok = ok && x > blo && x < bhi && conv;
        S += lam;
      }
    }
    F = 2 * kk <= N ? eta * lam0 + S : R(1) - (R(1) - eta) * lam0 - S;
    return ok;
  }

  // ---- continuation along one ray (the fused re-walk of stage two)
  //
  // Consecutive samples of a ray lie close in depth, and inside one gap the
  // roots a sample needs move smoothly with z -- except that the outer roots
  // run to infinity like 1 / (distance to one gap end).  Cont therefore holds
  // each root in the table's regularised coordinate (to_table), which stays
  // smooth up to both gap ends, and the previous sample's value, mapped back
  // with this sample's gap coordinate, is the Newton start.  Cont also holds
  // the gap of the last sample whose roots were found (-1: none).  A sample in
  // another gap (or after a failure) takes its starts from the closed forms.
  // Either way the roots must converge inside their gaps (the table path's
  // test), else the sample takes the closed-form bound, so the start changes
  // the cost of a sample but not its result beyond rounding.
  static constexpr int CONT_STEPS = 4;  // steps from a continued (or closed-form) start: 3 Newton, 1 chord
  struct Cont {
    int k;
    R v[Gaps<N>::NC > 0 ? Gaps<N>::NC : 1];  // regularised roots (to_table) of gap k
  };

  // Fraction of the absorbance in front of z; `how` says how the roots were
  // found: 0 none needed, 1 Newton from the previous sample's roots, 2 the
  // closed forms ran (a new gap, or no convergence).  zs: the sorted zeros.
  template <class Z>
  APC_HD R frac_before_cont(R z, R eta, const Z& zs, Cont& c, int& how) const {
    static_assert(N == 3 || N == 4, "the continuation serves m = 6 and m = 8");
    constexpr int NC = Gaps<N>::NC;
    bool closed = false;
    how = 0;
    if (mode == 1) {
      if (m_abs(z1 - z) <= Num<R>::same_depth) return eta;
      return z1 < z ? R(1) : R(0);
    }
    R P[N + 1];
    values(z, P);
    R K0 = R(0);
#pragma unroll
    for (int k = 0; k <= N; ++k) K0 += P[k] * P[k];
    const R lam0 = m_rcp1(K0);
    if (z < xlo) return eta * lam0;
    if (z > xhi) return R(1) - (R(1) - eta) * lam0;
    R q[N + 1];
    coeffs(P, q);
    int k = 0;
#pragma unroll
    for (int t = 0; t < N; ++t) k += zs[t] < z ? 1 : 0;
    bool ok = k >= 1 && k <= N - 1;
    const int kk = ok ? k : 1;
    // For N <= 4 the nodes on the fewer side of gap kk (side_gap) are the one
    // of gap 0 (left: 2 kk <= N) or of gap N (right), and for N = 4, kk = 2
    // also the one of gap 1 = (zs[0], zs[1]).  So root slot 0 always lies in
    // an outer gap and slot 1 in gap 1, and every zero is read at a constant
    // index (a run-time index costs a select over all N of them).
    const bool left = 2 * kk <= N;
    const bool two = N == 4 && kk == 2;  // slot 1 in use
    R lo = zs[0], hi = zs[1];            // the gap of z: (zs[kk - 1], zs[kk])
#pragma unroll
    for (int t = 2; t < N; ++t) {
      lo = kk == t ? zs[t - 1] : lo;
      hi = kk == t ? zs[t] : hi;
    }
    const R base = left ? zs[0] : zs[N - 1];  // slot 0: the finite end of its gap
    const R sz = (z - lo) * m_rcp_est(hi - z);  // the gap coordinate only maps Newton starts
    R x[NC];
    if (ok && kk == c.k) {  // from_table of each slot's root
      const R isz = (hi - z) * m_rcp_est(z - lo);  // the start needs no more
      x[0] = base + c.v[0] * (left ? isz : sz);
      if constexpr (NC > 1) {
        const R e = c.v[1] * sz;
        x[1] = two ? zs[0] + (zs[1] - zs[0]) * e * m_rcp_est(R(1) + e) : R(0);
      }
    } else {  // starts from the closed forms, sorted: gap j's root is r[j] below kk, r[j - 1] above
      closed = true;
      R r[N];
#pragma unroll
      for (int t = 0; t < N; ++t) r[t] = R(0);
      const int nr = poly_roots<N, R, 1>(q, r);
      sort_up(r);
      ok = ok && nr == N;
      x[0] = left ? r[0] : r[N - 1];
      if constexpr (NC > 1) x[1] = two ? r[1] : R(0);
    }
    R S = R(0);
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) {
      if (cc == 0 || two) {
        R xi = x[cc], d = R(0), rd = R(0);
#pragma unroll
        for (int it = 0; it < CONT_STEPS; ++it) {
          R p = q[N], dp = R(0);
          if (it < CONT_STEPS - 1) {  // Newton steps
#pragma unroll
            for (int t = N - 1; t >= 0; --t) {
              dp = dp * xi + p;
              p = p * xi + q[t];
            }
            rd = m_rcp_est(dp);
          } else {  // the last step keeps the previous slope
#pragma unroll
            for (int t = N - 1; t >= 0; --t) p = p * xi + q[t];
          }
          d = p * rd;
          xi -= d;
        }
        const R blo = cc == 0 ? (left ? -R(HUGE_VAL) : zs[N - 1]) : zs[0];
        const R bhi = cc == 0 ? (left ? zs[0] : R(HUGE_VAL)) : zs[1];
        const R lam = m_rcp1(kernel_diag(xi));
        const R ad = m_abs(d);
        // converged: a small last step, or (outer gaps, where K grows away
        // from the zeros) a weight too small for the step to matter -- from an
        // iterate that has settled against its distance to the gap's end
        const bool conv = ad <= R(1e-7) * m_max(R(1), m_abs(xi)) ||
                          (cc == 0 && lam * ad <= R(1e-12) * m_abs(xi - base) &&
                           ad <= R(1e-3) * m_abs(xi - base));
        ok = ok && xi > blo && xi < bhi && conv;
        x[cc] = xi;
        S += lam;
      }
    }
    if (!ok) {
      c.k = -1;
      how = 2;
      return closed_tail(z, eta, lam0, q);
    }
    how = closed ? 2 : 1;
    c.k = kk;
    c.v[0] = (x[0] - base) * (left ? sz : m_rcp_est(sz));  // to_table of slot 0
    if constexpr (NC > 1) {
      const R fr = (x[1] - zs[0]) * m_rcp_est(zs[1] - zs[0]);
      c.v[1] = two ? fr * m_rcp_est((R(1) - fr) * sz) : R(0);
    }
    return left ? eta * lam0 + S : R(1) - (R(1) - eta) * lam0 - S;
  }

};

}  // namespace apcm
