// Host build of the library's moment-bound header, for CPU tests that compare
// it with the FP64 oracle.  Test infrastructure only.
#include "../paper_2501_12581_amd/csrc/apc_mboit.h"

template <int N, class R>
static double run(const double* b, double alpha, const double* bias, double eta, double zf, int* floored) {
  R bb[2 * N + 1], bs[2 * N];
  for (int j = 0; j <= 2 * N; ++j) bb[j] = R(b[j]);
  for (int j = 0; j < 2 * N; ++j) bs[j] = R(bias[j]);
  apcm::Bound<N, R> B;
  *floored = B.setup(bb, R(alpha), bs);
  if (B.mode == 0) return 0.0;
  return double(B.frac_before(R(zf), R(eta)));
}

extern "C" double shim_bound(const double* b, int m, double alpha, const double* bias, double eta, double zf,
                             int fp64, int* floored) {
  if (fp64) {
    if (m == 4) return run<2, double>(b, alpha, bias, eta, zf, floored);
    if (m == 6) return run<3, double>(b, alpha, bias, eta, zf, floored);
    return run<4, double>(b, alpha, bias, eta, zf, floored);
  }
  if (m == 4) return run<2, float>(b, alpha, bias, eta, zf, floored);
  if (m == 6) return run<3, float>(b, alpha, bias, eta, zf, floored);
  return run<4, float>(b, alpha, bias, eta, zf, floored);
}

extern "C" int shim_roots(const double* q, int n, int fp64, double* out) {
  int k = 0;
  if (fp64) {
    double x[4];
    if (n == 2) k = apcm::kernel_roots<2, double>(q, x);
    if (n == 3) k = apcm::kernel_roots<3, double>(q, x);
    if (n == 4) k = apcm::kernel_roots<4, double>(q, x);
    for (int i = 0; i < k; ++i) out[i] = x[i];
  } else {
    float qq[5], x[4];
    for (int j = 0; j <= n; ++j) qq[j] = float(q[j]);
    if (n == 2) k = apcm::kernel_roots<2, float>(qq, x);
    if (n == 3) k = apcm::kernel_roots<3, float>(qq, x);
    if (n == 4) k = apcm::kernel_roots<4, float>(qq, x);
    for (int i = 0; i < k; ++i) out[i] = x[i];
  }
  return k;
}

// The gap-table path for one moment vector: builds the pixel's table node by
// node (as the lanes of a wavefront do), then evaluates n depths through the
// table and through the closed forms.  Returns the number of table fallbacks,
// or -1 when the pixel has no table (single-depth or no zeros).
template <int N>
static int run_table(const double* b, double alpha, const double* bias, double eta, const double* z, int n,
                     double* f_tab, double* f_closed) {
  double bb[2 * N + 1], bs[2 * N], zs[N];
  for (int j = 0; j <= 2 * N; ++j) bb[j] = b[j];
  for (int j = 0; j < 2 * N; ++j) bs[j] = bias[j];
  apcm::Bound<N, double> B;
  B.setup(bb, alpha, bs, zs);
  if (B.mode != 2 || !(B.xlo < B.xhi)) return -1;
  static apcm::TableArray<N, double> tab;
  for (int l = 0; l < apcm::Gaps<N>::NODES; ++l) B.gap_node(zs, l, tab);
  unsigned fb = 0;
  for (int i = 0; i < n; ++i) {
    f_closed[i] = B.frac_before(z[i], eta);
    if (!B.frac_before_tab(z[i], eta, zs, tab, f_tab[i])) {
      ++fb;
      f_tab[i] = f_closed[i];
    }
  }
  return int(fb);
}

extern "C" int shim_bound_table(const double* b, int m, double alpha, const double* bias, double eta,
                                const double* z, int n, double* f_tab, double* f_closed) {
  if (m == 6) return run_table<3>(b, alpha, bias, eta, z, n, f_tab, f_closed);
  if (m == 8) return run_table<4>(b, alpha, bias, eta, z, n, f_tab, f_closed);
  return -1;
}

// The continuation path of the fused re-walk for one moment vector: the
// depths z[0..n) in the order a ray's samples would meet them, each through
// frac_before_cont with the state the previous sample left, and through the
// closed forms.  Returns how many samples took the closed forms (a new gap or
// no convergence), or -1 when the pixel has no zeros.
template <int N>
static int run_cont(const double* b, double alpha, const double* bias, double eta, const double* z, int n,
                    double* f_cont, double* f_closed) {
  double bb[2 * N + 1], bs[2 * N];
  for (int j = 0; j <= 2 * N; ++j) bb[j] = b[j];
  for (int j = 0; j < 2 * N; ++j) bs[j] = bias[j];
  apcm::Bound<N, double> B;
  apcm::RegArray<N, double> zs;
  B.setup(bb, alpha, bs, zs.v);
  if (B.mode != 2 || !(B.xlo < B.xhi)) return -1;
  typename apcm::Bound<N, double>::Cont c;
  c.k = -1;
  for (auto& v : c.v) v = 0.0;
  int closed_n = 0;
  for (int i = 0; i < n; ++i) {
    int how = 0;
    f_cont[i] = B.frac_before_cont(z[i], eta, zs, c, how);
    closed_n += how == 2 ? 1 : 0;
    f_closed[i] = B.frac_before(z[i], eta);
  }
  return closed_n;
}

extern "C" int shim_bound_cont(const double* b, int m, double alpha, const double* bias, double eta,
                               const double* z, int n, double* f_cont, double* f_closed) {
  if (m == 6) return run_cont<3>(b, alpha, bias, eta, z, n, f_cont, f_closed);
  if (m == 8) return run_cont<4>(b, alpha, bias, eta, z, n, f_cont, f_closed);
  return -1;
}

// The zeros of the degree-n orthonormal polynomial of a moment vector (ascending), or 0 when the pixel has
// none; and the closed-form bound at one depth.
extern "C" int shim_zeros(const double* b, int m, double alpha, const double* bias, double* zeros) {
  double bb[9], bs[8];
  for (int j = 0; j <= m; ++j) bb[j] = b[j];
  for (int j = 0; j < m; ++j) bs[j] = bias[j];
  if (m == 6) {
    apcm::Bound<3, double> B;
    B.setup(bb, alpha, bs, zeros);
    return B.mode == 2 && B.xlo < B.xhi ? 3 : 0;
  }
  if (m == 8) {
    apcm::Bound<4, double> B;
    B.setup(bb, alpha, bs, zeros);
    return B.mode == 2 && B.xlo < B.xhi ? 4 : 0;
  }
  return 0;
}
