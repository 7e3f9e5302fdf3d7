// grprec_tables.h -- compile-time constants of the space-time predictor and of
// the reconstruction's nodal evaluation, per polynomial degree M.
//
// Nodes g_a: the (M+1)-point Gauss-Legendre points on [0,1] (closed forms).
// Lagrange basis l_a on these nodes; D[a][k] = l_k'(g_a); the time matrix of
// the space-time weak form K[b][l] = l_b(1) l_l(1) - int_0^1 l_b' l_l, which
// Gauss-Legendre at the nodes integrates exactly: l_b(1) l_l(1) - w_l l_b'(g_l);
// KW = K^{-1} diag(w).  Everything is evaluated by the compiler, so the
// kernels see the numbers as immediate operands.
#pragma once

namespace grp {
namespace tab {

constexpr double csqrt(double x) {
  if (x <= 0.0) return 0.0;
  double r = x > 1.0 ? x : 1.0;
  for (int i = 0; i < 200; ++i) {
    double n = 0.5 * (r + x / r);
    if (n == r) break;
    r = n;
  }
  return r;
}
constexpr double cabs(double x) { return x < 0.0 ? -x : x; }

template <int N>
struct Nodes {
  double x[N];
  double w[N];
};

// closed forms on [-1,1], mapped to [0,1]
template <int N>
constexpr Nodes<N> gauss_legendre() {
  Nodes<N> r{};
  double xs[5] = {0, 0, 0, 0, 0}, ws[5] = {0, 0, 0, 0, 0};
  if (N == 1) {
    xs[0] = 0.0; ws[0] = 2.0;
  } else if (N == 2) {
    const double a = 1.0 / csqrt(3.0);
    xs[0] = -a; xs[1] = a; ws[0] = ws[1] = 1.0;
  } else if (N == 3) {
    const double a = csqrt(0.6);
    xs[0] = -a; xs[1] = 0.0; xs[2] = a;
    ws[0] = ws[2] = 5.0 / 9.0; ws[1] = 8.0 / 9.0;
  } else if (N == 4) {
    const double r6 = 2.0 / 7.0 * csqrt(6.0 / 5.0);
    const double xi = csqrt(3.0 / 7.0 - r6), xo = csqrt(3.0 / 7.0 + r6);
    const double wi = (18.0 + csqrt(30.0)) / 36.0, wo = (18.0 - csqrt(30.0)) / 36.0;
    xs[0] = -xo; xs[1] = -xi; xs[2] = xi; xs[3] = xo;
    ws[0] = wo; ws[1] = wi; ws[2] = wi; ws[3] = wo;
  } else {
    const double r = 2.0 * csqrt(10.0 / 7.0);
    const double xi = csqrt(5.0 - r) / 3.0, xo = csqrt(5.0 + r) / 3.0;
    const double wi = (322.0 + 13.0 * csqrt(70.0)) / 900.0, wo = (322.0 - 13.0 * csqrt(70.0)) / 900.0;
    xs[0] = -xo; xs[1] = -xi; xs[2] = 0.0; xs[3] = xi; xs[4] = xo;
    ws[0] = wo; ws[1] = wi; ws[2] = 128.0 / 225.0; ws[3] = wi; ws[4] = wo;
  }
  for (int k = 0; k < N; ++k) {
    r.x[k] = 0.5 * (xs[k] + 1.0);
    r.w[k] = 0.5 * ws[k];
  }
  return r;
}

template <int N>
constexpr double lag(const double (&g)[N], int k, double t) {
  double v = 1.0;
  for (int j = 0; j < N; ++j)
    if (j != k) v *= (t - g[j]) / (g[k] - g[j]);
  return v;
}

template <int N>
constexpr double lag_d(const double (&g)[N], int k, double t) {
  double s = 0.0;
  for (int j = 0; j < N; ++j) {
    if (j == k) continue;
    double prod = 1.0 / (g[k] - g[j]);
    for (int l = 0; l < N; ++l)
      if (l != k && l != j) prod *= (t - g[l]) / (g[k] - g[l]);
    s += prod;
  }
  return s;
}

template <int M>
struct Predictor {
  static constexpr int N = M + 1;
  double g[N], w[N];
  double D[N][N];
  double KW[N][N];
  double l0[N], l1[N];
  double phi[N][4];  // xi, xi^2 - 1/12, xi^3, xi^4 - 1/80 at xi = g_a - 1/2
};

template <int M>
constexpr Predictor<M> predictor() {
  constexpr int N = M + 1;
  Predictor<M> P{};
  const Nodes<N> nw = gauss_legendre<N>();
  for (int a = 0; a < N; ++a) {
    P.g[a] = nw.x[a];
    P.w[a] = nw.w[a];
  }
  double K[N][2 * N] = {};
  for (int b = 0; b < N; ++b)
    for (int l = 0; l < N; ++l) {
      K[b][l] = lag<N>(P.g, b, 1.0) * lag<N>(P.g, l, 1.0) - P.w[l] * lag_d<N>(P.g, b, P.g[l]);
      K[b][N + l] = (b == l) ? 1.0 : 0.0;
    }
  for (int col = 0; col < N; ++col) {  // Gauss-Jordan with partial pivoting
    int piv = col;
    for (int r = col + 1; r < N; ++r)
      if (cabs(K[r][col]) > cabs(K[piv][col])) piv = r;
    for (int k = 0; k < 2 * N; ++k) {
      double t = K[col][k];
      K[col][k] = K[piv][k];
      K[piv][k] = t;
    }
    const double d = K[col][col];
    for (int k = 0; k < 2 * N; ++k) K[col][k] /= d;
    for (int r = 0; r < N; ++r) {
      if (r == col) continue;
      const double f = K[r][col];
      for (int k = 0; k < 2 * N; ++k) K[r][k] -= f * K[col][k];
    }
  }
  for (int b = 0; b < N; ++b)
    for (int l = 0; l < N; ++l) P.KW[b][l] = K[b][N + l] * P.w[l];
  for (int a = 0; a < N; ++a) {
    for (int k = 0; k < N; ++k) P.D[a][k] = lag_d<N>(P.g, k, P.g[a]);
    P.l0[a] = lag<N>(P.g, a, 0.0);
    P.l1[a] = lag<N>(P.g, a, 1.0);
    const double xi = P.g[a] - 0.5, x2 = xi * xi;
    P.phi[a][0] = xi;
    P.phi[a][1] = x2 - 1.0 / 12.0;
    P.phi[a][2] = x2 * xi;
    P.phi[a][3] = x2 * x2 - 1.0 / 80.0;
  }
  return P;
}

}  // namespace tab
}  // namespace grp
