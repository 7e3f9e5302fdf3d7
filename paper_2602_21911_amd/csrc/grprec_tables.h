// grprec_tables.h -- compile-time constants of the space-time predictor and of
// the reconstruction's nodal evaluation, per polynomial degree M.
//
// Nodes g_a: the (M+1)-point Gauss-Legendre points on [0,1] (closed forms).
// Lagrange basis l_a on these nodes; D[a][k] = l_k'(g_a); the time matrix of
// the space-time weak form K[b][l] = l_b(1) l_l(1) - int_0^1 l_b' l_l, which
// Gauss-Legendre at the nodes integrates exactly: l_b(1) l_l(1) - w_l l_b'(g_l);
// KW = K^{-1} diag(w).  K itself is kept for the implicit source term, whose
// time matrix is K + z diag(w) with z = kappa dt.  Everything is evaluated by
// the compiler, so the kernels see the numbers as immediate operands.
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
  double K[N][N];    // time matrix of the weak form
  double KW[N][N];
  double KWs[N];     // row sums of KW (the time solve of a time-constant argument)
  double l0[N], l1[N];
  double phi[N][4];  // xi, xi^2 - 1/12, xi^3, xi^4 - 1/80 at xi = g_a - 1/2
  // D split by the nodes' symmetry about 1/2, D[N-1-a][N-1-k] = -D[a][k]
  // (H = N/2): for a, k < H, De[a][k] = (D[a][k] + D[a][N-1-k]) / 2 acts on
  // the even part f_k + f_{N-1-k} and Do[a][k] = (D[a][k] - D[a][N-1-k]) / 2
  // on the odd part f_k - f_{N-1-k}; for odd N, Dm[a] = D[a][H] and the
  // middle row Dc[k] = D[H][k] (odd, so D[H][H] = 0).
  double De[N / 2][N / 2], Do[N / 2][N / 2], Dm[N / 2], Dc[N / 2];
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
      P.K[b][l] = K[b][l];
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
  for (int b = 0; b < N; ++b) {
    P.KWs[b] = 0.0;
    for (int l = 0; l < N; ++l) P.KWs[b] += P.KW[b][l];
  }
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
  for (int a = 0; a < N / 2; ++a) {
    for (int k = 0; k < N / 2; ++k) {
      P.De[a][k] = 0.5 * (P.D[a][k] + P.D[a][N - 1 - k]);
      P.Do[a][k] = 0.5 * (P.D[a][k] - P.D[a][N - 1 - k]);
      P.Dc[k] = P.D[N / 2][k];
    }
    P.Dm[a] = P.D[a][N / 2];
  }
  return P;
}

// ---------------------------------------------------------------- GRPrecNL
// Candidate polynomials of the nonlinear reconstruction (Sec. 3.3-3.4) in the
// zero-mean basis phi_1..phi_M of cell i (xi in [-1/2, 1/2]):
//   p = q_i + sum_j a_j phi_j,  a = A (d_sel - q_i),
// where d_sel are the data each candidate interpolates besides the mean of
// cell i, indexed 0 = mean of cell i-1, 2 = mean of cell i+1, 3 = value at
// xi = -1/2, 4 = at +1/2, 5 = at -3/2, 6 = at +3/2:
//   degree 1: left {3},          right {4}
//   degree 2: left {0, 4},       right {2, 3}
//   degree 3: left {0, 2, 3},    right {0, 2, 4}
//   degree 4: left {0, 2, 3, 5}, right {0, 2, 4, 6}.
// The oscillation indicator of a candidate is dx * a^T Gm a with
// Gm[j][k] = sum_l int_{-1/2}^{1/2} phi_j^(l) phi_k^(l) dxi.
constexpr double phi_at(int j, double x) {  // phi_{j+1}(x)
  const double x2 = x * x;
  return j == 0 ? x : j == 1 ? x2 - 1.0 / 12.0 : j == 2 ? x2 * x : x2 * x2 - 1.0 / 80.0;
}
constexpr double phi_prim(int j, double x) {  // an antiderivative of phi_{j+1}
  const double x2 = x * x;
  return j == 0 ? 0.5 * x2
       : j == 1 ? x2 * x / 3.0 - x / 12.0
       : j == 2 ? 0.25 * x2 * x2
                : 0.2 * x2 * x2 * x - x / 80.0;
}
constexpr double nl_functional(int cond, int j) {
  switch (cond) {
    case 0: return phi_prim(j, -0.5) - phi_prim(j, -1.5);  // mean over a unit cell
    case 2: return phi_prim(j, 1.5) - phi_prim(j, 0.5);
    case 3: return phi_at(j, -0.5);
    case 4: return phi_at(j, 0.5);
    case 5: return phi_at(j, -1.5);
    default: return phi_at(j, 1.5);
  }
}
constexpr double cfact(int n, int l) {  // n! / (n-l)!
  double r = 1.0;
  for (int t = 0; t < l; ++t) r *= (double)(n - t);
  return r;
}
constexpr double mono_int(int p) {  // int_{-1/2}^{1/2} xi^p dxi
  if (p % 2) return 0.0;
  double h = 1.0;
  for (int t = 0; t <= p; ++t) h *= 0.5;
  return 2.0 * h / (p + 1.0);
}

template <int M>
struct NLTab {
  int sel[2][M];        // [left/right][condition]
  double A[2][M][M];    // a = A (d_sel - q_i)
  double Gm[M][M];
};

template <int M>
constexpr NLTab<M> nl_tables() {
  NLTab<M> T{};
  const int sets[4][2][4] = {{{3}, {4}}, {{0, 4}, {2, 3}}, {{0, 2, 3}, {0, 2, 4}},
                             {{0, 2, 3, 5}, {0, 2, 4, 6}}};
  for (int side = 0; side < 2; ++side) {
    double K[M][2 * M] = {};
    for (int r = 0; r < M; ++r) {
      T.sel[side][r] = sets[M - 1][side][r];
      for (int j = 0; j < M; ++j) K[r][j] = nl_functional(T.sel[side][r], j);
      K[r][M + r] = 1.0;
    }
    for (int col = 0; col < M; ++col) {  // Gauss-Jordan with partial pivoting
      int piv = col;
      for (int r = col + 1; r < M; ++r)
        if (cabs(K[r][col]) > cabs(K[piv][col])) piv = r;
      for (int k = 0; k < 2 * M; ++k) {
        double t = K[col][k];
        K[col][k] = K[piv][k];
        K[piv][k] = t;
      }
      const double d = K[col][col];
      for (int k = 0; k < 2 * M; ++k) K[col][k] /= d;
      for (int r = 0; r < M; ++r) {
        if (r == col) continue;
        const double f = K[r][col];
        for (int k = 0; k < 2 * M; ++k) K[r][k] -= f * K[col][k];
      }
    }
    for (int j = 0; j < M; ++j)
      for (int r = 0; r < M; ++r) T.A[side][j][r] = K[j][M + r];
  }
  // phi_j^(l) = (j+1)!/(j+1-l)! xi^(j+1-l) for l >= 1 (constants drop out)
  for (int j = 0; j < M; ++j)
    for (int k = 0; k < M; ++k) {
      double g = 0.0;
      for (int l = 1; l <= (j < k ? j : k) + 1; ++l)
        g += cfact(j + 1, l) * cfact(k + 1, l) * mono_int(j + k + 2 - 2 * l);
      T.Gm[j][k] = g;
    }
  return T;
}

}  // namespace tab
}  // namespace grp
