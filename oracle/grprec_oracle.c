/*
 * grprec_oracle.c -- plain, slow, serial CPU reference for one time step of the
 * GRPrec finite-volume scheme (Montecinos, Toro & Mueller, "A generalized Riemann
 * problem-based compact reconstruction method for finite volume schemes").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is used by the test-suite, by the smoke
 * check and by the CPU-baseline leg of the benchmark.  The product library never
 * links, loads or calls it, and it shares no code, header or constant table with
 * the GPU library.
 *
 * Everything here is written to be checked by eye against the paper:
 *   - reconstruction: the defining conditions of Sec. 3.1 (eqs. interpleft,
 *     interpright, conservation and the two least-squares functionals) are
 *     assembled as a KKT system and solved by Gaussian elimination;
 *   - GRPrecNL (Sec. 3.3-3.4): left and right polynomials from their square
 *     condition systems, oscillation indicators by Gauss quadrature of the
 *     squared derivatives, weights of eq. omega; for the Euler equations in
 *     characteristic variables (Sec. 3.1);
 *   - the GRP_m solver is DET (Sec. 2 and Sec. 4.1): a local space-time DG
 *     predictor iterated to a fixed point, then classical Riemann problems at
 *     the time integration points of the flux integral (eq. numfluxes);
 *   - the interface datum for the next reconstruction is the Riemann solution at
 *     the interface at the end of the step, q_{i+1/2}(dt) (Sec. 3.1), from the
 *     exact solver or, for the Euler equations, optionally from the
 *     two-rarefaction approximation (Sec. 4.1);
 *   - time step from eq. (dt-FV) with S_max as in Sec. 4.1;
 *   - conservative one-step update, eq. (eq_finite_volume), optionally with the
 *     linear relaxation source S(Q) = -kappa Q: the predictor treats it
 *     implicitly (locally implicit space-time DG, Sec. 2) and the source
 *     integral of eq. (source) is the Gauss-Legendre quadrature of S over the
 *     cell's space-time polynomial.
 * The paper gives no details of the DET predictor, of the exact Euler Riemann
 * solver or of the first-step interface data; the readings used are stated at
 * each function.  Precision: IEEE double throughout.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_INVALID (-1)
#define ORC_E_NONPHYSICAL (-4)
#define ORC_E_VACUUM (-5)
#define ORC_E_NEWTON (-6)
#define ORC_E_PREDICTOR (-7)

#define MAXN 5 /* at most m+1 = 5 nodes */

typedef struct {
  int system;       /* 0 = linear advection, 1 = Euler */
  int m;            /* polynomial degree 1..4 (scheme order m+1) */
  double cfl;       /* C_CFL of eq. (dt-FV) */
  double lambda;    /* advection speed */
  double gamma;     /* ratio of specific heats */
  int bc_left;      /* 0 = periodic, 1 = transmissive */
  int bc_right;
  double newton_tol; /* relative pressure change that stops Newton */
  int newton_max;
  double picard_tol; /* predictor stop: max|change| <= tol*(1+max|q|) */
  int picard_max;
  int recon;        /* 0 = GRPrec (Sec. 3.1), 1 = GRPrecNL (Sec. 3.3-3.4) */
  double nl_lambda_c; /* GRPrecNL linear weight of the centred polynomial (1e9) */
  double nl_eps;      /* GRPrecNL epsilon (1e-14) */
  double nl_r;        /* GRPrecNL exponent r (4) */
  int datum;          /* Euler interface datum: 0 = exact Riemann solver, 1 = two-rarefaction */
  int source;         /* 0 = none, 1 = linear relaxation S(Q) = -kappa Q (every component) */
  double kappa;       /* relaxation rate of source 1, >= 0 */
} orc_cfg;

typedef struct {
  int64_t rs_calls;
  int64_t newton_iters;
  int64_t picard_iters;
  int picard_max_seen;
  int newton_max_seen;
} orc_stats;

/* ------------------------------------------------------------------ */
/* Small dense linear algebra: Gaussian elimination with partial pivoting. */

/* Solve A x = b in place (A is n x n row-major, b has nrhs columns, row-major
 * n x nrhs).  Returns 0, or -1 if a pivot vanishes. */
static int orc_gauss_solve(int n, double *A, int nrhs, double *b) {
  for (int col = 0; col < n; ++col) {
    int piv = col;
    double best = fabs(A[col * n + col]);
    for (int r = col + 1; r < n; ++r) {
      if (fabs(A[r * n + col]) > best) {
        best = fabs(A[r * n + col]);
        piv = r;
      }
    }
    if (best < 1e-300) return -1;
    if (piv != col) {
      for (int k = 0; k < n; ++k) {
        double t = A[col * n + k];
        A[col * n + k] = A[piv * n + k];
        A[piv * n + k] = t;
      }
      for (int k = 0; k < nrhs; ++k) {
        double t = b[col * nrhs + k];
        b[col * nrhs + k] = b[piv * nrhs + k];
        b[piv * nrhs + k] = t;
      }
    }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      double f = A[r * n + col] / A[col * n + col];
      if (f == 0.0) continue;
      for (int k = col; k < n; ++k) A[r * n + k] -= f * A[col * n + k];
      for (int k = 0; k < nrhs; ++k) b[r * nrhs + k] -= f * b[col * nrhs + k];
    }
  }
  for (int r = 0; r < n; ++r) {
    double d = A[r * n + r];
    for (int k = 0; k < nrhs; ++k) b[r * nrhs + k] /= d;
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Gauss-Legendre quadrature on [0,1] (used for the predictor nodes and for the
 * flux time integral of eq. numfluxes).  Roots of the Legendre polynomial P_n by
 * Newton's method on the three-term recurrence. */

static void orc_legendre(int n, double x, double *p, double *dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    *p = 1.0;
    *dp = 0.0;
    return;
  }
  for (int k = 2; k <= n; ++k) {
    double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = pk;
  }
  *p = p1;
  *dp = n * (x * p1 - p0) / (x * x - 1.0);
}

int orc_gauss_legendre(int n, double *x01, double *w01) {
  if (n < 1 || n > 16) return ORC_E_INVALID;
  for (int i = 0; i < n; ++i) {
    double x = cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      orc_legendre(n, x, &p, &dp);
      double dx = p / dp;
      x -= dx;
      if (fabs(dx) < 1e-17) break;
    }
    double p, dp;
    orc_legendre(n, x, &p, &dp);
    double w = 2.0 / ((1.0 - x * x) * dp * dp);
    /* ascending order on [0,1] */
    x01[n - 1 - i] = 0.5 * (x + 1.0);
    w01[n - 1 - i] = 0.5 * w;
  }
  return ORC_OK;
}

/* Lagrange basis on nodes g[0..n-1]: value and derivative of l_k at x. */
static double orc_lagr(int n, const double *g, int k, double x) {
  double v = 1.0;
  for (int j = 0; j < n; ++j)
    if (j != k) v *= (x - g[j]) / (g[k] - g[j]);
  return v;
}

static double orc_lagr_d(int n, const double *g, int k, double x) {
  double s = 0.0;
  for (int j = 0; j < n; ++j) {
    if (j == k) continue;
    double term = 1.0 / (g[k] - g[j]);
    for (int l = 0; l < n; ++l)
      if (l != k && l != j) term *= (x - g[l]) / (g[k] - g[l]);
    s += term;
  }
  return s;
}

/* ------------------------------------------------------------------ */
/* GRPrec reconstruction, Sec. 3.1.
 * Local coordinate xi = (x - x_i)/dx in [-1/2, 1/2]; p(xi) = sum_j c_j xi^j.
 * Data d = (q_{i-1}, q_i, q_{i+1}, V_{i-1/2}, V_{i+1/2}), where V are the GRP
 * interface states of the previous step.  The conditions are linear functionals
 * of c:
 *   mean over cell i-1 = [-3/2,-1/2], cell i = [-1/2,1/2], cell i+1 = [1/2,3/2],
 *   point values at xi = -1/2 and xi = +1/2.
 * Degree 1: cell-i mean exact (Lagrange multiplier), least squares on both
 *           interface values (first-degree functional).
 * Degree 2: cell-i mean and both interface values exact.
 * Degree 3: cell-i mean exact, least squares with unit weights on the means of
 *           cells i-1 and i+1 and both interface values (third-degree functional).
 * Degree 4: means of cells i-1, i, i+1 and both interface values exact.
 * KKT system for min |A c - b|^2 subject to C c = e:
 *   [ A^T A  C^T ] [c ]   [A^T b]
 *   [ C      0   ] [mu] = [ e   ]
 */

static void orc_cond_row(int m, int which, double *row) {
  /* which: 0 = mean cell i-1, 1 = mean cell i, 2 = mean cell i+1,
   *        3 = value at -1/2, 4 = value at +1/2,
   *        5 = value at -3/2, 6 = value at +3/2 (GRPrecNL, degree 4 only) */
  static const double point[7] = {0.0, 0.0, 0.0, -0.5, 0.5, -1.5, 1.5};
  for (int j = 0; j <= m; ++j) {
    double a, b;
    switch (which) {
      case 0: a = -1.5; b = -0.5; break;
      case 1: a = -0.5; b = 0.5; break;
      case 2: a = 0.5; b = 1.5; break;
      default: a = b = 0.0; break;
    }
    if (which <= 2)
      row[j] = (pow(b, j + 1) - pow(a, j + 1)) / (j + 1.0); /* interval length 1 */
    else
      row[j] = pow(point[which], j);
  }
}

int orc_recon_matrix(int m, double *R /* (m+1) x 5, row-major */) {
  if (m < 1 || m > 4) return ORC_E_INVALID;
  int exact[5], nexact = 0, ls[5], nls = 0;
  switch (m) {
    case 1: exact[nexact++] = 1; ls[nls++] = 3; ls[nls++] = 4; break;
    case 2: exact[nexact++] = 1; exact[nexact++] = 3; exact[nexact++] = 4; break;
    case 3:
      exact[nexact++] = 1;
      ls[nls++] = 2; ls[nls++] = 0; ls[nls++] = 3; ls[nls++] = 4;
      break;
    default:
      for (int k = 0; k < 5; ++k) exact[nexact++] = k;
      break;
  }
  int nc = m + 1, n = nc + nexact;
  double K[10 * 10], rhs[10 * 5];
  memset(K, 0, sizeof(K));
  memset(rhs, 0, sizeof(rhs));
  double row[MAXN], row2[MAXN];
  /* A^T A and A^T b (b = unit data vectors, one per column of rhs) */
  for (int l = 0; l < nls; ++l) {
    orc_cond_row(m, ls[l], row);
    for (int r = 0; r < nc; ++r) {
      for (int c = 0; c < nc; ++c) K[r * n + c] += row[r] * row[c];
      rhs[r * 5 + ls[l]] += row[r];
    }
  }
  for (int e = 0; e < nexact; ++e) {
    orc_cond_row(m, exact[e], row2);
    for (int c = 0; c < nc; ++c) {
      K[(nc + e) * n + c] = row2[c];
      K[c * n + (nc + e)] = row2[c];
    }
    rhs[(nc + e) * 5 + exact[e]] = 1.0;
  }
  if (orc_gauss_solve(n, K, 5, rhs) != 0) return ORC_E_INVALID;
  for (int r = 0; r < nc; ++r)
    for (int k = 0; k < 5; ++k) R[r * 5 + k] = rhs[r * 5 + k];
  return ORC_OK;
}

static double orc_poly(int m, const double *c, double xi) {
  double v = 0.0, x = 1.0;
  for (int j = 0; j <= m; ++j) {
    v += c[j] * x;
    x *= xi;
  }
  return v;
}

/* ------------------------------------------------------------------ */
/* GRPrecNL, Sec. 3.3-3.4: the polynomial of cell i is a convex combination of
 * a left, the centred (GRPrec) and a right polynomial of degree m, weighted by
 * oscillation indicators.  Data d = (q_{i-1}, q_i, q_{i+1}, V_{i-1/2},
 * V_{i+1/2}, V_{i-3/2}, V_{i+3/2}), indexed as in orc_cond_row.  The left and
 * right polynomials satisfy all their conditions exactly (square systems):
 *   degree 1: L = mean of i and the value at -1/2;
 *             R = mean of i and the value at +1/2;
 *   degree 2: L = means of i-1, i and the value at +1/2;
 *             R = means of i, i+1 and the value at -1/2;
 *   degree 3: L = means of i-1, i, i+1 and the value at -1/2;
 *             R = means of i-1, i, i+1 and the value at +1/2;
 *   degree 4: L = means of i-1, i, i+1 and the values at -1/2 and -3/2;
 *             R = means of i-1, i, i+1 and the values at +1/2 and +3/2
 *             (the paper's paragraph calls this polynomial "fifth degree"; it
 *             has five coefficients, so degree 4).
 * Weights: omega_k = lambda_k / (eps + OI_k)^r, beta_k = omega_k / sum omega,
 * lambda_L = lambda_R = 1; r, eps and lambda_C come from the configuration.
 * The paper prints r = 4, eps = 1e-14, lambda_C = 1e9 (eq. omega).  With
 * lambda_C = 1e9 the centred polynomial wins wherever the three indicators are
 * within a factor 1e9^(1/4) ~ 178 of each other, which on smooth data makes
 * GRPrecNL coincide with GRPrec; the paper's GRPrecNL table (Sec. 4.2.3) and
 * its square-wave remarks (Sec. 4.2.2) are reproduced with lambda_C ~ 10. */
#define ORC_NL_LAMBDA_SIDE 1.0

int orc_side_matrix(int m, int side /* 0 = left, 1 = right */, double *M /* (m+1) x 7 */) {
  static const int cond[4][2][5] = {{{1, 3}, {1, 4}},
                                    {{0, 1, 4}, {1, 2, 3}},
                                    {{0, 1, 2, 3}, {0, 1, 2, 4}},
                                    {{0, 1, 2, 3, 5}, {0, 1, 2, 4, 6}}};
  if (m < 1 || m > 4 || side < 0 || side > 1) return ORC_E_INVALID;
  int nc = m + 1;
  double A[MAXN * MAXN], rhs[MAXN * 7], row[MAXN];
  memset(rhs, 0, sizeof(rhs));
  for (int r = 0; r < nc; ++r) {
    orc_cond_row(m, cond[m - 1][side][r], row);
    for (int j = 0; j < nc; ++j) A[r * nc + j] = row[j];
    rhs[r * 7 + cond[m - 1][side][r]] = 1.0;
  }
  if (orc_gauss_solve(nc, A, 7, rhs) != 0) return ORC_E_INVALID;
  memcpy(M, rhs, sizeof(double) * nc * 7);
  return ORC_OK;
}

/* Oscillation indicator of Sec. 3.3 for p(x) = sum_j c_j ((x - x_i)/dx)^j on
 * cell i:  OI = sum_{l=1..m} integral over the cell of (d^l p/dx^l)^2 dx^(2l) dx,
 * the dx^(2l) factor as printed.  The integral is 5-point Gauss-Legendre,
 * exact here (the integrand has degree at most 6). */
static double orc_oi_q(int m, const double *c, double dx, const double *g, const double *w) {
  double oi = 0.0;
  for (int l = 1; l <= m; ++l) {
    for (int k = 0; k < 5; ++k) {
      double xi = g[k] - 0.5; /* x = x_i + xi dx */
      double d = 0.0;         /* d^l p / dx^l at x */
      for (int j = l; j <= m; ++j) {
        double f = 1.0;
        for (int t = 0; t < l; ++t) f *= (double)(j - t);
        d += c[j] * f * pow(xi, j - l) / pow(dx, l);
      }
      oi += dx * w[k] * d * d * pow(dx, 2 * l);
    }
  }
  return oi;
}

double orc_oi(int m, const double *c, double dx) {
  double g[5], w[5];
  orc_gauss_legendre(5, g, w);
  return orc_oi_q(m, c, dx, g, w);
}

/* The matrices and quadrature nodes GRPrecNL needs for one degree. */
typedef struct {
  double RC[MAXN * 5], ML[MAXN * 7], MR[MAXN * 7];
  double g5[5], w5[5];
} orc_nl;

static int orc_nl_init(int m, orc_nl *t) {
  if (orc_recon_matrix(m, t->RC) || orc_side_matrix(m, 0, t->ML) || orc_side_matrix(m, 1, t->MR))
    return ORC_E_INVALID;
  return orc_gauss_legendre(5, t->g5, t->w5);
}

/* One scalar component: coefficients of beta_L p_L + beta_C p_C + beta_R p_R
 * and the three weights. */
static void orc_nl_scalar(const orc_cfg *cf, double dx, const orc_nl *t, const double *d, double *c,
                          double *beta) {
  int m = cf->m;
  const double *RC = t->RC, *ML = t->ML, *MR = t->MR;
  double cl[MAXN], cc[MAXN], cr[MAXN];
  for (int r = 0; r <= m; ++r) {
    cl[r] = cc[r] = cr[r] = 0.0;
    for (int k = 0; k < 7; ++k) {
      cl[r] += ML[r * 7 + k] * d[k];
      cr[r] += MR[r * 7 + k] * d[k];
    }
    for (int k = 0; k < 5; ++k) cc[r] += RC[r * 5 + k] * d[k];
  }
  double wl = ORC_NL_LAMBDA_SIDE / pow(cf->nl_eps + orc_oi_q(m, cl, dx, t->g5, t->w5), cf->nl_r);
  double wc = cf->nl_lambda_c / pow(cf->nl_eps + orc_oi_q(m, cc, dx, t->g5, t->w5), cf->nl_r);
  double wr = ORC_NL_LAMBDA_SIDE / pow(cf->nl_eps + orc_oi_q(m, cr, dx, t->g5, t->w5), cf->nl_r);
  double ws = wl + wc + wr;
  double bl = wl / ws, bc = wc / ws, br = wr / ws;
  for (int r = 0; r <= m; ++r) c[r] = bl * cl[r] + bc * cc[r] + br * cr[r];
  if (beta) {
    beta[0] = bl;
    beta[1] = bc;
    beta[2] = br;
  }
}

/* ------------------------------------------------------------------ */
/* Physics (Sec. 4.2 and Sec. 4.3, eqs. Euler-gen, Euler-variables, ideal gas). */

static int orc_nvar(const orc_cfg *c) { return c->system == 0 ? 1 : 3; }

static void orc_flux(const orc_cfg *cf, const double *Q, double *F) {
  if (cf->system == 0) {
    F[0] = cf->lambda * Q[0];
    return;
  }
  double rho = Q[0], mom = Q[1], E = Q[2];
  double u = mom / rho;
  double p = (cf->gamma - 1.0) * (E - 0.5 * mom * u);
  F[0] = mom;
  F[1] = mom * u + p;
  F[2] = u * (E + p);
}

static void orc_cons_to_prim(double g, const double *Q, double *W) {
  W[0] = Q[0];
  W[1] = Q[1] / Q[0];
  W[2] = (g - 1.0) * (Q[2] - 0.5 * Q[1] * W[1]);
}

static void orc_prim_to_cons(double g, const double *W, double *Q) {
  Q[0] = W[0];
  Q[1] = W[0] * W[1];
  Q[2] = W[2] / (g - 1.0) + 0.5 * W[0] * W[1] * W[1];
}

/* Right eigenvectors of the Euler flux Jacobian at Q, as the columns of Rm
 * (row-major), for the eigenvalues u - c, u, u + c:
 *   (1, u - c, H - u c), (1, u, u^2/2), (1, u + c, H + u c),
 * H = (E + p)/rho the specific total enthalpy. */
int orc_eigvec(double g, const double *Q, double *Rm) {
  double W[3];
  orc_cons_to_prim(g, Q, W);
  if (!(W[0] > 0.0) || !(W[2] > 0.0) || !isfinite(W[1])) return ORC_E_NONPHYSICAL;
  double u = W[1], c = sqrt(g * W[2] / W[0]), H = (Q[2] + W[2]) / W[0];
  double col[3][3] = {{1.0, u - c, H - u * c}, {1.0, u, 0.5 * u * u}, {1.0, u + c, H + u * c}};
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) Rm[r * 3 + k] = col[k][r];
  return ORC_OK;
}

/* GRPrecNL polynomial of one cell.  d holds the seven data of every conserved
 * variable ([nv][7]); coef receives [nv][m+1] monomial coefficients in
 * xi = (x - x_i)/dx; beta (optional) the weights [nv][3].  For the Euler
 * equations the data are first written in characteristic variables with the
 * eigenvectors at the cell average q_i (the paper reconstructs systems in
 * characteristic variables, Sec. 3.1), each characteristic field is
 * reconstructed as a scalar, and the result is projected back; beta then
 * refers to the characteristic fields. */
static int orc_recon_nl_cell_t(const orc_cfg *cf, const orc_nl *t, double dx, const double *d,
                               double *coef, double *beta) {
  int m = cf->m;
  if (cf->system == 0) {
    orc_nl_scalar(cf, dx, t, d, coef, beta);
    return ORC_OK;
  }
  double Qbar[3] = {d[0 * 7 + 1], d[1 * 7 + 1], d[2 * 7 + 1]};
  double Rm[9], Lm[9], Rw[9];
  int rc = orc_eigvec(cf->gamma, Qbar, Rm);
  if (rc != ORC_OK) return rc;
  memcpy(Rw, Rm, sizeof(Rw));
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) Lm[r * 3 + k] = (r == k) ? 1.0 : 0.0;
  if (orc_gauss_solve(3, Rw, 3, Lm) != 0) return ORC_E_NONPHYSICAL; /* Lm = Rm^-1 */
  double w[3][7], cw[3][MAXN];
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 7; ++j) {
      w[k][j] = 0.0;
      for (int v = 0; v < 3; ++v) w[k][j] += Lm[k * 3 + v] * d[v * 7 + j];
    }
  for (int k = 0; k < 3; ++k) orc_nl_scalar(cf, dx, t, w[k], cw[k], beta ? beta + 3 * k : NULL);
  for (int v = 0; v < 3; ++v)
    for (int r = 0; r <= m; ++r) {
      coef[v * (m + 1) + r] = 0.0;
      for (int k = 0; k < 3; ++k) coef[v * (m + 1) + r] += Rm[v * 3 + k] * cw[k][r];
    }
  return ORC_OK;
}

int orc_recon_nl_cell(const orc_cfg *cf, double dx, const double *d, double *coef, double *beta) {
  orc_nl t;
  if (cf->m < 1 || cf->m > 4 || orc_nl_init(cf->m, &t)) return ORC_E_INVALID;
  return orc_recon_nl_cell_t(cf, &t, dx, d, coef, beta);
}

/* ------------------------------------------------------------------ */
/* Exact Riemann solver for the ideal-gas Euler equations, written from the
 * mathematics of the classical Riemann problem (the "classical non-linear
 * Riemann problems" that the DET interaction step solves, Sec. 2).
 *   f(p) = f_L(p) + f_R(p) + (u_R - u_L) = 0 for the star pressure,
 *   shock branch (p > p_K): f_K = (p - p_K) sqrt(A_K / (p + B_K)),
 *       A_K = 2/((g+1) rho_K), B_K = (g-1)/(g+1) p_K  (Rankine-Hugoniot),
 *   rarefaction branch (p <= p_K): f_K = 2 c_K/(g-1) ((p/p_K)^((g-1)/(2g)) - 1)
 *       (isentropic, generalised Riemann invariant).
 * Newton iteration from the guess; a non-positive iterate is replaced by half
 * the previous one; stop when 2|p_new - p|/(p_new + p) <= tol (at least one
 * iteration).  Solution sampled at x/t = 0. */

static void orc_pfun(double g, double p, double rk, double pk, double ck, double *f, double *fd) {
  if (p <= pk) {
    double pr = p / pk;
    *f = 2.0 * ck / (g - 1.0) * (pow(pr, (g - 1.0) / (2.0 * g)) - 1.0);
    *fd = 1.0 / (rk * ck) * pow(pr, -(g + 1.0) / (2.0 * g));
  } else {
    double ak = 2.0 / ((g + 1.0) * rk);
    double bk = (g - 1.0) / (g + 1.0) * pk;
    double s = sqrt(ak / (bk + p));
    *f = (p - pk) * s;
    *fd = (1.0 - 0.5 * (p - pk) / (bk + p)) * s;
  }
}

/* Pressure of the linearised (primitive-variable) Riemann solver, floored at
 * 1e-6 min(pL, pR) to keep the Newton start positive. */
double orc_pvrs_guess(double g, const double *WL, const double *WR) {
  double cl = sqrt(g * WL[2] / WL[0]), cr = sqrt(g * WR[2] / WR[0]);
  double ppv = 0.5 * (WL[2] + WR[2]) - 0.125 * (WR[1] - WL[1]) * (WL[0] + WR[0]) * (cl + cr);
  double floor_p = 1e-6 * fmin(WL[2], WR[2]);
  return ppv > floor_p ? ppv : floor_p;
}

/* Solve the Riemann problem (WL | WR) in primitive variables.  guess <= 0 means
 * use the PVRS guess.  Outputs: star pressure and velocity, the state at
 * x/t = 0 (primitive) and the number of Newton iterations. */
int orc_riemann(double g, const double *WL, const double *WR, double guess, double tol, int maxit,
                double *pstar, double *ustar, double *W0, int *iters) {
  double rl = WL[0], ul = WL[1], pl = WL[2];
  double rr = WR[0], ur = WR[1], pr = WR[2];
  if (!(rl > 0.0) || !(rr > 0.0) || !(pl > 0.0) || !(pr > 0.0)) return ORC_E_NONPHYSICAL;
  if (!isfinite(ul) || !isfinite(ur)) return ORC_E_NONPHYSICAL;
  double cl = sqrt(g * pl / rl), cr = sqrt(g * pr / rr);
  if (2.0 / (g - 1.0) * (cl + cr) <= ur - ul) return ORC_E_VACUUM;
  double p = guess > 0.0 ? guess : orc_pvrs_guess(g, WL, WR);
  int k = 0, conv = 0;
  for (k = 1; k <= maxit; ++k) {
    double fl, fld, fr, frd;
    orc_pfun(g, p, rl, pl, cl, &fl, &fld);
    orc_pfun(g, p, rr, pr, cr, &fr, &frd);
    double pn = p - (fl + fr + (ur - ul)) / (fld + frd);
    if (pn <= 0.0) pn = 0.5 * p;
    double change = 2.0 * fabs(pn - p) / (pn + p);
    p = pn;
    if (change <= tol) {
      conv = 1;
      break;
    }
  }
  if (iters) *iters = conv ? k : maxit;
  if (!conv) return ORC_E_NEWTON;
  double fl, fld, fr, frd;
  orc_pfun(g, p, rl, pl, cl, &fl, &fld);
  orc_pfun(g, p, rr, pr, cr, &fr, &frd);
  double u = 0.5 * (ul + ur) + 0.5 * (fr - fl);
  *pstar = p;
  *ustar = u;

  /* sampling at S = x/t = 0 */
  double gm1 = g - 1.0, gp1 = g + 1.0;
  if (u >= 0.0) {
    if (p <= pl) { /* left rarefaction */
      if (ul - cl >= 0.0) {
        W0[0] = rl; W0[1] = ul; W0[2] = pl;
      } else {
        double cml = cl * pow(p / pl, gm1 / (2.0 * g));
        if (u - cml < 0.0) {
          W0[0] = rl * pow(p / pl, 1.0 / g); W0[1] = u; W0[2] = p;
        } else { /* inside the fan: u - c = 0 and u + 2c/(g-1) = ul + 2cl/(g-1) */
          double c = 2.0 / gp1 * (cl + 0.5 * gm1 * ul);
          W0[0] = rl * pow(c / cl, 2.0 / gm1);
          W0[1] = c;
          W0[2] = pl * pow(c / cl, 2.0 * g / gm1);
        }
      }
    } else { /* left shock */
      double pml = p / pl;
      double sl = ul - cl * sqrt(gp1 / (2.0 * g) * pml + gm1 / (2.0 * g));
      if (sl >= 0.0) {
        W0[0] = rl; W0[1] = ul; W0[2] = pl;
      } else {
        W0[0] = rl * (pml + gm1 / gp1) / (pml * gm1 / gp1 + 1.0); W0[1] = u; W0[2] = p;
      }
    }
  } else {
    if (p > pr) { /* right shock */
      double pmr = p / pr;
      double sr = ur + cr * sqrt(gp1 / (2.0 * g) * pmr + gm1 / (2.0 * g));
      if (sr <= 0.0) {
        W0[0] = rr; W0[1] = ur; W0[2] = pr;
      } else {
        W0[0] = rr * (pmr + gm1 / gp1) / (pmr * gm1 / gp1 + 1.0); W0[1] = u; W0[2] = p;
      }
    } else { /* right rarefaction */
      if (ur + cr <= 0.0) {
        W0[0] = rr; W0[1] = ur; W0[2] = pr;
      } else {
        double cmr = cr * pow(p / pr, gm1 / (2.0 * g));
        if (u + cmr >= 0.0) {
          W0[0] = rr * pow(p / pr, 1.0 / g); W0[1] = u; W0[2] = p;
        } else { /* inside the fan: u + c = 0 and u - 2c/(g-1) = ur - 2cr/(g-1) */
          double c = 2.0 / gp1 * (cr - 0.5 * gm1 * ur);
          W0[0] = rr * pow(c / cr, 2.0 / gm1);
          W0[1] = -c;
          W0[2] = pr * pow(c / cr, 2.0 * g / gm1);
        }
      }
    }
  }
  return ORC_OK;
}

/* Two-rarefaction approximation of the Riemann problem, the solver Sec. 4.1
 * names for the Euler interface datum.  Both nonlinear waves are taken as
 * rarefactions, so across each the generalised Riemann invariant and the
 * isentrope hold (p_s, u_s: star pressure and velocity; c_sK star sound speeds):
 *   u_s + 2 c_sL/(g-1) = u_L + 2 c_L/(g-1),   c_sL = c_L (p_s / p_L)^z,
 *   u_s - 2 c_sR/(g-1) = u_R - 2 c_R/(g-1),   c_sR = c_R (p_s / p_R)^z,
 * z = (g-1)/(2 g).  Eliminating u_s gives
 *   p_s^z (c_L p_L^-z + c_R p_R^-z) = c_L + c_R - (g-1)/2 (u_R - u_L),
 * and u_s is the mean of the two invariant relations.  A non-positive
 * right-hand side means vacuum.  The solution at x/t = 0 is sampled from the
 * two-rarefaction pattern (left side when u_s >= 0). */
int orc_trrs(double g, const double *WL, const double *WR, double *pstar, double *ustar, double *W0) {
  double rl = WL[0], ul = WL[1], pl = WL[2];
  double rr = WR[0], ur = WR[1], pr = WR[2];
  if (!(rl > 0.0) || !(rr > 0.0) || !(pl > 0.0) || !(pr > 0.0)) return ORC_E_NONPHYSICAL;
  if (!isfinite(ul) || !isfinite(ur)) return ORC_E_NONPHYSICAL;
  double gm1 = g - 1.0, gp1 = g + 1.0, z = gm1 / (2.0 * g);
  double cl = sqrt(g * pl / rl), cr = sqrt(g * pr / rr);
  double num = cl + cr - 0.5 * gm1 * (ur - ul);
  if (!(num > 0.0)) return ORC_E_VACUUM;
  double p = pow(num / (cl * pow(pl, -z) + cr * pow(pr, -z)), 1.0 / z);
  double csl = cl * pow(p / pl, z), csr = cr * pow(p / pr, z);
  double u = 0.5 * (ul + ur) + ((csr - cr) - (csl - cl)) / gm1;
  *pstar = p;
  *ustar = u;
  if (u >= 0.0) {
    if (ul - cl >= 0.0) {
      W0[0] = rl; W0[1] = ul; W0[2] = pl;
    } else if (u - csl < 0.0) {
      W0[0] = rl * pow(p / pl, 1.0 / g); W0[1] = u; W0[2] = p;
    } else {
      double c = 2.0 / gp1 * (cl + 0.5 * gm1 * ul);
      W0[0] = rl * pow(c / cl, 2.0 / gm1);
      W0[1] = c;
      W0[2] = pl * pow(c / cl, 2.0 * g / gm1);
    }
  } else {
    if (ur + cr <= 0.0) {
      W0[0] = rr; W0[1] = ur; W0[2] = pr;
    } else if (u + csr >= 0.0) {
      W0[0] = rr * pow(p / pr, 1.0 / g); W0[1] = u; W0[2] = p;
    } else {
      double c = 2.0 / gp1 * (cr - 0.5 * gm1 * ur);
      W0[0] = rr * pow(c / cr, 2.0 / gm1);
      W0[1] = -c;
      W0[2] = pr * pow(c / cr, 2.0 * g / gm1);
    }
  }
  return ORC_OK;
}

/* Interface datum by the two-rarefaction solver (conserved in and out). */
static int orc_datum_trrs(const orc_cfg *cf, const double *QL, const double *QR, double *Q0) {
  double WL[3], WR[3], W0[3], ps, us;
  orc_cons_to_prim(cf->gamma, QL, WL);
  orc_cons_to_prim(cf->gamma, QR, WR);
  int rc = orc_trrs(cf->gamma, WL, WR, &ps, &us, W0);
  if (rc != ORC_OK) return rc;
  orc_prim_to_cons(cf->gamma, W0, Q0);
  return ORC_OK;
}

/* Interface interaction on conserved traces: returns the physical flux of the
 * Riemann solution at x/t = 0 and that state (conserved). */
static int orc_interact(const orc_cfg *cf, const double *QL, const double *QR, double *F, double *Q0,
                        orc_stats *st) {
  if (cf->system == 0) {
    /* exact Riemann solution of linear advection: the upwind state */
    Q0[0] = cf->lambda >= 0.0 ? QL[0] : QR[0];
    F[0] = cf->lambda * Q0[0];
    return ORC_OK;
  }
  double WL[3], WR[3], W0[3], ps, us;
  int it = 0;
  orc_cons_to_prim(cf->gamma, QL, WL);
  orc_cons_to_prim(cf->gamma, QR, WR);
  int rc = orc_riemann(cf->gamma, WL, WR, -1.0, cf->newton_tol, cf->newton_max, &ps, &us, W0, &it);
  if (st) {
    st->rs_calls++;
    st->newton_iters += it;
    if (it > st->newton_max_seen) st->newton_max_seen = it;
  }
  if (rc != ORC_OK) return rc;
  orc_prim_to_cons(cf->gamma, W0, Q0);
  orc_flux(cf, Q0, F);
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* DET predictor (local space-time DG), reading of the paper's cited solver:
 * unit cell xi in [0,1], unit time t in [0,1]; nodal tensor basis on the
 * (m+1)-point Gauss-Legendre nodes g_a in space and g_b in time; unknowns
 * q[a][b]; initial data w_a = p_i(g_a - 1/2) (the reconstruction at t^n).
 * Weak form of  dq/dt + nu dF(q)/dxi = 0  (nu = dt/dx), tested with
 * l_a(xi) l_b(t), integrated by parts in time only, upwind (initial data) at t=0,
 * flux replaced by its nodal interpolant.  With Gauss-Legendre quadrature at
 * the nodes (exact for the integrands that arise) this reads, per space node a,
 *   sum_l K[b][l] q[a][l] = l_b(0) w_a - nu w_b (D F)[a][b],
 *   K[b][l] = l_b(1) l_l(1) - int_0^1 l_b'(t) l_l(t) dt,  D[a][k] = l_k'(g_a).
 * Solved by Picard iteration from q = w (constant in time):
 *   q <- K^{-1} l(0) w_a - nu K^{-1} diag(w) (D F(q)),
 * until max|change| <= picard_tol (1 + max|q|), at most picard_max sweeps.
 * With the source S(q) = -kappa q of eq. (GRP) the weak form gains the nodal
 * source term dt w_b S(q[a][b]) on the right.  It is taken implicitly (the
 * predictor is locally implicit, Sec. 2, which is what admits stiff sources):
 * with z = kappa dt it moves to the left as z diag(w), so the same iteration
 * runs with K replaced by K_z = K + z diag(w); only the flux term is iterated. */

typedef struct {
  int n;
  double g[MAXN], w[MAXN];
  double D[MAXN][MAXN];
  double Kinv_l0[MAXN];        /* K_z^{-1} l(0) */
  double KinvW[MAXN][MAXN];    /* K_z^{-1} diag(w) */
  double l0[MAXN], l1[MAXN];   /* l_a(0), l_a(1) */
} orc_st;

/* z = kappa dt of the implicit source (0 without source). */
static int orc_st_init(int m, double z, orc_st *s) {
  int n = m + 1;
  s->n = n;
  orc_gauss_legendre(n, s->g, s->w);
  double K[MAXN * MAXN], I[MAXN * MAXN];
  for (int b = 0; b < n; ++b) {
    for (int l = 0; l < n; ++l) {
      double integral = 0.0; /* int_0^1 l_b' l_l by the n-point rule (exact, degree 2n-3) */
      for (int qn = 0; qn < n; ++qn)
        integral += s->w[qn] * orc_lagr_d(n, s->g, b, s->g[qn]) * orc_lagr(n, s->g, l, s->g[qn]);
      K[b * n + l] = orc_lagr(n, s->g, b, 1.0) * orc_lagr(n, s->g, l, 1.0) - integral;
      if (b == l) K[b * n + l] += z * s->w[b];
      I[b * n + l] = (b == l) ? 1.0 : 0.0;
    }
  }
  if (orc_gauss_solve(n, K, n, I) != 0) return ORC_E_INVALID; /* I <- K^{-1} */
  for (int a = 0; a < n; ++a) {
    s->l0[a] = orc_lagr(n, s->g, a, 0.0);
    s->l1[a] = orc_lagr(n, s->g, a, 1.0);
    for (int k = 0; k < n; ++k) s->D[a][k] = orc_lagr_d(n, s->g, k, s->g[a]);
  }
  for (int b = 0; b < n; ++b) {
    double acc = 0.0;
    for (int l = 0; l < n; ++l) {
      acc += I[b * n + l] * s->l0[l];
      s->KinvW[b][l] = I[b * n + l] * s->w[l];
    }
    s->Kinv_l0[b] = acc;
  }
  return ORC_OK;
}

/* q[v][a][b] flattened as q[(v*n + a)*n + b] */
static int orc_predict(const orc_cfg *cf, const orc_st *s, double nu, const double *w /* [nv][n] */,
                       double *q, int *iters) {
  int n = s->n, nv = orc_nvar(cf);
  double F[3 * MAXN * MAXN], G[3 * MAXN * MAXN], qn[3 * MAXN * MAXN];
  for (int v = 0; v < nv; ++v)
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) q[(v * n + a) * n + b] = w[v * n + a];
  for (int it = 1; it <= cf->picard_max; ++it) {
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        double Q[3], FF[3];
        for (int v = 0; v < nv; ++v) Q[v] = q[(v * n + a) * n + b];
        orc_flux(cf, Q, FF);
        for (int v = 0; v < nv; ++v) F[(v * n + a) * n + b] = FF[v];
      }
    for (int v = 0; v < nv; ++v)
      for (int a = 0; a < n; ++a)
        for (int l = 0; l < n; ++l) {
          double acc = 0.0;
          for (int k = 0; k < n; ++k) acc += s->D[a][k] * F[(v * n + k) * n + l];
          G[(v * n + a) * n + l] = acc;
        }
    double diff = 0.0, nrm = 0.0;
    for (int v = 0; v < nv; ++v)
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
          double acc = 0.0;
          for (int l = 0; l < n; ++l) acc += s->KinvW[b][l] * G[(v * n + a) * n + l];
          double val = s->Kinv_l0[b] * w[v * n + a] - nu * acc;
          qn[(v * n + a) * n + b] = val;
          double d = fabs(val - q[(v * n + a) * n + b]);
          if (d > diff || isnan(d)) diff = d;
          if (fabs(val) > nrm) nrm = fabs(val);
        }
    memcpy(q, qn, sizeof(double) * nv * n * n);
    if (isnan(diff) || isnan(nrm)) break;
    if (diff <= cf->picard_tol * (1.0 + nrm)) {
      if (iters) *iters = it;
      return ORC_OK;
    }
  }
  if (iters) *iters = cf->picard_max;
  return ORC_E_PREDICTOR;
}

/* Traces of the space-time polynomial at xi = 0 (left) and xi = 1 (right), at
 * the m+1 time nodes and at t = 1: T[v][b], b = 0..n (n+1 times). */
static void orc_traces(const orc_cfg *cf, const orc_st *s, const double *q, double *TL, double *TR) {
  int n = s->n, nv = orc_nvar(cf);
  for (int v = 0; v < nv; ++v) {
    for (int b = 0; b < n; ++b) {
      double l = 0.0, r = 0.0;
      for (int a = 0; a < n; ++a) {
        l += s->l0[a] * q[(v * n + a) * n + b];
        r += s->l1[a] * q[(v * n + a) * n + b];
      }
      TL[v * (n + 1) + b] = l;
      TR[v * (n + 1) + b] = r;
    }
    double l = 0.0, r = 0.0;
    for (int a = 0; a < n; ++a) {
      double qa1 = 0.0; /* q_a(t = 1) */
      for (int b = 0; b < n; ++b) qa1 += s->l1[b] * q[(v * n + a) * n + b];
      l += s->l0[a] * qa1;
      r += s->l1[a] * qa1;
    }
    TL[v * (n + 1) + n] = l;
    TR[v * (n + 1) + n] = r;
  }
}

/* ------------------------------------------------------------------ */
/* Public pin helpers. */

int orc_predictor_cell(const orc_cfg *cf, double nu, const double *w, double *q, double *TL, double *TR,
                       int *iters) {
  orc_st s;
  if (cf->m < 1 || cf->m > 4) return ORC_E_INVALID;
  orc_st_init(cf->m, 0.0, &s);
  int rc = orc_predict(cf, &s, nu, w, q, iters);
  orc_traces(cf, &s, q, TL, TR);
  return rc;
}

/* Predictor matrices, exposed so that a test can check the weak form
 * independently. */
int orc_predictor_matrices(int m, double *g, double *w, double *D, double *Kinv_l0, double *KinvW) {
  orc_st s;
  if (m < 1 || m > 4) return ORC_E_INVALID;
  orc_st_init(m, 0.0, &s);
  int n = m + 1;
  for (int a = 0; a < n; ++a) {
    g[a] = s.g[a];
    w[a] = s.w[a];
    Kinv_l0[a] = s.Kinv_l0[a];
    for (int k = 0; k < n; ++k) {
      D[a * n + k] = s.D[a][k];
      KinvW[a * n + k] = s.KinvW[a][k];
    }
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* One time step of one domain (segment), eqs. (dt-FV) and (eq_finite_volume).
 * q:  [nv][n] cell averages at t^n;  v: [nv][n+1] interface states from the
 * previous step (index k is x_{k-1/2}; for periodic domains v[0] and v[n] are
 * the same interface).  Ghosts: periodic wrap, or, at a transmissive end, a
 * ghost cell holding the end cell's average (zero-gradient extrapolation): it
 * enters the degree >= 3 reconstructions as a neighbour average and the
 * boundary Riemann problems as constant data. */

double orc_smax(const orc_cfg *cf, int n, const double *q) {
  if (cf->system == 0) return fabs(cf->lambda);
  double s = 0.0;
  for (int i = 0; i < n; ++i) {
    double Q[3] = {q[i], q[n + i], q[2 * n + i]}, W[3];
    orc_cons_to_prim(cf->gamma, Q, W);
    double c = sqrt(cf->gamma * W[2] / W[0]);
    double si = fabs(W[1]) + c;
    if (isnan(si) || isnan(s)) {
      s = NAN; /* a non-physical cell has no real wave speeds: keep the NaN */
    } else if (si > s) {
      s = si;
    }
  }
  return s;
}

/* dt rule: dt = cfl dx / S; if that reaches t_end the step ends exactly at t_end. */
static void orc_dt(double cfl, double dx, double S, double t, double t_end, double *dt, double *t_next) {
  double d = cfl * dx / S;
  if (d >= t_end - t) {
    *dt = t_end - t;
    *t_next = t_end;
  } else {
    *dt = d;
    *t_next = t + d;
  }
}

static int orc_check_state(const orc_cfg *cf, const double *Q) {
  if (cf->system == 0) return isfinite(Q[0]) ? ORC_OK : ORC_E_NONPHYSICAL;
  if (!isfinite(Q[0]) || !isfinite(Q[1]) || !isfinite(Q[2])) return ORC_E_NONPHYSICAL;
  double W[3];
  orc_cons_to_prim(cf->gamma, Q, W);
  if (!(W[0] > 0.0) || !(W[2] > 0.0)) return ORC_E_NONPHYSICAL;
  return ORC_OK;
}

int orc_segment_step(const orc_cfg *cf, int n, double dx, const double *q, const double *v, double t,
                     double t_end, double *q_out, double *v_out, double *dt_out, double *t_out,
                     orc_stats *st) {
  if (n < 1 || cf->m < 1 || cf->m > 4 || cf->recon < 0 || cf->recon > 1) return ORC_E_INVALID;
  if (cf->datum < 0 || cf->datum > 1) return ORC_E_INVALID;
  if (cf->source < 0 || cf->source > 1 || !(cf->kappa >= 0.0)) return ORC_E_INVALID;
  int m = cf->m, nv = orc_nvar(cf), nn = m + 1;
  int per = (cf->bc_left == 0);
  double R[5 * 5];
  orc_recon_matrix(m, R);
  orc_nl nlt;
  if (cf->recon == 1) orc_nl_init(m, &nlt);

  double S = orc_smax(cf, n, q);
  if (!(S > 0.0) || !isfinite(S)) return ORC_E_NONPHYSICAL;
  double dt, tn;
  orc_dt(cf->cfl, dx, S, t, t_end, &dt, &tn);
  double nu = dt / dx;
  /* predictor matrices with the implicit source of this step, z = kappa dt */
  const double kap = cf->source == 1 ? cf->kappa : 0.0;
  orc_st s;
  orc_st_init(m, kap * dt, &s);

  int ntr = nv * (nn + 1);
  double *TL = (double *)malloc(sizeof(double) * ntr * n);
  double *TR = (double *)malloc(sizeof(double) * ntr * n);
  double *Fb = (double *)malloc(sizeof(double) * nv * (n + 1));
  double *Si = (double *)malloc(sizeof(double) * nv * n); /* S^n_i of eq. (source) */
  int rc = ORC_OK;

  for (int i = 0; i < n && rc == ORC_OK; ++i) {
    int im = i - 1, ip = i + 1;
    if (per) {
      im = (im + n) % n;
      ip = ip % n;
    } else {
      if (im < 0) im = 0;
      if (ip > n - 1) ip = n - 1;
    }
    double w[3 * MAXN], qh[3 * MAXN * MAXN];
    /* the seven data of each variable; V_{i-3/2} and V_{i+3/2} are read by
     * GRPrecNL at degree 4 only.  Beyond a transmissive end they belong to the
     * ghost cell, a constant state equal to the end average. */
    double d[3 * 7], coef[3 * MAXN];
    for (int vv = 0; vv < nv; ++vv) {
      const double *qv = q + vv * n, *vvv = v + vv * (n + 1);
      double vm, vp;
      if (per) {
        vm = vvv[(i - 1 + n) % n];
        vp = vvv[(i + 2) % n];
      } else {
        vm = (i >= 1) ? vvv[i - 1] : qv[0];
        vp = (i + 2 <= n) ? vvv[i + 2] : qv[n - 1];
      }
      double dd[7] = {qv[im], qv[i], qv[ip], vvv[i], vvv[i + 1], vm, vp};
      memcpy(d + vv * 7, dd, sizeof(dd));
    }
    if (cf->recon == 1) {
      rc = orc_recon_nl_cell_t(cf, &nlt, dx, d, coef, NULL);
      if (rc != ORC_OK) break;
    } else {
      for (int vv = 0; vv < nv; ++vv)
        for (int r = 0; r <= m; ++r) {
          double acc = 0.0;
          for (int k = 0; k < 5; ++k) acc += R[r * 5 + k] * d[vv * 7 + k];
          coef[vv * (m + 1) + r] = acc;
        }
    }
    for (int vv = 0; vv < nv; ++vv)
      for (int a = 0; a < nn; ++a) w[vv * nn + a] = orc_poly(m, coef + vv * (m + 1), s.g[a] - 0.5);
    int it = 0;
    rc = orc_predict(cf, &s, nu, w, qh, &it);
    if (st) {
      st->picard_iters += it;
      if (it > st->picard_max_seen) st->picard_max_seen = it;
    }
    orc_traces(cf, &s, qh, TL + (size_t)ntr * i, TR + (size_t)ntr * i);
    /* eq. (source): the space-time mean of S over the cell, by the tensor
     * Gauss-Legendre rule on the predictor's nodes (exact for S linear) */
    for (int vv = 0; vv < nv; ++vv) {
      double acc = 0.0;
      for (int a = 0; a < nn; ++a)
        for (int b = 0; b < nn; ++b) acc += s.w[a] * s.w[b] * (-kap * qh[(vv * nn + a) * nn + b]);
      Si[vv * n + i] = acc;
    }
  }

  /* Transmissive ends: a ghost cell outside each end holds the end cell's
   * average as constant data (zero-gradient extrapolation).  Constant data
   * have no flux gradient, so the predictor only applies the source: the
   * solution at the time nodes is (K_z^{-1} l(0))_b times the average, and
   * l(1) . K_z^{-1} l(0) times it at the end of the step (without source a
   * constant state is its own evolution). */
  double *GL = (double *)malloc(sizeof(double) * ntr);
  double *GR = (double *)malloc(sizeof(double) * ntr);
  double gend = 0.0;
  for (int b = 0; b < nn; ++b) gend += s.l1[b] * s.Kinv_l0[b];
  for (int vv = 0; vv < nv; ++vv)
    for (int b = 0; b <= nn; ++b) {
      const double fac = kap == 0.0 ? 1.0 : (b < nn ? s.Kinv_l0[b] : gend);
      GL[vv * (nn + 1) + b] = fac * q[vv * n + 0];
      GR[vv * (nn + 1) + b] = fac * q[vv * n + n - 1];
    }

  /* interfaces k = 0..n; interface k lies between cells k-1 and k */
  for (int k = 0; k <= n && rc == ORC_OK; ++k) {
    const double *tl, *tr; /* right trace of left cell, left trace of right cell */
    if (per) {
      int cl = (k - 1 + n) % n, cr = k % n;
      tl = TR + (size_t)ntr * cl;
      tr = TL + (size_t)ntr * cr;
    } else if (k == 0) {
      tl = GL;
      tr = TL;
    } else if (k == n) {
      tl = TR + (size_t)ntr * (n - 1);
      tr = GR;
    } else {
      tl = TR + (size_t)ntr * (k - 1);
      tr = TL + (size_t)ntr * k;
    }
    double Fbar[3] = {0, 0, 0};
    for (int b = 0; b <= nn && rc == ORC_OK; ++b) {
      double QL[3], QR[3], F[3], Q0[3];
      for (int vv = 0; vv < nv; ++vv) {
        QL[vv] = tl[vv * (nn + 1) + b];
        QR[vv] = tr[vv * (nn + 1) + b];
      }
      if (b == nn && cf->system == 1 && cf->datum == 1)
        rc = orc_datum_trrs(cf, QL, QR, Q0); /* end-of-step datum only */
      else
        rc = orc_interact(cf, QL, QR, F, Q0, st);
      if (rc != ORC_OK) break;
      if (b < nn) {
        for (int vv = 0; vv < nv; ++vv) Fbar[vv] += s.w[b] * F[vv];
      } else {
        for (int vv = 0; vv < nv; ++vv) v_out[vv * (n + 1) + k] = Q0[vv];
      }
    }
    for (int vv = 0; vv < nv; ++vv) Fb[vv * (n + 1) + k] = Fbar[vv];
  }

  if (rc == ORC_OK) {
    for (int i = 0; i < n; ++i) {
      double Q[3];
      for (int vv = 0; vv < nv; ++vv) {
        q_out[vv * n + i] =
            q[vv * n + i] - nu * (Fb[vv * (n + 1) + i + 1] - Fb[vv * (n + 1) + i]) + dt * Si[vv * n + i];
        Q[vv] = q_out[vv * n + i];
      }
      if (orc_check_state(cf, Q) != ORC_OK) rc = ORC_E_NONPHYSICAL;
    }
  }
  free(TL);
  free(TR);
  free(Fb);
  free(Si);
  free(GL);
  free(GR);
  if (dt_out) *dt_out = dt;
  if (t_out) *t_out = tn;
  return rc;
}

/* Interface data at t = 0 (the paper does not say how the first step gets
 * them): the Riemann solution at x/t = 0 between the one-sided limits of the
 * initial condition at each interface (equal limits give the point value),
 * by the same solver that provides the datum in later steps. */
int orc_init_interfaces(const orc_cfg *cf, int nif, const double *vl, const double *vr, double *v) {
  int nv = orc_nvar(cf);
  for (int k = 0; k < nif; ++k) {
    double QL[3], QR[3], F[3], Q0[3];
    for (int vv = 0; vv < nv; ++vv) {
      QL[vv] = vl[vv * nif + k];
      QR[vv] = vr[vv * nif + k];
    }
    int rc = (cf->system == 1 && cf->datum == 1) ? orc_datum_trrs(cf, QL, QR, Q0)
                                                 : orc_interact(cf, QL, QR, F, Q0, NULL);
    if (rc != ORC_OK) return rc;
    for (int vv = 0; vv < nv; ++vv) v[vv * nif + k] = Q0[vv];
  }
  return ORC_OK;
}

/* Advance one domain in place until t_end or max_steps steps. */
int orc_run_segment(const orc_cfg *cf, int n, double dx, double *q, double *v, double t0, double t_end,
                    int64_t max_steps, double *t_out, int64_t *steps_out, orc_stats *st) {
  int nv = orc_nvar(cf);
  double *q2 = (double *)malloc(sizeof(double) * nv * n);
  double *v2 = (double *)malloc(sizeof(double) * nv * (n + 1));
  double t = t0;
  int64_t k = 0;
  int rc = ORC_OK;
  while (k < max_steps && t < t_end) {
    double dt, tn;
    rc = orc_segment_step(cf, n, dx, q, v, t, t_end, q2, v2, &dt, &tn, st);
    if (rc != ORC_OK) break;
    memcpy(q, q2, sizeof(double) * nv * n);
    memcpy(v, v2, sizeof(double) * nv * (n + 1));
    t = tn;
    ++k;
  }
  free(q2);
  free(v2);
  if (t_out) *t_out = t;
  if (steps_out) *steps_out = k;
  return rc;
}

/* Many independent domains stored back to back: cells of segment s are
 * [cell_off[s], cell_off[s+1]) of q (SoA [nv][total_cells]); its n_s + 1
 * interfaces are [cell_off[s] + s, cell_off[s+1] + s + 1) of v
 * (SoA [nv][total_cells + n_seg]).  Each segment advances with its own dt. */
int orc_run_segments(const orc_cfg *cf, int nseg, const int64_t *cell_off, const double *dx, double *q,
                     double *v, double *t, double t_end, int64_t max_steps, orc_stats *st) {
  int nv = orc_nvar(cf);
  int64_t total = cell_off[nseg], totif = total + nseg;
  int rc = ORC_OK;
  for (int s = 0; s < nseg && rc == ORC_OK; ++s) {
    int64_t c0 = cell_off[s], n = cell_off[s + 1] - c0, i0 = c0 + s;
    double *qs = (double *)malloc(sizeof(double) * nv * n);
    double *vs = (double *)malloc(sizeof(double) * nv * (n + 1));
    for (int vv = 0; vv < nv; ++vv) {
      memcpy(qs + vv * n, q + vv * total + c0, sizeof(double) * n);
      memcpy(vs + vv * (n + 1), v + vv * totif + i0, sizeof(double) * (n + 1));
    }
    double tout;
    int64_t k;
    rc = orc_run_segment(cf, (int)n, dx[s], qs, vs, t[s], t_end, max_steps, &tout, &k, st);
    t[s] = tout;
    for (int vv = 0; vv < nv; ++vv) {
      memcpy(q + vv * total + c0, qs + vv * n, sizeof(double) * n);
      memcpy(v + vv * totif + i0, vs + vv * (n + 1), sizeof(double) * (n + 1));
    }
    free(qs);
    free(vs);
  }
  return rc;
}
