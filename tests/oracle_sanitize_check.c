/* Runs every entry point of the C oracle on small problems (advection and
 * Euler, orders 2-5, periodic and transmissive, GRPrec and GRPrecNL, exact and
 * two-rarefaction datum, segments, error paths) so that the address and
 * undefined-behaviour sanitizers see every allocation and index of it.
 * Built and run by tests/test_oracle_sanitize.py; prints "ok <cases>". */
#include <math.h>
#include <stdio.h>

#include "grprec_oracle.c"

static int cases = 0;

static void fill_adv(int n, double *q, double *v) {
  for (int i = 0; i < n; ++i) q[i] = sin(2.0 * M_PI * (i + 0.5) / n);
  for (int k = 0; k <= n; ++k) v[k] = sin(2.0 * M_PI * k / n);
}

static void fill_euler(int n, double *q, double *v, double umean) {
  for (int i = 0; i < n; ++i) {
    double x = (i + 0.5) / n, r = 1.0 + 0.2 * sin(2.0 * M_PI * x), u = umean, p = 1.0;
    q[i] = r;
    q[n + i] = r * u;
    q[2 * n + i] = p / 0.4 + 0.5 * r * u * u;
  }
  for (int k = 0; k <= n; ++k) {
    double x = (double)k / n, r = 1.0 + 0.2 * sin(2.0 * M_PI * x), u = umean, p = 1.0;
    v[k] = r;
    v[(n + 1) + k] = r * u;
    v[2 * (n + 1) + k] = p / 0.4 + 0.5 * r * u * u;
  }
}

static orc_cfg base(int system, int m, int bc, int recon, int datum) {
  orc_cfg c = {system, m, 0.9, 1.0, 1.4, bc, bc, 1e-12, 50, 1e-13, 64, recon, 10.0, 1e-14, 4.0, datum};
  return c;
}

int main(void) {
  double x[8], w[8], R[25], M[35], g[5], D[25], kl[5], KW[25];
  for (int n = 1; n <= 5; ++n, ++cases) orc_gauss_legendre(n, x, w);
  for (int m = 1; m <= 4; ++m) {
    orc_recon_matrix(m, R);
    orc_side_matrix(m, 0, M);
    orc_side_matrix(m, 1, M);
    orc_predictor_matrices(m, g, w, D, kl, KW);
    double c[5] = {0.1, -0.2, 0.3, 0.05, -0.01};
    (void)orc_oi(m, c, 0.01);
    cases += 5;
  }
  /* Riemann problems: Sod, two rarefactions, two shocks, vacuum, Newton cap */
  double WL[3] = {1.0, 0.0, 1.0}, WR[3] = {0.125, 0.0, 0.1}, W0[3], ps, us;
  int it;
  orc_riemann(1.4, WL, WR, -1.0, 1e-12, 50, &ps, &us, W0, &it);
  double A[3] = {1.0, -2.0, 0.4}, B[3] = {1.0, 2.0, 0.4};
  orc_riemann(1.4, A, B, -1.0, 1e-12, 50, &ps, &us, W0, &it);
  orc_trrs(1.4, A, B, &ps, &us, W0);
  double C[3] = {1.0, 2.0, 1.0}, E[3] = {1.0, -2.0, 1.0};
  orc_riemann(1.4, C, E, -1.0, 1e-12, 50, &ps, &us, W0, &it);
  double V1[3] = {1.0, -20.0, 0.1}, V2[3] = {1.0, 20.0, 0.1};
  if (orc_riemann(1.4, V1, V2, -1.0, 1e-12, 50, &ps, &us, W0, &it) != ORC_E_VACUUM) return 2;
  if (orc_riemann(1.4, WL, WR, -1.0, 1e-12, 1, &ps, &us, W0, &it) != ORC_E_NEWTON) return 3;
  (void)orc_pvrs_guess(1.4, WL, WR);
  cases += 8;

  enum { NMAX = 64 };
  double q[3 * NMAX], v[3 * (NMAX + 1)], qo[3 * NMAX], vo[3 * (NMAX + 1)], dt, tn, t;
  int64_t k;
  orc_stats st = {0, 0, 0, 0, 0};
  for (int m = 1; m <= 4; ++m)
    for (int bc = 0; bc <= 1; ++bc)
      for (int recon = 0; recon <= 1; ++recon) {
        const int n = 23 + m;
        orc_cfg c = base(0, m, bc, recon, 0);
        fill_adv(n, q, v);
        if (orc_segment_step(&c, n, 1.0 / n, q, v, 0.0, 1.0, qo, vo, &dt, &tn, &st) != ORC_OK) return 4;
        if (orc_run_segment(&c, n, 1.0 / n, q, v, 0.0, 1.0, 5, &t, &k, &st) != ORC_OK) return 5;
        for (int datum = 0; datum <= 1; ++datum) {
          orc_cfg e = base(1, m, bc, recon, datum);
          fill_euler(n, q, v, bc ? 0.3 : 1.0);
          if (orc_run_segment(&e, n, 1.0 / n, q, v, 0.0, 1.0, 3, &t, &k, &st) != ORC_OK) return 6;
          double d[21], coef[15], beta[9];
          for (int j = 0; j < 21; ++j) d[j] = 1.0 + 0.01 * j;
          d[7] = 0.3; /* momentum row: small velocity */
          for (int j = 8; j < 14; ++j) d[j] = 0.3 + 0.001 * j;
          for (int j = 14; j < 21; ++j) d[j] = 3.0 + 0.01 * j;
          if (orc_recon_nl_cell(&e, 0.05, d, coef, beta) != ORC_OK) return 7;
          cases += 2;
        }
        cases += 2;
      }
  /* first-step interface data (Euler, both solvers) at a jump */
  {
    const int n = 10;
    double vl[3 * 11], vr[3 * 11], vv[3 * 11];
    for (int j = 0; j <= n; ++j) {
      vl[j] = 1.0; vl[11 + j] = 0.0; vl[22 + j] = 2.5;
      vr[j] = 0.5; vr[11 + j] = 0.0; vr[22 + j] = 1.25;
    }
    for (int datum = 0; datum <= 1; ++datum) {
      orc_cfg e = base(1, 2, 1, 0, datum);
      if (orc_init_interfaces(&e, n + 1, vl, vr, vv) != ORC_OK) return 8;
      ++cases;
    }
  }
  /* back-to-back segments */
  {
    int64_t off[4] = {0, 5, 17, 40};
    double dxs[3] = {0.2, 0.05, 0.03}, ts[3] = {0.0, 0.0, 0.0};
    double qq[3 * 40], vv[3 * 43];
    for (int s = 0; s < 3; ++s) {
      const int n = (int)(off[s + 1] - off[s]);
      double qs[3 * 40], vs[3 * 41];
      fill_euler(n, qs, vs, 0.5);
      for (int var = 0; var < 3; ++var) {
        for (int i = 0; i < n; ++i) qq[var * 40 + off[s] + i] = qs[var * n + i];
        for (int i = 0; i <= n; ++i) vv[var * 43 + off[s] + s + i] = vs[var * (n + 1) + i];
      }
    }
    orc_cfg e = base(1, 2, 1, 0, 0);
    if (orc_run_segments(&e, 3, off, dxs, qq, vv, ts, 1e9, 4, &st) != ORC_OK) return 9;
    ++cases;
  }
  /* a non-physical cell: S_max is NaN and the step reports it */
  {
    const int n = 12;
    orc_cfg e = base(1, 2, 0, 0, 0);
    fill_euler(n, q, v, 1.0);
    q[2 * n + 4] = -1.0;
    if (!isnan(orc_smax(&e, n, q))) return 10;
    if (orc_segment_step(&e, n, 1.0 / n, q, v, 0.0, 1.0, qo, vo, &dt, &tn, &st) != ORC_E_NONPHYSICAL) return 11;
    cases += 2;
  }
  printf("ok %d\n", cases);
  return 0;
}
