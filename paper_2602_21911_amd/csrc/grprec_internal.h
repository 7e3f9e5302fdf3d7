// grprec_internal.h -- structures shared by the library's host code and its
// gfx950 kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include "grprec_tiles.h"

namespace grp {

// Device control block.  Every per-step quantity lives in one of three slots:
// the step launched with slot p reads slot p, accumulates slot p+1 (atomics)
// and clears slot p+2, so a fixed launch sequence of period 3 can be captured
// once in a graph and replayed while all control stays on the device.
struct Ctl {
  int cur[3];          // buffer pair holding the state at the start of the step
  int active[3];       // domains with t < t_end at the start of the step
  long long steps[3];  // steps taken
  unsigned int err;    // sticky error bits (ErrBits)
  unsigned int stats_on;
  double t_end;
  unsigned long long stat[5];  // rs_calls, newton_iters, picard_sweeps, cells, mlp_guesses
  unsigned long long hash[2];  // bitwise digest used by the autotuner
};

enum ErrBits : unsigned int { ERR_NONPHYS = 1u, ERR_VACUUM = 2u, ERR_NEWTON = 4u, ERR_PICARD = 8u };

// Ideal-gas constants derived from gamma once on the host.
struct Gas {
  double g, gm1, gp1;
  double z;        // (g-1)/(2g)
  double inv_g;    // 1/g
  double two_gm1;  // 2/(g-1)
  double two_gp1;  // 2/(g+1)
  double gm1_gp1;  // (g-1)/(g+1)
  double twog_gm1; // 2g/(g-1)
  double gp1_2g;   // (g+1)/(2g)
  double inv_gm1;  // 1/(g-1)
  int root_n;      // 1/z when it is an integer (7 for g = 1.4), else 0
  int dens_k;      // 2/(g-1) when it is an integer (5 for g = 1.4), else 0
  double inv_n, nm1_n;  // 1/root_n, (root_n - 1)/root_n
  float inv_nf;
  // second-order coefficients of the weak-wave expansions about p = pK
  double k2;       // f_K  = (cK/g) d (1 - k2 d),        k2 = (g+1)/(4g)
  double z2;       // w    = 1 + z d + z2 d^2,          z2 = z (z-1)/2
  double dens2;    // rho* = rhoK (1 + d/g + dens2 d^2), dens2 = -(g-1)/(2g^2)
};

namespace gasc {
constexpr double cabs(double x) { return x < 0.0 ? -x : x; }
constexpr double cround(double x) { return (double)(long long)(x + 0.5); }
}  // namespace gasc

// Ideal-gas constants from gamma (usable at compile time).
constexpr Gas make_gas(double g) {
  Gas G{};
  G.g = g;
  G.gm1 = g - 1.0;
  G.gp1 = g + 1.0;
  G.z = (g - 1.0) / (2.0 * g);
  G.inv_g = 1.0 / g;
  G.two_gm1 = 2.0 / (g - 1.0);
  G.two_gp1 = 2.0 / (g + 1.0);
  G.gm1_gp1 = (g - 1.0) / (g + 1.0);
  G.twog_gm1 = 2.0 * g / (g - 1.0);
  G.gp1_2g = (g + 1.0) / (2.0 * g);
  G.inv_gm1 = 1.0 / (g - 1.0);
  const double n = 2.0 * g / (g - 1.0), k = 2.0 / (g - 1.0);
  G.root_n = (n < 32.0 && gasc::cabs(n - gasc::cround(n)) < 1e-9) ? (int)gasc::cround(n) : 0;
  G.dens_k = (k < 32.0 && gasc::cabs(k - gasc::cround(k)) < 1e-9) ? (int)gasc::cround(k) : 0;
  G.inv_n = G.root_n ? 1.0 / G.root_n : 0.0;
  G.nm1_n = G.root_n ? (G.root_n - 1.0) / G.root_n : 0.0;
  G.inv_nf = (float)G.inv_n;
  G.k2 = (g + 1.0) / (4.0 * g);
  G.z2 = 0.5 * G.z * (G.z - 1.0);
  G.dens2 = -(g - 1.0) / (2.0 * g * g);
  return G;
}

// Diatomic ideal gas, gamma = 1.4: the kernels carry a compile-time copy.
constexpr double kGammaAir = 1.4;
constexpr Gas kAir = make_gas(kGammaAir);

// Domain (segment) tables in the workspace.
struct Seg {
  const int *cell_off;         // [S+1] first cell of each domain
  const double *dx;            // [S]
  double *t;                   // [3][S] time per slot
  unsigned long long *smax;    // [3][S] S_max per slot (bits of a non-negative double)
  int S;
};

struct Harvest {
  double *ring;                // [cap][7] or null
  long long cap;
  unsigned long long *count;
};

template <int M>
struct EulerArgs {
  double *q0, *q1, *v0, *v1;
  int tc, ti;                  // total cells, total interfaces (SoA strides)
  const Tile *tiles;
  int ntiles;
  Seg seg;
  Ctl *ctl;
  int slot;
  int periodic;
  double cfl;
  Gas gas;
  int max_newton;
  double newton_tol;
  int max_picard;
  double picard_tol;
  int guess, warm;
  double gate;
  const float *mlp;
  Harvest hv;
  double nl_lambda_c, nl_eps;  // GRPrecNL weights (used by the NL instantiations)
  int datum;                   // end-of-step datum: 0 exact Riemann solver, 1 two-rarefaction
  int source;                  // 1: S(Q) = -kappa Q (the SRC instantiations)
  double kappa;
};

template <int M>
struct AdvArgs {
  double *q0, *q1, *v0, *v1;
  int n;                       // cells (single domain)
  Seg seg;
  Ctl *ctl;
  int slot;
  int periodic;
  double cfl, lambda;
  double nl_lambda_c, nl_eps;  // GRPrecNL weights (used by the NL instantiations)
  double kappa;                // S(q) = -kappa q (the SRC instantiations)
  double *src;                 // per-step linear maps of the predictor with source (SRC)
};

}  // namespace grp
