// grprec_internal.h -- structures shared by the library's host code and its
// gfx950 kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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
};

// Per-degree constants of the space-time predictor and of the reconstruction.
// Nodes g_a are the (M+1)-point Gauss-Legendre points on [0,1].
template <int M>
struct StConst {
  double D[M + 1][M + 1];   // D[a][k] = l_k'(g_a)
  double KW[M + 1][M + 1];  // K^{-1} diag(w), K the time matrix of the weak form
  double l0[M + 1];         // l_a(0)
  double l1[M + 1];         // l_a(1)
  double w[M + 1];          // Gauss-Legendre weights on [0,1]
  double phi[M + 1][4];     // zero-mean basis xi, xi^2-1/12, xi^3, xi^4-1/80 at xi = g_a - 1/2
};

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
  const int4 *tiles;           // (first cell, count, first domain, last domain)
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
  StConst<M> C;
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
};

}  // namespace grp
