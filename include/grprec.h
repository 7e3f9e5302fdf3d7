/*
 * grprec.h -- C ABI of libgrprec.so: the per-time-step hot path of the GRPrec
 * finite-volume scheme on AMD MI355X (gfx950), FP64.
 *
 * Method (Montecinos, Toro & Mueller, "A generalized Riemann problem-based
 * compact reconstruction method for finite volume schemes"):
 *   one step of the fully discrete ADER finite-volume scheme, eq. (eq_finite_volume)
 *   of Sec. 2 without source, with
 *   - time step dt = C_CFL dx / S_max, eq. (dt-FV), S_max as in Sec. 4.1;
 *   - GRPrec reconstruction of degree m = order-1 from the cell averages
 *     q_{i-1}, q_i, q_{i+1} and the previous step's GRP interface states
 *     q_{i-1/2}(dt^{n-1}), q_{i+1/2}(dt^{n-1}) (Sec. 3.1);
 *   - the DET solver of the generalized Riemann problem eq. (GRP): local
 *     space-time DG predictor per cell, then classical Riemann problems at the
 *     m+1 Gauss-Legendre times of the flux integral eq. (numfluxes) and at
 *     tau = dt, whose solution is the next step's interface state (Sec. 2, 4.1);
 *   - exact Riemann solvers: upwind state for linear advection (Sec. 4.2),
 *     Newton on the star pressure for the ideal-gas Euler equations (Sec. 4.3).
 *
 * Data layout (caller-owned device memory, float64, structure of arrays):
 *   q[var][cell]  : nvar x total_cells, cells of all domains back to back;
 *   v[var][iface] : nvar x (total_cells + n_segments); domain s with n_s cells
 *                   owns n_s + 1 interfaces starting at cell_off[s] + s
 *                   (interface k of a domain lies at x0 + k dx; for a periodic
 *                   domain entries 0 and n_s hold the same interface).
 * nvar = 1 (advection) or 3 (Euler: rho, rho u, E).
 *
 * Ownership: every device buffer belongs to the caller; the library keeps
 * pointers only.  Besides the caller's workspace the library allocates no
 * device memory.  The handle owns host-side plans, the tile lists' host copies
 * and any HIP graphs; grprec_destroy frees them.  A handle is bound to the
 * stream passed at init and is not thread-safe; use one handle per stream.
 *
 * Errors: every function returns GRPREC_OK (0) or a negative code.  Errors
 * raised inside kernels (non-physical states, vacuum, iteration caps) are
 * latched on the device and returned by the next call that synchronises
 * (grprec_step with dt_out, grprec_run, grprec_state).
 */
#ifndef GRPREC_H
#define GRPREC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GRPREC_OK 0
#define GRPREC_E_INVALID (-1)     /* bad argument: order, CFL, sizes, pointers */
#define GRPREC_E_UNSUPPORTED (-2) /* valid but not built, e.g. advection with several domains */
#define GRPREC_E_HIP (-3)         /* a HIP runtime call failed */
#define GRPREC_E_NONPHYSICAL (-4) /* rho <= 0, p <= 0 or non-finite value */
#define GRPREC_E_VACUUM (-5)      /* Riemann data generate vacuum */
#define GRPREC_E_NEWTON (-6)      /* star-pressure Newton hit its cap */
#define GRPREC_E_PREDICTOR (-7)   /* space-time predictor hit its sweep cap */

enum { GRPREC_ADVECTION = 0, GRPREC_EULER = 1 };
enum { GRPREC_BC_PERIODIC = 0, GRPREC_BC_TRANSMISSIVE = 1 };
/* Starting value of the star-pressure Newton iteration (Euler). */
enum {
  GRPREC_GUESS_PVRS = 0, /* linearised Riemann solver, floored at 1e-6 min(pL,pR) */
  GRPREC_GUESS_MLP = 1   /* learned proposal where the data jump is large, else PVRS */
};
/* Reconstruction operator. */
enum {
  GRPREC_RECON_LINEAR = 0, /* GRPrec, Sec. 3.1 */
  GRPREC_RECON_NL = 1      /* GRPrecNL, Sec. 3.3-3.4: convex combination of a left, the
                              centred (GRPrec) and a right polynomial with weights
                              omega_k = lambda_k / (eps + OI_k)^4, lambda_L = lambda_R = 1;
                              for the Euler equations in characteristic variables */
};
/* Solver of the end-of-step interface datum (Euler). */
enum {
  GRPREC_DATUM_EXACT = 0, /* exact Riemann solver, as for the fluxes */
  GRPREC_DATUM_TRRS = 1   /* two-rarefaction approximation (Sec. 4.1): closed form, no
                             iteration; also used for the first-step data */
};
/* How cells are grouped into workgroup tiles (Euler). */
enum {
  GRPREC_SCHED_AUTO = 0,          /* autotune at init over the others */
  GRPREC_SCHED_SEGMENT_TILES = 1, /* tiles never cross a domain boundary */
  GRPREC_SCHED_FLAT_TILES = 2,    /* fixed-size tiles over the concatenated cells */
  GRPREC_SCHED_PACKED = 3,        /* long domains split, short ones packed whole */
  GRPREC_SCHED_PER_DOMAIN = 4     /* one launch per domain per step (the plain form:
                                     the single-domain kernel applied domain by
                                     domain); always launched eagerly */
};

/* Learned star-pressure network: 6 -> 32 -> 32 -> 1, tanh, float32.
 * Parameter block (float32, this order): W1[32][6], b1[32], W2[32][32], b2[32],
 * W3[32], b3[1], then the feature normaliser mean[6], std[6].  Features of a
 * Riemann problem (primitive states L, R; bars are L/R means,
 * cbar = sqrt(gamma pbar / rhobar)):
 *   x = (ln(rhoL/rhobar), ln(rhoR/rhobar), ln(pL/pbar), ln(pR/pbar), uL/cbar, uR/cbar),
 * standardised with mean/std; output y approximates ln(p* / pbar). */
#define GRPREC_MLP_HIDDEN 32
#define GRPREC_MLP_IN 6
#define GRPREC_MLP_WEIGHTS 1313 /* 6*32+32 + 32*32+32 + 32+1 */
#define GRPREC_MLP_NPARAMS 1325 /* weights + 12 normaliser floats */

typedef struct grprec_handle grprec_handle;

typedef struct {
  int system;          /* GRPREC_ADVECTION or GRPREC_EULER */
  int order;           /* m + 1: 2..5 */
  double cfl;          /* C_CFL of eq. (dt-FV), 0 < cfl <= 1 */
  double lambda;       /* advection speed, nonzero */
  double gamma;        /* ratio of specific heats, > 1 */
  int bc;              /* GRPREC_BC_* at both ends of every domain */
  int n_segments;      /* number of independent domains, >= 1; periodic needs 1;
                          advection supports 1 */
  const int64_t *seg_cells;  /* host [n_segments], each >= 2 */
  const double *seg_length;  /* host [n_segments], each > 0 */
  int guess;           /* GRPREC_GUESS_* */
  int max_newton;      /* Newton cap (default 50 when 0) */
  double newton_tol;   /* stop at 2|p_new-p|/(p_new+p) <= tol (default 1e-12 when 0) */
  int max_picard;      /* predictor sweep cap (default 64 when 0) */
  double picard_tol;   /* predictor stop: max|change| <= tol (1 + max|q|) (default 1e-13) */
  const float *mlp_params; /* device, GRPREC_MLP_NPARAMS floats; needed for GUESS_MLP */
  double mlp_gate;     /* relative data jump |dp|/pbar + |drho|/rhobar + |du|/cbar of an
                          interface's first Riemann problem above which the learned and
                          warm starts are taken; below it Newton starts from PVRS
                          (default 0.1; negative: always) */
  int warm_start;      /* 1: at interfaces above the gate, the later Riemann problems start
                          from the first time's p* (implied by GUESS_MLP) */
  int schedule;        /* GRPREC_SCHED_* (Euler) */
  int block;           /* workgroup size 64, 128 or 256 (0 = choose) */
  int recon;           /* GRPREC_RECON_* */
  double nl_lambda_c;  /* GRPrecNL weight of the centred polynomial, (0, 1e30]
                          (default 10 when 0; the paper prints 1e9, with which
                          GRPrecNL equals GRPrec on smooth data, while its GRPrecNL
                          results are reproduced with 10) */
  double nl_eps;       /* GRPrecNL epsilon, [1e-30, 1] (default 1e-14 when 0) */
  int datum;           /* GRPREC_DATUM_* (Euler only) */
} grprec_problem;

typedef struct {
  double *q0, *q1; /* device [nvar][total_cells]: q0 holds the initial cell averages */
  double *v0, *v1; /* device [nvar][total_cells + n_segments]: at init v0 holds the
                      left and v1 the right limits of the initial condition at every
                      interface; init replaces v0 by the Riemann solution between
                      them at x/t = 0 (the point value where the data are continuous) */
  void *work;      /* device workspace, at least grprec_workspace_bytes() bytes */
  size_t work_bytes;
} grprec_buffers;

/* Bytes of device workspace needed for this problem (0 on invalid input). */
size_t grprec_workspace_bytes(const grprec_problem *p);

/* Validate the problem, build the plans, compute the first-step interface data
 * and the first S_max on `hip_stream` (a hipStream_t; NULL = default stream).
 * Time starts at 0.  With schedule AUTO the Euler tile schedule is autotuned
 * here (a few timed steps on a snapshot that is restored afterwards). */
int grprec_init(grprec_handle **out, const grprec_problem *p, const grprec_buffers *b,
                void *hip_stream);

/* One time step, clipped so that no domain passes t_stop.  Domains already at
 * t_stop do not move.  dt_out != NULL synchronises the stream and returns the
 * step of domain 0 (latched device errors are returned then). */
int grprec_step(grprec_handle *h, double t_stop, double *dt_out);

/* Steps until every domain reaches t_end or max_steps steps were taken.  Runs
 * captured HIP graphs of several steps; synchronises between graph chunks.
 * steps_out: steps taken by this call; t_out: time of domain 0. */
int grprec_run(grprec_handle *h, double t_end, int64_t max_steps, int64_t *steps_out,
               double *t_out);

/* Synchronise and report which buffer pair holds the current state
 * (0: q0/v0, 1: q1/v1), the smallest and largest domain time and the number
 * of steps taken since init.  Returns any latched device error. */
int grprec_state(grprec_handle *h, int *current, double *t_min, double *t_max, int64_t *steps);

/* Copy the per-domain times (host array of n_segments doubles). */
int grprec_segment_times(grprec_handle *h, double *t_host);

/* Restart from a saved state: the caller has written the state into the
 * buffers named by `current`; every domain time is set to t, the step counter
 * to steps, and S_max is recomputed.  Clears latched errors. */
int grprec_set_state(grprec_handle *h, int current, double t, int64_t steps);

/* Tile schedule in use, and a way to force one (Euler). */
int grprec_get_schedule(grprec_handle *h, int *schedule, int *block);
int grprec_set_schedule(grprec_handle *h, int schedule, int block);

/* Time each schedule candidate for `steps` steps from the current state (the
 * fastest of three runs) and keep the fastest candidate whose result is
 * bitwise equal to the first candidate's; the state is restored.  Writes
 * per-candidate milliseconds per step into ms_out[n_max] (candidate order:
 * schedules 1..3 x blocks 64,128,256; a single domain tries segment tiles
 * only; negative when the result differed), and the number written into
 * *n_out. */
int grprec_autotune(grprec_handle *h, int steps, double *ms_out, int n_max, int *n_out);

/* Counters accumulated since init when count_stats is on: Riemann solves,
 * Newton iterations, predictor sweeps, learned guesses used. */
typedef struct {
  uint64_t rs_calls, newton_iters, picard_sweeps, cells_predicted, mlp_guesses;
} grprec_stats;
int grprec_enable_stats(grprec_handle *h, int on);
int grprec_get_stats(grprec_handle *h, grprec_stats *out);

/* Message for a status code. */
const char *grprec_error_string(int code);
void grprec_destroy(grprec_handle *h);

/* ---- Riemann problems in bulk (exact Euler solver of the step) ----
 * wl, wr: device [n][3] primitive states (rho, u, p); outputs p* and Newton
 * iterations per problem (device, either may be NULL).  guess as above
 * (mlp_params needed for GRPREC_GUESS_MLP; gate < 0 uses the network for
 * every problem).  Problems that fail get p* = NaN and the negative error code
 * in iters. */
int grprec_riemann_batch(const double *wl, const double *wr, int64_t n, double gamma, int guess,
                         const float *mlp_params, double gate, double tol, int max_iter,
                         double *pstar, int *iters, void *hip_stream);

/* ---- learned star-pressure proposal: features, inference, training ----
 * Unnormalised features x[n][6] (float32) of primitive states wl, wr [n][3]
 * and, when pstar != NULL, targets y[n] = ln(p_star / pbar). */
int grprec_mlp_features(const double *wl, const double *wr, const double *pstar, int64_t n,
                        double gamma, float *x, float *y, void *hip_stream);
/* y[n] = network(standardise(x)) with params as laid out above. */
int grprec_mlp_forward(const float *params, const float *x, float *y, int64_t n,
                       void *hip_stream);
/* Mean-squared-error loss over the batch and its gradient with respect to the
 * GRPREC_MLP_WEIGHTS weights (grad: device float[GRPREC_MLP_WEIGHTS]; loss:
 * device float[1]).  work: device scratch of grprec_mlp_work_bytes(n) bytes. */
size_t grprec_mlp_work_bytes(int64_t n);
int grprec_mlp_loss_grad(const float *params, const float *x, const float *y, int64_t n,
                         float *grad, float *loss, void *work, void *hip_stream);
/* One Adam update of the weights (the normaliser is left alone); m, v: device
 * moment buffers of GRPREC_MLP_WEIGHTS floats; step counts from 1. */
int grprec_mlp_adam(float *params, const float *grad, float *m, float *v, int step, float lr,
                    float beta1, float beta2, float eps, void *hip_stream);

/* Record the Riemann problems solved by the following steps: each interface's
 * first flux problem is written as (rhoL, uL, pL, rhoR, uR, pR, p*) doubles into
 * the device ring [cap][7]; *count_dev (device int64) counts attempts (entries
 * beyond cap are dropped).  ring = NULL switches recording off. */
int grprec_harvest(grprec_handle *h, double *ring, int64_t cap, int64_t *count_dev);

#ifdef __cplusplus
}
#endif
#endif /* GRPREC_H */
