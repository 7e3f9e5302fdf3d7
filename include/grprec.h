/*
 * grprec.h -- C ABI of libgrprec.so: the per-time-step hot path of the GRPrec
 * finite-volume scheme on AMD MI355X (gfx950), FP64.
 *
 * Method (Montecinos, Toro & Mueller, "A generalized Riemann problem-based
 * compact reconstruction method for finite volume schemes"):
 *   one step of the fully discrete ADER finite-volume scheme, eq. (eq_finite_volume)
 *   of Sec. 2, without source or with a linear relaxation source, with
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
 * (grprec_step with dt_out, grprec_run, grprec_state, grprec_get_state).
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
/* Source term S(Q) of eq. (eq_hyperbolic_system). */
enum {
  GRPREC_SOURCE_NONE = 0,
  GRPREC_SOURCE_LINEAR = 1 /* S(Q) = -kappa Q, every component: taken implicitly in the
                              space-time predictor (the locally implicit DET of Sec. 2,
                              which admits stiff sources), and dt S^n_i of eq. (source) from
                              the predicted space-time polynomial in eq. (eq_finite_volume) */
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
                          warm starts are taken; below it Newton starts from PVRS, and so
                          does every problem the weak-wave path takes (both waves weak,
                          one Newton step from PVRS) (default 0.1; negative: the learned
                          start for every problem) */
  int warm_start;      /* 1: at interfaces above the gate, the later Riemann problems start
                          from the first time's p*, moved by the change of the PVRS
                          estimate between the two problems (implied by GUESS_MLP) */
  int schedule;        /* GRPREC_SCHED_* (Euler) */
  int block;           /* workgroup size 64, 128 or 256 (0 = choose) */
  int recon;           /* GRPREC_RECON_* */
  double nl_lambda_c;  /* GRPrecNL weight lambda_C of the centred polynomial in eq. (omega),
                          (0, 1e30]; default 1e9 when 0, the value Sec. 3.3 prints.  With
                          it GRPrecNL equals GRPrec on smooth data; the printed GRPrecNL
                          advection results (Sec. 4.2.3) are reproduced with 10 */
  double nl_eps;       /* GRPrecNL epsilon, [1e-30, 1] (default 1e-14 when 0) */
  int datum;           /* GRPREC_DATUM_* (Euler only) */
  int source;          /* GRPREC_SOURCE_*; for the Euler equations only with GRPrec and the
                          exact datum (else GRPREC_E_UNSUPPORTED) */
  double source_kappa; /* kappa >= 0 of GRPREC_SOURCE_LINEAR */
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

/* Bytes of device workspace needed for this problem (0 on invalid input).
 * The workspace holds the control block, the per-domain tables (cell offsets,
 * dx, times and S_max of eq. dt-FV), the tile lists and, with schedule AUTO,
 * an autotuning snapshot of one state. */
size_t grprec_workspace_bytes(const grprec_problem *p);

/* Set-up of the scheme of Sec. 2 on N uniform cells per domain (the grid of
 * Sec. 2): validates the problem (order 2..5 as in Sec. 3.1, 0 < C_CFL <= 1 as
 * the Courant limit of Sec. 4.1 and its table of methods), builds the plans,
 * computes the first-step interface data (the Riemann solution between the
 * one-sided limits of the initial condition; the paper is silent on the first
 * step) and the first S_max (Sec. 4.1) on `hip_stream` (a hipStream_t; NULL =
 * default stream).  Time starts at 0.  With schedule AUTO the Euler tile
 * schedule is autotuned here (a few timed steps on a snapshot that is
 * restored afterwards).  *out receives a handle owned by the caller until
 * grprec_destroy; on error *out is NULL and nothing is left allocated. */
int grprec_init(grprec_handle **out, const grprec_problem *p, const grprec_buffers *b,
                void *hip_stream);

/* One time step of eq. (eq_finite_volume), Sec. 2: dt from eq. (dt-FV) with
 * S_max of Sec. 4.1 per domain, GRPrec (Sec. 3.1) or GRPrecNL (Sec. 3.3-3.4)
 * reconstruction from the cell averages and the previous step's interface
 * states, the DET predictor and Riemann problems at the Gauss-Legendre times
 * of eq. (numfluxes) and at tau = dt (the next step's interface data), then the
 * conservative update.  The step is clipped so that no domain passes t_stop;
 * domains already at t_stop do not move.  Enqueued on the handle's stream.
 * dt_out != NULL synchronises the stream and returns the step of domain 0
 * (latched device errors are returned then). */
int grprec_step(grprec_handle *h, double t_stop, double *dt_out);

/* Repeated steps of eq. (eq_finite_volume) until every domain reaches t_end
 * (the last step of each domain is clipped to land on t_end) or max_steps
 * steps were taken.  Runs captured HIP graphs of several steps; synchronises
 * between graph chunks.  steps_out, t_out (host, may be NULL): steps taken by
 * this call and the time of domain 0. */
int grprec_run(grprec_handle *h, double t_end, int64_t max_steps, int64_t *steps_out,
               double *t_out);

/* Synchronise and report which buffer pair holds the current state
 * (0: q0/v0, 1: q1/v1), the smallest and largest domain time and the number
 * of steps taken since init.  Returns any latched device error.  Any output
 * pointer may be NULL. */
int grprec_state(grprec_handle *h, int *current, double *t_min, double *t_max, int64_t *steps);

/* Synchronise and report the time t^n of the current state (the smallest
 * domain time, i.e. the time of the state for a single domain) and the number
 * of steps taken since init (or since the last grprec_set_state).  The cell
 * averages Q^n and the interface states q_{i+1/2}^{n-1}(dt^{n-1}) of Sec. 3.1
 * stay in the caller's buffers; grprec_state names the current pair.  Either
 * pointer may be NULL.  Returns any latched device error. */
int grprec_get_state(grprec_handle *h, double *t, int64_t *step);

/* Copy the per-domain times t^n (host array of n_segments doubles; each domain
 * advances with its own dt of eq. dt-FV). */
int grprec_segment_times(grprec_handle *h, double *t_host);

/* Restart from a saved state (checkpoint/resume; not in the paper): the caller
 * has written the cell averages and interface states into the buffers named
 * by `current` (0: q0/v0, 1: q1/v1); every domain time is set to t, the step
 * counter to steps, and S_max (Sec. 4.1) is recomputed from the averages.
 * Clears latched errors; returns GRPREC_E_NONPHYSICAL if a cell is not a
 * physical state. */
int grprec_set_state(grprec_handle *h, int current, double t, int64_t steps);

/* Tile schedule in use, and a way to force one (Euler; not in the paper: how
 * the cells of many domains are grouped into workgroups).  set_schedule
 * rejects schedules and blocks outside the GRPREC_SCHED_* values and
 * 64/128/256 with GRPREC_E_INVALID. */
int grprec_get_schedule(grprec_handle *h, int *schedule, int *block);
int grprec_set_schedule(grprec_handle *h, int schedule, int block);

/* Autotuner (not in the paper).  Times each schedule candidate for `steps`
 * steps from the current state (the fastest of three runs) and keeps the
 * fastest candidate whose result is bitwise equal to the first candidate's;
 * the state is restored.  Writes per-candidate milliseconds per step into the
 * host array ms_out[n_max] (candidate order: schedules 1..3 x blocks
 * 64,128,256; a single domain tries segment tiles only; negative when the
 * result differed), and the number written into *n_out.  Needs the snapshot
 * area of a problem created with schedule AUTO (else GRPREC_E_INVALID). */
int grprec_autotune(grprec_handle *h, int steps, double *ms_out, int n_max, int *n_out);

/* Solver counters (not in the paper) accumulated while counting is on:
 * Riemann solves (the interaction step of Sec. 2), Newton iterations on the
 * star pressure, predictor sweeps, cells predicted (owned cells plus halo
 * recomputations), learned starts taken. */
typedef struct {
  uint64_t rs_calls, newton_iters, picard_sweeps, cells_predicted, mlp_guesses;
} grprec_stats;
int grprec_enable_stats(grprec_handle *h, int on);
int grprec_get_stats(grprec_handle *h, grprec_stats *out);

/* Static message for a status code ("unknown error" for other values). */
const char *grprec_error_string(int code);
/* Release the handle's host-side plans and graphs (NULL is ignored); the
 * caller's device buffers are untouched. */
void grprec_destroy(grprec_handle *h);

/* ---- Riemann problems in bulk ----
 * The exact Euler Riemann solver of the interaction step (Sec. 2, Sec. 4.3:
 * Newton on the star pressure from the pressure functions of the two waves),
 * applied to n independent problems: wl, wr are device [n][3] primitive
 * states (rho, u, p); outputs p* and Newton iterations per problem (device,
 * either may be NULL).  guess as above (mlp_params needed for
 * GRPREC_GUESS_MLP; gate < 0 uses the network for every problem).  Problems
 * that fail get p* = NaN and the negative error code in iters.  Enqueued on
 * hip_stream. */
int grprec_riemann_batch(const double *wl, const double *wr, int64_t n, double gamma, int guess,
                         const float *mlp_params, double gate, double tol, int max_iter,
                         double *pstar, int *iters, void *hip_stream);

/* ---- learned star-pressure proposal: features, inference, training ----
 * Not in the paper: a start value for the Newton iteration of the exact
 * Riemann solver.  Newton still runs to the same tolerance, so the solution
 * is that of the plain method.  All pointers are device pointers; calls are
 * enqueued on hip_stream; sizes n < 0 or missing pointers give
 * GRPREC_E_INVALID. */

/* Unnormalised features x[n][6] (float32) of primitive states wl, wr [n][3]
 * and, when pstar != NULL, targets y[n] = ln(p_star / pbar). */
int grprec_mlp_features(const double *wl, const double *wr, const double *pstar, int64_t n,
                        double gamma, float *x, float *y, void *hip_stream);
/* y[n] = network(standardise(x)) with params as laid out above. */
int grprec_mlp_forward(const float *params, const float *x, float *y, int64_t n,
                       void *hip_stream);
/* Bytes of device workspace that grprec_mlp_backward and grprec_mlp_loss_grad
 * need for n samples (per-block partial sums; 0 for n < 1). */
size_t grprec_mlp_work_bytes(int64_t n);
/* Backward pass: grad[k] = sum_s dy[s] d y_s / d theta_k over the n samples of
 * x[n][6] for the GRPREC_MLP_WEIGHTS weights theta (the normaliser is not
 * differentiated); dy[n] is the upstream gradient of the outputs.  grad:
 * device float[GRPREC_MLP_WEIGHTS], overwritten.  work: device scratch of at
 * least grprec_mlp_work_bytes(n) bytes; 1 <= n <= 64 * 2^20. */
int grprec_mlp_backward(const float *params, const float *x, const float *dy, float *grad,
                        int64_t n, void *work, void *hip_stream);
/* grprec_mlp_backward without caller workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the per-block partial sums live in a
 * fixed device array of the library (5.1 MiB per device, kept until the
 * process ends), so at most GRPREC_MLP_NOALLOC_MAX samples per call
 * (1 <= n <= 65536, else GRPREC_E_INVALID).  Same kernels and same result as
 * grprec_mlp_backward.  Every call on a device shares that device's array:
 * calls that overlap on one device (several streams or threads) race. */
#define GRPREC_MLP_NOALLOC_MAX 65536
int grprec_mlp_backward_noalloc(const float *params, const float *x, const float *dy, float *grad,
                                int64_t n, void *hip_stream);
/* Mean-squared-error loss (1/n) sum_s (y_s - t_s)^2 over the batch and its
 * gradient with respect to the GRPREC_MLP_WEIGHTS weights: the backward pass
 * with dy = 2 (y - t) / n.  grad: device float[GRPREC_MLP_WEIGHTS]; loss:
 * device float[1] or NULL.  work as for grprec_mlp_backward. */
int grprec_mlp_loss_grad(const float *params, const float *x, const float *y, int64_t n,
                         float *grad, float *loss, void *work, void *hip_stream);
/* One Adam update of the weights (the normaliser is left alone); m, v: device
 * moment buffers of GRPREC_MLP_WEIGHTS floats; step counts from 1. */
int grprec_mlp_adam(float *params, const float *grad, float *m, float *v, int step, float lr,
                    float beta1, float beta2, float eps, void *hip_stream);

/* Record the Riemann problems solved by the following steps (training data for
 * the learned start; not in the paper): each interface's first flux problem
 * (the interaction at the first Gauss-Legendre time, Sec. 2) is written as
 * (rhoL, uL, pL, rhoR, uR, pR, p*) doubles into the device ring [cap][7];
 * *count_dev (device int64) counts attempts (entries beyond cap are dropped).
 * ring = NULL switches recording off.  Euler only. */
int grprec_harvest(grprec_handle *h, double *ring, int64_t cap, int64_t *count_dev);

#ifdef __cplusplus
}
#endif
#endif /* GRPREC_H */
