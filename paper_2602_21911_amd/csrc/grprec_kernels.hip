// grprec_kernels.hip -- gfx950 kernels of the GRPrec finite-volume step for
// linear advection, and the set-up kernels of both systems (first-step
// interface data, S_max, control block, digests).  The Euler step kernel is
// in grprec_euler.h.
//
// FP64 throughout; no matrix cores: the work is a per-cell stencil, not a
// dense contraction.
#include <hip/hip_runtime.h>

#include "grprec_device.h"
#include "grprec_internal.h"
#include "grprec_step_common.h"
#include "grprec_tables.h"

namespace grp {

// ============================================================ advection step
// Linear advection q_t + lambda q_x = 0, single domain, one thread per cell.
// The predictor is the exact translation of the reconstruction, so the
// interface state at time tau is the upwind polynomial at the foot of the
// characteristic, and the Gauss-Legendre flux integral (exact for this degree)
// equals lambda times the mean of that polynomial over the swept interval.
// With the zero-mean basis phi_j of the reconstruction the mean and the point
// value are fixed linear combinations of the coefficients per step.
__device__ __forceinline__ void basis_at(double x, double P[4]) {
  const double x2 = x * x;
  P[0] = x;
  P[1] = x2 - 1.0 / 12.0;
  P[2] = x2 * x;
  P[3] = x2 * x2 - 1.0 / 80.0;
}
// mean of phi_j over [lo, hi]
__device__ __forceinline__ void basis_mean(double lo, double hi, double K[4]) {
  auto prim = [](double x, double R[4]) {
    const double x2 = x * x;
    R[0] = 0.5 * x2;
    R[1] = x2 * x * (1.0 / 3.0) - x * (1.0 / 12.0);
    R[2] = 0.25 * x2 * x2;
    R[3] = 0.2 * x2 * x2 * x - x * (1.0 / 80.0);
  };
  double A[4], Bv[4];
  prim(lo, A);
  prim(hi, Bv);
  const double inv = 1.0 / (hi - lo);
#pragma unroll
  for (int j = 0; j < 4; ++j) K[j] = (Bv[j] - A[j]) * inv;
}

// GRPrecNL coefficients of one cell (Sec. 3.3-3.4) from its seven data
// (vll = V_{i-3/2}, vrr = V_{i+3/2}; read at degree 4 only).
template <int M>
__device__ __forceinline__ void adv_coeffs_nl(double qm, double qc, double qp, double vl, double vr,
                                              double vll, double vrr, double dx, double lam_c,
                                              double eps, double a[4]) {
  const double del[7] = {qm - qc, 0.0, qp - qc, vl - qc, vr - qc, vll - qc, vrr - qc};
  double aC[M], o[M];
  grprec_from_diffs<M>(del[0], del[2], del[3], del[4], aC);
  nl_mix<M>(aC, del, dx, lam_c, eps, o);
  a[0] = a[1] = a[2] = a[3] = 0.0;
#pragma unroll
  for (int j = 0; j < M; ++j) a[j] = o[j];
}

template <int M>
__device__ __forceinline__ void adv_coeffs(double qm, double qc, double qp, double vl, double vr,
                                           double a[4]) {
  const double DI = vr - vl, SI = vl + vr - 2.0 * qc;
  a[0] = a[1] = a[2] = a[3] = 0.0;
  if (M == 1) {
    a[0] = DI;
  } else if (M == 2) {
    a[0] = DI;
    a[1] = 3.0 * SI;
  } else {
    const double DC = qp - qm, SC = qp + qm - 2.0 * qc;
    a[0] = 1.25 * DI - 0.125 * DC;
    a[2] = 0.5 * DC - DI;
    if (M == 3) {
      a[1] = (3.0 * SI + 18.0 * SC) * (1.0 / 37.0);
    } else {
      a[1] = 3.75 * SI - 0.125 * SC;
      a[3] = (5.0 / 12.0) * SC - 2.5 * SI;
    }
  }
}

// Lane shifts of the advection step: lane l receives lane l-1 (adv_prev) or
// l+1 (adv_next); the lane without a source (0, resp. 63) receives 0.  Only
// lanes that no updated lane reads are left without a source, and the result
// goes straight to a new register (no copy of the old value first).
__device__ __forceinline__ double adv_prev(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, 0x138, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x138, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double adv_next(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, 0x130, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x130, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Runs per wave per block chunk.  Measured at 2^25 cells over 1, 2, 3, 4, 8,
// 12 and 16: the memory-bound GRPrec kernels run best with 2 (more blocks in
// flight), the arithmetic-bound GRPrecNL kernels with 8.
template <bool NL>
constexpr int adv_passes() {
  return NL ? 8 : 2;
}

// Cells a wave updates per run.  A reconstruction reads the lanes on either
// side of its own (and the second one to the right for GRPrecNL at degree 4,
// which reads V_{i+3/2}), and an update reads its upwind neighbour's
// reconstruction, so of 64 lanes 61 (60) update cells and the rest only
// hold data; no lane loads anything beyond its own cell.
template <int M, bool NL>
constexpr int adv_run() {
  return (NL && M == 4) ? 60 : 61;
}

// SRC: with the relaxation source S(q) = -kappa q the predictor is the
// space-time DG evolution with the implicit source instead of the exact
// translation; being linear, its flux mean, end-of-step datum and space-time
// mean are fixed linear combinations of the cell mean and the coefficients,
// computed once per step by adv_source_prep into a.src.
template <int M, bool NL, bool SRC, bool POS>
__global__ __launch_bounds__(256) void adv_step(AdvArgs<M> a) {
  Ctl *ctl = a.ctl;
  const int slot = a.slot, s1 = (slot + 1) % 3, s2 = (slot + 2) % 3;
  if (ctl->active[slot] == 0) {
    carry_slot(a.seg, ctl, slot);
    return;
  }
  const int cur = ctl->cur[slot];
  const double *__restrict__ qin = cur ? a.q1 : a.q0;
  double *__restrict__ qout = cur ? a.q0 : a.q1;
  const double *__restrict__ vin = cur ? a.v1 : a.v0;
  double *__restrict__ vout = cur ? a.v0 : a.v1;
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid == 0) {
    ctl->cur[s1] = 1 - cur;
    ctl->steps[s1] = ctl->steps[slot] + 1;
    ctl->active[s2] = 0;
  }
  const int n = a.n;
  const double dx = a.seg.dx[0];
  const double t = a.seg.t[slot * a.seg.S];
  const double t_end = ctl->t_end;
  double dt, t_new;
  bool done;
  domain_dt(a.cfl, dx, fabs(a.lambda), t, t_end, dt, t_new, done);
  const double cn = a.lambda * dt / dx;  // signed Courant number
  constexpr bool pos = POS;  // lambda > 0: the upwind side is the left
  // per-step constants: mean of each basis function over the swept interval
  // and its value at the foot of the characteristic
  double Kin[4], Pin[4], Sin[4] = {0.0, 0.0, 0.0, 0.0};
  double K0 = 1.0, P0 = 1.0, S0 = 0.0, zs = 0.0;
  if constexpr (SRC) {
    // [0]: the constant mode, [1 + j]: phi_{j+1} (zero beyond the degree)
    K0 = a.src[0];
    P0 = a.src[M + 1];
    S0 = a.src[2 * (M + 1)];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      Kin[j] = j < M ? a.src[1 + j] : 0.0;
      Pin[j] = j < M ? a.src[M + 2 + j] : 0.0;
      Sin[j] = j < M ? a.src[2 * (M + 1) + 1 + j] : 0.0;
    }
    zs = a.kappa * dt;
  } else if (pos) {
    basis_mean(0.5 - cn, 0.5, Kin);
    basis_at(0.5 - cn, Pin);
  } else {
    basis_mean(-0.5, -0.5 - cn, Kin);
    basis_at(-0.5 - cn, Pin);
  }
  auto Q = [&](int k) -> double {
    if (a.periodic) {
      if (k < 0) k += n;
      if (k >= n) k -= n;
    } else {
      if (k < 0) k = 0;
      if (k >= n) k = n - 1;
    }
    return qin[k];
  };
  auto V = [&](int k) -> double {  // interface index 0..n
    if (a.periodic) {
      if (k < 0) k += n;
      if (k > n) k -= n;
    }
    return vin[k];
  };
  // interface value j: wrapped when periodic; beyond a transmissive end the
  // ghost cell's constant state (its average)
  auto VG = [&](int j) -> double {
    if (!a.periodic) {
      if (j < 0) return qin[0];
      if (j > n) return qin[n - 1];
    }
    return V(j);
  };
  // A wave advances runs of RUN consecutive cells.  Lane l holds cell
  // base + l - OFF: the run's upwind neighbour and the reconstructions' outer
  // data sit in the lanes around the updated ones, so every lane loads only
  // its own cell's data, neighbours' values arrive by lane shifts, and the
  // upwind lane's flux mean and end-of-step datum reach the next lane the same
  // way.  A block takes chunks of 4 waves x PASSES runs.  Blocks are
  // dispatched to the 8 XCDs round-robin, so block b works on chunk
  // (b % 8) * per + b / 8: consecutive chunks run on one XCD and the cache
  // lines they share at their ends are read once through its L2.
  constexpr int RUN = adv_run<M, NL>();
  constexpr int PASSES = adv_passes<NL>();
  constexpr int CH = 4 * PASSES * RUN;
  static_assert(PASSES % 2 == 0, "runs may be taken in pairs");
  const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
  const int nch = (n + CH - 1) / CH;
  const int per = (nch + 7) / 8;
  // Runs r and r + 1 of a wave are taken together, their arithmetic
  // interleaved (measured 1.5-4 % faster); GRPrecNL at degree 4 takes one run
  // at a time (the loop after this one), since the pair's registers cost it
  // two waves per SIMD and the branch-free form more instructions (2.5-3.5 %
  // slower).
  constexpr int STEP = (NL && M == 4) ? 1 : 2;
  // updated lanes OFF .. OFF + RUN - 1: for lambda > 0 the upwind lane and
  // the left neighbour it reads lie below them, for lambda < 0 one lane
  // below and the upwind lane with its right data above
  constexpr int OFF = pos ? 2 : 1;
  // The data of the run starting at cell base.  Every lane within two cells
  // of the domain holds the average of its cell and the value at the cell's
  // left interface (wrapped when periodic; the ghost state beyond a
  // transmissive end); a reconstruction takes its neighbours' values from the
  // adjacent lanes.  (Cells -2 .. n+1 and interfaces -2 .. n+2 are what
  // reconstructions of cells -1 .. n read; a single +-n wrap keeps them in
  // range for n >= 2.)  Interfaces 0 and n of a periodic domain are one
  // interface: the lanes of cells -1 and n also hold the value their
  // reconstruction takes from its other end (x).
  auto load_run = [&](int base, double &qk, double &vk, double &x) {
    const int i = base + lane - OFF;
    if (i >= -2 && i <= n + 2) {
      qk = i <= n + 1 ? Q(i) : 0.0;
      vk = VG(i);
      if (a.periodic && (i == -1 || i == n)) x = vin[i == -1 ? n : 0];
    }
  };
  // The lane's flux mean over the swept interval, its datum and (with the
  // source) its space-time mean.  Every lane computes them without a branch
  // and keeps the result only where it reconstructs, so the arithmetic of the
  // two runs of a pair can be interleaved.  At i = -1 and i = n the upwind
  // neighbour is the
  // periodic image or the ghost cell (a constant state: mean and point value
  // are the end average, scaled by the source's evolution of a constant).
  // (Lanes at the wave's edges reconstruct from zeros shifted in; no updated
  // lane reads their results.)
  auto recon_run = [&](int base, double qk, double vk, double x, double &mean_s, double &pt_s,
                       double &src_s) {
    const int i = base + lane - OFF;
    double qp = adv_next(qk), vp = adv_next(vk);
    const double qm = adv_prev(qk);
    double vm = 0.0, vpp = 0.0;
    if constexpr (NL && M == 4) {
      vm = adv_prev(vk);
      vpp = adv_next(adv_next(vk));
    }
    const bool per_lo = a.periodic && i == -1, per_hi = a.periodic && i == n;
    const bool recon = (i >= 0 && i < n) || per_lo || per_hi;
    // cell n-1 reads its right value at n, cell 0 its left value at 0
    vp = per_lo ? x : vp;
    const double vl = per_hi ? x : vk;
    double ac[4];
    if constexpr (NL) {
      adv_coeffs_nl<M>(qm, qk, qp, vl, vp, vm, vpp, dx, a.nl_lambda_c, a.nl_eps, ac);
    } else {
      adv_coeffs<M>(qm, qk, qp, vl, vp, ac);
    }
    double ms, ps, ss = 0.0;
    if constexpr (SRC) {
      ms = K0 * qk;
      ps = P0 * qk;
      ss = S0 * qk;
    } else {
      ms = qk;
      ps = qk;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      ms += ac[j] * Kin[j];
      ps += ac[j] * Pin[j];
      if constexpr (SRC) ss += ac[j] * Sin[j];
    }
    const bool ghost = !recon && (i == -1 || i == n);
    mean_s = recon ? ms : (ghost ? K0 * qk : 0.0);
    pt_s = recon ? ps : (ghost ? P0 * qk : 0.0);
    src_s = recon ? ss : 0.0;
  };
  auto update_run = [&](int base, double qk, double mean_s, double pt_s, double src_s) {
    const int i = base + lane - OFF;                      // this lane's cell
    const bool own = lane >= OFF && lane < OFF + RUN;     // updated by this run
    const double mean_u = pos ? adv_prev(mean_s) : adv_next(mean_s);
    const double pt_u = pos ? adv_prev(pt_s) : adv_next(pt_s);
    if (!own || i < 0 || i >= n) return;
    const double qc = qk;
    double qn;
    if (pos) {
      qn = qc - cn * (mean_s - mean_u);
      vout[i + 1] = pt_s;
      if (i == 0) vout[0] = pt_u;
    } else {
      qn = qc - cn * (mean_u - mean_s);
      vout[i] = pt_s;
      if (i == n - 1) vout[n] = pt_u;
    }
    if constexpr (SRC) qn -= zs * src_s;  // dt S^n_i, S = -kappa q
    qout[i] = qn;
    if (!isfinite(qn)) atomicOr(&ctl->err, ERR_NONPHYS);
  };
  // the step that only carries the state over (t has reached t_end)
  auto copy_run = [&](int base) {
    const int i = base + lane - OFF;
    const bool own = lane >= OFF && lane < OFF + RUN;
    if (!own || i < 0 || i >= n) return;
    qout[i] = qin[i];
    vout[i] = vin[i];
    if (i == n - 1) vout[n] = vin[n];
  };
  if constexpr (STEP == 2) {
  for (int blk = blockIdx.x; blk < 8 * per; blk += gridDim.x) {
  const int chunk = (blk % 8) * per + blk / 8;
  if (chunk >= nch) continue;
#pragma unroll
  for (int r = 0; r < PASSES; r += 2) {
    const int ba = chunk * CH + (r * 4 + wave) * RUN;  // first cell run r updates
    if (ba >= n) break;                                // uniform over the wave
    const int bb = ba + 4 * RUN;
    const bool has_b = bb < n;                         // uniform over the wave
    if (done) {
      copy_run(ba);
      if (has_b) copy_run(bb);
      continue;
    }
    double qa = 0.0, va = 0.0, xa = 0.0, qb = 0.0, vb = 0.0, xb = 0.0;
    load_run(ba, qa, va, xa);
    if (has_b) load_run(bb, qb, vb, xb);
    double ma, pa, sa, mb, pb, sb;
    recon_run(ba, qa, va, xa, ma, pa, sa);
    recon_run(bb, qb, vb, xb, mb, pb, sb);
    update_run(ba, qa, ma, pa, sa);
    if (has_b) update_run(bb, qb, mb, pb, sb);
  }
  }
  } else {
  // one run at a time
  for (int blk = blockIdx.x; blk < 8 * per; blk += gridDim.x) {
  const int chunk = (blk % 8) * per + blk / 8;
  if (chunk >= nch) continue;
#pragma unroll
  for (int r = 0; r < PASSES; ++r) {
    const int base = chunk * CH + (r * 4 + wave) * RUN;  // first cell the run updates
    if (base >= n) break;                                 // uniform over the wave
    const int i = base + lane - OFF;                      // this lane's cell
    const bool own = lane >= OFF && lane < OFF + RUN;     // updated by this run
    // Every lane within two cells of the domain holds the average of its cell
    // and the value at the cell's left interface (wrapped when periodic; the
    // ghost state beyond a transmissive end); a reconstruction takes its
    // neighbours' values from the adjacent lanes.
    // (cells -2 .. n+1 and interfaces -2 .. n+2 are what reconstructions of
    // cells -1 .. n read; a single +-n wrap keeps them in range for n >= 2)
    double qk = 0.0, vk = 0.0;
    if (i >= -2 && i <= n + 2) {
      qk = i <= n + 1 ? Q(i) : 0.0;
      vk = VG(i);
    }
    double qm = adv_prev(qk), qp = adv_next(qk), vp = adv_next(vk);
    double vm = 0.0, vpp = 0.0;
    if constexpr (NL && M == 4) {
      vm = adv_prev(vk);
      vpp = adv_next(adv_next(vk));
    }
    // the lane's flux mean over the swept interval and its datum; at i = -1
    // and i = n the upwind neighbour is the periodic image or the ghost cell
    // (a constant state: mean and point value are the end average, scaled by
    // the source's evolution of a constant)
    double mean_s = 0.0, pt_s = 0.0, src_s = 0.0;
    const bool recon = (i >= 0 && i < n) || (a.periodic && (i == -1 || i == n));
    if (!recon && (i == -1 || i == n)) {
      mean_s = K0 * qk;
      pt_s = P0 * qk;
    }
    // (lanes at the wave's edges reconstruct from shifted-in copies of their
    // own data; no updated lane reads their results)
    if (recon && !done) {
      // interfaces 0 and n of a periodic domain are one interface: cell n-1
      // reads its right value at n, cell 0 its left value at 0
      double vl = vk;
      if (a.periodic) {
        if (i == -1) vp = vin[n];
        if (i == n) vl = vin[0];
      }
      double ac[4];
      if constexpr (NL) {
        adv_coeffs_nl<M>(qm, qk, qp, vl, vp, vm, vpp, dx, a.nl_lambda_c, a.nl_eps, ac);
      } else {
        adv_coeffs<M>(qm, qk, qp, vl, vp, ac);
      }
      if constexpr (SRC) {
        mean_s = K0 * qk;
        pt_s = P0 * qk;
        src_s = S0 * qk;
      } else {
        mean_s = qk;
        pt_s = qk;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        mean_s += ac[j] * Kin[j];
        pt_s += ac[j] * Pin[j];
        if constexpr (SRC) src_s += ac[j] * Sin[j];
      }
    }
    const double mean_u = pos ? adv_prev(mean_s) : adv_next(mean_s);
    const double pt_u = pos ? adv_prev(pt_s) : adv_next(pt_s);
    if (!own || i < 0 || i >= n) continue;
    if (done) {
      qout[i] = qin[i];
      vout[i] = vin[i];
      if (i == n - 1) vout[n] = vin[n];
      continue;
    }
    const double qc = qk;
    double qn;
    if (pos) {
      qn = qc - cn * (mean_s - mean_u);
      vout[i + 1] = pt_s;
      if (i == 0) vout[0] = pt_u;
    } else {
      qn = qc - cn * (mean_u - mean_s);
      vout[i] = pt_s;
      if (i == n - 1) vout[n] = pt_u;
    }
    if constexpr (SRC) qn -= zs * src_s;  // dt S^n_i, S = -kappa q
    qout[i] = qn;
    if (!isfinite(qn)) atomicOr(&ctl->err, ERR_NONPHYS);
  }
  }
  }
  if (gid == 0) {
    a.seg.t[s1 * a.seg.S] = t_new;
    a.seg.smax[s1 * a.seg.S] = dbits(fabs(a.lambda));
    a.seg.smax[s2 * a.seg.S] = 0ull;
    if (t_new < t_end) atomicAdd(&ctl->active[s1], 1);
  }
}

// Per-step linear maps of the advection predictor with the implicit source
// (one thread): for the constant mode and each basis function phi_j the
// space-time DG predictor of q_t + lambda q_x = -kappa q is iterated to its
// fixed point (the linear flux makes it a fixed linear map of the data), then
//   src[j]             time mean of the upwind trace (the flux over lambda),
//   src[M+1+j]         the upwind trace at the end of the step (the datum),
//   src[2(M+1)+j]      the space-time mean (the source integral over -kappa).
// The upwind trace is the right one (xi = 1) for lambda > 0, else the left.
template <int M>
__global__ void adv_source_prep(AdvArgs<M> a) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  constexpr int N = M + 1;
  constexpr tab::Predictor<M> T = tab::predictor<M>();
  Ctl *ctl = a.ctl;
  const double dx = a.seg.dx[0];
  double dt, t_new;
  bool done;
  domain_dt(a.cfl, dx, fabs(a.lambda), a.seg.t[a.slot * a.seg.S], ctl->t_end, dt, t_new, done);
  const double cn = a.lambda * dt / dx;
  double A[N][N], c[N];
  source_time_mats<N>(T.K, T.w, T.l0, a.kappa * dt, A, c);
  const bool pos = a.lambda > 0.0;
  for (int j = 0; j <= M; ++j) {
    double w[N], q[N][N];
    for (int x = 0; x < N; ++x) {
      w[x] = j == 0 ? 1.0 : T.phi[x][j - 1];
      for (int b = 0; b < N; ++b) q[x][b] = w[x];
    }
    for (int it = 0; it < 200; ++it) {
      double qn[N][N], diff = 0.0, nrm = 0.0;
      for (int x = 0; x < N; ++x) {
        double Gd[N];
        for (int l = 0; l < N; ++l) {
          double g = 0.0;
          for (int k = 0; k < N; ++k) g = fma(T.D[x][k], q[k][l], g);
          Gd[l] = g;
        }
        for (int b = 0; b < N; ++b) {
          double acc = 0.0;
          for (int l = 0; l < N; ++l) acc = fma(A[b][l], Gd[l], acc);
          qn[x][b] = c[b] * w[x] - cn * acc;
          diff = fmax(diff, fabs(qn[x][b] - q[x][b]));
          nrm = fmax(nrm, fabs(qn[x][b]));
        }
      }
      for (int x = 0; x < N; ++x)
        for (int b = 0; b < N; ++b) q[x][b] = qn[x][b];
      if (diff <= 1e-17 * (1.0 + nrm)) break;
    }
    double fm = 0.0, end = 0.0, st = 0.0;
    for (int b = 0; b < N; ++b) {
      double tr = 0.0, row = 0.0;
      for (int x = 0; x < N; ++x) {
        tr = fma(pos ? T.l1[x] : T.l0[x], q[x][b], tr);
        row = fma(T.w[x], q[x][b], row);
      }
      fm = fma(T.w[b], tr, fm);
      end = fma(T.l1[b], tr, end);
      st = fma(T.w[b], row, st);
    }
    a.src[j] = fm;
    a.src[N + j] = end;
    a.src[2 * N + j] = st;
  }
}

// ============================================================ set-up kernels
// First-step interface data: the Riemann solution at x/t = 0 between the left
// (v0) and right (v1) limits of the initial condition; written into v0.
__global__ void init_interfaces_euler(double *v0, const double *v1, int ti, Gas G, int maxit,
                                      double tol, int datum, Ctl *ctl) {
  unsigned err = 0;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < ti; k += gridDim.x * blockDim.x) {
    double QL[3] = {v0[k], v0[ti + k], v0[2 * ti + k]};
    double QR[3] = {v1[k], v1[ti + k], v1[2 * ti + k]};
    RSOut o;
    err |= datum == 1 ? trrs_interact(G, QL, QR, o) : interact(G, QL, QR, 0.0, maxit, tol, o);
    v0[k] = o.Q[0];
    v0[ti + k] = o.Q[1];
    v0[2 * ti + k] = o.Q[2];
  }
  if (err) atomicOr(&ctl->err, err);
}

__global__ void init_interfaces_adv(double *v0, const double *v1, int ti, double lambda) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < ti; k += gridDim.x * blockDim.x)
    if (lambda < 0.0) v0[k] = v1[k];
}

// S_max over each domain's cells of the state in buffer `which` into slot.
__global__ __launch_bounds__(256) void domain_smax(const double *q, int tc, Seg seg, int slot, Gas G,
                                                   Ctl *ctl) {
  // cells are visited in order within a wave, so domains are non-decreasing
  const int stride = gridDim.x * blockDim.x;
  for (int base = blockIdx.x * blockDim.x; base < tc; base += stride) {
    const int c = base + threadIdx.x;
    int tag = -1;
    double sv = 0.0;
    if (c < tc) {
      tag = find_domain(seg.cell_off, c, 0, seg.S - 1);
      Prim W;
      if (to_prim(G, q[c], q[tc + c], q[2 * tc + c], W)) {
        sv = fabs(W.u) + W.c;
      } else {
        sv = __longlong_as_double(0x7ff8000000000000ll);
        atomicOr(&ctl->err, ERR_NONPHYS);
      }
    }
    wave_segmented_max(tag, sv, seg.smax + slot * seg.S);
  }
}

// Reset the control block and domain times.
__global__ void reset_ctl(Ctl *ctl, Seg seg, double t0, long long steps, int cur, double smax_const) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid == 0) {
    for (int k = 0; k < 3; ++k) {
      ctl->cur[k] = cur;
      ctl->active[k] = 0;
      ctl->steps[k] = steps;
    }
    ctl->err = 0;
    ctl->t_end = 0.0;
    for (int k = 0; k < 5; ++k) ctl->stat[k] = 0ull;
  }
  for (int s = gid; s < seg.S; s += gridDim.x * blockDim.x) {
    for (int k = 0; k < 3; ++k) {
      seg.t[k * seg.S + s] = t0;
      seg.smax[k * seg.S + s] = (k == 0 && smax_const > 0.0) ? dbits(smax_const) : 0ull;
    }
  }
}

// Before a run: set t_end and count active domains of the slot; clear the two
// following slots.  One block.
__global__ __launch_bounds__(256) void run_prologue(Ctl *ctl, Seg seg, int slot, double t_end) {
  __shared__ int cnt;
  const int s1 = (slot + 1) % 3, s2 = (slot + 2) % 3;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int local = 0;
  for (int s = threadIdx.x; s < seg.S; s += blockDim.x) {
    if (seg.t[slot * seg.S + s] < t_end) ++local;
    seg.smax[s1 * seg.S + s] = 0ull;
    seg.smax[s2 * seg.S + s] = 0ull;
  }
  atomicAdd(&cnt, local);
  __syncthreads();
  if (threadIdx.x == 0) {
    ctl->t_end = t_end;
    ctl->active[slot] = cnt;
    ctl->active[s1] = 0;
    ctl->active[s2] = 0;
  }
}

// Bitwise digest of a buffer (sum and xor of the 64-bit patterns).
__global__ void digest(const double *x, long long n, Ctl *ctl) {
  unsigned long long s = 0, xr = 0;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    unsigned long long b = dbits(x[k]);
    s += b * 0x9E3779B97F4A7C15ull + (unsigned long long)k;
    xr ^= b + 0x632BE59BD9B4E019ull * (unsigned long long)k;
  }
  s = wave_sum_u64(s);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) xr ^= __shfl_xor(xr, d, 64);
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&ctl->hash[0], s);
    atomicXor(&ctl->hash[1], xr);
  }
}
// ============================================================ launchers
template <int M>
hipError_t launch_adv(const AdvArgs<M> &a, int grid, bool nl, hipStream_t st) {
  (void)grid;
  const long long ch = nl ? 4LL * adv_passes<true>() * adv_run<M, true>()
                          : 4LL * adv_passes<false>() * adv_run<M, false>();
  const long long per = ((a.n + ch - 1) / ch + 7) / 8;
  const int g = (int)(8 * per < (1 << 20) ? 8 * per : (1 << 20));
  const bool pos = a.lambda > 0.0;
  if (a.src) {
    // the source's per-step maps first (stream order makes them visible)
    hipLaunchKernelGGL((adv_source_prep<M>), dim3(1), dim3(64), 0, st, a);
    if (nl) {
      if (pos) hipLaunchKernelGGL((adv_step<M, true, true, true>), dim3(g), dim3(256), 0, st, a);
      else hipLaunchKernelGGL((adv_step<M, true, true, false>), dim3(g), dim3(256), 0, st, a);
    } else {
      if (pos) hipLaunchKernelGGL((adv_step<M, false, true, true>), dim3(g), dim3(256), 0, st, a);
      else hipLaunchKernelGGL((adv_step<M, false, true, false>), dim3(g), dim3(256), 0, st, a);
    }
  } else if (nl) {
    if (pos) hipLaunchKernelGGL((adv_step<M, true, false, true>), dim3(g), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((adv_step<M, true, false, false>), dim3(g), dim3(256), 0, st, a);
  } else {
    if (pos) hipLaunchKernelGGL((adv_step<M, false, false, true>), dim3(g), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((adv_step<M, false, false, false>), dim3(g), dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

template hipError_t launch_adv<1>(const AdvArgs<1> &, int, bool, hipStream_t);
template hipError_t launch_adv<2>(const AdvArgs<2> &, int, bool, hipStream_t);
template hipError_t launch_adv<3>(const AdvArgs<3> &, int, bool, hipStream_t);
template hipError_t launch_adv<4>(const AdvArgs<4> &, int, bool, hipStream_t);

hipError_t launch_init_interfaces_euler(double *v0, const double *v1, int ti, const Gas &G, int maxit,
                                        double tol, int datum, Ctl *ctl, hipStream_t st) {
  int grid = (ti + 255) / 256;
  if (grid > 4096) grid = 4096;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(init_interfaces_euler, dim3(grid), dim3(256), 0, st, v0, v1, ti, G, maxit, tol, datum,
                     ctl);
  return hipGetLastError();
}

hipError_t launch_init_interfaces_adv(double *v0, const double *v1, int ti, double lambda,
                                      hipStream_t st) {
  int grid = (ti + 255) / 256;
  if (grid > 4096) grid = 4096;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(init_interfaces_adv, dim3(grid), dim3(256), 0, st, v0, v1, ti, lambda);
  return hipGetLastError();
}

hipError_t launch_domain_smax(const double *q, int tc, const Seg &seg, int slot, const Gas &G, Ctl *ctl,
                              hipStream_t st) {
  int grid = (tc + 255) / 256;
  if (grid > 8192) grid = 8192;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(domain_smax, dim3(grid), dim3(256), 0, st, q, tc, seg, slot, G, ctl);
  return hipGetLastError();
}

hipError_t launch_reset_ctl(Ctl *ctl, const Seg &seg, double t0, long long steps, int cur,
                            double smax_const, hipStream_t st) {
  int grid = (seg.S + 255) / 256;
  if (grid < 1) grid = 1;
  if (grid > 1024) grid = 1024;
  hipLaunchKernelGGL(reset_ctl, dim3(grid), dim3(256), 0, st, ctl, seg, t0, steps, cur, smax_const);
  return hipGetLastError();
}

hipError_t launch_run_prologue(Ctl *ctl, const Seg &seg, int slot, double t_end, hipStream_t st) {
  hipLaunchKernelGGL(run_prologue, dim3(1), dim3(256), 0, st, ctl, seg, slot, t_end);
  return hipGetLastError();
}

hipError_t launch_digest(const double *x, long long n, Ctl *ctl, hipStream_t st) {
  long long g = (n + 255) / 256;
  int grid = (int)(g > 2048 ? 2048 : (g < 1 ? 1 : g));
  hipLaunchKernelGGL(digest, dim3(grid), dim3(256), 0, st, x, n, ctl);
  return hipGetLastError();
}

}  // namespace grp
