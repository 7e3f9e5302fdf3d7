// grprec_euler.h -- the fused Euler step kernel of the GRPrec finite-volume
// scheme and its launch wrappers, as templates over the degree; each
// grprec_euler_m<M>.hip translation unit instantiates one degree.
//
// One launch advances every domain by one step:
//   dt from S_max (eq. dt-FV) -> GRPrec reconstruction (Sec. 3.1) -> DET
//   space-time predictor -> Riemann problems at the Gauss-Legendre times of the
//   flux integral (eq. numfluxes) and at tau = dt (next step's interface data)
//   -> conservative update (eq. eq_finite_volume) -> S_max of the new state.
// FP64 throughout; no matrix cores: the work is a per-cell stencil, not a
// dense contraction.
#pragma once

#include <hip/hip_runtime.h>

#include "grprec_device.h"
#include "grprec_internal.h"
#include "grprec_step_common.h"
#include "grprec_tables.h"

namespace grp {

// ============================================================ Euler step
// Waves per SIMD the register allocation must leave room for (1 = no limit):
// two up to order 3, whose kernels fit 256 registers per lane; order 4 and 5
// hold too many predictor unknowns for that.
#ifndef GRPREC_EULER_WAVES
#define GRPREC_EULER_WAVES(M) ((M) <= 2 ? 2 : 1)
#endif

// g = D f, the derivative at the nodes of the interpolant of nodal values f,
// through the even and odd parts of f about the centre (tab::Predictor's
// De, Do, Dm, Dc): 7 operations instead of 9 at N = 3, 20 instead of 25 at
// N = 5.  With the row sums of D zero, the even part's coefficients of one row
// sum to zero, which removes one term for even N (all of it at N = 2).
// With SCALE the result is c D f: the constants are multiplied by c (the
// products do not depend on f, so the compiler forms them once per cell).
template <int N, bool SCALE = false, class Tab>
__device__ __forceinline__ void deriv_sym(const Tab &T, const double (&f)[N], double (&g)[N],
                                          double c = 1.0) {
  constexpr int H = N / 2;
  auto k_ = [&](double v) { return SCALE ? c * v : v; };
  double s[H], d[H];
#pragma unroll
  for (int k = 0; k < H; ++k) {
    s[k] = f[k] + f[N - 1 - k];
    d[k] = f[k] - f[N - 1 - k];
  }
#pragma unroll
  for (int x = 0; x < H; ++x) {
    double o = k_(T.Do[x][0]) * d[0];
#pragma unroll
    for (int k = 1; k < H; ++k) o = fma(k_(T.Do[x][k]), d[k], o);
    if constexpr (N % 2 == 1) {
      double e = k_(T.Dm[x]) * f[H];
#pragma unroll
      for (int k = 0; k < H; ++k) e = fma(k_(T.De[x][k]), s[k], e);
      g[x] = o + e;
      g[N - 1 - x] = o - e;
    } else if constexpr (H > 1) {
      double e = k_(T.De[x][0]) * (s[0] - s[H - 1]);
#pragma unroll
      for (int k = 1; k < H - 1; ++k) e = fma(k_(T.De[x][k]), s[k] - s[H - 1], e);
      g[x] = o + e;
      g[N - 1 - x] = o - e;
    } else {
      g[x] = o;
      g[N - 1 - x] = o;
    }
  }
  if constexpr (N % 2 == 1) {
    double m = k_(T.Dc[0]) * d[0];
#pragma unroll
    for (int k = 1; k < H; ++k) m = fma(k_(T.Dc[k]), d[k], m);
    g[H] = m;
  }
}

template <bool B>
struct Flag {
  static constexpr bool value = B;
};

// AIR: gamma is 1.4 and the gas constants are compile-time values.
// NL: GRPrecNL reconstruction (Sec. 3.3-3.4) instead of GRPrec (Sec. 3.1).
// TR: end-of-step datum by the two-rarefaction solver (Sec. 4.1); a run-time
// branch in the Riemann loop would cost registers on every path.
// SRC: the linear relaxation source S(Q) = -kappa Q (eq. eq_finite_volume with
// S^n_i of eq. source): implicit in the predictor (time matrix K + z diag(w),
// z = kappa dt), the ghost states evolved by it, and dt S^n_i from the
// predicted space-time polynomial in the update.
template <int M, int B, bool AIR, bool NL, bool TR, bool SRC>
__global__ __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(GRPREC_EULER_WAVES(M))))
void euler_step(EulerArgs<M> a) {
  constexpr int N = M + 1;   // nodes per direction
  constexpr int NT = M + 2;  // trace times: N Gauss-Legendre times and tau = 1
  constexpr tab::Predictor<M> T = tab::predictor<M>();
  __shared__ double sTL[3 * NT][B];
  __shared__ double sTR[3 * NT][B];

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
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->cur[s1] = 1 - cur;
    ctl->steps[s1] = ctl->steps[slot] + 1;
    ctl->active[s2] = 0;
  }
  const double t_end = ctl->t_end;
  const bool stats = ctl->stats_on != 0;
  const Gas G = AIR ? kAir : a.gas;
  const int e = threadIdx.x;
  const int tc = a.tc, ti = a.ti;
  unsigned err = 0;
  unsigned st_rs = 0, st_newton = 0, st_sweeps = 0, st_cells = 0, st_mlp = 0;

  // this wave's words of a tile descriptor
  struct LaneTile {
    int start, count, cl, cr, w, base;
    unsigned long long first;
  };
  const int wj = (B > 64) ? (e >> 6) : 0;
  auto lane_tile = [&](int k) {
    const Tile *d = a.tiles + k;
    LaneTile r;
    r.start = d->start; r.count = d->count; r.cl = d->cl; r.cr = d->cr;
    r.w = d->w;
    r.base = d->base[wj];
    r.first = d->first[wj];
    return r;
  };
  // Which tiles this block takes.  Blocks are dispatched to the 8 XCDs
  // round-robin, so with a grid that is a multiple of 8 the tiles are split
  // into 8 contiguous ranges, one per XCD, and the XCD's blocks take its range
  // in turn: neighbouring tiles then run on one XCD and the cache lines their
  // halos share are fetched into that XCD's L2 once.  Otherwise the blocks
  // take the tiles in turn.
  int t_first = blockIdx.x, t_step = gridDim.x, t_last = a.ntiles;
  if ((gridDim.x & 7) == 0) {
    const int per = (a.ntiles + 7) >> 3, x = blockIdx.x & 7;
    t_first = x * per + (blockIdx.x >> 3);
    t_step = gridDim.x >> 3;
    t_last = min((x + 1) * per, a.ntiles);
  }
  // the next tile's descriptor is read one tile ahead
  LaneTile nx = {0, 0, -1, -1, 0, 0, 0ull};
  if (t_first < t_last) nx = lane_tile(t_first);
  // S_max of the new states: a tile's run maxima are compared with the
  // accumulating target, read at the end of the tile, at the head of the next
  // one, so that read's latency overlaps the next tile's own reads
  unsigned long long *const acc = a.seg.smax + s1 * a.seg.S;
  bool pend = false;
  int pseg = 0;
  unsigned long long pbits = 0, pseen = 0;

  for (int tile = t_first; tile < t_last; tile += t_step) {
    const LaneTile td = nx;
    if (tile + t_step < t_last) nx = lane_tile(tile + t_step);
    const int start = td.start, count = td.count;
    // ---- which slot this lane holds, and its domain.  Periodic runs (one
    // domain) index slots by cell.  Transmissive runs index them over each
    // domain's cells preceded by a ghost slot (slot off[s] + s of domain s,
    // the index of the domain's left interface), which solves the Riemann
    // problems of the left end like any interior slot solves those of its
    // right interface.
    bool valid = false, owned = false;
    int x = 0;
    if (e >= 1 && e <= count) {
      x = start + e - 1;
      valid = owned = true;
    } else if (e == 0) {
      x = td.cl;
      valid = x >= 0;
    } else if (e == count + 1) {
      x = td.cr;
      valid = x >= 0;
    }
    const int s = (e == count + 1) ? td.w : td.base + __popcll(td.first & ((2ull << (e & 63)) - 1ull));
    // every read of the slot depends on (x, s) alone, so they are issued
    // together; a ghost slot reads (and ignores) a neighbouring cell's data
    const int c = a.periodic ? x : max(x - s - 1, 0);
    int off = 0, n = 1, i = 0, io = 0;
    double dx = 1.0, dt = 0.0, t_new = 0.0, nu = 0.0, t = 0.0;
    bool done = true, ghost = false;
    double q0[3], vl0[3], vr0[3];
    if (valid) {
      off = a.seg.cell_off[s];
      n = a.seg.cell_off[s + 1] - off;
      dx = a.seg.dx[s];
      t = a.seg.t[slot * a.seg.S + s];
      const double S = bitsd(a.seg.smax[slot * a.seg.S + s]);
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        q0[v] = qin[v * tc + c];
        vl0[v] = vin[v * ti + c + s];
        vr0[v] = vin[v * ti + c + s + 1];
      }
      ghost = !a.periodic && x == off + s;
      i = ghost ? -1 : c - off;
      io = off + s;
      domain_dt(a.cfl, dx, S, t, t_end, dt, t_new, done);
      nu = dt / dx;
    }
    const bool useful = owned && !ghost;
    const bool work = valid && !done;
    // implicit source: the predictor's time matrices for this slot's dt, and
    // the factors of the constant-state evolution (ghost cells): gf[b] at the
    // time nodes, gf[N] at the end of the step
    double SA[SRC ? N : 1][SRC ? N : 1], gf[SRC ? N + 1 : 1];
    if constexpr (SRC) {
      double sc[N];
      source_time_mats<N>(T.K, T.w, T.l0, a.kappa * dt, SA, sc);
      double g1 = 0.0;
#pragma unroll
      for (int b = 0; b < N; ++b) {
        gf[b] = sc[b];
        g1 = fma(T.l1[b], sc[b], g1);
      }
      gf[N] = g1;
    }
    if (pend && pseen < pbits) atomicMax(acc + pseg, pbits);
    if (useful && !work) {  // a domain past its end time carries its data over
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        vout[v * ti + c + s + 1] = vr0[v];
        if (i == 0) vout[v * ti + c + s] = vl0[v];
      }
    }

    // ---- reconstruct, predict
    double src_dt[3] = {0.0, 0.0, 0.0};
    if (work && !ghost) {
      int im = i - 1, ip = i + 1;
      if (a.periodic) {
        if (im < 0) im += n;
        if (ip >= n) ip -= n;
      } else {
        if (im < 0) im = 0;
        if (ip >= n) ip = n - 1;
      }
      double w[3][N];
      if constexpr (NL) {
        // GRPrecNL in characteristic variables: differences of the stencil
        // data to the cell mean are projected with the left eigenvectors at
        // the cell mean, each field is reconstructed as a scalar, and the
        // coefficients are projected back
        double Lm[3][3], Rm[3][3];
        euler_eigen(G, q0, Lm, Rm);
        double dm[3] = {0.0, 0.0, 0.0}, dp[3] = {0.0, 0.0, 0.0}, dl[3], dr[3];
        double dll[3] = {0.0, 0.0, 0.0}, drr[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          if constexpr (M >= 2) {
            dm[v] = qin[v * tc + off + im] - q0[v];
            dp[v] = qin[v * tc + off + ip] - q0[v];
          }
          dl[v] = vl0[v] - q0[v];
          dr[v] = vr0[v] - q0[v];
          if constexpr (M == 4) {
            // V_{i-3/2} and V_{i+3/2}: wrapped when periodic; beyond a
            // transmissive end they belong to the ghost cell, a constant
            // state equal to the end average
            int kl = i - 1, kr = i + 2;
            double vll, vrr;
            if (a.periodic) {
              if (kl < 0) kl += n;
              if (kr > n) kr -= n;
              vll = vin[v * ti + io + kl];
              vrr = vin[v * ti + io + kr];
            } else {
              vll = kl >= 0 ? vin[v * ti + io + kl] : qin[v * tc + off];
              vrr = kr <= n ? vin[v * ti + io + kr] : qin[v * tc + off + n - 1];
            }
            dll[v] = vll - q0[v];
            drr[v] = vrr - q0[v];
          }
        }
        double ac[3][M];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
          double del[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int v = 0; v < 3; ++v) {
            del[0] = fma(Lm[f][v], dm[v], del[0]);
            del[2] = fma(Lm[f][v], dp[v], del[2]);
            del[3] = fma(Lm[f][v], dl[v], del[3]);
            del[4] = fma(Lm[f][v], dr[v], del[4]);
            if constexpr (M == 4) {
              del[5] = fma(Lm[f][v], dll[v], del[5]);
              del[6] = fma(Lm[f][v], drr[v], del[6]);
            }
          }
          double aC[M];
          grprec_from_diffs<M>(del[0], del[2], del[3], del[4], aC);
          nl_mix<M>(aC, del, dx, a.nl_lambda_c, a.nl_eps, ac[f]);
        }
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          double cv[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int j = 0; j < M; ++j)
            cv[j] = Rm[v][0] * ac[0][j] + Rm[v][1] * ac[1][j] + Rm[v][2] * ac[2][j];
#pragma unroll
          for (int k = 0; k < N; ++k)
            w[v][k] = q0[v] + cv[0] * T.phi[k][0] + cv[1] * T.phi[k][1] + cv[2] * T.phi[k][2] +
                      cv[3] * T.phi[k][3];
        }
      } else {
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        const double qc = q0[v];
        const double vl = vl0[v], vr = vr0[v];
        const double DI = vr - vl, SI = vl + vr - 2.0 * qc;
        double a1, a2 = 0.0, a3 = 0.0, a4 = 0.0;
        if (M == 1) {
          a1 = DI;
        } else if (M == 2) {
          a1 = DI;
          a2 = 3.0 * SI;
        } else {
          const double qm = qin[v * tc + off + im], qp = qin[v * tc + off + ip];
          const double DC = qp - qm, SC = qp + qm - 2.0 * qc;
          a1 = 1.25 * DI - 0.125 * DC;
          a3 = 0.5 * DC - DI;
          if (M == 3) {
            a2 = (3.0 * SI + 18.0 * SC) * (1.0 / 37.0);
          } else {
            a2 = 3.75 * SI - 0.125 * SC;
            a4 = (5.0 / 12.0) * SC - 2.5 * SI;
          }
        }
#pragma unroll
        for (int k = 0; k < N; ++k)
          w[v][k] = qc + a1 * T.phi[k][0] + a2 * T.phi[k][1] + a3 * T.phi[k][2] +
                    a4 * T.phi[k][3];
      }
      }
      // Picard iteration of the space-time Galerkin equations, from the data
      // held constant in time.  In the first sweep the nodal fluxes and their
      // space derivative therefore do not depend on the time node, and the
      // time solve reduces to the row sums of K^-1 W.  Its change is not
      // tested: it can only meet the tolerance when the flux gradient
      // vanishes, and then the second sweep reproduces it (and stops).
      double qh[3][N][N];
      // Up to N = 4 without the source, nu is folded into the derivative's
      // constants, so D F arrives scaled and each Picard update is N fused
      // multiply-adds (at N = 5 the twelve scaled constants would spill; the
      // source kernels keep the unscaled form).
      constexpr bool FOLD = (N <= 4) && !SRC;
      {
        double F1[3][N];
#pragma unroll
        for (int x = 0; x < N; ++x) euler_flux(G, w[0][x], w[1][x], w[2][x], F1[0][x], F1[1][x], F1[2][x]);
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          double Gd[N];
          if constexpr (FOLD) {
            deriv_sym<N, true>(T, F1[v], Gd, nu);
          } else {
            deriv_sym<N>(T, F1[v], Gd);
          }
#pragma unroll
          for (int x = 0; x < N; ++x) {
            double t;
            if constexpr (FOLD) {
              t = Gd[x];
            } else {
              t = nu * Gd[x];
            }
#pragma unroll
            for (int b = 0; b < N; ++b) {
              if constexpr (SRC) {
                double rs = 0.0;
#pragma unroll
                for (int l = 0; l < N; ++l) rs += SA[b][l];
                qh[v][x][b] = fma(-rs, t, gf[b] * w[v][x]);
              } else {
                qh[v][x][b] = fma(-T.KWs[b], t, w[v][x]);
              }
            }
          }
        }
      }
      // One sweep from qa into qb; with TEST, true when its change meets the
      // tolerance (without, the change is not formed).
      auto sweep = [&](const double (&qa)[3][N][N], double (&qb)[3][N][N], auto test) -> bool {
        constexpr bool TEST = decltype(test)::value;
        double F[3][N][N];
#pragma unroll
        for (int x = 0; x < N; ++x)
#pragma unroll
          for (int y = 0; y < N; ++y)
            euler_flux(G, qa[0][x][y], qa[1][x][y], qa[2][x][y], F[0][x][y], F[1][x][y], F[2][x][y]);
        double diff = 0.0, nrm = 0.0;
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          double Gd[N][N];  // [x][l]: space derivative at node x, time node l
#pragma unroll
          for (int l = 0; l < N; ++l) {
            double f[N], g[N];
#pragma unroll
            for (int k = 0; k < N; ++k) f[k] = F[v][k][l];
            if constexpr (FOLD) {
              deriv_sym<N, true>(T, f, g, nu);
            } else {
              deriv_sym<N>(T, f, g);
            }
#pragma unroll
            for (int x = 0; x < N; ++x) Gd[x][l] = g[x];
          }
#pragma unroll
          for (int x = 0; x < N; ++x) {
#pragma unroll
            for (int b = 0; b < N; ++b) {
              double acc = 0.0;
              double wb = w[v][x];
              if constexpr (SRC) {
#pragma unroll
                for (int l = 0; l < N; ++l) acc += SA[b][l] * Gd[x][l];
                wb *= gf[b];
              } else if constexpr (FOLD) {
#pragma unroll
                for (int l = 0; l < N; ++l) wb = fma(-T.KW[b][l], Gd[x][l], wb);
              } else {
#pragma unroll
                for (int l = 0; l < N; ++l) acc += T.KW[b][l] * Gd[x][l];
              }
              double nv;
              if constexpr (FOLD) {
                nv = wb;
              } else {
                nv = wb - nu * acc;
              }
              // non-finite values do not stop the sweep here: they reach the
              // traces and are caught by the physical-state checks
              if constexpr (TEST) {
                diff = fmax(diff, fabs(nv - qa[v][x][b]));
                nrm = fmax(nrm, fabs(nv));
              }
              qb[v][x][b] = nv;
            }
          }
        }
        return TEST && diff <= a.picard_tol * (1.0 + nrm);
      };
      // Later sweeps alternate between qh and qt (no register copies per
      // sweep); the iterate ends in qh.
      bool conv = false;
      int it = 1;
      if (a.max_picard <= 1) {  // a cap of one sweep: the first sweep's own test
        double diff = 0.0, nrm = 0.0;
#pragma unroll
        for (int v = 0; v < 3; ++v)
#pragma unroll
          for (int x = 0; x < N; ++x)
#pragma unroll
            for (int b = 0; b < N; ++b) {
              diff = fmax(diff, fabs(qh[v][x][b] - w[v][x]));
              nrm = fmax(nrm, fabs(qh[v][x][b]));
            }
        conv = diff <= a.picard_tol * (1.0 + nrm);
      }
      {
        double qt[3][N][N];
        if (N >= 3 && a.max_picard >= 3) {
          // The second sweep's change is not tested either: where it would
          // meet the tolerance the iteration has converged, the third sweep
          // changes the iterate by less again, and only the sweep count
          // differs from stopping at the second.
          sweep(qh, qt, Flag<false>{});
          conv = sweep(qt, qh, Flag<true>{});
          it = 3;
        }
        while (!conv && it < a.max_picard) {
          ++it;
          if (sweep(qh, qt, Flag<true>{})) {
            conv = true;
          } else if (it < a.max_picard) {
            ++it;
            conv = sweep(qt, qh, Flag<true>{});
            if (!conv) continue;
            break;
          }
#pragma unroll
          for (int v = 0; v < 3; ++v)
#pragma unroll
            for (int x = 0; x < N; ++x)
#pragma unroll
              for (int b = 0; b < N; ++b) qh[v][x][b] = qt[v][x][b];
          break;
        }
      }
      if (!conv) err |= ERR_PICARD;
      st_sweeps += conv ? it : a.max_picard;
      if constexpr (SRC) {  // dt S^n_i: Gauss-Legendre mean of -kappa q over the space-time cell
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          double acc = 0.0;
#pragma unroll
          for (int x = 0; x < N; ++x) {
            double row = 0.0;
#pragma unroll
            for (int b = 0; b < N; ++b) row = fma(T.w[b], qh[v][x][b], row);
            acc = fma(T.w[x], row, acc);
          }
          src_dt[v] = -(a.kappa * dt) * acc;
        }
      }
      st_cells += 1;
      // traces at xi = 0 and xi = 1, times g_b and 1 (the latter from the
      // former: evaluation in space and in time commute), staged in LDS
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        double l1sum = 0.0, r1sum = 0.0;
#pragma unroll
        for (int b = 0; b < N; ++b) {
          double l = 0.0, r = 0.0;
#pragma unroll
          for (int x = 0; x < N; ++x) {
            l += T.l0[x] * qh[v][x][b];
            r += T.l1[x] * qh[v][x][b];
          }
          sTL[v * NT + b][e] = l;
          sTR[v * NT + b][e] = r;
          l1sum = fma(T.l1[b], l, l1sum);
          r1sum = fma(T.l1[b], r, r1sum);
        }
        sTL[v * NT + N][e] = l1sum;
        sTR[v * NT + N][e] = r1sum;
      }
      // a domain's first cell gives its ghost slot the ghost state, the end
      // average (constant, or decaying with the source) at the trace times
      if (!a.periodic && i == 0 && e >= 1) {
#pragma unroll
        for (int b = 0; b < NT; ++b) {
          double f = 1.0;
          if constexpr (SRC) f = pick<N + 1>(gf, b);
#pragma unroll
          for (int v = 0; v < 3; ++v) sTR[v * NT + b][e - 1] = f * q0[v];
        }
      }
    }
    __syncthreads();

    // ---- interface x_{i+1/2}: Riemann problems at the trace times.  At a
    // transmissive end the outside data are a ghost cell holding the end
    // cell's average, constant in space and time.
    double FR[3] = {0.0, 0.0, 0.0}, VR[3] = {0.0, 0.0, 0.0};
    const bool rs_lane = work && (useful || ghost || e == 0);
    const bool boundary = (!a.periodic) && (i == n - 1);  // false for ghost slots (i = -1)
    const bool gated = a.warm || a.guess == 1;
    // data of the Riemann problem at trace time b: this slot's right trace
    // against the right neighbour's left trace (or the ghost state)
    auto load = [&](int b, double (&QL)[3], double (&QR)[3]) {
      QL[0] = sTR[0 * NT + b][e]; QL[1] = sTR[1 * NT + b][e]; QL[2] = sTR[2 * NT + b][e];
      if (boundary) {
        double f = 1.0;
        if constexpr (SRC) f = pick<N + 1>(gf, b);
        QR[0] = f * q0[0]; QR[1] = f * q0[1]; QR[2] = f * q0[2];
      } else {
        QR[0] = sTL[0 * NT + b][e + 1]; QR[1] = sTL[1 * NT + b][e + 1]; QR[2] = sTL[2 * NT + b][e + 1];
      }
    };
    // counts the solve, records it when harvesting, and adds the flux
    // sample or takes the datum
    auto take = [&](int b, const RSOut &o, const double (&QL)[3], const double (&QR)[3]) {
      st_mlp += o.learned ? 1 : 0;
      st_rs += 1;
      st_newton += o.iters;
      if (b == 0 && a.hv.ring != nullptr && useful) {
        unsigned long long k = atomicAdd(a.hv.count, 1ull);
        if ((long long)k < a.hv.cap) {
          Prim L, R;
          to_prim(G, QL[0], QL[1], QL[2], L);
          to_prim(G, QR[0], QR[1], QR[2], R);
          double *dst = a.hv.ring + 7 * k;
          dst[0] = L.r; dst[1] = L.u; dst[2] = L.p;
          dst[3] = R.r; dst[4] = R.u; dst[5] = R.p;
          dst[6] = o.pstar;
        }
      }
      if (b < N) {
        const double wb = pick<N>(T.w, b);
#pragma unroll
        for (int v = 0; v < 3; ++v) FR[v] += wb * o.F[v];
      } else {
#pragma unroll
        for (int v = 0; v < 3; ++v) VR[v] = o.Q[v];
      }
    };
    // The first time: the weak-wave solver.  With learned or warm starts on,
    // the problems it declines are tested against the gate (a problem it
    // takes is done in one Newton step from PVRS: no start would do better);
    // a negative gate takes the learned start for every problem.
    double QL0[3] = {1.0, 0.0, 1.0}, QR0[3] = {1.0, 0.0, 1.0};
    RSOut o0;
    bool fast0 = false, above0 = false;
    if (rs_lane) {
      load(0, QL0, QR0);
      const bool always = gated && a.gate < 0.0;
      fast0 = !always && weak_interact(G, QL0, QR0, a.newton_tol, o0);
      if (gated && !fast0) above0 = jump_exceeds_q(G, QL0, QR0, a.gate);
    }
    // learned starts of the interfaces above the gate, evaluated by the whole
    // wave (every lane is active here)
    double p_learn = 0.0;
    if (a.guess == 1 && __ballot(above0) != 0ull)
      p_learn = wave_learned_pressure(G.g, G.gm1, above0, QL0[0], QL0[1], QL0[2], QR0[0], QR0[1], QR0[2],
                                      a.mlp);
    if (rs_lane) {
      // The first time: the weak-wave solver's result, or where it declined
      // the general solver (a wave in which no lane declined skips that
      // code).  Above the gate the general solver starts from the learned
      // proposal, and the later times from the first time's star pressure
      // shifted by the change of the PVRS estimate; below it (and without
      // gating) every time starts from PVRS.
      RSOut og = o0;
      if (__builtin_expect(__ballot(!fast0) != 0ull, 0)) {
        if (!fast0) {
          err |= interact(G, QL0, QR0, p_learn, a.max_newton, a.newton_tol, og, nullptr, a.gate, gated);
          og.learned = og.strong && p_learn > 0.0;
        }
      }
      take(0, og, QL0, QR0);
      const double pg = og.strong ? og.pstar : 0.0, pvg = og.strong ? og.pv : 0.0;
      // The later times: the weak-wave solver in straight-line code (the
      // times are independent, and the unrolled loop gives the scheduler
      // that independent work), then the general solver for the problems it
      // declined.  A lane takes its results in the same order whatever the
      // other lanes of its wave do, so the results do not depend on the
      // tiling.
      unsigned slow = 0;
#pragma unroll
      for (int b = 1; b < NT; ++b) {
        double QL[3], QR[3];
        load(b, QL, QR);
        RSOut o;
        bool fast;
        if (TR && b == N) {  // end-of-step datum by the two-rarefaction solver
          err |= trrs_interact(G, QL, QR, o);
          fast = true;
        } else {
          fast = weak_interact(G, QL, QR, a.newton_tol, o);
        }
        if (fast) take(b, o, QL, QR);
        else slow |= 1u << b;
      }
      if (__builtin_expect(slow != 0, 0)) {
#pragma unroll
        for (int b = 1; b < NT; ++b) {
          if (!((slow >> b) & 1u)) continue;
          double QL[3], QR[3];
          load(b, QL, QR);
          RSOut o;
          err |= interact(G, QL, QR, pg, a.max_newton, a.newton_tol, o, nullptr, 0.0, false, pvg);
          take(b, o, QL, QR);
        }
      }
      // flux and datum go to the right neighbour through this slot's own
      // right-trace column, which no other thread reads
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        sTR[v][e] = FR[v];
        sTR[3 + v][e] = VR[v];
      }
    }
    double FL[3] = {0.0, 0.0, 0.0}, VL[3] = {0.0, 0.0, 0.0};
    __syncthreads();

    // ---- conservative update and S_max of the new state
    double smax_i = 0.0;
    int seg_tag = -1;
    if (useful) {
      double qn[3];
      if (work) {
        // the left interface's flux and datum: the left neighbour's, the
        // ghost slot's at a domain's left end
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          FL[v] = sTR[v][e - 1];
          VL[v] = sTR[3 + v][e - 1];
        }
#pragma unroll
        for (int v = 0; v < 3; ++v) qn[v] = q0[v] - nu * (FR[v] - FL[v]);
        if constexpr (SRC) {
#pragma unroll
          for (int v = 0; v < 3; ++v) qn[v] += src_dt[v];
        }
#pragma unroll
        for (int v = 0; v < 3; ++v) vout[v * ti + io + i + 1] = VR[v];
        if (i == 0) {
#pragma unroll
          for (int v = 0; v < 3; ++v) vout[v * ti + io] = VL[v];
        }
      } else {
#pragma unroll
        for (int v = 0; v < 3; ++v) qn[v] = q0[v];
      }
#pragma unroll
      for (int v = 0; v < 3; ++v) qout[v * tc + c] = qn[v];
      Prim W;
      if (!to_prim(G, qn[0], qn[1], qn[2], W)) {
        err |= ERR_NONPHYS;
        smax_i = __longlong_as_double(0x7ff8000000000000ll);
      } else {
        smax_i = fabs(W.u) + W.c;
      }
      seg_tag = s;
      if (i == 0) {  // one thread per domain owns its scalars
        a.seg.t[s1 * a.seg.S + s] = t_new;
        a.seg.smax[s2 * a.seg.S + s] = 0ull;
        if (t_new < t_end) atomicAdd(&ctl->active[s1], 1);
      }
    }
    pend = wave_segmented_lead(seg_tag, smax_i, pbits);
    pseg = seg_tag;
    pseen = pend ? __hip_atomic_load(acc + seg_tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : ~0ull;
    __syncthreads();
  }
  if (pend && pseen < pbits) atomicMax(acc + pseg, pbits);
  if (err) atomicOr(&ctl->err, err);
  if (stats) {
    const unsigned long long r0 = wave_sum_u64(st_rs), r1 = wave_sum_u64(st_newton),
                             r2 = wave_sum_u64(st_sweeps), r3 = wave_sum_u64(st_cells),
                             r4 = wave_sum_u64(st_mlp);
    if ((threadIdx.x & 63) == 0) {
      atomicAdd(&ctl->stat[0], r0);
      atomicAdd(&ctl->stat[1], r1);
      atomicAdd(&ctl->stat[2], r2);
      atomicAdd(&ctl->stat[3], r3);
      atomicAdd(&ctl->stat[4], r4);
    }
  }
}

// ============================================================ launchers
// (host-callable wrappers so that the API file needs no kernel templates)
// The source runs with GRPrec and the exact datum only (the host rejects the
// other combinations), which keeps the number of instantiations down.
template <int M, int B, bool NL>
static hipError_t launch_euler_mbn(const EulerArgs<M> &a, int grid, hipStream_t st) {
  if (a.gas.g == kGammaAir) {
    if (a.source) {
      if constexpr (!NL) hipLaunchKernelGGL((euler_step<M, B, true, false, false, true>), dim3(grid), dim3(B), 0, st, a);
    } else if (a.datum == 1) {
      hipLaunchKernelGGL((euler_step<M, B, true, NL, true, false>), dim3(grid), dim3(B), 0, st, a);
    } else {
      hipLaunchKernelGGL((euler_step<M, B, true, NL, false, false>), dim3(grid), dim3(B), 0, st, a);
    }
  } else {
    if (a.source) {
      if constexpr (!NL) hipLaunchKernelGGL((euler_step<M, B, false, false, false, true>), dim3(grid), dim3(B), 0, st, a);
    } else if (a.datum == 1) {
      hipLaunchKernelGGL((euler_step<M, B, false, NL, true, false>), dim3(grid), dim3(B), 0, st, a);
    } else {
      hipLaunchKernelGGL((euler_step<M, B, false, NL, false, false>), dim3(grid), dim3(B), 0, st, a);
    }
  }
  if (NL && a.source) return hipErrorInvalidValue;
  return hipGetLastError();
}

template <int M, int B>
static hipError_t launch_euler_mb(const EulerArgs<M> &a, int grid, bool nl, hipStream_t st) {
  return nl ? launch_euler_mbn<M, B, true>(a, grid, st) : launch_euler_mbn<M, B, false>(a, grid, st);
}

template <int M>
hipError_t launch_euler(const EulerArgs<M> &a, int block, int grid, bool nl, hipStream_t st) {
  switch (block) {
    case 64: return launch_euler_mb<M, 64>(a, grid, nl, st);
    case 128: return launch_euler_mb<M, 128>(a, grid, nl, st);
    case 256: return launch_euler_mb<M, 256>(a, grid, nl, st);
    default: return hipErrorInvalidValue;
  }
}

template <int M, int B>
static hipError_t euler_occ_b(bool nl, int *blocks_per_cu) {
  return nl ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, euler_step<M, B, true, true, false, false>, B, 0)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, euler_step<M, B, true, false, false, false>, B, 0);
}

template <int M>
hipError_t euler_occupancy(int block, bool nl, int *blocks_per_cu) {
  switch (block) {
    case 64: return euler_occ_b<M, 64>(nl, blocks_per_cu);
    case 128: return euler_occ_b<M, 128>(nl, blocks_per_cu);
    case 256: return euler_occ_b<M, 256>(nl, blocks_per_cu);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace grp
