// grprec_kernels.hip -- gfx950 kernels of the GRPrec finite-volume step.
//
// One launch advances every domain by one step:
//   dt from S_max (eq. dt-FV) -> GRPrec reconstruction (Sec. 3.1) -> DET
//   space-time predictor -> Riemann problems at the Gauss-Legendre times of the
//   flux integral (eq. numfluxes) and at tau = dt (next step's interface data)
//   -> conservative update (eq. eq_finite_volume) -> S_max of the new state.
// FP64 throughout; no matrix cores: the work is a per-cell stencil, not a
// dense contraction.
#include <hip/hip_runtime.h>

#include "grprec_device.h"
#include "grprec_internal.h"
#include "grprec_tables.h"

namespace grp {

// Per-domain step size from the slot's time and S_max: dt = cfl dx / S,
// clipped so that the domain lands exactly on t_end; dt = 0 for finished
// domains.
__device__ __forceinline__ void domain_dt(double cfl, double dx, double S, double t, double t_end,
                                          double &dt, double &t_new, bool &done) {
  // selects rather than branches: S is then read with the slot's other data
  // instead of behind the time test
  const double d = cfl * dx / S;
  done = !(t < t_end);
  const bool last = d >= t_end - t;
  dt = done ? 0.0 : (last ? t_end - t : d);
  t_new = done ? t : (last ? t_end : t + d);
}

// Step launched when no domain is active: carry the slot forward unchanged.
__device__ void carry_slot(const Seg &seg, Ctl *ctl, int slot) {
  const int s1 = (slot + 1) % 3, s2 = (slot + 2) % 3;
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid == 0) {
    ctl->cur[s1] = ctl->cur[slot];
    ctl->steps[s1] = ctl->steps[slot];
    ctl->active[s2] = 0;
  }
  for (int s = gid; s < seg.S; s += gridDim.x * blockDim.x) {
    seg.t[s1 * seg.S + s] = seg.t[slot * seg.S + s];
    seg.smax[s1 * seg.S + s] = seg.smax[slot * seg.S + s];
    seg.smax[s2 * seg.S + s] = 0ull;
  }
}

__device__ __forceinline__ int find_domain(const int *cell_off, int c, int lo, int hi) {
  // largest s in [lo, hi] with cell_off[s] <= c
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (cell_off[mid] <= c) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Element b of a small compile-time array with a uniform runtime index,
// as a chain of selects (no memory).
template <int N>
__device__ __forceinline__ double pick(const double (&t)[N], int b) {
  double r = t[0];
#pragma unroll
  for (int k = 1; k < N; ++k) r = (b == k) ? t[k] : r;
  return r;
}

// ============================================================ Euler step
// Waves per SIMD the register allocation must leave room for (1 = no limit):
// two up to order 3, whose kernels fit 256 registers per lane; order 4 and 5
// hold too many predictor unknowns for that.
#ifndef GRPREC_EULER_WAVES
#define GRPREC_EULER_WAVES(M) ((M) <= 2 ? 2 : 1)
#endif

// AIR: gamma is 1.4 and the gas constants are compile-time values.
// NL: GRPrecNL reconstruction (Sec. 3.3-3.4) instead of GRPrec (Sec. 3.1).
// TR: end-of-step datum by the two-rarefaction solver (Sec. 4.1); a run-time
// branch in the Riemann loop would cost registers on every path.
template <int M, int B, bool AIR, bool NL, bool TR>
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
  // the next tile's descriptor is read one tile ahead
  LaneTile nx = {0, 0, -1, -1, 0, 0, 0ull};
  if ((int)blockIdx.x < a.ntiles) nx = lane_tile(blockIdx.x);
  // S_max of the new states: a tile's run maxima are compared with the
  // accumulating target, read at the end of the tile, at the head of the next
  // one, so that read's latency overlaps the next tile's own reads
  unsigned long long *const acc = a.seg.smax + s1 * a.seg.S;
  bool pend = false;
  int pseg = 0;
  unsigned long long pbits = 0, pseen = 0;

  for (int tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    const LaneTile td = nx;
    if (tile + (int)gridDim.x < a.ntiles) nx = lane_tile(tile + gridDim.x);
    const int start = td.start, count = td.count;
    // ---- which cell this slot holds, and its domain
    bool valid = false, useful = false;
    int c = 0;
    if (e >= 1 && e <= count) {
      c = start + e - 1;
      valid = useful = true;
    } else if (e == 0) {
      c = td.cl;
      valid = c >= 0;
    } else if (e == count + 1) {
      c = td.cr;
      valid = c >= 0;
    }
    const int s = (e == count + 1) ? td.w : td.base + __popcll(td.first & ((2ull << (e & 63)) - 1ull));
    // every read of the slot depends on (c, s) alone, so they are issued together
    int off = 0, n = 1, i = 0, io = 0;
    double dx = 1.0, dt = 0.0, t_new = 0.0, nu = 0.0, t = 0.0;
    bool done = true;
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
      i = c - off;
      io = off + s;
      domain_dt(a.cfl, dx, S, t, t_end, dt, t_new, done);
      nu = dt / dx;
    }
    const bool work = valid && !done;
    if (pend && pseen < pbits) atomicMax(acc + pseg, pbits);
    if (useful && !work) {  // a domain past its end time carries its data over
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        vout[v * ti + c + s + 1] = vr0[v];
        if (i == 0) vout[v * ti + c + s] = vl0[v];
      }
    }

    // ---- reconstruct, predict
    if (work) {
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
      // time solve reduces to the row sums of K^-1 W.
      double qh[3][N][N];
      bool conv = false;
      int it = 1;
      {
        double F1[3][N];
#pragma unroll
        for (int x = 0; x < N; ++x) euler_flux(G, w[0][x], w[1][x], w[2][x], F1[0][x], F1[1][x], F1[2][x]);
        double diff = 0.0, nrm = 0.0;
#pragma unroll
        for (int v = 0; v < 3; ++v) {
#pragma unroll
          for (int x = 0; x < N; ++x) {
            double Gd = 0.0;
#pragma unroll
            for (int k = 0; k < N; ++k) Gd += T.D[x][k] * F1[v][k];
#pragma unroll
            for (int b = 0; b < N; ++b) {
              const double nv = w[v][x] - nu * (T.KWs[b] * Gd);
              diff = fmax(diff, fabs(nv - w[v][x]));
              nrm = fmax(nrm, fabs(nv));
              qh[v][x][b] = nv;
            }
          }
        }
        conv = diff <= a.picard_tol * (1.0 + nrm);
      }
      if (!conv) for (it = 2; it <= a.max_picard; ++it) {
        double F[3][N][N];
#pragma unroll
        for (int x = 0; x < N; ++x)
#pragma unroll
          for (int y = 0; y < N; ++y)
            euler_flux(G, qh[0][x][y], qh[1][x][y], qh[2][x][y], F[0][x][y], F[1][x][y], F[2][x][y]);
        double diff = 0.0, nrm = 0.0;
#pragma unroll
        for (int v = 0; v < 3; ++v) {
#pragma unroll
          for (int x = 0; x < N; ++x) {
            double Gd[N];
#pragma unroll
            for (int l = 0; l < N; ++l) {
              double acc = 0.0;
#pragma unroll
              for (int k = 0; k < N; ++k) acc += T.D[x][k] * F[v][k][l];
              Gd[l] = acc;
            }
#pragma unroll
            for (int b = 0; b < N; ++b) {
              double acc = 0.0;
#pragma unroll
              for (int l = 0; l < N; ++l) acc += T.KW[b][l] * Gd[l];
              const double nv = w[v][x] - nu * acc;
              // non-finite values do not stop the sweep here: they reach the
              // traces and are caught by the physical-state checks
              diff = fmax(diff, fabs(nv - qh[v][x][b]));
              nrm = fmax(nrm, fabs(nv));
              qh[v][x][b] = nv;
            }
          }
        }
        if (diff <= a.picard_tol * (1.0 + nrm)) {
          conv = true;
          break;
        }
      }
      if (!conv) err |= ERR_PICARD;
      st_sweeps += conv ? it : a.max_picard;
      st_cells += 1;
      // traces at xi = 0 and xi = 1, times g_b and 1, staged in LDS
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
        }
#pragma unroll
        for (int x = 0; x < N; ++x) {
          double at1 = 0.0;
#pragma unroll
          for (int b = 0; b < N; ++b) at1 += T.l1[b] * qh[v][x][b];
          l1sum += T.l0[x] * at1;
          r1sum += T.l1[x] * at1;
        }
        sTL[v * NT + N][e] = l1sum;
        sTR[v * NT + N][e] = r1sum;
      }
    }
    __syncthreads();

    // ---- interface x_{i+1/2}: Riemann problems at the trace times.  At a
    // transmissive end the outside data are a ghost cell holding the end
    // cell's average, constant in space and time.
    double FR[3] = {0.0, 0.0, 0.0}, VR[3] = {0.0, 0.0, 0.0};
    if (work && (useful || e == 0)) {
      const bool boundary = (!a.periodic) && (i == n - 1);
      // Riemann problem at trace time b with Newton start pguess (0: PVRS),
      // optionally testing the gate (learned start when mlp != nullptr);
      // adds the flux sample or takes the datum
      auto solve = [&](int b, double pguess, const float *mlp, bool test_gate) -> RSOut {
        double QL[3] = {sTR[0 * NT + b][e], sTR[1 * NT + b][e], sTR[2 * NT + b][e]};
        double QR[3];
        if (boundary) {
          QR[0] = q0[0]; QR[1] = q0[1]; QR[2] = q0[2];
        } else {
          QR[0] = sTL[0 * NT + b][e + 1]; QR[1] = sTL[1 * NT + b][e + 1]; QR[2] = sTL[2 * NT + b][e + 1];
        }
        RSOut o;
        if (TR && b == N)  // end-of-step datum by the two-rarefaction solver
          err |= trrs_interact(G, QL, QR, o);
        else
          err |= interact(G, QL, QR, pguess, a.max_newton, a.newton_tol, o, mlp, a.gate, test_gate);
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
        return o;
      };
      // With gating (learned or warm starts) the first time tests the
      // interface's jump against the gate; above it the first time starts from
      // the learned proposal and the later times from the first time's star
      // pressure, below it (and without gating) every time starts from PVRS.
      // The later times are independent of each other, and the unrolled loop
      // gives the scheduler that independent work.
      const bool gated = a.warm || a.guess == 1;
      const RSOut o0 = solve(0, 0.0, (gated && a.guess == 1) ? a.mlp : nullptr, gated);
      const double pg = o0.strong ? o0.pstar : 0.0;
#pragma unroll
      for (int b = 1; b < NT; ++b) (void)solve(b, pg, nullptr, false);
      // flux and datum go to the right neighbour through this slot's own
      // right-trace column, which no other thread reads
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        sTR[v][e] = FR[v];
        sTR[3 + v][e] = VR[v];
      }
    }
    // left end of a transmissive domain: ghost average against the left trace
    double FL[3] = {0.0, 0.0, 0.0}, VL[3] = {0.0, 0.0, 0.0};
    if (work && useful && i == 0 && !a.periodic) {
      const bool gated = a.warm || a.guess == 1;
      double pw = 0.0;
      bool strong = false;
#pragma unroll 1
      for (int b = 0; b < NT; ++b) {
        double QR[3] = {sTL[0 * NT + b][e], sTL[1 * NT + b][e], sTL[2 * NT + b][e]};
        const float *mlp = (b == 0 && a.guess == 1) ? a.mlp : nullptr;
        RSOut o;
        if (TR && b == N)  // end-of-step datum by the two-rarefaction solver
          err |= trrs_interact(G, q0, QR, o);
        else
          err |= interact(G, q0, QR, (b > 0 && strong) ? pw : 0.0, a.max_newton, a.newton_tol, o,
                          mlp, a.gate, b == 0 && gated);
        if (b == 0) {  // later times start from the first time's p* above the gate
          strong = o.strong;
          pw = o.pstar;
        }
        st_mlp += o.learned ? 1 : 0;
        st_rs += 1;
        st_newton += o.iters;
        if (b < N) {
          const double wb = pick<N>(T.w, b);
#pragma unroll
          for (int v = 0; v < 3; ++v) FL[v] += wb * o.F[v];
        } else {
#pragma unroll
          for (int v = 0; v < 3; ++v) VL[v] = o.Q[v];
        }
      }
    }
    __syncthreads();

    // ---- conservative update and S_max of the new state
    double smax_i = 0.0;
    int seg_tag = -1;
    if (useful) {
      double qn[3];
      if (work) {
        if (i > 0 || a.periodic) {
#pragma unroll
          for (int v = 0; v < 3; ++v) {
            FL[v] = sTR[v][e - 1];
            VL[v] = sTR[3 + v][e - 1];
          }
        }
#pragma unroll
        for (int v = 0; v < 3; ++v) qn[v] = q0[v] - nu * (FR[v] - FL[v]);
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

#ifndef ADV_PASSES
#define ADV_PASSES 4  // runs per wave per block chunk (4 measured best of 1, 2, 4, 6, 8)
#endif
#define ADV_RUN 63    // cells a wave updates per run (64 lanes, one upwind overlap)

template <int M, bool NL>
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
  const bool pos = a.lambda > 0.0;
  // per-step constants: mean of each basis function over the swept interval
  // and its value at the foot of the characteristic
  double Kin[4], Pin[4];
  if (pos) {
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
  // A wave advances runs of ADV_RUN = 63 consecutive cells.  Its 64th lane
  // holds the run's upwind neighbour (lane 0 for lambda > 0, lane 63 for
  // lambda < 0), so every lane reconstructs one cell and the upwind lane's
  // flux mean and end-of-step datum reach the next lane by a lane shift.  A block
  // takes chunks of 4 waves x ADV_PASSES runs.  Blocks are dispatched to the 8
  // XCDs round-robin, so block b works on chunk (b % 8) * per + b / 8:
  // consecutive chunks run on one XCD and the cache lines they share at their
  // ends are read once through its L2.
  constexpr int RUN = ADV_RUN;
  constexpr int CH = 4 * ADV_PASSES * RUN;
  const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
  const int nch = (n + CH - 1) / CH;
  const int per = (nch + 7) / 8;
  for (int blk = blockIdx.x; blk < 8 * per; blk += gridDim.x) {
  const int chunk = (blk % 8) * per + blk / 8;
  if (chunk >= nch) continue;
#pragma unroll
  for (int r = 0; r < ADV_PASSES; ++r) {
    const int base = chunk * CH + (r * 4 + wave) * RUN;  // first cell the run updates
    if (base >= n) break;                                 // uniform over the wave
    const int i = pos ? base + lane - 1 : base + lane;    // this lane's cell
    const bool own = pos ? lane >= 1 : lane < RUN;        // updated by this run
    // Every lane within two cells of the domain holds the average of its cell
    // and the value at the cell's left interface (wrapped when periodic; the
    // ghost state beyond a transmissive end); a reconstruction takes its
    // neighbours' values from the adjacent lanes, and only the wave's edge
    // lanes load theirs.
    // (cells -2 .. n+1 and interfaces -2 .. n+2 are what reconstructions of
    // cells -1 .. n read; a single +-n wrap keeps them in range for n >= 2)
    double qk = 0.0, vk = 0.0;
    if (i >= -2 && i <= n + 2) {
      qk = i <= n + 1 ? Q(i) : 0.0;
      vk = VG(i);
    }
    double qm = wave_prev(qk), qp = wave_next(qk), vp = wave_next(vk);
    double vm = 0.0, vpp = 0.0;
    if constexpr (NL && M == 4) {
      vm = wave_prev(vk);
      vpp = wave_next(wave_next(vk));
    }
    // the lane's flux mean over the swept interval and its datum; at i = -1
    // and i = n the upwind neighbour is the periodic image or the ghost cell
    // (a constant state: mean and point value are the end average)
    double mean_s = 0.0, pt_s = 0.0;
    const bool recon = (i >= 0 && i < n) || (a.periodic && (i == -1 || i == n));
    if (!recon && (i == -1 || i == n)) mean_s = pt_s = qk;
    if (recon && !done) {
      if (lane == 0) {
        qm = Q(i - 1);
        if constexpr (NL && M == 4) vm = VG(i - 1);
      }
      if (lane == 63) {
        qp = Q(i + 1);
        vp = VG(i + 1);
      }
      if constexpr (NL && M == 4) {
        if (lane >= 62) vpp = VG(i + 2);
      }
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
      mean_s = qk;
      pt_s = qk;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        mean_s += ac[j] * Kin[j];
        pt_s += ac[j] * Pin[j];
      }
    }
    const double mean_u = pos ? wave_prev(mean_s) : wave_next(mean_s);
    const double pt_u = pos ? wave_prev(pt_s) : wave_next(pt_s);
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
    qout[i] = qn;
    if (!isfinite(qn)) atomicOr(&ctl->err, ERR_NONPHYS);
  }
  }
  if (gid == 0) {
    a.seg.t[s1 * a.seg.S] = t_new;
    a.seg.smax[s1 * a.seg.S] = dbits(fabs(a.lambda));
    a.seg.smax[s2 * a.seg.S] = 0ull;
    if (t_new < t_end) atomicAdd(&ctl->active[s1], 1);
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
// (host-callable wrappers so that the API file needs no kernel templates)
template <int M, int B, bool NL>
static hipError_t launch_euler_mbn(const EulerArgs<M> &a, int grid, hipStream_t st) {
  if (a.gas.g == kGammaAir) {
    if (a.datum == 1) hipLaunchKernelGGL((euler_step<M, B, true, NL, true>), dim3(grid), dim3(B), 0, st, a);
    else hipLaunchKernelGGL((euler_step<M, B, true, NL, false>), dim3(grid), dim3(B), 0, st, a);
  } else {
    if (a.datum == 1) hipLaunchKernelGGL((euler_step<M, B, false, NL, true>), dim3(grid), dim3(B), 0, st, a);
    else hipLaunchKernelGGL((euler_step<M, B, false, NL, false>), dim3(grid), dim3(B), 0, st, a);
  }
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
  return nl ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, euler_step<M, B, true, true, false>, B, 0)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, euler_step<M, B, true, false, false>, B, 0);
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

template <int M>
hipError_t launch_adv(const AdvArgs<M> &a, int grid, bool nl, hipStream_t st) {
  (void)grid;
  const long long ch = 4LL * ADV_PASSES * ADV_RUN;
  const long long per = ((a.n + ch - 1) / ch + 7) / 8;
  const int g = (int)(8 * per < (1 << 20) ? 8 * per : (1 << 20));
  if (nl)
    hipLaunchKernelGGL((adv_step<M, true>), dim3(g), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((adv_step<M, false>), dim3(g), dim3(256), 0, st, a);
  return hipGetLastError();
}

template hipError_t launch_euler<1>(const EulerArgs<1> &, int, int, bool, hipStream_t);
template hipError_t launch_euler<2>(const EulerArgs<2> &, int, int, bool, hipStream_t);
template hipError_t launch_euler<3>(const EulerArgs<3> &, int, int, bool, hipStream_t);
template hipError_t launch_euler<4>(const EulerArgs<4> &, int, int, bool, hipStream_t);
template hipError_t euler_occupancy<1>(int, bool, int *);
template hipError_t euler_occupancy<2>(int, bool, int *);
template hipError_t euler_occupancy<3>(int, bool, int *);
template hipError_t euler_occupancy<4>(int, bool, int *);
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
