// grprec_device.h -- device functions of the GRPrec step for gfx950 (wave64, FP64).
#pragma once

#include <hip/hip_runtime.h>

#include "grprec_internal.h"

namespace grp {

__device__ __forceinline__ unsigned long long dbits(double x) {
  return (unsigned long long)__double_as_longlong(x);
}
__device__ __forceinline__ double bitsd(unsigned long long b) {
  return __longlong_as_double((long long)b);
}

// Largest of a and b, NaN wins (so a NaN reaches the error checks).
__device__ __forceinline__ double nanmax(double a, double b) { return (b > a || b != b) ? b : a; }

// x^e for x > 0 as 2^(e log2 x): a few ulp, cheaper than a general pow.
__device__ __forceinline__ double powpos(double x, double e) { return exp2(e * log2(x)); }

// ---------------------------------------------------------------- reductions
// Per-domain maximum over one wave: lanes hold (seg, val) with seg
// non-decreasing over the lanes that take part (seg >= 0); the first lane of
// each run of equal seg does one atomicMax on base[seg].  Values are
// non-negative doubles, whose bit patterns order like the values.
__device__ __forceinline__ void wave_segmented_max(int seg, double val, unsigned long long *base) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    double ov = __shfl_down(val, d, 64);
    int os = __shfl_down(seg, d, 64);
    if (lane + d < 64 && os == seg) val = nanmax(val, ov);
  }
  int prev = __shfl_up(seg, 1, 64);
  if (seg >= 0 && (lane == 0 || prev != seg)) atomicMax(base + seg, dbits(val));
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// ---------------------------------------------------------------- Euler physics
// Conserved Q = (rho, rho u, E), ideal gas p = (g-1)(E - rho u^2 / 2).
__device__ __forceinline__ void euler_flux(const Gas &G, double r, double m, double E, double &f0,
                                           double &f1, double &f2) {
  double u = m / r;
  double p = G.gm1 * (E - 0.5 * m * u);
  f0 = m;
  f1 = m * u + p;
  f2 = u * (E + p);
}

// Star-region pressure function of one side and its derivative (shock branch
// from the Rankine-Hugoniot conditions, rarefaction branch from the isentropic
// relation and the generalised Riemann invariant).
__device__ __forceinline__ void side_function(const Gas &G, double p, double rk, double pk, double ck,
                                              double &f, double &fd) {
  if (p <= pk) {
    double pr = p / pk;
    double pw = powpos(pr, G.z);
    f = G.two_gm1 * ck * (pw - 1.0);
    fd = pw / (pr * rk * ck);
  } else {
    double ak = G.two_gp1 / rk;
    double bk = G.gm1_gp1 * pk;
    double s = sqrt(ak / (bk + p));
    f = (p - pk) * s;
    fd = (1.0 - 0.5 * (p - pk) / (bk + p)) * s;
  }
}

struct Prim {
  double r, u, p, c;
};

// Primitive state and sound speed; false if not physical.
__device__ __forceinline__ bool to_prim(const Gas &G, double r, double m, double E, Prim &w) {
  w.r = r;
  w.u = m / r;
  w.p = G.gm1 * (E - 0.5 * m * w.u);
  bool ok = (r > 0.0) && (w.p > 0.0) && isfinite(w.u) && isfinite(w.p);
  w.c = ok ? sqrt(G.g * w.p / r) : 0.0;
  return ok;
}

__device__ __forceinline__ double pvrs(const Prim &L, const Prim &R) {
  double ppv = 0.5 * (L.p + R.p) - 0.125 * (R.u - L.u) * (L.r + R.r) * (L.c + R.c);
  double fl = 1e-6 * fmin(L.p, R.p);
  return ppv > fl ? ppv : fl;
}

// Newton iteration for the star pressure from p0 > 0; non-positive iterates
// are replaced by half the previous one; stop on relative change <= tol after
// at least one iteration.  Returns the iteration count (maxit+1 = no convergence).
__device__ __forceinline__ int newton_pstar(const Gas &G, const Prim &L, const Prim &R, double p,
                                            int maxit, double tol, double &pstar, double &ustar) {
  const double du = R.u - L.u;
  int k = 1;
  bool conv = false;
  for (; k <= maxit; ++k) {
    double fl, fld, fr, frd;
    side_function(G, p, L.r, L.p, L.c, fl, fld);
    side_function(G, p, R.r, R.p, R.c, fr, frd);
    double pn = p - (fl + fr + du) / (fld + frd);
    if (pn <= 0.0) pn = 0.5 * p;
    double change = 2.0 * fabs(pn - p) / (pn + p);
    p = pn;
    if (change <= tol) {
      conv = true;
      break;
    }
  }
  double fl, fld, fr, frd;
  side_function(G, p, L.r, L.p, L.c, fl, fld);
  side_function(G, p, R.r, R.p, R.c, fr, frd);
  pstar = p;
  ustar = 0.5 * (L.u + R.u) + 0.5 * (fr - fl);
  return conv ? k : maxit + 1;
}

// State of the exact Riemann solution on the line x/t = 0 (primitive).
__device__ __forceinline__ void sample_at_zero(const Gas &G, const Prim &L, const Prim &R, double ps,
                                               double us, double &r, double &u, double &p) {
  if (us >= 0.0) {
    if (ps <= L.p) {  // left rarefaction
      if (L.u - L.c >= 0.0) {
        r = L.r; u = L.u; p = L.p;
      } else {
        double prat = ps / L.p;
        double cs = L.c * powpos(prat, G.z);
        if (us - cs < 0.0) {
          r = L.r * powpos(prat, G.inv_g); u = us; p = ps;
        } else {  // fan: u - c = 0 and u + 2c/(g-1) is carried from the left
          double c = G.two_gp1 * (L.c + 0.5 * G.gm1 * L.u);
          double cr = c / L.c;
          r = L.r * powpos(cr, G.two_gm1);
          u = c;
          p = L.p * powpos(cr, G.twog_gm1);
        }
      }
    } else {  // left shock
      double pm = ps / L.p;
      double s = L.u - L.c * sqrt(G.gp1_2g * pm + 0.5 * G.gm1 * G.inv_g);
      if (s >= 0.0) {
        r = L.r; u = L.u; p = L.p;
      } else {
        r = L.r * (pm + G.gm1_gp1) / (pm * G.gm1_gp1 + 1.0); u = us; p = ps;
      }
    }
  } else {
    if (ps > R.p) {  // right shock
      double pm = ps / R.p;
      double s = R.u + R.c * sqrt(G.gp1_2g * pm + 0.5 * G.gm1 * G.inv_g);
      if (s <= 0.0) {
        r = R.r; u = R.u; p = R.p;
      } else {
        r = R.r * (pm + G.gm1_gp1) / (pm * G.gm1_gp1 + 1.0); u = us; p = ps;
      }
    } else {  // right rarefaction
      if (R.u + R.c <= 0.0) {
        r = R.r; u = R.u; p = R.p;
      } else {
        double prat = ps / R.p;
        double cs = R.c * powpos(prat, G.z);
        if (us + cs >= 0.0) {
          r = R.r * powpos(prat, G.inv_g); u = us; p = ps;
        } else {  // fan: u + c = 0 and u - 2c/(g-1) is carried from the right
          double c = G.two_gp1 * (R.c - 0.5 * G.gm1 * R.u);
          double cr = c / R.c;
          r = R.r * powpos(cr, G.two_gm1);
          u = -c;
          p = R.p * powpos(cr, G.twog_gm1);
        }
      }
    }
  }
}

// ---------------------------------------------------------------- learned guess
// 6 -> 32 -> 32 -> 1 tanh network, float32.  Weights are read with uniform
// (wave-wide) addresses, so they arrive through the scalar cache.
__device__ __forceinline__ float mlp_tanh(float x) {
  // tanh(x) = 1 - 2 / (exp(2x) + 1), saturating cleanly for large |x|
  float e = __expf(2.0f * x);
  return 1.0f - 2.0f / (e + 1.0f);
}

__device__ __forceinline__ void mlp_features(const Gas &G, const Prim &L, const Prim &R, float x[6],
                                             double &pbar) {
  double rbar = 0.5 * (L.r + R.r);
  pbar = 0.5 * (L.p + R.p);
  double cbar = sqrt(G.g * pbar / rbar);
  x[0] = (float)log(L.r / rbar);
  x[1] = (float)log(R.r / rbar);
  x[2] = (float)log(L.p / pbar);
  x[3] = (float)log(R.p / pbar);
  x[4] = (float)(L.u / cbar);
  x[5] = (float)(R.u / cbar);
}

__device__ __forceinline__ float mlp_eval(const float *__restrict__ P, const float xin[6]) {
  const float *W1 = P, *b1 = P + 192, *W2 = P + 224, *b2 = P + 1248, *W3 = P + 1280, *b3 = P + 1312;
  const float *mean = P + 1313, *stdv = P + 1319;
  float x[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) x[i] = (xin[i] - mean[i]) / stdv[i];
  float h1[32];
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    float a = b1[j];
#pragma unroll
    for (int i = 0; i < 6; ++i) a = fmaf(W1[j * 6 + i], x[i], a);
    h1[j] = mlp_tanh(a);
  }
  float y = b3[0];
#pragma unroll 4
  for (int j = 0; j < 32; ++j) {
    float a = b2[j];
#pragma unroll
    for (int i = 0; i < 32; ++i) a = fmaf(W2[j * 32 + i], h1[i], a);
    y = fmaf(W3[j], mlp_tanh(a), y);
  }
  return y;
}

// Starting pressure: learned proposal when asked for and the data jump is
// large (relative jump above the gate), else PVRS.  A non-finite or
// non-positive proposal falls back to PVRS.
__device__ __forceinline__ double start_pressure(const Gas &G, const Prim &L, const Prim &R, int guess,
                                                 double gate, const float *mlp, bool &used_mlp) {
  used_mlp = false;
  double pv = pvrs(L, R);
  if (guess == 1 && mlp != nullptr) {
    double pbar = 0.5 * (L.p + R.p);
    double rbar = 0.5 * (L.r + R.r);
    double cbar = sqrt(G.g * pbar / rbar);
    double jump = fabs(R.p - L.p) / pbar + fabs(R.r - L.r) / rbar + fabs(R.u - L.u) / cbar;
    if (gate < 0.0 || jump > gate) {
      float x[6];
      double pb;
      mlp_features(G, L, R, x, pb);
      float y = mlp_eval(mlp, x);
      double p0 = pb * exp((double)y);
      if (p0 > 0.0 && isfinite(p0)) {
        used_mlp = true;
        return p0;
      }
    }
  }
  return pv;
}

// Full interface interaction: exact Riemann solution at x/t = 0 between two
// conserved states; returns error bits, the physical flux there and the state.
// pguess > 0 overrides the start value (warm start).
struct RSOut {
  double F[3];
  double Q[3];
  double pstar;
  int iters;
  bool mlp;
};

__device__ __forceinline__ unsigned interact(const Gas &G, const double QL[3], const double QR[3],
                                             double pguess, int guess, double gate, const float *mlp,
                                             int maxit, double tol, RSOut &o) {
  Prim L, R;
  bool okl = to_prim(G, QL[0], QL[1], QL[2], L);
  bool okr = to_prim(G, QR[0], QR[1], QR[2], R);
  o.iters = 0;
  o.mlp = false;
  if (!(okl && okr)) {
    o.F[0] = o.F[1] = o.F[2] = 0.0;
    o.Q[0] = QL[0]; o.Q[1] = QL[1]; o.Q[2] = QL[2];
    o.pstar = 0.0;
    return ERR_NONPHYS;
  }
  if (G.two_gm1 * (L.c + R.c) <= R.u - L.u) {
    o.F[0] = o.F[1] = o.F[2] = 0.0;
    o.Q[0] = QL[0]; o.Q[1] = QL[1]; o.Q[2] = QL[2];
    o.pstar = 0.0;
    return ERR_VACUUM;
  }
  double p0 = pguess > 0.0 ? pguess : start_pressure(G, L, R, guess, gate, mlp, o.mlp);
  double ps, us;
  int it = newton_pstar(G, L, R, p0, maxit, tol, ps, us);
  o.iters = it;
  o.pstar = ps;
  double r, u, p;
  sample_at_zero(G, L, R, ps, us, r, u, p);
  double E = p * G.inv_gm1 + 0.5 * r * u * u;
  o.Q[0] = r;
  o.Q[1] = r * u;
  o.Q[2] = E;
  o.F[0] = r * u;
  o.F[1] = r * u * u + p;
  o.F[2] = u * (E + p);
  return it > maxit ? ERR_NEWTON : 0u;
}

}  // namespace grp
