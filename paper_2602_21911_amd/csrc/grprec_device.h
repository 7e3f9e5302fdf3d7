// grprec_device.h -- device functions of the GRPrec step for gfx950 (wave64, FP64).
#pragma once

#include <hip/hip_runtime.h>

#include "grprec_internal.h"
#include "grprec_tables.h"

namespace grp {

__device__ __forceinline__ unsigned long long dbits(double x) {
  return (unsigned long long)__double_as_longlong(x);
}
__device__ __forceinline__ double bitsd(unsigned long long b) {
  return __longlong_as_double((long long)b);
}

// x^e for x > 0 as 2^(e log2 x): a few ulp, cheaper than a general pow.
__device__ __forceinline__ double powpos(double x, double e) { return exp2(e * log2(x)); }

// ---------------------------------------------------------------- reductions
// One step of the segmented scan below: the value of the lane selected by the
// DPP control (the lane's own where there is none) is taken when it belongs to
// the same run and is larger.  Values are the bit patterns of non-negative
// doubles or NaN, which order as unsigned integers like the values, NaN
// above all.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void seg_max_step(int seg, unsigned long long &bits) {
  const int lo = (int)bits, hi = (int)(bits >> 32);
  const int olo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROW_MASK, 0xf, false);
  const int ohi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROW_MASK, 0xf, false);
  const int os = __builtin_amdgcn_update_dpp(seg, seg, CTRL, ROW_MASK, 0xf, false);
  const unsigned long long ob = ((unsigned long long)(unsigned)ohi << 32) | (unsigned)olo;
  if (os == seg && ob > bits) bits = ob;
}

// Per-domain maximum over one wave (every lane active): lanes hold (seg, val)
// with each seg >= 0 on one contiguous run of lanes (lanes with seg < 0 take
// no part), val >= 0 or NaN.  An inclusive segmented prefix maximum over the
// lanes -- shifts by 1, 2, 4 and 8 within each row of 16 lanes, then the last
// lane of rows 0 and 2 into rows 1 and 3, then the last lane of row 1 into
// rows 2 and 3 -- leaves each run's maximum on its last lane, which returns
// true and receives it as the bits of the double.
__device__ __forceinline__ bool wave_segmented_lead(int seg, double val, unsigned long long &bits) {
  bits = dbits(val);
  seg_max_step<0x111, 0xf>(seg, bits);  // row_shr:1
  seg_max_step<0x112, 0xf>(seg, bits);  // row_shr:2
  seg_max_step<0x114, 0xf>(seg, bits);  // row_shr:4
  seg_max_step<0x118, 0xf>(seg, bits);  // row_shr:8
  seg_max_step<0x142, 0xa>(seg, bits);  // row_bcast:15
  seg_max_step<0x143, 0xc>(seg, bits);  // row_bcast:31
  const int next = __builtin_amdgcn_update_dpp(seg, seg, 0x130, 0xf, 0xf, false);  // wave_shl:1
  return seg >= 0 && ((threadIdx.x & 63) == 63 || next != seg);
}

// One atomicMax per run on base[seg].  The target only grows while it
// accumulates, so a run whose maximum does not exceed the value already there
// has nothing to add; skipping it keeps a long domain's many waves from
// queueing on one address.
__device__ __forceinline__ void wave_segmented_max(int seg, double val, unsigned long long *base) {
  unsigned long long bits;
  if (wave_segmented_lead(seg, val, bits) &&
      __hip_atomic_load(base + seg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < bits)
    atomicMax(base + seg, bits);
}

// Whole-wave lane shifts of a double by DPP (wave_shr:1 / wave_shl:1): lane l
// receives lane l-1 (wave_prev) or lane l+1 (wave_next); the lane without a
// source (0, resp. 63) keeps its own value.
__device__ __forceinline__ double wave_prev(double x) {
  const long long b = __double_as_longlong(x);
  int lo = (int)b, hi = (int)(b >> 32);
  lo = __builtin_amdgcn_update_dpp(lo, lo, 0x138, 0xf, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(hi, hi, 0x138, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double wave_next(double x) {
  const long long b = __double_as_longlong(x);
  int lo = (int)b, hi = (int)(b >> 32);
  lo = __builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xf, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// ---------------------------------------------------------------- Euler physics
// 1/x from the hardware estimate refined by two Newton steps (within a few ulp
// of the correctly rounded value; x > 0 finite).
__device__ __forceinline__ double rcp(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}

// sqrt(x) for x > 0 finite: hardware 1/sqrt estimate and two Newton steps on
// the pair (g ~ sqrt(x), h ~ 1/(2 sqrt(x))) (within a few ulp).
__device__ __forceinline__ double sqrtpos(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  r = fma(-g, g, x);
  return fma(r, h, g);
}

// 1/x from the hardware estimate and one Newton step: within 11 ulp of the
// correctly rounded value (measured on MI355X over 4M arguments spanning
// 2^-20 .. 2^20; the raw estimate is good to about 2^-24).  Used for the
// predictor's nodal fluxes, whose sweeps stop at a relative change of 1e-13.
__device__ __forceinline__ double rcp1(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  return fma(y, fma(-x, y, 1.0), y);
}

// Conserved Q = (rho, rho u, E), ideal gas p = (g-1)(E - rho u^2 / 2).
__device__ __forceinline__ void euler_flux(const Gas &G, double r, double m, double E, double &f0,
                                           double &f1, double &f2) {
  double u = m * rcp1(r);
  double p = G.gm1 * (E - 0.5 * m * u);
  f0 = m;
  f1 = m * u + p;
  f2 = u * (E + p);
}

struct Prim {
  double r, u, p, c;
  double ir, ip, ic;  // 1/r, 1/p, 1/c
};

// Primitive state and sound speed; false if not physical.
__device__ __forceinline__ bool to_prim(const Gas &G, double r, double m, double E, Prim &w) {
  w.r = r;
  w.ir = rcp(r);
  w.u = m * w.ir;
  w.p = G.gm1 * (E - 0.5 * m * w.u);
  bool ok = (r > 0.0) && (w.p > 0.0) && isfinite(w.u) && isfinite(w.p);
  w.ip = ok ? rcp(w.p) : 0.0;
  w.c = ok ? sqrtpos(G.g * w.p * w.ir) : 0.0;
  w.ic = ok ? rcp(w.c) : 0.0;
  return ok;
}

// Prim from primitive values (r, p > 0 checked by the caller).
__device__ __forceinline__ void prim_from(const Gas &G, double r, double u, double p, Prim &w) {
  w.r = r;
  w.u = u;
  w.p = p;
  w.ir = rcp(r);
  w.ip = rcp(p);
  w.c = sqrtpos(G.g * p * w.ir);
  w.ic = rcp(w.c);
}

// y^k for a small non-negative integer k (binary powering).
__device__ __forceinline__ double ipow(double y, int k) {
  double r = 1.0;
  while (k > 0) {
    if (k & 1) r *= y;
    y *= y;
    k >>= 1;
  }
  return r;
}

// x^z, z = (g-1)/(2g), for x > 0.  When 1/z = n is an integer (n = 7 for
// g = 1.4) the n-th root starts from a float estimate and takes two Newton
// steps on y^n = x (each squares the relative error: 1e-7 -> 1e-14 -> 1e-28);
// otherwise 2^(z log2 x).
__device__ __forceinline__ double pow_z(const Gas &G, double x) {
  if (G.root_n > 0 && x > 1e-30 && x < 1e30) {
    const float xf = (float)x;
    double y = (double)__builtin_amdgcn_exp2f(__builtin_amdgcn_logf(xf) * G.inv_nf);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const double yn1 = ipow(y, G.root_n - 1);
      y = fma(G.nm1_n, y, x * rcp(yn1) * G.inv_n);
    }
    return y;
  }
  return powpos(x, G.z);
}

// (p/pK)^(1/g) from w = (p/pK)^z: w^(2/(g-1)).
__device__ __forceinline__ double dens_pow(const Gas &G, double w) {
  return G.dens_k > 0 ? ipow(w, G.dens_k) : powpos(w, G.two_gm1);
}

// Star-region pressure function of one side, its derivative and, on the
// rarefaction branch, w = (p/pK)^z (shock branch from the Rankine-Hugoniot
// conditions, rarefaction branch from the isentropic relation and the
// generalised Riemann invariant).  ip = 1/p.
struct Side {
  double f, fd, w;
  bool rare;
};

// Weak waves: for |p/pK - 1| <= kWeak both branches of f_K and of the star
// density agree with their second-order expansions about pK (the Hugoniot
// curve and the isentrope have second-order contact there); the neglected
// third-order terms, <= 2e-16 cK and 5e-17 rhoK, are below the round-off of
// the closed forms, which lose digits to cancellation at such d.  The
// expansions need no powers or square roots and no branch.
constexpr double kWeak = 1e-5;

__device__ __forceinline__ void side_eval(const Gas &G, double p, double ip, const Prim &K, Side &s) {
  const double d = (p - K.p) * K.ip;
  // weak waves dominate smooth flows: the other branches are laid out apart
  if (__builtin_expect(fabs(d) <= kWeak, 1)) {
    s.rare = false;  // w is not carried on this path
    s.w = 0.0;
    s.f = (K.c * G.inv_g) * d * fma(-G.k2, d, 1.0);
    s.fd = K.ir * K.ic * fma(-2.0 * G.k2, d, 1.0);
    return;
  }
  if (p <= K.p) {
    s.rare = true;
    s.w = pow_z(G, p * K.ip);
    s.f = G.two_gm1 * K.c * (s.w - 1.0);
    // (p/pK)^(-(g+1)/(2g)) / (rhoK cK) = w (pK / p) / (rhoK cK)
    s.fd = s.w * K.p * ip * K.ir * K.ic;
  } else {
    s.rare = false;
    s.w = 0.0;
    const double ak = G.two_gp1 * K.ir;
    const double bk = G.gm1_gp1 * K.p;
    const double ibp = rcp(bk + p);
    const double sq = sqrtpos(ak * ibp);
    s.f = (p - K.p) * sq;
    s.fd = (1.0 - 0.5 * (p - K.p) * ibp) * sq;
  }
}

__device__ __forceinline__ double pvrs(const Prim &L, const Prim &R) {
  double ppv = 0.5 * (L.p + R.p) - 0.125 * (R.u - L.u) * (L.r + R.r) * (L.c + R.c);
  double fl = 1e-6 * fmin(L.p, R.p);
  return ppv > fl ? ppv : fl;
}

// Newton iteration for the star pressure from p0 > 0; non-positive iterates
// are replaced by half the previous one; stop on relative change <= tol after
// at least one iteration.  Returns the iteration count (maxit+1 = no
// convergence).  f_K and w_K at the final pressure come from the last
// evaluation by a first-order correction: at convergence the step is at most
// tol p, so the neglected term is O(tol^2) relative.
__device__ __forceinline__ int newton_pstar(const Gas &G, const Prim &L, const Prim &R, double p,
                                            int maxit, double tol, double &pstar, double &ustar,
                                            Side &sl, Side &sr) {
  const double du = R.u - L.u;
  double pe = p;
  auto iterate = [&]() -> bool {
    pe = p;
    const double ip = rcp(p);
    side_eval(G, p, ip, L, sl);
    side_eval(G, p, ip, R, sr);
    double pn = p - (sl.f + sr.f + du) * rcp(sl.fd + sr.fd);
    if (pn <= 0.0) pn = 0.5 * p;
    const bool stop = 2.0 * fabs(pn - p) <= tol * (pn + p);
    p = pn;
    return stop;
  };
  // the first iteration, which is the last for most problems, outside the
  // loop: straight-line code that independent solves can interleave
  bool conv = iterate();
  int k = 1;
  if (__builtin_expect(!conv, 0)) {
    for (k = 2; k <= maxit; ++k) {
      if (iterate()) {
        conv = true;
        break;
      }
    }
  }
  const double dp = p - pe;
  sl.f = fma(sl.fd, dp, sl.f);
  sr.f = fma(sr.fd, dp, sr.f);
  const double rel = G.z * dp * rcp(pe);
  sl.w = fma(sl.w, rel, sl.w);
  sr.w = fma(sr.w, rel, sr.w);
  pstar = p;
  ustar = 0.5 * (L.u + R.u) + 0.5 * (sr.f - sl.f);
  return conv ? k : maxit + 1;
}

// State of the exact Riemann solution on the line x/t = 0 (primitive).
__device__ __forceinline__ void sample_at_zero(const Gas &G, const Prim &L, const Prim &R, double ps,
                                               double us, const Side &sl, const Side &sr, double &r,
                                               double &u, double &p) {
  if (us >= 0.0) {
    if (ps <= L.p) {  // left rarefaction
      if (L.u - L.c >= 0.0) {
        r = L.r; u = L.u; p = L.p;
      } else {
        const double d = (ps - L.p) * L.ip;
        const bool weak = fabs(d) <= kWeak;
        const double w = weak ? fma(fma(G.z2, d, G.z), d, 1.0) : (sl.rare ? sl.w : pow_z(G, ps * L.ip));
        const double cs = L.c * w;
        if (us - cs < 0.0) {
          r = L.r * (weak ? fma(fma(G.dens2, d, G.inv_g), d, 1.0) : dens_pow(G, w)); u = us; p = ps;
        } else {  // fan: u - c = 0 and u + 2c/(g-1) is carried from the left
          const double c = G.two_gp1 * (L.c + 0.5 * G.gm1 * L.u);
          const double cr = c * L.ic;
          r = L.r * powpos(cr, G.two_gm1);
          u = c;
          p = L.p * powpos(cr, G.twog_gm1);
        }
      }
    } else {  // left shock
      const double pm = ps * L.ip;
      const double s = L.u - L.c * sqrtpos(G.gp1_2g * pm + 0.5 * G.gm1 * G.inv_g);
      if (s >= 0.0) {
        r = L.r; u = L.u; p = L.p;
      } else {
        r = L.r * (pm + G.gm1_gp1) * rcp(pm * G.gm1_gp1 + 1.0); u = us; p = ps;
      }
    }
  } else {
    if (ps > R.p) {  // right shock
      const double pm = ps * R.ip;
      const double s = R.u + R.c * sqrtpos(G.gp1_2g * pm + 0.5 * G.gm1 * G.inv_g);
      if (s <= 0.0) {
        r = R.r; u = R.u; p = R.p;
      } else {
        r = R.r * (pm + G.gm1_gp1) * rcp(pm * G.gm1_gp1 + 1.0); u = us; p = ps;
      }
    } else {  // right rarefaction
      if (R.u + R.c <= 0.0) {
        r = R.r; u = R.u; p = R.p;
      } else {
        const double d = (ps - R.p) * R.ip;
        const bool weak = fabs(d) <= kWeak;
        const double w = weak ? fma(fma(G.z2, d, G.z), d, 1.0) : (sr.rare ? sr.w : pow_z(G, ps * R.ip));
        const double cs = R.c * w;
        if (us + cs >= 0.0) {
          r = R.r * (weak ? fma(fma(G.dens2, d, G.inv_g), d, 1.0) : dens_pow(G, w)); u = us; p = ps;
        } else {  // fan: u + c = 0 and u - 2c/(g-1) is carried from the right
          const double c = G.two_gp1 * (R.c - 0.5 * G.gm1 * R.u);
          const double cr = c * R.ic;
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
  // tanh(x) = 1 - 2 / (exp(2x) + 1), saturating cleanly for large |x|; the
  // hardware reciprocal (1 ulp) instead of a correctly rounded division
  const float e = __expf(2.0f * x);
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}

__device__ __forceinline__ void mlp_features(double g, double rl, double ul, double pl, double rr,
                                             double ur, double pr, float x[6], double &pbar) {
  double rbar = 0.5 * (rl + rr);
  pbar = 0.5 * (pl + pr);
  double cbar = sqrt(g * pbar / rbar);
  x[0] = (float)log(rl / rbar);
  x[1] = (float)log(rr / rbar);
  x[2] = (float)log(pl / pbar);
  x[3] = (float)log(pr / pbar);
  x[4] = (float)(ul / cbar);
  x[5] = (float)(ur / cbar);
}

__device__ __forceinline__ float mlp_eval(const float *__restrict__ P, const float xin[6]) {
  const float *W1 = P, *b1 = P + 192, *W2 = P + 224, *b2 = P + 1248, *W3 = P + 1280, *b3 = P + 1312;
  const float *mean = P + 1313, *stdv = P + 1319;
  float x[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) x[i] = (xin[i] - mean[i]) * __builtin_amdgcn_rcpf(stdv[i]);
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

// True when the data jump is large: |dp|/pbar + |drho|/rhobar + |du|/cbar
// above the gate (evaluated without divisions); a negative gate always passes.
__device__ __forceinline__ bool jump_exceeds(const Prim &L, const Prim &R, double gate) {
  const double pbar = 0.5 * (L.p + R.p), rbar = 0.5 * (L.r + R.r), cbar = 0.5 * (L.c + R.c);
  const double lhs = fabs(R.p - L.p) * rbar * cbar + fabs(R.r - L.r) * pbar * cbar +
                     fabs(R.u - L.u) * pbar * rbar;
  return gate < 0.0 || lhs > gate * pbar * rbar * cbar;
}

// jump_exceeds() on conserved data; false for a non-physical state (the
// general solver reports it).
__device__ __forceinline__ bool jump_exceeds_q(const Gas &G, const double QL[3], const double QR[3],
                                               double gate) {
  Prim L, R;
  const bool okl = to_prim(G, QL[0], QL[1], QL[2], L);
  const bool okr = to_prim(G, QR[0], QR[1], QR[2], R);
  return okl && okr && jump_exceeds(L, R, gate);
}

// The network's star-pressure proposal, or 0 when it is not positive and
// finite.  Kept out of line: it is large and, behind the gate, rarely taken.
// Arguments travel by value: a reference to a local would put that local in
// private memory on every path, taken or not.
__device__ __noinline__ double learned_pressure(double g, double rl, double ul, double pl, double rr,
                                                double ur, double pr, const float *mlp) {
  float x[6];
  double pb;
  mlp_features(g, rl, ul, pl, rr, ur, pr, x, pb);
  const float y = mlp_eval(mlp, x);
  const double p0 = pb * exp((double)y);
  return (p0 > 0.0 && isfinite(p0)) ? p0 : 0.0;
}

// The learned proposal evaluated by the whole wave, for the lanes whose
// `want` is set: lane j < 32 owns hidden unit j of both layers.  For each
// wanted lane in turn its six standardised features are broadcast, each lane
// evaluates its units, and the output is summed across the lanes; one
// sample costs about as much as one lane's share of the per-lane network
// (mlp_eval), so a wave with a few lanes above the gate no longer runs the
// whole network on every lane.  Returns pbar exp(y) on the wanted lanes (0
// where it is not positive and finite), 0 elsewhere.  Must be called with
// all 64 lanes of the wave active (cross-lane reads of the hidden units);
// L and R are read on the wanted lanes only.
__device__ __forceinline__ float lane_read(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

__device__ __forceinline__ double wave_learned_pressure(double g, double gm1, bool want, double r0, double m0, double e0,
                                                     double r1, double m1, double e1,
                                                     const float *__restrict__ P) {
  unsigned long long todo = __ballot(want);
  const int lane = threadIdx.x & 63, j = lane & 31;
  // this lane's rows of the parameters (lanes 32..63 repeat lanes 0..31)
  float w1[6], w2[32];
#pragma unroll
  for (int k = 0; k < 6; ++k) w1[k] = P[j * 6 + k];
#pragma unroll
  for (int k = 0; k < 32; ++k) w2[k] = P[224 + j * 32 + k];
  const float b1 = P[192 + j], b2 = P[1248 + j], w3 = lane < 32 ? P[1280 + j] : 0.0f, b3 = P[1312];
  // standardised features of the wanted lanes
  float z[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  double pb = 0.0;
  if (want) {  // conserved data (r, m, E) of both sides -> primitive -> features
    const double ul = m0 / r0, ur = m1 / r1;
    const double pl = gm1 * (e0 - 0.5 * m0 * ul), pr = gm1 * (e1 - 0.5 * m1 * ur);
    float x[6];
    mlp_features(g, r0, ul, pl, r1, ur, pr, x, pb);
#pragma unroll
    for (int k = 0; k < 6; ++k) z[k] = (x[k] - P[1313 + k]) * __builtin_amdgcn_rcpf(P[1319 + k]);
  }
  double p0 = 0.0;
  while (todo) {
    const int src = __ffsll((long long)todo) - 1;
    todo &= todo - 1ull;
    float a = b1;
#pragma unroll
    for (int k = 0; k < 6; ++k) a = fmaf(w1[k], lane_read(z[k], src), a);
    const float h1 = mlp_tanh(a);
    float a2 = b2;
#pragma unroll
    for (int k = 0; k < 32; ++k) a2 = fmaf(w2[k], lane_read(h1, k), a2);
    float t = w3 * mlp_tanh(a2);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) t += __shfl_xor(t, d, 64);
    if (lane == src) {
      const double p = pb * exp((double)(t + b3));
      p0 = (p > 0.0 && isfinite(p)) ? p : 0.0;
    }
  }
  return p0;
}

// Starting pressure: learned proposal when asked for and the data jump is
// large, else PVRS.  A non-finite or non-positive proposal falls back to PVRS.
__device__ __forceinline__ double start_pressure(const Gas &G, const Prim &L, const Prim &R, int guess,
                                                 double gate, const float *mlp, bool &used_mlp) {
  used_mlp = false;
  if (guess == 1 && mlp != nullptr && jump_exceeds(L, R, gate)) {
    const double p0 = learned_pressure(G.g, L.r, L.u, L.p, R.r, R.u, R.p, mlp);
    if (p0 > 0.0) {
      used_mlp = true;
      return p0;
    }
  }
  return pvrs(L, R);
}

// Full interface interaction: exact Riemann solution at x/t = 0 between two
// conserved states; returns error bits, the physical flux there and the state.
// Newton starts from pguess when it is positive, else from PVRS.
struct RSOut {
  double F[3];
  double Q[3];
  double pstar;
  double pv;    // PVRS estimate of the star pressure (general solver only)
  int iters;
  bool strong;  // the data jump passed the gate (when it was tested)
  bool learned; // Newton started from the learned proposal
};

// Start of the Newton iteration: pguess when positive, else PVRS.  With
// test_gate the data jump is first tested against the gate (o.strong); below
// the gate Newton starts from PVRS (already accurate to second order in the
// jump for weak waves), above it from the learned proposal when
// mlp != nullptr (o.learned), else from pguess when positive.  A warm start
// pguess taken from another problem's star pressure comes with that
// problem's PVRS estimate pv_ref > 0 and is moved by the difference of the
// two problems' PVRS estimates: the error of PVRS varies smoothly with the
// data, so the shifted start keeps only the change of that error between
// the two problems.
__device__ __forceinline__ unsigned interact(const Gas &G, const double QL[3], const double QR[3],
                                             double pguess, int maxit, double tol, RSOut &o,
                                             const float *mlp = nullptr, double gate = 0.0,
                                             bool test_gate = false, double pv_ref = 0.0) {
  Prim L, R;
  bool okl = to_prim(G, QL[0], QL[1], QL[2], L);
  bool okr = to_prim(G, QR[0], QR[1], QR[2], R);
  o.iters = 0;
  o.strong = false;
  o.learned = false;
  o.pv = 0.0;
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
  const double pv = pvrs(L, R);
  o.pv = pv;
  double p0 = 0.0;
  if (test_gate) {
    o.strong = jump_exceeds(L, R, gate);
    if (o.strong && mlp != nullptr) {
      p0 = learned_pressure(G.g, L.r, L.u, L.p, R.r, R.u, R.p, mlp);
      o.learned = p0 > 0.0;
    } else if (o.strong) {
      p0 = pguess;
    }
  } else {
    p0 = pguess;
  }
  if (p0 > 0.0 && pv_ref > 0.0) p0 += pv - pv_ref;
  if (!(p0 > 0.0)) p0 = pv;
  double ps, us;
  Side sl, sr;
  int it = newton_pstar(G, L, R, p0, maxit, tol, ps, us, sl, sr);
  o.iters = it;
  o.pstar = ps;
  double r, u, p;
  sample_at_zero(G, L, R, ps, us, sl, sr, r, u, p);
  double E = p * G.inv_gm1 + 0.5 * r * u * u;
  o.Q[0] = r;
  o.Q[1] = r * u;
  o.Q[2] = E;
  o.F[0] = r * u;
  o.F[1] = r * u * u + p;
  o.F[2] = u * (E + p);
  return it > maxit ? ERR_NEWTON : 0u;
}

// ---------------------------------------------------------------- weak waves in straight-line code
// The Riemann problems of smooth flow have two weak nonlinear waves: the PVRS
// start lies within kWeak of both data pressures, one Newton step meets the
// tolerance, and no rarefaction fan straddles x/t = 0.  weak_interact solves
// such a problem with the same start, the same Newton step and the same
// second-order expansions as interact() (its results agree to rounding), but
// without interact()'s branches: the sampled star density uses the expansion
// on both the shock and the rarefaction branch (Hugoniot and isentrope agree
// to second order, the third-order remainder is below 5e-17 rho_K), and the
// shock speed the expansion of its square root (remainder below 1e-16 c_K).
// It returns false, leaving o unspecified, whenever the problem needs the
// general solver: a non-physical or vacuum state, a start or star pressure
// outside the weak range, a Newton step that does not meet the tolerance, or
// a transonic rarefaction.
struct WeakPrim {
  double r, u, p, ip, c, irc;  // irc = 1/(rho c)
};

// The reciprocals and the reciprocal square root take one Newton step from
// the hardware estimates (within 11 and 20 ulp, measured on MI355X): the
// weak-wave solver's results then differ from interact()'s by a few 1e-15
// relative.
__device__ __forceinline__ bool weak_prim(const Gas &G, double r, double m, double E, WeakPrim &w) {
  const double ir = rcp1(r);
  w.r = r;
  w.u = m * ir;
  w.p = G.gm1 * (E - 0.5 * m * w.u);
  w.ip = rcp1(w.p);
  // 1/(rho c) = (g p rho)^(-1/2): hardware estimate and one Newton step;
  // c = g p / (rho c)
  const double x = G.g * w.p * r;
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x * y, y, 1.5);
  w.irc = y;
  w.c = G.g * w.p * y;
  // physical and finite: with r > 0 and g p r a normal positive number, p > 0
  // and u, c are finite (an infinite or NaN input drives p, hence g p r, to
  // NaN, -inf or +inf); states near the range limits go to the general solver
  return (r > 0.0) && (x > 1e-300) && (x < 1e300);
}

__device__ __forceinline__ bool weak_interact(const Gas &G, const double QL[3], const double QR[3], double tol,
                                              RSOut &o) {
  WeakPrim L, R;
  const bool okl = weak_prim(G, QL[0], QL[1], QL[2], L);
  const bool okr = weak_prim(G, QR[0], QR[1], QR[2], R);
  const double du = R.u - L.u;
  bool ok = okl && okr && (G.two_gm1 * (L.c + R.c) > du);
  // PVRS start, floored as in pvrs()
  const double ppv = 0.5 * (L.p + R.p) - 0.125 * du * (L.r + R.r) * (L.c + R.c);
  const double fl = 1e-6 * fmin(L.p, R.p);
  const double p = ppv > fl ? ppv : fl;
  const double dl = (p - L.p) * L.ip, dr = (p - R.p) * R.ip;
  ok = ok && fabs(dl) <= kWeak && fabs(dr) <= kWeak;
  // one Newton step with the weak-wave pressure functions of side_eval()
  double fL = (L.c * G.inv_g) * dl * fma(-G.k2, dl, 1.0);
  double fR = (R.c * G.inv_g) * dr * fma(-G.k2, dr, 1.0);
  const double fdL = L.irc * fma(-2.0 * G.k2, dl, 1.0);
  const double fdR = R.irc * fma(-2.0 * G.k2, dr, 1.0);
  const double pn = p - (fL + fR + du) * rcp1(fdL + fdR);
  ok = ok && pn > 0.0 && 2.0 * fabs(pn - p) <= tol * (pn + p);
  const double dp = pn - p;
  fL = fma(fdL, dp, fL);
  fR = fma(fdR, dp, fR);
  const double us = 0.5 * (L.u + R.u) + 0.5 * (fR - fL);
  // sample x/t = 0: the left wave when u* >= 0, else the right wave
  const bool left = us >= 0.0;
  const double rK = left ? L.r : R.r, uK = left ? L.u : R.u, pK = left ? L.p : R.p, cK = left ? L.c : R.c;
  const double d = (pn - pK) * (left ? L.ip : R.ip);
  ok = ok && fabs(d) <= kWeak;
  const double sg = left ? -1.0 : 1.0;  // the wave moves with uK + sg cK
  bool outside;                         // x/t = 0 lies outside the wave: the data state
  if (pn > pK) {                        // shock: speed uK + sg cK sqrt(1 + a d), a = (g+1)/(2g)
    const double a = G.gp1_2g;
    const double s = uK + sg * cK * fma(fma(-0.125 * a * a, d, 0.5 * a), d, 1.0);
    outside = left ? s >= 0.0 : s <= 0.0;
  } else {                              // rarefaction: head uK + sg cK, tail u* + sg c*
    const double cs = cK * fma(fma(G.z2, d, G.z), d, 1.0);
    const double head = uK + sg * cK, tail = us + sg * cs;
    outside = left ? head >= 0.0 : head <= 0.0;
    ok = ok && (outside || (left ? tail < 0.0 : tail >= 0.0));  // else a transonic fan
  }
  const double r = outside ? rK : rK * fma(fma(G.dens2, d, G.inv_g), d, 1.0);
  const double u = outside ? uK : us;
  const double pp = outside ? pK : pn;
  const double E = pp * G.inv_gm1 + 0.5 * r * u * u;
  o.Q[0] = r;
  o.Q[1] = r * u;
  o.Q[2] = E;
  o.F[0] = r * u;
  o.F[1] = r * u * u + pp;
  o.F[2] = u * (E + pp);
  o.pstar = pn;
  o.iters = 1;
  o.strong = false;
  o.learned = false;
  return ok;
}

// ---------------------------------------------------------------- two-rarefaction datum
// Two-rarefaction approximation of the Riemann problem (the solver Sec. 4.1
// names for the Euler interface datum): with both nonlinear waves taken as
// rarefactions the Riemann invariants and isentropes give
//   X = p_s^z = (c_L + c_R - (g-1)/2 (u_R - u_L)) / (c_L p_L^-z + c_R p_R^-z),
//   c_sK = c_K X / p_K^z,  u_s = (u_L + u_R)/2 + ((c_sR - c_R) - (c_sL - c_L))/(g-1),
// no iteration.  The state at x/t = 0 is sampled from the two-rarefaction
// pattern (left side when u_s >= 0); o.Q, o.F and o.pstar as interact().
__device__ __forceinline__ unsigned trrs_interact(const Gas &G, const double QL[3], const double QR[3],
                                                  RSOut &o) {
  Prim L, R;
  const bool okl = to_prim(G, QL[0], QL[1], QL[2], L);
  const bool okr = to_prim(G, QR[0], QR[1], QR[2], R);
  o.iters = 0;
  o.strong = false;
  o.learned = false;
  const double num = L.c + R.c - 0.5 * G.gm1 * (R.u - L.u);
  if (!(okl && okr) || !(num > 0.0)) {
    o.F[0] = o.F[1] = o.F[2] = 0.0;
    o.Q[0] = QL[0]; o.Q[1] = QL[1]; o.Q[2] = QL[2];
    o.pstar = 0.0;
    return (okl && okr) ? ERR_VACUUM : ERR_NONPHYS;
  }
  const double izl = rcp(pow_z(G, L.p)), izr = rcp(pow_z(G, R.p));  // p_K^-z
  const double X = num * rcp(L.c * izl + R.c * izr);
  const double ps = G.root_n > 0 ? ipow(X, G.root_n) : powpos(X, 1.0 / G.z);
  const double wl = X * izl, wr = X * izr;  // (p_s / p_K)^z
  const double csl = L.c * wl, csr = R.c * wr;
  const double us = 0.5 * (L.u + R.u) + ((csr - R.c) - (csl - L.c)) * G.inv_gm1;
  double r, u, p;
  if (us >= 0.0) {
    if (L.u - L.c >= 0.0) {
      r = L.r; u = L.u; p = L.p;
    } else if (us - csl < 0.0) {
      r = L.r * dens_pow(G, wl); u = us; p = ps;
    } else {  // fan: u - c = 0 and u + 2c/(g-1) is carried from the left
      const double c = G.two_gp1 * (L.c + 0.5 * G.gm1 * L.u);
      const double cr = c * L.ic;
      r = L.r * powpos(cr, G.two_gm1);
      u = c;
      p = L.p * powpos(cr, G.twog_gm1);
    }
  } else {
    if (R.u + R.c <= 0.0) {
      r = R.r; u = R.u; p = R.p;
    } else if (us + csr >= 0.0) {
      r = R.r * dens_pow(G, wr); u = us; p = ps;
    } else {  // fan: u + c = 0 and u - 2c/(g-1) is carried from the right
      const double c = G.two_gp1 * (R.c - 0.5 * G.gm1 * R.u);
      const double cr = c * R.ic;
      r = R.r * powpos(cr, G.two_gm1);
      u = -c;
      p = R.p * powpos(cr, G.twog_gm1);
    }
  }
  o.pstar = ps;
  const double E = p * G.inv_gm1 + 0.5 * r * u * u;
  o.Q[0] = r;
  o.Q[1] = r * u;
  o.Q[2] = E;
  o.F[0] = r * u;
  o.F[1] = r * u * u + p;
  o.F[2] = u * (E + p);
  return 0u;
}

// ---------------------------------------------------------------- implicit source
// Time matrices of the space-time predictor with the linear relaxation source
// S(q) = -kappa q taken implicitly: with z = kappa dt the weak form's time
// matrix is Kz = K + z diag(w), and the predictor iterates
//   q[a][.] <- c w_a - nu A (D F)[a][.],  A = Kz^{-1} diag(w),  c = Kz^{-1} l(0)
// (c = 1 and A = K^{-1} diag(w) without source).  Gauss-Jordan without pivot
// search: the pivots of K + z diag(w) stay above 0.4 of its largest entry for
// every z >= 0 at these degrees.
template <int N>
__device__ __forceinline__ void source_time_mats(const double (&K)[N][N], const double (&w)[N],
                                                 const double (&l0)[N], double z, double (&A)[N][N],
                                                 double (&c)[N]) {
  double M[N][N];
#pragma unroll
  for (int b = 0; b < N; ++b) {
#pragma unroll
    for (int l = 0; l < N; ++l) {
      M[b][l] = K[b][l] + (b == l ? z * w[b] : 0.0);
      A[b][l] = b == l ? w[b] : 0.0;  // right-hand sides diag(w) | l(0)
    }
    c[b] = l0[b];
  }
#pragma unroll
  for (int col = 0; col < N; ++col) {
    const double ip = rcp(M[col][col]);
#pragma unroll
    for (int k = 0; k < N; ++k) {
      M[col][k] *= ip;
      A[col][k] *= ip;
    }
    c[col] *= ip;
#pragma unroll
    for (int r = 0; r < N; ++r) {
      if (r == col) continue;
      const double f = M[r][col];
#pragma unroll
      for (int k = 0; k < N; ++k) {
        M[r][k] = fma(-f, M[col][k], M[r][k]);
        A[r][k] = fma(-f, A[col][k], A[r][k]);
      }
      c[r] = fma(-f, c[col], c[r]);
    }
  }
}

// ---------------------------------------------------------------- GRPrecNL
// Nonlinear combination of the left, centred and right candidates for one
// scalar field (Sec. 3.3).  aC: the centred (GRPrec) coefficients; del[k]:
// datum k minus the cell mean (indices as in tab::NLTab; del[1] unused).
// Indicators OI_k = dx a_k^T Gm a_k; weights omega_k = lambda_k/(eps+OI_k)^4
// with lambda_L = lambda_R = 1, normalised.  Scaling every omega by the
// product of the three (eps + OI)^4 leaves a single reciprocal:
//   beta_L : beta_C : beta_R = sC sR : lambda_C sL sR : sL sC.
template <int M>
__device__ __forceinline__ void nl_mix(const double (&aC)[M], const double (&del)[7], double dx,
                                       double lam_c, double eps, double (&out)[M]) {
  constexpr tab::NLTab<M> T = tab::nl_tables<M>();
  double aL[M], aR[M];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    double l = 0.0, r = 0.0;
#pragma unroll
    for (int k = 0; k < M; ++k) {
      if (T.A[0][j][k] != 0.0) l = fma(T.A[0][j][k], del[T.sel[0][k]], l);
      if (T.A[1][j][k] != 0.0) r = fma(T.A[1][j][k], del[T.sel[1][k]], r);
    }
    aL[j] = l;
    aR[j] = r;
  }
  auto ind = [&](const double (&a)[M]) {
    double sum = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      double row = T.Gm[j][j] * a[j];
#pragma unroll
      for (int k = j + 1; k < M; ++k)
        if (T.Gm[j][k] != 0.0) row = fma(2.0 * T.Gm[j][k], a[k], row);
      sum = fma(row, a[j], sum);
    }
    double s = fma(dx, sum, eps);
    s *= s;
    return s * s;
  };
  const double sL = ind(aL), sC = ind(aC), sR = ind(aR);
  const double wl = sC * sR, wc = lam_c * sL * sR, wr = sL * sC;
  const double inv = rcp(wl + wc + wr);
#pragma unroll
  for (int j = 0; j < M; ++j) out[j] = (wl * aL[j] + wc * aC[j] + wr * aR[j]) * inv;
}

// Centred GRPrec coefficients (zero-mean basis) from data differences to the
// cell mean: d0 = q_{i-1}, d2 = q_{i+1}, d3 = V_{i-1/2}, d4 = V_{i+1/2}, each
// minus q_i (Sec. 3.1 closed forms).
template <int M>
__device__ __forceinline__ void grprec_from_diffs(double d0, double d2, double d3, double d4,
                                                  double (&a)[M]) {
  const double DI = d4 - d3, SI = d3 + d4;
  if constexpr (M == 1) {
    a[0] = DI;
  } else if constexpr (M == 2) {
    a[0] = DI;
    a[1] = 3.0 * SI;
  } else {
    const double DC = d2 - d0, SC = d0 + d2;
    a[0] = 1.25 * DI - 0.125 * DC;
    a[2] = 0.5 * DC - DI;
    if constexpr (M == 3) {
      a[1] = (3.0 * SI + 18.0 * SC) * (1.0 / 37.0);
    } else {
      a[1] = 3.75 * SI - 0.125 * SC;
      a[3] = (5.0 / 12.0) * SC - 2.5 * SI;
    }
  }
}

// Eigenvectors of the Euler flux Jacobian at a conserved state, for the
// characteristic projection of the reconstruction (Sec. 3.1).  Right
// eigenvectors (columns of Rm) for u - c, u, u + c:
//   (1, u - c, H - u c), (1, u, u^2/2), (1, u + c, H + u c);
// rows of Lm = Rm^-1, with k = (g-1)/(2 c^2):
//   (u^2 k/2 + u/(2c), -(u k + 1/(2c)), k), (1 - u^2 k, 2 u k, -2 k),
//   (u^2 k/2 - u/(2c), -(u k - 1/(2c)), k).
// A non-physical state gives NaN, which the later state checks report.
__device__ __forceinline__ void euler_eigen(const Gas &G, const double (&Q)[3], double (&Lm)[3][3],
                                            double (&Rm)[3][3]) {
  const double ir = rcp(Q[0]);
  const double u = Q[1] * ir;
  const double p = G.gm1 * (Q[2] - 0.5 * Q[1] * u);
  const double c = sqrtpos(G.g * p * ir);
  const double ic = rcp(c), hic = 0.5 * ic;
  const double k = 0.5 * G.gm1 * ic * ic;
  const double H = (Q[2] + p) * ir;
  const double uk = u * k, u2k = 0.5 * u * uk, uhic = u * hic;
  Lm[0][0] = u2k + uhic; Lm[0][1] = -(uk + hic); Lm[0][2] = k;
  Lm[1][0] = 1.0 - 2.0 * u2k; Lm[1][1] = 2.0 * uk; Lm[1][2] = -2.0 * k;
  Lm[2][0] = u2k - uhic; Lm[2][1] = -(uk - hic); Lm[2][2] = k;
  const double uc = u * c;
  Rm[0][0] = 1.0; Rm[0][1] = 1.0; Rm[0][2] = 1.0;
  Rm[1][0] = u - c; Rm[1][1] = u; Rm[1][2] = u + c;
  Rm[2][0] = H - uc; Rm[2][1] = 0.5 * u * u; Rm[2][2] = H + uc;
}

}  // namespace grp
