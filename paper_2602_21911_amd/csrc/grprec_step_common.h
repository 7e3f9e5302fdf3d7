// grprec_step_common.h -- device helpers shared by the Euler and advection
// step kernels: per-domain step size, the idle-step carry, domain search and
// compile-time table selection.
#pragma once

#include <hip/hip_runtime.h>

#include "grprec_device.h"
#include "grprec_internal.h"

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
static __device__ void carry_slot(const Seg &seg, Ctl *ctl, int slot) {
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

}  // namespace grp
