// grprec_euler_m1.hip -- the fused Euler step at degree 1 (scheme order 2).
#include "grprec_euler.h"

namespace grp {
template hipError_t launch_euler<1>(const EulerArgs<1> &, int, int, bool, hipStream_t);
template hipError_t euler_occupancy<1>(int, bool, int *);
}  // namespace grp
