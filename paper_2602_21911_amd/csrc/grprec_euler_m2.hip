// grprec_euler_m2.hip -- the fused Euler step at degree 2 (scheme order 3).
#include "grprec_euler.h"

namespace grp {
template hipError_t launch_euler<2>(const EulerArgs<2> &, int, int, bool, hipStream_t);
template hipError_t euler_occupancy<2>(int, bool, int *);
}  // namespace grp
