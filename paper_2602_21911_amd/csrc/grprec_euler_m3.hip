// grprec_euler_m3.hip -- the fused Euler step at degree 3 (scheme order 4).
#include "grprec_euler.h"

namespace grp {
template hipError_t launch_euler<3>(const EulerArgs<3> &, int, int, bool, hipStream_t);
template hipError_t euler_occupancy<3>(int, bool, int *);
}  // namespace grp
