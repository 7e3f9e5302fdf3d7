// grprec_euler_m4.hip -- the fused Euler step at degree 4 (scheme order 5).
#include "grprec_euler.h"

namespace grp {
template hipError_t launch_euler<4>(const EulerArgs<4> &, int, int, bool, hipStream_t);
template hipError_t euler_occupancy<4>(int, bool, int *);
}  // namespace grp
