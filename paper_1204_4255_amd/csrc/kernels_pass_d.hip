// kernels_pass_d.hip -- instantiations of the plain propagator passes D1 and D2. The kernel template and its
// data flow are in pass_common.h; this file only instantiates them.
#include "pass_common.h"

namespace rk4ip {

hipError_t launch_axis_d(const GroupDev& g, int axis, int mode, const PassArgs& a, hipStream_t s) {
    if (mode == PASS_D1) return go_axis_mode<PASS_D1>(g, axis, a, s);
    if (mode == PASS_D2) return go_axis_mode<PASS_D2>(g, axis, a, s);
    return hipErrorInvalidValue;
}
}  // namespace rk4ip
