// kernels_pass_last.hip -- instantiations of the LF pass (D, the RK4 stage
// epilogue and D again on the last axis). The kernel template and its
// data flow are in pass_common.h; this file only instantiates them.
#include "pass_common.h"

namespace rk4ip {

hipError_t launch_axis_last(const GroupDev& g, int axis, int mode, const PassArgs& a, hipStream_t s) {
    if (mode == PASS_LF) return go_axis_mode<PASS_LF>(g, axis, a, s);
    return hipErrorInvalidValue;
}
}  // namespace rk4ip
