// kernels_pass_first.hip -- instantiations of the passes that open and close a
// run of steps on the contiguous axis: FIRST (h G, then D_0) and LAST2 (D_0, then the
// end of the step). The kernel template and its
// data flow are in pass_common.h; this file only instantiates them.
#include "pass_common.h"

namespace rk4ip {

hipError_t launch_axis_first(const GroupDev& g, int axis, int mode, const PassArgs& a, hipStream_t s) {
    if (mode == PASS_FIRST) return go_axis_mode<PASS_FIRST>(g, axis, a, s);
    if (mode == PASS_LAST2) return go_axis_mode<PASS_LAST2>(g, axis, a, s);
    return hipErrorInvalidValue;
}
}  // namespace rk4ip
