// kernels_pass_si.hip -- instantiations of the SI pass (the semi-implicit step on the last
// axis: D, the midpoint fixed-point iteration and D again, on one field in place). The
// kernel template and its data flow are in pass_common.h; this file only instantiates them.
#include "pass_common.h"

namespace rk4ip {

hipError_t launch_axis_si(const GroupDev& g, int axis, const PassArgs& a, hipStream_t s) {
    return go_axis_mode<PASS_SI>(g, axis, a, s);
}

}  // namespace rk4ip
