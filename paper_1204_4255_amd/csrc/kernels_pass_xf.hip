// kernels_pass_xf.hip -- instantiations of the XF pass (D_0, the end of one step and the
// start of the next, D_0 again). The kernel template and its data flow are in
// pass_common.h; this file only instantiates them.
#include "pass_common.h"

namespace rk4ip {

hipError_t launch_axis_xf(const GroupDev& g, int axis, const PassArgs& a, hipStream_t s) {
    return go_axis_mode<PASS_XF>(g, axis, a, s);
}

}  // namespace rk4ip
