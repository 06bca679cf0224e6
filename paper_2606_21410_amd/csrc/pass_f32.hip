// FP32 instantiations of the axis-pass kernel.
#include "pass_launch.h"

namespace cheb {
template int launch_axis_pass<float>(const cheb_plan*, int, int, int, const float*, const float*, float*,
                                     hipStream_t);
template int apply_t<float>(const cheb_plan*, const float*, const float*, float*, int, hipStream_t);
}  // namespace cheb
