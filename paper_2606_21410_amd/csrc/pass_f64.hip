// FP64 instantiations of the axis-pass kernel.
#include "pass_launch.h"

namespace cheb {
template int launch_axis_pass<double>(const cheb_plan*, int, int, int, const double*, const double*,
                                      double*, hipStream_t);
template int apply_t<double>(const cheb_plan*, const double*, const double*, double*, int, hipStream_t);
}  // namespace cheb
