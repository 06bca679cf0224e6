// Matrix-core axis pass (FP32 instantiation).
#include "dense_launch.h"

namespace cheb {

template int launch_dense_batch<float>(const cheb_plan*, int, int, const float*, const float*, float*, const DenseSys*,
                                      const int*, int, hipStream_t);
template int launch_dense_pass<float>(const cheb_plan*, int, int, int, const float*, const float*, float*,
                                       const float*, hipStream_t);
template int launch_dense_pair<float>(const cheb_plan*, int, const float*, const float*, float*, float*, hipStream_t);
template bool dense_pair_ok<float>(const cheb_plan*);

}  // namespace cheb
