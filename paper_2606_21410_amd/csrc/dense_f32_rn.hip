// Matrix-core axis pass, FP32, for plans with per-node Robin coefficients
// (each pencil's end-block inverse read from the plan).
#include "dense_launch.h"

namespace cheb {

template int launch_dense_rn<float, true>(const DenseArgs<float>&, int, int, int, int, hipStream_t);

}  // namespace cheb
