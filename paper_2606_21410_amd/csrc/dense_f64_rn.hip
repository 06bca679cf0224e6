// Matrix-core axis pass, FP64, for plans with per-node Robin coefficients
// (each pencil's end-block inverse read from the plan).
#include "dense_launch.h"

namespace cheb {

template int launch_dense_rn<double, true>(const DenseArgs<double>&, int, int, int, int, hipStream_t);

}  // namespace cheb
