// Instances of the slab-operator kernels for d = 2 in double (see apply_impl.hpp).
#include "apply_impl.hpp"

namespace sg {
template hipError_t apply_dim<2, double>(const ApplyOp<double>&, const double*, double*, hipStream_t);
}  // namespace sg
