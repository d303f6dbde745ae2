// Instances of the slab-operator kernels for d = 2 in float (see apply_impl.hpp).
#include "apply_impl.hpp"

namespace sg {
template hipError_t apply_dim<2, float>(const ApplyOp<float>&, const float*, float*, hipStream_t);
}  // namespace sg
