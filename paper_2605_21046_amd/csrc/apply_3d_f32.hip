// Instances of the slab-operator kernels for d = 3 in float (see apply_impl.hpp).
#include "apply_impl.hpp"

namespace sg {
template hipError_t apply_dim<3, float>(const ApplyOp<float>&, const float*, float*, hipStream_t);
}  // namespace sg
