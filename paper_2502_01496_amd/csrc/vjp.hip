// Vector-Jacobian product of the accelerations (tree and lists held fixed).
#include "fmm_internal.h"

namespace fmm {

hipError_t launch_vjp(Tree &, const void *, void *, void *, hipStream_t)
{
    return hipErrorNotSupported;
}

}  // namespace fmm
