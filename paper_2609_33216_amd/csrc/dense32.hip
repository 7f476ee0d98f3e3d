// The batched dense linear algebra of dense.hip in complex FP32 (FP32
// arithmetic, FP32 storage), for the mixed-precision factorisation: the
// diagonal-block LUs, X = D^{-1} L, A~ = (R X)^{-1} and the dense top-level
// system are factored in FP32 and the solution is refined against the FP64
// operator.
#include "kernels.hpp"

namespace symhss {
namespace f32 {

#include "dense_body.inc"

}  // namespace f32
}  // namespace symhss
