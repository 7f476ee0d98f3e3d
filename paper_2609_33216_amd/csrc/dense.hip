// Batched dense complex FP64 linear algebra for the compressed equations of
// paper Section 4.2: LU with partial pivoting of each diagonal block with its
// right-hand sides appended (so that X = D^{-1} L falls out of the same
// factorisation), the GEMMs R X, A~ R g, X z, triangular solves, and the
// gathers that assemble a parent's diagonal block from its children.
//
// All matrices are column-major.  A workgroup of 256 threads computes a
// 64 x 64 output tile of a GEMM as 16 x 16 threads with 4 x 4 accumulators
// each, staging 16-deep slices of both operands in LDS.
#include "kernels.hpp"

namespace symhss {

#include "dense_body.inc"

}  // namespace symhss
