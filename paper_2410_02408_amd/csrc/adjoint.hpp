// Gradient of a loss through a linear solve with respect to the stored
// values of A.  For x = A^-1 b and g = dL/dx, the adjoint solve
// lambda = A^-T g = A^-1 g (A symmetric) gives dL/db = lambda and
// dL/dA_ij = -lambda_i x_j for every stored entry (i, j) - an outer product
// restricted to A's sparsity pattern.
#pragma once

#include "common.hpp"

namespace bjp {

// GS lanes per row, rows in XCD-aware chunks; grad is written in CSR order.
template <int GS>
__global__ __launch_bounds__(kWG) void k_value_grad(int n, int chunk, const int32_t *__restrict__ rp,
                                                    const int32_t *__restrict__ ci,
                                                    const double *__restrict__ lambda,
                                                    const double *__restrict__ x,
                                                    double *__restrict__ grad) {
    constexpr int RWG = kWG / GS;
    const int tid = threadIdx.x, sub = tid & (GS - 1), grp = tid / GS;
    const int c = xcd_chunk(blockIdx.x, gridDim.x);
    const int r0 = c * chunk, r1 = min(r0 + chunk, n);
    for (int row = r0 + grp; row < r1; row += RWG) {
        const double li = -lambda[row];
        const int kb = rp[row], ke = rp[row + 1];
        for (int k = kb + sub; k < ke; k += GS) grad[k] = li * x[ci[k]];
    }
}

}  // namespace bjp
