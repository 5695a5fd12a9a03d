// CSR sparse matrix-vector product y = A x (or y = b - A x) with G lanes per
// row: the lanes of a group stride over the row's nonzeros (coalesced loads
// of colind / val), then reduce with cross-lane shuffles.  G is chosen from
// the mean row length so that short stencil rows do not leave most of a
// wavefront idle.
#pragma once
#include "gnp_internal.hpp"

namespace gnp {

template <typename VT> struct acc_of { using type = float; };
template <> struct acc_of<double> { using type = double; };

template <typename VT, typename XT, typename YT, int G>
__global__ __launch_bounds__(BLOCK) void k_spmv(int64_t n, const int32_t *__restrict__ rp,
                                                const int32_t *__restrict__ ci,
                                                const VT *__restrict__ val,
                                                const XT *__restrict__ x, YT *__restrict__ y,
                                                const double *__restrict__ bsub,
                                                const int *__restrict__ skip, int64_t xstep,
                                                int64_t ystride, int skip_step) {
    // batch: blockIdx.y selects a right-hand side; x is read at ci * xstep + b
    // (xstep = nrhs for a packed [n][nrhs] input), y at b * ystride
    const int bi = blockIdx.y;
    if (skip && skip[bi * skip_step]) return;
    x += bi;
    y += bi * ystride;
    using Acc = typename acc_of<VT>::type;
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int lg = threadIdx.x % G;
    Acc acc = 0;
    if (row < n) {
        const int32_t e = rp[row + 1];
        for (int32_t k = rp[row] + lg; k < e; k += G) acc += (Acc)val[k] * (Acc)x[ci[k] * xstep];
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
    if (row < n && lg == 0) y[row] = bsub ? (YT)(bsub[row] - (double)acc) : (YT)acc;
}

template <typename VT, typename XT, typename YT>
inline void spmv_launch(int64_t n, const int32_t *rp, const int32_t *ci, const VT *val,
                        const XT *x, YT *y, const double *bsub, const int *skip, int64_t nnz,
                        hipStream_t st, int nb = 1, int64_t xstep = 1, int64_t ystride = 0,
                        int skip_step = 0) {
    // lanes per row from the mean row length: 4 lanes for stencil-like rows
    // (at 7 nonzeros per row, 4 lanes beat 8 by a third on MI355X)
    const double avg = (double)nnz / (double)n;
    if (avg <= 12.0) {
        hipLaunchKernelGGL((k_spmv<VT, XT, YT, 4>), dim3(grid_for(n * 4, BLOCK), nb), dim3(BLOCK), 0,
                           st, n, rp, ci, val, x, y, bsub, skip, xstep, ystride, skip_step);
    } else if (avg <= 24.0) {
        hipLaunchKernelGGL((k_spmv<VT, XT, YT, 8>), dim3(grid_for(n * 8, BLOCK), nb), dim3(BLOCK), 0,
                           st, n, rp, ci, val, x, y, bsub, skip, xstep, ystride, skip_step);
    } else if (avg <= 48.0) {
        hipLaunchKernelGGL((k_spmv<VT, XT, YT, 16>), dim3(grid_for(n * 16, BLOCK), nb), dim3(BLOCK), 0,
                           st, n, rp, ci, val, x, y, bsub, skip, xstep, ystride, skip_step);
    } else {
        hipLaunchKernelGGL((k_spmv<VT, XT, YT, 32>), dim3(grid_for(n * 32, BLOCK), nb), dim3(BLOCK), 0,
                           st, n, rp, ci, val, x, y, bsub, skip, xstep, ystride, skip_step);
    }
}

}  // namespace gnp
