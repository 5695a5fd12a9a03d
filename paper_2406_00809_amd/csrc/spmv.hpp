// CSR sparse matrix-vector product y = A x (or y = b - A x) with G lanes per
// row: the lanes of a group stride over the row's nonzeros (coalesced loads
// of colind / val), then reduce with cross-lane shuffles.  G is chosen from
// the mean row length so that short stencil rows do not leave most of a
// wavefront idle.
#pragma once
#include <type_traits>
#include "gnp_internal.hpp"

namespace gnp {

template <typename VT> struct acc_of { using type = float; };
template <> struct acc_of<double> { using type = double; };

template <typename VT, typename XT, typename YT, int G, int NB, bool STRIDED>
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
        // G lanes per row; each lane takes entries lg, lg + G, ... in order,
        // NB at a time: all column / value loads of a batch, then all
        // gathers of x, then the adds (slots past the row's end re-read its
        // last entry and add nothing)
        const int32_t e = rp[row + 1];
        for (int32_t k0 = rp[row] + lg; k0 < e; k0 += G * NB) {
            int32_t c[NB];
            VT a[NB];
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                const int32_t k = k0 + u * G < e ? k0 + u * G : e - 1;
                c[u] = ci[k];
                a[u] = val[k];
            }
            XT xv[NB];
#pragma unroll
            for (int u = 0; u < NB; ++u) xv[u] = STRIDED ? x[c[u] * xstep] : x[c[u]];
#pragma unroll
            for (int u = 0; u < NB; ++u)
                if (k0 + u * G < e) acc += (Acc)a[u] * (Acc)xv[u];
        }
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
    if (row < n && lg == 0) y[row] = bsub ? (YT)(bsub[row] - (double)acc) : (YT)acc;
}

template <typename VT, typename XT, typename YT, int G, int NB>
inline void spmv_launch_g(int64_t n, const int32_t *rp, const int32_t *ci, const VT *val,
                          const XT *x, YT *y, const double *bsub, const int *skip, hipStream_t st,
                          int nb, int64_t xstep, int64_t ystride, int skip_step) {
    if (xstep == 1)  // contiguous x: no 64-bit index product per gather
        hipLaunchKernelGGL((k_spmv<VT, XT, YT, G, NB, false>), dim3(grid_for(n * G, BLOCK), nb),
                           dim3(BLOCK), 0, st, n, rp, ci, val, x, y, bsub, skip, xstep, ystride,
                           skip_step);
    else
        hipLaunchKernelGGL((k_spmv<VT, XT, YT, G, NB, true>), dim3(grid_for(n * G, BLOCK), nb),
                           dim3(BLOCK), 0, st, n, rp, ci, val, x, y, bsub, skip, xstep, ystride,
                           skip_step);
}

// Lanes per row from the mean row length (4 lanes for stencil-like rows: at
// 7 nonzeros per row, 4 lanes beat 8 by a third on MI355X), with 4 entries
// per lane in flight for irregular rows (the longest row above four times the
// mean) and 2 otherwise.  Irregular rows of a short mean take 8 lanes rather
// than 4 (a wavefront waits for its longest row); longer means keep their
// width: on the n = 2^20 power-law matrix (mean 12, rows of 3..64, random
// columns) 8 lanes take 76 us, 16 lanes 87 us.  max_row: the longest row (0
// if unknown).
template <typename VT, typename XT, typename YT>
inline void spmv_launch(int64_t n, const int32_t *rp, const int32_t *ci, const VT *val,
                        const XT *x, YT *y, const double *bsub, const int *skip, int64_t nnz,
                        hipStream_t st, int nb = 1, int64_t xstep = 1, int64_t ystride = 0,
                        int skip_step = 0, int max_row = 0) {
    const double avg = (double)nnz / (double)n;
    const bool irregular = max_row > 4.0 * avg;
    int level = avg <= 12.0 ? 0 : (avg <= 24.0 ? 1 : (avg <= 48.0 ? 2 : 3));
    if (irregular && level == 0) level = 1;
    const auto go = [&](auto g, auto nbv) {
        spmv_launch_g<VT, XT, YT, decltype(g)::value, decltype(nbv)::value>(
            n, rp, ci, val, x, y, bsub, skip, st, nb, xstep, ystride, skip_step);
    };
    using I2 = std::integral_constant<int, 2>;
    using I4 = std::integral_constant<int, 4>;
    switch (level) {
        case 0: return irregular ? go(I4{}, I4{}) : go(I4{}, I2{});
        case 1: return irregular ? go(std::integral_constant<int, 8>{}, I4{})
                                 : go(std::integral_constant<int, 8>{}, I2{});
        case 2: return irregular ? go(std::integral_constant<int, 16>{}, I4{})
                                 : go(std::integral_constant<int, 16>{}, I2{});
        default: return irregular ? go(std::integral_constant<int, 32>{}, I4{})
                                  : go(std::integral_constant<int, 32>{}, I2{});
    }
}

}  // namespace gnp
