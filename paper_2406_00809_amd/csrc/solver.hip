// Restarted flexible GMRES (Algorithm 1) with the network as nonlinear right
// preconditioner.  Per Arnoldi step j the stream holds: z_j = M(v_j), the
// SpMV w = A z_j, classical Gram-Schmidt applied twice with float64 inner
// products (pass 0: dots; pass 1: update + dots + ||w||^2; pass 2: update),
// the Givens update of the Hessenberg column on the device (its finaliser
// also forms h_{j+1,j} from pass 1's sums), and the normalisation
// v_{j+1} = w / h_{j+1,j}.  With a float32/bfloat16 network the next step's
// encoder does the normalisation, and with a basis pitch of 32 also pass 2,
// as it reads w; the network takes tau = 1 for every basis vector (unit norm,
// Eq. (6)).  Otherwise pass 2 writes v_{j+1} itself.
//
// Layout: the Arnoldi basis is stored row-interleaved, V[i * MP + k]
// (MP = m + 1 rounded up to a multiple of 32), so that the j + 1 basis
// entries of one row sit in one 128-byte line: a Gram-Schmidt pass reads
// each row once with eight lanes per row (float4 per lane) instead of j + 1
// separate streams.  The current v_j is also kept contiguous (vcur) as the
// network input.  Z (network outputs) is column-major: z_j is the SpMV input.
//
// Reductions are deterministic: each block writes its partial sums, and a
// one-block finalize kernel adds the partials in block order (lanes over
// columns, wavefronts over block subsets, up to 64 independent loads per lane in
// one round).
// The host synchronises once per restart cycle; every kernel of a step exits
// at entry once the device-side control block says the cycle is over.
#include <float.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "solver.hpp"
#include "spmv.hpp"

namespace gnp {

constexpr int RPP = BLOCK / 8;  // rows per pass in the Gram-Schmidt kernels
constexpr int MAXCOL = 258;     // columns of a finalize reduction (m + 2)

static int stream_grid(int64_t n) { return grid_for(n, 4 * BLOCK, 1024); }

// ---------------------------------------------------------------------------
// one-block finalize helper: out[c] = sum over blk < nblk of
// partial[blk * stride + c] for c < ncol, and with extra >= 0 also
// out[ncol] = the same sum of column `extra`; fixed summation order.
// ---------------------------------------------------------------------------
__device__ void reduce_columns(int nblk, int ncol, const double *__restrict__ partial, int stride,
                               double *out /* shared, >= ncol + 1 */, int extra = -1) {
    __shared__ double sh[BLOCK];
    const int t = threadIdx.x;
    const int nc = ncol + (extra >= 0 ? 1 : 0);
    if (nc == 1) {
        const double s = sum_partials(nblk, partial + (ncol == 1 ? 0 : extra), stride, sh);
        if (t == 0) out[0] = s;
        __syncthreads();
        return;
    }
    // lanes over output columns (CP per chunk), the rest over block subsets;
    // each thread issues all its loads of a round (U) before adding them in
    // block order: one memory round trip for up to S * U blocks
    constexpr int U = 64;
    const int CP = nc <= 32 ? 32 : 64;
    const int S = BLOCK / CP;
    const int cl = t % CP, sub = t / CP;
    for (int c0 = 0; c0 < nc; c0 += CP) {
        const int oc = c0 + cl;
        const int src = oc < ncol ? oc : (oc == ncol && extra >= 0 ? extra : 0);
        double s = 0.0;
        for (int blk0 = sub * U; blk0 < nblk; blk0 += S * U) {
            double v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {  // clamped, unconditional loads
                const int blk = (blk0 + u < nblk) ? blk0 + u : nblk - 1;
                v[u] = partial[(int64_t)blk * stride + src];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) s += (blk0 + u < nblk && oc < nc) ? v[u] : 0.0;
        }
        sh[t] = s;
        __syncthreads();
        if (t < CP && c0 + t < nc) {
            double v = 0.0;
            for (int q = 0; q < S; ++q) v += sh[q * CP + t];
            out[c0 + t] = v;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// ||b||^2 partials and finalize
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_sumsq(int64_t n, const double *__restrict__ x,
                                                 double *__restrict__ partial, Bat bt) {
    __shared__ double sh[BLOCK / WAVE];
    x += blockIdx.y * bt.vec;
    partial += blockIdx.y * bt.part;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * BLOCK)
        s += x[i] * x[i];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(BLOCK) void k_fin_bnorm(int nblk, const double *partial, double rtol,
                                                     Ctl *ctl, Bat bt) {
    __shared__ double res[1];
    partial += blockIdx.y * bt.part;
    ctl += blockIdx.y;
    reduce_columns(nblk, 1, partial, 1, res);
    if (threadIdx.x == 0) {
        ctl->bnorm = sqrt(res[0]);
        ctl->target = rtol * sqrt(res[0]);
    }
}

// ---------------------------------------------------------------------------
// true residual r = b - A x (float64 values and x), partial ||r||^2
// ---------------------------------------------------------------------------
template <int G>
__global__ __launch_bounds__(BLOCK) void k_residual(int64_t n, const int32_t *__restrict__ rp,
                                                    const int32_t *__restrict__ ci,
                                                    const double *__restrict__ val,
                                                    const double *__restrict__ x,
                                                    const double *__restrict__ b,
                                                    double *__restrict__ r,
                                                    double *__restrict__ partial, Bat bt) {
    __shared__ double sh[BLOCK / WAVE];
    x += blockIdx.y * bt.vec;
    b += blockIdx.y * bt.vec;
    r += blockIdx.y * bt.vec;
    partial += blockIdx.y * bt.part;
    const int lg = threadIdx.x % G;
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * (BLOCK / G);
    for (int64_t row = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) / G; row < n; row += stride) {
        double acc = 0.0;
        const int32_t e = rp[row + 1];
        for (int32_t k = rp[row] + lg; k < e; k += G) acc += val[k] * x[ci[k]];
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
        if (lg == 0) {
            const double ri = b[row] - acc;
            r[row] = ri;
            s += ri * ri;
        }
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// beta = ||r||; convergence / iteration-limit decision; restart bookkeeping
__global__ __launch_bounds__(BLOCK) void k_fin_residual(int nblk, const double *partial, Ctl *ctl,
                                                        double *g, double *hist, int initial,
                                                        Bat bt, uint64_t *tstamp) {
    __shared__ double res[1];
    partial += blockIdx.y * bt.part;
    ctl += blockIdx.y;
    g += blockIdx.y * bt.small;
    if (hist) hist += blockIdx.y * bt.hist;
    reduce_columns(nblk, 1, partial, 1, res);
    const double beta = sqrt(res[0]);
    if (threadIdx.x == 0) {
        const double rel = ctl->bnorm > 0.0 ? beta / ctl->bnorm : 0.0;
        ctl->rel_true = rel;
        ctl->beta = beta;
        if (initial) {
            if (hist) hist[0] = rel;
            const uint64_t now = (uint64_t)wall_clock64();
            if (tstamp) tstamp[0] = now;
            if (ctl->timeout_ticks) ctl->deadline = now + ctl->timeout_ticks;
            ctl->est_rel = rel;
        }
        if (!isfinite(beta)) {
            ctl->nonfinite = 1;
            ctl->solve_done = 1;
        } else if (beta <= ctl->target) {
            ctl->converged = 1;
            ctl->solve_done = 1;
        } else if (ctl->timed_out) {
            ctl->solve_done = 1;
        } else if (ctl->it >= ctl->maxiters) {
            ctl->solve_done = 1;
        } else if (!initial) {
            ctl->restarts += 1;
        }
        ctl->cycle_done = ctl->solve_done;
        ctl->kcols = 0;
        ctl->kuse = 0;
    }
    for (int k = threadIdx.x; k <= ctl->m; k += BLOCK) g[k] = (k == 0) ? beta : 0.0;
}

// ---------------------------------------------------------------------------
// Jacobi preconditioner (the weak baseline of Sec. 3, "Compared methods"):
// dinv = 1 / a_ii of the system matrix (prescaled when the system is), then
// z = dinv * v per Arnoldi step.  flag is set when a row has no nonzero
// diagonal entry.
// ---------------------------------------------------------------------------
__global__ void k_diag_inv(int64_t n, const int32_t *__restrict__ rp,
                           const int32_t *__restrict__ ci, const double *__restrict__ val,
                           double *__restrict__ dinv, int *flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double d = 0.0;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
        if (ci[k] == i) d = val[k];
    if (d == 0.0) atomicOr(flag, 1);
    dinv[i] = d != 0.0 ? 1.0 / d : 0.0;
}

template <typename KT>
__global__ __launch_bounds__(BLOCK) void k_jacobi(int64_t n, const double *__restrict__ dinv,
                                                  const KT *__restrict__ v, KT *__restrict__ z,
                                                  const Ctl *ctl) {
    if (ctl->cycle_done) return;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * BLOCK)
        z[i] = (KT)(dinv[i] * (double)v[i]);
}

// ---------------------------------------------------------------------------
// Inner-outer GMRES (the comparison method of Sec. 3, "Compared methods"):
// z_j is the result of one cycle of at most k unpreconditioned Arnoldi steps
// on A z = v_j from z = 0, ended once the Givens estimate is <= tol ||v_j||.
// The inner cycle runs on the step kernels below with a context of its own;
// k_inner_begin/k_inner_start set it up from v_j (r = v_j, x = 0, beta =
// ||v_j||), k_inner_end hands its float64 solution back as z_j.  Once the
// outer cycle is over they do nothing, and k_inner_start marks the inner
// cycle over too, so that every kernel of the inner cycle exits at entry.
// ---------------------------------------------------------------------------
template <typename KT>
__global__ __launch_bounds__(BLOCK) void k_inner_begin(int64_t n, const KT *__restrict__ v,
                                                       double *__restrict__ r,
                                                       double *__restrict__ x,
                                                       double *__restrict__ partial,
                                                       const Ctl *outer) {
    __shared__ double sh[BLOCK / WAVE];
    if (outer->cycle_done) return;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * BLOCK) {
        const double vi = (double)v[i];
        r[i] = vi;
        x[i] = 0.0;
        s += vi * vi;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(BLOCK) void k_inner_start(int nblk, const double *partial,
                                                       double tol, int k, Ctl *ctl, double *g,
                                                       const Ctl *outer) {
    __shared__ double res[1];
    if (outer->cycle_done) {
        if (threadIdx.x == 0) {
            ctl->cycle_done = 1;
            ctl->kcols = 0;
            ctl->kuse = 0;
        }
        return;
    }
    reduce_columns(nblk, 1, partial, 1, res);
    const double beta = sqrt(res[0]);
    if (threadIdx.x == 0) {
        Ctl c;
        memset(&c, 0, sizeof(c));
        c.m = k;
        c.maxiters = k;
        c.bnorm = beta;
        c.beta = beta;
        c.target = tol * beta;
        c.est = beta;
        c.est_rel = 1.0;
        c.rel_true = 1.0;
        c.cycle_done = beta > c.target ? 0 : 1;  // v = 0 or tol >= 1: z = 0
        *ctl = c;
    }
    for (int i = threadIdx.x; i <= k; i += BLOCK) g[i] = (i == 0) ? beta : 0.0;
}

template <typename KT>
__global__ __launch_bounds__(BLOCK) void k_inner_end(int64_t n, const double *__restrict__ x,
                                                     KT *__restrict__ z, const Ctl *outer) {
    if (outer->cycle_done) return;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * BLOCK)
        z[i] = (KT)x[i];
}

// ---------------------------------------------------------------------------
// v = src / div into vcur (contiguous), div = beta (cycle start) or
// h_{j+1,j}.  The basis column of v is written by the next step's first
// Gram-Schmidt pass, which reads that row of the basis anyway.  (For j >= 1
// of a single solve the division is done with the same expression by the
// encoder of a float32/bfloat16 network, else by the third Gram-Schmidt
// pass.)
// ---------------------------------------------------------------------------
template <typename KT, typename ST>
__global__ __launch_bounds__(BLOCK) void k_normalize(int64_t n, const ST *__restrict__ src,
                                                     KT *__restrict__ vcur, const Ctl *ctl,
                                                     int use_beta, Bat bt) {
    const int bi = blockIdx.y;
    ctl += bi;
    const int done = ctl->cycle_done;  // tested with the divisor in hand
    src += bi * bt.vec;
    const double div = use_beta ? ctl->beta : ctl->hnext;
    if (done) return;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * BLOCK)
        vcur[i * bt.vstep + bi] = (KT)((double)src[i] / div);
}

// tau triple (tau, sqrt(n)/tau, tau/sqrt(n)) of the network input, Eq. (6).
// Every network input of the solver is a basis vector v = w / ||w||, whose
// norm is 1 in exact arithmetic; tau is taken as that 1 (the norm of the
// rounded vector differs from it by about one unit of its precision), which
// spares a global reduction per Arnoldi step.  In a batch (gridDim.y
// right-hand sides) block (0, 0) also records in *all_done whether every
// right-hand side has ended its cycle (the network launches of the next step
// are then skipped).  scaled = 0 (a network without Eq. (6)): (1, 1, 1).
__global__ void k_unit_tau(int64_t n, double *tau, const Ctl *ctl, int *all_done, int scaled) {
    if (threadIdx.x != 0) return;
    if (all_done && blockIdx.y == 0) {
        int done = 1;
        for (int k = 0; k < (int)gridDim.y; ++k) done &= ctl[k].cycle_done ? 1 : 0;
        *all_done = done;
    }
    ctl += blockIdx.y;
    if (ctl->cycle_done) return;
    tau += 3 * blockIdx.y;
    const double tv = 1.0, sqn = scaled ? sqrt((double)n) : 1.0;
    tau[0] = tv;
    tau[1] = sqn / tv;
    tau[2] = tv / sqn;
}

// ---------------------------------------------------------------------------
// Gram-Schmidt passes over the interleaved basis (8 lanes per row, lane q
// owns entries k = 4 (q + 8 u) + e).  MODE 0: dots V_j^T w and ||w||^2;
// column j (v_j) is taken from vcur and stored into the basis here.
// MODE 1: w -= V_j hprev, then dots and ||w||^2 of the updated w.  MODE 2:
// w -= V_j hprev only (its norm follows from MODE 1's sums, k_fin_givens).
// MODE 3 (one right-hand side): MODE 2, and the next basis vector
// v_{j+1} = w / h_{j+1,j} into vout with the expression of k_normalize.
// MODE 4: MODE 0 with the SpMV w = A z_j fused in front: the eight lanes of a
// row take its nonzeros q, q + 8, ... in order (FP32 products and sums, FP64
// for a float64 basis), add their partial sums across the lanes by xor 4, 2,
// 1, and lane 0 stores w_i; the dots then use w_i as MODE 0 uses w.
// Entries k > j are masked by selection (they may hold an older cycle).
// ---------------------------------------------------------------------------
// The SpMV operands of the first pass when it forms w = A z_j itself
// (MODE 4): CSR of the system matrix in the Krylov precision and z_j, read
// at ci * zstep + (right-hand side) for a batch whose network outputs are
// packed [n][nb].
template <typename KT> struct SpIn {
    const int32_t *rp = nullptr, *ci = nullptr;
    const KT *val = nullptr, *z = nullptr;
    int64_t zstep = 1;
};

template <typename KT> struct Quad;
template <> struct Quad<float> {
    static __device__ __forceinline__ void load_raw(const float *p, float *o) {
        const float4 v = *reinterpret_cast<const float4 *>(p);
        o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
    }
};
template <> struct Quad<double> {
    static __device__ __forceinline__ void load_raw(const double *p, double *o) {
        const double2 a = *reinterpret_cast<const double2 *>(p);
        const double2 b = *reinterpret_cast<const double2 *>(p + 2);
        o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
    }
};

template <typename KT, int MP, int MODE>
__global__ __launch_bounds__(BLOCK) void k_cgs(int64_t n, int64_t rpb, KT *__restrict__ V,
                                               int j, KT *__restrict__ w,
                                               const double *__restrict__ hprev,
                                               double *__restrict__ partial, int pstride,
                                               const Ctl *ctl, Bat bt,
                                               const KT *__restrict__ vcur,
                                               KT *__restrict__ vout, int vj_in_V = 0,
                                               SpIn<KT> sp = SpIn<KT>()) {
    ctl += blockIdx.y;
    // the end-of-cycle flag is tested only after the first round of loads
    // has been issued (the loads are in bounds either way), so its latency
    // overlaps theirs
    const int done = ctl->cycle_done;
    constexpr bool D0 = MODE == 0 || MODE == 4;  // the first pass (dots, column j)
    V += blockIdx.y * bt.basis;
    w += blockIdx.y * bt.vec;
    if (D0) vcur += blockIdx.y;
    if (MODE == 4) sp.z += blockIdx.y;
    if (hprev) hprev += blockIdx.y * bt.small;
    partial += blockIdx.y * bt.part;
    constexpr int NU = MP / 32, NA = 4 * NU;
    const int t = threadIdx.x, q = t % 8, g = t / 8;
    const int64_t i0 = (int64_t)blockIdx.x * rpb;
    const int64_t i1 = (i0 + rpb < n) ? i0 + rpb : n;
    double acc[NA], hp[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) {
        acc[a] = 0.0;
        const int k = 4 * (q + 8 * (a / 4)) + a % 4;
        hp[a] = (MODE >= 1 && MODE <= 3 && k <= j) ? hprev[k] : 0.0;
    }
    double nrm = 0.0;
    // every row of the block in one round of loads (rpb = RPP * RU at a
    // basis pitch of 32)
    constexpr int RU0 = 8 * 32 / MP;
    constexpr int RU = RU0 < 2 ? 2 : RU0;
    // the lane owning column j (MODE 0 stores it)
    const bool owner_j = q == ((j >> 2) & 7);
    double hdiv = 1.0;
    bool first = true;
    using Acc = typename std::conditional<sizeof(KT) == 8, double, float>::type;
    for (int64_t ib = i0 + g; ib < i1; ib += (int64_t)RPP * RU) {
        KT v[RU][NA];
        KT wold[RU], vj[RU];
        int32_t kb[RU], ke[RU];
#pragma unroll
        for (int ru = 0; ru < RU; ++ru) {
            const int64_t i = ib + (int64_t)ru * RPP;
            const int64_t ic = i < i1 ? i : i1 - 1;
            if (MODE == 4) {
                kb[ru] = sp.rp[ic];
                ke[ru] = sp.rp[ic + 1];
            }
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int c = q + 8 * u;
                if (4 * c <= j) {
                    Quad<KT>::load_raw(V + ic * MP + 4 * c, &v[ru][4 * u]);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[ru][4 * u + e] = (KT)0;
                }
            }
            if (MODE != 4) wold[ru] = w[ic];
            if (D0 && !vj_in_V) vj[ru] = vcur[ic * bt.vstep];
        }
        if (MODE == 4) {
            // w_i = (A z)_i: every lane's first nonzero in flight for all rows,
            // then the rest of longer rows
            int32_t cc[RU];
            KT av[RU];
#pragma unroll
            for (int ru = 0; ru < RU; ++ru) {
                const int32_t k = kb[ru] + q;
                const int32_t kk = k < ke[ru] ? k : (ke[ru] > 0 ? ke[ru] - 1 : 0);
                cc[ru] = sp.ci[kk];
                av[ru] = sp.val[kk];
            }
            KT xv[RU];
#pragma unroll
            for (int ru = 0; ru < RU; ++ru) xv[ru] = sp.z[(int64_t)cc[ru] * sp.zstep];
#pragma unroll
            for (int ru = 0; ru < RU; ++ru) {
                Acc p = kb[ru] + q < ke[ru] ? (Acc)av[ru] * (Acc)xv[ru] : (Acc)0;
                for (int32_t k = kb[ru] + q + 8; k < ke[ru]; k += 8)
                    p += (Acc)sp.val[k] * (Acc)sp.z[(int64_t)sp.ci[k] * sp.zstep];
                p += __shfl_xor(p, 4, WAVE);
                p += __shfl_xor(p, 2, WAVE);
                p += __shfl_xor(p, 1, WAVE);
                wold[ru] = (KT)p;
            }
        }
        if (first) {
            if (done) return;
            if (MODE == 3) hdiv = ctl->hnext;
            first = false;
        }
#pragma unroll
        for (int ru = 0; ru < RU; ++ru) {
            const int64_t i = ib + (int64_t)ru * RPP;
            const bool ok = i < i1;
            if (D0 && !vj_in_V) {  // column j from vcur, stored into the basis
#pragma unroll
                for (int a = 0; a < NA; ++a)
                    if (4 * (q + 8 * (a / 4)) + a % 4 == j) v[ru][a] = vj[ru];
                if (ok && owner_j) V[i * MP + j] = vj[ru];
            }
            double vv[NA];
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                const int k = 4 * (q + 8 * (a / 4)) + a % 4;
                vv[a] = (k <= j) ? (double)v[ru][a] : 0.0;
            }
            double wi;
            if (D0) {
                if (MODE == 4 && ok && q == 0) w[i] = wold[ru];
                wi = ok ? (double)wold[ru] : 0.0;
            } else {
                double corr = 0.0;
#pragma unroll
                for (int a = 0; a < NA; ++a) corr += hp[a] * vv[a];
                corr += __shfl_xor(corr, 1, WAVE);
                corr += __shfl_xor(corr, 2, WAVE);
                corr += __shfl_xor(corr, 4, WAVE);
                const KT wn = (KT)((double)wold[ru] - corr);
                if (ok && q == 0) w[i] = wn;
                if (MODE == 3 && ok && q == 0) vout[i] = (KT)((double)wn / hdiv);
                wi = ok ? (double)wn : 0.0;
            }
            if (MODE <= 1 || MODE == 4) {
#pragma unroll
                for (int a = 0; a < NA; ++a) acc[a] += vv[a] * wi;
            }
            if ((MODE <= 1 || MODE == 4) && q == 0) nrm += wi * wi;
        }
    }
    if (done) return;                              // rows of no round (the tail block)
    if constexpr (MODE == 2 || MODE == 3) return;  // no sums
    __shared__ double sh[BLOCK / WAVE][8 * NA + 1];
    const int lane = t % WAVE, wv = t / WAVE;
    if (MODE <= 1 || MODE == 4) {
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            double s = acc[a];
            s += __shfl_xor(s, 8, WAVE);
            s += __shfl_xor(s, 16, WAVE);
            s += __shfl_xor(s, 32, WAVE);
            if (lane < 8) sh[wv][lane * NA + a] = s;
        }
    }
    {
        const double s = wave_sum(nrm);
        if (lane == 0) sh[wv][8 * NA] = s;
    }
    __syncthreads();
    double *dst = partial + (int64_t)blockIdx.x * pstride;
    if (MODE <= 1 || MODE == 4) {
        for (int k = t; k <= j; k += BLOCK) {
            const int c = k / 4, e = k % 4, qq = c % 8, u = c / 8;
            double s = 0.0;
            for (int w2 = 0; w2 < BLOCK / WAVE; ++w2) s += sh[w2][qq * NA + 4 * u + e];
            dst[k] = s;
        }
    }
    if (t == 0) {
        double s = 0.0;
        for (int w2 = 0; w2 < BLOCK / WAVE; ++w2) s += sh[w2][8 * NA];
        dst[pstride - 1] = s;
    }
}

// First dots finalize, one block per column: block k <= j sums h1[k] = (V^T w)_k,
// block j + 1 the squared norm slot (||A z_j||), each over the pass's block
// partials in one fixed order (sum_partials), so the bits do not depend on
// scheduling.  Launched with j + 2 blocks per right-hand side.
__global__ __launch_bounds__(BLOCK) void k_fin_dots(int nblk, int j, const double *partial,
                                                    int pstride, double *hout, Ctl *ctl, Bat bt) {
    ctl += blockIdx.y;
    // the end-of-cycle flag is tested once the partials have been read (in
    // range either way), so that the two loads share one round trip
    const int done = ctl->cycle_done;
    const int k = blockIdx.x;
    partial += blockIdx.y * bt.part;
    hout += blockIdx.y * bt.small;
    __shared__ double sh[BLOCK / WAVE];
    const double s = sum_partials(nblk, partial + (k <= j ? k : pstride - 1), pstride, sh);
    if (done) return;
    if (threadIdx.x == 0) {
        if (k <= j) hout[k] = s;
        else ctl->wnorm0 = sqrt(s);
    }
}

// End of an Arnoldi step: h2[0..j] = V^T w1 and h2[j + 1] = ||w1||^2 (w1: w
// after the first projection);
// h_{j+1,j} = ||w1 - V h2|| = sqrt(||w1||^2 - ||h2||^2), exact for
// orthonormal V and h2 = V^T w1 (h2 is a small correction, so nothing
// cancels; a negative difference from rounding counts as 0, a breakdown);
// column j of H-bar = h1 + h2, Givens rotation, residual estimate,
// end-of-cycle decision.  The third pass then only updates w.  Inputs are
// staged in LDS by all threads, the sequential rotation runs in one thread.
// done: the block's end-of-cycle flag, read by the caller and tested here
// once the inputs are staged (nothing is written when it is set).
__device__ void givens_step(int j, const double *h1, const double *h2, Ctl *ctl, double *H,
                            double *H0, double *cs, double *sn, double *g, double *hist,
                            uint64_t *tstamp, int done) {
    __shared__ double res[MAXCOL + 1];
    __shared__ double col[MAXCOL], scs[MAXCOL], ssn[MAXCOL];
    __shared__ double gj_s;
    const int m = ctl->m;
    for (int i = threadIdx.x; i < j; i += BLOCK) {
        scs[i] = cs[i];
        ssn[i] = sn[i];
    }
    if (threadIdx.x == 0) gj_s = g[j];
    for (int i = threadIdx.x; i <= j + 1; i += BLOCK) res[i] = h2[i];
    __syncthreads();
    if (done) return;
    for (int i = threadIdx.x; i <= j; i += BLOCK) {
        col[i] = h1[i] + res[i];
        H0[(int64_t)i * m + j] = col[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double hh = 0.0;
        for (int i = 0; i <= j; ++i) hh += res[i] * res[i];
        const double d2 = res[j + 1] - hh;
        const double hn = d2 < 0.0 ? 0.0 : sqrt(d2);  // NaN stays NaN
        H0[(int64_t)(j + 1) * m + j] = hn;
        col[j + 1] = hn;
        // previous rotations (Saad 2003, Sec. 6.5.3), then a new one
        for (int i = 0; i < j; ++i) {
            const double a0 = col[i], b0 = col[i + 1];
            col[i] = scs[i] * a0 + ssn[i] * b0;
            col[i + 1] = -ssn[i] * a0 + scs[i] * b0;
        }
        const double a0 = col[j];
        const double rho = hypot(a0, hn);
        double c = 1.0, s = 0.0;
        if (rho != 0.0) {
            c = a0 / rho;
            s = hn / rho;
        }
        cs[j] = c;
        sn[j] = s;
        col[j] = rho;
        col[j + 1] = 0.0;
        const double gj = gj_s;
        g[j + 1] = -s * gj;
        g[j] = c * gj;
        const double est = fabs(s * gj);
        ctl->est = est;
        ctl->est_rel = est / ctl->bnorm;
        ctl->it += 1;
        ctl->kcols = j + 1;
        if (hist) hist[ctl->it] = est / ctl->bnorm;
        if (tstamp) tstamp[ctl->it] = (uint64_t)wall_clock64();
        if (!isfinite(hn) || !isfinite(rho) || !isfinite(est)) {
            ctl->nonfinite = 1;
            ctl->solve_done = 1;
            ctl->cycle_done = 1;
        } else if (hn <= 1e-14 * ctl->wnorm0) {
            ctl->breakdowns += 1;
            ctl->cycle_done = 1;
        } else {
            ctl->hnext = hn;
            if (est <= ctl->target || j + 1 >= m || ctl->it >= ctl->maxiters) ctl->cycle_done = 1;
        }
        if (ctl->deadline && (uint64_t)wall_clock64() >= ctl->deadline) {
            ctl->timed_out = 1;
            ctl->cycle_done = 1;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= j + 1; i += BLOCK) H[(int64_t)i * m + j] = col[i];
}

// The second pass's sums, one block per column, the same way as k_fin_dots:
// h2[k] = (V^T w1)_k for k <= j and h2[j + 1] = ||w1||^2, for k_fin_givens.
// Launched with j + 2 blocks per right-hand side.  (Completing the step in
// the last block to finish, behind a ticket, was measured slower: the
// fences that make the other blocks' sums visible cost more than a launch.)
__global__ __launch_bounds__(BLOCK) void k_fin_sums2(int nblk, int j, const double *partial,
                                                     int pstride, double *h2, const Ctl *ctl,
                                                     Bat bt) {
    ctl += blockIdx.y;
    const int k = blockIdx.x;
    partial += blockIdx.y * bt.part;
    h2 += blockIdx.y * bt.small;
    __shared__ double sh[BLOCK / WAVE];
    const int done = ctl->cycle_done;  // tested after the partials, as in k_fin_dots
    const double s = sum_partials(nblk, partial + (k <= j ? k : pstride - 1), pstride, sh);
    if (done) return;
    if (threadIdx.x == 0) h2[k] = s;
}

// One block: the rest of the Arnoldi step (givens_step) from h1 and h2.
__global__ __launch_bounds__(BLOCK) void k_fin_givens(int j, const double *h1, const double *h2,
                                                      Ctl *ctl, double *H, double *H0,
                                                      double *cs, double *sn, double *g,
                                                      double *hist, Bat bt, uint64_t *tstamp) {
    const int bi = blockIdx.y;
    ctl += bi;
    givens_step(j, h1 + bi * bt.small, h2 + bi * bt.small, ctl, H + bi * bt.hess,
                H0 + bi * bt.hess, cs + bi * bt.small, sn + bi * bt.small, g + bi * bt.small,
                hist ? hist + bi * bt.hist : nullptr, tstamp, ctl->cycle_done);
}

// y = R^{-1} g on the leading columns with nonzero pivots: the triangle and g
// are staged in LDS by all threads, then one thread substitutes backwards.
__global__ __launch_bounds__(BLOCK) void k_backsolve(Ctl *ctl, const double *H, const double *g,
                                                     double *y, Bat bt) {
    ctl += blockIdx.y;
    H += blockIdx.y * bt.hess;
    g += blockIdx.y * bt.small;
    y += blockIdx.y * bt.small;
    __shared__ double R[64 * 64];
    __shared__ double gs[64], ys[64];
    __shared__ int kk_s;
    const int m = ctl->m;
    const int kc = ctl->kcols;
    const bool staged = kc <= 64;
    if (staged) {
        for (int e = threadIdx.x; e < kc * kc; e += BLOCK) {
            const int i = e / kc, q = e % kc;
            R[i * 64 + q] = (q >= i) ? H[(int64_t)i * m + q] : 0.0;
        }
        for (int i = threadIdx.x; i < kc; i += BLOCK) gs[i] = g[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int kk = kc;
        if (staged) {
            while (kk > 0 && R[(kk - 1) * 64 + (kk - 1)] == 0.0) --kk;
            for (int i = kk - 1; i >= 0; --i) {
                double acc = gs[i];
                for (int q = i + 1; q < kk; ++q) acc -= R[i * 64 + q] * ys[q];
                ys[i] = acc / R[i * 64 + i];
            }
        } else {
            while (kk > 0 && H[(int64_t)(kk - 1) * m + (kk - 1)] == 0.0) --kk;
            for (int i = kk - 1; i >= 0; --i) {
                double acc = g[i];
                for (int q = i + 1; q < kk; ++q) acc -= H[(int64_t)i * m + q] * y[q];
                y[i] = acc / H[(int64_t)i * m + i];
            }
        }
        kk_s = kk;
        ctl->kuse = kk;
    }
    __syncthreads();
    if (staged)
        for (int i = threadIdx.x; i < kk_s; i += BLOCK) y[i] = ys[i];
}

// x += Z y (float64 accumulation).  Z column-major (network outputs), or the
// interleaved basis itself when M = I (then z_k = v_k).
template <typename KT, int MP, bool FROM_V>
__global__ __launch_bounds__(BLOCK) void k_update_x(int64_t n, const KT *__restrict__ Z,
                                                    const double *__restrict__ y, const Ctl *ctl,
                                                    double *__restrict__ x) {
    const int ku = ctl->kuse;
    if (ku == 0) return;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * BLOCK) {
        double acc = 0.0;
        if (FROM_V)
            for (int k = 0; k < ku; ++k) acc += (double)Z[i * MP + k] * y[k];
        else
            for (int k = 0; k < ku; ++k) acc += (double)Z[(int64_t)k * n + i] * y[k];
        x[i] += acc;
    }
}

// x_b += Z_b y_b for a batch whose network outputs are packed: Zp holds step
// k's outputs of all right-hand sides at Zp[k * n * nb + i * nb + b].  One
// thread per (row, right-hand side), right-hand side fastest; the sum over k
// runs in the order of k_update_x.
template <typename KT>
__global__ __launch_bounds__(BLOCK) void k_update_x_pk(int64_t n, int nb, const KT *__restrict__ Zp,
                                                       const double *__restrict__ y,
                                                       const Ctl *ctl, double *__restrict__ x,
                                                       Bat bt) {
    const int64_t total = n * nb;
    for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * BLOCK) {
        const int b = (int)(e % nb);
        const int64_t i = e / nb;
        const int ku = ctl[b].kuse;
        if (ku == 0) continue;
        const double *yb = y + b * bt.small;
        double acc = 0.0;
        for (int k = 0; k < ku; ++k) acc += (double)Zp[(int64_t)k * total + e] * yb[k];
        x[b * bt.vec + i] += acc;
    }
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
static int basis_pitch(int m) {
    int mp = 32;
    while (mp < m + 1) mp *= 2;
    return mp;
}

// rows per block of the Gram-Schmidt kernels: one round of loads per lane
// (RPP * 8 rows) unless n needs more than 1024 such blocks.  (RPP * 16 rows
// per block, half the blocks with twice the loads in flight per lane, held
// 233 registers against about half that and ran the unpreconditioned step
// 54.3 us against 48.0 at n = 2^18, the network step 153.9 against 152.2.)
static int64_t cgs_rpb(int64_t n) {
    int64_t rpb = RPP * 8;
    while ((n + rpb - 1) / rpb > 1024) rpb *= 2;
    return rpb;
}

void solve_ctx_free(SolveCtx *c) {
    if (!c) return;
    if (c->inner) {
        solve_ctx_free(c->inner);
        delete c->inner;
    }
    if (c->inner_x) (void)hipFree(c->inner_x);
    void *ptrs[] = {c->V,  c->Z,  c->w,  c->r,  c->act[0], c->act[1], c->tau, c->H,
                    c->H0, c->cs, c->sn, c->g,  c->y,      c->h1,     c->h2,  c->hist,
                    c->partial, c->counters, c->ctl, c->vcur, c->tstamp};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (c->ctl_host) (void)hipHostFree(c->ctl_host);
    if (c->ev) (void)hipEventDestroy(c->ev);
    *c = SolveCtx();
}

size_t solve_ctx_bytes(int64_t n, int m, int maxiters, gnp_precision prec, int act_d) {
    const size_t kb = (prec == GNP_F64) ? 8 : 4;
    const int mp = basis_pitch(m);
    const int64_t cap = std::max(maxiters, 128);
    const int64_t nb_cgs = (n + cgs_rpb(n) - 1) / cgs_rpb(n);
    const int64_t npartial = std::max<int64_t>(nb_cgs * (mp + 1), 2048);
    size_t b = kb * (size_t)n * (mp + m + 2) + sizeof(double) * n;
    if (act_d > 0) b += 2 * kb * (size_t)n * act_d;
    b += sizeof(double) * (4 + 2 * (m + 1) * m + 3 * m + 3 * (m + 1) + 2 * (cap + 1) + npartial);
    b += sizeof(Ctl);
    return b;
}

gnp_status solve_ctx_prepare(SolveCtx *c, gnp_system *sys, int m, int maxiters,
                             gnp_precision prec, int act_d) {
    const size_t kb = (prec == GNP_F64) ? 8 : 4;
    if (c->sys == sys && c->m == m && c->kbytes == kb && c->maxiters_cap >= maxiters &&
        c->act_d >= act_d)
        return GNP_OK;
    solve_ctx_free(c);
    c->sys = sys;
    c->m = m;
    c->mp = basis_pitch(m);
    c->n = sys->n;
    c->prec = prec;
    c->kbytes = kb;
    c->maxiters_cap = std::max(maxiters, 128);
    c->act_d = act_d;
    const int64_t n = sys->n;
    GNP_HIP(hipMalloc(&c->V, kb * (size_t)n * c->mp));
    GNP_HIP(hipMemset(c->V, 0, kb * (size_t)n * c->mp));
    GNP_HIP(hipMalloc(&c->Z, kb * (size_t)n * m));
    GNP_HIP(hipMalloc(&c->vcur, kb * (size_t)n));
    GNP_HIP(hipMalloc(&c->w, kb * (size_t)n));
    GNP_HIP(hipMalloc(&c->r, sizeof(double) * n));
    // activations: float64 / float32 elements (bfloat16 uses half of a float32 buffer)
    if (act_d > 0)
        for (int i = 0; i < 2; ++i) GNP_HIP(hipMalloc(&c->act[i], kb * (size_t)n * act_d));
    GNP_HIP(hipMalloc(&c->tau, sizeof(double) * 4));
    GNP_HIP(hipMalloc(&c->H, sizeof(double) * (m + 1) * m));
    GNP_HIP(hipMalloc(&c->H0, sizeof(double) * (m + 1) * m));
    GNP_HIP(hipMalloc(&c->cs, sizeof(double) * m));
    GNP_HIP(hipMalloc(&c->sn, sizeof(double) * m));
    GNP_HIP(hipMalloc(&c->g, sizeof(double) * (m + 1)));
    GNP_HIP(hipMalloc(&c->y, sizeof(double) * m));
    GNP_HIP(hipMalloc(&c->h1, sizeof(double) * (m + 1)));
    GNP_HIP(hipMalloc(&c->h2, sizeof(double) * (m + 1)));
    GNP_HIP(hipMalloc(&c->hist, sizeof(double) * (c->maxiters_cap + 1)));
    GNP_HIP(hipMalloc(&c->tstamp, sizeof(uint64_t) * (c->maxiters_cap + 1)));
    const int64_t nb_cgs = (n + cgs_rpb(n) - 1) / cgs_rpb(n);
    c->npartial = std::max<int64_t>(nb_cgs * (c->mp + 1), 2048);
    GNP_HIP(hipMalloc(&c->partial, sizeof(double) * c->npartial));
    GNP_HIP(hipMalloc(&c->ctl, sizeof(Ctl)));
    GNP_HIP(hipHostMalloc(&c->ctl_host, sizeof(Ctl), hipHostMallocDefault));
    GNP_HIP(hipEventCreateWithFlags(&c->ev, hipEventDisableTiming));
    return GNP_OK;
}

template <typename KT, int MP>
static gnp_status launch_cycle_mp(SolveCtx *c, gnp_model *model, int nsteps, double *x,
                                  hipStream_t st) {
    gnp_system *s = c->sys;
    const int64_t n = s->n;
    KT *V = (KT *)c->V, *Z = (KT *)c->Z, *w = (KT *)c->w, *vcur = (KT *)c->vcur;
    const KT *val;
    if constexpr (sizeof(KT) == 8) val = (const KT *)s->val64;
    else val = (const KT *)s->val32;
    const int sg = stream_grid(n);
    const int64_t rpb = cgs_rpb(n);
    const int gcgs = (int)((n + rpb - 1) / rpb);
    const int pstride = MP + 1;
    const int *skip = &c->ctl->cycle_done;
    // the basis vector v_j (j >= 1) = w / h_{j,j-1}: formed by the encoder of
    // a float32/bfloat16 network as it reads w (it also stores v_j to vcur),
    // else by its own kernel at the end of step j - 1; with a basis of pitch
    // 32 that encoder also applies step j - 1's second correction w -= V h2,
    // so that pass is not launched (the encoder takes the tau triple of Eq. (6),
    // so a network without that scaling keeps the separate kernels)
    const bool v_in_encoder = model && c->prec != GNP_F64 && model->scaled;
    const bool corr_in_encoder = v_in_encoder && MP == 32;
    // Jacobi: z_j = D^{-1} v_j; with any preconditioner z_j is kept in Z
    const bool jac = !model && c->precond == PRECOND_JACOBI;
    const bool inner = !model && c->precond == PRECOND_GMRES;
    const bool flex = model || jac || inner;
    hipLaunchKernelGGL((k_normalize<KT, double>), dim3(sg), dim3(BLOCK), 0, st, n, c->r, vcur,
                       c->ctl, 1, Bat{});
    if (model)
        hipLaunchKernelGGL(k_unit_tau, dim3(1), dim3(WAVE), 0, st, n, c->tau, c->ctl,
                           (int *)nullptr, model->scaled);
    for (int j = 0; j < nsteps; ++j) {
        KT *zj = flex ? Z + (int64_t)j * n : vcur;
        const bool fuse = v_in_encoder && j > 0;
        BasisNext bn;
        if (fuse) {
            bn.hdiv = &c->ctl->hnext;
            bn.vout = (float *)vcur;
            if (corr_in_encoder) {
                bn.V = (const float *)V;
                bn.h = c->h2;
                bn.j = j - 1;
                bn.Vout = (float *)V;  // v_j into column j of the basis ...
                bn.vout = nullptr;     // ... which the first pass then reads as it is
            }
        }
        if (model)
            GNP_TRY(forward_launch(model, c->prec, fuse ? w : vcur, zj, 1, c->tau, c->act[0],
                                   c->act[1], skip, st, nullptr, fuse ? &bn : nullptr));
        else if (jac)
            hipLaunchKernelGGL((k_jacobi<KT>), dim3(sg), dim3(BLOCK), 0, st, n,
                               (const double *)s->dinv64, (const KT *)vcur, zj,
                               (const Ctl *)c->ctl);
        else if (inner) {
            // float64 bases accumulate the inner solution in z_j itself
            SolveCtx *ic = c->inner;
            double *xin = sizeof(KT) == 8 ? (double *)zj : c->inner_x;
            hipLaunchKernelGGL((k_inner_begin<KT>), dim3(sg), dim3(BLOCK), 0, st, n,
                               (const KT *)vcur, ic->r, xin, ic->partial, (const Ctl *)c->ctl);
            hipLaunchKernelGGL(k_inner_start, dim3(1), dim3(BLOCK), 0, st, sg,
                               (const double *)ic->partial, c->inner_tol, c->inner_k, ic->ctl,
                               ic->g, (const Ctl *)c->ctl);
            GNP_TRY((launch_cycle_mp<KT, 32>(ic, nullptr, c->inner_k, xin, st)));
            if (sizeof(KT) != 8)
                hipLaunchKernelGGL((k_inner_end<KT>), dim3(sg), dim3(BLOCK), 0, st, n,
                                   (const double *)xin, zj, (const Ctl *)c->ctl);
        }
        // w = A z_j and the first Gram-Schmidt pass in one kernel
        SpIn<KT> sp;
        sp.rp = s->rp;
        sp.ci = s->ci;
        sp.val = val;
        sp.z = zj;
        hipLaunchKernelGGL((k_cgs<KT, MP, 4>), dim3(gcgs), dim3(BLOCK), 0, st, n, rpb, V, j, w,
                           (const double *)nullptr, c->partial, pstride, (const Ctl *)c->ctl,
                           Bat{}, (const KT *)vcur, (KT *)nullptr,
                           (int)(fuse && corr_in_encoder), sp);
        hipLaunchKernelGGL(k_fin_dots, dim3(j + 2), dim3(BLOCK), 0, st, gcgs, j,
                           (const double *)c->partial, pstride, c->h1, c->ctl, Bat{});
        hipLaunchKernelGGL((k_cgs<KT, MP, 1>), dim3(gcgs), dim3(BLOCK), 0, st, n, rpb, V, j, w,
                           (const double *)c->h1, c->partial, pstride, (const Ctl *)c->ctl,
                           Bat{}, (const KT *)nullptr, (KT *)nullptr);
        hipLaunchKernelGGL(k_fin_sums2, dim3(j + 2), dim3(BLOCK), 0, st, gcgs, j,
                           (const double *)c->partial, pstride, c->h2, (const Ctl *)c->ctl,
                           Bat{});
        hipLaunchKernelGGL(k_fin_givens, dim3(1), dim3(BLOCK), 0, st, j, (const double *)c->h1,
                           (const double *)c->h2, c->ctl, c->H, c->H0, c->cs, c->sn, c->g,
                           c->hist, Bat{}, c->tstamp);
        if (!v_in_encoder)  // third pass and v_{j+1} = w / h_{j+1,j} in one kernel
            hipLaunchKernelGGL((k_cgs<KT, MP, 3>), dim3(gcgs), dim3(BLOCK), 0, st, n, rpb, V, j,
                               w, (const double *)c->h2, c->partial, pstride,
                               (const Ctl *)c->ctl, Bat{}, (const KT *)nullptr, vcur);
        else if (!corr_in_encoder)
            hipLaunchKernelGGL((k_cgs<KT, MP, 2>), dim3(gcgs), dim3(BLOCK), 0, st, n, rpb, V, j,
                               w, (const double *)c->h2, c->partial, pstride,
                               (const Ctl *)c->ctl, Bat{}, (const KT *)nullptr, (KT *)nullptr);
        if (!v_in_encoder) {
            if (model)
                hipLaunchKernelGGL(k_unit_tau, dim3(1), dim3(WAVE), 0, st, n, c->tau, c->ctl,
                                   (int *)nullptr, model->scaled);
        }
    }
    hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(BLOCK), 0, st, c->ctl, c->H, c->g, c->y, Bat{});
    if (flex)
        hipLaunchKernelGGL((k_update_x<KT, MP, false>), dim3(sg), dim3(BLOCK), 0, st, n,
                           (const KT *)Z, c->y, c->ctl, x);
    else
        hipLaunchKernelGGL((k_update_x<KT, MP, true>), dim3(sg), dim3(BLOCK), 0, st, n,
                           (const KT *)V, c->y, c->ctl, x);
    GNP_HIP(hipGetLastError());
    return GNP_OK;
}

template <typename KT>
static gnp_status launch_cycle(SolveCtx *c, gnp_model *model, int nsteps, double *x,
                               hipStream_t st) {
    switch (c->mp) {
        case 32: return launch_cycle_mp<KT, 32>(c, model, nsteps, x, st);
        case 64: return launch_cycle_mp<KT, 64>(c, model, nsteps, x, st);
        case 128: return launch_cycle_mp<KT, 128>(c, model, nsteps, x, st);
        case 256: return launch_cycle_mp<KT, 256>(c, model, nsteps, x, st);
        default: return fail(GNP_EINVAL, "unsupported basis pitch");
    }
}

static void launch_residual(SolveCtx *c, const double *b, const double *x, int initial,
                            hipStream_t st) {
    gnp_system *s = c->sys;
    const int64_t n = s->n;
    const double avg = (double)s->nnz / (double)n;
    const int G = avg <= 12.0 ? 4 : (avg <= 24.0 ? 8 : 16);
    const int grid = grid_for(n, BLOCK / G, 1024);
    if (G == 4)
        hipLaunchKernelGGL(k_residual<4>, dim3(grid), dim3(BLOCK), 0, st, n, s->rp, s->ci,
                           s->val64, x, b, c->r, c->partial, Bat{});
    else if (G == 8)
        hipLaunchKernelGGL(k_residual<8>, dim3(grid), dim3(BLOCK), 0, st, n, s->rp, s->ci,
                           s->val64, x, b, c->r, c->partial, Bat{});
    else
        hipLaunchKernelGGL(k_residual<16>, dim3(grid), dim3(BLOCK), 0, st, n, s->rp, s->ci,
                           s->val64, x, b, c->r, c->partial, Bat{});
    hipLaunchKernelGGL(k_fin_residual, dim3(1), dim3(BLOCK), 0, st, grid,
                       (const double *)c->partial, c->ctl, c->g, c->hist, initial, Bat{},
                       c->tstamp);
}

gnp_status solve_begin(SolveCtx *c, const double *b, const double *x, int m, double rtol,
                       int maxiters, hipStream_t st) {
    const int64_t n = c->sys->n;
    Ctl init;
    memset(&init, 0, sizeof(init));
    init.m = m;
    init.maxiters = maxiters;
    if (c->timeout_s > 0.0) {
        int dev = 0, khz = 0;
        GNP_HIP(hipGetDevice(&dev));
        GNP_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        if (khz <= 0) return fail(GNP_EDEVICE, "device reports no wall-clock rate");
        const double ticks = c->timeout_s * 1e3 * (double)khz;
        init.timeout_ticks = ticks < 1.0 ? 1 : ticks > 1e18 ? (uint64_t)1e18 : (uint64_t)ticks;
    }
    *c->ctl_host = init;
    GNP_HIP(hipMemcpyAsync(c->ctl, c->ctl_host, sizeof(Ctl), hipMemcpyHostToDevice, st));
    const int sg = stream_grid(n);
    hipLaunchKernelGGL(k_sumsq, dim3(sg), dim3(BLOCK), 0, st, n, b, c->partial, Bat{});
    hipLaunchKernelGGL(k_fin_bnorm, dim3(1), dim3(BLOCK), 0, st, sg, (const double *)c->partial,
                       rtol, c->ctl, Bat{});
    launch_residual(c, b, x, 1, st);
    GNP_HIP(hipMemcpyAsync(c->ctl_host, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    return GNP_OK;
}

gnp_status solve_next(SolveCtx *c, gnp_model *model, const double *b, double *x, int m,
                      int maxiters, hipStream_t st) {
    const int it0 = c->ctl_host->it;
    const int nsteps = std::min(m, maxiters - it0);
    if (c->prec == GNP_F64) GNP_TRY(launch_cycle<double>(c, model, nsteps, x, st));
    else GNP_TRY(launch_cycle<float>(c, model, nsteps, x, st));
    launch_residual(c, b, x, 0, st);
    GNP_HIP(hipMemcpyAsync(c->ctl_host, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    return GNP_OK;
}

void solve_info_from(const Ctl &h, gnp_solve_info *info) {
    if (!info) return;
    info->iters = h.it;
    info->restarts = h.restarts;
    info->converged = h.converged;
    info->breakdowns = h.breakdowns;
    info->rel_res_true = h.rel_true;
    info->rel_res_est = h.est_rel;
    info->mismatch = (h.est_rel > 0.0 && h.rel_true > 10.0 * h.est_rel) ? 1 : 0;
}

gnp_status solve_run(SolveCtx *c, gnp_model *model, const double *b, double *x, int m,
                     double rtol, int maxiters, double *hist_host, gnp_solve_info *info,
                     hipStream_t st) {
    const int64_t n = c->sys->n;
    GNP_TRY(solve_begin(c, b, x, m, rtol, maxiters, st));
    GNP_HIP(hipStreamSynchronize(st));
    if (!std::isfinite(c->ctl_host->bnorm)) return fail(GNP_ENUMERIC, "b is not finite");
    if (c->ctl_host->bnorm == 0.0) {
        GNP_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, st));
        GNP_HIP(hipStreamSynchronize(st));
        if (hist_host) hist_host[0] = 0.0;
        if (info) {
            memset(info, 0, sizeof(*info));
            info->converged = 1;
        }
        return GNP_OK;
    }
    while (!c->ctl_host->solve_done) {
        const int it0 = c->ctl_host->it;
        GNP_TRY(solve_next(c, model, b, x, m, maxiters, st));
        GNP_HIP(hipStreamSynchronize(st));
        if (c->ctl_host->it <= it0 && !c->ctl_host->solve_done)
            return fail(GNP_EDEVICE, "solver made no progress in a cycle");
    }
    const Ctl &h = *c->ctl_host;
    if (hist_host)
        GNP_HIP(hipMemcpy(hist_host, c->hist, sizeof(double) * (h.it + 1), hipMemcpyDeviceToHost));
    solve_info_from(h, info);
    if (h.nonfinite) return fail(GNP_ENUMERIC, "non-finite value in the Arnoldi process");
    return GNP_OK;
}

// ---------------------------------------------------------------------------
// Batched solve: nb right-hand sides of one system in lockstep.  Every solver
// kernel runs once per stage with gridDim.y = nb on per-right-hand-side
// slices (Bat strides); the network input of all right-hand sides is packed
// [n][nb] so that one network launch per step serves the whole batch, and
// the network outputs stay packed (Zp) for the update of x.  Each right-hand
// side follows the single-solve arithmetic step for step.
// ---------------------------------------------------------------------------
struct BatchCtx {
    gnp_system *sys = nullptr;
    int m = 0, mp = 32, nb = 0, cap = 0, d = 0;
    gnp_precision prec = GNP_BF16;
    int64_t n = 0, npartial = 0;
    float *V = nullptr, *Zp = nullptr, *vpk = nullptr, *w = nullptr;
    void *act[2] = {nullptr, nullptr};
    double *r = nullptr, *tau = nullptr, *H = nullptr, *H0 = nullptr, *cs = nullptr,
           *sn = nullptr, *g = nullptr, *y = nullptr, *h1 = nullptr, *h2 = nullptr,
           *hist = nullptr, *partial = nullptr;
    Ctl *ctl = nullptr, *ctl_host = nullptr;
    int *all_done = nullptr;
    Bat bt;
};

static void batch_free(BatchCtx *c) {
    if (!c) return;
    void *ptrs[] = {c->V,  c->Zp, c->vpk, c->w,  c->act[0], c->act[1], c->r,  c->tau,
                    c->H,  c->H0, c->cs,  c->sn, c->g,      c->y,      c->h1, c->h2,
                    c->hist, c->partial, c->ctl, c->all_done};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    if (c->ctl_host) (void)hipHostFree(c->ctl_host);
    *c = BatchCtx();
}

static gnp_status batch_prepare(BatchCtx *c, gnp_system *sys, int m, int maxiters, int nb,
                                int d) {
    if (c->sys == sys && c->m == m && c->nb == nb && c->cap >= maxiters && c->d == d)
        return GNP_OK;
    batch_free(c);
    const int64_t n = sys->n;
    c->sys = sys;
    c->m = m;
    c->mp = basis_pitch(m);
    c->nb = nb;
    c->cap = std::max(maxiters, 128);
    c->d = d;
    c->n = n;
    const int64_t nb_cgs = (n + cgs_rpb(n) - 1) / cgs_rpb(n);
    c->npartial = std::max<int64_t>(nb_cgs * (c->mp + 1), 2048);
    c->bt.vec = n;
    c->bt.basis = n * c->mp;
    c->bt.part = c->npartial;
    c->bt.hess = (int64_t)(m + 1) * m;
    c->bt.small = m + 1;
    c->bt.hist = c->cap + 1;
    c->bt.vstep = nb;
    auto al = [&](auto **q, size_t count) -> gnp_status {
        GNP_HIP(hipMalloc((void **)q, sizeof(**q) * count));
        return GNP_OK;
    };
    GNP_TRY(al(&c->V, (size_t)nb * n * c->mp));
    GNP_HIP(hipMemset(c->V, 0, sizeof(float) * (size_t)nb * n * c->mp));
    GNP_TRY(al(&c->Zp, (size_t)m * n * nb));
    GNP_TRY(al(&c->vpk, (size_t)n * nb));
    GNP_TRY(al(&c->w, (size_t)n * nb));
    for (int i = 0; i < 2; ++i) GNP_HIP(hipMalloc(&c->act[i], sizeof(float) * n * nb * d));
    GNP_TRY(al(&c->r, (size_t)n * nb));
    GNP_TRY(al(&c->tau, (size_t)3 * nb));
    GNP_TRY(al(&c->H, (size_t)nb * c->bt.hess));
    GNP_TRY(al(&c->H0, (size_t)nb * c->bt.hess));
    for (double **q : {&c->cs, &c->sn, &c->g, &c->y, &c->h1, &c->h2})
        GNP_TRY(al(q, (size_t)nb * c->bt.small));
    GNP_TRY(al(&c->hist, (size_t)nb * c->bt.hist));
    GNP_TRY(al(&c->partial, (size_t)nb * c->npartial));
    GNP_TRY(al(&c->ctl, (size_t)nb));
    GNP_TRY(al(&c->all_done, 1));
    GNP_HIP(hipHostMalloc(&c->ctl_host, sizeof(Ctl) * nb, hipHostMallocDefault));
    return GNP_OK;
}

template <int MP>
static gnp_status batch_cycle(BatchCtx *c, gnp_model *model, int nsteps, double *x,
                              hipStream_t st) {
    gnp_system *s = c->sys;
    const int64_t n = s->n;
    const int nb = c->nb;
    const Bat &bt = c->bt;
    const int sg = stream_grid(n);
    const int64_t rpb = cgs_rpb(n);
    const int gcgs = (int)((n + rpb - 1) / rpb);
    const int pstride = MP + 1;
    float *V = c->V, *w = c->w;
    hipLaunchKernelGGL((k_normalize<float, double>), dim3(sg, nb), dim3(BLOCK), 0, st, n,
                       (const double *)c->r, c->vpk, (const Ctl *)c->ctl, 1, bt);
    hipLaunchKernelGGL(k_unit_tau, dim3(1, nb), dim3(WAVE), 0, st, n, c->tau,
                       (const Ctl *)c->ctl, c->all_done, model->scaled);
    for (int j = 0; j < nsteps; ++j) {
        float *zj = c->Zp + (int64_t)j * n * nb;
        GNP_TRY(forward_launch(model, c->prec, c->vpk, zj, nb, c->tau, c->act[0], c->act[1],
                               c->all_done, st));
        SpIn<float> sp;  // z_j packed [n][nb]
        sp.rp = s->rp;
        sp.ci = s->ci;
        sp.val = s->val32;
        sp.z = zj;
        sp.zstep = nb;
        hipLaunchKernelGGL((k_cgs<float, MP, 4>), dim3(gcgs, nb), dim3(BLOCK), 0, st, n, rpb, V, j,
                           w, (const double *)nullptr, c->partial, pstride, (const Ctl *)c->ctl,
                           bt, (const float *)c->vpk, (float *)nullptr, 0, sp);
        hipLaunchKernelGGL(k_fin_dots, dim3(j + 2, nb), dim3(BLOCK), 0, st, gcgs, j,
                           (const double *)c->partial, pstride, c->h1, c->ctl, bt);
        hipLaunchKernelGGL((k_cgs<float, MP, 1>), dim3(gcgs, nb), dim3(BLOCK), 0, st, n, rpb, V, j,
                           w, (const double *)c->h1, c->partial, pstride, (const Ctl *)c->ctl,
                           bt, (const float *)nullptr, (float *)nullptr);
        hipLaunchKernelGGL(k_fin_sums2, dim3(j + 2, nb), dim3(BLOCK), 0, st, gcgs, j,
                           (const double *)c->partial, pstride, c->h2, (const Ctl *)c->ctl, bt);
        hipLaunchKernelGGL(k_fin_givens, dim3(1, nb), dim3(BLOCK), 0, st, j, (const double *)c->h1,
                           (const double *)c->h2, c->ctl, c->H, c->H0, c->cs, c->sn, c->g,
                           c->hist, bt, (uint64_t *)nullptr);
        hipLaunchKernelGGL((k_cgs<float, MP, 2>), dim3(gcgs, nb), dim3(BLOCK), 0, st, n, rpb, V, j,
                           w, (const double *)c->h2, c->partial, pstride, (const Ctl *)c->ctl,
                           bt, (const float *)nullptr, (float *)nullptr);
        hipLaunchKernelGGL((k_normalize<float, float>), dim3(sg, nb), dim3(BLOCK), 0, st, n,
                           (const float *)w, c->vpk, (const Ctl *)c->ctl, 0, bt);
        hipLaunchKernelGGL(k_unit_tau, dim3(1, nb), dim3(WAVE), 0, st, n, c->tau,
                           (const Ctl *)c->ctl, c->all_done, model->scaled);
    }
    hipLaunchKernelGGL(k_backsolve, dim3(1, nb), dim3(BLOCK), 0, st, c->ctl, (const double *)c->H,
                       (const double *)c->g, c->y, bt);
    hipLaunchKernelGGL((k_update_x_pk<float>), dim3(grid_for(n * nb, BLOCK, 4096)), dim3(BLOCK), 0,
                       st, n, nb, (const float *)c->Zp, (const double *)c->y, (const Ctl *)c->ctl,
                       x, bt);
    GNP_HIP(hipGetLastError());
    return GNP_OK;
}

static void batch_residual(BatchCtx *c, const double *b, const double *x, int initial,
                           hipStream_t st) {
    gnp_system *s = c->sys;
    const int64_t n = s->n;
    const double avg = (double)s->nnz / (double)n;
    const int G = avg <= 12.0 ? 4 : (avg <= 24.0 ? 8 : 16);
    const int grid = grid_for(n, BLOCK / G, 1024);
    const dim3 gg(grid, c->nb);
    if (G == 4)
        hipLaunchKernelGGL(k_residual<4>, gg, dim3(BLOCK), 0, st, n, s->rp, s->ci, s->val64, x, b,
                           c->r, c->partial, c->bt);
    else if (G == 8)
        hipLaunchKernelGGL(k_residual<8>, gg, dim3(BLOCK), 0, st, n, s->rp, s->ci, s->val64, x, b,
                           c->r, c->partial, c->bt);
    else
        hipLaunchKernelGGL(k_residual<16>, gg, dim3(BLOCK), 0, st, n, s->rp, s->ci, s->val64, x,
                           b, c->r, c->partial, c->bt);
    hipLaunchKernelGGL(k_fin_residual, dim3(1, c->nb), dim3(BLOCK), 0, st, grid,
                       (const double *)c->partial, c->ctl, c->g, c->hist, initial, c->bt,
                       (uint64_t *)nullptr);
}

static gnp_status batch_run(BatchCtx *c, gnp_model *model, const double *b, double *x, int m,
                            double rtol, int maxiters, gnp_solve_info *infos, hipStream_t st) {
    const int64_t n = c->n;
    const int nb = c->nb;
    Ctl init;
    memset(&init, 0, sizeof(init));
    init.m = m;
    init.maxiters = maxiters;
    for (int k = 0; k < nb; ++k) c->ctl_host[k] = init;
    GNP_HIP(hipMemcpyAsync(c->ctl, c->ctl_host, sizeof(Ctl) * nb, hipMemcpyHostToDevice, st));
    const int sg = stream_grid(n);
    hipLaunchKernelGGL(k_sumsq, dim3(sg, nb), dim3(BLOCK), 0, st, n, b, c->partial, c->bt);
    hipLaunchKernelGGL(k_fin_bnorm, dim3(1, nb), dim3(BLOCK), 0, st, sg, (const double *)c->partial,
                       rtol, c->ctl, c->bt);
    batch_residual(c, b, x, 1, st);
    GNP_HIP(hipMemcpyAsync(c->ctl_host, c->ctl, sizeof(Ctl) * nb, hipMemcpyDeviceToHost, st));
    GNP_HIP(hipStreamSynchronize(st));
    bool zero_rhs = false;
    for (int k = 0; k < nb; ++k) {
        Ctl &h = c->ctl_host[k];
        if (!std::isfinite(h.bnorm)) return fail(GNP_ENUMERIC, "a right-hand side is not finite");
        if (h.bnorm == 0.0) {  // x = 0, nothing to iterate
            GNP_HIP(hipMemsetAsync(x + (int64_t)k * n, 0, sizeof(double) * n, st));
            h.converged = 1;
            h.solve_done = 1;
            h.cycle_done = 1;
            h.rel_true = 0.0;
            h.est_rel = 0.0;
            zero_rhs = true;
        }
    }
    if (zero_rhs)
        GNP_HIP(hipMemcpyAsync(c->ctl, c->ctl_host, sizeof(Ctl) * nb, hipMemcpyHostToDevice, st));
    auto all_done = [&]() {
        for (int k = 0; k < nb; ++k)
            if (!c->ctl_host[k].solve_done) return false;
        return true;
    };
    std::vector<int> it0(nb);
    while (!all_done()) {
        int nsteps = 0;
        for (int k = 0; k < nb; ++k) {
            it0[k] = c->ctl_host[k].it;
            if (!c->ctl_host[k].solve_done) nsteps = std::max(nsteps, std::min(m, maxiters - it0[k]));
        }
        switch (c->mp) {
            case 32: GNP_TRY(batch_cycle<32>(c, model, nsteps, x, st)); break;
            case 64: GNP_TRY(batch_cycle<64>(c, model, nsteps, x, st)); break;
            case 128: GNP_TRY(batch_cycle<128>(c, model, nsteps, x, st)); break;
            case 256: GNP_TRY(batch_cycle<256>(c, model, nsteps, x, st)); break;
            default: return fail(GNP_EINVAL, "unsupported basis pitch");
        }
        batch_residual(c, b, x, 0, st);
        GNP_HIP(hipMemcpyAsync(c->ctl_host, c->ctl, sizeof(Ctl) * nb, hipMemcpyDeviceToHost, st));
        GNP_HIP(hipStreamSynchronize(st));
        bool progress = false;
        for (int k = 0; k < nb; ++k)
            if (c->ctl_host[k].it > it0[k] || c->ctl_host[k].solve_done) progress = true;
        if (!progress) return fail(GNP_EDEVICE, "batched solver made no progress in a cycle");
    }
    bool nonfinite = false;
    for (int k = 0; k < nb; ++k) {
        solve_info_from(c->ctl_host[k], infos ? infos + k : nullptr);
        nonfinite |= c->ctl_host[k].nonfinite != 0;
    }
    if (nonfinite) return fail(GNP_ENUMERIC, "non-finite value in the Arnoldi process");
    return GNP_OK;
}

void batch_cache_free(void *p) {
    if (!p) return;
    BatchCtx *c = (BatchCtx *)p;
    batch_free(c);
    delete c;
}

}  // namespace gnp

using namespace gnp;

extern "C" gnp_status fgmres_solve(gnp_system *sys, gnp_model *model, const double *b_dev,
                                   double *x_dev, int m, double rtol, int maxiters,
                                   gnp_precision prec, double *hist, gnp_solve_info *info,
                                   void *hip_stream) {
    if (!sys || !b_dev || !x_dev) return fail(GNP_EINVAL, "null argument");
    if (m < 1 || m > 255) return fail(GNP_EINVAL, "m must be in [1, 255]");
    if (!(rtol > 0.0)) return fail(GNP_EINVAL, "rtol must be > 0");
    if (maxiters < 1) return fail(GNP_EINVAL, "maxiters must be >= 1");
    if (!valid_precision(prec)) return fail(GNP_EINVAL, "bad precision");
    if (model && model->sys != sys) return fail(GNP_EINVAL, "model belongs to another system");
    if (!sys->solve_cache) sys->solve_cache = new SolveCtx();
    SolveCtx *c = (SolveCtx *)sys->solve_cache;
    GNP_TRY(solve_ctx_prepare(c, sys, m, maxiters, prec, model ? model->d : 0));
    c->prec = prec;
    c->timeout_s = sys->solve_timeout;
    return solve_run(c, model, b_dev, x_dev, m, rtol, maxiters, hist, info,
                     (hipStream_t)hip_stream);
}

// D^{-1} of the system, made once (GNP_EINVAL for a zero or missing diagonal entry)
static gnp_status system_dinv(gnp_system *s, hipStream_t st) {
    if (s->dinv64) return GNP_OK;
    double *d = nullptr;
    int *flag = nullptr;
    GNP_HIP(hipMalloc(&d, sizeof(double) * s->n));
    if (hipMalloc(&flag, sizeof(int)) != hipSuccess) {
        (void)hipFree(d);
        return fail(GNP_ENOMEM, "hipMalloc failed");
    }
    int h = 0;
    hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_diag_inv, dim3(grid_for(s->n, BLOCK)), dim3(BLOCK), 0, st, s->n, s->rp,
                           s->ci, (const double *)s->val64, d, flag);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(flag);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return check_hip(e, "Jacobi diagonal");
    }
    if (h) {
        (void)hipFree(d);
        return fail(GNP_EINVAL, "Jacobi needs a nonzero diagonal entry in every row");
    }
    s->dinv64 = d;
    return GNP_OK;
}

extern "C" gnp_status fgmres_solve_jacobi(gnp_system *sys, const double *b_dev, double *x_dev,
                                          int m, double rtol, int maxiters, gnp_precision prec,
                                          double *hist, gnp_solve_info *info, void *hip_stream) {
    if (!sys || !b_dev || !x_dev) return fail(GNP_EINVAL, "null argument");
    if (m < 1 || m > 255) return fail(GNP_EINVAL, "m must be in [1, 255]");
    if (!(rtol > 0.0)) return fail(GNP_EINVAL, "rtol must be > 0");
    if (maxiters < 1) return fail(GNP_EINVAL, "maxiters must be >= 1");
    if (prec != GNP_F32 && prec != GNP_F64)
        return fail(GNP_EINVAL, "the Jacobi solve runs in float32 or float64");
    hipStream_t st = (hipStream_t)hip_stream;
    GNP_TRY(system_dinv(sys, st));
    if (!sys->solve_cache) sys->solve_cache = new SolveCtx();
    SolveCtx *c = (SolveCtx *)sys->solve_cache;
    GNP_TRY(solve_ctx_prepare(c, sys, m, maxiters, prec, 0));
    c->prec = prec;
    c->timeout_s = sys->solve_timeout;
    c->precond = PRECOND_JACOBI;
    const gnp_status r = solve_run(c, nullptr, b_dev, x_dev, m, rtol, maxiters, hist, info, st);
    c->precond = PRECOND_MODEL;
    return r;
}

extern "C" gnp_status fgmres_solve_gmres(gnp_system *sys, const double *b_dev, double *x_dev,
                                         int m, double rtol, int maxiters, int inner_k,
                                         double inner_tol, gnp_precision prec, double *hist,
                                         gnp_solve_info *info, void *hip_stream) {
    if (!sys || !b_dev || !x_dev) return fail(GNP_EINVAL, "null argument");
    if (m < 1 || m > 255) return fail(GNP_EINVAL, "m must be in [1, 255]");
    if (!(rtol > 0.0)) return fail(GNP_EINVAL, "rtol must be > 0");
    if (maxiters < 1) return fail(GNP_EINVAL, "maxiters must be >= 1");
    if (inner_k < 1 || inner_k > 31) return fail(GNP_EINVAL, "inner_k must be in [1, 31]");
    if (!(inner_tol >= 0.0) || !std::isfinite(inner_tol))
        return fail(GNP_EINVAL, "inner_tol must be finite and >= 0");
    if (prec != GNP_F32 && prec != GNP_F64)
        return fail(GNP_EINVAL, "inner-outer GMRES runs in float32 or float64");
    hipStream_t st = (hipStream_t)hip_stream;
    if (!sys->solve_cache) sys->solve_cache = new SolveCtx();
    SolveCtx *c = (SolveCtx *)sys->solve_cache;
    GNP_TRY(solve_ctx_prepare(c, sys, m, maxiters, prec, 0));
    c->prec = prec;
    if (!c->inner) c->inner = new SolveCtx();
    GNP_TRY(solve_ctx_prepare(c->inner, sys, inner_k, inner_k, prec, 0));
    c->inner->prec = prec;
    c->inner->precond = PRECOND_MODEL;
    if (!c->inner_x) GNP_HIP(hipMalloc(&c->inner_x, sizeof(double) * sys->n));
    c->inner_k = inner_k;
    c->inner_tol = inner_tol;
    c->timeout_s = sys->solve_timeout;
    c->precond = PRECOND_GMRES;
    const gnp_status r = solve_run(c, nullptr, b_dev, x_dev, m, rtol, maxiters, hist, info, st);
    c->precond = PRECOND_MODEL;
    return r;
}

extern "C" gnp_status gnp_system_set_timeout(gnp_system *sys, double seconds) {
    if (!sys) return fail(GNP_EINVAL, "null system");
    if (!(seconds >= 0.0) || !std::isfinite(seconds))
        return fail(GNP_EINVAL, "seconds must be finite and >= 0");
    sys->solve_timeout = seconds;
    return GNP_OK;
}

extern "C" gnp_status fgmres_step_times(gnp_system *sys, double *t_host, int count) {
    if (!sys || !t_host) return fail(GNP_EINVAL, "null argument");
    SolveCtx *c = (SolveCtx *)sys->solve_cache;
    if (!c || !c->tstamp || !c->ctl_host) return fail(GNP_EINVAL, "no solve on this system yet");
    if (count < 1 || count > c->ctl_host->it + 1)
        return fail(GNP_EINVAL, "count must be in [1, iters + 1] of the last solve");
    int dev = 0, khz = 0;
    GNP_HIP(hipGetDevice(&dev));
    GNP_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    if (khz <= 0) return fail(GNP_EDEVICE, "device reports no wall-clock rate");
    std::vector<uint64_t> ts(count);
    GNP_HIP(hipMemcpy(ts.data(), c->tstamp, sizeof(uint64_t) * count, hipMemcpyDeviceToHost));
    for (int i = 0; i < count; ++i)
        t_host[i] = (double)(int64_t)(ts[i] - ts[0]) / (1e3 * (double)khz);
    return GNP_OK;
}

extern "C" gnp_status gnp_auc(const double *r, const double *t, int iters, double rtol,
                              double *iter_auc, double *time_auc) {
    if (!r || iters < 0 || !(rtol > 0.0) || (time_auc && !t))
        return fail(GNP_EINVAL, "bad argument");
    // a zero residual (b = 0, an exact step) is taken at the smallest normal double
    auto lg = [&](double v) { return log10(v > DBL_MIN ? v : DBL_MIN) - log10(rtol); };
    if (iter_auc) {
        double a = 0.0;
        for (int i = 0; i <= iters; ++i) a += lg(r[i]);
        *iter_auc = a;
    }
    if (time_auc) {
        double a = 0.0;
        for (int i = 1; i <= iters; ++i) a += lg(r[i]) * (t[i] - t[i - 1]);
        *time_auc = a;
    }
    return GNP_OK;
}

extern "C" gnp_status fgmres_solve_batch(gnp_system *sys, gnp_model *model, const double *b_dev,
                                         double *x_dev, int nrhs, int m, double rtol,
                                         int maxiters, gnp_precision prec, gnp_solve_info *infos,
                                         void *hip_stream) {
    if (!sys || !model || !b_dev || !x_dev) return fail(GNP_EINVAL, "null argument");
    if (nrhs < 1 || nrhs > 256) return fail(GNP_EINVAL, "nrhs must be in [1, 256]");
    if (m < 1 || m > 255) return fail(GNP_EINVAL, "m must be in [1, 255]");
    if (!(rtol > 0.0)) return fail(GNP_EINVAL, "rtol must be > 0");
    if (maxiters < 1) return fail(GNP_EINVAL, "maxiters must be >= 1");
    if (prec != GNP_F32 && prec != GNP_BF16)
        return fail(GNP_EINVAL, "batched solves run the float32 or bfloat16 network");
    if (model->sys != sys) return fail(GNP_EINVAL, "model belongs to another system");
    if (!sys->batch_cache) sys->batch_cache = new BatchCtx();
    BatchCtx *c = (BatchCtx *)sys->batch_cache;
    GNP_TRY(batch_prepare(c, sys, m, maxiters, nrhs, model->d));
    c->prec = prec;
    return batch_run(c, model, b_dev, x_dev, m, rtol, maxiters, infos, (hipStream_t)hip_stream);
}

namespace gnp {
void solve_cache_free(void *p) {
    if (!p) return;
    SolveCtx *c = (SolveCtx *)p;
    solve_ctx_free(c);
    delete c;
}
}  // namespace gnp
