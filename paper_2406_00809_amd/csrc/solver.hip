// Restarted flexible GMRES (Algorithm 1) with the network as nonlinear right
// preconditioner.  Per Arnoldi step j the stream holds: z_j = M(v_j), the
// SpMV w = A z_j, three classical Gram-Schmidt passes (dots; update + dots;
// update + norm, i.e. CGS applied twice with float64 inner products), the
// Givens update of the Hessenberg column on the device, and the
// normalisation v_{j+1} = w / h_{j+1,j} fused with the float64 norm that the
// next network input needs for its scaling (Eq. (6)).  All reductions are
// two-stage and deterministic.  The host synchronises once per cycle.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "solver.hpp"
#include "spmv.hpp"

namespace gnp {

constexpr int CH = 32;  // basis vectors per dot-product chunk

static int stream_grid(int64_t n) { return grid_for(n, 4 * BLOCK, 2048); }

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_bnorm(int64_t n, const double *__restrict__ b,
                                                 double rtol, double *partial, unsigned *counter,
                                                 Ctl *ctl) {
    __shared__ double sh[BLOCK / WAVE];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * BLOCK)
        s += b[i] * b[i];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
    if (last_block(counter)) {
        double a = 0.0;
        for (unsigned k = threadIdx.x; k < gridDim.x; k += BLOCK) a += partial[k];
        a = block_sum(a, sh);
        if (threadIdx.x == 0) {
            ctl->bnorm = sqrt(a);
            ctl->target = rtol * sqrt(a);
        }
    }
}

// r = b - A x (float64 values, float64 x), beta = ||r||, restart bookkeeping
template <int G>
__global__ __launch_bounds__(BLOCK) void k_residual(
    int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const double *__restrict__ val, const double *__restrict__ x, const double *__restrict__ b,
    double *__restrict__ r, double *partial, unsigned *counter, Ctl *ctl, double *g, double *hist,
    int initial) {
    __shared__ double sh[BLOCK / WAVE];
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
    if (last_block(counter)) {
        double a = 0.0;
        for (unsigned k = threadIdx.x; k < gridDim.x; k += BLOCK) a += partial[k];
        a = block_sum(a, sh);
        if (threadIdx.x == 0) {
            const double beta = sqrt(a);
            const double rel = beta / ctl->bnorm;
            ctl->rel_true = rel;
            ctl->beta = beta;
            if (initial) {
                if (hist) hist[0] = rel;
                ctl->est_rel = rel;
            }
            if (!isfinite(beta)) {
                ctl->nonfinite = 1;
                ctl->solve_done = 1;
            } else if (beta <= ctl->target) {
                ctl->converged = 1;
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
        for (int k = threadIdx.x; k <= ctl->m; k += BLOCK) g[k] = (k == 0) ? sqrt(a) : 0.0;
    }
}

// v = src / div (div = beta or h_{j+1,j}); tau triple from ||v||_2 of the
// stored (rounded) v, for the scaling s of the next network input.
template <typename KT, typename ST>
__global__ __launch_bounds__(BLOCK) void k_scale_norm(int64_t n, const ST *__restrict__ src,
                                                      KT *__restrict__ v, double *partial,
                                                      unsigned *counter, const Ctl *ctl,
                                                      int use_beta, double *tau) {
    if (ctl->cycle_done) return;
    __shared__ double sh[BLOCK / WAVE];
    const double div = use_beta ? ctl->beta : ctl->hnext;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * BLOCK) {
        const KT t = (KT)((double)src[i] / div);
        v[i] = t;
        s += (double)t * (double)t;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
    if (last_block(counter)) {
        double a = 0.0;
        for (unsigned k = threadIdx.x; k < gridDim.x; k += BLOCK) a += partial[k];
        a = block_sum(a, sh);
        if (threadIdx.x == 0) {
            const double tv = sqrt(a), sqn = sqrt((double)n);
            tau[0] = tv;
            tau[1] = tv > 0.0 ? sqn / tv : 0.0;
            tau[2] = tv / sqn;
        }
    }
}

// Block-reduce CH accumulators into partial[blk * stride + base + k].
__device__ __forceinline__ void block_reduce_chunk(double (&acc)[CH], double *sh, double *dst,
                                                   int count) {
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const double v = wave_sum(acc[k]);
        if (lane == 0) sh[wv * CH + k] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < count) {
        double s = 0.0;
        for (int q = 0; q < BLOCK / WAVE; ++q) s += sh[q * CH + threadIdx.x];
        dst[threadIdx.x] = s;
    }
    __syncthreads();
}

// Classical Gram-Schmidt pass over V_0..V_j (float64 arithmetic on the
// stored vectors).  MODE 0: h = V^T w and ||w||^2.  MODE 1: w -= V hprev,
// then h = V^T w.  MODE 2: w -= V hprev, then ||w||^2 and the Givens update.
template <typename KT, int MODE>
__global__ __launch_bounds__(BLOCK) void k_cgs(int64_t n, int64_t rpb, const KT *__restrict__ V,
                                               int j, KT *__restrict__ w,
                                               const double *__restrict__ hprev,
                                               double *__restrict__ hout, double *partial,
                                               int pstride, unsigned *counter, Ctl *ctl,
                                               double *H, double *H0, double *cs, double *sn,
                                               double *g, double *hist) {
    if (ctl->cycle_done) return;
    __shared__ double sh[(BLOCK / WAVE) * CH];
    const int64_t i0 = (int64_t)blockIdx.x * rpb;
    const int64_t i1 = (i0 + rpb < n) ? i0 + rpb : n;
    double nrm = 0.0;
    if (MODE >= 1) {
        for (int64_t i = i0 + threadIdx.x; i < i1; i += BLOCK) {
            double corr = 0.0;
            for (int k = 0; k <= j; ++k) corr += hprev[k] * (double)V[(int64_t)k * n + i];
            const KT wi = (KT)((double)w[i] - corr);
            w[i] = wi;
            if (MODE == 2) nrm += (double)wi * (double)wi;
        }
    }
    if (MODE <= 1) {
        for (int kc = 0; kc <= j; kc += CH) {
            double acc[CH];
#pragma unroll
            for (int k = 0; k < CH; ++k) acc[k] = 0.0;
            for (int64_t i = i0 + threadIdx.x; i < i1; i += BLOCK) {
                const double wi = (double)w[i];
                if (MODE == 0 && kc == 0) nrm += wi * wi;
#pragma unroll
                for (int k = 0; k < CH; ++k)
                    if (kc + k <= j) acc[k] += (double)V[(int64_t)(kc + k) * n + i] * wi;
            }
            const int cnt = std::min(CH, j + 1 - kc);
            block_reduce_chunk(acc, sh, partial + (int64_t)blockIdx.x * pstride + kc, cnt);
        }
    }
    if (MODE != 1) {
        const double s = block_sum(nrm, sh);
        if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * pstride + (pstride - 1)] = s;
    }
    if (!last_block(counter)) return;
    // ---- last block: combine partials in block order
    if (MODE <= 1) {
        for (int t = threadIdx.x; t <= j; t += BLOCK) {
            double a = 0.0;
            for (unsigned blk = 0; blk < gridDim.x; ++blk) a += partial[(int64_t)blk * pstride + t];
            hout[t] = a;
        }
    }
    if (MODE == 0) {
        if (threadIdx.x == 0) {
            double a = 0.0;
            for (unsigned blk = 0; blk < gridDim.x; ++blk)
                a += partial[(int64_t)blk * pstride + (pstride - 1)];
            ctl->wnorm0 = sqrt(a);
        }
    }
    if (MODE == 2 && threadIdx.x == 0) {
        double a = 0.0;
        for (unsigned blk = 0; blk < gridDim.x; ++blk)
            a += partial[(int64_t)blk * pstride + (pstride - 1)];
        const double hn = sqrt(a);
        const int m = ctl->m;
        // column j of H-bar: h1 + h2 (hout holds h1, hprev holds h2), then ||w||
        for (int i = 0; i <= j; ++i) {
            const double v = hout[i] + hprev[i];
            H0[(int64_t)i * m + j] = v;
            H[(int64_t)i * m + j] = v;
        }
        H0[(int64_t)(j + 1) * m + j] = hn;
        // previous rotations (Saad 2003, Sec. 6.5.3), then a new one
        for (int i = 0; i < j; ++i) {
            const double a0 = H[(int64_t)i * m + j], b0 = H[(int64_t)(i + 1) * m + j];
            H[(int64_t)i * m + j] = cs[i] * a0 + sn[i] * b0;
            H[(int64_t)(i + 1) * m + j] = -sn[i] * a0 + cs[i] * b0;
        }
        const double a0 = H[(int64_t)j * m + j];
        const double rho = hypot(a0, hn);
        double c = 1.0, s = 0.0;
        if (rho != 0.0) {
            c = a0 / rho;
            s = hn / rho;
        }
        cs[j] = c;
        sn[j] = s;
        H[(int64_t)j * m + j] = rho;
        H[(int64_t)(j + 1) * m + j] = 0.0;
        const double gj = g[j];
        g[j + 1] = -s * gj;
        g[j] = c * gj;
        const double est = fabs(g[j + 1]);
        ctl->est = est;
        ctl->est_rel = est / ctl->bnorm;
        ctl->it += 1;
        ctl->kcols = j + 1;
        if (hist) hist[ctl->it] = est / ctl->bnorm;
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
    }
}

// y = R^{-1} g on the leading columns with nonzero pivots (one thread)
__global__ void k_backsolve(Ctl *ctl, const double *H, const double *g, double *y) {
    if (threadIdx.x != 0) return;
    const int m = ctl->m;
    int kk = ctl->kcols;
    while (kk > 0 && H[(int64_t)(kk - 1) * m + (kk - 1)] == 0.0) --kk;
    for (int i = kk - 1; i >= 0; --i) {
        double acc = g[i];
        for (int q = i + 1; q < kk; ++q) acc -= H[(int64_t)i * m + q] * y[q];
        y[i] = acc / H[(int64_t)i * m + i];
    }
    ctl->kuse = kk;
}

// x += Z y  (float64 accumulation)
template <typename KT>
__global__ __launch_bounds__(BLOCK) void k_update_x(int64_t n, const KT *__restrict__ Z,
                                                    const double *__restrict__ y, const Ctl *ctl,
                                                    double *__restrict__ x) {
    const int ku = ctl->kuse;
    if (ku == 0) return;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * BLOCK) {
        double acc = 0.0;
        for (int k = 0; k < ku; ++k) acc += (double)Z[(int64_t)k * n + i] * y[k];
        x[i] += acc;
    }
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
void solve_ctx_free(SolveCtx *c) {
    if (!c) return;
    void *ptrs[] = {c->V,  c->Z,  c->w,  c->r,  c->act[0], c->act[1], c->tau,     c->H,
                    c->H0, c->cs, c->sn, c->g,  c->y,      c->h1,     c->h2,      c->hist,
                    c->partial, c->counters, c->ctl};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (c->ctl_host) (void)hipHostFree(c->ctl_host);
    if (c->ev) (void)hipEventDestroy(c->ev);
    *c = SolveCtx();
}

static int64_t cgs_rpb(int64_t n) {
    int64_t nb = 512;
    int64_t rpb = (n + nb - 1) / nb;
    rpb = ((rpb + BLOCK - 1) / BLOCK) * BLOCK;
    return rpb < BLOCK ? BLOCK : rpb;
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
    c->n = sys->n;
    c->prec = prec;
    c->kbytes = kb;
    c->maxiters_cap = std::max(maxiters, 128);
    c->act_d = act_d;
    const int64_t n = sys->n;
    GNP_HIP(hipMalloc(&c->V, kb * (size_t)n * (m + 1)));
    GNP_HIP(hipMalloc(&c->Z, kb * (size_t)n * m));
    GNP_HIP(hipMalloc(&c->w, kb * (size_t)n));
    GNP_HIP(hipMalloc(&c->r, sizeof(double) * n));
    if (act_d > 0)
        for (int i = 0; i < 2; ++i) GNP_HIP(hipMalloc(&c->act[i], sizeof(double) * n * act_d));
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
    const int64_t nb_cgs = (n + cgs_rpb(n) - 1) / cgs_rpb(n);
    c->npartial = std::max<int64_t>(nb_cgs * (m + 2), 4096);
    GNP_HIP(hipMalloc(&c->partial, sizeof(double) * c->npartial));
    GNP_HIP(hipMalloc(&c->counters, sizeof(unsigned) * 16));
    GNP_HIP(hipMemset(c->counters, 0, sizeof(unsigned) * 16));
    GNP_HIP(hipMalloc(&c->ctl, sizeof(Ctl)));
    GNP_HIP(hipHostMalloc(&c->ctl_host, sizeof(Ctl), hipHostMallocDefault));
    GNP_HIP(hipEventCreateWithFlags(&c->ev, hipEventDisableTiming));
    return GNP_OK;
}

template <typename KT>
static gnp_status launch_cycle(SolveCtx *c, gnp_model *model, int nsteps, double *x,
                               hipStream_t st) {
    gnp_system *s = c->sys;
    const int64_t n = s->n;
    KT *V = (KT *)c->V, *Z = model ? (KT *)c->Z : (KT *)c->V, *w = (KT *)c->w;
    const KT *val;
    if constexpr (sizeof(KT) == 8) val = (const KT *)s->val64;
    else val = (const KT *)s->val32;
    const int sg = stream_grid(n);
    const int64_t rpb = cgs_rpb(n);
    const int gcgs = (int)((n + rpb - 1) / rpb);
    const int pstride = c->m + 2;
    int *skip = &c->ctl->cycle_done;
    hipLaunchKernelGGL((k_scale_norm<KT, double>), dim3(sg), dim3(BLOCK), 0, st, n, c->r, V,
                       c->partial, c->counters + 0, c->ctl, 1, c->tau);
    for (int j = 0; j < nsteps; ++j) {
        KT *vj = V + (int64_t)j * n, *zj = Z + (int64_t)j * n;
        if (model)
            GNP_TRY(forward_launch(model, c->prec, vj, zj, 1, c->tau, c->act[0], c->act[1], skip,
                                   st));
        spmv_launch<KT, KT, KT>(n, s->rp, s->ci, val, zj, w, nullptr, skip, s->nnz, st);
        hipLaunchKernelGGL((k_cgs<KT, 0>), dim3(gcgs), dim3(BLOCK), 0, st, n, rpb, V, j, w,
                           (const double *)nullptr, c->h1, c->partial, pstride, c->counters + 1,
                           c->ctl, c->H, c->H0, c->cs, c->sn, c->g, c->hist);
        hipLaunchKernelGGL((k_cgs<KT, 1>), dim3(gcgs), dim3(BLOCK), 0, st, n, rpb, V, j, w,
                           (const double *)c->h1, c->h2, c->partial, pstride, c->counters + 2,
                           c->ctl, c->H, c->H0, c->cs, c->sn, c->g, c->hist);
        hipLaunchKernelGGL((k_cgs<KT, 2>), dim3(gcgs), dim3(BLOCK), 0, st, n, rpb, V, j, w,
                           (const double *)c->h2, c->h1, c->partial, pstride, c->counters + 3,
                           c->ctl, c->H, c->H0, c->cs, c->sn, c->g, c->hist);
        hipLaunchKernelGGL((k_scale_norm<KT, KT>), dim3(sg), dim3(BLOCK), 0, st, n, w,
                           V + (int64_t)(j + 1) * n, c->partial, c->counters + 4, c->ctl, 0,
                           c->tau);
    }
    hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(WAVE), 0, st, c->ctl, c->H, c->g, c->y);
    hipLaunchKernelGGL((k_update_x<KT>), dim3(sg), dim3(BLOCK), 0, st, n, Z, c->y, c->ctl, x);
    GNP_HIP(hipGetLastError());
    return GNP_OK;
}

static void launch_residual(SolveCtx *c, const double *b, const double *x, int initial,
                            hipStream_t st) {
    gnp_system *s = c->sys;
    const int64_t n = s->n;
    const double avg = (double)s->nnz / (double)n;
    const int grid = grid_for(n, BLOCK / 8, 2048);
    if (avg <= 8.0)
        hipLaunchKernelGGL(k_residual<8>, dim3(grid), dim3(BLOCK), 0, st, n, s->rp, s->ci,
                           s->val64, x, b, c->r, c->partial, c->counters + 5, c->ctl, c->g,
                           c->hist, initial);
    else
        hipLaunchKernelGGL(k_residual<16>, dim3(grid), dim3(BLOCK), 0, st, n, s->rp, s->ci,
                           s->val64, x, b, c->r, c->partial, c->counters + 5, c->ctl, c->g,
                           c->hist, initial);
}

gnp_status solve_run(SolveCtx *c, gnp_model *model, const double *b, double *x, int m,
                     double rtol, int maxiters, double *hist_host, gnp_solve_info *info,
                     hipStream_t st) {
    gnp_system *s = c->sys;
    const int64_t n = s->n;
    Ctl init;
    memset(&init, 0, sizeof(init));
    init.m = m;
    init.maxiters = maxiters;
    *c->ctl_host = init;
    GNP_HIP(hipMemcpyAsync(c->ctl, c->ctl_host, sizeof(Ctl), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_bnorm, dim3(stream_grid(n)), dim3(BLOCK), 0, st, n, b, rtol, c->partial,
                       c->counters + 6, c->ctl);
    launch_residual(c, b, x, 1, st);
    GNP_HIP(hipMemcpyAsync(c->ctl_host, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
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
        const int nsteps = std::min(m, maxiters - it0);
        if (c->prec == GNP_F64) GNP_TRY(launch_cycle<double>(c, model, nsteps, x, st));
        else GNP_TRY(launch_cycle<float>(c, model, nsteps, x, st));
        launch_residual(c, b, x, 0, st);
        GNP_HIP(hipMemcpyAsync(c->ctl_host, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
        GNP_HIP(hipStreamSynchronize(st));
        if (c->ctl_host->it <= it0 && !c->ctl_host->solve_done)
            return fail(GNP_EDEVICE, "solver made no progress in a cycle");
    }
    const Ctl &h = *c->ctl_host;
    if (hist_host)
        GNP_HIP(hipMemcpy(hist_host, c->hist, sizeof(double) * (h.it + 1), hipMemcpyDeviceToHost));
    if (info) {
        info->iters = h.it;
        info->restarts = h.restarts;
        info->converged = h.converged;
        info->breakdowns = h.breakdowns;
        info->rel_res_true = h.rel_true;
        info->rel_res_est = h.est_rel;
        info->mismatch = (h.est_rel > 0.0 && h.rel_true > 10.0 * h.est_rel) ? 1 : 0;
    }
    if (h.nonfinite) return fail(GNP_ENUMERIC, "non-finite value in the Arnoldi process");
    return GNP_OK;
}

}  // namespace gnp

using namespace gnp;

extern "C" gnp_status fgmres_solve(gnp_system *sys, gnp_model *model, const double *b_dev,
                                   double *x_dev, int m, double rtol, int maxiters,
                                   gnp_precision prec, double *hist, gnp_solve_info *info,
                                   void *hip_stream) {
    if (!sys || !b_dev || !x_dev) return fail(GNP_EINVAL, "null argument");
    if (m < 1 || m > 256) return fail(GNP_EINVAL, "m must be in [1, 256]");
    if (!(rtol > 0.0)) return fail(GNP_EINVAL, "rtol must be > 0");
    if (maxiters < 1) return fail(GNP_EINVAL, "maxiters must be >= 1");
    if (!valid_precision(prec)) return fail(GNP_EINVAL, "bad precision");
    if (model && model->sys != sys) return fail(GNP_EINVAL, "model belongs to another system");
    if (!sys->solve_cache) sys->solve_cache = new SolveCtx();
    SolveCtx *c = (SolveCtx *)sys->solve_cache;
    GNP_TRY(solve_ctx_prepare(c, sys, m, maxiters, prec, model ? model->d : 0));
    c->prec = prec;
    return solve_run(c, model, b_dev, x_dev, m, rtol, maxiters, hist, info,
                     (hipStream_t)hip_stream);
}

namespace gnp {
void solve_cache_free(void *p) {
    if (!p) return;
    SolveCtx *c = (SolveCtx *)p;
    solve_ctx_free(c);
    delete c;
}
}  // namespace gnp
