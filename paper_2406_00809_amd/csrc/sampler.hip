// Training-pair sampler of Sec. 2.2 (Eqs. (2)-(3)).
//
// m steps of the Arnoldi process without a preconditioner give
// A V_m = V_{m+1} Hbar_m (Eq. (2)); with the thin SVD Hbar_m = W S Z^T the
// sampler draws x = V_m Z S^{-1} eps, eps ~ N(0, I_m) (Eq. (3)), so that
// b = A x = V_{m+1} W eps has a projector as covariance and the x cover the
// bottom of A's spectrum better than x ~ N(0, I).
//
// The Arnoldi run is the solver's own unpreconditioned FGMRES cycle in FP64
// (CGS2, FP64 dots), stopped after m steps by a zero target; V stays in the
// solver's row-interleaved layout, which suits the per-row product x = V c.
// The SVD is a one-sided Jacobi (Hestenes) on one workgroup in FP64, written
// in a canonical form: singular values in decreasing order, each column of Z
// with its entry of largest magnitude positive.  G = Z S^+ (columns of
// singular values <= 1e-12 s_max are zero) turns eps into the coefficients
// c = G eps of x in the basis V_m.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "gnp_internal.hpp"
#include "philox.hpp"
#include "sampler.hpp"
#include "solver.hpp"

struct gnp_sampler {
    gnp_system *sys = nullptr;
    int m = 0, k = 0;
    uint64_t seed = 0;
    gnp::SolveCtx ctx;       // FP64 Arnoldi workspace; ctx.V holds V_k after the run
    double *xi = nullptr;    // start vector (n)
    double *x0 = nullptr;    // the cycle's solution (unused, n)
    double *U = nullptr;     // (k + 1) x k, column-major: Hbar, rotated into W S
    double *Zr = nullptr;    // k x k, column-major: accumulated rotations
    double *G = nullptr;     // k x k, row-major: G[j * k + c]
    double *sv = nullptr;    // k singular values, decreasing
    double *coef = nullptr;  // [coef_cap][k] coefficients of the last draw
    int coef_cap = 0;
};

namespace gnp {

constexpr int SAMPLER_MAX_M = 64;
constexpr double SV_DROP = 1e-12;

__global__ void k_normals_stream(int64_t count, uint64_t seed, uint32_t step, uint32_t stream,
                                 double *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) out[e] = normal_at(seed, step, stream, (uint64_t)e);
}

// Hbar (rows 0..k, columns 0..k-1 of the solver's row-major H0 with row
// stride m) into U, column-major with k + 1 rows.  Hbar is upper
// Hessenberg: the solver writes rows r <= c + 1 of column c only, the rest
// is zero by definition.
__global__ void k_hbar_cols(int k, int m, const double *__restrict__ H0, double *__restrict__ U) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (k + 1) * k) return;
    const int c = e / (k + 1), r = e % (k + 1);
    U[e] = r <= c + 1 ? H0[(int64_t)r * m + c] : 0.0;
}

// One-sided Jacobi SVD of U ((rows) x k, column-major) on one workgroup:
// sweeps of the round-robin pairing (every pair of columns once per sweep,
// disjoint pairs of a round handled by different wavefronts in parallel),
// each pair rotated until its columns are orthogonal to 1e-15, until a sweep
// rotates nothing.  Then s_c = ||u_c||, canonical order and signs, and G.
__global__ __launch_bounds__(BLOCK) void k_jacobi_svd(int rows, int k, double *__restrict__ U,
                                                      double *__restrict__ Zr,
                                                      double *__restrict__ G,
                                                      double *__restrict__ sv) {
    const int t = threadIdx.x, lane = t % WAVE, wv = t / WAVE;
    constexpr int NW = BLOCK / WAVE;
    __shared__ int pos[SAMPLER_MAX_M];
    __shared__ int rotated;
    __shared__ double snorm[SAMPLER_MAX_M], sgn[SAMPLER_MAX_M];
    __shared__ int ord[SAMPLER_MAX_M];
    const int kk = k + (k & 1);  // an odd k pairs with a dummy column
    for (int e = t; e < k * k; e += BLOCK) Zr[e] = (e / k == e % k) ? 1.0 : 0.0;
    for (int i = t; i < kk; i += BLOCK) pos[i] = i;
    __syncthreads();
    for (int sweep = 0; sweep < 60; ++sweep) {
        if (t == 0) rotated = 0;
        __syncthreads();
        for (int r = 0; r + 1 < kk; ++r) {
            for (int pr = wv; pr < kk / 2; pr += NW) {
                int p = pos[pr], q = pos[kk - 1 - pr];
                if (p > q) {
                    const int tmp = p;
                    p = q;
                    q = tmp;
                }
                if (q >= k) continue;
                double a = 0.0, b = 0.0, g = 0.0;
                for (int i = lane; i < rows; i += WAVE) {
                    const double up = U[(int64_t)p * rows + i], uq = U[(int64_t)q * rows + i];
                    a += up * up;
                    b += uq * uq;
                    g += up * uq;
                }
                a = wave_sum(a);
                b = wave_sum(b);
                g = wave_sum(g);
                if (g == 0.0 || fabs(g) <= 1e-15 * sqrt(a * b)) continue;
                const double zeta = (b - a) / (2.0 * g);
                const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + tt * tt), s = c * tt;
                for (int i = lane; i < rows; i += WAVE) {
                    const double up = U[(int64_t)p * rows + i], uq = U[(int64_t)q * rows + i];
                    U[(int64_t)p * rows + i] = c * up - s * uq;
                    U[(int64_t)q * rows + i] = s * up + c * uq;
                }
                for (int i = lane; i < k; i += WAVE) {
                    const double zp = Zr[(int64_t)p * k + i], zq = Zr[(int64_t)q * k + i];
                    Zr[(int64_t)p * k + i] = c * zp - s * zq;
                    Zr[(int64_t)q * k + i] = s * zp + c * zq;
                }
                if (lane == 0) rotated = 1;
            }
            __syncthreads();
            if (t == 0) {  // next round: position 0 fixed, the others rotate by one
                const int last = pos[kk - 1];
                for (int i = kk - 1; i > 1; --i) pos[i] = pos[i - 1];
                if (kk > 1) pos[1] = last;
            }
            __syncthreads();
        }
        const int again = rotated;
        __syncthreads();
        if (!again) break;
    }
    // singular values, decreasing order (ties: lower column first)
    for (int c = wv; c < k; c += NW) {
        double a = 0.0;
        for (int i = lane; i < rows; i += WAVE) a += U[(int64_t)c * rows + i] * U[(int64_t)c * rows + i];
        a = wave_sum(a);
        if (lane == 0) snorm[c] = sqrt(a);
    }
    __syncthreads();
    if (t == 0) {
        for (int c = 0; c < k; ++c) ord[c] = c;
        for (int i = 1; i < k; ++i) {
            const int v = ord[i];
            int j = i - 1;
            while (j >= 0 && snorm[ord[j]] < snorm[v]) {
                ord[j + 1] = ord[j];
                --j;
            }
            ord[j + 1] = v;
        }
    }
    __syncthreads();
    // sign: the entry of largest magnitude of each Z column positive (first on ties)
    if (t < k) {
        const int c = ord[t];
        double best = -1.0, val = 0.0;
        for (int i = 0; i < k; ++i) {
            const double z = Zr[(int64_t)c * k + i];
            if (fabs(z) > best) {
                best = fabs(z);
                val = z;
            }
        }
        sgn[t] = val < 0.0 ? -1.0 : 1.0;
        sv[t] = snorm[c];
    }
    __syncthreads();
    const double smax = k > 0 ? snorm[ord[0]] : 0.0;
    for (int e = t; e < k * k; e += BLOCK) {
        const int j = e / k, c2 = e % k, c = ord[c2];
        const double s = snorm[c];
        G[e] = s > SV_DROP * smax ? sgn[c2] * Zr[(int64_t)c * k + j] / s : 0.0;
    }
}

// c = G eps for `count` draws: block d, lane j (k <= 64)
__global__ void k_sampler_coef(int k, const double *__restrict__ G, uint64_t seed, uint32_t step,
                               double *__restrict__ coef) {
    __shared__ double eps[SAMPLER_MAX_M];
    const int d = blockIdx.x, j = threadIdx.x;
    if (j < k) eps[j] = normal_at(seed, step, 1u, (uint64_t)d * k + j);
    __syncthreads();
    if (j < k) {
        double s = 0.0;
        for (int c = 0; c < k; ++c) s += G[j * k + c] * eps[c];
        coef[(int64_t)d * k + j] = s;
    }
}

// x[i * B + d] = sum_j V[i * mp + j] c_d[j] for d < count (one thread per (i, d))
template <typename T>
__global__ void k_sampler_x(int64_t n, int k, int mp, const double *__restrict__ V,
                            const double *__restrict__ coef, int count, int B, T *__restrict__ x) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * count) return;
    const int64_t i = e / count;
    const int d = (int)(e - i * count);
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += V[i * mp + j] * coef[(int64_t)d * k + j];
    x[i * B + d] = (T)s;
}

template <typename T>
gnp_status sampler_draw_launch(gnp_sampler *sp, uint32_t step, int count, int B, T *x,
                               hipStream_t st) {
    if (count <= 0) return GNP_OK;
    if (count > sp->coef_cap) return fail(GNP_EINVAL, "sampler draw larger than its buffer");
    hipLaunchKernelGGL(k_sampler_coef, dim3(count), dim3(WAVE), 0, st, sp->k,
                       (const double *)sp->G, sp->seed, step, sp->coef);
    const int64_t n = sp->sys->n;
    hipLaunchKernelGGL((k_sampler_x<T>), dim3(grid_for(n * count, BLOCK)), dim3(BLOCK), 0, st, n,
                       sp->k, sp->ctx.mp, (const double *)sp->ctx.V, (const double *)sp->coef,
                       count, B, x);
    GNP_HIP(hipGetLastError());
    return GNP_OK;
}
template gnp_status sampler_draw_launch<float>(gnp_sampler *, uint32_t, int, int, float *,
                                               hipStream_t);
template gnp_status sampler_draw_launch<double>(gnp_sampler *, uint32_t, int, int, double *,
                                                hipStream_t);

static void sampler_free(gnp_sampler *sp) {
    if (!sp) return;
    solve_ctx_free(&sp->ctx);
    for (double *p : {sp->xi, sp->x0, sp->U, sp->Zr, sp->G, sp->sv, sp->coef})
        if (p) (void)hipFree(p);
    delete sp;
}

gnp_status sampler_create(gnp_system *sys, int m, uint64_t seed, int max_count, hipStream_t st,
                          gnp_sampler **out) {
    if (!sys || !out) return fail(GNP_EINVAL, "null argument");
    if (m < 1 || m > SAMPLER_MAX_M) return fail(GNP_EINVAL, "sampler steps m must be in [1, 64]");
    if (m >= sys->n) return fail(GNP_EINVAL, "sampler steps m must be below n");
    if (max_count < 1 || max_count > BLOCK) return fail(GNP_EINVAL, "draws per call must be in [1, 256]");
    gnp_sampler *sp = new gnp_sampler();
    sp->sys = sys;
    sp->m = m;
    sp->seed = seed;
    const int64_t n = sys->n;
    auto fin = [&](gnp_status s) {
        if (s != GNP_OK) sampler_free(sp);
        return s;
    };
    if (solve_ctx_prepare(&sp->ctx, sys, m, m, GNP_F64, 0) != GNP_OK) return fin(GNP_ENOMEM);
    if (hipMalloc(&sp->xi, sizeof(double) * n) != hipSuccess ||
        hipMalloc(&sp->x0, sizeof(double) * n) != hipSuccess ||
        hipMalloc(&sp->U, sizeof(double) * (m + 1) * m) != hipSuccess ||
        hipMalloc(&sp->Zr, sizeof(double) * m * m) != hipSuccess ||
        hipMalloc(&sp->G, sizeof(double) * m * m) != hipSuccess ||
        hipMalloc(&sp->sv, sizeof(double) * m) != hipSuccess ||
        hipMalloc(&sp->coef, sizeof(double) * (int64_t)max_count * m) != hipSuccess)
        return fin(fail(GNP_ENOMEM, "sampler: device allocation failed"));
    sp->coef_cap = max_count;
    // start vector xi ~ N(0, I) (stream 2, step 0), x0 = 0; one cycle of m
    // unpreconditioned steps with a zero target
    hipLaunchKernelGGL(k_normals_stream, dim3(grid_for(n, BLOCK)), dim3(BLOCK), 0, st, n, seed, 0u,
                       2u, sp->xi);
    if (hipMemsetAsync(sp->x0, 0, sizeof(double) * n, st) != hipSuccess)
        return fin(fail(GNP_EDEVICE, "sampler: memset failed"));
    gnp_status s = solve_begin(&sp->ctx, sp->xi, sp->x0, m, 0.0, m, st);
    if (s != GNP_OK) return fin(s);
    if (hipStreamSynchronize(st) != hipSuccess) return fin(fail(GNP_EDEVICE, "sampler: sync failed"));
    if (!(sp->ctx.ctl_host->bnorm > 0.0) || !std::isfinite(sp->ctx.ctl_host->bnorm))
        return fin(fail(GNP_ENUMERIC, "sampler: start vector is zero or not finite"));
    s = solve_next(&sp->ctx, nullptr, sp->xi, sp->x0, m, m, st);
    if (s != GNP_OK) return fin(s);
    if (hipStreamSynchronize(st) != hipSuccess) return fin(fail(GNP_EDEVICE, "sampler: sync failed"));
    const Ctl &h = *sp->ctx.ctl_host;
    if (h.nonfinite) return fin(fail(GNP_ENUMERIC, "sampler: non-finite value in the Arnoldi process"));
    sp->k = h.it;  // Arnoldi steps of the one cycle (the breakdown step included)
    if (sp->k < 1) return fin(fail(GNP_ENUMERIC, "sampler: the Arnoldi process made no step"));
    const int k = sp->k;
    hipLaunchKernelGGL(k_hbar_cols, dim3(grid_for((k + 1) * k, BLOCK)), dim3(BLOCK), 0, st, k, m,
                       (const double *)sp->ctx.H0, sp->U);
    hipLaunchKernelGGL(k_jacobi_svd, dim3(1), dim3(BLOCK), 0, st, k + 1, k, sp->U, sp->Zr, sp->G,
                       sp->sv);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
        return fin(fail(GNP_EDEVICE, "sampler: SVD launch failed"));
    *out = sp;
    return GNP_OK;
}

void sampler_destroy(gnp_sampler *sp) { sampler_free(sp); }

}  // namespace gnp

using namespace gnp;

extern "C" {

gnp_status gnp_sampler_create(gnp_system *sys, int m, uint64_t seed, int max_count,
                              void *hip_stream, gnp_sampler **out) {
    if (out) *out = nullptr;
    return sampler_create(sys, m, seed, max_count, (hipStream_t)hip_stream, out);
}

gnp_status gnp_sampler_info(const gnp_sampler *sp, int *k, double *hbar, double *sv,
                            double *G) {
    if (!sp) return fail(GNP_EINVAL, "null sampler");
    const int kk = sp->k, m = sp->m;
    if (k) *k = kk;
    if (hbar) {
        std::vector<double> h0((size_t)(m + 1) * m);
        GNP_HIP(hipMemcpy(h0.data(), sp->ctx.H0, sizeof(double) * h0.size(), hipMemcpyDeviceToHost));
        for (int r = 0; r <= kk; ++r)  // upper Hessenberg: zero below the subdiagonal
            for (int c = 0; c < kk; ++c)
                hbar[(size_t)r * kk + c] = r <= c + 1 ? h0[(size_t)r * m + c] : 0.0;
    }
    if (sv) GNP_HIP(hipMemcpy(sv, sp->sv, sizeof(double) * kk, hipMemcpyDeviceToHost));
    if (G) GNP_HIP(hipMemcpy(G, sp->G, sizeof(double) * kk * kk, hipMemcpyDeviceToHost));
    return GNP_OK;
}

gnp_status gnp_sampler_draw(gnp_sampler *sp, uint32_t step, int count, double *x_dev,
                            void *hip_stream) {
    if (!sp || !x_dev) return fail(GNP_EINVAL, "null argument");
    if (count < 1 || count > sp->coef_cap) return fail(GNP_EINVAL, "count must be in [1, max_count]");
    return sampler_draw_launch<double>(sp, step, count, count, x_dev, (hipStream_t)hip_stream);
}

void gnp_sampler_destroy(gnp_sampler *sp) { sampler_free(sp); }

}  // extern "C"
