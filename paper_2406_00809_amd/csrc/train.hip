// Training of the graph neural preconditioner (Sec. 2.2 streaming (b, x)
// pairs with x ~ N(0, I), b = A x; Sec. 3: l1 residual loss, Adam, keep the
// best-loss model).  Forward saves the input of every layer; the backward is
// written by hand:
//   decoder:  o = ReLU(X_L W3 + c3) W4 + c4,  z = (tau / sqrt n) o
//   layer:    Y = ReLU(P), P = X U + T W, T = A-hat X   (Eq. (5))
//             dP = dY * [Y > 0], dU = X^T dP, dW = T^T dP,
//             dX = dP U^T + A-hat^T (dP W^T)   (A-hat^T from the transposed CSR)
//   encoder:  E = ReLU(u W1 + c1) W2 + c2
//   loss:     l = mean |A z - b|, dl/dz = A^T sign(A z - b) / (n B)
// Weight gradients are sums over all rows: every block keeps its own sums
// over a fixed set of row tiles and writes one partial per parameter; one
// kernel then adds the partials in block order (deterministic).  The FP32
// backward runs on MFMA (bwd_mfma.hpp); FP64 uses the VALU kernels below.
// The whole training loop is stream-ordered with no host synchronisation.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "bwd_mfma.hpp"
#include "gnp_fwd.hpp"
#include "model.hpp"
#include "philox.hpp"
#include "sampler.hpp"

namespace gnp {

constexpr int TB = 64;       // rows per block tile
constexpr int NBG_MAX = 1024;  // blocks of the gradient kernels

// ---------------------------------------------------------------------------
// x ~ N(0, I) batches: stream 0 of the counter-based generator (philox.hpp)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_normals(int64_t count, uint64_t seed, uint32_t step, T *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    out[e] = (T)normal_at(seed, step, 0u, (uint64_t)e);
}

template <typename S, typename T>
__global__ void k_convert(int64_t count, const S *__restrict__ a, T *__restrict__ b) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) b[e] = (T)a[e];
}

// Y[i, k] = sum_j A_ij X[j, k] for nrhs columns (one thread per (i, k))
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_spmm_rhs(int64_t n, int B, const int32_t *__restrict__ rp,
                                                    const int32_t *__restrict__ ci,
                                                    const T *__restrict__ val,
                                                    const T *__restrict__ X, T *__restrict__ Y) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * B) return;
    const int64_t i = e / B;
    const int k = (int)(e - i * B);
    T acc = 0;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) acc += val[q] * X[(int64_t)ci[q] * B + k];
    Y[e] = acc;
}

// R = A z - b;  S = sign(R) / (n B);  loss = mean |R|  (deterministic)
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_loss(int64_t n, int B, const int32_t *__restrict__ rp,
                                                const int32_t *__restrict__ ci,
                                                const T *__restrict__ val, const T *__restrict__ z,
                                                const T *__restrict__ b, T *__restrict__ S,
                                                double *partial, unsigned *counter,
                                                double *loss_out) {
    __shared__ double sh[BLOCK / WAVE];
    const int64_t rows = n * B;
    double s = 0.0;
    const T inv = (T)(1.0 / (double)rows);
    // four rows of the thread's stride in flight at once; |r| is added in
    // row order
    constexpr int U = 4;
    const int64_t step = (int64_t)gridDim.x * BLOCK;
    for (int64_t e0 = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e0 < rows; e0 += U * step) {
        T r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = e0 + u * step < rows ? e0 + u * step : e0;
            const int64_t i = e / B;
            const int k = (int)(e - i * B);
            T acc = 0;
            for (int32_t q = rp[i]; q < rp[i + 1]; ++q) acc += val[q] * z[(int64_t)ci[q] * B + k];
            r[u] = acc - b[e];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = e0 + u * step;
            if (e < rows) {
                S[e] = r[u] > (T)0 ? inv : (r[u] < (T)0 ? -inv : (T)0);
                s += fabs((double)r[u]);
            }
        }
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
    if (last_block(counter)) {
        double a = 0.0;
        for (unsigned k = threadIdx.x; k < gridDim.x; k += BLOCK) a += partial[k];
        a = block_sum(a, sh);
        if (threadIdx.x == 0) *loss_out = a / (double)rows;
    }
}

// ---------------------------------------------------------------------------
// decoder forward (training: reads the saved X_L)
// ---------------------------------------------------------------------------
template <typename T, int D, int H>
__global__ __launch_bounds__(BLOCK) void k_dec_fwd(int64_t rows, int B, const T *__restrict__ X,
                                                   const T *__restrict__ th, int64_t oW3,
                                                   int64_t oc3, int64_t oW4, int64_t oc4,
                                                   const double *__restrict__ tau,
                                                   T *__restrict__ z) {
    __shared__ T Xs[TB][D + 1];
    const T *W3 = th + oW3, *c3 = th + oc3, *W4 = th + oW4;
    const int rl = threadIdx.x / 4, q = threadIdx.x % 4;
    const int64_t nbt = (rows + TB - 1) / TB;
    for (int64_t bt = blockIdx.x; bt < nbt; bt += gridDim.x) {
        const int64_t r = bt * TB + rl;
#pragma unroll
        for (int e = 0; e < D / 4; ++e)
            Xs[rl][q * (D / 4) + e] = r < rows ? X[r * D + q * (D / 4) + e] : (T)0;
        __syncthreads();
        T part = 0;
        for (int kk = 0; kk < H / 4; ++kk) {
            const int k = q * (H / 4) + kk;
            T hs = c3[k];
            for (int f = 0; f < D; ++f) hs += Xs[rl][f] * W3[f * H + k];
            part += relu(hs) * W4[k];
        }
        part += __shfl_xor(part, 1, 4);
        part += __shfl_xor(part, 2, 4);
        if (q == 0 && r < rows) z[r] = (T)(tau[3 * (r % B) + 2] * (double)(part + th[oc4]));
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// decoder backward: dX_L and partial gradients of W3, c3, W4, c4
// ---------------------------------------------------------------------------
template <typename T, int D, int H>
__global__ __launch_bounds__(BLOCK) void k_dec_bwd(int64_t rows, int B, const T *__restrict__ X,
                                                   const T *__restrict__ dz,
                                                   const T *__restrict__ th, int64_t oW3,
                                                   int64_t oc3, int64_t oW4, int64_t oc4,
                                                   const double *__restrict__ tau,
                                                   T *__restrict__ dX, double *__restrict__ gpart,
                                                   int64_t np) {
    __shared__ T Xs[TB][D + 1];
    __shared__ T PR[TB][H + 1];  // decoder hidden pre-activations
    __shared__ T DO[TB];         // dl/do = (tau / sqrt n) dl/dz
    const T *W3 = th + oW3, *c3 = th + oc3, *W4 = th + oW4;
    const int t = threadIdx.x, rl = t / 4, q = t % 4;
    constexpr int NW3 = D * H / BLOCK;
    T gW3[NW3];
#pragma unroll
    for (int s = 0; s < NW3; ++s) gW3[s] = 0;
    T gc3 = 0, gW4 = 0, gc4 = 0;
    const int64_t nbt = (rows + TB - 1) / TB;
    for (int64_t bt = blockIdx.x; bt < nbt; bt += gridDim.x) {
        const int64_t r = bt * TB + rl;
#pragma unroll
        for (int e = 0; e < D / 4; ++e)
            Xs[rl][q * (D / 4) + e] = r < rows ? X[r * D + q * (D / 4) + e] : (T)0;
        if (q == 0) DO[rl] = r < rows ? (T)(tau[3 * (r % B) + 2] * (double)dz[r]) : (T)0;
        __syncthreads();
        for (int kk = 0; kk < H / 4; ++kk) {
            const int k = q * (H / 4) + kk;
            T pre = c3[k];
            for (int f = 0; f < D; ++f) pre += Xs[rl][f] * W3[f * H + k];
            PR[rl][k] = pre;
        }
        __syncthreads();
        if (r < rows) {
            const T dout = DO[rl];
#pragma unroll
            for (int e = 0; e < D / 4; ++e) {
                const int f = q * (D / 4) + e;
                T acc = 0;
                for (int k = 0; k < H; ++k)
                    if (PR[rl][k] > (T)0) acc += W3[f * H + k] * W4[k];
                dX[r * D + f] = acc * dout;
            }
        }
#pragma unroll
        for (int s = 0; s < NW3; ++s) {
            const int e = t + BLOCK * s, f = e / H, k = e % H;
            T acc = 0;
            for (int row = 0; row < TB; ++row)
                if (PR[row][k] > (T)0) acc += Xs[row][f] * DO[row];
            gW3[s] += W4[k] * acc;
        }
        if (t < H) {
            T a3 = 0, a4 = 0;
            for (int row = 0; row < TB; ++row) {
                const T pre = PR[row][t];
                if (pre > (T)0) {
                    a3 += DO[row];
                    a4 += pre * DO[row];
                }
            }
            gc3 += W4[t] * a3;
            gW4 += a4;
        }
        if (t == 0) {
            T a = 0;
            for (int row = 0; row < TB; ++row) a += DO[row];
            gc4 += a;
        }
        __syncthreads();
    }
    double *gp = gpart + (int64_t)blockIdx.x * np;
#pragma unroll
    for (int s = 0; s < NW3; ++s) gp[oW3 + t + BLOCK * s] = (double)gW3[s];
    if (t < H) {
        gp[oc3 + t] = (double)gc3;
        gp[oW4 + t] = (double)gW4;
    }
    if (t == 0) gp[oc4] = (double)gc4;
}

// ---------------------------------------------------------------------------
// Res-GCONV backward, part 1: recompute T = A-hat X, dP = dY [Y > 0],
// G = dP W^T, Hx = dP U^T, and partial dU = X^T dP, dW = T^T dP.
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ __launch_bounds__(BLOCK) void k_layer_bwd1(
    int64_t rows, int B, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const T *__restrict__ ahat, const T *__restrict__ X, const T *__restrict__ Y,
    const T *__restrict__ dY, const T *__restrict__ th, int64_t oU, T *__restrict__ G,
    T *__restrict__ Hx, double *__restrict__ gpart, int64_t np) {
    __shared__ T Xs[TB][D + 1];
    __shared__ T Ts[TB][D + 1];
    __shared__ T Ps[TB][D + 1];
    const T *U = th + oU, *W = th + oU + D * D;
    const int t = threadIdx.x, rl = t / 4, q = t % 4;
    constexpr int NE = D * D / BLOCK;
    T gU[NE], gW[NE];
#pragma unroll
    for (int s = 0; s < NE; ++s) gU[s] = gW[s] = 0;
    const int64_t nbt = (rows + TB - 1) / TB;
    for (int64_t bt = blockIdx.x; bt < nbt; bt += gridDim.x) {
        const int64_t r = bt * TB + rl;
        T tv[D / 4], xv[D / 4], pv[D / 4];
#pragma unroll
        for (int e = 0; e < D / 4; ++e) tv[e] = xv[e] = pv[e] = 0;
        if (r < rows) {
            const int64_t i = (B == 1) ? r : r / B;
            const int b = (int)(r - i * B);
            for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
                const T a = ahat[k];
                const T *xs = X + ((int64_t)ci[k] * B + b) * D + q * (D / 4);
#pragma unroll
                for (int e = 0; e < D / 4; ++e) tv[e] += a * xs[e];
            }
#pragma unroll
            for (int e = 0; e < D / 4; ++e) {
                const int64_t o = r * D + q * (D / 4) + e;
                xv[e] = X[o];
                pv[e] = Y[o] > (T)0 ? dY[o] : (T)0;
            }
        }
#pragma unroll
        for (int e = 0; e < D / 4; ++e) {
            Xs[rl][q * (D / 4) + e] = xv[e];
            Ts[rl][q * (D / 4) + e] = tv[e];
            Ps[rl][q * (D / 4) + e] = pv[e];
        }
        __syncthreads();
        if (r < rows) {
#pragma unroll
            for (int e = 0; e < D / 4; ++e) {
                const int p = q * (D / 4) + e;
                T g = 0, hx = 0;
                for (int c = 0; c < D; ++c) {
                    g += Ps[rl][c] * W[p * D + c];
                    hx += Ps[rl][c] * U[p * D + c];
                }
                G[r * D + p] = g;
                Hx[r * D + p] = hx;
            }
        }
#pragma unroll
        for (int s = 0; s < NE; ++s) {
            const int e = t + BLOCK * s, p = e / D, c = e % D;
            T au = 0, aw = 0;
            for (int row = 0; row < TB; ++row) {
                au += Xs[row][p] * Ps[row][c];
                aw += Ts[row][p] * Ps[row][c];
            }
            gU[s] += au;
            gW[s] += aw;
        }
        __syncthreads();
    }
    double *gp = gpart + (int64_t)blockIdx.x * np;
#pragma unroll
    for (int s = 0; s < NE; ++s) {
        gp[oU + t + BLOCK * s] = (double)gU[s];
        gp[oU + D * D + t + BLOCK * s] = (double)gW[s];
    }
}

// part 2: dX = Hx + A-hat^T G (gather over the transposed CSR), in place on Hx
template <typename T, int D>
__global__ __launch_bounds__(BLOCK) void k_layer_bwd2(int64_t rows, int B,
                                                      const int32_t *__restrict__ trp,
                                                      const int32_t *__restrict__ tci,
                                                      const T *__restrict__ tahat,
                                                      const T *__restrict__ G,
                                                      T *__restrict__ dX) {
    const int64_t r = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) / 4;
    const int q = threadIdx.x % 4;
    if (r >= rows) return;
    const int64_t i = (B == 1) ? r : r / B;
    const int b = (int)(r - i * B);
    T acc[D / 4];
#pragma unroll
    for (int e = 0; e < D / 4; ++e) acc[e] = dX[r * D + q * (D / 4) + e];
    gather_rows<T, D / 4, sizeof(T) == 8 ? 4 : 8>(tci, tahat, trp[i], trp[i + 1], G,
                                                  (uint32_t)B, (uint32_t)b, q, acc);
#pragma unroll
    for (int e = 0; e < D / 4; ++e) dX[r * D + q * (D / 4) + e] = acc[e];
}

// ---------------------------------------------------------------------------
// encoder backward: partial gradients of W1, c1, W2, c2
// ---------------------------------------------------------------------------
template <typename T, int D, int H>
__global__ __launch_bounds__(BLOCK) void k_enc_bwd(int64_t rows, int B, const T *__restrict__ bin,
                                                   const double *__restrict__ tau,
                                                   const T *__restrict__ th, int64_t oW1,
                                                   int64_t oc1, int64_t oW2, int64_t oc2,
                                                   const T *__restrict__ dE,
                                                   double *__restrict__ gpart, int64_t np) {
    __shared__ T Hb[TB][H + 1];  // ReLU(u W1 + c1), then dl/d(u W1 + c1)
    __shared__ T Es[TB][D + 1];
    __shared__ T Us[TB];
    const T *W1 = th + oW1, *c1 = th + oc1, *W2 = th + oW2;
    const int t = threadIdx.x, rl = t / 4, q = t % 4;
    constexpr int NW2 = H * D / BLOCK;
    T gW2[NW2];
#pragma unroll
    for (int s = 0; s < NW2; ++s) gW2[s] = 0;
    T gc2 = 0, gW1 = 0, gc1 = 0;
    const int64_t nbt = (rows + TB - 1) / TB;
    for (int64_t bt = blockIdx.x; bt < nbt; bt += gridDim.x) {
        const int64_t r = bt * TB + rl;
        const T u = r < rows ? (T)(tau[3 * (r % B) + 1] * (double)bin[r]) : (T)0;
        if (q == 0) Us[rl] = u;
#pragma unroll
        for (int e = 0; e < D / 4; ++e)
            Es[rl][q * (D / 4) + e] = r < rows ? dE[r * D + q * (D / 4) + e] : (T)0;
        __syncthreads();
        T dp[H / 4];
#pragma unroll
        for (int kk = 0; kk < H / 4; ++kk) {
            const int k = q * (H / 4) + kk;
            const T pre = u * W1[k] + c1[k];
            Hb[rl][k] = relu(pre);
            T dh = 0;
            for (int f = 0; f < D; ++f) dh += W2[k * D + f] * Es[rl][f];
            dp[kk] = pre > (T)0 ? dh : (T)0;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < NW2; ++s) {
            const int e = t + BLOCK * s, k = e / D, f = e % D;
            T acc = 0;
            for (int row = 0; row < TB; ++row) acc += Hb[row][k] * Es[row][f];
            gW2[s] += acc;
        }
        if (t < D) {
            T a = 0;
            for (int row = 0; row < TB; ++row) a += Es[row][t];
            gc2 += a;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < H / 4; ++kk) Hb[rl][q * (H / 4) + kk] = dp[kk];
        __syncthreads();
        if (t < H) {
            T a1 = 0, a2 = 0;
            for (int row = 0; row < TB; ++row) {
                a1 += Us[row] * Hb[row][t];
                a2 += Hb[row][t];
            }
            gW1 += a1;
            gc1 += a2;
        }
        __syncthreads();
    }
    double *gp = gpart + (int64_t)blockIdx.x * np;
#pragma unroll
    for (int s = 0; s < NW2; ++s) gp[oW2 + t + BLOCK * s] = (double)gW2[s];
    if (t < D) gp[oc2 + t] = (double)gc2;
    if (t < H) {
        gp[oW1 + t] = (double)gW1;
        gp[oc1 + t] = (double)gc1;
    }
}

// grad[p] = sum over blocks of gpart[blk * np + p], in block order; the
// loads go out 16 at a time ahead of their adds (one round trip per 16
// blocks instead of one per block), the adds keep the block order
__global__ void k_grad_reduce(int64_t np, int nblk, const double *__restrict__ gpart,
                              double *__restrict__ grad) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    constexpr int U = 16;
    double a = 0.0;
    for (int b0 = 0; b0 < nblk; b0 += U) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int b = b0 + u < nblk ? b0 + u : nblk - 1;
            v[u] = gpart[(int64_t)b * np + p];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (b0 + u < nblk) a += v[u];
    }
    grad[p] = a;
}

// best-loss snapshot (two kernels so that every block reads the old best)
__global__ void k_snapshot_copy(int64_t np, const double *loss, const double *best,
                                const double *__restrict__ th, double *__restrict__ th_best) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < np && *loss < *best) th_best[p] = th[p];
}

__global__ void k_snapshot_update(const double *loss, double *best, int *best_step, int step,
                                  int *flag) {
    if (threadIdx.x != 0) return;
    const double l = *loss;
    if (!isfinite(l)) *flag = 1;
    if (l < *best) {
        *best = l;
        *best_step = step;
    }
}

// Adam (Kingma & Ba), bias-corrected, float64 master parameters
__global__ void k_adam(int64_t np, double *__restrict__ th, const double *__restrict__ g,
                       double *__restrict__ m, double *__restrict__ v, int t, double lr, double b1,
                       double b2, double eps, const int *flag) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np || *flag) return;
    const double bc1 = 1.0 - pow(b1, (double)t), bc2 = 1.0 - pow(b2, (double)t);
    const double gp = g[p];
    const double mp = b1 * m[p] + (1.0 - b1) * gp;
    const double vp = b2 * v[p] + (1.0 - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    th[p] -= lr * (mp / bc1) / (sqrt(vp / bc2) + eps);
}

__global__ void k_init_best(double *best, int *best_step, int *flag) {
    *best = INFINITY;
    *best_step = -1;
    *flag = 0;
}

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
struct TrainCtx {
    gnp_precision prec = GNP_F32;
    int nrhs = 0;
    int64_t rows = 0;
    size_t es = 4;  // element size
    void *x = nullptr, *b = nullptr, *z = nullptr, *S = nullptr, *dz = nullptr;
    void *acts = nullptr;             // (L+1) * rows * d
    void *dA = nullptr, *dB = nullptr, *G = nullptr;
    double *tau = nullptr;
    double *gpart = nullptr;          // NBG * np
    double *grad = nullptr, *am = nullptr, *av = nullptr, *th_best = nullptr;
    double *loss = nullptr;           // per step
    int loss_cap = 0;
    double *best = nullptr;
    int *best_step = nullptr, *flag = nullptr;
    double *partial = nullptr;
    unsigned *counters = nullptr;
    int nbg = 0;
    int have_fwd = 0;                 // a saved forward exists (gnp_forward_save)
};

void train_ctx_free(void *p) {
    if (!p) return;
    TrainCtx *c = (TrainCtx *)p;
    void *ptrs[] = {c->x,     c->b,     c->z,       c->S,       c->dz,   c->acts,      c->dA,
                    c->dB,    c->G,     c->tau,     c->gpart,   c->grad, c->am,        c->av,
                    c->th_best, c->loss, c->best,   c->best_step, c->flag, c->partial, c->counters};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    delete c;
}

static gnp_status train_ctx_get(gnp_model *m, gnp_precision prec, int nrhs, int steps,
                                TrainCtx **out) {
    TrainCtx *c = (TrainCtx *)m->train_ctx;
    const size_t es = prec == GNP_F64 ? 8 : 4;
    const int64_t rows = m->sys->n * (int64_t)nrhs;
    if (rows * m->d * (int64_t)es >= (int64_t)1 << 32)
        return fail(GNP_EINVAL,
                    "an activation block (n * batch * d elements) must stay below 4 GiB "
                    "(32-bit gather offsets)");
    if (c && c->nrhs == nrhs && c->es == es && c->loss_cap >= steps) {
        c->prec = prec;
        *out = c;
        return GNP_OK;
    }
    train_ctx_free(c);
    m->train_ctx = nullptr;
    c = new TrainCtx();
    m->train_ctx = c;
    c->prec = prec;
    c->nrhs = nrhs;
    c->rows = rows;
    c->es = es;
    const int64_t d = m->d;
    c->nbg = (int)std::min<int64_t>(NBG_MAX, (rows + TB - 1) / TB);
    GNP_HIP(hipMalloc(&c->x, es * rows));
    GNP_HIP(hipMalloc(&c->b, es * rows));
    GNP_HIP(hipMalloc(&c->z, es * rows));
    GNP_HIP(hipMalloc(&c->S, es * rows));
    GNP_HIP(hipMalloc(&c->dz, es * rows));
    GNP_HIP(hipMalloc(&c->acts, es * rows * d * (m->L + 1)));
    GNP_HIP(hipMalloc(&c->dA, es * rows * d));
    GNP_HIP(hipMalloc(&c->dB, es * rows * d));
    GNP_HIP(hipMalloc(&c->G, es * rows * d));
    GNP_HIP(hipMalloc(&c->tau, sizeof(double) * 3 * nrhs));
    GNP_HIP(hipMalloc(&c->gpart, sizeof(double) * c->nbg * m->np));
    GNP_HIP(hipMalloc(&c->grad, sizeof(double) * m->np));
    GNP_HIP(hipMalloc(&c->am, sizeof(double) * m->np));
    GNP_HIP(hipMalloc(&c->av, sizeof(double) * m->np));
    GNP_HIP(hipMalloc(&c->th_best, sizeof(double) * m->np));
    c->loss_cap = std::max(steps, 1);
    GNP_HIP(hipMalloc(&c->loss, sizeof(double) * c->loss_cap));
    GNP_HIP(hipMalloc(&c->best, sizeof(double)));
    GNP_HIP(hipMalloc(&c->best_step, sizeof(int)));
    GNP_HIP(hipMalloc(&c->flag, sizeof(int)));
    const int64_t npart = std::max<int64_t>(4096, (int64_t)colnorm_blocks(m->sys->n) * nrhs);
    GNP_HIP(hipMalloc(&c->partial, sizeof(double) * npart));
    GNP_HIP(hipMalloc(&c->counters, sizeof(unsigned) * 8));
    GNP_HIP(hipMemset(c->counters, 0, sizeof(unsigned) * 8));
    *out = c;
    return GNP_OK;
}

// ---------------------------------------------------------------------------
// forward (saving layer inputs) and backward
// ---------------------------------------------------------------------------
template <typename T, int D, int H>
static void fwd_save(gnp_model *m, TrainCtx *c, const T *bin, T *z, hipStream_t st) {
    gnp_system *s = m->sys;
    const int B = c->nrhs;
    const int64_t rows = c->rows;
    const ParamOffsets &po = m->po;
    launch_colnorm<T>(m, bin, B, c->tau, c->partial, c->counters + 0, nullptr, st);
    T *acts = (T *)c->acts;
    const int grid = grid_for(rows, 64);
    const T *vec;
    const void *w2;
    const T *ahat;
    if constexpr (sizeof(T) == 8) {
        vec = (const T *)m->theta64;
        w2 = m->theta64 + po.W2;
        ahat = (const T *)s->ahat64;
    } else {
        vec = (const T *)m->theta32;
        w2 = m->pk_f32 + m->pf.W2;
        ahat = (const T *)s->ahat32;
    }
    if constexpr (sizeof(T) == 8) {
        hipLaunchKernelGGL((k_encoder<T, T, D, H>), dim3(grid), dim3(BLOCK), 0, st, rows, B, bin,
                           c->tau, vec, po.W1, po.c1, po.c2, w2, acts, (const int *)nullptr);
    } else {  // the persistent MFMA encoder of the apply path
        const int ge = std::min(grid, resident_blocks<k_encoder_p<T, T, D, H>>());
        hipLaunchKernelGGL((k_encoder_p<T, T, D, H>), dim3(ge), dim3(BLOCK), 0, st, rows, B, bin,
                           c->tau, vec, po.W1, po.c1, po.c2, w2, acts, (const int *)nullptr,
                           BasisNext{}, s->n);
    }
    for (int l = 0; l < m->L; ++l) {
        const void *wc;
        if constexpr (sizeof(T) == 8) wc = m->theta64 + po.U0 + (int64_t)l * 2 * D * D;
        else wc = m->pk_f32 + m->pf.Wcat0 + l * m->pf.Wcat_stride;
        hipLaunchKernelGGL((layer_kernel<T, D, H, false, T>(B, s->max_row)),
                           dim3(layer_grid<T, D, H, false, T>(rows, B, s->max_row)),
                           dim3(BLOCK), 0, st, rows, B,
                           s->rp, s->ci, ahat, acts + (int64_t)l * rows * D,
                           acts + (int64_t)(l + 1) * rows * D, wc, (const void *)nullptr, vec,
                           po.c3, po.W4, po.c4, (const double *)c->tau, (T *)nullptr,
                           (const int *)nullptr);
    }
    const int gd = (int)std::min<int64_t>(4096, (rows + TB - 1) / TB);
    if constexpr (sizeof(T) == 4)
        hipLaunchKernelGGL((k_dec_fwd_mfma<D, H>), dim3(gd), dim3(BLOCK), 0, st, rows, B,
                           acts + (int64_t)m->L * rows * D, vec, po.W3, po.c3, po.W4, po.c4,
                           (const double *)c->tau, z);
    else
        hipLaunchKernelGGL((k_dec_fwd<T, D, H>), dim3(gd), dim3(BLOCK), 0, st, rows, B,
                           acts + (int64_t)m->L * rows * D, vec, po.W3, po.c3, po.W4, po.c4,
                           (const double *)c->tau, z);
}

template <typename T, int D, int H>
static void bwd(gnp_model *m, TrainCtx *c, const T *bin, const T *dz, hipStream_t st) {
    gnp_system *s = m->sys;
    const int B = c->nrhs;
    const int64_t rows = c->rows;
    const ParamOffsets &po = m->po;
    const T *th = sizeof(T) == 8 ? (const T *)m->theta64 : (const T *)m->theta32;
    const T *ahat = sizeof(T) == 8 ? (const T *)s->ahat64 : (const T *)s->ahat32;
    const T *tahat = sizeof(T) == 8 ? (const T *)s->tahat64 : (const T *)s->tahat32;
    T *acts = (T *)c->acts;
    T *dA = (T *)c->dA, *dB = (T *)c->dB, *G = (T *)c->G;
    const int nbg = c->nbg;
    // FP32: MFMA kernels; FP64: VALU kernels (reference precision)
    constexpr bool MF = sizeof(T) == 4;
    if constexpr (MF)
        hipLaunchKernelGGL((k_dec_bwd_mfma<D, H>), dim3(nbg), dim3(BLOCK), 0, st, rows, B,
                           acts + (int64_t)m->L * rows * D, dz, th, po.W3, po.c3, po.W4, po.c4,
                           (const double *)c->tau, dA, c->gpart, m->np);
    else
        hipLaunchKernelGGL((k_dec_bwd<T, D, H>), dim3(nbg), dim3(BLOCK), 0, st, rows, B,
                           acts + (int64_t)m->L * rows * D, dz, th, po.W3, po.c3, po.W4, po.c4,
                           (const double *)c->tau, dA, c->gpart, m->np);
    for (int l = m->L - 1; l >= 0; --l) {
        const int64_t oU = po.U0 + (int64_t)l * 2 * D * D;
        if constexpr (MF)
            hipLaunchKernelGGL((k_layer_bwd1_mfma<D>), dim3(nbg), dim3(BLOCK), 0, st, rows, B,
                               s->rp, s->ci, ahat, acts + (int64_t)l * rows * D,
                               acts + (int64_t)(l + 1) * rows * D, dA, th, oU, G, dB, c->gpart,
                               m->np);
        else
            hipLaunchKernelGGL((k_layer_bwd1<T, D>), dim3(nbg), dim3(BLOCK), 0, st, rows, B,
                               s->rp, s->ci, ahat, acts + (int64_t)l * rows * D,
                               acts + (int64_t)(l + 1) * rows * D, dA, th, oU, G, dB, c->gpart,
                               m->np);
        hipLaunchKernelGGL((k_layer_bwd2<T, D>), dim3(grid_for(rows * 4, BLOCK)), dim3(BLOCK), 0,
                           st, rows, B, s->trp, s->tci, tahat, G, dB);
        std::swap(dA, dB);
    }
    if constexpr (MF)
        hipLaunchKernelGGL((k_enc_bwd_mfma<D, H>), dim3(nbg), dim3(BLOCK), 0, st, rows, B, bin,
                           (const double *)c->tau, th, po.W1, po.c1, po.W2, po.c2, dA, c->gpart,
                           m->np);
    else
        hipLaunchKernelGGL((k_enc_bwd<T, D, H>), dim3(nbg), dim3(BLOCK), 0, st, rows, B, bin,
                           (const double *)c->tau, th, po.W1, po.c1, po.W2, po.c2, dA, c->gpart,
                           m->np);
    hipLaunchKernelGGL(k_grad_reduce, dim3(grid_for(m->np, BLOCK)), dim3(BLOCK), 0, st, m->np,
                       nbg, c->gpart, c->grad);
}

template <typename T>
static void loss_dz(gnp_model *m, TrainCtx *c, const T *bin, const T *z, double *loss_slot,
                    hipStream_t st) {
    gnp_system *s = m->sys;
    const T *val = sizeof(T) == 8 ? (const T *)s->val64 : (const T *)s->val32;
    const T *tval = sizeof(T) == 8 ? (const T *)s->tval64 : (const T *)s->tval32;
    const int B = c->nrhs;
    hipLaunchKernelGGL((k_loss<T>), dim3(grid_for(c->rows, BLOCK, 2048)), dim3(BLOCK), 0, st,
                       s->n, B, s->rp, s->ci, val, z, bin, (T *)c->S, c->partial,
                       c->counters + 1, loss_slot);
    hipLaunchKernelGGL((k_spmm_rhs<T>), dim3(grid_for(c->rows, BLOCK)), dim3(BLOCK), 0, st, s->n,
                       B, s->trp, s->tci, tval, (const T *)c->S, (T *)c->dz);
}

template <typename T, int D, int H>
static gnp_status train_typed(gnp_model *m, TrainCtx *c, const gnp_train_opts *o,
                              const double *x_fixed, gnp_sampler *samp, hipStream_t st) {
    gnp_system *s = m->sys;
    const int64_t rows = c->rows;
    const T *val = sizeof(T) == 8 ? (const T *)s->val64 : (const T *)s->val32;
    T *x = (T *)c->x, *b = (T *)c->b, *z = (T *)c->z;
    const int ge = grid_for(rows, BLOCK), gp = grid_for(m->np, BLOCK);
    GNP_HIP(hipMemsetAsync(c->am, 0, sizeof(double) * m->np, st));
    GNP_HIP(hipMemsetAsync(c->av, 0, sizeof(double) * m->np, st));
    GNP_HIP(hipMemcpyAsync(c->th_best, m->theta64, sizeof(double) * m->np,
                           hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_init_best, dim3(1), dim3(1), 0, st, c->best, c->best_step, c->flag);
    if (x_fixed)
        hipLaunchKernelGGL((k_convert<double, T>), dim3(ge), dim3(BLOCK), 0, st, rows, x_fixed, x);
    for (int t = 0; t < o->steps; ++t) {
        if (!x_fixed) {
            hipLaunchKernelGGL((k_normals<T>), dim3(ge), dim3(BLOCK), 0, st, rows, o->seed,
                               (uint32_t)t, x);
            if (samp)  // the first sampler_count columns from Eq. (3)
                GNP_TRY(sampler_draw_launch<T>(samp, (uint32_t)t, o->sampler_count, c->nrhs, x,
                                               st));
        }
        hipLaunchKernelGGL((k_spmm_rhs<T>), dim3(ge), dim3(BLOCK), 0, st, s->n, c->nrhs, s->rp,
                           s->ci, val, (const T *)x, b);
        fwd_save<T, D, H>(m, c, b, z, st);
        loss_dz<T>(m, c, b, z, c->loss + t, st);
        bwd<T, D, H>(m, c, b, (const T *)c->dz, st);
        hipLaunchKernelGGL(k_snapshot_copy, dim3(gp), dim3(BLOCK), 0, st, m->np, c->loss + t,
                           c->best, m->theta64, c->th_best);
        hipLaunchKernelGGL(k_snapshot_update, dim3(1), dim3(1), 0, st, c->loss + t, c->best,
                           c->best_step, t, c->flag);
        hipLaunchKernelGGL(k_adam, dim3(gp), dim3(BLOCK), 0, st, m->np, m->theta64, c->grad, c->am,
                           c->av, t + 1, o->lr, o->beta1, o->beta2, o->eps, c->flag);
        GNP_TRY(model_repack(m, st));
    }
    GNP_HIP(hipMemcpyAsync(m->theta64, c->th_best, sizeof(double) * m->np,
                           hipMemcpyDeviceToDevice, st));
    GNP_TRY(model_repack(m, st));
    GNP_HIP(hipGetLastError());
    return GNP_OK;
}

template <int D, int H>
static gnp_status train_dispatch(gnp_model *m, TrainCtx *c, const gnp_train_opts *o,
                                 const double *x_fixed, gnp_sampler *samp, hipStream_t st) {
    if (o->prec == GNP_F64) return train_typed<double, D, H>(m, c, o, x_fixed, samp, st);
    return train_typed<float, D, H>(m, c, o, x_fixed, samp, st);
}

template <typename T, int D, int H>
static void fwd_save_any(gnp_model *m, TrainCtx *c, const void *b, void *z, hipStream_t st) {
    fwd_save<T, D, H>(m, c, (const T *)b, (T *)z, st);
}

static void fwd_save_dispatch(gnp_model *m, TrainCtx *c, const void *b, void *z, hipStream_t st) {
    const bool f64 = c->prec == GNP_F64;
    if (m->d == 16) {
        if (f64) fwd_save_any<double, 16, 32>(m, c, b, z, st);
        else fwd_save_any<float, 16, 32>(m, c, b, z, st);
    } else {
        if (f64) fwd_save_any<double, 32, 64>(m, c, b, z, st);
        else fwd_save_any<float, 32, 64>(m, c, b, z, st);
    }
}

static void bwd_dispatch(gnp_model *m, TrainCtx *c, const void *b, const void *dz,
                         hipStream_t st) {
    const bool f64 = c->prec == GNP_F64;
    if (m->d == 16) {
        if (f64) bwd<double, 16, 32>(m, c, (const double *)b, (const double *)dz, st);
        else bwd<float, 16, 32>(m, c, (const float *)b, (const float *)dz, st);
    } else {
        if (f64) bwd<double, 32, 64>(m, c, (const double *)b, (const double *)dz, st);
        else bwd<float, 32, 64>(m, c, (const float *)b, (const float *)dz, st);
    }
}

static gnp_status check_train_prec(gnp_precision p) {
    if (p != GNP_F32 && p != GNP_F64)
        return fail(GNP_EINVAL, "training precision must be GNP_F32 or GNP_F64");
    return GNP_OK;
}

}  // namespace gnp

using namespace gnp;

extern "C" {

gnp_status gnp_train(gnp_model *m, const gnp_train_opts *o, const double *x_fixed_dev,
                     double *loss_hist, int *best_step, void *hip_stream) {
    if (!m || !o) return fail(GNP_EINVAL, "null argument");
    if (o->steps < 1) return fail(GNP_EINVAL, "steps must be >= 1");
    if (o->batch < 1 || o->batch > BLOCK) return fail(GNP_EINVAL, "batch must be in [1, 256]");
    if (!(o->lr > 0.0) || !(o->beta1 >= 0.0 && o->beta1 < 1.0) ||
        !(o->beta2 >= 0.0 && o->beta2 < 1.0) || !(o->eps > 0.0))
        return fail(GNP_EINVAL, "bad Adam hyperparameters");
    GNP_TRY(check_train_prec(o->prec));
    if (o->sampler_m < 0 || (o->sampler_m > 0 && (o->sampler_count < 0 ||
                                                  o->sampler_count > o->batch)))
        return fail(GNP_EINVAL, "sampler_m must be >= 0 and sampler_count in [0, batch]");
    hipStream_t st = (hipStream_t)hip_stream;
    TrainCtx *c = nullptr;
    GNP_TRY(train_ctx_get(m, o->prec, o->batch, o->steps, &c));
    c->have_fwd = 0;
    // the sampler lives for this call; freeing its device memory waits for
    // the kernels that still use it
    struct SamplerGuard {
        gnp_sampler *p = nullptr;
        ~SamplerGuard() { sampler_destroy(p); }
    } samp;
    if (o->sampler_m > 0 && o->sampler_count > 0 && !x_fixed_dev)
        GNP_TRY(sampler_create(m->sys, o->sampler_m, o->seed, o->batch, st, &samp.p));
    if (m->d == 16) GNP_TRY((train_dispatch<16, 32>(m, c, o, x_fixed_dev, samp.p, st)));
    else GNP_TRY((train_dispatch<32, 64>(m, c, o, x_fixed_dev, samp.p, st)));
    int flag = 0, bs = -1;
    GNP_HIP(hipMemcpyAsync(&flag, c->flag, sizeof(int), hipMemcpyDeviceToHost, st));
    GNP_HIP(hipMemcpyAsync(&bs, c->best_step, sizeof(int), hipMemcpyDeviceToHost, st));
    if (loss_hist)
        GNP_HIP(hipMemcpyAsync(loss_hist, c->loss, sizeof(double) * o->steps,
                               hipMemcpyDeviceToHost, st));
    GNP_HIP(hipStreamSynchronize(st));
    if (best_step) *best_step = bs;
    if (flag) return fail(GNP_ENUMERIC, "non-finite training loss");
    return GNP_OK;
}

gnp_status gnp_forward_save(gnp_model *m, const void *b_dev, void *z_dev, int nrhs,
                            gnp_precision prec, void *hip_stream) {
    if (!m || !b_dev || !z_dev) return fail(GNP_EINVAL, "null argument");
    if (nrhs < 1 || nrhs > BLOCK) return fail(GNP_EINVAL, "nrhs must be in [1, 256]");
    GNP_TRY(check_train_prec(prec));
    TrainCtx *c = nullptr;
    GNP_TRY(train_ctx_get(m, prec, nrhs, 1, &c));
    const int64_t bytes = (int64_t)c->es * c->rows;
    hipStream_t st = (hipStream_t)hip_stream;
    GNP_HIP(hipMemcpyAsync(c->b, b_dev, bytes, hipMemcpyDeviceToDevice, st));
    fwd_save_dispatch(m, c, c->b, z_dev, st);
    GNP_HIP(hipGetLastError());
    c->have_fwd = 1;
    return GNP_OK;
}

gnp_status gnp_backward(gnp_model *m, const void *dz_dev, double *dparams_dev, void *hip_stream) {
    if (!m || !dz_dev || !dparams_dev) return fail(GNP_EINVAL, "null argument");
    TrainCtx *c = (TrainCtx *)m->train_ctx;
    if (!c || !c->have_fwd) return fail(GNP_EINVAL, "gnp_backward needs a prior gnp_forward_save");
    hipStream_t st = (hipStream_t)hip_stream;
    bwd_dispatch(m, c, c->b, dz_dev, st);
    GNP_HIP(hipMemcpyAsync(dparams_dev, c->grad, sizeof(double) * m->np,
                           hipMemcpyDeviceToDevice, st));
    GNP_HIP(hipGetLastError());
    return GNP_OK;
}

gnp_status gnp_loss_grad(gnp_model *m, const double *b_dev, int nrhs, gnp_precision prec,
                         double *loss, double *grad, void *hip_stream) {
    if (!m || !b_dev) return fail(GNP_EINVAL, "null argument");
    if (nrhs < 1 || nrhs > BLOCK) return fail(GNP_EINVAL, "nrhs must be in [1, 256]");
    GNP_TRY(check_train_prec(prec));
    TrainCtx *c = nullptr;
    GNP_TRY(train_ctx_get(m, prec, nrhs, 1, &c));
    hipStream_t st = (hipStream_t)hip_stream;
    const int ge = grid_for(c->rows, BLOCK);
    if (prec == GNP_F64)
        hipLaunchKernelGGL((k_convert<double, double>), dim3(ge), dim3(BLOCK), 0, st, c->rows,
                           b_dev, (double *)c->b);
    else
        hipLaunchKernelGGL((k_convert<double, float>), dim3(ge), dim3(BLOCK), 0, st, c->rows,
                           b_dev, (float *)c->b);
    fwd_save_dispatch(m, c, c->b, c->z, st);
    if (prec == GNP_F64) loss_dz<double>(m, c, (const double *)c->b, (const double *)c->z, c->loss, st);
    else loss_dz<float>(m, c, (const float *)c->b, (const float *)c->z, c->loss, st);
    bwd_dispatch(m, c, c->b, c->dz, st);
    c->have_fwd = 1;
    double l = 0.0;
    GNP_HIP(hipMemcpyAsync(&l, c->loss, sizeof(double), hipMemcpyDeviceToHost, st));
    if (grad)
        GNP_HIP(hipMemcpyAsync(grad, c->grad, sizeof(double) * m->np, hipMemcpyDeviceToHost, st));
    GNP_HIP(hipStreamSynchronize(st));
    if (loss) *loss = l;
    if (!std::isfinite(l)) return fail(GNP_ENUMERIC, "non-finite loss");
    return GNP_OK;
}

}  // extern "C"
