// FP32 training kernels of the network on MFMA (v_mfma_f32_16x16x4_f32):
// the decoder forward and the backward of decoder, layers and encoder.
//
// Each wavefront walks 16-row tiles (tile stride = wavefronts in the grid)
// with LDS regions of its own.  Weight gradients are sums over rows of outer
// products, acc += Atile^T Btile, kept in MFMA accumulators across all tiles
// of the wavefront; bias-like gradients are kept per lane in the MFMA result
// layout and summed over the 16 row lanes at the end.  Products with a weight
// matrix are formed transposed (weights as the A operand), so a lane's four
// results are four consecutive features of one row and leave as one 16-byte
// store.  The four wavefronts of a block add their sums in a fixed order
// through LDS, and the block writes one float64 partial per parameter; a
// separate kernel adds the block partials in block order, so the gradient is
// deterministic.
#pragma once
#include "gnp_fwd.hpp"

namespace gnp {

// LDS row stride (floats) of a tile with N features
template <int N> constexpr int ldp() { return N + 1; }

// acc[mt][nt] += sum over the 16 tile rows of A[r][mt*16 + i] * B[r][nt*16 + jj]
template <int M, int N>
__device__ __forceinline__ void outer_acc(const float *A, int lda, const float *Bm, int ldb,
                                          f32x4 (&acc)[M / 16][N / 16], int lane) {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        const int row = 4 * ks + lane / 16;
        float a[M / 16], b[N / 16];
#pragma unroll
        for (int mt = 0; mt < M / 16; ++mt) a[mt] = A[row * lda + mt * 16 + lane % 16];
#pragma unroll
        for (int nt = 0; nt < N / 16; ++nt) b[nt] = Bm[row * ldb + nt * 16 + lane % 16];
#pragma unroll
        for (int mt = 0; mt < M / 16; ++mt)
#pragma unroll
            for (int nt = 0; nt < N / 16; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mt], b[nt], acc[mt][nt], 0, 0, 0);
    }
}

// out^T (P x 16) = Wm (P x K, LDS row stride ldw) * Tile^T with Tile[r][k] in
// LDS; lane l gets out[r = l % 16][p = pt * 16 + 4 (l / 16) + j]
template <int P, int K>
__device__ __forceinline__ void wt_tile(const float *Wm, int ldw, const float *Tile, int ldt,
                                        f32x4 (&out)[P / 16], int lane) {
#pragma unroll
    for (int pt = 0; pt < P / 16; ++pt) out[pt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
    for (int ks = 0; ks < K / 4; ++ks) {
        const int k = 4 * ks + lane / 16;
        const float b = Tile[(lane % 16) * ldt + k];
#pragma unroll
        for (int pt = 0; pt < P / 16; ++pt)
            out[pt] = __builtin_amdgcn_mfma_f32_16x16x4f32(Wm[(pt * 16 + lane % 16) * ldw + k], b,
                                                          out[pt], 0, 0, 0);
    }
}

// acc += sum over k in [k0, k1) of av[k] * X[(ci[k] * B + b) * NF*4 + q * NF + e]
// for the lane's NF features.  Neighbour indices and values are fetched NB at
// a time (clamped, unconditional loads), so NB row loads are in flight at once
// instead of a dependent index -> row chain per neighbour; the sum is taken in
// k order.
template <typename T, int NF, int NB>
__device__ __forceinline__ void gather_rows(const int32_t *__restrict__ ci,
                                            const T *__restrict__ av, int32_t k0, int32_t k1,
                                            const T *__restrict__ X, uint32_t B, uint32_t b,
                                            int q, T (&acc)[NF]) {
    for (int32_t kb = k0; kb < k1; kb += NB) {
        uint32_t c[NB];
        T a[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int32_t k = kb + u < k1 ? kb + u : k1 - 1;
            c[u] = (uint32_t)ci[k];
            a[u] = kb + u < k1 ? av[k] : (T)0;
        }
        T nv[NB][NF];
#pragma unroll
        for (int u = 0; u < NB; ++u)
            load_feats<T, NF>(X + (c[u] * B + b) * (uint32_t)(4 * NF) + q * NF, nv[u]);
#pragma unroll
        for (int u = 0; u < NB; ++u)
#pragma unroll
            for (int e = 0; e < NF; ++e) acc[e] += a[u] * nv[u][e];
    }
}

// sum over the lanes of a 16-lane group (the row lanes of the result layout)
__device__ __forceinline__ float sum16(float v) {
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    return v;
}

// Block partial of an (M x N) outer-product gradient: the wavefronts add into
// buf (M * N floats) one after another, then the block writes float64 values
// to gp[off + p * N + q].
template <int M, int N>
__device__ __forceinline__ void flush_outer(const f32x4 (&acc)[M / 16][N / 16], float *buf,
                                            double *gp, int64_t off, int lane, int wv) {
    for (int w = 0; w < BLOCK / WAVE; ++w) {
        if (wv == w) {
#pragma unroll
            for (int mt = 0; mt < M / 16; ++mt)
#pragma unroll
                for (int nt = 0; nt < N / 16; ++nt)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int e = (mt * 16 + 4 * (lane / 16) + j) * N + nt * 16 + lane % 16;
                        buf[e] = w == 0 ? acc[mt][nt][j] : buf[e] + acc[mt][nt][j];
                    }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < M * N; e += BLOCK) gp[off + e] = (double)buf[e];
    __syncthreads();
}

// Block partial of a length-K vector gradient held per lane in the result
// layout, v[kt][j] for feature kt * 16 + 4 (l / 16) + j (summed over the row
// lanes first).
template <int K>
__device__ __forceinline__ void flush_vec(const float (&v)[K / 16][4], float *buf, double *gp,
                                          int64_t off, int lane, int wv) {
    float s[K / 16][4];
#pragma unroll
    for (int kt = 0; kt < K / 16; ++kt)
#pragma unroll
        for (int j = 0; j < 4; ++j) s[kt][j] = sum16(v[kt][j]);
    for (int w = 0; w < BLOCK / WAVE; ++w) {
        if (wv == w && lane % 16 == 0) {
#pragma unroll
            for (int kt = 0; kt < K / 16; ++kt)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int e = kt * 16 + 4 * (lane / 16) + j;
                    buf[e] = w == 0 ? s[kt][j] : buf[e] + s[kt][j];
                }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < K; e += BLOCK) gp[off + e] = (double)buf[e];
    __syncthreads();
}

// Block partial of a scalar (lane 0 of each wavefront holds the wave's sum)
__device__ __forceinline__ void flush_scalar(float v, float *buf, double *gp, int64_t off,
                                             int lane, int wv) {
    if (lane == 0) buf[wv] = v;
    __syncthreads();
    if (threadIdx.x == 0) gp[off] = (double)(((buf[0] + buf[1]) + buf[2]) + buf[3]);
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Decoder forward of training (reads the saved X_L):
//   z = (tau / sqrt n) (ReLU(X_L W3 + c3) W4 + c4)   (Eq. (6))
// ---------------------------------------------------------------------------
template <int D, int H>
__global__ __launch_bounds__(BLOCK) void k_dec_fwd_mfma(int64_t rows, int B,
                                                        const float *__restrict__ X,
                                                        const float *__restrict__ th, int64_t oW3,
                                                        int64_t oc3, int64_t oW4, int64_t oc4,
                                                        const double *__restrict__ tau,
                                                        float *__restrict__ z) {
    constexpr int LX = ldp<D>(), LH = ldp<H>();
    __shared__ float smem[4 * 16 * LX];
    __shared__ float W3s[D * LH];  // W3[f][k]
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    float *Xs = smem + wv * 16 * LX;
    for (int e = threadIdx.x; e < D * H; e += BLOCK) W3s[(e / H) * LH + e % H] = th[oW3 + e];
    __syncthreads();
    float c3r[H / 16][4], w4r[H / 16][4];
#pragma unroll
    for (int kt = 0; kt < H / 16; ++kt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            c3r[kt][j] = th[oc3 + kt * 16 + 4 * (lane / 16) + j];
            w4r[kt][j] = th[oW4 + kt * 16 + 4 * (lane / 16) + j];
        }
    const float c4 = th[oc4];
    const int64_t ntiles = (rows + 15) / 16, nw = (int64_t)gridDim.x * (BLOCK / WAVE);
    for (int64_t t = (int64_t)blockIdx.x * (BLOCK / WAVE) + wv; t < ntiles; t += nw) {
        const int64_t r0 = t * 16;
        {
            const int rl = lane / 4, q = lane % 4;
            const int64_t r = r0 + rl;
            float xv[D / 4];
#pragma unroll
            for (int e = 0; e < D / 4; ++e) xv[e] = 0.f;
            if (r < rows) load_feats<float, D / 4>(X + r * D + q * (D / 4), xv);
#pragma unroll
            for (int e = 0; e < D / 4; ++e) Xs[rl * LX + q * (D / 4) + e] = xv[e];
        }
        wave_lds_sync();
        f32x4 pre[H / 16];
#pragma unroll
        for (int kt = 0; kt < H / 16; ++kt) pre[kt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
        for (int ks = 0; ks < D / 4; ++ks) {
            const int f = 4 * ks + lane / 16;
            const float b = Xs[(lane % 16) * LX + f];
#pragma unroll
            for (int kt = 0; kt < H / 16; ++kt)
                pre[kt] = __builtin_amdgcn_mfma_f32_16x16x4f32(W3s[f * LH + kt * 16 + lane % 16], b,
                                                              pre[kt], 0, 0, 0);
        }
        float part = 0.f;
#pragma unroll
        for (int kt = 0; kt < H / 16; ++kt)
#pragma unroll
            for (int j = 0; j < 4; ++j) part += fmaxf(pre[kt][j] + c3r[kt][j], 0.f) * w4r[kt][j];
        part += __shfl_xor(part, 16);
        part += __shfl_xor(part, 32);
        const int64_t r = r0 + lane;
        if (lane < 16 && r < rows) z[r] = (float)(tau[3 * (r % B) + 2] * (double)(part + c4));
        wave_lds_sync();
    }
}

// ---------------------------------------------------------------------------
// Decoder backward.  Forward: pre = X_L W3 + c3, o = ReLU(pre) W4 + c4,
// z = (tau / sqrt n) o (Eq. (6)).  With do = (tau / sqrt n) dz and
// dh = [pre > 0] W4 do:
//   dX_L = dh W3^T, dW3 += X_L^T dh, dc3 += sum dh, dW4 += sum ReLU(pre) do,
//   dc4 += sum do.
// ---------------------------------------------------------------------------
template <int D, int H>
__global__ __launch_bounds__(BLOCK) void k_dec_bwd_mfma(int64_t rows, int B,
                                                        const float *__restrict__ X,
                                                        const float *__restrict__ dz,
                                                        const float *__restrict__ th, int64_t oW3,
                                                        int64_t oc3, int64_t oW4, int64_t oc4,
                                                        const double *__restrict__ tau,
                                                        float *__restrict__ dX,
                                                        double *__restrict__ gpart, int64_t np) {
    constexpr int LX = ldp<D>(), LH = ldp<H>();
    constexpr int WAVE_F = 16 * LX + 16 * LH + 16;  // floats per wavefront
    constexpr int SM = 4 * WAVE_F > D * H ? 4 * WAVE_F : D * H;
    __shared__ float smem[SM];
    __shared__ float W3s[D * LH];  // W3[f][k]
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    float *Xs = smem + wv * WAVE_F, *DH = Xs + 16 * LX, *DO = DH + 16 * LH;
    for (int e = threadIdx.x; e < D * H; e += BLOCK) W3s[(e / H) * LH + e % H] = th[oW3 + e];
    __syncthreads();
    float c3r[H / 16][4], w4r[H / 16][4];
#pragma unroll
    for (int kt = 0; kt < H / 16; ++kt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            c3r[kt][j] = th[oc3 + kt * 16 + 4 * (lane / 16) + j];
            w4r[kt][j] = th[oW4 + kt * 16 + 4 * (lane / 16) + j];
        }
    f32x4 gW3[D / 16][H / 16];
    float gc3[H / 16][4], gW4[H / 16][4];
#pragma unroll
    for (int a = 0; a < D / 16; ++a)
#pragma unroll
        for (int b = 0; b < H / 16; ++b) gW3[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < H / 16; ++kt)
#pragma unroll
        for (int j = 0; j < 4; ++j) gc3[kt][j] = gW4[kt][j] = 0.f;
    float gc4 = 0.f;
    const int64_t ntiles = (rows + 15) / 16, nw = (int64_t)gridDim.x * (BLOCK / WAVE);
    for (int64_t t = (int64_t)blockIdx.x * (BLOCK / WAVE) + wv; t < ntiles; t += nw) {
        const int64_t r0 = t * 16;
        {
            const int rl = lane / 4, q = lane % 4;
            const int64_t r = r0 + rl;
            float xv[D / 4];
#pragma unroll
            for (int e = 0; e < D / 4; ++e) xv[e] = 0.f;
            if (r < rows) load_feats<float, D / 4>(X + r * D + q * (D / 4), xv);
#pragma unroll
            for (int e = 0; e < D / 4; ++e) Xs[rl * LX + q * (D / 4) + e] = xv[e];
            if (lane < 16) {
                const int64_t rr = r0 + lane;
                DO[lane] = rr < rows ? (float)(tau[3 * (rr % B) + 2] * (double)dz[rr]) : 0.f;
            }
        }
        wave_lds_sync();
        // pre^T = W3^T X^T  (A operand: A[k][f] = W3[f][k])
        f32x4 pre[H / 16];
#pragma unroll
        for (int kt = 0; kt < H / 16; ++kt) pre[kt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
        for (int ks = 0; ks < D / 4; ++ks) {
            const int f = 4 * ks + lane / 16;
            const float b = Xs[(lane % 16) * LX + f];
#pragma unroll
            for (int kt = 0; kt < H / 16; ++kt)
                pre[kt] = __builtin_amdgcn_mfma_f32_16x16x4f32(W3s[f * LH + kt * 16 + lane % 16], b,
                                                              pre[kt], 0, 0, 0);
        }
        const float dout = DO[lane % 16];
#pragma unroll
        for (int kt = 0; kt < H / 16; ++kt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float p = pre[kt][j] + c3r[kt][j];
                const float dh = p > 0.f ? w4r[kt][j] * dout : 0.f;
                DH[(lane % 16) * LH + kt * 16 + 4 * (lane / 16) + j] = dh;
                gc3[kt][j] += dh;
                gW4[kt][j] += (p > 0.f ? p : 0.f) * dout;
            }
        if (lane == 0) {
            float s = 0.f;
            for (int row = 0; row < 16; ++row) s += DO[row];
            gc4 += s;
        }
        wave_lds_sync();
        // dX^T = W3 DH^T
        f32x4 dx[D / 16];
        wt_tile<D, H>(W3s, LH, DH, LH, dx, lane);
        const int64_t r = r0 + lane % 16;
        if (r < rows) {
#pragma unroll
            for (int ft = 0; ft < D / 16; ++ft)
                store4<float>(dX + r * D + ft * 16 + 4 * (lane / 16), dx[ft][0], dx[ft][1],
                              dx[ft][2], dx[ft][3]);
        }
        outer_acc<D, H>(Xs, LX, DH, LH, gW3, lane);
        wave_lds_sync();
    }
    __syncthreads();
    double *gp = gpart + (int64_t)blockIdx.x * np;
    flush_outer<D, H>(gW3, smem, gp, oW3, lane, wv);
    flush_vec<H>(gc3, smem, gp, oc3, lane, wv);
    flush_vec<H>(gW4, smem, gp, oW4, lane, wv);
    flush_scalar(gc4, smem, gp, oc4, lane, wv);
}

// ---------------------------------------------------------------------------
// Res-GCONV backward, part 1 (Eq. (5), Y = ReLU(X U + A-hat X W)):
// recompute T = A-hat X, dP = dY [Y > 0], store G = dP W^T and Hx = dP U^T,
// and accumulate dU += X^T dP, dW += T^T dP.
// When B is a multiple of 16 (the training batches), the 16 rows of a tile
// are right-hand sides of one node and share its CSR row: the row pointers
// are fetched two tiles ahead and the row's first NE entries one tile ahead,
// so a tile costs one memory round trip (its own rows and all neighbour rows
// in flight together).  Either way T is summed in CSR order.
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(BLOCK) void k_layer_bwd1_mfma(
    int64_t rows, int B, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const float *__restrict__ ahat, const float *__restrict__ X, const float *__restrict__ Y,
    const float *__restrict__ dY, const float *__restrict__ th, int64_t oU,
    float *__restrict__ G, float *__restrict__ Hx, double *__restrict__ gpart, int64_t np) {
    constexpr int LX = ldp<D>();
    constexpr int WAVE_F = 3 * 16 * LX;
    constexpr int SM = 4 * WAVE_F > D * D ? 4 * WAVE_F : D * D;
    __shared__ float smem[SM];
    __shared__ float Us[D * LX], Ws[D * LX];
    const int lane = threadIdx.x % WAVE;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    float *Xs = smem + wv * WAVE_F, *Ts = Xs + 16 * LX, *Ps = Ts + 16 * LX;
    for (int e = threadIdx.x; e < D * D; e += BLOCK) {
        Us[(e / D) * LX + e % D] = th[oU + e];
        Ws[(e / D) * LX + e % D] = th[oU + D * D + e];
    }
    __syncthreads();
    f32x4 gU[D / 16][D / 16], gW[D / 16][D / 16];
#pragma unroll
    for (int a = 0; a < D / 16; ++a)
#pragma unroll
        for (int b = 0; b < D / 16; ++b) gU[a][b] = gW[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int64_t ntiles = (rows + 15) / 16, nw = (int64_t)gridDim.x * (BLOCK / WAVE);
    const int rl = lane / 4, q = lane % 4;
    // the tile's rows staged in LDS: products with the weights, stores, and
    // the weight-gradient outer products
    auto stage = [&](const float (&xv)[D / 4], const float (&tv)[D / 4], const float (&yv)[D / 4],
                     const float (&gv)[D / 4]) {
#pragma unroll
        for (int e = 0; e < D / 4; ++e) {
            Xs[rl * LX + q * (D / 4) + e] = xv[e];
            Ts[rl * LX + q * (D / 4) + e] = tv[e];
            Ps[rl * LX + q * (D / 4) + e] = yv[e] > 0.f ? gv[e] : 0.f;
        }
    };
    auto finish = [&](int64_t r0) {
        wave_lds_sync();
        f32x4 o[D / 16];
        const int64_t r = r0 + lane % 16;
        wt_tile<D, D>(Ws, LX, Ps, LX, o, lane);  // G^T = W dP^T
        if (r < rows) {
#pragma unroll
            for (int pt = 0; pt < D / 16; ++pt)
                store4<float>(G + r * D + pt * 16 + 4 * (lane / 16), o[pt][0], o[pt][1], o[pt][2],
                              o[pt][3]);
        }
        wt_tile<D, D>(Us, LX, Ps, LX, o, lane);  // Hx^T = U dP^T
        if (r < rows) {
#pragma unroll
            for (int pt = 0; pt < D / 16; ++pt)
                store4<float>(Hx + r * D + pt * 16 + 4 * (lane / 16), o[pt][0], o[pt][1], o[pt][2],
                              o[pt][3]);
        }
        outer_acc<D, D>(Xs, LX, Ps, LX, gU, lane);
        outer_acc<D, D>(Ts, LX, Ps, LX, gW, lane);
        wave_lds_sync();
    };
    int64_t t = (int64_t)blockIdx.x * (BLOCK / WAVE) + wv;
    if (B % 16 == 0) {
        constexpr int NE = 8;  // entries of the shared CSR row prefetched per tile
        // node of tile tt (clamped past the end: loads stay in range, results unused)
        auto node = [&](int64_t tt) -> int64_t { return (tt < ntiles ? tt : ntiles - 1) * 16 / B; };
        // entries rs.. of a row ending at re: column and weight, 0 past the end
        auto entries = [&](int32_t rs, int32_t re, int32_t (&c)[NE], float (&w)[NE]) {
#pragma unroll
            for (int u = 0; u < NE; ++u) {
                const int32_t k = rs + u;
                const int32_t kc = k < re ? k : (re > 0 ? re - 1 : 0);
                c[u] = ci[kc];
                w[u] = k < re ? ahat[kc] : 0.f;
            }
        };
        int64_t i0 = node(t);
        int32_t rs0 = rp[i0], re0 = rp[i0 + 1];
        int32_t c0[NE];
        float a0[NE];
        entries(rs0, re0, c0, a0);
        const int64_t i1 = node(t + nw);
        int32_t rs1 = rp[i1], re1 = rp[i1 + 1];
        for (; t < ntiles; t += nw) {
            // next tile's entries and the row pointers of the one after, in
            // flight with this tile's loads
            int32_t c1[NE];
            float a1[NE];
            entries(rs1, re1, c1, a1);
            const int64_t i2 = node(t + 2 * nw);
            const int32_t rs2 = rp[i2], re2 = rp[i2 + 1];
            const int64_t r0 = t * 16;
            {
                const int64_t r = r0 + rl;  // rows is a multiple of 16 here
                const uint32_t b = (uint32_t)(r % B);
                float tv[D / 4], xv[D / 4], yv[D / 4], gv[D / 4];
                load_feats<float, D / 4>(X + r * D + q * (D / 4), xv);
                load_feats<float, D / 4>(Y + r * D + q * (D / 4), yv);
                load_feats<float, D / 4>(dY + r * D + q * (D / 4), gv);
                float nv[NE][D / 4];
#pragma unroll
                for (int u = 0; u < NE; ++u)
                    load_feats<float, D / 4>(X + ((int64_t)c0[u] * B + b) * D + q * (D / 4), nv[u]);
#pragma unroll
                for (int e = 0; e < D / 4; ++e) tv[e] = 0.f;
#pragma unroll
                for (int u = 0; u < NE; ++u)
#pragma unroll
                    for (int e = 0; e < D / 4; ++e) tv[e] += a0[u] * nv[u][e];
                if (re0 - rs0 > NE)  // the rest of a longer row, in order
                    gather_rows<float, D / 4, 4>(ci, ahat, rs0 + NE, re0, X, (uint32_t)B, b, q, tv);
                stage(xv, tv, yv, gv);
            }
            finish(r0);
#pragma unroll
            for (int u = 0; u < NE; ++u) {
                c0[u] = c1[u];
                a0[u] = a1[u];
            }
            rs0 = rs1;
            re0 = re1;
            rs1 = rs2;
            re1 = re2;
        }
    } else {
        for (; t < ntiles; t += nw) {
            const int64_t r0 = t * 16;
            {
                const int64_t r = r0 + rl;
                float tv[D / 4], xv[D / 4], yv[D / 4], gv[D / 4];
#pragma unroll
                for (int e = 0; e < D / 4; ++e) tv[e] = xv[e] = yv[e] = gv[e] = 0.f;
                if (r < rows) {
                    const int64_t i = (B == 1) ? r : r / B;
                    const int b = (int)(r - i * B);
                    load_feats<float, D / 4>(X + r * D + q * (D / 4), xv);
                    load_feats<float, D / 4>(Y + r * D + q * (D / 4), yv);
                    load_feats<float, D / 4>(dY + r * D + q * (D / 4), gv);
                    gather_rows<float, D / 4, 4>(ci, ahat, rp[i], rp[i + 1], X, (uint32_t)B,
                                                 (uint32_t)b, q, tv);
                }
                stage(xv, tv, yv, gv);
            }
            finish(r0);
        }
    }
    __syncthreads();
    double *gp = gpart + (int64_t)blockIdx.x * np;
    flush_outer<D, D>(gU, smem, gp, oU, lane, wv);
    flush_outer<D, D>(gW, smem, gp, oU + D * D, lane, wv);
}

// ---------------------------------------------------------------------------
// Encoder backward.  Forward: pre = u W1 + c1, hid = ReLU(pre),
// E = hid W2 + c2 with u = (sqrt n / tau) b (Eq. (6)).  With dE given:
//   dpre = [pre > 0] dE W2^T, dW2 += hid^T dE, dc2 += sum dE,
//   dW1 += sum u dpre, dc1 += sum dpre.
// ---------------------------------------------------------------------------
template <int D, int H>
__global__ __launch_bounds__(BLOCK) void k_enc_bwd_mfma(int64_t rows, int B,
                                                        const float *__restrict__ bin,
                                                        const double *__restrict__ tau,
                                                        const float *__restrict__ th, int64_t oW1,
                                                        int64_t oc1, int64_t oW2, int64_t oc2,
                                                        const float *__restrict__ dE,
                                                        double *__restrict__ gpart, int64_t np) {
    constexpr int LX = ldp<D>();
    constexpr int WAVE_F = 16 * LX + 16;
    constexpr int SM = 4 * WAVE_F > H * D ? 4 * WAVE_F : H * D;
    __shared__ float smem[SM];
    __shared__ float W2s[H * LX];  // W2[k][f]
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    float *Es = smem + wv * WAVE_F, *Us = Es + 16 * LX;
    for (int e = threadIdx.x; e < H * D; e += BLOCK) W2s[(e / D) * LX + e % D] = th[oW2 + e];
    __syncthreads();
    // W1, c1 in the two layouts used below: A operand (feature mt*16 + l%16)
    // and result (feature kt*16 + 4 (l/16) + j)
    float w1a[H / 16], c1a[H / 16], w1r[H / 16][4], c1r[H / 16][4];
#pragma unroll
    for (int kt = 0; kt < H / 16; ++kt) {
        w1a[kt] = th[oW1 + kt * 16 + lane % 16];
        c1a[kt] = th[oc1 + kt * 16 + lane % 16];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            w1r[kt][j] = th[oW1 + kt * 16 + 4 * (lane / 16) + j];
            c1r[kt][j] = th[oc1 + kt * 16 + 4 * (lane / 16) + j];
        }
    }
    f32x4 gW2[H / 16][D / 16];
    float gW1[H / 16][4], gc1[H / 16][4], gc2[D / 4];
#pragma unroll
    for (int a = 0; a < H / 16; ++a)
#pragma unroll
        for (int b = 0; b < D / 16; ++b) gW2[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < H / 16; ++kt)
#pragma unroll
        for (int j = 0; j < 4; ++j) gW1[kt][j] = gc1[kt][j] = 0.f;
#pragma unroll
    for (int e = 0; e < D / 4; ++e) gc2[e] = 0.f;
    const int64_t ntiles = (rows + 15) / 16, nw = (int64_t)gridDim.x * (BLOCK / WAVE);
    for (int64_t t = (int64_t)blockIdx.x * (BLOCK / WAVE) + wv; t < ntiles; t += nw) {
        const int64_t r0 = t * 16;
        {
            const int rl = lane / 4, q = lane % 4;
            const int64_t r = r0 + rl;
            float ev[D / 4];
#pragma unroll
            for (int e = 0; e < D / 4; ++e) ev[e] = 0.f;
            if (r < rows) load_feats<float, D / 4>(dE + r * D + q * (D / 4), ev);
#pragma unroll
            for (int e = 0; e < D / 4; ++e) {
                Es[rl * LX + q * (D / 4) + e] = ev[e];
                gc2[e] += ev[e];
            }
            if (lane < 16) {
                const int64_t rr = r0 + lane;
                Us[lane] = rr < rows ? (float)(tau[3 * (rr % B) + 1] * (double)bin[rr]) : 0.f;
            }
        }
        wave_lds_sync();
        // dhid^T = W2 dE^T
        f32x4 dh[H / 16];
        wt_tile<H, D>(W2s, LX, Es, LX, dh, lane);
        const float u = Us[lane % 16];
#pragma unroll
        for (int kt = 0; kt < H / 16; ++kt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float dp = u * w1r[kt][j] + c1r[kt][j] > 0.f ? dh[kt][j] : 0.f;
                gW1[kt][j] += u * dp;
                gc1[kt][j] += dp;
            }
        // dW2 += hid^T dE with hid rebuilt in the A-operand layout
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int row = 4 * ks + lane / 16;
            const float ur = Us[row];
            float b[D / 16];
#pragma unroll
            for (int nt = 0; nt < D / 16; ++nt) b[nt] = Es[row * LX + nt * 16 + lane % 16];
#pragma unroll
            for (int mt = 0; mt < H / 16; ++mt) {
                const float a = fmaxf(ur * w1a[mt] + c1a[mt], 0.f);
#pragma unroll
                for (int nt = 0; nt < D / 16; ++nt)
                    gW2[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[nt], gW2[mt][nt], 0, 0, 0);
            }
        }
        wave_lds_sync();
    }
    // gc2: lanes with equal l % 4 hold the same features; sum them
#pragma unroll
    for (int e = 0; e < D / 4; ++e) {
        float v = gc2[e];
        v += __shfl_xor(v, 4);
        v += __shfl_xor(v, 8);
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        gc2[e] = v;
    }
    __syncthreads();
    double *gp = gpart + (int64_t)blockIdx.x * np;
    flush_outer<H, D>(gW2, smem, gp, oW2, lane, wv);
    flush_vec<H>(gW1, smem, gp, oW1, lane, wv);
    flush_vec<H>(gc1, smem, gp, oc1, lane, wv);
    for (int w = 0; w < BLOCK / WAVE; ++w) {
        if (wv == w && lane < 4) {
#pragma unroll
            for (int e = 0; e < D / 4; ++e) {
                const int f = lane * (D / 4) + e;
                smem[f] = w == 0 ? gc2[e] : smem[f] + gc2[e];
            }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < D; e += BLOCK) gp[oc2 + e] = (double)smem[e];
}

}  // namespace gnp
