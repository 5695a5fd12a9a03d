// Forward kernels of the graph neural preconditioner (Sec. 2.3).
//
// Rows of the activation matrices are (node, right-hand side) pairs,
// r = i * nrhs + k, node-major, with d features per row.  Every kernel runs
// 256-thread blocks of four wavefronts; each wavefront owns one tile of 16
// consecutive rows, so a block covers 64 rows.
//
// Arithmetic per activation storage type G:
//   double   : FP64 VALU (reference-precision instantiation)
//   float    : FP32 MFMA v_mfma_f32_16x16x4_f32
//   uint16_t : bf16 storage, MFMA v_mfma_f32_16x16x32_bf16, FP32 accumulation
//
// MFMA operand layouts (64 lanes, l = lane):
//   A (16 x K):  row = l % 16, k-slot = l / 16 (f32: 1 value; bf16: 8 values)
//   B (K x 16):  col = l % 16, same k-slot as A
//   D (16 x 16): col = l % 16, rows 4 * (l / 16) + j, j = 0..3
#pragma once
#include "model.hpp"

namespace gnp {

template <int BYTES> struct alignas(BYTES >= 16 ? 16 : BYTES) Chunk {
    uint32_t w[BYTES / 4];
};

template <typename G> struct Act;
template <> struct Act<double> {
    using acc = double;  // accumulation type
    using mt = double;   // LDS tile type
    using vt = double;   // A-hat value type
    static __device__ __forceinline__ double get(double v) { return v; }
    static __device__ __forceinline__ double put(double v) { return v; }
};
template <> struct Act<float> {
    using acc = float;
    using mt = float;
    using vt = float;
    static __device__ __forceinline__ float get(float v) { return v; }
    static __device__ __forceinline__ float put(float v) { return v; }
};
template <> struct Act<uint16_t> {
    using acc = float;
    using mt = uint16_t;
    using vt = float;
    static __device__ __forceinline__ float get(uint16_t v) { return bf2f(v); }
    static __device__ __forceinline__ uint16_t put(float v) { return f2bf(v); }
};

template <typename G, int N>
__device__ __forceinline__ void load_feats(const G *p, typename Act<G>::acc (&out)[N]) {
    constexpr int BYTES = N * (int)sizeof(G);
    Chunk<BYTES> c = *reinterpret_cast<const Chunk<BYTES> *>(p);
    const G *e = reinterpret_cast<const G *>(&c);
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] = Act<G>::get(e[i]);
}

template <typename G, int N>
__device__ __forceinline__ void store_feats(G *p, const typename Act<G>::acc (&in)[N]) {
    constexpr int BYTES = N * (int)sizeof(G);
    Chunk<BYTES> c;
    G *e = reinterpret_cast<G *>(&c);
#pragma unroll
    for (int i = 0; i < N; ++i) e[i] = Act<G>::put(in[i]);
    *reinterpret_cast<Chunk<BYTES> *>(p) = c;
}

template <typename T> __device__ __forceinline__ T relu(T x) { return x > (T)0 ? x : (T)0; }

// Every LDS region of these kernels belongs to one wavefront, and a
// wavefront's LDS operations execute in order, so a wavefront-scope fence
// (ordering for the compiler) replaces a block barrier between the write and
// read phases; the four wavefronts of a block never wait for each other.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ bf16x8 load_bf16x8(const uint16_t *p) {
    uint4 u = *reinterpret_cast<const uint4 *>(p);
    return __builtin_bit_cast(bf16x8, u);
}

template <typename G> constexpr int lds_pad() {
    return sizeof(G) == 2 ? 8 : (sizeof(G) == 4 ? 4 : 2);
}

// ---------------------------------------------------------------------------
// Encoder: E = ReLU(u W1 + c1) W2 + c2 with u = (sqrt(n)/tau) v  (Eq. (6)).
// The hidden activations form the MFMA A operand directly in registers.
// ---------------------------------------------------------------------------
template <typename G, typename IN, int D, int H>
__global__ __launch_bounds__(BLOCK) void k_encoder(int64_t rows, int B, const IN *__restrict__ v,
                                                   const double *__restrict__ tau,
                                                   const typename Act<G>::acc *__restrict__ vec,
                                                   int64_t oW1, int64_t oc1, int64_t oc2,
                                                   const void *__restrict__ w2,
                                                   G *__restrict__ E, const int *__restrict__ skip) {
    if (skip && *skip) return;
    using acc_t = typename Act<G>::acc;
    const acc_t *W1 = vec + oW1, *c1 = vec + oc1, *c2 = vec + oc2;
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    const int64_t r0 = ((int64_t)blockIdx.x * (BLOCK / WAVE) + wv) * 16;
    if constexpr (sizeof(G) == 8) {
        const double *W2 = (const double *)w2;
        const int q = lane % 4;
        const int64_t r = r0 + lane / 4;
        if (r >= rows) return;
        const double u = tau[3 * (r % B) + 1] * (double)v[r];
        double out[D / 4];
#pragma unroll
        for (int e = 0; e < D / 4; ++e) out[e] = 0.0;
        for (int k = 0; k < H; ++k) {
            const double hk = relu(u * W1[k] + c1[k]);
#pragma unroll
            for (int e = 0; e < D / 4; ++e) out[e] += hk * W2[(int64_t)k * D + q * (D / 4) + e];
        }
#pragma unroll
        for (int e = 0; e < D / 4; ++e) out[e] += c2[q * (D / 4) + e];
        store_feats<G, D / 4>(E + r * D + q * (D / 4), out);
    } else {
        __shared__ __attribute__((aligned(16))) G Es[BLOCK / WAVE][16][D + 8];
        const int64_t ra = r0 + lane % 16;
        const float u = ra < rows ? (float)(tau[3 * (ra % B) + 1] * (double)v[ra]) : 0.f;
        f32x4 o[D / 16];
#pragma unroll
        for (int nt = 0; nt < D / 16; ++nt) o[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
        if constexpr (sizeof(G) == 4) {
            const float *pk = (const float *)w2;
#pragma unroll 4
            for (int ks = 0; ks < H / 4; ++ks) {
                const int k = ks * 4 + lane / 16;
                const float a = fmaxf(u * W1[k] + c1[k], 0.f);
#pragma unroll
                for (int nt = 0; nt < D / 16; ++nt)
                    o[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                        a, pk[(ks * (D / 16) + nt) * 64 + lane], o[nt], 0, 0, 0);
            }
        } else {
            const uint16_t *pk = (const uint16_t *)w2;
#pragma unroll
            for (int kb = 0; kb < H / 32; ++kb) {
                uint16_t av[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int k = kb * 32 + 8 * (lane / 16) + i;
                    av[i] = f2bf(fmaxf(u * W1[k] + c1[k], 0.f));
                }
                const bf16x8 af = __builtin_bit_cast(bf16x8, av);
#pragma unroll
                for (int nt = 0; nt < D / 16; ++nt)
                    o[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        af, load_bf16x8(pk + ((int64_t)(kb * (D / 16) + nt) * 64 + lane) * 8),
                        o[nt], 0, 0, 0);
            }
        }
        // stage the 16 x D output tile in LDS, then 16-byte coalesced stores
#pragma unroll
        for (int nt = 0; nt < D / 16; ++nt) {
            const int col = nt * 16 + lane % 16;
            const float cb = c2[col];
#pragma unroll
            for (int j = 0; j < 4; ++j) Es[wv][4 * (lane / 16) + j][col] = Act<G>::put(o[nt][j] + cb);
        }
        wave_lds_sync();
        const int rl = lane / 4, q = lane % 4;
        const int64_t r = r0 + rl;
        if (r < rows) {
            typename Act<G>::acc ov[D / 4];
#pragma unroll
            for (int e = 0; e < D / 4; ++e) ov[e] = Act<G>::get(Es[wv][rl][q * (D / 4) + e]);
            store_feats<G, D / 4>(E + r * D + q * (D / 4), ov);
        }
    }
}

// ---------------------------------------------------------------------------
// Res-GCONV layer (Eq. (5)), fused:  T = A-hat X (CSR gather, 4 lanes per
// row, d/4 features per lane) -> LDS tile [X | T] -> [X | T] [U; W] on MFMA
// -> ReLU -> store.  With DEC the output tile stays in LDS and feeds the
// decoder  o = ReLU(Y W3 + c3) W4 + c4,  z = (tau/sqrt(n)) o  (Eq. (6)).
// ---------------------------------------------------------------------------
template <typename G, int D, int H, bool DEC, typename ZT>
__global__ __launch_bounds__(BLOCK) void k_layer(
    int64_t rows, int B, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const typename Act<G>::vt *__restrict__ ahat, const G *__restrict__ X, G *__restrict__ Y,
    const void *__restrict__ wcat, const void *__restrict__ w3,
    const typename Act<G>::acc *__restrict__ vec, int64_t oc3, int64_t oW4, int64_t oc4,
    const double *__restrict__ tau, ZT *__restrict__ z, const int *__restrict__ skip) {
    if (skip && *skip) return;
    using acc_t = typename Act<G>::acc;
    using mt = typename Act<G>::mt;
    constexpr int LD = 2 * D + lds_pad<G>();
    __shared__ __attribute__((aligned(16))) mt As[BLOCK / WAVE][16][LD];
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    const int64_t r0 = ((int64_t)blockIdx.x * (BLOCK / WAVE) + wv) * 16;

    // ---- stage the tile's slice of the CSR arrays (rows r0 .. r0+15 touch
    // nodes ifirst .. ilast, whose nonzeros are contiguous) in LDS
    using vt_t = typename Act<G>::vt;
    constexpr int CAP = 256;
    __shared__ int32_t sRp[BLOCK / WAVE][17];
    __shared__ int32_t sCi[BLOCK / WAVE][CAP];
    __shared__ vt_t sVa[BLOCK / WAVE][CAP];
    const bool live = r0 < rows;
    const int64_t rlast = (r0 + 15 < rows) ? r0 + 15 : rows - 1;
    const int64_t ifirst = live ? ((B == 1) ? r0 : r0 / B) : 0;
    const int64_t ilast = live ? ((B == 1) ? rlast : rlast / B) : 0;
    const int32_t kbeg = live ? rp[ifirst] : 0;
    const int32_t cnt = live ? rp[ilast + 1] - kbeg : 0;
    const bool staged = cnt <= CAP;
    if (live && lane <= (int)(ilast - ifirst)) sRp[wv][lane] = rp[ifirst + lane] - kbeg;
    if (live && lane == 0) sRp[wv][ilast - ifirst + 1] = cnt;
    if (live && staged) {
        for (int t2 = lane; t2 < cnt; t2 += WAVE) {
            sCi[wv][t2] = ci[kbeg + t2];
            sVa[wv][t2] = ahat[kbeg + t2];
        }
    }
    wave_lds_sync();

    // ---- phase 1: gather T = A-hat X and the row's own X into LDS
    {
        const int rl = lane / 4, q = lane % 4;
        const int64_t r = r0 + rl;
        acc_t t[D / 4], s[D / 4];
#pragma unroll
        for (int e = 0; e < D / 4; ++e) t[e] = s[e] = (acc_t)0;
        if (r < rows) {
            const int64_t i = (B == 1) ? r : r / B;
            const int b = (int)(r - i * B);
            const int li = (int)(i - ifirst);
            const int32_t ks = sRp[wv][li], ke = sRp[wv][li + 1];
            load_feats<G, D / 4>(X + r * D + q * (D / 4), s);
            if (staged) {
                // neighbours in batches of NB: all gathers issued before the FMAs;
                // short rows re-load a valid neighbour with weight 0
                constexpr int NB = sizeof(G) == 2 ? 8 : 4;
                constexpr int CB = (D / 4) * (int)sizeof(G);
                for (int32_t k0 = ks; k0 < ke; k0 += NB) {
                    Chunk<CB> raw[NB];  // packed until the FMAs (register economy)
                    acc_t av[NB];
#pragma unroll
                    for (int u = 0; u < NB; ++u) {
                        const bool ok = k0 + u < ke;
                        const int32_t kk = ok ? k0 + u : ks;
                        const int64_t c = sCi[wv][kk];
                        av[u] = ok ? (acc_t)sVa[wv][kk] : (acc_t)0;
                        raw[u] = *reinterpret_cast<const Chunk<CB> *>(X + (c * B + b) * D +
                                                                      q * (D / 4));
                    }
#pragma unroll
                    for (int u = 0; u < NB; ++u) {
                        const G *e8 = reinterpret_cast<const G *>(&raw[u]);
#pragma unroll
                        for (int e = 0; e < D / 4; ++e) t[e] += av[u] * Act<G>::get(e8[e]);
                    }
                }
            } else {
                for (int32_t k = kbeg + ks; k < kbeg + ke; ++k) {
                    const int64_t c = ci[k];
                    const acc_t a = (acc_t)ahat[k];
                    acc_t xv[D / 4];
                    load_feats<G, D / 4>(X + (c * B + b) * D + q * (D / 4), xv);
#pragma unroll
                    for (int e = 0; e < D / 4; ++e) t[e] += a * xv[e];
                }
            }
        }
#pragma unroll
        for (int e = 0; e < D / 4; ++e) {
            As[wv][rl][q * (D / 4) + e] = Act<G>::put(s[e]);
            As[wv][rl][D + q * (D / 4) + e] = Act<G>::put(t[e]);
        }
    }
    wave_lds_sync();

    if constexpr (sizeof(G) == 8) {
        // ---- FP64 VALU path
        const double *Wc = (const double *)wcat;
        const int rl = lane / 4, q = lane % 4;
        const int64_t r = r0 + rl;
        double y[D / 4];
#pragma unroll
        for (int e = 0; e < D / 4; ++e) {
            const int col = q * (D / 4) + e;
            double sacc = 0.0;
            for (int k = 0; k < 2 * D; ++k) sacc += As[wv][rl][k] * Wc[(int64_t)k * D + col];
            y[e] = relu(sacc);
        }
        if constexpr (!DEC) {
            if (r < rows) store_feats<G, D / 4>(Y + r * D + q * (D / 4), y);
        } else {
            wave_lds_sync();
#pragma unroll
            for (int e = 0; e < D / 4; ++e) As[wv][rl][q * (D / 4) + e] = y[e];
            wave_lds_sync();
            const double *W3 = (const double *)w3;
            const double *c3 = vec + oc3, *W4 = vec + oW4;
            double part = 0.0;
            for (int kk = 0; kk < H / 4; ++kk) {
                const int k = q * (H / 4) + kk;
                double hs = c3[k];
                for (int f = 0; f < D; ++f) hs += As[wv][rl][f] * W3[(int64_t)f * H + k];
                part += relu(hs) * W4[k];
            }
            part += __shfl_xor(part, 1, 4);
            part += __shfl_xor(part, 2, 4);
            if (q == 0 && r < rows) {
                const int b = (int)(r % B);
                z[r] = (ZT)(tau[3 * b + 2] * (part + vec[oc4]));
            }
        }
    } else {
        // ---- MFMA path: [X | T] (16 x 2D) times [U; W] (2D x D)
        f32x4 o[D / 16];
#pragma unroll
        for (int nt = 0; nt < D / 16; ++nt) o[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
        if constexpr (sizeof(G) == 4) {
            const float *pk = (const float *)wcat;
#pragma unroll 8
            for (int ks = 0; ks < 2 * D / 4; ++ks) {
                const float a = As[wv][lane % 16][ks * 4 + lane / 16];
#pragma unroll
                for (int nt = 0; nt < D / 16; ++nt)
                    o[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                        a, pk[(ks * (D / 16) + nt) * 64 + lane], o[nt], 0, 0, 0);
            }
        } else {
            const uint16_t *pk = (const uint16_t *)wcat;
#pragma unroll
            for (int kb = 0; kb < 2 * D / 32; ++kb) {
                const bf16x8 af = load_bf16x8(&As[wv][lane % 16][kb * 32 + 8 * (lane / 16)]);
#pragma unroll
                for (int nt = 0; nt < D / 16; ++nt)
                    o[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        af, load_bf16x8(pk + ((int64_t)(kb * (D / 16) + nt) * 64 + lane) * 8),
                        o[nt], 0, 0, 0);
            }
        }
        if constexpr (!DEC) {
            wave_lds_sync();  // every lane has read its A fragments
#pragma unroll
            for (int nt = 0; nt < D / 16; ++nt) {
                const int col = nt * 16 + lane % 16;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    As[wv][4 * (lane / 16) + j][col] = Act<G>::put(relu(o[nt][j]));
            }
            wave_lds_sync();
            const int rl = lane / 4, q = lane % 4;
            const int64_t r = r0 + rl;
            if (r < rows) {
                acc_t ov[D / 4];
#pragma unroll
                for (int e = 0; e < D / 4; ++e) ov[e] = Act<G>::get(As[wv][rl][q * (D / 4) + e]);
                store_feats<G, D / 4>(Y + r * D + q * (D / 4), ov);
            }
        } else {
            wave_lds_sync();
            constexpr int KP = (sizeof(G) == 2) ? ((D + 31) / 32) * 32 : D;
#pragma unroll
            for (int nt = 0; nt < D / 16; ++nt) {
                const int col = nt * 16 + lane % 16;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    As[wv][4 * (lane / 16) + j][col] = Act<G>::put(relu(o[nt][j]));
                    if constexpr (KP > D) As[wv][4 * (lane / 16) + j][D + col] = Act<G>::put(0.f);
                }
            }
            wave_lds_sync();
            f32x4 hacc[H / 16];
#pragma unroll
            for (int nt = 0; nt < H / 16; ++nt) hacc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
            if constexpr (sizeof(G) == 4) {
                const float *pk = (const float *)w3;
#pragma unroll 4
                for (int ks = 0; ks < D / 4; ++ks) {
                    const float a = As[wv][lane % 16][ks * 4 + lane / 16];
#pragma unroll
                    for (int nt = 0; nt < H / 16; ++nt)
                        hacc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            a, pk[(ks * (H / 16) + nt) * 64 + lane], hacc[nt], 0, 0, 0);
                }
            } else {
                const uint16_t *pk = (const uint16_t *)w3;
#pragma unroll
                for (int kb = 0; kb < KP / 32; ++kb) {
                    const bf16x8 af = load_bf16x8(&As[wv][lane % 16][kb * 32 + 8 * (lane / 16)]);
#pragma unroll
                    for (int nt = 0; nt < H / 16; ++nt)
                        hacc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            af, load_bf16x8(pk + ((int64_t)(kb * (H / 16) + nt) * 64 + lane) * 8),
                            hacc[nt], 0, 0, 0);
                }
            }
            const float *c3 = vec + oc3, *W4 = vec + oW4;
            float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int nt = 0; nt < H / 16; ++nt) {
                const int col = nt * 16 + lane % 16;
                const float cb = c3[col], w4 = W4[col];
#pragma unroll
                for (int j = 0; j < 4; ++j) part[j] += fmaxf(hacc[nt][j] + cb, 0.f) * w4;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
#pragma unroll
                for (int off = 8; off > 0; off >>= 1) part[j] += __shfl_xor(part[j], off, 16);
            }
            if (lane % 16 == 0) {
                const float c4 = vec[oc4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int64_t r = r0 + 4 * (lane / 16) + j;
                    if (r < rows) z[r] = (ZT)(tau[3 * (r % B) + 2] * (double)(part[j] + c4));
                }
            }
        }
    }
}

}  // namespace gnp
