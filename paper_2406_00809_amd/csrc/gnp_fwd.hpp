// Forward kernels of the graph neural preconditioner (Sec. 2.3).
//
// Rows of the activation matrices are (node, right-hand side) pairs,
// r = i * nrhs + k, node-major, with d features per row.  Kernels run
// 256-thread blocks of four wavefronts; a wavefront works on tiles of 16
// consecutive rows.
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
// The products are formed transposed, Y^T = W^T X^T: the packed weight
// fragments are the A operand and the activation tile the B operand, so a
// lane's four results are four consecutive features (4 (l/16) + j) of one row
// (l % 16) and leave as a single 8- or 16-byte store.
#pragma once
#include <type_traits>

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
    static __device__ __forceinline__ double wf(double a) { return a; }
};
template <> struct Act<float> {
    using acc = float;
    using mt = float;
    using vt = float;
    static __device__ __forceinline__ float get(float v) { return v; }
    static __device__ __forceinline__ float put(float v) { return v; }
    static __device__ __forceinline__ float wf(float a) { return a; }
};
template <> struct Act<uint16_t> {
    using acc = float;
    using mt = uint16_t;
    using vt = uint16_t;  // A-hat stored in bfloat16 as well
    static __device__ __forceinline__ float get(uint16_t v) { return bf2f(v); }
    static __device__ __forceinline__ uint16_t put(float v) { return f2bf(v); }
    static __device__ __forceinline__ float wf(uint16_t a) { return bf2f(a); }
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

// Store four consecutive features held by one lane.
template <typename G> __device__ __forceinline__ void store4(G *p, float a, float b, float c, float d);
template <>
__device__ __forceinline__ void store4<float>(float *p, float a, float b, float c, float d) {
    *reinterpret_cast<float4 *>(p) = make_float4(a, b, c, d);
}
template <>
__device__ __forceinline__ void store4<uint16_t>(uint16_t *p, float a, float b, float c, float d) {
    uint2 u;
    u.x = (uint32_t)f2bf(a) | ((uint32_t)f2bf(b) << 16);
    u.y = (uint32_t)f2bf(c) | ((uint32_t)f2bf(d) << 16);
    *reinterpret_cast<uint2 *>(p) = u;
}

template <typename T> __device__ __forceinline__ T relu(T x) { return x > (T)0 ? x : (T)0; }

// ReLU of two features rounded to bf16 (RNE) and packed: the rounding keeps
// the sign, so clearing negative halves of the rounded pair equals rounding
// the ReLU (a NaN keeps or loses its value with its sign bit).
__device__ __forceinline__ uint32_t relu_pk_bf16(float a, float b) {
    typedef __bf16 bf16v2 __attribute__((ext_vector_type(2)));
    typedef float f32v2 __attribute__((ext_vector_type(2)));
    typedef short i16v2 __attribute__((ext_vector_type(2)));
    const bf16v2 h = __builtin_convertvector((f32v2){a, b}, bf16v2);
    const i16v2 z = {0, 0};
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(i16v2, h), z));
}

// Buffer resource over `bytes` bytes at p (raw, stride 0): a load whose
// offset lies past `bytes` returns zeros instead of touching memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, (int)bytes, 0x00020000);
}
constexpr uint32_t BUF_OOB = 0xFFFFFFF0u;  // an offset past any buffer here (< 2^32 - 16 bytes)

template <int BYTES>
__device__ __forceinline__ Chunk<BYTES> buffer_chunk(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    if constexpr (BYTES == 16)
        return __builtin_bit_cast(Chunk<16>, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    else if constexpr (BYTES == 8)
        return __builtin_bit_cast(Chunk<8>, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    else {
        static_assert(BYTES == 4, "chunk of 4, 8 or 16 bytes");
        return __builtin_bit_cast(Chunk<4>, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    }
}

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
// The hidden activations of row l % 16 are built in registers as the B
// operand of E^T = W2^T hid^T.
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
                        pk[(ks * (D / 16) + nt) * 64 + lane], a, o[nt], 0, 0, 0);
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
                const bf16x8 hf = __builtin_bit_cast(bf16x8, av);
#pragma unroll
                for (int nt = 0; nt < D / 16; ++nt)
                    o[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        load_bf16x8(pk + ((int64_t)(kb * (D / 16) + nt) * 64 + lane) * 8), hf,
                        o[nt], 0, 0, 0);
            }
        }
        if (ra < rows) {
#pragma unroll
            for (int nt = 0; nt < D / 16; ++nt) {
                const int f = nt * 16 + 4 * (lane / 16);
                store4<G>(E + ra * D + f, o[nt][0] + c2[f], o[nt][1] + c2[f + 1],
                          o[nt][2] + c2[f + 2], o[nt][3] + c2[f + 3]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Persistent encoder for the MFMA paths (float32 / bfloat16 activations):
// the weights a lane needs are loaded once, and the input of the next tile
// is requested before the current one is computed.  With bn.hdiv (one
// right-hand side, inside the solver) the input is the solver's vector w and
// the network input is the next basis vector formed here (BasisNext): with
// bn.V, w - V[:, 0..j] h first, in the solver's correction arithmetic (8
// lanes per row, lane q owning columns 4q..4q+3, FP64 products summed in
// column order, then across the 8 lanes by xor 1, 2, 4), then the division
// by *hdiv.  v is written to bn.vout and, with bn.Vout, into column j + 1 of
// the basis (the lane holding that column stores its four columns whole); its
// tau of Eq. (6) is 1 (v has unit
// norm), and block 0 publishes that triple for the decoder.
// ---------------------------------------------------------------------------
template <typename G, typename IN, int D, int H>
__global__ __launch_bounds__(BLOCK) void k_encoder_p(
    int64_t rows, int B, const IN *__restrict__ v, double *__restrict__ tau,
    const float *__restrict__ vec, int64_t oW1, int64_t oc1, int64_t oc2,
    const void *__restrict__ w2, G *__restrict__ E, const int *__restrict__ skip,
    BasisNext bn, int64_t n) {
    static_assert(sizeof(G) <= 4, "MFMA encoder");
    // the skip flag is tested after the weights are loaded (overlapped)
    const int skipped = skip ? *skip : 0;
    const double *hdiv = bn.hdiv;
    const bool corr = hdiv && bn.V;  // the second Gram-Schmidt correction here
    const int lane = threadIdx.x % WAVE;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const float *W1 = vec + oW1, *c1 = vec + oc1, *c2 = vec + oc2;
    // hidden-unit weights in the layout of the MFMA B operand, output bias in
    // the result layout, W2 fragments as the A operand
    constexpr int KG = sizeof(G) == 2 ? H / 32 : H / 4;  // k groups
    constexpr int KE = sizeof(G) == 2 ? 8 : 1;           // k per group per lane
    float w1r[KG][KE], c1r[KG][KE], c2r[D / 16][4];
#pragma unroll
    for (int g = 0; g < KG; ++g)
#pragma unroll
        for (int i = 0; i < KE; ++i) {
            const int k = sizeof(G) == 2 ? g * 32 + 8 * (lane / 16) + i : g * 4 + lane / 16;
            w1r[g][i] = W1[k];
            c1r[g][i] = c1[k];
        }
#pragma unroll
    for (int nt = 0; nt < D / 16; ++nt)
#pragma unroll
        for (int j = 0; j < 4; ++j) c2r[nt][j] = c2[nt * 16 + 4 * (lane / 16) + j];
    using Frag = typename std::conditional<sizeof(G) == 2, bf16x8, float>::type;
    Frag pk[KG][D / 16];
#pragma unroll
    for (int g = 0; g < KG; ++g)
#pragma unroll
        for (int nt = 0; nt < D / 16; ++nt) {
            if constexpr (sizeof(G) == 2)
                pk[g][nt] = load_bf16x8((const uint16_t *)w2 +
                                        ((int64_t)(g * (D / 16) + nt) * 64 + lane) * 8);
            else
                pk[g][nt] = ((const float *)w2)[(g * (D / 16) + nt) * 64 + lane];
        }
    const int64_t ntiles = (rows + 15) / 16, nw = (int64_t)gridDim.x * (BLOCK / WAVE);
    int64_t t = (int64_t)blockIdx.x * (BLOCK / WAVE) + wv;
    IN vn = v[t * 16 + lane % 16 < rows ? t * 16 + lane % 16 : rows - 1];
    // with the correction: rows t*16 + 8 rho + lane/8 (rho = 0, 1), lane
    // q = lane % 8 holding basis columns 4q..4q+3 of its row and the row's w;
    // columns past j are masked below (they may hold an older cycle)
    const int cq = lane % 8;
    double hc[4];
    float4 vq[2];
    float wq[2];
    auto load_corr = [&](int64_t tt) {
#pragma unroll
        for (int rho = 0; rho < 2; ++rho) {
            const int64_t r = tt * 16 + 8 * rho + lane / 8;
            const int64_t rc = r < rows ? r : rows - 1;
            vq[rho] = *reinterpret_cast<const float4 *>(bn.V + rc * 32 + 4 * cq);
            wq[rho] = (float)v[rc];
        }
    };
    __shared__ float s_vb[BLOCK / WAVE][16];  // the tile's basis values, by row
    if (corr) {
#pragma unroll
        for (int a = 0; a < 4; ++a) hc[a] = 4 * cq + a <= bn.j ? bn.h[4 * cq + a] : 0.0;
        load_corr(t);
    }
    // without hdiv: sqrt(n)/tau of every right-hand side (B <= 256) staged in
    // LDS once, so the tile loop waits on no global load but its input
    // prefetch
    __shared__ double s_tau1[BLOCK];
    double tau1 = 0.0, div = 1.0;  // with hdiv: sqrt(n) / 1 and the divisor
    if (!hdiv) {
        for (int b = threadIdx.x; b < B; b += BLOCK) s_tau1[b] = tau[3 * b + 1];
        __syncthreads();
    } else {
        const double sqn = sqrt((double)n), tv = 1.0;
        tau1 = sqn / tv;
        div = *hdiv;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            tau[0] = tv;
            tau[1] = tau1;
            tau[2] = tv / sqn;
        }
    }
    // the flag is tested once the first tile's loads (input, correction rows
    // and coefficients, divisor) are in flight: all in range, unused if set
    if (skipped) return;
    for (; t < ntiles; t += nw) {
        const int64_t ra = t * 16 + lane % 16;
        IN vc;
        if (corr) {
            // w - V h for rows 8 rho + lane/8, then / h_{j+1,j}; exchanged
            // through LDS into the row-per-lane layout of the network
#pragma unroll
            for (int rho = 0; rho < 2; ++rho) {
                const float qv[4] = {vq[rho].x, vq[rho].y, vq[rho].z, vq[rho].w};
                double c = 0.0;
#pragma unroll
                for (int a = 0; a < 4; ++a)
                    c += hc[a] * (4 * cq + a <= bn.j ? (double)qv[a] : 0.0);
                c += __shfl_xor(c, 1, WAVE);
                c += __shfl_xor(c, 2, WAVE);
                c += __shfl_xor(c, 4, WAVE);
                const IN wn = (IN)((double)wq[rho] - c);
                const IN vb = (IN)((double)wn / div);
                const int64_t r = t * 16 + 8 * rho + lane / 8;
                if (cq == 0) {
                    s_vb[wv][8 * rho + lane / 8] = vb;
                    if (bn.vout && r < rows) bn.vout[r] = vb;
                }
                // the basis column j + 1: the lane holding it writes its four
                // columns back whole (one 16-byte store; the columns past
                // j + 1 keep what they held)
                if (bn.Vout && cq == ((bn.j + 1) >> 2) && r < rows) {
                    float4 nv = vq[rho];
                    const int e = (bn.j + 1) & 3;
                    nv.x = e == 0 ? (float)vb : nv.x;
                    nv.y = e == 1 ? (float)vb : nv.y;
                    nv.z = e == 2 ? (float)vb : nv.z;
                    nv.w = e == 3 ? (float)vb : nv.w;
                    *reinterpret_cast<float4 *>(bn.Vout + r * 32 + 4 * cq) = nv;
                }
            }
            load_corr(t + nw);  // the next tile's rows (clamped past the end)
            wave_lds_sync();
            vc = s_vb[wv][lane % 16];
            wave_lds_sync();  // read before the next tile's writes
        } else {
            // with hdiv: the basis vector, as the solver's normalisation forms it
            vc = hdiv ? (IN)((double)vn / div) : vn;
            if (hdiv && bn.vout && lane < 16 && ra < rows) bn.vout[ra] = vc;
        }
        // this tile's scale first, then the next tile's input: waiting for
        // the scale leaves the prefetch in flight
        const double ts = hdiv ? tau1 : s_tau1[(uint32_t)ra % (uint32_t)B];
        const int64_t rn = (t + nw) * 16 + lane % 16;
        vn = v[rn < rows ? rn : rows - 1];  // next tile's input, clamped
        const float u = ra < rows ? (float)(ts * (double)vc) : 0.f;
        f32x4 o[D / 16];
#pragma unroll
        for (int nt = 0; nt < D / 16; ++nt) o[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int g = 0; g < KG; ++g) {
            if constexpr (sizeof(G) == 2) {
                uint16_t av[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) av[i] = f2bf(fmaxf(u * w1r[g][i] + c1r[g][i], 0.f));
                const bf16x8 hf = __builtin_bit_cast(bf16x8, av);
#pragma unroll
                for (int nt = 0; nt < D / 16; ++nt)
                    o[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pk[g][nt], hf, o[nt], 0, 0, 0);
            } else {
                const float a = fmaxf(u * w1r[g][0] + c1r[g][0], 0.f);
#pragma unroll
                for (int nt = 0; nt < D / 16; ++nt)
                    o[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(pk[g][nt], a, o[nt], 0, 0, 0);
            }
        }
        if (ra < rows) {
#pragma unroll
            for (int nt = 0; nt < D / 16; ++nt)
                store4<G>(E + ra * D + nt * 16 + 4 * (lane / 16), o[nt][0] + c2r[nt][0],
                          o[nt][1] + c2r[nt][1], o[nt][2] + c2r[nt][2], o[nt][3] + c2r[nt][3]);
        }
    }
}

// Blocks of a kernel that fit on the device at once (occupancy x CUs).
template <auto K> inline int resident_blocks() {
    static const int resident = [] {  // initialised once, thread-safe
        int dev = 0, cus = 0, per_cu = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, K, BLOCK, 0);
        return (cus > 0 ? cus : 256) * (per_cu > 0 ? per_cu : 1);
    }();
    return resident;
}

// ---------------------------------------------------------------------------
// Res-GCONV layer (Eq. (5)), fused:  T = A-hat X (CSR gather, 4 lanes per
// row, d/4 features per lane) -> LDS tile [X | T] -> [X | T] [U; W] on MFMA
// -> ReLU -> store.  With DEC the output tile stays in LDS and feeds the
// decoder  o = ReLU(Y W3 + c3) W4 + c4,  z = (tau/sqrt(n)) o  (Eq. (6)).
//
// Persistent, software-pipelined walk over 16-row tiles (XCD-aware order,
// see xcd_walk).  Tile t touches nodes ifirst..ilast whose nonzeros
// are contiguous in CSR; that slice (colind, values, rowptr offsets) is
// staged in the wavefront's LDS.  The rowptr slice of the next tile is
// requested before the gathers of the current one, and its colind / value
// slice (into registers) before the current tile's MFMA and stores.
// Gather offsets are 32-bit (the launchers check rows * d < 2^31).
// ---------------------------------------------------------------------------
template <typename G, int D, int H, bool DEC, typename ZT>
__device__ __forceinline__ void layer_tiles(
    int64_t rows, int B, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const typename Act<G>::vt *__restrict__ ahat, const G *__restrict__ X, G *__restrict__ Y,
    const void *__restrict__ wcat, const void *__restrict__ w3,
    const typename Act<G>::acc *__restrict__ vec, int64_t oc3, int64_t oW4, int64_t oc4,
    const double *__restrict__ tau, ZT *__restrict__ z, const int *__restrict__ skip) {
    if (skip && *skip) return;
    using acc_t = typename Act<G>::acc;
    using mt = typename Act<G>::mt;
    using vt_t = typename Act<G>::vt;
    constexpr int LD = 2 * D + lds_pad<G>();
    constexpr int CAP = 256, NC = CAP / WAVE;
    __shared__ __attribute__((aligned(16))) mt As[BLOCK / WAVE][16][LD];
    __shared__ int32_t sRp[BLOCK / WAVE][17];
    __shared__ uint32_t sCo[BLOCK / WAVE][CAP];  // byte offset of row (column, rhs 0) in X
    __shared__ vt_t sVa[BLOCK / WAVE][CAP];
    // the wavefront index is uniform: keep it (and the whole tile walk, the
    // rowptr slice and the CSR slice bounds) in scalar registers
    const int lane = threadIdx.x % WAVE;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const TileWalk walk = xcd_walk((rows + 15) / 16, BLOCK / WAVE, wv);
    const int64_t ntiles = walk.end, nw = walk.stride;
    const uint32_t rowbytes = (uint32_t)B * (uint32_t)(D * sizeof(G));

    auto node_range = [&](int64_t t, int64_t &ifirst, int &nn) {
        const int64_t r0 = t * 16;
        const int64_t rlast = (r0 + 15 < rows) ? r0 + 15 : rows - 1;
        ifirst = (B == 1) ? r0 : r0 / B;
        nn = (int)(((B == 1) ? rlast : rlast / B) - ifirst) + 1;
    };
    auto fetch_rp = [&](int64_t t, int32_t &rpv) {
        int64_t ifirst;
        int nn;
        node_range(t, ifirst, nn);
        rpv = lane <= nn ? rp[ifirst + lane] : 0;
    };
    auto fetch_csr = [&](int64_t t, int32_t rpv, int32_t &kbeg, int32_t &cnt, int32_t (&cv)[NC],
                         vt_t (&av)[NC]) {
        int64_t ifirst;
        int nn;
        node_range(t, ifirst, nn);
        kbeg = __builtin_amdgcn_readfirstlane(rpv);
        cnt = __builtin_amdgcn_readlane(rpv, nn) - kbeg;
        if (cnt > 0 && cnt <= CAP) {  // cnt = 0: empty rows, nothing to load
#pragma unroll
            for (int u = 0; u < NC; ++u) {
                const int idx = lane + WAVE * u;
                const int idc = idx < cnt ? idx : 0;
                cv[u] = ci[kbeg + idc];
                av[u] = ahat[kbeg + idc];
            }
        }
    };

    int64_t t = walk.t;
    int32_t rpv = 0, kbeg = 0, cnt = 0;
    int32_t cv[NC];
    vt_t av[NC];
    if (t < ntiles) {
        fetch_rp(t, rpv);
        fetch_csr(t, rpv, kbeg, cnt, cv, av);
    }
    for (; t < ntiles; t += nw) {
        const int64_t r0 = t * 16;
        int64_t ifirst;
        int nn;
        node_range(t, ifirst, nn);
        const bool staged = cnt <= CAP;
        // ---- commit this tile's CSR slice to LDS
        if (lane <= nn) sRp[wv][lane] = rpv - kbeg;
        if (staged) {
#pragma unroll
            for (int u = 0; u < NC; ++u) {
                const int idx = lane + WAVE * u;
                if (idx < cnt) {
                    sCo[wv][idx] = (uint32_t)cv[u] * rowbytes;
                    sVa[wv][idx] = av[u];
                }
            }
        }
        const int64_t tn = t + nw;
        int32_t rpn = 0;
        if (tn < ntiles) fetch_rp(tn, rpn);
        wave_lds_sync();

        // ---- phase 1: gather T = A-hat X and the row's own X into the LDS tile
        {
            const int rl = lane / 4, q = lane % 4;
            const int64_t r = r0 + rl;
            acc_t ta[D / 4], sv[D / 4];
#pragma unroll
            for (int e = 0; e < D / 4; ++e) ta[e] = sv[e] = (acc_t)0;
            if (r < rows) {
                const int64_t i = (B == 1) ? r : r / B;
                const int b = (int)(r - i * B);
                const int li = (int)(i - ifirst);
                const int32_t ks = sRp[wv][li], ke = sRp[wv][li + 1];
                load_feats<G, D / 4>(X + r * D + q * (D / 4), sv);
                if (staged) {
                    // neighbours in batches of NB, kept packed until the FMAs;
                    // short rows re-load a valid neighbour with weight 0.
                    // Byte offsets from the uniform base (the launchers keep
                    // the activation block below 4 GiB).
                    constexpr int NB = sizeof(G) == 2 ? 8 : 4;
                    constexpr int CB = (D / 4) * (int)sizeof(G);
                    const uint32_t lane_off =
                        ((uint32_t)b * D + (uint32_t)(q * (D / 4))) * (uint32_t)sizeof(G);
                    const char *Xb = reinterpret_cast<const char *>(X);
                    for (int32_t k0 = ks; k0 < ke; k0 += NB) {
                        Chunk<CB> raw[NB];
                        vt_t wgt[NB];
#pragma unroll
                        for (int u = 0; u < NB; ++u) {
                            const bool ok = k0 + u < ke;
                            const int32_t kk = ok ? k0 + u : ks;
                            wgt[u] = ok ? sVa[wv][kk] : (vt_t)0;
                            raw[u] = *reinterpret_cast<const Chunk<CB> *>(Xb + sCo[wv][kk] +
                                                                          lane_off);
                        }
                        if constexpr (sizeof(G) == 2) {
                            // bf16 pairs times packed weights (a, 0) and (0, a):
                            // one v_dot2 per element, no unpacking
#pragma unroll
                            for (int u = 0; u < NB; ++u) {
                                const uint32_t wlo = (uint32_t)wgt[u], whi = wlo << 16;
#pragma unroll
                                for (int j = 0; j < CB / 4; ++j) {
                                    const bf16x2 xv = __builtin_bit_cast(bf16x2, raw[u].w[j]);
                                    ta[2 * j] = __builtin_amdgcn_fdot2_f32_bf16(
                                        xv, __builtin_bit_cast(bf16x2, wlo), ta[2 * j], false);
                                    ta[2 * j + 1] = __builtin_amdgcn_fdot2_f32_bf16(
                                        xv, __builtin_bit_cast(bf16x2, whi), ta[2 * j + 1], false);
                                }
                            }
                        } else {
#pragma unroll
                            for (int u = 0; u < NB; ++u) {
                                const G *e8 = reinterpret_cast<const G *>(&raw[u]);
#pragma unroll
                                for (int e = 0; e < D / 4; ++e)
                                    ta[e] += Act<G>::wf(wgt[u]) * Act<G>::get(e8[e]);
                            }
                        }
                    }
                } else {
                    // (the same per-neighbour arithmetic as the staged path,
                    // so that a row's result does not depend on its tile)
                    for (int32_t k = kbeg + ks; k < kbeg + ke; ++k) {
                        const uint32_t c = (uint32_t)ci[k];
                        const G *xr =
                            X + (c * (uint32_t)B + (uint32_t)b) * (uint32_t)D + q * (D / 4);
                        if constexpr (sizeof(G) == 2) {
                            constexpr int CB = (D / 4) * (int)sizeof(G);
                            const Chunk<CB> raw = *reinterpret_cast<const Chunk<CB> *>(xr);
                            const uint32_t wlo = (uint32_t)ahat[k], whi = wlo << 16;
#pragma unroll
                            for (int j = 0; j < CB / 4; ++j) {
                                const bf16x2 xv = __builtin_bit_cast(bf16x2, raw.w[j]);
                                ta[2 * j] = __builtin_amdgcn_fdot2_f32_bf16(
                                    xv, __builtin_bit_cast(bf16x2, wlo), ta[2 * j], false);
                                ta[2 * j + 1] = __builtin_amdgcn_fdot2_f32_bf16(
                                    xv, __builtin_bit_cast(bf16x2, whi), ta[2 * j + 1], false);
                            }
                        } else {
                            const acc_t a = Act<G>::wf(ahat[k]);
                            acc_t xv[D / 4];
                            load_feats<G, D / 4>(xr, xv);
#pragma unroll
                            for (int e = 0; e < D / 4; ++e) ta[e] += a * xv[e];
                        }
                    }
                }
            }
            store_feats<mt, D / 4>(&As[wv][rl][q * (D / 4)], sv);
            store_feats<mt, D / 4>(&As[wv][rl][D + q * (D / 4)], ta);
        }
        // ---- prefetch the next tile's colind / value slice into registers
        int32_t kbeg_n = 0, cnt_n = 0;
        int32_t cv_n[NC];
        vt_t av_n[NC];
        if (tn < ntiles) fetch_csr(tn, rpn, kbeg_n, cnt_n, cv_n, av_n);
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
            // ---- MFMA path: Y^T = [U; W]^T [X | T]^T, lane gets row l % 16
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
                            pk[(ks * (D / 16) + nt) * 64 + lane], a, o[nt], 0, 0, 0);
                }
            } else {
                const uint16_t *pk = (const uint16_t *)wcat;
#pragma unroll
                for (int kb = 0; kb < 2 * D / 32; ++kb) {
                    const bf16x8 xf = load_bf16x8(&As[wv][lane % 16][kb * 32 + 8 * (lane / 16)]);
#pragma unroll
                    for (int nt = 0; nt < D / 16; ++nt)
                        o[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            load_bf16x8(pk + ((int64_t)(kb * (D / 16) + nt) * 64 + lane) * 8), xf,
                            o[nt], 0, 0, 0);
                }
            }
            const int64_t r = r0 + lane % 16;
            if constexpr (!DEC) {
                if (r < rows) {
#pragma unroll
                    for (int nt = 0; nt < D / 16; ++nt)
                        store4<G>(Y + r * D + nt * 16 + 4 * (lane / 16), relu(o[nt][0]),
                                  relu(o[nt][1]), relu(o[nt][2]), relu(o[nt][3]));
                }
            } else {
                // ---- decoder on the tile: Y -> LDS (row-major, K padded to
                // KP with zeros), hidden^T = W3^T Y^T, then ReLU(. + c3) W4
                constexpr int KP = (sizeof(G) == 2) ? ((D + 31) / 32) * 32 : D;
                wave_lds_sync();  // every lane has read its tile fragments
#pragma unroll
                for (int nt = 0; nt < D / 16; ++nt) {
                    const int f = nt * 16 + 4 * (lane / 16);
                    store4<mt>(&As[wv][lane % 16][f], relu(o[nt][0]), relu(o[nt][1]),
                               relu(o[nt][2]), relu(o[nt][3]));
                    if constexpr (KP > D) store4<mt>(&As[wv][lane % 16][D + f], 0.f, 0.f, 0.f, 0.f);
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
                                pk[(ks * (H / 16) + nt) * 64 + lane], a, hacc[nt], 0, 0, 0);
                    }
                } else {
                    const uint16_t *pk = (const uint16_t *)w3;
#pragma unroll
                    for (int kb = 0; kb < KP / 32; ++kb) {
                        const bf16x8 yf = load_bf16x8(&As[wv][lane % 16][kb * 32 + 8 * (lane / 16)]);
#pragma unroll
                        for (int nt = 0; nt < H / 16; ++nt)
                            hacc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                load_bf16x8(pk + ((int64_t)(kb * (H / 16) + nt) * 64 + lane) * 8),
                                yf, hacc[nt], 0, 0, 0);
                    }
                }
                // lane holds hidden units nt*16 + 4 (l/16) + j of row l % 16
                const float *c3 = vec + oc3, *W4 = vec + oW4;
                float part = 0.f;
#pragma unroll
                for (int nt = 0; nt < H / 16; ++nt) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int k = nt * 16 + 4 * (lane / 16) + j;
                        part += fmaxf(hacc[nt][j] + c3[k], 0.f) * W4[k];
                    }
                }
                part += __shfl_xor(part, 16, WAVE);
                part += __shfl_xor(part, 32, WAVE);
                if (lane < 16 && r < rows)
                    z[r] = (ZT)(tau[3 * (r % B) + 2] * (double)(part + vec[oc4]));
            }
        }
        // ---- rotate the prefetched CSR state; every lane is done with this
        // tile's LDS before the next commit
        wave_lds_sync();
        rpv = rpn;
        kbeg = kbeg_n;
        cnt = cnt_n;
#pragma unroll
        for (int u = 0; u < NC; ++u) {
            cv[u] = cv_n[u];
            av[u] = av_n[u];
        }
    }
}

// ---------------------------------------------------------------------------
// BF16 Res-GCONV layer (Eq. (5)) without the decoder, pipelined so that a tile
// costs one memory round trip: while tile t is gathered, the colind / value
// slice of tile t + nw and the rowptr slice of tile t + 2 nw are already in
// flight (issued just before the gather, so that the single wait for the
// gather covers them too), and the tile's own CSR slice was fetched during the
// previous tile.  All loads are unconditional (clamped addresses, results
// unused when out of range), so the compiler can count them.  The rowptr
// slice stays in registers (cross-lane reads), the MFMA weight fragments are
// staged in LDS once per block.  With DEC the layer is the last one and the
// decoder follows on the tile: z = tau_2 (ReLU(Y W3 + c3) W4 + c4), Eq. (6).
// ---------------------------------------------------------------------------
template <int D, int H, bool DEC, bool B1, bool SHORT, typename ZT>
__device__ __forceinline__ void layer_tiles_bf16(
    int64_t rows, int B, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const uint16_t *__restrict__ ahat, const uint16_t *__restrict__ X, uint16_t *__restrict__ Y,
    const void *__restrict__ wcat, const void *__restrict__ w3, const float *__restrict__ vec,
    int64_t oc3, int64_t oW4, int64_t oc4, const double *__restrict__ tau, ZT *__restrict__ z,
    const int *__restrict__ skip) {
    // the skip flag (end of a solver cycle) is tested after the weights are
    // staged, so that its load overlaps theirs
    const int skipped = skip ? *skip : 0;
    using G = uint16_t;
    constexpr int LD = 2 * D + lds_pad<G>();
    // SHORT (every row has at most 7 entries): 7 neighbour slots per batch
    // and a 128-entry CSR slice (16 rows x 7 fit); otherwise 8 and 256
    constexpr int CAP = SHORT ? 128 : 256, NC = CAP / WAVE;
    constexpr int KB = 2 * D / 32, NT = D / 16;  // MFMA k-blocks and n-tiles
    constexpr int CB = (D / 4) * (int)sizeof(G);  // bytes per lane per row
    constexpr int NB = SHORT ? 7 : 8;             // neighbour loads per batch
    constexpr int KP = ((D + 31) / 32) * 32;      // decoder K, zero-padded
    constexpr int NW3 = DEC ? (KP / 32) * (H / 16) * WAVE : 1;  // W3 fragments (x 8 bf16)
    __shared__ __attribute__((aligned(16))) G As[BLOCK / WAVE][16][LD];
    __shared__ uint32_t sCo[BLOCK / WAVE][CAP];  // byte offset of row (column, rhs 0) in X
    __shared__ uint16_t sVa[BLOCK / WAVE][CAP];
    __shared__ __attribute__((aligned(16))) uint16_t sW[KB * NT * WAVE * 8];
    __shared__ __attribute__((aligned(16))) uint16_t sW3[NW3 * 8];
    __shared__ __attribute__((aligned(16))) float sC3[DEC ? H : 4], sW4[DEC ? H : 4];
    const int lane = threadIdx.x % WAVE;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const TileWalk walk = xcd_walk((rows + 15) / 16, BLOCK / WAVE, wv, B1);
    const int64_t ntiles = walk.end, nw = walk.stride;
    const uint32_t rowbytes = (uint32_t)B * (uint32_t)(D * sizeof(G));
    const int rshift = (rowbytes & (rowbytes - 1)) == 0 ? __builtin_ctz(rowbytes) : -1;
    // X holds rows * D features (< 2^32 bytes)
    const __amdgpu_buffer_rsrc_t xr = buffer_rsrc(X, (uint32_t)rows * (uint32_t)(D * sizeof(G)));

    // nodes of tile t (clamped to the last tile, so that a wave past the end
    // loads valid addresses whose results it never uses); row indices fit in
    // 32 bits because rows * D * sizeof(G) < 2^32
    auto node_range = [&](int64_t t, uint32_t &ifirst, int &nn) {
        const uint32_t tt = (uint32_t)(t < ntiles ? t : ntiles - 1);
        const uint32_t r0 = tt * 16u;
        const uint32_t rlast = r0 + 15u < (uint32_t)rows ? r0 + 15u : (uint32_t)rows - 1u;
        // B1: one right-hand side, rows are nodes (no division)
        ifirst = B1 ? r0 : r0 / (uint32_t)B;
        nn = (int)((B1 ? rlast : rlast / (uint32_t)B) - ifirst) + 1;
    };
    auto fetch_rp = [&](int64_t t) -> int32_t {
        uint32_t ifirst;
        int nn;
        node_range(t, ifirst, nn);
        return rp[ifirst + (uint32_t)(lane <= nn ? lane : nn)];
    };
    // the row pointers of the wavefront's first two tiles go out before the
    // weights are staged, so that the two round trips overlap
    const int32_t rp_first = fetch_rp(walk.t), rp_second = fetch_rp(walk.t + nw);
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(wcat);
        for (int e = threadIdx.x; e < KB * NT * WAVE; e += BLOCK)
            reinterpret_cast<uint4 *>(sW)[e] = src[e];
        if constexpr (DEC) {
            const uint4 *src3 = reinterpret_cast<const uint4 *>(w3);
            for (int e = threadIdx.x; e < NW3; e += BLOCK) reinterpret_cast<uint4 *>(sW3)[e] = src3[e];
            for (int e = threadIdx.x; e < H; e += BLOCK) {
                sC3[e] = vec[oc3 + e];
                sW4[e] = vec[oW4 + e];
            }
        }
        __syncthreads();
    }
    if (skipped) return;
    // colind / value slice of tile t (rowptr slice rpv) into registers; lanes
    // past the slice re-read its last entry (an empty slice reads the entry
    // before it, or entry 0: nnz >= 1)
    // entry range [kbeg, kbeg + cnt) of tile t from its rowptr slice rpv
    // (wave-uniform results)
    auto slice_range = [&](int64_t t, int32_t rpv, int32_t &kbeg, int32_t &cnt) {
        uint32_t ifirst;
        int nn;
        node_range(t, ifirst, nn);
        kbeg = __builtin_amdgcn_readfirstlane(rpv);
        cnt = __builtin_amdgcn_readlane(rpv, nn) - kbeg;
    };
    // colind / value slice [kbeg, kbeg + cnt) into registers; lanes past the
    // slice re-read its last entry (an empty slice reads the entry before
    // it, or entry 0: nnz >= 1)
    auto fetch_csr = [&](int32_t kbeg, int32_t cnt, int32_t (&cv)[NC], uint16_t (&av)[NC]) {
        const int32_t base = cnt > 0 ? kbeg : (kbeg > 0 ? kbeg - 1 : 0);
        const int32_t lim = cnt > 0 ? cnt - 1 : 0;
#pragma unroll
        for (int u = 0; u < NC; ++u) {
            const int idx = lane + WAVE * u;
            const uint32_t k = (uint32_t)(base + (idx < lim ? idx : lim));
            cv[u] = ci[k];
            av[u] = ahat[k];
        }
    };
    // a slice of at most CAP entries goes to LDS as byte offsets and weights
    auto commit = [&](int32_t cnt, const int32_t (&cv)[NC], const uint16_t (&av)[NC]) {
        if (cnt <= CAP) {
#pragma unroll
            for (int u = 0; u < NC; ++u) {
                const int idx = lane + WAVE * u;
                sCo[wv][idx] = rshift >= 0 ? (uint32_t)cv[u] << rshift : (uint32_t)cv[u] * rowbytes;
                sVa[wv][idx] = av[u];
            }
        }
    };

    // Prologue: tile t's slice in LDS, tile t + nw's rowptr slice and entry
    // range known.  Everything loaded here is consumed here, so the loop
    // starts with no loads in flight.
    int64_t t = walk.t;
    int32_t rp0 = rp_first;     // rowptr slice of the current tile
    int32_t kb0, cnt0;          // its entry range
    slice_range(t, rp0, kb0, cnt0);
    int32_t rp1 = rp_second;    // of the next tile
    {
        int32_t cv[NC];
        uint16_t av[NC];
        fetch_csr(kb0, cnt0, cv, av);
        commit(cnt0, cv, av);
    }
    int32_t kb1, cnt1;
    slice_range(t + nw, rp1, kb1, cnt1);
    wave_lds_sync();
    for (; t < ntiles; t += nw) {
        const int64_t r0 = t * 16;
        uint32_t ifirst;
        int nn;
        node_range(t, ifirst, nn);
        const int32_t kbeg = kb0;
        const bool staged = cnt0 <= CAP;
        // ---- next tiles' slices, in flight during this tile's gather
        int32_t cv1[NC];
        uint16_t av1[NC];
        fetch_csr(kb1, cnt1, cv1, av1);
        const int32_t rp2 = fetch_rp(t + 2 * nw);
        // ---- gather T = A-hat X and the row's own X into the LDS tile
        {
            const int rl = lane / 4, q = lane % 4;
            const int64_t r = r0 + rl;
            const bool valid = r < rows;
            const uint32_t rr = (uint32_t)(valid ? r : r0);
            const uint32_t i = B1 ? rr : rr / (uint32_t)B;
            const uint32_t b = rr - i * (uint32_t)B;
            const int li = (int)(i - ifirst);
            const int32_t ks = valid ? __shfl(rp0, li, WAVE) - kbeg : 0;
            const int32_t ke = valid ? __shfl(rp0, li + 1, WAVE) - kbeg : 0;
            const uint32_t lane_off = (b * D + (uint32_t)(q * (D / 4))) * (uint32_t)sizeof(G);
            const uint32_t own_off = (rr * D + (uint32_t)(q * (D / 4))) * (uint32_t)sizeof(G);
            // rows past the end read zeros
            const Chunk<CB> own = buffer_chunk<CB>(xr, valid ? own_off : BUF_OOB);
            float ta[D / 4];
#pragma unroll
            for (int e = 0; e < D / 4; ++e) ta[e] = 0.f;
            auto acc_chunk = [&](const Chunk<CB> &raw, uint32_t wlo) {
                const uint32_t whi = wlo << 16;
#pragma unroll
                for (int j = 0; j < CB / 4; ++j) {
                    const bf16x2 xv = __builtin_bit_cast(bf16x2, raw.w[j]);
                    ta[2 * j] = __builtin_amdgcn_fdot2_f32_bf16(xv, __builtin_bit_cast(bf16x2, wlo),
                                                                ta[2 * j], false);
                    ta[2 * j + 1] = __builtin_amdgcn_fdot2_f32_bf16(
                        xv, __builtin_bit_cast(bf16x2, whi), ta[2 * j + 1], false);
                }
            };
            if (staged) {
                for (int32_t k0 = ks; k0 < ke; k0 += NB) {
                    Chunk<CB> raw[NB];
                    uint32_t wgt[NB];
                    // slots past the row read zeros: their (finite, staged)
                    // weights then add nothing
#pragma unroll
                    for (int u = 0; u < NB; ++u) {
                        const int32_t kk = k0 + u < CAP ? k0 + u : CAP - 1;
                        wgt[u] = sVa[wv][kk];
                        // past the row: the offset OR-ed up to BUF_OOB (the
                        // staged value stays in use, so its read is not
                        // moved into a branch)
                        const uint32_t oob = k0 + u < ke ? 0u : BUF_OOB;
                        raw[u] = buffer_chunk<CB>(xr, (sCo[wv][kk] + lane_off) | oob);
                    }
#pragma unroll
                    for (int u = 0; u < NB; ++u) acc_chunk(raw[u], wgt[u]);
                }
            } else {
                for (int32_t k = kbeg + ks; k < kbeg + ke; ++k) {
                    const uint32_t c = (uint32_t)ci[k];
                    acc_chunk(buffer_chunk<CB>(xr, c * rowbytes + lane_off), (uint32_t)ahat[k]);
                }
            }
            *reinterpret_cast<Chunk<CB> *>(&As[wv][rl][q * (D / 4)]) = own;  // already bf16
            store_feats<G, D / 4>(&As[wv][rl][D + q * (D / 4)], ta);
        }
        wave_lds_sync();
        // ---- Y^T = [U; W]^T [X | T]^T on MFMA, lane gets row l % 16
        {
            f32x4 o[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) o[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                const bf16x8 xf = load_bf16x8(&As[wv][lane % 16][kb * 32 + 8 * (lane / 16)]);
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    o[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        load_bf16x8(sW + ((kb * NT + nt) * WAVE + lane) * 8), xf, o[nt], 0, 0, 0);
            }
            const int64_t r = r0 + lane % 16;
            if constexpr (!DEC) {
                if (r < rows) {
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
                        *reinterpret_cast<uint2 *>(Y + r * D + nt * 16 + 4 * (lane / 16)) =
                            make_uint2(relu_pk_bf16(o[nt][0], o[nt][1]),
                                       relu_pk_bf16(o[nt][2], o[nt][3]));
                }
            } else {
                // ---- decoder: Y (bf16, K zero-padded to KP) to LDS, then
                // hidden^T = W3^T Y^T on MFMA, then ReLU(. + c3) W4 per row
                wave_lds_sync();  // every lane has read its tile fragments
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const int f = nt * 16 + 4 * (lane / 16);
                    *reinterpret_cast<uint2 *>(&As[wv][lane % 16][f]) = make_uint2(
                        relu_pk_bf16(o[nt][0], o[nt][1]), relu_pk_bf16(o[nt][2], o[nt][3]));
                    if constexpr (KP > D)
                        *reinterpret_cast<uint2 *>(&As[wv][lane % 16][D + f]) = make_uint2(0u, 0u);
                }
                wave_lds_sync();
                f32x4 hacc[H / 16];
#pragma unroll
                for (int nt = 0; nt < H / 16; ++nt) hacc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < KP / 32; ++kb) {
                    const bf16x8 yf = load_bf16x8(&As[wv][lane % 16][kb * 32 + 8 * (lane / 16)]);
#pragma unroll
                    for (int nt = 0; nt < H / 16; ++nt)
                        hacc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            load_bf16x8(sW3 + ((kb * (H / 16) + nt) * WAVE + lane) * 8), yf,
                            hacc[nt], 0, 0, 0);
                }
                // lane holds hidden units nt*16 + 4 (l/16) + j of row l % 16
                float part = 0.f;
#pragma unroll
                for (int nt = 0; nt < H / 16; ++nt) {
                    const int k0 = nt * 16 + 4 * (lane / 16);
                    const float4 c3 = *reinterpret_cast<const float4 *>(&sC3[k0]);
                    const float4 w4 = *reinterpret_cast<const float4 *>(&sW4[k0]);
                    part += fmaxf(hacc[nt][0] + c3.x, 0.f) * w4.x;
                    part += fmaxf(hacc[nt][1] + c3.y, 0.f) * w4.y;
                    part += fmaxf(hacc[nt][2] + c3.z, 0.f) * w4.z;
                    part += fmaxf(hacc[nt][3] + c3.w, 0.f) * w4.w;
                }
                part += __shfl_xor(part, 16, WAVE);
                part += __shfl_xor(part, 32, WAVE);
                if (lane < 16 && r < rows)
                    z[r] = (ZT)(tau[3 * ((uint32_t)r % (uint32_t)B) + 2] *
                                (double)(part + vec[oc4]));
            }
        }
        // ---- the next tile's slice to LDS (this tile's gather has read its
        // own), the entry range of the one after
        commit(cnt1, cv1, av1);
        int32_t kb2, cnt2;
        slice_range(t + 2 * nw, rp2, kb2, cnt2);
        wave_lds_sync();
        rp0 = rp1;
        rp1 = rp2;
        kb0 = kb1;
        cnt0 = cnt1;
        kb1 = kb2;
        cnt1 = cnt2;
    }
}

// ---------------------------------------------------------------------------
// Float32 Res-GCONV layer (Eq. (5)), pipelined like layer_tiles_bf16: the
// same tile walk, CSR slice staging and one memory round trip per tile, with
// float32 activations (32 bytes per lane and row for d = 32, two buffer
// loads), A-hat in float32, FP32 FMA gathers and the [X | T] [U; W] product
// on v_mfma_f32_16x16x4f32 with the weight fragments staged in LDS.  With
// DEC the decoder follows on the tile (W3 on MFMA as well).  Per row the
// arithmetic is that of the one-right-hand-side and the several-right-hand-
// side variants alike (neighbours in CSR order, the same MFMA sequence).
// ---------------------------------------------------------------------------
template <int BYTES>
__device__ __forceinline__ Chunk<BYTES> buffer_chunk_f(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    if constexpr (BYTES <= 16) {
        return buffer_chunk<BYTES>(r, off);
    } else {
        static_assert(BYTES == 32, "chunk of up to 32 bytes");
        // off is either in range or at least BUF_OOB (out of range for both halves)
        const uint32_t off2 = off >= BUF_OOB ? off : off + 16u;
        Chunk<32> c;
        const Chunk<16> a = buffer_chunk<16>(r, off), b = buffer_chunk<16>(r, off2);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            c.w[i] = a.w[i];
            c.w[4 + i] = b.w[i];
        }
        return c;
    }
}

template <int D, int H, bool DEC, bool B1, bool SHORT, typename ZT>
__device__ __forceinline__ void layer_tiles_f32p(
    int64_t rows, int B, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const float *__restrict__ ahat, const float *__restrict__ X, float *__restrict__ Y,
    const void *__restrict__ wcat, const void *__restrict__ w3, const float *__restrict__ vec,
    int64_t oc3, int64_t oW4, int64_t oc4, const double *__restrict__ tau, ZT *__restrict__ z,
    const int *__restrict__ skip) {
    const int skipped = skip ? *skip : 0;
    using G = float;
    constexpr int LD = 2 * D + lds_pad<G>();
    constexpr int CAP = SHORT ? 128 : 256, NC = CAP / WAVE;
    constexpr int KS = 2 * D / 4, NT = D / 16;    // MFMA k-steps and n-tiles
    constexpr int CB = (D / 4) * (int)sizeof(G);  // bytes per lane per row
    constexpr int NB = SHORT ? 7 : 8;             // neighbour loads per batch
    constexpr int NW3 = DEC ? (D / 4) * (H / 16) * WAVE : 1;  // W3 fragments
    __shared__ __attribute__((aligned(16))) G As[BLOCK / WAVE][16][LD];
    __shared__ uint32_t sCo[BLOCK / WAVE][CAP];  // byte offset of row (column, rhs 0) in X
    __shared__ float sVa[BLOCK / WAVE][CAP];
    __shared__ __attribute__((aligned(16))) float sW[KS * NT * WAVE];
    __shared__ __attribute__((aligned(16))) float sW3[NW3];
    __shared__ __attribute__((aligned(16))) float sC3[DEC ? H : 4], sW4[DEC ? H : 4];
    const int lane = threadIdx.x % WAVE;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const TileWalk walk = xcd_walk((rows + 15) / 16, BLOCK / WAVE, wv, B1);
    const int64_t ntiles = walk.end, nw = walk.stride;
    const uint32_t rowbytes = (uint32_t)B * (uint32_t)(D * sizeof(G));
    const int rshift = (rowbytes & (rowbytes - 1)) == 0 ? __builtin_ctz(rowbytes) : -1;
    // X holds rows * D features (< 2^32 bytes, checked by the launcher)
    const __amdgpu_buffer_rsrc_t xr = buffer_rsrc(X, (uint32_t)rows * (uint32_t)(D * sizeof(G)));

    auto node_range = [&](int64_t t, uint32_t &ifirst, int &nn) {
        const uint32_t tt = (uint32_t)(t < ntiles ? t : ntiles - 1);
        const uint32_t r0 = tt * 16u;
        const uint32_t rlast = r0 + 15u < (uint32_t)rows ? r0 + 15u : (uint32_t)rows - 1u;
        ifirst = B1 ? r0 : r0 / (uint32_t)B;
        nn = (int)((B1 ? rlast : rlast / (uint32_t)B) - ifirst) + 1;
    };
    auto fetch_rp = [&](int64_t t) -> int32_t {
        uint32_t ifirst;
        int nn;
        node_range(t, ifirst, nn);
        return rp[ifirst + (uint32_t)(lane <= nn ? lane : nn)];
    };
    // the row pointers of the wavefront's first two tiles go out before the
    // weights are staged, so that the two round trips overlap
    const int32_t rp_first = fetch_rp(walk.t), rp_second = fetch_rp(walk.t + nw);
    {
        const float4 *src = reinterpret_cast<const float4 *>(wcat);
        for (int e = threadIdx.x; e < KS * NT * WAVE / 4; e += BLOCK)
            reinterpret_cast<float4 *>(sW)[e] = src[e];
        if constexpr (DEC) {
            const float4 *src3 = reinterpret_cast<const float4 *>(w3);
            for (int e = threadIdx.x; e < NW3 / 4; e += BLOCK)
                reinterpret_cast<float4 *>(sW3)[e] = src3[e];
            for (int e = threadIdx.x; e < H; e += BLOCK) {
                sC3[e] = vec[oc3 + e];
                sW4[e] = vec[oW4 + e];
            }
        }
        __syncthreads();
    }
    if (skipped) return;
    auto slice_range = [&](int64_t t, int32_t rpv, int32_t &kbeg, int32_t &cnt) {
        uint32_t ifirst;
        int nn;
        node_range(t, ifirst, nn);
        kbeg = __builtin_amdgcn_readfirstlane(rpv);
        cnt = __builtin_amdgcn_readlane(rpv, nn) - kbeg;
    };
    auto fetch_csr = [&](int32_t kbeg, int32_t cnt, int32_t (&cv)[NC], float (&av)[NC]) {
        const int32_t base = cnt > 0 ? kbeg : (kbeg > 0 ? kbeg - 1 : 0);
        const int32_t lim = cnt > 0 ? cnt - 1 : 0;
#pragma unroll
        for (int u = 0; u < NC; ++u) {
            const int idx = lane + WAVE * u;
            const uint32_t k = (uint32_t)(base + (idx < lim ? idx : lim));
            cv[u] = ci[k];
            av[u] = ahat[k];
        }
    };
    auto commit = [&](int32_t cnt, const int32_t (&cv)[NC], const float (&av)[NC]) {
        if (cnt <= CAP) {
#pragma unroll
            for (int u = 0; u < NC; ++u) {
                const int idx = lane + WAVE * u;
                sCo[wv][idx] = rshift >= 0 ? (uint32_t)cv[u] << rshift : (uint32_t)cv[u] * rowbytes;
                sVa[wv][idx] = av[u];
            }
        }
    };

    int64_t t = walk.t;
    int32_t rp0 = rp_first;
    int32_t kb0, cnt0;
    slice_range(t, rp0, kb0, cnt0);
    int32_t rp1 = rp_second;
    {
        int32_t cv[NC];
        float av[NC];
        fetch_csr(kb0, cnt0, cv, av);
        commit(cnt0, cv, av);
    }
    int32_t kb1, cnt1;
    slice_range(t + nw, rp1, kb1, cnt1);
    wave_lds_sync();
    for (; t < ntiles; t += nw) {
        const int64_t r0 = t * 16;
        uint32_t ifirst;
        int nn;
        node_range(t, ifirst, nn);
        const int32_t kbeg = kb0;
        const bool staged = cnt0 <= CAP;
        int32_t cv1[NC];
        float av1[NC];
        fetch_csr(kb1, cnt1, cv1, av1);
        const int32_t rp2 = fetch_rp(t + 2 * nw);
        // ---- gather T = A-hat X and the row's own X into the LDS tile
        {
            const int rl = lane / 4, q = lane % 4;
            const int64_t r = r0 + rl;
            const bool valid = r < rows;
            const uint32_t rr = (uint32_t)(valid ? r : r0);
            const uint32_t i = B1 ? rr : rr / (uint32_t)B;
            const uint32_t b = rr - i * (uint32_t)B;
            const int li = (int)(i - ifirst);
            const int32_t ks = valid ? __shfl(rp0, li, WAVE) - kbeg : 0;
            const int32_t ke = valid ? __shfl(rp0, li + 1, WAVE) - kbeg : 0;
            const uint32_t lane_off = (b * D + (uint32_t)(q * (D / 4))) * (uint32_t)sizeof(G);
            const uint32_t own_off = (rr * D + (uint32_t)(q * (D / 4))) * (uint32_t)sizeof(G);
            const Chunk<CB> own = buffer_chunk_f<CB>(xr, valid ? own_off : BUF_OOB);
            float ta[D / 4];
#pragma unroll
            for (int e = 0; e < D / 4; ++e) ta[e] = 0.f;
            auto acc_chunk = [&](const Chunk<CB> &raw, float a) {
#pragma unroll
                for (int e = 0; e < CB / 4; ++e)
                    ta[e] = __builtin_fmaf(a, __builtin_bit_cast(float, raw.w[e]), ta[e]);
            };
            if (staged) {
                for (int32_t k0 = ks; k0 < ke; k0 += NB) {
                    Chunk<CB> raw[NB];
                    float wgt[NB];
#pragma unroll
                    for (int u = 0; u < NB; ++u) {
                        const int32_t kk = k0 + u < CAP ? k0 + u : CAP - 1;
                        wgt[u] = sVa[wv][kk];
                        const uint32_t oob = k0 + u < ke ? 0u : BUF_OOB;
                        raw[u] = buffer_chunk_f<CB>(xr, (sCo[wv][kk] + lane_off) | oob);
                    }
#pragma unroll
                    for (int u = 0; u < NB; ++u) acc_chunk(raw[u], wgt[u]);
                }
            } else {
                for (int32_t k = kbeg + ks; k < kbeg + ke; ++k) {
                    const uint32_t c = (uint32_t)ci[k];
                    acc_chunk(buffer_chunk_f<CB>(xr, c * rowbytes + lane_off), ahat[k]);
                }
            }
            *reinterpret_cast<Chunk<CB> *>(&As[wv][rl][q * (D / 4)]) = own;
            store_feats<G, D / 4>(&As[wv][rl][D + q * (D / 4)], ta);
        }
        wave_lds_sync();
        // ---- Y^T = [U; W]^T [X | T]^T on MFMA, lane gets row l % 16
        {
            f32x4 o[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) o[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < KS; ++kk) {
                const float a = As[wv][lane % 16][kk * 4 + lane / 16];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    o[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(sW[(kk * NT + nt) * WAVE + lane], a,
                                                                 o[nt], 0, 0, 0);
            }
            const int64_t r = r0 + lane % 16;
            if constexpr (!DEC) {
                if (r < rows) {
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
                        *reinterpret_cast<float4 *>(Y + r * D + nt * 16 + 4 * (lane / 16)) =
                            make_float4(relu(o[nt][0]), relu(o[nt][1]), relu(o[nt][2]),
                                        relu(o[nt][3]));
                }
            } else {
                // ---- decoder: Y to LDS, hidden^T = W3^T Y^T on MFMA, then
                // ReLU(. + c3) W4 per row
                wave_lds_sync();
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const int f = nt * 16 + 4 * (lane / 16);
                    *reinterpret_cast<float4 *>(&As[wv][lane % 16][f]) =
                        make_float4(relu(o[nt][0]), relu(o[nt][1]), relu(o[nt][2]), relu(o[nt][3]));
                }
                wave_lds_sync();
                f32x4 hacc[H / 16];
#pragma unroll
                for (int nt = 0; nt < H / 16; ++nt) hacc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kk = 0; kk < D / 4; ++kk) {
                    const float y = As[wv][lane % 16][kk * 4 + lane / 16];
#pragma unroll
                    for (int nt = 0; nt < H / 16; ++nt)
                        hacc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            sW3[(kk * (H / 16) + nt) * WAVE + lane], y, hacc[nt], 0, 0, 0);
                }
                float part = 0.f;
#pragma unroll
                for (int nt = 0; nt < H / 16; ++nt) {
                    const int k0 = nt * 16 + 4 * (lane / 16);
                    const float4 c3 = *reinterpret_cast<const float4 *>(&sC3[k0]);
                    const float4 w4 = *reinterpret_cast<const float4 *>(&sW4[k0]);
                    part += fmaxf(hacc[nt][0] + c3.x, 0.f) * w4.x;
                    part += fmaxf(hacc[nt][1] + c3.y, 0.f) * w4.y;
                    part += fmaxf(hacc[nt][2] + c3.z, 0.f) * w4.z;
                    part += fmaxf(hacc[nt][3] + c3.w, 0.f) * w4.w;
                }
                part += __shfl_xor(part, 16, WAVE);
                part += __shfl_xor(part, 32, WAVE);
                if (lane < 16 && r < rows)
                    z[r] = (ZT)(tau[3 * ((uint32_t)r % (uint32_t)B) + 2] *
                                (double)(part + vec[oc4]));
            }
        }
        commit(cnt1, cv1, av1);
        int32_t kb2, cnt2;
        slice_range(t + 2 * nw, rp2, kb2, cnt2);
        wave_lds_sync();
        rp0 = rp1;
        rp1 = rp2;
        kb0 = kb1;
        cnt0 = cnt1;
        kb1 = kb2;
        cnt1 = cnt2;
    }
}

#define GNP_LAYER_PARAMS                                                                       \
    int64_t rows, int B, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,       \
        const typename Act<G>::vt *__restrict__ ahat, const G *__restrict__ X,                 \
        G *__restrict__ Y, const void *__restrict__ wcat, const void *__restrict__ w3,         \
        const typename Act<G>::acc *__restrict__ vec, int64_t oc3, int64_t oW4, int64_t oc4,   \
        const double *__restrict__ tau, ZT *__restrict__ z, const int *__restrict__ skip
#define GNP_LAYER_ARGS rows, B, rp, ci, ahat, X, Y, wcat, w3, vec, oc3, oW4, oc4, tau, z, skip

template <typename G, int D, int H, bool DEC, typename ZT>
__global__ __launch_bounds__(BLOCK) void k_layer(GNP_LAYER_PARAMS) {
    layer_tiles<G, D, H, DEC, ZT>(GNP_LAYER_ARGS);
}

// The bfloat16 layers (and the last one with the decoder), held to 128
// registers: at least 4 wavefronts per SIMD.
template <typename G, int D, int H, bool DEC, typename ZT, bool B1 = false, bool SHORT = false>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_layer_w4(
    GNP_LAYER_PARAMS) {
    static_assert(sizeof(G) == 2, "bfloat16 layer");
    layer_tiles_bf16<D, H, DEC, B1, SHORT, ZT>(rows, B, rp, ci, ahat, X, Y, wcat, w3, vec, oc3, oW4,
                                               oc4, tau, z, skip);
}
// The pipelined float32 layers, held to 128 registers (4 wavefronts per SIMD).
template <typename G, int D, int H, bool DEC, typename ZT, bool B1 = false, bool SHORT = false>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_layer_f32p(
    GNP_LAYER_PARAMS) {
    static_assert(sizeof(G) == 4, "float32 layer");
    layer_tiles_f32p<D, H, DEC, B1, SHORT, ZT>(rows, B, rp, ci, ahat, X, Y, wcat, w3, vec, oc3,
                                               oW4, oc4, tau, z, skip);
}

#undef GNP_LAYER_PARAMS
#undef GNP_LAYER_ARGS

// The layer kernel to launch for a configuration (B: right-hand sides
// interleaved in the activations; max_row: the longest row of the matrix).
// The bfloat16 kernel has variants for one right-hand side and for rows of
// at most 7 entries (7-point stencils and sparser).
template <typename G, int D, int H, bool DEC, typename ZT>
inline void (*layer_kernel(int B = 0, int max_row = 0))(
    int64_t, int, const int32_t *, const int32_t *, const typename Act<G>::vt *, const G *, G *,
    const void *, const void *, const typename Act<G>::acc *, int64_t, int64_t, int64_t,
    const double *, ZT *, const int *) {
    if constexpr (sizeof(G) == 2) {
        const bool shrt = max_row > 0 && max_row <= 7;
        if (B == 1)
            return shrt ? &k_layer_w4<G, D, H, DEC, ZT, true, true>
                        : &k_layer_w4<G, D, H, DEC, ZT, true, false>;
        return shrt ? &k_layer_w4<G, D, H, DEC, ZT, false, true>
                    : &k_layer_w4<G, D, H, DEC, ZT, false, false>;
    } else if constexpr (sizeof(G) == 4) {
        const bool shrt = max_row > 0 && max_row <= 7;
        if (B == 1)
            return shrt ? &k_layer_f32p<G, D, H, DEC, ZT, true, true>
                        : &k_layer_f32p<G, D, H, DEC, ZT, true, false>;
        return shrt ? &k_layer_f32p<G, D, H, DEC, ZT, false, true>
                    : &k_layer_f32p<G, D, H, DEC, ZT, false, false>;
    } else {
        return &k_layer<G, D, H, DEC, ZT>;
    }
}

// Grid of the persistent layer kernel: as many blocks as can be resident at
// once (the occupancy of the variant launched x compute units), at most one
// 64-row block per tile group.  B, max_row: as for layer_kernel.
template <typename G, int D, int H, bool DEC, typename ZT>
inline int layer_grid(int64_t rows, int B = 0, int max_row = 0) {
    int resident;
    if constexpr (sizeof(G) == 2) {
        const bool shrt = max_row > 0 && max_row <= 7;
        if (B == 1)
            resident = shrt ? resident_blocks<&k_layer_w4<G, D, H, DEC, ZT, true, true>>()
                            : resident_blocks<&k_layer_w4<G, D, H, DEC, ZT, true, false>>();
        else
            resident = shrt ? resident_blocks<&k_layer_w4<G, D, H, DEC, ZT, false, true>>()
                            : resident_blocks<&k_layer_w4<G, D, H, DEC, ZT, false, false>>();
    } else if constexpr (sizeof(G) == 4) {
        const bool shrt = max_row > 0 && max_row <= 7;
        if (B == 1)
            resident = shrt ? resident_blocks<&k_layer_f32p<G, D, H, DEC, ZT, true, true>>()
                            : resident_blocks<&k_layer_f32p<G, D, H, DEC, ZT, true, false>>();
        else
            resident = shrt ? resident_blocks<&k_layer_f32p<G, D, H, DEC, ZT, false, true>>()
                            : resident_blocks<&k_layer_f32p<G, D, H, DEC, ZT, false, false>>();
    } else {
        resident = resident_blocks<&k_layer<G, D, H, DEC, ZT>>();
    }
    const int64_t need = (rows + 63) / 64;
    int g = (int)(need < resident ? need : resident);
    return g >= XCDS ? g - g % XCDS : g;  // whole rounds over the XCDs
}

}  // namespace gnp
