// Network object and the internal launch interface of the forward pass.
#pragma once
#include "gnp_internal.hpp"

namespace gnp {

// bf16 held as raw 16-bit words in memory; conversions are explicit.
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
// float -> bf16, round to nearest even (v_cvt_pk_bf16_f32 on gfx950)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

struct ParamOffsets {
    int64_t W1, c1, W2, c2, W3, c3, W4, c4;
    int64_t U0;  // U_l at U0 + l * 2 d^2, W_l right after it
    int64_t total;
};

inline ParamOffsets param_offsets(int L, int d, int h) {
    ParamOffsets o;
    o.W1 = 0;
    o.c1 = h;
    o.W2 = 2 * h;
    o.c2 = o.W2 + (int64_t)h * d;
    o.U0 = o.c2 + d;
    o.W3 = o.U0 + (int64_t)L * 2 * d * d;
    o.c3 = o.W3 + (int64_t)d * h;
    o.W4 = o.c3 + h;
    o.c4 = o.W4 + h;
    o.total = o.c4 + 1;
    return o;
}

// Offsets (in elements) of the MFMA-fragment packings of the three matrix
// kinds.  bf16 fragments: 16x16x32 B-operand, K padded to a multiple of 32;
// f32 fragments: 16x16x4 B-operand.
struct PackOffsets {
    int64_t W2, Wcat0, Wcat_stride, W3, total;
};

inline int64_t pack_count_bf16(int K, int N) { return (int64_t)((K + 31) / 32) * (N / 16) * 512; }
inline int64_t pack_count_f32(int K, int N) { return (int64_t)(K / 4) * (N / 16) * 64; }

inline PackOffsets pack_offsets(int L, int d, int h, bool bf16) {
    PackOffsets p;
    auto cnt = [&](int K, int N) { return bf16 ? pack_count_bf16(K, N) : pack_count_f32(K, N); };
    p.W2 = 0;
    p.Wcat0 = cnt(h, d);
    p.Wcat_stride = cnt(2 * d, d);
    p.W3 = p.Wcat0 + (int64_t)L * p.Wcat_stride;
    p.total = p.W3 + cnt(d, h);
    return p;
}

struct ApplyWorkspace {
    int nrhs = 0;
    void *act[2] = {nullptr, nullptr};  // ping-pong activations, n*nrhs*d (sized for f64)
    double *tau = nullptr;              // [3 * nrhs]: tau, sqrt(n)/tau, tau/sqrt(n)
    double *partial = nullptr;          // column-norm partials
    unsigned *counter = nullptr;
    int partial_blocks = 0;
};

}  // namespace gnp

struct gnp_model {
    gnp_system *sys = nullptr;
    int L = 0, d = 0, h = 0;
    int64_t np = 0;
    int scaled = 1;                // 0: without s, s^-1 of Eq. (6) (ablation)
    double *theta64 = nullptr;     // master parameters (device, float64)
    float *theta32 = nullptr;      // float32 copy (biases and vectors)
    uint16_t *pk_bf16 = nullptr;   // bf16 MFMA fragments
    float *pk_f32 = nullptr;       // f32 MFMA fragments
    gnp::ParamOffsets po;
    gnp::PackOffsets pb, pf;
    gnp::ApplyWorkspace ws;
    void *train_ctx = nullptr;     // training workspace (train.hip)
};

namespace gnp {

void train_ctx_free(void *p);

// Repack the fragment layouts and float32 copy from theta64 (stream-ordered).
gnp_status model_repack(gnp_model *m, hipStream_t st);

// Make sure the apply workspace can hold nrhs right-hand sides.
gnp_status model_workspace(gnp_model *m, int nrhs);

// Number of blocks (and partials per column) of launch_colnorm for n rows.
int colnorm_blocks(int64_t n);

// Column norms of v ([n][nrhs], float or double) into tau triples
// (tau, sqrt(n)/tau, tau/sqrt(n)) at tau_out[3*k .. 3*k+2]; (tau, 1, 1)
// for a model without the scaling of Eq. (6).
template <typename IN>
void launch_colnorm(gnp_model *m, const IN *v, int nrhs, double *tau_out, double *partial,
                    unsigned *counter, const int *skip, hipStream_t st);

// The solver's next basis vector, formed by the encoder as it reads w (one
// right-hand side, float32 basis): with V given, the second Gram-Schmidt
// correction first, w - V[:, 0..j] h (basis pitch 32, the arithmetic of the
// solver's correction pass), then v = (that) / *hdiv, rounded as the basis
// stores it and written to vout.  The network takes v with tau = 1 (v has
// unit norm) and the encoder writes that tau triple.
struct BasisNext {
    const double *hdiv = nullptr;  // h_{j+1,j}
    float *vout = nullptr;         // v, the solver's contiguous copy
    const float *V = nullptr;      // basis (pitch 32); nullptr: w is already final
    const double *h = nullptr;     // correction coefficients h[0..j]
    float *Vout = nullptr;         // with V: also store v as column j + 1 of the basis
    int j = 0;
};

// z = M(v) given precomputed tau triples.  act0/act1: activation buffers.
// When layers != nullptr, X_0 (encoder output) and every layer output X_l
// are kept in block l of layers ((L+1) blocks of n * nrhs * d activations)
// instead of ping-ponging between act0 and act1.  With bn (one
// float32/bfloat16 right-hand side, inside the solver) v is the solver's
// vector w and the encoder forms the next basis vector itself (BasisNext).
gnp_status forward_launch(gnp_model *m, gnp_precision prec, const void *v, void *z, int nrhs,
                          const double *tau, void *act0, void *act1, const int *skip,
                          hipStream_t st, void *layers = nullptr,
                          const struct BasisNext *bn = nullptr);

}  // namespace gnp
