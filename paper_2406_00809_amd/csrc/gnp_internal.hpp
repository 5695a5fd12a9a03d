// Internal declarations shared by the HIP translation units of libgnp.
// Device helpers: wavefront/block reductions, the deterministic "last block"
// grid reduction, bf16 conversion and MFMA operand vector types.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <string>

#include "../../include/gnp.h"

namespace gnp {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

constexpr int WAVE = 64;
constexpr int BLOCK = 256;

// ---------------------------------------------------------------------------
// error plumbing (host)
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);
gnp_status fail(gnp_status st, const std::string &msg);
gnp_status check_hip(hipError_t e, const char *what);

#define GNP_HIP(call)                                                   \
    do {                                                                \
        hipError_t e__ = (call);                                        \
        if (e__ != hipSuccess) return ::gnp::check_hip(e__, #call);     \
    } while (0)

#define GNP_TRY(call)                                                   \
    do {                                                                \
        gnp_status s__ = (call);                                        \
        if (s__ != GNP_OK) return s__;                                  \
    } while (0)

// ---------------------------------------------------------------------------
// conversions
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ float to_f32(T v) { return (float)v; }
template <> __device__ __forceinline__ float to_f32<__bf16>(__bf16 v) { return (float)v; }

template <typename T> __device__ __forceinline__ T from_acc(float v) { return (T)v; }
template <typename T> __device__ __forceinline__ T from_acc(double v) { return (T)v; }

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// Sum over the block in a fixed order (deterministic).  All threads must
// call it; the result is valid in every thread.  `scratch` holds BLOCK/WAVE
// doubles.
__device__ __forceinline__ double block_sum(double v, double *scratch) {
    const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) scratch[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x / WAVE); ++i) s += scratch[i];
    return s;
}

// Sum of partial[k * stride] over k < nblk in one fixed order (every thread
// of the block takes part and receives the sum): any block that calls it on
// the same data gets the same bits.  scratch: >= BLOCK / WAVE doubles.
__device__ __forceinline__ double sum_partials(int nblk, const double *__restrict__ partial,
                                               int stride, double *scratch) {
    const int t = threadIdx.x;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int blk0 = t; blk0 < nblk; blk0 += 4 * BLOCK) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {  // clamped, unconditional loads
            const int blk = blk0 + u * BLOCK;
            v[u] = partial[(int64_t)(blk < nblk ? blk : nblk - 1) * stride];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] += (blk0 + u * BLOCK < nblk) ? v[u] : 0.0;
    }
    return block_sum((a[0] + a[1]) + (a[2] + a[3]), scratch);
}

// Grid-level "last block" detection for deterministic two-stage reductions:
// every block writes its partials, then calls this; exactly one block (the
// last to arrive) gets true and may read all partials, which it sums in
// block order.  The ticket counter is reset by that block.
__device__ __forceinline__ bool last_block(unsigned *counter) {
    __shared__ int is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned t = atomicAdd(counter, 1u);
        is_last = (t == gridDim.x - 1) ? 1 : 0;
    }
    __syncthreads();
    if (is_last) {
        __threadfence();
        if (threadIdx.x == 0) atomicExch(counter, 0u);
    }
    return is_last != 0;
}

// ---------------------------------------------------------------------------
// tile walk of the persistent kernels
// ---------------------------------------------------------------------------
// Tile walk of a persistent grid that keeps every XCD on one contiguous range
// of tiles.  MI355X dispatches workgroups to its 8 XCDs round-robin (block b
// runs on XCD b % 8), and each XCD has an L2 of its own: with XCD x taking
// tiles [x T/8, (x+1) T/8) and its wavefronts striding through that range,
// the rows a tile gathers from its graph neighbours were mostly brought into
// that XCD's L2 by nearby tiles.  The walk covers every tile exactly once for
// any grid (grids that are not a multiple of 8 fall back to a plain stride);
// the placement only affects speed.
constexpr int XCDS = 8;
struct TileWalk {
    int64_t t, end, stride;
};
// ranges = false: the plain stride for every grid.  With several right-hand
// sides stored node-major a node's rows are B d elements long and the graph
// neighbours lie far apart in memory (a 64^3 stencil's z neighbours 16 MB
// away at B = 32 in float32), beyond any L2; the plain stride keeps all XCDs
// in one window of the activations, which the Infinity Cache then holds
// (the float32 layer at B = 32: 1.31 -> 1.11 ms).
__device__ __forceinline__ TileWalk xcd_walk(int64_t ntiles, int waves_per_block, int wv,
                                             bool ranges = true) {
    TileWalk w;
    if (ranges && gridDim.x % XCDS == 0) {
        const int64_t nbx = gridDim.x / XCDS;
        const int64_t x = blockIdx.x % XCDS, lb = blockIdx.x / XCDS;
        const int64_t per = (ntiles + XCDS - 1) / XCDS;
        const int64_t beg = x * per;
        w.end = beg + per < ntiles ? beg + per : ntiles;
        w.t = beg + lb * waves_per_block + wv;
        w.stride = nbx * waves_per_block;
    } else {
        w.t = (int64_t)blockIdx.x * waves_per_block + wv;
        w.end = ntiles;
        w.stride = (int64_t)gridDim.x * waves_per_block;
    }
    return w;
}

// precision selection
inline bool valid_precision(int p) { return p == GNP_F64 || p == GNP_F32 || p == GNP_BF16; }

inline int grid_for(int64_t work, int per_block, int cap = 1 << 20) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace gnp

// ---------------------------------------------------------------------------
// objects behind the opaque handles
// ---------------------------------------------------------------------------
struct gnp_system {
    int64_t n = 0, nnz = 0;
    int max_row = 0;
    int32_t *rp = nullptr, *ci = nullptr;        // CSR of A (device)
    double *val64 = nullptr;                     // system A, float64
    float *val32 = nullptr;                      // system A, float32
    double *ahat64 = nullptr;                    // A-hat = A / gamma
    float *ahat32 = nullptr;
    uint16_t *ahat16 = nullptr;                  // A-hat in bfloat16 (the BF16 network)
    int32_t *trp = nullptr, *tci = nullptr;      // CSR of A^T
    int32_t *tperm = nullptr;                    // entry k of A^T is entry tperm[k] of A
    int prescale = 0;                            // A was divided by its own gamma
    double *tval64 = nullptr;                    // A^T
    float *tval32 = nullptr;
    double *tahat64 = nullptr;                   // A-hat^T
    float *tahat32 = nullptr;
    double gamma_raw = 0.0, gamma = 0.0;
    unsigned *counters = nullptr;                // tickets for last-block reductions
    double *scratch = nullptr;                   // small reduction scratch
    int nscratch = 0;
    double *dinv64 = nullptr;                    // 1 / a_ii (Jacobi preconditioner), made on first use
    double solve_timeout = 0.0;                  // seconds per single solve, 0 = none
    void *solve_cache = nullptr;                 // FGMRES workspace of fgmres_solve
    void *batch_cache = nullptr;                 // workspace of fgmres_solve_batch
};

namespace gnp {
void solve_cache_free(void *p);
void batch_cache_free(void *p);
}
