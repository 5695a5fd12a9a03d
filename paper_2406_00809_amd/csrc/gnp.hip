// Graph neural preconditioner: model object, weight packing into MFMA
// fragment layouts, column norms for the scaling s of Eq. (6), and the
// forward launch sequence (encoder, L Res-GCONV layers, decoder).
#include <math.h>

#include <mutex>
#include <unordered_map>
#include <vector>

#include "gnp_fwd.hpp"
#include "model.hpp"
#include "philox.hpp"

namespace gnp {

// ---------------------------------------------------------------------------
// packing
// ---------------------------------------------------------------------------
__global__ void k_pack_bf16(const double *__restrict__ th, int64_t off, int K, int N,
                            uint16_t *__restrict__ out, int64_t count) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= count) return;
    const int i = (int)(p % 8), lane = (int)((p / 8) % 64);
    const int64_t f = p / 512;
    const int ntiles = N / 16;
    const int nt = (int)(f % ntiles), kb = (int)(f / ntiles);
    const int k = kb * 32 + 8 * (lane / 16) + i, col = nt * 16 + lane % 16;
    const float v = k < K ? (float)th[off + (int64_t)k * N + col] : 0.f;
    out[p] = f2bf(v);
}

__global__ void k_pack_f32(const double *__restrict__ th, int64_t off, int K, int N,
                           float *__restrict__ out, int64_t count) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= count) return;
    const int lane = (int)(p % 64);
    const int64_t f = p / 64;
    const int ntiles = N / 16;
    const int nt = (int)(f % ntiles), ks = (int)(f / ntiles);
    const int k = ks * 4 + lane / 16, col = nt * 16 + lane % 16;
    out[p] = (float)th[off + (int64_t)k * N + col];
}

__global__ void k_copy_f32(const double *__restrict__ a, float *__restrict__ b, int64_t n) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) b[p] = (float)a[p];
}

// Stores v into every element of p[0, count) (evicts caches for cold timing).
__global__ void k_fill_f32(float *__restrict__ p, int64_t count, float v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

gnp_status model_repack(gnp_model *m, hipStream_t st) {
    const int L = m->L, d = m->d, h = m->h;
    hipLaunchKernelGGL(k_copy_f32, dim3(grid_for(m->np, BLOCK)), dim3(BLOCK), 0, st, m->theta64,
                       m->theta32, m->np);
    struct Mat { int64_t off; int K, N; int64_t pb, pf; };
    std::vector<Mat> mats;
    mats.push_back({m->po.W2, h, d, m->pb.W2, m->pf.W2});
    for (int l = 0; l < L; ++l)
        mats.push_back({m->po.U0 + (int64_t)l * 2 * d * d, 2 * d, d,
                        m->pb.Wcat0 + l * m->pb.Wcat_stride, m->pf.Wcat0 + l * m->pf.Wcat_stride});
    mats.push_back({m->po.W3, d, h, m->pb.W3, m->pf.W3});
    for (const Mat &x : mats) {
        const int64_t cb = pack_count_bf16(x.K, x.N), cf = pack_count_f32(x.K, x.N);
        hipLaunchKernelGGL(k_pack_bf16, dim3(grid_for(cb, BLOCK)), dim3(BLOCK), 0, st, m->theta64,
                           x.off, x.K, x.N, m->pk_bf16 + x.pb, cb);
        hipLaunchKernelGGL(k_pack_f32, dim3(grid_for(cf, BLOCK)), dim3(BLOCK), 0, st, m->theta64,
                           x.off, x.K, x.N, m->pk_f32 + x.pf, cf);
    }
    GNP_HIP(hipGetLastError());
    return GNP_OK;
}

// ---------------------------------------------------------------------------
// column norms: tau_k = ||v(:, k)||_2 in float64, deterministic two stages
// ---------------------------------------------------------------------------
static int64_t colnorm_chunk(int64_t n) {
    int64_t c = (n + 1023) / 1024;
    return c < 512 ? 512 : c;
}

int colnorm_blocks(int64_t n) { return grid_for(n, (int)colnorm_chunk(n)); }

template <typename IN>
__global__ __launch_bounds__(BLOCK) void k_colnorm(int64_t n, int B, int64_t chunk,
                                                   const IN *__restrict__ v, double *partial,
                                                   unsigned *counter, double *tau,
                                                   const int *__restrict__ skip, int scaled) {
    if (skip && *skip) return;
    __shared__ double sh[BLOCK];
    const int t = threadIdx.x;
    const int S = BLOCK / B;
    const int c = t % B, p = t / B;
    double s = 0.0;
    if (p < S) {
        const int64_t i0 = (int64_t)blockIdx.x * chunk;
        const int64_t i1 = (i0 + chunk < n) ? i0 + chunk : n;
        // eight rows in flight at once, squares added in row order
        constexpr int U = 8;
        for (int64_t ib = i0 + p; ib < i1; ib += U * S) {
            double x[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i = ib + u * S < i1 ? ib + u * S : ib;
                x[u] = (double)v[i * B + c];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (ib + u * S < i1) s += x[u] * x[u];
        }
    }
    sh[t] = s;
    __syncthreads();
    if (t < B) {
        double a = 0.0;
        for (int k = 0; k < S; ++k) a += sh[t + k * B];
        partial[(int64_t)blockIdx.x * B + t] = a;
    }
    if (last_block(counter)) {
        if (t < B) {
            double a = 0.0;
            for (unsigned blk = 0; blk < gridDim.x; ++blk) a += partial[(int64_t)blk * B + t];
            const double tv = sqrt(a), sqn = sqrt((double)n);
            tau[3 * t] = tv;
            tau[3 * t + 1] = scaled ? (tv > 0.0 ? sqn / tv : 0.0) : 1.0;
            tau[3 * t + 2] = scaled ? tv / sqn : 1.0;
        }
    }
}

template <typename IN>
void launch_colnorm(gnp_model *m, const IN *v, int nrhs, double *tau_out, double *partial,
                    unsigned *counter, const int *skip, hipStream_t st) {
    const int64_t n = m->sys->n, chunk = colnorm_chunk(n);
    const int nb = grid_for(n, (int)chunk);
    hipLaunchKernelGGL(k_colnorm<IN>, dim3(nb), dim3(BLOCK), 0, st, n, nrhs, chunk, v, partial,
                       counter, tau_out, skip, m->scaled);
}
template void launch_colnorm<float>(gnp_model *, const float *, int, double *, double *,
                                    unsigned *, const int *, hipStream_t);
template void launch_colnorm<double>(gnp_model *, const double *, int, double *, double *,
                                     unsigned *, const int *, hipStream_t);

gnp_status model_workspace(gnp_model *m, int nrhs) {
    ApplyWorkspace &w = m->ws;
    if (w.nrhs >= nrhs) return GNP_OK;
    for (int i = 0; i < 2; ++i)
        if (w.act[i]) (void)hipFree(w.act[i]);
    if (w.tau) (void)hipFree(w.tau);
    if (w.partial) (void)hipFree(w.partial);
    if (w.counter) (void)hipFree(w.counter);
    w = ApplyWorkspace();
    const int64_t n = m->sys->n;
    const size_t act_bytes = sizeof(double) * (size_t)n * nrhs * m->d;
    for (int i = 0; i < 2; ++i) GNP_HIP(hipMalloc(&w.act[i], act_bytes));
    GNP_HIP(hipMalloc(&w.tau, sizeof(double) * 3 * nrhs));
    w.partial_blocks = grid_for(n, (int)colnorm_chunk(n));
    GNP_HIP(hipMalloc(&w.partial, sizeof(double) * (size_t)w.partial_blocks * nrhs));
    GNP_HIP(hipMalloc(&w.counter, sizeof(unsigned) * 4));
    GNP_HIP(hipMemset(w.counter, 0, sizeof(unsigned) * 4));
    w.nrhs = nrhs;
    return GNP_OK;
}

// ---------------------------------------------------------------------------
// forward launch sequence
// ---------------------------------------------------------------------------
// layers (optional): (L+1) blocks of rows*D activations; when given, X_0 and
// every layer output X_l go to block l (the last layer then runs once more
// without the decoder to materialise X_L).
// bn (optional, one right-hand side, MFMA paths): v is the solver's vector
// w; the encoder forms the next basis vector from it (BasisNext), takes
// tau = 1 for it and stores that triple in tau.
template <typename G, typename IN, typename ZT, int D, int H>
static void forward_typed(gnp_model *m, const IN *v, ZT *z, int nrhs, const double *tau,
                          G *act0, G *act1, const typename Act<G>::acc *vec, const void *wmat,
                          const int *skip, hipStream_t st, G *layers = nullptr,
                          const BasisNext *bn = nullptr) {
    gnp_system *s = m->sys;
    const int64_t rows = s->n * (int64_t)nrhs;
    const int grid = grid_for(rows, 64);
    const ParamOffsets &po = m->po;
    const typename Act<G>::vt *ahat;
    const void *w2, *w3;
    int64_t wstride, w0;
    if constexpr (sizeof(G) == 8) {
        ahat = (const typename Act<G>::vt *)s->ahat64;
        w2 = m->theta64 + po.W2;
        w3 = m->theta64 + po.W3;
        w0 = po.U0;
        wstride = 2 * (int64_t)D * D;
    } else if constexpr (sizeof(G) == 4) {
        ahat = (const typename Act<G>::vt *)s->ahat32;
        w2 = m->pk_f32 + m->pf.W2;
        w3 = m->pk_f32 + m->pf.W3;
        w0 = m->pf.Wcat0;
        wstride = m->pf.Wcat_stride;
    } else {
        ahat = (const typename Act<G>::vt *)s->ahat16;
        w2 = m->pk_bf16 + m->pb.W2;
        w3 = m->pk_bf16 + m->pb.W3;
        w0 = m->pb.Wcat0;
        wstride = m->pb.Wcat_stride;
    }
    auto wcat = [&](int l) -> const void * {
        if constexpr (sizeof(G) == 8) return m->theta64 + w0 + l * wstride;
        else if constexpr (sizeof(G) == 4) return m->pk_f32 + w0 + l * wstride;
        else return m->pk_bf16 + w0 + l * wstride;
    };
    (void)wmat;
    G *bufs[2] = {act0, act1};
    auto buf = [&](int l) -> G * {  // holds X_l
        return layers ? layers + (int64_t)l * rows * D : bufs[l % 2];
    };
    if constexpr (sizeof(G) == 8) {
        hipLaunchKernelGGL((k_encoder<G, IN, D, H>), dim3(grid), dim3(BLOCK), 0, st, rows, nrhs,
                           v, tau, vec, po.W1, po.c1, po.c2, w2, buf(0), skip);
    } else {
        const int ge = std::min(grid, resident_blocks<k_encoder_p<G, IN, D, H>>());
        hipLaunchKernelGGL((k_encoder_p<G, IN, D, H>), dim3(ge), dim3(BLOCK), 0, st, rows, nrhs,
                           v, const_cast<double *>(tau), vec, po.W1, po.c1, po.c2, w2, buf(0),
                           skip, bn ? *bn : BasisNext{}, s->n);
    }
    for (int l = 0; l < m->L; ++l) {
        const G *X = buf(l);
        if (l < m->L - 1 || layers) {
            hipLaunchKernelGGL((layer_kernel<G, D, H, false, ZT>(nrhs, s->max_row)),
                               dim3(layer_grid<G, D, H, false, ZT>(rows, nrhs, s->max_row)), dim3(BLOCK), 0, st, rows,
                               nrhs, s->rp, s->ci, ahat, X, buf(l + 1), wcat(l), w3, vec,
                               po.c3, po.W4, po.c4, tau, z, skip);
        }
        if (l == m->L - 1) {
            hipLaunchKernelGGL((layer_kernel<G, D, H, true, ZT>(nrhs, s->max_row)),
                               dim3(layer_grid<G, D, H, true, ZT>(rows, nrhs, s->max_row)), dim3(BLOCK), 0, st, rows,
                               nrhs, s->rp, s->ci, ahat, X, (G *)nullptr, wcat(l), w3, vec, po.c3,
                               po.W4, po.c4, tau, z, skip);
        }
    }
}

template <int D, int H>
static void forward_dispatch(gnp_model *m, gnp_precision prec, const void *v, void *z, int nrhs,
                             const double *tau, void *a0, void *a1, const int *skip,
                             hipStream_t st, void *layers, const BasisNext *bn) {
    if (prec == GNP_F64)
        forward_typed<double, double, double, D, H>(m, (const double *)v, (double *)z, nrhs, tau,
                                                    (double *)a0, (double *)a1, m->theta64,
                                                    nullptr, skip, st, (double *)layers);
    else if (prec == GNP_F32)
        forward_typed<float, float, float, D, H>(m, (const float *)v, (float *)z, nrhs, tau,
                                                 (float *)a0, (float *)a1, m->theta32, nullptr,
                                                 skip, st, (float *)layers, bn);
    else
        forward_typed<uint16_t, float, float, D, H>(m, (const float *)v, (float *)z, nrhs, tau,
                                                    (uint16_t *)a0, (uint16_t *)a1, m->theta32,
                                                    nullptr, skip, st, (uint16_t *)layers,
                                                    bn);
}

gnp_status forward_launch(gnp_model *m, gnp_precision prec, const void *v, void *z, int nrhs,
                          const double *tau, void *act0, void *act1, const int *skip,
                          hipStream_t st, void *layers, const BasisNext *bn) {
    if (bn && (nrhs != 1 || prec == GNP_F64 || !bn->hdiv))
        return fail(GNP_EINVAL, "the encoder forms basis vectors only for one float32/bfloat16 rhs");
    const int64_t elem = prec == GNP_F64 ? 8 : (prec == GNP_F32 ? 4 : 2);
    if (m->sys->n * (int64_t)nrhs * m->d * elem >= (int64_t)1 << 32)
        return fail(GNP_EINVAL,
                    "an activation block (n * nrhs * d elements) must stay below 4 GiB "
                    "(32-bit gather offsets)");
    if (m->d == 16)
        forward_dispatch<16, 32>(m, prec, v, z, nrhs, tau, act0, act1, skip, st, layers, bn);
    else
        forward_dispatch<32, 64>(m, prec, v, z, nrhs, tau, act0, act1, skip, st, layers, bn);
    GNP_HIP(hipGetLastError());
    return GNP_OK;
}

// One Res-GCONV layer launch, exactly as in the forward sequence (nrhs
// right-hand sides on the apply workspace, layer `l`, non-final variant).
template <typename G, int D, int H>
static void layer_once(gnp_model *m, int nrhs, int l, hipStream_t st) {
    gnp_system *s = m->sys;
    const int64_t rows = s->n * (int64_t)nrhs;
    const int grid = layer_grid<G, D, H, false, float>(rows, nrhs, s->max_row);
    const void *wc;
    const typename Act<G>::vt *ahat;
    const typename Act<G>::acc *vec;
    if constexpr (sizeof(G) == 8) {
        wc = m->theta64 + m->po.U0 + (int64_t)l * 2 * D * D;
        ahat = (const typename Act<G>::vt *)s->ahat64;
        vec = (const typename Act<G>::acc *)m->theta64;
    } else if constexpr (sizeof(G) == 4) {
        wc = m->pk_f32 + m->pf.Wcat0 + l * m->pf.Wcat_stride;
        ahat = (const typename Act<G>::vt *)s->ahat32;
        vec = (const typename Act<G>::acc *)m->theta32;
    } else {
        wc = m->pk_bf16 + m->pb.Wcat0 + l * m->pb.Wcat_stride;
        ahat = (const typename Act<G>::vt *)s->ahat16;
        vec = (const typename Act<G>::acc *)m->theta32;
    }
    hipLaunchKernelGGL((layer_kernel<G, D, H, false, float>(nrhs, s->max_row)), dim3(grid), dim3(BLOCK), 0, st, rows,
                       nrhs, s->rp, s->ci, ahat, (const G *)m->ws.act[0], (G *)m->ws.act[1], wc,
                       (const void *)nullptr, vec, m->po.c3, m->po.W4, m->po.c4,
                       (const double *)m->ws.tau, (float *)nullptr, (const int *)nullptr);
}

template <int D, int H>
static void layer_once_prec(gnp_model *m, int nrhs, gnp_precision prec, hipStream_t st) {
    if (prec == GNP_F64) layer_once<double, D, H>(m, nrhs, 0, st);
    else if (prec == GNP_F32) layer_once<float, D, H>(m, nrhs, 0, st);
    else layer_once<uint16_t, D, H>(m, nrhs, 0, st);
}

// Default initial weights (the paper leaves the initialisation open): each
// weight and bias uniform on +-1/sqrt(fan_in) of its linear map, parameter k
// from the uniform of Philox stream 3 at element k (philox.hpp).
static void default_init(int L, int d, int h, uint64_t seed, std::vector<double> &th) {
    const ParamOffsets po = param_offsets(L, d, h);
    th.resize(po.total);
    for (int64_t k = 0; k < po.total; ++k) {
        int fan;
        if (k < po.W2) fan = 1;           // W1, c1
        else if (k < po.U0) fan = h;      // W2, c2
        else if (k < po.W4) fan = d;      // U_l, W_l, W3, c3
        else fan = h;                     // W4, c4
        th[k] = (2.0 * uniform_at(seed, 0u, 3u, (uint64_t)k) - 1.0) / sqrt((double)fan);
    }
}

static void model_free(gnp_model *m) {
    if (!m) return;
    void *ptrs[] = {m->theta64, m->theta32, m->pk_bf16, m->pk_f32, m->ws.act[0], m->ws.act[1],
                    m->ws.tau, m->ws.partial, m->ws.counter};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    train_ctx_free(m->train_ctx);
    delete m;
}

// ---------------------------------------------------------------------------
// Scratch memory of gnp_apply_noalloc: a fixed array in device memory (one
// copy per GPU, held until the process ends) instead of the model's apply
// workspace, for callers that cannot allocate.  Layout for one call: the
// column-norm ticket counter, the tau triples, the column-norm partials, the
// two ping-pong activation blocks, each at a 256-byte boundary.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[GNP_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::unordered_map<int, unsigned char *> g_scratch_ptr;  // device -> address of its copy
}  // namespace

// Device address of this GPU's copy of `scratch` (looked up once per device,
// with that device current; the array's name is not a device address in
// host code).
static gnp_status scratch_address(unsigned char **out) {
    int dev = 0;
    GNP_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void *p = nullptr;
        GNP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        it = g_scratch_ptr.emplace(dev, (unsigned char *)p).first;
    }
    *out = it->second;
    return GNP_OK;
}

__global__ void k_zero_u32(unsigned *p, int count) {
    if ((int)threadIdx.x < count) p[threadIdx.x] = 0u;
}

static size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace gnp

using namespace gnp;

extern "C" {

gnp_status gnp_apply_noalloc(gnp_model *m, const void *v_dev, void *z_dev, int nrhs,
                             gnp_precision prec, void *hip_stream) {
    if (!m || !v_dev || !z_dev) return fail(GNP_EINVAL, "null argument");
    if (nrhs < 1 || nrhs > BLOCK) return fail(GNP_EINVAL, "nrhs must be in [1, 256]");
    if (!valid_precision(prec)) return fail(GNP_EINVAL, "bad precision");
    hipStream_t st = (hipStream_t)hip_stream;
    const int64_t n = m->sys->n;
    const size_t elem = prec == GNP_F64 ? 8 : (prec == GNP_F32 ? 4 : 2);
    const size_t o_tau = 256;
    const size_t o_part = o_tau + round256(sizeof(double) * 3 * (size_t)nrhs);
    const size_t o_act0 =
        o_part + round256(sizeof(double) * (size_t)colnorm_blocks(n) * (size_t)nrhs);
    const size_t act = round256((size_t)n * (size_t)nrhs * (size_t)m->d * elem);
    const size_t need = o_act0 + 2 * act;
    if (need > (size_t)GNP_NOALLOC_SCRATCH_BYTES)
        return fail(GNP_EINVAL, "this apply needs " + std::to_string(need) +
                                    " bytes of scratch; the no-allocation apply holds " +
                                    std::to_string((size_t)GNP_NOALLOC_SCRATCH_BYTES));
    unsigned char *base = nullptr;
    GNP_TRY(scratch_address(&base));
    unsigned *counter = (unsigned *)base;
    double *tau = (double *)(base + o_tau), *partial = (double *)(base + o_part);
    void *act0 = base + o_act0, *act1 = base + o_act0 + act;
    // the ticket counter must start at zero (an earlier call may have ended
    // early); a kernel, not a memset, so that the sequence can be captured
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, counter, 4);
    if (prec == GNP_F64)
        launch_colnorm<double>(m, (const double *)v_dev, nrhs, tau, partial, counter, nullptr,
                               st);
    else
        launch_colnorm<float>(m, (const float *)v_dev, nrhs, tau, partial, counter, nullptr, st);
    return forward_launch(m, prec, v_dev, z_dev, nrhs, tau, act0, act1, nullptr, st);
}


gnp_status gnp_model_create(gnp_system *sys, int L, int d, int h, const double *init_params,
                            uint64_t seed, gnp_model **out) {
    if (!out) return fail(GNP_EINVAL, "out is null");
    *out = nullptr;
    if (!sys) return fail(GNP_EINVAL, "sys is null");
    if (L < 1 || L > 64) return fail(GNP_EINVAL, "L must be in [1, 64]");
    if (!((d == 16 && h == 32) || (d == 32 && h == 64)))
        return fail(GNP_EINVAL, "supported (d, h): (16, 32), (32, 64)");
    std::vector<double> dflt;
    if (!init_params) {
        default_init(L, d, h, seed, dflt);
        init_params = dflt.data();
    }
    gnp_model *m = new gnp_model();
    m->sys = sys;
    m->L = L;
    m->d = d;
    m->h = h;
    m->po = param_offsets(L, d, h);
    m->np = m->po.total;
    for (int64_t k = 0; k < m->np; ++k)
        if (!std::isfinite(init_params[k])) {
            delete m;
            return fail(GNP_ENUMERIC, "non-finite initial parameter at " + std::to_string(k));
        }
    m->pb = pack_offsets(L, d, h, true);
    m->pf = pack_offsets(L, d, h, false);
    auto run = [&]() -> gnp_status {
        GNP_HIP(hipMalloc(&m->theta64, sizeof(double) * m->np));
        GNP_HIP(hipMalloc(&m->theta32, sizeof(float) * m->np));
        GNP_HIP(hipMalloc(&m->pk_bf16, sizeof(uint16_t) * m->pb.total));
        GNP_HIP(hipMalloc(&m->pk_f32, sizeof(float) * m->pf.total));
        GNP_HIP(hipMemcpy(m->theta64, init_params, sizeof(double) * m->np, hipMemcpyHostToDevice));
        GNP_TRY(model_repack(m, nullptr));
        GNP_HIP(hipStreamSynchronize(nullptr));
        return GNP_OK;
    };
    gnp_status rc = run();
    if (rc != GNP_OK) {
        model_free(m);
        return rc;
    }
    *out = m;
    return GNP_OK;
}

void gnp_model_destroy(gnp_model *model) { model_free(model); }

size_t gnp_model_nparams(const gnp_model *model) { return model ? (size_t)model->np : 0; }

gnp_status gnp_model_set_scaling(gnp_model *model, int on) {
    if (!model) return fail(GNP_EINVAL, "null argument");
    if (on != 0 && on != 1) return fail(GNP_EINVAL, "on must be 0 or 1");
    model->scaled = on;
    return GNP_OK;
}

gnp_status gnp_params_get(const gnp_model *m, double *buf, size_t count) {
    if (!m || !buf) return fail(GNP_EINVAL, "null argument");
    if (count != (size_t)m->np) return fail(GNP_EINVAL, "count must equal the parameter count");
    GNP_HIP(hipMemcpy(buf, m->theta64, sizeof(double) * m->np, hipMemcpyDeviceToHost));
    return GNP_OK;
}

gnp_status gnp_params_set(gnp_model *m, const double *buf, size_t count) {
    if (!m || !buf) return fail(GNP_EINVAL, "null argument");
    if (count != (size_t)m->np) return fail(GNP_EINVAL, "count must equal the parameter count");
    for (size_t k = 0; k < count; ++k)
        if (!std::isfinite(buf[k])) return fail(GNP_ENUMERIC, "non-finite parameter");
    GNP_HIP(hipDeviceSynchronize());
    GNP_HIP(hipMemcpy(m->theta64, buf, sizeof(double) * m->np, hipMemcpyHostToDevice));
    GNP_TRY(model_repack(m, nullptr));
    GNP_HIP(hipStreamSynchronize(nullptr));
    return GNP_OK;
}

gnp_status gnp_params_set_device(gnp_model *m, const double *buf_dev, size_t count,
                                 void *hip_stream) {
    if (!m || !buf_dev) return fail(GNP_EINVAL, "null argument");
    if (count != (size_t)m->np) return fail(GNP_EINVAL, "count must equal the parameter count");
    hipStream_t st = (hipStream_t)hip_stream;
    GNP_HIP(hipMemcpyAsync(m->theta64, buf_dev, sizeof(double) * m->np, hipMemcpyDeviceToDevice,
                           st));
    GNP_TRY(model_repack(m, st));
    return GNP_OK;
}

gnp_status gnp_time_layer(gnp_model *m, int nrhs, gnp_precision prec, int reps,
                          double *ms_per_launch, void *hip_stream) {
    if (!m || !ms_per_launch) return fail(GNP_EINVAL, "null argument");
    if (nrhs < 1 || nrhs > BLOCK || reps < 1) return fail(GNP_EINVAL, "bad nrhs or reps");
    if (!valid_precision(prec)) return fail(GNP_EINVAL, "bad precision");
    hipStream_t st = (hipStream_t)hip_stream;
    GNP_TRY(model_workspace(m, nrhs));
    hipEvent_t e0, e1;
    GNP_HIP(hipEventCreate(&e0));
    GNP_HIP(hipEventCreate(&e1));
    auto once = [&]() {
        if (m->d == 16) layer_once_prec<16, 32>(m, nrhs, prec, st);
        else layer_once_prec<32, 64>(m, nrhs, prec, st);
    };
    once();  // warm the instruction cache and the workspace
    GNP_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < reps; ++r) once();
    GNP_HIP(hipEventRecord(e1, st));
    GNP_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    GNP_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_per_launch = (double)ms / reps;
    return GNP_OK;
}

gnp_status gnp_time_layer_cold(gnp_model *m, int nrhs, gnp_precision prec, int reps,
                               void *flush_dev, size_t flush_bytes, double *ms_per_launch,
                               double *ms_flush, void *hip_stream) {
    if (!m || !flush_dev || !ms_per_launch) return fail(GNP_EINVAL, "null argument");
    if (nrhs < 1 || nrhs > BLOCK || reps < 1) return fail(GNP_EINVAL, "bad nrhs or reps");
    if (flush_bytes < 4) return fail(GNP_EINVAL, "flush_bytes must be >= 4");
    if (!valid_precision(prec)) return fail(GNP_EINVAL, "bad precision");
    hipStream_t st = (hipStream_t)hip_stream;
    GNP_TRY(model_workspace(m, nrhs));
    const int64_t nf = (int64_t)(flush_bytes / 4);
    auto layer = [&]() {
        if (m->d == 16) layer_once_prec<16, 32>(m, nrhs, prec, st);
        else layer_once_prec<32, 64>(m, nrhs, prec, st);
    };
    auto flush = [&](int r) {
        hipLaunchKernelGGL(k_fill_f32, dim3(2048), dim3(BLOCK), 0, st, (float *)flush_dev, nf,
                           (float)r);
    };
    hipEvent_t e0, e1, e2;
    GNP_HIP(hipEventCreate(&e0));
    GNP_HIP(hipEventCreate(&e1));
    GNP_HIP(hipEventCreate(&e2));
    flush(0);
    layer();  // instruction cache and workspace
    GNP_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < reps; ++r) {
        flush(r + 1);
        layer();
    }
    GNP_HIP(hipEventRecord(e1, st));
    for (int r = 0; r < reps; ++r) flush(reps + r + 1);
    GNP_HIP(hipEventRecord(e2, st));
    GNP_HIP(hipEventSynchronize(e2));
    float both = 0.f, fl = 0.f;
    GNP_HIP(hipEventElapsedTime(&both, e0, e1));
    GNP_HIP(hipEventElapsedTime(&fl, e1, e2));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipEventDestroy(e2);
    *ms_per_launch = (double)(both - fl) / reps;
    if (ms_flush) *ms_flush = (double)fl / reps;
    GNP_HIP(hipGetLastError());
    return GNP_OK;
}

gnp_status gnp_apply(gnp_model *m, const void *v_dev, void *z_dev, int nrhs, gnp_precision prec,
                     void *hip_stream) {
    if (!m || !v_dev || !z_dev) return fail(GNP_EINVAL, "null argument");
    if (nrhs < 1 || nrhs > BLOCK) return fail(GNP_EINVAL, "nrhs must be in [1, 256]");
    if (!valid_precision(prec)) return fail(GNP_EINVAL, "bad precision");
    hipStream_t st = (hipStream_t)hip_stream;
    GNP_TRY(model_workspace(m, nrhs));
    ApplyWorkspace &w = m->ws;
    if (prec == GNP_F64)
        launch_colnorm<double>(m, (const double *)v_dev, nrhs, w.tau, w.partial, w.counter,
                               nullptr, st);
    else
        launch_colnorm<float>(m, (const float *)v_dev, nrhs, w.tau, w.partial, w.counter, nullptr,
                              st);
    return forward_launch(m, prec, v_dev, z_dev, nrhs, w.tau, w.act[0], w.act[1], nullptr, st);
}

gnp_status gnp_apply_layers(gnp_model *m, const void *v_dev, void *z_dev, void *acts_dev,
                            int nrhs, gnp_precision prec, void *hip_stream) {
    if (!m || !v_dev || !z_dev || !acts_dev) return fail(GNP_EINVAL, "null argument");
    if (nrhs < 1 || nrhs > BLOCK) return fail(GNP_EINVAL, "nrhs must be in [1, 256]");
    if (!valid_precision(prec)) return fail(GNP_EINVAL, "bad precision");
    hipStream_t st = (hipStream_t)hip_stream;
    GNP_TRY(model_workspace(m, nrhs));
    ApplyWorkspace &w = m->ws;
    if (prec == GNP_F64)
        launch_colnorm<double>(m, (const double *)v_dev, nrhs, w.tau, w.partial, w.counter,
                               nullptr, st);
    else
        launch_colnorm<float>(m, (const float *)v_dev, nrhs, w.tau, w.partial, w.counter, nullptr,
                              st);
    return forward_launch(m, prec, v_dev, z_dev, nrhs, w.tau, w.act[0], w.act[1], nullptr, st,
                          acts_dev);
}

}  // extern "C"
