// Linear-system side of libgnp: CSR ingest and validation, gamma of Eq. (4)
// with the optional harness prescaling (Sec. 3), the transposed CSR built by a
// counting sort on the device, and the CSR SpMV.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "gnp_internal.hpp"
#include "spmv.hpp"

namespace gnp {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

gnp_status fail(gnp_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

gnp_status check_hip(hipError_t e, const char *what) {
    std::string m = std::string("HIP error '") + hipGetErrorString(e) + "' in " + what;
    g_err = m;
    return (e == hipErrorOutOfMemory) ? GNP_ENOMEM : GNP_EDEVICE;
}

// ---------------------------------------------------------------------------
// gamma (Eq. (4)): row sums in storage order, column sums as row sums of the
// transposed CSR (rows of A in increasing order), maxima by integer atomics
// on the bit patterns of non-negative doubles (order-independent, exact).
// ---------------------------------------------------------------------------
__global__ void k_abs_rowsum_max(int64_t n, const int32_t *__restrict__ rp,
                                 const double *__restrict__ val, unsigned long long *out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (i < n) {
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) s += fabs(val[k]);
    }
    // block max, then one atomic per block
    unsigned long long b = (unsigned long long)__double_as_longlong(s);
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        unsigned long long t = __shfl_xor(b, o, WAVE);
        b = t > b ? t : b;
    }
    if ((threadIdx.x % WAVE) == 0) atomicMax(out, b);
}

__global__ void k_gamma_finish(const unsigned long long *rowmax, const unsigned long long *colmax,
                               double *gamma) {
    double r = __longlong_as_double((long long)*rowmax);
    double c = __longlong_as_double((long long)*colmax);
    *gamma = r < c ? r : c;
}

__global__ void k_div(int64_t nnz, const double *__restrict__ v, const double *__restrict__ g,
                      double *__restrict__ out64, float *__restrict__ out32) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nnz) {
        double q = v[k] / *g;
        out64[k] = q;
        if (out32) out32[k] = (float)q;
    }
}

__global__ void k_to_f32(int64_t nnz, const double *__restrict__ v, float *__restrict__ out) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nnz) out[k] = (float)v[k];
}

// ---------------------------------------------------------------------------
// transpose by counting sort
// ---------------------------------------------------------------------------
__global__ void k_count_cols(int64_t nnz, const int32_t *__restrict__ ci, int32_t *cnt) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nnz) atomicAdd(&cnt[ci[k] + 1], 1);
}

// exclusive scan helpers: per-block inclusive scan of 4 elements per thread
constexpr int SCAN_PER_BLOCK = BLOCK * 4;

__global__ void k_scan_blocks(int64_t len, int32_t *data, int32_t *block_sums) {
    __shared__ int32_t s[BLOCK];
    int64_t base = (int64_t)blockIdx.x * SCAN_PER_BLOCK + threadIdx.x * 4;
    int32_t v[4];
    int32_t run = 0;
    for (int q = 0; q < 4; ++q) {
        int64_t idx = base + q;
        int32_t x = idx < len ? data[idx] : 0;
        run += x;
        v[q] = run;
    }
    s[threadIdx.x] = run;
    __syncthreads();
    for (int off = 1; off < BLOCK; off <<= 1) {
        int32_t t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    int32_t prefix = threadIdx.x > 0 ? s[threadIdx.x - 1] : 0;
    for (int q = 0; q < 4; ++q) {
        int64_t idx = base + q;
        if (idx < len) data[idx] = v[q] + prefix;
    }
    if (threadIdx.x == BLOCK - 1) block_sums[blockIdx.x] = s[BLOCK - 1];
}

__global__ void k_scan_add(int64_t len, int32_t *data, const int32_t *block_offsets) {
    int64_t base = (int64_t)blockIdx.x * SCAN_PER_BLOCK;
    int32_t off = block_offsets[blockIdx.x];
    for (int q = threadIdx.x; q < SCAN_PER_BLOCK; q += BLOCK) {
        int64_t idx = base + q;
        if (idx < len) data[idx] += off;
    }
}

// in-place inclusive scan of len int32 values on the device (recursive over
// block sums); tmp must hold enough room for the block-sum levels.
static gnp_status scan_inclusive(int32_t *data, int64_t len, int32_t *tmp, hipStream_t st) {
    int nb = grid_for(len, SCAN_PER_BLOCK);
    hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(BLOCK), 0, st, len, data, tmp);
    if (nb > 1) {
        GNP_TRY(scan_inclusive(tmp, nb, tmp + nb, st));
        // tmp now holds inclusive sums of blocks; block b needs tmp[b-1]
        hipLaunchKernelGGL(k_scan_add, dim3(nb - 1), dim3(BLOCK), 0, st, len - SCAN_PER_BLOCK,
                           data + SCAN_PER_BLOCK, tmp);
    }
    GNP_HIP(hipGetLastError());
    return GNP_OK;
}

__global__ void k_fill_transpose(int64_t n, const int32_t *__restrict__ rp,
                                 const int32_t *__restrict__ ci, int32_t *cursor,
                                 int32_t *__restrict__ trow, int32_t *__restrict__ tperm) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
        int32_t pos = atomicAdd(&cursor[ci[k]], 1);
        trow[pos] = (int32_t)i;
        tperm[pos] = k;
    }
}

// sort each column segment by row index (insertion sort; segments are short)
__global__ void k_sort_segments(int64_t n, const int32_t *__restrict__ trp, int32_t *trow,
                                int32_t *tperm) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int32_t a = trp[j], b = trp[j + 1];
    for (int32_t p = a + 1; p < b; ++p) {
        int32_t r = trow[p], q = tperm[p];
        int32_t s = p - 1;
        while (s >= a && trow[s] > r) {
            trow[s + 1] = trow[s];
            tperm[s + 1] = tperm[s];
            --s;
        }
        trow[s + 1] = r;
        tperm[s + 1] = q;
    }
}

__global__ void k_gather(int64_t nnz, const int32_t *__restrict__ perm,
                         const double *__restrict__ src, double *__restrict__ dst64,
                         float *__restrict__ dst32) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nnz) {
        double v = src[perm[k]];
        dst64[k] = v;
        dst32[k] = (float)v;
    }
}

__global__ void k_to_bf16(int64_t count, const float *__restrict__ src, uint16_t *__restrict__ dst) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) dst[k] = __builtin_bit_cast(uint16_t, (__bf16)src[k]);  // round to nearest even
}

static void sys_free(gnp_system *s) {
    if (!s) return;
    void *ptrs[] = {s->rp,     s->ci,      s->val64,  s->val32,   s->ahat64,  s->ahat32,
                    s->trp,    s->tci,     s->tval64, s->tval32,  s->tahat64, s->tahat32,
                    s->ahat16,   s->counters, s->scratch, s->dinv64, s->tperm};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    solve_cache_free(s->solve_cache);
    batch_cache_free(s->batch_cache);
    delete s;
}

template <typename T> static gnp_status dalloc(T **p, int64_t count) {
    size_t bytes = sizeof(T) * (size_t)(count > 0 ? count : 1);
    hipError_t e = hipMalloc((void **)p, bytes);
    if (e != hipSuccess) return check_hip(e, "hipMalloc");
    return GNP_OK;
}

static gnp_status validate_csr(int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci,
                               const double *val, int *max_row) {
    if (n < 1) return fail(GNP_EINVAL, "n must be >= 1");
    if (nnz < 1) return fail(GNP_EINVAL, "nnz must be >= 1");
    if (n >= (int64_t)INT32_MAX || nnz >= (int64_t)INT32_MAX)
        return fail(GNP_EINVAL, "n and nnz must be below 2^31 - 1");
    if (!rp || !ci || !val) return fail(GNP_EINVAL, "null CSR array");
    if (rp[0] != 0) return fail(GNP_EINVAL, "rowptr[0] must be 0");
    if ((int64_t)rp[n] != nnz) return fail(GNP_EINVAL, "rowptr[n] must equal nnz");
    int mr = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t a = rp[i], b = rp[i + 1];
        if (b < a) return fail(GNP_EINVAL, "rowptr must be non-decreasing (row " +
                                               std::to_string(i) + ")");
        if (b - a > mr) mr = b - a;
        for (int32_t k = a; k < b; ++k) {
            if (ci[k] < 0 || (int64_t)ci[k] >= n)
                return fail(GNP_EINVAL, "column index out of range at nnz " + std::to_string(k));
            if (k > a && ci[k] <= ci[k - 1])
                return fail(GNP_EINVAL, "columns must be strictly increasing within row " +
                                            std::to_string(i));
            if (!std::isfinite(val[k]))
                return fail(GNP_EINVAL, "non-finite value at nnz " + std::to_string(k));
        }
    }
    *max_row = mr;
    return GNP_OK;
}

// Finite values, and finite, nonzero absolute row and column sums (so that
// gamma of the input and of the prescaled matrix is finite and positive).
static gnp_status validate_values(int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci,
                                  const double *val) {
    if (!val) return fail(GNP_EINVAL, "null value array");
    std::vector<double> col(n, 0.0);
    double rmax = 0.0, cmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double r = 0.0;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            if (!std::isfinite(val[k]))
                return fail(GNP_EINVAL, "non-finite value at nnz " + std::to_string(k));
            r += fabs(val[k]);
            col[ci[k]] += fabs(val[k]);
        }
        rmax = r > rmax ? r : rmax;
    }
    for (int64_t j = 0; j < n; ++j) cmax = col[j] > cmax ? col[j] : cmax;
    (void)nnz;
    if (!(rmax > 0.0) || !std::isfinite(rmax) || !std::isfinite(cmax))
        return fail(GNP_EINVAL, "gamma is zero or not finite (all-zero matrix?)");
    return GNP_OK;
}

static gnp_status gamma_dev(gnp_system *s, const double *val, double *g_dev,
                            unsigned long long *maxes, hipStream_t st) {
    GNP_HIP(hipMemsetAsync(maxes, 0, 2 * sizeof(unsigned long long), st));
    hipLaunchKernelGGL(k_abs_rowsum_max, dim3(grid_for(s->n, BLOCK)), dim3(BLOCK), 0, st, s->n,
                       s->rp, val, maxes);
    // column sums are the row sums of A^T, whose values are gathered from val
    hipLaunchKernelGGL(k_abs_rowsum_max, dim3(grid_for(s->n, BLOCK)), dim3(BLOCK), 0, st, s->n,
                       s->trp, s->tval64, maxes + 1);
    hipLaunchKernelGGL(k_gamma_finish, dim3(1), dim3(1), 0, st, maxes, maxes + 1, g_dev);
    GNP_HIP(hipGetLastError());
    return GNP_OK;
}

}  // namespace gnp

using namespace gnp;

extern "C" {

const char *gnp_last_error(void) { return g_err.c_str(); }

const char *gnp_version(void) { return "libgnp 0.1 (gfx950)"; }

}  // extern "C"

namespace gnp {
// Everything on the device that follows from the values (input values on
// the device in tmp64, the transposed pattern already built): gamma of the
// input, the (prescaled) A and its transpose in float64/float32, gamma of
// that matrix, A-hat in three precisions and its transpose.  gam: 2
// doubles, maxes: 2 words of device scratch.  Waits for the stream.
static gnp_status derive_values(gnp_system *s, double *tmp64, double *gam,
                                unsigned long long *maxes, hipStream_t st) {
    const int64_t nnz = s->nnz;
    const int gk = grid_for(nnz, BLOCK);
    hipLaunchKernelGGL(k_gather, dim3(gk), dim3(BLOCK), 0, st, nnz, s->tperm, tmp64, s->tval64,
                       s->tval32);
    GNP_TRY(gamma_dev(s, tmp64, gam, maxes, st));
    if (s->prescale) {
        hipLaunchKernelGGL(k_div, dim3(gk), dim3(BLOCK), 0, st, nnz, tmp64, gam, s->val64,
                           s->val32);
        hipLaunchKernelGGL(k_gather, dim3(gk), dim3(BLOCK), 0, st, nnz, s->tperm, s->val64,
                           s->tval64, s->tval32);
        GNP_TRY(gamma_dev(s, s->val64, gam + 1, maxes, st));
    } else {
        GNP_HIP(hipMemcpyAsync(s->val64, tmp64, sizeof(double) * nnz, hipMemcpyDeviceToDevice,
                               st));
        hipLaunchKernelGGL(k_to_f32, dim3(gk), dim3(BLOCK), 0, st, nnz, s->val64, s->val32);
        GNP_HIP(hipMemcpyAsync(gam + 1, gam, sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    // A-hat = A / gamma and its transpose
    hipLaunchKernelGGL(k_div, dim3(gk), dim3(BLOCK), 0, st, nnz, s->val64, gam + 1, s->ahat64,
                       s->ahat32);
    hipLaunchKernelGGL(k_to_bf16, dim3(gk), dim3(BLOCK), 0, st, nnz, (const float *)s->ahat32,
                       s->ahat16);
    hipLaunchKernelGGL(k_gather, dim3(gk), dim3(BLOCK), 0, st, nnz, s->tperm, s->ahat64,
                       s->tahat64, s->tahat32);
    GNP_HIP(hipGetLastError());
    double gh[2];
    GNP_HIP(hipMemcpyAsync(gh, gam, sizeof(gh), hipMemcpyDeviceToHost, st));
    GNP_HIP(hipStreamSynchronize(st));
    s->gamma_raw = gh[0];
    s->gamma = gh[1];
    if (!(gh[0] > 0.0) || !(gh[1] > 0.0) || !std::isfinite(gh[1]))
        return fail(GNP_EINVAL, "gamma is zero or not finite (all-zero matrix?)");
    return GNP_OK;
}
}  // namespace gnp

extern "C" {

gnp_status gnp_system_create(int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *colind,
                             const double *val, int prescale, void *hip_stream,
                             gnp_system **out) {
    if (!out) return fail(GNP_EINVAL, "out is null");
    *out = nullptr;
    int max_row = 0;
    GNP_TRY(validate_csr(n, nnz, rowptr, colind, val, &max_row));
    GNP_TRY(validate_values(n, nnz, rowptr, colind, val));
    hipStream_t st = (hipStream_t)hip_stream;
    gnp_system *s = new gnp_system();
    s->n = n;
    s->nnz = nnz;
    s->max_row = max_row;
    s->prescale = prescale ? 1 : 0;
    int32_t *cnt = nullptr, *scan_tmp = nullptr;
    double *tmp64 = nullptr, *gam = nullptr;
    unsigned long long *maxes = nullptr;
    gnp_status rc = GNP_OK;
    auto run = [&]() -> gnp_status {
        GNP_TRY(dalloc(&s->rp, n + 1));
        GNP_TRY(dalloc(&s->ci, nnz));
        GNP_TRY(dalloc(&s->val64, nnz));
        GNP_TRY(dalloc(&s->val32, nnz));
        GNP_TRY(dalloc(&s->ahat64, nnz));
        GNP_TRY(dalloc(&s->ahat32, nnz));
        GNP_TRY(dalloc(&s->ahat16, nnz));
        GNP_TRY(dalloc(&s->trp, n + 1));
        GNP_TRY(dalloc(&s->tci, nnz));
        GNP_TRY(dalloc(&s->tval64, nnz));
        GNP_TRY(dalloc(&s->tval32, nnz));
        GNP_TRY(dalloc(&s->tahat64, nnz));
        GNP_TRY(dalloc(&s->tahat32, nnz));
        GNP_TRY(dalloc(&s->counters, 64));
        s->nscratch = 4096;
        GNP_TRY(dalloc(&s->scratch, s->nscratch));
        GNP_TRY(dalloc(&cnt, n + 1));
        GNP_TRY(dalloc(&s->tperm, nnz));
        GNP_TRY(dalloc(&scan_tmp, 2 * (n / SCAN_PER_BLOCK + 16)));
        GNP_TRY(dalloc(&tmp64, nnz));
        GNP_TRY(dalloc(&gam, 2));
        GNP_TRY(dalloc(&maxes, 2));
        GNP_HIP(hipMemsetAsync(s->counters, 0, 64 * sizeof(unsigned), st));
        GNP_HIP(hipMemcpyAsync(s->rp, rowptr, sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, st));
        GNP_HIP(hipMemcpyAsync(s->ci, colind, sizeof(int32_t) * nnz, hipMemcpyHostToDevice, st));
        GNP_HIP(hipMemcpyAsync(tmp64, val, sizeof(double) * nnz, hipMemcpyHostToDevice, st));
        // transposed pattern: count, scan, fill, sort each column by row
        GNP_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (n + 1), st));
        const int gk = grid_for(nnz, BLOCK), gn = grid_for(n, BLOCK);
        hipLaunchKernelGGL(k_count_cols, dim3(gk), dim3(BLOCK), 0, st, nnz, s->ci, cnt);
        GNP_TRY(scan_inclusive(cnt, n + 1, scan_tmp, st));
        GNP_HIP(hipMemcpyAsync(s->trp, cnt, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL(k_fill_transpose, dim3(gn), dim3(BLOCK), 0, st, n, s->rp, s->ci, cnt,
                           s->tci, s->tperm);
        hipLaunchKernelGGL(k_sort_segments, dim3(gn), dim3(BLOCK), 0, st, n, s->trp, s->tci,
                           s->tperm);
        return derive_values(s, tmp64, gam, maxes, st);
    };
    rc = run();
    void *tmps[] = {cnt, scan_tmp, tmp64, gam, maxes};
    for (void *p : tmps)
        if (p) (void)hipFree(p);
    if (rc != GNP_OK) {
        sys_free(s);
        return rc;
    }
    *out = s;
    return GNP_OK;
}

gnp_status gnp_system_set_values(gnp_system *sys, const double *val, void *hip_stream) {
    if (!sys) return fail(GNP_EINVAL, "null system");
    std::vector<int32_t> rp(sys->n + 1), ci(sys->nnz);
    GNP_HIP(hipMemcpy(rp.data(), sys->rp, sizeof(int32_t) * rp.size(), hipMemcpyDeviceToHost));
    GNP_HIP(hipMemcpy(ci.data(), sys->ci, sizeof(int32_t) * ci.size(), hipMemcpyDeviceToHost));
    GNP_TRY(validate_values(sys->n, sys->nnz, rp.data(), ci.data(), val));
    hipStream_t st = (hipStream_t)hip_stream;
    double *tmp64 = nullptr, *gam = nullptr;
    unsigned long long *maxes = nullptr;
    auto run = [&]() -> gnp_status {
        GNP_TRY(dalloc(&tmp64, sys->nnz));
        GNP_TRY(dalloc(&gam, 2));
        GNP_TRY(dalloc(&maxes, 2));
        GNP_HIP(hipMemcpyAsync(tmp64, val, sizeof(double) * sys->nnz, hipMemcpyHostToDevice, st));
        if (sys->dinv64) {  // the Jacobi diagonal is made again on its next use
            GNP_HIP(hipStreamSynchronize(st));
            GNP_HIP(hipFree(sys->dinv64));
            sys->dinv64 = nullptr;
        }
        return derive_values(sys, tmp64, gam, maxes, st);
    };
    const gnp_status rc = run();
    void *tmps[] = {tmp64, gam, maxes};
    for (void *p : tmps)
        if (p) (void)hipFree(p);
    return rc;
}

void gnp_system_destroy(gnp_system *sys) { sys_free(sys); }

gnp_status gnp_system_gamma(const gnp_system *sys, double *gamma_input, double *gamma_system) {
    if (!sys) return fail(GNP_EINVAL, "sys is null");
    if (gamma_input) *gamma_input = sys->gamma_raw;
    if (gamma_system) *gamma_system = sys->gamma;
    return GNP_OK;
}

int64_t gnp_system_n(const gnp_system *sys) { return sys ? sys->n : -1; }
int64_t gnp_system_nnz(const gnp_system *sys) { return sys ? sys->nnz : -1; }

gnp_status gnp_system_export(const gnp_system *sys, double *val, double *ahat, int32_t *t_rowptr,
                             int32_t *t_colind, double *t_val) {
    if (!sys) return fail(GNP_EINVAL, "sys is null");
    const int64_t n = sys->n, nnz = sys->nnz;
    if (val) GNP_HIP(hipMemcpy(val, sys->val64, sizeof(double) * nnz, hipMemcpyDeviceToHost));
    if (ahat) GNP_HIP(hipMemcpy(ahat, sys->ahat64, sizeof(double) * nnz, hipMemcpyDeviceToHost));
    if (t_rowptr)
        GNP_HIP(hipMemcpy(t_rowptr, sys->trp, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
    if (t_colind)
        GNP_HIP(hipMemcpy(t_colind, sys->tci, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
    if (t_val) GNP_HIP(hipMemcpy(t_val, sys->tval64, sizeof(double) * nnz, hipMemcpyDeviceToHost));
    return GNP_OK;
}

gnp_status gnp_spmv(const gnp_system *sys, const void *x_dev, void *y_dev, gnp_precision prec,
                    void *hip_stream) {
    if (!sys || !x_dev || !y_dev) return fail(GNP_EINVAL, "null argument");
    if (!valid_precision(prec)) return fail(GNP_EINVAL, "bad precision");
    hipStream_t st = (hipStream_t)hip_stream;
    if (prec == GNP_F64)
        spmv_launch<double, double, double>(sys->n, sys->rp, sys->ci, sys->val64,
                                            (const double *)x_dev, (double *)y_dev, nullptr,
                                            nullptr, sys->nnz, st, 1, 1, 0, 0, sys->max_row);
    else
        spmv_launch<float, float, float>(sys->n, sys->rp, sys->ci, sys->val32,
                                         (const float *)x_dev, (float *)y_dev, nullptr,
                                         nullptr, sys->nnz, st, 1, 1, 0, 0, sys->max_row);
    GNP_HIP(hipGetLastError());
    return GNP_OK;
}

}  // extern "C"

extern "C" gnp_status gnp_time_spmv(const gnp_system *sys, const void *x_dev, void *y_dev,
                                    gnp_precision prec, int reps, double *ms_per_launch,
                                    void *hip_stream) {
    if (!sys || !x_dev || !y_dev || !ms_per_launch || reps < 1)
        return fail(GNP_EINVAL, "bad argument");
    hipStream_t st = (hipStream_t)hip_stream;
    hipEvent_t e0, e1;
    GNP_HIP(hipEventCreate(&e0));
    GNP_HIP(hipEventCreate(&e1));
    GNP_TRY(gnp_spmv(sys, x_dev, y_dev, prec, hip_stream));
    GNP_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < reps; ++r) GNP_TRY(gnp_spmv(sys, x_dev, y_dev, prec, hip_stream));
    GNP_HIP(hipEventRecord(e1, st));
    GNP_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    GNP_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_per_launch = (double)ms / reps;
    return GNP_OK;
}
