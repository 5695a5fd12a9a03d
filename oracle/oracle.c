/*
 * FP64 CPU oracle for graph-neural-preconditioned FGMRES.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may call,
 * link or load this file; it exists so that the tests, the smoke check and the
 * CPU baseline of the benchmark can compare the HIP path against a plain,
 * slow, obviously correct implementation written from the paper
 * (Chen, "Graph Neural Preconditioners for Iterative Solutions of Sparse
 * Linear Systems", ICLR 2025).  It shares no code, header or constant with the
 * HIP library.
 *
 * Everything is IEEE double.  Every reduction is a single sequential sum in
 * index order, so results do not depend on the OpenMP thread count; OpenMP is
 * used only across independent rows.
 *
 * Readings of points the paper leaves open (stated once here, used below):
 *  - stopping: converged iff the true ||b - A x||_2 <= rtol * ||b||_2; the
 *    Givens estimate is checked after every Arnoldi step and ends a cycle
 *    early, the true residual confirms it (Sec. 3 "Stopping criteria" and the
 *    robustness discussion in Sec. 4 that tracks the residual through the QR
 *    factorisation of the Hessenberg matrix).
 *  - one "iteration" is one Arnoldi step (one application of M), counted
 *    across restarts.
 *  - breakdown: if h_{j+1,j} <= 1e-14 * ||A z_j|| the cycle ends at step j.
 *  - network: MLP = Lin -> ReLU -> Lin with biases; Res-GCONV has no bias and
 *    is followed by ReLU in every layer; no activation at the encoder output
 *    or at the decoder output; tau = ||b||_2 in FP64; b = 0 maps to 0.
 *  - loss: mean over the n*B entries of |A M(b) - b|; sign(0) = 0 and
 *    ReLU'(0) = 0.
 *  - Adam: beta1 0.9, beta2 0.999, eps 1e-8 with bias correction; the model
 *    kept is the one with the smallest minibatch loss, earliest on ties.
 *
 * Parameter packing (input index first, y = x M, row-major):
 *   W1[1 x h] c1[h] W2[h x d] c2[d] | L x (U_l[d x d] W_l[d x d]) |
 *   W3[d x h] c3[h] W4[h x 1] c4[1]
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_API __attribute__((visibility("default")))

#ifdef _OPENMP
#include <omp.h>
#endif

/* Number of OpenMP threads the oracle's parallel loops use. */
OR_API int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set that number (timing with one thread and with all of them); results do
   not depend on it (fixed-size chunks, summed in index order). */
OR_API void or_set_num_threads(int k)
{
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

/* ------------------------------------------------------------------------ */
/* Sparse matrix basics                                                     */
/* ------------------------------------------------------------------------ */

/* y = A x for B right-hand sides stored node-major: x[j*B + b]. */
OR_API void or_spmm(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                    int B, const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int b = 0; b < B; ++b) {
            double s = 0.0;
            for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
                s += v[k] * x[(int64_t)ci[k] * B + b];
            y[i * B + b] = s;
        }
    }
}

/* Eq. (4): gamma = min( max_i sum_j |a_ij| , max_j sum_i |a_ij| ).
 * Row sums run over the row in storage order; column sums accumulate in
 * increasing row order. */
OR_API double or_gamma(int64_t n, const int32_t *rp, const int32_t *ci, const double *v)
{
    double *colsum = (double *)calloc((size_t)n, sizeof(double));
    double rmax = 0.0, cmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            s += fabs(v[k]);
            colsum[ci[k]] += fabs(v[k]);
        }
        if (s > rmax) rmax = s;
    }
    for (int64_t j = 0; j < n; ++j)
        if (colsum[j] > cmax) cmax = colsum[j];
    free(colsum);
    return rmax < cmax ? rmax : cmax;
}

/* out = v / s elementwise (A-hat = A / gamma, Eq. (4); harness prescale). */
OR_API void or_scale(int64_t nnz, const double *v, double s, double *out)
{
    for (int64_t k = 0; k < nnz; ++k) out[k] = v[k] / s;
}

/* CSR of A^T by counting sort; within a column, rows stay in increasing order. */
OR_API void or_transpose(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                         int32_t *trp, int32_t *tci, double *tv)
{
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t k = 0; k < rp[n]; ++k) cnt[ci[k] + 1] += 1;
    for (int64_t j = 0; j < n; ++j) cnt[j + 1] += cnt[j];
    for (int64_t j = 0; j <= n; ++j) trp[j] = (int32_t)cnt[j];
    for (int64_t i = 0; i < n; ++i) {
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            int64_t pos = cnt[ci[k]]++;
            tci[pos] = (int32_t)i;
            tv[pos] = v[k];
        }
    }
    free(cnt);
}

static double dot_seq(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static double nrm2_seq(int64_t n, const double *a) { return sqrt(dot_seq(n, a, a)); }

/* ------------------------------------------------------------------------ */
/* Graph neural preconditioner, Sec. 2.3                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    const double *W1, *c1, *W2, *c2, *W3, *c3, *W4, *c4;
    const double *U[64], *W[64];
} gnp_view;

static int64_t gnp_nparams(int L, int d, int h)
{
    return (int64_t)h + h + (int64_t)h * d + d + (int64_t)L * 2 * d * d + (int64_t)d * h + h + h + 1;
}

OR_API int64_t or_gnp_nparams(int L, int d, int h) { return gnp_nparams(L, d, h); }

static void gnp_unpack(const double *th, int L, int d, int h, gnp_view *g)
{
    const double *p = th;
    g->W1 = p; p += h;
    g->c1 = p; p += h;
    g->W2 = p; p += (int64_t)h * d;
    g->c2 = p; p += d;
    for (int l = 0; l < L; ++l) {
        g->U[l] = p; p += (int64_t)d * d;
        g->W[l] = p; p += (int64_t)d * d;
    }
    g->W3 = p; p += (int64_t)d * h;
    g->c3 = p; p += h;
    g->W4 = p; p += h;
    g->c4 = p;
}

/* Saved intermediates of one forward pass (rows are (node, rhs) pairs,
 * r = i*B + b).  X[l] is the input of layer l (X[0] = encoder output,
 * X[L] = input of the decoder); T[l] = A-hat X[l]. */
typedef struct {
    int64_t rows;
    double *tau, *si, *so;  /* per rhs: ||b||, sqrt(n)/tau, tau/sqrt(n) */
    double *u;              /* rows: scaled input s(b) */
    double *pre1;           /* rows x h: u W1 + c1 */
    double **X;             /* L+1 arrays of rows x d */
    double **T;             /* L arrays of rows x d */
    double *pre3;           /* rows x h: X_L W3 + c3 */
    double *o;              /* rows: decoder output before s^{-1} */
} fwd_state;

static void fwd_alloc(fwd_state *s, int64_t n, int B, int L, int d, int h)
{
    int64_t rows = n * B;
    s->rows = rows;
    s->tau = (double *)malloc(sizeof(double) * B);
    s->si = (double *)malloc(sizeof(double) * B);
    s->so = (double *)malloc(sizeof(double) * B);
    s->u = (double *)malloc(sizeof(double) * rows);
    s->pre1 = (double *)malloc(sizeof(double) * rows * h);
    s->X = (double **)malloc(sizeof(double *) * (L + 1));
    s->T = (double **)malloc(sizeof(double *) * (L > 0 ? L : 1));
    for (int l = 0; l <= L; ++l) s->X[l] = (double *)malloc(sizeof(double) * rows * d);
    for (int l = 0; l < L; ++l) s->T[l] = (double *)malloc(sizeof(double) * rows * d);
    s->pre3 = (double *)malloc(sizeof(double) * rows * h);
    s->o = (double *)malloc(sizeof(double) * rows);
}

static void fwd_free(fwd_state *s, int L)
{
    free(s->tau); free(s->si); free(s->so); free(s->u); free(s->pre1);
    for (int l = 0; l <= L; ++l) free(s->X[l]);
    for (int l = 0; l < L; ++l) free(s->T[l]);
    free(s->X); free(s->T); free(s->pre3); free(s->o);
}

static double relu(double x) { return x > 0.0 ? x : 0.0; }

/* 0: the network without the scaling of Eq. (6), s = s^-1 = identity (the
 * ablation of Sec. 3 that asks whether scale equivariance is needed); it
 * applies to every forward pass, loss, gradient, training run and solve. */
static int g_scaled = 1;
OR_API void or_set_scaling(int on) { g_scaled = on ? 1 : 0; }

/* s(b) of Eq. (6) per right-hand side: tau = ||b||_2, the input factor
 * sqrt(n)/tau (0 for b = 0) and the output factor tau/sqrt(n). */
static void scale_factors(int64_t n, int B, const double *bin, double *tau, double *si, double *so)
{
    const double sqn = sqrt((double)n);
    for (int b = 0; b < B; ++b) {
        double ss = 0.0;
        for (int64_t i = 0; i < n; ++i) ss += bin[i * B + b] * bin[i * B + b];
        double t = sqrt(ss);
        if (tau) tau[b] = t;
        si[b] = g_scaled ? (t > 0.0 ? sqn / t : 0.0) : 1.0;
        so[b] = g_scaled ? t / sqn : 1.0;
    }
}

/* MLP encoder of Sec. 2.3 on the scaled input, row by row:
 * u = si * b, E = ReLU(u W1 + c1) W2 + c2 (pre1 keeps u W1 + c1). */
static void encoder_rows(int64_t rows, int B, int d, int h, const gnp_view *g, const double *si,
                         const double *bin, double *u_out, double *pre1, double *E_out)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < rows; ++r) {
        double u = si[r % B] * bin[r];
        u_out[r] = u;
        double *p1 = pre1 + r * h;
        for (int k = 0; k < h; ++k) p1[k] = u * g->W1[k] + g->c1[k];
        double *E = E_out + r * d;
        for (int f = 0; f < d; ++f) {
            double acc = 0.0;
            for (int k = 0; k < h; ++k) acc += relu(p1[k]) * g->W2[(int64_t)k * d + f];
            E[f] = acc + g->c2[f];
        }
    }
}

/* One Res-GCONV layer, Eq. (5): T = A-hat X, Y = ReLU(X U + T W), for B
 * right-hand sides (rows r = i*B + b, d features each). */
static void layer_rows(int64_t n, const int32_t *rp, const int32_t *ci, const double *ahat, int B,
                       int d, const double *U, const double *W, const double *X, double *T,
                       double *Y)
{
    const int64_t rows = n * B;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int b = 0; b < B; ++b) {
            double *Tr = T + (i * B + b) * d;
            for (int f = 0; f < d; ++f) {
                double acc = 0.0;
                for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
                    acc += ahat[k] * X[((int64_t)ci[k] * B + b) * d + f];
                Tr[f] = acc;
            }
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < rows; ++r) {
        const double *Xr = X + r * d, *Tr = T + r * d;
        for (int q = 0; q < d; ++q) {
            double acc = 0.0;
            for (int p = 0; p < d; ++p) acc += Xr[p] * U[(int64_t)p * d + q];
            for (int p = 0; p < d; ++p) acc += Tr[p] * W[(int64_t)p * d + q];
            Y[r * d + q] = relu(acc);
        }
    }
}

/* MLP decoder and s^-1 of Eq. (6), row by row: o = ReLU(X_L W3 + c3) W4 + c4,
 * z = so * o (pre3 keeps X_L W3 + c3). */
static void decoder_rows(int64_t rows, int B, int d, int h, const gnp_view *g, const double *so,
                         const double *XL, double *pre3, double *o_out, double *z)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < rows; ++r) {
        double *p3 = pre3 + r * h;
        for (int k = 0; k < h; ++k) {
            double acc = 0.0;
            for (int f = 0; f < d; ++f) acc += XL[r * d + f] * g->W3[(int64_t)f * h + k];
            p3[k] = acc + g->c3[k];
        }
        double acc = 0.0;
        for (int k = 0; k < h; ++k) acc += relu(p3[k]) * g->W4[k];
        o_out[r] = acc + g->c4[0];
        z[r] = so[r % B] * o_out[r];
    }
}

/* Forward pass: Eq. (6) scaling, MLP encoder, L Res-GCONV layers (Eq. (5))
 * with A-hat from Eq. (4), MLP decoder, back-scaling. */
static void gnp_forward_state(int64_t n, const int32_t *rp, const int32_t *ci, const double *ahat,
                              int L, int d, int h, const double *theta, int B,
                              const double *bin, double *z, fwd_state *s)
{
    gnp_view g;
    gnp_unpack(theta, L, d, h, &g);
    const int64_t rows = n * B;
    scale_factors(n, B, bin, s->tau, s->si, s->so);
    encoder_rows(rows, B, d, h, &g, s->si, bin, s->u, s->pre1, s->X[0]);
    for (int l = 0; l < L; ++l)
        layer_rows(n, rp, ci, ahat, B, d, g.U[l], g.W[l], s->X[l], s->T[l], s->X[l + 1]);
    decoder_rows(rows, B, d, h, &g, s->so, s->X[L], s->pre3, s->o, z);
}

/* The three stages of the forward pass one at a time (the same functions as
 * or_gnp_forward runs), so that one stage can be evaluated on inputs taken
 * from elsewhere.  Encoder (with the s(b) of Eq. (6)): E = X_0 for b
 * ([n][B]); layer l of Eq. (5): Y = X_{l+1} from X = X_l; decoder with
 * s^-1 of Eq. (6): z from X_L, tau taken from b. */
OR_API void or_gnp_encoder(int64_t n, int L, int d, int h, const double *theta, int B,
                           const double *bin, double *E)
{
    gnp_view g;
    gnp_unpack(theta, L, d, h, &g);
    const int64_t rows = n * B;
    double *si = (double *)malloc(sizeof(double) * B), *so = (double *)malloc(sizeof(double) * B);
    double *u = (double *)malloc(sizeof(double) * rows);
    double *pre1 = (double *)malloc(sizeof(double) * rows * h);
    scale_factors(n, B, bin, NULL, si, so);
    encoder_rows(rows, B, d, h, &g, si, bin, u, pre1, E);
    free(si); free(so); free(u); free(pre1);
}

OR_API void or_gnp_layer(int64_t n, const int32_t *rp, const int32_t *ci, const double *ahat,
                         int L, int d, int h, const double *theta, int l, int B, const double *X,
                         double *Y)
{
    gnp_view g;
    gnp_unpack(theta, L, d, h, &g);
    double *T = (double *)malloc(sizeof(double) * n * B * d);
    layer_rows(n, rp, ci, ahat, B, d, g.U[l], g.W[l], X, T, Y);
    free(T);
}

OR_API void or_gnp_decoder(int64_t n, int L, int d, int h, const double *theta, int B,
                           const double *bin, const double *XL, double *z)
{
    gnp_view g;
    gnp_unpack(theta, L, d, h, &g);
    const int64_t rows = n * B;
    double *si = (double *)malloc(sizeof(double) * B), *so = (double *)malloc(sizeof(double) * B);
    double *pre3 = (double *)malloc(sizeof(double) * rows * h);
    double *o = (double *)malloc(sizeof(double) * rows);
    scale_factors(n, B, bin, NULL, si, so);
    decoder_rows(rows, B, d, h, &g, so, XL, pre3, o, z);
    free(si); free(so); free(pre3); free(o);
}

/* M(b) for B right-hand sides; acts (optional) receives X_0..X_L, each
 * n*B*d, node-major [i][b][f]. */
OR_API void or_gnp_forward(int64_t n, const int32_t *rp, const int32_t *ci, const double *ahat,
                           int L, int d, int h, const double *theta, int B,
                           const double *bin, double *z, double *acts)
{
    fwd_state s;
    fwd_alloc(&s, n, B, L, d, h);
    gnp_forward_state(n, rp, ci, ahat, L, d, h, theta, B, bin, z, &s);
    if (acts) {
        for (int l = 0; l <= L; ++l)
            memcpy(acts + (int64_t)l * n * B * d, s.X[l], sizeof(double) * n * B * d);
    }
    fwd_free(&s, L);
}

/* Training loss (Sec. 3 "Hyperparameters"): l = mean |A M(b) - b| over the
 * n*B entries (b = A x), and its gradient with respect to theta by reverse
 * mode, written out by hand.  A is the system matrix, ahat = A / gamma. */
OR_API double or_gnp_loss_grad(int64_t n, const int32_t *rp, const int32_t *ci,
                               const double *aval, const double *ahat,
                               int L, int d, int h, const double *theta, int B,
                               const double *bin, double *grad, double *zout)
{
    const int64_t rows = n * B;
    fwd_state s;
    fwd_alloc(&s, n, B, L, d, h);
    double *z = (double *)malloc(sizeof(double) * rows);
    gnp_forward_state(n, rp, ci, ahat, L, d, h, theta, B, bin, z, &s);
    if (zout) memcpy(zout, z, sizeof(double) * rows);
    /* residual R = A z - b and the loss */
    double *R = (double *)malloc(sizeof(double) * rows);
    or_spmm(n, rp, ci, aval, B, z, R);
    double loss = 0.0;
    for (int64_t r = 0; r < rows; ++r) {
        R[r] -= bin[r];
        loss += fabs(R[r]);
    }
    loss /= (double)rows;
    if (!grad) {
        free(z); free(R); fwd_free(&s, L);
        return loss;
    }
    gnp_view g;
    gnp_unpack(theta, L, d, h, &g);
    const int64_t np = gnp_nparams(L, d, h);
    memset(grad, 0, sizeof(double) * np);
    double *gW1 = grad, *gc1 = gW1 + h, *gW2 = gc1 + h, *gc2 = gW2 + (int64_t)h * d;
    double *gU[64], *gWl[64];
    double *p = gc2 + d;
    for (int l = 0; l < L; ++l) { gU[l] = p; p += (int64_t)d * d; gWl[l] = p; p += (int64_t)d * d; }
    double *gW3 = p, *gc3 = gW3 + (int64_t)d * h, *gW4 = gc3 + h, *gc4 = gW4 + h;

    /* dl/dz = A^T sign(R) / (n B), as a scatter over the nonzeros of A */
    double *dz = (double *)calloc((size_t)rows, sizeof(double));
    for (int64_t i = 0; i < n; ++i)
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
            for (int b = 0; b < B; ++b) {
                double rr = R[i * B + b];
                double sg = rr > 0.0 ? 1.0 : (rr < 0.0 ? -1.0 : 0.0);
                dz[(int64_t)ci[k] * B + b] += aval[k] * sg / (double)rows;
            }
    /* decoder backward */
    double *dX = (double *)calloc((size_t)(rows * d), sizeof(double));
    double *dp3 = (double *)malloc(sizeof(double) * h);
    for (int64_t r = 0; r < rows; ++r) {
        double dout = s.so[r % B] * dz[r];
        gc4[0] += dout;
        const double *p3 = s.pre3 + r * h;
        for (int k = 0; k < h; ++k) {
            gW4[k] += relu(p3[k]) * dout;
            dp3[k] = p3[k] > 0.0 ? g.W4[k] * dout : 0.0;
            gc3[k] += dp3[k];
        }
        const double *XL = s.X[L] + r * d;
        for (int f = 0; f < d; ++f) {
            double acc = 0.0;
            for (int k = 0; k < h; ++k) {
                gW3[(int64_t)f * h + k] += XL[f] * dp3[k];
                acc += g.W3[(int64_t)f * h + k] * dp3[k];
            }
            dX[r * d + f] = acc;
        }
    }
    /* Res-GCONV backward, layers L-1 .. 0 (Eq. (5)):
     *   dP = dY * [P > 0],  dU = X^T dP,  dW = T^T dP,
     *   dX = dP U^T + A-hat^T (dP W^T). */
    double *dP = (double *)malloc(sizeof(double) * rows * d);
    double *G = (double *)malloc(sizeof(double) * rows * d);
    double *dXn = (double *)malloc(sizeof(double) * rows * d);
    for (int l = L - 1; l >= 0; --l) {
        const double *X = s.X[l], *T = s.T[l], *Y = s.X[l + 1];
        for (int64_t e = 0; e < rows * d; ++e) dP[e] = Y[e] > 0.0 ? dX[e] : 0.0;
        for (int64_t r = 0; r < rows; ++r)
            for (int pp = 0; pp < d; ++pp)
                for (int q = 0; q < d; ++q) {
                    gU[l][(int64_t)pp * d + q] += X[r * d + pp] * dP[r * d + q];
                    gWl[l][(int64_t)pp * d + q] += T[r * d + pp] * dP[r * d + q];
                }
        for (int64_t r = 0; r < rows; ++r)
            for (int pp = 0; pp < d; ++pp) {
                double au = 0.0, aw = 0.0;
                for (int q = 0; q < d; ++q) {
                    au += g.U[l][(int64_t)pp * d + q] * dP[r * d + q];
                    aw += g.W[l][(int64_t)pp * d + q] * dP[r * d + q];
                }
                dXn[r * d + pp] = au;
                G[r * d + pp] = aw;
            }
        /* A-hat^T G as a scatter: row i of A-hat sends a_ij G_i to node j */
        for (int64_t i = 0; i < n; ++i)
            for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
                for (int b = 0; b < B; ++b)
                    for (int pp = 0; pp < d; ++pp)
                        dXn[((int64_t)ci[k] * B + b) * d + pp] += ahat[k] * G[(i * B + b) * d + pp];
        memcpy(dX, dXn, sizeof(double) * rows * d);
    }
    /* encoder backward: E = ReLU(u W1 + c1) W2 + c2 */
    for (int64_t r = 0; r < rows; ++r) {
        const double *p1 = s.pre1 + r * h;
        const double *dE = dX + r * d;
        for (int f = 0; f < d; ++f) gc2[f] += dE[f];
        for (int k = 0; k < h; ++k) {
            double a = relu(p1[k]);
            double acc = 0.0;
            for (int f = 0; f < d; ++f) {
                gW2[(int64_t)k * d + f] += a * dE[f];
                acc += g.W2[(int64_t)k * d + f] * dE[f];
            }
            double dp1 = p1[k] > 0.0 ? acc : 0.0;
            gW1[k] += s.u[r] * dp1;
            gc1[k] += dp1;
        }
    }
    free(dp3); free(dP); free(G); free(dXn); free(dX); free(dz); free(z); free(R);
    fwd_free(&s, L);
    return loss;
}

/* ------------------------------------------------------------------------ */
/* Adam (Kingma & Ba), bias-corrected; t counts from 1                      */
/* ------------------------------------------------------------------------ */
OR_API void or_adam(int64_t np, double *th, const double *g, double *m, double *v, int t,
                    double lr, double b1, double b2, double eps)
{
    double bc1 = 1.0 - pow(b1, (double)t), bc2 = 1.0 - pow(b2, (double)t);
    for (int64_t k = 0; k < np; ++k) {
        m[k] = b1 * m[k] + (1.0 - b1) * g[k];
        v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k];
        double mh = m[k] / bc1, vh = v[k] / bc2;
        th[k] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* ------------------------------------------------------------------------ */
/* Counter-based normal sampler: Philox4x32-10 (Salmon, Moraes, Dror, Shaw,  */
/* SC'11) followed by the Box-Muller transform (Box & Muller 1958)          */
/* ------------------------------------------------------------------------ */
OR_API void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Standard normal number e of stream `stream`, training step `step`, for
 * seed `seed`: counter = (e_lo, e_hi, step, stream), key = (seed_lo,
 * seed_hi); two 53-bit uniforms in (0,1) from the four output words;
 * z = sqrt(-2 ln u1) cos(2 pi u2).  Stream 0: the x ~ N(0, I) training
 * batches; 1: the coefficients eps of Eq. (3); 2: the Arnoldi start vector. */
OR_API double or_normal_stream(uint64_t seed, uint32_t step, uint32_t stream, uint64_t e)
{
    uint32_t ctr[4] = {(uint32_t)e, (uint32_t)(e >> 32), step, stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    or_philox4x32_10(ctr, key, o);
    const double two53 = 9007199254740992.0;
    double u1 = ((double)(((uint64_t)(o[0] >> 5) << 26) | (o[1] >> 6)) + 0.5) / two53;
    double u2 = ((double)(((uint64_t)(o[2] >> 5) << 26) | (o[3] >> 6)) + 0.5) / two53;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
}

OR_API double or_normal(uint64_t seed, uint32_t step, uint64_t e)
{
    return or_normal_stream(seed, step, 0u, e);
}

OR_API void or_normals(uint64_t seed, uint32_t step, int64_t count, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < count; ++e) out[e] = or_normal(seed, step, (uint64_t)e);
}

OR_API void or_normals_stream(uint64_t seed, uint32_t step, uint32_t stream, int64_t count,
                              double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < count; ++e) out[e] = or_normal_stream(seed, step, stream, (uint64_t)e);
}

/* Default initial weights (the paper does not state its initialisation):
 * every weight and bias uniform on (-1/sqrt(fan_in), 1/sqrt(fan_in)), fan_in
 * the input width of its linear map (W1, c1: 1; W2, c2: h; U_l, W_l: d;
 * W3, c3: d; W4, c4: h).  Parameter k takes the 53-bit uniform u in (0, 1)
 * from the first two output words of Philox4x32-10 at counter
 * (k_lo, k_hi, 0, 3) and key (seed_lo, seed_hi), and becomes
 * (2u - 1) / sqrt(fan_in). */
OR_API void or_init_params(int L, int d, int h, uint64_t seed, double *theta)
{
    const int64_t np = gnp_nparams(L, d, h);
    const int64_t end_enc = (int64_t)h + h + (int64_t)h * d + d;
    const int64_t end_layers = end_enc + (int64_t)L * 2 * d * d;
    const int64_t end_w3c3 = end_layers + (int64_t)d * h + h;
    const double two53 = 9007199254740992.0;
    for (int64_t k = 0; k < np; ++k) {
        int fan;
        if (k < 2 * (int64_t)h) fan = 1;             /* W1, c1 */
        else if (k < end_enc) fan = h;                /* W2, c2 */
        else if (k < end_layers) fan = d;             /* U_l, W_l */
        else if (k < end_w3c3) fan = d;               /* W3, c3 */
        else fan = h;                                 /* W4, c4 */
        uint32_t ctr[4] = {(uint32_t)k, (uint32_t)((uint64_t)k >> 32), 0u, 3u};
        uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
        uint32_t o[4];
        or_philox4x32_10(ctr, key, o);
        double u = ((double)(((uint64_t)(o[0] >> 5) << 26) | (o[1] >> 6)) + 0.5) / two53;
        theta[k] = (2.0 * u - 1.0) / sqrt((double)fan);
    }
}

/* ------------------------------------------------------------------------ */
/* Training loop (Sec. 2.2 streaming pairs, Sec. 3 hyperparameters)        */
/* ------------------------------------------------------------------------ */
/* x_fixed != NULL: the same n*B batch x every step; otherwise x is drawn
 * fresh each step from or_normal(seed, step, i*B + b).  b = A x.  theta is
 * replaced by the parameters of the step with the smallest loss. */
OR_API int or_train(int64_t n, const int32_t *rp, const int32_t *ci, const double *aval,
                    const double *ahat, int L, int d, int h, double *theta, int steps, int B,
                    double lr, double b1, double b2, double eps, uint64_t seed,
                    const double *x_fixed, double *loss_hist, int *best_step)
{
    const int64_t np = gnp_nparams(L, d, h), rows = n * B;
    double *grad = (double *)malloc(sizeof(double) * np);
    double *m = (double *)calloc((size_t)np, sizeof(double));
    double *v = (double *)calloc((size_t)np, sizeof(double));
    double *best = (double *)malloc(sizeof(double) * np);
    double *x = (double *)malloc(sizeof(double) * rows);
    double *bb = (double *)malloc(sizeof(double) * rows);
    double best_loss = INFINITY;
    int bs = -1, status = 0;
    memcpy(best, theta, sizeof(double) * np);
    for (int t = 0; t < steps; ++t) {
        if (x_fixed) memcpy(x, x_fixed, sizeof(double) * rows);
        else or_normals(seed, (uint32_t)t, rows, x);
        or_spmm(n, rp, ci, aval, B, x, bb);
        double loss = or_gnp_loss_grad(n, rp, ci, aval, ahat, L, d, h, theta, B, bb, grad, NULL);
        if (loss_hist) loss_hist[t] = loss;
        if (!isfinite(loss)) { status = 1; break; }
        if (loss < best_loss) {
            best_loss = loss;
            bs = t;
            memcpy(best, theta, sizeof(double) * np);
        }
        or_adam(np, theta, grad, m, v, t + 1, lr, b1, b2, eps);
    }
    memcpy(theta, best, sizeof(double) * np);
    if (best_step) *best_step = bs;
    free(grad); free(m); free(v); free(best); free(x); free(bb);
    return status;
}

/* ------------------------------------------------------------------------ */
/* FGMRES with a nonlinear right preconditioner (Algorithm 1, Sec. 2.1)     */
/* ------------------------------------------------------------------------ */

enum { OR_M_IDENTITY = 0, OR_M_GNP = 1, OR_M_DENSE = 2, OR_M_DIAG = 3, OR_M_GMRES = 4 };

typedef struct {
    int kind;
    /* GNP: graph of A-hat and weights */
    const int32_t *rp, *ci;
    const double *ahat;
    int L, d, h;
    const double *theta;
    /* DENSE: n x n row-major matrix; DIAG: n entries */
    const double *mat;
    /* GMRES (inner-outer GMRES, Sec. 3 "Compared methods"): z = one cycle of
       at most inner_k unpreconditioned Arnoldi steps on A z = v from z = 0,
       ended early once the Givens estimate is <= inner_tol ||v||; A is
       (rp, ci, aval) */
    const double *aval;
    int inner_k;
    double inner_tol;
    int inner_ortho;
} or_precond;

typedef struct {
    int iters, restarts, converged, mismatch, breakdowns;
    double rel_res_true, rel_res_est;
} or_info;

static int fgmres_core(int64_t n, const int32_t *rp, const int32_t *ci, const double *val,
                       const or_precond *M, const double *b, double *x, int m, double rtol,
                       int maxiters, int ortho, double *hist, or_info *info, double *dumpV,
                       double *dumpZ, double *dumpH, int *dump_k, int max_cycles);

static void apply_precond(int64_t n, const or_precond *M, const double *v, double *z)
{
    if (!M || M->kind == OR_M_IDENTITY) {
        memcpy(z, v, sizeof(double) * n);
    } else if (M->kind == OR_M_GNP) {
        or_gnp_forward(n, M->rp, M->ci, M->ahat, M->L, M->d, M->h, M->theta, 1, v, z, NULL);
    } else if (M->kind == OR_M_DENSE) {
        for (int64_t i = 0; i < n; ++i) z[i] = dot_seq(n, M->mat + i * n, v);
    } else if (M->kind == OR_M_GMRES) {
        or_info inner;
        memset(z, 0, sizeof(double) * n);
        fgmres_core(n, M->rp, M->ci, M->aval, NULL, v, z, M->inner_k, M->inner_tol, M->inner_k,
                    M->inner_ortho, NULL, &inner, NULL, NULL, NULL, NULL, 1);
    } else {
        for (int64_t i = 0; i < n; ++i) z[i] = M->mat[i] * v[i];
    }
}

/* ortho: 0 = modified Gram-Schmidt as printed in Algorithm 1,
 *        1 = classical Gram-Schmidt applied twice (CGS2).
 * hist (optional, maxiters+1): hist[0] = ||b - A x0|| / ||b||, hist[i] =
 * Givens estimate of the relative residual after iteration i.
 * dumpV/dumpZ/dumpH (optional): the last cycle's V (n x (m+1), column k at
 * k*n), Z (n x m) and the unrotated H-bar ((m+1) x m, row-major); *dump_k
 * receives its number of Arnoldi steps. */
OR_API int or_fgmres(int64_t n, const int32_t *rp, const int32_t *ci, const double *val,
                     const or_precond *M, const double *b, double *x, int m, double rtol,
                     int maxiters, int ortho, double *hist, or_info *info,
                     double *dumpV, double *dumpZ, double *dumpH, int *dump_k)
{
    return fgmres_core(n, rp, ci, val, M, b, x, m, rtol, maxiters, ortho, hist, info, dumpV,
                       dumpZ, dumpH, dump_k, 0);
}

/* Algorithm 1 as described at or_fgmres; max_cycles > 0 stops after that
 * many restart cycles (the inner solve of inner-outer GMRES runs one). */
static int fgmres_core(int64_t n, const int32_t *rp, const int32_t *ci, const double *val,
                       const or_precond *M, const double *b, double *x, int m, double rtol,
                       int maxiters, int ortho, double *hist, or_info *info, double *dumpV,
                       double *dumpZ, double *dumpH, int *dump_k, int max_cycles)
{
    memset(info, 0, sizeof(*info));
    int cycles = 0;
    double *V = (double *)malloc(sizeof(double) * n * (m + 1));
    double *Z = (double *)malloc(sizeof(double) * n * m);
    double *H = (double *)calloc((size_t)(m + 1) * m, sizeof(double));  /* rotated */
    double *H0 = (double *)calloc((size_t)(m + 1) * m, sizeof(double)); /* as built */
    double *cs = (double *)malloc(sizeof(double) * m), *sn = (double *)malloc(sizeof(double) * m);
    double *gv = (double *)malloc(sizeof(double) * (m + 1));
    double *y = (double *)malloc(sizeof(double) * m);
    double *r = (double *)malloc(sizeof(double) * n);
    double *w = (double *)malloc(sizeof(double) * n);
    double *hc = (double *)malloc(sizeof(double) * (m + 1));
    const double bnorm = nrm2_seq(n, b);
    int it = 0;
    if (bnorm == 0.0) {
        memset(x, 0, sizeof(double) * n);
        info->converged = 1;
        if (hist) hist[0] = 0.0;
        goto done;
    }
    const double target = rtol * bnorm;
    /* r0 = b - A x0, beta = ||r0|| */
    or_spmm(n, rp, ci, val, 1, x, r);
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
    double beta = nrm2_seq(n, r);
    if (hist) hist[0] = beta / bnorm;
    info->rel_res_true = info->rel_res_est = beta / bnorm;
    if (beta <= target) { info->converged = 1; goto done; }
    while (it < maxiters) {
        for (int64_t i = 0; i < n; ++i) V[i] = r[i] / beta;
        memset(gv, 0, sizeof(double) * (m + 1));
        gv[0] = beta;
        memset(H0, 0, sizeof(double) * (m + 1) * m);
        int k = 0;
        double est = beta;
        for (int j = 0; j < m && it < maxiters; ++j) {
            double *vj = V + (int64_t)j * n, *zj = Z + (int64_t)j * n;
            apply_precond(n, M, vj, zj);           /* z_j = M(v_j) */
            or_spmm(n, rp, ci, val, 1, zj, w);     /* w = A z_j */
            double wnorm0 = nrm2_seq(n, w);
            for (int i = 0; i <= j + 1; ++i) hc[i] = 0.0;
            if (ortho == 0) {
                for (int i = 0; i <= j; ++i) {     /* modified Gram-Schmidt */
                    const double *vi = V + (int64_t)i * n;
                    double hij = dot_seq(n, w, vi);
                    for (int64_t q = 0; q < n; ++q) w[q] -= hij * vi[q];
                    hc[i] = hij;
                }
            } else {
                for (int pass = 0; pass < 2; ++pass) { /* classical Gram-Schmidt, twice */
                    double hp[1024];
                    for (int i = 0; i <= j; ++i) hp[i] = dot_seq(n, w, V + (int64_t)i * n);
                    for (int64_t q = 0; q < n; ++q) {
                        double acc = 0.0;
                        for (int i = 0; i <= j; ++i) acc += hp[i] * V[(int64_t)i * n + q];
                        w[q] -= acc;
                    }
                    for (int i = 0; i <= j; ++i) hc[i] += hp[i];
                }
            }
            hc[j + 1] = nrm2_seq(n, w);
            for (int i = 0; i <= j + 1; ++i) {
                H0[(int64_t)i * m + j] = hc[i];
                H[(int64_t)i * m + j] = hc[i];
            }
            /* apply the previous rotations, then a new one (Saad 2003, Sec. 6.5.3) */
            for (int i = 0; i < j; ++i) {
                double a = H[(int64_t)i * m + j], bb = H[(int64_t)(i + 1) * m + j];
                H[(int64_t)i * m + j] = cs[i] * a + sn[i] * bb;
                H[(int64_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * bb;
            }
            double a = H[(int64_t)j * m + j], bb = H[(int64_t)(j + 1) * m + j];
            double rho = hypot(a, bb);
            if (rho == 0.0) { cs[j] = 1.0; sn[j] = 0.0; }
            else { cs[j] = a / rho; sn[j] = bb / rho; }
            H[(int64_t)j * m + j] = rho;
            H[(int64_t)(j + 1) * m + j] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            est = fabs(gv[j + 1]);
            ++it;
            k = j + 1;
            if (hist) hist[it] = est / bnorm;
            if (hc[j + 1] <= 1e-14 * wnorm0) { info->breakdowns++; break; }
            double *vn = V + (int64_t)(j + 1) * n;
            for (int64_t q = 0; q < n; ++q) vn[q] = w[q] / hc[j + 1];
            if (est <= target) break;
        }
        /* y = argmin || beta e1 - H-bar y ||: back substitution on the rotated
         * triangle; trailing columns with a zero pivot are dropped. */
        int kk = k;
        while (kk > 0 && H[(int64_t)(kk - 1) * m + (kk - 1)] == 0.0) --kk;
        for (int i = kk - 1; i >= 0; --i) {
            double acc = gv[i];
            for (int q = i + 1; q < kk; ++q) acc -= H[(int64_t)i * m + q] * y[q];
            y[i] = acc / H[(int64_t)i * m + i];
        }
        for (int64_t q = 0; q < n; ++q) {
            double acc = 0.0;
            for (int i = 0; i < kk; ++i) acc += Z[(int64_t)i * n + q] * y[i];
            x[q] += acc;
        }
        if (dumpV) memcpy(dumpV, V, sizeof(double) * n * (m + 1));
        if (dumpZ) memcpy(dumpZ, Z, sizeof(double) * n * m);
        if (dumpH) memcpy(dumpH, H0, sizeof(double) * (m + 1) * m);
        if (dump_k) *dump_k = k;
        /* true residual */
        or_spmm(n, rp, ci, val, 1, x, r);
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
        beta = nrm2_seq(n, r);
        info->rel_res_true = beta / bnorm;
        info->rel_res_est = est / bnorm;
        if (!isfinite(beta)) break;
        if (beta <= target) { info->converged = 1; break; }
        if (it >= maxiters) break;
        if (max_cycles > 0 && ++cycles >= max_cycles) break;
        info->restarts++;
    }
    if (info->rel_res_est > 0.0 && info->rel_res_true > 10.0 * info->rel_res_est) info->mismatch = 1;
done:
    info->iters = it;
    free(V); free(Z); free(H); free(H0); free(cs); free(sn); free(gv); free(y); free(r); free(w);
    free(hc);
    return 0;
}
