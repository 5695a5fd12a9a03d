/*
 * gnp.h -- C ABI of libgnp: graph-neural-preconditioned flexible GMRES on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: J. Chen, "Graph Neural Preconditioners for Iterative Solutions of
 * Sparse Linear Systems" (ICLR 2025).  Section numbers below refer to it.
 *
 * Conventions for every entry point
 *  - Every call returns a gnp_status; no C++ exception crosses the ABI.  On a
 *    status other than GNP_OK a thread-local message is available from
 *    gnp_last_error().  Non-convergence of a solve is NOT an error: it returns
 *    GNP_OK with info.converged = 0.
 *  - Pointers named *_dev are device pointers (for example from PyTorch's
 *    caching allocator); every other pointer is host memory.  The library
 *    never frees memory it did not allocate.
 *  - hip_stream is a hipStream_t (NULL = the default stream).  Work is
 *    ordered on that stream; calls that return host results synchronise it.
 *  - Dense vectors with several right-hand sides are node-major: element
 *    (i, k) of an n x nrhs block lives at [i * nrhs + k].
 *  - CSR input: int32 rowptr[n+1] and colind[nnz], column indices sorted
 *    and unique within each row, float64 values.
 */
#ifndef GNP_H
#define GNP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GNP_API __attribute__((visibility("default")))

typedef enum {
    GNP_OK = 0,
    GNP_EINVAL = 1,   /* invalid argument or malformed CSR */
    GNP_ENOMEM = 2,   /* device or host allocation failed */
    GNP_EDEVICE = 3,  /* HIP runtime error */
    GNP_ENUMERIC = 4, /* non-finite value met (b, weights, beta, h, tau, loss) */
    GNP_EBUSY = 5     /* a served request is not finished yet */
} gnp_status;

/* Arithmetic of the preconditioned path.
 *   GNP_F64 : everything in float64 (reference-precision instantiation).
 *   GNP_F32 : network activations, SpMV and Krylov basis V, Z in float32.
 *   GNP_BF16: network activations stored in bfloat16, products on MFMA with
 *             float32 accumulation; SpMV and V, Z in float32.
 * In every mode the Arnoldi inner products and norms, the Hessenberg
 * least-squares (Givens), the solution x and the true residual b - A x are
 * float64. */
typedef enum { GNP_F64 = 0, GNP_F32 = 1, GNP_BF16 = 2 } gnp_precision;

typedef struct gnp_system gnp_system;
typedef struct gnp_model gnp_model;
typedef struct gnp_sampler gnp_sampler;

/* Message describing the last failure on the calling thread. */
GNP_API const char *gnp_last_error(void);

/* Library version string. */
GNP_API const char *gnp_version(void);

/* ------------------------------------------------------------------------ */
/* Linear system                                                            */
/* ------------------------------------------------------------------------ */

/* Create a device-resident system from a host CSR matrix A (n x n).
 *
 * The host arrays are copied; the caller keeps them.  On the device the
 * library computes gamma of Eq. (4) (an upper bound of the spectral radius
 * by Gershgorin: min of the largest absolute row sum and the largest
 * absolute column sum).  If prescale != 0, A is first divided by its own
 * gamma (the harness normalisation of Sec. 3), and gamma is then recomputed
 * for the scaled matrix.  A-hat = A / gamma (Eq. (4)) feeds the network; the
 * (possibly prescaled) A is the matrix that fgmres_solve solves with.  The
 * transposed CSR of A (needed by training) is built on the device by a
 * counting sort.
 *
 * Errors: GNP_EINVAL when n < 1, nnz < 1, rowptr[0] != 0, rowptr is
 * decreasing, rowptr[n] != nnz, a column index lies outside [0, n), columns
 * in a row are not strictly increasing, a value is not finite, or gamma = 0.
 */
GNP_API gnp_status gnp_system_create(int64_t n, int64_t nnz, const int32_t *rowptr,
                                     const int32_t *colind, const double *val, int prescale,
                                     void *hip_stream, gnp_system **out);

/* Replace the values of a system's matrix, keeping its sparsity pattern: the
 * slowly evolving systems for which the paper proposes to keep training the
 * same network (Sec. 5, "Discussions and Conclusions").  val: host array of nnz
 * values in the CSR order of gnp_system_create.  Everything that follows from
 * the values is made again on the device exactly as gnp_system_create makes
 * it (gamma, the prescaled A and A-hat of Eq. (4) in every precision, their
 * transposes), so the system then equals one created from the new values.
 * Networks of the system stay valid and keep their weights (training
 * continues from them); the Jacobi diagonal is made again on its next use.
 * No solve, training run or server request may be in flight on the system.
 * Errors: GNP_EINVAL for a null system or val, a non-finite value, or
 * values whose gamma would be zero or not finite; the system is then
 * unchanged. */
GNP_API gnp_status gnp_system_set_values(gnp_system *sys, const double *val, void *hip_stream);
GNP_API void gnp_system_destroy(gnp_system *sys);

/* gamma of the input matrix, and gamma of the matrix after the optional
 * prescaling (the A-hat divisor).  Either pointer may be NULL. */
GNP_API gnp_status gnp_system_gamma(const gnp_system *sys, double *gamma_input,
                                    double *gamma_system);

/* Copy device-resident arrays back to host buffers (any pointer may be NULL):
 * val[nnz] = system A (float64), ahat[nnz] = A-hat (float64),
 * t_rowptr[n+1], t_colind[nnz] = CSR of A^T, t_val[nnz] = values of A^T. */
GNP_API gnp_status gnp_system_export(const gnp_system *sys, double *val, double *ahat,
                                     int32_t *t_rowptr, int32_t *t_colind, double *t_val);

GNP_API int64_t gnp_system_n(const gnp_system *sys);
GNP_API int64_t gnp_system_nnz(const gnp_system *sys);

/* y_dev = A x_dev (system matrix, Sec. 2.1).  prec = GNP_F64: float64 values,
 * x and y float64; GNP_F32 / GNP_BF16: float32 values, x and y float32. */
GNP_API gnp_status gnp_spmv(const gnp_system *sys, const void *x_dev, void *y_dev,
                            gnp_precision prec, void *hip_stream);

/* ------------------------------------------------------------------------ */
/* Graph neural preconditioner (Sec. 2.3)                                   */
/* ------------------------------------------------------------------------ */

/* Create the network M for a system: an MLP encoder lifting 1 -> d (hidden
 * h), L Res-GCONV layers X <- ReLU(X U_l + A-hat X W_l) (Eq. (5)), an MLP
 * decoder d -> 1 (hidden h), wrapped in the scale-equivariant s, s^-1 of
 * Eq. (6) with tau = ||b||_2.
 *
 * Parameters are a float64 vector in this packing (matrices row-major with
 * the input index first, y = x M):
 *   W1[1 x h] c1[h] W2[h x d] c2[d] | for l < L: U_l[d x d] W_l[d x d] |
 *   W3[d x h] c3[h] W4[h x 1] c4[1]
 * count = 2h + 2hd + d + 2 L d^2 + 2h + 1.  init_params (host) holds that
 * many values, or is NULL for the seeded default initialisation (the paper
 * does not state one): every weight and bias uniform on
 * (-1/sqrt(fan_in), 1/sqrt(fan_in)), fan_in the input width of its linear
 * map (W1, c1: 1; W2, c2: h; U_l, W_l: d; W3, c3: d; W4, c4: h), parameter k
 * = (2u - 1)/sqrt(fan_in) with u the 53-bit uniform in (0, 1) from the first
 * two output words of Philox4x32-10 at counter (k_lo, k_hi, 0, 3) and key
 * (seed_lo, seed_hi).  seed is used only when init_params is NULL.
 * Supported (d, h): (16, 32) and (32, 64); 1 <= L <= 64 (the network has at
 * least one Res-GCONV layer: the decoder runs fused into the last one).
 * The model keeps a reference to sys, which must outlive it.
 * Errors: GNP_EINVAL for a null sys or out, an unsupported (d, h) or L out
 * of range; GNP_ENUMERIC for a non-finite initial parameter. */
GNP_API gnp_status gnp_model_create(gnp_system *sys, int L, int d, int h,
                                    const double *init_params, uint64_t seed, gnp_model **out);
GNP_API void gnp_model_destroy(gnp_model *model);
GNP_API size_t gnp_model_nparams(const gnp_model *model);
/* Switch the scale-equivariant wrapping of Eq. (6) off (on = 0) or back on
 * (on = 1, the default) for every later apply, training step and solve: off,
 * the network is applied to b itself, z = decoder(layers(encoder(b))), the
 * alternative the paper's ablation compares against (Sec. 3, whether the
 * scale-equivariance design is necessary).  Off, M(0) is the network's
 * output for a zero input instead of 0.  Errors: GNP_EINVAL for a null model
 * or another value of on. */
GNP_API gnp_status gnp_model_set_scaling(gnp_model *model, int on);
GNP_API gnp_status gnp_params_get(const gnp_model *model, double *buf, size_t count);
GNP_API gnp_status gnp_params_set(gnp_model *model, const double *buf, size_t count);
/* Same as gnp_params_set from a float64 device buffer, stream-ordered (no
 * host synchronisation, no finiteness check). */
GNP_API gnp_status gnp_params_set_device(gnp_model *model, const double *buf_dev, size_t count,
                                         void *hip_stream);

/* z_dev = M(v_dev) for nrhs right-hand sides, node-major [n][nrhs].
 * prec = GNP_F64: v, z float64; GNP_F32 / GNP_BF16: v, z float32.
 * A zero column maps to a zero column (tau = 0).  Stream-ordered; uses the
 * model's workspace (allocated on first use for a given nrhs, then reused).
 * Errors: GNP_EINVAL for nrhs < 1 or a bad precision. */
GNP_API gnp_status gnp_apply(gnp_model *model, const void *v_dev, void *z_dev, int nrhs,
                             gnp_precision prec, void *hip_stream);

/* gnp_apply for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results as gnp_apply, with its workspace (column-norm
 * partials and counter, tau, two activation blocks) in a fixed array of
 * GNP_NOALLOC_SCRATCH_BYTES in device memory that the library holds on
 * every GPU it runs on until the process ends, instead of the model's apply
 * workspace.  No allocation of any kind; the launches are a fill kernel for
 * the counter and the apply's kernels, all on hip_stream.
 * Limit: 256 + 256-rounded (24 nrhs + 8 nrhs * column-norm blocks) + 2 x
 * 256-rounded (n * nrhs * d * element size: 8, 4 or 2 bytes for F64, F32,
 * BF16) bytes must fit (the column-norm blocks are at most 1024); the
 * 64^3 system with d = 32 fits with one right-hand side in float32 and
 * bfloat16 (80 MiB; float64 needs 128 MiB there).
 * Every call on a GPU uses that GPU's one array: calls that overlap on one
 * GPU (other streams, other threads) race and give wrong results; order them
 * on one stream.  Errors: as gnp_apply, plus GNP_EINVAL when the apply does
 * not fit in the array. */
#define GNP_NOALLOC_SCRATCH_BYTES (80u << 20)
GNP_API gnp_status gnp_apply_noalloc(gnp_model *model, const void *v_dev, void *z_dev, int nrhs,
                                     gnp_precision prec, void *hip_stream);

/* gnp_apply that also keeps every activation of the network: acts_dev holds
 * (L+1) blocks of n * nrhs * d activations in the precision's storage type
 * (float64, float32, or bfloat16 bit patterns as uint16 for GNP_BF16), node-
 * major [n][nrhs][d]; block 0 = the encoder output X_0, block l = the output
 * X_l of Res-GCONV layer l (Eq. (5)).  z_dev receives M(v) exactly as from
 * gnp_apply (same kernels; the last layer additionally runs once without the
 * fused decoder to store X_L).  For per-layer precision studies. */
GNP_API gnp_status gnp_apply_layers(gnp_model *model, const void *v_dev, void *z_dev,
                                    void *acts_dev, int nrhs, gnp_precision prec,
                                    void *hip_stream);

/* ------------------------------------------------------------------------ */
/* FGMRES(m) with the network as right preconditioner (Algorithm 1)         */
/* ------------------------------------------------------------------------ */

typedef struct {
    int iters;          /* Arnoldi steps (applications of M), across restarts */
    int restarts;       /* completed cycles that did not converge */
    int converged;      /* 1 iff ||b - A x||_2 <= rtol ||b||_2 (true residual) */
    int mismatch;       /* 1 iff true residual > 10 x the Givens estimate */
    int breakdowns;     /* cycles ended by h_{j+1,j} <= 1e-14 ||A z_j|| */
    double rel_res_true;/* ||b - A x|| / ||b|| at exit, float64 */
    double rel_res_est; /* Givens least-squares estimate at exit */
} gnp_solve_info;

/* Solve A x = b (A = the system matrix) by restarted flexible GMRES.
 *
 * b_dev, x_dev: float64 device vectors of length n; x_dev holds x0 on entry
 * and the solution on exit.  model = NULL runs unpreconditioned GMRES (M = I).
 * m: restart length; rtol: relative tolerance on the true residual;
 * maxiters: bound on Arnoldi steps across restarts.  After every Arnoldi step
 * the Givens residual estimate is checked and ends the cycle early once it is
 * below rtol ||b||; the float64 true residual confirms or restarts.
 * Orthogonalisation is classical Gram-Schmidt applied twice with float64
 * inner products.
 * hist (optional, host, maxiters + 1 doubles): hist[0] = ||b - A x0||/||b||,
 * hist[i] = estimated relative residual after Arnoldi step i; entries past
 * info.iters are left untouched.
 * b = 0 gives x = 0, iters = 0, converged = 1.
 * Errors: GNP_EINVAL for m < 1, m > 255, rtol <= 0, maxiters < 1, a model of
 * another system or a bad precision; GNP_ENUMERIC when b, the residual, a
 * norm or a Hessenberg entry becomes non-finite. */
GNP_API gnp_status fgmres_solve(gnp_system *sys, gnp_model *model, const double *b_dev,
                                double *x_dev, int m, double rtol, int maxiters,
                                gnp_precision prec, double *hist, gnp_solve_info *info,
                                void *hip_stream);

/* fgmres_solve with the Jacobi preconditioner M = D^{-1}, D the diagonal of
 * the system matrix (prescaled when the system is): the simple baseline the
 * paper compares the network against (Sec. 3, "Compared methods").  Each
 * Arnoldi step applies z_j = D^{-1} v_j in float64 and rounds to the Krylov
 * precision; everything else is as in fgmres_solve.  D^{-1} is formed on the
 * device on first use and kept with the system.
 * prec: GNP_F32 or GNP_F64.  Errors: as fgmres_solve, plus GNP_EINVAL when a
 * row has no nonzero diagonal entry or for another precision. */
GNP_API gnp_status fgmres_solve_jacobi(gnp_system *sys, const double *b_dev, double *x_dev,
                                       int m, double rtol, int maxiters, gnp_precision prec,
                                       double *hist, gnp_solve_info *info, void *hip_stream);

/* fgmres_solve with inner-outer GMRES: the preconditioner z_j = M(v_j) is
 * itself an unpreconditioned GMRES solve of A z = v_j, the other comparison
 * method of Sec. 3 ("Compared methods"; the paper runs inner_k = 10,
 * inner_tol = 1e-6 with an outer restart of 10).  Each inner solve is one
 * cycle of at most inner_k Arnoldi steps from z = 0, on the same kernels and
 * in the same Krylov precision as the outer one (classical Gram-Schmidt
 * twice, float64 inner products), ended early once its Givens estimate is at
 * most inner_tol ||v_j||; it takes no true residual.  info.iters counts
 * outer steps.  The inner workspace (inner_k + 1 basis vectors and a
 * float64 vector, pitch 32) is kept with the system.
 * inner_k: 1..31; inner_tol: finite, >= 0 (>= 1 gives z = 0 and a breakdown).
 * prec: GNP_F32 or GNP_F64.  Errors: as fgmres_solve, plus GNP_EINVAL for
 * inner_k or inner_tol out of range or another precision. */
GNP_API gnp_status fgmres_solve_gmres(gnp_system *sys, const double *b_dev, double *x_dev,
                                      int m, double rtol, int maxiters, int inner_k,
                                      double inner_tol, gnp_precision prec, double *hist,
                                      gnp_solve_info *info, void *hip_stream);


/* Time limit for the single solves on this system (fgmres_solve,
 * fgmres_solve_jacobi, fgmres_solve_gmres), the stopping criterion the paper
 * uses for its time comparisons besides rtol (Sec. 3, "Stopping criteria"):
 * once the initial residual is known the device takes a deadline `seconds`
 * later on its own wall clock; the first Arnoldi step that ends after it
 * ends the cycle, x is updated, and the solve returns with converged = 0
 * unless that cycle reached rtol.  maxiters still bounds the steps.  0 (the
 * default) means no limit.  Served requests and the sampler are not
 * affected.  Errors: GNP_EINVAL for a null system or a negative or
 * non-finite value. */
GNP_API gnp_status gnp_system_set_timeout(gnp_system *sys, double seconds);

/* Elapsed wall-clock time of the last single solve on this system
 * (fgmres_solve, fgmres_solve_jacobi or fgmres_solve_gmres), for the
 * Time-AUC metric of Sec. 3 ("Evaluation metrics"): t_host[i] = seconds from
 * the moment the initial residual r_0 was known to the moment the residual
 * estimate of Arnoldi step i was known (t_host[0] = 0), stamped on the device
 * with its wall clock, so host waits between restart cycles are included.
 * t_host: host array of count doubles, count in [1, iters + 1] of that solve.
 * Errors: GNP_EINVAL for no solve yet or count out of range. */
GNP_API gnp_status fgmres_step_times(gnp_system *sys, double *t_host, int count);

/* The two metrics of Sec. 3 ("Evaluation metrics") from a residual history
 * (host arrays): Iter-AUC = sum over i = 0..iters of log10 r_i - log10 rtol,
 * Time-AUC = sum over i = 1..iters of (log10 r_i - log10 rtol)(t_i - t_{i-1}).
 * r: iters + 1 relative residuals (the hist of a solve: r_0 true, then the
 * Givens estimates); t: iters + 1 times (fgmres_step_times), needed only for
 * time_auc.  A residual of 0 counts as the smallest normal double.  Either
 * output may be NULL.  Errors: GNP_EINVAL for r = NULL, iters < 0, rtol <= 0,
 * or time_auc without t.  Host-only: no device work. */
GNP_API gnp_status gnp_auc(const double *r, const double *t, int iters, double rtol,
                           double *iter_auc, double *time_auc);

/* Solve A x_k = b_k for nrhs right-hand sides at once (each one exactly as
 * fgmres_solve would, step for step), with one network application per
 * Arnoldi step for the whole batch (Sec. 2.2: one preconditioner serves every
 * right-hand side of its system).  b_dev, x_dev: nrhs float64 vectors of
 * length n, one after the other (b_k at b_dev + k n); x_dev holds the x0 on
 * entry and the solutions on exit.  The right-hand sides run in lockstep
 * restart cycles; one that has converged (or reached maxiters) idles while
 * the others go on.  infos (host, nrhs entries, optional) receives each
 * solve's gnp_solve_info.  model is required; prec is GNP_F32 or GNP_BF16.
 * Errors: as fgmres_solve, plus GNP_EINVAL for nrhs outside [1, 256]. */
GNP_API gnp_status fgmres_solve_batch(gnp_system *sys, gnp_model *model, const double *b_dev,
                                      double *x_dev, int nrhs, int m, double rtol, int maxiters,
                                      gnp_precision prec, gnp_solve_info *infos,
                                      void *hip_stream);

/* ------------------------------------------------------------------------ */
/* Training (Sec. 2.2 and Sec. 3 "Hyperparameters")                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    int steps;           /* Adam steps */
    int batch;           /* right-hand sides per step, 1..256 */
    double lr;           /* Adam learning rate (the paper uses 1e-3) */
    double beta1, beta2; /* Adam moment decay rates (0.9, 0.999) */
    double eps;          /* Adam epsilon (1e-8) */
    uint64_t seed;       /* seed of the samplers */
    gnp_precision prec;  /* GNP_F32 or GNP_F64 */
    int sampler_m;       /* 0: every x ~ N(0, I); 1..64: Arnoldi steps of the
                            Eq. (3) sampler (the paper uses 40) */
    int sampler_count;   /* with sampler_m > 0: the first sampler_count columns
                            of every batch are drawn from Eq. (3), the others
                            from N(0, I) (the paper: 8 of 16); 0..batch */
} gnp_train_opts;

/* Train the network on streaming pairs (b = A x, x): every step draws
 * x ~ N(0, I) ([n][batch]) with a counter-based Philox4x32-10 generator
 * (counter = (element index low, high, step, 0), key = seed) and the
 * Box-Muller transform, unless x_fixed_dev (float64 device, [n][batch]) is
 * given, in which case that batch is used at every step.  With
 * opts->sampler_m > 0 a sampler as gnp_sampler_create(system, sampler_m,
 * seed) is built first and columns 0..sampler_count-1 of every drawn batch
 * are replaced by its draws for that step (gnp_sampler_draw).  Loss: mean over the
 * n*batch entries of |A M(b) - b| (the l1 residual of Sec. 3); gradient by the
 * hand-written backward; update: bias-corrected Adam on float64 master
 * weights.  At the end the model holds the weights of the step with the
 * smallest loss (earliest on ties), as the paper keeps the best epoch.
 * loss_hist (host, optional, [steps]) receives the loss of every step;
 * *best_step its index.  Synchronises the stream.
 * Errors: GNP_EINVAL for bad options or precision GNP_BF16; GNP_ENUMERIC if a
 * loss is not finite (updates stop at that step). */
GNP_API gnp_status gnp_train(gnp_model *model, const gnp_train_opts *opts,
                             const double *x_fixed_dev, double *loss_hist, int *best_step,
                             void *hip_stream);

/* ------------------------------------------------------------------------ */
/* Training-pair sampler (Sec. 2.2, Eqs. (2)-(3))                            */
/* ------------------------------------------------------------------------ */

/* Run m steps (1..64, below n) of the Arnoldi process without a
 * preconditioner, A V_m = V_{m+1} Hbar_m (Eq. (2)), in FP64 with CGS2,
 * from xi / ||xi||, xi ~ N(0, I) drawn from the Philox generator with
 * counter (element low, high, 0, 2) and key seed; then the thin SVD
 * Hbar_m = W S Z^T on the device (one-sided Jacobi, FP64) in canonical form
 * (singular values decreasing, the entry of largest magnitude of each
 * column of Z positive) and G = Z S^+ (singular values <= 1e-12 s_max
 * dropped).  A breakdown ends the process early: k < m steps are used.
 * max_count: most draws per gnp_sampler_draw call (1..256).  The sampler
 * keeps V_k and G on the device (n * pitch + ... doubles) and refers to
 * the system, which must outlive it.  Synchronises the stream.
 * Errors: GNP_EINVAL for bad arguments; GNP_ENUMERIC for a non-finite
 * Arnoldi process; GNP_ENOMEM. */
GNP_API gnp_status gnp_sampler_create(gnp_system *sys, int m, uint64_t seed, int max_count,
                                      void *hip_stream, gnp_sampler **out);

/* Host copies of what the sampler built (each optional): *k = steps used,
 * hbar = Hbar_k ((k+1) x k, row-major), sv = the k singular values
 * (decreasing), G = Z S^+ (k x k, row-major).  Synchronous. */
GNP_API gnp_status gnp_sampler_info(const gnp_sampler *s, int *k, double *hbar, double *sv,
                                    double *G);

/* x_dev (float64 device, [n][count]): column d = V_k G eps_d, the draw of
 * Eq. (3), with eps_d[j] the Philox normal of counter (d k + j, 0, step, 1)
 * and key seed.  count in 1..max_count.  Stream-ordered. */
GNP_API gnp_status gnp_sampler_draw(gnp_sampler *s, uint32_t step, int count, double *x_dev,
                                    void *hip_stream);
GNP_API void gnp_sampler_destroy(gnp_sampler *s);

/* Loss and gradient at the current weights for one batch b_dev (float64
 * device, [n][nrhs]): *loss = mean |A M(b) - b|, grad (host, optional,
 * [nparams]) = its gradient in the packing of gnp_model_create.  prec:
 * GNP_F32 or GNP_F64.  Synchronises the stream. */
GNP_API gnp_status gnp_loss_grad(gnp_model *model, const double *b_dev, int nrhs,
                                 gnp_precision prec, double *loss, double *grad,
                                 void *hip_stream);

/* Forward pass that keeps every layer input for a later gnp_backward (the
 * pair behind a torch.autograd.Function).  b_dev, z_dev: [n][nrhs] in the
 * precision's type (float64 or float32).  The saved state belongs to the
 * model and is replaced by the next call. */
GNP_API gnp_status gnp_forward_save(gnp_model *model, const void *b_dev, void *z_dev, int nrhs,
                                    gnp_precision prec, void *hip_stream);

/* Vector-Jacobian product of the last gnp_forward_save: given dz_dev
 * ([n][nrhs], same type), write d<dz, M(b)>/dtheta to dparams_dev (float64
 * device, [nparams]).  Errors: GNP_EINVAL without a saved forward. */
GNP_API gnp_status gnp_backward(gnp_model *model, const void *dz_dev, double *dparams_dev,
                                void *hip_stream);

/* ------------------------------------------------------------------------ */
/* Solve server: continuous batching over resident systems                   */
/* ------------------------------------------------------------------------ */

/* The paper applies one trained preconditioner to any number of right-hand
 * sides of its system (Sec. 2.2 trains on a distribution of b).  The server
 * keeps registered systems (CSR, A-hat) and their networks resident and
 * solves a stream of requests, each one FGMRES(m) from x0 = 0 exactly as
 * fgmres_solve runs it (same kernels, buffers of its own), so a result does
 * not depend on the other requests in flight.
 *
 * A worker thread admits queued requests into up to max_slots slots whenever
 * a slot and HBM free up (continuous batching): each slot needs a solve
 * workspace for its system (Krylov basis, network outputs and activations,
 * b, x; gnp_server_workspace_bytes), and the workspaces held never exceed
 * hbm_budget bytes.  A finished request leaves its workspace resident for the
 * next request on the same system; idle workspaces of other systems are
 * evicted, least recently used first, when a new one would not fit.  A request
 * whose workspace alone exceeds the budget fails with GNP_ENOMEM.  Requests
 * that fit may overtake one that waits for memory, at most 8 while the same
 * request heads the queue.  Every slot has its own HIP stream, so the solves
 * in flight overlap on the device.
 *
 * Latency of a request: from gnp_server_submit to the moment its solution is
 * in host memory.  All server entry points are thread-safe. */
typedef struct gnp_server gnp_server;

typedef struct {
    int64_t submitted, completed, failed, rejected; /* rejected: larger than the budget */
    int64_t queued, active, max_active;             /* requests waiting / in slots now / peak */
    double latency_p50_s, latency_p99_s, latency_mean_s; /* completed requests, nearest rank */
    double solves_per_s;  /* completed / (last completion - first submission) */
    size_t hbm_budget, hbm_used, hbm_peak; /* bytes of solve workspaces held */
    int64_t workspaces_allocated, workspaces_reused, workspaces_evicted;
    /* requests that completed with a true residual <= their rtol (completed
     * counts also the ones that stopped at maxiters or a time limit) */
    int64_t converged;
    double converged_per_s;                        /* converged / (last converged - first submission) */
    double conv_latency_p50_s, conv_latency_p99_s; /* over the converged requests */
} gnp_server_stats;

/* Start a server on the current device.  m: restart length of every solve
 * (1..255); max_iters: largest maxiters a request may ask for; prec: the
 * network / Krylov precision (as in fgmres_solve).
 * Errors: GNP_EINVAL for max_slots outside [1, 256], bad m, max_iters < 1,
 * hbm_budget = 0 or a bad precision; GNP_EDEVICE if streams cannot be made. */
GNP_API gnp_status gnp_server_create(size_t hbm_budget, int max_slots, int m, int max_iters,
                                     gnp_precision prec, gnp_server **out);

/* Register a system and its network (model = NULL: unpreconditioned GMRES).
 * Both must outlive the server.  *id receives the system's id. */
GNP_API gnp_status gnp_server_register(gnp_server *srv, gnp_system *sys, gnp_model *model,
                                       int *id);

/* Device bytes one solve workspace of system `id` takes. */
GNP_API gnp_status gnp_server_workspace_bytes(gnp_server *srv, int id, size_t *bytes);

/* Queue a solve of A_id x = b: b_host (host, n doubles) is copied before the
 * call returns.  rtol > 0, 1 <= maxiters <= max_iters.  *ticket identifies
 * the request for gnp_server_poll. */
GNP_API gnp_status gnp_server_submit(gnp_server *srv, int id, const double *b_host, double rtol,
                                     int maxiters, uint64_t *ticket);

/* Collect a request: GNP_EBUSY while it is queued or running; otherwise the
 * request's own status (GNP_OK, or the error that ended it), and the ticket is
 * released.  On GNP_OK: x_host (n doubles), info and latency_s (seconds from
 * submission to completion) are filled (each may be NULL). */
GNP_API gnp_status gnp_server_poll(gnp_server *srv, uint64_t ticket, double *x_host,
                                   gnp_solve_info *info, double *latency_s);

/* Block until no request is queued or running, or until timeout_s seconds
 * have passed (GNP_EBUSY). */
GNP_API gnp_status gnp_server_drain(gnp_server *srv, double timeout_s);

/* Replace the values of registered system `id` while the server runs (the
 * slowly evolving systems for which the paper keeps training the same
 * network, Sec. 5 "Discussions and Conclusions"): its queued and newly
 * submitted requests wait, the requests of it already in slots finish on
 * the old values, then gnp_system_set_values(sys, val) runs and, with
 * tune != NULL, gnp_train(model, tune, NULL, loss_hist, best_step) trains
 * the registered network further on the new matrix; then its requests are
 * admitted again (the other systems are served throughout).  Blocks the
 * caller until done.  Training memory is outside the HBM budget.
 * Errors: GNP_EINVAL for an unknown id, a null val, tune without a
 * registered network, or what gnp_system_set_values / gnp_train reject (the
 * system then keeps its old values, or the weights of the failed training);
 * GNP_EBUSY if an update of the same system is already in progress. */
GNP_API gnp_status gnp_server_update_system(gnp_server *srv, int id, const double *val,
                                            const gnp_train_opts *tune, double *loss_hist,
                                            int *best_step);

GNP_API gnp_status gnp_server_get_stats(gnp_server *srv, gnp_server_stats *out);

/* Stop the server: requests still queued fail with GNP_EBUSY, running ones
 * finish first; uncollected results are dropped. */
GNP_API void gnp_server_destroy(gnp_server *srv);

/* ------------------------------------------------------------------------ */
/* Measurement helpers                                                      */
/* ------------------------------------------------------------------------ */

/* Mean duration (ms) of one launch of the Res-GCONV layer kernel (Eq. (5)),
 * in the launch configuration of gnp_apply / fgmres_solve for nrhs
 * right-hand sides and precision prec: `reps` back-to-back launches on
 * hip_stream between two hipEvents recorded on that stream.  Operates on the
 * model's apply workspace (run gnp_apply with the same nrhs first so that it
 * holds real activations).  Synchronises the stream. */
GNP_API gnp_status gnp_time_layer(gnp_model *model, int nrhs, gnp_precision prec, int reps,
                                  double *ms_per_launch, void *hip_stream);

/* The same launch timed with cold caches: before every layer launch a fill
 * kernel writes flush_bytes of flush_dev (device memory of the caller, at
 * least twice the 256 MB Infinity Cache to evict it and every L2), and the
 * time of `reps` fills alone is subtracted: *ms_per_launch = ((fill + layer)
 * x reps - fill x reps) / reps, all between hipEvents on hip_stream;
 * *ms_flush (optional) = one fill.  Synchronises the stream. */
GNP_API gnp_status gnp_time_layer_cold(gnp_model *model, int nrhs, gnp_precision prec, int reps,
                                       void *flush_dev, size_t flush_bytes, double *ms_per_launch,
                                       double *ms_flush, void *hip_stream);

/* Mean duration (ms) of one gnp_spmv launch (y = A x), measured the same way. */
GNP_API gnp_status gnp_time_spmv(const gnp_system *sys, const void *x_dev, void *y_dev,
                                 gnp_precision prec, int reps, double *ms_per_launch,
                                 void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* GNP_H */
