// FGMRES(m) solve context: device workspace and the device-resident control
// block that lets every kernel of an Arnoldi step exit early once the cycle
// has ended (Givens estimate below target, breakdown, or iteration limit),
// so the host synchronises only once per restart cycle.
#pragma once
#include "gnp_internal.hpp"
#include "model.hpp"

namespace gnp {

struct Ctl {
    int cycle_done;  // step kernels exit at entry when set
    int kcols;       // Arnoldi steps completed in the current cycle
    int kuse;        // columns used by the least-squares solution
    int it;          // Arnoldi steps in total
    int converged;
    int breakdowns;
    int restarts;
    int nonfinite;
    int solve_done;
    int m, maxiters, pad_;
    double bnorm, target, beta, est, rel_true, wnorm0, hnext, est_rel;
    // time limit (the paper's timeout criterion): 0 = none; the deadline is
    // set on the device when r_0 is known, and a step that ends after it
    // ends the solve
    uint64_t timeout_ticks, deadline;
    int timed_out, pad2_;
};

// Per-right-hand-side strides (elements) of a batched solve: right-hand
// side b = blockIdx.y of every solver kernel works on its own slices.  All
// zero (and vstep = 1) for a single solve.
struct Bat {
    int64_t vec = 0;    // n-vectors: b, x, r, w
    int64_t basis = 0;  // Krylov basis V (n * MP)
    int64_t part = 0;   // per-block partial sums
    int64_t hess = 0;   // H, H0 ((m + 1) * m)
    int64_t small = 0;  // cs, sn, g, y, h1, h2 (m + 1)
    int64_t hist = 0;   // residual history
    int vstep = 1;      // stride of the network input vector (nrhs when packed [n][nrhs])
};

// Preconditioner of a solve besides the network (which is passed as a model)
enum PrecondKind { PRECOND_MODEL = 0, PRECOND_JACOBI = 1, PRECOND_GMRES = 2 };

struct SolveCtx {
    gnp_system *sys = nullptr;
    int precond = PRECOND_MODEL;  // PRECOND_JACOBI: z_j = D^{-1} v_j (sys->dinv64);
                                  // PRECOND_GMRES: z_j = inner GMRES on A z = v_j
    int m = 0;
    int mp = 32;            // row pitch of the interleaved basis
    int maxiters_cap = 0;
    gnp_precision prec = GNP_F32;
    int64_t n = 0;
    size_t kbytes = 4;      // bytes per Krylov element
    void *V = nullptr;      // n x mp, row-interleaved basis (entries k <= m used)
    void *Z = nullptr;      // m x n, column-major network outputs
    void *vcur = nullptr;   // n, the current basis vector (network input)
    void *w = nullptr;      // n
    double *r = nullptr;    // n, float64 residual
    void *act[2] = {nullptr, nullptr};
    int act_d = 0;
    double *tau = nullptr;  // tau triple for the network input
    double *H = nullptr;    // (m+1) x m, rotated (upper triangle + zeros)
    double *H0 = nullptr;   // (m+1) x m, as built
    double *cs = nullptr, *sn = nullptr, *g = nullptr, *y = nullptr;
    double *h1 = nullptr, *h2 = nullptr;  // CGS2 pass coefficients
    double *hist = nullptr;               // maxiters_cap + 1
    // wall-clock stamps (wall_clock64 ticks): [0] once r_0 is known, [i] once
    // step i's residual estimate is known; maxiters_cap + 1
    uint64_t *tstamp = nullptr;
    double *partial = nullptr;
    int64_t npartial = 0;
    unsigned *counters = nullptr;
    Ctl *ctl = nullptr;
    Ctl *ctl_host = nullptr;  // pinned
    hipEvent_t ev = nullptr;
    // inner-outer GMRES: the inner solve's own context (m = inner_k, no
    // preconditioner) and its float64 solution
    SolveCtx *inner = nullptr;
    double *inner_x = nullptr;
    int inner_k = 0;
    double inner_tol = 0.0;
    double timeout_s = 0.0;  // time limit of the next solve_begin (0: none)
};

gnp_status solve_ctx_prepare(SolveCtx *c, gnp_system *sys, int m, int maxiters,
                             gnp_precision prec, int act_d);
// Device bytes solve_ctx_prepare allocates for these arguments.
size_t solve_ctx_bytes(int64_t n, int m, int maxiters, gnp_precision prec, int act_d);
void solve_ctx_free(SolveCtx *c);

// Stages of a solve, each enqueued on `st` without waiting; each ends with a
// copy of the control block to c->ctl_host, valid once the stream has
// reached that point.  solve_begin: ||b||, target and the initial residual;
// solve_next: one restart cycle (<= m Arnoldi steps, update of x, true
// residual).  The caller stops when ctl_host->solve_done is set (or b = 0,
// or ||b|| is not finite after solve_begin).
gnp_status solve_begin(SolveCtx *c, const double *b, const double *x, int m, double rtol,
                       int maxiters, hipStream_t st);
gnp_status solve_next(SolveCtx *c, gnp_model *model, const double *b, double *x, int m,
                      int maxiters, hipStream_t st);
void solve_info_from(const Ctl &h, gnp_solve_info *info);

// Enqueue the whole solve on `st` and run it to completion (one host sync per
// cycle).  x holds x0 on entry.
gnp_status solve_run(SolveCtx *c, gnp_model *model, const double *b, double *x, int m,
                     double rtol, int maxiters, double *hist_host, gnp_solve_info *info,
                     hipStream_t st);

}  // namespace gnp
