"""GPU parity of training: loss and hand-written gradient against the oracle,
central finite differences on the float64 instantiation (also at the full
64^3 / 32-right-hand-side training shape), the Philox sampler and Adam loop
against the oracle's training loop, and the torch.autograd binding."""
import os
import time

import numpy as np
import pytest

import oracle as O
from paper_2406_00809_amd import inputs as I

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available()
    from paper_2406_00809_amd import api as A
    return A


def _dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _nrel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


GRAD_CASES = {
    "laplace2d_16_d16": (lambda: I.laplace2d(16), 3, 16, 32, 4),
    "convdiff3d_8_d32": (lambda: I.convdiff3d(8), 4, 32, 64, 3),
    "powerlaw_3000_d32": (lambda: I.powerlaw_random(3000, seed_structure=3, seed_values=4),
                          2, 32, 64, 2),
    # rows (nodes x batch) not a multiple of the 16-row tile
    "ragged_laplace2d_13_d16": (lambda: I.laplace2d(13), 2, 16, 32, 3),
    # fewer rows than one tile
    "tiny_laplace2d_3_d32": (lambda: I.laplace2d(3), 1, 32, 64, 1),
    # batches that are multiples of 16 (a tile = right-hand sides of one node)
    "laplace2d_16_d16_b16": (lambda: I.laplace2d(16), 2, 16, 32, 16),
    # ... with rows longer than the 8 prefetched entries
    "powerlaw_3000_d32_b32": (lambda: I.powerlaw_random(3000, seed_structure=3, seed_values=4),
                              2, 32, 64, 32),
}


@pytest.mark.parametrize("case", list(GRAD_CASES))
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_loss_grad_matches_oracle(api, case, prec):
    mk, L, d, h, B = GRAD_CASES[case]
    A = mk()
    S = api.System(A)
    ref = O.System(A)
    th = I.init_params(L, d, h, 21)
    M = api.Model(S, L, d, h, th)
    b = O.spmm(ref.A, np.random.default_rng(22).standard_normal((A.n, B)))
    loss, g = M.loss_grad(_dev(b), prec=prec)
    lr, gr = O.loss_grad(ref, L, d, h, th, b)
    el, eg = abs(loss - lr) / lr, _nrel(g, gr)
    print(f"{case} {prec}: loss err {el:.2e} grad err {eg:.2e}")
    if prec == "f64":
        assert el < 1e-12 and eg < 1e-10
    else:
        assert el < 1e-5 and eg < 2e-3


def _roundings(n, B, L, d, h, row_max):
    """Roundings along one path from an input to the FP64 loss, counted
    with every product and sum rounded once (FMA rounds less): the scaling
    u = s b (1), the encoder's W1 u + c1 (2) and W2 with c2 (h + 1), per
    layer A-hat X (row_max) and [X | T] [U; W] (2 d), the decoder's W3 with
    c3 (d + 1), W4 with c4 (h + 1) and tau / sqrt(n) (1), the residual A z - b
    (row_max + 1), and the mean of the n B absolute residuals as the loss
    kernel adds them: a strided chain per thread over a grid of G =
    min(ceil(nB / 256), 2048) blocks of 256, a 64-lane butterfly (6) and the
    4 wavefronts (4), the same over the block partials, and the division."""
    rows = n * B
    G = min(-(-rows // 256), 2048)
    d_sum = -(-rows // (G * 256)) + 10 + -(-G // 256) + 10 + 1
    return (1 + 2 + (h + 1) + L * (row_max + 2 * d) + (d + 1) + (h + 1) + 1 + (row_max + 1)
            + d_sum)


def _fd_check(M, th, b, prec, rng, ndir, K, h=1e-6):
    """Central differences along random unit directions, with the Richardson
    guard: a direction counts only when the h and h/2 quotients agree.

    Roundoff floor: the loss is computed with K roundings along each path
    (_roundings).  In the probabilistic model of rounding errors (Higham and
    Mary, SIAM J. Sci. Comput. 41 (2019)), K independent relative errors of
    at most u = eps / 2 give a relative error below lambda sqrt(K) u except
    with probability about 2 exp(-lambda^2 / 2); lambda = 6 (1.5e-8), with
    |loss| as the scale of the sums (the loss is a mean of absolute values).
    The worst-case bound, gamma_K times the loss of the network with
    absolute weights, grows like the product of the layers' absolute gains
    and is of no use here.  Each loss value then errs by at most
    e = 6 sqrt(K) u |loss|, the h quotient by N = e / h, the h/2 quotient by
    2 N: the two quotients may differ by 3 N from roundoff (4 N taken, the
    rest for the O(h^2) terms), and the h quotient differs from g . v by N
    (2 N taken) plus the gradient's own rounding (1e-6 relative)."""
    loss, g = M.loss_grad(b, prec=prec)
    noise = 6.0 * np.sqrt(K) * (np.finfo(float).eps / 2) * abs(loss) / h
    used = 0
    for _ in range(4 * ndir):
        v = rng.standard_normal(th.size)
        v /= np.linalg.norm(v)
        f = {}
        for s in (h, -h, h / 2, -h / 2):
            M.set_params(th + s * v)
            f[s] = M.loss_grad(b, prec=prec)[0]
        q1 = (f[h] - f[-h]) / (2 * h)
        q2 = (f[h / 2] - f[-h / 2]) / h
        if abs(q1 - q2) > 4 * noise + 1e-7 * abs(q1):
            continue  # a ReLU or |.| kink lies inside the stencil
        used += 1
        assert abs(q1 - g @ v) <= 2 * noise + 1e-6 * abs(q1), (q1, g @ v, noise)
        if used >= ndir:
            break
    M.set_params(th)
    return used


def test_finite_differences_gpu_f64(api):
    A = I.convdiff3d(12)
    S = api.System(A)
    ref = O.System(A)
    L, d, h, B = 3, 32, 64, 2
    th = I.init_params(L, d, h, 23)
    M = api.Model(S, L, d, h, th)
    b = _dev(O.spmm(ref.A, np.random.default_rng(24).standard_normal((A.n, B))))
    K = _roundings(A.n, B, L, d, h, int(np.diff(A.rowptr).max()))
    assert _fd_check(M, th, b, "f64", np.random.default_rng(25), 6, K) >= 6


@pytest.mark.slow
def test_finite_differences_gpu_f64_full_training_shape(api):
    """64^3 convection-diffusion, 32 right-hand sides, L=8, d=32, h=64."""
    A = I.convdiff3d(64)
    S = api.System(A)
    L, d, h, B = 8, 32, 64, 32
    th = I.init_params(L, d, h, 12)
    M = api.Model(S, L, d, h, th)
    x = np.random.default_rng(26).standard_normal((A.n, B))
    b = _dev(A.to_scipy() @ x / S.gamma_input)
    t0 = time.time()
    K = _roundings(A.n, B, L, d, h, int(np.diff(A.rowptr).max()))
    used = _fd_check(M, th, b, "f64", np.random.default_rng(27), 3, K)
    print(f"full-shape FD: {used} directions in {time.time() - t0:.1f}s")
    assert used >= 3


def test_train_f64_fixed_batch_matches_oracle(api):
    """C1 protocol: 200 Adam steps on 16 fixed pairs; loss history, best step
    and weights against the oracle's training loop."""
    import torch
    A = I.laplace2d(32)
    S = api.System(A)
    L, d, h, B = 4, 16, 32, 16
    th0 = I.init_params(L, d, h, 10)
    M = api.Model(S, L, d, h, th0)
    xf = np.random.default_rng(1).standard_normal((A.n, B))
    hist, best = M.train(200, B, lr=1e-3, prec="f64", x_fixed=_dev(xf))
    ref_loss = np.load(os.path.join(GOLD, "c1_gnp_oracle_loss.npy"))
    ref_th = np.load(os.path.join(GOLD, "c1_gnp_oracle_trained.npy"))
    print("loss", hist[0], hist[best], "ref", ref_loss[0], ref_loss.min())
    np.testing.assert_allclose(hist[:20], ref_loss[:20], rtol=1e-10)
    np.testing.assert_allclose(hist, ref_loss, rtol=1e-6)
    assert best == int(np.argmin(ref_loss))
    assert _nrel(M.get_params(), ref_th) < 1e-6


def test_train_sampler_matches_oracle(api):
    """Philox4x32-10 + Box-Muller sampler and Adam: 3 steps, float64."""
    A = I.convdiff3d(8)
    S = api.System(A)
    ref = O.System(A)
    L, d, h, B = 3, 32, 64, 4
    th0 = I.init_params(L, d, h, 31)
    M = api.Model(S, L, d, h, th0)
    hist, best = M.train(3, B, lr=1e-3, seed=12345, prec="f64")
    th_r, hist_r, best_r, st = O.train(ref, L, d, h, th0, 3, B, lr=1e-3, seed=12345)
    np.testing.assert_allclose(hist, hist_r, rtol=1e-11)
    assert best == best_r
    assert _nrel(M.get_params(), th_r) < 1e-10


def test_gpu_trained_c1_solves_like_oracle_trained(api):
    A = I.laplace2d(32)
    S = api.System(A)
    L, d, h, B = 4, 16, 32, 16
    M = api.Model(S, L, d, h, I.init_params(L, d, h, 10))
    xf = np.random.default_rng(1).standard_normal((A.n, B))
    M.train(200, B, lr=1e-3, prec="f32", x_fixed=_dev(xf))
    ref = O.System(A)
    ref_th = np.load(os.path.join(GOLD, "c1_gnp_oracle_trained.npy"))
    b = I.rhs_normal(A.n, 0)
    x, info, _ = api.fgmres_solve(S, _dev(b), M, m=10, rtol=1e-8, maxiters=3000, prec="f32")
    r = O.fgmres(ref, b, 10, 1e-8, 3000, M="gnp", theta=ref_th, arch=(L, d, h), ortho=O.CGS2)
    print("gpu-trained", info, "oracle-trained", r["info"])
    assert info["converged"] == 1
    it, itr = info["iters"], r["info"]["iters"]
    assert abs(it - itr) <= max(1, int(np.ceil(0.1 * itr))), (it, itr)


def test_train_f32_full_shape_loss_decreases(api):
    """64^3 convection-diffusion, batch 32, fresh Philox batches: 30 steps."""
    import torch
    A = I.convdiff3d(64)
    S = api.System(A)
    L, d, h, B = 8, 32, 64, 32
    M = api.Model(S, L, d, h, I.init_params(L, d, h, 12))
    torch.cuda.synchronize()
    t0 = time.time()
    hist, best = M.train(30, B, lr=1e-3, seed=2, prec="f32")
    dt = time.time() - t0
    print(f"30 steps in {dt:.2f}s ({1e3 * dt / 30:.1f} ms/step); loss {hist[0]:.4f} -> "
          f"{hist[best]:.4f}")
    assert np.all(np.isfinite(hist))
    assert hist[best] < 0.9 * hist[0]


def test_teacher_forcing_full_shape(api):
    """Gradients at weights the GPU has trained: the full training shape
    (64^3 convection-diffusion, L = 8, d = 32, h = 64) is trained on the GPU
    in FP32 with fresh batches of 32; at steps 0, 100 and 400 the weights are
    handed to the oracle, and the loss and gradient on a fixed two-column
    batch are compared in FP64 and FP32.  The oracle cannot afford the
    training run itself; this checks the backward pass where training
    actually goes, with ReLU patterns unlike those of the initial weights.
    (Adam restarts at each stage: any weights the GPU produced will do.)"""
    A = I.convdiff3d(64)
    S = api.System(A)
    ref = O.System(A)
    L, d, h = 8, 32, 64
    M = api.Model(S, L, d, h, I.init_params(L, d, h, 12))
    b_np = O.spmm(ref.A, np.random.default_rng(28).standard_normal((A.n, 2)))
    b = _dev(b_np)
    done = 0
    for k in (0, 100, 400):
        if k > done:
            M.train(k - done, 32, lr=1e-3, seed=2 + k, prec="f32")
            done = k
        th = M.get_params()
        lr, gr = O.loss_grad(ref, L, d, h, th, b_np)
        for prec, tl, tg in (("f64", 1e-12, 1e-10), ("f32", 1e-5, 2e-3)):
            loss, g = M.loss_grad(b, prec=prec)
            el, eg = abs(loss - lr) / lr, _nrel(g, gr)
            print(f"step {k} {prec}: loss {loss:.6f} (oracle {lr:.6f}) err {el:.2e}, grad err {eg:.2e}")
            assert el < tl and eg < tg, (k, prec, el, eg)


def test_autograd_function_matches_oracle(api):
    import torch
    from paper_2406_00809_amd.autograd import gnp
    A = I.laplace2d(12)
    S = api.System(A)
    ref = O.System(A)
    L, d, h, B = 2, 16, 32, 3
    th0 = I.init_params(L, d, h, 41)
    M = api.Model(S, L, d, h, th0)
    theta = torch.tensor(th0, dtype=torch.float64, device="cuda", requires_grad=True)
    x = np.random.default_rng(42).standard_normal((A.n, B))
    b_np = O.spmm(ref.A, x)
    b = _dev(b_np)
    Ad = torch.tensor(ref.A.to_scipy().toarray(), dtype=torch.float64, device="cuda")
    z = gnp(b, theta, M, "f64")
    loss = (Ad @ z - b).abs().mean()
    loss.backward()
    lr, gr = O.loss_grad(ref, L, d, h, th0, b_np)
    assert abs(loss.item() - lr) <= 1e-12 * lr
    assert _nrel(theta.grad.cpu().numpy(), gr) < 1e-10
    # a linear functional <c, z>: gradient against central differences of gnp_apply
    c = torch.tensor(np.random.default_rng(43).standard_normal((A.n, B)), device="cuda")
    theta.grad = None
    (gnp(b, theta, M, "f64") * c).sum().backward()
    g = theta.grad.cpu().numpy()
    v = np.random.default_rng(44).standard_normal(th0.size)
    v /= np.linalg.norm(v)
    fv = []
    for s in (1e-6, -1e-6):
        M.set_params(th0 + s * v)
        fv.append(float((M.apply(b, prec="f64") * c).sum()))
    q = (fv[0] - fv[1]) / 2e-6
    assert abs(q - g @ v) <= 1e-6 * max(abs(q), 1e-4)
