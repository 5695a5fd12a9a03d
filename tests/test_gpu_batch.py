"""Batched FGMRES (fgmres_solve_batch) on the GPU, through the C ABI.

Every right-hand side of a batch runs the single-solve arithmetic step for
step (the network is applied to the whole batch at once, each row with the
same operations), so its iteration count and solution must equal those of
fgmres_solve bit for bit; solutions are also checked against the matrix.
"""
import numpy as np
import pytest

from paper_2406_00809_amd import inputs as I

pytestmark = pytest.mark.gpu

RTOL = 1e-8


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    from paper_2406_00809_amd import api as A
    return A


def _model(api, A, L, d, h, seed, steps=60):
    S = api.System(A)
    M = api.Model(S, L, d, h, I.init_params(L, d, h, seed))
    M.train(steps, 8, lr=1e-3, seed=seed + 1, prec="f32")
    return S, M


def _single(api, S, M, b, m, prec, maxiters):
    import torch
    bd = torch.as_tensor(b, dtype=torch.float64, device="cuda")
    x, info, _ = api.fgmres_solve(S, bd, M, m=m, rtol=RTOL, maxiters=maxiters, prec=prec,
                                  want_hist=False)
    return x.cpu().numpy(), info


CASES = {
    "laplace2d_40_d16_nb5": (lambda: I.laplace2d(40), (4, 16, 32), 5, 20),
    "convdiff3d_16_d32_nb16": (lambda: I.convdiff3d(16), (8, 32, 64), 16, 30),
    "powerlaw_4000_d32_nb3": (lambda: I.powerlaw_random(4000, seed_structure=11,
                                                        seed_values=12), (4, 32, 64), 3, 30),
    "laplace2d_30_d16_nb1": (lambda: I.laplace2d(30), (3, 16, 32), 1, 10),
    # restart 40: basis pitch 64, where single solves launch the third
    # Gram-Schmidt pass themselves
    "convdiff3d_12_d32_nb4_m40": (lambda: I.convdiff3d(12), (4, 32, 64), 4, 40),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("prec", ["bf16", "f32"])
def test_batch_equals_single_solves(api, case, prec):
    import torch
    mk, (L, d, h), nb, m = CASES[case]
    A = mk()
    S, M = _model(api, A, L, d, h, 70)
    maxiters = 600
    Bh = np.stack([I.rhs_normal(A.n, 900 + k) for k in range(nb)])
    X, infos = api.fgmres_solve_batch(S, torch.as_tensor(Bh, device="cuda"), M, m=m, rtol=RTOL,
                                      maxiters=maxiters, prec=prec)
    Xh = X.cpu().numpy()
    Ad = A.to_scipy() / S.gamma_input
    for k in range(nb):
        xs, info = _single(api, S, M, Bh[k], m, prec, maxiters)
        assert infos[k]["iters"] == info["iters"], (k, infos[k], info)
        assert infos[k]["converged"] == info["converged"]
        assert np.array_equal(Xh[k], xs), (k, np.max(np.abs(Xh[k] - xs)))
        if infos[k]["converged"]:
            res = np.linalg.norm(Bh[k] - Ad @ Xh[k]) / np.linalg.norm(Bh[k])
            assert res <= 1.5 * RTOL


def test_batch_zero_rhs_and_errors(api):
    import torch
    A = I.laplace2d(20)
    S, M = _model(api, A, 3, 16, 32, 80, steps=20)
    Bh = np.stack([I.rhs_normal(A.n, 1), np.zeros(A.n), I.rhs_normal(A.n, 2)])
    X0 = torch.ones((3, A.n), dtype=torch.float64, device="cuda")
    X, infos = api.fgmres_solve_batch(S, torch.as_tensor(Bh, device="cuda"), M, X=X0, m=10,
                                      rtol=RTOL, maxiters=400, prec="bf16")
    Xh = X.cpu().numpy()
    assert not np.any(Xh[1]) and infos[1]["converged"] == 1 and infos[1]["iters"] == 0
    for k in (0, 2):  # the others run as single solves from the same x0
        x0 = torch.ones(A.n, dtype=torch.float64, device="cuda")
        xs, info, _ = api.fgmres_solve(S, torch.as_tensor(Bh[k], device="cuda"), M, x=x0, m=10,
                                       rtol=RTOL, maxiters=400, prec="bf16", want_hist=False)
        assert infos[k]["iters"] == info["iters"] and infos[k]["converged"] == info["converged"]
        assert np.array_equal(Xh[k], xs.cpu().numpy())
    with pytest.raises(api.GNPError):
        api.fgmres_solve_batch(S, torch.as_tensor(Bh, device="cuda"), M, prec="f64")
    Bn = Bh.copy()
    Bn[2, 3] = np.inf
    with pytest.raises(api.GNPError) as e:
        api.fgmres_solve_batch(S, torch.as_tensor(Bn, device="cuda"), M, prec="bf16")
    assert "GNP_ENUMERIC" in str(e.value)
