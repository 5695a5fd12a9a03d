"""Pins of the oracle's FGMRES (Algorithm 1, Sec. 2.1 and Eq. (1)).

* M = I reproduces GMRES: the per-iteration residual equals the minimum
  residual over the Krylov space, computed independently with numpy QR and
  lstsq on the explicit Krylov basis.
* Jacobi M = D^-1 reproduces right-preconditioned GMRES on A D^-1.
* M = A^-1 (dense) solves in one step and breaks down there.
* a dense direct solve bounds the error of the converged x.
* the Arnoldi relation A Z = V H-bar and orthonormality of V (Eq. (1)).
* for the nonlinear GNP preconditioner the cycle's x minimises the residual
  over x0 + span(Z) (numpy lstsq on A Z).
* monotone residuals; MGS and CGS2 agree; edge cases.
"""
import numpy as np
import pytest

import oracle as O
from paper_2406_00809_amd import inputs as I


def _sys(A):
    return O.System(A, prescale=True)


def _krylov_minres(Ad, b, kmax):
    """min_y ||b - A K_k y|| / ||b|| for k = 1..kmax via QR of the Krylov basis."""
    n = b.size
    out = []
    K = np.zeros((n, kmax))
    v = b / np.linalg.norm(b)
    for k in range(kmax):
        K[:, k] = v
        v = Ad @ v
        v /= np.linalg.norm(v)
        Q, _ = np.linalg.qr(K[:, :k + 1])
        AQ = Ad @ Q
        y, *_ = np.linalg.lstsq(AQ, b, rcond=None)
        out.append(np.linalg.norm(b - AQ @ y) / np.linalg.norm(b))
    return np.array(out)


@pytest.mark.parametrize("ortho", [O.MGS, O.CGS2])
def test_identity_preconditioner_is_gmres(ortho):
    A = I.random_small(60, 0.1, 1, diag_shift=4.0)
    S = _sys(A)
    b = np.random.default_rng(2).standard_normal(60)
    r = O.fgmres(S, b, m=20, rtol=1e-14, maxiters=12, ortho=ortho)
    ref = _krylov_minres(S.A.to_scipy().toarray(), b, 12)
    np.testing.assert_allclose(r["hist"][1:], ref, rtol=1e-9)


def test_jacobi_is_gmres_on_right_preconditioned_matrix():
    A = I.random_small(50, 0.12, 3, diag_shift=3.0)
    S = _sys(A)
    Ad = S.A.to_scipy().toarray()
    dinv = 1.0 / np.diag(Ad)
    b = np.random.default_rng(4).standard_normal(50)
    r = O.fgmres(S, b, m=15, rtol=1e-14, maxiters=10, M="diag", mat=dinv)
    ref = _krylov_minres(Ad * dinv[None, :], b, 10)
    np.testing.assert_allclose(r["hist"][1:], ref, rtol=1e-9)


def test_exact_inverse_one_step_breakdown():
    A = I.random_small(30, 0.2, 5, diag_shift=5.0)
    S = _sys(A)
    Ad = S.A.to_scipy().toarray()
    b = np.random.default_rng(6).standard_normal(30)
    r = O.fgmres(S, b, m=10, rtol=1e-10, maxiters=10, M="dense", mat=np.linalg.inv(Ad), dump=True)
    assert r["info"]["iters"] == 1 and r["info"]["converged"] == 1
    assert r["info"]["breakdowns"] == 1
    np.testing.assert_allclose(r["x"], np.linalg.solve(Ad, b), rtol=1e-12)
    # H-bar_1 = [1, ~0]^T
    assert abs(r["H"][0, 0] - 1.0) < 1e-12 and abs(r["H"][1, 0]) < 1e-13


def test_converged_solution_vs_direct_solve():
    A = I.laplace2d(8)
    S = _sys(A)
    Ad = S.A.to_scipy().toarray()
    b = np.random.default_rng(7).standard_normal(S.n)
    r = O.fgmres(S, b, m=10, rtol=1e-10, maxiters=500)
    assert r["info"]["converged"] == 1
    xs = np.linalg.solve(Ad, b)
    kappa = np.linalg.cond(Ad)
    assert np.linalg.norm(r["x"] - xs) / np.linalg.norm(xs) <= kappa * 1e-10
    assert r["info"]["rel_res_true"] <= 1e-10
    assert np.linalg.norm(b - Ad @ r["x"]) / np.linalg.norm(b) == pytest.approx(
        r["info"]["rel_res_true"], rel=1e-6)


@pytest.mark.parametrize("ortho", [O.MGS, O.CGS2])
def test_arnoldi_relation_and_orthonormality_gnp(ortho):
    A = I.convdiff3d(5)
    S = _sys(A)
    L, d, h = 2, 6, 12
    th = I.init_params(L, d, h, 8)
    b = np.random.default_rng(9).standard_normal(S.n)
    m = 12
    r = O.fgmres(S, b, m=m, rtol=1e-14, maxiters=m, M="gnp", theta=th, arch=(L, d, h),
                 ortho=ortho, dump=True)
    k = r["k"]
    assert k == m
    V, Z, H = r["V"][:k + 1].T, r["Z"][:k].T, r["H"][:k + 1, :k]
    Ad = S.A.to_scipy()
    lhs = Ad @ Z
    err = np.linalg.norm(lhs - V @ H) / (np.linalg.norm(Ad.toarray(), 2) * np.linalg.norm(Z))
    assert err < 1e-13
    tol = 1e-13 if ortho == O.CGS2 else 1e-10
    assert np.linalg.norm(V.T @ V - np.eye(k + 1)) < tol
    # z_j = M(v_j) with the oracle's own forward
    np.testing.assert_array_equal(Z[:, 3], O.gnp_forward(S, L, d, h, th, V[:, 3].copy()))


def test_flexible_cycle_minimises_over_span_of_Z():
    """x_m = x0 + Z y with y = argmin ||b - A(x0 + Z y)|| (Algorithm 1)."""
    A = I.convdiff3d(5)
    S = _sys(A)
    L, d, h = 2, 6, 12
    th = I.init_params(L, d, h, 10)
    b = np.random.default_rng(11).standard_normal(S.n)
    x0 = np.random.default_rng(12).standard_normal(S.n) * 0.1
    m = 8
    r = O.fgmres(S, b, m=m, rtol=1e-14, maxiters=m, M="gnp", theta=th, arch=(L, d, h), x0=x0,
                 dump=True)
    Ad = S.A.to_scipy()
    Z = r["Z"][:m].T
    r0 = b - Ad @ x0
    y, *_ = np.linalg.lstsq(Ad @ Z, r0, rcond=None)
    np.testing.assert_allclose(r["x"], x0 + Z @ y, rtol=1e-9, atol=1e-11)
    best = np.linalg.norm(r0 - (Ad @ Z) @ y) / np.linalg.norm(b)
    assert r["info"]["rel_res_true"] == pytest.approx(best, rel=1e-9)
    assert r["hist"][-1] == pytest.approx(best, rel=1e-8)


def test_monotone_residuals_and_restart():
    A = I.convdiff3d(6)
    S = _sys(A)
    b = np.random.default_rng(13).standard_normal(S.n)
    m = 5
    r = O.fgmres(S, b, m=m, rtol=1e-9, maxiters=400)
    hist = r["hist"]
    assert r["info"]["converged"] == 1 and r["info"]["restarts"] > 0
    for c in range(0, len(hist) - 1, m):  # within a cycle the estimate never rises
        seg = hist[c + 1:c + m + 1]
        assert np.all(np.diff(seg) <= 1e-15)
    # across cycles (true residual restarts) nondecreasing is impossible
    assert np.all(np.diff(hist[::m]) <= 1e-12)


def test_mgs_and_cgs2_same_iterations():
    A = I.convdiff3d(5)
    S = _sys(A)
    L, d, h = 2, 8, 16
    th = I.init_params(L, d, h, 14)
    b = np.random.default_rng(15).standard_normal(S.n)
    r1 = O.fgmres(S, b, 10, 1e-8, 600, M="gnp", theta=th, arch=(L, d, h), ortho=O.MGS)
    r2 = O.fgmres(S, b, 10, 1e-8, 600, M="gnp", theta=th, arch=(L, d, h), ortho=O.CGS2)
    i1, i2 = r1["info"]["iters"], r2["info"]["iters"]
    assert r1["info"]["converged"] and r2["info"]["converged"]
    assert abs(i1 - i2) <= max(1, int(np.ceil(0.1 * i1)))
    # first cycle agrees to rounding; later cycles drift because M is nonlinear
    np.testing.assert_allclose(r1["hist"][:11], r2["hist"][:11], rtol=1e-9)


def test_edge_cases():
    S = _sys(I.laplace2d(6))
    r = O.fgmres(S, np.zeros(S.n), 5, 1e-8, 50)
    assert r["info"]["iters"] == 0 and r["info"]["converged"] == 1
    assert np.all(r["x"] == 0)
    b = np.random.default_rng(16).standard_normal(S.n)
    r = O.fgmres(S, b, 5, 1e-8, 1)
    assert r["info"]["iters"] == 1 and r["info"]["converged"] == 0
    # already converged initial guess
    xs = np.linalg.solve(S.A.to_scipy().toarray(), b)
    r = O.fgmres(S, b, 5, 1e-8, 50, x0=xs)
    assert r["info"]["iters"] == 0 and r["info"]["converged"] == 1
    # m = 1 still converges (restarted GMRES(1) on an SPD-shifted matrix)
    r = O.fgmres(_sys(I.random_small(20, 0.1, 17, diag_shift=6.0)),
                 np.ones(20), 1, 1e-8, 500)
    assert r["info"]["converged"] == 1


# --- inner-outer GMRES (Sec. 3, "Compared methods") ---------------------------

def _krylov_argmin(Ad, v, k):
    """z = argmin over K_k(A, v) of ||v - A z|| (QR of the explicit Krylov basis)."""
    n = v.size
    K = np.zeros((n, k))
    u = v / np.linalg.norm(v)
    for i in range(k):
        K[:, i] = u
        u = Ad @ u
        u /= np.linalg.norm(u)
    Q, _ = np.linalg.qr(K)
    c, *_ = np.linalg.lstsq(Ad @ Q, v, rcond=None)
    z = Q @ c
    return z, np.linalg.norm(v - Ad @ z) / np.linalg.norm(v)


@pytest.mark.parametrize("ortho", [O.MGS, O.CGS2])
def test_inner_gmres_is_krylov_minimiser(ortho):
    """Each z_j is the minimum-residual point of K_k(A, v_j), found independently."""
    A = I.random_small(40, 0.15, 31, diag_shift=3.0)
    S = _sys(A)
    Ad = S.A.to_scipy().toarray()
    b = np.random.default_rng(32).standard_normal(40)
    k, m = 5, 4
    r = O.fgmres(S, b, m=m, rtol=1e-14, maxiters=m, M="gmres", inner=(k, 1e-15), ortho=ortho,
                 dump=True)
    assert r["k"] == m
    for j in range(m):
        v = r["V"][j]
        zb, _ = _krylov_argmin(Ad, v, k)
        np.testing.assert_allclose(r["Z"][j], zb, rtol=1e-9, atol=1e-11 * np.abs(zb).max())


def test_inner_gmres_one_step_closed_form():
    """k = 1: the minimiser over span{v} is z = (v^T A v / ||A v||^2) v."""
    A = I.convdiff3d(4)
    S = _sys(A)
    Ad = S.A.to_scipy()
    b = np.random.default_rng(33).standard_normal(S.n)
    m = 6
    r = O.fgmres(S, b, m=m, rtol=1e-14, maxiters=m, M="gmres", inner=(1, 1e-15), dump=True)
    for j in range(r["k"]):
        v = r["V"][j]
        Av = Ad @ v
        np.testing.assert_allclose(r["Z"][j], (v @ Av) / (Av @ Av) * v, rtol=1e-12, atol=1e-15)


def test_inner_gmres_stops_at_its_tolerance():
    """With tol between the minimal residuals of K_2 and K_3 the inner solve ends after
    three steps: z_0 is the K_3 minimiser although k = 8."""
    A = I.random_small(40, 0.15, 34, diag_shift=2.5)
    S = _sys(A)
    Ad = S.A.to_scipy().toarray()
    b = np.random.default_rng(35).standard_normal(40)
    v = b / np.linalg.norm(b)
    _, r2 = _krylov_argmin(Ad, v, 2)
    z3, r3 = _krylov_argmin(Ad, v, 3)
    assert r3 < 0.95 * r2
    tol = np.sqrt(r2 * r3)
    r = O.fgmres(S, b, m=1, rtol=1e-14, maxiters=1, M="gmres", inner=(8, tol), dump=True)
    np.testing.assert_allclose(r["Z"][0], z3, rtol=1e-9, atol=1e-11 * np.abs(z3).max())
    assert np.linalg.norm(v - Ad @ r["Z"][0]) <= tol


def test_inner_gmres_full_space_is_exact_inverse():
    """k >= n with a tiny tolerance: z = A^{-1} v, so the outer solve needs one step."""
    A = I.random_small(20, 0.2, 36, diag_shift=4.0)
    S = _sys(A)
    Ad = S.A.to_scipy().toarray()
    b = np.random.default_rng(37).standard_normal(20)
    r = O.fgmres(S, b, m=5, rtol=1e-10, maxiters=20, M="gmres", inner=(25, 1e-13))
    assert r["info"]["iters"] == 1 and r["info"]["converged"] == 1
    np.testing.assert_allclose(r["x"], np.linalg.solve(Ad, b), rtol=1e-9)


def test_inner_gmres_converges_where_restarted_gmres_stalls_less():
    """Outer FGMRES(10) with inner GMRES(10) needs fewer outer steps than GMRES(10)."""
    S = _sys(I.convdiff3d(6))
    b = np.random.default_rng(38).standard_normal(S.n)
    plain = O.fgmres(S, b, 10, 1e-8, 2000)
    io = O.fgmres(S, b, 10, 1e-8, 2000, M="gmres", inner=(10, 1e-6))
    assert plain["info"]["converged"] and io["info"]["converged"]
    assert io["info"]["iters"] < plain["info"]["iters"]
    assert io["info"]["rel_res_true"] <= 1e-8
