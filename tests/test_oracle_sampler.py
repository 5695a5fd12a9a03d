"""Pins of the oracle's training-pair sampler (Sec. 2.2, Eqs. (2)-(3)).

The sampler runs m unpreconditioned Arnoldi steps, A V_m = V_{m+1} Hbar_m,
takes the thin SVD Hbar_m = W S Z^T and draws x = V_m Z S^{-1} eps.  What
fixes it, independently of its own code:
* the algebra the paper states: b = A x = V_{m+1} W eps exactly, x lies in
  range(V_m), and the covariance of b, (V_{m+1} W)(V_{m+1} W)^T, is a
  projector;
* the limit the paper names: with a full Arnoldi run (m = n, no breakdown
  before step n) the covariance of b is the identity and that of x is
  A^{-1} A^{-T};
* the SVD factors against the definition (orthonormal, Hbar = W S Z^T) and
  the canonical form (decreasing values, sign rule);
* the random streams: stream 0 is the training sampler's, stream 1 differs.
"""
import numpy as np
import pytest

import oracle as O
from paper_2406_00809_amd import inputs as I


def _dense_csr(M):
    n = M.shape[0]
    rp = np.zeros(n + 1, dtype=np.int32)
    ci, va = [], []
    for i in range(n):
        nz = np.nonzero(M[i])[0]
        ci.extend(nz.tolist())
        va.extend(M[i, nz].tolist())
        rp[i + 1] = len(ci)
    return I.CSR(n, rp, np.asarray(ci, dtype=np.int32), np.asarray(va), "dense")


@pytest.fixture(scope="module")
def cd():
    A = I.convdiff3d(6)  # n = 216, nonsymmetric
    S = O.System(A)
    return S, O.arnoldi_sampler(S, 12, seed=3)


def test_svd_factors_and_canonical_form(cd):
    S, sp = cd
    k = sp["k"]
    assert k == 12
    W, s, Z, Hb = sp["W"], sp["s"], sp["Z"], sp["Hbar"]
    assert Hb.shape == (13, 12)
    np.testing.assert_allclose(W.T @ W, np.eye(k), atol=1e-13)
    np.testing.assert_allclose(Z.T @ Z, np.eye(k), atol=1e-13)
    np.testing.assert_allclose(W @ np.diag(s) @ Z.T, Hb, atol=1e-13 * s[0])
    assert np.all(np.diff(s) <= 0)
    for c in range(k):
        i = int(np.argmax(np.abs(Z[:, c])))
        assert Z[i, c] > 0
    # Arnoldi relation of Eq. (2) holds for the basis returned
    V = sp["V"]
    A = S.A.to_scipy()
    np.testing.assert_allclose(A @ V[:, :k], V @ Hb, atol=1e-12)
    np.testing.assert_allclose(V.T @ V, np.eye(k + 1), atol=1e-12)


def test_b_equals_V_W_eps(cd):
    """A x = V_{m+1} Hbar Z S^{-1} eps = V_{m+1} W eps."""
    S, sp = cd
    k = sp["k"]
    eps = O.sampler_eps(sp, step=4, count=5)
    x = O.sampler_draw(sp, step=4, count=5)
    b = S.A.to_scipy() @ x
    b2 = sp["V"] @ (sp["W"] @ eps.T)
    assert np.linalg.norm(b - b2) <= 1e-12 * np.linalg.norm(b)
    # x in range(V_m)
    Vm = sp["V"][:, :k]
    assert np.linalg.norm(x - Vm @ (Vm.T @ x)) <= 1e-12 * np.linalg.norm(x)


def test_cov_b_is_projector(cd):
    S, sp = cd
    Q = sp["V"] @ sp["W"]  # n x m, orthonormal columns
    P = Q @ Q.T
    np.testing.assert_allclose(P @ P, P, atol=1e-12)
    assert abs(np.trace(P) - sp["k"]) <= 1e-10


def test_full_arnoldi_covariances():
    """m = n on a matrix with distinct eigenvalues: Cov(b) = I and
    Cov(x) = A^{-1} A^{-T}."""
    rng = np.random.default_rng(17)
    n = 10
    M = rng.standard_normal((n, n)) + 8.0 * np.eye(n)
    A = _dense_csr(M)
    S = O.System(A, prescale=False)
    sp = O.arnoldi_sampler(S, n, seed=9)
    assert sp["k"] == n
    Q = sp["V"] @ sp["W"]
    np.testing.assert_allclose(Q @ Q.T, np.eye(n), atol=1e-10)
    X = sp["V"][:, :n] @ sp["G"]  # x = X eps, Cov(x) = X X^T
    Ainv = np.linalg.inv(M)
    np.testing.assert_allclose(X @ X.T, Ainv @ Ainv.T, rtol=1e-8, atol=1e-12)


def test_streams():
    assert np.array_equal(O.normals_stream(5, 3, 0, 64), O.normals(5, 3, 64))
    a, b = O.normals_stream(5, 3, 1, 64), O.normals_stream(5, 3, 0, 64)
    assert not np.any(a == b)
    assert np.array_equal(O.normals_stream(5, 3, 1, 64), a)  # reproducible
