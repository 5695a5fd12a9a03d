"""Pins of the oracle's CSR layer: generators, gamma (Eq. (4)), transpose, SpMV.

Closed forms are derived in the docstrings; library cross-checks use scipy.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from paper_2406_00809_amd import inputs as I


def test_nnz_closed_forms():
    # 2D 5-point: 5n - 4N (each of the 4 boundary sides drops N couplings)
    A = I.laplace2d(32)
    assert A.n == 1024 and A.nnz == 5 * 1024 - 4 * 32 == 4992
    # 3D 7-point: 7n - 6N^2 (each of the 6 faces drops N^2 couplings)
    A = I.convdiff3d(64)
    assert A.n == 262144 and A.nnz == 7 * 262144 - 6 * 64 ** 2 == 1810432


@pytest.mark.parametrize("N", [4, 9, 32])
def test_gamma_laplace_closed_form(N):
    # Eq. (4): interior rows of the 2D Laplacian have |4| + 4*|-1| = 8,
    # 3D: 6 + 6 = 12; the matrices are symmetric so both maxima agree.
    assert O.gamma(I.laplace2d(N)) == 8.0
    assert O.gamma(I.laplace3d(N)) == 12.0


def test_gamma_convdiff_closed_form():
    # interior row: (6 + h*sum w) + 3*(1 + h*w_k) + 3*1 = 12 + 2*h*sqrt(3)*Pe
    # (column sums equal the row sums by the stencil's translation symmetry)
    N, Pe = 64, 10.0
    h = 1.0 / (N + 1)
    expect = 12.0 + 6.0 * h * Pe / math.sqrt(3.0)
    assert abs(O.gamma(I.convdiff3d(N, Pe)) - expect) <= 4e-15 * expect


def test_gamma_takes_min_of_row_and_col():
    # rows: |1|+|-2| = 3, |0.5| = 0.5  -> max row sum 3
    # cols: |1| = 1,  |-2|+|0.5| = 2.5 -> max col sum 2.5; gamma = 2.5
    dense = np.array([[1.0, -2.0], [0.0, 0.5]])
    A = I.dense_to_csr(dense)
    assert O.gamma(A) == 2.5
    assert O.gamma(I.dense_to_csr(dense.T.copy())) == 2.5


def test_gamma_matches_scipy_abs_sums():
    A = I.powerlaw_random(3000, seed_structure=7, seed_values=8)
    S = abs(A.to_scipy())
    expect = min(S.sum(axis=1).max(), S.sum(axis=0).max())
    assert abs(O.gamma(A) - expect) <= 1e-13 * expect


def test_transpose_matches_scipy_and_involution():
    A = I.powerlaw_random(5000, seed_structure=9, seed_values=10)
    T = O.transpose(A)
    ref = A.to_scipy().T.tocsr()
    ref.sort_indices()
    np.testing.assert_array_equal(T.rowptr, ref.indptr)
    np.testing.assert_array_equal(T.colind, ref.indices)
    np.testing.assert_array_equal(T.val, ref.data)
    TT = O.transpose(T)
    np.testing.assert_array_equal(TT.rowptr, A.rowptr)
    np.testing.assert_array_equal(TT.colind, A.colind)
    np.testing.assert_array_equal(TT.val, A.val)


def test_spmm_matches_scipy():
    A = I.powerlaw_random(4000, seed_structure=11, seed_values=12)
    x = np.random.default_rng(1).standard_normal((4000, 3))
    y = O.spmm(A, x)
    ref = A.to_scipy() @ x
    np.testing.assert_allclose(y, ref, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(O.spmm(A, x[:, 0].copy()), ref[:, 0], rtol=1e-13, atol=1e-13)


def test_prescale_makes_gamma_one():
    S = O.System(I.convdiff3d(12))
    assert abs(S.gamma - 1.0) <= 4e-16
    np.testing.assert_array_equal(S.ahat, S.A.val / S.gamma)


def test_powerlaw_generator_statistics():
    A = I.powerlaw_random(1 << 16)
    deg = np.diff(A.rowptr)
    assert deg.min() >= 3 and deg.max() <= 64
    assert abs(deg.mean() - 12.0) < 0.3
    assert int(np.median(deg)) == 7
    # every row holds its diagonal, columns sorted and unique
    for i in np.random.default_rng(0).integers(0, A.n, 200):
        cols = A.colind[A.rowptr[i]:A.rowptr[i + 1]]
        assert np.all(np.diff(cols) > 0) and i in cols
