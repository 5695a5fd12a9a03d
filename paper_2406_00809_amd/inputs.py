"""Seeded synthetic inputs shared by the HIP path, the tests and the oracle.

This module holds no arithmetic of the method itself: it only builds CSR
matrices of fixed families, right-hand sides and initial network weights from
explicit seeds.  The normalisation by gamma (Eq. (4)), the network and the
solver are computed independently by the library and by the oracle.

Families (stand-ins for the paper's SuiteSparse selection, Sec. 3 "Problems"):

* ``laplace2d(N)``   2D 5-point Dirichlet Laplacian, lexicographic p = i + N*j.
* ``laplace3d(N)``   3D 7-point Dirichlet Laplacian, p = i + N*j + N^2*k.
* ``convdiff3d(N, Pe)``  3D 7-point convection-diffusion -Lap(u) + w.grad(u) on
  (0,1)^3 with w = (Pe/sqrt(3)) (1,1,1), first-order upwind, rows scaled by h^2.
* ``powerlaw_random(n, ...)``  nonsymmetric random sparse matrix whose row
  lengths follow a discrete power law on {kmin..kmax}, N(0,1) off-diagonals and
  a diagonal of random sign with magnitude log-uniform in [1e-4, 1].

Every matrix is returned as CSR with int32 ``rowptr``/``colind`` (columns sorted
and unique within a row) and float64 ``val``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class CSR:
    n: int
    rowptr: np.ndarray  # int32 [n+1]
    colind: np.ndarray  # int32 [nnz]
    val: np.ndarray     # float64 [nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.colind, self.rowptr), shape=(self.n, self.n))

    def spmv_host(self, x: np.ndarray) -> np.ndarray:
        """Plain FP64 product used only to build right-hand sides b = A x."""
        return self.to_scipy() @ x


def _stencil(shape, offsets_vals, diag):
    """Build a CSR stencil matrix on a tensor grid with Dirichlet boundaries.

    offsets_vals: list of (axis, step, value) for off-diagonal couplings.
    Grid index p = i0 + N0*(i1 + N1*i2) (axis 0 fastest).
    """
    dims = len(shape)
    n = int(np.prod(shape))
    idx = np.arange(n, dtype=np.int64)
    coords = []
    rem = idx.copy()
    for a in range(dims):
        coords.append(rem % shape[a])
        rem //= shape[a]
    strides = [int(np.prod(shape[:a])) for a in range(dims)]
    rows, cols, vals = [idx], [idx], [np.full(n, diag, dtype=np.float64)]
    for axis, step, v in offsets_vals:
        c = coords[axis] + step
        ok = (c >= 0) & (c < shape[axis])
        rows.append(idx[ok])
        cols.append(idx[ok] + step * strides[axis])
        vals.append(np.full(int(ok.sum()), v, dtype=np.float64))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr.astype(np.int32), c.astype(np.int32), v


def laplace2d(N: int) -> CSR:
    """2D 5-point Dirichlet Laplacian on an N x N grid: diagonal 4, neighbours -1."""
    rp, ci, v = _stencil((N, N), [(0, -1, -1.0), (0, 1, -1.0), (1, -1, -1.0), (1, 1, -1.0)], 4.0)
    return CSR(N * N, rp, ci, v, f"laplace2d_{N}")


def laplace3d(N: int) -> CSR:
    """3D 7-point Dirichlet Laplacian on an N^3 grid: diagonal 6, neighbours -1."""
    offs = [(a, s, -1.0) for a in range(3) for s in (-1, 1)]
    rp, ci, v = _stencil((N, N, N), offs, 6.0)
    return CSR(N ** 3, rp, ci, v, f"laplace3d_{N}")


def convdiff3d(N: int, Pe: float = 10.0) -> CSR:
    """3D convection-diffusion -Lap(u) + w.grad(u), w = (Pe/sqrt 3)(1,1,1), upwind.

    h = 1/(N+1).  Row p (scaled by h^2): a_pp = 6 + h*(w1+w2+w3),
    a_{p,p-e_k} = -1 - h*w_k (upwind side), a_{p,p+e_k} = -1.
    """
    h = 1.0 / (N + 1)
    wk = Pe / math.sqrt(3.0)
    diag = 6.0 + h * 3.0 * wk
    offs = []
    for a in range(3):
        offs.append((a, -1, -1.0 - h * wk))
        offs.append((a, 1, -1.0))
    rp, ci, v = _stencil((N, N, N), offs, diag)
    return CSR(N ** 3, rp, ci, v, f"convdiff3d_{N}_Pe{Pe:g}")


def powerlaw_degrees(n: int, alpha: float, kmin: int, kmax: int, rng) -> np.ndarray:
    k = np.arange(kmin, kmax + 1)
    p = k.astype(np.float64) ** (-alpha)
    p /= p.sum()
    return rng.choice(k, size=n, p=p).astype(np.int64)


def powerlaw_random(n: int, alpha: float = 1.57461, kmin: int = 3, kmax: int = 64,
                    seed_structure: int = 3, seed_values: int = 4) -> CSR:
    """Random nonsymmetric sparse matrix with power-law row lengths.

    Row i has k_i entries (diagonal included), k_i ~ P(k) proportional to
    k^-alpha on {kmin..kmax}.  The k_i - 1 off-diagonal columns are uniform
    without replacement over [0,n) minus {i}; off-diagonal values are N(0,1);
    the diagonal is +-10^U(-4,0) with a random sign.
    """
    rs = np.random.default_rng(seed_structure)
    deg = powerlaw_degrees(n, alpha, kmin, kmax, rs)
    off = deg - 1
    rowptr_off = np.zeros(n + 1, dtype=np.int64)
    rowptr_off[1:] = np.cumsum(off)
    total = int(rowptr_off[-1])
    rows = np.repeat(np.arange(n, dtype=np.int64), off)
    cols = rs.integers(0, n - 1, size=total, dtype=np.int64)
    cols = cols + (cols >= rows)  # skip the diagonal: uniform over [0,n) \ {i}
    # redraw duplicated columns inside a row until every row is duplicate-free
    while True:
        order = np.lexsort((cols, rows))
        rows, cols = rows[order], cols[order]
        dup = np.zeros(total, dtype=bool)
        dup[1:] = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
        nd = int(dup.sum())
        if nd == 0:
            break
        redraw = rs.integers(0, n - 1, size=nd, dtype=np.int64)
        cols[dup] = redraw + (redraw >= rows[dup])
    rv = np.random.default_rng(seed_values)
    offv = rv.standard_normal(total)
    dmag = 10.0 ** rv.uniform(-4.0, 0.0, size=n)
    dsgn = np.where(rv.integers(0, 2, size=n) == 0, -1.0, 1.0)
    r_all = np.concatenate([rows, np.arange(n, dtype=np.int64)])
    c_all = np.concatenate([cols, np.arange(n, dtype=np.int64)])
    v_all = np.concatenate([offv, dsgn * dmag])
    order = np.lexsort((c_all, r_all))
    rowptr = np.zeros(n + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum(deg)
    return CSR(n, rowptr.astype(np.int32), c_all[order].astype(np.int32), v_all[order],
               f"powerlaw_{n}")


def random_small(n: int, density: float, seed: int, diag_shift: float = 0.0,
                 nonneg: bool = False) -> CSR:
    """Small random sparse matrix (tests): Bernoulli(density) pattern plus diagonal."""
    rng = np.random.default_rng(seed)
    mask = rng.random((n, n)) < density
    np.fill_diagonal(mask, True)
    vals = rng.random((n, n)) if nonneg else rng.standard_normal((n, n))
    dense = np.where(mask, vals, 0.0)
    dense[np.diag_indices(n)] += diag_shift
    dense[~mask] = 0.0
    return dense_to_csr(dense, f"random_{n}_{seed}", keep_pattern=mask)


def dense_to_csr(dense: np.ndarray, name: str = "dense", keep_pattern=None) -> CSR:
    n = dense.shape[0]
    pat = (dense != 0) if keep_pattern is None else keep_pattern
    rows, cols = np.nonzero(pat)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    return CSR(n, rowptr.astype(np.int32), cols.astype(np.int32),
               dense[rows, cols].astype(np.float64), name)


def permute(A: CSR, perm: np.ndarray) -> CSR:
    """P A P^T for the permutation new_index = perm[old_index]."""
    import scipy.sparse as sp
    S = A.to_scipy()
    P = sp.csr_matrix((np.ones(A.n), (perm, np.arange(A.n))), shape=(A.n, A.n))
    B = (P @ S @ P.T).tocsr()
    B.sort_indices()
    return CSR(A.n, B.indptr.astype(np.int32), B.indices.astype(np.int32),
               B.data.astype(np.float64), A.name + "_perm")


# ---------------------------------------------------------------------------
# network shapes and initial weights
# ---------------------------------------------------------------------------

def n_params(L: int, d: int, h: int) -> int:
    """Parameter count of the packed layout (encoder, L Res-GCONV, decoder)."""
    return (h + h + h * d + d) + L * 2 * d * d + (d * h + h + h + 1)


def param_layout(L: int, d: int, h: int):
    """Offsets of the packed parameter vector.

    Order: W1[1 x h], c1[h], W2[h x d], c2[d], then per layer l the keys
    "U_l", "W_l" ([d x d] each), then W3[d x h], c3[h], W4[h x 1], c4[1]; every matrix is
    row-major with the input index first (y = x @ M).
    """
    off = {}
    p = 0
    for name, size in (("W1", h), ("c1", h), ("W2", h * d), ("c2", d)):
        off[name] = (p, size)
        p += size
    for l in range(L):
        off[f"U_{l}"] = (p, d * d)
        p += d * d
        off[f"W_{l}"] = (p, d * d)
        p += d * d
    for name, size in (("W3", d * h), ("c3", h), ("W4", h), ("c4", 1)):
        off[name] = (p, size)
        p += size
    assert p == n_params(L, d, h)
    return off


def init_params(L: int, d: int, h: int, seed: int) -> np.ndarray:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) for every weight and bias, FP64."""
    rng = np.random.default_rng(seed)
    lay = param_layout(L, d, h)
    fan = {"W1": 1, "c1": 1, "W2": h, "c2": h, "W3": d, "c3": d, "W4": h, "c4": h}
    for l in range(L):
        fan[f"U_{l}"] = d
        fan[f"W_{l}"] = d
    out = np.empty(n_params(L, d, h), dtype=np.float64)
    for name, (o, s) in lay.items():
        bnd = 1.0 / math.sqrt(fan[name])
        out[o:o + s] = rng.uniform(-bnd, bnd, size=s)
    return out


def rhs_normal(n: int, seed: int, nrhs: int | None = None) -> np.ndarray:
    """b ~ N(0, I) drawn from numpy.random.default_rng(seed); shape [n] or [n, nrhs]."""
    rng = np.random.default_rng(seed)
    if nrhs is None:
        return rng.standard_normal(n)
    return rng.standard_normal((n, nrhs))


# ---------------------------------------------------------------------------
# the named workloads
# ---------------------------------------------------------------------------

WORKLOADS = {
    "c1_laplace2d_32": dict(family="laplace2d", N=32, L=4, d=16, h=32, m=10,
                            init_seed=10, rhs_seed=0),
    "c2_convdiff3d_64": dict(family="convdiff3d", N=64, Pe=10.0, L=8, d=32, h=64, m=30,
                             init_seed=12, rhs_seed=0),
    "c3_powerlaw_1m": dict(family="powerlaw", n=1 << 20, L=8, d=32, h=64,
                           init_seed=11, rhs_seed=5),
}


def make_matrix(spec: dict) -> CSR:
    fam = spec["family"]
    if fam == "laplace2d":
        return laplace2d(spec["N"])
    if fam == "laplace3d":
        return laplace3d(spec["N"])
    if fam == "convdiff3d":
        return convdiff3d(spec["N"], spec.get("Pe", 10.0))
    if fam == "powerlaw":
        return powerlaw_random(spec["n"])
    raise ValueError(fam)
