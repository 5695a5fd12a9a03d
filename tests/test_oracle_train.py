"""Pins of the oracle's training pieces (Sec. 2.2 streaming pairs, Sec. 3
hyperparameters): Philox known answers, the normal sampler's distribution,
Adam against torch.optim.Adam, and the best-loss snapshot."""
import os

import numpy as np
import pytest

import oracle as O
from paper_2406_00809_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(t, 16) for t in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        np.testing.assert_array_equal(O.philox(ctr, key), np.array(out, dtype=np.uint32))


def test_normal_sampler_distribution():
    from scipy import stats
    z = O.normals(2, 0, 200000)
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # different steps and seeds give independent-looking streams
    z1 = O.normals(2, 1, 200000)
    assert abs(np.corrcoef(z, z1)[0, 1]) < 5 / np.sqrt(z.size)
    assert not np.array_equal(O.normals(3, 0, 10), z[:10])
    # element e depends only on (seed, step, e)
    np.testing.assert_array_equal(O.normals(2, 0, 10), z[:10])


def test_box_muller_from_philox_words():
    """One element by hand: 53-bit uniforms from the four Philox words."""
    seed, step, e = 123456789012, 7, 99
    w = O.philox([e & 0xffffffff, e >> 32, step, 0], [seed & 0xffffffff, seed >> 32])
    w = [int(t) for t in w]
    u1 = (((w[0] >> 5) << 26 | (w[1] >> 6)) + 0.5) / 2.0 ** 53
    u2 = (((w[2] >> 5) << 26 | (w[3] >> 6)) + 0.5) / 2.0 ** 53
    z = np.sqrt(-2 * np.log(u1)) * np.cos(2 * np.pi * u2)
    assert O.lib().or_normal(seed, step, e) == pytest.approx(z, rel=1e-15, abs=1e-15)


def test_adam_matches_torch():
    import torch
    rng = np.random.default_rng(1)
    th = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    p = torch.tensor(th.copy(), requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 30):
        g = rng.standard_normal(50) * (10.0 ** rng.uniform(-6, 1))
        O.adam(th, g, m, v, t)
        p.grad = torch.tensor(g)
        opt.step()
        np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-14, atol=1e-15)


def test_train_keeps_best_step_and_reduces_loss():
    S = O.System(I.laplace2d(8))
    L, d, h, B = 2, 8, 16, 4
    th0 = I.init_params(L, d, h, 3)
    th, hist, best, st = O.train(S, L, d, h, th0, steps=40, B=B, lr=1e-2, seed=5)
    assert st == 0
    assert best == int(np.argmin(hist))
    assert hist[best] < hist[0]
    # the returned parameters reproduce the best loss on that step's batch
    x = O.normals(5, best, S.n * B).reshape(S.n, B)
    b = O.spmm(S.A, x)
    assert O.loss_grad(S, L, d, h, th, b, want_grad=False) == hist[best]


def test_train_fixed_batch_is_deterministic():
    S = O.System(I.laplace2d(6))
    L, d, h, B = 1, 4, 8, 3
    th0 = I.init_params(L, d, h, 4)
    xf = np.random.default_rng(1).standard_normal((S.n, B))
    a = O.train(S, L, d, h, th0, steps=15, B=B, x_fixed=xf)
    b = O.train(S, L, d, h, th0, steps=15, B=B, x_fixed=xf)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    # first step's loss equals a direct evaluation at the initial weights
    bb = O.spmm(S.A, xf)
    assert a[1][0] == O.loss_grad(S, L, d, h, th0, bb, want_grad=False)


def test_loss_of_exact_inverse_is_zero():
    """The loss vanishes iff A M(b) = b: check with a 'network' that is exact
    on a diagonal system (A = 2I, prescaled to I): L = 0, d = h = 1, identity
    MLP on positive inputs; then M(b) = b = A^-1 b for b > 0."""
    n = 16
    A = I.dense_to_csr(2.0 * np.eye(n))
    S = O.System(A)
    th = np.zeros(I.n_params(0, 1, 1))
    lay = I.param_layout(0, 1, 1)
    for k in ("W1", "W2", "W3", "W4"):
        th[lay[k][0]] = 1.0
    b = np.random.default_rng(2).random((n, 2)) + 0.5
    loss, g = O.loss_grad(S, 0, 1, 1, th, b)
    assert loss < 1e-15


def _fans(L, d, h):
    """fan_in of every parameter in the packing order: W1, c1 (1), W2, c2
    (h), L x (U_l, W_l) (d), W3, c3 (d), W4, c4 (h)."""
    return np.concatenate([np.full(2 * h, 1.0), np.full(h * d + d, float(h)),
                           np.full(2 * L * d * d, float(d)), np.full(d * h + h, float(d)),
                           np.full(h + 1, float(h))])


@pytest.mark.parametrize("arch", [(4, 16, 32), (8, 32, 64)])
def test_default_init_params(arch):
    """The default initialisation (uniform on +-1/sqrt(fan_in), Philox stream
    3): within each block's bound, mean 0 and variance 1/(3 fan_in) within
    sampling error, one element rebuilt from the known-answer-pinned Philox
    words, deterministic in the seed and different across seeds."""
    from scipy import stats
    L, d, h = arch
    th = O.init_params(L, d, h, 7)
    fan = _fans(L, d, h)
    assert th.size == fan.size == O.nparams(L, d, h)
    assert np.all(np.abs(th) < 1 / np.sqrt(fan))
    w = th * np.sqrt(fan)  # uniform on (-1, 1) if the definition holds
    assert abs(w.mean()) < 5 * np.sqrt(1 / 3 / w.size)
    assert abs(w.var() - 1 / 3) < 5 * np.sqrt(4 / 45 / w.size)
    assert stats.kstest((w + 1) / 2, "uniform").pvalue > 1e-4
    for k in (0, 2 * h + 5, th.size - 1):
        o = O.philox([k & 0xFFFFFFFF, k >> 32, 0, 3], [7, 0])
        u = ((int(o[0] >> 5) << 26 | int(o[1] >> 6)) + 0.5) / 2.0 ** 53
        assert th[k] == (2 * u - 1) / np.sqrt(fan[k])
    assert np.array_equal(th, O.init_params(L, d, h, 7))
    assert not np.any(th == O.init_params(L, d, h, 8))
