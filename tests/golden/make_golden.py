"""Write the stored fixtures of tests/golden/ by calling only the oracle.

c1_gnp_oracle_trained.npy: GNP weights (L=4, d=16, h=32) trained by the
oracle for 200 full-batch Adam steps (lr 1e-3) on the 2D 5-point Laplacian
32 x 32 (prescaled by gamma) with the fixed 16 pairs x = N(0, I) from
numpy.random.default_rng(1), b = A x, l1 loss; initial weights from
inputs.init_params(4, 16, 32, seed=10).  The best-loss step is kept.

c1_gnp_oracle_trained_noscale.npy / c1_gnp_oracle_loss_noscale.npy: the same
protocol for the network without the scaling of Eq. (6) (the ablation of
Sec. 3).
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2406_00809_amd import inputs as I  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def c1_weights(scaled=True):
    if not scaled:
        with O.without_scaling():
            return c1_weights(True)
    S = O.System(I.laplace2d(32))
    L, d, h = 4, 16, 32
    th0 = I.init_params(L, d, h, 10)
    xf = np.random.default_rng(1).standard_normal((S.n, 16))
    th, hist, best, st = O.train(S, L, d, h, th0, 200, 16, lr=1e-3, x_fixed=xf)
    assert st == 0
    return th, hist


if __name__ == "__main__":
    th, hist = c1_weights()
    np.save(os.path.join(HERE, "c1_gnp_oracle_trained.npy"), th)
    np.save(os.path.join(HERE, "c1_gnp_oracle_loss.npy"), hist)
    print("wrote", th.size, "weights; loss", hist[0], "->", hist.min())
    th, hist = c1_weights(scaled=False)
    np.save(os.path.join(HERE, "c1_gnp_oracle_trained_noscale.npy"), th)
    np.save(os.path.join(HERE, "c1_gnp_oracle_loss_noscale.npy"), hist)
    print("without Eq. (6) scaling: loss", hist[0], "->", hist.min())
