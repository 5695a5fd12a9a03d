"""CPU checks of the stage-wise comparison used by the GPU parity tests.

1. The oracle's stages (encoder with s(b), Res-GCONV layer of Eq. (5),
   decoder with s^-1 of Eq. (6)) composed in order give exactly the oracle's
   forward pass (bit for bit, activations included), so the per-stage
   references inherit every pin of the forward pass.
2. The elementwise bounds of tests/_bounds.py hold for an emulation of the
   reduced-precision arithmetic the GPU kernels perform (bfloat16 storage of
   A-hat, activations, gathered sums and weights with FP32 accumulation; and
   all-FP32), so they are not too tight for correct kernels.
3. Mistakes planted in an otherwise correctly rounded stage output (one
   16-row tile zeroed, one neighbour missing from a row, the rows of a tile
   shifted by one, two features of one row swapped, one right-hand side's
   gather read from another) each exceed the bound, so the GPU tests catch
   them.
"""
import numpy as np
import pytest

import oracle as O
from paper_2406_00809_amd import inputs as I

from _bounds import (_unpack, bf16_round, convdiff_lambda_min_sym, decoder_bound, encoder_bound,
                     layer_bound, quantize, quantized_system, worst)

L, D, H = 3, 32, 64


def _f32(x):
    return np.asarray(x, dtype=np.float32)


def _round(x, mode):
    return bf16_round(x) if mode == "bf16" else _f32(x).astype(np.float64)


@pytest.fixture(scope="module", params=["convdiff10_b2", "powerlaw3000_b1"])
def case(request):
    if request.param == "convdiff10_b2":
        A, B = I.convdiff3d(10, 10.0), 2
    else:
        A, B = I.powerlaw_random(3000, seed_structure=21, seed_values=22), 1
    S = O.System(A)
    th = I.init_params(L, D, H, 31)
    v = I.rhs_normal(A.n, 32, B)
    v = v.reshape(A.n, B)
    return A, S, th, v, B


def test_stages_compose_to_the_forward_pass(case):
    A, S, th, v, B = case
    z, acts = O.gnp_forward(S, L, D, H, th, v, return_acts=True)
    X = O.gnp_encoder(S, L, D, H, th, v)
    assert np.array_equal(X, acts[0])
    for l in range(L):
        X = O.gnp_layer(S, L, D, H, th, l, X)
        assert np.array_equal(X, acts[l + 1])
    assert np.array_equal(O.gnp_decoder(S, L, D, H, th, v, X), z)
    with O.without_scaling():
        z0 = O.gnp_forward(S, L, D, H, th, v)
        X = O.gnp_encoder(S, L, D, H, th, v)
        for l in range(L):
            X = O.gnp_layer(S, L, D, H, th, l, X)
        assert np.array_equal(O.gnp_decoder(S, L, D, H, th, v, X), z0)


def _emulate_layer(S, P, l, X, mode):
    """The GPU layer's arithmetic in numpy: A-hat in the storage type, T
    summed in FP32 neighbour by neighbour, rounded to the operand type, FP32
    product with the rounded weights, ReLU, output rounded."""
    n, B, d = X.shape
    a = _round(S.ahat, mode).astype(np.float32)
    Xf = _f32(X)
    T = np.zeros((n, B, d), dtype=np.float32)
    rp, ci = S.A.rowptr, S.A.colind
    lens = np.diff(rp)
    for j in range(int(lens.max())):
        rows = np.nonzero(lens > j)[0]
        k = rp[rows] + j
        T[rows] = T[rows] + a[k][:, None, None] * Xf[ci[k]]
    Tq = _f32(_round(T, mode)) if mode == "bf16" else T
    Uq, Wq = _f32(_round(P["U"][l], mode)), _f32(_round(P["W"][l], mode))
    p = Xf.reshape(-1, d) @ Uq + Tq.reshape(-1, d) @ Wq
    return _round(np.maximum(p, 0), mode).reshape(n, B, d)


def _emulate_encoder(P, v, mode):
    n = v.shape[0]
    tau = np.sqrt((v * v).sum(axis=0))
    u = _f32(np.sqrt(n) / tau * v).reshape(-1)
    hid = np.maximum(u[:, None] * _f32(P["W1"]) + _f32(P["c1"]), 0).astype(np.float32)
    hid = _f32(_round(hid, mode)) if mode == "bf16" else hid
    E = hid @ _f32(_round(P["W2"], mode)) + _f32(P["c2"])
    return _round(E, mode).reshape(n, v.shape[1], -1)


def _emulate_decoder(P, v, XL, mode):
    n, B, d = XL.shape
    tau = np.sqrt((v * v).sum(axis=0))
    hid = np.maximum(_f32(XL).reshape(-1, d) @ _f32(_round(P["W3"], mode)) + _f32(P["c3"]), 0)
    o = hid @ _f32(P["W4"]) + np.float32(P["c4"][0])
    return _f32((tau / np.sqrt(n)) * o.reshape(n, B)).astype(np.float64)


@pytest.mark.parametrize("mode", ["bf16", "f32"])
def test_bounds_hold_for_the_kernel_arithmetic(case, mode):
    A, S, th, v, B = case
    thq, Sq = quantize(th, L, D, H, mode), quantized_system(S, mode)
    P = _unpack(thq, L, D, H)
    mr = int(np.diff(A.rowptr).max())
    E = _emulate_encoder(P, v, mode)
    E_ref = O.gnp_encoder(Sq, L, D, H, thq, v)
    r_enc = worst(E - E_ref, encoder_bound(thq, L, D, H, v, E_ref, mode))
    X = E
    r_lay = []
    for l in range(L):
        Y = _emulate_layer(Sq, P, l, X, mode)
        Y_ref = O.gnp_layer(Sq, L, D, H, thq, l, X)
        r_lay.append(worst(Y - Y_ref, layer_bound(Sq, thq, L, D, H, l, X, Y_ref, mode, mr)))
        X = Y
    z_ref = O.gnp_decoder(Sq, L, D, H, thq, v, X)
    r_dec = worst(_emulate_decoder(P, v, X, mode) - z_ref,
                  decoder_bound(thq, L, D, H, v, X, z_ref, mode))
    print(mode, "worst error / bound: encoder", r_enc, "layers", r_lay, "decoder", r_dec)
    assert r_enc <= 1 and max(r_lay) <= 1 and r_dec <= 1
    # the bfloat16 bounds of the encoder and the layers, which the storage
    # roundings dominate, are not loose: the emulated errors reach a good
    # part of them (the FP32 accumulation terms are worst-case sums)
    if mode == "bf16":
        assert min(r_enc, min(r_lay)) > 0.2


def test_planted_mistakes_exceed_the_layer_bound(case):
    A, S, th, v, B = case
    mr = int(np.diff(A.rowptr).max())
    thq, Sq = quantize(th, L, D, H, "bf16"), quantized_system(S, "bf16")
    X = bf16_round(O.gnp_encoder(Sq, L, D, H, thq, v))
    Y_ref = O.gnp_layer(Sq, L, D, H, thq, 0, X)
    bnd = layer_bound(Sq, thq, L, D, H, 0, X, Y_ref, "bf16", mr)
    good = bf16_round(Y_ref)
    assert worst(good - Y_ref, bnd) <= 1
    n = A.n
    rows = good.reshape(n * B, D)
    planted = {}
    # (a) one 16-row tile zeroed
    t = (n * B // 16) // 2
    w = rows.copy()
    w[16 * t:16 * t + 16] = 0
    planted["tile zeroed"] = w
    # (b) one neighbour missing from one row (the oracle on A-hat without
    # it), in a shortest and in a longest row
    lens = np.diff(A.rowptr)
    for what, i in (("short", int(np.argmin(lens))), ("long", int(np.argmax(lens)))):
        ks = [k for k in range(A.rowptr[i], A.rowptr[i + 1]) if A.colind[k] != i]
        S2 = quantized_system(S, "bf16")
        S2.ahat = Sq.ahat.copy()
        S2.ahat[max(ks, key=lambda k: abs(Sq.ahat[k]))] = 0.0
        Y_drop = bf16_round(O.gnp_layer(S2, L, D, H, thq, 0, X)).reshape(n * B, D)
        w = rows.copy()
        w[i * B] = Y_drop[i * B]
        planted[f"neighbour missing ({what} row, {lens[i]} entries)"] = w
    # (c) the rows of one tile shifted by one
    w = rows.copy()
    w[16 * t:16 * t + 16] = rows[16 * t + 1:16 * t + 17]
    planted["tile shifted"] = w
    # (d) two features of one row swapped
    w = rows.copy()
    r = 16 * t + 5
    f = int(np.argmax(np.abs(rows[r, :16] - rows[r, 16:])))
    w[r, f], w[r, 16 + f] = rows[r, 16 + f], rows[r, f]
    planted["features swapped"] = w
    # (e) with several right-hand sides: one row of right-hand side 0
    # computed from right-hand side 1's activations
    if B > 1:
        Xs = X.copy()
        Xs[:, 0, :] = X[:, 1, :]
        Y_mix = bf16_round(O.gnp_layer(Sq, L, D, H, thq, 0, Xs)).reshape(n * B, D)
        w = rows.copy()
        w[16 * t] = Y_mix[16 * t]
        planted["other right-hand side read"] = w
    for what, w in planted.items():
        r = worst(w.reshape(good.shape) - Y_ref, bnd)
        print(f"{what}: worst error / bound {r:.1f}")
        assert r > 1, what


def test_convdiff_lambda_min_closed_form_small_grid():
    """The closed-form smallest eigenvalue of the symmetric part of the
    prescaled convection-diffusion matrix (used to bound the distance of two
    solutions of residual <= rtol) against a dense eigensolver, and the
    singular values of A above it."""
    A = I.convdiff3d(6, 10.0)
    ref = O.System(A)
    Ad = ref.A.to_scipy().toarray()
    lam = np.linalg.eigvalsh((Ad + Ad.T) / 2).min()
    assert abs(lam - convdiff_lambda_min_sym(6, 10.0, ref.gamma_raw)) <= 1e-12 * abs(lam)
    assert np.linalg.svd(Ad, compute_uv=False).min() >= lam * (1 - 1e-12)
