"""Elementwise error bounds for one stage of the network, by the arithmetic
each precision mode performs (rounding-error analysis in the standard model
fl(a op b) = (a op b)(1 + e), |e| <= u).

A stage's GPU output is compared with the oracle's FP64 evaluation of the
same stage (Sec. 2.3 encoder, Eq. (5) layer, decoder with s^-1 of Eq. (6))
on the GPU's own input and on the parameters as the kernels hold them
(`quantize`: A-hat and the MFMA weight operands rounded to bfloat16 through
float32, or to float32; the bias and output vectors to float32; rounding
these is deterministic, so the oracle takes them as given).  What remains is
the rounding done inside the stage, bounded element by element:

Res-GCONV layer, Y = ReLU(X U + (A-hat X) W), input X exact (the stored
activations).  The GPU sums T = A-hat X in FP32, rounds T to the operand
type of the product (u_t: 2^-8 for bfloat16, none for float32), forms
[X | T] [U; W] with FP32 accumulation and rounds ReLU of the result to the
storage type (u_y).  With T = A-hat X, S1 = |X| |U| and S2 = |A-hat| |X| |W|
(elementwise absolute values), ReLU 1-Lipschitz:

    |Y_gpu - Y_ref| <= c [ u_t |T| |W| + 2 g (S1 + S2) ] + u_y |Y_ref|

where g = (row length + 2d + 2) 2^-24 covers the FP32 accumulations and
c = 1.01 the second-order terms.  The encoder (hidden = ReLU(u W1 + c1)
rounded to the operand type, then W2 and c2, rounded to the storage type)
and the decoder (hidden = ReLU(X W3 + c3), then W4, c4, the FP64 factor
tau/sqrt(n), z stored as FP32) follow the same pattern.

For bfloat16 the bound is about 2^-8 of |T| |W| plus 2^-8 of |Y|: a wrong,
missing or shifted neighbour, a wrong row or mixed-up features move an
element by a term of the size of one neighbour's share of S2 or more, far
above it (tests/test_oracle_bounds.py plants such mistakes).
"""
from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24
UBF = 2.0 ** -8
C2ND = 1.01

# rounding inside a stage: T (and the encoder's hidden units) to the MFMA
# operand type, the stored output
UNITS = {"bf16": dict(t=UBF, y=UBF), "f32": dict(t=0.0, y=U32)}


def bf16_round(x):
    """Round to float32, then to the nearest bfloat16, ties to even (the
    conversions the library performs)."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def f32_round(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def _layout(L, d, h):
    out, p = {}, 0
    for name, size in [("W1", h), ("c1", h), ("W2", h * d), ("c2", d)]:
        out[name] = (p, size)
        p += size
    for l in range(L):
        out[f"layer{l}.U"] = (p, d * d)
        p += d * d
        out[f"layer{l}.W"] = (p, d * d)
        p += d * d
    for name, size in [("W3", d * h), ("c3", h), ("W4", h), ("c4", 1)]:
        out[name] = (p, size)
        p += size
    return out


def _unpack(theta, L, d, h):
    lay = _layout(L, d, h)
    g = {k: theta[o:o + s] for k, (o, s) in lay.items()}
    g["W2"] = g["W2"].reshape(h, d)
    g["W3"] = g["W3"].reshape(d, h)
    g["U"] = [g[f"layer{l}.U"].reshape(d, d) for l in range(L)]
    g["W"] = [g[f"layer{l}.W"].reshape(d, d) for l in range(L)]
    return g


def quantize(theta, L, d, h, mode):
    """The parameters as the kernels use them: the MFMA operands (W2, U_l,
    W_l, W3) in bfloat16 (through float32) or float32, the vectors (W1, c1,
    c2, c3, W4, c4) in float32."""
    th = np.array(theta, dtype=np.float64)
    rnd = bf16_round if mode == "bf16" else f32_round
    for name, (o, s) in _layout(L, d, h).items():
        mat = name in ("W2", "W3") or name.startswith("layer")
        th[o:o + s] = rnd(th[o:o + s]) if mat else f32_round(th[o:o + s])
    return th


def quantized_system(S, mode):
    """A copy of an oracle System whose A-hat is rounded as the kernels hold
    it (bfloat16 through float32, or float32)."""
    import copy
    Q = copy.copy(S)
    Q.ahat = bf16_round(S.ahat) if mode == "bf16" else f32_round(S.ahat)
    return Q


def _gather(S, X, absolute):
    import oracle as O
    from paper_2406_00809_amd.inputs import CSR
    n, B, d = X.shape
    a = np.abs(S.ahat) if absolute else S.ahat
    A = CSR(S.n, S.A.rowptr, S.A.colind, np.ascontiguousarray(a), "ahat")
    return O.spmm(A, (np.abs(X) if absolute else X).reshape(n, B * d)).reshape(n * B, d)


def layer_bound(Sq, thq, L, d, h, l, X, Y_ref, mode, max_row):
    """Bound of |Y_gpu - Y_ref| for Res-GCONV layer l; Sq, thq: the
    quantized system and parameters the reference was computed with."""
    u = UNITS[mode]
    g = (max_row + 2 * d + 2) * U32
    P = _unpack(thq, L, d, h)
    n, B, _ = X.shape
    Ua, Wa = np.abs(P["U"][l]), np.abs(P["W"][l])
    S1 = np.abs(X).reshape(n * B, d) @ Ua
    S2 = _gather(Sq, X, True) @ Wa
    bnd = 2 * g * (S1 + S2)
    del S1, S2
    if u["t"]:
        bnd += u["t"] * (np.abs(_gather(Sq, X, False)) @ Wa)
    return (C2ND * bnd).reshape(n, B, d) + u["y"] * np.abs(Y_ref)


def scale_factors(v, n):
    """sqrt(n) / ||v_k|| (0 for a zero column) and ||v_k|| / sqrt(n), FP64."""
    v2 = np.asarray(v, dtype=np.float64).reshape(n, -1)
    tau = np.sqrt((v2 * v2).sum(axis=0))
    return np.where(tau > 0, np.sqrt(n) / np.where(tau > 0, tau, 1.0), 0.0), tau / np.sqrt(n)


def encoder_bound(thq, L, d, h, v, E_ref, mode):
    """Bound of |X0_gpu - X0_ref| for the encoder with s(b)."""
    u = UNITS[mode]
    g = (h + 4) * U32
    P = _unpack(thq, L, d, h)
    n = E_ref.shape[0]
    si, _ = scale_factors(v, n)
    uu = (np.asarray(v, dtype=np.float64).reshape(n, -1) * si).reshape(-1)  # rows n B
    W2a = np.abs(P["W2"])
    bnd = np.empty((uu.size, d))
    for r0 in range(0, uu.size, 1 << 18):  # in row chunks
        ur = uu[r0:r0 + (1 << 18), None]
        hid = np.maximum(ur * P["W1"] + P["c1"], 0.0)
        habs = np.abs(ur) * np.abs(P["W1"]) + np.abs(P["c1"])
        bnd[r0:r0 + (1 << 18)] = u["t"] * (hid @ W2a) + 2 * g * (habs @ W2a + np.abs(P["c2"]))
    return C2ND * bnd.reshape(E_ref.shape) + u["y"] * np.abs(E_ref)


def decoder_bound(thq, L, d, h, v, XL, z_ref, mode):
    """Bound of |z_gpu - z_ref| for the decoder with s^-1 (FP32 sums, z
    stored as FP32)."""
    g = (d + h + 4) * U32
    P = _unpack(thq, L, d, h)
    n, B, _ = XL.shape
    _, so = scale_factors(v, n)
    Xa = np.abs(XL).reshape(n * B, d)
    S = np.empty(n * B)
    for r0 in range(0, n * B, 1 << 18):  # in row chunks
        hid = Xa[r0:r0 + (1 << 18)] @ np.abs(P["W3"]) + np.abs(P["c3"])
        S[r0:r0 + (1 << 18)] = hid @ np.abs(P["W4"]) + abs(P["c4"][0])
    bnd = C2ND * np.abs(so) * (2 * g * S.reshape(n, B)) + U32 * np.abs(
        np.asarray(z_ref).reshape(n, B))
    return bnd.reshape(np.shape(z_ref))


def convdiff_lambda_min_sym(N, pe, gamma):
    """Smallest eigenvalue of the symmetric part (A + A^T) / 2 of the
    prescaled N^3 upwind convection-diffusion matrix (diagonal 6 + h sum w,
    backward neighbours -1 - h w_k, forward -1; w = pe / sqrt(3) (1, 1, 1),
    h = 1 / (N + 1)), in closed form: a constant-coefficient 7-point operator
    with Dirichlet ends has eigenvalues a + sum_k 2 s_k cos(pi j_k / (N + 1)),
    s_k = -(1 + h w_k / 2), smallest at j_k = 1.  It bounds sigma_min(A) from
    below (||A x|| >= x^T A x for unit x)."""
    h = 1.0 / (N + 1)
    hw = h * pe / np.sqrt(3.0)
    return (6 + 3 * hw) * (1 - np.cos(np.pi * h)) / gamma


def worst(err, bound):
    """Largest err / bound (0 where both vanish; inf where only the bound does)."""
    err = np.abs(err)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(bound > 0, err / np.where(bound > 0, bound, 1.0),
                     np.where(err > 0, np.inf, 0.0))
    return float(r.max()) if r.size else 0.0


def maxnorm_rel(x, ref):
    """max_i |x_i - ref_i| / max_i |ref_i|."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(x - ref).max() / max(np.abs(ref).max(), 1e-300))
