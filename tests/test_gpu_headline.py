"""The timed workload, solved to rtol 1e-8, against the oracle's solve.

Workload: 3D 7-point convection-diffusion on a 64^3 grid (n = 262144,
Peclet 10, upwind), prescaled by gamma; b = A 1, x0 = 0; network L = 8,
d = 32, h = 64 trained on the GPU exactly as the benchmark trains it (init
seed 12, 2000 Adam steps, lr 1e-3, batch 32 of fresh x ~ N(0, I), Philox
seed 2, float32 training, the best-loss weights kept).  The weights go to
the oracle as data (gnp_params_get), and FGMRES(30) to rtol 1e-8
(Algorithm 1; Sec. 3, stopping criteria) runs on both sides:

* the bfloat16 network (the timed solve) and the float32 network (the
  paper's arithmetic) each converge, with a true relative residual, checked
  on the host in FP64, of at most 1e-8, and with an iteration count within
  max(1, ceil(10 %)) of the oracle's FP64 solve (classical Gram-Schmidt
  twice) with the same weights;
* both solutions are within the distance that two points of residual
  <= 1e-8 ||b|| can have, measured against the oracle's: ||x - x_ref|| <=
  2e-8 ||b|| / sigma_min(A), with sigma_min bounded below by the smallest
  eigenvalue of the symmetric part (closed form, checked against a dense
  eigensolver on a 6^3 grid in tests/test_oracle_bounds.py);
* one request served by the solve server (continuous batching, bfloat16)
  returns the single solve's iterations and solution bit for bit;
* every stage of the trained bfloat16 network on one basis vector stays
  within its elementwise rounding bound (tests/_bounds.py).
"""
import numpy as np
import pytest

import oracle as O
from paper_2406_00809_amd import inputs as I

from _bounds import (convdiff_lambda_min_sym, decoder_bound, encoder_bound, layer_bound,
                     quantize, quantized_system, worst)

pytestmark = pytest.mark.gpu

L, D, H, M_RESTART = 8, 32, 64, 30


@pytest.fixture(scope="module")
def trained():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    from paper_2406_00809_amd import api
    A = I.convdiff3d(64, 10.0)
    S = api.System(A)
    M = api.Model(S, L, D, H, I.init_params(L, D, H, 12))
    hist, best = M.train(2000, 32, lr=1e-3, seed=2, prec="f32")
    print(f"\ntrained: loss {hist[0]:.4f} -> {hist[best]:.5f} (best step {best})")
    th = M.get_params()
    ref = O.System(A)
    b = O.spmm(ref.A, np.ones(A.n))  # b = A 1 in the prescaled system
    r = O.fgmres(ref, b, M_RESTART, 1e-8, 3000, M="gnp", theta=th, arch=(L, D, H),
                 ortho=O.CGS2)
    print("oracle:", r["info"])
    return api, A, S, M, th, ref, b, r


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["bf16", "f32"])
def test_headline_solve_matches_oracle(trained, prec):
    import torch
    api, A, S, M, th, ref, b, r = trained
    bd = torch.as_tensor(b, dtype=torch.float64, device="cuda")
    x, info, hist = api.fgmres_solve(S, bd, M, m=M_RESTART, rtol=1e-8, maxiters=3000, prec=prec)
    xs = x.cpu().numpy()
    Asp = ref.A.to_scipy()
    true = np.linalg.norm(b - Asp @ xs) / np.linalg.norm(b)
    it, it_ref = info["iters"], r["info"]["iters"]
    dx = np.linalg.norm(xs - r["x"])
    smin = convdiff_lambda_min_sym(64, 10.0, ref.gamma_raw)
    print(f"{prec}: {it} iterations (oracle {it_ref}), true rel res {true:.2e}, "
          f"||x - x_ref|| = {dx:.2e}, bound {2e-8 * np.linalg.norm(b) / smin:.2e}")
    assert r["info"]["converged"] == 1
    assert info["converged"] == 1 and true <= 1e-8
    assert abs(it - it_ref) <= max(1, int(np.ceil(0.1 * it_ref)))
    assert smin > 0
    assert dx <= 2e-8 * np.linalg.norm(b) / smin


@pytest.mark.timeout(600)
def test_served_request_equals_single_solve(trained):
    import torch
    api, A, S, M, th, ref, b, r = trained
    bd = torch.as_tensor(b, dtype=torch.float64, device="cuda")
    x, info, _ = api.fgmres_solve(S, bd, M, m=M_RESTART, rtol=1e-8, maxiters=3000, prec="bf16",
                                  want_hist=False)
    srv = api.Server(8 << 30, max_slots=4, m=M_RESTART, max_iters=3000, prec="bf16")
    try:
        sid = srv.register(S, M)
        t = srv.submit(sid, b, rtol=1e-8, maxiters=3000)
        srv.drain(300)
        xs, inf_s, lat = srv.poll(t, A.n)
    finally:
        srv.close()
    it_ref = r["info"]["iters"]
    print(f"served: {inf_s['iters']} iterations (single {info['iters']}, oracle {it_ref}), "
          f"latency {lat * 1e3:.1f} ms")
    assert inf_s["iters"] == info["iters"] and inf_s["converged"] == 1
    assert np.array_equal(xs, x.cpu().numpy())
    assert abs(inf_s["iters"] - it_ref) <= max(1, int(np.ceil(0.1 * it_ref)))


@pytest.mark.timeout(600)
def test_trained_network_stage_bounds(trained):
    import torch
    api, A, S, M, th, ref, b, r = trained
    v = b / np.linalg.norm(b)  # a basis vector of the first cycle
    vd = torch.as_tensor(v, dtype=torch.float32, device="cuda")
    z, acts = M.apply_layers(vd, prec="bf16")
    vv = vd.cpu().numpy().astype(np.float64).reshape(A.n, 1)
    thq, Sq = quantize(th, L, D, H, "bf16"), quantized_system(ref, "bf16")
    mr = int(np.diff(A.rowptr).max())
    X = acts[0].float().cpu().numpy().astype(np.float64)
    E_ref = O.gnp_encoder(Sq, L, D, H, thq, vv)
    ratios = [("encoder", worst(X - E_ref, encoder_bound(thq, L, D, H, vv, E_ref, "bf16")))]
    for l in range(L):
        Xn = acts[l + 1].float().cpu().numpy().astype(np.float64)
        Y_ref = O.gnp_layer(Sq, L, D, H, thq, l, X)
        ratios.append((f"layer {l + 1}",
                       worst(Xn - Y_ref, layer_bound(Sq, thq, L, D, H, l, X, Y_ref, "bf16", mr))))
        X = Xn
    z_ref = O.gnp_decoder(Sq, L, D, H, thq, vv, X)
    zg = z.cpu().numpy().astype(np.float64).reshape(A.n, 1)
    ratios.append(("decoder", worst(zg - z_ref, decoder_bound(thq, L, D, H, vv, X, z_ref, "bf16"))))
    print("trained network, worst error / bound:", ", ".join(f"{s} {q:.3f}" for s, q in ratios))
    assert all(q <= 1.0 for _, q in ratios)
