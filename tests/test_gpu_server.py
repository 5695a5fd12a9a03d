"""Solve server (continuous batching, HBM admission) on the GPU, through the C ABI.

Every served request runs the same kernels as a single fgmres_solve from
x0 = 0 on buffers of its own, so a result must be the same alone and in the
mix: same iteration count and the same solution bit for bit.  Solutions are
also checked against the matrix on the host (true residual).
"""
import time

import numpy as np
import pytest

from paper_2406_00809_amd import inputs as I

pytestmark = pytest.mark.gpu

M_RESTART, RTOL, MAXIT = 20, 1e-8, 1500


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    from paper_2406_00809_amd import api as A
    return A


@pytest.fixture(scope="module")
def fleet(api):
    """Four resident systems of different families and sizes, each with a
    briefly trained network (one unpreconditioned)."""
    specs = [("laplace2d_40", I.laplace2d(40), (4, 16, 32)),
             ("laplace3d_12", I.laplace3d(12), (4, 16, 32)),
             ("convdiff3d_16", I.convdiff3d(16), (8, 32, 64)),
             ("powerlaw_3000", I.powerlaw_random(3000, seed_structure=5, seed_values=6), None)]
    out = []
    for k, (name, A, arch) in enumerate(specs):
        S = api.System(A)
        M = None
        if arch is not None:
            L, d, h = arch
            M = api.Model(S, L, d, h, I.init_params(L, d, h, 40 + k))
            M.train(60, 8, lr=1e-3, seed=7 + k, prec="f32")
        out.append((name, A, S, M))
    return out


def _solve_alone(api, S, M, b):
    import torch
    bd = torch.as_tensor(b, dtype=torch.float64, device="cuda")
    x, info, _ = api.fgmres_solve(S, bd, M, m=M_RESTART, rtol=RTOL, maxiters=MAXIT,
                                  prec="bf16", want_hist=False)
    return x.cpu().numpy(), info


def _true_rel_res(A, S, x, b):
    Ad = A.to_scipy() / S.gamma_input
    return np.linalg.norm(b - Ad @ x) / np.linalg.norm(b)


def _collect(srv, tickets, timeout=300.0):
    res, t0 = {}, time.time()
    while len(res) < len(tickets):
        for t, n in tickets.items():
            if t in res:
                continue
            r = srv.poll(t, n)
            if r is not None:
                res[t] = r
        assert time.time() - t0 < timeout, "served requests did not finish"
        time.sleep(0.002)
    return res


def test_same_result_alone_and_in_the_mix(api, fleet):
    srv = api.Server(hbm_budget=8 << 30, max_slots=6, m=M_RESTART, max_iters=MAXIT, prec="bf16")
    ids = [srv.register(S, M) for _, _, S, M in fleet]
    reqs = []
    for rep in range(4):
        for k, (name, A, S, M) in enumerate(fleet):
            b = I.rhs_normal(A.n, 1000 + 10 * k + rep)
            reqs.append((k, b))
    tickets = {}
    order = []
    for k, b in reqs:
        t = srv.submit(ids[k], b, rtol=RTOL, maxiters=MAXIT)
        tickets[t] = fleet[k][1].n
        order.append((t, k, b))
    res = _collect(srv, tickets)
    st = srv.stats()
    print("stats", st)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["max_active"] > 1  # solves were in flight together
    for t, k, b in order:
        name, A, S, M = fleet[k]
        x, info, lat = res[t]
        xa, ia = _solve_alone(api, S, M, b)
        assert info["iters"] == ia["iters"], (name, info, ia)
        assert info["converged"] == ia["converged"]
        assert np.array_equal(x, xa), (name, np.max(np.abs(x - xa)))
        if info["converged"]:
            assert _true_rel_res(A, S, x, b) <= 1.5 * RTOL
    srv.close()


def test_hbm_budget_bounds_resident_workspaces(api, fleet):
    probe = api.Server(hbm_budget=1 << 40, max_slots=1, m=M_RESTART, max_iters=MAXIT)
    wsb = [probe.workspace_bytes(probe.register(S, M)) for _, _, S, M in fleet]
    probe.close()
    budget = max(wsb) + min(wsb)  # the fleet's workspaces never fit at once
    srv = api.Server(hbm_budget=budget, max_slots=8, m=M_RESTART, max_iters=MAXIT, prec="bf16")
    ids = [srv.register(S, M) for _, _, S, M in fleet]
    tickets = {}
    for rep in range(3):
        for k, (_, A, _, _) in enumerate(fleet):
            tickets[srv.submit(ids[k], I.rhs_normal(A.n, 2000 + 10 * k + rep), rtol=RTOL,
                               maxiters=MAXIT)] = A.n
    _collect(srv, tickets)
    st = srv.stats()
    print("stats", st, "workspace bytes", wsb)
    assert st["completed"] == len(tickets)
    assert st["hbm_peak"] <= budget
    assert st["workspaces_evicted"] > 0  # the fleet does not fit at once
    assert st["workspaces_reused"] > 0
    srv.close()


def test_oversized_request_is_rejected_others_run(api, fleet):
    probe = api.Server(hbm_budget=1 << 40, max_slots=1, m=M_RESTART, max_iters=MAXIT)
    wsb = [probe.workspace_bytes(probe.register(S, M)) for _, _, S, M in fleet]
    probe.close()
    big = int(np.argmax(wsb))
    small = int(np.argmin(wsb))
    srv = api.Server(hbm_budget=wsb[small] + 1, max_slots=4, m=M_RESTART, max_iters=MAXIT)
    ids = [srv.register(S, M) for _, _, S, M in fleet]
    A_big, A_small = fleet[big][1], fleet[small][1]
    t_big = srv.submit(ids[big], I.rhs_normal(A_big.n, 3), rtol=RTOL, maxiters=MAXIT)
    t_small = srv.submit(ids[small], I.rhs_normal(A_small.n, 4), rtol=RTOL, maxiters=MAXIT)
    srv.drain(300.0)
    with pytest.raises(api.GNPError) as e:
        srv.poll(t_big, A_big.n)
    assert "GNP_ENOMEM" in str(e.value)
    x, info, _ = srv.poll(t_small, A_small.n)
    assert info["iters"] > 0
    st = srv.stats()
    assert st["rejected"] == 1 and st["completed"] == 1
    srv.close()


def test_requests_admitted_while_others_run(api, fleet):
    """Continuous batching: short requests submitted after long ones start in
    the free slots and finish while the long ones still run."""
    srv = api.Server(hbm_budget=8 << 30, max_slots=3, m=M_RESTART, max_iters=MAXIT, prec="bf16")
    name, A_long, S_long, _ = fleet[2]                # convdiff3d_16, unpreconditioned: long
    sid_long = srv.register(S_long, None)
    _, A_short, S_short, M_short = fleet[0]           # laplace2d_40 with its network: short
    sid_short = srv.register(S_short, M_short)
    # an rtol below double precision: the long requests run all MAXIT steps;
    # the short ones stop after 40 steps
    long_t = [srv.submit(sid_long, I.rhs_normal(A_long.n, 50 + i), rtol=1e-30, maxiters=MAXIT)
              for i in range(2)]
    time.sleep(0.01)
    short_t = [srv.submit(sid_short, I.rhs_normal(A_short.n, 60 + i), rtol=RTOL, maxiters=40)
               for i in range(6)]
    tickets = {t: A_long.n for t in long_t}
    tickets.update({t: A_short.n for t in short_t})
    res = _collect(srv, tickets)
    lat_long = [res[t][2] for t in long_t]
    lat_short = [res[t][2] for t in short_t]
    assert all(res[t][1]["iters"] == MAXIT for t in long_t)
    assert all(res[t][1]["iters"] <= 40 for t in short_t)
    print("long latencies", lat_long, "short latencies", lat_short, srv.stats())
    # the six short requests went through the single free slot one after the
    # other while both long solves were running
    assert max(lat_short) < min(lat_long)
    st = srv.stats()
    assert st["max_active"] == 3
    assert st["latency_p50_s"] <= st["latency_p99_s"]
    srv.close()


def test_zero_and_nonfinite_rhs(api, fleet):
    srv = api.Server(hbm_budget=8 << 30, max_slots=2, m=M_RESTART, max_iters=MAXIT)
    _, A, S, M = fleet[0]
    sid = srv.register(S, M)
    t0 = srv.submit(sid, np.zeros(A.n), rtol=RTOL, maxiters=MAXIT)
    bn = I.rhs_normal(A.n, 9)
    bn[5] = np.nan
    t1 = srv.submit(sid, bn, rtol=RTOL, maxiters=MAXIT)
    srv.drain(60.0)
    x, info, _ = srv.poll(t0, A.n)
    assert info["converged"] == 1 and info["iters"] == 0 and not np.any(x)
    with pytest.raises(api.GNPError) as e:
        srv.poll(t1, A.n)
    assert "GNP_ENUMERIC" in str(e.value)
    with pytest.raises(api.GNPError):
        srv.submit(sid, bn, rtol=-1.0)
    srv.close()


def test_converged_counted_apart_from_completed(api, fleet):
    """Requests that stop at maxiters complete but do not count as converged:
    throughput and latency percentiles over the converged ones are reported
    separately."""
    srv = api.Server(hbm_budget=8 << 30, max_slots=4, m=M_RESTART, max_iters=MAXIT, prec="bf16")
    _, A, S, M = fleet[2]  # convdiff3d_16 with its network
    sid = srv.register(S, M)
    full = [srv.submit(sid, I.rhs_normal(A.n, 70 + i), rtol=RTOL, maxiters=MAXIT)
            for i in range(3)]
    short = [srv.submit(sid, I.rhs_normal(A.n, 80 + i), rtol=RTOL, maxiters=3) for i in range(2)]
    tickets = {t: A.n for t in full + short}
    res = _collect(srv, tickets)
    st = srv.stats()
    print(st, [res[t][1] for t in full])
    assert all(res[t][1]["converged"] == 1 for t in full)
    assert all(res[t][1]["converged"] == 0 for t in short)
    assert st["completed"] == 5 and st["converged"] == 3 and st["failed"] == 0
    assert 0 < st["converged_per_s"] and 0 < st["solves_per_s"]
    assert 0 < st["conv_latency_p50_s"] <= st["conv_latency_p99_s"]
    srv.close()


def test_register_while_requests_in_flight(api, fleet):
    """Systems registered while requests run (the registry grows many times)
    leave the running requests intact, and requests on the new ids run too."""
    srv = api.Server(hbm_budget=8 << 30, max_slots=6, m=M_RESTART, max_iters=MAXIT, prec="bf16")
    ids = [srv.register(S, M) for _, _, S, M in fleet]
    order, tickets = [], {}
    for k, (_, A, S, M) in enumerate(fleet):
        b = I.rhs_normal(A.n, 500 + k)
        t = srv.submit(ids[k], b, rtol=RTOL, maxiters=MAXIT)
        tickets[t] = A.n
        order.append((t, k, b))
    for rep in range(40):  # re-register the fleet under new ids while they run
        k = rep % len(fleet)
        _, A, S, M = fleet[k]
        nid = srv.register(S, M)
        if rep % 8 == 0:
            b = I.rhs_normal(A.n, 600 + rep)
            t = srv.submit(nid, b, rtol=RTOL, maxiters=MAXIT)
            tickets[t] = A.n
            order.append((t, k, b))
    res = _collect(srv, tickets)
    for t, k, b in order:
        name, A, S, M = fleet[k]
        x, info, _ = res[t]
        xa, ia = _solve_alone(api, S, M, b)
        assert info["iters"] == ia["iters"] and np.array_equal(x, xa), name
    srv.close()


def test_update_system_while_serving(api, fleet):
    """Evolving systems (Sec. 5): new values for a registered system while
    the server runs, with a short fine-tuning of its network.  Requests
    submitted after the update are solved on the new matrix: the same result
    as a single solve with the tuned network, the true residual of the new
    matrix below rtol, and the oracle's iteration count (FP64, the same tuned
    weights, the new matrix) within max(1, ceil(10 %)).  Requests queued
    before it converge on the old or the new values; the other systems are
    served throughout, unchanged."""
    import oracle as O
    import torch
    A0, A1 = I.convdiff3d(16, 10.0), I.convdiff3d(16, 15.0)
    assert np.array_equal(A0.colind, A1.colind) and np.array_equal(A0.rowptr, A1.rowptr)
    S = api.System(A0)
    M = api.Model(S, 8, 32, 64, I.init_params(8, 32, 64, 44))
    M.train(100, 8, lr=1e-3, seed=3, prec="f32")
    srv = api.Server(hbm_budget=8 << 30, max_slots=4, m=M_RESTART, max_iters=MAXIT, prec="bf16")
    sid = srv.register(S, M)
    _, Ao, So, Mo = fleet[0]
    oid = srv.register(So, Mo)
    before, others, tickets = [], [], {}
    for i in range(4):
        b = I.rhs_normal(A0.n, 700 + i)
        t = srv.submit(sid, b, rtol=RTOL, maxiters=MAXIT)
        before.append((t, b))
        tickets[t] = A0.n
        bo = I.rhs_normal(Ao.n, 710 + i)
        t = srv.submit(oid, bo, rtol=RTOL, maxiters=MAXIT)
        others.append((t, bo))
        tickets[t] = Ao.n
    hist, best = srv.update_system(sid, A1.val, tune_steps=40, batch=8, lr=1e-4, seed=9)
    print(f"tuning on the new values: loss {hist[0]:.4f} -> {hist[best]:.4f}")
    after = []
    for i in range(4):
        b = I.rhs_normal(A1.n, 720 + i)
        t = srv.submit(sid, b, rtol=RTOL, maxiters=MAXIT)
        after.append((t, b))
        tickets[t] = A1.n
    res = _collect(srv, tickets)
    srv.close()
    ref1 = O.System(A1)
    assert S.gamma_input == ref1.gamma_raw
    th = M.get_params()
    Ad0 = A0.to_scipy() / O.gamma(A0)
    Ad1 = ref1.A.to_scipy()
    for t, b in before:
        x, info, _ = res[t]
        assert info["converged"] == 1
        r0 = np.linalg.norm(b - Ad0 @ x) / np.linalg.norm(b)
        r1 = np.linalg.norm(b - Ad1 @ x) / np.linalg.norm(b)
        assert min(r0, r1) <= 1.5 * RTOL, (r0, r1)
    for t, b in after:
        x, info, _ = res[t]
        xa, ia = _solve_alone(api, S, M, b)
        assert info["iters"] == ia["iters"] and np.array_equal(x, xa)
        assert info["converged"] == 1
        assert np.linalg.norm(b - Ad1 @ x) / np.linalg.norm(b) <= 1.5 * RTOL
        r = O.fgmres(ref1, b, M_RESTART, RTOL, MAXIT, M="gnp", theta=th, arch=(8, 32, 64),
                     ortho=O.CGS2)
        it, it_ref = info["iters"], r["info"]["iters"]
        print(f"after the update: {it} iterations, oracle {it_ref}")
        assert abs(it - it_ref) <= max(1, int(np.ceil(0.1 * it_ref)))
    for t, bo in others:
        x, info, _ = res[t]
        xa, ia = _solve_alone(api, So, Mo, bo)
        assert info["iters"] == ia["iters"] and np.array_equal(x, xa)
