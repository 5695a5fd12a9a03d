"""The no-allocation network apply (gnp_apply_noalloc), through the C ABI.

It runs gnp_apply's kernels on a fixed device array instead of the model's
workspace, so its output must equal gnp_apply's bit for bit (the parity
bar of gnp_apply against the oracle carries over).  Checked on two calls in
a row, the second with a smaller input, in every precision; the device's
free memory does not change across calls made before the model has any
apply workspace (after one earlier call, which lets the HIP runtime set up
its private memory for register spills); an apply that does not fit the
array is rejected.
"""
import ctypes as C

import numpy as np
import pytest

from paper_2406_00809_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    from paper_2406_00809_amd import api as A
    return A


def _noalloc(api, M, v, z, nrhs, prec):
    import torch
    from paper_2406_00809_amd import _lib
    st = _lib.load().gnp_apply_noalloc(M.handle, C.c_void_p(v.data_ptr()),
                                       C.c_void_p(z.data_ptr()), int(nrhs), api.PREC[prec],
                                       C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


@pytest.mark.parametrize("prec", ["bf16", "f32", "f64"])
def test_noalloc_equals_apply_two_calls(api, prec):
    import torch
    from paper_2406_00809_amd._lib import GNP_OK
    dt = torch.float64 if prec == "f64" else torch.float32
    cases = [(I.convdiff3d(20, 10.0), 3, (8, 32, 64), 31),   # n = 8000, 3 right-hand sides
             (I.laplace2d(23), 1, (4, 16, 32), 32)]           # smaller: n = 529, one
    models = []
    for A, nrhs, (L, d, h), seed in cases:
        S = api.System(A)
        models.append((A, nrhs, S, api.Model(S, L, d, h, I.init_params(L, d, h, seed))))
    outs = []
    for A, nrhs, S, M in models:  # every tensor of the test allocated up front
        v = torch.as_tensor(I.rhs_normal(A.n, 5, nrhs if nrhs > 1 else None), dtype=dt,
                            device="cuda").contiguous()
        outs.append((v, torch.full_like(v, float("nan"))))
    # one untimed call first: the HIP runtime sets up its per-queue private
    # memory (register spills of the float64 kernels) on a kernel's first
    # launch; that is the runtime's, not a workspace of the call
    A, nrhs, S, M = models[0]
    warm = torch.empty_like(outs[0][0])
    assert _noalloc(api, M, outs[0][0], warm, nrhs, prec) == GNP_OK
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for (A, nrhs, S, M), (v, z) in zip(models, outs):  # two calls, the second smaller
        assert _noalloc(api, M, v, z, nrhs, prec) == GNP_OK
    torch.cuda.synchronize()
    # no allocation: the models have no apply workspace yet, and the
    # device's free memory is unchanged
    assert torch.cuda.mem_get_info()[0] == free0
    for (A, nrhs, S, M), (v, z) in zip(models, outs):
        z_ref = M.apply(v, prec=prec)
        assert torch.equal(z, z_ref), (A.name, prec)
    # and again after gnp_apply ran (the array keeps the last call's data)
    A, nrhs, S, M = models[0]
    v, _ = outs[0]
    z = torch.empty_like(v)
    assert _noalloc(api, M, v, z, nrhs, prec) == GNP_OK
    assert torch.equal(z, M.apply(v, prec=prec))


def test_noalloc_rejects_what_does_not_fit(api):
    import torch
    from paper_2406_00809_amd._lib import GNP_EINVAL
    A = I.convdiff3d(64, 10.0)
    S = api.System(A)
    M = api.Model(S, 2, 32, 64, I.init_params(2, 32, 64, 3))
    v = torch.ones((A.n, 4), dtype=torch.float32, device="cuda")
    z = torch.empty_like(v)
    assert _noalloc(api, M, v, z, 4, "f32") == GNP_EINVAL  # 2 x 128 MiB of activations
    v1 = torch.ones(A.n, dtype=torch.float32, device="cuda")
    z1 = torch.empty_like(v1)
    assert _noalloc(api, M, v1, z1, 1, "bf16") == 0
    assert torch.equal(z1, M.apply(v1, prec="bf16"))
