"""Python-facing objects over the C ABI (include/gnp.h).

Tensors are PyTorch device tensors; this module only checks shapes, dtypes
and devices, and passes raw pointers and the current HIP stream.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import GNP_BF16, GNP_F32, GNP_F64, GNPError, SolveInfo, TrainOpts, check

PREC = {"f64": GNP_F64, "f32": GNP_F32, "bf16": GNP_BF16,
        GNP_F64: GNP_F64, GNP_F32: GNP_F32, GNP_BF16: GNP_BF16}
KDTYPE = {GNP_F64: torch.float64, GNP_F32: torch.float32, GNP_BF16: torch.float32}


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_ptr(t: torch.Tensor, dtype, numel=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, has {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.c_void_p)


class System:
    """Device-resident sparse system (gnp_system_create)."""

    def __init__(self, csr=None, *, n=None, rowptr=None, colind=None, val=None,
                 prescale: bool = True, stream=None):
        if csr is not None:
            n, rowptr, colind, val = csr.n, csr.rowptr, csr.colind, csr.val
        L = _lib.load()
        rp, prp = _host(rowptr, np.int32)
        ci, pci = _host(colind, np.int32)
        v, pv = _host(val, np.float64)
        nnz = int(ci.size)
        h = C.c_void_p()
        check(L.gnp_system_create(int(n), nnz, prp, pci, pv, int(bool(prescale)),
                                  _stream(stream), C.byref(h)))
        self._h = h
        self.n = int(n)
        self.nnz = nnz
        g0, g1 = C.c_double(), C.c_double()
        check(L.gnp_system_gamma(h, C.byref(g0), C.byref(g1)))
        self.gamma_input, self.gamma = g0.value, g1.value

    @property
    def handle(self):
        return self._h

    def refresh(self):
        """Re-read gamma after the values changed elsewhere (a server update)."""
        g0, g1 = C.c_double(), C.c_double()
        check(_lib.load().gnp_system_gamma(self._h, C.byref(g0), C.byref(g1)))
        self.gamma_input, self.gamma = g0.value, g1.value

    def set_timeout(self, seconds: float):
        """Time limit of every later single solve on this system, 0 = none
        (gnp_system_set_timeout)."""
        check(_lib.load().gnp_system_set_timeout(self._h, float(seconds)))

    def set_values(self, val, stream=None):
        """New values on the same pattern (gnp_system_set_values)."""
        v, pv = _host(val, np.float64)
        if v.size != self.nnz:
            raise ValueError("val must have nnz entries")
        L = _lib.load()
        check(L.gnp_system_set_values(self._h, pv, _stream(stream)))
        g0, g1 = C.c_double(), C.c_double()
        check(L.gnp_system_gamma(self._h, C.byref(g0), C.byref(g1)))
        self.gamma_input, self.gamma = g0.value, g1.value

    def export(self):
        L = _lib.load()
        val = np.empty(self.nnz)
        ahat = np.empty(self.nnz)
        trp = np.empty(self.n + 1, dtype=np.int32)
        tci = np.empty(self.nnz, dtype=np.int32)
        tv = np.empty(self.nnz)
        p = lambda a: a.ctypes.data_as(C.c_void_p)
        check(L.gnp_system_export(self._h, p(val), p(ahat), p(trp), p(tci), p(tv)))
        return dict(val=val, ahat=ahat, t_rowptr=trp, t_colind=tci, t_val=tv)

    def spmv(self, x: torch.Tensor, y: torch.Tensor | None = None, prec="f32", stream=None):
        p = PREC[prec]
        dt = KDTYPE[p]
        if y is None:
            y = torch.empty(self.n, dtype=dt, device=x.device)
        check(_lib.load().gnp_spmv(self._h, _dev_ptr(x, dt, self.n, "x"),
                                   _dev_ptr(y, dt, self.n, "y"), p, _stream(stream)))
        return y

    def time_spmv(self, x: torch.Tensor, y: torch.Tensor, prec="f32", reps=50, stream=None):
        """Mean ms per SpMV launch (HIP events on the launch stream)."""
        p = PREC[prec]
        dt = KDTYPE[p]
        ms = C.c_double()
        check(_lib.load().gnp_time_spmv(self._h, _dev_ptr(x, dt, self.n, "x"),
                                        _dev_ptr(y, dt, self.n, "y"), p, int(reps),
                                        C.byref(ms), _stream(stream)))
        return ms.value

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().gnp_system_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Model:
    """Graph neural preconditioner bound to a System (gnp_model_create)."""

    def __init__(self, system: System, L: int, d: int, h: int, params=None, seed: int = 0):
        """params: initial weights (float64, the packing of gnp_model_create),
        or None for the library's seeded default initialisation."""
        lib = _lib.load()
        pth = None
        if params is not None:
            th, pth = _host(params, np.float64)
        hm = C.c_void_p()
        check(lib.gnp_model_create(system.handle, L, d, h, pth, int(seed), C.byref(hm)))
        self._h = hm
        self.system = system  # keeps the system alive
        self.L, self.d, self.h = L, d, h
        self.nparams = int(lib.gnp_model_nparams(hm))

    @property
    def handle(self):
        return self._h

    def get_params(self) -> np.ndarray:
        out = np.empty(self.nparams)
        check(_lib.load().gnp_params_get(self._h, out.ctypes.data_as(C.c_void_p), self.nparams))
        return out

    def set_params(self, params):
        th, pth = _host(params, np.float64)
        check(_lib.load().gnp_params_set(self._h, pth, th.size))

    def set_scaling(self, on: bool):
        """Eq. (6) scaling on (default) or off, the ablation (gnp_model_set_scaling)."""
        check(_lib.load().gnp_model_set_scaling(self._h, 1 if on else 0))

    def apply(self, v: torch.Tensor, z: torch.Tensor | None = None, prec="f32", stream=None):
        """z = M(v); v of shape [n] or [n, nrhs] (node-major)."""
        p = PREC[prec]
        dt = KDTYPE[p]
        nrhs = 1 if v.dim() == 1 else v.shape[1]
        if z is None:
            z = torch.empty_like(v)
        check(_lib.load().gnp_apply(self._h, _dev_ptr(v, dt, self.system.n * nrhs, "v"),
                                    _dev_ptr(z, dt, self.system.n * nrhs, "z"), nrhs, p,
                                    _stream(stream)))
        return z

    def apply_layers(self, v: torch.Tensor, prec="f32", stream=None):
        """(z, acts): z = M(v) as from apply, and every activation of the
        network, acts[l] = X_l of shape [n, nrhs, d] (l = 0: encoder output),
        in the precision's storage type (bfloat16 for "bf16")."""
        p = PREC[prec]
        dt = KDTYPE[p]
        nrhs = 1 if v.dim() == 1 else v.shape[1]
        z = torch.empty_like(v)
        sdt = {GNP_F64: torch.float64, GNP_F32: torch.float32, GNP_BF16: torch.bfloat16}[p]
        acts = torch.empty((self.L + 1, self.system.n, nrhs, self.d), dtype=sdt, device=v.device)
        check(_lib.load().gnp_apply_layers(self._h, _dev_ptr(v, dt, self.system.n * nrhs, "v"),
                                           _dev_ptr(z, dt, self.system.n * nrhs, "z"),
                                           C.c_void_p(acts.data_ptr()), nrhs, p, _stream(stream)))
        return z, acts

    def train(self, steps: int, batch: int, lr: float = 1e-3, seed: int = 2, prec="f32",
              x_fixed: torch.Tensor | None = None, betas=(0.9, 0.999), eps: float = 1e-8,
              sampler_m: int = 0, sampler_count: int | None = None, stream=None):
        """gnp_train: returns (loss history ndarray, best step).  sampler_m > 0
        draws the first sampler_count (default batch // 2) columns of every
        batch from the Arnoldi sampler of Eq. (3) with sampler_m steps."""
        if sampler_count is None:
            sampler_count = batch // 2 if sampler_m > 0 else 0
        o = TrainOpts(int(steps), int(batch), float(lr), float(betas[0]), float(betas[1]),
                      float(eps), int(seed), PREC[prec], int(sampler_m), int(sampler_count))
        hist = np.empty(steps)
        best = C.c_int(-1)
        xf = None
        if x_fixed is not None:
            xf = _dev_ptr(x_fixed, torch.float64, self.system.n * batch, "x_fixed")
        check(_lib.load().gnp_train(self._h, C.byref(o), xf, hist.ctypes.data_as(C.c_void_p),
                                    C.byref(best), _stream(stream)))
        return hist, best.value

    def time_layer(self, nrhs=1, prec="bf16", reps=50, stream=None):
        """Mean ms per Res-GCONV layer launch (HIP events on the launch stream)."""
        ms = C.c_double()
        check(_lib.load().gnp_time_layer(self._h, int(nrhs), PREC[prec], int(reps), C.byref(ms),
                                         _stream(stream)))
        return ms.value

    def time_layer_cold(self, flush: torch.Tensor, nrhs=1, prec="bf16", reps=50, stream=None):
        """(ms per layer launch, ms per flush) with the caches evicted before
        every launch by writing the float32 tensor `flush` (gnp_time_layer_cold)."""
        ms, mf = C.c_double(), C.c_double()
        if flush.dtype != torch.float32 or not flush.is_cuda or not flush.is_contiguous():
            raise TypeError("flush must be a contiguous float32 device tensor")
        check(_lib.load().gnp_time_layer_cold(self._h, int(nrhs), PREC[prec], int(reps),
                                              C.c_void_p(flush.data_ptr()),
                                              flush.numel() * 4, C.byref(ms), C.byref(mf),
                                              _stream(stream)))
        return ms.value, mf.value

    def loss_grad(self, b: torch.Tensor, prec="f64", stream=None):
        """gnp_loss_grad on b ([n] or [n, nrhs], float64 device)."""
        nrhs = 1 if b.dim() == 1 else b.shape[1]
        loss = C.c_double()
        g = np.empty(self.nparams)
        check(_lib.load().gnp_loss_grad(self._h, _dev_ptr(b, torch.float64,
                                                          self.system.n * nrhs, "b"),
                                        nrhs, PREC[prec], C.byref(loss),
                                        g.ctypes.data_as(C.c_void_p), _stream(stream)))
        return loss.value, g

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().gnp_model_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fgmres_solve(system: System, b: torch.Tensor, model: Model | None = None,
                 x: torch.Tensor | None = None, m: int = 30, rtol: float = 1e-8,
                 maxiters: int = 100, prec="f32", want_hist: bool = True, stream=None):
    """Algorithm 1 on the device.  Returns (x, info dict, hist ndarray or None)."""
    p = PREC[prec]
    if x is None:
        x = torch.zeros(system.n, dtype=torch.float64, device=b.device)
    hist = np.full(maxiters + 1, np.nan) if want_hist else None
    info = SolveInfo()
    check(_lib.load().fgmres_solve(
        system.handle, model.handle if model is not None else None,
        _dev_ptr(b, torch.float64, system.n, "b"), _dev_ptr(x, torch.float64, system.n, "x"),
        int(m), float(rtol), int(maxiters), p,
        hist.ctypes.data_as(C.c_void_p) if hist is not None else None, C.byref(info),
        _stream(stream)))
    d = info.as_dict()
    if hist is not None:
        hist = hist[: d["iters"] + 1]
    return x, d, hist


def fgmres_solve_jacobi(system: System, b: torch.Tensor, x: torch.Tensor | None = None,
                        m: int = 30, rtol: float = 1e-8, maxiters: int = 100, prec="f32",
                        want_hist: bool = True, stream=None):
    """Algorithm 1 with the Jacobi preconditioner M = D^{-1} (fgmres_solve_jacobi).
    Returns (x, info dict, hist ndarray or None)."""
    p = PREC[prec]
    if x is None:
        x = torch.zeros(system.n, dtype=torch.float64, device=b.device)
    hist = np.full(maxiters + 1, np.nan) if want_hist else None
    info = SolveInfo()
    check(_lib.load().fgmres_solve_jacobi(
        system.handle, _dev_ptr(b, torch.float64, system.n, "b"),
        _dev_ptr(x, torch.float64, system.n, "x"), int(m), float(rtol), int(maxiters), p,
        hist.ctypes.data_as(C.c_void_p) if hist is not None else None, C.byref(info),
        _stream(stream)))
    d = info.as_dict()
    if hist is not None:
        hist = hist[: d["iters"] + 1]
    return x, d, hist


def fgmres_solve_gmres(system: System, b: torch.Tensor, x: torch.Tensor | None = None,
                       m: int = 10, rtol: float = 1e-8, maxiters: int = 100, inner_k: int = 10,
                       inner_tol: float = 1e-6, prec="f32", want_hist: bool = True,
                       stream=None):
    """Algorithm 1 with inner-outer GMRES as M (fgmres_solve_gmres): z_j = one
    cycle of at most inner_k GMRES steps on A z = v_j, ended at inner_tol.
    Returns (x, info dict, hist ndarray or None)."""
    p = PREC[prec]
    if x is None:
        x = torch.zeros(system.n, dtype=torch.float64, device=b.device)
    hist = np.full(maxiters + 1, np.nan) if want_hist else None
    info = SolveInfo()
    check(_lib.load().fgmres_solve_gmres(
        system.handle, _dev_ptr(b, torch.float64, system.n, "b"),
        _dev_ptr(x, torch.float64, system.n, "x"), int(m), float(rtol), int(maxiters),
        int(inner_k), float(inner_tol), p,
        hist.ctypes.data_as(C.c_void_p) if hist is not None else None, C.byref(info),
        _stream(stream)))
    d = info.as_dict()
    if hist is not None:
        hist = hist[: d["iters"] + 1]
    return x, d, hist


def fgmres_step_times(system: System, count: int) -> np.ndarray:
    """Seconds from r_0 to each Arnoldi step's residual estimate of the last
    single solve on `system` (fgmres_step_times); count = iters + 1."""
    t = np.zeros(int(count))
    check(_lib.load().fgmres_step_times(system.handle, t.ctypes.data_as(C.c_void_p), int(count)))
    return t


def auc(hist, rtol: float, t=None):
    """(Iter-AUC, Time-AUC or None) of a residual history (gnp_auc, Sec. 3)."""
    r = np.ascontiguousarray(hist, dtype=np.float64)
    tt = None if t is None else np.ascontiguousarray(t, dtype=np.float64)
    if tt is not None and tt.size != r.size:
        raise ValueError("t must have one entry per residual")
    ia, ta = C.c_double(), C.c_double()
    check(_lib.load().gnp_auc(r.ctypes.data_as(C.c_void_p),
                              None if tt is None else tt.ctypes.data_as(C.c_void_p),
                              r.size - 1, float(rtol), C.byref(ia),
                              None if tt is None else C.byref(ta)))
    return ia.value, (None if tt is None else ta.value)


def fgmres_solve_batch(system: System, B: torch.Tensor, model: Model, X: torch.Tensor | None = None,
                       m: int = 30, rtol: float = 1e-8, maxiters: int = 100, prec="bf16",
                       stream=None):
    """Solve A x_k = b_k for the rows of B ([nrhs, n], float64, device) in one
    lockstep batch.  Returns (X, list of info dicts)."""
    if B.dim() != 2 or B.shape[1] != system.n:
        raise ValueError("B must have shape [nrhs, n]")
    nrhs = B.shape[0]
    if X is None:
        X = torch.zeros_like(B)
    infos = (SolveInfo * nrhs)()
    check(_lib.load().fgmres_solve_batch(
        system.handle, model.handle, _dev_ptr(B, torch.float64, nrhs * system.n, "B"),
        _dev_ptr(X, torch.float64, nrhs * system.n, "X"), int(nrhs), int(m), float(rtol),
        int(maxiters), PREC[prec], C.cast(infos, C.c_void_p), _stream(stream)))
    return X, [infos[k].as_dict() for k in range(nrhs)]


class Sampler:
    """Training-pair sampler of Eqs. (2)-(3) (gnp_sampler_*): m Arnoldi steps
    of the system's matrix without a preconditioner, SVD of Hbar; draw()
    returns x = V_m Z S^+ eps ([n, count] float64, device)."""

    def __init__(self, system: System, m: int = 40, seed: int = 2, max_count: int = 256,
                 stream=None):
        h = C.c_void_p()
        check(_lib.load().gnp_sampler_create(system.handle, int(m), int(seed), int(max_count),
                                             _stream(stream), C.byref(h)))
        self._h = h
        self.system = system

    def info(self):
        """(k, Hbar [(k+1) x k], singular values [k], G [k x k]) as numpy arrays."""
        k = C.c_int()
        check(_lib.load().gnp_sampler_info(self._h, C.byref(k), None, None, None))
        k = k.value
        hb = np.empty((k + 1, k))
        sv = np.empty(k)
        G = np.empty((k, k))
        check(_lib.load().gnp_sampler_info(self._h, None, hb.ctypes.data_as(C.c_void_p),
                                           sv.ctypes.data_as(C.c_void_p),
                                           G.ctypes.data_as(C.c_void_p)))
        return k, hb, sv, G

    def draw(self, step: int, count: int, stream=None) -> torch.Tensor:
        x = torch.empty((self.system.n, count), dtype=torch.float64, device="cuda")
        check(_lib.load().gnp_sampler_draw(self._h, int(step), int(count),
                                           _dev_ptr(x, torch.float64, self.system.n * count, "x"),
                                           _stream(stream)))
        return x

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().gnp_sampler_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching solve server (gnp_server_*): requests for any
    registered system are admitted into slots as slots and HBM free up and
    solved concurrently on the device; results are collected by ticket."""

    def __init__(self, hbm_budget: int, max_slots: int = 16, m: int = 30,
                 max_iters: int = 3000, prec="bf16"):
        h = C.c_void_p()
        check(_lib.load().gnp_server_create(int(hbm_budget), int(max_slots), int(m),
                                            int(max_iters), PREC[prec], C.byref(h)))
        self._h = h
        self._n = {}
        self._sys = {}
        self._keep = []  # systems / models must outlive the server

    def register(self, system: System, model: Model | None = None) -> int:
        i = C.c_int()
        check(_lib.load().gnp_server_register(self._h, system.handle,
                                              model.handle if model is not None else None,
                                              C.byref(i)))
        self._n[i.value] = system.n
        self._sys[i.value] = system
        self._keep.append((system, model))
        return i.value

    def workspace_bytes(self, sid: int) -> int:
        b = C.c_size_t()
        check(_lib.load().gnp_server_workspace_bytes(self._h, int(sid), C.byref(b)))
        return b.value

    def submit(self, sid: int, b, rtol: float = 1e-8, maxiters: int = 3000) -> int:
        arr, ptr = _host(b, np.float64)
        if arr.size != self._n[sid]:
            raise ValueError(f"b must have {self._n[sid]} entries")
        t = C.c_uint64()
        check(_lib.load().gnp_server_submit(self._h, int(sid), ptr, float(rtol), int(maxiters),
                                            C.byref(t)))
        return t.value

    def poll(self, ticket: int, n: int):
        """(x, info dict, latency seconds), or None while the request runs."""
        x = np.empty(n, dtype=np.float64)
        info = SolveInfo()
        lat = C.c_double()
        st = _lib.load().gnp_server_poll(self._h, C.c_uint64(ticket),
                                         x.ctypes.data_as(C.c_void_p), C.byref(info),
                                         C.byref(lat))
        if st == _lib.GNP_EBUSY:
            return None
        check(st)
        return x, info.as_dict(), lat.value

    def update_system(self, sid: int, val, tune_steps: int = 0, batch: int = 16,
                      lr: float = 1e-3, seed: int = 2, prec="f32", betas=(0.9, 0.999),
                      eps: float = 1e-8):
        """New values for registered system `sid` while serving
        (gnp_server_update_system); with tune_steps > 0 its network is
        trained further on the new matrix.  Returns (loss history, best step)
        of that training, or None."""
        v, pv = _host(val, np.float64)
        if tune_steps > 0:
            o = TrainOpts(int(tune_steps), int(batch), float(lr), float(betas[0]),
                          float(betas[1]), float(eps), int(seed), PREC[prec], 0, 0)
            hist = np.empty(tune_steps)
            best = C.c_int(-1)
            check(_lib.load().gnp_server_update_system(self._h, int(sid), pv, C.byref(o),
                                                       hist.ctypes.data_as(C.c_void_p),
                                                       C.byref(best)))
            self._sys[sid].refresh()
            return hist, best.value
        check(_lib.load().gnp_server_update_system(self._h, int(sid), pv, None, None, None))
        self._sys[sid].refresh()
        return None

    def drain(self, timeout_s: float = 600.0):
        check(_lib.load().gnp_server_drain(self._h, float(timeout_s)))

    def stats(self) -> dict:
        s = _lib.ServerStats()
        check(_lib.load().gnp_server_get_stats(self._h, C.byref(s)))
        return s.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().gnp_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
