"""Randomized quasi-Monte Carlo pricing on MI355X (gfx950).

Thin Python binding over the C ABI of ``librqmc.so`` (declared in
``include/rqmc.h``): argument marshalling only.  Every step of the path --
random starts, radical inverses, inverse normal, LIBOR / MBS paths,
payoffs, reductions -- runs in the library's HIP kernels.  PyTorch provides
device memory and the stream.  There is no CPU fallback: if the library is
missing or no GPU is present the calls raise.

The method is the one of Xu & Okten, "High Performance Financial Simulation
Using Randomized Quasi-Monte Carlo Methods": M independent random-start
(optionally permuted) Halton replications (Algorithm 3), theta_N^m per
replication, the grand average RQ_{M,N} and its spread (Introduction), for
LIBOR market model caplets (caplet section) and Caflisch MBS (MBS section).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librqmc.so")

RQ_OK, RQ_EINVAL, RQ_ERANGE, RQ_ENOMEM, RQ_EHIP, RQ_EWORKSPACE, RQ_EUNSUPPORTED = range(7)
FP64, FP32 = 0, 1
START_RANDOM, START_ZERO, PERM_RANDOM, OUT_DIGITS, MC_PHILOX, LMM_EULER, PERM_PER_REP = 0, 1, 2, 4, 8, 16, 32

_dp = C.POINTER(C.c_double)


class RqError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"rq status {status}: {msg}")
        self.status = status


class rq_lmm_model(C.Structure):
    _fields_ = [("n_fwd", C.c_int), ("n_factors", C.c_int), ("delta", C.c_double),
                ("L0", _dp), ("sigma", _dp), ("loadings", _dp), ("strike", _dp)]


class rq_mbs_params(C.Structure):
    _fields_ = [("months", C.c_int), ("i0", C.c_double), ("sigma", C.c_double),
                ("K1", C.c_double), ("K2", C.c_double), ("K3", C.c_double), ("K4", C.c_double)]


class rq_instrument(C.Structure):
    _fields_ = [("kind", C.c_int), ("lmm", C.POINTER(rq_lmm_model)), ("mbs", C.POINTER(rq_mbs_params)),
                ("N", C.c_int64), ("M", C.c_int), ("seed", C.c_uint64), ("m_offset", C.c_int64),
                ("flags", C.c_int)]


class rq_tuning(C.Structure):
    _fields_ = [("chunk", C.c_int), ("waves_per_cu", C.c_int), ("order", C.c_int)]


INST_LMM, INST_MBS = 0, 1
ORDER_COST, ORDER_GIVEN = 0, 1


class rq_result(C.Structure):
    _fields_ = [("theta", C.c_void_p), ("mean", C.c_void_p), ("sd", C.c_void_p),
                ("se", C.c_void_p)]


_lib = None


def lib():
    """The loaded C library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(LIB_PATH)
    L.rq_last_error.restype = C.c_char_p
    L.rq_last_error.argtypes = []
    L.rq_version.restype = C.c_char_p
    L.rq_version.argtypes = []
    L.rq_sequence_workspace.restype = C.c_size_t
    L.rq_sequence_workspace.argtypes = [C.c_int, C.c_int64, C.c_int, C.c_int]
    L.rq_caplets_workspace.restype = C.c_size_t
    L.rq_caplets_workspace.argtypes = [C.POINTER(rq_lmm_model), C.c_int64, C.c_int, C.c_int, C.c_int, C.c_int]
    L.rq_mbs_workspace.restype = C.c_size_t
    L.rq_mbs_workspace.argtypes = [C.POINTER(rq_mbs_params), C.c_int64, C.c_int, C.c_int, C.c_int, C.c_int]
    L.rq_sequence.restype = C.c_int
    L.rq_sequence.argtypes = [C.c_int, C.c_int64, C.c_int, C.c_uint64, C.c_int, C.c_int64,
                              C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
    L.rq_price_caplets.restype = C.c_int
    L.rq_price_caplets.argtypes = [C.POINTER(rq_lmm_model), C.c_int64, C.c_int, C.c_uint64, C.c_int64,
                                   C.c_int, C.c_int, C.POINTER(rq_result), C.POINTER(rq_result),
                                   C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
    L.rq_price_caplets_noalloc.restype = C.c_int
    L.rq_price_caplets_noalloc.argtypes = [C.POINTER(rq_lmm_model), C.c_int64, C.c_int, C.c_uint64, C.c_int64,
                                           C.c_int, C.c_int, C.POINTER(rq_result), C.POINTER(rq_result),
                                           C.c_void_p, C.c_void_p]
    L.rq_price_mbs.restype = C.c_int
    L.rq_price_mbs.argtypes = [C.POINTER(rq_mbs_params), C.c_int64, C.c_int, C.c_uint64, C.c_int64,
                               C.c_int, C.c_int, C.POINTER(rq_result), C.POINTER(rq_result),
                               C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
    L.rq_inv_normal.restype = C.c_int
    L.rq_inv_normal.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]
    L.rq_batch_workspace.restype = C.c_size_t
    L.rq_batch_workspace.argtypes = [C.POINTER(rq_instrument), C.c_int, C.c_int, C.c_int]
    L.rq_price_batch.restype = C.c_int
    L.rq_price_batch.argtypes = [C.POINTER(rq_instrument), C.c_int, C.c_int, C.c_int, C.POINTER(rq_tuning),
                                 C.POINTER(rq_result), C.POINTER(rq_result), C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_size_t, C.c_void_p]
    L.rq_autotune_batch.restype = C.c_int
    L.rq_autotune_batch.argtypes = [C.POINTER(rq_instrument), C.c_int, C.c_int, C.c_int,
                                    C.POINTER(rq_result), C.POINTER(rq_result), C.POINTER(rq_tuning),
                                    C.POINTER(C.c_double), C.c_void_p, C.c_size_t, C.c_void_p]
    L.rq_batch_tuning.restype = C.c_int
    L.rq_batch_tuning.argtypes = [C.POINTER(rq_instrument), C.c_int, C.c_int, C.c_int, C.POINTER(rq_tuning),
                                  C.POINTER(C.c_int)]
    L.rq_realtime_hz.restype = C.c_int
    L.rq_realtime_hz.argtypes = [C.POINTER(C.c_double)]
    L.rq_lmm_pca_loadings.restype = C.c_int
    L.rq_lmm_pca_loadings.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.POINTER(C.c_double)]
    L.rq_timer_begin.restype = C.c_int
    L.rq_timer_begin.argtypes = [C.c_int]
    L.rq_timer_end.restype = C.c_int
    L.rq_timer_end.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_int)]
    L.rq_set_adjoint_store_limit.restype = C.c_int
    L.rq_set_adjoint_store_limit.argtypes = [C.c_size_t]
    L.rq_timer_part.restype = C.c_int
    L.rq_timer_part.argtypes = [C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int)]
    _lib = L
    return L


def last_error() -> str:
    return lib().rq_last_error().decode()


def _check(st: int):
    if st != RQ_OK:
        raise RqError(st, last_error())


def _torch():
    import torch
    return torch


def _device(device):
    torch = _torch()
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the RQMC library runs on MI355X only")
    return torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())


def _stream(device):
    return C.c_void_p(_torch().cuda.current_stream(device).cuda_stream)


def _workspace(nbytes: int, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


# ---------------------------------------------------------------------------
# model marshalling (host arrays stay alive for the duration of the call)
# ---------------------------------------------------------------------------
class _LmmHost:
    def __init__(self, model):
        self.L0 = np.ascontiguousarray(model.L0, dtype=np.float64)
        self.sigma = np.ascontiguousarray(model.sigma, dtype=np.float64)
        self.b = np.ascontiguousarray(model.loadings, dtype=np.float64).reshape(-1)
        self.K = np.ascontiguousarray(model.strike, dtype=np.float64)
        self.c = rq_lmm_model(int(model.n_fwd), int(model.n_factors), float(model.delta),
                              self.L0.ctypes.data_as(_dp), self.sigma.ctypes.data_as(_dp),
                              self.b.ctypes.data_as(_dp), self.K.ctypes.data_as(_dp))


def _mbs_c(p) -> rq_mbs_params:
    return rq_mbs_params(int(p.months), float(p.i0), float(p.sigma), float(p.K1), float(p.K2),
                         float(p.K3), float(p.K4))


@dataclass
class Result:
    """Per-replication estimates theta [M][n_out], RQ, sd (M-1), SE, all FP64
    device tensors; per_path [M][N][n_out] when requested; greeks (another
    Result) when requested."""
    theta: object
    mean: object
    sd: object
    se: object
    per_path: Optional[object] = None
    greeks: Optional["Result"] = None


def _result(M: int, n_out: int, device):
    # one allocation, four views: theta [M][n_out], then mean, sd, se
    torch = _torch()
    buf = torch.empty((M + 3) * n_out, dtype=torch.float64, device=device)
    theta = buf[:M * n_out].view(M, n_out)
    mean, sd, se = (buf[(M + r) * n_out:(M + r + 1) * n_out] for r in range(3))
    c = rq_result(theta.data_ptr(), mean.data_ptr(), sd.data_ptr(), se.data_ptr())
    return Result(theta, mean, sd, se), c


def _prec(precision) -> int:
    if precision in (FP64, "fp64", "f64", "float64"):
        return FP64
    if precision in (FP32, "fp32", "f32", "float32"):
        return FP32
    raise ValueError(f"unknown precision {precision!r}")


# ---------------------------------------------------------------------------
# entry points
# ---------------------------------------------------------------------------
def sequence_workspace(s: int, N: int, M: int, flags: int = 0) -> int:
    n = lib().rq_sequence_workspace(s, N, M, flags)
    if n == 0:
        raise RqError(RQ_EINVAL, last_error())
    return n


def sequence(s: int, N: int, M: int, seed: int, flags: int = 0, m_offset: int = 0,
             device=None, out=None, ws=None):
    """Points of M random-start Halton replications: tensor [M][N][s], FP64
    (or uint64 integers R = x * P_j with flags | OUT_DIGITS)."""
    torch = _torch()
    dev = _device(device)
    dtype = torch.int64 if flags & OUT_DIGITS else torch.float64
    if out is None:
        out = torch.empty((M, N, s), dtype=dtype, device=dev)
    need = sequence_workspace(s, N, M, flags)
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    _check(lib().rq_sequence(s, N, M, seed, flags, m_offset, C.c_void_p(out.data_ptr()),
                             C.c_void_p(ws.data_ptr()), ws.numel(), _stream(dev)))
    return out


def caplets_workspace(model, N: int, M: int, flags: int = 0, precision="fp64",
                      greeks: bool = False) -> int:
    h = _LmmHost(model)
    n = lib().rq_caplets_workspace(C.byref(h.c), N, M, flags, _prec(precision), int(greeks))
    if n == 0:
        raise RqError(RQ_EINVAL, last_error())
    return n


def price_caplets(model, N: int, M: int, seed: int, m_offset: int = 0, flags: int = 0,
                  precision="fp64", per_path: bool = False, greeks: bool = False,
                  device=None, ws=None) -> Result:
    """Caplets on every forward with a strike, plus the book (last output),
    n_out = n_fwd + 1.  greeks=True runs the adjoint kernel and adds
    result.greeks with 2 n_fwd + 1 outputs: dbook/dL_n(0) (n = 1..n_fwd),
    dbook/dL_0(0), dbook/dsigma_n (n = 1..n_fwd)."""
    torch = _torch()
    dev = _device(device)
    h = _LmmHost(model)
    prec = _prec(precision)
    n_out = model.n_fwd + 1
    res, c = _result(M, n_out, dev)
    gres, gc = _result(M, 2 * model.n_fwd + 1, dev) if greeks else (None, None)
    pp = torch.empty((M, N, n_out), dtype=torch.float64, device=dev) if per_path else None
    need = lib().rq_caplets_workspace(C.byref(h.c), N, M, flags, prec, int(greeks))
    if need == 0:
        raise RqError(RQ_EINVAL, last_error())
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    _check(lib().rq_price_caplets(C.byref(h.c), N, M, seed, m_offset, flags, prec, C.byref(c),
                                  C.byref(gc) if greeks else None,
                                  C.c_void_p(pp.data_ptr() if pp is not None else 0),
                                  C.c_void_p(ws.data_ptr()), ws.numel(), _stream(dev)))
    res.per_path = pp
    res.greeks = gres
    return res


def price_caplets_noalloc(model, N: int, M: int, seed: int, m_offset: int = 0, flags: int = 0,
                          precision="fp64", greeks: bool = False, out=None, grad=None,
                          device=None) -> Result:
    """price_caplets on the library's own device scratch array (no
    workspace; RQ_ERANGE beyond its size).  out / grad: optional
    preallocated (Result, rq_result) pairs from a previous call, so that a
    caller can run with no allocation at all."""
    dev = _device(device)
    h = _LmmHost(model)
    res, c = out if out is not None else _result(M, model.n_fwd + 1, dev)
    if greeks:
        gres, gc = grad if grad is not None else _result(M, 2 * model.n_fwd + 1, dev)
    else:
        gres, gc = None, None
    _check(lib().rq_price_caplets_noalloc(C.byref(h.c), N, M, seed, m_offset, flags, _prec(precision),
                                          C.byref(c), C.byref(gc) if greeks else None, None, _stream(dev)))
    res.greeks = gres
    return res


def mbs_workspace(params, N: int, M: int, flags: int = 0, precision="fp64", greeks: bool = False) -> int:
    p = _mbs_c(params)
    n = lib().rq_mbs_workspace(C.byref(p), N, M, flags, _prec(precision), int(greeks))
    if n == 0:
        raise RqError(RQ_EINVAL, last_error())
    return n


def price_mbs(params, N: int, M: int, seed: int, m_offset: int = 0, flags: int = 0,
              precision="fp64", per_path: bool = False, greeks: bool = False,
              device=None, ws=None) -> Result:
    """Present value of the MBS pool, n_out = 1; greeks=True adds the
    pathwise total derivative dPV/di0 as result.greeks."""
    torch = _torch()
    dev = _device(device)
    p = _mbs_c(params)
    prec = _prec(precision)
    res, c = _result(M, 1, dev)
    gres, gc = _result(M, 1, dev) if greeks else (None, None)
    pp = torch.empty((M, N, 1), dtype=torch.float64, device=dev) if per_path else None
    need = lib().rq_mbs_workspace(C.byref(p), N, M, flags, prec, int(greeks))
    if need == 0:
        raise RqError(RQ_EINVAL, last_error())
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    _check(lib().rq_price_mbs(C.byref(p), N, M, seed, m_offset, flags, prec, C.byref(c),
                              C.byref(gc) if greeks else None,
                              C.c_void_p(pp.data_ptr() if pp is not None else 0),
                              C.c_void_p(ws.data_ptr()), ws.numel(), _stream(dev)))
    res.per_path = pp
    res.greeks = gres
    return res


# ---------------------------------------------------------------------------
# batches of instruments (one persistent launch)
# ---------------------------------------------------------------------------
@dataclass
class BatchResult:
    """results[k] (and greeks in results[k].greeks) per instrument, in the
    caller's order; t_first / t_last [n] int64 device tensors of real-time
    counter ticks (rq_realtime_hz) when timestamps were requested."""
    results: list
    t_first: Optional[object] = None
    t_last: Optional[object] = None


class _BatchHost:
    """C instrument array for a list of instruments (objects with kind
    "lmm"/"mbs", model, N, M, seed and optional m_offset, flags); the host
    model arrays stay referenced while this object lives."""

    def __init__(self, instruments):
        n = len(instruments)
        self.keep = []
        self.arr = (rq_instrument * max(n, 1))()
        self.n = n
        self.n_out, self.n_g = [], []
        for k, ins in enumerate(instruments):
            e = self.arr[k]
            if ins.kind == "lmm":
                h = _LmmHost(ins.model)
                self.keep.append(h)
                e.kind = INST_LMM
                e.lmm = C.pointer(h.c)
                self.n_out.append(ins.model.n_fwd + 1)
                self.n_g.append(2 * ins.model.n_fwd + 1)
            elif ins.kind == "mbs":
                p = _mbs_c(ins.model)
                self.keep.append(p)
                e.kind = INST_MBS
                e.mbs = C.pointer(p)
                self.n_out.append(1)
                self.n_g.append(1)
            else:
                raise ValueError(f"unknown instrument kind {ins.kind!r}")
            e.N = int(ins.N)
            e.M = int(ins.M)
            e.seed = int(ins.seed)
            e.m_offset = int(getattr(ins, "m_offset", 0))
            e.flags = int(getattr(ins, "flags", 0))


def batch_workspace(instruments, precision="fp32", greeks: bool = False) -> int:
    h = _BatchHost(instruments)
    n = lib().rq_batch_workspace(h.arr, h.n, _prec(precision), int(greeks))
    if n == 0:
        raise RqError(RQ_EINVAL, last_error())
    return n


def _batch_outputs(h, instruments, greeks, dev):
    res, cres, gcres = [], (rq_result * max(h.n, 1))(), (rq_result * max(h.n, 1))()
    for k, ins in enumerate(instruments):
        r, c = _result(int(ins.M), h.n_out[k], dev)
        cres[k] = c
        if greeks:
            g, gc = _result(int(ins.M), h.n_g[k], dev)
            gcres[k] = gc
            r.greeks = g
        res.append(r)
    return res, cres, gcres


def price_batch(instruments, precision="fp32", greeks: bool = False, tuning=None,
                timestamps: bool = True, device=None, ws=None) -> BatchResult:
    """Price every instrument of the list in one persistent launch.
    tuning: None (automatic) or (chunk, waves_per_cu, order)."""
    torch = _torch()
    dev = _device(device)
    h = _BatchHost(instruments)
    prec = _prec(precision)
    res, cres, gcres = _batch_outputs(h, instruments, greeks, dev)
    need = lib().rq_batch_workspace(h.arr, h.n, prec, int(greeks))
    if need == 0:
        raise RqError(RQ_EINVAL, last_error())
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    tf = tl = None
    if timestamps:
        tf = torch.empty(max(h.n, 1), dtype=torch.int64, device=dev)
        tl = torch.empty(max(h.n, 1), dtype=torch.int64, device=dev)
    tu = rq_tuning(*tuning) if tuning is not None else None
    _check(lib().rq_price_batch(h.arr, h.n, prec, int(greeks), C.byref(tu) if tu is not None else None,
                                cres, gcres if greeks else None,
                                C.c_void_p(tf.data_ptr() if tf is not None else 0),
                                C.c_void_p(tl.data_ptr() if tl is not None else 0),
                                C.c_void_p(ws.data_ptr()), ws.numel(), _stream(dev)))
    return BatchResult(res, tf, tl)


def autotune_batch(instruments, precision="fp32", greeks: bool = False, device=None, ws=None):
    """(chunk, waves_per_cu, order) of the fastest launch shape for this
    batch, and its time in ms (rq_autotune_batch: the automatic shape,
    (0, 0, order), and 20 fixed ones; a large batch screened on a probe of
    itself).  price_batch with
    tuning=None then uses the choice for this list."""
    dev = _device(device)
    h = _BatchHost(instruments)
    prec = _prec(precision)
    res, cres, gcres = _batch_outputs(h, instruments, greeks, dev)
    need = lib().rq_batch_workspace(h.arr, h.n, prec, int(greeks))
    if need == 0:
        raise RqError(RQ_EINVAL, last_error())
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    best = rq_tuning()
    ms = C.c_double(0.0)
    _check(lib().rq_autotune_batch(h.arr, h.n, prec, int(greeks), cres, gcres if greeks else None,
                                   C.byref(best), C.byref(ms), C.c_void_p(ws.data_ptr()), ws.numel(),
                                   _stream(dev)))
    return (best.chunk, best.waves_per_cu, best.order), ms.value


def batch_tuning(instruments, precision="fp32", greeks: bool = False):
    """((chunk, waves_per_cu, order), from_autotuner): the launch shape
    price_batch uses for this list with tuning=None -- the autotuner's
    choice for the list's signature, else all zero (automatic)."""
    h = _BatchHost(instruments)
    t = rq_tuning()
    hit = C.c_int(0)
    _check(lib().rq_batch_tuning(h.arr, h.n, _prec(precision), int(greeks), C.byref(t), C.byref(hit)))
    return (t.chunk, t.waves_per_cu, t.order), bool(hit.value)


def realtime_hz() -> float:
    """Frequency of the device real-time counter of the batch timestamps."""
    hz = C.c_double(0.0)
    _check(lib().rq_realtime_hz(C.byref(hz)))
    return hz.value


# ---------------------------------------------------------------------------
# autograd wrappers: the Greeks come from the adjoint kernel (LIBOR) and the
# pathwise tangent (MBS); backward only scales them by the incoming gradient
# ---------------------------------------------------------------------------
def _autograd():
    import torch

    class CapletBook(torch.autograd.Function):
        """RQ_{M,N} of the caplet book as a function of the initial forward
        curve L0 [n_fwd+1] and the vols sigma [n_fwd+1] (CPU float64
        tensors); backward returns g * dRQ/dL0 and g * dRQ/dsigma from the
        adjoint kernel.  The per-replication Greek estimates and their SE are
        kept in ctx.greeks (a Result) and returned by CapletBook.last."""

        last = None

        @staticmethod
        def forward(ctx, L0, sigma, model, N, M, seed, precision="fp32", device=None):
            m = model.copy()
            m.L0 = L0.detach().cpu().double().numpy().copy()
            m.sigma = sigma.detach().cpu().double().numpy().copy()
            r = price_caplets(m, N, M, seed, precision=precision, greeks=True, device=device)
            gm = r.greeks.mean.cpu()
            nf = m.n_fwd
            dL0 = torch.zeros(nf + 1, dtype=torch.float64)
            dL0[0] = gm[nf]
            dL0[1:] = gm[:nf]
            dsig = torch.zeros(nf + 1, dtype=torch.float64)
            dsig[1:] = gm[nf + 1:]
            ctx.save_for_backward(dL0, dsig)
            CapletBook.last = r
            return r.mean[-1].detach().cpu().reshape(())

        @staticmethod
        def backward(ctx, g):
            dL0, dsig = ctx.saved_tensors
            return g * dL0, g * dsig, None, None, None, None, None, None

    class MBSPrice(torch.autograd.Function):
        """RQ_{M,N} of the MBS as a function of i0 (0-dim CPU float64
        tensor); backward returns g * dRQ/di0 from the pathwise tangent."""

        last = None

        @staticmethod
        def forward(ctx, i0, params, N, M, seed, precision="fp32", device=None):
            from dataclasses import replace
            p = replace(params, i0=float(i0.detach().cpu()))
            r = price_mbs(p, N, M, seed, precision=precision, greeks=True, device=device)
            ctx.save_for_backward(r.greeks.mean.cpu().reshape(()))
            MBSPrice.last = r
            return r.mean[0].detach().cpu().reshape(())

        @staticmethod
        def backward(ctx, g):
            (d,) = ctx.saved_tensors
            return g * d, None, None, None, None, None, None

    return CapletBook, MBSPrice


def __getattr__(name):
    if name in ("CapletBook", "MBSPrice"):
        cb, mp = _autograd()
        globals()["CapletBook"], globals()["MBSPrice"] = cb, mp
        return globals()[name]
    raise AttributeError(name)


def inv_normal(u, precision="fp64"):
    """Inverse standard normal CDF of a device FP64 tensor (elementwise)."""
    torch = _torch()
    if not u.is_cuda or u.dtype != torch.float64:
        raise ValueError("u must be a float64 device tensor")
    u = u.contiguous()
    prec = _prec(precision)
    z = torch.empty(u.shape, dtype=torch.float64 if prec == FP64 else torch.float32, device=u.device)
    _check(lib().rq_inv_normal(u.numel(), C.c_void_p(u.data_ptr()), C.c_void_p(z.data_ptr()), prec,
                               _stream(u.device)))
    return z


def lmm_pca_loadings(n_fwd: int, n_factors: int, delta: float, beta: float):
    """Unit-row PCA loadings [n_fwd][n_factors] of rho_ij = exp(-beta|T_i - T_j|)
    (host computation; returns a numpy array)."""
    import numpy as np
    out = np.zeros((n_fwd, n_factors), dtype=np.float64)
    _check(lib().rq_lmm_pca_loadings(n_fwd, n_factors, delta, beta,
                                     out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def timer_begin(max_launches: int = 1000) -> None:
    """Start recording HIP events around every main path kernel launch."""
    _check(lib().rq_timer_begin(max_launches))


def timer_end():
    """(total kernel ms, number of timed launches) since timer_begin."""
    ms = C.c_double(0.0)
    n = C.c_int(0)
    _check(lib().rq_timer_end(C.byref(ms), C.byref(n)))
    return ms.value, n.value


def set_adjoint_store_limit(nbytes: int) -> None:
    """Bytes (FP64-counted) of the two-kernel adjoint's store region per
    chunk of tasks; 0 restores the default (64 GiB).  Results never depend
    on it; the workspace size does."""
    _check(lib().rq_set_adjoint_store_limit(nbytes))


def timer_part(part: int):
    """After timer_end: (ms, launches) of the adjoint's forward (part 1) or
    reverse (part 2) kernel over the timed calls."""
    ms = C.c_double(0.0)
    n = C.c_int(0)
    _check(lib().rq_timer_part(part, C.byref(ms), C.byref(n)))
    return ms.value, n.value


def version() -> str:
    return lib().rq_version().decode()


# ---------------------------------------------------------------------------
# the CPU baseline generator (librqmc_cpu.so, include/rqmc_cpu.h): the
# paper's recursive Halton method (Algorithm 2) on the host's cores, the
# comparison for rq_sequence; no GPU entry point uses it
# ---------------------------------------------------------------------------
CPU_LIB_PATH = os.path.join(HERE, "librqmc_cpu.so")
_cpu_lib = None


def cpu_lib():
    """The loaded CPU generator library (raises if it has not been built)."""
    global _cpu_lib
    if _cpu_lib is not None:
        return _cpu_lib
    if not os.path.exists(CPU_LIB_PATH):
        raise RuntimeError(f"CPU generator library {CPU_LIB_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(CPU_LIB_PATH)
    L.rq_cpu_last_error.restype = C.c_char_p
    L.rq_cpu_last_error.argtypes = []
    L.rq_cpu_max_threads.restype = C.c_int
    L.rq_cpu_max_threads.argtypes = []
    L.rq_cpu_sequence.restype = C.c_int
    L.rq_cpu_sequence.argtypes = [C.c_int, C.c_int64, C.c_int, C.c_uint64, C.c_int, C.c_int64, C.c_void_p,
                                  C.c_int]
    L.rq_cpu_alg2_run.restype = C.c_int
    L.rq_cpu_alg2_run.argtypes = [C.c_uint32, C.c_void_p, C.c_uint64, C.c_int64, C.c_void_p]
    _cpu_lib = L
    return L


def _cpu_check(st: int):
    if st != RQ_OK:
        raise RqError(st, cpu_lib().rq_cpu_last_error().decode())


def cpu_max_threads() -> int:
    return int(cpu_lib().rq_cpu_max_threads())


def cpu_sequence(s: int, N: int, M: int, seed: int, flags: int = 0, m_offset: int = 0,
                 threads: int = 0, out=None) -> np.ndarray:
    """The points of sequence() computed on the host by the recursive
    generator: numpy [M][N][s] FP64, bit-identical to the GPU's."""
    if out is None:
        out = np.empty((M, N, s), dtype=np.float64)
    if out.dtype != np.float64 or not out.flags.c_contiguous or out.size < M * N * s:
        raise ValueError("out must be a C-contiguous float64 array of M*N*s elements")
    _cpu_check(cpu_lib().rq_cpu_sequence(s, N, M, seed, flags, m_offset, out.ctypes.data, threads))
    return out


def cpu_alg2_run(p: int, n: int, count: int, sigma=None) -> np.ndarray:
    """The exact integers R of `count` consecutive indices from n in base p
    (uint64), by the recursive generator."""
    out = np.empty(count, dtype=np.uint64)
    sg = None
    if sigma is not None:
        sg = np.ascontiguousarray(sigma, dtype=np.int32)
    _cpu_check(cpu_lib().rq_cpu_alg2_run(p, sg.ctypes.data if sg is not None else None, n, count,
                                         out.ctypes.data))
    return out
