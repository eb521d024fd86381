"""CPU oracle for the RQMC pricing path (TEST INFRASTRUCTURE ONLY).

Plain FP64 implementation in C (``rqmc_oracle.c``), wrapped with ctypes.
Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
may import this package; the GPU library never does, and the two share no
code.  Each wrapper names the passage of the paper it follows; the C file
carries the full derivations.

Pins (tests/test_oracle_*.py) tie every function to something other than
itself: van der Corput leading points, Struckmeier's transformation in exact
rationals, the stratification invariant, mpmath / erfc for the inverse
normal, the sigma = 0 closed forms, 1-D / 2-D quadrature, the Black caplet
formula and the MBS par invariant.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "librqmc_oracle.so")
_lib = None

START_RANDOM = 0
START_ZERO = 1
PERM_RANDOM = 2
MC_PHILOX = 8
LMM_EULER = 16
PERM_PER_REP = 32

_dp = C.POINTER(C.c_double)
_u64p = C.POINTER(C.c_uint64)
_ip = C.POINTER(C.c_int)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(os.path.join(HERE, "rqmc_oracle.c"))):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    lib.orc_splitmix64.restype = C.c_uint64
    lib.orc_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
    lib.orc_nth_prime.restype = C.c_int
    lib.orc_nth_prime.argtypes = [C.c_int]
    lib.orc_digits.restype = C.c_int
    lib.orc_digits.argtypes = [C.c_uint64, _u64p]
    lib.orc_start.restype = C.c_int
    lib.orc_start.argtypes = [C.c_uint64, C.c_uint64, C.c_int, C.c_uint64, C.c_int, _u64p]
    lib.orc_perm.restype = C.c_int
    lib.orc_perm.argtypes = [C.c_uint64, C.c_int, C.c_int, _ip]
    lib.orc_radinv_R.restype = C.c_uint64
    lib.orc_radinv_R.argtypes = [C.c_uint64, C.c_int, _ip, C.c_uint64]
    lib.orc_point_from_R.restype = C.c_double
    lib.orc_point_from_R.argtypes = [C.c_uint64, C.c_uint64]
    lib.orc_perm_rep.restype = C.c_int
    lib.orc_perm_rep.argtypes = [C.c_uint64, C.c_uint64, C.c_int, C.c_int, _ip]
    lib.orc_perm_rep_seed.restype = C.c_uint64
    lib.orc_perm_rep_seed.argtypes = [C.c_uint64, C.c_uint64]
    lib.orc_philox4x64.restype = None
    lib.orc_philox4x64.argtypes = [_u64p, _u64p, _u64p]
    lib.orc_mc_point.restype = C.c_double
    lib.orc_mc_point.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.c_int]
    lib.orc_ppnd16.restype = C.c_double
    lib.orc_ppnd16.argtypes = [C.c_double]
    lib.orc_ppnd16_vec.restype = None
    lib.orc_ppnd16_vec.argtypes = [C.c_int64, _dp, _dp]
    lib.orc_sequence.restype = C.c_int
    lib.orc_sequence.argtypes = [C.c_int, C.c_int64, C.c_int, C.c_uint64, C.c_int, C.c_int64,
                                 C.c_int, _dp, _u64p]
    lib.orc_lmm_paths.restype = None
    lib.orc_lmm_paths.argtypes = [C.c_int64, C.c_int, C.c_int, C.c_double, _dp, _dp, _dp, _dp,
                                  C.c_int, C.c_int, _dp, _dp]
    lib.orc_mbs_paths.restype = None
    lib.orc_mbs_paths.argtypes = [C.c_int64, C.c_int, C.c_double, C.c_double, C.c_double,
                                  C.c_double, C.c_double, C.c_double, _dp, _dp]
    lib.orc_mbs_annuity.restype = None
    lib.orc_mbs_annuity.argtypes = [C.c_int, C.c_double, _dp]
    lib.orc_price_caplets.restype = C.c_int
    lib.orc_price_caplets.argtypes = [C.c_int, C.c_int, C.c_double, _dp, _dp, _dp, _dp,
                                      C.c_int64, C.c_int, C.c_uint64, C.c_int64, C.c_int, _dp, _dp]
    lib.orc_price_mbs.restype = C.c_int
    lib.orc_price_mbs.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                                  C.c_double, C.c_double, C.c_int64, C.c_int, C.c_uint64,
                                  C.c_int64, C.c_int, _dp, _dp]
    lib.orc_finalize.restype = None
    lib.orc_finalize.argtypes = [_dp, C.c_int, C.c_int, _dp, _dp, _dp]
    lib.orc_alg2_run.restype = None
    lib.orc_alg2_run.argtypes = [C.c_uint64, _ip, C.c_uint64, C.c_int64, _u64p]
    lib.orc_num_threads.restype = C.c_int
    lib.orc_num_threads.argtypes = []
    lib.orc_set_num_threads.restype = None
    lib.orc_set_num_threads.argtypes = [C.c_int]
    _lib = lib
    return lib


def _d(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def num_threads() -> int:
    return _load().orc_num_threads()


def set_num_threads(n: int) -> None:
    """OpenMP threads of the following oracle calls (timing only)."""
    _load().orc_set_num_threads(n)


# -- generator primitives --------------------------------------------------

def splitmix64(seed: int, k: int) -> int:
    """Output k (0-based) of SplitMix64 seeded with `seed`."""
    return int(_load().orc_splitmix64(seed, k))


def nth_prime(j: int) -> int:
    return int(_load().orc_nth_prime(j))


def digits(p: int) -> Tuple[int, int]:
    """(D, P): D = max{D : p^D <= 2^53}, P = p^D."""
    P = C.c_uint64(0)
    D = _load().orc_digits(p, C.byref(P))
    return int(D), int(P.value)


def start(seed: int, m_global: int, j: int, flags: int = 0) -> int:
    """Random start n_j^m in [0, P_j) (Algorithm 3, step 1)."""
    p = nth_prime(j)
    _, P = digits(p)
    n = C.c_uint64(0)
    st = _load().orc_start(seed, m_global, j, P, flags, C.byref(n))
    if st:
        raise RuntimeError(f"orc_start status {st}")
    return int(n.value)


def perm(seed: int, j: int) -> np.ndarray:
    """Random digit permutation of base j (eq. (3))."""
    p = nth_prime(j)
    out = np.zeros(p, dtype=np.int32)
    st = _load().orc_perm(seed, j, p, out.ctypes.data_as(_ip))
    if st:
        raise RuntimeError(f"orc_perm status {st}")
    return out


def perm_rep(seed: int, m_global: int, j: int) -> np.ndarray:
    """The digit permutation of base j drawn by replication m_global."""
    p = nth_prime(j)
    out = np.empty(p, dtype=np.int32)
    if _load().orc_perm_rep(seed, m_global, j, p, out.ctypes.data_as(_ip)):
        raise RuntimeError("orc_perm_rep failed")
    return out


def perm_rep_seed(seed: int, m_global: int) -> int:
    return int(_load().orc_perm_rep_seed(seed, m_global))


def radinv_R(p: int, idx: int, sigma: Optional[np.ndarray] = None) -> int:
    """R = P * phi_p^sigma(idx) (eqs. (1)-(3)), an exact integer."""
    D, _ = digits(p)
    sp = None
    if sigma is not None:
        sigma = np.ascontiguousarray(sigma, dtype=np.int32)
        sp = sigma.ctypes.data_as(_ip)
    return int(_load().orc_radinv_R(p, D, sp, idx))


def alg2_run(p: int, n: int, count: int, sigma: Optional[np.ndarray] = None) -> np.ndarray:
    """R values of `count` consecutive terms from index n by the Algorithm-2
    recursion (exact integers)."""
    out = np.empty(count, dtype=np.uint64)
    sp = None
    if sigma is not None:
        sigma = np.ascontiguousarray(sigma, dtype=np.int32)
        sp = sigma.ctypes.data_as(_ip)
    _load().orc_alg2_run(p, sp, n, count, out.ctypes.data_as(_u64p))
    return out


def point_from_R(R: int, P: int) -> float:
    return float(_load().orc_point_from_R(R, P))


def ppnd16(u) -> np.ndarray:
    """Inverse standard normal CDF (AS241, PPND16)."""
    u = _f64(u)
    flat = u.reshape(-1).copy()
    out = np.empty_like(flat)
    _load().orc_ppnd16_vec(flat.size, _d(flat), _d(out))
    return out.reshape(u.shape)


def sequence(s: int, N: int, M: int, seed: int, flags: int = 0, m_offset: int = 0,
             gen: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """Points x[M][N][s] and integers R[M][N][s] of the random-start Halton
    replications (gen 0: definition, gen 1: Algorithm 2).  With
    flags & MC_PHILOX the points are Philox4x64-10 uniforms and R is None."""
    x = np.empty((M, N, s), dtype=np.float64)
    if flags & MC_PHILOX:
        st = _load().orc_sequence(s, N, M, seed, flags, m_offset, gen, _d(x), None)
        if st:
            raise RuntimeError(f"orc_sequence status {st}")
        return x, None
    R = np.empty((M, N, s), dtype=np.uint64)
    st = _load().orc_sequence(s, N, M, seed, flags, m_offset, gen, _d(x), R.ctypes.data_as(_u64p))
    if st:
        raise RuntimeError(f"orc_sequence status {st}")
    return x, R


def philox4x64(ctr, key) -> Tuple[int, int, int, int]:
    """Philox4x64-10 (Salmon et al., SC'11) of a 4-word counter under a
    2-word key."""
    c = (C.c_uint64 * 4)(*[int(v) for v in ctr])
    k = (C.c_uint64 * 2)(*[int(v) for v in key])
    o = (C.c_uint64 * 4)()
    _load().orc_philox4x64(c, k, o)
    return tuple(int(v) for v in o)


def mc_point(seed: int, m_global: int, i: int, j: int) -> float:
    """Pseudo-random coordinate j of point i of replication m_global."""
    return float(_load().orc_mc_point(seed, m_global, i, j))


# -- models ---------------------------------------------------------------

def _lmm_arrays(model):
    return (_f64(model.L0), _f64(model.sigma), _f64(model.loadings).reshape(-1),
            _f64(model.strike))


def lmm_paths(model, z: np.ndarray, n_sub: int = 1, euler: bool = False) -> np.ndarray:
    """Discounted caplet payoffs (+ book) of paths driven by the given
    standard normals z[n_paths][n_fwd*n_sub*d] (caplet section)."""
    z = _f64(z)
    n_paths = z.shape[0]
    assert z.shape[1] == model.n_fwd * n_sub * model.n_factors
    L0, sig, b, K = _lmm_arrays(model)
    pay = np.empty((n_paths, model.n_fwd + 1), dtype=np.float64)
    _load().orc_lmm_paths(n_paths, model.n_fwd, model.n_factors, model.delta, _d(L0), _d(sig),
                          _d(b), _d(K), n_sub, int(euler), _d(z), _d(pay))
    return pay


def mbs_paths(params, z: np.ndarray) -> np.ndarray:
    """Present values of MBS paths driven by z[n_paths][months] (MBS section)."""
    z = _f64(z)
    assert z.shape[1] == params.months
    pv = np.empty(z.shape[0], dtype=np.float64)
    _load().orc_mbs_paths(z.shape[0], params.months, params.i0, params.sigma, params.K1,
                          params.K2, params.K3, params.K4, _d(z), _d(pv))
    return pv


def mbs_annuity(months: int, i0: float) -> np.ndarray:
    ck = np.empty(months + 1, dtype=np.float64)
    _load().orc_mbs_annuity(months, i0, _d(ck))
    return ck


def price_caplets(model, N: int, M: int, seed: int, m_offset: int = 0, flags: int = 0,
                  per_path: bool = False):
    """theta[M][n_fwd+1] (and per-path payoffs [M][N][n_fwd+1] if asked)."""
    L0, sig, b, K = _lmm_arrays(model)
    n_out = model.n_fwd + 1
    theta = np.empty((M, n_out), dtype=np.float64)
    pp = np.empty((M, N, n_out), dtype=np.float64) if per_path else None
    st = _load().orc_price_caplets(model.n_fwd, model.n_factors, model.delta, _d(L0), _d(sig),
                                   _d(b), _d(K), N, M, seed, m_offset, flags, _d(theta),
                                   _d(pp) if pp is not None else None)
    if st:
        raise RuntimeError(f"orc_price_caplets status {st}")
    return (theta, pp) if per_path else theta


def price_mbs(params, N: int, M: int, seed: int, m_offset: int = 0, flags: int = 0,
              per_path: bool = False):
    """theta[M][1] (and per-path PVs [M][N][1] if asked)."""
    theta = np.empty((M, 1), dtype=np.float64)
    pp = np.empty((M, N, 1), dtype=np.float64) if per_path else None
    st = _load().orc_price_mbs(params.months, params.i0, params.sigma, params.K1, params.K2,
                               params.K3, params.K4, N, M, seed, m_offset, flags, _d(theta),
                               _d(pp) if pp is not None else None)
    if st:
        raise RuntimeError(f"orc_price_mbs status {st}")
    return (theta, pp) if per_path else theta


def finalize(theta: np.ndarray):
    """(RQ, sd, SE) per output over the M replication estimates."""
    theta = _f64(theta)
    M, n_out = theta.shape
    mean = np.empty(n_out)
    sd = np.empty(n_out)
    se = np.empty(n_out)
    _load().orc_finalize(_d(theta), M, n_out, _d(mean), _d(sd), _d(se))
    return mean, sd, se
