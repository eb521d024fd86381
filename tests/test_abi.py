"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function the public header declares, and rejects bad arguments before
touching the device."""
import ctypes as C
import math
import os
import re
import sys

import numpy as np
import pytest

import paper_1408_5526_amd as rq
import rqmc_inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header="rqmc.h"):
    txt = open(os.path.join(ROOT, "include", header)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rq_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = rq.lib()
    names = _declared()
    assert {"rq_sequence", "rq_price_caplets", "rq_price_mbs", "rq_last_error", "rq_batch_tuning"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    assert "gfx950" in rq.version()


def test_cpu_generator_library_exports_its_header():
    lib = rq.cpu_lib()
    names = _declared("rqmc_cpu.h")
    assert {"rq_cpu_sequence", "rq_cpu_alg2_run", "rq_cpu_last_error", "rq_cpu_max_threads"} == set(names)
    for n in names:
        assert hasattr(lib, n), n
    assert not any(hasattr(rq.lib(), n) for n in names)   # two libraries, nothing shared


def test_workspace_sizes_and_validation():
    lib = rq.lib()
    n = lib.rq_sequence_workspace(10, 4096, 32, 0)
    assert n >= 32 * 10 * 32
    assert lib.rq_sequence_workspace(0, 4096, 32, 0) == 0
    assert "s must be" in rq.last_error()
    assert lib.rq_sequence_workspace(5000, 4096, 32, 0) == 0
    assert "beyond" in rq.last_error()
    assert lib.rq_sequence_workspace(1, 2 ** 53 + 1, 1, 0) == 0       # N > P_0 = 2^53
    assert lib.rq_sequence_workspace(4, 100, 1, 64) == 0              # unknown flag


def _call_caplets(model, N=256, M=2, ws_bytes=1 << 20, flags=0, prec=0, theta=1):
    h = rq._LmmHost(model)
    res = rq.rq_result(theta, 0, 0, 0)
    return rq.lib().rq_price_caplets(C.byref(h.c), N, M, 1, 0, flags, prec, C.byref(res), None, None,
                                     C.c_void_p(256), ws_bytes, None)


def test_caplet_argument_errors_return_before_launch():
    m = I.cfg1().model
    bad = m.copy(); bad.L0[3] = -0.01
    assert _call_caplets(bad) == rq.RQ_EINVAL and "L0[3]" in rq.last_error()
    bad = m.copy(); bad.sigma[2] = -1.0
    assert _call_caplets(bad) == rq.RQ_EINVAL
    bad = I.small_lmm(4, 2); bad.loadings[1] *= 1.1
    assert _call_caplets(bad) == rq.RQ_EINVAL and "norm" in rq.last_error()
    big = I.lmm_curve80(n_fwd=80, n_factors=3)
    big.n_fwd = 81
    big.L0 = np.append(big.L0, 0.06); big.sigma = np.append(big.sigma, 0.1)
    big.loadings = np.vstack([big.loadings, big.loadings[-1:]]); big.strike = np.append(big.strike, 0.06)
    assert _call_caplets(big) == rq.RQ_EUNSUPPORTED
    assert _call_caplets(m, N=0) == rq.RQ_EINVAL
    assert _call_caplets(m, M=0) == rq.RQ_EINVAL
    assert _call_caplets(m, theta=0) == rq.RQ_EINVAL
    assert _call_caplets(m, flags=rq.OUT_DIGITS) == rq.RQ_EINVAL
    assert _call_caplets(m, prec=7) == rq.RQ_EINVAL
    assert _call_caplets(m, ws_bytes=16) == rq.RQ_EWORKSPACE and "needed" in rq.last_error()
    # the Greeks need a larger workspace than the prices alone
    h = rq._LmmHost(m)
    assert rq.lib().rq_caplets_workspace(C.byref(h.c), 4096, 4, 0, 1, 1) > \
        rq.lib().rq_caplets_workspace(C.byref(h.c), 4096, 4, 0, 1, 0)


def test_adjoint_store_limit_sizes_the_workspace():
    # the two-kernel adjoint stores w and the final states for one chunk of
    # 64-path tasks: (20 x 3 + 32) x 64 x 8 B = 47,104 B per task counted in
    # FP64; a limit of 7 tasks shrinks the Greeks workspace accordingly, and
    # 0 restores the default (64 GiB, i.e. all 64 tasks here)
    m = I.lmm_curve80(20, 3)
    h = rq._LmmHost(m)
    per = (20 * 3 + 32) * 64 * 8
    full = rq.lib().rq_caplets_workspace(C.byref(h.c), 4096, 1, 0, 1, 1)
    try:
        rq.set_adjoint_store_limit(7 * per)
        small = rq.lib().rq_caplets_workspace(C.byref(h.c), 4096, 1, 0, 1, 1)
        rq.set_adjoint_store_limit(1)          # below one task: still one task
        one = rq.lib().rq_caplets_workspace(C.byref(h.c), 4096, 1, 0, 1, 1)
    finally:
        rq.set_adjoint_store_limit(0)
    assert full - small == (64 - 7) * per
    assert small - one == 6 * per
    assert rq.lib().rq_caplets_workspace(C.byref(h.c), 4096, 1, 0, 1, 1) == full


def test_mbs_argument_errors_return_before_launch():
    p = rq._mbs_c(I.MbsParams(0, 0.007, 0.02, 0.01, -0.005, 10, 0.5))
    res = rq.rq_result(1, 0, 0, 0)
    st = rq.lib().rq_price_mbs(C.byref(p), 64, 1, 1, 0, 0, 0, C.byref(res), None, None, C.c_void_p(256), 1 << 20, None)
    assert st == rq.RQ_EINVAL and "months" in rq.last_error()
    p = rq._mbs_c(I.MbsParams(12, 0.007, -0.02, 0.01, -0.005, 10, 0.5))
    st = rq.lib().rq_price_mbs(C.byref(p), 64, 1, 1, 0, 0, 0, C.byref(res), None, None, C.c_void_p(256), 1 << 20, None)
    assert st == rq.RQ_EINVAL
    bad = rq.rq_result(0, 0, 0, 0)
    p = rq._mbs_c(I.mbs_paper(12))
    st = rq.lib().rq_price_mbs(C.byref(p), 64, 1, 1, 0, 0, 0, C.byref(res), C.byref(bad), None, C.c_void_p(256), 1 << 20, None)
    assert st == rq.RQ_EINVAL and "grad" in rq.last_error()


def test_misaligned_workspace_rejected():
    st = rq.lib().rq_sequence(4, 64, 1, 1, 0, 0, C.c_void_p(1 << 20), C.c_void_p(257), 1 << 30, None)
    assert st == rq.RQ_EWORKSPACE and "aligned" in rq.last_error()


def test_python_api_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError, match="no GPU"):
        rq.sequence(2, 8, 1, 1)


@pytest.mark.parametrize("n,d,delta,beta", [(80, 3, 0.25, 0.1), (20, 2, 0.25, 0.1), (33, 1, 0.5, 0.3),
                                            (3, 3, 0.25, 2.0), (1, 1, 0.25, 0.1)])
def test_pca_loadings_match_numpy_eigh(n, d, delta, beta):
    # host-only entry: the same reduction as the model inputs (numpy eigh)
    got = rq.lmm_pca_loadings(n, d, delta, beta)
    want = I.pca_loadings(np.arange(1, n + 1) * delta, beta, d)
    assert np.abs(got - want).max() < 1e-12
    assert np.allclose(np.linalg.norm(got, axis=1), 1.0, rtol=0, atol=1e-15)


def test_pca_loadings_validation():
    out = (C.c_double * 16)()
    lib = rq.lib()
    assert lib.rq_lmm_pca_loadings(0, 1, 0.25, 0.1, out) == rq.RQ_ERANGE
    assert lib.rq_lmm_pca_loadings(81, 1, 0.25, 0.1, out) == rq.RQ_ERANGE
    assert lib.rq_lmm_pca_loadings(2, 3, 0.25, 0.1, out) == rq.RQ_ERANGE
    assert lib.rq_lmm_pca_loadings(4, 4, 0.25, 0.1, out) == rq.RQ_ERANGE
    assert lib.rq_lmm_pca_loadings(4, 2, 0.0, 0.1, out) == rq.RQ_EINVAL
    assert lib.rq_lmm_pca_loadings(4, 2, 0.25, 0.0, out) == rq.RQ_EINVAL
    assert lib.rq_lmm_pca_loadings(4, 2, 0.25, 0.1, None) == rq.RQ_EINVAL
    assert "NULL" in rq.last_error()


def test_scheme_and_generator_flag_combinations():
    m = I.lmm_treasury_caplet()
    h = rq._LmmHost(m)
    res = rq.rq_result(1, 0, 0, 0)
    g = rq.rq_result(1, 0, 0, 0)

    def call(flags, grad=None):
        return rq.lib().rq_price_caplets(C.byref(h.c), 64, 1, 1, 0, flags, 0, C.byref(res),
                                         C.byref(grad) if grad is not None else None, None,
                                         C.c_void_p(256), 16, None)
    # Euler with Greeks or permutations is refused; Philox excludes the Halton options
    assert call(rq.LMM_EULER, g) == rq.RQ_EUNSUPPORTED and "log-Euler" in rq.last_error()
    assert call(rq.LMM_EULER | rq.PERM_RANDOM) == rq.RQ_EUNSUPPORTED
    assert call(rq.MC_PHILOX | rq.PERM_RANDOM) == rq.RQ_EINVAL and "RQ_MC_PHILOX" in rq.last_error()
    assert call(rq.MC_PHILOX | rq.START_ZERO) == rq.RQ_EINVAL
    # valid combinations get as far as the (too small) workspace
    assert call(rq.LMM_EULER) == rq.RQ_EWORKSPACE
    assert call(rq.LMM_EULER | rq.MC_PHILOX) == rq.RQ_EWORKSPACE
    assert call(rq.MC_PHILOX) == rq.RQ_EWORKSPACE
    # Euler is a LIBOR option only
    p = rq._mbs_c(I.mbs_paper(12))
    st = rq.lib().rq_price_mbs(C.byref(p), 64, 1, 1, 0, rq.LMM_EULER, 0, C.byref(res), None, None,
                               C.c_void_p(256), 1 << 20, None)
    assert st == rq.RQ_EINVAL and "caplets" in rq.last_error()
    st = rq.lib().rq_sequence(4, 64, 1, 1, rq.LMM_EULER, 0, C.c_void_p(256), C.c_void_p(256), 1 << 20, None)
    assert st == rq.RQ_EINVAL


def _fnv_signature(insts, prec, greeks):
    # the batch signature as the library defines it (FNV-1a 64 over the
    # little-endian bytes of each field), written again here
    h = 0xcbf29ce484222325

    def mix(v):
        nonlocal h
        for b in int(v).to_bytes(8, "little", signed=True):
            h ^= b
            h = (h * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF

    mix(prec)
    mix(1 if greeks else 0)
    mix(len(insts))
    for c in insts:
        mix(0 if c.kind == "lmm" else 1)
        mix(c.N)
        mix(c.M)
        mix(getattr(c, "flags", 0))
        if c.kind == "lmm":
            mix(c.model.n_fwd)
            mix(c.model.n_factors)
        else:
            mix(c.model.months)
    return h


def test_batch_tuning_cache_file_is_read(tmp_path):
    # a tuning kept in the RQ_TUNING_CACHE file by an earlier process is what
    # price_batch would use for that list; another list stays automatic
    import subprocess
    insts = I.cfg5()[:5]
    sig = _fnv_signature(insts, 1, True)
    f = tmp_path / "tuning.txt"
    f.write_text(f"{sig:016x} 4 3 1\n")
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_1408_5526_amd as rq, rqmc_inputs as I\n"
            "L = I.cfg5()\n"
            "print(rq.batch_tuning(L[:5], 'fp32', greeks=True), rq.batch_tuning(L[:5], 'fp32', greeks=False),"
            " rq.batch_tuning(L[:6], 'fp32', greeks=True))\n") % ROOT
    env = dict(os.environ, RQ_TUNING_CACHE=str(f))
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "((4, 3, 1), True) ((0, 0, 0), False) ((0, 0, 0), False)", out.stdout
