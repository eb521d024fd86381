"""The no-allocation LIBOR entry point (rq_price_caplets_noalloc): the same
results as rq_price_caplets with a caller workspace, bit for bit (the same
kernels; each 64-path task writes its own partial row, so the adjoint's
chunking does not enter the results), on consecutive calls that reuse the
library's scratch array with a smaller input the second time, and a clear
range error, with nothing launched, for a call too large for the array."""
import sys

import numpy as np
import pytest

import paper_1408_5526_amd as rq
import rqmc_inputs as I

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _same(a, b):
    return np.array_equal(_np(a).view(np.uint64), _np(b).view(np.uint64))


# (label, model, N, M, seed, flags, precision, greeks); each list runs in
# order, the second call smaller than the first
CALLS = [
    [("cfg1 greeks fp64", I.cfg1().model, 4096, 32, 1, 0, "fp64", True),
     ("cfg1 greeks fp64 smaller", I.cfg1().model, 1000, 3, 2, 0, "fp64", True)],
    # 80 forwards, 3 factors with Greeks: 384 tasks of 160 KiB (FP64
    # count) do not fit 64 MiB at once, so the adjoint runs in chunks
    [("nf80d3 greeks fp32", I.lmm_curve80(80, 3), 4096, 6, 3, 0, "fp32", True),
     ("nf80d3 prices fp32 smaller", I.lmm_curve80(80, 3), 2000, 2, 4, 0, "fp32", False)],
    [("nf20d2 perm prices fp64", I.lmm_curve80(20, 2), 3000, 8, 5, rq.PERM_RANDOM, "fp64", False),
     ("nf12d2 philox greeks fp32 smaller", I.lmm_curve80(12, 2), 700, 2, 6, rq.MC_PHILOX, "fp32", True)],
]


@pytest.mark.parametrize("calls", CALLS, ids=["cfg1", "nf80d3", "mixed"])
def test_noalloc_equals_workspace_entry_point(calls):
    for label, model, N, M, seed, flags, prec, greeks in calls:
        _say("noalloc", label, N, M, seed, flags, prec, greeks)
        got = rq.price_caplets_noalloc(model, N, M, seed, flags=flags, precision=prec, greeks=greeks)
        ref = rq.price_caplets(model, N, M, seed, flags=flags, precision=prec, greeks=greeks)
        for a, b in ((got.theta, ref.theta), (got.mean, ref.mean), (got.se, ref.se)):
            assert _same(a, b), label
        if greeks:
            for a, b in ((got.greeks.theta, ref.greeks.theta), (got.greeks.mean, ref.greeks.mean)):
                assert _same(a, b), label


def test_noalloc_rejects_a_call_beyond_the_scratch_array():
    # 1024 replications x 256 blocks x 81 outputs of FP64 partial sums: 170 MB
    c = I.cfg3()
    _say("noalloc too large")
    with pytest.raises(rq.RqError, match="scratch array"):
        rq.price_caplets_noalloc(c.model, c.N, c.M, c.seed, precision="fp32")
    # and the array still serves the next call
    got = rq.price_caplets_noalloc(c.model, 512, 2, c.seed, precision="fp32")
    ref = rq.price_caplets(c.model, 512, 2, c.seed, precision="fp32")
    assert _same(got.theta, ref.theta)
