#!/usr/bin/env python3
"""Throughput benchmark of the RQMC pricing path on one MI355X.

Workload (default): the 80-forward, 3-factor LIBOR market model caplet book
(quarterly forwards over 20 years, 4%->6% curve, humped vol, PCA-reduced
exponential correlation, 80 ATM caplets + book), s = 240 Halton bases,
N = 2^16 points x M = 1024 random-start replications, seed 3.  One step is
one full pricing call: random starts, radical inverses, inverse normal,
log-Euler paths, payoffs, theta_N^m, RQ_{M,N}, sd and SE -- inputs resident
on the device, outputs left on the device.

The headline form computes the paths in FP32 (digits, points, numeraire
and reductions in FP64); the plain FP64 form is timed beside it on the same
points, so both reach the same standard error.  The dominant kernel's
launches are timed with HIP events recorded by the library on the launch
stream; the CPU oracle is timed on a bounded sample of the same workload.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Work per path of the 80-forward, 3-factor book, counted from the kernels'
# arithmetic as written (flops: FMA = 2, add/sub/mul = 1, each special
# function = 1, FP32 and FP64 alike; integer digit work not counted):
#  * forward-step (3,240 per path): drift factor 1/(1 + kappa 2^-X) (exp2,
#    FMA, rcp: 4), w += g delta a (3 FMA: 6), the increment
#    log2(e)(c + a.w) (3 FMA: 6), the state add (1): 17;
#  * coordinate (240): the point R RN(1/P) (1), the FP32 inverse normal's
#    main branch (u(1-u): 2, log: 1, FMA: 2, 2u-1: 2, t: 1, 9 FMA: 18,
#    product: 1 = 27): 28;
#  * payoff (80, pricing kernel): 2^X and the fixing value (2), 1 + delta L
#    (2), L - K (1), numeraire product (1), Newton reciprocal (rcp and 4
#    FMA: 9), delta (L - K) / num times the caplet flag (3), the book (1): 19;
#  * reverse forward-step (3,240, adjoint): the increment e = log2(e)(c +
#    a.w) (3 FMA: 6), the pre-step state X - e (1), the drift factor (4),
#    Wbar += Xbar log2(e) a (3 FMA: 6), delta a.Wbar (mul, 2 FMA: 5), h = g
#    (delta a.Wbar) (1), the vega entry (e + c, FMA, add: 4), Xbar += ln2 h
#    (1 - g) (2 FMA: 4), the w rewind (3 FMA: 6): 37;
#  * payoff section of the reverse kernel (80): the book over a common
#    denominator (10), the payoffs again with their adjoint (27), the delta
#    and vega outputs (4): 41.
FLOPS_FWD_STEP, FLOPS_COORD, FLOPS_PAYOFF, FLOPS_REV_STEP, FLOPS_PAYOFF_ADJ = 17, 28, 19, 37, 41
N_FS, N_COORD, N_FWD = 3_240, 240, 80
FLOPS_PER_PATH_LMM80 = N_FS * FLOPS_FWD_STEP + N_COORD * FLOPS_COORD + N_FWD * FLOPS_PAYOFF
# The adjoint's two kernels: the forward passes (no payoffs), then the
# payoffs with the reverse sweep.
FLOPS_PER_PATH_LMM80_FWD = N_FS * FLOPS_FWD_STEP + N_COORD * FLOPS_COORD
FLOPS_PER_PATH_LMM80_REV = N_FS * FLOPS_REV_STEP + N_FWD * FLOPS_PAYOFF_ADJ
FLOPS_PER_PATH_LMM80_GREEKS = FLOPS_PER_PATH_LMM80_FWD + FLOPS_PER_PATH_LMM80_REV
# The survey's algorithmic count of the textbook scheme (26 flops per
# forward-step, 32 per inverse normal, 12 per payoff, one division per
# point), reported beside the as-written count for the pricing kernel.
FLOPS_PER_PATH_LMM80_SURVEY = 93_040
N_GREEKS_LMM80 = 2 * 80 + 1
PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}   # MI355X vector peaks (published)


ADJ_SOURCES = ("rq_lmm_adj.h", "rq_lmm_adj32.hip", "rq_device.h", "rq_internal.h")
PRICE_SOURCES = ("rq_lmm.h", "rq_lmm.hip", "rq_device.h", "rq_internal.h")


def _kernel_source_hash(names) -> str:
    """Hash of the kernel sources' code: comments, blank lines and trailing
    spaces are dropped first (the sources hold no comment markers inside
    string literals), so a profile stays matched across comment edits."""
    import hashlib
    import re
    m = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_1408_5526_amd", "csrc", name)) as f:
            text = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
        lines = (re.sub(r"//.*", "", ln).rstrip() for ln in text.split("\n"))
        m.update("\n".join(ln for ln in lines if ln).encode())
    return m.hexdigest()[:16]


def _traffic_bytes(profile: str, sources):
    """HBM bytes per launch of a kernel from a committed rocprofv3
    FETCH_SIZE / WRITE_SIZE measurement, scaled by the copy-probe factors --
    or None when there is none or the kernel source has changed since."""
    path = os.path.join(ROOT, "profiles", profile)
    try:
        kv = {}
        with open(path) as f:
            for line in f:
                if line.strip() and not line.startswith("#"):
                    k, v = line.split()
                    kv[k] = v
        if kv.get("source_hash") != _kernel_source_hash(sources):
            return None
        return (float(kv["fetch_kib"]) * float(kv["fetch_factor"]) +
                float(kv["write_kib"]) * float(kv["write_factor"])) * 1024.0
    except (OSError, KeyError, ValueError):
        return None


def _executed_flops(profile: str, sources):
    """FLOP-type instructions one launch of a kernel executed, from a
    committed rocprofv3 counter run (SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_{F32,
    F64} per dispatch): 64 lanes x (ADD + MUL + 2 FMA + TRANS), every lane
    counted -- or None when there is none or the kernel source has changed
    since."""
    path = os.path.join(ROOT, "profiles", profile)
    try:
        kv = {}
        with open(path) as f:
            for line in f:
                if line.strip() and not line.startswith("#"):
                    k, v = line.split()
                    kv[k] = v
        if kv.get("source_hash") != _kernel_source_hash(sources):
            return None
        tot = 0.0
        for prec in ("F32", "F64"):
            tot += float(kv[f"SQ_INSTS_VALU_ADD_{prec}"]) + float(kv[f"SQ_INSTS_VALU_MUL_{prec}"])
            tot += 2.0 * float(kv[f"SQ_INSTS_VALU_FMA_{prec}"]) + float(kv[f"SQ_INSTS_VALU_TRANS_{prec}"])
        return 64.0 * tot
    except (OSError, KeyError, ValueError):
        return None


def _time_steps(fn, steps: int, warmup: int):
    import torch
    import paper_1408_5526_amd as rq
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    rq.timer_begin(steps)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    last = None
    for _ in range(steps):
        last = fn()
    stop.record()
    torch.cuda.synchronize()
    kernel_ms, n = rq.timer_end()
    total_ms = start.elapsed_time(stop)
    _time_steps.parts = (rq.timer_part(1), rq.timer_part(2))   # adjoint halves: (ms, launches)
    return total_ms / steps, kernel_ms / max(n, 1), last


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(model, N: int, seed: int, m_per_core: int):
    import oracle as O
    cores = O.num_threads()
    m_sub = m_per_core * cores
    t0 = time.perf_counter()
    cpu_baseline.theta = O.price_caplets(model, N, m_sub, seed)   # kept for the error statement
    dt = time.perf_counter() - t0
    # the same oracle on one core (2 replications)
    O.set_num_threads(1)
    t1 = time.perf_counter()
    O.price_caplets(model, N, 2, seed)
    dt1 = time.perf_counter() - t1
    O.set_num_threads(cores)
    return {"value": m_sub * N / dt, "unit": "paths/s", "cores": cores, "kind": "oracle",
            "sample": f"{m_sub} of the 1024 replications at full N = {N} "
                      f"({m_per_core} per thread), FP64, {dt:.1f} s",
            "value_1core": 2 * N / dt1, "sample_1core": f"2 replications at N = {N} on one thread, {dt1:.1f} s",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count()}


def generator_leg(rq, torch, dev, steps: int):
    """Halton point generation alone on the GPU (the counter-based form, one
    thread per number, written to HBM as FP64): numbers per second for the
    random-start sequence with and without random digit permutations
    (Rasrap), 240 dimensions.  Context for the paper's generator tables."""
    s, n, m = 240, 1 << 16, 16
    out = {"s": s, "N": n, "M": m}
    for name, flags in (("random_start", 0), ("rasrap", rq.PERM_RANDOM)):
        buf = torch.empty((m, n, s), dtype=torch.float64, device=dev)
        ws = torch.empty(rq.sequence_workspace(s, n, m, flags), dtype=torch.uint8, device=dev)
        _, kms, _ = _time_steps(lambda: rq.sequence(s, n, m, 5, flags, device=dev, out=buf, ws=ws), steps, 1)
        out[name + "_gnumbers_per_s"] = s * n * m / (kms / 1e3) / 1e9
        out[name + "_kernel_ms"] = kms
        out[name + "_write_tb_s"] = s * n * m * 8 / (kms / 1e3) / 1e12
        del buf, ws
    # a plain write of the same bytes (torch's fill kernel), for the rate that
    # writes alone reach on this device beside the published 8 TB/s
    buf = torch.empty((m, n, s), dtype=torch.float64, device=dev)
    buf.fill_(0.0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        buf.fill_(1.0)
    e1.record()
    torch.cuda.synchronize()
    out["fill_write_tb_s"] = buf.numel() * 8 / (e0.elapsed_time(e1) / steps / 1e3) / 1e12
    del buf
    out["note"] = ("FP64 digit expansion per number, 8 B written per number; the pricing kernels "
                   "generate the same points in registers and never store them")
    return out


def cpu_generator_baseline():
    """The oracle's recursive generator (Algorithm 2, exact integer partial
    sums, one thread) on consecutive indices of the first 240 bases."""
    import numpy as np
    import oracle as O
    count, n0, total = 1 << 18, 123456789, 0
    t0 = time.perf_counter()
    for j in range(240):
        p = O.nth_prime(j)
        total += O.alg2_run(p, n0 % (p ** 4), count).size
    dt = time.perf_counter() - t0
    return {"value": total / dt / 1e9, "unit": "GNumbers/s", "cores": 1, "kind": "oracle",
            "sample": f"Algorithm 2, {count} consecutive terms in each of 240 bases, {dt:.2f} s"}


def cpu_simd_generator():
    """The recursive generator built as a CPU baseline (librqmc_cpu.so:
    Algorithm 2 on exact integer partial sums, blocks of low digits in SIMD
    lanes, OpenMP over (replication, index range)), producing the same
    [M][N][s] FP64 points as the GPU leg: all host threads on the GPU leg's
    shape, and one thread on one replication of it."""
    import numpy as np
    import paper_1408_5526_amd as rq
    s, n, m = 240, 1 << 16, 16
    out = np.empty((m, n, s), dtype=np.float64)
    rq.cpu_sequence(s, n, 1, 5, out=out)                 # first touch of the pages
    rq.cpu_sequence(s, n, m, 5, out=out)
    t0 = time.perf_counter()
    rq.cpu_sequence(s, n, m, 5, out=out)
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()
    rq.cpu_sequence(s, n, 1, 5, threads=1, out=out)
    dt1 = time.perf_counter() - t1
    return {"value": s * n * m / dt / 1e9, "unit": "GNumbers/s", "cores": rq.cpu_max_threads(),
            "kind": "recursive generator (Algorithm 2), multi-core SIMD",
            "sample": f"s = {s}, N = 2^16, M = {m} FP64 points ([M][N][s]), {dt:.2f} s",
            "value_1core": s * n / dt1 / 1e9, "sample_1core": f"M = 1 on one thread, {dt1:.2f} s",
            "cpu_model": _cpu_model()}


def mbs_leg(rq, I, torch, dev, steps: int):
    """The 360-month MBS pool (s = 360, N = 2^14, M = 64): paths/s in FP64 and
    FP32 (and FP32 with the pathwise dPV/di0), and the paper's efficiency
    (sample sd of the estimates x time) of the Halton replications against
    Philox points."""
    c = I.cfg2()
    out = {"workload": "mbs360_N2^14_M64", "N": c.N, "M": c.M}
    ws = torch.empty(rq.mbs_workspace(c.model, c.N, c.M, 0, "fp64", greeks=True), dtype=torch.uint8, device=dev)
    for name, prec, flags, gr in (("fp64", "fp64", 0, False), ("fp32", "fp32", 0, False),
                                  ("fp32_philox", "fp32", rq.MC_PHILOX, False), ("fp32_greeks", "fp32", 0, True)):
        ms, kms, r = _time_steps(lambda: rq.price_mbs(c.model, c.N, c.M, c.seed, flags=flags, precision=prec,
                                                      greeks=gr, device=dev, ws=ws), steps, 1)
        sd = r.sd[0].item()
        out[name] = {"paths_per_s": c.N * c.M / (ms / 1e3), "ms_per_step": ms, "kernel_ms": kms,
                     "pv": r.mean[0].item(), "sd": sd, "efficiency_sd_x_s": sd * ms / 1e3}
        if gr:
            out[name]["dpv_di0"] = r.greeks.mean[0].item()
            out[name]["dpv_di0_se"] = r.greeks.se[0].item()
    return out


def small_call_leg(rq, I, torch, dev, calls: int = 50):
    """The small 1-factor caplet (10 forwards, s = 10, N = 4096, M = 32):
    host-to-result latency of one call (median wall time, stream synced),
    and the device time of its main kernel."""
    import statistics
    c = I.cfg1()
    ws = torch.empty(rq.caplets_workspace(c.model, c.N, c.M, 0, "fp64"), dtype=torch.uint8, device=dev)
    out = {"workload": "lmm10_1f_caplet_N4096_M32"}
    for prec in ("fp32", "fp64"):
        f = lambda: rq.price_caplets(c.model, c.N, c.M, c.seed, precision=prec, device=dev, ws=ws)
        f()
        torch.cuda.synchronize()
        walls = []
        for _ in range(calls):
            t0 = time.perf_counter()
            f()
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
        _, kms, r = _time_steps(f, 5, 1)
        out[prec] = {"call_us_median": statistics.median(walls) * 1e6, "kernel_us": kms * 1e3,
                     "price": r.mean[-1].item()}
    return out


def cpu_mbs_baseline():
    """The oracle on the same MBS workload, a bounded sample of replications."""
    import oracle as O
    import rqmc_inputs as I
    c = I.cfg2()
    cores = O.num_threads()
    m_sub = min(c.M, 4 * cores)
    t0 = time.perf_counter()
    O.price_mbs(c.model, c.N, m_sub, c.seed)
    dt = time.perf_counter() - t0
    return {"value": m_sub * c.N / dt, "unit": "paths/s", "cores": cores, "kind": "oracle",
            "sample": f"{m_sub} of the {c.M} replications at full N = {c.N}, FP64, {dt:.1f} s"}


def batch_leg(rq, I, torch, dev, n_cap: int, m_cap: int, steps: int, autotune: bool = True):
    """The 256-instrument batch (FP32 prices + Greeks) in one persistent
    launch: the autotuner picks the launch shape for the list (kept for its
    signature, so the timed calls pass no tuning), then whole-batch paths/s
    and the per-instrument completion times (from the batch start) and
    spans, from the device real-time counter."""
    import numpy as np
    insts = I.cfg5()
    if n_cap or m_cap:
        import dataclasses
        insts = [dataclasses.replace(c, N=min(c.N, n_cap or c.N), M=min(c.M, m_cap or c.M)) for c in insts]
    paths = sum(c.N * c.M for c in insts)
    ws = torch.empty(rq.batch_workspace(insts, "fp32", greeks=True), dtype=torch.uint8, device=dev)
    tune = {}
    if autotune:
        t0 = time.perf_counter()
        (chunk, per_cu, order), tms = rq.autotune_batch(insts, "fp32", greeks=True, device=dev, ws=ws)
        tune = {"chunk": chunk or "automatic", "waves_per_cu": per_cu or "resident",
                "order": "cost" if order == rq.ORDER_COST else "given",
                "autotune_ms": tms, "autotune_wall_s": time.perf_counter() - t0}
    used, from_tuner = rq.batch_tuning(insts, "fp32", greeks=True)
    tune["used_by_price_batch"] = {"chunk": used[0], "waves_per_cu": used[1], "order": used[2],
                                   "from_autotuner": from_tuner}
    rq.price_batch(insts, "fp32", greeks=True, device=dev, ws=ws)   # warm-up
    torch.cuda.synchronize()
    walls, br = [], None
    for _ in range(max(1, steps)):
        t0 = time.perf_counter()
        br = rq.price_batch(insts, "fp32", greeks=True, device=dev, ws=ws)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
    hz = rq.realtime_hz()
    tf = br.t_first.cpu().numpy().view(np.uint64).astype(np.float64)
    tl = br.t_last.cpu().numpy().view(np.uint64).astype(np.float64)
    done = (tl - tf.min()) / hz * 1e3
    span = (tl - tf) / hz * 1e3
    wall = float(np.median(walls))
    return {"workload": "cfg5_256_instruments" + ("" if not (n_cap or m_cap) else f"_N<=2^{n_cap.bit_length() - 1}_M<={m_cap}"),
            "n_instruments": len(insts), "paths": paths, "precision": "fp32", "greeks": True,
            "tuning": tune,
            "paths_per_s": paths / wall, "ms_per_batch": wall * 1e3,
            "kernel_span_ms": float((tl.max() - tf.min()) / hz * 1e3),
            "completion_ms_p50": float(np.percentile(done, 50)), "completion_ms_p99": float(np.percentile(done, 99)),
            "span_ms_p50": float(np.percentile(span, 50)), "span_ms_p99": float(np.percentile(span, 99))}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--skip-fp64", action="store_true", help="do not time the FP64 comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-m-per-core", type=int, default=4)
    ap.add_argument("--batch", default="full", choices=["capped", "full", "off"],
                    help="256-instrument batch leg: as drawn (full), N <= 2^14 and M <= 64 (capped), or none")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="batch leg: skip the autotuner (automatic launch shape)")
    ap.add_argument("--no-generators", dest="generators", action="store_false",
                    help="skip the point-generation leg")
    ap.add_argument("--no-mbs", dest="mbs", action="store_false", help="skip the MBS leg")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy MIB mebibytes device-to-device (calibrates HBM byte counters)")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(replications would shard across GPUs by m_offset)", file=sys.stderr)
        return 2

    import torch
    import paper_1408_5526_amd as rq
    import rqmc_inputs as I

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_probe:
        n = args.copy_probe << 20
        src = torch.ones(n // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        scratch = torch.empty(n // 4, dtype=torch.float32, device=dev)
        scratch.fill_(2.0)          # evicts src from the caches
        torch.cuda.synchronize()
        dst.copy_(src)              # reads n bytes, writes n bytes
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n}), flush=True)
        return 0
    c = I.cfg3()
    model, N, M, seed = c.model, c.N, c.M, c.seed

    ws = torch.empty(max(rq.caplets_workspace(model, N, M, 0, "fp32"),
                         rq.caplets_workspace(model, N, M, 0, "fp64")), dtype=torch.uint8, device=dev)

    def step(prec):
        return lambda: rq.price_caplets(model, N, M, seed, precision=prec, device=dev, ws=ws)

    # 1) the full hot path: FP32 prices + 161 Greeks (adjoint kernel)
    wsg = torch.empty(rq.caplets_workspace(model, N, M, 0, "fp32", greeks=True), dtype=torch.uint8, device=dev)
    ms_g, kms_g, res_g = _time_steps(
        lambda: rq.price_caplets(model, N, M, seed, precision="fp32", greeks=True, device=dev, ws=wsg),
        args.steps, args.warmup)
    (fwd_ms, fwd_n), (rev_ms, rev_n) = _time_steps.parts
    # 2) prices only, FP32 and the plain FP64 form, same points
    head = args.precision
    ms, kms, res = _time_steps(step(head), args.steps, args.warmup)
    out_extra = {}
    res64 = None
    if not args.skip_fp64 and head != "fp64":
        ms64, kms64, res64 = _time_steps(step("fp64"), args.steps, args.warmup)
        rq64, se64 = res64.mean[-1].item(), res64.se[-1].item()
        # the like-for-like comparison: FP64 prices + the same 161 Greeks
        wsg64 = torch.empty(rq.caplets_workspace(model, N, M, 0, "fp64", greeks=True), dtype=torch.uint8,
                            device=dev)
        ms64g, kms64g, res64g = _time_steps(
            lambda: rq.price_caplets(model, N, M, seed, precision="fp64", greeks=True, device=dev, ws=wsg64),
            args.steps, args.warmup)
        del wsg64
        out_extra = {
            "fp64_paths_per_s": N * M / (ms64 / 1e3),
            "fp64_ms_per_step": ms64,
            "fp64_kernel_ms": kms64,
            "fp64_greeks_paths_per_s": N * M / (ms64g / 1e3),
            "fp64_greeks_ms_per_step": ms64g,
            "speedup_vs_fp64_greeks": ms64g / ms_g,
            "fp64_greeks_vs_fp32_greeks_max_rel": float(
                ((res64g.greeks.mean - res_g.greeks.mean).abs().max() / res64g.greeks.mean.abs().max()).item()),
            "speedup_vs_fp64": ms64 / ms_g,
            "book_rq": {"fp32_greeks": res_g.mean[-1].item(), "fp32": res.mean[-1].item(), "fp64": rq64},
            "book_se": {"fp32_greeks": res_g.se[-1].item(), "fp32": res.se[-1].item(), "fp64": se64},
            "se_ratio": res_g.se[-1].item() / se64,
            "book_rel_diff_fp32_vs_fp64": abs(res_g.mean[-1].item() - rq64) / abs(rq64),
        }
    gm, gse = res_g.greeks.mean, res_g.greeks.se
    out_extra["greeks"] = {
        "n": N_GREEKS_LMM80,
        "delta_L40": gm[39].item(), "delta_L40_se": gse[39].item(),
        "vega_s40": gm[81 + 39].item(), "vega_s40_se": gse[81 + 39].item(),
        "delta_spot": gm[80].item(),
    }
    # the paper's comparison: the same kernels on Philox pseudo-random points
    ms_mc, kms_mc, res_mc = _time_steps(
        lambda: rq.price_caplets(model, N, M, seed, flags=rq.MC_PHILOX, precision="fp32", device=dev, ws=ws),
        args.steps, args.warmup)
    out_extra["mc_philox_fp32"] = {
        "paths_per_s": N * M / (ms_mc / 1e3), "kernel_ms": kms_mc,
        "book_rq": res_mc.mean[-1].item(), "book_se": res_mc.se[-1].item(),
        "se_ratio_mc_over_rqmc": res_mc.se[-1].item() / res.se[-1].item()}
    # the paper's efficiency: sample sd of the M estimates x execution time
    # (lower is better), book price, FP32 prices only
    out_extra["efficiency_sd_x_s"] = {"rqmc_halton": res.sd[-1].item() * ms / 1e3,
                                      "mc_philox": res_mc.sd[-1].item() * ms_mc / 1e3}
    out_extra["prices_only_fp32"] = {
        "paths_per_s": N * M / (ms / 1e3), "ms_per_step": ms, "kernel_ms": kms,
        "achieved_tflops": FLOPS_PER_PATH_LMM80 * N * M / (kms / 1e3) / 1e12,
        "flops_per_path": FLOPS_PER_PATH_LMM80,
        "achieved_tflops_survey_count": FLOPS_PER_PATH_LMM80_SURVEY * N * M / (kms / 1e3) / 1e12,
        "flops_per_path_survey": FLOPS_PER_PATH_LMM80_SURVEY,
        "traffic": _traffic_bytes("lmm80_3f_fp32_traffic.txt", PRICE_SOURCES)}

    dtype = "f32"
    peak = PEAK_TFLOPS[dtype]
    # the dominant kernel is the reverse half; its launches cover equal
    # chunks of the N M paths, so flops per launch / mean launch time is the
    # whole count over the summed launch times
    paths_timed = N * M * args.steps
    achieved = FLOPS_PER_PATH_LMM80_REV * paths_timed / (rev_ms / 1e3) / 1e12
    achieved_fwd = FLOPS_PER_PATH_LMM80_FWD * paths_timed / (fwd_ms / 1e3) / 1e12
    rev_launch_s = rev_ms / max(rev_n, 1) / 1e3
    fwd_launch_s = fwd_ms / max(fwd_n, 1) / 1e3
    ex_rev = _executed_flops("lmm80_3f_fp32_greeks_rev_flops.txt", ADJ_SOURCES)
    ex_fwd = _executed_flops("lmm80_3f_fp32_greeks_fwd_flops.txt", ADJ_SOURCES)
    line = {
        "metric": "RQMC paths/s + Greeks/s (LMM 80-fwd caplets) vs plain FP64, at equal std err",
        "value": N * M / (ms_g / 1e3),
        "unit": "paths/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_g,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": "lmm80_3f_caplet_book_greeks", "n_fwd": 80, "n_factors": 3, "s": 240,
                   "N": N, "M": M, "seed": seed, "precision": "fp32", "greeks": N_GREEKS_LMM80},
        "greeks_per_s": N * M * N_GREEKS_LMM80 / (ms_g / 1e3),
        "greeks_per_s_lmm160": N * M * (N_GREEKS_LMM80 - 1) / (ms_g / 1e3),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": _traffic_bytes("lmm80_3f_fp32_greeks_rev_traffic.txt", ADJ_SOURCES),
                     "kernel": "lmm_adj_rev_kernel<80,3,float,false>", "kernel_ms": rev_ms / max(rev_n, 1),
                     "launches_per_step": rev_n / args.steps,
                     "flops_per_path": FLOPS_PER_PATH_LMM80_REV, "flops_basis": "kernel arithmetic as written",
                     "executed": ex_rev / rev_launch_s / 1e12 if ex_rev else None,
                     "executed_frac": ex_rev / rev_launch_s / 1e12 / peak if ex_rev else None,
                     "peak_single_issue": 78.6},
        "roofline_fwd": {"bound": "alu", "achieved": achieved_fwd, "peak": peak, "unit": "TFLOP/s",
                         "frac": achieved_fwd / peak,
                         "traffic": _traffic_bytes("lmm80_3f_fp32_greeks_fwd_traffic.txt", ADJ_SOURCES),
                         "kernel": "lmm_adj_fwd_kernel<80,3,float,false>", "kernel_ms": fwd_ms / max(fwd_n, 1),
                         "launches_per_step": fwd_n / args.steps,
                         "flops_per_path": FLOPS_PER_PATH_LMM80_FWD, "flops_basis": "kernel arithmetic as written",
                         "executed": ex_fwd / fwd_launch_s / 1e12 if ex_fwd else None,
                         "executed_frac": ex_fwd / fwd_launch_s / 1e12 / peak if ex_fwd else None},
        "adjoint_pass": {"kernel_ms": kms_g, "flops_per_path": FLOPS_PER_PATH_LMM80_GREEKS,
                         "achieved": FLOPS_PER_PATH_LMM80_GREEKS * N * M / (kms_g / 1e3) / 1e12},
    }
    line.update(out_extra)
    if args.batch != "off":
        caps = (1 << 14, 64) if args.batch == "capped" else (0, 0)
        line["batch"] = batch_leg(rq, I, torch, dev, caps[0], caps[1], 3, args.autotune)
    if args.generators:
        line["generators"] = generator_leg(rq, torch, dev, 3)
    if args.mbs:
        line["mbs"] = mbs_leg(rq, I, torch, dev, 3)
        line["small_call"] = small_call_leg(rq, I, torch, dev)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(model, N, seed, args.cpu_m_per_core)
        # every GPU form's estimates against the FP64 oracle on the replications
        # the oracle computed (all 81 outputs: 80 caplets and the book)
        import numpy as np
        th_o = cpu_baseline.theta
        errs = {}
        for name, r in (("fp32_greeks", res_g), ("fp32", res), ("fp64", res64)):
            if r is None:
                continue
            th = r.theta[:th_o.shape[0]].cpu().numpy()
            rel = np.abs(th - th_o) / np.abs(th_o)
            errs[name] = {"max_rel": float(rel.max()), "book_max_rel": float(rel[:, -1].max())}
        line["error_vs_oracle"] = {"replications": int(th_o.shape[0]), "outputs": int(th_o.shape[1]),
                                   "theta_rel_err": errs}
        if args.generators:
            line["generators"]["cpu_recursive"] = cpu_generator_baseline()
            line["generators"]["cpu_recursive_simd"] = cpu_simd_generator()
        if args.mbs:
            line["mbs"]["cpu_baseline"] = cpu_mbs_baseline()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
