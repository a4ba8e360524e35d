#!/usr/bin/env python3
"""Throughput benchmark of the negacyclic RNS NTT on one MI355X.

Workload (the CKKS-shaped configuration): 4 polynomials (2 ciphertexts) of
N = 2^16 in RNS form over the 36 largest primes q = 1 (mod 2^17) below 2^50,
64-bit words, coefficients uniform in [0, q) (seeded SplitMix64).

One step = the whole hot path over one batch:
    forward NTT of all 4 polynomials            144 limb transforms
    pointwise product of the 2 pairs            (72 limb products)
    inverse NTT of all 4 polynomials            144 limb transforms
    polymul of the 2 pairs (Eq. (1))            144 forward + 72 inverse
=> 504 limb transforms per step; `value` = limb transforms per second.
The forward and the pointwise products run as one call (ntt_forward_mul: the
row pass that finishes both transforms of a pair also writes their product);
--unfused-step times them as two calls, and the other form is always reported
beside the headline.

Inputs are resident in HBM before timing starts.  The step rotates over
`--sets` independent copies of its buffers (151 MB each, 1.2 GB for 8) so that
no step finds its data in the 256 MB Infinity Cache.  Twiddle tables stay
resident, as they are meant to.

`roofline` is the whole forward transform of the 4 x 36 limb-rows (its column
and row launches, timed per call with HIP events on the library's stream over
the rotating sets) against 1.25 MiB of algorithmic bytes per limb transform
(coefficients read and written once, 16 N bytes of twiddles per modulus shared
by its 4 polynomials); its `valu` entry is the fraction of the chip's VALU issue
slots the two kernels fill, from their committed rocprofv3 instruction counts
(profiles/counters.json, used only when taken on the current kernel sources).
Per-kernel figures (duration, share, algorithmic GB/s, measured HBM bytes, VALU
issue fraction) are in extra.breakdown and roofline.per_kernel.

Also reported: step-time percentiles, the CPU oracle's throughput on this host
(all cores and one core), and auxiliary figures (TFHE-shaped batch cold and
warm, external product and CMux step, batched vs one launch per polynomial,
single-transform latency, ragged batches, serving, automorphism, basis
conversion, ModUp and ModDown).

`--summarize-counters` reduces rocprofv3 counter CSVs to profiles/counters.json.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "NTTs/sec and % HBM peak at N=2^16×36 limbs and N=2^10 batch; batched vs plain"
HBM_PEAK_GBS = 8000.0


def _log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2410_05934_amd", "csrc")
    for fn in sorted(os.listdir(csrc)):
        if fn.endswith((".hpp", ".hip", ".cpp")):
            with open(os.path.join(csrc, fn), "rb") as f:
                h.update(fn.encode())
                h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(name: str, words: int, N: int, limbs: int, word_bytes: int) -> float:
    """Bytes a launch must move at minimum, by kernel kind.

    row / col pass: every coefficient read once and written once (2 * W per
    word) -- the pass cannot do less; a row pass also reads one twiddle table
    of N entries per modulus (8 B per fp64 entry, 16 B per Shoup pair).
    polymul_row: two operands read, one result written, both tables read.
    pointwise: two operands read, one result written.
    fwdmul_row: the forward rows of a and b with their product (five words moved
    per word of one operand, plus one table).
    """
    tw = 16 if "_i64_" in name else 8
    if name.startswith("fwdmul_row"):
        # a and b read, a and b written back transformed, the product written
        return 5.0 * words * word_bytes + 1.0 * limbs * N * tw
    if name.startswith("polymul_row"):
        return 3.0 * words * word_bytes + 2.0 * limbs * N * tw
    if name.startswith("row"):
        return 2.0 * words * word_bytes + 1.0 * limbs * N * tw
    if name.startswith("col"):
        return 2.0 * words * word_bytes
    if name.startswith("pointwise"):
        return 3.0 * words * word_bytes
    return 0.0


COUNTERS_PATH = os.path.join(ROOT, "profiles", "counters.json")
# VALU issue peak: 256 CUs x 4 SIMDs, one wave64 VALU instruction per SIMD per
# 4 cycles (16 lanes), at 2.4 GHz.  The fp64 operations the kernels use (add,
# mul, fma, rint) all issue at that rate on gfx950 (measured).
SIMDS = 1024
CLOCK_HZ = 2.4e9
VALU_CYCLES_PER_INST = 4


def load_counters():
    """Per-kernel figures of the committed rocprofv3 counter runs (HBM bytes and
    VALU instructions per launch), if they were taken on the current kernel
    sources; else {}."""
    if not os.path.exists(COUNTERS_PATH):
        return {}
    with open(COUNTERS_PATH) as f:
        rec = json.load(f)
    if rec.get("source_hash") != kernel_source_hash():
        return {}
    return rec.get("kernels", {})


def valu_frac(valu_insts: float, seconds: float) -> float:
    """Fraction of the chip's VALU issue slots that `valu_insts` wave
    instructions fill in `seconds`."""
    return valu_insts * VALU_CYCLES_PER_INST / (SIMDS * CLOCK_HZ * seconds)


def percentiles(ms_list) -> dict:
    import numpy as np
    a = np.asarray(ms_list, dtype=float)
    return {"median_ms": round(float(np.median(a)), 5), "p10_ms": round(float(np.percentile(a, 10)), 5),
            "p90_ms": round(float(np.percentile(a, 90)), 5), "mean_ms": round(float(a.mean()), 5),
            "samples": int(a.size)}


def timed_calls(torch, fn, reps, stream):
    """Per-call durations (ms) from HIP events recorded on `stream` around each call."""
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record(stream)
    for i in range(reps):
        fn(i)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    return [ev[i].elapsed_time(ev[i + 1]) for i in range(reps)]


def kernel_breakdown(stats: dict, counters: dict, N: int, L: int) -> dict:
    """Per kernel: launches, mean duration, share of the time, algorithmic GB/s
    and fraction of HBM peak, and (when the committed counter runs match the
    sources) measured HBM bytes and the fraction of VALU issue slots used."""
    total = sum(v["total_ms"] for v in stats.values()) or 1e-9
    out = {}
    for name, st in stats.items():
        sec = st["avg_ms"] * 1e-3
        b = algorithmic_bytes(name, st["words"] // max(1, st["launches"]), N, L, 8)
        rec = {"launches": st["launches"], "avg_us": round(st["avg_ms"] * 1e3, 2),
               "share": round(st["total_ms"] / total, 4),
               "alg_GBps": round(b / sec / 1e9, 1) if b else None,
               "hbm_frac": round(b / sec / 1e9 / HBM_PEAK_GBS, 4) if b else None}
        c = counters.get(name)
        if c:
            rec["hbm_bytes_measured"] = c.get("hbm_bytes_per_launch")
            if c.get("valu_insts_per_launch") is not None:
                rec["valu_issue_frac"] = round(valu_frac(c["valu_insts_per_launch"], sec), 4)
        out[name] = rec
    return out


def run_gpu(args):
    import numpy as np
    import torch

    import paper_2410_05934_amd as ntt
    from paper_2410_05934_amd import synth
    from paper_2410_05934_amd.tensors import empty_device, to_device

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    N, L, P = 1 << 16, 36, 4
    moduli = synth.c2_primes(L)
    tuned = {}
    if args.tune_file and os.path.exists(args.tune_file):
        # the choices of an earlier tuned run (so that a profiled run launches
        # the same kernels as the timed one)
        ntt.tune_load(args.tune_file)
        tuned["loaded"] = args.tune_file
    elif not args.no_tune:
        # The autotuner picks the pass split for this shape (and for the pairs
        # inside polymul) before anything is timed.
        for batch in (P, P // 2):
            n1, us = ntt.tune_split(N, moduli, 64, batch)
            tuned[f"split_b{batch}"] = {"n1": n1, "fwd_inv_us": round(us, 2)}
        _log(f"[bench] tuned: {tuned}")
        if args.tune_file:
            ntt.tune_save(args.tune_file)
    plan = ntt.Plan(N, moduli, 64, flags=ntt.FLAG_ROW_RADIX8 if args.row_radix8 else 0)
    _log(f"[bench] plan N={N} L={L} split n1={plan.split}; generating inputs")
    host = synth.uniform_poly(args.seed, moduli, P, N)
    X = [to_device(host, 64) for _ in range(args.sets)]
    # Output buffers are written once here (zeros), so that no set's memory is
    # first touched inside the timed region (the warm-up steps cover only some sets).
    PW = [torch.zeros((2, L, N), dtype=torch.int64, device="cuda") for _ in range(args.sets)]
    C = [torch.zeros((2, L, N), dtype=torch.int64, device="cuda") for _ in range(args.sets)]
    stream = torch.cuda.current_stream()

    def step(i, unfused=args.unfused_step, noalloc=False):
        r = i % args.sets
        x = X[r]
        if unfused:
            plan.forward(x, stream)
            plan.pointwise_mul(PW[r], x[0:2], x[2:4], stream)
        else:
            # the same forward of all four polynomials and the same products, with the
            # products written by the row pass that finishes the transforms
            plan.forward_mul(PW[r], x[0:2], x[2:4], stream)
        plan.inverse(x, stream)
        if noalloc:
            plan.polymul_noalloc(C[r], x[0:2], x[2:4], stream)
        else:
            plan.polymul(C[r], x[0:2], x[2:4], stream)

    transforms_per_step = 144 + 144 + 144 + 72
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    _log(f"[bench] warmup done ({args.warmup} steps)")

    # Timed region: K steps bracketed by events on the stream the library
    # launches on (and a device synchronisation on both sides).
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    for i in range(args.steps):
        step(args.warmup + i)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t0.elapsed_time(t1)
    ms_per_step = ms / args.steps
    value = transforms_per_step * args.steps / (ms / 1e3)
    _log(f"[bench] timed {args.steps} steps: {ms_per_step:.4f} ms/step, {value:.4g} limb-NTT/s (wall {wall:.3f}s)")

    # The same K steps with an event between consecutive steps: the spread of
    # the step time (median, p10, p90).
    step_ms = timed_calls(torch, lambda i: step(i), args.steps, stream)

    # The same K steps again with the library's per-launch events (two HIP
    # events on the kernel's own stream around every launch): per-kernel
    # durations for the breakdown.  The events add a little time between
    # launches, so `value` comes from the run above.
    counters = load_counters()
    ntt.stats_reset()
    ntt.stats_enable(True)
    t0.record(stream)
    for i in range(args.steps):
        step(i)
    t1.record(stream)
    torch.cuda.synchronize()
    ntt.stats_enable(False)
    stats = ntt.stats_collect()
    ms_events = t0.elapsed_time(t1) / args.steps
    _log(f"[bench] with per-launch events: {ms_events:.4f} ms/step")
    breakdown = kernel_breakdown(stats, counters, N, L)

    # The same steps with the forward and the pointwise product as two calls.
    t0.record(stream)
    for i in range(args.steps):
        step(i, unfused=not args.unfused_step)
    t1.record(stream)
    torch.cuda.synchronize()
    ms_other = t0.elapsed_time(t1) / args.steps
    # The same steps with the product's workspace from the library's fixed per-GPU
    # scratch (ntt_polymul_noalloc) instead of the stream-ordered pool.  Its first
    # call on a device looks up the scratch array's address (tens of ms, once per
    # process): one untimed step first.
    step(0, noalloc=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for i in range(args.steps):
        step(i, noalloc=True)
    t1.record(stream)
    torch.cuda.synchronize()
    ms_noalloc = t0.elapsed_time(t1) / args.steps

    import itertools
    rot = itertools.count()
    # Roofline: the whole forward transform of the 4 x 36 limb-rows (column pass
    # and row pass, two launches) over the rotating sets, one HIP event pair per
    # call on the library's stream.  Algorithmic bytes per limb transform:
    # 2 N W (every coefficient read and written once) + the twiddles, 16 N bytes
    # per modulus per launch shared by the 4 polynomials of that modulus: 1.25 MiB
    # at N = 2^16, W = 8 B; 144 limb transforms per call.
    reps = 16 * args.sets
    fwd_mean = _time(torch, lambda: plan.forward(X[next(rot) % args.sets], stream), reps, stream)
    inv_mean = _time(torch, lambda: plan.inverse(X[next(rot) % args.sets], stream), reps, stream)
    fwd_ms = timed_calls(torch, lambda i: plan.forward(X[i % args.sets], stream), reps, stream)
    inv_ms = timed_calls(torch, lambda i: plan.inverse(X[i % args.sets], stream), reps, stream)
    ntt.stats_reset()
    ntt.stats_enable(True)
    for i in range(reps):
        plan.forward(X[i % args.sets], stream)
    torch.cuda.synchronize()
    ntt.stats_enable(False)
    fstats = ntt.stats_collect()
    fwd_kernels = {k: v for k, v in kernel_breakdown(fstats, counters, N, L).items()}
    limb_ntt_bytes = 2 * N * 8 + 16 * N // P  # 1.25 MiB
    alg = 144 * limb_ntt_bytes
    t_fwd = percentiles(fwd_ms)
    t_avg_s = fwd_mean * 1e-3
    achieved = alg / t_avg_s / 1e9
    hbm = [counters.get(k, {}).get("hbm_bytes_per_launch") for k in fwd_kernels]
    traffic = sum(hbm) if hbm and all(h is not None for h in hbm) else None
    vi = [counters.get(k, {}).get("valu_insts_per_launch") for k in fwd_kernels]
    valu = None
    if vi and all(v is not None for v in vi):
        valu = {"insts_per_launch": sum(vi), "issue_frac": round(valu_frac(sum(vi), t_avg_s), 4),
                "peak": "1024 SIMDs x one wave64 VALU instruction per 4 cycles at 2.4 GHz"}
    # The measured copy rate for the same coefficients: a device copy of one 75.5 MB
    # set (cold, over the rotating sets) into one of two destination buffers.
    dst = [torch.empty_like(X[0]) for _ in range(2)]
    copy_mean = _time(torch, lambda: dst[next(rot) % 2].copy_(X[next(rot) % args.sets]), reps, stream)
    copy_gbps = 2 * X[0].numel() * 8 / (copy_mean * 1e-3) / 1e9
    del dst
    roofline = {"bound": "hbm", "kernel": "forward transform, 4 x 36 x 2^16: " + " + ".join(sorted(fwd_kernels)),
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "alg_bytes_per_launch": alg, "avg_launch_us": round(fwd_mean * 1e3, 2),
                "time_percentiles_ms_event_per_call": t_fwd, "valu": valu,
                "copy_GBps": round(copy_gbps, 1), "frac_of_copy": round(achieved / copy_gbps, 4),
                "per_kernel": fwd_kernels}
    _log(f"[bench] forward transform: {fwd_mean * 1e3:.2f} us, {achieved:.1f} GB/s = "
         f"{achieved / HBM_PEAK_GBS:.4f} of HBM peak; kernels {fwd_kernels}")
    extra = {"breakdown": breakdown, "ms_per_step_with_launch_events": round(ms_events, 4),
             "step_time_percentiles": percentiles(step_ms),
             ("ms_per_step_fused_forward_mul" if args.unfused_step else "ms_per_step_unfused"):
                 round(ms_other, 4),
             "ms_per_step_polymul_noalloc": round(ms_noalloc, 4),
             "rotating_sets": args.sets, "split_used": plan.split_for(P), "tuned": tuned}
    coeff_bytes = 144 * 2 * N * 8
    whole = {}
    for name, ms_list, t in (("forward", fwd_ms, fwd_mean), ("inverse", inv_ms, inv_mean)):
        pc = percentiles(ms_list)
        whole[name] = {"us": round(t * 1e3, 2), "limb_ntt_per_s": 144 / (t * 1e-3),
                       "rns_poly_ntt_per_s": 4 / (t * 1e-3),
                       "hbm_frac_coefficients": round(coeff_bytes / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                       "hbm_frac_with_tables": round(alg / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                       "percentiles_ms": pc}
    _log(f"[bench] whole transforms: {whole}")
    extra["c2_whole_transform"] = whole
    if not args.no_aux:
        import itertools
        ctr = itertools.count()
        dst = synth.primes_below(1 << 50, 1 << 17, 2 * L)[L:]
        if want(args, "automorph"):
            # Automorphism sigma_5 of every limb (coefficient domain, then the forward
            # transform's slot order) from the rotating sets into two output buffers:
            # algorithmic bytes = every word read once and written once.
            outs = [empty_device((P, L, N), 64) for _ in range(2)]
            auto = {}
            k_inv5 = pow(5, -1, 2 * N)
            for name, k, tr in (("coefficient", 5, False), ("coefficient_k_inv5", k_inv5, False),
                                ("transformed", 5, True)):
                def call(k=k, tr=tr):
                    j = next(ctr)
                    plan.automorph(outs[j % 2], X[j % args.sets], k, tr, stream)
                t = _time(torch, call, 4 * args.sets, stream)
                auto[name] = {"us": round(t * 1e3, 2),
                              "alg_GBps": round(coeff_bytes / (t * 1e-3) / 1e9, 1),
                              "hbm_frac": round(coeff_bytes / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            del outs
            _log(f"[bench] automorphism k=5: {auto}")
            extra["c2_automorph_k5"] = auto
        if want(args, "bconv"):
            # Basis conversion of the 4 x 36-limb polynomials to 36 other 50-bit primes:
            # 36 x (36 + 5) Shoup products per coefficient (five chunks of output moduli).
            conv = ntt.BasisConversion(N, moduli, dst, 64)
            yb = empty_device((P, L, N), 64)

            def bcall():
                conv(yb, X[next(ctr) % args.sets], stream)
            t = _time(torch, bcall, 2 * args.sets, stream)
            prods = P * N * L * (L + (L + 7) // 8)
            extra["c2_bconv_36_to_36"] = {"us": round(t * 1e3, 2),
                                          "modmul_per_s": prods / (t * 1e-3),
                                          "alg_GBps": round(2 * P * L * N * 8 / (t * 1e-3) / 1e9, 1)}
            del yb, conv
            _log(f"[bench] basis conversion 36 -> 36: {extra['c2_bconv_36_to_36']}")
        if want(args, "modup"):
            # ModUp of the 4 x 36-limb polynomials to Q u P with 36 special primes (the
            # next 36 primes = 1 mod 2^17 below the CKKS ones), and ModDown back: each
            # reads 36 (up) or 72 (down) limbs and writes 72 or 36, 108 limb-rows of
            # 2^16 words per polynomial.  Two wide buffers alternate.
            ext = ntt.BasisExtension(N, moduli, dst, 64)
            ups = [empty_device((P, 2 * L, N), 64) for _ in range(2)]
            dn = empty_device((P, L, N), 64)
            for j in range(2):
                ext.mod_up(ups[j], X[j], stream)

            def upcall():
                j = next(ctr)
                ext.mod_up(ups[j % 2], X[j % args.sets], stream)

            def downcall():
                ext.mod_down(dn, ups[next(ctr) % 2], stream)
            ks_bytes = P * 3 * L * N * 8
            ks = {}
            for name, fn in (("mod_up", upcall), ("mod_down", downcall)):
                t = _time(torch, fn, 2 * args.sets, stream)
                ks[name] = {"us": round(t * 1e3, 2), "alg_GBps": round(ks_bytes / (t * 1e-3) / 1e9, 1),
                            "hbm_frac": round(ks_bytes / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            del ups, dn, ext
            _log(f"[bench] ModUp / ModDown 36 + 36: {ks}")
            extra["c2_modup_moddown_36_36"] = ks
        extra.update(run_aux(args, torch, ntt, synth, np, to_device, empty_device, plan, X, stream))
    return value, ms_per_step, roofline, extra


def want(args, section: str) -> bool:
    """Whether an auxiliary section runs (--sections restricts them)."""
    return args.sections is None or section in args.sections.split(",")


def _time(torch, fn, reps, stream):
    fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def run_aux(args, torch, ntt, synth, np, to_device, empty_device, plan2, X, stream):
    out = {}
    # C2 batched (one call over 4 polynomials) vs plain (one call per RNS
    # polynomial): cold over the rotating sets, and warm on one set (75.5 MB,
    # resident in the 256 MB Infinity Cache after the first call).
    import itertools
    ctr = itertools.count()
    x2 = X[0]
    if want(args, "batched"):
        run_batched_vs_plain(args, torch, plan2, X, x2, ctr, stream, out)
    if want(args, "c3"):
        run_c3(args, torch, ntt, synth, to_device, empty_device, stream, out)
    if want(args, "c1"):
        N = 1 << 10
        q1 = synth.c1_prime(0)
        p1 = ntt.Plan(N, [q1], 32)
        x1 = to_device(synth.uniform_poly(7, [q1], 1, N), 32)
        t1 = _time(torch, lambda: (p1.forward(x1, stream), p1.inverse(x1, stream)), 200, stream)
        out["c1_fwd_inv_us"] = round(t1 * 1e3, 2)
    if want(args, "latency"):
        out["single_polynomial_56bit"] = run_latency(args, torch, ntt, synth, to_device, stream)
    if not args.no_ragged and want(args, "ragged"):
        out["c4_ragged"] = run_ragged(args, torch, ntt, synth, to_device, stream)
    if not args.no_serving and want(args, "serving"):
        run_serving(args, out)
    return out


def run_batched_vs_plain(args, torch, plan2, X, x2, ctr, stream, out):

    def cold_batched():
        plan2.forward(X[next(ctr) % args.sets], stream)

    def cold_plain():
        x = X[next(ctr) % args.sets]
        for i in range(4):
            plan2.forward(x[i:i + 1], stream)
    t_bc = _time(torch, cold_batched, 4 * args.sets, stream)
    t_pc = _time(torch, cold_plain, 4 * args.sets, stream)
    t_b = _time(torch, lambda: plan2.forward(x2, stream), 20, stream)
    t_p = _time(torch, lambda: [plan2.forward(x2[i:i + 1], stream) for i in range(4)], 20, stream)
    # One launch per (polynomial, limb): a one-modulus plan per limb, each call on one
    # limb-row of the same buffers (144 calls per forward).
    import paper_2410_05934_amd as ntt
    from paper_2410_05934_amd import synth
    limb_plans = [ntt.Plan(plan2.N, [q], 64) for q in synth.c2_primes(36)]

    def per_limb(x):
        for i in range(4):
            for l, pl in enumerate(limb_plans):
                pl.forward(x[i:i + 1, l:l + 1], stream)
    t_lc = _time(torch, lambda: per_limb(X[next(ctr) % args.sets]), 2 * args.sets, stream)
    t_l = _time(torch, lambda: per_limb(x2), 10, stream)
    for pl in limb_plans:
        pl.close()
    out["c2_forward"] = {"batched_us": round(t_bc * 1e3, 2), "per_poly_launch_us": round(t_pc * 1e3, 2),
                         "per_limb_launch_us": round(t_lc * 1e3, 2),
                         "batched_limb_ntt_per_s": 144 / (t_bc * 1e-3),
                         "batched_over_plain": round(t_pc / t_bc, 3),
                         "batched_over_per_limb": round(t_lc / t_bc, 3),
                         "warm_batched_us": round(t_b * 1e3, 2), "warm_per_poly_launch_us": round(t_p * 1e3, 2),
                         "warm_per_limb_launch_us": round(t_l * 1e3, 2),
                         "warm_batched_over_plain": round(t_p / t_b, 3),
                         "warm_batched_over_per_limb": round(t_l / t_b, 3),
                         "note": "cold: rotating sets; warm: one 75.5 MB set, Infinity-Cache resident; plain: one "
                                 "call per RNS polynomial (all its limbs); per limb: one call per (polynomial, limb)"}


def run_c3(args, torch, ntt, synth, to_device, empty_device, stream, out):
    """TFHE-shaped: 2048 x 2^10 u32 forward, MAC (6 rows x 2 cols), 684 inverse;
    the fused external product, its decomposing form and the CMux step."""
    import itertools
    N, Pn, rows, cols = 1 << 10, 2048, 6, 2
    q = synth.c3_prime()
    p3 = ntt.Plan(N, [q], 32)
    a = to_device(synth.uniform_poly(5, [q], Pn, N), 32)
    key = to_device(synth.uniform_poly(6, [q], rows * cols, N), 32)
    G = (Pn + rows - 1) // rows
    acc = empty_device((G * cols, 1, N), 32)
    work = a.clone()

    def c3_batched():
        work.copy_(a)
        p3.forward(work, stream)
        p3.mac(acc, work, key, rows, cols, stream)
        p3.inverse(acc, stream)

    def c3_plain():
        work.copy_(a)
        for i in range(Pn):
            p3.forward(work[i:i + 1], stream)
        p3.mac(acc, work, key, rows, cols, stream)
        for i in range(G * cols):
            p3.inverse(acc[i:i + 1], stream)

    acc2 = empty_device((G * cols, 1, N), 32)

    def c3_fused():
        p3.external_product(acc2, a, key, rows, cols, stream)

    # The same product from the ciphertexts themselves: G RLWE ciphertexts of
    # k+1 = 2 components, each coefficient split into 3 signed digits of base
    # 2^11 inside the kernel (rows = 2 x 3 = 6 operands per ciphertext).
    ct = to_device(synth.uniform_poly(8, [q], G * 2, N), 32).reshape(G, 2, 1, N)
    key4 = key.reshape(rows, cols, 1, N)
    acc3 = empty_device((G, cols, 1, N), 32)

    def c3_decomposed():
        p3.external_product_decomposed(acc3, ct, key4, 3, 11, stream)

    # One batched CMux step of blind rotation over the same ciphertexts:
    # acc + ExtProd(key, X^a acc - acc), a different rotation per ciphertext.
    rot3 = torch.tensor([(37 * g + 11) % (2 * N) for g in range(G)], dtype=torch.int32, device="cuda")
    cm_out = empty_device((G, 2, 1, N), 32)

    def c3_cmux():
        p3.cmux(cm_out, ct, rot3, key4, 3, 11, stream)

    # The 2048-operand forward alone: cold over 40 copies of the operands
    # (336 MB, more than the Infinity Cache) and warm on one copy (8.4 MB).
    sets3 = [a.clone() for _ in range(40)]
    ctr3 = itertools.count()
    t_fc = _time(torch, lambda: p3.forward(sets3[next(ctr3) % 40], stream), 80, stream)
    t_fw = _time(torch, lambda: p3.forward(work, stream), 80, stream)
    del sets3
    tb = _time(torch, c3_batched, 20, stream)
    tp = _time(torch, c3_plain, 3, stream)
    tf = _time(torch, c3_fused, 20, stream)
    td = _time(torch, c3_decomposed, 20, stream)
    tcm = _time(torch, c3_cmux, 20, stream)
    copy_ms = _time(torch, lambda: work.copy_(a), 20, stream)
    torch.cuda.synchronize()
    n3 = Pn + G * cols
    # Algorithmic bytes (u32 words, N = 2^10): a limb transform reads and writes
    # its 4 KiB (8 KiB); the MAC reads the 2048 operands and the 12 key rows and
    # writes the 684 accumulators; the fused external product moves the same
    # words as the MAC; the decomposing form and the CMux step read the 342 x 2
    # ciphertext rows instead of the 2048 digit operands.
    row_b = N * 4
    b_fwd = Pn * 2 * row_b
    b_mac = (Pn + rows * cols + G * cols) * row_b
    b_inv = G * cols * 2 * row_b
    b_dec = (G * 2 + rows * cols + G * cols) * row_b

    def frac(b, ms):
        return round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    out["c3_tfhe"] = {"forward_2048_cold_us": round(t_fc * 1e3, 2),
                      "forward_2048_cold_hbm_frac": frac(b_fwd, t_fc),
                      "forward_2048_cold_limb_ntt_per_s": Pn / (t_fc * 1e-3),
                      "forward_2048_warm_us": round(t_fw * 1e3, 2),
                      "forward_2048_warm_hbm_frac": frac(b_fwd, t_fw),
                      "fwd_mac_inv_hbm_frac": frac(b_fwd + b_mac + b_inv, tb - copy_ms),
                      "external_product_hbm_frac": frac(b_mac, tf),
                      "external_product_decomposed_hbm_frac": frac(b_dec, td),
                      "cmux_step_hbm_frac": frac(b_dec, tcm),
                      "note": "8.4 MB of operands fit in the Infinity Cache: every figure but "
                              "forward_2048_cold is warm",
                      "batched_us": round(tb * 1e3, 2), "plain_us": round(tp * 1e3, 2),
                      "input_copy_us": round(copy_ms * 1e3, 2),
                      "batched_ntt_per_s": n3 / ((tb - copy_ms) * 1e-3),
                      "batched_over_plain": round(tp / tb, 2),
                      "external_product_us": round(tf * 1e3, 2),
                      "external_product_ntt_per_s": n3 / (tf * 1e-3),
                      "external_product_same_words": bool(torch.equal(acc, acc2)),
                      "decomposed_ciphertexts": G,
                      "external_product_decomposed_us": round(td * 1e3, 2),
                      "external_product_decomposed_ntt_per_s": (G * rows + G * cols) / (td * 1e-3),
                      "cmux_step_us": round(tcm * 1e3, 2),
                      "cmux_per_s": G / (tcm * 1e-3)}


def run_serving(args, out):
    from paper_2410_05934_amd import serving
    res = serving.sweep(args.serving_requests, [0.1, 0.3, 0.5, 0.7, 0.9, 1.1, 1.2], 64 << 30, 4,
                        args.seed, True)
    keep = ("offered_rate", "achieved_req_per_s", "p50_ms", "p99_ms", "p99_ms_small",
            "p99_ms_large", "mean_batch", "mean_batch_large")
    out["c5_serving"] = {
        "requests": res["requests"], "budget_bytes": res["budget_bytes"], "streams": res["streams"],
        "batched_capacity_req_per_s": res["batched"]["capacity_req_per_s"],
        "batched_burst_launches": res["batched"]["burst"]["launches"],
        "merged_capacity_req_per_s": res["merged"]["capacity_req_per_s"],
        "merged_burst_launches": res["merged"]["burst"]["launches"],
        "merged_burst_merged_launches": res["merged"]["burst"]["merged_launches"],
        "serial_capacity_req_per_s": res["serial"]["capacity_req_per_s"],
        "batched_over_serial_capacity": res["batched_over_serial_capacity"],
        "merged_over_batched_capacity": res["merged_over_batched_capacity"],
        "small_budget": res["small_budget"],
        "batched": [{"fraction": o["fraction"], **{k: o[k] for k in keep}} for o in res["batched"]["open_loop"]],
        "serial": [{"fraction": o["fraction"], **{k: o[k] for k in keep}} for o in res["serial"]["open_loop"]],
    }


def run_latency(args, torch, ntt, synth, to_device, stream):
    """One polynomial over one 56-bit prime, N = 2^12 .. 2^16 (the single-transform
    setting of the paper's Tab. ntt-mix, Sec. VI-A): the forward time at every pass
    split (the paper's switching-point sweep, Sec. V-C), then the forward and inverse
    with the split and row radix the autotuner picks for this shape.  Times are
    means over back-to-back calls on one stream."""
    q = synth.latency_prime()
    out = {"q_bits": q.bit_length(), "reps": 200}
    for logn in (args.latency_logn or range(12, 17)):
        N = 1 << logn
        x = to_device(synth.uniform_poly(900 + logn, [q], 1, N), 64)
        sweep = {}
        for n1 in range(0, 6):
            if not ((n1 == 0 and logn <= 14) or (n1 >= 1 and 4 <= logn - n1 <= 14)):
                continue
            p = ntt.Plan(N, [q], 64, flags=ntt.flag_split(n1))
            sweep[str(n1)] = round(_time(torch, lambda: p.forward(x, stream), 200, stream) * 1e3, 2)
            p.close()
        if not args.no_tune:
            ntt.tune_split(N, [q], 64, 1)
        p = ntt.Plan(N, [q], 64)
        fwd = _time(torch, lambda: p.forward(x, stream), 200, stream) * 1e3
        inv = _time(torch, lambda: p.inverse(x, stream), 200, stream) * 1e3
        out[f"N=2^{logn}"] = {"split_sweep_fwd_us": sweep, "split": p.split_for(1),
                              "fwd_us": round(fwd, 2), "inv_us": round(inv, 2)}
        p.close()
    _log(f"[bench] single polynomial, 56-bit q: {out}")
    return out


def run_ragged(args, torch, ntt, synth, to_device, stream):
    """Ragged mix: 256 instances, N = 2^(10+U{0..6}), L = U{1..40} primes of 30..60
    bits from a 64-prime pool, u64 words.  Forward then inverse of everything as
    two ragged batches replayed from hipGraphs (persistent kernel for N <= 2^12,
    grouped two-pass launches for larger N), against one forward and one inverse
    call per polynomial (batch 1 each); also the variant that runs every size in
    the persistent kernel (one workgroup per large transform)."""
    inst = synth.c4_instances(args.seed)
    if not args.no_tune:
        big = sorted({it.N for it in inst if it.N >= (1 << 13)})
        pool = synth.c4_pool(args.seed)
        for N in big:
            ntt.tune_ragged(N, [q for q in pool if q < (1 << 50)][:8], 4)
    plans, tens = [], []
    words = 0
    limb_ntts = 0
    for i, it in enumerate(inst):
        p = ntt.Plan(it.N, it.moduli, 64)
        h = synth.uniform_poly(args.seed * 7919 + i, it.moduli, 1, it.N)
        plans.append(p)
        tens.append(to_device(h, 64))
        words += h.size
        limb_ntts += len(it.moduli)
    _log(f"[bench] ragged: {len(inst)} instances, {words * 8 / 1e9:.3f} GB, {limb_ntts} limb-rows")
    fwd = ntt.RaggedBatch([(p, ntt.OP_FORWARD, t) for p, t in zip(plans, tens)])
    inv = ntt.RaggedBatch([(p, ntt.OP_INVERSE, t) for p, t in zip(plans, tens)])
    items, wgs = fwd.info()
    fwd_wg = ntt.RaggedBatch([(p, ntt.OP_FORWARD, t) for p, t in zip(plans, tens)], ntt.RAGGED_IN_WORKGROUP)
    inv_wg = ntt.RaggedBatch([(p, ntt.OP_INVERSE, t) for p, t in zip(plans, tens)], ntt.RAGGED_IN_WORKGROUP)

    def persistent():
        fwd.run(stream)
        inv.run(stream)

    def persistent_wg():
        fwd_wg.run(stream)
        inv_wg.run(stream)

    def plain():
        for p, t in zip(plans, tens):
            p.forward(t, stream)
        for p, t in zip(plans, tens):
            p.inverse(t, stream)

    t_pers = _time(torch, persistent, 10, stream)
    t_wg = _time(torch, persistent_wg, 10, stream)
    t_plain = _time(torch, plain, 5, stream)
    n = 2 * limb_ntts
    return {"instances": len(inst), "gbytes": round(words * 8 / 1e9, 3), "limb_rows": limb_ntts,
            "items": items, "persistent_workgroups": wgs,
            "persistent_graph_ms": round(t_pers, 3), "one_launch_per_poly_ms": round(t_plain, 3),
            "persistent_limb_ntt_per_s": n / (t_pers * 1e-3),
            "plain_limb_ntt_per_s": n / (t_plain * 1e-3),
            "persistent_over_plain": round(t_plain / t_pers, 3),
            "all_in_persistent_kernel_ms": round(t_wg, 3),
            "alg_GBps_persistent": round(2 * 2 * words * 8 / (t_pers * 1e-3) / 1e9, 1)}


def run_cpu_baseline(args):
    """The oracle (plain radix-2, unsigned __int128 %, one thread per core)
    timed on a bounded sample: whole C2 steps repeated until cpu_seconds pass."""
    import oracle
    from paper_2410_05934_amd import synth
    N, L = 1 << 16, 36
    moduli = synth.c2_primes(L)
    x = synth.uniform_poly(args.seed, moduli, 4, N)
    cores = oracle.num_cores()
    t0 = time.perf_counter()
    steps = 0
    while True:
        f = oracle.forward(x, moduli, cores)
        oracle.pointwise_mul(f[0:2], f[2:4], moduli)
        oracle.inverse(f, moduli, cores)
        oracle.polymul(x[0:2], x[2:4], moduli, cores)
        steps += 1
        el = time.perf_counter() - t0
        if el >= args.cpu_seconds:
            break
    # One core: forward + inverse of one of the polynomials (72 limb transforms)
    # repeated for about a quarter of the time.
    t1 = time.perf_counter()
    reps1 = 0
    while True:
        oracle.inverse(oracle.forward(x[0:1], moduli, 1), moduli, 1)
        reps1 += 1
        el1 = time.perf_counter() - t1
        if el1 >= args.cpu_seconds / 4:
            break
    return {"value": 504 * steps / el, "unit": "limb-NTT/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} whole steps of the same workload (4x36x2^16, fwd+pointwise+inv+polymul), "
                      f"{el:.1f} s, {cores} threads over (poly, limb) rows",
            "one_core": {"value": 72 * reps1 / el1, "unit": "limb-NTT/s", "cores": 1,
                         "sample": f"{reps1} x forward + inverse of one 36-limb 2^16 polynomial, {el1:.1f} s"},
            "host": _host_cpu(), "per_config": run_cpu_per_config(args, cores)}


def _host_cpu() -> dict:
    """The host's CPU model (/proc/cpuinfo) and the threads the OS reports."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "os_cpu_count": os.cpu_count()}


def run_cpu_per_config(args, cores: int) -> dict:
    """The oracle on the other configurations, each repeated for about an eighth
    of cpu_seconds (at least once): C1 latency shape on one core, the C3 TFHE
    batch (2048 forward, MAC 6 x 2, 684 inverse), the first 16 instances of the
    C4 ragged mix (forward + inverse), and the C5 request mix (polymul per
    request, in arrival order)."""
    import oracle
    from paper_2410_05934_amd import synth
    budget = args.cpu_seconds / 8

    def repeat(fn):
        t0 = time.perf_counter()
        n = 0
        while True:
            fn(n)
            n += 1
            el = time.perf_counter() - t0
            if el >= budget:
                return n, el

    out = {}
    q1 = synth.c1_prime(0)
    x1 = synth.uniform_poly(args.seed, [q1], 1, 1 << 10)
    n, el = repeat(lambda i: oracle.inverse(oracle.forward(x1, [q1], 1), [q1], 1))
    out["c1"] = {"value": round(n / el, 1), "unit": "forward+inverse pairs/s", "cores": 1,
                 "sample": f"{n} x forward + inverse of one 2^10 polynomial, {el:.1f} s"}
    q3 = synth.c3_prime()
    x3 = synth.uniform_poly(args.seed, [q3], 2048, 1 << 10)
    k3 = synth.uniform_poly(6, [q3], 12, 1 << 10).reshape(6, 2, 1, 1 << 10)

    def c3(i):
        acc = oracle.mac(oracle.forward(x3, [q3], cores), k3, [q3], 6, 2)
        oracle.inverse(acc.reshape(-1, 1, 1 << 10), [q3], cores)

    n, el = repeat(c3)
    out["c3"] = {"value": round((2048 + 684) * n / el, 1), "unit": "limb-NTT/s", "cores": cores,
                 "sample": f"{n} x (2048 forward, MAC, 684 inverse) at 2^10, {el:.1f} s"}
    inst = synth.c4_instances(args.seed)[:16]
    xs = [synth.uniform_poly(synth.derive_seed(args.seed, j), r.moduli, 1, r.N) for j, r in enumerate(inst)]
    rows = sum(len(r.moduli) for r in inst)

    def c4(i):
        for r, x in zip(inst, xs):
            oracle.inverse(oracle.forward(x, r.moduli, cores), r.moduli, cores)

    n, el = repeat(c4)
    out["c4"] = {"value": round(2 * rows * n / el, 1), "unit": "limb-NTT/s", "cores": cores,
                 "sample": f"{n} x forward + inverse of the first 16 ragged instances ({rows} limb-rows), {el:.1f} s"}
    reqs = synth.c5_requests(args.seed, 64, 1000.0)
    ops = [(synth.uniform_poly(r.seed, r.moduli, r.pairs, r.N), synth.uniform_poly(r.seed + 1, r.moduli, r.pairs, r.N),
            r.moduli) for r in reqs]
    done = [0]

    def c5(i):
        a, b, m = ops[i % len(ops)]
        oracle.polymul(a, b, m, cores)
        done[0] += 1

    n, el = repeat(c5)
    out["c5"] = {"value": round(n / el, 1), "unit": "req/s", "cores": cores,
                 "sample": f"{n} requests of the serving mix (polymul each, in arrival order), {el:.1f} s"}
    return out


_CLS = {"ArF64S": "f64s", "ArF64L": "f64l", "ArI64": "i64"}


def bench_name(symbol: str, log_n: int = 16):
    """The library's per-launch timer name of a HIP kernel symbol as rocprofv3
    prints it (for the kernels of the CKKS-shaped workload, N = 2^log_n), or None."""
    import re
    m = re.search(r"nttk::(\w+)<([^>]*)>", symbol)
    if not m:
        return None
    kind, targs = m.group(1), [t.strip().replace("nttk::", "") for t in m.group(2).split(",")]
    if kind == "col_kernel":
        a, n1, inv, two = targs[:4]
        return f"col_{'inv' if inv == 'true' else 'fwd'}_{_CLS[a]}_log{n1}{'_2pass' if two == 'true' else ''}"
    if kind == "row_kernel":
        a, n2, inv, two, rb = targs[:5]
        pre = {"4": "row", "3": "row8", "2": "row4"}[rb]
        return f"{pre}_{'inv' if inv == 'true' else 'fwd'}_{_CLS[a]}_log{n2}{'_2pass' if two == 'true' else ''}"
    if kind == "polymul_row_kernel":
        a, n2, two, rb = targs[:4]
        fm = len(targs) > 4 and targs[4] == "true"
        pre = ("fwdmul_row" if fm else "polymul_row") + ("8" if rb == "3" else "")
        return f"{pre}_fwd_{_CLS[a]}_log{n2}{'_2pass' if two == 'true' else ''}"
    if kind == "pointwise_kernel":
        return f"pointwise_fwd_{_CLS[targs[0]]}_log{log_n}"
    if kind in ("bconv_mfma_kernel", "bconv_f64_kernel", "bconv_kernel"):
        w = "u32" if "unsigned int" in targs[0] else "u64"
        mode = int(targs[-1])
        base = ["bconv", "modup", "moddown"][mode]
        form = {"bconv_mfma_kernel": "_mfma", "bconv_f64_kernel": "_f64", "bconv_kernel": ""}[kind]
        return f"{base}{form}_fwd_{w}_log{log_n}"
    return None


def _per_dispatch(csv_paths: str) -> dict:
    """{kernel symbol: {counter: mean per dispatch (summed over instances)}, "_n": dispatches}
    over one or more comma-separated rocprofv3 counter CSVs."""
    import csv
    from collections import defaultdict
    sums = defaultdict(lambda: defaultdict(float))
    disp = defaultdict(set)
    for path in csv_paths.split(","):
        with open(path) as f:
            for r in csv.DictReader(f):
                k = r["Kernel_Name"]
                sums[k][r["Counter_Name"]] += float(r["Counter_Value"])
                disp[k].add((path, r["Dispatch_Id"]))
    return {k: {**{c: v / len(disp[k]) for c, v in cs.items()}, "_n": len(disp[k])} for k, cs in sums.items()}


def summarize_counters(args) -> None:
    """Reduce rocprofv3 counter runs (FETCH_SIZE, WRITE_SIZE, the same two on the
    calibration copy, and the VALU / LDS set) to profiles/counters.json: per
    kernel, HBM bytes and VALU instructions per launch, keyed by the hash of the
    kernel sources they were taken on."""
    cal_f = _per_dispatch(args.cal_fetch_csv)
    cal_w = _per_dispatch(args.cal_write_csv)
    copy_bytes = float(1 << 30)
    fcopy = max((v for v in cal_f.values()), key=lambda v: v.get("FETCH_SIZE", 0))["FETCH_SIZE"] * 1024
    wcopy = max((v for v in cal_w.values()), key=lambda v: v.get("WRITE_SIZE", 0))["WRITE_SIZE"] * 1024
    ff, wf = copy_bytes / fcopy, copy_bytes / wcopy
    fetch = _per_dispatch(args.fetch_csv)
    write = _per_dispatch(args.write_csv)
    valu = _per_dispatch(args.valu_csv) if args.valu_csv else {}
    kernels = {}
    for sym in sorted(set(fetch) | set(write) | set(valu)):
        name = bench_name(sym)
        if name is None:
            continue
        rec = {"symbol": sym.split("(")[0].replace("void ", "").replace("nttk::", "")}
        if sym in fetch and sym in write:
            rec["launches_sampled"] = int(fetch[sym]["_n"])
            rec["fetch_bytes_per_launch"] = round(fetch[sym]["FETCH_SIZE"] * 1024 * ff)
            rec["write_bytes_per_launch"] = round(write[sym]["WRITE_SIZE"] * 1024 * wf)
            rec["hbm_bytes_per_launch"] = rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
        if sym in valu:
            v = valu[sym]
            for key, c in (("valu_insts_per_launch", "SQ_INSTS_VALU"), ("valu_active_quads_per_launch", "SQ_ACTIVE_INST_VALU"),
                           ("lds_insts_per_launch", "SQ_INSTS_LDS"), ("lds_bank_conflict_cycles", "SQ_LDS_BANK_CONFLICT"),
                           ("lds_active_cycles", "SQ_LDS_IDX_ACTIVE"), ("waves_per_launch", "SQ_WAVES"),
                           ("gui_active_cycles_sum_xcc", "GRBM_GUI_ACTIVE")):
                if c in v:
                    rec[key] = round(v[c])
            if "SQ_ACTIVE_INST_VALU" in v and "GRBM_GUI_ACTIVE" in v:
                # rocprofv3's VALUBusy: quad-cycles of VALU work per CU over the
                # busy cycles of one XCD (GRBM_GUI_ACTIVE is summed over 8 here)
                rec["valu_busy_frac"] = round(v["SQ_ACTIVE_INST_VALU"] / 256 / (v["GRBM_GUI_ACTIVE"] / 8), 4)
            if "SQ_LDS_IDX_ACTIVE" in v and "SQ_LDS_BANK_CONFLICT" in v and v["SQ_LDS_IDX_ACTIVE"] > 0:
                rec["lds_conflicts_per_access"] = round(
                    v["SQ_LDS_BANK_CONFLICT"] / max(1.0, v["SQ_LDS_IDX_ACTIVE"] - v["SQ_LDS_BANK_CONFLICT"]), 4)
        kernels[name] = rec
    out = {"source_hash": kernel_source_hash(),
           "calibration": {"kernel": "device copy of 1 GiB (torch copy_)", "fetch_factor": round(ff, 4),
                           "write_factor": round(wf, 4)},
           "command": args.counters_command, "kernels": kernels}
    with open(COUNTERS_PATH, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def calibrate_copy(gib: int = 1, reps: int = 4) -> None:
    """A plain device copy of known size, for scaling the HBM byte counters:
    each launch reads and writes exactly `gib` GiB."""
    import torch
    n = (gib << 30) // 8
    a = torch.ones(n, dtype=torch.int64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes_each_way": n * 8, "launches": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--sets", type=int, default=8, help="rotating buffer sets (defeats the 256 MB MALL)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-aux", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--tune-file", default=None,
                    help="load the tuning table from this file if it exists, else tune and save it there")
    ap.add_argument("--no-ragged", action="store_true")
    ap.add_argument("--sections", default=None,
                    help="comma list of auxiliary sections to run (automorph, bconv, modup, batched, "
                         "c3, c1, latency, ragged, serving); default all")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--row-radix8", action="store_true", help="radix-8 row passes")
    ap.add_argument("--unfused-step", action="store_true",
                    help="forward and pointwise product as two calls instead of ntt_forward_mul")
    ap.add_argument("--serving-requests", type=int, default=10000)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration) and exit")
    ap.add_argument("--latency-only", action="store_true",
                    help="only run the single-polynomial 56-bit section (one JSON line) and exit")
    ap.add_argument("--latency-logn", type=int, nargs="*", default=None,
                    help="log2 N of the single-polynomial section (default 12 .. 16)")
    ap.add_argument("--summarize-counters", action="store_true",
                    help="reduce rocprofv3 counter CSVs (--fetch-csv, --write-csv, --cal-fetch-csv, "
                         "--cal-write-csv, --valu-csv) to profiles/counters.json and exit")
    ap.add_argument("--fetch-csv")
    ap.add_argument("--write-csv")
    ap.add_argument("--cal-fetch-csv")
    ap.add_argument("--cal-write-csv")
    ap.add_argument("--valu-csv")
    ap.add_argument("--counters-command", default="", help="the rocprofv3 commands, recorded in the JSON")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(args)
        return
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.latency_only:
        import torch
        import paper_2410_05934_amd as ntt
        from paper_2410_05934_amd import synth
        from paper_2410_05934_amd.tensors import to_device
        torch.cuda.init()
        res = run_latency(args, torch, ntt, synth, to_device, torch.cuda.current_stream())
        print(json.dumps({"single_polynomial_56bit": res}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (every "
              "(poly, limb) transform is independent, so limbs would be dealt to GPUs "
              "round-robin with no exchange). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    value, ms_per_step, roofline, extra = run_gpu(args)
    cpu = None if args.no_cpu else run_cpu_baseline(args)
    line = {
        "metric": METRIC, "value": value, "unit": "limb-NTT/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": "ckks-rns: 4 polys x 36 limbs x N=2^16, 36 largest primes q=1 mod 2^17 "
                               "below 2^50, u64 words; step = fwd + pointwise "
                               + ("(separate calls)" if args.unfused_step else "(one row pass, ntt_forward_mul)")
                               + " + inv + polymul",
                   "N": 1 << 16, "limbs": 36, "polys": 4, "word_bits": 64,
                   "transforms_per_step": 504, "parallelism": "single-gpu"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
