"""Load driver for the request server: Poisson arrivals of polymul requests,
latency percentiles and throughput, continuous batching against a serial FIFO.

Request mix (the serving configuration): 70% are 1..64 polymul pairs at
N = 2^10 over one 32-bit prime (32-bit words); 30% are one pair at N = 2^16 over
the first L = 8..36 of the ~50-bit primes (64-bit words).  Operands are resident
on the device (inputs drawn from a pool, one output buffer per request); the
server admits requests by its HBM budget and batches requests of identical
shape, against the same server also merging requests of different moduli in one
arithmetic class (the 2^16 requests of different L) and a serial FIFO.

    python -m paper_2410_05934_amd.serving --requests 10000 --fractions 0.1,0.5,0.9,1.2
"""
from __future__ import annotations

import argparse
import json

import numpy as np

from . import synth


class Workload:
    """Device operands for a list of requests.

    Inputs come from a pool per (N, width): `copies` random batches shaped like
    the largest request of that group ([pairs][L][N]), whose rows every other
    request of the group reuses as a prefix (its moduli are the first L of the
    same list, or its pairs the first of the same one-modulus batch).  Request i
    reads copy i mod `copies`, so requests of one shape read different memory and
    a launch's gathers do not hit in cache more for one batching rule than for
    another; the large pool (16 x 36 limbs x 2^16 x 8 B = 302 MB per operand)
    exceeds the 256 MB Infinity Cache.  One output buffer per request."""

    def __init__(self, reqs, seed: int = 0, copies: int = 16):
        import torch
        from .tensors import empty_device, to_device
        self.reqs = reqs
        self.copies = copies
        self.pools = {}
        self.outs = []
        groups = {}
        for r in reqs:
            g = groups.setdefault((r.N, r.word_bits), r)
            if r.pairs * len(r.moduli) > g.pairs * len(g.moduli):
                groups[(r.N, r.word_bits)] = r
        for (N, wb), big in groups.items():
            shape = (big.pairs, len(big.moduli))
            for r in reqs:
                if (r.N, r.word_bits) != (N, wb):
                    continue
                if len(r.moduli) == 1 and shape[1] == 1:
                    ok = r.moduli[0] == big.moduli[0] and r.pairs <= shape[0]
                else:
                    ok = r.pairs == 1 and shape[0] == 1 and list(r.moduli) == list(big.moduli[:len(r.moduli)])
                assert ok, "request rows are not a prefix of the pool's"
            pool = []
            for k in range(copies):
                a = synth.uniform_poly(synth.derive_seed(seed, N, k, 1), big.moduli, big.pairs, N)
                b = synth.uniform_poly(synth.derive_seed(seed, N, k, 2), big.moduli, big.pairs, N)
                pool.append((to_device(a, wb), to_device(b, wb)))
            self.pools[(N, wb)] = pool
        for r in reqs:
            self.outs.append(empty_device((r.pairs, len(r.moduli), r.N), r.word_bits))
        torch.cuda.synchronize()

    def operands(self, i):
        """Device tensors (a, b, out) of request i; a and b are views of its pool copy's
        first pairs x L rows (the same words as a [pairs][L][N] batch)."""
        r = self.reqs[i]
        da, db = self.pools[(r.N, r.word_bits)][i % self.copies]
        rows = r.pairs * len(r.moduli)
        flat_a = da.reshape(-1, r.N)[:rows]
        flat_b = db.reshape(-1, r.N)[:rows]
        return flat_a, flat_b, self.outs[i]


def run_load(server, work: Workload, rate: float | None, ntt_mod) -> dict:
    """Replay every request at its arrival time (rate None: all at t = 0, a
    burst) through the library's native load generator, then collect the
    completion records and return latency statistics."""
    reqs = work.reqs
    n = len(reqs)
    gaps = np.diff([0.0] + [r.arrival_s for r in reqs])
    base_rate = n / max(reqs[-1].arrival_s, 1e-9)
    scale = 0.0 if rate is None else base_rate / rate
    arrivals = np.cumsum(gaps * scale)
    batch = []
    for i, r in enumerate(reqs):
        da, db, out = work.operands(i)
        batch.append((ntt_mod.REQ_POLYMUL, r.N, r.moduli, r.word_bits, r.pairs,
                      da.data_ptr(), db.data_ptr(), out.data_ptr()))
    ids = server.replay(batch, arrivals)
    infos = [server.wait(i, 600000) for i in ids]
    lat = np.array([x["t_done"] - x["t_submit"] for x in infos])
    t_first = min(x["t_submit"] for x in infos)
    t_last = max(x["t_done"] for x in infos)
    big = np.array([r.N == (1 << 16) for r in reqs])
    c = server.counters()
    return {
        "requests": n,
        "offered_rate": rate,
        "achieved_req_per_s": n / (t_last - t_first),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "p50_ms_small": float(np.percentile(lat[~big], 50) * 1e3) if (~big).any() else None,
        "p99_ms_small": float(np.percentile(lat[~big], 99) * 1e3) if (~big).any() else None,
        "p50_ms_large": float(np.percentile(lat[big], 50) * 1e3) if big.any() else None,
        "p99_ms_large": float(np.percentile(lat[big], 99) * 1e3) if big.any() else None,
        "mean_batch": float(np.mean([x["batched_with"] for x in infos])),
        "mean_batch_large": float(np.mean([x["batched_with"] for x, b in zip(infos, big) if b]))
        if big.any() else None,
        "launches": c["launches"],
        "merged_launches": c["merged_launches"],
        "max_inflight_bytes": c["max_inflight_bytes"],
    }


def sweep(n_requests: int, fractions, budget: int = 64 << 30, streams: int = 4, seed: int = 0,
          serial_too: bool = True, merged_too: bool = True, small_budget: int = 1 << 30) -> dict:
    """Capacity (all requests at t = 0) and open-loop load at `fractions` of it,
    per server mode: "batched" (the default server), "merged" (also merging
    moduli; capacity alone) and "serial"; then the default server's capacity
    under `small_budget` bytes (0: skipped)."""
    import paper_2410_05934_amd as ntt
    reqs = synth.c5_requests(seed, n_requests, 1000.0)
    work = Workload(reqs, seed)
    out = {"budget_bytes": budget, "streams": streams, "requests": n_requests}
    modes = [("batched", 0, True)]
    if merged_too:
        modes.append(("merged", ntt.SERVER_MERGE_MODULI, False))
    if serial_too:
        modes.append(("serial", ntt.SERVER_SERIAL, True))
    for name, flags, open_loop in modes:
        with ntt.Server(budget, streams, 0, flags) as srv:
            # warm-up: plans and twiddles resident, pools grown
            run_load(srv, _subset(work, 256), None, ntt)
            cap = run_load(srv, work, None, ntt)
            res = {"capacity_req_per_s": cap["achieved_req_per_s"], "burst": cap, "open_loop": []}
            for f in (fractions if open_loop else []):
                rate = f * cap["achieved_req_per_s"]
                res["open_loop"].append({"fraction": f, **run_load(srv, work, rate, ntt)})
            out[name] = res
    if serial_too:
        out["batched_over_serial_capacity"] = (out["batched"]["capacity_req_per_s"]
                                               / out["serial"]["capacity_req_per_s"])
    if merged_too:
        out["merged_over_batched_capacity"] = (out["merged"]["capacity_req_per_s"]
                                               / out["batched"]["capacity_req_per_s"])
    if small_budget:
        # The same burst under a small HBM budget: admission holds requests back
        # and the staging arenas stay inside the budget.
        with ntt.Server(small_budget, streams, 0, 0) as srv:
            run_load(srv, _subset(work, 256), None, ntt)
            cap = run_load(srv, work, None, ntt)
            c = srv.counters()
        out["small_budget"] = {"budget_bytes": small_budget, "capacity_req_per_s": cap["achieved_req_per_s"],
                               "p99_ms": cap["p99_ms"], "launches": cap["launches"],
                               "max_inflight_bytes": c["max_inflight_bytes"],
                               "max_arena_bytes": c["max_arena_bytes"], "rejected": c["rejected"]}
    return out


def _subset(work: Workload, k: int) -> Workload:
    w = Workload.__new__(Workload)
    w.reqs = work.reqs[:k]
    w.copies = work.copies
    w.pools = work.pools
    w.outs = work.outs[:k]
    return w


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=10000)
    ap.add_argument("--fractions", default="0.1,0.3,0.5,0.7,0.9,1.1,1.2")
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-serial", action="store_true")
    ap.add_argument("--no-merged", action="store_true")
    args = ap.parse_args()
    res = sweep(args.requests, [float(x) for x in args.fractions.split(",")],
                int(args.budget_gb * (1 << 30)), args.streams, args.seed, not args.no_serial,
                not args.no_merged)
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main()
