"""GPU tests of the request server: every result equals the oracle's and is
the same alone (serial server) and in the mix (continuous batching)."""
import numpy as np
import pytest

import oracle
from paper_2410_05934_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2410_05934_amd as ntt  # noqa: E402
from paper_2410_05934_amd.tensors import empty_device, to_device, to_host  # noqa: E402


def _requests(n, seed):
    """A serving mix with its own inputs per request (small limb counts keep the oracle quick)."""
    small_q = synth.c3_prime()
    big = synth.c2_primes(6)
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        if rng.random() < 0.7:
            N, mods, wb, pairs = 1 << 10, [small_q], 32, int(rng.integers(1, 9))
        else:
            N, mods, wb, pairs = 1 << 16, big[: int(rng.integers(1, 4))], 64, 1
        op = [ntt.REQ_POLYMUL, ntt.REQ_FORWARD, ntt.REQ_INVERSE][int(rng.integers(0, 3))] if i % 4 == 0 else ntt.REQ_POLYMUL
        a = synth.uniform_poly(seed * 100000 + 2 * i, mods, pairs, N)
        b = synth.uniform_poly(seed * 100000 + 2 * i + 1, mods, pairs, N)
        out.append((op, N, mods, wb, pairs, a, b))
    return out


def _want(req):
    op, N, mods, wb, pairs, a, b = req
    if op == ntt.REQ_POLYMUL:
        return oracle.polymul(a, b, mods)
    if op == ntt.REQ_FORWARD:
        return oracle.forward(a, mods)
    return oracle.inverse(a, mods)


def _run(reqs, flags, streams=4, budget=8 << 30, memory=ntt.REQ_DEVICE):
    results = []
    bufs, ptr_list = [], []
    for op, N, mods, wb, pairs, a, b in reqs:
        if memory == ntt.REQ_DEVICE:
            da, db = to_device(a, wb), to_device(b, wb)
            out = empty_device(a.shape, wb)
        else:
            dt = np.uint64 if wb == 64 else np.uint32
            da = torch.from_numpy(a.astype(dt).view(np.int64 if wb == 64 else np.int32)).pin_memory()
            db = torch.from_numpy(b.astype(dt).view(np.int64 if wb == 64 else np.int32)).pin_memory()
            out = torch.empty_like(da).pin_memory()
        bufs.append((da, db, out))
        ptr_list.append((da.data_ptr(), db.data_ptr(), out.data_ptr()))
    torch.cuda.synchronize()
    with ntt.Server(budget, streams, 0, flags) as srv:
        # all buffers exist before the first submit, and the native load generator
        # submits every request at t = 0: the requests arrive as a burst
        batch = [(op, N, mods, wb, pairs, *ptrs, memory)
                 for (op, N, mods, wb, pairs, a, b), ptrs in zip(reqs, ptr_list)]
        ids = srv.replay(batch, [0.0] * len(batch))
        infos = [srv.wait(i, 120000) for i in ids]
        counters = srv.counters()
    torch.cuda.synchronize()
    for (op, N, mods, wb, pairs, a, b), (da, db, out) in zip(reqs, bufs):
        if memory == ntt.REQ_DEVICE:
            results.append(to_host(out, wb).astype(np.uint64))
        else:
            results.append(out.numpy().view(np.uint64 if wb == 64 else np.uint32).astype(np.uint64))
    return results, infos, counters


def test_mix_matches_oracle_and_alone():
    reqs = _requests(48, 1)
    mixed, infos, c = _run(reqs, 0, streams=1)
    alone, infos1, c1 = _run(reqs, ntt.SERVER_SERIAL)
    assert max(x["batched_with"] for x in infos) > 1, "the mix should have batched something"
    assert all(x["batched_with"] == 1 for x in infos1)
    for req, m, s in zip(reqs, mixed, alone):
        w = _want(req)
        assert np.array_equal(m, w)
        assert np.array_equal(s, w)
    assert c["max_inflight_bytes"] <= c["budget_bytes"]


def test_host_memory_requests_and_a_small_budget():
    reqs = _requests(24, 2)
    big = max(4 * 8 * r[4] * len(r[2]) * r[1] for r in reqs)
    got, infos, c = _run(reqs, 0, streams=2, budget=big + (1 << 20), memory=ntt.REQ_HOST)
    for req, g in zip(reqs, got):
        assert np.array_equal(g, _want(req))
    assert c["max_inflight_bytes"] <= big + (1 << 20)


@pytest.mark.parametrize("flags", [0, ntt.SERVER_MERGE_MODULI])
def test_serving_mix_at_full_size(flags):
    """The serving configuration itself: 70% 1..64 polymul pairs at 2^10 over the
    32-bit prime, 30% one pair at 2^16 over 8..36 of the 50-bit primes, each with
    its own inputs; continuous batching on 4 streams (identical moduli only, and
    merging moduli) against the serial server and the oracle, word for word."""
    reqs = []
    for i, r in enumerate(synth.c5_requests(7, 40, 1000.0)):
        a = synth.uniform_poly(r.seed, r.moduli, r.pairs, r.N)
        b = synth.uniform_poly(r.seed + 1, r.moduli, r.pairs, r.N)
        reqs.append((ntt.REQ_POLYMUL, r.N, r.moduli, r.word_bits, r.pairs, a, b))
    assert any(q[1] == 1 << 16 and len(q[2]) >= 30 for q in reqs)
    assert any(q[1] == 1 << 10 and q[4] >= 40 for q in reqs)
    mixed, infos, c = _run(reqs, flags, streams=4, budget=64 << 30)
    alone, _, _ = _run(reqs, ntt.SERVER_SERIAL, streams=1, budget=64 << 30)
    assert max(x["batched_with"] for x in infos) > 1, "the mix should have batched something"
    if flags & ntt.SERVER_MERGE_MODULI:
        # batched 2^16 products run in place through row tables, without staging copies
        assert any(x["batched_with"] > 1 for x, q in zip(infos, reqs) if q[1] == 1 << 16)
        assert c["direct_launches"] >= 1
    for req, m, s in zip(reqs, mixed, alone):
        w = oracle.polymul(req[5], req[6], req[2])
        assert np.array_equal(m, w)
        assert np.array_equal(s, w)


def _mixed_moduli_requests(seed):
    """Requests whose moduli differ but share a class: 50-bit primes at N = 2^12
    (on-chip polymul) and 2^14 (two-pass polymul with workspace), 32-bit primes
    at N = 2^10, with 1..5 limbs, 1..3 polynomials, polymul / forward / inverse;
    plus requests whose two moduli fall in two classes."""
    p50 = synth.c2_primes(5)
    p32 = synth.primes_below(1 << 32, 1 << 17, 4)
    wide = [p50[0], synth.primes_below(1 << 61, 1 << 17, 1)[0]]
    rng = np.random.default_rng(seed)
    out = []
    for i in range(36):
        kind = i % 6
        if kind == 5:
            N, mods, wb = 1 << 12, wide, 64
        elif kind == 4:
            N, mods, wb = 1 << 10, p32[: 1 + i % 4], 32
        else:
            N, mods, wb = (1 << 12) if kind < 2 else (1 << 14), p50[: 1 + int(rng.integers(0, 5))], 64
        pairs = 1 + int(rng.integers(0, 3))
        op = [ntt.REQ_POLYMUL, ntt.REQ_FORWARD, ntt.REQ_INVERSE][(i // 6) % 3]
        a = synth.uniform_poly(seed * 1000 + 2 * i, mods, pairs, N)
        b = synth.uniform_poly(seed * 1000 + 2 * i + 1, mods, pairs, N)
        out.append((op, N, mods, wb, pairs, a, b))
    return out


@pytest.mark.parametrize("memory", [ntt.REQ_DEVICE, ntt.REQ_HOST])
def test_requests_of_different_moduli_share_launches_word_for_word(memory):
    """With NTT_SERVER_MERGE_MODULI, a launch over requests of different moduli
    (one virtual plan over their limbs laid end to end) gives every request the
    oracle's words and the words of the default server, which batches identical
    moduli only."""
    reqs = _mixed_moduli_requests(3)
    merged, infos, c = _run(reqs, ntt.SERVER_MERGE_MODULI, streams=1, memory=memory)
    same, _, c_same = _run(reqs, 0, streams=1, memory=memory)
    assert c["merged_launches"] >= 1 and c_same["merged_launches"] == 0
    assert c["launches"] < c_same["launches"]
    if memory == ntt.REQ_DEVICE:
        assert c["direct_launches"] >= 1      # two-pass products at 2^12 and 2^14
    else:
        assert c["direct_launches"] == 0 and c_same["direct_launches"] == 0
    for req, m, s in zip(reqs, merged, same):
        w = _want(req)
        assert np.array_equal(m, w)
        assert np.array_equal(s, w)


_CLASS_PRIMES = {
    "f64": (64, lambda: synth.c2_primes(4)),                                  # fp64 class, < 2^50
    "i64": (64, lambda: synth.primes_below(1 << 61, 1 << 17, 4)),             # 64-bit integer class
    "u32": (32, lambda: synth.primes_below(1 << 32, 1 << 17, 4)),             # 32-bit words
}


@pytest.mark.parametrize("cls", ["f64", "i64", "u32"])
@pytest.mark.parametrize("flags", [0, ntt.SERVER_MERGE_MODULI])
def test_batched_two_pass_products_read_and_write_the_requests_in_place(flags, cls):
    """Two-pass products (N = 2^16 and 2^14) batched from a burst run straight
    from the requests' buffers through row tables, in every arithmetic class:
    every result equals the oracle's, including a request whose output buffer is
    its own first operand."""
    wb, primes = _CLASS_PRIMES[cls]
    pool = primes()
    reqs = []
    for i in range(14):
        N = 1 << 16 if i % 2 == 0 else 1 << 14
        L = 3 if not flags else 1 + i % 4
        pairs = 1 + (i % 3 == 0)
        a = synth.uniform_poly(7000 + 2 * i, pool[:L], pairs, N)
        b = synth.uniform_poly(7001 + 2 * i, pool[:L], pairs, N)
        reqs.append((ntt.REQ_POLYMUL, N, pool[:L], wb, pairs, a, b))
    got, infos, c = _run(reqs, flags, streams=1)
    assert c["direct_launches"] >= 1
    assert max(x["batched_with"] for x in infos) > 1
    for req, g in zip(reqs, got):
        assert np.array_equal(g, oracle.polymul(req[5], req[6], req[2]))
    # out aliasing a: the operands are consumed by the first launch before the
    # last one writes
    da = [to_device(r[5], wb) for r in reqs]
    db = [to_device(r[6], wb) for r in reqs]
    torch.cuda.synchronize()
    with ntt.Server(8 << 30, 1, 0, flags) as srv:
        batch = [(op, N, mods, w, pairs, x.data_ptr(), y.data_ptr(), x.data_ptr())
                 for (op, N, mods, w, pairs, _, _), x, y in zip(reqs, da, db)]
        ids = srv.replay(batch, [0.0] * len(batch))
        [srv.wait(i, 120000) for i in ids]
        assert srv.counters()["direct_launches"] >= 1
    torch.cuda.synchronize()
    for req, x in zip(reqs, da):
        assert np.array_equal(to_host(x, wb).astype(np.uint64), oracle.polymul(req[5], req[6], req[2]))
