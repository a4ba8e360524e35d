"""GPU parity of ragged batches (one persistent launch, hipGraph replay) and of
the autotuner: results must be bit-identical to the oracle whatever the
schedule.  Chameleon (arXiv 2410.05934), Sec. V-D (single launch)."""
import os
import random

import numpy as np
import pytest

import oracle
from paper_2410_05934_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2410_05934_amd as ntt  # noqa: E402
from paper_2410_05934_amd.tensors import to_device, to_host  # noqa: E402

Q50 = synth.c2_primes(4)
Q60 = synth.primes_below(1 << 61, 1 << 17, 3)
Q30 = synth.primes_below(1 << 30, 1 << 17, 2)
Q32 = synth.primes_below(1 << 32, 1 << 17, 3)


def _mixed_jobs(seed):
    rng = random.Random(seed)
    specs = []
    for logn in range(4, 17):
        for wb in (64, 32):
            pool = Q32 if wb == 32 else Q50 + Q60 + Q30
            L = rng.randint(1, 3)
            mods = rng.sample(pool, L)
            batch = rng.randint(1, 3)
            op = rng.randint(0, 2)
            specs.append((1 << logn, mods, wb, batch, op))
    return specs


def _build(specs, seed):
    """Transform jobs are (plan, op, tensor); product jobs (plan, OP_POLYMUL,
    out, a, b).  hosts[i] is the input (a product job: the pair (a, b))."""
    jobs, hosts = [], []
    for i, (N, mods, wb, batch, op) in enumerate(specs):
        plan = ntt.Plan(N, mods, wb)
        h = synth.uniform_poly(seed * 1000 + i, mods, batch, N)
        if op == ntt.OP_POLYMUL:
            h2 = synth.uniform_poly(seed * 1000 + i + 500, mods, batch, N)
            out = to_device(np.zeros_like(h), wb)
            jobs.append((plan, op, out, to_device(h, wb), to_device(h2, wb)))
            hosts.append((h, h2))
        else:
            jobs.append((plan, op, to_device(h, wb)))
            hosts.append(h)
    return jobs, hosts


def _expected(specs, hosts):
    out = []
    for (N, mods, wb, batch, op), h in zip(specs, hosts):
        if op == ntt.OP_POLYMUL:
            out.append(oracle.polymul(h[0], h[1], mods))
        else:
            out.append(oracle.forward(h, mods) if op == 0 else oracle.inverse(h, mods))
    return out


def _check(specs, jobs, want, hosts=None):
    torch.cuda.synchronize()
    for i, ((N, mods, wb, batch, op), job, w) in enumerate(zip(specs, jobs, want)):
        assert np.array_equal(to_host(job[2], wb).astype(np.uint64), w), (N, mods, wb, batch, op)
        if op == ntt.OP_POLYMUL and hosts is not None:   # operands untouched
            assert np.array_equal(to_host(job[3], wb).astype(np.uint64), hosts[i][0])
            assert np.array_equal(to_host(job[4], wb).astype(np.uint64), hosts[i][1])


def _reset(specs, jobs, hosts):
    for (N, mods, wb, batch, op), job, h in zip(specs, jobs, hosts):
        if op == ntt.OP_POLYMUL:
            job[2].zero_()
        else:
            job[2].copy_(to_device(h, wb))


@pytest.mark.parametrize("flags", [0, ntt.RAGGED_NO_GRAPH,
                                   ntt.RAGGED_IN_WORKGROUP,
                                   ntt.RAGGED_IN_WORKGROUP | ntt.ragged_row_log(11),
                                   ntt.RAGGED_IN_WORKGROUP | ntt.ragged_row_log(12) | ntt.RAGGED_NO_GRAPH])
def test_ragged_mixed_sizes_classes_widths(flags):
    specs = _mixed_jobs(1)
    jobs, hosts = _build(specs, 1)
    want = _expected(specs, hosts)
    assert any(sp[4] == ntt.OP_POLYMUL and sp[0] >= 1 << 13 for sp in specs)
    assert any(sp[4] == ntt.OP_POLYMUL and sp[0] <= 1 << 12 for sp in specs)
    rb = ntt.RaggedBatch(jobs, flags)
    items, wgs = rb.info()
    assert items >= len(specs) and wgs >= 1
    rb.run()
    _check(specs, jobs, want, hosts)


def test_ragged_graph_replays_after_eager_work():
    """Replay the captured graph several times with eager work in between."""
    specs = _mixed_jobs(2)
    jobs, hosts = _build(specs, 2)
    want = _expected(specs, hosts)
    rb = ntt.RaggedBatch(jobs)
    for rep in range(3):
        _reset(specs, jobs, hosts)             # eager reset of the inputs
        torch.cuda.synchronize()
        rb.run()
        _check(specs, jobs, want, hosts)


def test_batch_ragged_one_shot_and_plain_launches_agree():
    specs = _mixed_jobs(3)
    jobs, hosts = _build(specs, 3)
    want = _expected(specs, hosts)
    ntt.batch_ragged(jobs)
    _check(specs, jobs, want, hosts)
    # the same jobs one launch per polynomial through the plain calls
    _reset(specs, jobs, hosts)
    for (N, mods, wb, batch, op), job in zip(specs, jobs):
        plan, t = job[0], job[2]
        for b in range(batch):
            if op == ntt.OP_POLYMUL:
                plan.polymul(t[b:b + 1], job[3][b:b + 1], job[4][b:b + 1])
            else:
                (plan.forward if op == 0 else plan.inverse)(t[b:b + 1])
    _check(specs, jobs, want, hosts)


def test_ragged_rejects_bad_product_jobs():
    plan = ntt.Plan(1 << 10, Q32[:1], 32)
    a = to_device(synth.uniform_poly(1, Q32[:1], 2, 1 << 10), 32)
    with pytest.raises(ntt.NTTError):               # out overlaps a
        ntt.RaggedBatch([(plan, ntt.OP_POLYMUL, a, a[1:2].reshape(1, 1, -1).repeat(2, 1, 1), a)])
    lib = ntt.lib()
    arr = ntt._jobs_array([(plan, ntt.OP_FORWARD, a)])
    arr[0].op = 3                                   # unknown kind
    h = ntt._vp()
    assert lib.ntt_ragged_create(ntt.ctypes.byref(h), ntt.ctypes.cast(arr, ntt._vp), 1, 0) == 1
    arr = ntt._jobs_array([(plan, ntt.OP_FORWARD, a)])
    arr[0].a = a[1:2].data_ptr()                    # a transform job works in place only
    assert lib.ntt_ragged_create(ntt.ctypes.byref(h), ntt.ctypes.cast(arr, ntt._vp), 1, 0) == 1


@pytest.mark.parametrize("flags", [0, ntt.RAGGED_IN_WORKGROUP])
def test_ragged_products_at_serving_shapes(flags):
    """The request mix of the serving workload as one ragged batch of products:
    1..64 pairs at 2^10 over the 32-bit prime, and single pairs at 2^16 over
    8..36 of the 50-bit primes; every product against the oracle."""
    rng = random.Random(7)
    q3 = synth.c3_prime()
    big = synth.c2_primes(36)
    specs = []
    for i in range(12):
        if i % 3 == 2:
            specs.append((1 << 16, big[:rng.randint(8, 36)], 64, 1, ntt.OP_POLYMUL))
        else:
            specs.append((1 << 10, [q3], 32, rng.randint(1, 64), ntt.OP_POLYMUL))
    jobs, hosts = _build(specs, 11)
    want = _expected(specs, hosts)
    ntt.RaggedBatch(jobs, flags).run()
    _check(specs, jobs, want, hosts)


def test_c4_shape_full():
    """256 instances, N = 2^(10..16), 1..40 limbs from a 64-prime pool of 30..60 bits;
    forward then inverse in two ragged batches; every limb-row of the forward
    against the oracle and the round trip checked in full."""
    inst = synth.c4_instances(0)
    plans, tens, hosts = [], [], []
    for i, it in enumerate(inst):
        p = ntt.Plan(it.N, it.moduli, 64)
        h = synth.uniform_poly(5000 + i, it.moduli, 1, it.N)
        plans.append(p)
        hosts.append(h)
        tens.append(to_device(h, 64))
    fwd = ntt.RaggedBatch([(p, ntt.OP_FORWARD, t) for p, t in zip(plans, tens)])
    inv = ntt.RaggedBatch([(p, ntt.OP_INVERSE, t) for p, t in zip(plans, tens)])
    fwd.run()
    torch.cuda.synchronize()
    # every limb-row of every instance against the oracle's forward transform
    for i, it in enumerate(inst):
        got = to_host(tens[i], 64)
        assert np.array_equal(got, oracle.forward(hosts[i], it.moduli)), (i, it.N)
    inv.run()
    torch.cuda.synchronize()
    for t, h in zip(tens, hosts):
        assert np.array_equal(to_host(t, 64), h)


def test_tuner_records_and_uses_a_valid_split(tmp_path):
    ntt.tune_clear()
    mods = Q50[:2]
    N = 1 << 15
    best, us = ntt.tune_split(N, mods, 64, 4)
    assert us > 0
    plan = ntt.Plan(N, mods, 64)
    assert plan.split_for(4) == best
    a = synth.uniform_poly(9, mods, 4, N)
    d = to_device(a, 64)
    plan.forward(d)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(d, 64), oracle.forward(a, mods))
    path = str(tmp_path / "tune.json")
    ntt.tune_save(path)
    import json
    kinds = {e["kind"]: e["value"] for e in json.load(open(path))["entries"]}
    assert kinds[0] == best and kinds[2] in (2, 3, 4) and kinds[3] in (2, 3, 4)
    if best > 0:  # a column pass: its workgroup size was measured too
        assert kinds[5] in (64, 128, 256)
    ntt.tune_clear()
    assert plan.split_for(4) == plan.split
    ntt.tune_load(path)
    assert plan.split_for(4) == best
    row_log, us2 = ntt.tune_ragged(1 << 16, Q50[:2], 2)
    assert row_log in (11, 12) and us2 > 0
    ntt.tune_clear()
