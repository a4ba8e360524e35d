"""Admission and batching logic of the request server, on the CPU: the server's
dry-run executor models each launch's duration instead of touching a device."""
import threading

import pytest

import paper_2410_05934_amd as ntt
from paper_2410_05934_amd import synth

Q_SMALL = synth.c3_prime()
Q_BIG = synth.c2_primes(9)


def _small(srv, pairs=4):
    return srv.submit(ntt.REQ_POLYMUL, 1 << 10, [Q_SMALL], 32, pairs)


def _big(srv, L=8):
    return srv.submit(ntt.REQ_POLYMUL, 1 << 16, Q_BIG[:L], 64, 1)


def test_budget_is_never_exceeded_and_everything_completes():
    big_bytes = 4 * 8 * (1 << 16) * 8          # 4 buffers x 8 limbs x 2^16 x 8 B
    budget = 2 * big_bytes + 64 * 1024
    with ntt.Server(budget, n_streams=4, flags=ntt.SERVER_DRY_RUN) as srv:
        ids = []
        for i in range(60):
            ids.append(_big(srv) if i % 3 == 0 else _small(srv, 1 + i % 5))
        infos = [srv.wait(i, 10000) for i in ids]
        c = srv.counters()
    assert all(x["status"] == 0 for x in infos)
    assert c["completed"] == 60 and c["rejected"] == 0
    assert 0 < c["max_inflight_bytes"] <= budget
    for x in infos:
        assert x["t_submit"] <= x["t_admit"] <= x["t_launch"] <= x["t_done"]


def test_oversize_request_is_rejected():
    with ntt.Server(1 << 20, flags=ntt.SERVER_DRY_RUN) as srv:
        with pytest.raises(ntt.NTTError) as e:
            _big(srv, 8)
        assert e.value.name == "NTT_ENOMEM"
        assert srv.counters()["rejected"] == 1


def test_bad_requests_are_rejected():
    with ntt.Server(1 << 30, flags=ntt.SERVER_DRY_RUN) as srv:
        with pytest.raises(ntt.NTTError):
            srv.submit(ntt.REQ_POLYMUL, 1 << 10, [Q_SMALL + 2], 32, 1)     # composite
        with pytest.raises(ntt.NTTError):
            srv.submit(ntt.REQ_POLYMUL, 1000, [Q_SMALL], 32, 1)            # N not a power of two
        with pytest.raises(ntt.NTTError):
            srv.submit(7, 1 << 10, [Q_SMALL], 32, 1)                       # bad op


def _two_big_shapes_and_small(srv):
    shapes, ids = {}, []
    for i in range(200):
        if i % 10 == 0:
            rid = _big(srv, 8 + (i // 10) % 2)           # two different big shapes
            shapes[rid] = ("big", 8 + (i // 10) % 2)
        else:
            rid = _small(srv, 1 + i % 7)
            shapes[rid] = ("small", 0)
        ids.append(rid)
    return shapes, {i: srv.wait(i, 10000) for i in ids}


def _shapes_per_launch(shapes, infos):
    by_launch = {}
    for rid, x in infos.items():
        by_launch.setdefault(x["launch_id"], set()).add(shapes[rid])
    return by_launch


def test_same_shape_requests_share_launches_and_shapes_never_mix():
    with ntt.Server(1 << 32, n_streams=1, max_batch=4096, flags=ntt.SERVER_DRY_RUN) as srv:
        shapes, infos = _two_big_shapes_and_small(srv)
        c = srv.counters()
    assert c["launches"] < 200 and c["merged_launches"] == 0
    assert max(x["batched_with"] for x in infos.values()) > 1
    assert all(len(s) == 1 for s in _shapes_per_launch(shapes, infos).values())


def test_requests_of_different_moduli_in_one_class_share_launches():
    """With NTT_SERVER_MERGE_MODULI, big requests of 8 and of 9 limbs (same op, N,
    width and class) may share a launch; big and small requests (other N, other
    width) never do."""
    with ntt.Server(1 << 32, n_streams=1, max_batch=4096,
                    flags=ntt.SERVER_DRY_RUN | ntt.SERVER_MERGE_MODULI) as srv:
        shapes, infos = _two_big_shapes_and_small(srv)
        c = srv.counters()
    by_launch = _shapes_per_launch(shapes, infos)
    assert c["merged_launches"] >= 1
    assert any(s == {("big", 8), ("big", 9)} for s in by_launch.values())
    assert all(len({k for k, _ in s}) == 1 for s in by_launch.values())


def test_moduli_spanning_classes_only_batch_with_identical_moduli():
    """A request whose moduli fall in two arithmetic classes (one below 2^50,
    one above) runs only beside requests of exactly its moduli."""
    wide = synth.primes_below(1 << 61, 1 << 17, 2)
    mixed_cls = [Q_BIG[0], wide[0]]
    with ntt.Server(1 << 32, n_streams=1, flags=ntt.SERVER_DRY_RUN | ntt.SERVER_MERGE_MODULI) as srv:
        kinds, ids = {}, []
        for i in range(60):
            if i % 3 == 0:
                rid = srv.submit(ntt.REQ_POLYMUL, 1 << 16, mixed_cls, 64, 1)
                kinds[rid] = "two-class"
            else:
                L = 2 + i % 2
                rid = srv.submit(ntt.REQ_POLYMUL, 1 << 16, Q_BIG[:L], 64, 1)
                kinds[rid] = "fp64"
            ids.append(rid)
        infos = {i: srv.wait(i, 10000) for i in ids}
    by_launch = {}
    for rid, x in infos.items():
        by_launch.setdefault(x["launch_id"], set()).add(kinds[rid])
    assert all(len(s) == 1 for s in by_launch.values())
    assert any(x["batched_with"] > 1 for rid, x in infos.items() if kinds[rid] == "two-class")


def test_a_launch_of_different_moduli_holds_at_most_4096_limb_rows():
    """Requests of 9 limbs x 100 polynomials and of 8 limbs x 100 polynomials:
    a launch that mixes them stays within 4096 limb-rows."""
    with ntt.Server(1 << 40, n_streams=1, flags=ntt.SERVER_DRY_RUN | ntt.SERVER_MERGE_MODULI) as srv:
        limbs, ids = {}, []
        for i in range(40):
            L = 8 + i % 2
            rid = srv.submit(ntt.REQ_FORWARD, 1 << 10, Q_BIG[:L], 64, 100)
            limbs[rid] = (L, 100 * L)
            ids.append(rid)
        infos = {i: srv.wait(i, 10000) for i in ids}
        c = srv.counters()
    rows, kinds = {}, {}
    for rid, x in infos.items():
        rows[x["launch_id"]] = rows.get(x["launch_id"], 0) + limbs[rid][1]
        kinds.setdefault(x["launch_id"], set()).add(limbs[rid][0])
    assert c["merged_launches"] >= 1
    assert all(rows[k] <= 4096 for k in rows if len(kinds[k]) > 1)


def test_max_batch_caps_polynomials_per_launch():
    with ntt.Server(1 << 32, n_streams=1, max_batch=16, flags=ntt.SERVER_DRY_RUN) as srv:
        ids = [_small(srv, 4) for _ in range(40)]
        infos = [srv.wait(i, 10000) for i in ids]
    per_launch = {}
    for x in infos:
        per_launch[x["launch_id"]] = per_launch.get(x["launch_id"], 0) + 4
    assert max(per_launch.values()) <= 16


def test_serial_mode_is_one_at_a_time_in_order():
    with ntt.Server(1 << 32, n_streams=4, flags=ntt.SERVER_SERIAL | ntt.SERVER_DRY_RUN) as srv:
        ids = [_small(srv, 2) if i % 2 else _big(srv) for i in range(30)]
        infos = [srv.wait(i, 10000) for i in ids]
        c = srv.counters()
    assert all(x["batched_with"] == 1 for x in infos)
    assert c["max_inflight_requests"] == 1
    done = [x["t_done"] for x in infos]
    assert done == sorted(done)


def test_requests_arriving_during_flight_are_admitted_continuously():
    """Submit from another thread while launches are in flight: later arrivals
    join later launches rather than waiting for the whole queue to drain."""
    with ntt.Server(1 << 32, n_streams=2, flags=ntt.SERVER_DRY_RUN) as srv:
        ids = []
        lock = threading.Lock()

        def producer():
            for i in range(100):
                rid = _small(srv, 3)
                with lock:
                    ids.append(rid)

        t = threading.Thread(target=producer)
        t.start()
        t.join()
        infos = [srv.wait(i, 10000) for i in ids]
        c = srv.counters()
    assert c["completed"] == 100
    assert len({x["launch_id"] for x in infos}) >= 2


def test_replay_submits_at_the_given_times():
    arrivals = [i * 200e-6 for i in range(50)]
    reqs = [(ntt.REQ_POLYMUL, 1 << 10, [Q_SMALL], 32, 2, 0, 0, 0)] * 50
    with ntt.Server(1 << 32, n_streams=2, flags=ntt.SERVER_DRY_RUN) as srv:
        ids = srv.replay(reqs, arrivals)
        infos = [srv.wait(i, 10000) for i in ids]
    t = [x["t_submit"] for x in infos]
    span = t[-1] - t[0]
    assert 0.9 * arrivals[-1] <= span <= arrivals[-1] + 0.05
    assert all(b >= a for a, b in zip(t, t[1:]))


def test_a_launch_stays_below_2_to_32_words():
    """64 forward requests of 64 polynomials x 16 limbs x 2^16 (u32) fit the
    64 GB budget together but make exactly 2^32 words, the library's per-call
    limit: the server must split them over launches, so that every request
    succeeds as it would alone."""
    mods = synth.primes_below(1 << 32, 1 << 17, 16)
    words = 64 * 16 * (1 << 16)
    with ntt.Server(64 << 30, n_streams=1, flags=ntt.SERVER_DRY_RUN) as srv:
        ids = [srv.submit(ntt.REQ_FORWARD, 1 << 16, mods, 32, 64) for _ in range(64)]
        infos = [srv.wait(i, 60000) for i in ids]
    assert all(x["status"] == 0 for x in infos)
    per_launch = {}
    for x in infos:
        per_launch[x["launch_id"]] = per_launch.get(x["launch_id"], 0) + 1
    assert max(per_launch.values()) * words < (1 << 32)
    assert max(x["batched_with"] for x in infos) > 1


def test_request_of_2_to_32_words_is_rejected_at_submit():
    mods = synth.primes_below(1 << 32, 1 << 17, 16)
    with ntt.Server(1 << 40, flags=ntt.SERVER_DRY_RUN) as srv:
        with pytest.raises(ntt.NTTError) as e:
            srv.submit(ntt.REQ_FORWARD, 1 << 16, mods, 32, 4096)   # 2^12 x 2^4 x 2^16 words
        assert e.value.name == "NTT_EINVAL"
