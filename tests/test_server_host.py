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


def test_same_shape_requests_share_launches_and_shapes_never_mix():
    with ntt.Server(1 << 32, n_streams=1, max_batch=4096, flags=ntt.SERVER_DRY_RUN) as srv:
        shapes = {}
        ids = []
        for i in range(200):
            if i % 10 == 0:
                rid = _big(srv, 8 + (i // 10) % 2)           # two different big shapes
                shapes[rid] = ("big", 8 + (i // 10) % 2)
            else:
                rid = _small(srv, 1 + i % 7)
                shapes[rid] = ("small", 0)
            ids.append(rid)
        infos = {i: srv.wait(i, 10000) for i in ids}
        c = srv.counters()
    assert c["launches"] < 200
    assert max(x["batched_with"] for x in infos.values()) > 1
    by_launch = {}
    for rid, x in infos.items():
        by_launch.setdefault(x["launch_id"], set()).add(shapes[rid])
    assert all(len(s) == 1 for s in by_launch.values())


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
