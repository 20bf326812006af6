"""Served form: continuous batching over resident trees.  Every request's keys equal the
oracle's exhaustive float32-contract search (bit-exact) and the same query answered alone,
whatever else is in flight; admission respects the slot budget; waiting requests can be
cancelled; the server keeps a request's arrays until it is released."""
from __future__ import annotations

import sys
import threading
import time

import numpy as np
import pytest

import datagen
import oracle
import paper_1512_02831_amd as bkd

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def keys_of(idx, d2):
    """(float32 squared distance bits << 32) | index, the order the oracle's lists use."""
    return (d2.view(np.uint32).astype(np.uint64) << np.uint64(32)) | idx.astype(np.uint64)


def trees():
    PA, _ = datagen.mixture_pq(seed=31, n=40_000, m=1, d=10, comps=16)
    PB, _ = datagen.mixture_pq(seed=32, n=12_000, m=1, d=15, comps=16)
    return (PA, 7), (PB, 5)


@pytest.mark.parametrize("hA", [7, 4])  # h = 4: leaves of 2500 points, 512-lane tail workgroups
def test_requests_same_alone_and_in_the_mix(hA):
    say(f"case: 80 requests, two trees (hA={hA}), mixed k, two submitting threads")
    (PA, _), (PB, hB) = trees()
    ta = bkd.build(PA, hA, flags=bkd.FLAG_SQUARED)
    tb = bkd.build(PB, hB, flags=bkd.FLAG_SQUARED)
    rng = np.random.default_rng(5)
    reqs = []
    for i in range(80):
        tree = int(rng.integers(0, 2))
        m = int(np.floor(2 ** rng.uniform(0, 11.5)))
        k = int(rng.choice([1, 10, 32]))
        P = PA if tree == 0 else PB
        comps = 16
        _, Q = datagen.mixture_pq(seed=31 + tree, n=1, m=m, d=P.shape[1], comps=comps)
        Q = Q + np.float32(rng.normal(0, 0.01))  # distinct queries per request
        reqs.append((tree, Q.astype(np.float32), k))
    # requests of 3000-6000 queries on the d = 15 tree (32 leaves): rounds with more than
    # 2048 pending queries and buffers of more than 32, so the two-step (d + 2 = 17
    # products) matrix-core filter runs inside the session
    for i in range(3):
        _, Q = datagen.mixture_pq(seed=60 + i, n=1, m=3000 * (i + 1), d=15, comps=16)
        reqs.insert(10 * i + 3, (1, Q, [10, 32, 1][i]))
    with bkd.server_create(flags=bkd.FLAG_SQUARED) as srv:
        ida = bkd.server_add_tree(srv, ta)
        idb = bkd.server_add_tree(srv, tb)
        handles = [None] * len(reqs)

        def feed(part):
            for i in part:
                tree, Q, k = reqs[i]
                handles[i] = bkd.submit(srv, ida if tree == 0 else idb, Q, k)
                time.sleep(0.001 * ((i * 7919) % 3))

        th = [threading.Thread(target=feed, args=(range(j, len(reqs), 2),)) for j in range(2)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        for h in handles:
            bkd.wait(srv, h, 60_000_000)
            assert bkd.poll(srv, h) == bkd.REQ_DONE
        for i, ((tree, Q, k), h) in enumerate(zip(reqs, handles)):
            t = ta if tree == 0 else tb
            ref = oracle.brute_f32c(PA if tree == 0 else PB, Q, k)
            assert np.array_equal(keys_of(h.idx, h.dist), ref), f"request {i}: m={len(Q)} k={k} tree={tree}"
            idx, d2 = bkd.query(t, Q, k)
            assert np.array_equal(idx, h.idx) and np.array_equal(d2, h.dist)
            s, a, d = bkd.request_times(srv, h)
            assert s <= a <= d
    ta.free()
    tb.free()


def test_admission_by_slots_and_cancel():
    say("case: slot budget and cancel")
    (PA, hA), _ = trees()
    ta = bkd.build(PA, hA, flags=bkd.FLAG_SQUARED)
    _, Q = datagen.mixture_pq(seed=40, n=1, m=450, d=10, comps=16)
    want = oracle.brute_f32c(PA, Q, 10)
    with bkd.server_create(slots_per_session=500, flags=bkd.FLAG_SQUARED) as srv:
        tid = bkd.server_add_tree(srv, ta)
        with pytest.raises(bkd.BkdError) as e:
            bkd.submit(srv, tid, np.zeros((501, 10), np.float32), 10)
        assert e.value.code == bkd.EBUSY
        hs = [bkd.submit(srv, tid, Q, 10) for _ in range(6)]  # only one fits at a time
        bkd.cancel(srv, hs[-1])
        for h in hs[:-1]:
            bkd.wait(srv, h, 60_000_000)
        bkd.wait(srv, hs[-1], 60_000_000)
        assert bkd.poll(srv, hs[-1]) == bkd.REQ_CANCELLED
        for h in hs[:-1]:
            assert np.array_equal(keys_of(h.idx, h.dist), want)
        times = [bkd.request_times(srv, h) for h in hs[:-1]]
        for (s0, a0, d0), (s1, a1, d1) in zip(times, times[1:]):
            assert a1 >= d0 - 1e-3  # admitted after the previous one released its slots
        with pytest.raises(bkd.BkdError) as e:
            bkd.submit(srv, 7, Q, 10)
        assert e.value.code == bkd.ENOTFOUND
    ta.free()


def test_dropped_handles_are_kept_until_release():
    say("case: request handles dropped before completion, waited for by id")
    import gc
    (PA, hA), _ = trees()
    ta = bkd.build(PA, hA, flags=bkd.FLAG_SQUARED)
    _, Q = datagen.mixture_pq(seed=41, n=1, m=3000, d=10, comps=16)
    want = oracle.brute_f32c(PA, Q, 10)
    with bkd.server_create(flags=bkd.FLAG_SQUARED) as srv:
        tid = bkd.server_add_tree(srv, ta)
        ids = [bkd.submit(srv, tid, Q, 10).id for _ in range(4)]
        bkd.cancel(srv, ids[3])  # cancelled, possibly while running: still written at completion
        gc.collect()  # no handle is referenced by the caller any more
        for rid in ids:
            bkd.wait(srv, rid, 60_000_000)
        for rid in ids[:3]:
            idx, d2 = bkd.wait(srv, rid)
            assert np.array_equal(keys_of(idx, d2), want)
        for rid in ids:
            bkd.release(srv, rid)
        assert not srv.requests
        with pytest.raises(bkd.BkdError) as e:
            bkd.poll(srv, ids[0])
        assert e.value.code == bkd.ENOTFOUND
    ta.free()


# straggle_max 3000: the 3000-query request leaves the rounds at its first routing, the others
# once 3000 of theirs are left, so hand-overs are certain; with 64 they depend on how the
# traversal lengths spread on these small trees, and only the results are checked
@pytest.mark.parametrize("age_max,straggle_max", [(1, 0), (4, 0), (0, 3000), (0, 64), (8, 64)])
def test_aged_queries_leave_the_rounds(age_max, straggle_max):
    say(f"case: served age_max={age_max} straggle_max={straggle_max}: walks handed from the rounds to single walks")
    (PA, hA), (PB, hB) = trees()
    ta = bkd.build(PA, hA, flags=bkd.FLAG_SQUARED)
    tb = bkd.build(PB, hB, flags=bkd.FLAG_SQUARED)
    reqs = []
    for i, (P, m, k) in enumerate(((PA, 5000, 10), (PB, 4000, 32), (PA, 3000, 1), (PB, 100, 10))):
        _, Q = datagen.mixture_pq(seed=70 + i, n=1, m=m, d=P.shape[1], comps=16)
        reqs.append((P, Q, k))
    # tail_max=-1: the rounds never hand the whole remainder to the tail, so these few
    # thousand queries stay in the rounds long enough to age
    with bkd.server_create(flags=bkd.FLAG_SQUARED, age_max=age_max, tail_max=-1, straggle_max=straggle_max) as srv:
        ids = [bkd.server_add_tree(srv, t) for t in (ta, tb)]
        hs = [bkd.submit(srv, ids[0] if P is PA else ids[1], Q, k) for P, Q, k in reqs]
        for (P, Q, k), h in zip(reqs, hs):
            idx, d2 = bkd.wait(srv, h, 60_000_000)
            assert np.array_equal(keys_of(idx, d2), oracle.brute_f32c(P, Q, k)), (len(Q), k)
        st = bkd.server_stats(srv)
    if age_max > 0 or straggle_max >= 3000:
        assert st["aged_queries"] > 0
    ta.free()
    tb.free()
