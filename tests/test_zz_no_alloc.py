"""bkd_query_async_noalloc (the library's fixed device workspace) against bkd_query_async.

Two calls in a row on the same tree, the second with fewer queries (and another k), so
the second call runs in a workspace that still holds the first call's contents; both
must equal bkd_query_async's outputs bit for bit, for the lock-step and the Algorithm 1
schedules.  A query whose workspace exceeds the fixed size is refused before any launch.
"""
from __future__ import annotations

import ctypes
import sys

import numpy as np
import pytest

import datagen
import paper_1512_02831_amd as bkd

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run(fn, tree, dQ, k):
    import torch
    m = dQ.shape[0]
    di = torch.full((m, k), -7, dtype=torch.int64, device="cuda")
    dd = torch.full((m, k), -7.0, dtype=torch.float32, device="cuda")
    s = torch.cuda.Stream()
    rc = fn(tree.handle, dQ.data_ptr(), m, k, di.data_ptr(), dd.data_ptr(), ctypes.c_void_p(s.cuda_stream))
    assert rc == bkd.OK, bkd.lib().bkd_last_error()
    s.synchronize()
    return di.cpu().numpy(), dd.cpu().numpy()


@pytest.mark.parametrize("schedule", ["lockstep", "algorithm1"])
def test_noalloc_matches_query_async(schedule):
    import torch
    say(f"case: no-alloc entry point, {schedule}, two calls (m 20000 then 3000)")
    P, Q = datagen.mixture_pq(seed=77, n=200_000, m=20_000, d=10, comps=16)
    opts = dict(fetch_size=-1, buffer_size=-1) if schedule == "lockstep" else dict(buffer_size=512, fetch_size=4096)
    L = bkd.lib()
    with bkd.build(P, 9, flags=bkd.FLAG_SQUARED, **opts) as t:
        for m, k in ((20_000, 10), (3000, 5)):
            dQ = torch.from_numpy(np.ascontiguousarray(Q[:m])).to("cuda")
            ref = run(L.bkd_query_async, t, dQ, k)
            got = run(L.bkd_query_async_noalloc, t, dQ, k)
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), (m, k)
            assert np.all(got[0] >= 0)


def test_noalloc_refuses_oversized_and_streamed():
    import torch
    say("case: no-alloc entry point refuses a workspace beyond its size and a streamed tree")
    P, Q = datagen.mixture_pq(seed=78, n=20_000, m=1, d=10, comps=4)
    L = bkd.lib()
    with bkd.build(P, 5, fetch_size=-1, buffer_size=-1) as t:
        m, k = 200_000, 64  # 64 keys of 8 bytes per query: more than 64 MiB in all
        dQ = torch.zeros((m, 10), dtype=torch.float32, device="cuda")
        di = torch.empty((m, k), dtype=torch.int64, device="cuda")
        dd = torch.empty((m, k), dtype=torch.float32, device="cuda")
        rc = L.bkd_query_async_noalloc(t.handle, dQ.data_ptr(), m, k, di.data_ptr(), dd.data_ptr(), None)
        assert rc == bkd.EINVAL and b"workspace" in L.bkd_last_error()
    with bkd.build(P, 5, fetch_size=-1, buffer_size=-1, num_chunks=2) as t:
        dQ = torch.zeros((10, 10), dtype=torch.float32, device="cuda")
        di = torch.empty((10, 3), dtype=torch.int64, device="cuda")
        dd = torch.empty((10, 3), dtype=torch.float32, device="cuda")
        rc = L.bkd_query_async_noalloc(t.handle, dQ.data_ptr(), 10, 3, di.data_ptr(), dd.data_ptr(), None)
        assert rc == bkd.EINVAL and b"resident" in L.bkd_last_error()
