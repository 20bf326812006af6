"""Disk-backed leaf structure (Section 3.2: the structure kept on disk when host memory is too
small, every chunk copied disk -> host -> device): a tree built with a leaf file and forced
into N chunks gives the resident run's results and the oracle's, under Algorithm 1 (per-call
buffer contents equal to the oracle's replay) and under lock-step rounds with the chunk sweep;
its chunk plan is the oracle's leaf-aligned plan; the file exists while the tree does."""
from __future__ import annotations

import os
import sys
import tempfile

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
    return (d2.view(np.uint32).astype(np.uint64) << np.uint64(32)) | idx.astype(np.uint64)


@pytest.mark.parametrize("N,mode,schedule", [(3, bkd.CHUNK_LEAF, "lockstep"), (5, bkd.CHUNK_LEAF, "algorithm1"),
                                             (4, bkd.CHUNK_POSITION, "lockstep"), (0, bkd.CHUNK_LEAF, "lockstep")])
def test_leaf_file_matches_resident_and_oracle(N, mode, schedule):
    say(f"case: leaf file, N={N} mode={mode} {schedule}")
    P, Q = datagen.mixture_pq(seed=61, n=200_003, m=6000, d=8, comps=8)
    k, h = 10, 7
    sched = dict(fetch_size=-1, buffer_size=-1) if schedule == "lockstep" else dict(buffer_size=4096, fetch_size=16384)
    flags = bkd.FLAG_SQUARED | (bkd.FLAG_TRACE if schedule == "algorithm1" else 0)
    with bkd.build(P, h, flags=bkd.FLAG_SQUARED, **sched) as t:
        ref_i, ref_d = bkd.query(t, Q, k)
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "leaves.bin")
        budget = 0 if N else 2 * 1_900_000  # N = 0: chunks packed up to a budget of two leaf buffers
        with bkd.build(P, h, flags=flags, chunk_mode=mode, num_chunks=N, leaf_budget_bytes=budget,
                       leaf_path=path, **sched) as t:
            info = bkd.tree_info(t)
            assert info.on_disk == 1 and not info.resident
            assert os.path.getsize(path) == (4 * 8 + 4) * len(P)
            if N:
                assert info.num_chunks == N
            lo = np.zeros(info.num_chunks, dtype=np.int64)
            hi = np.zeros(info.num_chunks, dtype=np.int64)
            bkd.lib().bkd_chunk_plan(t.handle, lo.ctypes.data, hi.ctypes.data)
            idx, d2 = bkd.query(t, Q, k)
            st = bkd.last_stats(t)
            tr = bkd.trace(t) if schedule == "algorithm1" else None
            idx2, d22 = bkd.query(t, Q[:500], k)  # a second call on the same file
        assert not os.path.exists(path)  # removed with the tree
    say("  stats", {key: st[key] for key in ("chunk_copies", "bytes_h2d", "bytes_disk", "disk_ms", "wait_ms")},
        "direct I/O" if info.direct_io else "buffered I/O")
    # a chunk still held by a staging buffer is copied again without a second read
    assert st["bytes_disk"] > 0 and st["bytes_h2d"] > 0
    assert np.array_equal(idx, ref_i) and np.array_equal(d2, ref_d)
    assert np.array_equal(idx2, ref_i[:500]) and np.array_equal(d22, ref_d[:500])
    t_or = oracle.build_tree(P, h)
    assert np.array_equal(keys_of(idx, d2), oracle.brute_f32c(P, Q, k))
    if mode == bkd.CHUNK_LEAF:
        first = oracle.leaf_chunks(t_or, N, 0 if N else budget // 2)
        assert lo.tolist() == t_or.leaf_off[first[:-1]].tolist()
        assert hi.tolist() == t_or.leaf_off[first[1:]].tolist()
    else:
        olo, ohi = oracle.chunk_bounds(len(P), N)
        assert lo.tolist() == olo.tolist() and hi.tolist() == ohi.tolist()
    if tr is not None:
        rep = oracle.replay(P, t_or, Q, k, B=4096, M=16384)
        off, q, leaf = tr
        assert np.array_equal(off, rep.call_off)
        assert np.array_equal(q, rep.trace_q) and np.array_equal(leaf, rep.trace_r)


def test_leaf_file_bad_path():
    say("case: leaf file in a missing directory")
    P, _ = datagen.mixture_pq(seed=62, n=5000, m=1, d=4, comps=4)
    with pytest.raises(bkd.BkdError) as e:
        bkd.build(P, 4, num_chunks=2, leaf_path="/nonexistent-dir/leaves.bin")
    assert e.value.code == bkd.EINVAL
