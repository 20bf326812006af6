"""The bigger-than-budget workload at full size, checked against the oracle on a sample.

n = 2^28 reference points of the d = 10, 16-component mixture, height 14 (16384 leaves
of 16384 points), leaf structure streamed through a 2 GB device budget (12 leaf-aligned
chunks, Section 3.2), lock-step rounds with the chunk sweep, as the benchmark runs it.
The structure holds about 2.9e9 words, so leaf-block offsets pass 2^31.  4096 queries
drawn from the workload's query stream are answered and their keys compared bit-exactly
with the oracle's traversal of its own canonical tree (built from P alone).

The same reference set also serves as one leaf of 2^28 points (height 0, brute force,
resident): every scan kernel then addresses coordinate rows past 2^31 words inside a
single leaf (row j starts at word j * 2^28).  The tail path and, with the tail switched
off, the dense and sparse scans must return the same keys.

These are the slowest GPU tests (the oracle's build of 2^28 points takes about a minute
on the host); they run after the others.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import datagen
import oracle
import paper_1512_02831_amd as bkd

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

N, M, D, K, H = 1 << 28, 1 << 24, 10, 10, 14
BUDGET = 2_000_000_000
SAMPLE = 4096


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def f32_keys(idx, d2):
    return (d2.astype(np.float32).view(np.uint32).astype(np.uint64) << np.uint64(32)) | idx.astype(np.uint64)


@pytest.fixture(scope="module")
def workload():
    say(f"case: bigger-than-budget inputs n=2^28 m=2^24 d={D} (generating)")
    P, Q = datagen.mixture_pq(datagen.DEFAULT_SEED, N, M, D, 16)
    rng = np.random.default_rng(28)
    sample = np.sort(rng.choice(M, SAMPLE, replace=False))
    Qs = np.ascontiguousarray(Q[sample])
    del Q
    say("  oracle: canonical tree of 2^28 points, traversal of the sample")
    t_or = oracle.build_tree(P, H)
    okeys, _, _ = oracle.traverse_many_f32(P, t_or, Qs, K)
    return P, Qs, t_or, okeys


def test_bigger_than_budget_sampled_parity(workload):
    P, Qs, t_or, okeys = workload
    say("case: streamed n=2^28 h=14, 2 GB leaf budget, 4096 sampled queries")
    with bkd.build(P, H, fetch_size=-1, buffer_size=-1, leaf_budget_bytes=BUDGET,
                   flags=bkd.FLAG_SQUARED | bkd.FLAG_DEVICE_BUILD) as t:
        info = bkd.tree_info(t)
        assert not info.resident and info.num_chunks == 12
        assert info.leaf_bytes // 4 > 1 << 31
        split, leaf_off, _ = bkd.tree_export(t)
        assert np.array_equal(split.view(np.uint32), t_or.split.view(np.uint32))
        assert np.array_equal(leaf_off, t_or.leaf_off)
        idx, d2 = bkd.query(t, Qs, K)
        st = bkd.last_stats(t)
    say("  gpu done", st)
    assert st["chunk_copies"] > 0
    assert np.array_equal(f32_keys(idx, d2), okeys)


@pytest.mark.parametrize("flags", [0, bkd.FLAG_NO_TAIL])
def test_single_leaf_past_2p31_words(workload, flags):
    P, Qs, _, okeys = workload
    say(f"case: one resident leaf of 2^28 points (h=0), 64 queries, flags={flags}")
    with bkd.build(P, 0, fetch_size=-1, buffer_size=-1, flags=bkd.FLAG_SQUARED | flags) as t:
        idx, d2 = bkd.query(t, Qs[:64], K)
        st = bkd.last_stats(t)
    say("  gpu done", st)
    if flags & bkd.FLAG_NO_TAIL:
        assert st["dense_launches"] > 0  # 64 queries in one buffer: the dense scan
    assert np.array_equal(f32_keys(idx, d2), okeys[:64])
