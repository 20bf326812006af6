"""Variant tree (Section 2.3) on the GPU: the longest-side splitting rule and bounding-box
pruning, through the C ABI, against the oracle.

Bars: the tree (split values, dimensions, leaf bounds, permutation, node boxes) bit-exact
with the oracle's variant build; every query's leaf sequence (from the trace) equal to the
oracle's walk under the same rules; keys bit-exact with the exhaustive float32 search, under
Algorithm 1, lock-step rounds with the tail, a streamed structure and the served form.
"""
from __future__ import annotations

import sys

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


def anisotropic_mixture(seed, n, m, d):
    """The mixture generator with each dimension scaled by its own power of two, so that the
    longest side of a node's box is often not the level's dimension."""
    P, Q = datagen.mixture_pq(seed=seed, n=n, m=m, d=d, comps=8)
    scale = (2.0 ** np.random.default_rng(seed).integers(-2, 3, size=d)).astype(np.float32)
    return (P * scale).astype(np.float32), (Q * scale).astype(np.float32)


def sequences(tr):
    off, q, leaf = tr
    seq = {}
    for qi, lf in zip(q.tolist(), leaf.tolist()):
        if lf >= 0:
            seq.setdefault(qi, []).append(lf)
    return seq


RULES = [(bkd.SPLIT_LONGEST, bkd.PRUNE_PLANE), (bkd.SPLIT_CYCLIC, bkd.PRUNE_BOX), (bkd.SPLIT_LONGEST, bkd.PRUNE_BOX)]


@pytest.mark.parametrize("rule,prune", RULES)
def test_variant_tree_and_walks_match_oracle(rule, prune):
    say(f"case: variant tree rule={rule} prune={prune}, Algorithm 1 with trace")
    P, Q = anisotropic_mixture(51, 60_000, 3000, 8)
    k, h = 10, 7
    with bkd.build(P, h, split_rule=rule, prune=prune, flags=bkd.FLAG_TRACE | bkd.FLAG_SQUARED,
                   buffer_size=2048, fetch_size=8192) as t:
        split, leaf_off, perm = bkd.tree_export(t)
        dims, boxes = bkd.tree_rules_export(t, boxes=prune == bkd.PRUNE_BOX)
        idx, d2 = bkd.query(t, Q, k)
        tr = bkd.trace(t)
        st = bkd.last_stats(t)
    t_or = oracle.build_tree_rules(P, h, rule)
    assert np.array_equal(split.view(np.uint32), t_or.split.view(np.uint32))
    assert np.array_equal(leaf_off, t_or.leaf_off) and np.array_equal(perm, t_or.perm)
    assert np.array_equal(dims, t_or.dims)
    ob = oracle.node_boxes(P, t_or) if prune == bkd.PRUNE_BOX else None
    if ob is not None:
        assert np.array_equal(boxes.view(np.uint32), ob.view(np.uint32))
    assert np.array_equal(keys_of(idx, d2), oracle.brute_f32c(P, Q, k))
    seq = sequences(tr)
    for qi in np.random.default_rng(0).choice(len(Q), 300, replace=False):
        lv, _ = oracle.traverse_f32_rules(P, t_or, Q[qi], k, boxes=ob)
        assert seq[int(qi)] == lv.tolist(), int(qi)
    _, visits = oracle.traverse_many_f32_rules(P, t_or, Q, k, boxes=ob)
    assert st["visits"] == int(visits.sum())


@pytest.mark.parametrize("chunks", [0, 3])
def test_variant_lockstep_tail_and_streamed(chunks):
    say(f"case: variant tree (longest side, boxes), lock-step rounds, chunks={chunks}")
    P, Q = anisotropic_mixture(52, 80_000, 20_000, 10)
    k, h = 10, 8
    ref = oracle.brute_f32c(P, Q, k)
    t_or = oracle.build_tree_rules(P, h, bkd.SPLIT_LONGEST)
    _, visits = oracle.traverse_many_f32_rules(P, t_or, Q, k, boxes=oracle.node_boxes(P, t_or))
    for tail_max in (0, 2048, -1):  # default tail, a later hand-over, rounds to the end
        with bkd.build(P, h, split_rule=bkd.SPLIT_LONGEST, prune=bkd.PRUNE_BOX, flags=bkd.FLAG_SQUARED,
                       fetch_size=-1, buffer_size=-1, num_chunks=chunks, tail_max=tail_max) as t:
            idx, d2 = bkd.query(t, Q, k)
            st = bkd.last_stats(t)
        assert np.array_equal(keys_of(idx, d2), ref), tail_max
        assert st["visits"] == int(visits.sum()), tail_max


def test_variant_served():
    say("case: variant tree (longest side, boxes) in the served form")
    P, Q = anisotropic_mixture(53, 50_000, 6000, 6)
    with bkd.build(P, 7, split_rule=bkd.SPLIT_LONGEST, prune=bkd.PRUNE_BOX, flags=bkd.FLAG_SQUARED) as t:
        with bkd.server_create(flags=bkd.FLAG_SQUARED) as srv:
            tid = bkd.server_add_tree(srv, t)
            parts = [(0, 5), (5, 900), (900, 6000)]  # direct path (small requests) and rounds
            hs = [bkd.submit(srv, tid, Q[a:b], k) for (a, b), k in zip(parts, (1, 10, 32))]
            for h_, (a, b), k in zip(hs, parts, (1, 10, 32)):
                idx, d2 = bkd.wait(srv, h_, 60_000_000)
                assert np.array_equal(keys_of(idx, d2), oracle.brute_f32c(P, Q[a:b], k))


def test_variant_options_rejected():
    say("case: variant tree option errors")
    P, _ = anisotropic_mixture(54, 2000, 1, 3)
    for kw in (dict(split_rule=2), dict(prune=-1),
               dict(split_rule=bkd.SPLIT_LONGEST, flags=bkd.FLAG_DEVICE_BUILD)):
        with pytest.raises(bkd.BkdError) as e:
            bkd.build(P, 4, **kw)
        assert e.value.code == bkd.EINVAL
    with bkd.build(P, 4) as t:
        dims, _ = bkd.tree_rules_export(t)
        assert dims.tolist() == [int(np.floor(np.log2(v + 1))) % 3 for v in range(15)]
        with pytest.raises(bkd.BkdError) as e:
            bkd.tree_rules_export(t, boxes=True)
        assert e.value.code == bkd.EINVAL
