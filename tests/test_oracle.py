"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: exact rational arithmetic,
integer lattices (every float operation exact), the d = 1 closed form, the
Q = P special case, a hand-worked example from the paper's rules, the error
bound of the float32 distance, and independent pure-Python implementations of
the tree, the search and the Algorithm 1 schedule.
"""
from __future__ import annotations

import json
import math
import os
from collections import deque
from fractions import Fraction

import numpy as np
import pytest

import datagen
import oracle
from tests import exact_ref as X

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# --------------------------------------------------------------------------
# float32 distance reading

def test_fmaf_chain_matches_exact_rounding():
    rng = np.random.default_rng(7)
    for d in (1, 2, 3, 5, 10):
        P = (rng.standard_normal((40, d)) * rng.choice([1e-3, 1.0, 1e3], size=(40, 1))).astype(np.float32)
        Q = (rng.standard_normal((3, d)) * 2).astype(np.float32)
        keys = oracle.brute_f32c(P, Q, 40)
        d2, idx = oracle.keys_split(keys)
        for qi in range(3):
            for r in range(40):
                want = X.dist2_f32_exact(Q[qi], P[idx[qi, r]])
                assert X.f32_bits(want) == int(np.float32(d2[qi, r]).view(np.uint32)), (d, qi, r)


def test_f32_distance_within_error_bound():
    # |fl32 chain - exact| <= ((1+u)^(d+2) - 1) * exact, u = 2^-24 (monotone rounding of non-negative terms)
    rng = np.random.default_rng(11)
    u = 2.0 ** -24
    for d in (3, 10, 15, 30):
        P = rng.standard_normal((200, d)).astype(np.float32)
        Q = rng.standard_normal((5, d)).astype(np.float32)
        keys = oracle.brute_f32c(P, Q, 200)
        d2, idx = oracle.keys_split(keys)
        bound = (1 + u) ** (d + 2) - 1
        for qi in range(5):
            for r in range(0, 200, 17):
                ex = X.dist2_exact(Q[qi], P[idx[qi, r]])
                err = abs(Fraction(float(d2[qi, r])) - ex)
                assert err <= Fraction(bound) * ex


def test_plane_term_never_exceeds_far_side_distance():
    # Pruning lemma: for every point on the far side of a splitting hyperplane, the float32 plane term
    # (q[dim]-s)^2 is <= the float32 squared distance, so pruning never drops a closer point.
    P, Q = datagen.mixture_pq(seed=3, n=2000, m=50, d=6, comps=4)
    h = 5
    t = oracle.build_tree(P, h)
    keys = oracle.brute_f32c(P, Q, P.shape[0])
    d2, idx = oracle.keys_split(keys)
    dmap = np.empty((Q.shape[0], P.shape[0]), dtype=np.float32)
    for qi in range(Q.shape[0]):
        dmap[qi, idx[qi]] = d2[qi]
    nleaf = 1 << h
    # points of each subtree: union of its leaves
    for v in range(nleaf - 1):
        level = int(math.floor(math.log2(v + 1)))
        dim = level % P.shape[1]
        s = t.split[v]

        def subtree_points(u):
            lo = u
            while lo < nleaf - 1:
                lo = 2 * lo + 1
            hi = u
            while hi < nleaf - 1:
                hi = 2 * hi + 2
            a, b = lo - (nleaf - 1), hi - (nleaf - 1)
            return t.perm[t.leaf_off[a]: t.leaf_off[b + 1]]

        left, right = subtree_points(2 * v + 1), subtree_points(2 * v + 2)
        for qi in range(Q.shape[0]):
            q = Q[qi]
            far = right if q[dim] < s else left
            tt = np.float32(q[dim]) - np.float32(s)
            h2 = np.float32(tt * tt)
            assert np.all(h2 <= dmap[qi, far])


# --------------------------------------------------------------------------
# exhaustive search

def test_brute_f64_matches_exact_rationals():
    rng = np.random.default_rng(5)
    P = rng.standard_normal((60, 3)).astype(np.float32)
    Q = rng.standard_normal((12, 3)).astype(np.float32)
    k = 6
    idx, d2 = oracle.brute_f64(P, Q, k)
    ref = X.knn_exact(P, Q, k)
    for qi in range(len(Q)):
        assert [i for _, i in ref[qi]] == list(idx[qi])
        for r in range(k):
            assert abs(d2[qi, r] - float(ref[qi][r][0])) <= 1e-15 * float(ref[qi][r][0])


def test_lattice_every_method_exact_with_ties():
    # Integer coordinates: all float32/float64 arithmetic is exact, ties are frequent and
    # the answer (ties by smaller index) is fixed by integer arithmetic.
    P = datagen.lattice(1, 1, 400, 4, side=6)
    Q = datagen.lattice(1, 2, 60, 4, side=6)
    k = 9
    exact = []
    for q in Q.astype(np.int64):
        dd = ((P.astype(np.int64) - q) ** 2).sum(axis=1)
        order = np.lexsort((np.arange(len(P)), dd))[:k]
        exact.append((order, dd[order]))
    idx64, d64 = oracle.brute_f64(P, Q, k)
    keys = oracle.brute_f32c(P, Q, k)
    d32, i32 = oracle.keys_split(keys)
    kidx, kd2 = oracle.kdtree_f64(P, Q, k, leaf_size=4)
    for h in (0, 3, 6):
        t = oracle.build_tree(P, h)
        rep = oracle.replay(P, t, Q, k, B=8, M=16)
        rd2, ri = oracle.keys_split(rep.keys)
        for qi in range(len(Q)):
            o, dd = exact[qi]
            assert list(ri[qi]) == list(o)
            assert list(rd2[qi]) == list(dd.astype(np.float32))
    for qi in range(len(Q)):
        o, dd = exact[qi]
        assert list(idx64[qi]) == list(o) and list(d64[qi]) == list(dd.astype(float))
        assert list(i32[qi]) == list(o) and list(d32[qi]) == list(dd.astype(np.float32))
        assert list(kidx[qi]) == list(o)


def test_d1_window_closed_form():
    # d = 1: the k nearest neighbours of q form a contiguous window of the sorted values.
    rng = np.random.default_rng(9)
    vals = rng.permutation(5000).astype(np.float32)[:800] * np.float32(0.5)
    P = vals.reshape(-1, 1)
    Q = (rng.random((40, 1)) * 2500).astype(np.float32)
    k = 7
    idx, _ = oracle.brute_f64(P, Q, k)
    order = np.argsort(vals, kind="stable")
    sv = vals[order]
    for qi, q in enumerate(Q[:, 0]):
        lo = int(np.searchsorted(sv, q))
        a, b = lo, lo  # window [a, b)
        while b - a < k:
            left = q - sv[a - 1] if a > 0 else math.inf
            right = sv[b] - q if b < len(sv) else math.inf
            if left <= right:
                a -= 1
            else:
                b += 1
        assert set(order[a:b]) == set(idx[qi])


def test_self_query_finds_itself():
    P = datagen.uniform(4, 1, 3000, 5)
    Q = P[::7]
    t = oracle.build_tree(P, 6)
    rep = oracle.replay(P, t, Q, 4, B=0, M=0, trace=False)
    d2, idx = oracle.keys_split(rep.keys)
    assert np.all(idx[:, 0] == np.arange(0, 3000, 7))
    assert np.all(d2[:, 0] == 0)


def test_hand_worked_example():
    g = _golden("tiny_knn_2d.json")
    P = np.array(g["P"], dtype=np.float32)
    t = oracle.build_tree(P, g["height"])
    assert list(t.split) == g["split"]
    assert list(t.leaf_off) == g["leaf_off"]
    assert list(t.perm) == g["perm"]
    q = np.array(g["query"], dtype=np.float32)
    leaves, keys = oracle.traverse_f32(P, t, q, g["k"])
    assert list(leaves) == g["leaf_sequence"]
    d2, idx = oracle.keys_split(keys)
    assert list(idx) == g["knn_idx"] and list(d2) == g["knn_d2"]
    rep = oracle.replay(P, t, q.reshape(1, -1), g["k"], B=2, M=1)
    assert np.array_equal(rep.keys[0], keys)


# --------------------------------------------------------------------------
# canonical build

def test_build_matches_python_recursion():
    for seed, n, d, h in ((1, 37, 3, 3), (2, 64, 2, 6), (3, 100, 5, 4), (4, 9, 1, 3)):
        P = datagen.uniform(seed, 1, n, d)
        P[::5, 0] = P[0, 0]  # duplicates in dimension 0
        t = oracle.build_tree(P, h)
        split, leaves = X.build_py(P, h)
        assert list(t.split) == [np.float32(s) for s in split]
        flat = [i for lf in leaves for i in lf]
        assert list(t.perm) == flat
        assert list(np.diff(t.leaf_off)) == [len(lf) for lf in leaves]


def test_build_invariants():
    P, _ = datagen.mixture_pq(seed=8, n=50_000, m=1, d=7, comps=16)
    h = 9
    t = oracle.build_tree(P, h)
    n = P.shape[0]
    assert np.array_equal(np.sort(t.perm), np.arange(n))
    sizes = np.diff(t.leaf_off)
    assert set(sizes.tolist()) <= {n >> h, -(-n >> h)}
    # every leaf is ascending in original index
    for a, b in zip(t.leaf_off[:-1], t.leaf_off[1:]):
        assert np.all(np.diff(t.perm[a:b]) > 0)
    # routing: descending with q = the point itself lands in its own leaf or, on equal values,
    # at or right of it; each subtree's points lie on the correct side of every ancestor split
    leaf_of = np.empty(n, dtype=np.int64)
    for lf in range(1 << h):
        leaf_of[t.perm[t.leaf_off[lf]:t.leaf_off[lf + 1]]] = lf
    for v in range(min((1 << h) - 1, 200)):
        level = int(math.floor(math.log2(v + 1)))
        dim = level % P.shape[1]
        span = 1 << (h - level)
        first = (v - ((1 << level) - 1)) * span
        left = np.isin(leaf_of, np.arange(first, first + span // 2))
        right = np.isin(leaf_of, np.arange(first + span // 2, first + span))
        assert np.all(P[left, dim] <= t.split[v])
        assert np.all(P[right, dim] >= t.split[v])


# --------------------------------------------------------------------------
# search: k-d tree, stackless traversal, Algorithm 1 replay

def test_kdtree_f64_equals_brute_f64():
    P, Q = datagen.mixture_pq(seed=2, n=4000, m=300, d=5, comps=8)
    for k in (1, 10, 33):
        i1, d1 = oracle.brute_f64(P, Q, k)
        i2, d2 = oracle.kdtree_f64(P, Q, k, leaf_size=16)
        assert np.array_equal(i1, i2) and np.array_equal(d1, d2)


def test_traversal_matches_recursive_search():
    P = datagen.uniform(12, 1, 96, 3)
    Q = datagen.uniform(12, 2, 8, 3)
    for h in (0, 2, 4):
        t = oracle.build_tree(P, h)
        split, leaves = X.build_py(P, h)
        for k in (1, 5):
            for q in Q:
                order, best = X.search_py(P, split, leaves, h, q, k)
                lv, keys = oracle.traverse_f32(P, t, q, k)
                assert list(lv) == order
                d2, idx = oracle.keys_split(keys)
                assert list(idx) == [i for _, i in best]
                assert [X.f32_bits(float(v)) for v in d2] == [X.f32_bits(v) for v, _ in best]


def _alg1_model(sequences, m, B, M):
    """Algorithm 1 in plain Python over fixed per-query leaf sequences.

    Each query's leaf sequence does not depend on the schedule, so FindLeafBatch
    is 'next leaf of the sequence, or -1'.  Returns the trace per call.
    """
    inp = deque(range(m))
    rein = deque()
    pos = [0] * m
    bufs = {}
    calls, cur = [], []
    half = (B + 1) // 2 if B > 0 else math.inf
    while inp or rein:
        fetched = []
        while len(fetched) < (M if M > 0 else math.inf) and rein:
            fetched.append(rein.popleft())
        while len(fetched) < (M if M > 0 else math.inf) and inp:
            fetched.append(inp.popleft())
        for i in fetched:
            seq = sequences[i]
            r = seq[pos[i]] if pos[i] < len(seq) else -1
            pos[i] += 1
            cur.append((i, r))
            if r != -1:
                bufs.setdefault(r, []).append(i)
        if any(len(b) >= half for b in bufs.values()) or (not inp and not rein):
            for leaf in sorted(bufs):
                rein.extend(bufs[leaf])
            bufs = {}
            calls.append(cur)
            cur = []
    return calls


@pytest.mark.parametrize("B,M", [(0, 0), (16, 40), (3, 7), (1, 1), (64, 0), (0, 25)])
def test_replay_schedule_matches_python_model(B, M):
    P, Q = datagen.mixture_pq(seed=6, n=3000, m=150, d=4, comps=4)
    h, k = 5, 6
    t = oracle.build_tree(P, h)
    seqs = [list(oracle.traverse_f32(P, t, q, k)[0]) for q in Q]
    rep = oracle.replay(P, t, Q, k, B=B, M=M)
    model = _alg1_model(seqs, len(Q), B, M)
    assert rep.ncalls == len(model)
    for c, trace in enumerate(model):
        q, r = rep.call(c)
        assert list(zip(q.tolist(), r.tolist())) == trace


def test_replay_results_schedule_invariant():
    P, Q = datagen.mixture_pq(seed=10, n=20_000, m=700, d=8, comps=16)
    k, h = 10, 7
    t = oracle.build_tree(P, h)
    ref = oracle.brute_f32c(P, Q, k)
    visits = None
    for B, M in ((1 << (24 - h), 10 << (24 - h)), (0, 0), (32, 50), (5, 3)):
        rep = oracle.replay(P, t, Q, k, B=B, M=M)
        assert np.array_equal(rep.keys, ref)
        pairs = sorted(zip(rep.trace_q.tolist(), rep.trace_r.tolist()))
        if visits is None:
            visits = pairs
        assert pairs == visits
    keys, nv, npairs = oracle.traverse_many_f32(P, t, Q, k)
    assert np.array_equal(keys, ref)
    assert rep.pairs == int(npairs.sum())


def test_chunk_bounds_golden_and_partition():
    for c in _golden("chunk_bounds.json")["cases"]:
        lo, hi = oracle.chunk_bounds(c["n"], c["N"])
        assert list(lo) == c["lo"] and list(hi) == c["hi"]
    for n in (1, 2, 17, 1000, 123457):
        for N in (1, 2, 3, 10, 64):
            if N > n:
                continue
            lo, hi = oracle.chunk_bounds(n, N)
            assert lo[0] == 0 and hi[-1] == n
            assert np.all(lo[1:] == hi[:-1]) and np.all(hi > lo)


def test_leaf_chunk_plan_golden_and_partition():
    for c in _golden("leaf_chunks.json")["cases"]:
        t = oracle.Tree(None, np.array(c["leaf_off"], dtype=np.int64), None, c["height"], c["d"])
        assert oracle.leaf_chunks(t, c["N"], c["cap_bytes"]).tolist() == c["first"], c["note"]
    P, _ = datagen.mixture_pq(seed=13, n=10_007, m=1, d=5, comps=4)
    t = oracle.build_tree(P, 6)
    bpp = 4 * 5 + 4
    for cap in (bpp * 400, bpp * 1000, bpp * 5000):
        first = oracle.leaf_chunks(t, 0, cap)
        assert first[0] == 0 and first[-1] == 64 and np.all(np.diff(first) > 0)
        sizes = (t.leaf_off[first[1:]] - t.leaf_off[first[:-1]]) * bpp
        assert np.all(sizes <= cap)
        # packing is greedy: no chunk could also hold the next chunk's first leaf
        nxt = (t.leaf_off[np.minimum(first[1:-1] + 1, 64)] - t.leaf_off[first[:-2]]) * bpp
        assert np.all(nxt > cap)
    for N in (1, 3, 7, 64, 100):
        first = oracle.leaf_chunks(t, N)
        assert len(first) == min(N, 64) + 1 and first[0] == 0 and first[-1] == 64 and np.all(np.diff(first) > 0)
