"""Pins of the oracle's variant tree (Section 2.3): the footnote's longest-side splitting rule
and bounding-box pruning in the search phase.

What fixes the expected values, none of it the oracle itself:
  * a hand-worked example (tests/golden/variant_tree_2d.json) where the longest side picks
    another dimension than the level rule and the box term prunes a leaf the plane term visits;
  * independent pure-Python recursions (exact rational float32 emulation) of the build, the
    boxes and the depth-first search;
  * the box lemma checked with exact rationals: the box term never exceeds the float32
    distance of a point inside the box, and is never below the plane term of the far side;
  * exhaustive search: with either rule and either bound the keys equal the exhaustive
    float32 keys, on mixtures and on integer lattices (ties);
  * the box walk visits a subsequence of the plane walk's leaves.
"""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

import datagen
import oracle
from tests import exact_ref as X

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "variant_tree_2d.json")


def test_hand_worked_variant_example():
    g = json.load(open(GOLDEN))
    P = np.array(g["points"], dtype=np.float32)
    h = g["height"]
    t = oracle.build_tree_rules(P, h, oracle.SPLIT_LONGEST)
    assert t.split.tolist() == g["longest"]["split"]
    assert t.dims.tolist() == g["longest"]["dims"]
    assert t.leaf_off.tolist() == g["longest"]["leaf_off"]
    assert t.perm.tolist() == g["longest"]["perm"]
    c = oracle.build_tree_rules(P, h, oracle.SPLIT_CYCLIC)
    assert c.split.tolist() == g["cyclic"]["split"] and c.dims.tolist() == g["cyclic"]["dims"]
    boxes = oracle.node_boxes(P, t)
    assert boxes.tolist() == g["boxes_longest"]
    q = np.array(g["query"], dtype=np.float32)
    lv_plane, keys_plane = oracle.traverse_f32_rules(P, t, q, g["k"])
    lv_box, keys_box = oracle.traverse_f32_rules(P, t, q, g["k"], boxes=boxes)
    assert lv_plane.tolist() == g["plane_leaves"] and lv_box.tolist() == g["box_leaves"]
    for keys in (keys_plane, keys_box):
        d2, idx = oracle.keys_split(keys)
        assert idx.tolist() == g["idx"] and d2.tolist() == g["d2"]


def anisotropic(seed, n, d, dup=False):
    rng = np.random.default_rng(seed)
    scale = 2.0 ** rng.integers(-3, 4, size=d)
    P = (rng.standard_normal((n, d)) * scale).astype(np.float32)
    if dup:
        P[::4, 0] = P[0, 0]
        P[1::5] = P[2]
    return P


@pytest.mark.parametrize("rule", [oracle.SPLIT_CYCLIC, oracle.SPLIT_LONGEST])
def test_build_rules_match_python_recursion(rule):
    for seed, n, d, h, dup in ((1, 37, 3, 3, False), (2, 64, 2, 6, True), (3, 100, 5, 4, True), (4, 90, 7, 3, False)):
        P = anisotropic(seed, n, d, dup)
        t = oracle.build_tree_rules(P, h, rule)
        split, dims, leaves = X.build_rules_py(P, h, rule)
        assert list(t.split) == [np.float32(s) for s in split]
        assert list(t.dims) == dims
        assert list(t.perm) == [i for lf in leaves for i in lf]
        assert list(np.diff(t.leaf_off)) == [len(lf) for lf in leaves]
        boxes = oracle.node_boxes(P, t)
        ref = X.boxes_py(P, h, leaves)
        for v, (lo, hi) in enumerate(ref):
            assert boxes[v, 0].tolist() == lo and boxes[v, 1].tolist() == hi


def test_cyclic_rule_is_the_original_build():
    P, _ = datagen.mixture_pq(seed=5, n=5000, m=1, d=6, comps=8)
    a = oracle.build_tree(P, 7)
    b = oracle.build_tree_rules(P, 7, oracle.SPLIT_CYCLIC)
    assert np.array_equal(a.split.view(np.uint32), b.split.view(np.uint32))
    assert np.array_equal(a.perm, b.perm) and np.array_equal(a.leaf_off, b.leaf_off)
    assert b.dims.tolist() == [int(np.floor(np.log2(v + 1))) % 6 for v in range(127)]


def test_longest_side_invariants():
    P = anisotropic(9, 20_000, 6)
    h = 7
    t = oracle.build_tree_rules(P, h, oracle.SPLIT_LONGEST)
    boxes = oracle.node_boxes(P, t)
    first = (1 << h) - 1
    for v in range(first):
        lo, hi = boxes[v]
        sides = (hi - lo).astype(np.float32)
        assert t.dims[v] == int(np.argmax(sides))  # argmax takes the first maximum
        # every point below the left child is <= the split value, below the right child >=
        lchild, rchild = boxes[2 * v + 1], boxes[2 * v + 2]
        assert lchild[1, t.dims[v]] <= t.split[v] <= rchild[0, t.dims[v]]
    # boxes contain their points
    for lf in range(1 << h):
        pts = P[t.perm[t.leaf_off[lf]:t.leaf_off[lf + 1]]]
        assert np.all(pts >= boxes[first + lf, 0]) and np.all(pts <= boxes[first + lf, 1])


def test_box_term_bounds_every_point_and_the_plane():
    """Box lemma, exact rationals: for every far child, its box term is <= the float32 distance
    of each of its points and >= the plane term of its parent's split."""
    P = anisotropic(11, 300, 4)
    Q = anisotropic(12, 20, 4) * np.float32(1.5)
    h = 4
    split, dims, leaves = X.build_rules_py(P, h, 1)
    boxes = X.boxes_py(P, h, leaves)
    first = (1 << h) - 1

    def points_below(v):
        if v >= first:
            return leaves[v - first]
        return points_below(2 * v + 1) + points_below(2 * v + 2)

    checked = 0
    for q in Q:
        for v in range(first):
            dim = dims[v]
            far = 2 * v + 2 if float(q[dim]) < split[v] else 2 * v + 1
            b = X.box2_f32_exact(q, *boxes[far])
            assert b >= X.plane2_f32_exact(q[dim], split[v])
            for i in points_below(far):
                assert b <= X.dist2_f32_exact(q, P[i])
                checked += 1
    assert checked > 10_000


@pytest.mark.parametrize("rule,use_box", [(0, True), (1, False), (1, True)])
def test_rules_traversal_matches_python_search(rule, use_box):
    P = anisotropic(21, 120, 3, dup=True)
    Q = anisotropic(22, 10, 3)
    for h in (0, 2, 4):
        t = oracle.build_tree_rules(P, h, rule)
        split, dims, leaves = X.build_rules_py(P, h, rule)
        boxes = oracle.node_boxes(P, t) if use_box else None
        pyboxes = X.boxes_py(P, h, leaves) if use_box else None
        for k in (1, 5):
            for q in Q:
                order, best = X.search_rules_py(P, split, dims, leaves, h, q, k, pyboxes)
                lv, keys = oracle.traverse_f32_rules(P, t, q, k, boxes=boxes)
                assert list(lv) == order
                d2, idx = oracle.keys_split(keys)
                assert list(idx) == [i for _, i in best]
                assert [X.f32_bits(float(v)) for v in d2] == [X.f32_bits(v) for v, _ in best]


@pytest.mark.parametrize("kind", ["mixture", "lattice"])
def test_rules_give_the_exhaustive_keys(kind):
    if kind == "mixture":
        P, Q = datagen.mixture_pq(seed=31, n=20_000, m=300, d=8, comps=8)
    else:
        P = datagen.lattice(32, 1, 6000, 4, side=6)
        Q = datagen.lattice(32, 2, 200, 4, side=6)
    for k in (1, 7, 16):
        ref = oracle.brute_f32c(P, Q, k)
        for rule in (oracle.SPLIT_CYCLIC, oracle.SPLIT_LONGEST):
            t = oracle.build_tree_rules(P, 7, rule)
            boxes = oracle.node_boxes(P, t)
            for bx in (None, boxes):
                keys, _ = oracle.traverse_many_f32_rules(P, t, Q, k, boxes=bx)
                assert np.array_equal(keys, ref), (kind, k, rule, bx is not None)


def test_box_walk_is_a_subsequence_of_the_plane_walk():
    """A pruned subtree holds no point below the current k-th distance, so both walks keep the
    same list at every step and the box walk skips only leaves the plane walk gains nothing from."""
    P, Q = datagen.mixture_pq(seed=41, n=30_000, m=60, d=6, comps=8)
    t = oracle.build_tree_rules(P, 8, oracle.SPLIT_LONGEST)
    boxes = oracle.node_boxes(P, t)
    fewer = 0
    for q in Q:
        plane, kp = oracle.traverse_f32_rules(P, t, q, 10)
        box, kb = oracle.traverse_f32_rules(P, t, q, 10, boxes=boxes)
        assert np.array_equal(kp, kb)
        it = iter(plane.tolist())
        assert all(any(x == y for y in it) for x in box.tolist())
        fewer += len(box) < len(plane)
    assert fewer > 0
