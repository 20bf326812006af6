"""Independent pure-Python references used to pin the oracle.

Nothing here calls the oracle or the HIP library.  The arithmetic is exact
(Python integers and fractions), so these functions are slow and only run on
tiny inputs.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def round_f32(x: Fraction) -> float:
    """Round an exact rational to the nearest float32 (ties to even), as a Python float."""
    if x == 0:
        return 0.0
    neg = x < 0
    a = -x if neg else x
    e = a.numerator.bit_length() - a.denominator.bit_length()
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    q = max(e - 23, -149)  # quantum of the float32 binade (or of the subnormals)
    scaled = a / (Fraction(2) ** q)
    n = scaled.numerator // scaled.denominator
    rem = scaled - n
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and n % 2 == 1):
        n += 1
    v = float(Fraction(n) * Fraction(2) ** q)  # exactly representable
    return -v if neg else v


def f32_bits(v: float) -> int:
    return int(np.array([v], dtype=np.float32).view(np.uint32)[0])


def dist2_f32_exact(q, x) -> float:
    """float32 squared distance: t = fl32(q_j - x_j); acc = fl32(t*t + acc), one rounding per step."""
    acc = Fraction(0)
    for qj, xj in zip(q, x):
        t = Fraction(round_f32(Fraction(float(qj)) - Fraction(float(xj))))
        acc = Fraction(round_f32(t * t + acc))
    return float(acc)


def plane2_f32_exact(qd: float, s: float) -> float:
    t = Fraction(round_f32(Fraction(float(qd)) - Fraction(float(s))))
    return round_f32(t * t)


def dist2_exact(q, x) -> Fraction:
    return sum((Fraction(float(a)) - Fraction(float(b))) ** 2 for a, b in zip(q, x))


def knn_exact(P, Q, k):
    """Exact kNN by rational arithmetic: list of index lists, ties by smaller index."""
    out = []
    for q in Q:
        d = [(dist2_exact(q, P[i]), i) for i in range(len(P))]
        d.sort()
        out.append(d[:k])
    return out


def build_py(P, h):
    """Recursive median split: rank floor(c/2) under (coordinate, index); leaves by index."""
    n, d = P.shape
    split = [0.0] * ((1 << h) - 1)
    leaves = [None] * (1 << h)

    def rec(v, level, idx):
        if level == h:
            leaves[v - ((1 << h) - 1)] = sorted(idx)
            return
        dim = level % d
        s = sorted(idx, key=lambda i: (float(P[i, dim]), i))
        c = len(s)
        split[v] = float(P[s[c // 2], dim])
        rec(2 * v + 1, level + 1, s[: c // 2])
        rec(2 * v + 2, level + 1, s[c // 2:])

    rec(0, 0, list(range(n)))
    return split, leaves


def search_py(P, split, leaves, h, q, k):
    """Recursive depth-first k-d search, near child first, float32 arithmetic emulated exactly.

    Returns (leaf visit order, final list of (d2 bits, index)).
    """
    d = P.shape[1]
    first = (1 << h) - 1
    best = []  # sorted list of (d2 float, idx)
    order = []

    def kth():
        return best[k - 1][0] if len(best) >= k else math.inf

    def visit(v, level):
        if v >= first:
            leaf = v - first
            order.append(leaf)
            for i in leaves[leaf]:
                best.append((dist2_f32_exact(q, P[i]), i))
            best.sort()
            del best[k:]
            return
        dim = level % d
        near, far = (2 * v + 1, 2 * v + 2) if float(q[dim]) < split[v] else (2 * v + 2, 2 * v + 1)
        visit(near, level + 1)
        if plane2_f32_exact(q[dim], split[v]) <= kth():
            visit(far, level + 1)

    visit(0, 0)
    return order, best


# --------------------------------------------------------------------------
# Variant tree: longest-side splits and bounding-box pruning (Section 2.3)

def side_f32(vals) -> float:
    """Longest-side measure of one dimension: fl32(max - min) of its float32 values."""
    return round_f32(Fraction(float(max(vals))) - Fraction(float(min(vals))))


def build_rules_py(P, h, rule):
    """Recursive median split with a splitting rule: 0 = level mod d, 1 = the dimension whose
    bounding-box side fl32(max - min) over the node's points is largest (smallest d on ties).
    Returns (split, dims, leaves)."""
    n, d = P.shape
    split = [0.0] * ((1 << h) - 1)
    dims = [0] * ((1 << h) - 1)
    leaves = [None] * (1 << h)

    def rec(v, level, idx):
        if level == h:
            leaves[v - ((1 << h) - 1)] = sorted(idx)
            return
        if rule == 0:
            dim = level % d
        else:
            sides = [side_f32([float(P[i, j]) for i in idx]) for j in range(d)]
            dim = max(range(d), key=lambda j: (sides[j], -j))
        dims[v] = dim
        s = sorted(idx, key=lambda i: (float(P[i, dim]), i))
        c = len(s)
        split[v] = float(P[s[c // 2], dim])
        rec(2 * v + 1, level + 1, s[: c // 2])
        rec(2 * v + 2, level + 1, s[c // 2:])

    rec(0, 0, list(range(n)))
    return split, dims, leaves


def boxes_py(P, h, leaves):
    """(lo, hi) lists of every heap node: the bounding box of the points of the leaves below it."""
    first = (1 << h) - 1
    out = [None] * (2 * first + 1)

    def rec(v):
        if v >= first:
            pts = P[leaves[v - first]]
        else:
            rec(2 * v + 1)
            rec(2 * v + 2)
            pts = None
        if pts is not None:
            out[v] = ([float(x) for x in pts.min(axis=0)], [float(x) for x in pts.max(axis=0)])
        else:
            a, b = out[2 * v + 1], out[2 * v + 2]
            out[v] = ([min(x, y) for x, y in zip(a[0], b[0])], [max(x, y) for x, y in zip(a[1], b[1])])
        return out[v]

    rec(0)
    return out


def box2_f32_exact(q, lo, hi) -> float:
    """float32 box term: g_j = fl32 distance of q_j to [lo_j, hi_j], acc = fl32(g*g + acc)."""
    acc = Fraction(0)
    for qj, a, b in zip(q, lo, hi):
        qj = Fraction(float(qj))
        if qj < Fraction(a):
            g = Fraction(round_f32(Fraction(a) - qj))
        elif qj > Fraction(b):
            g = Fraction(round_f32(qj - Fraction(b)))
        else:
            g = Fraction(0)
        acc = Fraction(round_f32(g * g + acc))
    return float(acc)


def search_rules_py(P, split, dims, leaves, h, q, k, boxes=None):
    """Recursive depth-first search, near child first, per-node dimensions, and the far child
    entered when its bound (the box term with boxes, else the plane term) does not exceed the
    current k-th float32 squared distance.  Returns (leaf order, final list)."""
    first = (1 << h) - 1
    best = []
    order = []

    def kth():
        return best[k - 1][0] if len(best) >= k else math.inf

    def visit(v):
        if v >= first:
            leaf = v - first
            order.append(leaf)
            for i in leaves[leaf]:
                best.append((dist2_f32_exact(q, P[i]), i))
            best.sort()
            del best[k:]
            return
        dim = dims[v]
        near, far = (2 * v + 1, 2 * v + 2) if float(q[dim]) < split[v] else (2 * v + 2, 2 * v + 1)
        visit(near)
        bound = box2_f32_exact(q, *boxes[far]) if boxes is not None else plane2_f32_exact(q[dim], split[v])
        if bound <= kth():
            visit(far)

    visit(0)
    return order, best
