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
