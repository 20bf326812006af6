"""Pin of the dense leaf scan's matrix-core filter bound.

The filter works in each leaf's own frame: centred coordinates (relative to
the leaf's bounding-box centre c, rounded to float32) times the leaf's scale
s, a power of two with every centred point coordinate in [-1, 1].  Both sides
are rounded to float16 (x~, q~) and G = <q~,x~> - |x~|^2/2 is formed from the
products x~_j q~_j (exact in float32) and the norm term's float16 hi and lo
parts, accumulated in float32 in an unspecified order with either rounding.
A pair passes when

    G >= (|q~|^2 - T)/2 - 2^-18 (|q~|^2 + d + 1) - 2^-100,
    T = (sqrt(thr s^2) + delta)^2,
    delta = 2^-10 (1 + 2^-8)(|p| + sqrt d) + 2^-13 sqrt d,

with p the scaled query offset and thr the query's current K-th float32
squared distance; the square root in T is the hardware's approximate one,
modelled at its worst (2^-21 relative low, zero below 2^-126).  The claim:
every pair whose float32 distance (the oracle's arithmetic) is at most thr
passes.  These tests emulate every rounding
exactly with rationals, float16 rounding to nearest even, toward zero, or
with subnormals flushed, float32 accumulation in random orders and in the
matrix cores' steps of sixteen products (one step at d <= 14, two or three at
d = 15..32), at thresholds equal to the pair's own distance and one ulp
either side, and check the claim; a negative control shows that the
widening delta is needed.  The GPU parity tests check that results stay
bit-identical.
"""
from __future__ import annotations

from fractions import Fraction as F

import numpy as np
import pytest

from tests.exact_ref import round_f32


def round_f16(x: F, mode: str) -> F:
    """Round an exact rational to float16 (11 significant bits, subnormals down to 2^-24)."""
    if x == 0:
        return F(0)
    neg = x < 0
    a = -x if neg else x
    e = a.numerator.bit_length() - a.denominator.bit_length()
    while F(2) ** e > a:
        e -= 1
    while F(2) ** (e + 1) <= a:
        e += 1
    q = max(e - 10, -24)
    sc = a / F(2) ** q
    n = sc.numerator // sc.denominator
    rem = sc - n
    if mode != "rz" and (rem > F(1, 2) or (rem == F(1, 2) and n % 2 == 1)):
        n += 1
    v = F(n) * F(2) ** q
    if mode == "flush" and v < F(2) ** -14:
        v = F(0)
    return -v if neg else v


def f32(x: F) -> F:
    return F(round_f32(x))


def round_rz(x: F) -> F:
    r = F(round_f32(x))
    if abs(r) > abs(x):
        r = F(float(np.nextafter(np.float32(float(r)), np.float32(0.0))))
    return r


def sqrt32(x: F) -> F:
    return F(float(np.sqrt(np.float32(float(x)))))


def hw_sqrt(v: F) -> F:
    """The kernel's approximate square root, taken at its worst: two float32 ulps low
    (2^-21 relative), and zero for inputs below the normal range."""
    if v < F(2) ** -126:
        return F(0)
    return f32(sqrt32(v) * (1 - F(2) ** -21))


def filter_margin(q, x, c, e, thr: F, rng, mode: str, widen: bool = True):
    """min over accumulation orders and roundings of G - aq (>= 0: the pair passes), and the
    pair's float32 squared distance."""
    d = len(q)
    s = F(2) ** (-e)
    p = [f32(F(float(q[j])) - F(float(c[j]))) * s for j in range(d)]
    u = [f32(F(float(x[j])) - F(float(c[j]))) * s for j in range(d)]
    assert all(abs(v) <= 1 for v in u)
    qt = [round_f16(v, mode) for v in p]
    xt = [round_f16(v, mode) for v in u]
    d2 = F(0)
    for j in range(d):
        t = f32(F(float(q[j])) - F(float(x[j])))
        d2 = f32(t * t + d2)
    Qn = Pn = Xn = F(0)
    for j in range(d):
        Qn = f32(qt[j] * qt[j] + Qn)
        Pn = f32(p[j] * p[j] + Pn)
        Xn = f32(xt[j] * xt[j] + Xn)
    nb = f32(-Xn / 2)
    bh = round_f16(nb, "rne")
    bl = round_f16(f32(nb - bh), "rne")
    prods = [qt[j] * xt[j] for j in range(d)] + [bh, bl]
    sqd = sqrt32(F(d))
    delta = f32(f32(F(2) ** -10 * F(257, 256) * f32(sqrt32(Pn) + sqd)) + f32(F(2) ** -13 * sqd)) if widen else F(0)
    r = f32(hw_sqrt(f32(f32(thr * s) * s)) + delta)
    aq = f32(f32(F(1, 2) * f32(Qn - f32(r * r))) - f32(F(2) ** -18 * f32(Qn + d + 1))) - F(2) ** -100
    worst = None
    for rnd in (lambda v: F(round_f32(v)), round_rz):
        for _ in range(2):
            acc = F(0)
            for o in rng.permutation(len(prods)):
                acc = rnd(acc + prods[o])
            m = acc - aq
            worst = m if worst is None else min(worst, m)
        # the matrix cores take the products in steps of sixteen (operand order); within a
        # step the sum may be formed in any order or with a single rounding, and each
        # step's result is added to the running float32 accumulator
        steps = [prods[i:i + 16] for i in range(0, len(prods), 16)]
        for single in (True, False):
            acc = F(0)
            for st in steps:
                if single:
                    acc = rnd(acc + sum(st, F(0)))
                else:
                    part = F(0)
                    for o in rng.permutation(len(st)):
                        part = rnd(part + st[o])
                    acc = rnd(acc + part)
            m = acc - aq
            worst = min(worst, m)
    return worst, d2


def borderline_thresholds(q, x):
    t = np.float32(np.sum((q.astype(np.float64) - x.astype(np.float64)) ** 2))
    return [F(float(v)) for v in (t, np.nextafter(t, np.float32(np.inf)), np.nextafter(t, np.float32(0.0)))]


def scale_exponent(ext: float) -> int:
    return int(np.ceil(np.log2(ext)))


# one matrix-core step of sixteen products (d <= 14), and two or three steps (d >= 15)
ONE_STEP_DIMS = [3, 5, 10, 14]
MULTI_STEP_DIMS = [15, 16, 20, 24, 32]


@pytest.mark.parametrize("dims,seed", [(ONE_STEP_DIMS, 1), (MULTI_STEP_DIMS, 11)])
def test_scaled_f16_band_random(dims, seed):
    rng = np.random.default_rng(seed)
    cases = 0
    for _ in range(120):
        d = int(rng.choice(dims))
        cen = rng.uniform(-20, 20, d).astype(np.float32)
        ext = float(rng.choice([1e-3, 0.5, 3.0, 50.0]))
        e = scale_exponent(ext)
        x = (cen + rng.uniform(-1, 1, d) * ext * 0.999).astype(np.float32)
        q = (cen + rng.normal(0, float(rng.choice([0.1, 1.0, 5.0, 50.0])) * ext, d)).astype(np.float32)
        for thr in borderline_thresholds(q, x):
            for mode in ("rne", "rz", "flush"):
                m, d2 = filter_margin(q, x, cen, e, thr, rng, mode)
                if d2 <= thr:
                    assert m >= 0, (d, ext, float(thr), float(m))
                    cases += 1
    assert cases > 500


@pytest.mark.parametrize("dims,seed", [([3, 10, 14], 2), (MULTI_STEP_DIMS, 12)])
def test_scaled_f16_band_adversarial(dims, seed):
    rng = np.random.default_rng(seed)
    for _ in range(60):
        d = int(rng.choice(dims))
        cen = rng.uniform(-1e3, 1e3, d).astype(np.float32)
        ext = float(rng.choice([1e-30, 1e-6, 1.0, 1e4]))
        e = scale_exponent(ext)
        # a point on the box's corner; queries: the point itself, its neighbour float, a far one
        x = (cen + np.sign(rng.uniform(-1, 1, d)) * np.float32(ext) * np.float32(0.9999)).astype(np.float32)
        for q in (x.copy(), np.nextafter(x, np.float32(np.inf)).astype(np.float32),
                  (cen + rng.normal(0, 1000 * ext, d)).astype(np.float32)):
            if np.any(np.abs((q.astype(np.float64) - cen) / 2.0 ** e) > 2 ** 14):
                continue  # such a query takes the exact path
            for thr in borderline_thresholds(q, x)[:2]:
                for mode in ("rne", "rz", "flush"):
                    m, d2 = filter_margin(q, x, cen, e, thr, rng, mode)
                    if d2 <= thr:
                        assert m >= 0


@pytest.mark.parametrize("d", [10, 20])
def test_scaled_f16_band_needs_the_widening(d):
    """Negative control: with delta = 0 some pair at its own threshold is dropped."""
    rng = np.random.default_rng(3)
    broke = False
    for _ in range(60):
        cen = rng.uniform(-5, 5, d).astype(np.float32)
        x = (cen + rng.uniform(-1, 1, d) * np.float32(0.999)).astype(np.float32)
        q = (cen + rng.normal(0, 1.0, d)).astype(np.float32)
        thr = borderline_thresholds(q, x)[0]
        m, d2 = filter_margin(q, x, cen, 0, thr, rng, "rne", widen=False)
        broke |= d2 <= thr and m < 0
    assert broke


def test_threshold_widening_is_small_for_typical_geometry():
    """The squared threshold grows by (1 + delta/r)^2 for a k-th radius r (in leaf units):
    at most 6% for queries within ten leaf radii of the centre and r >= half a radius."""
    for pnorm in (0.5, 1.0, 3.0, 10.0):
        delta = 2 ** -10 * (1 + 2 ** -8) * (pnorm + np.sqrt(10)) + 2 ** -13 * np.sqrt(10)
        assert ((0.5 + delta) / 0.5) ** 2 < 1.06


def _sign_test(c, aq):
    """The dense scan's mask bit: the sign of c - aq (float32) is clear."""
    with np.errstate(invalid="ignore", over="ignore"):
        t = np.float32(c) - np.float32(aq)
    return not np.signbit(t)


def test_mask_sign_bit_matches_comparison():
    """With aq never zero, 'sign of G - aq clear' is exactly G >= aq in float32, subnormals kept:
    x - y is +0 only for x == y and is never -0 for y != 0."""
    rng = np.random.default_rng(4)
    f32v = np.float32
    specials = [f32v(0.0), f32v(-0.0), f32v(1e-45), f32v(-1e-45), f32v(1.17549435e-38), f32v(-3e-39),
                f32v(1.0), f32v(-1.0), f32v(3.4e38), f32v(-3.4e38)]
    aqs = [v for v in specials if v != 0] + [f32v(np.inf), f32v(-np.inf), f32v(-1e-45)]
    vals = specials + list(rng.standard_normal(200).astype(np.float32)) + \
        list((rng.standard_normal(100) * 1e-40).astype(np.float32))
    checked = 0
    for aq in aqs + list(rng.standard_normal(50).astype(np.float32)):
        near = [aq, np.nextafter(aq, f32v(np.inf)), np.nextafter(aq, f32v(-np.inf))] if np.isfinite(aq) else []
        for c in vals + near:
            if not np.isfinite(c):
                continue
            assert _sign_test(c, aq) == bool(c >= aq), (float(c), float(aq))
            checked += 1
    assert checked > 10000
    # the guard is needed: with aq = +0, G = -0 passes the comparison but not the sign test
    assert f32v(-0.0) >= f32v(0.0) and not _sign_test(f32v(-0.0), f32v(0.0))
