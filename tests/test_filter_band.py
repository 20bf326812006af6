"""Pin of the dense leaf scan's inner-product filter bound.

The filter compares (1 - c(d)) S - 2<q',x'> with the current K-th squared
distance, where q' = q - centre and x' = x - centre are rounded to float32,
S = |q'|^2 + |x'|^2 and every quantity is accumulated with float32 fused
multiply-adds.  It is exact (never drops a point that the float32 distance
would keep) provided |(S - 2<q',x'>)_float32 - d2_float32| <= (4d + 14) 2^-24 S,
with c(d) four times that.  Here the float32 arithmetic is emulated exactly
with rationals (round to nearest even after every operation) and the bound is
checked on random and adversarial inputs.  This pins the constant; the GPU
parity tests check that results stay bit-identical.

The inner product may also come from a matrix unit that adds two products
per step in an unspecified order and may truncate instead of rounding to
nearest (error up to 2^-23 per operation).  The second set of tests emulates
that arithmetic in every add order, with both rounding modes, and checks the
expansion against twice the bound.

The dense scan itself forms the inner product from bfloat16 parts: each
centred float32 coordinate v is split as hi = bf16(v), lo = bf16(v - hi), and
<q',x'> is taken as sum(xl qh + xh ql + xh qh) over three matrix-unit calls
whose float32 accumulation may round either way in any order.  The dropped
terms are at most 3 2^-16 sum |q'_j x'_j|, so the expansion stays within
2^-14 S of the float32 distance; the kernel's band is c = 2^-12, four times
that.  The third set of tests emulates this exactly and checks 2^-14 S, and
checks that dropping one of the three products breaks it.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from tests.exact_ref import round_f32

U = Fraction(1, 1 << 24)


def f(x):
    return Fraction(float(x))


def fmaf(a, b, c):
    return Fraction(round_f32(a * b + c))


def sub(a, b):
    return Fraction(round_f32(a - b))


def round_rz(x: Fraction) -> Fraction:
    """Round an exact rational to float32 toward zero."""
    r = Fraction(round_f32(x))
    if abs(r) > abs(x):
        r = Fraction(float(np.nextafter(np.float32(float(r)), np.float32(0.0))))
    return r


def mx_dot(qc, xc, rnd, order):
    """Inner product in steps of two coordinates, every product and sum rounded by rnd."""
    acc = Fraction(0)
    for j in range(0, len(qc), 2):
        p0 = rnd(qc[j] * xc[j])
        p1 = rnd(qc[j + 1] * xc[j + 1]) if j + 1 < len(qc) else Fraction(0)
        if order == 0:
            acc = rnd(rnd(acc + p0) + p1)
        elif order == 1:
            acc = rnd(rnd(acc + p1) + p0)
        else:
            acc = rnd(acc + rnd(p0 + p1))
    return acc


def filter_terms(q, x, cen, dot_fn=None):
    d = len(q)
    qc = [sub(f(q[j]), f(cen[j])) for j in range(d)]
    xc = [sub(f(x[j]), f(cen[j])) for j in range(d)]
    Qn = Xn = dot = Fraction(0)
    for j in range(d):
        Qn = fmaf(qc[j], qc[j], Qn)
        Xn = fmaf(xc[j], xc[j], Xn)
        dot = fmaf(qc[j], xc[j], dot)
    if dot_fn is not None:
        dot = dot_fn(qc, xc)
    d2 = Fraction(0)
    for j in range(d):
        t = sub(f(q[j]), f(x[j]))
        d2 = fmaf(t, t, d2)
    S = Qn + Xn
    approx = S - 2 * dot  # exact combination; the kernel's own rounding of it is covered by the factor 4
    return approx, d2, S


def check(q, x, cen):
    d = len(q)
    approx, d2, S = filter_terms(q, x, cen)
    bound = (4 * d + 14) * U * S
    assert abs(approx - d2) <= bound + Fraction(1, 10 ** 40), (float(approx), float(d2), float(S))


def check_mx(q, x, cen):
    d = len(q)
    bound = 2 * (4 * d + 14) * U
    worst = Fraction(0)
    for rnd in (lambda v: Fraction(round_f32(v)), round_rz):
        for order in range(3):
            approx, d2, S = filter_terms(q, x, cen, lambda a, b: mx_dot(a, b, rnd, order))
            assert abs(approx - d2) <= bound * S + Fraction(1, 10 ** 40), (float(approx), float(d2), float(S))
            if S > 0:
                worst = max(worst, abs(approx - d2) / (bound * S))
    return worst


def test_band_random_mixture_scale():
    rng = np.random.default_rng(1)
    for d in (3, 10, 15):
        for _ in range(150):
            cen = (rng.uniform(0, 20, d)).astype(np.float32)
            spread = rng.choice([1e-3, 0.1, 2.0, 30.0])
            q = (cen + rng.normal(0, spread, d)).astype(np.float32)
            x = (cen + rng.normal(0, spread, d)).astype(np.float32)
            check(q, x, cen)


def test_band_adversarial():
    rng = np.random.default_rng(2)
    d = 10
    for _ in range(100):
        # far from the origin, tiny separation (cancellation), centre off to one side
        base = rng.uniform(1e3, 1e4, d).astype(np.float32)
        q = base
        x = np.nextafter(base, np.float32(np.inf)) if rng.random() < 0.5 else (base + np.float32(1e-3))
        cen = (base + rng.normal(0, 50, d)).astype(np.float32)
        check(q, x.astype(np.float32), cen)
        check(q, q.copy(), cen)  # identical points: distance 0
        # subnormal-sized differences
        tiny = (rng.normal(0, 1e-39, d)).astype(np.float32)
        check(tiny, np.zeros(d, np.float32), np.zeros(d, np.float32))


def test_band_matrix_unit_model_random():
    rng = np.random.default_rng(3)
    worst = Fraction(0)
    for d in (3, 10, 15):
        for _ in range(40):
            cen = (rng.uniform(0, 20, d)).astype(np.float32)
            spread = rng.choice([1e-3, 0.1, 2.0, 30.0])
            q = (cen + rng.normal(0, spread, d)).astype(np.float32)
            x = (cen + rng.normal(0, spread, d)).astype(np.float32)
            worst = max(worst, check_mx(q, x, cen))
    assert worst < 1


def test_band_matrix_unit_model_adversarial():
    rng = np.random.default_rng(4)
    d = 10
    for _ in range(30):
        base = rng.uniform(1e3, 1e4, d).astype(np.float32)
        x = np.nextafter(base, np.float32(np.inf)) if rng.random() < 0.5 else (base + np.float32(1e-3))
        cen = (base + rng.normal(0, 50, d)).astype(np.float32)
        check_mx(base, x.astype(np.float32), cen)
        check_mx(base, base.copy(), cen)
    # the wrong model fails: an inner product that loses one step's rounding twice over breaks the bound
    q = np.float32([3.0, -1.0, 2.5]); x = np.float32([2.9, -1.2, 2.4]); cen = np.float32([0.0, 0.0, 0.0])
    approx, d2, S = filter_terms(q, x, cen, lambda a, b: sum(a[j] * b[j] for j in range(3)) * (1 + 200 * U))
    assert abs(approx - d2) > 2 * (4 * 3 + 14) * U * S


def round_bf16(x: Fraction) -> Fraction:
    """Round an exact rational to the nearest bfloat16 (8 significant bits, ties to even)."""
    if x == 0:
        return Fraction(0)
    neg = x < 0
    a = -x if neg else x
    e = a.numerator.bit_length() - a.denominator.bit_length()
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    q = max(e - 7, -133)
    scaled = a / (Fraction(2) ** q)
    n = scaled.numerator // scaled.denominator
    rem = scaled - n
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and n % 2 == 1):
        n += 1
    v = Fraction(n) * Fraction(2) ** q
    return -v if neg else v


def split_dot(qc, xc, rnd, rng, terms=(0, 1, 2)):
    """sum(xl qh + xh ql + xh qh): three accumulations of 16 products each, in random order."""
    qh = [round_bf16(v) for v in qc]
    ql = [round_bf16(v - h) for v, h in zip(qc, qh)]
    xh = [round_bf16(v) for v in xc]
    xl = [round_bf16(v - h) for v, h in zip(xc, xh)]
    calls = [[xl[j] * qh[j] for j in range(len(qc))], [xh[j] * ql[j] for j in range(len(qc))],
             [xh[j] * qh[j] for j in range(len(qc))]]
    acc = Fraction(0)
    for t in terms:
        prods = calls[t]
        order = rng.permutation(len(prods))
        sacc = Fraction(0)
        for o in order:
            sacc = rnd(sacc + prods[o])
        acc = rnd(acc + sacc)
    return acc


def check_split(q, x, cen, rng):
    worst = Fraction(0)
    for rnd in (lambda v: Fraction(round_f32(v)), round_rz):
        approx, d2, S = filter_terms(q, x, cen, lambda a, b: split_dot(a, b, rnd, rng))
        bound = Fraction(1, 1 << 14) * S
        assert abs(approx - d2) <= bound + Fraction(1, 10 ** 40), (float(approx), float(d2), float(S))
        if S > 0:
            worst = max(worst, abs(approx - d2) / bound)
    return worst


def test_band_bf16_split_random():
    rng = np.random.default_rng(5)
    worst = Fraction(0)
    for d in (3, 10, 15, 16):
        for _ in range(40):
            cen = (rng.uniform(0, 20, d)).astype(np.float32)
            spread = rng.choice([1e-3, 0.1, 2.0, 30.0])
            q = (cen + rng.normal(0, spread, d)).astype(np.float32)
            x = (cen + rng.normal(0, spread, d)).astype(np.float32)
            worst = max(worst, check_split(q, x, cen, rng))
    assert worst < 1


def test_band_bf16_split_adversarial():
    rng = np.random.default_rng(6)
    d = 10
    for _ in range(30):
        base = rng.uniform(1e3, 1e4, d).astype(np.float32)
        x = np.nextafter(base, np.float32(np.inf)) if rng.random() < 0.5 else (base + np.float32(1e-3))
        cen = (base + rng.normal(0, 50, d)).astype(np.float32)
        check_split(base, x.astype(np.float32), cen, rng)
        check_split(base, base.copy(), cen, rng)
        # coordinates whose bfloat16 parts round half-way
        hw = (cen + np.float32(1.0 + 2.0 ** -8 + 2.0 ** -17)).astype(np.float32)
        check_split(hw, cen.copy(), cen, rng)


def test_band_bf16_split_needs_all_three_products():
    rng = np.random.default_rng(7)
    broke = False
    for _ in range(20):
        d = 10
        cen = np.zeros(d, np.float32)
        q = rng.normal(0, 3, d).astype(np.float32)
        x = rng.normal(0, 3, d).astype(np.float32)
        approx, d2, S = filter_terms(q, x, cen, lambda a, b: split_dot(a, b, lambda v: Fraction(round_f32(v)), rng,
                                                                         terms=(1, 2)))
        broke |= abs(approx - d2) > Fraction(1, 1 << 14) * S
    assert broke


def folded_terms(q, x, cen, rnd, rng):
    """Qn - 2 G with G = <q',x'> - |x'|^2/2 formed in one split accumulation (the norm
    rides as one more coordinate pair (-|x'|^2/2, 1)), as the kernel does when a slot is free."""
    d = len(q)
    qc = [sub(f(q[j]), f(cen[j])) for j in range(d)]
    xc = [sub(f(x[j]), f(cen[j])) for j in range(d)]
    Qn = Xn = Fraction(0)
    for j in range(d):
        Qn = fmaf(qc[j], qc[j], Qn)
        Xn = fmaf(xc[j], xc[j], Xn)
    bs = Fraction(round_f32(Xn / 2))
    G = split_dot(qc + [Fraction(1)], xc + [-bs], rnd, rng)
    d2 = Fraction(0)
    for j in range(d):
        t = sub(f(q[j]), f(x[j]))
        d2 = fmaf(t, t, d2)
    return Qn - 2 * G, d2, Qn + Xn


def test_band_bf16_split_with_folded_norm():
    rng = np.random.default_rng(8)
    worst = Fraction(0)
    for d in (3, 10, 15):
        for _ in range(40):
            cen = (rng.uniform(0, 20, d)).astype(np.float32)
            spread = rng.choice([1e-3, 0.1, 2.0, 30.0])
            q = (cen + rng.normal(0, spread, d)).astype(np.float32)
            x = (cen + rng.normal(0, spread, d)).astype(np.float32)
            for rnd in (lambda v: Fraction(round_f32(v)), round_rz):
                approx, d2, S = folded_terms(q, x, cen, rnd, rng)
                bound = Fraction(1, 1 << 13) * S
                assert abs(approx - d2) <= bound + Fraction(1, 10 ** 40)
                if S > 0:
                    worst = max(worst, abs(approx - d2) / bound)
    assert worst < 1


def packed_dot(qc, xc, bs, rnd, rng):
    """<q',x'> - bs as the dense scan forms it: the 3d + 2 bfloat16 products
    xh.qh, xl.qh, xh.ql (d each) and bs_hi.1, bs_lo.1 laid end to end and cut
    into matrix-unit steps of sixteen; each step adds its products and the
    running accumulator in a random order, every sum rounded by rnd."""
    d = len(qc)
    qh = [round_bf16(v) for v in qc]
    ql = [round_bf16(v - h) for v, h in zip(qc, qh)]
    xh = [round_bf16(v) for v in xc]
    xl = [round_bf16(v - h) for v, h in zip(xc, xh)]
    bh = round_bf16(-bs)
    bl = round_bf16(-bs - bh)
    prods = ([xh[j] * qh[j] for j in range(d)] + [xl[j] * qh[j] for j in range(d)]
             + [xh[j] * ql[j] for j in range(d)] + [bh, bl])
    acc = Fraction(0)
    for s in range(0, len(prods), 16):
        group = prods[s:s + 16] + [acc]
        sacc = Fraction(0)
        for o in rng.permutation(len(group)):
            sacc = rnd(sacc + group[o])
        acc = sacc
    return acc


def test_band_bf16_packed_steps():
    """The packed, folded form keeps the folded bound 2^-13 S at every padded dimension."""
    rng = np.random.default_rng(9)
    worst = Fraction(0)
    for d in (2, 5, 10, 15, 16, 20, 32):
        for _ in range(12):
            cen = (rng.uniform(0, 20, d)).astype(np.float32)
            spread = rng.choice([1e-3, 0.1, 2.0, 30.0])
            q = (cen + rng.normal(0, spread, d)).astype(np.float32)
            x = (cen + rng.normal(0, spread, d)).astype(np.float32)
            qc = [sub(f(q[j]), f(cen[j])) for j in range(d)]
            xc = [sub(f(x[j]), f(cen[j])) for j in range(d)]
            Qn = Xn = Fraction(0)
            for j in range(d):
                Qn = fmaf(qc[j], qc[j], Qn)
                Xn = fmaf(xc[j], xc[j], Xn)
            bs = Fraction(round_f32(Xn / 2))
            d2 = Fraction(0)
            for j in range(d):
                t = sub(f(q[j]), f(x[j]))
                d2 = fmaf(t, t, d2)
            S = Qn + Xn
            for rnd in (lambda v: Fraction(round_f32(v)), round_rz):
                approx = Qn - 2 * packed_dot(qc, xc, bs, rnd, rng)
                bound = Fraction(1, 1 << 13) * S
                assert abs(approx - d2) <= bound + Fraction(1, 10 ** 40)
                if S > 0:
                    worst = max(worst, abs(approx - d2) / bound)
    assert worst < 1


def test_band_bf16_packed_steps_need_every_term():
    """Negative control: losing the low part of the folded norm (one of the two
    norm terms) breaks the bound."""
    rng = np.random.default_rng(10)
    broke = False
    for _ in range(20):
        d = 10
        qc = [Fraction(float(v)) for v in rng.normal(0, 3, d).astype(np.float32)]
        xc = [Fraction(float(v)) for v in rng.normal(0, 3, d).astype(np.float32)]
        Qn = sum(v * v for v in qc)
        Xn = sum(v * v for v in xc)
        bs = Fraction(round_f32(Xn / 2))
        exact = sum(a * b for a, b in zip(qc, xc)) - bs
        full = packed_dot(qc, xc, bs, lambda v: Fraction(round_f32(v)), rng)
        lost = full - (round_bf16(-bs - round_bf16(-bs)))
        assert abs(full - exact) <= Fraction(1, 1 << 14) * (Qn + Xn)
        broke |= abs(lost - exact) > Fraction(1, 1 << 14) * (Qn + Xn)
    assert broke
