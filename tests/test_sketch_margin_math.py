"""The fast sketch's sign test, checked against the exact error bound (CPU).

The MFMA sketch trusts the sign of a window's fast sum S (fp16 products, fp32
accumulation) when, in float32,
    y = |S| - b0 > 0  and  y*y > a2 * fma(E, 1 + 2^-6, W 2^-28),
with a2 = alpha^2 (1 + 2^-18) and b0 = beta (1 + 2^-20) rounded up, where the
error of S is at most alpha ||w|| + beta (alpha = c1 ||r|| + c2 sqrt(W),
beta = c2 sqrt(W) ||r||) and ||w||^2 <= E (1 + 2^-6) + W 2^-28 (Section 4.1's
sign bits stay exact only if S is trusted just when the bound allows it).  This
test emulates the float32 steps with numpy and checks, on values packed around
the decision boundary, that every accepted S satisfies the bound in exact
(float64 and rational) arithmetic: the rounding slack is never eaten.
"""
from fractions import Fraction

import numpy as np

F32 = np.float32


def round_up_f32(v: float) -> np.float32:
    f = F32(v)
    if float(f) < v:
        f = np.nextafter(f, F32(np.inf))
    return f


def constants(W: int, rnorm: float):
    u = 2.0 ** -11
    e32 = 2.0 ** -23
    k = W + 2
    gam = k * e32 / (1.0 - k * e32)
    bound = (2 * u + u * u + gam * (1 + u) * (1 + u) + (W + 1) * 2.0 ** -53) * 1.01
    c1 = round_up_f32(max(bound, 1e-3))
    c2 = round_up_f32(2.0 ** -14 * (1 + u) * 1.01)
    rn = round_up_f32(rnorm * (1 + 2.0 ** -40))
    sw = round_up_f32(np.sqrt(W))
    alpha = float(c1) * float(rn) + float(c2) * float(sw)
    a2 = round_up_f32(alpha * alpha * (1 + 2.0 ** -18))
    b0 = round_up_f32(float(c2) * float(sw) * float(rn) * (1 + 2.0 ** -20))
    return c1, c2, rn, sw, a2, b0


def trusted_f32(S: np.ndarray, E: np.ndarray, W: int, a2, b0) -> np.ndarray:
    k = 1.0 + 2.0 ** -6
    c = W * 2.0 ** -28
    Q = (E.astype(np.float64) * k + c).astype(F32)  # one rounding to float32
    y = (np.abs(S) - b0).astype(F32)
    return (y > 0) & ((y * y).astype(F32) > (a2 * Q).astype(F32))


def test_trusted_sign_implies_exact_bound():
    rng = np.random.default_rng(5)
    for W, rnorm in [(80, 9.1), (64, 0.003), (128, 2000.0), (30, 1.0)]:
        c1, c2, rn, sw, a2, b0 = constants(W, rnorm)
        alpha = Fraction(float(c1)) * Fraction(float(rn)) + Fraction(float(c2)) * Fraction(float(sw))
        beta = Fraction(float(c2)) * Fraction(float(sw)) * Fraction(float(rn))
        E = (10.0 ** rng.uniform(-12, 9, 4000)).astype(F32)
        E[:10] = 0
        q_exact = E.astype(np.float64) * (1 + 2.0 ** -6) + W * 2.0 ** -28
        edge = float(alpha) * np.sqrt(q_exact) + float(beta)
        # from a few ulps below the exact edge to past the slack (about 2^-19 above it)
        rel = rng.uniform(-8.0, 64.0, E.size) * 2.0 ** -24
        S = (edge * (1 + rel) * rng.choice([-1.0, 1.0], E.size)).astype(F32)
        ok = trusted_f32(S, E, W, a2, b0)
        assert ok.any() and (~ok).any()
        for s, e in zip(S[ok], E[ok]):
            # |S| - beta > alpha sqrt(Q), squared, in rational arithmetic
            q = Fraction(float(e)) * (1 + Fraction(1, 64)) + Fraction(W, 2 ** 28)
            y = abs(Fraction(float(s))) - beta
            assert y > 0 and y * y > alpha * alpha * q, (W, float(s), float(e))


def test_zero_sum_is_never_trusted():
    for W, rnorm in [(80, 9.1), (30, 1e-6)]:
        _, _, _, _, a2, b0 = constants(W, rnorm)
        E = np.array([0.0, 1.0, 1e6], F32)
        assert not trusted_f32(np.zeros(3, F32), E, W, a2, b0).any()


# ---------------------------------------------------------------------------
# the L1 margin (filters without fp16-subnormal entries)
# ---------------------------------------------------------------------------
def l1_constants(r: np.ndarray):
    W = len(r)
    u = 2.0 ** -11
    e32 = 2.0 ** -23
    k = W + 2
    gam = k * e32 / (1.0 - k * e32)
    v = u / (1 - u)
    e64 = (W + 1) * 2.0 ** -53
    l1r = float(np.abs(r.astype(np.float16).astype(np.float64)).sum())
    rel = (2 * v + v * v + gam + e64 * (1 + v) * (1 + v)) / (1 - gam)
    c1a = round_up_f32(rel * 1.01 * (1 + 2.0 ** -20))
    c0a = round_up_f32(2.0 ** -14 * (1 + v) * (1 + e64) * l1r / (1 - gam) * 1.01 * (1 + 2.0 ** -20))
    return c1a, c0a


def to_f16(a: np.ndarray, flush: bool) -> np.ndarray:
    h = a.astype(np.float16)  # round to nearest, subnormals kept
    if flush:
        h = np.where(np.abs(a) < 2.0 ** -14, np.float16(0), h)
    return h


def test_l1_margin_bounds_the_fast_sum_error():
    """|s16 - s| <= c1a A + c0a for the exact sum s of float32 r x, with s16 the
    float32 sum of the exact fp16 products in a shuffled order and A the float32
    sum of |r^||x^|, fp16 subnormals kept or flushed; and a sign the float32 test
    trusts is the sign of s (up to the float64 sum's own rounding, also in the
    bound)."""
    rng = np.random.default_rng(9)
    for W in (80, 30, 128):
        r = rng.standard_normal(W).astype(np.float32)
        r[np.abs(r) < 2.0 ** -13] = 0.25  # no fp16-subnormal entries
        c1a, c0a = l1_constants(r)
        trusted_wrong = 0
        for trial in range(300):
            x = rng.standard_normal(W).astype(np.float64)
            if trial % 3 == 0:
                x *= 2.0 ** rng.integers(-30, 8)
            if trial % 2 == 0:  # put the exact sum near zero
                x[-1] = -float(np.dot(r[:-1].astype(np.float64), x[:-1])) / float(r[-1])
            x = x.astype(np.float32)
            x[rng.random(W) < 0.1] *= np.float32(2.0 ** -16)  # some samples below 2^-14
            s = sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(r, x))
            for flush in (False, True):
                rh, xh = to_f16(r, False), to_f16(x, flush)
                prods = rh.astype(np.float32) * xh.astype(np.float32)  # exact in float32
                order = rng.permutation(W)
                s16 = np.float32(0)
                A = np.float32(0)
                for i in order:
                    s16 = np.float32(s16 + prods[i])
                    A = np.float32(A + np.abs(prods[i]))
                bound = Fraction(float(c1a)) * Fraction(float(A)) + Fraction(float(c0a))
                assert abs(Fraction(float(s16)) - s) <= bound, (W, trial, flush)
                M = np.float32(float(c1a) * float(A) + float(c0a))  # one rounding, as fma
                if abs(s16) > M and (s16 > 0) != (s > 0):
                    trusted_wrong += 1
        assert trusted_wrong == 0
        # worst case: every value just below an fp16 rounding midpoint and every
        # product of one sign, so each rounding takes close to u off each factor
        # and the errors add up to about 2u sum |r x|, close to the bound
        for trial in range(20):
            j = rng.integers(0, 16, size=(2, W))  # near 1: relative rounding close to u
            e = rng.integers(-3, 4, size=(2, W))
            vals = (1 + (j + 0.4999) * 2.0 ** -10) * 2.0 ** e
            rr, xx = vals[0].astype(np.float32), vals[1].astype(np.float32)
            ca, cz = l1_constants(rr)
            rh, xh = to_f16(rr, False), to_f16(xx, False)
            prods = rh.astype(np.float32) * xh.astype(np.float32)
            s16 = np.float32(0)
            A = np.float32(0)
            for i in rng.permutation(W):
                s16 = np.float32(s16 + prods[i])
                A = np.float32(A + prods[i])
            ss = sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(rr, xx))
            err = abs(Fraction(float(s16)) - ss)
            bound = Fraction(float(ca)) * Fraction(float(A)) + Fraction(float(cz))
            assert err <= bound and err > bound * Fraction(85, 100), (W, trial, float(err / bound))
