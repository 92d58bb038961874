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
