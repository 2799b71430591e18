"""The one-expression form of the cutoff function that the force and adjoint
kernels evaluate, checked in exact rational arithmetic against the two
pieces of eq. (cutoff) (Sec. 2):

    g(xi) = 1 - 8/5 xi^3 + 8/5 xi^5 - 1/2 xi^6 - 12/35 xi^7 + 3/20 xi^8    0 <= xi <= 1
    g(xi) = -(xi - 2)^5 (7 xi^3 + 22 xi^2 + 10 xi + 4) / 140              1 <= xi <= 2

With T = 1 - xi/2 and W = 1 - xi, each clamped to [0, 1], the kernels take

    g        = 32 T^5 R + W^6 Q,        R = (7 xi^3 + 22 xi^2 + 10 xi + 4) / 140,
                                        Q = 3/35 + 18/35 xi + xi^2 / 5,
    g'(xi)/xi = -16 T^4 P5 + W^5 L,     P5 = (2 xi^2 + 4 xi - 1) / 5,
                                        L = -16/5 - 8/5 xi,

which rests on the polynomial identities (no rounding involved)

    g_[0,1] - g_[1,2]             = (1 - xi)^6 Q,
    (g'_[0,1] - g'_[1,2]) / xi    = (1 - xi)^5 L,
    g'_[1,2] / xi                 = -(2 - xi)^4 P5.

No GPU and no oracle code: plain polynomial algebra over the rationals.
"""
from fractions import Fraction as F

import pytest

P = list  # ascending coefficient lists of Fractions


def padd(a, b):
    n = max(len(a), len(b))
    return [(a[i] if i < len(a) else F(0)) + (b[i] if i < len(b) else F(0)) for i in range(n)]


def pscale(a, s):
    return [s * c for c in a]


def pmul(a, b):
    r = [F(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            r[i + j] += x * y
    return r


def ppow(a, k):
    r = [F(1)]
    for _ in range(k):
        r = pmul(r, a)
    return r


def pder(a):
    return [i * a[i] for i in range(1, len(a))] or [F(0)]


def trim(a):
    a = list(a)
    while len(a) > 1 and a[-1] == 0:
        a.pop()
    return a


def peval(a, x):
    return sum(c * x ** i for i, c in enumerate(a))


# the two pieces as printed (the [1,2] one in the factored form of R17,
# itself pinned against the printed expansion in the oracle's tests)
G01 = [F(1), F(0), F(0), F(-8, 5), F(0), F(8, 5), F(-1, 2), F(-12, 35), F(3, 20)]
R = [F(4, 140), F(10, 140), F(22, 140), F(7, 140)]
TWO_MINUS_XI = [F(2), F(-1)]
ONE_MINUS_XI = [F(1), F(-1)]
G12 = pmul(ppow(TWO_MINUS_XI, 5), R)
Q = [F(3, 35), F(18, 35), F(1, 5)]
L = [F(-16, 5), F(-8, 5)]
P5 = [F(-1, 5), F(4, 5), F(2, 5)]


def div_by_xi(a):
    assert a[0] == 0, "not divisible by xi"
    return a[1:]


def test_value_difference_is_sixth_order_at_one():
    assert trim(padd(G01, pscale(G12, F(-1)))) == trim(pmul(ppow(ONE_MINUS_XI, 6), Q))


def test_derivative_difference_over_xi():
    d = padd(pder(G01), pscale(pder(G12), F(-1)))
    assert trim(div_by_xi(d)) == trim(pmul(ppow(ONE_MINUS_XI, 5), L))


def test_outer_derivative_over_xi():
    assert trim(div_by_xi(pder(G12))) == trim(pscale(pmul(ppow(TWO_MINUS_XI, 4), P5), F(-1)))


def clamp01(v):
    return min(max(v, F(0)), F(1))


def g_kernel_form(xi):
    t, w = clamp01(1 - xi / 2), clamp01(1 - xi)
    return 32 * t ** 5 * peval(R, xi) + w ** 6 * peval(Q, xi)


def h_kernel_form(xi):
    """g'(xi)/xi as the kernels form it (before the factor k^2)."""
    t, w = clamp01(1 - xi / 2), clamp01(1 - xi)
    return -16 * t ** 4 * peval(P5, xi) + w ** 5 * peval(L, xi)


@pytest.mark.parametrize("xi", [F(0), F(1, 7), F(1, 2), F(99, 100), F(1), F(101, 100), F(3, 2), F(199, 100),
                                F(2), F(9, 4), F(3)])
def test_kernel_form_equals_the_piecewise_function(xi):
    if xi <= 1:
        g, gp = peval(G01, xi), peval(pder(G01), xi)
    elif xi <= 2:
        g, gp = peval(G12, xi), peval(pder(G12), xi)
    else:
        g, gp = F(0), F(0)
    assert g_kernel_form(xi) == g
    if xi > 0:
        assert h_kernel_form(xi) == gp / xi
    else:
        # g'(xi)/xi -> -24/5 xi -> 0 at the origin; the form gives it exactly
        assert h_kernel_form(xi) == 0


def test_both_terms_are_nonnegative_on_the_support():
    for j in range(0, 201):
        xi = F(j, 100)
        t, w = clamp01(1 - xi / 2), clamp01(1 - xi)
        assert 32 * t ** 5 * peval(R, xi) >= 0 and w ** 6 * peval(Q, xi) >= 0
