"""The excess-pivot recursion of the r = 1 float32 precision mode, checked
against the plain pivot recursion of the banded LDL^T (Sec. 2.2) on the
tridiagonal A = I + lambda L of a path (Eq. 4 at r = 1), without a GPU.

Plain:  alpha_0 = 1 + c_0,  alpha_k = 1 + c_{k-1} + c_k - c_{k-1}^2 / alpha_{k-1}.
Excess: delta_0 = 1,  alpha_k = delta_k + c_k,  delta_{k+1} = 1 + c_k delta_k / alpha_k.

In exact arithmetic both give the same pivots (delta_k = alpha_k - c_k is the
pivot's excess over the coupling still to be eliminated), and the product of
the pivots is det(A).  In float32 with c up to 1e7 (lambda * omega^frac at the
paper's detail-enhancement setting) the plain recursion loses the excess, which
is what makes A well conditioned, while the excess recursion keeps it to a few
float32 ulps."""
from fractions import Fraction

import numpy as np
import pytest


def plain(c, dtype):
    c = c.astype(dtype)
    one = dtype(1)
    a = np.empty_like(c)
    a[0] = one + c[0]
    for k in range(1, len(c)):
        a[k] = one + c[k - 1] + c[k] - c[k - 1] * c[k - 1] / a[k - 1]
    return a


def excess(c, dtype):
    c = c.astype(dtype)
    one = dtype(1)
    d = np.empty_like(c)
    d[0] = one
    for k in range(len(c) - 1):
        d[k + 1] = one + c[k] * (d[k] / (d[k] + c[k]))
    return d   # alpha_k = d_k + c_k


def chain(n, scale, seed):
    rng = np.random.default_rng(seed)
    c = scale * rng.uniform(0.0, 1.0, n)
    c[-1] = 0.0   # the last element has no coupling beyond it
    return c


def exact_excess(c):
    """Pivot excesses alpha_k - c_k by the plain recursion in exact rational
    arithmetic (no rounding at all)."""
    c = [Fraction(float(v)) for v in c]
    a = [1 + c[0]]
    for k in range(1, len(c)):
        a.append(1 + c[k - 1] + c[k] - c[k - 1] * c[k - 1] / a[k - 1])
    return np.array([float(a[k] - c[k]) for k in range(len(c))])


@pytest.mark.parametrize("scale", [1e-3, 1.0, 1e3, 1e7])
def test_excess_matches_exact_arithmetic(scale):
    c = chain(60, scale, seed=int(np.log10(scale) + 20))
    np.testing.assert_allclose(excess(c, np.float64), exact_excess(c), rtol=1e-13)


@pytest.mark.parametrize("scale", [1e-3, 1.0, 1e3])
def test_excess_equals_plain_pivots_in_float64(scale):
    # (at these scales the plain float64 recursion is itself accurate)
    c = chain(300, scale, seed=int(np.log10(scale) + 10))
    a = plain(c, np.float64)
    d = excess(c, np.float64)
    np.testing.assert_allclose(d + c, a, rtol=1e-12)
    # the pivots factor A: their product is det(A), checked against a dense determinant
    n = 12
    cs = c[:n].copy()
    cs[-1] = 0.0
    A = np.eye(n)
    for k in range(n - 1):
        A[k, k] += cs[k]
        A[k + 1, k + 1] += cs[k]
        A[k, k + 1] = A[k + 1, k] = -cs[k]
    sign, logdet = np.linalg.slogdet(A)
    assert sign > 0
    np.testing.assert_allclose(np.sum(np.log(excess(cs, np.float64) + cs)), logdet, rtol=1e-12)


def test_excess_is_bounded_below_by_one():
    # every Schur complement of I + lambda L keeps the identity: delta_k >= 1
    d = excess(chain(500, 1e7, seed=3), np.float64)
    assert (d >= 1.0).all()


def test_float32_keeps_the_excess_where_the_plain_recursion_loses_it():
    c = chain(120, 1e7, seed=5).astype(np.float32).astype(np.float64)   # exactly representable
    ref = exact_excess(c)
    d32 = excess(c, np.float32).astype(np.float64)
    e_excess = np.max(np.abs(d32 - ref) / ref)
    a32 = plain(c, np.float32).astype(np.float64)
    e_plain = np.max(np.abs((a32 - c.astype(np.float32).astype(np.float64)) - ref) / ref)
    assert e_excess < 1e-5, e_excess
    assert e_plain > 1e-1, e_plain                    # the plain pivots lost it
