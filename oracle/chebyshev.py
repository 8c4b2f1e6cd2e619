"""Polynomial P_K: Chebyshev acceleration of the Jacobi iteration on K_m.

TEST INFRASTRUCTURE ONLY (see the package header).

Sec. 5.3 leaves the choice of P_1 ~ S_1 and P_K ~ K_m open: any classical
preconditioner of the elliptic / parabolic matrix fits the block-LU
framework of Def. 2.  This module defines one such P_K by its polynomial.
With D = diag(K), A = D^-1 K, an interval [lo, hi] for the spectrum of A,
theta = (hi + lo) / 2, delta = (hi - lo) / 2 and m steps from z_0 = 0, the
Chebyshev method returns z = q(A) D^-1 t where the residual polynomial is

    R_m(lam) = 1 - lam q(lam) = T_m((theta - lam) / delta) / T_m(theta / delta)

(T_m the Chebyshev polynomial of the first kind; R_m(0) = 1, so q has
degree m - 1).  The oracle builds q from that closed form with numpy's
polynomial classes and applies it by Horner's rule; it does not run the
three-term recurrence.  Monomial coefficients grow with m, so this plain
form is meant for m of at most about ten.
"""
import numpy as np
from numpy.polynomial import Chebyshev, Polynomial


def residual_polynomial(lo, hi, m):
    """R_m as a Polynomial in lam."""
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    tm = Chebyshev.basis(m).convert(kind=Polynomial)        # T_m(x), power basis
    x_of_lam = Polynomial([theta / delta, -1.0 / delta])     # x = (theta - lam) / delta
    return tm(x_of_lam) / tm(theta / delta)


def q_polynomial(lo, hi, m):
    """q with 1 - lam q(lam) = R_m(lam) (degree m - 1)."""
    one_minus_r = Polynomial([1.0]) - residual_polynomial(lo, hi, m)
    quo, rem = divmod(one_minus_r, Polynomial([0.0, 1.0]))
    assert np.allclose(rem.coef, 0.0, atol=1e-9 * max(1.0, np.abs(one_minus_r.coef).max()))
    c = np.zeros(m)
    c[:len(quo.coef)] = quo.coef[:m]
    return c


def chebyshev_jacobi(K, t, lo, hi, m):
    """z = q(D^-1 K) D^-1 t for a sparse or dense symmetric K."""
    d = K.diagonal() if hasattr(K, "diagonal") else np.diag(K)
    v = t / d
    c = q_polynomial(lo, hi, m)
    z = c[-1] * v
    for j in range(m - 2, -1, -1):          # Horner: z <- A z + c_j v
        z = (K @ z) / d + c[j] * v
    return z


def chebyshev_t(m, x):
    """T_m(x) from its trigonometric / hyperbolic definition."""
    x = np.asarray(x, dtype=float)
    inside = np.abs(x) <= 1.0
    out = np.empty_like(x)
    out[inside] = np.cos(m * np.arccos(x[inside]))
    xo = x[~inside]
    out[~inside] = np.sign(xo) ** m * np.cosh(m * np.arccosh(np.abs(xo)))
    return out
