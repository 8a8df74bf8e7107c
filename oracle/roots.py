"""Polynomial approximation of 1/z and the multi-boson roots (oracle).

Test infrastructure only.

Section 4 approximates 1/z by P_N(z) = (1 - R_{N+1}(z))/z = c_N prod_k (z - z_k)
and gives the shifted roots u_k = 1 - z_k = cos(2 pi k/(N+1)) + i sqrt(1-c^2) sin(2 pi k/(N+1)).
The paper does not define R_{N+1} or c.  The reading used here (it reproduces
the printed roots exactly) is the Chebyshev remainder
    R_{N+1}(z) = T_{N+1}((1 - z)/c) / T_{N+1}(1/c),   0 < c < 1,
which is 1 at z = 0 and small on the disc-like region around z = 1.
"""
from __future__ import annotations

import numpy as np

__all__ = ["chebyshev_T", "remainder", "poly_P", "mb_roots", "leading_coeff"]


def chebyshev_T(n: int, x):
    """T_n(x) by the three-term recurrence (works for complex x)."""
    x = np.asarray(x, dtype=np.complex128)
    t0 = np.ones_like(x)
    if n == 0:
        return t0
    t1 = x.copy()
    for _ in range(n - 1):
        t0, t1 = t1, 2 * x * t1 - t0
    return t1


def remainder(N: int, c: float, z):
    """R_{N+1}(z) = T_{N+1}((1 - z)/c) / T_{N+1}(1/c)."""
    z = np.asarray(z, dtype=np.complex128)
    return chebyshev_T(N + 1, (1 - z) / c) / chebyshev_T(N + 1, np.asarray(1.0 / c))


def poly_P(N: int, c: float, z):
    """P_N(z) = (1 - R_{N+1}(z)) / z."""
    z = np.asarray(z, dtype=np.complex128)
    return (1 - remainder(N, c, z)) / z


def mb_roots(N: int, c: float) -> np.ndarray:
    """u_k = 1 - z_k for k = 1..N (Section 4)."""
    k = np.arange(1, N + 1)
    th = 2 * np.pi * k / (N + 1)
    return np.cos(th) + 1j * np.sqrt(1 - c * c) * np.sin(th)


def leading_coeff(N: int, c: float) -> float:
    """c_N, the leading coefficient of P_N: -(coefficient of z^{N+1} in R_{N+1}).

    T_{N+1}(y) has leading coefficient 2^N, and y = (1 - z)/c contributes
    (-1/c)^{N+1}.
    """
    lead_R = 2.0 ** N * (-1.0 / c) ** (N + 1) / float(np.real(chebyshev_T(N + 1, np.asarray(1.0 / c))))
    return -lead_R
