"""Dense-matrix checks of the block factorisation (oracle, tiny lattices only).

Test infrastructure only.  The dense matrix of D is assembled column by column
from the C operator (``dirac_full`` applied to unit vectors); restrictions D_X
and off-diagonal blocks D_{X,Y} are sub-matrices of it, and determinants come
from LU factorisations (``numpy.linalg.slogdet``).

Row/column index of (site n, spin s, colour c) is 12 n + 3 s + c.
"""
from __future__ import annotations

import numpy as np

from . import wilson

__all__ = [
    "dense_dirac_full",
    "dense_dirac_box",
    "dof",
    "sub",
    "logdet",
    "schur",
]


def dense_dirac_full(L, tbc, kappa, U) -> np.ndarray:
    V = int(np.prod(L))
    n = 12 * V
    M = np.empty((n, n), dtype=np.complex128)
    e = np.zeros((V, 4, 3), dtype=np.complex128)
    ef = e.reshape(-1)
    for j in range(n):
        ef[j] = 1.0
        M[:, j] = wilson.dirac_full(L, tbc, kappa, U, e).reshape(-1)
        ef[j] = 0.0
    return M


def dense_dirac_box(L, tbc, kappa, U, origin, extent) -> np.ndarray:
    S = int(np.prod(extent))
    n = 12 * S
    M = np.empty((n, n), dtype=np.complex128)
    e = np.zeros((S, 4, 3), dtype=np.complex128)
    ef = e.reshape(-1)
    for j in range(n):
        ef[j] = 1.0
        M[:, j] = wilson.dirac_box(L, tbc, kappa, U, origin, extent, e).reshape(-1)
        ef[j] = 0.0
    return M


def dof(sites) -> np.ndarray:
    """Matrix indices of all spin-colour components of the given sites."""
    sites = np.asarray(sites, dtype=np.int64)
    return (12 * sites[:, None] + np.arange(12)[None, :]).reshape(-1)


def sub(M, rows, cols=None) -> np.ndarray:
    """D_{X,Y}: rows of the sites X, columns of the sites Y (Y = X if omitted)."""
    r = dof(rows)
    c = r if cols is None else dof(cols)
    return M[np.ix_(r, c)]


def logdet(A) -> complex:
    """ln det A (complex: ln|det| + i arg det) from an LU factorisation."""
    if A.shape[0] == 0:
        return 0.0 + 0.0j
    sign, ld = np.linalg.slogdet(A)
    return ld + 1j * np.angle(sign)


def schur(A, B, C, Dm) -> np.ndarray:
    """A - B Dm^{-1} C."""
    if Dm.shape[0] == 0:
        return A.copy()
    return A - B @ np.linalg.solve(Dm, C)
