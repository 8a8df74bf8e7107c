"""The Sheikholeslami-Wohlert (clover) term of the Dirac operator (oracle, small lattices only).

Test infrastructure only.  Section 3 takes D to be the Wilson-Dirac operator,
naming the Sheikholeslami-Wohlert improvement beside it; the paper prints no
formula for the term, so the textbook one is taken (reading R24):

  D_sw = D_w + A - 1,   A(x) = 1 + i kappa c_sw sum_{mu<nu} sigma_{mu nu} Fhat_{mu nu}(x),

in the hopping normalisation D_w = 1 - kappa H of wilson.py (the usual
c_sw (i/4) sum_{mu,nu} sigma F of the lattice-spacing normalisation, times
2 kappa).  sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu] in the chiral basis of
wilson.gamma; Fhat_{mu nu}(x) = (Q_{mu nu}(x) - Q_{mu nu}(x)^+) / 8, with
Q_{mu nu}(x) the sum of the four plaquettes in the (mu, nu) plane that start
and end at x, each traversed mu-then-nu (counter-clockwise).  The gauge field
is periodic in every direction (the antiperiodic time condition belongs to
the fermion hops, not to the plaquettes).  A(x) is diagonal in the site, acts
on spin and colour, is hermitian and commutes with gamma_5.

The restriction to a box keeps A(x) of the full lattice at every box site: D_X
is the principal sub-matrix of D (the plaquettes of a boundary site reach
links outside the box).

Spin-colour index of a site: 3 s + c (as everywhere in the oracle).
"""
from __future__ import annotations

import numpy as np

from . import geometry, wilson

__all__ = ["sigma", "field_strength", "clover_matrix", "dirac_clover_full", "dirac_clover_box", "PLANES"]

PLANES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def sigma(mu: int, nu: int) -> np.ndarray:
    """sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu], 4x4."""
    g_mu, g_nu = wilson.gamma(mu), wilson.gamma(nu)
    return 0.5j * (g_mu @ g_nu - g_nu @ g_mu)


def _shift(L, mu, step):
    """Index map x -> x + step * mu-hat (periodic) over the canonical site order."""
    x = geometry.coords(L)
    x[:, mu] = (x[:, mu] + step) % int(L[mu])
    Lv = [int(v) for v in L]
    return ((x[:, 0] * Lv[1] + x[:, 1]) * Lv[2] + x[:, 2]) * Lv[3] + x[:, 3]


def _dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


def field_strength(L, U) -> np.ndarray:
    """Fhat_{mu nu}(x) for the six planes of PLANES: [V, 6, 3, 3] (anti-hermitian)."""
    U = np.asarray(U, dtype=np.complex128)
    V = U.shape[0]
    F = np.empty((V, 6, 3, 3), dtype=np.complex128)
    for k, (mu, nu) in enumerate(PLANES):
        p_mu, p_nu = _shift(L, mu, 1), _shift(L, nu, 1)
        m_mu, m_nu = _shift(L, mu, -1), _shift(L, nu, -1)
        m_mu_p_nu = _shift(L, nu, 1)[m_mu]   # x - mu + nu
        m_mu_m_nu = _shift(L, nu, -1)[m_mu]  # x - mu - nu
        p_mu_m_nu = _shift(L, mu, 1)[m_nu]   # x + mu - nu
        Umu, Unu = U[:, mu], U[:, nu]
        # the four leaves at x, each a closed loop mu-then-nu
        q1 = Umu @ Unu[p_mu] @ _dag(Umu[p_nu]) @ _dag(Unu)
        q2 = Unu @ _dag(Umu[m_mu_p_nu]) @ _dag(Unu[m_mu]) @ Umu[m_mu]
        q3 = _dag(Umu[m_mu]) @ _dag(Unu[m_mu_m_nu]) @ Umu[m_mu_m_nu] @ Unu[m_nu]
        q4 = _dag(Unu[m_nu]) @ Umu[m_nu] @ Unu[p_mu_m_nu] @ _dag(Umu)
        Q = q1 + q2 + q3 + q4
        F[:, k] = (Q - _dag(Q)) / 8.0
    return F


def clover_matrix(L, U, kappa: float, csw: float) -> np.ndarray:
    """A(x) = 1 + i kappa c_sw sum_{mu<nu} sigma_{mu nu} (x) Fhat_{mu nu}(x): [V, 12, 12]."""
    F = field_strength(L, U)
    V = F.shape[0]
    A = np.zeros((V, 12, 12), dtype=np.complex128)
    for k, (mu, nu) in enumerate(PLANES):
        s = sigma(mu, nu)
        # (sigma (x) F)[3a + c, 3b + d] = sigma[a, b] F[c, d]
        A += np.einsum("ab,vcd->vacbd", s, F[:, k]).reshape(V, 12, 12)
    A *= 1j * kappa * csw
    A += np.eye(12)[None]
    return A


def _apply_site(A, psi):
    """(A psi)(x) for site matrices A[n, 12, 12] and psi[n, 4, 3]."""
    n = psi.shape[0]
    return np.einsum("vij,vj->vi", A, np.asarray(psi, dtype=np.complex128).reshape(n, 12)).reshape(n, 4, 3)


def dirac_clover_full(L, tbc: int, kappa: float, csw: float, U, psi, A=None) -> np.ndarray:
    """D_sw psi on the full lattice (canonical site order).  A: clover_matrix of the lattice, if
    already computed."""
    if A is None:
        A = clover_matrix(L, U, kappa, csw)
    psi = np.asarray(psi, dtype=np.complex128)
    return wilson.dirac_full(L, tbc, kappa, U, psi) + _apply_site(A, psi) - psi


def dirac_clover_box(L, tbc: int, kappa: float, csw: float, U, origin, extent, psi, A=None) -> np.ndarray:
    """D_sw restricted to a box (Dirichlet hops, A of the full lattice at the box sites); psi and the
    result in box-local canonical order.  A: clover_matrix of the lattice, if already computed."""
    if A is None:
        A = clover_matrix(L, U, kappa, csw)
    sites = geometry.box_sites(L, origin, extent)
    psi = np.asarray(psi, dtype=np.complex128)
    return wilson.dirac_box(L, tbc, kappa, U, origin, extent, psi) + _apply_site(A[sites], psi) - psi
