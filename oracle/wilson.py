"""FP64 Wilson-Dirac operator, its box restrictions and block solves (oracle).

Thin numpy wrappers over the plain C code in ``dd_oracle.c``.  Test
infrastructure only.

Operator (paper Section 3 takes D to be the Wilson-Dirac operator; only its
locality is used by the derivation):
    D = 1 - kappa H,
    (H psi)(x) = sum_mu [(1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu)],
chiral gamma basis, periodic space, antiperiodic time when ``tbc = -1``.
D_X for a site set X is the restriction with Dirichlet boundary: hops whose
source lies outside X are dropped (the D_X of Section 3).
"""
from __future__ import annotations

import ctypes

import numpy as np

from ._clib import lib

__all__ = [
    "gamma",
    "hop_full",
    "dirac_full",
    "hop_box",
    "dirac_box",
    "box_parity",
    "solve_box",
    "solve_many",
    "num_threads",
]


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _i4(v) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(v, dtype=np.int32).reshape(-1))


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


def gamma(mu: int) -> np.ndarray:
    """gamma_mu (mu = 0..3) or gamma_5 (mu = 4) of the chiral basis, 4x4."""
    out = np.zeros((4, 4), dtype=np.complex128)
    lib().or_gamma(int(mu), _ptr(out))
    return out


def hop_full(L, tbc: int, U: np.ndarray, psi: np.ndarray) -> np.ndarray:
    L4 = _i4(L)
    U = _c128(U)
    psi = _c128(psi)
    out = np.empty_like(psi)
    lib().or_hop_full(_ptr(L4), int(tbc), _ptr(U), _ptr(psi), _ptr(out))
    return out


def dirac_full(L, tbc: int, kappa: float, U: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """D psi on the full lattice; psi[V,4,3] in canonical site order."""
    L4 = _i4(L)
    U = _c128(U)
    psi = _c128(psi)
    out = np.empty_like(psi)
    lib().or_dirac_full(_ptr(L4), int(tbc), float(kappa), _ptr(U), _ptr(psi), _ptr(out))
    return out


def hop_box(L, tbc, U, origin, extent, psi) -> np.ndarray:
    L4, o, e = _i4(L), _i4(origin), _i4(extent)
    U = _c128(U)
    psi = _c128(psi)
    out = np.empty_like(psi)
    lib().or_hop_box(_ptr(L4), int(tbc), _ptr(U), _ptr(o), _ptr(e), _ptr(psi), _ptr(out))
    return out


def dirac_box(L, tbc, kappa, U, origin, extent, psi) -> np.ndarray:
    """D_Lambda psi for the box Lambda = (origin, extent); psi in box-local canonical order."""
    L4, o, e = _i4(L), _i4(origin), _i4(extent)
    U = _c128(U)
    psi = _c128(psi)
    out = np.empty_like(psi)
    lib().or_dirac_box(_ptr(L4), int(tbc), float(kappa), _ptr(U), _ptr(o), _ptr(e), _ptr(psi),
                       _ptr(out))
    return out


def frame_mask(extent, hole_off, hole_ext) -> np.ndarray:
    """Box-local canonical mask of a frame: the box sites outside the hole (hole_off, hole_ext)."""
    y = np.indices([int(v) for v in extent]).reshape(4, -1).T
    ho, he = np.asarray(hole_off), np.asarray(hole_ext)
    return ~np.all((y >= ho) & (y < ho + he), axis=1)


def dirac_frame(L, tbc, kappa, U, origin, extent, hole_off, hole_ext, psi) -> np.ndarray:
    """D_Phi psi for the frame Phi = box minus hole (Section 2's Phi_1^a = Omega_0^a minus
    Lambda_0^a): the principal sub-matrix of D on Phi, i.e. D_box applied to psi restricted to
    Phi, then restricted to Phi.  psi and the result are box-local canonical, zero on the hole."""
    m = frame_mask(extent, hole_off, hole_ext)
    p = np.array(_c128(psi), copy=True)
    p[~m] = 0
    out = dirac_box(L, tbc, kappa, U, origin, extent, p)
    out[~m] = 0
    return out


def box_parity(L, origin, extent) -> np.ndarray:
    L4, o, e = _i4(L), _i4(origin), _i4(extent)
    S = int(np.prod(e))
    par = np.empty(S, dtype=np.int32)
    lib().or_box_parity(_ptr(L4), _ptr(o), _ptr(e), _ptr(par))
    return par


def solve_box(L, tbc, kappa, U, origin, extent, b, tol=1e-12, maxit=5000):
    """x = D_Lambda^{-1} b on one box; returns (x, inner iterations, true relres)."""
    L4, o, e = _i4(L), _i4(origin), _i4(extent)
    U = _c128(U)
    b = _c128(b)
    x = np.zeros_like(b)
    rr = np.zeros(1, dtype=np.float64)
    it = lib().or_solve_box(_ptr(L4), int(tbc), float(kappa), _ptr(U), _ptr(o), _ptr(e), _ptr(b),
                            _ptr(x), float(tol), int(maxit), _ptr(rr))
    return x, int(it), float(rr[0])


def solve_many(L, tbc, kappa, U, boxes, b, tol=1e-12, maxit=5000, nthreads=0):
    """Independent solves for every (block, rhs) pair.

    boxes: int [n_blk, 8] (origin, extent); b: complex [n_rhs, sum_b S_b, 4, 3].
    Returns (x, iters[n_rhs, n_blk], relres[n_rhs, n_blk], n_failed).
    """
    L4 = _i4(L)
    bx = _i4(boxes)
    nblk = bx.size // 8
    U = _c128(U)
    b = _c128(b)
    nrhs = b.shape[0]
    x = np.zeros_like(b)
    iters = np.zeros(nrhs * nblk, dtype=np.int32)
    rel = np.zeros(nrhs * nblk, dtype=np.float64)
    fails = lib().or_solve_many(_ptr(L4), int(tbc), float(kappa), _ptr(U), int(nblk), _ptr(bx),
                                int(nrhs), _ptr(b), _ptr(x), float(tol), int(maxit), _ptr(iters),
                                _ptr(rel), int(nthreads))
    return x, iters.reshape(nrhs, nblk), rel.reshape(nrhs, nblk), int(fails)


def num_threads() -> int:
    return int(lib().or_num_threads())
