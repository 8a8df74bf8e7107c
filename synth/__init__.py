"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module draws random numbers and builds the input fields only: it holds
none of the method's arithmetic (no Dirac operator, no solver, no action).
Both the CPU oracle and the HIP library consume what it returns.

Conventions (fixed here so every consumer agrees):
  * Lattice L = (L0, L1, L2, L3), direction 0 is time.
  * Canonical site index n = ((x0*L1 + x1)*L2 + x2)*L3 + x3 (x3 fastest).
  * Link field U[n, mu, row, col], complex128; U_mu(x) sits on the link
    (x, x + mu_hat) (Section 1 of the paper places links between adjacent
    sites).
  * Spinor field psi[n, spin(4), colour(3)], complex128.

Gauge field: H(x,mu) = sum_a h_a lambda_a / 2 with h_a iid N(0,1) (lambda_a
the Gell-Mann matrices), drawn in the order site, mu, a from numpy PCG64
``default_rng(seed)``; U = exp(i eps H) through an FP64 eigendecomposition,
so U is unitary with det U = 1 (tr H = 0).

Sources: real and imaginary parts iid N(0,1), drawn as one array of shape
[n_rhs, V, 4, 3, 2] (last axis re, im).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gell_mann",
    "volume",
    "site_index",
    "gauge_field",
    "unit_gauge",
    "spinor_field",
    "random_su3",
]


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices lambda_1..lambda_8 as a [8,3,3] array."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    s3 = 1.0 / np.sqrt(3.0)
    lam[7][0, 0] = s3
    lam[7][1, 1] = s3
    lam[7][2, 2] = -2 * s3
    return lam


def volume(L) -> int:
    L = tuple(int(v) for v in L)
    return L[0] * L[1] * L[2] * L[3]


def site_index(L, x0, x1, x2, x3):
    """Canonical site index (x3 fastest); works on ints or numpy arrays."""
    return ((x0 * L[1] + x1) * L[2] + x2) * L[3] + x3


def _expi_hermitian(H: np.ndarray, eps: float) -> np.ndarray:
    w, v = np.linalg.eigh(H)
    return (v * np.exp(1j * eps * w)[..., None, :]) @ np.conj(np.swapaxes(v, -1, -2))


def gauge_field(L, eps: float, seed: int, chunk: int = 1 << 19) -> np.ndarray:
    """SU(3) link field U[V,4,3,3] = exp(i eps H), H Gaussian traceless Hermitian."""
    V = volume(L)
    rng = np.random.default_rng(seed)
    h = rng.standard_normal((V, 4, 8))
    lam_half = gell_mann() / 2.0
    U = np.empty((V, 4, 3, 3), dtype=np.complex128)
    hf = h.reshape(V * 4, 8)
    Uf = U.reshape(V * 4, 3, 3)
    for s in range(0, V * 4, chunk):
        e = min(s + chunk, V * 4)
        H = np.einsum("na,aij->nij", hf[s:e], lam_half)
        Uf[s:e] = _expi_hermitian(H, eps)
    return U


def unit_gauge(L) -> np.ndarray:
    V = volume(L)
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1
    return U


def spinor_field(L, n_rhs: int, seed: int) -> np.ndarray:
    """Gaussian complex spinors psi[n_rhs, V, 4, 3]."""
    V = volume(L)
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n_rhs, V, 4, 3, 2))
    return z[..., 0] + 1j * z[..., 1]


def gaussian_complex(shape, seed: int) -> np.ndarray:
    """Generic Gaussian complex array (re, im interleaved on a trailing axis)."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(tuple(shape) + (2,))
    return z[..., 0] + 1j * z[..., 1]


def random_su3(n: int, seed: int) -> np.ndarray:
    """n Haar-ish SU(3) matrices (QR of a Gaussian matrix, phases fixed, det 1)."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q[:, :, 0] /= det[:, None]
    return q
