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
``default_rng(seed)``; U = exp(i eps H), unitary with det U = 1 (tr H = 0).
The exponential of the traceless Hermitian 3x3 matrix Q = eps H is evaluated
exactly by the Cayley-Hamilton form exp(iQ) = f0 + f1 Q + f2 Q^2 with the
coefficients of Morningstar and Peardon (Phys. Rev. D 69 (2004) 054501),
vectorised over links; it agrees with an eigendecomposition to rounding.

Sources: real and imaginary parts iid N(0,1), drawn as one array of shape
[n_rhs, V, 4, 3, 2] (last axis re, im).
"""
from __future__ import annotations

import concurrent.futures
import os

import numpy as np

__all__ = [
    "gell_mann",
    "volume",
    "site_index",
    "gauge_field",
    "gauge_field_device",
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


def _expi_cayley_hamilton(Q: np.ndarray) -> np.ndarray:
    """exp(iQ) for traceless Hermitian Q[n,3,3] (Cayley-Hamilton form)."""
    d0, d1, d2 = Q[:, 0, 0].real, Q[:, 1, 1].real, Q[:, 2, 2].real
    q01, q02, q12 = Q[:, 0, 1], Q[:, 0, 2], Q[:, 1, 2]
    a01, a02, a12 = np.abs(q01) ** 2, np.abs(q02) ** 2, np.abs(q12) ** 2
    # Q^2 (Hermitian): diagonal and upper triangle
    s00 = d0 * d0 + a01 + a02
    s11 = d1 * d1 + a01 + a12
    s22 = d2 * d2 + a02 + a12
    s01 = q01 * (d0 + d1) + q02 * np.conj(q12)
    s02 = q02 * (d0 + d2) + q01 * q12
    s12 = np.conj(q01) * q02 + q12 * (d1 + d2)
    c1 = 0.5 * (s00 + s11 + s22)
    c0 = d0 * d1 * d2 + 2 * np.real(q01 * q12 * np.conj(q02)) - d0 * a12 - d1 * a02 - d2 * a01
    neg = c0 < 0
    c0 = np.abs(c0)
    with np.errstate(divide="ignore", invalid="ignore", under="ignore"):
        c1s = np.maximum(c1, 1e-300)
        c0max = 2.0 * (c1s / 3.0) ** 1.5
        theta = np.arccos(np.clip(np.where(c0max > 0, c0 / c0max, 1.0), -1.0, 1.0))
        u = np.sqrt(c1s / 3.0) * np.cos(theta / 3.0)
        w = np.sqrt(c1s) * np.sin(theta / 3.0)
        w2 = w * w
        small = np.abs(w) < 0.05
        xi0 = np.where(small, 1 - w2 / 6 * (1 - w2 / 20 * (1 - w2 / 42)), np.sin(w) / np.where(small, 1.0, w))
        e2iu = np.exp(2j * u)
        emiu = np.exp(-1j * u)
        cw = np.cos(w)
        u2 = u * u
        den = 9 * u2 - w2
        f0 = ((u2 - w2) * e2iu + emiu * (8 * u2 * cw + 2j * u * (3 * u2 + w2) * xi0)) / den
        f1 = (2 * u * e2iu - emiu * (2 * u * cw - 1j * (3 * u2 - w2) * xi0)) / den
        f2 = (e2iu - emiu * (cw + 3j * u * xi0)) / den
    # c0 < 0: f_j(-c0) = (-1)^j conj(f_j(c0))
    f0 = np.where(neg, np.conj(f0), f0)
    f1 = np.where(neg, -np.conj(f1), f1)
    f2 = np.where(neg, np.conj(f2), f2)
    zero = c1 < 1e-30
    f0 = np.where(zero, 1.0, f0)
    f1 = np.where(zero, 0.0, f1)
    f2 = np.where(zero, 0.0, f2)
    out = np.empty((Q.shape[0], 3, 3), dtype=np.complex128)
    out[:, 0, 0] = f0 + f1 * d0 + f2 * s00
    out[:, 1, 1] = f0 + f1 * d1 + f2 * s11
    out[:, 2, 2] = f0 + f1 * d2 + f2 * s22
    out[:, 0, 1] = f1 * q01 + f2 * s01
    out[:, 0, 2] = f1 * q02 + f2 * s02
    out[:, 1, 2] = f1 * q12 + f2 * s12
    out[:, 1, 0] = f1 * np.conj(q01) + f2 * np.conj(s01)
    out[:, 2, 0] = f1 * np.conj(q02) + f2 * np.conj(s02)
    out[:, 2, 1] = f1 * np.conj(q12) + f2 * np.conj(s12)
    return out


def gauge_field(L, eps: float, seed: int, chunk: int = 1 << 16) -> np.ndarray:
    """SU(3) link field U[V,4,3,3] = exp(i eps H), H Gaussian traceless Hermitian."""
    V = volume(L)
    rng = np.random.default_rng(seed)
    U = np.empty((V, 4, 3, 3), dtype=np.complex128)
    Uf = U.reshape(V * 4, 3, 3)
    lam = gell_mann() * (0.5 * eps)
    lam_flat = lam.reshape(8, 9)

    def work(s, h):
        Q = (h @ lam_flat).reshape(h.shape[0], 3, 3)
        Uf[s:s + h.shape[0]] = _expi_cayley_hamilton(Q)

    # the normals are drawn in (site, mu, a) order, chunk by chunk; the
    # exponentials of different chunks are independent and run in threads
    nthr = max(1, min(16, os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(nthr) as ex:
        futs = []
        for s in range(0, V * 4, chunk):
            e = min(s + chunk, V * 4)
            futs.append(ex.submit(work, s, rng.standard_normal((e - s, 8))))
            if len(futs) >= 2 * nthr:
                futs.pop(0).result()
        for f in futs:
            f.result()
    return U


def _expi_cayley_hamilton_torch(Q):
    """exp(iQ) for traceless Hermitian Q[n,3,3] (torch complex128), the same
    Cayley-Hamilton form as _expi_cayley_hamilton, evaluated on Q's device."""
    import torch

    d0, d1, d2 = Q[:, 0, 0].real, Q[:, 1, 1].real, Q[:, 2, 2].real
    q01, q02, q12 = Q[:, 0, 1], Q[:, 0, 2], Q[:, 1, 2]
    a01, a02, a12 = q01.abs() ** 2, q02.abs() ** 2, q12.abs() ** 2
    s00 = d0 * d0 + a01 + a02
    s11 = d1 * d1 + a01 + a12
    s22 = d2 * d2 + a02 + a12
    s01 = q01 * (d0 + d1) + q02 * q12.conj()
    s02 = q02 * (d0 + d2) + q01 * q12
    s12 = q01.conj() * q02 + q12 * (d1 + d2)
    c1 = 0.5 * (s00 + s11 + s22)
    c0 = d0 * d1 * d2 + 2 * (q01 * q12 * q02.conj()).real - d0 * a12 - d1 * a02 - d2 * a01
    neg = c0 < 0
    c0 = c0.abs()
    c1s = torch.clamp(c1, min=1e-300)
    c0max = 2.0 * (c1s / 3.0) ** 1.5
    theta = torch.arccos(torch.clamp(c0 / c0max, -1.0, 1.0))
    u = torch.sqrt(c1s / 3.0) * torch.cos(theta / 3.0)
    w = torch.sqrt(c1s) * torch.sin(theta / 3.0)
    w2 = w * w
    small = w.abs() < 0.05
    xi0 = torch.where(small, 1 - w2 / 6 * (1 - w2 / 20 * (1 - w2 / 42)),
                      torch.sin(w) / torch.where(small, torch.ones_like(w), w))
    e2iu = torch.exp(2j * u)
    emiu = torch.exp(-1j * u)
    cw = torch.cos(w)
    u2 = u * u
    den = 9 * u2 - w2
    f0 = ((u2 - w2) * e2iu + emiu * (8 * u2 * cw + 2j * u * (3 * u2 + w2) * xi0)) / den
    f1 = (2 * u * e2iu - emiu * (2 * u * cw - 1j * (3 * u2 - w2) * xi0)) / den
    f2 = (e2iu - emiu * (cw + 3j * u * xi0)) / den
    f0 = torch.where(neg, f0.conj(), f0)
    f1 = torch.where(neg, -f1.conj(), f1)
    f2 = torch.where(neg, f2.conj(), f2)
    zero = c1 < 1e-30
    f0 = torch.where(zero, torch.ones_like(f0), f0)
    f1 = torch.where(zero, torch.zeros_like(f1), f1)
    f2 = torch.where(zero, torch.zeros_like(f2), f2)
    out = torch.empty((Q.shape[0], 3, 3), dtype=torch.complex128, device=Q.device)
    out[:, 0, 0] = f0 + f1 * d0 + f2 * s00
    out[:, 1, 1] = f0 + f1 * d1 + f2 * s11
    out[:, 2, 2] = f0 + f1 * d2 + f2 * s22
    out[:, 0, 1] = f1 * q01 + f2 * s01
    out[:, 0, 2] = f1 * q02 + f2 * s02
    out[:, 1, 2] = f1 * q12 + f2 * s12
    out[:, 1, 0] = f1 * q01.conj() + f2 * s01.conj()
    out[:, 2, 0] = f1 * q02.conj() + f2 * s02.conj()
    out[:, 2, 1] = f1 * q12.conj() + f2 * s12.conj()
    return out


def gauge_field_device(L, eps: float, seed: int, device="cuda", chunk: int = 1 << 22):
    """SU(3) link field U[V,4,3,3] = exp(i eps H) (torch complex128 on a torch
    device), H = sum_a h_a lambda_a / 2 with h_a iid N(0,1) drawn by torch's
    seeded generator for that device, in (site, mu, a) order chunk by chunk.
    For lattices too large to draw on the host; the values are a function of
    (L, eps, seed, device type) only and differ from gauge_field's."""
    import torch

    V = volume(L)
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    lam = torch.from_numpy(gell_mann().reshape(8, 9) * (0.5 * eps)).to(device)
    U = torch.empty((V * 4, 3, 3), dtype=torch.complex128, device=device)
    for s in range(0, V * 4, chunk):
        e = min(s + chunk, V * 4)
        h = torch.randn((e - s, 8), generator=g, dtype=torch.float64, device=device)
        Q = (h.to(torch.complex128) @ lam).reshape(e - s, 3, 3)
        U[s:e] = _expi_cayley_hamilton_torch(Q)
    return U.reshape(V, 4, 3, 3)


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


def spinor_field_device(n_rhs: int, n_sites: int, seed: int, device="cuda"):
    """Gaussian complex spinors [n_rhs, n_sites, 4, 3] (complex128) drawn on a
    torch device by torch's seeded generator for that device (re, im
    interleaved on a trailing axis).  For workloads whose sources are too large
    to draw on the host; the values are a function of (seed, device type) only."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    z = torch.randn((n_rhs, n_sites, 4, 3, 2), generator=g, dtype=torch.float64, device=device)
    return torch.view_as_complex(z)


def convnet_weights(seed: int, scale: float = 0.1, identity: bool = True) -> np.ndarray:
    """Initial FP32 weights of the 24 -> 32 -> 32 -> 24 block network, layers
    back to back, each [81][c_in][c_out]: Gaussian with standard deviation
    scale / sqrt(81 c_in), plus (identity=True) the identity between the first
    min(c_in, c_out) channels on the centre tap, so that the untrained linear
    network is close to the identity map."""
    rng = np.random.default_rng(seed)
    out = []
    for cin, cout in ((24, 32), (32, 32), (32, 24)):
        w = rng.standard_normal((81, cin, cout)) * (scale / np.sqrt(81 * cin))
        if identity:
            k = min(cin, cout)
            w[40, np.arange(k), np.arange(k)] += 1.0
        out.append(w.reshape(-1))
    return np.concatenate(out).astype(np.float32)


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
