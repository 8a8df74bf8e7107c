"""Block-local multi-boson action (oracle).  Test infrastructure only.

Section 4 writes the multi-boson action |W_z chi|^2 as a sum of block-local
terms S_MB^a plus a global rest.  The block-local term is the squared norm, on
the internal boundary dLambda_0^a, of
    z chi + [Dhat_{dLambda_0^a}]^{-1} Dhat^h chi + D_{Omega_0^a}^{-1} D_{Phi_1^a, dOmega^{a*}} chi.
Reading used here:
  * field k is taken at z = u_k (because z_k - W_1 = -W_{u_k});
  * [Dhat_{dLambda_0^a}]^{-1} equals the dLambda_0^a block of D_{Omega_0^a}^{-1}
    (Dhat_{dLambda_0^a} is the Schur complement of D_{Omega_0^a} onto
    dLambda_0^a, since the block bulk and the frame do not touch), so both
    operator terms are one solve with D_{Omega_0^a} restricted to dLambda_0^a;
  * the caller supplies the source xi_k^a on Omega_0^a that collects both
    hop-in terms (the one through Dhat^h depends on inactive links only).
Hence  S^a = sum_k sum_{x in dLambda_0^a} |u_k chi_k(x) + (D_{Omega_0^a}^{-1} xi_k^a)(x)|^2.
"""
from __future__ import annotations

import numpy as np

from . import geometry, wilson

__all__ = ["boundary_lists", "mb_local_action"]


def boundary_lists(L, boxes, inner):
    """dLambda_0^a as box-local canonical indices for every block.

    inner[b] = (offset[4], extent[4]) of the active box inside block b.
    """
    out = []
    for b in range(len(boxes)):
        out.append(geometry.inner_boundary_local(L, boxes[b], inner[b][:4], inner[b][4:8]))
    return out


def mb_local_action(L, tbc, kappa, U, boxes, inner, u, chi, xi, tol=1e-12, nthreads=0):
    """Per-block actions S^a and their sum.

    boxes [nb, 8]; inner [nb, 8]; u [n_fields] complex;
    chi [n_fields, sum_b |dLambda_0^b|, 4, 3]; xi [n_fields, sum_b S_b, 4, 3].
    """
    boxes = np.asarray(boxes, dtype=np.int32).reshape(-1, 8)
    nb = boxes.shape[0]
    u = np.asarray(u, dtype=np.complex128).reshape(-1)
    nf = u.size
    chi = np.asarray(chi, dtype=np.complex128)
    xi = np.asarray(xi, dtype=np.complex128)
    y, _, rel, fails = wilson.solve_many(L, tbc, kappa, U, boxes, xi, tol=tol, nthreads=nthreads)
    if fails:
        raise RuntimeError("oracle block solve did not converge")
    bl = boundary_lists(L, boxes, inner)
    S = np.zeros(nb, dtype=np.float64)
    soff = 0
    boff = 0
    for b in range(nb):
        Sb = int(np.prod(boxes[b, 4:8]))
        nbd = bl[b].size
        for k in range(nf):
            v = u[k] * chi[k, boff:boff + nbd] + y[k, soff + bl[b]]
            S[b] += float(np.sum(np.abs(v) ** 2))
        soff += Sb
        boff += nbd
    return S, float(np.sum(S))
