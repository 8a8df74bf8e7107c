"""The Schur-complement pieces of the factorisation of Section 3 as dense
matrices (oracle, tiny lattices only).  Test infrastructure only.

Notation of Section 3 with the domains of Section 2 (geometry.PaperDomains or
geometry.BoxDomains): dLambda_0 = union of the internal boundaries,
Lambda0bar = active bulk, Lambda_1 = inactive rest, dPi_1 = hyperplane sites
in Lambda_1, Lambda1bar = Lambda_1 minus dPi_1, Phi_1^a the frames.

Defined exactly (first Schur step):
  Dtilde = D_{dL0} - D_{dL0,L0bar} D_{L0bar}^{-1} D_{L0bar,dL0} - D_{dL0,L1} D_{L1}^{-1} D_{L1,dL0}
  Dhat^d = sum_a Dhat_{dL0^a},
  Dhat_{dL0^a} = D_{dL0^a} - D_{dL0^a,L0bar^a} D_{L0bar^a}^{-1} D_{L0bar^a,dL0^a}
                 - D_{dL0^a,Phi^a} D_{Phi^a}^{-1} D_{Phi^a,dL0^a}
  Dhat_{dPi1} = D_{dPi1} - D_{dPi1,L1bar} D_{L1bar}^{-1} D_{L1bar,dPi1}    (D_{L1bar}^{-1}: the
                Schur complement must eliminate Lambda1bar, not Lambda_1)
  Dhat_{dL0,dPi1} = - sum_a D_{dL0^a,Phi^a} D_{Phi^a}^{-1} D_{Phi^a, dOmega^{a*}}
                (so that [Dhat^d]^{-1} Dhat_{dL0,dPi1} is the W_{dL0,dPi1} of eq. offdiagW1).

The hopping term Dhat^h and Dhat_{dPi1,dL0} are printed garbled or not
defined.  Reading taken: for a != a',
  Dhat^h_{aa'}     = - D_{dL0^a,Phi^a} D_{Phi^a}^{-1} P_{Phi^a} D_{Phi^{a'},dL0^{a'}},
  Dhat_{dPi1,dL0}  = D_{dPi1,dL0} - D_{dPi1,L1bar} D_{L1bar}^{-1} D_{L1bar,dL0}.
It follows from splitting Lambda_1 = Phi^a u (Lambda_1 minus Phi^a), whose
coupling goes through dOmega^{a*} only: for y supported on Lambda_1,
  (D_{L1}^{-1} y)|_{Phi^a} = D_{Phi^a}^{-1} (P_{Phi^a} y - D_{Phi^a,dOmega^{a*}} (D_{L1}^{-1} y)|_{dOmega^{a*}}),
and (D_{L1}^{-1} y)|_{dPi1} = Dhat_{dPi1}^{-1} (y - D_{dPi1,L1bar} D_{L1bar}^{-1} y)|_{dPi1}; with it
  Dtilde = Dhat^d + Dhat^h - Dhat_{dL0,dPi1} Dhat_{dPi1}^{-1} Dhat_{dPi1,dL0}
holds exactly, which is the second decomposition of Section 3.  In one
dimension (dPi_1 empty) Dhat^h equals the printed bracket term for term.
W_z of eq. (Wz) is assembled from these pieces (rows and columns dL0, then dPi1).

Row/column order of every matrix: sites in increasing canonical index (the
order of the masks' nonzeros), 12 components each.
"""
from __future__ import annotations

import numpy as np

from . import dense

__all__ = ["pieces", "printed_dhat_h", "w_z"]


def _inv_apply(M, X, Y):
    return np.linalg.solve(M, Y) if M.shape[0] else np.zeros((0, Y.shape[1]), dtype=Y.dtype)


def pieces(M, P):
    """Dense pieces of the decomposition for the full matrix M of D on the lattice of the domains P.

    Returns a dict with the site lists ("dl0", "dp1"), "Dtilde", "Dd", "Dh", "Bl" (Dhat_{dL0,dPi1}),
    "Dp" (Dhat_{dPi1}), "Kp" (Dhat_{dPi1,dL0}) and "blk" (for each block the positions of its
    dLambda_0^a sites in dl0).
    """
    s = P.sites
    dl0, l0b, l1, dp1 = s(P.dlam0), s(P.lam0bar), s(P.lam1), s(P.dPi1)
    l1b = s(P.lam1 & ~P.dPi1)
    sub = lambda r, c=None: dense.sub(M, r, c)  # noqa: E731
    Dt = sub(dl0)
    if l0b.size:
        Dt = Dt - sub(dl0, l0b) @ np.linalg.solve(sub(l0b), sub(l0b, dl0))
    Dt = Dt - sub(dl0, l1) @ np.linalg.solve(sub(l1), sub(l1, dl0))
    n0, n1 = 12 * dl0.size, 12 * dp1.size
    pos0 = {int(v): i for i, v in enumerate(dl0)}
    pos1 = {int(v): i for i, v in enumerate(dp1)}
    Dd = np.zeros((n0, n0), dtype=complex)
    Dh = np.zeros((n0, n0), dtype=complex)
    Bl = np.zeros((n0, n1), dtype=complex)
    nb = len(P.lam0_a)
    dl = [s(m) for m in P.dlam0_a]
    bulk = [s(m & ~d) for m, d in zip(P.lam0_a, P.dlam0_a)]
    ph = [s(m) for m in P.phi_a]
    ext_star = [s(e & P.dPi1) for e in (P.ext_omega_a if hasattr(P, "ext_omega_a") else P.ext_a)]
    rows = [dense.dof(np.array([pos0[int(v)] for v in d], dtype=np.int64)) for d in dl]
    for a in range(nb):
        H = sub(dl[a])
        if bulk[a].size:
            H = H - sub(dl[a], bulk[a]) @ np.linalg.solve(sub(bulk[a]), sub(bulk[a], dl[a]))
        if ph[a].size:
            H = H - sub(dl[a], ph[a]) @ np.linalg.solve(sub(ph[a]), sub(ph[a], dl[a]))
        Dd[np.ix_(rows[a], rows[a])] = H
        if ext_star[a].size:
            cols = dense.dof(np.array([pos1[int(v)] for v in ext_star[a]], dtype=np.int64))
            Bl[np.ix_(rows[a], cols)] += -sub(dl[a], ph[a]) @ np.linalg.solve(sub(ph[a]), sub(ph[a], ext_star[a]))
    for a in range(nb):
        if not ph[a].size:
            continue
        # P_{Phi^a} D_{Phi^{a'}, dL0^{a'}} = D_{Phi^a, dL0^{a'}} (every Lambda_1 neighbour of
        # dLambda_0^{a'} lies in Phi^{a'})
        G = np.linalg.solve(sub(ph[a]), np.eye(12 * ph[a].size))
        left = -sub(dl[a], ph[a]) @ G
        for b in range(nb):
            if b != a:
                Dh[np.ix_(rows[a], rows[b])] = left @ sub(ph[a], dl[b])
    if n1:
        Dp = sub(dp1)
        Kp = sub(dp1, dl0)
        if l1b.size:
            Dp = Dp - sub(dp1, l1b) @ np.linalg.solve(sub(l1b), sub(l1b, dp1))
            Kp = Kp - sub(dp1, l1b) @ np.linalg.solve(sub(l1b), sub(l1b, dl0))
    else:
        Dp = np.zeros((0, 0), dtype=complex)
        Kp = np.zeros((0, n0), dtype=complex)
    return {"dl0": dl0, "dp1": dp1, "Dtilde": Dt, "Dd": Dd, "Dh": Dh, "Bl": Bl, "Dp": Dp, "Kp": Kp,
            "blk": rows}


def printed_dhat_h(M, P):
    """The hopping term as printed in Section 3, read with every D_{Phi}^{-1} zero-extended to the
    lattice:  Dhat_{aa'} = -1/2 D_{dL0^a,Phi^a} [ D_{Phi^a}^{-1} - D_{Phi^a}^{-1} D_{Phi^a,dOmega^{a*}}
    D_{Phi^{a'}}^{-1} + D_{Phi^{a'}}^{-1} - D_{Phi^a}^{-1} D_{dOmega^{a'*},Phi^{a'}} D_{Phi^{a'}}^{-1} ]
    D_{Phi^{a'},dL0^{a'}} (a != a'), in the dl0 order of pieces().  Each term is applied to the
    columns D_{Phi^{a'},dL0^{a'}} as lattice-wide vectors."""
    s = P.sites
    dl0 = s(P.dlam0)
    N = 12 * P.V
    pos0 = {int(v): i for i, v in enumerate(dl0)}
    nb = len(P.lam0_a)
    dl = [s(m) for m in P.dlam0_a]
    ph = [s(m) for m in P.phi_a]
    exts = P.ext_omega_a if hasattr(P, "ext_omega_a") else P.ext_a
    est = [s(e & P.dPi1) for e in exts]
    fi = [dense.dof(v) for v in ph]
    ei = [dense.dof(v) for v in est]

    def zinv(a, Y):  # D_{Phi^a}^{-1} P_{Phi^a} Y, zero outside Phi^a
        out = np.zeros_like(Y)
        if fi[a].size:
            out[fi[a]] = np.linalg.solve(M[np.ix_(fi[a], fi[a])], Y[fi[a]])
        return out

    def hop(rows, cols, Y):  # D_{rows, cols} Y[cols], zero outside rows
        out = np.zeros_like(Y)
        if rows.size and cols.size:
            out[rows] = M[np.ix_(rows, cols)] @ Y[cols]
        return out

    out = np.zeros((12 * dl0.size, 12 * dl0.size), dtype=complex)
    for b in range(nb):
        db = dense.dof(dl[b])
        rb = dense.dof(np.array([pos0[int(v)] for v in dl[b]], dtype=np.int64))
        Y0 = np.zeros((N, db.size), dtype=complex)
        Y0[fi[b]] = M[np.ix_(fi[b], db)]  # D_{Phi^b, dL0^b}
        Wb = zinv(b, Y0)  # D_{Phi^b}^{-1} D_{Phi^b, dL0^b}
        for a in range(nb):
            if a == b:
                continue
            ra = dense.dof(np.array([pos0[int(v)] for v in dl[a]], dtype=np.int64))
            t1 = zinv(a, Y0)
            t2 = zinv(a, hop(fi[a], ei[a], Wb))
            t3 = np.zeros_like(Wb)
            t3[fi[a]] = Wb[fi[a]]
            t4 = zinv(a, hop(ei[b], fi[b], Wb))
            br = t1 - t2 + t3 - t4
            out[np.ix_(ra, rb)] = -0.5 * M[np.ix_(dense.dof(dl[a]), fi[a])] @ br[fi[a]]
    return out


def w_z(pc, z):
    """W_z of eq. (Wz) on dL0 u dPi1 (rows/columns dl0 first):
    [[z + Dd^{-1} Dh, Dd^{-1} Bl], [Dp^{-1} Kp, z]]."""
    n0, n1 = pc["Dd"].shape[0], pc["Dp"].shape[0]
    W = np.zeros((n0 + n1, n0 + n1), dtype=complex)
    W[:n0, :n0] = z * np.eye(n0) + np.linalg.solve(pc["Dd"], pc["Dh"])
    if n1:
        W[:n0, n0:] = np.linalg.solve(pc["Dd"], pc["Bl"])
        W[n0:, :n0] = np.linalg.solve(pc["Dp"], pc["Kp"])
        W[n0:, n0:] = z * np.eye(n1)
    return W
