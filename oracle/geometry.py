"""Domain decomposition geometry (oracle, pure numpy).  Test infrastructure only.

Paper Section 2 builds the overlapping decomposition in three steps:
  1. active hyperrectangular blocks Lambda_0^a, their union Lambda_0 (disconnected)
     and the connected inactive rest Lambda_1;
  2. internal block boundaries dLambda_0^a (sites of a block that touch its
     outside), the hyperplanes dPi holding them, and dPi_1 = dPi \\ dLambda_0;
  3. frames Phi_1^a inside Lambda_1 and framed blocks Omega_0^a = Lambda_0^a u Phi_1^a,
     with exterior boundary dOmega_0^a and its part dOmega_0^{a*} on dPi_1.
The paper defers the precise shapes to an appendix of another article, which
is not available; the reading used here ("box reading") is:
  * per decomposed direction an active extent b and a gap d >= 1; blocks start
    at multiples of b + d; a direction may be left undecomposed (full extent);
  * dPi = sites with some decomposed coordinate equal to a block-face
    coordinate s or s + b - 1;
  * Omega_0^a = the box [s - d, s + b - 1 + d] in the decomposed directions;
    Phi_1^a = Omega_0^a \\ Lambda_0^a.

Tile mode (the benchmark blocks) simply tiles the lattice with boxes.

Ordering conventions (shared with the library by specification, not code):
  * blocks of a tiling are listed with the tile coordinate of direction 3
    fastest, direction 0 slowest;
  * sites inside a box are in box-local canonical order (local x3 fastest);
  * even-odd order inside a box: the sites of even global parity first, then
    the odd ones, each in box-local canonical order.
"""
from __future__ import annotations

import itertools

import numpy as np

__all__ = [
    "volume",
    "coords",
    "neighbours",
    "tile_boxes",
    "box_sites",
    "box_mask",
    "box_parity",
    "box_eo_order",
    "inner_boundary_local",
    "boundary_of",
    "exterior_boundary_of",
    "PaperDomains",
    "BoxDomains",
]


def volume(L) -> int:
    return int(np.prod([int(v) for v in L]))


def coords(L) -> np.ndarray:
    """Global coordinates [V, 4] of every site in canonical order."""
    L = [int(v) for v in L]
    g = np.indices(L).reshape(4, -1).T
    return g.astype(np.int64)


def _index(L, x):
    return ((x[..., 0] * L[1] + x[..., 1]) * L[2] + x[..., 2]) * L[3] + x[..., 3]


def neighbours(L) -> np.ndarray:
    """[V, 8] global neighbours: columns 2*mu = x + mu, 2*mu + 1 = x - mu (periodic)."""
    L = [int(v) for v in L]
    x = coords(L)
    out = np.empty((x.shape[0], 8), dtype=np.int64)
    for mu in range(4):
        for k, step in enumerate((1, -1)):
            y = x.copy()
            y[:, mu] = (y[:, mu] + step) % L[mu]
            out[:, 2 * mu + k] = _index(L, y)
    return out


def tile_boxes(L, segs, shift=(0, 0, 0, 0)) -> np.ndarray:
    """Boxes [n, 8] (origin, extent) of a tiling.

    segs[mu] lists the consecutive tile extents along direction mu (they must
    sum to L[mu]); tiles start at shift[mu] and wrap around the lattice.
    """
    L = [int(v) for v in L]
    starts, exts = [], []
    for mu in range(4):
        s = [int(v) for v in segs[mu]]
        if sum(s) != L[mu] or min(s) < 1:
            raise ValueError("tile extents along direction %d must be >= 1 and sum to %d" % (mu, L[mu]))
        o = np.concatenate([[0], np.cumsum(s)[:-1]])
        starts.append([(int(v) + int(shift[mu])) % L[mu] for v in o])
        exts.append(s)
    boxes = []
    for t in itertools.product(*[range(len(exts[m])) for m in range(4)]):
        boxes.append([starts[m][t[m]] for m in range(4)] + [exts[m][t[m]] for m in range(4)])
    return np.asarray(boxes, dtype=np.int32).reshape(-1, 8)


def box_sites(L, origin, extent) -> np.ndarray:
    """Global site index of every box site, in box-local canonical order."""
    L = [int(v) for v in L]
    e = [int(v) for v in extent]
    y = np.indices(e).reshape(4, -1).T
    x = (y + np.asarray(origin, dtype=np.int64)[None, :]) % np.asarray(L)[None, :]
    return _index(L, x)


def box_mask(L, origin, extent) -> np.ndarray:
    m = np.zeros(volume(L), dtype=bool)
    m[box_sites(L, origin, extent)] = True
    return m


def box_parity(L, origin, extent) -> np.ndarray:
    """Global parity (x0+x1+x2+x3) mod 2 of the box sites, box-local canonical order."""
    x = coords(L)[box_sites(L, origin, extent)]
    return (x.sum(axis=1) % 2).astype(np.int32)


def box_eo_order(L, origin, extent):
    """Even-odd order of a box.

    Returns (perm, pos): perm[k] = box-local canonical index of the k-th site
    in even-odd order; pos[i] = even-odd position of canonical site i.
    """
    par = box_parity(L, origin, extent)
    perm = np.concatenate([np.nonzero(par == 0)[0], np.nonzero(par == 1)[0]]).astype(np.int64)
    pos = np.empty_like(perm)
    pos[perm] = np.arange(perm.size)
    return perm, pos


def boundary_of(mask: np.ndarray, nbr: np.ndarray) -> np.ndarray:
    """Sites of a set with at least one neighbour outside it (internal boundary)."""
    return mask & np.any(~mask[nbr], axis=1)


def exterior_boundary_of(mask: np.ndarray, nbr: np.ndarray) -> np.ndarray:
    """Sites outside a set with at least one neighbour inside it."""
    return (~mask) & np.any(mask[nbr], axis=1)


def inner_boundary_local(L, box, inner_off, inner_ext) -> np.ndarray:
    """Box-local canonical indices of dLambda_0 for an inner box of a block.

    The inner (active) box starts inner_off sites into the block and has extent
    inner_ext; its boundary is the set of its sites with a lattice neighbour
    outside it.
    """
    L = [int(v) for v in L]
    o = np.asarray(box[:4], dtype=np.int64)
    e = [int(v) for v in box[4:8]]
    io = o + np.asarray(inner_off, dtype=np.int64)
    inner = box_mask(L, io, inner_ext)
    bnd = boundary_of(inner, neighbours(L))
    sites = box_sites(L, o, e)
    return np.nonzero(bnd[sites])[0].astype(np.int64)


class PaperDomains:
    """The sets of Section 2 on a small lattice, as boolean masks over sites.

    spec[mu] is None (direction not decomposed) or (b, d): active extent b and
    gap d >= 1 with L[mu] divisible by b + d.
    """

    def __init__(self, L, spec):
        self.L = [int(v) for v in L]
        self.spec = spec
        V = volume(self.L)
        self.V = V
        self.nbr = neighbours(self.L)
        starts = []
        for mu in range(4):
            if spec[mu] is None:
                starts.append([None])
            else:
                b, d = spec[mu]
                if d < 1 or self.L[mu] % (b + d) != 0:
                    raise ValueError("direction %d: need d >= 1 and (b+d) | L" % mu)
                starts.append(list(range(0, self.L[mu], b + d)))
        self.blocks = []  # list of dicts with lambda0 and omega boxes
        for t in itertools.product(*starts):
            lo, le, oo, oe = [], [], [], []
            for mu in range(4):
                if spec[mu] is None:
                    lo.append(0); le.append(self.L[mu]); oo.append(0); oe.append(self.L[mu])
                else:
                    b, d = spec[mu]
                    lo.append(t[mu]); le.append(b)
                    oo.append((t[mu] - d) % self.L[mu]); oe.append(b + 2 * d)
            self.blocks.append({"lambda0": (lo, le), "omega": (oo, oe)})
        x = coords(self.L)
        # dPi: some decomposed coordinate on a block face (s or s + b - 1)
        dpi = np.zeros(V, dtype=bool)
        for mu in range(4):
            if spec[mu] is None:
                continue
            b, _ = spec[mu]
            faces = set()
            for s in range(0, self.L[mu], b + spec[mu][1]):
                faces.add(s)
                faces.add(s + b - 1)
            dpi |= np.isin(x[:, mu], sorted(faces))
        self.dPi = dpi
        self.lam0_a = [box_mask(self.L, *blk["lambda0"]) for blk in self.blocks]
        self.omega_a = [box_mask(self.L, *blk["omega"]) for blk in self.blocks]
        self.lam0 = np.any(self.lam0_a, axis=0)
        self.lam1 = ~self.lam0
        self.dlam0_a = [boundary_of(m, self.nbr) for m in self.lam0_a]
        self.dlam0 = np.any(self.dlam0_a, axis=0)
        self.lam0bar_a = [m & ~d for m, d in zip(self.lam0_a, self.dlam0_a)]
        self.lam0bar = self.lam0 & ~self.dlam0
        self.dPi1 = self.dPi & self.lam1
        self.lam1bar = self.lam1 & ~self.dPi1
        self.phi_a = [o & ~l for o, l in zip(self.omega_a, self.lam0_a)]
        self.ext_omega_a = [exterior_boundary_of(o, self.nbr) for o in self.omega_a]
        self.ext_omega_star_a = [e & self.dPi1 for e in self.ext_omega_a]

    def sites(self, mask) -> np.ndarray:
        return np.nonzero(mask)[0].astype(np.int64)


class BoxDomains:
    """The sets of Section 2 for an explicit list of blocks: each block b is a
    box Omega_0^b (origin, extent) holding an active box Lambda_0^b (an inner
    offset and extent relative to it).  Masks over lattice sites:

      lam0     union of the active boxes;  lam1 = its complement;
      dlam0_b  sites of Lambda_0^b with a neighbour outside it;
      dPi      sites with some coordinate on a face coordinate (first or last)
               of an active box, in the directions where that box does not
               span the lattice (the hyperplanes of step 2);
      dPi1     dPi minus the active boxes;
      omega_b  Omega_0^b;  phi_b = Omega_0^b minus Lambda_0^b (the frame);
      ext_b    exterior boundary of Omega_0^b (outside, with a neighbour inside).
    With the paper-mode boxes (Omega = [s - d, s + b - 1 + d]) these are the
    sets of PaperDomains.
    """

    def __init__(self, L, boxes, inner):
        self.L = [int(v) for v in L]
        V = volume(self.L)
        self.V = V
        self.nbr = neighbours(self.L)
        boxes = np.asarray(boxes, dtype=np.int64).reshape(-1, 8)
        inner = np.asarray(inner, dtype=np.int64).reshape(-1, 8)
        self.boxes, self.inner = boxes, inner
        x = coords(self.L)
        self.omega_a, self.lam0_a = [], []
        faces = [set() for _ in range(4)]
        for bx, ib in zip(boxes, inner):
            o = bx[:4]
            io = (o + ib[:4]) % np.asarray(self.L)
            self.omega_a.append(box_mask(self.L, o, bx[4:8]))
            self.lam0_a.append(box_mask(self.L, io, ib[4:8]))
            for mu in range(4):
                if ib[4 + mu] < self.L[mu]:
                    faces[mu].add(int(io[mu]))
                    faces[mu].add(int((io[mu] + ib[4 + mu] - 1) % self.L[mu]))
        dpi = np.zeros(V, dtype=bool)
        for mu in range(4):
            if faces[mu]:
                dpi |= np.isin(x[:, mu], sorted(faces[mu]))
        self.dPi = dpi
        self.lam0 = np.any(self.lam0_a, axis=0) if len(self.lam0_a) else np.zeros(V, dtype=bool)
        self.lam1 = ~self.lam0
        self.dlam0_a = [boundary_of(m, self.nbr) for m in self.lam0_a]
        self.dlam0 = np.any(self.dlam0_a, axis=0) if len(self.dlam0_a) else np.zeros(V, dtype=bool)
        self.lam0bar = self.lam0 & ~self.dlam0
        self.dPi1 = self.dPi & self.lam1
        self.phi_a = [o & ~l for o, l in zip(self.omega_a, self.lam0_a)]
        self.ext_a = [exterior_boundary_of(o, self.nbr) for o in self.omega_a]

    def sites(self, mask) -> np.ndarray:
        return np.nonzero(mask)[0].astype(np.int64)
