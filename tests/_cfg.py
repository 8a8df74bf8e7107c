"""Workload definitions and helpers shared by the tests.

The five configurations: plain FP64 4^4 (two overlapping tilings by 2^4 blocks), the 32^4 lattice
with 256 blocks of 8^4, the 48^3 x 96 lattice with uneven 8^4 / 8^3 x 12 blocks, the learned
preconditioner's training blocks, and the 64^4 multi-boson lattice with 4096 blocks of 8^4.
"""
import numpy as np

import synth
from oracle import geometry

C1 = dict(L=(4, 4, 4, 4), kappa=0.12, eps=0.5, seed_u=1101, seed_src=1102, nrhs=12,
          segs=[[2, 2]] * 4)
C2 = dict(L=(32, 32, 32, 32), kappa=0.1355, eps=0.3, seed_u=2101, seed_src=2102, nrhs=12,
          segs=[[8] * 4] * 4)
C3 = dict(L=(96, 48, 48, 48), kappa=0.1355, eps=0.3, seed_u=3101, seed_src=3102, nrhs=12,
          segs=[[12, 8, 12, 8, 12, 8, 12, 8, 8, 8]] + [[8] * 6] * 3)
C5 = dict(L=(64, 64, 64, 64), kappa=0.1365, eps=0.2, seed_u=5101, seed_chi=5102, seed_xi=5103, nfields=12,
          N=24, c=0.5, segs=[[8] * 8] * 4, inner_d=1)


def c1_boxes():
    """16 tiles of 2^4 plus the same tiling shifted by (1,1,1,1): 32 overlapping blocks."""
    a = geometry.tile_boxes(C1["L"], C1["segs"])
    b = geometry.tile_boxes(C1["L"], C1["segs"], shift=(1, 1, 1, 1))
    return np.concatenate([a, b])


def block_sites(L, boxes):
    return np.concatenate([geometry.box_sites(L, bx[:4], bx[4:8]) for bx in boxes])


def site_offsets(boxes):
    S = [int(np.prod(bx[4:8])) for bx in boxes]
    return np.concatenate([[0], np.cumsum(S)]).astype(np.int64)


def rel_err(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def max_err(a, b):
    """Largest element-wise difference relative to the largest element of b (complex modulus)."""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b), initial=0.0) / max(np.max(np.abs(b), initial=0.0), 1e-300))
