"""CPU FP64 oracle for the block Wilson-Dirac path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  It shares no code
with the HIP library (no kernels, headers, helpers, tables or constant
generators) and imports nothing from it; both consume the seeded inputs of
the separate ``synth`` module.

Contents (each module cites the part of the paper it follows):
  wilson     Wilson-Dirac operator D, box restrictions D_Lambda, block solves (C, FP64)
  geometry   tilings and the domains of Section 2 (box reading)
  dense      dense-matrix determinant identities of Section 3 on tiny lattices
  factor     the Schur-complement pieces of Section 3 (Dtilde, Dhat^d, Dhat^h, W_z) as dense matrices
  roots      polynomial P_N, remainder R_{N+1} and roots u_k of Section 4
  mb         multi-boson action of Section 4 (block-local S_MB^a, global rest S^r_MB), W_z chi as a
             vector, field generation chi = W_u^{-1} eta, the remainder R_{N+1}(W_1) and the
             stochastic estimate of ln W_N (eq. rw)
  clover     the Sheikholeslami-Wohlert term named in Section 3
  precision  FP64 -> FP32 -> BF16 rounding rules
  convnet    the learned block preconditioner: 4D conv net, gradients, loss, Adam
             (not in the paper; parity pinned by independent identities)
"""
from . import clover, convnet, dense, factor, geometry, mb, precision, roots, wilson  # noqa: F401
from ._clib import build  # noqa: F401
