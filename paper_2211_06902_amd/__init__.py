"""MI355X-native block Wilson-Dirac library: D_Lambda, batched block solves
D_Lambda^{-1} b and the block-local multi-boson action of the overlapping
four-dimensional domain decomposition of det D (Saccardi & Giusti, Lattice
2022).  The compute path is the HIP library ``libdd.so`` (C ABI in
``include/dd.h``); ``dd`` is its ctypes binding."""

__all__ = ["dd"]
