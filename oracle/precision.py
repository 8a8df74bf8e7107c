"""Reduced-precision rounding rules (oracle).  Test infrastructure only.

The mixed-precision stencil stores links and spinors in FP32 or links in
BF16.  The rule: FP64 -> FP32 round-to-nearest-even (IEEE default), then
FP32 -> BF16 round-to-nearest-even on the top 16 bits; NaN maps to the quiet
NaN 0x7FC0 with the sign kept.

Links are stored as their first two rows; the third row of an SU(3) matrix
is the complex conjugate of the cross product of the first two, and is
rebuilt from the stored (possibly rounded) rows.
"""
from __future__ import annotations

import numpy as np

__all__ = ["to_f32", "f32_to_bf16_bits", "bf16_bits_to_f32", "round_bf16", "rebuild_third_row",
           "links_two_rows"]


def to_f32(a) -> np.ndarray:
    return np.asarray(a, dtype=np.float64).astype(np.float32)


def f32_to_bf16_bits(a) -> np.ndarray:
    """uint16 bit patterns of BF16 values, rounding FP32 to nearest even."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16).astype(np.uint16)
    nan = np.isnan(f)
    if np.any(nan):
        r[nan] = ((u[nan] >> 16) & 0x8000).astype(np.uint16) | np.uint16(0x7FC0)
    return r


def bf16_bits_to_f32(bits) -> np.ndarray:
    b = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return b.view(np.float32)


def round_bf16(a) -> np.ndarray:
    """FP64 values rounded FP64 -> FP32 -> BF16, returned as FP64."""
    return bf16_bits_to_f32(f32_to_bf16_bits(to_f32(a))).astype(np.float64)


def rebuild_third_row(U: np.ndarray) -> np.ndarray:
    """[..., 3, 3] complex: row 2 replaced by conj(row 0 x row 1) (exact for SU(3))."""
    V = np.array(U, dtype=np.complex128, copy=True)
    a, b = V[..., 0, :], V[..., 1, :]
    V[..., 2, :] = np.conj(np.cross(a, b))
    return V


def links_two_rows(U: np.ndarray, rounding=None) -> np.ndarray:
    """The links a two-row store reproduces: rows 0 and 1 passed through `rounding`
    (a function on real arrays, e.g. round_bf16; None keeps them), row 2 rebuilt."""
    V = np.array(U, dtype=np.complex128, copy=True)
    if rounding is not None:
        V[..., :2, :] = rounding(V[..., :2, :].real) + 1j * rounding(V[..., :2, :].imag)
    return rebuild_third_row(V)
