"""Pin of the FP64 -> FP32 -> BF16 rounding rule against torch's CPU conversion."""
import numpy as np
import torch

from oracle import precision


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    x = np.concatenate([
        rng.standard_normal(100000),
        rng.standard_normal(1000) * 1e-30,
        rng.standard_normal(1000) * 1e30,
        np.array([0.0, -0.0, 1.0, -1.0, 1.00390625, 1.01171875, 3.0e38, np.inf, -np.inf]),
    ])
    f32 = precision.to_f32(x)
    bits = precision.f32_to_bf16_bits(f32)
    ref = torch.from_numpy(f32).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(bits, ref)


def test_bf16_ties_to_even():
    # 1 + 2^-8 lies halfway between two BF16 values: rounds to the even one (1.0)
    assert precision.f32_to_bf16_bits(np.float32(1.0 + 2**-8)) == 0x3F80
    # 1 + 3*2^-8 is halfway between 1+2^-7 and 1+2^-6: rounds to 1+2^-6 (even mantissa)
    assert precision.f32_to_bf16_bits(np.float32(1.0 + 3 * 2**-8)) == 0x3F82


def test_nan_is_quiet():
    assert precision.f32_to_bf16_bits(np.float32(np.nan)) & 0x7FC0 == 0x7FC0


def test_third_row_of_su3_links_is_rebuilt_exactly():
    """For SU(3) links conj(row0 x row1) is row 2; the check uses the generator's links and the identity."""
    import synth

    U = synth.gauge_field((4, 4, 4, 4), 0.5, 31).reshape(-1, 3, 3)
    assert np.max(np.abs(precision.rebuild_third_row(U) - U)) <= 1e-14
    I = np.broadcast_to(np.eye(3, dtype=complex), (5, 3, 3))
    assert np.array_equal(precision.rebuild_third_row(I), I)
    # a phase on row 2 alone is not SU(3) and is undone
    W = U.copy()
    W[:, 2, :] *= 1j
    assert np.max(np.abs(precision.rebuild_third_row(W) - U)) <= 1e-14


def test_two_row_bf16_links_round_only_the_stored_rows():
    import synth

    U = synth.gauge_field((2, 2, 2, 2), 0.3, 32).reshape(-1, 3, 3)
    V = precision.links_two_rows(U, precision.round_bf16)
    assert np.array_equal(V[:, :2].real, precision.round_bf16(U[:, :2].real))
    assert np.array_equal(V[:, :2].imag, precision.round_bf16(U[:, :2].imag))
    assert np.allclose(V[:, 2], np.conj(np.cross(V[:, 0], V[:, 1])), rtol=0, atol=1e-15)
    # the rebuilt row differs from the rounded original row by about the BF16 step
    assert 1e-4 < np.max(np.abs(V[:, 2] - U[:, 2])) < 2e-2
