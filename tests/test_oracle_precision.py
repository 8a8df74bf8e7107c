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
