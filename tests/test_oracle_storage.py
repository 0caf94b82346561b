"""Pins of the FP16 / BF16 storage rounding emulation."""

import numpy as np
import torch

from oracle import storage


def test_bf16_matches_torch_cast():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000) * 10 ** rng.uniform(-5, 5, 10000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875]])
    want = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(storage.round_bf16(x), want)


def test_bf16_ties_to_even():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties go to the even mantissa (1)
    assert storage.round_bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    assert storage.round_bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6


def test_f16_matches_numpy_and_exact_values_pass():
    rng = np.random.default_rng(1)
    x = rng.standard_normal(1000) * 100
    assert np.array_equal(storage.round_f16(x), x.astype(np.float16).astype(np.float64))
    exact = np.array([0.5, 0.25, 1024.0, -3.0])
    assert np.array_equal(storage.round_f16(exact), exact)
    assert np.array_equal(storage.round_bf16(exact), exact)
