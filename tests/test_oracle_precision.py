"""Pins of the BF16x3 emulation: the rounding is RNE on the bit pattern, the
split is exact to 16 bits, and on a small fit the emulated coefficients sit
between FP32-level and BF16-level error."""
import numpy as np

import oracle
from oracle import precision


def test_bf16_round_is_nearest_even():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 0.0], np.float32)
    r = precision.bf16_round(x)
    # 1+2^-8 is a tie between 1 and 1+2^-7: even mantissa (1) wins;
    # 1+3*2^-8 ties between 1+2^-7 and 1+2^-6: even (1+2^-6) wins
    assert list(r) == [1.0, 1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -6, -2.5, 0.0]


def test_split_error_bound():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(100000) * 10 ** rng.uniform(-3, 3, 100000)).astype(np.float32)
    hi, lo = precision.split(x)
    rel = np.abs(hi + lo - x.astype(np.float64)) / np.abs(x)
    assert rel.max() <= 2.0 ** -16
    prod_err = np.abs((hi * hi + 2 * hi * lo) - x.astype(np.float64) ** 2) / x.astype(np.float64) ** 2
    assert prod_err.max() <= 2.0 ** -14


def test_emulated_fit_error_scale():
    from test_oracle_pins import _star_ref
    H, W = 90, 100
    ref = _star_ref(W, H, 40, 5)
    rng = np.random.default_rng(6)
    sci = 1.02 * ref + rng.standard_normal((H, W)) * 3
    v = np.full((H, W), 9.0)
    z = np.zeros((H, W), np.uint8)
    # a small, well-conditioned basis: dropping lo*lo keeps it positive definite
    spec = oracle.KernelSpec(sigmas=(1.2,), degrees=(2,), half_width=4)
    co, st, nf = oracle.fit_kernel(ref, v, z, sci, v, z, spec)
    cb, sb, nb = precision.fit_kernel_bf16x3(ref, v, z, sci, v, z, spec)
    assert st[0] == 0 and sb[0] == 0
    err = np.abs(cb - co).max() / np.abs(co).max()
    assert 1e-9 < err < 1e-1
