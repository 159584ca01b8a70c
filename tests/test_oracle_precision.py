"""Pins of the BF16x3 emulation (the oracle's model of the split-precision
normal equations):

* the rounding is round-to-nearest-even on the bit pattern and the split
  keeps 16 significant bits;
* with operands that bf16 holds exactly (lo = 0) the emulated moments equal
  the exact sums bit for bit;
* with operands of exactly 16 significant bits (x = hi + lo exactly) the
  emulated moments equal the exact sums minus sum lo*lo', the one term the
  scheme drops, bit for bit;
* with the split and the FP32 rounding switched off, the moment form gives
  the FP64 normal equations of the plain definition (oracle.normal_equations)
  and the same solution, in both fit modes and with a spatially varying
  kernel and background.
"""
import numpy as np
import pytest

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


def test_bf16_exact_operands_give_exact_moments():
    rng = np.random.default_rng(11)
    N = 40
    c = rng.integers(-8, 9, (N, 64, 32)) / 4.0                 # at most 4 significant bits
    B = c * 2.0 ** rng.integers(-3, 4, (N, 64, 1))             # w xt^a c: still 4 bits
    hi, lo = precision.split(c)
    assert np.all(lo == 0) and np.all(precision.split(B)[1] == 0)
    got = precision.segment_moments(c, B, True)
    exact = np.matmul(c.transpose(0, 2, 1), B)
    assert np.array_equal(got, exact)


def test_sixteen_bit_operands_lose_exactly_lo_times_lo():
    rng = np.random.default_rng(12)
    N = 16
    # x = g (1 + s1 2^-4 + s2 2^-9), g = +-1: hi = g (1 + s1 2^-4), lo = g s2 2^-9;
    # one exponent keeps every FP32 step sum exact, so only the dropped term differs
    def draw(shape):
        g = rng.choice([-1.0, 1.0], shape)
        s1 = rng.integers(-1, 2, shape)
        s2 = rng.choice([-1.0, 1.0], shape)
        return g * (1.0 + s1 * 2.0 ** -4 + s2 * 2.0 ** -9), g * s2 * 2.0 ** -9
    c, clo = draw((N, 64, 32))
    B, blo = draw((N, 64, 32))
    hi, lo = precision.split(c)
    assert np.array_equal(lo, clo) and np.array_equal(hi + lo, c)
    assert np.array_equal(precision.split(B)[1], blo)
    got = precision.segment_moments(c, B, True)
    exact = np.matmul(c.transpose(0, 2, 1), B)
    dropped = np.matmul(clo.transpose(0, 2, 1), blo)
    assert np.abs(dropped).max() > 0
    assert np.array_equal(got, exact - dropped)


def _pair(W, H, seed):
    from test_oracle_pins import _star_ref
    ref = _star_ref(W, H, 40, seed)
    rng = np.random.default_rng(seed + 1)
    xt, yt = oracle.norm_coords(W, H)
    sci = (1.02 + 0.01 * xt[None, :]) * ref + 3.0 * yt[:, None] + rng.standard_normal((H, W)) * 3
    vr = np.full((H, W), 4.0) + rng.uniform(0, 1, (H, W))
    vs = np.full((H, W), 9.0) + rng.uniform(0, 1, (H, W))
    mr = np.zeros((H, W), np.uint8)
    ms = np.zeros((H, W), np.uint8)
    mr[30, 40] = oracle.BAD
    ms[50, 20] = oracle.SAT
    return ref, vr, mr, sci, vs, ms


@pytest.mark.parametrize("mode,D", [(oracle.core.GLOBAL, 1), (oracle.core.PER_TILE, 0),
                                    (oracle.core.GLOBAL, 2)])
def test_moment_form_equals_plain_normal_equations(mode, D):
    W, H = 150, 90                     # several 64-column segments and a ragged one
    planes = _pair(W, H, 3)
    spec = oracle.KernelSpec(sigmas=(1.0, 2.0), degrees=(2, 1), half_width=5, spatial_degree=D,
                             bg_degree=D, tiles_x=2, tiles_y=2, mode=mode)
    A, b, nf = precision.moment_system(*planes, spec, split_products=False, fp32_operands=False)
    Ao, bo, nfo = oracle.normal_equations(*planes, spec)
    if mode == oracle.core.GLOBAL:
        Ao, bo, nfo = Ao.sum(0)[None], bo.sum(0)[None], nfo.sum()[None]
    assert np.array_equal(nf, nfo)
    assert np.abs(A - Ao).max() <= 1e-12 * np.abs(Ao).max()
    assert np.abs(b - bo).max() <= 1e-12 * np.abs(bo).max()
    co, st, _ = precision.fit_kernel_bf16x3(*planes, spec, split_products=False,
                                            fp32_operands=False)
    coo, sto, _ = oracle.fit_kernel(*planes, spec)
    assert np.array_equal(st, sto) and np.all(st == 0)
    assert np.abs(co - coo).max() <= 1e-9 * np.abs(coo).max()


def test_emulated_error_sits_between_fp32_and_bf16():
    """On a small fit the split's coefficient error is far above what the FP32
    operands alone give and far below plain BF16 (8-bit) operands."""
    planes = _pair(150, 90, 5)
    spec = oracle.KernelSpec(sigmas=(1.2,), degrees=(2,), half_width=4)
    co, _, _ = oracle.fit_kernel(*planes, spec)
    e3, s3, _ = precision.fit_kernel_bf16x3(*planes, spec)
    e32, s32, _ = precision.fit_kernel_bf16x3(*planes, spec, split_products=False)
    assert s3[0] == 0 and s32[0] == 0
    scale = np.abs(co).max()
    err3 = np.abs(e3 - co).max() / scale
    err32 = np.abs(e32 - co).max() / scale
    assert err32 < err3 < 2.0 ** -8, (err32, err3)
