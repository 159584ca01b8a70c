"""The seeded input generators (host side): the device generator's
fixed-order accumulation of overlapping stars, checked on the CPU against
numpy's unbuffered add, and reproducibility of a render."""
import numpy as np
import pytest

from paper_2207_14304_amd import synth_torch


def test_add_at_sums_repeated_indices():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    idx = rng.integers(0, 50, 2000)
    vals = rng.standard_normal(2000).astype(np.float32)
    img = torch.zeros(50, dtype=torch.float32)
    synth_torch._add_at(img, torch.from_numpy(idx), torch.from_numpy(vals))
    ref = np.zeros(50, np.float64)
    np.add.at(ref, idx, vals.astype(np.float64))
    assert np.allclose(img.numpy(), ref, rtol=1e-5, atol=1e-4)


def test_render_is_reproducible_and_conserves_flux():
    torch = pytest.importorskip("torch")
    g = torch.Generator().manual_seed(5)
    W, H, n = 160, 120, 200
    xs = (torch.rand(n, generator=g) * (W - 40) + 20).float()
    ys = (torch.rand(n, generator=g) * (H - 40) + 20).float()
    fl = (torch.rand(n, generator=g) * 1e4 + 100).float()
    a = synth_torch.render(W, H, xs, ys, fl, 2.0, "cpu")
    b = synth_torch.render(W, H, xs, ys, fl, 2.0, "cpu")
    assert torch.equal(a, b)
    # stars at least 20 px from the border keep their whole 8-FWHM disk (16 px)
    assert abs(float(a.double().sum()) / float(fl.double().sum()) - 1.0) < 1e-5
