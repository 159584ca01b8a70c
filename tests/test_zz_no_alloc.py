"""argus_subtract_noalloc (the subtraction for callers that cannot allocate)
against argus_subtract through the C ABI: every output bit-identical, on two
calls in a row (a spatially varying 21x21 global fit's frame, then a smaller
frame with per-tile constant kernels), and the scratch limit rejected on the
host before any launch."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_2207_14304_amd import argus, synth
from gpu_util import dev, host, empty

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = argus.Context(0)
    yield c
    c.close()


def _planes(W, H, seed):
    fp = synth.make_pair(W, H, 300, seed, 2.0, 2.6, n_transients=5)
    cs, vs, ms = oracle.calibrate(fp.sci_raw, fp.dark, fp.flat, fp.bpm)
    cr, vr, mr = oracle.calibrate(fp.ref_raw[0], fp.dark, fp.flat, fp.bpm)
    rng = np.random.default_rng(seed)
    mr[rng.random(mr.shape) < 3e-4] |= oracle.SAT
    f = lambda a: a.astype(np.float32)
    return [dev(p) for p in (f(cr), f(vr), mr, f(cs), f(vs), ms)]


def _stamps(spec, ns, seed):
    """A kernel near the science/reference PSF ratio, per solve and monomial."""
    os_ = oracle.KernelSpec(half_width=spec.half_width, spatial_degree=spec.spatial_degree,
                            bg_degree=spec.bg_degree)
    n = oracle.n_unknowns(os_)
    rng = np.random.default_rng(seed)
    co = 0.01 * rng.standard_normal((ns, n))
    nP = (spec.spatial_degree + 1) * (spec.spatial_degree + 2) // 2
    co[:, 0] = 1.05
    co[:, 31 * nP] = -40.0
    st, bg = oracle.expand_kernel(co, os_)
    return dev(st.astype(np.float32)), dev(bg.astype(np.float32))


def _both(ctx, spec, planes):
    import torch
    H, W = planes[0].shape
    n, ns = argus.kernel_dims(spec)
    stamps, bg = _stamps(spec, ns, W + H)
    out = []
    for noalloc in (False, True):
        o = [empty((H, W), torch.float32), empty((H, W), torch.float32),
             empty((H, W), torch.uint8), empty(ns, torch.float64), empty(ns, torch.int64),
             empty(ns, torch.float64), empty(ns, torch.float64)]
        ctx.subtract(spec, stamps, bg, *planes, *o, noalloc=noalloc)
        out.append([host(t).copy() for t in o])
    return out


def test_noalloc_matches_subtract_on_two_calls(ctx):
    big = argus.make_spec(half_width=10, spatial_degree=2, bg_degree=2, tiles_x=16, tiles_y=16)
    small = argus.make_spec(half_width=7, tiles_x=3, tiles_y=2, mode=argus.FIT_PER_TILE)
    for spec, (W, H, seed) in ((big, (1100, 700, 5)), (small, (400, 300, 6))):
        ref, got = _both(ctx, spec, _planes(W, H, seed))
        for a, b in zip(ref, got):
            assert np.array_equal(a, b)
        assert np.all(ref[4] > 0) and np.all(np.isfinite(ref[3]))


def test_noalloc_rejects_beyond_its_scratch(ctx):
    import torch
    lib = argus.load()
    spec = argus.make_spec(half_width=7)
    t = torch.zeros(64, dtype=torch.float32, device="cuda")
    m = torch.zeros(64, dtype=torch.uint8, device="cuda")
    W, H = 128 * 257, 16 * 256                 # 65792 blocks of 128x16: over the 65536 limit
    d = argus.Dims(W, H, W)
    p, q = C.c_void_p(t.data_ptr()), C.c_void_p(m.data_ptr())
    rc = lib.argus_subtract_noalloc(ctx.h, d, C.byref(spec), p, p, p, p, q, p, p, q, p, p, q,
                                    None, None, None, None)
    assert rc == argus.ESHAPE
    assert b"scratch" in lib.argus_last_error(ctx.h)
