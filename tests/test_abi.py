"""The C-ABI library builds, loads and exports every symbol the header
declares; host-only calls work without a GPU."""
import ctypes
import os
import re

import pytest

from paper_2207_14304_amd import argus

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _ensure_built():
    if not os.path.exists(argus.LIB_PATH):
        from paper_2207_14304_amd import build
        build.build()


def test_header_and_binding_agree():
    hdr = open(os.path.join(ROOT, "include", "argus.h")).read()
    declared = set(re.findall(r"\b(argus_[a-z_]+)\s*\(", hdr))
    assert declared == set(argus.SYMBOLS)


def test_library_exports_every_symbol():
    _ensure_built()
    lib = ctypes.CDLL(argus.LIB_PATH)
    for name in argus.SYMBOLS:
        assert hasattr(lib, name), name


def test_kernel_dims_host_only():
    _ensure_built()
    s = argus.make_spec(half_width=7)
    assert argus.kernel_dims(s) == (32, 1)
    s = argus.make_spec(half_width=10, spatial_degree=2, bg_degree=2, tiles_x=16, tiles_y=16)
    assert argus.kernel_dims(s) == (192, 1)
    s = argus.make_spec(half_width=7, tiles_x=4, tiles_y=4, mode=argus.FIT_PER_TILE)
    assert argus.kernel_dims(s) == (32, 16)
    with pytest.raises(argus.ArgusError):
        argus.kernel_dims(argus.make_spec(half_width=16))
    with pytest.raises(argus.ArgusError):
        argus.kernel_dims(argus.make_spec(spatial_degree=1, bg_degree=2))
    with pytest.raises(argus.ArgusError):
        argus.kernel_dims(argus.make_spec(sigmas=(1.0,) * 4, degrees=(3, 3, 3, 3)))


def test_null_context_is_rejected():
    _ensure_built()
    lib = argus.load()
    d = argus.Dims(8, 8, 8)
    assert lib.argus_calibrate(None, d, None, None, None, None, 1.0, 1.0, 65535, None, None,
                               None) == argus.EINVAL
    assert lib.argus_ctx_create(0, None) == argus.EINVAL
    assert lib.argus_last_error(None) == b"null ctx"


def test_batch_candidates_host_only():
    _ensure_built()
    shapes = [argus.batch_candidate(i) for i in range(6)]
    assert shapes == [(16, 1), (16, 2), (16, 3), (32, 1), (32, 2), (32, 3)]
    for bad in (-1, 6):
        with pytest.raises(argus.ArgusError):
            argus.batch_candidate(bad)
