"""The CPU actors' kernel of the CPU+GPU split (Sec. 7.5), on the host:
counts equal the oracle's, bit for bit, in both precisions; bad arguments
are refused.  Needs the built library, not a GPU."""
import numpy as np
import pytest

import oracle
from paper_1505_07368_amd import binding as cg
from paper_1505_07368_amd import gen


def _args(vp, fp):
    return cg.caf_mandel_args(vp.re_min, vp.im_min, vp.step_re, vp.step_im, vp.width, vp.height,
                              0, vp.height, vp.max_iter, fp)


@pytest.mark.parametrize("fp", [cg.F32, cg.F64])
def test_tiny_image_matches_oracle(fp):
    vp = gen.tiny_viewport()
    got = cg.cpu_mandel_rows(_args(vp, fp), 0, vp.height)
    ref = oracle.mandelbrot(vp.re_min, vp.im_min, vp.step_re, vp.step_im, vp.width, 0,
                            vp.height, vp.max_iter, "f32" if fp == cg.F32 else "f64")
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("fp", [cg.F32, cg.F64])
@pytest.mark.parametrize("max_iter", [120, 1200])
def test_paper_viewport_rows_match_oracle(fp, max_iter):
    """A band of the Sec. 7.5 image, away from row 0: rows are sampled with
    their global index."""
    vp = gen.paper_replica_viewport(max_iter)
    r0, r1 = 517, 531
    got = cg.cpu_mandel_rows(_args(vp, fp), r0, r1)
    ref = oracle.mandelbrot(vp.re_min, vp.im_min, vp.step_re, vp.step_im, vp.width, r0, r1 - r0,
                            max_iter, "f32" if fp == cg.F32 else "f64")
    assert np.array_equal(got, ref)
    assert got.max() == max_iter and got.min() >= 1  # interior and exterior both present


def test_bad_arguments_refused():
    vp = gen.tiny_viewport()
    L = cg.load()
    out = np.zeros((4, vp.width), np.uint16)
    a = _args(vp, cg.F32)
    assert L.caf_cpu_mandel_rows(None, 0, 1, out.ctypes.data) == cg.E_INVALID
    assert L.caf_cpu_mandel_rows(a, 0, 1, None) == cg.E_INVALID
    assert L.caf_cpu_mandel_rows(a, 2, 1, out.ctypes.data) == cg.E_INVALID
    assert L.caf_cpu_mandel_rows(a, vp.height - 1, vp.height + 1, out.ctypes.data) == cg.E_INVALID
    for field, bad in (("max_iter", 0), ("max_iter", 65536), ("fp", cg.I32), ("width", 0)):
        b = _args(vp, cg.F32)
        setattr(b, field, bad)
        assert L.caf_cpu_mandel_rows(b, 0, 1, out.ctypes.data) == cg.E_INVALID, field
    assert L.caf_cpu_mandel_rows(a, 3, 3, out.ctypes.data) == cg.OK  # empty range
