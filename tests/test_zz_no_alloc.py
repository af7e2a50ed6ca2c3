"""caf_offload_mandel_noalloc, the split for callers that cannot allocate:
through the C ABI, its image equals caf_offload_mandel's bit for bit, on
two calls in a row (the second smaller, so it reads only what it staged
itself), and sizes beyond the fixed staging array are refused on the host."""
import ctypes as C

import numpy as np
import pytest

from paper_1505_07368_amd import gen

pytestmark = pytest.mark.gpu


def _image(cg, vp, fp):
    return cg.caf_mandel_args(vp.re_min, vp.im_min, vp.step_re, vp.step_im, vp.width,
                              vp.height, 0, vp.height, vp.max_iter, fp)


def _viewport(width, height, max_iter):
    vp = gen.paper_replica_viewport(max_iter)
    return gen.Viewport(vp.re_min, vp.im_min, 0.6 / width, 0.6 / height, width, height, max_iter)


@pytest.mark.parametrize("mode", ["batched", "plain"])
def test_noalloc_split_matches_the_allocating_split(mode):
    from paper_1505_07368_amd import binding as cg
    big = _viewport(1920, 1080, 120)
    small = _viewport(640, 360, 1200)
    with cg.System(mode=mode, arena_bytes=64 << 20, ring_slots=256) as s:
        a = s.spawn(cg.BHV_MANDELBROT)
        for vp, fp, gpu_rows, threads in ((big, cg.F32, 700, 4), (small, cg.F64, 150, 4)):
            image = _image(cg, vp, fp)
            # the allocating call also starts the CPU actors with `threads` workers
            ref, _ = s.offload_mandel(a, image, gpu_rows, cpu_threads=threads)
            got, t = s.offload_mandel_noalloc(a, image, gpu_rows, cpu_threads=threads)
            assert np.array_equal(got, ref), (vp.width, gpu_rows, int((got != ref).sum()))
            assert t["gpu_done_ns"] > 0 and t["cpu_done_ns"] > 0
            # all rows on the GPU actor: needs no CPU actors
            got_all, t = s.offload_mandel_noalloc(a, image, vp.height, cpu_threads=threads)
            ref_all, _ = s.offload_mandel(a, image, vp.height, cpu_threads=threads)
            assert np.array_equal(got_all, ref_all)
            assert np.array_equal(got_all, ref)


def test_noalloc_split_limits():
    from paper_1505_07368_amd import binding as cg
    L = cg.load()
    with cg.System(mode="batched", arena_bytes=16 << 20, ring_slots=64) as s:
        a = s.spawn(cg.BHV_MANDELBROT)
        wide = _viewport(8192, 1100, 120)  # 1100 rows x 8192 x 2 B > 16 MiB
        out = np.zeros((wide.height, wide.width), np.uint16)
        image = _image(cg, wide, cg.F32)
        assert L.caf_offload_mandel_noalloc(s.h, a, C.byref(image), wide.height, 4,
                                            out.ctypes.data, None) == cg.E_INVALID
        assert L.caf_offload_mandel_noalloc(s.h, a, C.byref(image), 8, 4, None,
                                            None) == cg.E_INVALID
        # a CPU share before any CPU actors run: refused (starting them allocates)
        assert L.caf_offload_mandel_noalloc(s.h, a, C.byref(image), 8, 3,
                                            out.ctypes.data, None) == cg.E_INVALID
        small = _viewport(256, 64, 120)
        out = np.zeros((small.height, small.width), np.uint16)
        img = _image(cg, small, cg.F32)
        assert L.caf_offload_mandel_noalloc(s.h, a, C.byref(img), small.height, 3,
                                            out.ctypes.data, None) == cg.OK
