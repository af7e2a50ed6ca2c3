"""The CPU+GPU split of one Mandelbrot image (Sec. 7.5): whatever share the
GPU actor gets, the assembled image equals the oracle's bit for bit."""
import numpy as np
import pytest

import oracle
from paper_1505_07368_amd import gen

pytestmark = pytest.mark.gpu


def _scaled_replica(max_iter, width=320, height=200):
    vp = gen.paper_replica_viewport(max_iter)
    return gen.Viewport(vp.re_min, vp.im_min, 0.6 / width, 0.6 / height, width, height, max_iter)


@pytest.mark.parametrize("fp", ["f32", "f64"])
@pytest.mark.parametrize("max_iter", [120, 1200])
def test_split_image_matches_oracle(fp, max_iter):
    from paper_1505_07368_amd import binding as cg
    vp = _scaled_replica(max_iter)
    code = cg.F32 if fp == "f32" else cg.F64
    ref = oracle.mandelbrot(vp.re_min, vp.im_min, vp.step_re, vp.step_im, vp.width, 0,
                            vp.height, max_iter, fp)
    with cg.System(mode="batched", arena_bytes=64 << 20, ring_slots=64) as s:
        a = s.spawn(cg.BHV_MANDELBROT)
        image = cg.caf_mandel_args(vp.re_min, vp.im_min, vp.step_re, vp.step_im, vp.width,
                                   vp.height, 0, vp.height, max_iter, code)
        for gpu_rows in (0, 77, 130, vp.height):  # 77: a partial 64-row request
            img, t = s.offload_mandel(a, image, gpu_rows, cpu_threads=4)
            assert np.array_equal(img, ref), gpu_rows
            assert t["total_ns"] >= max(t["gpu_done_ns"], t["cpu_done_ns"]) >= 0
            assert (t["gpu_done_ns"] > 0) == (gpu_rows > 0)
            assert (t["cpu_done_ns"] > 0) == (gpu_rows < vp.height)


def test_split_refuses_bad_arguments():
    import torch
    from paper_1505_07368_amd import binding as cg
    vp = _scaled_replica(120, 64, 32)
    with cg.System(mode="batched", arena_bytes=16 << 20, ring_slots=16) as s:
        a = s.spawn(cg.BHV_MANDELBROT)
        L = cg.load()
        out = np.zeros((vp.height, vp.width), np.uint16)
        stage = torch.empty(vp.height * vp.width, dtype=torch.uint16, device="cuda")
        good = cg.caf_mandel_args(vp.re_min, vp.im_min, vp.step_re, vp.step_im, vp.width,
                                  vp.height, 0, vp.height, 120, cg.F32)
        o, st = out.ctypes.data, stage.data_ptr()
        assert L.caf_offload_mandel(s.h, a, good, vp.height + 1, 2, st, o, None) == cg.E_INVALID
        assert L.caf_offload_mandel(s.h, a, good, 8, 2, None, o, None) == cg.E_INVALID
        assert L.caf_offload_mandel(s.h, a, good, 8, 2, st, None, None) == cg.E_INVALID
        assert L.caf_offload_mandel(s.h, a, good, 8, 1025, st, o, None) == cg.E_INVALID
        tile = cg.caf_mandel_args(vp.re_min, vp.im_min, vp.step_re, vp.step_im, vp.width,
                                  vp.height, 8, 8, 120, cg.F32)  # not the whole image
        assert L.caf_offload_mandel(s.h, a, tile, 8, 2, st, o, None) == cg.E_INVALID
        g = s.spawn(cg.BHV_GEMM)  # not a Mandelbrot actor: the request is refused
        assert L.caf_offload_mandel(s.h, g, good, 8, 2, st, o, None) == cg.E_INVALID
        assert L.caf_offload_mandel(s.h, a, good, 8, 2, st, o, None) == cg.OK
