"""Autotuner for the compute-actor drain: work-tile sizes and grid.

It times candidate configurations on the actual workload through the C ABI
(the native driver issues the messages; the same kernels run as in
production) and keeps the fastest.  Results are cached in a JSON file keyed
by the device name and a workload signature, so a later run can reuse them
without re-timing.

Tuned knobs:
  * Mandelbrot: pixels per work tile (512, 1024, 2048, 4096) and the drain grid
    (all workgroups resident, or half of them);
  * GEMM: output-tile edge (64 or 128) per size class (n <= 64, <= 128,
    <= 256, > 256).
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import binding as cg


def _device_name(torch) -> str:
    # the device and the kernel sources: a cache written for other kernels
    # is not reused
    from . import profsum
    return f"{torch.cuda.get_device_name(0)}|src:{profsum.source_digest()[:16]}"


def _load_cache(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _store_cache(path, cache):
    if not path:
        return
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_drive(s, msgs, keep, window, reps):
    """Median wall time of `reps` runs after a warm-up (the median, not the
    minimum: candidates a few percent apart are otherwise ranked by luck)."""
    cg.drive_array(s, msgs, keep, window=window)  # warm-up
    times = []
    for _ in range(reps):
        t = time.perf_counter()
        rc, _, st, _ = cg.drive_array(s, msgs, keep, window=window)
        times.append(time.perf_counter() - t)
        if rc != cg.OK or not (st == cg.OK).all():
            return float("inf")
    return sorted(times)[len(times) // 2]


def mandel_messages(actor, viewports, tile_rows=64, fp=cg.F32):
    """NP_MSG array of row-tile requests for the given viewports."""
    from . import gen
    rows = []
    for vp in viewports:
        for r0, nr in gen.row_tiles(vp.height, tile_rows):
            rows.append((vp.re_min, vp.im_min, vp.step_re, vp.step_im, vp.width, vp.height, r0,
                         nr, vp.max_iter, fp))
    args = np.array(rows, dtype=cg.NP_MANDEL)
    msgs = np.zeros(len(rows), cg.NP_MSG)
    msgs["actor"] = actor
    msgs["args"] = args.ctypes.data + np.arange(len(rows), dtype=np.uint64) * args.itemsize
    msgs["args_bytes"] = args.itemsize
    return msgs, args


def tune_mandel(torch, viewports, mode="batched", cache_path=None, reps=5,
                pxs=(512, 1024, 2048, 4096), fp=cg.F32):
    """Returns {"mandel_tile_px": px, "grid": g} for the image workload."""
    key = f"{_device_name(torch)}|mandel|{mode}|fp{fp}|{len(viewports)}x" \
          f"{viewports[0].width}x{viewports[0].height}|{viewports[0].max_iter}"
    cache = _load_cache(cache_path)
    if key in cache:
        return cache[key]
    best, best_t = None, float("inf")
    for px in pxs:
        for grid_scale in (1.0, 0.5):
            s = cg.System(mode=mode, arena_bytes=1 << 30, mandel_tile_px=px)
            grid = 0
            if grid_scale != 1.0:
                # half of the resident grid of the light variant (5 per CU)
                grid = int(torch.cuda.get_device_properties(0).multi_processor_count * 5 *
                           grid_scale)
                s.shutdown()
                s = cg.System(mode=mode, arena_bytes=1 << 30, mandel_tile_px=px, grid=grid)
            try:
                a = s.spawn(cg.BHV_MANDELBROT)
                msgs, args = mandel_messages(a, viewports, fp=fp)
                t = _time_drive(s, msgs, (args,), len(msgs), reps)
            finally:
                s.shutdown()
            if t < best_t:
                best, best_t = {"mandel_tile_px": px, "grid": grid}, t
    cache[key] = best
    _store_cache(cache_path, cache)
    return best


def tune_gemm(torch, mode="batched", dtype="f32", count_per_size=256, cache_path=None, reps=5):
    """Returns the gemm_tile_class list (tile edge per size class)."""
    key = f"{_device_name(torch)}|gemm|{mode}|{dtype}|{count_per_size}"
    cache = _load_cache(cache_path)
    if key in cache:
        return cache[key]
    classes = [64, 128, 256, 512]  # a representative n per class
    choice = []
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    for n in classes:
        A = torch.rand(count_per_size * n * n, generator=g, device="cuda") * 2 - 1
        B = torch.rand(count_per_size * n * n, generator=g, device="cuda") * 2 - 1
        code = cg.F32
        if dtype == "bf16":
            A, B, code = A.to(torch.bfloat16), B.to(torch.bfloat16), cg.BF16
        esz = A.element_size()
        best_te, best_t = 0, float("inf")
        for te in (64, 128):
            s = cg.System(mode=mode, arena_bytes=2 << 30, ring_slots=max(4, count_per_size),
                          gemm_tile=te)
            try:
                act = s.spawn(cg.BHV_GEMM)
                args = np.zeros(1, cg.NP_GEMM)
                args["n"] = n
                args["in_dtype"] = code
                idx = np.arange(count_per_size, dtype=np.uint64)
                bufs = np.zeros(2 * count_per_size, cg.NP_BUF)
                bufs["data"][0::2] = A.data_ptr() + idx * (n * n * esz)
                bufs["data"][1::2] = B.data_ptr() + idx * (n * n * esz)
                bufs["numel"] = n * n
                bufs["dtype"] = code
                bufs["on_device"] = 1
                msgs = np.zeros(count_per_size, cg.NP_MSG)
                msgs["actor"] = act
                msgs["n_in"] = 2
                msgs["args"] = args.ctypes.data
                msgs["args_bytes"] = args.itemsize
                msgs["in_"] = bufs.ctypes.data + idx * 2 * bufs.itemsize
                torch.cuda.synchronize()
                t = _time_drive(s, msgs, (args, bufs), count_per_size, reps)
            finally:
                s.shutdown()
            if t < best_t:
                best_te, best_t = te, t
        choice.append(best_te)
        del A, B
    cache[key] = choice
    _store_cache(cache_path, cache)
    return choice
