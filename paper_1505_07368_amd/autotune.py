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
    <= 256, > 256);
  * a mix of escape-time tiles and products: the full drain variant's
    workgroups per compute unit (2 or 3) and the drain batch (max_batch).
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
        # 256: 128 x 256 bf16 tiles (products that do not qualify get 128)
        for te in ((64, 128, 256) if dtype == "bf16" else (64, 128)):
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


def mix_messages(cg, torch, d, m_actor, g_actor, pool_seed=0):
    """NP_MSG array of a serving mix (gen.serving_mix_arrays output d):
    Mandelbrot squares to m_actor, fp32 GEMMs to g_actor with inputs from
    eight device pairs per size.  Returns (msgs, keep): keep holds every
    buffer the messages point into."""
    from . import gen
    cnt = d["arrival_ns"].size
    pool = {}
    gg = torch.Generator(device="cuda")
    gg.manual_seed(pool_seed)
    for n in gen.SERVE_GEMM_N:
        pool[n] = [(torch.rand(n * n, generator=gg, device="cuda") * 2 - 1,
                    torch.rand(n * n, generator=gg, device="cuda") * 2 - 1) for _ in range(8)]
    margs = np.zeros(cnt, cg.NP_MANDEL)
    margs["re_min"] = d["re_min"]
    margs["im_min"] = d["im_min"]
    margs["step_re"] = d["step"]
    margs["step_im"] = d["step"]
    margs["width"] = d["side"]
    margs["height"] = d["side"]
    margs["rows"] = d["side"]
    margs["max_iter"] = d["max_iter"]
    margs["fp"] = cg.F32
    gargs = np.zeros(cnt, cg.NP_GEMM)
    gargs["n"] = d["gemm_n"]
    gargs["in_dtype"] = cg.F32
    bufs = np.zeros(cnt * 2, cg.NP_BUF)
    pick = np.arange(cnt) % 8
    for n in gen.SERVE_GEMM_N:
        sel = np.nonzero((d["gemm_n"] == n) & ~d["is_mandel"])[0]
        for k in range(8):
            ss = sel[pick[sel] == k]
            bufs["data"][2 * ss] = pool[n][k][0].data_ptr()
            bufs["data"][2 * ss + 1] = pool[n][k][1].data_ptr()
            bufs["numel"][2 * ss] = n * n
            bufs["numel"][2 * ss + 1] = n * n
    bufs["dtype"] = cg.F32
    bufs["on_device"] = 1
    idx = np.arange(cnt, dtype=np.uint64)
    msgs = np.zeros(cnt, cg.NP_MSG)
    ism = d["is_mandel"]
    msgs["actor"] = np.where(ism, m_actor, g_actor)
    msgs["n_in"] = np.where(ism, 0, 2)
    msgs["args"] = np.where(ism, margs.ctypes.data + idx * margs.itemsize,
                            gargs.ctypes.data + idx * gargs.itemsize)
    msgs["args_bytes"] = np.where(ism, margs.itemsize, gargs.itemsize)
    msgs["in_"] = np.where(ism, 0, bufs.ctypes.data + idx * 2 * bufs.itemsize)
    return msgs, (margs, gargs, bufs, pool)


def tune_mix(torch, cache_path=None, seed=7, count=6000, window=2048, reps=3,
             wgs=(2, 3), batches=(256, 1024)):
    """Returns {"full_wgs_per_cu": w, "max_batch": b} for a serving mix (70 %
    escape-time squares, 30 % fp32 products), timed closed loop through a
    persistent system on a seeded mix of `count` messages."""
    from . import gen
    key = f"{_device_name(torch)}|mix|{count}|{window}"
    cache = _load_cache(cache_path)
    if key in cache:
        return cache[key]
    d = gen.serving_mix_arrays(seed, 1e5, count / 1e5)
    best, best_t = None, float("inf")
    for w in wgs:
        for mb in batches:
            s = cg.System(mode="persistent", arena_bytes=4 << 30, ring_slots=8192,
                          max_batch=mb, full_wgs_per_cu=w)
            try:
                m = s.spawn(cg.BHV_MANDELBROT)
                g = s.spawn(cg.BHV_GEMM)
                msgs, keep = mix_messages(cg, torch, d, m, g)
                torch.cuda.synchronize()
                t = _time_drive(s, msgs, keep, window, reps)
            finally:
                s.shutdown()
            if t < best_t:
                best, best_t = {"full_wgs_per_cu": w, "max_batch": mb}, t
    cache[key] = best
    _store_cache(cache_path, cache)
    return best
