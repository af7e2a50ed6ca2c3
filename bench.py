"""Benchmark of the compute-actor hot path on one MI355X.

Workload (the headline): Mandelbrot 1920x1080 at max_iter 1000, eight
seeded viewports on the main cardioid's boundary (zoom 1 to 1e4), each image
split into 17 row-tile messages of 64 rows (the last 56) sent to one GPU
actor.  One step = all 8 x 17 = 136 tile requests through the C ABI,
issued by the native driver and waited for.  `value` is Mandelbrot Giter/s
(sum of the exact escape counts of the replies per second) of the batched
mailbox-drain form in float; the same step in double, the persistent form
and the one-launch-per-message form are reported beside it, with reply
latency percentiles, plus the small-message comparison (int32 echo
ping-pong, 64x64 tiles, n = 64 GEMMs) of the three forms.

Prints ONE JSON line.  Only --gpus 1 is supported.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Vector peaks, from the published MI355X figures (256 CUs at 2.4 GHz):
# 157.3 TFLOP/s fp32 and 78.6 TFLOP/s fp64, which count a fused multiply-add
# as two flops, i.e. 128 fp32 and 64 fp64 lane operations per clock per CU.
# The escape loop has no multiply-add (exact counts), so its ceiling is that
# many plain adds, multiplies or compares per lane per clock: 78.6e12 fp32
# and 39.3e12 fp64 operations per second.  (For plain fp32 instructions
# gfx950 reaches the fp32 rate by issuing two VALU instructions per SIMD in
# one quad cycle, from two waves.)
VALU_PEAK = {"f32": 157.3e12 / 2, "f64": 78.6e12 / 2}
# Algorithmic operations per escape-time iteration: 3 multiplies, 5 adds or
# subtracts, and the |z|^2 > 4 compare.
OPS_PER_ITER = 9
HBM_PEAK = 8.0e12


# time of the last progress line (the leg watchdog's clock)
_PROGRESS = [time.monotonic()]
# a leg that prints no progress line for this long is taken to be stuck
LEG_STALL_S = 150.0


def log(*a):
    _PROGRESS[0] = time.monotonic()
    print(*a, file=sys.stderr, flush=True)


def start_leg_watchdog(result, tuned, current):
    """Ends the run if a leg beside the headline stops making progress: the
    leg is recorded as timed out, the legs after it as not run, and the one
    JSON line (headline included) is printed before the process exits.  A
    leg stuck in a library call cannot be interrupted from Python, and the
    process's exit ends its GPU work."""
    import threading

    def watch():
        while True:
            time.sleep(1.0)
            leg = current[0]
            if leg is None or time.monotonic() - _PROGRESS[0] < LEG_STALL_S:
                continue
            log(f"[bench] leg {leg}: no progress for {LEG_STALL_S:g} s; ending the run")
            out = None
            for _ in range(10):  # the stuck thread is inside a library call
                try:
                    out = json.loads(json.dumps(result))
                    break
                except RuntimeError:
                    time.sleep(0.1)
            if out is None:
                out = {k: result[k] for k in ("metric", "value", "unit")}
            msg = (f"no progress for {LEG_STALL_S:g} s; this leg and the legs after it did "
                   "not finish")
            if isinstance(out.get(leg), dict):
                out[leg]["error"] = msg  # keep what the leg measured before it stalled
            else:
                out[leg] = {"error": msg}
            try:
                out["tuned"] = json.loads(json.dumps(tuned))
            except (RuntimeError, TypeError, ValueError):
                pass
            print(json.dumps(out), flush=True)
            os._exit(0)

    threading.Thread(target=watch, daemon=True).start()


# rocprofv3 summary of the headline's dominant kernel (durations and counters).
PROFILE = os.path.join(ROOT, "profiles", "drain_kernel_light_mandelbrot_8x1920x1080_i1000_f32.md")


def measured_traffic():
    """HBM bytes per drain launch from the committed counter summary, or
    None if the device sources changed since the counters were taken."""
    from paper_1505_07368_amd import profsum
    kv = profsum.read_summary(PROFILE)
    if kv.get("source_digest") != profsum.source_digest() or "traffic_bytes_per_dispatch" not in kv:
        return None
    return int(kv["traffic_bytes_per_dispatch"])


def percentiles(lat_ns):
    lat = np.asarray(lat_ns, np.float64)
    lat = lat[lat >= 0] / 1e3
    if lat.size == 0:
        return None, None
    return float(np.percentile(lat, 50)), float(np.percentile(lat, 99))


def interior_viewport(width=1920, height=1080, max_iter=1000):
    """A viewport inside the main cardioid (re in [-0.5, 0.1], square
    pixels, centred on the real axis): no pixel escapes, so every lane runs
    max_iter iterations with no divergence and no escape bookkeeping -- the
    attainable rate of the escape loop's own instruction mix."""
    from paper_1505_07368_amd import gen
    step = 0.6 / width
    return gen.Viewport(-0.5, -step * height / 2, step, step, width, height, max_iter)


def mandel_leg(cg, torch, mode, fp, steps, warmup, seeds, timed_kernel=False, tune=None,
               palette=None, viewports=None, dispersion_reps=0):
    """Runs the image workload in one delivery mode; returns a dict.  With a
    palette (device int32 tensor) the timed steps go to an actor spawned with
    it, so every reply is a colour image; the work per step is still the sum
    of the escape counts, taken from a counts run of the same messages.
    viewports replaces the seeded boundary viewports.  dispersion_reps > 0
    times that many further steps one by one (mean and standard deviation).

    The timed steps are bracketed by device synchronisation, except for the
    persistent form: its drain kernel stays resident for a long idle linger
    by design, and a device-wide synchronize would wait for that linger, so
    the closing synchronisation there is of the caller's stream (every reply
    has already been received when the last step returns)."""
    from paper_1505_07368_amd import autotune, gen
    tune = tune or {}
    vps = viewports or [gen.boundary_viewport(sd) for sd in seeds]
    s = cg.System(mode=mode, arena_bytes=1 << 30, ring_slots=4096,
                  mandel_tile_px=tune.get("mandel_tile_px", 0), grid=tune.get("grid", 0))
    try:
        a = s.spawn(cg.BHV_MANDELBROT)
        arr, arr_args = autotune.mandel_messages(a, vps, fp=fp)
        # exact algorithmic work of one step: the sum of the reply counts
        outs = [torch.empty(int(r["rows"]) * int(r["width"]), dtype=torch.uint16, device="cuda")
                for r in arr_args]
        chk = arr.copy()
        chk["out"]["data"] = [o.data_ptr() for o in outs]
        chk["out"]["numel"] = [o.numel() for o in outs]
        chk["out"]["dtype"] = cg.U16
        chk["out"]["on_device"] = 1
        torch.cuda.synchronize()
        rc, _, st, _ = cg.drive_array(s, chk, (arr_args, outs), window=len(chk))
        assert rc == cg.OK and (st == cg.OK).all(), (rc, st)
        torch.cuda.synchronize()
        iters = int(sum(int(o.to(torch.int64).sum()) for o in outs))
        del outs
        # the timed steps issue a prebuilt message array (the caller's
        # marshalling is not part of a step)
        timed = a if palette is None else s.spawn(cg.BHV_MANDELBROT, palette=palette)
        arr["actor"] = timed
        step = cg.PreparedDrive(s, arr, window=len(arr))
        for _ in range(warmup):
            step()
        s.drain_kernel_ms()  # reset the launch timers
        torch.cuda.synchronize()
        lats, step_s, bad = [], [], 0
        t0 = time.perf_counter()
        t = t0
        for _ in range(steps):
            rc = step()
            t1 = time.perf_counter()
            step_s.append(t1 - t)
            t = t1
            bad += rc != cg.OK or not (step.st == cg.OK).all()
            lats.append(step.lat.copy())
        assert bad == 0
        if mode == "persistent":
            torch.cuda.current_stream().synchronize()
        else:
            torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        kms, launches = s.drain_kernel_ms()
        p50, p99 = percentiles(np.concatenate(lats))
        st_ms = np.asarray(step_s) * 1e3
        out = {"giter_s": iters * steps / dt / 1e9, "msgs_per_s": len(arr) * steps / dt,
               "ms_per_step": dt / steps * 1e3, "iters_per_step": iters,
               "step_ms_mean": float(st_ms.mean()), "step_ms_std": float(st_ms.std(ddof=1))
               if steps > 1 else 0.0,
               "p50_us": p50, "p99_us": p99, "messages_per_step": len(arr)}
        if timed_kernel and launches:
            out["kernel_ms_total"] = kms
            out["kernel_launches"] = launches
        if dispersion_reps:
            ds = []
            for _ in range(dispersion_reps):
                t = time.perf_counter()
                rc = step()
                ds.append(time.perf_counter() - t)
                assert rc == cg.OK and (step.st == cg.OK).all()
            ds = np.asarray(ds)
            g = iters / ds / 1e9
            out["dispersion"] = {"reps": dispersion_reps, "step_ms_mean": float(ds.mean() * 1e3),
                                 "step_ms_std": float(ds.std(ddof=1) * 1e3),
                                 "giter_s_mean": float(g.mean()), "giter_s_std": float(g.std(ddof=1))}
        return out
    finally:
        s.shutdown()


def small_leg(cg, torch, mode, kind, count, window):
    """Small messages through one form: echo (int32), 64x64 Mandelbrot tile,
    n = 64 fp32 GEMM, or a stateful hash-chain step (device-resident state,
    updated strictly in mailbox order).  Returns msgs/s and latency
    percentiles."""
    from paper_1505_07368_amd import gen
    s = cg.System(mode=mode, arena_bytes=256 << 20, ring_slots=4096, idle_exit_us=200000)
    try:
        keep = []
        if kind == "echo":
            a = s.spawn(cg.BHV_NOOP)
            x = np.array([42], np.int32)
            keep.append(x)
            msgs = [{"actor": a, "inputs": [x]} for _ in range(count)]
        elif kind == "hash":
            a = s.spawn(cg.BHV_HASHCHAIN)
            msgs = [{"actor": a, "args": cg.caf_hash_args(i * 2654435761)} for i in range(count)]
        elif kind == "mandel64":
            a = s.spawn(cg.BHV_MANDELBROT)
            vp = gen.tiny_viewport()
            msgs = [{"actor": a, "args": cg.caf_mandel_args(
                vp.re_min + 64 * vp.step_re * (i % 8), vp.im_min, vp.step_re, vp.step_im,
                64, 512, 64 * ((i // 8) % 8), 64, 100, cg.F32)} for i in range(count)]
        else:
            a = s.spawn(cg.BHV_GEMM)
            A, B = gen.gemm_pair(3, 64)
            At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
            keep += [At, Bt]
            msgs = [{"actor": a, "args": cg.caf_gemm_args(64, cg.F32), "inputs": [At, Bt]}
                    for _ in range(count)]
        torch.cuda.synchronize()
        s.drive(msgs[: min(len(msgs), 256)], window=window)  # warm-up
        rc, lat, st, el = s.drive(msgs, window=window)
        assert rc == cg.OK and (st == cg.OK).all(), (rc, np.unique(st))
        p50, p99 = percentiles(lat)
        return {"msgs_per_s": count / el, "p50_us": p50, "p99_us": p99}
    finally:
        s.shutdown()


MFMA_PEAK = {"f32": 157.3e12, "bf16": 2.5e15}


def _bufs_array(cg, pairs):
    """NP_BUF array (2 per message) for (ptrA, ptrB, numel, dtype) rows."""
    arr = np.zeros(len(pairs) * 2, cg.NP_BUF)
    pa = np.asarray(pairs, dtype=np.uint64)
    arr["data"][0::2] = pa[:, 0]
    arr["data"][1::2] = pa[:, 1]
    arr["numel"][0::2] = pa[:, 2]
    arr["numel"][1::2] = pa[:, 2]
    arr["dtype"][:] = pa[0, 3] if len(pa) else 0
    arr["on_device"][:] = 1
    return arr


def gemm_leg(cg, torch, dtype, count=4096, seed=0, reps=3, tile_class=(0, 0, 0, 0),
             max_batch=1024, grid=0, full_wgs_per_cu=0):
    """The grouped-GEMM workload: `count` requests with n drawn from
    {64, 128, 256, 512}, entries U(-1, 1) (bf16: rounded to nearest even),
    every request with its own inputs resident in HBM."""
    from paper_1505_07368_amd import gen
    sizes = gen.gemm_sizes(seed, count).astype(np.int64)
    nn = sizes * sizes
    offs = np.concatenate([[0], np.cumsum(nn)[:-1]])
    total = int(nn.sum())
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    A = torch.rand(total, generator=g, device="cuda") * 2 - 1
    B = torch.rand(total, generator=g, device="cuda") * 2 - 1
    code = cg.F32
    if dtype == "bf16":
        A, B, code = A.to(torch.bfloat16), B.to(torch.bfloat16), cg.BF16
    esz = A.element_size()
    flops = float((2 * sizes ** 3).sum())
    bytes_ = float((nn * (2 * esz + 4)).sum())
    s = cg.System(mode="batched", arena_bytes=4 << 30, ring_slots=count, max_batch=max_batch,
                  grid=grid, gemm_tile_class=tuple(tile_class), full_wgs_per_cu=full_wgs_per_cu)
    try:
        a = s.spawn(cg.BHV_GEMM)
        args = np.zeros(count, cg.NP_GEMM)
        args["n"] = sizes
        args["in_dtype"] = code
        bufs = _bufs_array(cg, [(A.data_ptr() + int(o) * esz, B.data_ptr() + int(o) * esz,
                                 int(m), code) for o, m in zip(offs, nn)])
        msgs = np.zeros(count, cg.NP_MSG)
        msgs["actor"] = a
        msgs["n_in"] = 2
        msgs["args"] = args.ctypes.data + np.arange(count, dtype=np.uint64) * args.itemsize
        msgs["args_bytes"] = args.itemsize
        msgs["in_"] = bufs.ctypes.data + np.arange(count, dtype=np.uint64) * 2 * bufs.itemsize
        torch.cuda.synchronize()
        keep = (args, bufs, A, B)
        cg.drive_array(s, msgs, keep, window=count)  # warm-up
        s.drain_kernel_ms()
        t0 = time.perf_counter()
        for _ in range(reps):
            rc, lat, st, el = cg.drive_array(s, msgs, keep, window=count)
            assert rc == cg.OK and (st == cg.OK).all(), (rc, np.unique(st))
        dt = (time.perf_counter() - t0) / reps
        kms, nl = s.drain_kernel_ms()
        kdt = kms * 1e-3 / reps
        # The same batch from a pre-filled mailbox: the drain is held while
        # the host submits every request, then one launch runs them all, so
        # its time excludes the host's submission.
        L = cg.load()
        pk = []
        for _ in range(reps):
            assert s.drain() == cg.OK
            s.drain_kernel_ms()  # the last launch has exited
            s.hold(True)
            futs = []
            for i in range(count):
                f = C.c_void_p()
                rc = L.caf_gpu_request(s.h, int(msgs["actor"][i]), 0, int(msgs["args"][i]),
                                       int(msgs["args_bytes"][i]),
                                       C.cast(int(msgs["in_"][i]), C.POINTER(cg.caf_buf)), 2,
                                       None, 0, C.byref(f))
                assert rc == cg.OK, rc
                futs.append(f)
            s.hold(False)
            res, st = cg.caf_buf(), C.c_int32()
            for f in futs:
                assert L.caf_future_wait(f, -1, C.byref(res), C.byref(st)) == cg.OK
                assert st.value == cg.OK
                L.caf_future_release(f)
            kms1, nl1 = s.drain_kernel_ms()
            pk.append((kms1, nl1))
        pdt = sum(k for k, _ in pk) * 1e-3 / reps
        attain = float(np.maximum(2 * sizes ** 3 / MFMA_PEAK[dtype],
                                  nn * (2 * esz + 4) / HBM_PEAK).sum())
        return {"msgs_per_s": count / dt, "tflops": flops / dt / 1e12,
                "kernel_tflops": flops / kdt / 1e12, "kernel_ms_per_batch": kdt * 1e3,
                "mfma_frac": flops / kdt / MFMA_PEAK[dtype],
                "hbm_gbs": bytes_ / kdt / 1e9, "hbm_frac": bytes_ / kdt / HBM_PEAK,
                "attainable_ms": attain * 1e3, "frac_of_attainable": attain / kdt,
                "prefilled": {"kernel_ms_per_batch": pdt * 1e3,
                              "launches_per_batch": sum(n for _, n in pk) / reps,
                              "kernel_tflops": flops / pdt / 1e12,
                              "mfma_frac": flops / pdt / MFMA_PEAK[dtype],
                              "hbm_frac": bytes_ / pdt / HBM_PEAK,
                              "frac_of_attainable": attain / pdt},
                "flop_per_batch": flops, "bytes_per_batch": bytes_}
    finally:
        s.shutdown()


def pipeline_leg(cg, torch, chains=100000, n=128, window=1024, seed=0):
    """GEMM (n = 128, fp32) -> tanh -> row sum chains: device forwarding vs
    host-mediated forwarding through the same actors."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    A = torch.rand(chains * n * n, generator=g, device="cuda") * 2 - 1
    B = torch.rand(chains * n * n, generator=g, device="cuda") * 2 - 1
    out = {}
    # device: the drain forwards each reply on the GPU; host: the driver
    # re-sends each reply; plain / plain_graph: one launch per stage in
    # stream order (direct, or one replayed graph per chain).
    for form in ("device", "host", "plain", "plain_graph"):
        mode = form if form.startswith("plain") else "persistent"
        s = cg.System(mode=mode, arena_bytes=4 << 30, ring_slots=4096)
        try:
            rs = s.spawn(cg.BHV_ROWSUM, n=n)
            th_fwd = s.spawn(cg.BHV_TANH, n=n, forward_to=rs)
            th = s.spawn(cg.BHV_TANH, n=n)
            gm = s.spawn(cg.BHV_GEMM, n=n)
            args = np.zeros(1, cg.NP_GEMM)
            args["n"] = n
            args["in_dtype"] = cg.F32
            idx = np.arange(chains, dtype=np.uint64)
            bufs = np.zeros(chains * 2, cg.NP_BUF)
            bufs["data"][0::2] = A.data_ptr() + idx * (n * n * 4)
            bufs["data"][1::2] = B.data_ptr() + idx * (n * n * 4)
            bufs["numel"] = n * n
            bufs["dtype"] = cg.F32
            bufs["on_device"] = 1
            msgs = np.zeros(chains, cg.NP_MSG)
            msgs["actor"] = gm
            msgs["n_in"] = 2
            msgs["args"] = args.ctypes.data
            msgs["args_bytes"] = args.itemsize
            msgs["in_"] = bufs.ctypes.data + idx * 2 * bufs.itemsize
            if form != "host":
                msgs["forward_to"] = th_fwd
            torch.cuda.synchronize()
            keep = (args, bufs)
            hops = (th, rs) if form == "host" else ()
            cg.drive_array(s, msgs[:2048], keep, window=window, chain_hops=len(hops),
                           hop_actors=hops)
            rc, lat, st, el = cg.drive_array(s, msgs, keep, window=window,
                                             chain_hops=len(hops), hop_actors=hops)
            assert rc == cg.OK and (st == cg.OK).all(), (rc, np.unique(st))
            p50, p99 = percentiles(lat)
            out[form] = {"chains_per_s": chains / el, "p50_us": p50, "p99_us": p99}
        finally:
            s.shutdown()
    # per chain: 2 n^3 flop; unfused bytes: GEMM reads A, B and writes C, tanh
    # reads and writes n^2 floats, the row sum reads n^2 and writes n floats
    flop = 2.0 * n ** 3
    nbytes = 4.0 * (3 * n * n + 2 * n * n + n * n + n)
    for form in ("device", "host", "plain", "plain_graph"):
        r = out[form]["chains_per_s"]
        out[form]["hbm_frac"] = round(r * nbytes / HBM_PEAK, 4)
        out[form]["mfma_frac"] = round(r * flop / MFMA_PEAK["f32"], 4)
    out["bytes_per_chain"] = nbytes
    out["flop_per_chain"] = flop
    out["device_over_host"] = round(out["device"]["chains_per_s"] / out["host"]["chains_per_s"], 2)
    out["device_over_plain"] = round(out["device"]["chains_per_s"] / out["plain"]["chains_per_s"], 2)
    return out


def offload_leg(cg, torch, reps=3, threads=None):
    """The Sec. 7.5 experiment: the paper's 1920x1080 image of
    [-0.5-0.7375i, 0.1-0.1375i] in float at max_iter 1200 and 120, with the
    GPU actor's share of the rows going from 0 to 100% in steps of 10% and
    the rest on the CPU actors (host worker threads).  Median wall time per
    image of `reps` runs, and when each share was complete.  The whole image
    ends in host memory either way (the GPU share is copied back)."""
    from paper_1505_07368_amd import gen
    threads = threads or min(16, os.cpu_count() or 1)
    s = cg.System(mode="batched", arena_bytes=1 << 30, ring_slots=256)
    try:
        a = s.spawn(cg.BHV_MANDELBROT)
        out = {"cpu_threads": threads, "image": "1920x1080 [-0.5-0.7375i, 0.1-0.1375i], fp32"}
        for mi in (1200, 120):
            vp = gen.paper_replica_viewport(mi)
            image = cg.caf_mandel_args(vp.re_min, vp.im_min, vp.step_re, vp.step_im, vp.width,
                                       vp.height, 0, vp.height, mi, cg.F32)
            stage = torch.empty(vp.height * vp.width, dtype=torch.uint16, device="cuda")
            host = np.zeros((vp.height, vp.width), np.uint16)
            s.offload_mandel(a, image, vp.height, threads, stage, host)  # warm-up
            iters = int(host.astype(np.int64).sum())
            rows = []
            for k in range(11):
                g = round(vp.height * k / 10)
                ts = [s.offload_mandel(a, image, g, threads, stage, host)[1] for _ in range(reps)]
                med = lambda key: sorted(t[key] for t in ts)[reps // 2] / 1e6
                rows.append({"gpu_share": k / 10, "gpu_rows": g, "ms": med("total_ns"),
                             "gpu_done_ms": med("gpu_done_ns"), "cpu_done_ms": med("cpu_done_ns")})
                log(f"[bench] offload max_iter {mi}: GPU share {k * 10}% -> {rows[-1]['ms']:.2f} ms")
            out[f"max_iter_{mi}"] = {"iters_per_image": iters, "by_share": rows}
        return out
    finally:
        s.shutdown()


def serving_leg(cg, torch, rate, duration_s=2.0, seed=0, ring=8192, budget=32 << 30,
                blocking=False, tune=None):
    """Open-loop Poisson arrivals: 70 % Mandelbrot squares (64^2..512^2,
    max_iter 256..4096, boundary viewports, fp32), 30 % fp32 GEMM with n in
    {32..512}; admission by HBM budget and mailbox slots; latency from the
    scheduled arrival.  Non-blocking: a request that does not fit is refused
    (counted).  Blocking: it waits, in arrival order, until earlier replies
    free a slot and arena memory.  Replies are library-allocated from the
    arena, so the budget binds.  The work done is counted over the completed
    requests: Mandelbrot iterations (each message's exact count sum, from a
    closed-loop pass over the same messages before the timed run) and GEMM
    flops (2 n^3).  tune: the autotuner's full_wgs_per_cu and max_batch."""
    from paper_1505_07368_amd import autotune, gen
    tune = tune or {}
    d = gen.serving_mix_arrays(seed, rate, duration_s)
    cnt = d["arrival_ns"].size
    s = cg.System(mode="persistent", arena_bytes=budget, ring_slots=ring, blocking=blocking,
                  max_batch=tune.get("max_batch", 1024),
                  full_wgs_per_cu=tune.get("full_wgs_per_cu", 0))
    try:
        m = s.spawn(cg.BHV_MANDELBROT)
        gm = s.spawn(cg.BHV_GEMM)
        msgs, keep = autotune.mix_messages(cg, torch, d, m, gm, pool_seed=seed)
        ism = d["is_mandel"]
        iters = mandel_work(cg, torch, s, msgs[ism], keep, d["side"][ism], window=ring // 2)
        torch.cuda.synchronize()
        # the driver's own bookkeeping never limits: the library admits
        rc, lat, st, el = cg.drive_array(s, msgs, keep, window=cnt, arrival_ns=d["arrival_ns"])
        ok = st == cg.OK
        rej = st == cg.E_OVERLOAD
        assert ((st == cg.OK) | rej).all(), np.unique(st)
        p50, p99 = percentiles(lat[ok])
        pm50, pm99 = percentiles(lat[ok & ism])
        gn = d["gemm_n"].astype(np.float64)
        return {"offered_per_s": cnt / duration_s, "messages": int(cnt), "budget_bytes": budget,
                "admission": "blocking" if blocking else "non-blocking",
                "completed": int(ok.sum()), "rejected": int(rej.sum()),
                "goodput_per_s": float(ok.sum()) / el, "elapsed_s": el,
                "p50_us": p50, "p99_us": p99, "mandel_p50_us": pm50, "mandel_p99_us": pm99,
                "mandel_giter_s": float(iters[ok[ism]].sum()) / el / 1e9,
                "gemm_tflops": float((2 * gn[ok & ~ism] ** 3).sum()) / el / 1e12}
    finally:
        s.shutdown()


def mandel_work(cg, torch, s, msgs, keep, side, window, chunk_px=1 << 27):
    """Exact iterations of each Mandelbrot message: messages of one square
    size at a time are run in closed-loop chunks with their replies written
    into a device pool [k, side * side], and each reply's counts are summed
    (counts <= 4096 fit int16)."""
    out = np.zeros(msgs.size, np.int64)
    side = side.astype(np.int64)
    for sd in np.unique(side):
        sel = np.nonzero(side == sd)[0]
        px = int(sd * sd)
        k = max(1, min(len(sel), chunk_px // px))
        for c0 in range(0, len(sel), k):
            ids = sel[c0:c0 + k]
            buf = torch.empty((len(ids), px), dtype=torch.int16, device="cuda")
            part = msgs[ids].copy()
            part["out"]["data"] = buf.data_ptr() + 2 * px * np.arange(len(ids), dtype=np.uint64)
            part["out"]["numel"] = px
            part["out"]["dtype"] = cg.U16
            part["out"]["on_device"] = 1
            torch.cuda.synchronize()
            rc, _, st, _ = cg.drive_array(s, part, keep, window=min(len(part), window))
            assert rc == cg.OK and (st == cg.OK).all(), (rc, np.unique(st))
            torch.cuda.synchronize()
            out[ids] = buf.to(torch.int32).sum(1, dtype=torch.int64).cpu().numpy()
            del buf
    return out


def cpu_oracle_tile(args):
    import oracle
    vp, r0, rows = args
    t = time.perf_counter()
    img = oracle.mandelbrot(vp.re_min, vp.im_min, vp.step_re, vp.step_im, vp.width, r0, rows,
                            vp.max_iter, "f32")
    return int(img.sum(dtype=np.int64)), time.perf_counter() - t


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def usable_cores(cap=16) -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(cap, n))


def cpu_baseline(seeds=tuple(range(8)), single_seed=0):
    """The oracle, as it stands, on the host's cores, over the headline
    workload's tile messages: K independent single-threaded instances over a
    disjoint partition of all 136 messages (K = the usable cores, at most 16),
    and one instance alone over the 17 messages of one image."""
    import multiprocessing as mp
    from paper_1505_07368_amd import gen
    import oracle
    oracle.lib()  # built before forking
    work = []
    for seed in seeds:
        vp = gen.boundary_viewport(seed)
        work += [(vp, r0, rows) for r0, rows in gen.row_tiles(vp.height, 64)]
    cores = usable_cores()
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(cpu_oracle_tile, work, chunksize=1)
    dt = time.perf_counter() - t0
    iters = sum(r[0] for r in res)
    vp = gen.boundary_viewport(single_seed)
    one = [(vp, r0, rows) for r0, rows in gen.row_tiles(vp.height, 64)]
    t1 = time.perf_counter()
    it1 = sum(cpu_oracle_tile(w)[0] for w in one)
    dt1 = time.perf_counter() - t1
    return {"value": iters / dt / 1e9, "unit": "Giter/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"all {len(work)} tile messages of one step ({len(seeds)} images "
                      f"1920x1080, max_iter 1000, fp32), {iters / 1e9:.2f} Giter in "
                      f"{dt:.2f} s wall on {cores} single-threaded oracle processes",
            "single_core": {"value": it1 / dt1 / 1e9, "unit": "Giter/s", "cores": 1,
                            "sample": f"the {len(one)} tile messages of image {single_seed}, "
                                      f"{it1 / 1e9:.2f} Giter in {dt1:.2f} s"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--quick", action="store_true", help="headline leg only")
    ap.add_argument("--legs", default="fp64,colour,forms,small,gemm,pipeline,serving,offload",
                    help="comma list of the legs to run beside the headline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serving-tight-nonblocking", action="store_true",
                    help="also run the 64 MiB serving case with non-blocking admission")
    ap.add_argument("--gemm-dtypes", default="f32,bf16", help="GEMM leg input types")
    ap.add_argument("--gemm-tile-class", default="",
                    help="GEMM leg tile choice per size class (e.g. 64,128,256,256) instead "
                    "of the autotuned one")
    ap.add_argument("--headline-fp", default="f32", choices=("f32", "f64"),
                    help="precision of the headline leg (f64: for profiling the double "
                    "path; the reported metric is defined in f32)")
    ap.add_argument("--interior", action="store_true",
                    help="with --quick: also time the no-divergence interior viewport")
    ap.add_argument("--dispersion", type=int, default=100,
                    help="further headline steps timed one by one (mean, std); 0: none")
    ap.add_argument("--no-tune", action="store_true", help="library defaults, no autotuning")
    ap.add_argument("--mandel-tile-px", type=int, default=0,
                    help="headline work tile (pixels) instead of the autotuned one")
    ap.add_argument("--grid", type=int, default=-1,
                    help="headline drain grid (0: all resident) instead of the autotuned one")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the compute-actor path runs on a single MI355X; "
              "--gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1505_07368_amd import binding as cg
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.init()
    seeds = list(range(8))

    from paper_1505_07368_amd import autotune, gen
    cache = os.path.join(ROOT, "paper_1505_07368_amd", "autotune_cache.json")
    vps = [gen.boundary_viewport(sd) for sd in seeds]
    tuned = {}
    if args.mandel_tile_px or args.grid >= 0:
        tuned["mandel"] = {"mandel_tile_px": args.mandel_tile_px, "grid": max(0, args.grid)}
    elif not args.no_tune:
        log("[bench] autotune (mandelbrot work tile, grid)")
        tuned["mandel"] = autotune.tune_mandel(torch, vps, cache_path=cache)
    log("[bench] batched fp32 (headline)")
    hfp = args.headline_fp
    head = mandel_leg(cg, torch, "batched", cg.F32 if hfp == "f32" else cg.F64, args.steps,
                      args.warmup, seeds, True, tune=tuned.get("mandel"),
                      dispersion_reps=args.dispersion)
    result = {
        "metric": "GPU-actor msgs/s + Mandelbrot Giter/s; p50/p99 reply latency vs 1-launch/msg",
        "value": round(head["giter_s"], 2),
        "unit": "Giter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": hfp,
        "data": "synthetic",
        "config": {"workload": "mandelbrot 1920x1080 max_iter 1000, 8 seeded boundary "
                               "viewports x 17 row-tile messages (64 rows, last 56), "
                               f"{'fp32' if hfp == 'f32' else 'fp64'}, batched mailbox drain",
                   "images": len(seeds), "tile_rows": 64, "max_iter": 1000,
                   "messages_per_step": head["messages_per_step"],
                   "iters_per_step": head["iters_per_step"]},
        "msgs_per_s": round(head["msgs_per_s"], 1),
        "p50_us": head["p50_us"],
        "p99_us": head["p99_us"],
        "step_ms_mean": round(head["step_ms_mean"], 4),
        "step_ms_std": round(head["step_ms_std"], 4),
    }
    if "dispersion" in head:
        result["dispersion"] = head["dispersion"]
    kms = head.get("kernel_ms_total")
    if kms:
        per_launch_ms = kms / head["kernel_launches"]
        ops = head["iters_per_step"] * args.steps * OPS_PER_ITER
        achieved = ops / (kms * 1e-3)
        result["roofline"] = {
            "bound": "alu", "achieved": round(achieved / 1e12, 3),
            "peak": round(VALU_PEAK[hfp] / 1e12, 3), "unit": "TFLOP/s",
            "frac": round(achieved / VALU_PEAK[hfp], 4),
            "traffic": measured_traffic() if hfp == "f32" else None,
            "kernel": "drain_kernel_light", "launches": head["kernel_launches"],
            "avg_launch_ms": round(per_launch_ms, 4), "ops_per_iter": OPS_PER_ITER,
            "ops_per_launch": head["iters_per_step"] * OPS_PER_ITER}
    if not args.quick or args.interior:
        # the loop's attainable rate: the same 136 messages over a viewport
        # where no pixel escapes (every lane busy until max_iter)
        log("[bench] batched fp32, interior viewport (no divergence)")
        ivp = [interior_viewport()] * len(seeds)
        inner = mandel_leg(cg, torch, "batched", cg.F32, max(2, args.steps // 2), 1, seeds,
                           True, tune=tuned.get("mandel"), viewports=ivp)
        result["interior"] = {k: inner[k] for k in ("giter_s", "iters_per_step", "ms_per_step")}
        if inner.get("kernel_ms_total"):
            ops_s = (inner["iters_per_step"] * max(2, args.steps // 2) * OPS_PER_ITER
                     / (inner["kernel_ms_total"] * 1e-3))
            result["interior"]["alu_frac"] = round(ops_s / VALU_PEAK["f32"], 4)
            if "roofline" in result:
                result["roofline"]["of_interior"] = round(
                    result["roofline"]["achieved"] * 1e12 / ops_s, 4)
    legs = set() if args.quick else set(args.legs.split(","))

    current = [None]
    start_leg_watchdog(result, tuned, current)

    def run_leg(name, fn):
        """Runs one leg beside the headline; a failure is recorded in its
        place (with the traceback on stderr) so the headline line still
        prints, and a leg that stops making progress ends the run with the
        results so far (start_leg_watchdog)."""
        current[0] = name
        _PROGRESS[0] = time.monotonic()
        try:
            fn()
        except Exception as e:  # noqa: BLE001 -- any leg failure is reported, not fatal
            import traceback
            traceback.print_exc()
            result[name] = {"error": f"{type(e).__name__}: {e}"}
        finally:
            current[0] = None

    def leg_fp64():
        log("[bench] batched fp64")
        f64 = mandel_leg(cg, torch, "batched", cg.F64, max(2, args.steps // 2), 1, seeds, True,
                         tune=tuned.get("mandel"))
        result["fp64"] = {k: f64[k] for k in ("giter_s", "msgs_per_s", "p50_us", "p99_us",
                                              "iters_per_step")}
        if f64.get("kernel_ms_total"):
            result["fp64"]["alu_frac"] = round(
                f64["iters_per_step"] * max(2, args.steps // 2) * OPS_PER_ITER
                / (f64["kernel_ms_total"] * 1e-3) / VALU_PEAK["f64"], 4)

    def leg_colour():
        # the same batch through an actor spawned with a 256-entry palette:
        # the colour map is fused into the tile's store (4-byte pixels)
        log("[bench] batched fp32, colour replies")
        g = torch.Generator(device="cuda")
        g.manual_seed(3)
        pal = torch.randint(-2 ** 31, 2 ** 31 - 1, (256,), generator=g, device="cuda",
                            dtype=torch.int32)
        col = mandel_leg(cg, torch, "batched", cg.F32, args.steps, args.warmup, seeds, True,
                         tune=tuned.get("mandel"), palette=pal)
        result["colour"] = {k: col[k] for k in ("giter_s", "msgs_per_s", "p50_us", "p99_us")}
        result["colour"]["vs_counts"] = round(col["giter_s"] / result["value"], 4)

    def leg_forms():
        for mode in ("persistent", "plain", "plain_graph"):
            log(f"[bench] {mode} fp32")
            r = mandel_leg(cg, torch, mode, cg.F32, max(2, args.steps // 2), 1, seeds,
                           tune=tuned.get("mandel") if mode != "plain" else None)
            result[mode] = {k: r[k] for k in ("giter_s", "msgs_per_s", "p50_us", "p99_us")}

    def leg_small():
        small = {}
        result["small_messages"] = small
        for kind, count in (("echo", 10000), ("mandel64", 4096), ("gemm64", 4096),
                            ("hash", 4096)):
            for window in ((1, 64, 1024) if kind == "echo" else (256,)):
                row = {}
                for mode in ("plain", "plain_graph", "batched", "persistent"):
                    log(f"[bench] small {kind} window {window} {mode}")
                    row[mode] = small_leg(cg, torch, mode, kind, count, window)
                row["persistent_over_plain"] = round(
                    row["persistent"]["msgs_per_s"] / row["plain"]["msgs_per_s"], 2)
                row["batched_over_plain"] = round(
                    row["batched"]["msgs_per_s"] / row["plain"]["msgs_per_s"], 2)
                small[f"{kind}_w{window}"] = row

    def leg_gemm(dt):
        tc = (0, 0, 0, 0)
        if args.gemm_tile_class:
            tc = tuple(int(x) for x in args.gemm_tile_class.split(","))
            assert len(tc) == 4, "--gemm-tile-class takes four edges"
        elif not args.no_tune:
            log(f"[bench] autotune gemm {dt}")
            tc = autotune.tune_gemm(torch, dtype=dt, cache_path=cache)
            tuned[f"gemm_{dt}_tile_class"] = tc
        log(f"[bench] gemm batch {dt}")
        result[f"gemm_{dt}"] = gemm_leg(cg, torch, dt, tile_class=tc)
        result[f"gemm_{dt}"]["tile_class"] = list(tc)

    def leg_pipeline():
        log("[bench] pipeline")
        result["pipeline"] = pipeline_leg(cg, torch)

    def leg_serving():
        mix = {}
        if not args.no_tune:
            log("[bench] autotune (serving mix: full-variant occupancy, max_batch)")
            mix = autotune.tune_mix(torch, cache_path=cache)
            tuned["serving_mix"] = mix
        serving = {}
        result["serving"] = serving
        for rate in (1e4, 1e5, 1e6):
            # at most 2e5 arrivals per rate: above capacity the backlog, not
            # the arrival window, sets the run time
            dur = min(2.0, 2e5 / rate)
            log(f"[bench] serving {rate:g}/s for {dur:g} s")
            serving[f"{rate:g}"] = serving_leg(cg, torch, rate, duration_s=dur, tune=mix)
        # a 64 MiB budget: admission binds on arena memory.  The non-blocking
        # form stalled once (no reply for minutes, cause not found) and runs
        # only when asked for.
        for blocking in ((False, True) if args.serving_tight_nonblocking else (True,)):
            log(f"[bench] serving 1e5/s for 0.5 s, 64 MiB budget, blocking={blocking}")
            serving["1e5_64MiB_" + ("blocking" if blocking else "nonblocking")] = serving_leg(
                cg, torch, 1e5, duration_s=0.5, budget=64 << 20, blocking=blocking, tune=mix)

    def leg_offload():
        result["offload"] = offload_leg(cg, torch)

    def leg_cpu():
        log("[bench] cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline()

    for name, fn in (("fp64", leg_fp64), ("colour", leg_colour), ("forms", leg_forms),
                     ("small", leg_small)):
        if name in legs:
            run_leg(name, fn)
    # the CPU baseline and the offload leg before serving, the longest and
    # most loaded leg: if a leg stalls, the watchdog's line still has them.
    # The GEMM batches, bound by memory traffic, run late: right after a
    # heavy run (a test suite) their first minutes have been slower.
    if not args.no_cpu:
        run_leg("cpu_baseline", leg_cpu)
    for name, fn in (("pipeline", leg_pipeline), ("offload", leg_offload)):
        if name in legs:
            run_leg(name, fn)
    if "gemm" in legs:
        for dt in args.gemm_dtypes.split(","):
            run_leg(f"gemm_{dt}", lambda dt=dt: leg_gemm(dt))
    if "serving" in legs:
        run_leg("serving", leg_serving)
    result["tuned"] = tuned
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
