"""Parity at the benchmark workloads' full sizes (GPU).

Each test runs a workload the benchmark times, through the same entry points
and the same System configuration (delivery mode, ring, work-tile size and
grid candidates of the autotuner), and compares the outputs with the oracle:

  * the headline image batch: 8 boundary viewports of 1920x1080 at max_iter
    1000, 17 row-tile messages each (the last has 56 rows), fp32 and fp64:
    every pixel of every image against the oracle, and the escape-count sums
    against the oracle's stored sums (tests/golden/headline_sums.json);
  * the grouped GEMM batch: n drawn from {64, 128, 256, 512}, fp32 and bf16,
    both output-tile edges;
  * the serving mix: Mandelbrot squares 64^2..512^2 at max_iter 256..4096 and
    fp32 GEMMs n = 32..512 through the non-blocking persistent system, every
    reply compared in full;
  * the GEMM leg's 4096-request batch (every 64th product against the
    oracle) and the pipeline leg's 100,000 chains as the benchmark runs them.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1505_07368_amd import gen
from tests import oracle_par
from tests.gpu_util import rel_fro

pytestmark = pytest.mark.gpu

SEEDS = list(range(8))
GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "headline_sums.json")))

_ORACLE_IMAGES = {}


def oracle_images(fp):
    """The oracle's eight headline images (computed once per session)."""
    if fp not in _ORACLE_IMAGES:
        _ORACLE_IMAGES[fp] = oracle_par.mandel_images([gen.boundary_viewport(sd) for sd in SEEDS],
                                                      fp)
    return _ORACLE_IMAGES[fp]


def _image_batch(cg, torch, s, fp):
    a = s.spawn(cg.BHV_MANDELBROT)
    msgs, imgs = [], []
    for seed in SEEDS:
        vp = gen.boundary_viewport(seed)
        img = torch.zeros(vp.height * vp.width, dtype=torch.uint16, device="cuda")
        imgs.append((vp, img))
        for r0, rows in gen.row_tiles(vp.height, 64):
            view = img[r0 * vp.width:(r0 + rows) * vp.width]
            msgs.append({"actor": a, "args": cg.mandel_args(vp, row0=r0, rows=rows, fp=fp),
                         "out": view})
    torch.cuda.synchronize()
    rc, _, st, _ = s.drive(msgs, window=len(msgs))
    assert rc == cg.OK and (st == cg.OK).all(), (rc, np.unique(st))
    assert len(msgs) == 136
    return imgs


def _check_images(imgs, fp):
    """Every pixel of every image against the oracle, and the sums against
    the oracle's stored sums."""
    refs = oracle_images(fp)
    total = 0
    for seed, (vp, img), ref in zip(SEEDS, imgs, refs):
        host = img.cpu().numpy().reshape(vp.height, vp.width)
        bad = host != ref
        assert not bad.any(), (seed, int(bad.sum()), np.argwhere(bad)[:4].tolist())
        s = int(host.sum(dtype=np.int64))
        assert s == GOLDEN[fp]["images"][seed]["sum"], (seed, s)
        total += s
    assert total == GOLDEN[fp]["total"]


@pytest.mark.parametrize("px,half_grid", [(512, False), (1024, False), (2048, False),
                                          (4096, False), (2048, True)])
def test_headline_batch_tile_candidates(px, half_grid):
    """Every (work tile, grid) candidate the autotuner may pick, in float."""
    import torch
    from paper_1505_07368_amd import binding as cg
    grid = 0
    if half_grid:
        grid = int(torch.cuda.get_device_properties(0).multi_processor_count * 5 * 0.5)
    s = cg.System(mode="batched", arena_bytes=1 << 30, ring_slots=4096, mandel_tile_px=px,
                  grid=grid)
    try:
        imgs = _image_batch(cg, torch, s, cg.F32)
    finally:
        s.shutdown()
    _check_images(imgs, "f32")


@pytest.mark.parametrize("mode", ["batched", "persistent", "plain"])
def test_headline_batch_double(mode):
    import torch
    from paper_1505_07368_amd import binding as cg
    s = cg.System(mode=mode, arena_bytes=1 << 30, ring_slots=4096)
    try:
        imgs = _image_batch(cg, torch, s, cg.F64)
    finally:
        s.shutdown()
    _check_images(imgs, "f64")


def _gemm_batch(cg, torch, s, sizes, dtype):
    a = s.spawn(cg.BHV_GEMM)
    code = cg.F32 if dtype == "f32" else cg.BF16
    msgs, io = [], []
    for i, n in enumerate(sizes):
        A, B = gen.gemm_pair(1000 + i, int(n), dtype)
        if dtype == "f32":
            At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        else:
            At = torch.from_numpy(A.view(np.int16)).cuda().view(torch.bfloat16)
            Bt = torch.from_numpy(B.view(np.int16)).cuda().view(torch.bfloat16)
        C = torch.full((int(n) * int(n),), float("nan"), device="cuda")
        io.append((A, B, C, At, Bt))
        msgs.append({"actor": a, "args": cg.caf_gemm_args(int(n), code), "inputs": [At, Bt],
                     "out": C})
    torch.cuda.synchronize()
    rc, _, st, _ = s.drive(msgs, window=len(msgs))
    assert rc == cg.OK and (st == cg.OK).all(), (rc, np.unique(st))
    return io


@pytest.mark.parametrize("wgs", [2, 3])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("te", [64, 128, 256])
def test_gemm_batch_sampled(dtype, te, wgs):
    """A drained batch of mixed sizes with every tile choice and both full
    drain variants (2 workgroups per CU with 64-deep bf16 slices, 3 with
    32-deep ones; 256 = 128 x 256 bf16 tiles in the wide variant, whose
    square tiles are calls -- fp32 products run there as 128 x 128, and the
    3-workgroup variant replaces 256 by 128); one message of each size
    (n = 512 included) checked against the FP64 oracle, every output
    checked finite."""
    import torch
    from paper_1505_07368_amd import binding as cg
    sizes = gen.gemm_sizes(0, 48)
    s = cg.System(mode="batched", arena_bytes=1 << 30, ring_slots=64, max_batch=1024,
                  gemm_tile_class=(te, te, te, te), full_wgs_per_cu=wgs)
    try:
        io = _gemm_batch(cg, torch, s, sizes, dtype)
    finally:
        s.shutdown()
    seen = set()
    for n, (A, B, C, _, _) in zip(sizes, io):
        c = C.cpu().numpy()
        assert np.isfinite(c).all(), n
        if int(n) in seen:
            continue
        seen.add(int(n))
        err = rel_fro(c.reshape(int(n), int(n)), oracle.gemm(A, B, dtype))
        assert err <= 1e-5, (int(n), err)
    assert seen == {64, 128, 256, 512}


@pytest.mark.parametrize("wgs, grouping", [(2, "kind"), (3, "kind"), (2, "lpt"), (3, "fifo")])
def test_serving_mix_full(wgs, grouping):
    """Every request of a 0.1 s serving-mix run at 1e4 arrivals/s (about
    1,000 messages, issued as one burst through the same system
    configuration as the serving benchmark, with either full drain variant
    and each layout of a drained batch): every Mandelbrot square compared
    pixel for pixel, every GEMM in full (relative Frobenius error)."""
    import torch
    from paper_1505_07368_amd import binding as cg
    d = gen.serving_mix_arrays(0, 1e4, 0.1)
    cnt = d["arrival_ns"].size
    assert cnt >= 900
    s = cg.System(mode="persistent", arena_bytes=32 << 30, ring_slots=8192, blocking=False,
                  full_wgs_per_cu=wgs, grouping=grouping)
    try:
        m = s.spawn(cg.BHV_MANDELBROT)
        gm = s.spawn(cg.BHV_GEMM)
        msgs, cases = [], []
        for i in range(cnt):
            if d["is_mandel"][i]:
                side, mi = int(d["side"][i]), int(d["max_iter"][i])
                vp = gen.Viewport(float(d["re_min"][i]), float(d["im_min"][i]),
                                  float(d["step"][i]), float(d["step"][i]), side, side, mi)
                out = torch.zeros(side * side, dtype=torch.uint16, device="cuda")
                msgs.append({"actor": m, "args": cg.mandel_args(vp), "out": out})
                cases.append(("mandel", vp, out))
            else:
                n = int(d["gemm_n"][i])
                A, B = gen.gemm_pair(2000 + i, n)
                At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
                C = torch.full((n * n,), float("nan"), device="cuda")
                msgs.append({"actor": gm, "args": cg.caf_gemm_args(n, cg.F32),
                             "inputs": [At, Bt], "out": C})
                cases.append(("gemm", (A, B), C))
        torch.cuda.synchronize()
        rc, _, st, _ = s.drive(msgs, window=len(msgs))
        assert rc == cg.OK and (st == cg.OK).all(), (rc, np.unique(st))
    finally:
        s.shutdown()
    from concurrent.futures import ThreadPoolExecutor
    oracle.lib()

    def ref_of(case):
        kind, x, _ = case
        if kind == "mandel":
            vp = x
            return oracle.mandelbrot(vp.re_min, vp.im_min, vp.step_re, vp.step_im, vp.width, 0,
                                     vp.height, vp.max_iter, "f32")
        return oracle.gemm(x[0], x[1])

    with ThreadPoolExecutor(oracle_par.threads()) as ex:
        refs = list(ex.map(ref_of, cases))
    nm = 0
    for (kind, x, out), ref in zip(cases, refs):
        if kind == "mandel":
            vp = x
            host = out.cpu().numpy().reshape(vp.height, vp.width)
            assert (host == ref).all(), (vp, int((host != ref).sum()))
            nm += 1
        else:
            n = x[0].shape[0]
            err = rel_fro(out.cpu().numpy().reshape(n, n), ref)
            assert err <= 1e-5, (n, err)
    assert nm >= 600


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_gemm_bench_batch_full_size(dtype, tile_class=(0, 0, 0, 0)):
    """The benchmark's GEMM leg as timed: 4096 requests, n ~ U{64..512},
    inputs drawn on the device, batched drain with max_batch 1024.  Every
    output is checked finite; every 64th product (and one of each size)
    against the oracle (inputs copied back)."""
    import torch
    from paper_1505_07368_amd import binding as cg
    count = 4096
    sizes = gen.gemm_sizes(0, count).astype(np.int64)
    nn = sizes * sizes
    offs = np.concatenate([[0], np.cumsum(nn)[:-1]])
    total = int(nn.sum())
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    A = torch.rand(total, generator=g, device="cuda") * 2 - 1
    B = torch.rand(total, generator=g, device="cuda") * 2 - 1
    code = cg.F32
    if dtype == "bf16":
        A, B, code = A.to(torch.bfloat16), B.to(torch.bfloat16), cg.BF16
    C = torch.full((total,), float("nan"), device="cuda")
    esz = A.element_size()
    s = cg.System(mode="batched", arena_bytes=1 << 30, ring_slots=count, max_batch=1024,
                  gemm_tile_class=tile_class)
    try:
        a = s.spawn(cg.BHV_GEMM)
        args = np.zeros(count, cg.NP_GEMM)
        args["n"] = sizes
        args["in_dtype"] = code
        bufs = np.zeros(2 * count, cg.NP_BUF)
        bufs["data"][0::2] = A.data_ptr() + offs.astype(np.uint64) * esz
        bufs["data"][1::2] = B.data_ptr() + offs.astype(np.uint64) * esz
        bufs["numel"][0::2] = nn
        bufs["numel"][1::2] = nn
        bufs["dtype"] = code
        bufs["on_device"] = 1
        idx = np.arange(count, dtype=np.uint64)
        msgs = np.zeros(count, cg.NP_MSG)
        msgs["actor"] = a
        msgs["n_in"] = 2
        msgs["args"] = args.ctypes.data + idx * args.itemsize
        msgs["args_bytes"] = args.itemsize
        msgs["in_"] = bufs.ctypes.data + idx * 2 * bufs.itemsize
        msgs["out"]["data"] = C.data_ptr() + offs.astype(np.uint64) * 4
        msgs["out"]["numel"] = nn
        msgs["out"]["dtype"] = cg.F32
        msgs["out"]["on_device"] = 1
        torch.cuda.synchronize()
        rc, _, st, _ = cg.drive_array(s, msgs, (args, bufs, A, B, C), window=count)
        assert rc == cg.OK and (st == cg.OK).all(), (rc, np.unique(st))
    finally:
        s.shutdown()
    assert torch.isfinite(C).all()
    picks = list(range(0, count, 64))
    for size in (64, 128, 256, 512):  # and at least one product of every size
        picks.append(int(np.nonzero(sizes == size)[0][0]))
    pairs, outs = [], []
    for i in sorted(set(picks)):
        size, o = int(sizes[i]), int(offs[i])
        m = size * size
        if dtype == "bf16":
            Ah = A[o:o + m].view(torch.int16).cpu().numpy().view(np.uint16).reshape(size, size)
            Bh = B[o:o + m].view(torch.int16).cpu().numpy().view(np.uint16).reshape(size, size)
        else:
            Ah = A[o:o + m].cpu().numpy().reshape(size, size)
            Bh = B[o:o + m].cpu().numpy().reshape(size, size)
        pairs.append((Ah, Bh))
        outs.append((i, C[o:o + m].cpu().numpy().reshape(size, size)))
    for (i, got), ref in zip(outs, oracle_par.gemms(pairs, dtype)):
        err = rel_fro(got, ref)
        assert err <= 1e-5, (i, got.shape[0], err)


@pytest.mark.parametrize("wgs", [2, 3])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_gemm_ragged_runs_sampled(dtype, wgs):
    """2048 requests with ragged n (72, 100, 136, 200, 264: partial last
    k slice, both tile edges, n % 8 != 0 for 100) published in two drained
    batches, so workgroups claim several consecutive tiles of one product and
    run them as one stream.  Every output finite; 40 products spread over
    the batch against the FP64 oracle."""
    import torch
    from paper_1505_07368_amd import binding as cg
    count = 2048
    sizes = np.resize(np.array([72, 100, 136, 200, 264], np.int64), count)
    nn = sizes * sizes
    offs = np.concatenate([[0], np.cumsum(nn)[:-1]])
    total = int(nn.sum())
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    A = torch.rand(total, generator=g, device="cuda") * 2 - 1
    B = torch.rand(total, generator=g, device="cuda") * 2 - 1
    code = cg.F32
    if dtype == "bf16":
        A, B, code = A.to(torch.bfloat16), B.to(torch.bfloat16), cg.BF16
    C = torch.full((total,), float("nan"), device="cuda")
    esz = A.element_size()
    s = cg.System(mode="batched", arena_bytes=1 << 30, ring_slots=count, max_batch=1024,
                  full_wgs_per_cu=wgs)
    try:
        a = s.spawn(cg.BHV_GEMM)
        args = np.zeros(count, cg.NP_GEMM)
        args["n"] = sizes
        args["in_dtype"] = code
        bufs = np.zeros(2 * count, cg.NP_BUF)
        bufs["data"][0::2] = A.data_ptr() + offs.astype(np.uint64) * esz
        bufs["data"][1::2] = B.data_ptr() + offs.astype(np.uint64) * esz
        bufs["numel"][0::2] = nn
        bufs["numel"][1::2] = nn
        bufs["dtype"] = code
        bufs["on_device"] = 1
        idx = np.arange(count, dtype=np.uint64)
        msgs = np.zeros(count, cg.NP_MSG)
        msgs["actor"] = a
        msgs["n_in"] = 2
        msgs["args"] = args.ctypes.data + idx * args.itemsize
        msgs["args_bytes"] = args.itemsize
        msgs["in_"] = bufs.ctypes.data + idx * 2 * bufs.itemsize
        msgs["out"]["data"] = C.data_ptr() + offs.astype(np.uint64) * 4
        msgs["out"]["numel"] = nn
        msgs["out"]["dtype"] = cg.F32
        msgs["out"]["on_device"] = 1
        torch.cuda.synchronize()
        rc, _, st, _ = cg.drive_array(s, msgs, (args, bufs, A, B, C), window=count)
        assert rc == cg.OK and (st == cg.OK).all(), (rc, np.unique(st))
    finally:
        s.shutdown()
    assert torch.isfinite(C).all()
    for i in np.linspace(0, count - 1, 40).astype(int):
        size, o = int(sizes[i]), int(offs[i])
        m = size * size
        if dtype == "bf16":
            Ah = A[o:o + m].view(torch.int16).cpu().numpy().view(np.uint16).reshape(size, size)
            Bh = B[o:o + m].view(torch.int16).cpu().numpy().view(np.uint16).reshape(size, size)
        else:
            Ah = A[o:o + m].cpu().numpy().reshape(size, size)
            Bh = B[o:o + m].cpu().numpy().reshape(size, size)
        err = rel_fro(C[o:o + m].cpu().numpy().reshape(size, size), oracle.gemm(Ah, Bh, dtype))
        assert err <= 1e-5, (int(i), size, err)


def test_pipeline_bench_size_sampled():
    """The benchmark's pipeline leg at full size: 100,000 GEMM(128) -> tanh ->
    row-sum chains with device forwarding (persistent drain); every reply
    finite, sampled chains against the oracle chain."""
    import torch
    from paper_1505_07368_amd import binding as cg
    n, chains = 128, 100000
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    A = torch.rand(chains * n * n, generator=g, device="cuda") * 2 - 1
    B = torch.rand(chains * n * n, generator=g, device="cuda") * 2 - 1
    Y = torch.full((chains * n,), float("nan"), device="cuda")
    s = cg.System(mode="persistent", arena_bytes=4 << 30, ring_slots=4096)
    try:
        rs = s.spawn(cg.BHV_ROWSUM, n=n)
        th = s.spawn(cg.BHV_TANH, n=n, forward_to=rs)
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
        msgs["forward_to"] = th
        msgs["out"]["data"] = Y.data_ptr() + idx * (n * 4)
        msgs["out"]["numel"] = n
        msgs["out"]["dtype"] = cg.F32
        msgs["out"]["on_device"] = 1
        torch.cuda.synchronize()
        rc, _, st, _ = cg.drive_array(s, msgs, (args, bufs), window=1024)
        assert rc == cg.OK and (st == cg.OK).all(), (rc, np.unique(st))
    finally:
        s.shutdown()
    assert torch.isfinite(Y).all()
    for c in (0, 1, 4321, 77777, chains - 1):
        a = A[c * n * n:(c + 1) * n * n].cpu().numpy().reshape(n, n)
        b = B[c * n * n:(c + 1) * n * n].cpu().numpy().reshape(n, n)
        err = rel_fro(Y[c * n:(c + 1) * n].cpu().numpy(), oracle.chain(a, b))
        assert err <= 1e-5, (c, err)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_gemm_large_single_message(dtype):
    """One n = 1024 request (64 tiles of 128, 16 k slices) through the
    batched drain, against the FP64 oracle."""
    import torch
    from paper_1505_07368_amd import binding as cg
    n = 1024
    A, B = gen.gemm_pair(4242, n, dtype)
    if dtype == "f32":
        At, Bt, code = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), cg.F32
    else:
        At = torch.from_numpy(A.view(np.int16)).cuda().view(torch.bfloat16)
        Bt = torch.from_numpy(B.view(np.int16)).cuda().view(torch.bfloat16)
        code = cg.BF16
    s = cg.System(mode="batched", arena_bytes=64 << 20)
    try:
        g = s.spawn(cg.BHV_GEMM)
        torch.cuda.synchronize()
        st, C = s.request(g, cg.caf_gemm_args(n, code), inputs=[At, Bt]).result()
        assert st == cg.OK
        c = C.cpu().numpy().reshape(n, n)
    finally:
        s.shutdown()
    err = rel_fro(c, oracle.gemm(A, B, dtype))
    assert err <= 1e-5, err


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_gemm_bench_batch_full_size_wide(dtype):
    """The benchmark's batch in a system that asks for 128 x 256 tiles from
    n = 256 on (the wide variant: every bf16 product gets them, fp32
    products run the square tiles as calls), checked as above."""
    test_gemm_bench_batch_full_size(dtype, tile_class=(128, 128, 256, 256))


@pytest.mark.parametrize("mode", ["batched", "persistent"])
def test_gemm_bf16_wide_tiles(mode):
    """128 x 256 bf16 tiles (direct-to-LDS ring, transposing B reads) for
    every n % 32 == 0 from 32 to 544, ragged against both tile dimensions;
    n % 32 != 0 and an input 8 bytes off 16-byte alignment fall back to
    128 x 128 tiles.  Every product compared in full with the FP64 oracle."""
    import torch
    from paper_1505_07368_amd import binding as cg
    sizes = [32, 64, 96, 128, 160, 224, 256, 288, 384, 512, 544, 100, 200, 520]
    with cg.System(mode=mode, arena_bytes=1 << 30, ring_slots=64, gemm_tile=256) as s:
        a = s.spawn(cg.BHV_GEMM)
        cases = []
        for i, n in enumerate(sizes):
            A, B = gen.gemm_pair(1500 + i, n, "bf16")
            tA = torch.from_numpy(A.view(np.int16)).cuda().view(torch.bfloat16)
            tB = torch.from_numpy(B.view(np.int16)).cuda().view(torch.bfloat16)
            cases.append((n, A, B, tA, tB))
        # an operand 8 bytes past a 16-byte boundary
        n = 256
        A, B = gen.gemm_pair(1600, n, "bf16")
        pad = torch.zeros(n * n + 4, dtype=torch.int16, device="cuda")
        pad[4:] = torch.from_numpy(A.view(np.int16).ravel()).cuda()
        tA = pad[4:].view(torch.bfloat16)
        assert tA.data_ptr() % 16 == 8
        tB = torch.from_numpy(B.view(np.int16)).cuda().view(torch.bfloat16)
        cases.append((n, A, B, tA, tB))
        torch.cuda.synchronize()
        futs = [s.request(a, cg.caf_gemm_args(n, cg.BF16), inputs=[tA, tB])
                for n, _, _, tA, tB in cases]
        for (n, A, B, _, _), f in zip(cases, futs):
            st, C = f.result()
            assert st == cg.OK, (n, st)
            err = rel_fro(C.cpu().numpy().reshape(n, n), oracle.gemm(A, B, "bf16"))
            assert err <= 1e-5, (n, err)


@pytest.mark.parametrize("wgs", [2, 3])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_gemm_sizes_each_full_variant(dtype, wgs):
    """Single products of n = 1 .. 512, across slice and tile boundaries of
    both full drain variants (64- and 32-deep bf16 slices, 64- and 128-wide
    tiles), each compared in full with the FP64 oracle."""
    import torch
    from paper_1505_07368_amd import binding as cg
    sizes = [1, 7, 8, 16, 24, 31, 32, 33, 40, 64, 65, 100, 128, 129, 200, 256, 264, 512]
    with cg.System(mode="batched", arena_bytes=1 << 30, ring_slots=64,
                   full_wgs_per_cu=wgs) as s:
        a = s.spawn(cg.BHV_GEMM)
        cases = []
        for i, n in enumerate(sizes):
            A, B = gen.gemm_pair(900 + i, n, dtype)
            if dtype == "bf16":
                tA = torch.from_numpy(A.view(np.int16)).cuda().view(torch.bfloat16)
                tB = torch.from_numpy(B.view(np.int16)).cuda().view(torch.bfloat16)
            else:
                tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
            cases.append((n, A, B, tA, tB))
        torch.cuda.synchronize()
        code = cg.BF16 if dtype == "bf16" else cg.F32
        futs = [s.request(a, cg.caf_gemm_args(n, code), inputs=[tA, tB])
                for n, _, _, tA, tB in cases]
        for (n, A, B, _, _), f in zip(cases, futs):
            st, C = f.result()
            assert st == cg.OK, (n, st)
            err = rel_fro(C.cpu().numpy().reshape(n, n), oracle.gemm(A, B, dtype))
            assert err <= 1e-5, (n, err)
