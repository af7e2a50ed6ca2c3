"""Serving with admission that binds (GPU): requests arrive open loop while
others are on the device, are admitted as mailbox slots and arena memory
free up, and every result equals the oracle's (the result of the message
alone), whatever else shared the device with it.

  * a Python open loop against a non-blocking system with an 8 MiB arena
    and library-allocated replies: a refused request is retried after the
    oldest outstanding reply has been read and released, so admission binds
    on the budget; every reply is compared in full;
  * the native driver against a blocking system with a 4 MiB arena: the
    driver keeps requests that do not fit yet in arrival order and retries
    them as replies free room, so every request completes; its replies are
    written to caller buffers and compared in full as well, and the arena
    use stays within the budget.
"""
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_1505_07368_amd import gen
from tests import oracle_par
from tests.gpu_util import rel_fro

pytestmark = pytest.mark.gpu


def _mix(seed, rate, duration_s):
    d = gen.serving_mix_arrays(seed, rate, duration_s)
    cases = []
    for i in range(d["arrival_ns"].size):
        if d["is_mandel"][i]:
            side, mi = int(d["side"][i]), int(d["max_iter"][i])
            vp = gen.Viewport(float(d["re_min"][i]), float(d["im_min"][i]), float(d["step"][i]),
                              float(d["step"][i]), side, side, mi)
            cases.append(("mandel", int(d["arrival_ns"][i]), vp))
        else:
            n = int(d["gemm_n"][i])
            cases.append(("gemm", int(d["arrival_ns"][i]), gen.gemm_pair(5000 + i, n)))
    return cases


def _oracle(cases):
    oracle.lib()

    def ref_of(c):
        kind, _, x = c
        if kind == "mandel":
            return oracle.mandelbrot(x.re_min, x.im_min, x.step_re, x.step_im, x.width, 0,
                                     x.height, x.max_iter, "f32")
        return oracle.gemm(x[0], x[1])

    with ThreadPoolExecutor(oracle_par.threads()) as ex:
        return list(ex.map(ref_of, cases))


def _check(cases, refs, got):
    for (kind, _, x), ref, g in zip(cases, refs, got):
        if kind == "mandel":
            img = g.reshape(x.height, x.width)
            assert (img == ref).all(), (x, int((img != ref).sum()))
        else:
            n = x[0].shape[0]
            assert rel_fro(g.reshape(n, n), ref) <= 1e-5, n


def test_open_loop_small_budget_retries_and_matches_oracle():
    import torch
    from paper_1505_07368_amd import binding as cg
    cases = _mix(1, 1e4, 0.06)
    assert len(cases) >= 400
    dev = {}
    for i, (kind, _, x) in enumerate(cases):
        if kind == "gemm":
            dev[i] = (torch.from_numpy(x[0]).cuda(), torch.from_numpy(x[1]).cuda())
    torch.cuda.synchronize()
    got = [None] * len(cases)
    outstanding = []  # (index, future), oldest first
    max_inflight = retries = 0
    with cg.System(mode="persistent", arena_bytes=8 << 20, ring_slots=256,
                   blocking=False) as s:
        m = s.spawn(cg.BHV_MANDELBROT)
        gm = s.spawn(cg.BHV_GEMM)

        def harvest_oldest():
            i, f = outstanding.pop(0)
            st, v = f.result()
            assert st == cg.OK, (i, st)
            got[i] = v.cpu().numpy().copy()
            f.release()  # gives the reply's arena memory back

        t0 = time.perf_counter_ns()
        for i, (kind, t_arr, x) in enumerate(cases):
            while time.perf_counter_ns() - t0 < t_arr:
                pass
            while True:
                if kind == "mandel":
                    rc, f = s.request_raw(m, cg.mandel_args(x))
                else:
                    rc, f = s.request_raw(gm, cg.caf_gemm_args(x[0].shape[0], cg.F32),
                                          inputs=list(dev[i]))
                if rc == cg.OK:
                    break
                assert rc == cg.E_OVERLOAD, rc
                retries += 1
                assert outstanding, "refused with nothing outstanding"
                harvest_oldest()
            outstanding.append((i, f))
            max_inflight = max(max_inflight, len(outstanding))
        while outstanding:
            harvest_oldest()
        stats = s.stats()
    assert retries > 0 and stats["rejected"] == retries  # the budget bound
    assert max_inflight >= 2  # later requests were admitted while others ran
    assert stats["arena_peak"] <= 8 << 20
    _check(cases, _oracle(cases), got)


def test_driver_blocking_admission_small_budget():
    import torch
    from paper_1505_07368_amd import binding as cg
    cases = _mix(2, 2e4, 0.03)
    assert len(cases) >= 400
    msgs, outs = [], []
    with cg.System(mode="batched", arena_bytes=4 << 20, ring_slots=64, blocking=True) as s:
        m = s.spawn(cg.BHV_MANDELBROT)
        gm = s.spawn(cg.BHV_GEMM)
        for kind, _, x in cases:
            if kind == "mandel":
                out = torch.zeros(x.width * x.height, dtype=torch.uint16, device="cuda")
                msgs.append({"actor": m, "args": cg.mandel_args(x), "out": out})
            else:
                n = x[0].shape[0]
                # host inputs: staged into the arena, so GEMMs hold budget
                out = torch.full((n * n,), float("nan"), device="cuda")
                msgs.append({"actor": gm, "args": cg.caf_gemm_args(n, cg.F32),
                             "inputs": [x[0], x[1]], "out": out})
            outs.append(out)
        torch.cuda.synchronize()
        arrival = np.array([c[1] for c in cases], np.int64)
        rc, lat, st, el = s.drive(msgs, window=len(msgs), arrival_ns=arrival)
        assert rc == cg.OK and (st == cg.OK).all(), (rc, np.unique(st))
        stats = s.stats()
    assert stats["rejected"] == 0 and stats["completions"] >= len(cases)
    assert stats["arena_peak"] <= 4 << 20
    assert (lat > 0).all()
    torch.cuda.synchronize()
    _check(cases, _oracle(cases), [o.cpu().numpy() for o in outs])


@pytest.mark.parametrize("arena_kib", [3072, 512])
def test_driver_host_chains_under_blocking_budget(arena_kib):
    """Host-mediated chains GEMM (n = 128) -> tanh -> row sum through the
    native driver with a blocking system and 32 chains in flight.  With
    3 MiB the first stages' replies (2 MiB at most) leave room for the next
    stages, which wait in the driver, in order, until earlier replies are
    released: every chain completes.  With 512 KiB the first stages' replies
    fill the arena and no next stage could ever be admitted: the driver
    refuses the oldest waiting chain (CAF_E_OVERLOAD) and releases its reply
    rather than waiting forever.  Every completed chain equals the oracle's."""
    import torch
    from paper_1505_07368_amd import binding as cg
    n, chains = 128, 48
    inputs, outs = [], []
    for c in range(chains):
        A, B = gen.gemm_pair(3000 + c, n)
        inputs.append((A, B, torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()))
        outs.append(torch.zeros(n, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    with cg.System(mode="batched", arena_bytes=arena_kib << 10, ring_slots=64,
                   blocking=True) as s:
        rs = s.spawn(cg.BHV_ROWSUM, n=n)
        th = s.spawn(cg.BHV_TANH, n=n)
        gm = s.spawn(cg.BHV_GEMM, n=n)
        msgs = [{"actor": gm, "args": cg.caf_gemm_args(n, cg.F32), "inputs": [At, Bt], "out": o}
                for (_, _, At, Bt), o in zip(inputs, outs)]
        rc, lat, st, _ = s.drive(msgs, window=32, chain_hops=2, hop_actors=(th, rs))
        assert rc == cg.OK and ((st == cg.OK) | (st == cg.E_OVERLOAD)).all(), np.unique(st)
        stats = s.stats()
    assert stats["arena_peak"] <= arena_kib << 10
    if arena_kib == 3072:
        assert (st == cg.OK).all()
    assert (st == cg.OK).sum() > 0
    torch.cuda.synchronize()
    for (A, B, _, _), o, sti in zip(inputs, outs, st):
        if sti == cg.OK:
            assert rel_fro(o.cpu().numpy(), oracle.chain(A, B)) <= 1e-5
