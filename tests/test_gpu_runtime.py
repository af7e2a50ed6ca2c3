"""Actor semantics of the GPU runtime, checked against the CPU oracle and the
paper's rules (GPU).

Sec. 2 / 4.3: a mailbox is FIFO with a single reader.  Sec. 5: a request has
a unique id and exactly one reply, an error if the receiver is gone, and the
waiter may give up after a timeout.  Sec. 4.4: inputs are passed by value.
Sec. 4.6: the reply is the kernel's output; signatures are checked.
"""
import numpy as np
import pytest

import oracle
from paper_1505_07368_amd import gen
from tests.gpu_util import rel_fro

pytestmark = pytest.mark.gpu

MODES = ["plain", "plain_graph", "batched", "persistent"]


@pytest.fixture(scope="module", params=MODES)
def sysm(request):
    import torch
    from paper_1505_07368_amd import binding as cg
    assert torch.cuda.is_available()
    s = cg.System(mode=request.param, arena_bytes=256 << 20, idle_exit_us=0)
    yield s
    s.shutdown()


def slow_mandel_args(cg, rows=64):
    """A tile entirely inside the main cardioid at max_iter 65535: every
    pixel runs the full count (slow on purpose, ~1 ms)."""
    return cg.caf_mandel_args(-0.4, -0.2, 0.4 / 512, 0.4 / 512, 512, 512, 0, rows, 65535, cg.F32)


def test_fifo_hash_chain_three_senders(sysm):
    from paper_1505_07368_amd import binding as cg
    a = sysm.spawn(cg.BHV_HASHCHAIN)
    g = gen.rng(5)
    futs, xs = [], []
    for i in range(240):
        x = int(g.integers(0, 2 ** 62))
        xs.append(x)
        futs.append(sysm.request(a, cg.caf_hash_args(x), sender=int(g.integers(0, 3))))
    state = 0
    for x, f in zip(xs, futs):
        state = oracle.hash_step(state, x)
        st, v = f.result()
        assert st == cg.OK and int(v[0]) == state


def test_hash_chains_interleaved_with_sends_and_echo(sysm):
    """Five stateful actors whose messages are interleaved in the mailbox
    with sends (no reply) and echo requests: each actor's state follows its
    own messages in mailbox order (Sec. 2: one mailbox per actor, FIFO), so
    a drain pass holding entries of several applies each chain in order."""
    from paper_1505_07368_amd import binding as cg
    nact = 5
    acts = [sysm.spawn(cg.BHV_HASHCHAIN) for _ in range(nact)]
    e = sysm.spawn(cg.BHV_NOOP)
    g = gen.rng(9)
    state = [0] * nact
    checks, echoes = [], []
    for i in range(900):
        k = int(g.integers(0, nact + 1))
        if k == nact:
            x = np.array([i], np.int32)
            echoes.append((i, sysm.request(e, inputs=[x])))
            continue
        x = int(g.integers(0, 2 ** 62))
        state[k] = oracle.hash_step(state[k], x)
        if g.integers(0, 4) == 0:
            assert sysm.send(acts[k], cg.caf_hash_args(x)) == cg.OK
        else:
            checks.append((state[k], sysm.request(acts[k], cg.caf_hash_args(x))))
    for want, f in checks:
        st, v = f.result()
        assert st == cg.OK and int(v[0]) == want
    for i, f in echoes:
        st, v = f.result()
        assert st == cg.OK and int(v[0]) == i
    # the chains continue from the state the sends advanced
    for k in range(nact):
        st, v = sysm.request(acts[k], cg.caf_hash_args(7)).result()
        assert st == cg.OK and int(v[0]) == oracle.hash_step(state[k], 7)


def test_exactly_once_and_sends(sysm):
    from paper_1505_07368_amd import binding as cg
    before = sysm.stats()
    e = sysm.spawn(cg.BHV_NOOP)
    futs = []
    for i in range(300):
        x = np.array([i], np.int32)
        if i % 3 == 0:
            assert sysm.send(e, inputs=[x]) == cg.OK
        else:
            futs.append((i, sysm.request(e, inputs=[x])))
    for i, f in futs:
        st, v = f.result()
        assert st == cg.OK and int(v[0]) == i
    assert sysm.drain(30) == cg.OK
    after = sysm.stats()
    assert after["duplicate_completions"] == before["duplicate_completions"] == 0
    assert after["sends"] - before["sends"] == 100
    assert after["requests"] - before["requests"] == 200
    assert after["completions"] - before["completions"] == 300
    assert after["outstanding"] == 0


def test_pingpong_echo_lengths_and_sends(sysm):
    """Window-1 echoes of 1..4 int32 (input and reply inline: in the ring
    forms the drain answers them itself) and of 5 and 64 int32 (tile path),
    with sends between them: every reply exact, one completion each."""
    from paper_1505_07368_amd import binding as cg
    before = sysm.stats()
    e = sysm.spawn(cg.BHV_NOOP)
    g = gen.rng(23)
    nreq = nsend = 0
    for i in range(240):
        n = (1, 2, 3, 4, 5, 64)[i % 6]
        x = g.integers(-2 ** 31, 2 ** 31 - 1, size=n).astype(np.int32)
        if i % 5 == 4:
            assert sysm.send(e, inputs=[x]) == cg.OK
            nsend += 1
            continue
        st, v = sysm.request(e, inputs=[x]).result()
        nreq += 1
        got = v if isinstance(v, np.ndarray) else v.cpu().numpy()
        assert st == cg.OK and np.array_equal(np.asarray(got).reshape(-1)[:n], x), (i, n)
    assert sysm.drain(30) == cg.OK
    after = sysm.stats()
    assert after["duplicate_completions"] == 0
    assert after["completions"] - before["completions"] == nreq + nsend
    assert after["outstanding"] == 0


def test_quit_answers_unstarted_requests(sysm):
    from paper_1505_07368_amd import binding as cg
    m = sysm.spawn(cg.BHV_MANDELBROT)
    futs = [sysm.request(m, slow_mandel_args(cg)) for _ in range(12)]
    assert sysm.quit(m) == cg.OK
    statuses = [f.wait(60)[0] for f in futs]
    assert set(statuses) <= {cg.OK, cg.E_QUIT}
    # dequeue order is FIFO: the handled ones are a prefix
    k = statuses.count(cg.OK)
    assert statuses == [cg.OK] * k + [cg.E_QUIT] * (len(statuses) - k)
    rc, f = sysm.request_raw(m, slow_mandel_args(cg))
    assert rc == cg.E_NO_ACTOR and f is None
    assert sysm.quit(m) == cg.E_NO_ACTOR
    assert sysm.drain(30) == cg.OK
    assert sysm.stats()["duplicate_completions"] == 0


def test_timeout_then_late_reply_swallowed(sysm):
    from paper_1505_07368_amd import binding as cg
    m = sysm.spawn(cg.BHV_MANDELBROT)
    before = sysm.stats()["swallowed"]
    f = sysm.request(m, slow_mandel_args(cg, rows=256))
    with pytest.raises(cg.CafError) as ei:
        f.wait(1e-5)
    assert ei.value.status == cg.E_TIMEOUT
    assert f.poll()[1] == cg.E_TIMEOUT  # resolved once, as a timeout
    assert sysm.drain(60) == cg.OK
    assert f.poll()[1] == cg.E_TIMEOUT
    assert sysm.stats()["swallowed"] == before + 1
    f.release()


def test_signature_mismatch_and_unknown_actor(sysm):
    import torch
    from paper_1505_07368_amd import binding as cg
    g = sysm.spawn(cg.BHV_GEMM, n=16)
    A = torch.zeros(16 * 16, dtype=torch.float32, device="cuda")
    ok = cg.caf_gemm_args(16, cg.F32)
    assert sysm.request_raw(g, ok, [A, A])[0] == cg.OK
    assert sysm.request_raw(g, ok, [A.double(), A])[0] == cg.E_INVALID   # dtype
    assert sysm.request_raw(g, ok, [A[:100], A])[0] == cg.E_INVALID      # element count
    assert sysm.request_raw(g, ok, [A])[0] == cg.E_INVALID               # arity
    assert sysm.request_raw(g, cg.caf_gemm_args(8, cg.F32),
                            [A[:64], A[:64]])[0] == cg.E_INVALID         # n fixed at spawn
    m = sysm.spawn(cg.BHV_MANDELBROT)
    vp = gen.tiny_viewport()
    assert sysm.request_raw(m, cg.mandel_args(vp, max_iter=0))[0] == cg.E_INVALID
    assert sysm.request_raw(m, cg.mandel_args(vp, row0=500, rows=64))[0] == cg.E_INVALID
    assert sysm.request_raw(999, ok, [A, A])[0] == cg.E_NO_ACTOR
    assert sysm.drain(30) == cg.OK


def test_inputs_unchanged_and_fault(sysm):
    import torch
    from paper_1505_07368_amd import binding as cg
    n = 64
    g = sysm.spawn(cg.BHV_GEMM)
    A, B = gen.gemm_pair(8, n)
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    torch.cuda.synchronize()
    st, C = sysm.request(g, cg.caf_gemm_args(n, cg.F32), inputs=[At, Bt]).result()
    assert st == cg.OK
    assert (At.cpu().numpy() == A).all() and (Bt.cpu().numpy() == B).all()
    f = sysm.spawn(cg.BHV_FAULT)
    for _ in range(2):  # the actor stays alive after a fault reply
        st, v = sysm.request(f).result()
        assert st == cg.E_FAULT and v is None


def test_host_inputs_and_caller_output(sysm):
    import torch
    from paper_1505_07368_amd import binding as cg
    n = 48
    g = sysm.spawn(cg.BHV_GEMM)
    A, B = gen.gemm_pair(9, n)
    out = torch.full((n * n,), -1.0, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    f = sysm.request(g, cg.caf_gemm_args(n, cg.F32), inputs=[A, B], out=out)  # host inputs
    st, v = f.result()
    assert st == cg.OK and v is None  # written into the caller's tensor
    err = rel_fro(out.cpu().numpy().reshape(n, n), oracle.gemm(A, B))
    assert err <= 1e-5, err


def test_nonblocking_admission_overload():
    import torch
    from paper_1505_07368_amd import binding as cg
    with cg.System(mode="persistent", arena_bytes=64 << 20, ring_slots=2, blocking=False,
                   idle_exit_us=20000) as s:
        m = s.spawn(cg.BHV_MANDELBROT)
        a = slow_mandel_args(cg, rows=512)
        f1 = s.request(m, a)
        f2 = s.request(m, a)
        rc, f3 = s.request_raw(m, a)
        assert rc == cg.E_OVERLOAD and f3 is None
        assert f1.wait(60)[0] == cg.OK and f2.wait(60)[0] == cg.OK
        f1.release()
        f2.release()
        assert s.drain(30) == cg.OK
        assert s.stats()["rejected"] >= 1
        f4 = s.request(m, cg.caf_mandel_args(-2, -1, 0.1, 0.1, 8, 8, 0, 8, 10, cg.F32))
        assert f4.wait(30)[0] == cg.OK


def test_become_matches_oracle_sequence(sysm):
    """become (Sec. 6) through the mailbox: hash-chain, echo and Mandelbrot
    messages with swaps in between, all submitted before any reply is read;
    every reply and the final state equal the oracle's run of the same
    sequence, and the state survives swaps away and back."""
    from paper_1505_07368_amd import binding as cg
    vp = gen.tiny_viewport()
    margs = cg.caf_mandel_args(vp.re_min, vp.im_min, vp.step_re, vp.step_im, vp.width,
                               vp.height, 40, 9, vp.max_iter, cg.F32)
    x = np.array([7, -8, 9], np.int32)
    a = sysm.spawn(cg.BHV_HASHCHAIN)
    ref = oracle.System()
    ra = ref.spawn(oracle.BHV_HASHCHAIN)
    futs, rreqs = [], []

    def hash_(v):
        futs.append(sysm.request(a, cg.caf_hash_args(v)))
        rreqs.append(ref.request(ra, 0, args=np.uint64(v).tobytes())[1])

    def swap(beh, rbeh):
        assert sysm.become(a, beh) == cg.OK
        assert ref.become(ra, rbeh) == oracle.OK

    hash_(11)
    hash_(22)
    swap(cg.BHV_NOOP, oracle.BHV_NOOP)
    rc, f = sysm.request_raw(a, cg.caf_hash_args(5))  # checked against the new behaviour
    assert rc == cg.E_INVALID and f is None
    futs.append(sysm.request(a, inputs=[x]))
    rreqs.append(ref.request(ra, 0, inputs=[(x, oracle.I32)])[1])
    swap(cg.BHV_HASHCHAIN, oracle.BHV_HASHCHAIN)
    hash_(33)
    swap(cg.BHV_MANDELBROT, oracle.BHV_MANDELBROT)
    futs.append(sysm.request(a, margs))
    rreqs.append(ref.request(ra, 0, args=oracle.mandel_args(
        vp.re_min, vp.im_min, vp.step_re, vp.step_im, vp.width, vp.height, 40, 9,
        vp.max_iter))[1])
    swap(cg.BHV_HASHCHAIN, oracle.BHV_HASHCHAIN)
    hash_(44)
    ref.run()
    for f, r in zip(futs, rreqs):
        st, v = f.result()
        ok, rst, data, _ = ref.reply(r)
        assert ok and st == rst == cg.OK
        got = v.cpu().numpy() if hasattr(v, "cpu") else np.asarray(v)
        assert np.array_equal(got.ravel(), data.ravel())
    assert sysm.become(a, 99) == cg.E_INVALID
    assert sysm.quit(a) == cg.OK
    assert sysm.become(a, cg.BHV_NOOP) == cg.E_NO_ACTOR


def test_become_gemm_while_a_light_launch_runs():
    """An echo actor becomes a GEMM actor while the drain kernel without
    matrix tiles is running: the product is still computed."""
    import torch
    from paper_1505_07368_amd import binding as cg
    with cg.System(mode="batched", arena_bytes=64 << 20, ring_slots=64,
                   idle_exit_us=200000) as s:
        e = s.spawn(cg.BHV_NOOP)
        st, v = s.request(e, inputs=[np.array([3], np.int32)]).result()
        assert st == cg.OK and int(v[0]) == 3
        assert s.become(e, cg.BHV_GEMM) == cg.OK
        A, B = gen.gemm_pair(77, 64)
        At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        st, C = s.request(e, cg.caf_gemm_args(64, cg.F32), inputs=[At, Bt]).result()
        assert st == cg.OK
        assert rel_fro(C.cpu().numpy().reshape(64, 64), oracle.gemm(A, B)) <= 1e-5


def test_become_gemm_multi_tile_products_during_light_launch():
    """Multi-tile products (n = 256 at 64-wide tiles: 16 tiles each) sent
    while a light drain launch (no matrix tiles) is busy with Mandelbrot
    tiles: the first full launch starts only after every light workgroup has
    left, so no product tile is claimed by a light workgroup (which would
    fail it).  Every product and every Mandelbrot reply against the oracle."""
    import torch
    from paper_1505_07368_amd import binding as cg
    with cg.System(mode="batched", arena_bytes=256 << 20, ring_slots=256, gemm_tile=64,
                   idle_exit_us=200000) as s:
        e = s.spawn(cg.BHV_NOOP)
        m = s.spawn(cg.BHV_MANDELBROT)
        vp = gen.tiny_viewport()
        first = [s.request(m, cg.mandel_args(vp, row0=r0, rows=64)) for r0 in range(0, 512, 64)]
        first.append(s.request(m, slow_mandel_args(cg, rows=128)))
        assert s.become(e, cg.BHV_GEMM) == cg.OK
        n = 256
        pairs = [gen.gemm_pair(300 + k, n) for k in range(8)]
        dev = [(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()) for A, B in pairs]
        torch.cuda.synchronize()
        gf = [s.request(e, cg.caf_gemm_args(n, cg.F32), inputs=[At, Bt]) for At, Bt in dev]
        later = [s.request(m, cg.mandel_args(vp, row0=r0, rows=64)) for r0 in range(0, 512, 64)]
        for k, f in enumerate(gf):
            st, C = f.result()
            assert st == cg.OK, (k, st)
            A, B = pairs[k]
            assert rel_fro(C.cpu().numpy().reshape(n, n), oracle.gemm(A, B)) <= 1e-5, k
        ref = oracle.mandelbrot(vp.re_min, vp.im_min, vp.step_re, vp.step_im, 512, 0, 512, 100)
        for fs in (first[:8], later):
            for r0, f in zip(range(0, 512, 64), fs):
                st, img = f.result()
                assert st == cg.OK
                assert (img.cpu().numpy().reshape(64, 512) == ref[r0:r0 + 64]).all(), r0
        st, _ = first[8].result()
        assert st == cg.OK


def test_hash_reply_into_caller_buffer(sysm):
    """A hash-chain request with a caller-owned device output buffer: the
    new state is written there (the request goes the tile way, since its
    reply does not travel in the completion record), in every form."""
    import torch
    from paper_1505_07368_amd import binding as cg
    a = sysm.spawn(cg.BHV_HASHCHAIN)
    xs = [int(v) for v in gen.rng(17).integers(0, 2 ** 62, size=12)]
    outs = [torch.zeros(1, dtype=torch.uint64, device="cuda") for _ in xs]
    torch.cuda.synchronize()
    futs = [sysm.request(a, cg.caf_hash_args(x), out=o) for x, o in zip(xs, outs)]
    state = 0
    for x, f, o in zip(xs, futs, outs):
        state = oracle.hash_step(state, x)
        st, v = f.result()
        assert st == cg.OK and v is None
        got = int(o.view(torch.int64).cpu().item()) & (2 ** 64 - 1)
        assert got == state, (got, state)


def test_blocking_request_larger_than_arena_is_refused():
    """In blocking mode a request whose buffers can never fit the arena is
    refused at once (it would otherwise wait forever)."""
    import torch
    from paper_1505_07368_amd import binding as cg
    with cg.System(mode="batched", arena_bytes=1 << 20, blocking=True) as s:
        g = s.spawn(cg.BHV_GEMM)
        n = 1024  # a 4 MiB reply into a 1 MiB arena
        A = torch.zeros(n * n, device="cuda")
        rc, f = s.request_raw(g, cg.caf_gemm_args(n, cg.F32), inputs=[A, A])
        assert rc == cg.E_OVERLOAD and f is None
        m = s.spawn(cg.BHV_MANDELBROT)
        st, img = s.request(m, cg.caf_mandel_args(-2, -1, 0.1, 0.1, 8, 8, 0, 8, 10,
                                                  cg.F32)).result()
        assert st == cg.OK and img.numel() == 64


def test_batched_pingpong_keeps_its_launch():
    """Window-1 ping-pong in batched mode (default 50 us linger): the drain
    launch stays up between requests instead of retiring in every gap (a
    sentinel once judged idleness by its own last work alone, which
    relaunched the kernel for about 13% of the requests)."""
    from paper_1505_07368_amd import binding as cg
    with cg.System(mode="batched", arena_bytes=64 << 20, ring_slots=256) as s:
        a = s.spawn(cg.BHV_NOOP)
        x = np.array([7], np.int32)
        msgs = [{"actor": a, "inputs": [x]} for _ in range(1000)]
        s.drive(msgs[:50], window=1)
        before = s.stats()["drain_launches"]
        rc, _, st, _ = s.drive(msgs, window=1)
        assert rc == cg.OK and (st == cg.OK).all()
        assert s.stats()["drain_launches"] - before <= 50


def test_arena_reuse_then_coalesce():
    """Replies in the arena: freed blocks are reused by size, merged when a
    larger reply needs the space, and a reply larger than the arena is
    refused without blocking."""
    import torch
    from paper_1505_07368_amd import binding as cg
    with cg.System(mode="batched", arena_bytes=16 << 20, ring_slots=64, blocking=False) as s:
        g = s.spawn(cg.BHV_GEMM)
        A, B = gen.gemm_pair(21, 512)
        At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        A2, B2 = gen.gemm_pair(22, 1024)
        At2, Bt2 = torch.from_numpy(A2).cuda(), torch.from_numpy(B2).cuda()
        torch.cuda.synchronize()
        for _ in range(2):  # the second round reuses the freed 1 MB blocks
            futs = [s.request(g, cg.caf_gemm_args(512, cg.F32), inputs=[At, Bt])
                    for _ in range(12)]
            outs = [f.result() for f in futs]
            assert all(st == cg.OK for st, _ in outs)
            err = rel_fro(outs[-1][1].cpu().numpy().reshape(512, 512), oracle.gemm(A, B))
            assert err <= 1e-5, err
            for f in futs:
                f.release()
            assert s.drain(30) == cg.OK
            assert s.stats()["arena_in_use"] == 0
        # 2 x 4 MB replies only fit once the freed 1 MB blocks are merged
        futs = [s.request(g, cg.caf_gemm_args(1024, cg.F32), inputs=[At2, Bt2])
                for _ in range(2)]
        outs = [f.result() for f in futs]
        assert all(st == cg.OK for st, _ in outs)
        err = rel_fro(outs[0][1].cpu().numpy().reshape(1024, 1024), oracle.gemm(A2, B2))
        assert err <= 1e-5, err
        assert s.stats()["arena_in_use"] == 8 << 20
        for f in futs:
            f.release()
        assert s.drain(30) == cg.OK
        # a 17.6 MB reply (n = 2100) cannot fit a 16 MiB arena
        A3 = torch.zeros(2100 * 2100, device="cuda")
        rc, f3 = s.request_raw(g, cg.caf_gemm_args(2100, cg.F32), inputs=[A3, A3])
        assert rc == cg.E_OVERLOAD and f3 is None
        assert s.stats()["arena_in_use"] == 0


@pytest.mark.parametrize("n,chains", [(128, 24), (512, 3)])
def test_pipeline_device_vs_host_forwarding(sysm, n, chains):
    """n = 128: the tanh and row-sum stages are small enough to run in the
    workgroup that finished the previous stage; n = 512: they are published
    as work tiles for every workgroup."""
    import torch
    from paper_1505_07368_amd import binding as cg
    rs = sysm.spawn(cg.BHV_ROWSUM, n=n)
    th = sysm.spawn(cg.BHV_TANH, n=n)
    gm = sysm.spawn(cg.BHV_GEMM, n=n)
    inputs, outs_dev, outs_host = [], [], []
    for c in range(chains):
        A, B = gen.gemm_pair(100 + c, n)
        inputs.append((A, B, torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()))
        outs_dev.append(torch.zeros(n, dtype=torch.float32, device="cuda"))
        outs_host.append(torch.zeros(n, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    # device forwarding: gemm -> tanh (spawned without a target) -> rowsum
    th2 = sysm.spawn(cg.BHV_TANH, n=n, forward_to=rs)
    msgs = [{"actor": gm, "args": cg.caf_gemm_args(n, cg.F32), "inputs": [At, Bt], "out": o,
             "forward_to": th2} for (_, _, At, Bt), o in zip(inputs, outs_dev)]
    rc, lat, st, _ = sysm.drive(msgs, window=8)
    assert rc == cg.OK and (st == cg.OK).all(), st
    # host-mediated: the driver re-sends each reply to tanh, then rowsum
    msgs = [{"actor": gm, "args": cg.caf_gemm_args(n, cg.F32), "inputs": [At, Bt], "out": o}
            for (_, _, At, Bt), o in zip(inputs, outs_host)]
    rc, lat, st, _ = sysm.drive(msgs, window=8, chain_hops=2, hop_actors=(th, rs))
    assert rc == cg.OK and (st == cg.OK).all(), st
    torch.cuda.synchronize()
    for (A, B, _, _), od, oh in zip(inputs, outs_dev, outs_host):
        ref = oracle.chain(A, B)
        assert rel_fro(od.cpu().numpy(), ref) <= 1e-5
        assert rel_fro(oh.cpu().numpy(), ref) <= 1e-5


def test_batching_invariance(sysm):
    """A message gives the same reply alone and inside a mixed batch:
    bit-exact for Mandelbrot, identical for GEMM (same tile shape)."""
    import torch
    from paper_1505_07368_amd import binding as cg
    vp = gen.boundary_viewport(2, width=320, height=192, max_iter=700)
    m = sysm.spawn(cg.BHV_MANDELBROT)
    g = sysm.spawn(cg.BHV_GEMM)
    n = 96
    A, B = gen.gemm_pair(21, n)
    At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    torch.cuda.synchronize()
    st, alone_m = sysm.request(m, cg.mandel_args(vp, row0=64, rows=64)).result()
    alone_m = alone_m.cpu().numpy().copy()
    st, alone_g = sysm.request(g, cg.caf_gemm_args(n, cg.F32), inputs=[At, Bt]).result()
    alone_g = alone_g.cpu().numpy().copy()
    futs = []
    for i in range(40):
        if i % 2:
            futs.append(("g", sysm.request(g, cg.caf_gemm_args(n, cg.F32), inputs=[At, Bt])))
        else:
            futs.append(("m", sysm.request(m, cg.mandel_args(vp, row0=64, rows=64))))
        futs.append(("x", sysm.request(m, cg.mandel_args(vp, row0=(i * 7) % 128, rows=64,
                                                          fp=cg.F64))))
    for kind, f in futs:
        st, v = f.result()
        assert st == cg.OK
        if kind == "m":
            assert (v.cpu().numpy() == alone_m).all()
        elif kind == "g":
            assert (v.cpu().numpy() == alone_g).all()
    ref = oracle.mandelbrot(vp.re_min, vp.im_min, vp.step_re, vp.step_im, 320, 64, 64, 700)
    assert (alone_m.reshape(64, 320) == ref).all()


def test_plain_graph_replays_match_oracle():
    """CAF_MODE_PLAIN_GRAPH: one graph per stage shape, replayed with each
    message's arguments.  Every replay is checked against the oracle, with
    eager device work and host synchronisation between replays."""
    import torch
    from paper_1505_07368_amd import binding as cg
    s = cg.System(mode="plain_graph", arena_bytes=256 << 20)
    try:
        g = s.spawn(cg.BHV_GEMM)
        m = s.spawn(cg.BHV_MANDELBROT)
        vp = gen.boundary_viewport(4, width=256, height=64, max_iter=300)
        whole = oracle.mandelbrot(vp.re_min, vp.im_min, vp.step_re, vp.step_im, 256, 0, 64, 300)
        scratch = torch.ones(1 << 20, device="cuda")
        for i in range(12):
            A, B = gen.gemm_pair(300 + i, 64)
            At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
            torch.cuda.synchronize()
            st, C = s.request(g, cg.caf_gemm_args(64, cg.F32), inputs=[At, Bt]).result()
            assert st == cg.OK
            assert rel_fro(C.cpu().numpy().reshape(64, 64), oracle.gemm(A, B)) <= 1e-5, i
            r0 = (i * 16) % 48
            st, img = s.request(m, cg.mandel_args(vp, row0=r0, rows=16)).result()
            assert st == cg.OK
            assert (img.cpu().numpy().reshape(16, 256) == whole[r0:r0 + 16]).all(), i
            scratch.mul_(1.0001)  # eager work between replays
            if i % 3 == 0:
                torch.cuda.synchronize()
        stats = s.stats()
        assert stats["launches"] >= 24
    finally:
        s.shutdown()


def test_degenerate_and_maximum_arguments(sysm):
    """Boundaries of the signatures: empty or oversized requests are refused
    with CAF_E_INVALID before anything reaches the device; the largest
    max_iter and a 1-pixel / 1x1 request are served exactly."""
    import torch
    from paper_1505_07368_amd import binding as cg
    from paper_1505_07368_amd.gen import Viewport
    g = sysm.spawn(cg.BHV_GEMM)
    A = torch.zeros(4, dtype=torch.float32, device="cuda")
    assert sysm.request_raw(g, cg.caf_gemm_args(0, cg.F32), [A[:0], A[:0]])[0] == cg.E_INVALID
    assert sysm.request_raw(g, cg.caf_gemm_args(16385, cg.F32), [A, A])[0] == cg.E_INVALID
    assert sysm.request_raw(g, cg.caf_gemm_args(2, cg.F64), [A, A])[0] == cg.E_INVALID
    m = sysm.spawn(cg.BHV_MANDELBROT)
    vp = gen.tiny_viewport()
    assert sysm.request_raw(m, cg.mandel_args(vp, max_iter=65536))[0] == cg.E_INVALID
    assert sysm.request_raw(m, cg.mandel_args(Viewport(0, 0, 1, 1, 0, 1, 10)))[0] == cg.E_INVALID
    assert sysm.request_raw(m, cg.mandel_args(vp, fp=cg.I32))[0] == cg.E_INVALID
    # more than 2^32 pixels (each side within its own limit of 2^20)
    huge = Viewport(0, 0, 1e-6, 1e-6, 1 << 20, 1 << 13, 10)
    assert sysm.request_raw(m, cg.mandel_args(huge))[0] == cg.E_INVALID
    e = sysm.spawn(cg.BHV_NOOP)
    assert sysm.request_raw(e, None, [np.zeros(0, np.int32)])[0] == cg.E_INVALID
    # max_iter = 65535 at c = 0 (never escapes) and 1 at c = 3 (escapes at once)
    for c, mi, expect in [(0j, 65535, 65535), (3 + 0j, 1, 1), (3 + 0j, 65535, 1)]:
        st, img = sysm.request(m, cg.mandel_args(Viewport(c.real, c.imag, 0, 0, 1, 1, mi))).result()
        assert st == cg.OK and int(img.cpu()[0]) == expect, (c, mi)
    # 1x1 GEMM in both input types
    for code, dt in ((cg.F32, torch.float32), (cg.BF16, torch.bfloat16)):
        a1 = torch.full((1,), 3.0, dtype=dt, device="cuda")
        b1 = torch.full((1,), -2.0, dtype=dt, device="cuda")
        torch.cuda.synchronize()
        st, c1 = sysm.request(g, cg.caf_gemm_args(1, code), inputs=[a1, b1]).result()
        assert st == cg.OK and float(c1.cpu()[0]) == -6.0
    assert sysm.drain(30) == cg.OK


@pytest.mark.parametrize("mode", ["batched", "persistent"])
def test_hold_collects_one_batch(mode):
    """caf_gpu_hold: held messages wait in the mailbox (no reply, no new
    launch); letting go runs them in one drain launch, each reply equal to
    the oracle's."""
    import time
    import torch
    from paper_1505_07368_amd import binding as cg
    with cg.System(mode=mode, arena_bytes=64 << 20, ring_slots=256, idle_exit_us=50) as s:
        g = s.spawn(cg.BHV_GEMM)
        e = s.spawn(cg.BHV_NOOP)
        # a first message, so a launch has come and gone
        st, v = s.request(e, inputs=[np.array([1], np.int32)]).result()
        assert st == cg.OK
        assert s.drain() == cg.OK
        s.drain_kernel_ms()  # waits until that launch has exited
        before = s.stats()["drain_launches"]
        assert s.hold(True) == cg.OK
        pairs = [gen.gemm_pair(700 + i, 96) for i in range(24)]
        dev = [(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()) for A, B in pairs]
        torch.cuda.synchronize()
        futs = [s.request(g, cg.caf_gemm_args(96, cg.F32), inputs=list(ab)) for ab in dev]
        futs += [s.request(e, inputs=[np.array([i, -i], np.int32)]) for i in range(40)]
        time.sleep(0.05)
        assert not any(f.poll()[0] for f in futs)  # nothing ran while held
        assert s.drain(timeout_s=0.01) == cg.E_TIMEOUT
        assert s.stats()["drain_launches"] == before
        assert s.hold(False) == cg.OK
        for (A, B), f in zip(pairs, futs[:24]):
            st, C = f.result()
            assert st == cg.OK
            assert rel_fro(C.cpu().numpy().reshape(96, 96), oracle.gemm(A, B)) <= 1e-5
        for i, f in enumerate(futs[24:]):
            st, v = f.result()
            assert st == cg.OK and v.tolist() == [i, -i]
        assert s.drain() == cg.OK
        assert s.stats()["drain_launches"] == before + 1
    with cg.System(mode="plain", arena_bytes=16 << 20) as p:
        assert p.hold(True) == cg.E_INVALID


def test_shutdown_while_held_answers_quit():
    """Requests still held in the mailbox at shutdown never ran: each
    future resolves once, with CAF_E_QUIT.  Each round follows a busy
    persistent system, the condition under which a poller that had checked
    the hold just before it started once launched a drain for the held
    messages (the hold is now set and checked under the launch lock)."""
    import torch
    from paper_1505_07368_amd import binding as cg
    for rnd in range(6):
        with cg.System(mode="persistent", arena_bytes=64 << 20, ring_slots=256,
                       idle_exit_us=50) as s0:
            g = s0.spawn(cg.BHV_GEMM)
            A, B = gen.gemm_pair(710 + rnd, 96)
            dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
            torch.cuda.synchronize()
            for f in [s0.request(g, cg.caf_gemm_args(96, cg.F32), inputs=[dA, dB])
                      for _ in range(8)]:
                assert f.result()[0] == cg.OK
        s = cg.System(mode="batched", arena_bytes=16 << 20, ring_slots=64)
        e = s.spawn(cg.BHV_NOOP)
        st, v = s.request(e, inputs=[np.array([5], np.int32)]).result()
        assert st == cg.OK and v.tolist() == [5]
        assert s.drain() == cg.OK
        s.drain_kernel_ms()
        assert s.hold(True) == cg.OK
        futs = [s.request(e, inputs=[np.array([i], np.int32)]) for i in range(10)]
        s.shutdown()
        got = []
        for f in futs:
            st, _ = f.wait(5.0)
            got.append(st)
            f.release()
        assert got == [cg.E_QUIT] * 10, (rnd, got)
