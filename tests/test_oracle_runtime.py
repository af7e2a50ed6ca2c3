"""Pins of the oracle's actor runtime against the paper's semantics.

Sec. 2 / 4.3: a mailbox is a FIFO read only by its owner.  Sec. 5: a
synchronous request carries a unique id and receives exactly one response,
an error if the receiver is gone, or a timeout.  Sec. 4.4: call-by-value
messages.  Sec. 4.6: a compute actor replies with its kernel's output and
its input counts are fixed at spawn.
"""
import itertools

import numpy as np
import pytest

import oracle as o
from paper_1505_07368_amd import gen


def u64(x):
    return np.uint64(x).tobytes()


def test_fifo_per_sender_and_fold_order():
    s = o.System()
    a = s.spawn(o.BHV_HASHCHAIN)
    sent = []
    g = gen.rng(0)
    seqs = {0: 0, 1: 0, 2: 0}
    reqs = []
    for i in range(60):
        sender = int(g.integers(0, 3))
        x = int(g.integers(0, 2 ** 62))
        st, r = s.request(a, sender, args=u64(x))
        assert st == o.OK
        sent.append((sender, seqs[sender], x))
        seqs[sender] += 1
        reqs.append(r)
    assert len(set(reqs)) == len(reqs)  # unique request ids
    s.run()
    log = s.dequeue_log(a)
    # single reader, FIFO: dequeue order is the enqueue order
    assert log == [(snd, q) for snd, q, _ in sent]
    state = 0
    for (snd, q, x), r in zip(sent, reqs):
        state = o.hash_step(state, x)
        ok, st, data, res = s.reply(r)
        assert ok and st == o.OK and res == 1
        assert int(data[0]) == state  # each reply is the state after its own message
    assert s.state(a) == state


def test_exactly_one_reply_and_reply_is_output():
    s = o.System()
    echo = s.spawn(o.BHV_NOOP)
    mand = s.spawn(o.BHV_MANDELBROT)
    reqs = []
    for i in range(20):
        x = np.array([i, -i, 7], np.int32)
        st, r = s.request(echo, 0, inputs=[(x, o.I32)])
        reqs.append((r, x.copy()))
    vp = gen.tiny_viewport()
    args = o.mandel_args(vp.re_min, vp.im_min, vp.step_re, vp.step_im, 512, 512, 64, 32, 100)
    st, rm = s.request(mand, 1, args=args)
    assert st == o.OK
    assert s.run() == 21
    for r, x in reqs:
        ok, st, data, res = s.reply(r)
        assert ok and st == o.OK and res == 1 and (data == x).all()
    ok, st, data, res = s.reply(rm)
    direct = o.mandelbrot(vp.re_min, vp.im_min, vp.step_re, vp.step_im, 512, 64, 32, 100)
    assert ok and res == 1 and (data.reshape(32, 512) == direct).all()


def test_quit_answers_pending_and_refuses_later():
    s = o.System()
    a = s.spawn(o.BHV_NOOP)
    x = np.array([1], np.int32)
    rs = [s.request(a, 0, inputs=[(x, o.I32)])[1] for _ in range(5)]
    assert s.send(a, 0, inputs=[(x, o.I32)]) == o.OK
    assert s.quit(a) == o.OK
    for r in rs:
        ok, st, _, res = s.reply(r)
        assert ok and st == o.E_QUIT and res == 1
    st, _ = s.request(a, 0, inputs=[(x, o.I32)])
    assert st == o.E_NO_ACTOR
    assert s.quit(a) == o.E_NO_ACTOR
    assert s.run() == 0


def test_timeout_then_late_reply_swallowed():
    s = o.System()
    a = s.spawn(o.BHV_NOOP)
    x = np.array([3], np.int32)
    _, r = s.request(a, 0, inputs=[(x, o.I32)])
    assert s.timeout(r) == o.OK
    s.run()
    ok, st, _, res = s.reply(r)
    assert ok and st == o.E_TIMEOUT and res == 1


def test_signature_mismatch():
    s = o.System()
    g = s.spawn(o.BHV_GEMM, n=4)
    A = np.zeros((4, 4), np.float32)
    good = o.GemmArgs(4, o.F32)
    assert s.request(g, 0, args=good, inputs=[(A, o.F32), (A, o.F32)])[0] == o.OK
    # wrong dtype, wrong element count, wrong arity, wrong n vs spawn
    assert s.request(g, 0, args=good, inputs=[(A, o.F64), (A, o.F32)])[0] == o.E_INVALID
    assert s.request(g, 0, args=good, inputs=[(A[:3], o.F32), (A, o.F32)])[0] == o.E_INVALID
    assert s.request(g, 0, args=good, inputs=[(A, o.F32)])[0] == o.E_INVALID
    assert s.request(g, 0, args=o.GemmArgs(5, o.F32),
                     inputs=[(A, o.F32), (A, o.F32)])[0] == o.E_INVALID
    m = s.spawn(o.BHV_MANDELBROT)
    bad = o.mandel_args(-2, -1, 0.1, 0.1, 8, 8, 0, 8, 0)
    assert s.request(m, 0, args=bad)[0] == o.E_INVALID
    bad = o.mandel_args(-2, -1, 0.1, 0.1, 8, 8, 4, 8, 10)  # rows beyond height
    assert s.request(m, 0, args=bad)[0] == o.E_INVALID
    assert s.request(99, 0)[0] == o.E_NO_ACTOR


def test_inputs_unchanged_call_by_value():
    s = o.System()
    g = s.spawn(o.BHV_GEMM)
    A, B = gen.gemm_pair(3, 16)
    A0, B0 = A.copy(), B.copy()
    _, r = s.request(g, 0, args=o.GemmArgs(16, o.F32), inputs=[(A, o.F32), (B, o.F32)])
    A[:] = 0  # the message holds its own copy
    s.run()
    ok, st, C, _ = s.reply(r)
    assert (C.reshape(16, 16) == o.gemm(A0, B0)).all()
    assert (B == B0).all()


def test_forward_chain_gemm_tanh_rowsum():
    s = o.System()
    rsum = s.spawn(o.BHV_ROWSUM, n=8)
    th = s.spawn(o.BHV_TANH, n=8, forward_to=rsum)
    gm = s.spawn(o.BHV_GEMM, n=8)
    A, B = gen.gemm_pair(4, 8)
    _, r = s.request(gm, 0, args=o.GemmArgs(8, o.F32), inputs=[(A, o.F32), (B, o.F32)],
                     forward_to=th)
    s.run()
    ok, st, y, res = s.reply(r)
    assert ok and st == o.OK and res == 1
    assert (y == o.chain(A, B)).all()


def test_fault_behaviour_replies_error_and_stays_alive():
    s = o.System()
    f = s.spawn(o.BHV_FAULT)
    _, r1 = s.request(f, 0)
    _, r2 = s.request(f, 0)
    s.run()
    for r in (r1, r2):
        ok, st, _, res = s.reply(r)
        assert ok and st == o.E_FAULT and res == 1


def test_interleaving_is_valid_merge():
    """Two actors each keep FIFO order per sender whatever run() interleaves."""
    s = o.System()
    a, b = s.spawn(o.BHV_HASHCHAIN), s.spawn(o.BHV_HASHCHAIN)
    order = {a: [], b: []}
    for i, (dst, snd) in enumerate(itertools.product([a, b, a], [0, 1])):
        s.send(dst, snd, args=u64(i))
        order[dst].append(snd)
    s.run()
    for act in (a, b):
        log = s.dequeue_log(act)
        assert [snd for snd, _ in log] == order[act]
        for snd in (0, 1):
            qs = [q for sd, q in log if sd == snd]
            assert qs == sorted(qs) == list(range(len(qs)))


def test_become_swaps_behaviour_in_mailbox_order_and_keeps_state():
    """become (Sec. 6): messages enqueued before a swap meet the old
    behaviour and later ones the new; the actor's state survives a swap away
    and back; the enqueue-time signature check follows the latest swap."""
    s = o.System()
    a = s.spawn(o.BHV_HASHCHAIN)
    _, r1 = s.request(a, 0, args=u64(11))
    _, r2 = s.request(a, 0, args=u64(22))
    assert s.become(a, o.BHV_NOOP) == o.OK
    assert s.request(a, 0, args=u64(5))[0] == o.E_INVALID  # before anything ran
    x = np.array([7, 8], np.int32)
    st, r3 = s.request(a, 0, inputs=[(x, o.I32)])
    assert st == o.OK
    assert s.become(a, o.BHV_HASHCHAIN) == o.OK
    _, r4 = s.request(a, 0, args=u64(33))
    assert s.run() == 6  # four messages and two swaps
    h1 = o.hash_step(0, 11)
    h2 = o.hash_step(h1, 22)
    h3 = o.hash_step(h2, 33)
    assert int(s.reply(r1)[2][0]) == h1 and int(s.reply(r2)[2][0]) == h2
    ok, st, data, _ = s.reply(r3)
    assert ok and st == o.OK and (data == x).all()
    assert int(s.reply(r4)[2][0]) == h3 and s.state(a) == h3
    assert s.dequeue_log(a) == [(0, 0), (0, 1), (0, 2), (0, 3)]  # messages, not swaps
    assert s.become(a, 99) == o.E_INVALID
    assert s.quit(a) == o.OK
    assert s.become(a, o.BHV_NOOP) == o.E_NO_ACTOR
