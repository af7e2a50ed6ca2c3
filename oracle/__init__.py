"""CPU oracle for the compute-actor hot path (ctypes binding of libcafref).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The
product library (``paper_1505_07368_amd``) never imports it and shares no
code with it.

What it computes is documented in ``cafref.h``: an escape-time Mandelbrot in
float and double (the workloads of the paper's Sec. 7.4 and 7.5), the dense
product of flat n x n matrices in double (Sec. 4.6, the matrix_multiply
kernel), tanh, row sums, echo, a non-commutative hash chain, and a
single-threaded mailbox runtime with request ids, exactly-once replies and
quit (Sec. 2, 4.3, 5, 6).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcafref.so")
SOURCES = [os.path.join(HERE, "cafref.cpp")]

OK, E_INVALID, E_NO_ACTOR, E_OVERLOAD, E_TIMEOUT, E_DEVICE, E_QUIT, E_FAULT = (
    0, -1, -2, -3, -4, -5, -6, -7)
I32, U16, F32, F64, BF16, U64 = 0, 1, 2, 3, 4, 5
BHV_NOOP, BHV_MANDELBROT, BHV_GEMM, BHV_TANH, BHV_ROWSUM, BHV_HASHCHAIN, BHV_FAULT = range(7)

_NP = {I32: np.int32, U16: np.uint16, F32: np.float32, F64: np.float64, BF16: np.uint16,
       U64: np.uint64}


def build(verbose: bool = False) -> str:
    """Compiles libcafref.so with g++ (-O2, no FMA contraction, no fast-math)."""
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-Wall", "-o", LIB_PATH] + SOURCES
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return LIB_PATH


class RefBuf(C.Structure):
    _fields_ = [("data", C.c_void_p), ("numel", C.c_uint64), ("dtype", C.c_int32)]


class MandelArgs(C.Structure):
    _fields_ = [("re_min", C.c_double), ("im_min", C.c_double), ("step_re", C.c_double),
                ("step_im", C.c_double), ("width", C.c_uint32), ("height", C.c_uint32),
                ("row0", C.c_uint32), ("rows", C.c_uint32), ("max_iter", C.c_uint32),
                ("fp", C.c_int32)]


class GemmArgs(C.Structure):
    _fields_ = [("n", C.c_uint32), ("in_dtype", C.c_int32)]


class ShapeArgs(C.Structure):
    _fields_ = [("rows", C.c_uint32), ("cols", C.c_uint32)]


class SpawnArgs(C.Structure):
    _fields_ = [("n", C.c_uint32), ("forward_to", C.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or any(
                os.path.getmtime(s) > os.path.getmtime(LIB_PATH) for s in SOURCES):
            build()
        L = C.CDLL(LIB_PATH)
        vp, u32, u64, i32, dbl = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int32, C.c_double
        for name in ("caf_ref_mandelbrot_f32", "caf_ref_mandelbrot_f64"):
            f = getattr(L, name)
            f.argtypes = [dbl, dbl, dbl, dbl, u32, u32, u32, u32, vp]
            f.restype = None
        for name in ("caf_ref_gemm_f32", "caf_ref_gemm_bf16"):
            f = getattr(L, name)
            f.argtypes = [u32, vp, vp, vp]
            f.restype = None
        L.caf_ref_tanh_f64.argtypes = [u64, vp, vp]
        L.caf_ref_rowsum_f64.argtypes = [u32, u32, vp, vp]
        L.caf_ref_hash_step.argtypes = [u64, u64]
        L.caf_ref_hash_step.restype = u64
        L.caf_ref_new.restype = vp
        L.caf_ref_free.argtypes = [vp]
        L.caf_ref_spawn.argtypes = [vp, i32, C.POINTER(SpawnArgs), C.POINTER(u64)]
        L.caf_ref_send.argtypes = [vp, u64, u32, vp, u64, C.POINTER(RefBuf), u32]
        L.caf_ref_request.argtypes = [vp, u64, u32, vp, u64, C.POINTER(RefBuf), u32, u64,
                                      C.POINTER(u64)]
        L.caf_ref_run.argtypes = [vp]
        L.caf_ref_run.restype = u64
        L.caf_ref_quit.argtypes = [vp, u64, u32]
        L.caf_ref_reply.argtypes = [vp, u64, C.POINTER(i32), vp, u64, C.POINTER(u64),
                                    C.POINTER(i32), C.POINTER(u32)]
        L.caf_ref_timeout.argtypes = [vp, u64]
        L.caf_ref_dequeue_log.argtypes = [vp, u64, vp, vp, u64]
        L.caf_ref_dequeue_log.restype = u64
        L.caf_ref_actor_state.argtypes = [vp, u64]
        L.caf_ref_actor_state.restype = u64
        L.caf_ref_become.argtypes = [vp, u64, i32, C.POINTER(SpawnArgs)]
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags.c_contiguous
    return a.ctypes.data


# ---- scalar kernels ------------------------------------------------------

def mandelbrot(re_min, im_min, step_re, step_im, width, row0, rows, max_iter, fp="f32"):
    """Escape-time counts, uint16 [rows][width] (see cafref.h)."""
    out = np.zeros((rows, width), dtype=np.uint16)
    f = lib().caf_ref_mandelbrot_f32 if fp in ("f32", F32) else lib().caf_ref_mandelbrot_f64
    if rows and width:
        f(re_min, im_min, step_re, step_im, width, row0, rows, max_iter, _ptr(out))
    return out


def colour_map(counts: np.ndarray, palette: np.ndarray) -> np.ndarray:
    """A Mandelbrot reply after the spawn-time post-processing step (the
    transformation spawn_cl accepts beside the kernel, Sec. 4.6): each count
    n becomes palette[min(n, len(palette) - 1)], uint32."""
    palette = np.asarray(palette, dtype=np.uint32)
    idx = np.minimum(np.asarray(counts, dtype=np.int64), len(palette) - 1)
    return palette[idx]


def escape(c: complex, max_iter: int, fp="f32") -> int:
    """Count of a single point c (a 1x1 request whose corner is c)."""
    return int(mandelbrot(c.real, c.imag, 0.0, 0.0, 1, 0, 1, max_iter, fp)[0, 0])


def gemm(A: np.ndarray, B: np.ndarray, dtype="f32") -> np.ndarray:
    """C = A @ B in float64; A, B float32, or uint16 bfloat16 bit patterns."""
    n = A.shape[0]
    assert A.shape == (n, n) and B.shape == (n, n)
    C_ = np.zeros((n, n), dtype=np.float64)
    if dtype in ("f32", F32):
        A = np.ascontiguousarray(A, np.float32)
        B = np.ascontiguousarray(B, np.float32)
        lib().caf_ref_gemm_f32(n, _ptr(A), _ptr(B), _ptr(C_))
    else:
        A = np.ascontiguousarray(A, np.uint16)
        B = np.ascontiguousarray(B, np.uint16)
        lib().caf_ref_gemm_bf16(n, _ptr(A), _ptr(B), _ptr(C_))
    return C_


def tanh(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float64)
    y = np.empty_like(x)
    lib().caf_ref_tanh_f64(x.size, _ptr(x), _ptr(y))
    return y


def rowsum(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float64)
    y = np.empty(x.shape[0], np.float64)
    lib().caf_ref_rowsum_f64(x.shape[0], x.shape[1], _ptr(x), _ptr(y))
    return y


def hash_step(s: int, x: int) -> int:
    return int(lib().caf_ref_hash_step(s, x))


def chain(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """The pipeline GEMM -> tanh -> row-sum, in float64 throughout."""
    return rowsum(tanh(gemm(A, B, "f32")))


# ---- runtime ---------------------------------------------------------------

class System:
    """A single-threaded oracle actor system."""

    def __init__(self):
        self.L = lib()
        self.h = self.L.caf_ref_new()
        self._keep = []

    def close(self):
        if self.h:
            self.L.caf_ref_free(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def spawn(self, behavior: int, n: int = 0, forward_to: int = 0) -> int:
        out = C.c_uint64()
        sa = SpawnArgs(n, forward_to)
        st = self.L.caf_ref_spawn(self.h, behavior, C.byref(sa), C.byref(out))
        if st != OK:
            raise ValueError(f"spawn failed: {st}")
        return out.value

    def _bufs(self, inputs):
        arr = (RefBuf * max(1, len(inputs)))()
        for i, (a, dt) in enumerate(inputs):
            a = np.ascontiguousarray(a)
            self._keep.append(a)
            arr[i] = RefBuf(a.ctypes.data, a.size, dt)
        return arr

    def send(self, actor, sender, args=None, inputs=()):
        ab = bytes(args) if args is not None else b""
        bufs = self._bufs(inputs)
        return self.L.caf_ref_send(self.h, actor, sender, ab, len(ab), bufs, len(inputs))

    def request(self, actor, sender, args=None, inputs=(), forward_to=0):
        """Returns (status, request id)."""
        ab = bytes(args) if args is not None else b""
        bufs = self._bufs(inputs)
        rid = C.c_uint64(0)
        st = self.L.caf_ref_request(self.h, actor, sender, ab, len(ab), bufs, len(inputs),
                                    forward_to, C.byref(rid))
        return st, rid.value

    def run(self) -> int:
        n = self.L.caf_ref_run(self.h)
        self._keep.clear()
        return n

    def quit(self, actor, reason=0) -> int:
        return self.L.caf_ref_quit(self.h, actor, reason)

    def become(self, actor, behavior: int, n: int = 0, forward_to: int = 0) -> int:
        sa = SpawnArgs(n, forward_to)
        return self.L.caf_ref_become(self.h, actor, behavior, C.byref(sa))

    def timeout(self, req) -> int:
        return self.L.caf_ref_timeout(self.h, req)

    def reply(self, req):
        """Returns (resolved, status, ndarray or None, resolutions)."""
        st = C.c_int32(0)
        nb = C.c_uint64(0)
        dt = C.c_int32(0)
        res = C.c_uint32(0)
        r = self.L.caf_ref_reply(self.h, req, C.byref(st), None, 0, C.byref(nb), C.byref(dt),
                                 C.byref(res))
        if r < 0:
            raise KeyError(req)
        if r == 0:
            return False, None, None, res.value
        buf = np.zeros(nb.value, np.uint8)
        if nb.value:
            self.L.caf_ref_reply(self.h, req, None, _ptr(buf), nb.value, None, None, None)
        data = buf.view(_NP[dt.value]) if nb.value else None
        return True, st.value, data, res.value

    def dequeue_log(self, actor):
        n = self.L.caf_ref_dequeue_log(self.h, actor, None, None, 0)
        s = np.zeros(n, np.uint32)
        q = np.zeros(n, np.uint32)
        if n:
            self.L.caf_ref_dequeue_log(self.h, actor, _ptr(s), _ptr(q), n)
        return list(zip(s.tolist(), q.tolist()))

    def state(self, actor) -> int:
        return int(self.L.caf_ref_actor_state(self.h, actor))


def mandel_args(re_min, im_min, step_re, step_im, width, height, row0, rows, max_iter, fp=F32):
    return MandelArgs(re_min, im_min, step_re, step_im, width, height, row0, rows, max_iter, fp)
