"""Seeded synthetic inputs for the compute-actor workloads.

This module only draws inputs: viewports, matrices, message mixes and
arrival times.  It contains none of the arithmetic the actors compute, so
that the GPU path and the CPU oracle can both be fed from it while sharing
no code.  Every generator takes a seed and uses numpy's PCG64.

Workload shapes follow the paper's experiments (Sec. 7.4: an N x N image of
[-1.5-i, 0.5+i]; Sec. 7.5: a 1920x1080 image of [-0.5-0.7375i, 0.1-0.1375i]
at 1,200 and 120 iterations) and the matrix-multiply actor of Sec. 4.6.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass(frozen=True)
class Viewport:
    """Lower-left corner and pixel steps; pixel (x, y) samples
    re_min + x*step_re + i*(im_min + y*step_im)."""
    re_min: float
    im_min: float
    step_re: float
    step_im: float
    width: int
    height: int
    max_iter: int


def tiny_viewport() -> Viewport:
    """512x512 over re in [-2.5, 1], im in [-1.25, 1.25], 100 iterations.
    Both steps are dyadic (7/1024 and 5/1024), so every sample point is
    exactly representable in float."""
    return Viewport(-2.5, -1.25, 3.5 / 512, 2.5 / 512, 512, 512, 100)


def paper_replica_viewport(max_iter: int = 1200) -> Viewport:
    """The Sec. 7.5 workload: 1920x1080 over [-0.5-0.7375i, 0.1-0.1375i]
    (non-square pixels: 0.6 wide and 0.6 high on a 16:9 grid)."""
    return Viewport(-0.5, -0.7375, 0.6 / 1920, 0.6 / 1080, 1920, 1080, max_iter)


def boundary_viewport(seed: int, width: int = 1920, height: int = 1080,
                      max_iter: int = 1000) -> Viewport:
    """A viewport centred on a seeded point of the main cardioid's boundary,
    c0 = e^{i t}/2 - e^{2 i t}/4 with t ~ U[0, 2 pi), zoomed by Z = 10^{4u},
    u ~ U[0, 1] (zoom 1 to 1e4), 3.5/Z wide, square pixels."""
    g = rng(seed)
    t = g.uniform(0.0, 2.0 * math.pi)
    u = g.uniform(0.0, 1.0)
    c0 = complex(math.cos(t), math.sin(t)) / 2 - complex(math.cos(2 * t), math.sin(2 * t)) / 4
    zoom = 10.0 ** (4.0 * u)
    step = 3.5 / zoom / width
    return Viewport(c0.real - 0.5 * width * step, c0.imag - 0.5 * height * step, step, step,
                    width, height, max_iter)


def random_square_viewport(g: np.random.Generator, side: int, max_iter: int) -> Viewport:
    """Serving-mix tile: a side x side square at a boundary viewport."""
    t = g.uniform(0.0, 2.0 * math.pi)
    u = g.uniform(0.0, 1.0)
    c0 = complex(math.cos(t), math.sin(t)) / 2 - complex(math.cos(2 * t), math.sin(2 * t)) / 4
    zoom = 10.0 ** (4.0 * u)
    step = 3.5 / zoom / side
    return Viewport(c0.real - 0.5 * side * step, c0.imag - 0.5 * side * step, step, step,
                    side, side, max_iter)


def row_tiles(height: int, tile_rows: int = 64) -> list[tuple[int, int]]:
    """(row0, rows) of each tile message; the last tile keeps the remainder
    (1080 = 16*64 + 56)."""
    return [(r, min(tile_rows, height - r)) for r in range(0, height, tile_rows)]


def uniform_matrix(g: np.random.Generator, n: int) -> np.ndarray:
    return g.uniform(-1.0, 1.0, size=(n, n)).astype(np.float32)


def to_bf16_bits(a: np.ndarray) -> np.ndarray:
    """Round float32 to bfloat16 (round to nearest, ties to even) and return
    the 16-bit patterns.  These rounded values *are* the message content of
    a bfloat16 request; inputs are finite."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)
    return r.astype(np.uint16)


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    return (np.ascontiguousarray(b, np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


def gemm_pair(seed: int, n: int, dtype: str = "f32"):
    """A, B with entries U(-1, 1); bf16 requests carry the RNE-rounded bits."""
    g = rng(seed)
    A = uniform_matrix(g, n)
    B = uniform_matrix(g, n)
    if dtype == "bf16":
        return to_bf16_bits(A), to_bf16_bits(B)
    return A, B


def integer_matrix(seed: int, n: int, lo: int = -4, hi: int = 4) -> np.ndarray:
    """Small integers: products and sums are exact in float32 and bfloat16."""
    return rng(seed).integers(lo, hi + 1, size=(n, n)).astype(np.float32)


def gemm_sizes(seed: int, count: int, choices=(64, 128, 256, 512)) -> np.ndarray:
    return rng(seed).choice(np.asarray(choices, np.int64), size=count)


def poisson_arrivals(seed: int, rate: float, duration_s: float) -> np.ndarray:
    """Open-loop arrival times in ns (exponential inter-arrival gaps)."""
    g = rng(seed)
    n_est = int(rate * duration_s * 1.2) + 16
    gaps = g.exponential(1.0 / rate, size=n_est)
    t = np.cumsum(gaps)
    t = t[t < duration_s]
    return (t * 1e9).astype(np.int64)


MAX_ITERS = (256, 512, 1024, 2048, 4096)
SQUARES = (64, 128, 256, 512)
SERVE_GEMM_N = (32, 64, 128, 256, 512)


@dataclass
class ServeMsg:
    kind: str           # "mandel" or "gemm"
    arrival_ns: int
    vp: Viewport | None = None
    n: int = 0
    seed: int = 0


def serving_mix(seed: int, rate: float, duration_s: float, mandel_frac: float = 0.7):
    """Poisson arrivals; 70 % Mandelbrot squares (64^2..512^2, max_iter in
    256..4096, random boundary viewport, float), 30 % float GEMM with n in
    {32, ..., 512}."""
    g = rng(seed + 1000)
    arr = poisson_arrivals(seed, rate, duration_s)
    msgs = []
    for i, t in enumerate(arr):
        if g.uniform() < mandel_frac:
            side = int(g.choice(SQUARES))
            mi = int(g.choice(MAX_ITERS))
            msgs.append(ServeMsg("mandel", int(t), vp=random_square_viewport(g, side, mi)))
        else:
            msgs.append(ServeMsg("gemm", int(t), n=int(g.choice(SERVE_GEMM_N)),
                                 seed=int(g.integers(0, 2**31))))
    return msgs


def serving_mix_arrays(seed: int, rate: float, duration_s: float, mandel_frac: float = 0.7):
    """Vectorised serving_mix: returns a dict of numpy arrays (arrival_ns,
    is_mandel, side, max_iter, re_min, im_min, step, gemm_n) with the same
    distributions (boundary viewports of the main cardioid, zoom 1 to 1e4)."""
    g = rng(seed + 1000)
    arr = poisson_arrivals(seed, rate, duration_s)
    n = arr.size
    is_m = g.uniform(size=n) < mandel_frac
    side = g.choice(np.asarray(SQUARES), size=n)
    mi = g.choice(np.asarray(MAX_ITERS), size=n)
    t = g.uniform(0.0, 2.0 * math.pi, size=n)
    u = g.uniform(0.0, 1.0, size=n)
    c0 = np.exp(1j * t) / 2 - np.exp(2j * t) / 4
    zoom = 10.0 ** (4.0 * u)
    step = 3.5 / zoom / side
    gn = g.choice(np.asarray(SERVE_GEMM_N), size=n)
    return {"arrival_ns": arr, "is_mandel": is_m, "side": side.astype(np.uint32),
            "max_iter": mi.astype(np.uint32), "re_min": c0.real - 0.5 * side * step,
            "im_min": c0.imag - 0.5 * side * step, "step": step, "gemm_n": gn.astype(np.uint32)}
