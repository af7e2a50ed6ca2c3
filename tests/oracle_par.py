"""Runs the CPU oracle over many independent rows or messages in threads.

The oracle's ctypes calls release the GIL, so a thread pool runs disjoint
row blocks (or whole messages) in parallel without forking a process that
may already hold the GPU.  Nothing here computes anything itself: every
value comes from one oracle call on one disjoint piece of the work, and the
pieces are put back in place.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle


def threads() -> int:
    # At most 16 worker processes: a test host may grant fewer CPUs than
    # os.cpu_count() reports.
    return max(1, min(16, os.cpu_count() or 1))


def mandel_image(vp, fp: str, block_rows: int = 8) -> np.ndarray:
    """The whole image [height][width] of viewport vp, by the oracle."""
    oracle.lib()  # built and loaded once, before the threads start
    out = np.zeros((vp.height, vp.width), np.uint16)

    def run(r0):
        rows = min(block_rows, vp.height - r0)
        out[r0:r0 + rows] = oracle.mandelbrot(vp.re_min, vp.im_min, vp.step_re, vp.step_im,
                                              vp.width, r0, rows, vp.max_iter, fp)

    with ThreadPoolExecutor(threads()) as ex:
        list(ex.map(run, range(0, vp.height, block_rows)))
    return out


def mandel_images(vps, fp: str) -> list[np.ndarray]:
    return [mandel_image(vp, fp) for vp in vps]


def gemms(pairs, dtype: str = "f32") -> list[np.ndarray]:
    """The oracle product of each (A, B) pair."""
    oracle.lib()
    with ThreadPoolExecutor(threads()) as ex:
        return list(ex.map(lambda ab: oracle.gemm(ab[0], ab[1], dtype), pairs))
