"""Writes headline_sums.json: the oracle's escape-count sums of the headline
image workload (eight seeded 1920x1080 boundary viewports at max_iter 1000),
in float and in double, per image and in total, with a SHA-256 digest of
each whole count image (uint16, row-major, little-endian).

Only the oracle computes here; the viewports come from the seeded input
generator.  Run from the repository root:

    python tests/golden/make_headline_sums.py
"""
from __future__ import annotations

import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from paper_1505_07368_amd import gen  # noqa: E402
from tests import oracle_par  # noqa: E402

SEEDS = list(range(8))
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "headline_sums.json")


def summarise(img: np.ndarray, max_iter: int) -> dict:
    return {"sum": int(img.sum(dtype=np.int64)),
            "at_max_iter": int((img == max_iter).sum()),
            "sha256": hashlib.sha256(np.ascontiguousarray(img, "<u2").tobytes()).hexdigest()}


def main():
    doc = {"_provenance": "oracle escape counts of the headline workload: eight boundary "
                          "viewports (seeds 0-7) of 1920x1080 at max_iter 1000, written by "
                          "tests/golden/make_headline_sums.py (oracle only)",
           "seeds": SEEDS, "width": 1920, "height": 1080, "max_iter": 1000}
    for fp in ("f32", "f64"):
        per = []
        for seed in SEEDS:
            vp = gen.boundary_viewport(seed)
            per.append(summarise(oracle_par.mandel_image(vp, fp), vp.max_iter))
            print(fp, seed, per[-1]["sum"], flush=True)
        doc[fp] = {"images": per, "total": sum(p["sum"] for p in per)}
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    print("wrote", OUT, doc["f32"]["total"], doc["f64"]["total"])


if __name__ == "__main__":
    main()
