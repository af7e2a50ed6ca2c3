"""The stored oracle sums of the headline workload (tests/golden/
headline_sums.json, written by tests/golden/make_headline_sums.py) are the
oracle's own: two images are recomputed here and must match the stored sum,
count of pixels at max_iter and digest bit for bit."""
import hashlib
import json
import os

import numpy as np
import pytest

from paper_1505_07368_amd import gen
from tests import oracle_par

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "headline_sums.json")))


@pytest.mark.parametrize("fp,seed", [("f32", 0), ("f64", 5)])
def test_golden_headline_image_matches_oracle(fp, seed):
    vp = gen.boundary_viewport(seed)
    assert (vp.width, vp.height, vp.max_iter) == (GOLDEN["width"], GOLDEN["height"],
                                                 GOLDEN["max_iter"])
    img = oracle_par.mandel_image(vp, fp)
    g = GOLDEN[fp]["images"][seed]
    assert int(img.sum(dtype=np.int64)) == g["sum"]
    assert int((img == vp.max_iter).sum()) == g["at_max_iter"]
    assert hashlib.sha256(np.ascontiguousarray(img, "<u2").tobytes()).hexdigest() == g["sha256"]


def test_golden_totals_are_the_sums_of_the_images():
    for fp in ("f32", "f64"):
        assert GOLDEN[fp]["total"] == sum(im["sum"] for im in GOLDEN[fp]["images"])
    # float and double counts differ on this workload (precision-specific),
    # and every image has pixels that never escape within max_iter
    assert GOLDEN["f32"]["total"] != GOLDEN["f64"]["total"]
    assert all(im["at_max_iter"] > 0 for im in GOLDEN["f32"]["images"])
