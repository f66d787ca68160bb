"""The oracle on hand-worked examples stored under tests/golden/ (each file
cites the passage it follows and shows the derivation; the expected values
are exact and were worked out by hand from the paper's equations, not
produced by the oracle).  CPU only."""
import json
import math
import os

import numpy as np
import pytest

import gen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def test_golden_files_cite_their_passage():
    names = sorted(f for f in os.listdir(GOLDEN) if f.endswith(".json"))
    assert len(names) >= 4
    for f in names:
        g = load(f)
        assert g["citation"] and g["derivation"], f


def test_eq3_composite_three_gaussians(orc):
    g = load("eq3_composite_three_gaussians.json")
    cam = gen.make_camera(g["width"], g["height"])
    coef, fT, last, _ = orc.composite(cam, np.asarray(g["tile_ranges"], np.uint32), np.asarray(g["ids"], np.uint32),
                                      np.asarray(g["mean2d"], np.float64), np.asarray(g["conic"], np.float64),
                                      np.asarray(g["opacity"], np.float64), np.asarray(g["topk_idx"], np.int32),
                                      np.asarray(g["topk_w"], np.float32), g["L"])
    for e in g["expected"]:
        x, y = e["pixel"]
        np.testing.assert_allclose(coef[0, y, x], e["coef"], rtol=0, atol=1e-15)
        assert fT[y, x] == pytest.approx(e["final_T"], abs=1e-15)
        assert last[y, x] == e["last"]


def test_eq7_decode_small(orc):
    g = load("eq7_decode_small.json")
    F = orc.decode(np.asarray(g["W"], np.float64), np.asarray(g["S"], np.float32))
    np.testing.assert_array_equal(F, np.asarray(g["F"]))


def test_sec32_lerf_relevancy(orc):
    g = load("sec32_lerf_relevancy.json")
    r = orc.query(np.asarray(g["feat"], np.float64), np.asarray(g["pos"], np.float32),
                  np.asarray(g["neg"], np.float32), tau=g["tau"])
    np.testing.assert_allclose(r, g["relevancy"], rtol=0, atol=1e-12)


def test_sec33_topk_softmax_codes(orc):
    g = load("sec33_topk_softmax_codes.json")
    for row, K, idx, w in zip(g["logits_ln_of"], g["K"], g["idx"], g["w"]):
        logits = np.log(np.asarray([row], np.float64))
        got_idx, got_w = orc.sparse_codes(logits, K)
        assert got_idx[0].tolist() == idx
        np.testing.assert_allclose(got_w[0], [a / b for a, b in w], rtol=0, atol=1e-12)
    assert math.isclose(sum(a / b for a, b in g["w"][0]), 1.0)
