"""The oracle's held-box righting moments at 128^3 (tests/golden/
righting_moment_128.json, written by make_righting_moment.py, which calls
only the oracle) checked against the closed form: the exact moment of the
immersed polygon of a cuboid held with its centre of gravity on the water
plane (Sec. 4 stability of a floating box).  The discrete wall sits on the
staircase of mapped cells, so the lattice moment differs from the
continuous one by a few percent at this resolution (32 x 16 cells of
section); the bound below is the one the resolution study of the oracle
shows, and the sign and the growth with heel are exact requirements."""
import json
import math
import os

import pytest

from oracle import analytic as A

PATH = os.path.join(os.path.dirname(__file__), "golden", "righting_moment_128.json")


def _gold():
    with open(PATH) as f:
        return json.load(f)


def test_golden_file_complete():
    g = _gold()
    assert [r["heel_deg"] for r in g["runs"]] == [10.0, 20.0, 30.0]
    for r in g["runs"]:
        assert r["steps"] == 5000 and r["window"] == 1000 and r["every"] == 10


def test_golden_moments_match_closed_form():
    for r in _gold()["runs"]:
        ana = A.righting_moment_polygon(32, 16, 32, math.radians(r["heel_deg"]), 5e-6, zw=0.0)
        assert r["analytic_polygon"] == pytest.approx(ana, rel=1e-12)
        assert r["m_s"] > 0  # restoring
        assert abs(r["m_s"] - ana) / ana < 0.05, (r["heel_deg"], r["m_s"], ana)


def test_golden_moments_grow_with_heel():
    ms = [r["m_s"] for r in _gold()["runs"]]
    assert ms[0] < ms[1] < ms[2]
