"""The oracle's righting moments of four instances of the 48-instance heel
sweep, each run alone (tests/golden/batch48_righting.json, written by
make_batch_righting.py, which calls only the oracle), checked against the
workload generator and the closed form: the exact moment of the immersed
polygon of a cuboid held with its centre of gravity at a fixed height over
the water plane (Sec. 4, stability of a floating box).  The staircase of
mapped cells sets how far the lattice moment can be from the continuous one:
the coarsest section here is 16 x 8 cells (half the 128^3 case's), the
others 28 x 14 and 32 x 16."""
import json
import math
import os

from oracle import analytic as A
from paper_1201_0351_amd import workloads as W

PATH = os.path.join(os.path.dirname(__file__), "golden", "batch48_righting.json")


def _gold():
    with open(PATH) as f:
        return json.load(f)


def test_golden_batch_file_matches_the_workload():
    g = _gold()
    assert (g["steps"], g["window"], g["every"]) == (3000, 1000, 10)
    insts = W.config4()["instances"]
    assert [r["instance"] for r in g["runs"]] == [43, 36, 13, 11]
    for r in g["runs"]:
        i = insts[r["instance"]]
        lat, b = i["lattice"], i["bodies"][0]
        assert r["shape"] == [lat["nx"], lat["ny"], lat["nz"]]
        assert r["density"] == b["density"]
        assert abs(r["heel_deg"] - math.degrees(2.0 * math.atan2(b["quat"][1], b["quat"][0]))) < 1e-9


def test_golden_batch_moments_match_closed_form():
    """Restoring at every heel (up to 59 deg) and within 20% of the closed
    form on the 16 x 8 section, 4% on the finer ones (measured: 17.0% and
    1.5%, 0.14%, 2.7%)."""
    insts = W.config4()["instances"]
    for r in _gold()["runs"]:
        i = insts[r["instance"]]
        b = i["bodies"][0]
        hx, hy, hz = b["half"]
        zw = 0.5 * i["lattice"]["nz"] - b["pos"][2]  # water plane over G (filled to half depth)
        ana = A.righting_moment_polygon(2 * hy, 2 * hz, 2 * hx, math.radians(r["heel_deg"]), 5e-6, zw=zw)
        assert r["m_s"] > 0 and ana > 0
        bound = 0.20 if 2 * hy < 20 else 0.04
        assert abs(r["m_s"] - ana) / ana < bound, (r["instance"], r["m_s"], ana)


def test_golden_batch_thin_film_realisations():
    """Instances whose low deck edge lies less than 1.5 cells under the water
    carry oracle runs from initial noise of 1e-7 (seeds 1..4), and those
    spread by more than 1%: the reason such an instance is compared as an
    ensemble on the GPU (measured: 3.9% for the 16 x 8 section at 29.6 deg).
    The others are well clear of the waterline or deep under it."""
    for r in _gold()["runs"]:
        d = r["deck_edge_depth"]
        if 0.0 < d < 1.5:
            ens = [r["m_s"]] + r["m_s_noise_1e-7"]
            assert len(ens) == 5
            assert (max(ens) - min(ens)) / min(ens) > 0.01
        else:
            assert "m_s_noise_1e-7" not in r and abs(d) > 5.0
