"""The analytic floating-stability module against the paper's printed numbers
(Sec. 3.3) and against itself (Scribanti is exact while wall-sided)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import analytic as A
from oracle.oracle import integrate_body

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


@pytest.mark.parametrize("rho_s", [0.25, 0.5, 0.75])
def test_cube_stable_heel_matches_paper(rho_s):
    want = GOLD["stable_heel_deg"]["rho_%s" % rho_s]
    got = A.stable_heel_angles(1.0, 1.0, rho_s)
    assert min(abs(a - want) for a in got) < 2e-3


@pytest.mark.parametrize("b,h", [(32, 16), (24, 16), (20, 16), (64, 32)])
def test_scribanti_equals_polygon_while_wall_sided(b, h):
    lim = A.wall_sided_limit(b, h, 0.5)
    for frac in (0.1, 0.5, 0.9, 0.999):
        a = frac * lim
        assert A.righting_moment_polygon(b, h, 2 * h, a, 1e-4, zw=0.0) == pytest.approx(
            A.righting_moment_scribanti(b, h, 2 * h, a, 1e-4), rel=1e-9)
    # beyond the wall-sided range the formula overestimates
    a = 1.2 * lim
    assert A.righting_moment_scribanti(b, h, 2 * h, a, 1e-4) > A.righting_moment_polygon(b, h, 2 * h, a, 1e-4,
                                                                                        zw=0.0)


def test_cube_upright_is_unstable_and_wide_box_stable():
    """Fig. stabilityCurves: the cube's stability curve starts with a negative
    slope (upright unstable); wider boxes are stable."""
    assert A.righting_moment_scribanti(4, 4, 1, 0.05, 1.0) < 0
    assert A.righting_moment_scribanti(6, 4, 1, 0.05, 1.0) > 0


def test_half_immersed_area_is_half():
    for a in np.linspace(0, 1.2, 7):
        assert A.immersed_section(32, 16, a, 0.0)[0] == pytest.approx(256.0, rel=1e-12)


def test_integrator_free_fall_and_spin():
    half = np.array([2.0, 3.0, 4.0])
    M = 0.5 * 8 * 24
    g = np.array([0.0, 0.0, -1e-3])
    b = dict(pos=np.array([10.0, 10.0, 10.0]), quat=np.array([1.0, 0, 0, 0]), vel=np.zeros(3), omega=np.zeros(3))
    T = np.array([0.3, 0.0, 0.0])
    Ixx = M / 3 * (3 ** 2 + 4 ** 2)
    for k in range(1, 11):
        nb = integrate_body(half, b["pos"], b["quat"], b["vel"], b["omega"], 0.5, np.zeros(3), T, g, 0x3F)
        b.update(nb)
        np.testing.assert_allclose(b["vel"], k * g, rtol=1e-14)
        assert b["omega"][0] == pytest.approx(k * 0.3 / Ixx, rel=1e-12)
    # positions: semi-implicit Euler sum_k k*g = 55 g
    np.testing.assert_allclose(b["pos"], np.array([10, 10, 10]) + 55 * g, rtol=1e-14)
    # rotation about x only: quaternion angle = sum_k k * 0.3 / Ixx
    ang = 55 * 0.3 / Ixx
    np.testing.assert_allclose(b["quat"], [math.cos(ang / 2), math.sin(ang / 2), 0, 0], atol=1e-15)


def test_integrator_dof_mask_roll_only():
    half = np.array([16.0, 16.0, 8.0])
    q = np.array([math.cos(0.2), math.sin(0.2), 0, 0])
    nb = integrate_body(half, np.zeros(3), q, np.zeros(3), np.zeros(3), 0.5, np.array([1.0, 2, 3]),
                        np.array([0.5, 0.7, 0.9]), np.array([0, 0, -1e-4]), 0x08)
    assert np.all(nb["vel"] == 0) and nb["omega"][1] == 0 and nb["omega"][2] == 0
    M = 0.5 * 8 * 16 * 16 * 8
    # roll about the world x axis: I_xx of the body rotated about x is its body I_xx
    assert nb["omega"][0] == pytest.approx(0.5 / (M / 3 * (16 ** 2 + 8 ** 2)), rel=1e-12)


@pytest.mark.parametrize("zw", [-4.0, 0.0, 4.0, 4.5])
@pytest.mark.parametrize("alpha_deg", [5.0, 20.7, 40.0])
def test_offset_waterline_moment_matches_grid_integral(zw, alpha_deg):
    """Brute force: the immersed area and buoyancy lever of a heeled 16 x 16
    section with the water plane zw above G, summed over a fine grid of
    sample points, agree with the clipped-polygon moment."""
    n, b, h, g = 1000, 16.0, 16.0, 7.5e-4
    a = math.radians(alpha_deg)
    u = (np.arange(n) + 0.5) / n
    yb, zb = np.meshgrid((u - 0.5) * b, (u - 0.5) * h, indexing="ij")
    y = yb * math.cos(a) - zb * math.sin(a)
    z = yb * math.sin(a) + zb * math.cos(a)
    wet = z <= zw
    area = wet.sum() * (b / n) * (h / n)
    cy = y[wet].mean()
    brute = -g * area * 32.0 * cy
    exact = A.righting_moment_polygon(b, h, 32.0, a, g, zw=zw)
    assert exact == pytest.approx(brute, rel=2e-3, abs=2e-3 * g * b * h * 32.0 * 0.05)


def test_fixed_centre_stable_heel_of_cubes():
    """A cube held at its upright equilibrium draft and free to turn only
    about its long axis: 45 deg at density 1/2 (the half-immersed square is
    symmetric about its diagonal), the same angle for densities 1/4 and 3/4
    (the wet part of one is the point reflection of the dry part of the
    other through G), and that angle lies below the free-floating 26.565 deg."""
    s = 16.0
    half = A.stable_heel_angles(s, s, 0.5, zw=0.5 * s - s / 2)
    assert min(abs(x - 45.0) for x in half) < 1e-3
    lo = A.stable_heel_angles(s, s, 0.25, zw=0.25 * s - s / 2)
    hi = A.stable_heel_angles(s, s, 0.75, zw=0.75 * s - s / 2)
    assert lo[0] == pytest.approx(hi[0], abs=1e-6)
    assert 15.0 < lo[0] < 26.0
