"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/lgs_lbm.h declares, validates configurations on the host, and its
host rigid-body update agrees with the oracle's (no device calls here)."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from oracle.oracle import SPHERE
from oracle.oracle import integrate_body as oracle_integrate
from paper_1201_0351_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            names |= set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = lbm.library()
    names = declared_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n


def test_struct_sizes_match_header_layout():
    assert C.sizeof(lbm.lbm_config) == 4 * 4 + 8 + 24 + 8 * 4 + 4 + 4 + 8 + 8 + 8 + 4 + 4 + 24 + 8
    # 17 doubles, then fixed, dof_mask and shape (uint32), padded to 8 bytes
    assert C.sizeof(lbm.lbm_body) == 8 * (3 + 3 + 4 + 3 + 3 + 1) + 4 * 3 + 4


def _ws(cfg):
    n = C.c_size_t(0)
    arr = (lbm.lbm_config * 1)(lbm.make_config(cfg))
    rc = lbm.library().lbm_workspace_size(arr, 1, C.byref(n))
    return rc, n.value


def test_workspace_size_and_validation():
    base = dict(nx=32, ny=32, nz=32, tau=0.6, accel=(0, 0, -1e-5), fill_height=16)
    rc, n = _ws(base)
    assert rc == 0 and n > 32 ** 3 * 19 * 4 * 2
    rc16, n16 = _ws(dict(base, storage="fp16"))
    assert rc16 == 0 and n16 < n
    # surface tension adds one float per cell (the curvature), and only then
    rcs, ns = _ws(dict(base, surface_tension=1e-3))
    assert rcs == 0 and ns - n >= 32 ** 3 * 4
    for bad in (dict(tau=0.5), dict(tau=0.3), dict(accel=(0, 0, -2e-3)), dict(nx=0), dict(eps=-1.0),
                dict(rho_gas=0.0), dict(storage="fp16", fp16_scale=3.0), dict(recon_mode=7),
                dict(surface_tension=-1e-3), dict(surface_tension=0.1), dict(surface_tension=float("nan")),
                dict(wall_vel=(0.2, 0.0, 0.0))):
        rc, _ = _ws(dict(base, **bad))
        assert rc == -1, bad
        assert lbm.library().lbm_last_error().decode()


@pytest.mark.parametrize("dof", [0x3F, 0x08, 0x07, 0x28])
def test_host_integrator_matches_oracle(dof):
    rng = np.random.default_rng(dof)
    half = rng.uniform(2, 9, 3)
    ax = rng.normal(size=3)
    ax /= np.linalg.norm(ax)
    ang = 0.4
    q = np.array([math.cos(ang / 2), *(math.sin(ang / 2) * ax)])
    body = dict(half=half, pos=rng.uniform(10, 20, 3), quat=q, vel=rng.normal(0, 1e-3, 3),
                omega=rng.normal(0, 1e-4, 3), density=0.6)
    F, T, a = rng.normal(0, 1e-2, 3), rng.normal(0, 1e-1, 3), np.array([0, 0, -5e-6])
    got = lbm.integrate_body(body, F, T, a, dof)
    want = oracle_integrate(half, body["pos"], q, body["vel"], body["omega"], 0.6, F, T, a, dof)
    for k in ("pos", "vel", "omega", "quat"):
        np.testing.assert_allclose(got[k], want[k], rtol=1e-13, atol=1e-18)


def test_host_integrator_matches_oracle_fast_spin():
    """A rotation of 0.27 rad per step: the half-angle comes from sin and cos
    rather than from the small-angle series."""
    half = np.array([3.0, 5.0, 7.0])
    q = np.array([math.cos(0.2), math.sin(0.2), 0.0, 0.0])
    body = dict(half=half, pos=np.array([15.0, 16.0, 17.0]), quat=q, vel=np.zeros(3),
                omega=np.array([0.15, -0.1, 0.2]), density=0.6)
    F, T, a = np.zeros(3), np.array([0.5, -0.2, 0.1]), np.array([0, 0, -5e-6])
    got = lbm.integrate_body(body, F, T, a, 0x38)
    want = oracle_integrate(half, body["pos"], q, body["vel"], body["omega"], 0.6, F, T, a, 0x38)
    for k in ("pos", "vel", "omega", "quat"):
        np.testing.assert_allclose(got[k], want[k], rtol=1e-13, atol=1e-18)


@pytest.mark.parametrize("dof", [0x3F, 0x38, 0x07])
def test_host_integrator_matches_oracle_sphere(dof):
    """A sphere (radius half_ext[0]): mass 4/3 pi r^3 rho_s and the isotropic
    inertia 2/5 M r^2 on both sides."""
    rng = np.random.default_rng(100 + dof)
    r = 6.5
    ax = rng.normal(size=3)
    ax /= np.linalg.norm(ax)
    q = np.array([math.cos(0.3), *(math.sin(0.3) * ax)])
    body = dict(half=np.array([r, 1.0, 2.0]), pos=rng.uniform(10, 20, 3), quat=q, vel=rng.normal(0, 1e-3, 3),
                omega=rng.normal(0, 1e-4, 3), density=0.5, shape=lbm.SHAPE_SPHERE)
    F, T, a = rng.normal(0, 1e-2, 3), rng.normal(0, 1e-1, 3), np.array([0, 0, -5e-6])
    got = lbm.integrate_body(body, F, T, a, dof)
    want = oracle_integrate((r, r, r), body["pos"], q, body["vel"], body["omega"], 0.5, F, T, a, dof, shape=SPHERE)
    for k in ("pos", "vel", "omega", "quat"):
        np.testing.assert_allclose(got[k], want[k], rtol=1e-13, atol=1e-18)
