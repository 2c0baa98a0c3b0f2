"""Pins of the oracle's spherical bodies (Sec. 2.3 mapping by cell centres;
Sec. 3, the sphere of radius 5 whose discretised volume the paper plots
around 523.6, and the free advection test of a sphere in uniform flow)
against closed forms."""
import math
import os

import numpy as np
import pytest

from oracle.oracle import PH_REMAP, SPHERE, Oracle, feq, integrate_body, lattice

C, WTS, OPP = lattice()
NT = min(8, os.cpu_count() or 1)


def _mapped_count(r, centre, n=16):
    o = Oracle(n, n, n, 0.7, threads=NT)
    o.init_basin(0.0)
    o.set_body(0, (r, r, r), tuple(centre), shape=SPHERE)
    o.step(1, PH_REMAP)
    c = int((o.types() == 3).sum())
    o.close()
    return c


def test_sphere_mean_discrete_volume_is_the_volume():
    """Cell centres form a unit lattice, so the number of centres inside a
    sphere placed at a uniformly random offset has the sphere's volume as its
    expectation: 4/3 pi r^3 = 523.6 for r = 5 (the paper's ideal volume)."""
    r = 5.0
    rng = np.random.default_rng(7)
    counts = np.array([_mapped_count(r, 8.0 + rng.uniform(0.0, 1.0, 3)) for _ in range(96)])
    vol = 4.0 / 3.0 * math.pi * r ** 3
    sem = counts.std() / math.sqrt(len(counts))
    assert abs(counts.mean() - vol) < 4.0 * sem + 1e-9, (counts.mean(), vol, sem)
    # the discretised volume moves with the position (the paper's Fig.
    # volumeerror: a few cells around 523.6)
    assert counts.min() < vol < counts.max()


def test_sphere_volume_is_periodic_along_an_axis_path():
    """Moving along an axis by one cell maps the same number of cells (the
    paper's curve repeats after 10000 steps of 1e-4), and the count depends on
    the sub-cell position."""
    r = 5.0
    path = [np.array([7.0 + t, 8.25, 8.5]) for t in np.arange(0.0, 1.0, 0.125)]
    a = [_mapped_count(r, p) for p in path]
    b = [_mapped_count(r, p + np.array([1.0, 0.0, 0.0])) for p in path]
    assert a == b
    assert len(set(a)) > 1


def test_sphere_integrator_mass_and_inertia():
    """Rigid-body update of a sphere: M = rho_s 4/3 pi r^3, and the inertia
    2/5 M r^2 is the same about every axis, whatever the orientation."""
    r, rho_s = 6.0, 0.5
    M = rho_s * 4.0 / 3.0 * math.pi * r ** 3
    I = 0.4 * M * r * r
    F = np.array([3e-3, -2e-3, 5e-3])
    T = np.array([4e-2, 1e-2, -3e-2])
    for q in [(1.0, 0.0, 0.0, 0.0), (math.cos(0.4), 0.0, math.sin(0.4) * 0.6, math.sin(0.4) * 0.8)]:
        out = integrate_body((r, r, r), (10.0, 10.0, 10.0), q, (0, 0, 0), (0, 0, 0), rho_s, F, T, (0, 0, 0), 0x3F,
                             shape=SPHERE)
        np.testing.assert_allclose(out["vel"], F / M, rtol=1e-14)
        np.testing.assert_allclose(out["omega"], T / I, rtol=1e-13)


def test_sphere_in_uniform_flow_keeps_the_flow_velocity():
    """Sec. 3.2, first free advection run (all liquid, no gravity): a free
    sphere of diameter 12 in a uniform flow moves with the flow to the last
    digit while it is remapped: moving-wall bounce-back of f_eq(rho, u) with
    u_w = u returns f_eq, and refilled cells get f_eq(1, u_w)."""
    n = 24
    u = np.array([0.025, -0.013, 0.006])
    o = Oracle(n, n, n, 0.7, periodic=7, threads=NT)
    o.init_basin(1e9)
    fe = feq(1.0, u)
    o.set_f(np.broadcast_to(fe[:, None, None, None], (19, n, n, n)).copy())
    body = dict(r=6.0, pos=np.array([11.7, 12.2, 11.9]), vel=u.copy(), omega=np.zeros(3))
    moved = 0
    for k in range(50):
        o.set_body(0, (body["r"],) * 3, body["pos"], (1, 0, 0, 0), body["vel"], body["omega"], 1.0, 0,
                   shape=SPHERE)
        before = o.get_flags()
        o.step(1)
        moved += int((o.get_flags() != before).sum())
        F, T = o.body_forces(0)
        assert np.abs(F).max() < 1e-12 and np.abs(T).max() < 1e-11
        nb = integrate_body((body["r"],) * 3, body["pos"], (1, 0, 0, 0), body["vel"], body["omega"], 1.0, F, T,
                            (0, 0, 0), 0x3F, shape=SPHERE)
        body.update(pos=nb["pos"], vel=nb["vel"], omega=nb["omega"])
    assert moved > 50
    np.testing.assert_allclose(body["vel"], u, rtol=0, atol=1e-14)
    f = o.get_f()
    rho = f.sum(0)
    t = o.types()
    vel = np.einsum("ia,izyx->azyx", C, f) / np.where(rho > 0, rho, 1.0)
    np.testing.assert_allclose(vel[:, t == 1].max(axis=1), u, atol=1e-13)
    np.testing.assert_allclose(vel[:, t == 1].min(axis=1), u, atol=1e-13)


def test_sphere_archimedes_relaxed():
    """A fixed, fully submerged sphere of radius 5: after the liquid relaxes,
    F_z = rho g V with V the discretised volume (its obstacle cells) and rho
    the liquid density at its centre; no sideways force."""
    g, r = 1e-4, 5.0
    o = Oracle(20, 20, 32, 1.0, accel=(0, 0, -g), periodic=3, threads=NT)
    o.init_basin(28.0)
    centre = (10.3, 9.8, 12.4)
    o.set_body(0, (r, r, r), centre, shape=SPHERE)
    o.step(2500)
    F, _ = o.body_forces(0)
    vol = int((o.types() == 3).sum())
    rho_c = 1.0 + 3.0 * g * (28.0 - centre[2])
    assert F[2] / (rho_c * g * vol) == pytest.approx(1.0, abs=0.002)
    assert abs(F[0]) < 1e-3 * F[2] and abs(F[1]) < 1e-3 * F[2]
