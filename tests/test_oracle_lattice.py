"""Pins of the oracle's lattice, equilibrium, force term, stream and collide
against closed forms (Sec. 2.1 of the paper)."""
from fractions import Fraction

import numpy as np
import pytest

from oracle.oracle import Oracle, feq, force_term, lattice

# Fig. d3q19 caption order; a direction's vector follows from its letters
# (E/W = +-x, N/S = +-y, T/B = +-z).
CAPTION = ["C", "W", "E", "N", "S", "T", "B", "TW", "TE", "TN", "TS", "NW", "NE", "SW", "SE", "BW", "BE", "BN",
           "BS"]
LETTER = {"E": (1, 0, 0), "W": (-1, 0, 0), "N": (0, 1, 0), "S": (0, -1, 0), "T": (0, 0, 1), "B": (0, 0, -1)}


def test_velocity_set_follows_caption_names():
    c, w, opp = lattice()
    for i, name in enumerate(CAPTION):
        v = np.zeros(3, dtype=int)
        for ch in name.replace("C", ""):
            v += LETTER[ch]
        assert tuple(c[i]) == tuple(v), name
    for i in range(19):
        assert tuple(c[opp[i]]) == tuple(-c[i])
    # weights: 1/3 centre, 1/18 axis, 1/36 diagonal (caption)
    assert w[0] == pytest.approx(1 / 3, abs=0)
    assert all(w[i] == 1 / 18 for i in range(1, 7))
    assert all(w[i] == 1 / 36 for i in range(7, 19))


def test_isotropy_exact_rationals():
    c, w, _ = lattice()
    W = [Fraction(1, 3)] + [Fraction(1, 18)] * 6 + [Fraction(1, 36)] * 12
    assert sum(W) == 1
    for a in range(3):
        assert sum(W[i] * c[i][a] for i in range(19)) == 0
        for b in range(3):
            assert sum(W[i] * c[i][a] * c[i][b] for i in range(19)) == (Fraction(1, 3) if a == b else 0)
            for g in range(3):
                assert sum(W[i] * c[i][a] * c[i][b] * c[i][g] for i in range(19)) == 0
                for d in range(3):
                    want = Fraction(int(a == b and g == d) + int(a == g and b == d) + int(a == d and b == g), 9)
                    assert sum(W[i] * c[i][a] * c[i][b] * c[i][g] * c[i][d] for i in range(19)) == want


@pytest.mark.parametrize("seed", range(4))
def test_equilibrium_moments(seed):
    rng = np.random.default_rng(seed)
    c, _, _ = lattice()
    rho = rng.uniform(0.8, 1.2)
    u = rng.uniform(-0.1, 0.1, 3)
    f = feq(rho, u)
    assert f.sum() == pytest.approx(rho, rel=1e-14)
    np.testing.assert_allclose(c.T @ f, rho * u, atol=1e-15)
    P = np.einsum("ia,ib,i->ab", c, c, f)
    np.testing.assert_allclose(P, rho * np.outer(u, u) + rho / 3 * np.eye(3), atol=1e-15)


@pytest.mark.parametrize("seed", range(4))
def test_force_term_moments(seed):
    """Luo's term: zero mass, momentum rho*a, second moment rho(ua + au).  A
    factor 1/2 on the (c.u) c term, as printed, would break all of these but
    the first order one."""
    rng = np.random.default_rng(10 + seed)
    c, _, _ = lattice()
    rho = rng.uniform(0.8, 1.2)
    u = rng.uniform(-0.1, 0.1, 3)
    a = rng.uniform(-1e-3, 1e-3, 3)
    F = force_term(rho, u, a)
    assert abs(F.sum()) < 1e-17
    np.testing.assert_allclose(c.T @ F, rho * a, atol=1e-18)
    np.testing.assert_allclose(np.einsum("ia,ib,i->ab", c, c, F), rho * (np.outer(u, a) + np.outer(a, u)),
                               atol=1e-18)


def test_single_cell_collide_conserves_mass_adds_momentum():
    """A 1x1x1 periodic liquid cell streams onto itself: one step is one
    collision, which keeps rho and adds rho*a to the momentum."""
    c, _, _ = lattice()
    a = np.array([1e-4, -2e-4, 3e-4])
    o = Oracle(1, 1, 1, 0.7, accel=a, periodic=7)
    o.init_basin(10.0)
    rng = np.random.default_rng(0)
    f0 = rng.uniform(0.9, 1.1, (19, 1, 1, 1)) / 19
    o.set_f(f0)
    o.step(1)
    f1 = o.get_f()
    rho0 = f0.sum()
    assert f1.sum() == pytest.approx(rho0, rel=1e-14)
    np.testing.assert_allclose(np.einsum("ia,izyx->a", c, f1) - np.einsum("ia,izyx->a", c, f0), rho0 * a,
                               atol=1e-16)


@pytest.mark.parametrize("i", range(1, 19))
def test_stream_moves_one_cell(i):
    """With collisions switched off (tau huge) a perturbation of population i
    moves by exactly c_i per step (Eq. stream), across the periodic wrap."""
    c, w, _ = lattice()
    n = 5
    o = Oracle(n, n, n, 1e300, periodic=7)
    o.init_basin(100.0)
    f = np.broadcast_to(w[:, None, None, None], (19, n, n, n)).copy()
    src = np.array([0, 2, 4])  # (x, y, z)
    f[i, src[2], src[1], src[0]] += 1e-3
    o.set_f(f)
    o.step(1)
    d = o.get_f() - w[:, None, None, None]
    dst = (src + c[i]) % n
    assert d[i, dst[2], dst[1], dst[0]] == pytest.approx(1e-3, rel=1e-12)
    d[i, dst[2], dst[1], dst[0]] = 0
    assert np.abs(d).max() < 1e-15


def test_periodic_box_conserves_mass_and_momentum():
    c, _, _ = lattice()
    o = Oracle(6, 5, 4, 0.7, periodic=7)
    o.init_basin(100.0, seed=3, noise_amp=1e-3)
    f0 = o.get_f()
    o.step(25)
    f1 = o.get_f()
    assert abs(f1.sum() - f0.sum()) < 1e-12
    np.testing.assert_allclose(np.einsum("ia,izyx->a", c, f1), np.einsum("ia,izyx->a", c, f0), atol=1e-13)


def test_body_force_adds_total_momentum():
    c, _, _ = lattice()
    a = np.array([2e-5, 0.0, -1e-5])
    o = Oracle(5, 4, 3, 0.9, accel=a, periodic=7)
    o.init_basin(100.0, seed=5, noise_amp=1e-3)
    f0 = o.get_f()
    M = f0.sum()
    o.step(10)
    dJ = np.einsum("ia,izyx->a", c, o.get_f()) - np.einsum("ia,izyx->a", c, f0)
    np.testing.assert_allclose(dJ, 10 * M * a, rtol=1e-10, atol=1e-13)
