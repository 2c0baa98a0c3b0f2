"""Hand-built small lattices whose conversion outcomes were worked out by hand
from the rules of Sec. 2.2 (interface conversions) and Sec. 2.4 (obstacle
conversions on B(x)).  Each case states the expected cell types and masses."""
import numpy as np
import pytest

from oracle.oracle import GAS, IF, LIQ, OBS, PH_CONVERT, PH_REMAP, Oracle, feq, lattice

C, W, _ = lattice()


def layered(nx, ny, nz, layers, phis, periodic=3):
    """Types per z-layer, uniform f = w (rho = 1, u = 0), fill phi per layer."""
    o = Oracle(nx, ny, nz, 0.8, periodic=periodic)
    t = np.zeros((nz, ny, nx), np.uint8)
    phi = np.zeros((nz, ny, nx))
    for z, (tp, ph) in enumerate(zip(layers, phis)):
        t[z] = tp
        phi[z] = ph
    f = np.zeros((19, nz, ny, nx))
    fl = (t == LIQ) | (t == IF)
    for i in range(19):
        f[i][fl] = W[i]
    o.set_flags(t)
    o.set_f(f)
    o.set_phi(phi)
    o.set_mass(np.where(t == IF, phi, 0.0))
    return o


def test_filled_layer():
    """IF layer at phi 1.05 over liquid, gas above: it becomes liquid, the gas
    layer above becomes interface (f = f_eq of the old liquid/interface
    neighbours' mean rho, u = w here), each filled cell's excess 0.05 is split
    over its 5 new interface neighbours and each of those receives 5 shares."""
    o = layered(4, 4, 6, [LIQ, LIQ, IF, GAS, GAS, GAS], [1, 1, 1.05, 0, 0, 0])
    o.step(1, PH_CONVERT)
    t = o.types()
    assert (t[:3] == LIQ).all() and (t[3] == IF).all() and (t[4:] == GAS).all()
    np.testing.assert_allclose(o.get_mass()[3], 0.05, rtol=1e-13)
    np.testing.assert_allclose(o.get_phi()[3], 0.05, rtol=1e-13)
    np.testing.assert_allclose(o.get_f()[:, 3], np.broadcast_to(W[:, None, None], (19, 4, 4)), rtol=1e-15)
    c = o.last_conversions()
    assert c["filled"] == 16 and c["new_from_gas"] == 16 and c["emptied"] == 0 and c["new_from_liquid"] == 0
    M, led = o.mass_total()
    assert led == 0.0 and M == pytest.approx(2 * 16 + 16 * 1.0 + 16 * 0.05, rel=1e-14)


def test_emptied_layer():
    """IF layer at phi -0.02 under gas: it becomes gas, the liquid layer below
    becomes interface with m = rho = 1 and receives 5 shares of -0.02/5."""
    o = layered(4, 4, 6, [LIQ, LIQ, LIQ, IF, GAS, GAS], [1, 1, 1, -0.02, 0, 0])
    o.step(1, PH_CONVERT)
    t = o.types()
    assert (t[:2] == LIQ).all() and (t[2] == IF).all() and (t[3:] == GAS).all()
    np.testing.assert_allclose(o.get_mass()[2], 0.98, rtol=1e-14)
    np.testing.assert_allclose(o.get_phi()[2], 0.98, rtol=1e-14)
    assert np.abs(o.get_f()[:, 3]).max() == 0.0
    c = o.last_conversions()
    assert c["emptied"] == 16 and c["new_from_liquid"] == 16


def test_filling_wins_checkerboard():
    """A checkerboard of filled (phi 1.05) and emptied (phi -0.05) interface
    cells: every emptied cell touches a filled one, so none empties.  Filled
    cells become liquid and share 0.05 over 9 interface neighbours (4 kept
    in-plane, 5 new above)."""
    o = layered(4, 4, 6, [LIQ, LIQ, IF, GAS, GAS, GAS], [1, 1, 0, 0, 0, 0])
    phi = o.get_phi()
    yy, xx = np.mgrid[0:4, 0:4]
    even = (xx + yy) % 2 == 0
    phi[2] = np.where(even, 1.05, -0.05)
    o.set_phi(phi)
    o.set_mass(np.where(o.types() == IF, phi, 0.0))
    o.step(1, PH_CONVERT)
    t = o.types()
    assert (t[2][even] == LIQ).all() and (t[2][~even] == IF).all()
    assert (t[3] == IF).all() and (t[4:] == GAS).all()
    m = o.get_mass()
    np.testing.assert_allclose(m[2][~even], -0.05 + 4 * 0.05 / 9, rtol=1e-13)
    np.testing.assert_allclose(m[3][even], 0.05 / 9, rtol=1e-13)
    np.testing.assert_allclose(m[3][~even], 4 * 0.05 / 9, rtol=1e-13)
    assert o.liq_gas_contacts() == 0
    c = o.last_conversions()
    assert c["filled"] == 8 and c["emptied"] == 0 and c["new_from_gas"] == 16


def test_excess_without_receivers_goes_to_ledger():
    o = layered(5, 5, 5, [LIQ] * 5, [1] * 5, periodic=0)
    t = o.types()
    t[2, 2, 2] = IF
    o.set_flags(t)
    phi = o.get_phi()
    phi[2, 2, 2] = 1.2
    o.set_phi(phi)
    o.set_mass(np.where(t == IF, phi, 0.0))
    M0, _ = o.mass_total()
    o.step(1, PH_CONVERT)
    assert (o.types() == LIQ).all()
    M1, led = o.mass_total()
    assert led == pytest.approx(-0.2, rel=1e-13)
    assert M1 - led == pytest.approx(M0, rel=1e-15)


def test_remap_in_gas_and_in_liquid():
    """A 2x2x2 body moved by one cell: in gas the uncovered cells become gas
    (no liquid in B(x)); in liquid they become liquid with rho the mean of B
    and f = f_eq(rho, u_w) at the closest surface point (= V for a pure
    translation).  Covered liquid leaves the fluid, refilled liquid enters."""
    V = np.array([0.02, 0.0, 0.01])
    for H, want in [(0.0, GAS), (1e9, LIQ)]:
        o = Oracle(10, 10, 10, 0.8)
        o.init_basin(H)
        o.set_body(0, (1, 1, 1), (5.1, 5.1, 5.1), vel=V)
        o.step(1, PH_REMAP)
        t = o.types()
        assert (t == OBS).sum() == 8 and (t[4:6, 4:6, 4:6] == OBS).all()
        o.set_body(0, (1, 1, 1), (6.1, 5.1, 5.1), vel=V)
        o.step(1, PH_REMAP)
        t = o.types()
        assert (t[4:6, 4:6, 5:7] == OBS).all() and (t == OBS).sum() == 8
        assert (t[4:6, 4:6, 4] == want).all()
        M, led = o.mass_total()
        if want == LIQ:
            f = o.get_f()
            fe = feq(1.0, V)
            for z in (4, 5):
                for y in (4, 5):
                    np.testing.assert_allclose(f[:, z, y, 4], fe, rtol=1e-14)
            assert led == pytest.approx(-8.0, rel=1e-14)
            assert M == pytest.approx(1000 - 8, rel=1e-14)
        else:
            assert led == 0.0 and M == 0.0


def test_remap_across_surface():
    """A 2x4x4 body straddling an interface layer (phi 0.5) moves by one cell
    along x.  In the uncovered column: the liquid-level cell sees liquid and
    interface only -> LIQ; the interface-level cell sees liquid and gas ->
    IF with phi = mean interface fill 0.5; cells above see no liquid -> GAS."""
    o = Oracle(12, 8, 12, 0.8)
    o.init_basin(5.5)
    assert (o.types()[5] == IF).all() and (o.types()[4] == LIQ).all()
    o.set_body(0, (1, 2, 2), (4.0, 4.0, 5.6))
    o.step(1, PH_REMAP)
    o.set_body(0, (1, 2, 2), (5.0, 4.0, 5.6))
    o.step(1, PH_REMAP)
    t = o.types()
    col = t[:, 2:6, 3]
    assert (col[4] == LIQ).all() and (col[5] == IF).all() and (col[6] == GAS).all() and (col[7] == GAS).all()
    np.testing.assert_allclose(o.get_phi()[5, 2:6, 3], 0.5, rtol=1e-14)
    assert (t[4:8, 2:6, 4:6] == OBS).all() and (t == OBS).sum() == 2 * 4 * 4
    assert o.liq_gas_contacts() == 0


def test_remap_fixup_new_liquid_next_to_new_gas():
    """Uncovered cells (3,y,3) see liquid and interface only (rule: LIQ) while
    (3,y,4) above them see no liquid (rule: GAS); a new liquid cell touching a
    new gas cell is turned into interface, with phi the mean fill of the
    interface cells of its B(x): (5 x 0.3 + 2 x 0.7) / 7."""
    nx = ny = nz = 8
    o = Oracle(nx, ny, nz, 0.8)
    t = np.zeros((nz, ny, nx), np.uint8)
    t[:3] = LIQ
    t[3] = IF
    t[4] = IF
    phi = np.zeros((nz, ny, nx))
    phi[:3] = 1
    phi[3] = 0.3
    phi[4] = 0.7
    t[3:5, 3:5, 3:5] = OBS  # old obstacle block x, y, z in {3, 4}; body 0
    phi[3:5, 3:5, 3:5] = 0
    f = np.zeros((19, nz, ny, nx))
    fl = (t == LIQ) | (t == IF)
    for i in range(19):
        f[i][fl] = W[i]
    o.set_flags(t)
    o.set_f(f)
    o.set_phi(phi)
    o.set_mass(np.where(t == IF, phi, 0.0))
    o.set_body(0, (0.5, 1, 1), (4.6, 4.0, 4.0))  # new pose: only the x = 4 column
    o.step(1, PH_REMAP)
    t2 = o.types()
    assert (t2[3:5, 3:5, 4] == OBS).all() and (t2 == OBS).sum() == 4
    assert (t2[3, 3:5, 3] == IF).all()
    assert (t2[4, 3:5, 3] == GAS).all()
    np.testing.assert_allclose(o.get_phi()[3, 3:5, 3], 2.9 / 7, rtol=1e-14)
    assert o.liq_gas_contacts() == 0
