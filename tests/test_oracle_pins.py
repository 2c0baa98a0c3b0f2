"""Pins of oracle parts that the physics tests cannot tell apart from a
plausible mistake: the interface-interface weight of the mass exchange, the
rotational part of the moving-wall velocity and the lever of the torque, the
wall velocity of refilled cells under rotation, and the initialisation of new
interface cells from gas.  Each expected value is derived by hand (or by a
brute-force sum written here) from the paper's definitions, not by calling
the oracle's own arithmetic."""
import numpy as np
import pytest

from oracle.oracle import Oracle, PH_CONVERT, PH_REMAP, PH_SWEEP, lattice

C, WTS, OPP = lattice()
GAS, LIQ, IF, OBS = 0, 1, 2, 3
# link indices of the six axis directions (Fig. d3q19 caption order)
W_, E_ = 1, 2


def test_mass_exchange_weights_and_orientation():
    """Sec. 2.2, the mass-exchange cases: an interface cell x exchanges
    f_ibar(x + c_i) - f_i(x) with a liquid neighbour and (phi_x + phi_y)/2
    times that with an interface neighbour y; walls exchange nothing.

    A 3 x 1 x 1 lattice (walls all round): cell 0 liquid, cells 1 and 2
    interface with phi 0.2 and 0.6.  The only links that reach a fluid cell
    are E/W along x.  With every population at its rest weight except four,
      dm_1 = [f_E(0) - f_W(1)] + (0.2 + 0.6)/2 [f_W(2) - f_E(1)]
           = (0.010 + 0.002) + 0.4 (0.004 - 0.001) = 0.0132
      dm_2 = (0.2 + 0.6)/2 [f_E(1) - f_W(2)]                 = -0.0012.
    A weight of 1 gives 0.015, a dropped 1/2 gives 0.0144, phi_y alone
    0.0138, phi_x alone 0.0126, the reversed orientation -0.0132."""
    o = Oracle(3, 1, 1, 0.8, accel=(0, 0, 0))
    t = np.array([LIQ, IF, IF], np.uint8).reshape(1, 1, 3)
    f = np.zeros((19, 1, 1, 3))
    for i in range(19):
        f[i] = WTS[i]
    f[E_, 0, 0, 0] += 0.010
    f[W_, 0, 0, 1] -= 0.002
    f[W_, 0, 0, 2] += 0.004
    f[E_, 0, 0, 1] += 0.001
    phi = np.array([1.0, 0.2, 0.6]).reshape(1, 1, 3)
    m = np.array([0.0, 0.21, 0.59]).reshape(1, 1, 3)
    o.set_flags(t)
    o.set_f(f)
    o.set_phi(phi)
    o.set_mass(m)
    o.step(1, PH_SWEEP)
    dm = o.get_mass()[0, 0] - m[0, 0]
    assert dm[1] == pytest.approx(0.0132, abs=1e-15)
    assert dm[2] == pytest.approx(-0.0012, abs=1e-15)


def _s2(n):
    """Sum of squared offsets of n cell centres from their middle: n(n^2 - 1)/12."""
    return n * (n * n - 1) / 12.0


def _spin_moments(a, b, h):
    """Diagonal of M = sum over the links from fluid cells into an axis-aligned
    a x b x h obstacle block of w_i (s x c_i)(s x c_i)^T, s the obstacle
    cell's offset from the block centre, derived by pairing the links of each
    face, edge and direction (the z entry; x and y by permuting the axes):
      axis links +-x, +-y (w 1/18):  2h S2(b) + 2h S2(a)
      in-plane diagonals (w 1/36):   4h [b A^2 + S2(b) + a B^2 + S2(a) - (A - B)^2]
      x-z and y-z diagonals (w 1/36): 4 (h + a - 1) S2(b) + 4 (h + b - 1) S2(a)
    with A = (a - 1)/2, B = (b - 1)/2 the offsets of the face cells."""
    def mzz(a, b, h):
        A, B = (a - 1) / 2.0, (b - 1) / 2.0
        axis = (2 * h * _s2(b) + 2 * h * _s2(a)) / 18.0
        inplane = 4 * h * (b * A * A + _s2(b) + a * B * B + _s2(a) - (A - B) ** 2) / 36.0
        outplane = (4 * (h + a - 1) * _s2(b) + 4 * (h + b - 1) * _s2(a)) / 36.0
        return axis + inplane + outplane
    return np.array([mzz(b, h, a), mzz(h, a, b), mzz(a, b, h)])


def _drag_moments(a, b, h):
    """Diagonal of K = sum over the same links of w_i c_i c_i^T, by pairing:
      axis links (w 1/18):             2 b h
      in-plane diagonals (w 1/36):     4 (b h + a h - h)   (x or y face)
      x-z diagonals (w 1/36):          4 (b h + a b - b)   (x or z face)
    (the x entry; y and z by permuting the axes)."""
    def kxx(a, b, h):
        return 2 * b * h / 18.0 + 4 * (b * h + a * h - h) / 36.0 + 4 * (b * h + a * b - b) / 36.0
    return np.array([kxx(a, b, h), kxx(b, a, h), kxx(h, b, a)])


def _link_sums_brute(a, b, h):
    """M and K by enumerating every obstacle cell and link."""
    s_all = [np.array([x - (a - 1) / 2, y - (b - 1) / 2, z - (h - 1) / 2])
             for z in range(h) for y in range(b) for x in range(a)]
    half = np.array([a, b, h]) / 2.0
    M, K = np.zeros((3, 3)), np.zeros((3, 3))
    for s in s_all:
        for i in range(1, 19):
            if np.all(np.abs(s + C[i]) < half):
                continue  # the neighbour is an obstacle cell too
            v = np.cross(s, C[i])
            M += WTS[i] * np.outer(v, v)
            K += WTS[i] * np.outer(C[i], C[i])
    return M, K


def test_link_sum_closed_forms_match_brute_force():
    for dims in [(4, 6, 8), (5, 3, 7)]:
        M, K = _link_sums_brute(*dims)
        assert np.allclose(np.diag(M), _spin_moments(*dims), rtol=1e-13)
        assert np.allclose(np.diag(K), _drag_moments(*dims), rtol=1e-13)
        assert np.abs(M - np.diag(np.diag(M))).max() < 1e-12
        assert np.abs(K - np.diag(np.diag(K))).max() < 1e-12


def test_spinning_box_torque_and_fluid_momentum():
    """Sec. 2.3, Eqs. noslip and momentumexchange with u_w = V + Omega x
    (x_c - c_i/2 - o), and Eqs. netforce / torque, on a held box moving at V
    and spinning at Omega in liquid of uniform density rho at rest (no
    gravity), one step.

    At rest f_ibar = w_i rho, whose terms cancel over the closed surface; the
    velocity term of a link is 6 w_i rho c_i (c_i.u_w), and
    c_i.(Omega x (x_c - c_i/2 - o)) = Omega.(s x c_i) with s the obstacle
    cell's offset (x_c - o = s + c_i).  The parts odd in (s, c_i) cancel over
    the symmetric box, leaving F = -6 rho K V and T = -6 rho M Omega with the
    link sums K, M of _drag_moments / _spin_moments: drag opposes the motion
    and the torque opposes the spin.  A sign error in Omega x r, a lever about
    another point (T would pick up (o - o') x F) or a missing rho fails this.
    The fluid gains exactly the momentum and angular momentum about o that
    the body loses (Sec. 2.3: the momentum transferred to the wall equals the
    change of the fluid's momentum)."""
    a, b, h = 4, 6, 8
    rho = 1.05
    nx, ny, nz = 18, 20, 22
    o_ = np.array([8.0, 9.0, 12.0])  # face planes on cell faces: no mapping ties
    Om = np.array([0.004, -0.003, 0.006])
    V = np.array([0.002, 0.005, -0.003])
    o = Oracle(nx, ny, nz, 0.8, accel=(0, 0, 0), rho_gas=rho)
    o.init_basin(1e9)  # all liquid at rho_G, walls all round
    o.set_body(0, (a / 2, b / 2, h / 2), tuple(o_), vel=tuple(V), omega=tuple(Om), fixed=1)
    o.step(1, PH_REMAP)
    t = o.types()
    fluid = t != OBS
    zc, yc, xc = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    r = np.stack([xc - o_[0], yc - o_[1], zc - o_[2]])

    def momenta(f):
        j = np.einsum("ia,izyx->azyx", C.astype(float), f) * fluid
        return j.reshape(3, -1).sum(1), np.cross(r, j, axis=0).reshape(3, -1).sum(1)

    P0, L0 = momenta(o.get_f())
    o.step(1, PH_SWEEP)
    F, T = o.body_forces(0)
    P1, L1 = momenta(o.get_f())
    assert np.allclose(T, -6.0 * rho * _spin_moments(a, b, h) * Om, rtol=1e-10, atol=0)
    assert np.allclose(F, -6.0 * rho * _drag_moments(a, b, h) * V, rtol=1e-10, atol=0)
    assert np.allclose(P1 - P0, -F, atol=1e-13)
    assert np.allclose(L1 - L0, -T, rtol=1e-9, atol=1e-13)


def test_refilled_cells_take_the_velocity_of_the_closest_surface_point():
    """Sec. 2.4: an obstacle cell uncovered by the body's motion, with only
    liquid around it, becomes liquid with f = f_eq(rho_bar, u_w(p*)), p* the
    point of the body surface closest to its centre and u_w = V + Omega x
    (p* - o).  The box [6, 10]^3 moves to centre o = (7.4, 7.4, 8) (spanning
    [5.4, 9.4] x [5.4, 9.4] x [6, 10]) with V = (-0.006, -0.003, 0) and
    Omega = (0.004, 0, 0.01).  By hand, p* - o and u_w are
      cell (9, 9, 8): p* = (9.4, 9.4, 8.5), d = (2.0, 2.0, 0.5),
                      Omega x d = (-0.02, 0.018, 0.008)
      cell (9, 7, 8): p* = (9.4, 7.5, 8.5), d = (2.0, 0.1, 0.5),
                      Omega x d = (-0.001, 0.018, 0.0004)
      cell (7, 9, 8): p* = (7.5, 9.4, 8.5), d = (0.1, 2.0, 0.5),
                      Omega x d = (-0.02, -0.001, 0.008)
    and the equilibrium's moments return rho_bar = 1 and u_w exactly."""
    o = Oracle(16, 16, 16, 0.8, accel=(0, 0, 0))
    o.init_basin(1e9)
    o.set_body(0, (2, 2, 2), (8.0, 8.0, 8.0), fixed=1)
    o.step(1, PH_REMAP)
    V = np.array([-0.006, -0.003, 0.0])
    Om = (0.004, 0.0, 0.01)
    o.set_body(0, (2, 2, 2), (7.4, 7.4, 8.0), vel=tuple(V), omega=Om, fixed=1)
    o.step(1, PH_REMAP)
    f = o.get_f()
    t = o.types()
    for (x, y, z), w in [((9, 9, 8), (-0.02, 0.018, 0.008)), ((9, 7, 8), (-0.001, 0.018, 0.0004)),
                         ((7, 9, 8), (-0.02, -0.001, 0.008))]:
        assert t[z, y, x] == LIQ
        fc = f[:, z, y, x]
        rho = fc.sum()
        u = C.T.astype(float) @ fc / rho
        assert rho == pytest.approx(1.0, abs=1e-14)
        assert np.allclose(u, V + np.array(w), atol=1e-15)


def test_new_interface_cell_from_gas_takes_mean_density_and_velocity():
    """Sec. 2.2 conversions (the reading of this implementation): a gas cell
    next to a filled interface cell becomes interface with
    f = f_eq(mean rho, mean u) over its neighbours that were liquid or
    interface and are not emptying (m = 0).  The neighbours here carry
    different densities and velocities, so the plain mean of u differs from
    the density-weighted one; the emptying neighbour is left out."""
    n = 5
    o = Oracle(n, n, n, 0.8, accel=(0, 0, 0))
    t = np.zeros((n, n, n), np.uint8)
    rng = np.random.default_rng(7)
    f = np.zeros((19, n, n, n))
    phi = np.zeros((n, n, n))
    m = np.zeros((n, n, n))
    g = (2, 2, 2)  # the gas cell, (x, y, z)
    cells = {(1, 2, 2): (IF, 1.2),   # filled (phi >= 1 + eps): g becomes interface
             (2, 1, 2): (LIQ, 1.0),
             (2, 2, 1): (LIQ, 1.0),
             (2, 3, 3): (IF, 0.5),
             (2, 4, 4): (LIQ, 1.0),  # liquid next to (2, 3, 3) only: not stranded
             (3, 3, 2): (IF, -0.3)}  # emptied, not next to the filled cell
    for (x, y, z), (ty, ph) in cells.items():
        t[z, y, x] = ty
        f[:, z, y, x] = WTS * rng.uniform(0.9, 1.1) * (1.0 + 0.3 * rng.uniform(-1, 1, 19))
        phi[z, y, x] = ph
        m[z, y, x] = ph * f[:, z, y, x].sum() if ty == IF else 0.0
    o.set_flags(t)
    o.set_f(f)
    o.set_phi(phi)
    o.set_mass(m)
    o.step(1, PH_CONVERT)
    used = [(1, 2, 2), (2, 1, 2), (2, 2, 1), (2, 3, 3)]
    rhos = np.array([f[:, z, y, x].sum() for (x, y, z) in used])
    us = np.array([C.T.astype(float) @ f[:, z, y, x] / f[:, z, y, x].sum() for (x, y, z) in used])
    rho_bar, u_bar = rhos.mean(), us.mean(axis=0)
    u_weighted = (rhos[:, None] * us).sum(0) / rhos.sum()
    assert np.abs(u_bar - u_weighted).max() > 1e-3  # the two readings are told apart
    x, y, z = g
    assert o.types()[z, y, x] == IF
    fg = o.get_f()[:, z, y, x]
    assert fg.sum() == pytest.approx(rho_bar, abs=1e-14)
    assert np.allclose(C.T.astype(float) @ fg / fg.sum(), u_bar, atol=1e-14)
    # the emptied cell turned gas and its liquid neighbours (none here) stay
    assert o.types()[2, 3, 3] == GAS


def _isolated_cell(rule):
    """One interface cell at rest in gas (all 18 neighbours gas, no gravity),
    f_0 = 1.2 and the other populations 0.075 w_i (rho = 1.25, u = 0)."""
    n = 5
    o = Oracle(n, n, n, 0.526, accel=(0, 0, 0))
    o.set_stranded_rule(rule)
    t = np.zeros((n, n, n), np.uint8)
    t[2, 2, 2] = IF
    f = np.zeros((19, n, n, n))
    f[:, 2, 2, 2] = 0.075 * WTS
    f[0, 2, 2, 2] = 1.2
    phi = np.zeros((n, n, n))
    phi[2, 2, 2] = 0.02
    o.set_flags(t)
    o.set_f(f)
    o.set_phi(phi)
    o.set_mass(phi * 1.25)
    return o


def test_stranded_interface_cell_empties_before_its_density_turns_negative():
    """Interface cells with no liquid neighbour (the reading taken for a case
    the paper leaves open).  An isolated interface cell at rest rebuilds all
    18 links from the gas (Eq. reconstruct with rho_G = 1, u = 0):
      rho' = f_0 + sum_i (2 w_i - f_ibar) = 2 f_0 - rho + 4/3,
    and BGK leaves f_0 <- (1 - omega) f_0 + omega rho'/3 (f_eq,0 = rho/3).
    With f_0 = 1.2, rho = 1.25, omega = 1/0.526:
      step 1: rho_1 = 2.4833..., f_0 = 0.49235...
      step 2: rho_2 = 2 (0.49235...) - 2.4833... + 4/3 = -0.1653...
    Without a rule the cell stays interface (phi = 0.025 / 2.48 is inside the
    thresholds) and the second step's sweep computes a negative density.  With the
    stranded rule it is emptied at the end of step 1: it turns gas, its mass
    m = 0.025 leaves the fluid to the ledger (no interface neighbour
    receives it), and nothing negative is ever computed."""
    om = 1.0 / 0.526
    rho1 = 2 * 1.2 - 1.25 + 4.0 / 3.0
    f01 = (1 - om) * 1.2 + om * rho1 / 3.0
    rho2 = 2 * f01 - rho1 + 4.0 / 3.0
    assert rho2 < -0.16
    o = _isolated_cell(False)
    o.step(1)
    assert o.types()[2, 2, 2] == IF
    assert o.get_f()[:, 2, 2, 2].sum() == pytest.approx(rho1, abs=1e-12)
    assert o.get_f()[0, 2, 2, 2] == pytest.approx(f01, abs=1e-12)
    o.step(1, PH_SWEEP)  # the second step's sweep (its conversions would empty the cell: phi < -eps)
    assert o.get_f()[:, 2, 2, 2].sum() == pytest.approx(rho2, abs=1e-12)
    o = _isolated_cell(True)
    o.step(1)
    assert o.types()[2, 2, 2] == GAS
    M, led = o.mass_total()
    assert M == 0.0 and led == pytest.approx(-0.025, abs=1e-15)
    assert o.last_conversions()["emptied"] == 1
    o.step(5)
    assert (o.types() == GAS).all()


def test_stranded_means_cut_off_from_the_liquid():
    """The stranded rule reaches two cells: a 4 x 4 periodic column with
    liquid at z = 0..3, interface at z = 4 (fill 0.8) and z = 5 (fill 0.2)
    over it, gas at z = 6, 7, and a detached interface film at z = 8, 9
    (fill 0.5).  The outer interface layer z = 5 has no liquid neighbour but
    its interface neighbours below have one, so it stays; the film at
    z = 8, 9 reaches no liquid and empties.  Fill levels are inside the
    thresholds, so nothing else converts."""
    n = 4
    o = Oracle(n, n, 12, 0.8, accel=(0, 0, 0), periodic=3)
    t = np.zeros((12, n, n), np.uint8)
    t[:4] = LIQ
    t[4:6] = IF
    t[8:10] = IF
    phi = np.zeros((12, n, n))
    phi[:4] = 1.0
    phi[4], phi[5], phi[8:10] = 0.8, 0.2, 0.5
    f = np.zeros((19, 12, n, n))
    for i in range(19):
        f[i][t > 0] = WTS[i]
    o.set_flags(t)
    o.set_f(f)
    o.set_phi(phi)
    o.set_mass(np.where(t == IF, phi, 0.0))
    o.step(1, PH_CONVERT)
    tt = o.types()
    assert (tt[4:6] == IF).all() and (tt[:4] == LIQ).all()
    assert (tt[8:10] == GAS).all()
    assert o.last_conversions() == dict(filled=0, emptied=32, new_from_gas=0, new_from_liquid=0)
    M, led = o.mass_total()
    assert led == pytest.approx(-16.0, abs=1e-12)  # the film's mass 32 x 0.5 has no receiver
