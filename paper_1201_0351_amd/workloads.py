"""Seeded synthetic workloads and injected states shared by the tests and the
benchmark.

This module only describes inputs: lattice sizes, physical parameters, body
shapes and poses, and random cell-type / population / fill-level fields.  It
holds none of the method's arithmetic (no equilibrium, no streaming, no
collision, no mapping); both the GPU library and the CPU oracle receive the
same numbers from here and compute everything else themselves.

The workloads stand in for the paper's floating-box and channel experiments
(Sec. 3.2 free-advection channel, Sec. 3.3 heeled boxes in a half-filled
basin); the paper uses no dataset.
"""
import math

import numpy as np

GAS, LIQ, IF, OBS = 0, 1, 2, 3


def heel_quat(deg, axis=0):
    """Unit quaternion (w, x, y, z) for a rotation of `deg` degrees about a
    coordinate axis."""
    a = math.radians(deg)
    q = [math.cos(a / 2), 0.0, 0.0, 0.0]
    q[1 + axis] = math.sin(a / 2)
    return tuple(q)


def basin(n, H, tau, g, rho_gas=1.0, eps=1e-2, periodic=0, seed=0, noise_amp=0.0, u_surface=0.0,
          accel_x=0.0, storage="fp32"):
    """A basin of n = (nx, ny, nz) cells filled to height H (cells below z = H are
    liquid), gravity g along -z."""
    nx, ny, nz = n
    return dict(nx=nx, ny=ny, nz=nz, tau=tau, accel=(accel_x, 0.0, -g), rho_gas=rho_gas, eps=eps,
                fill_height=H, init_ux_surface=u_surface, periodic=periodic, seed=seed,
                noise_amp=noise_amp, storage=storage)


def box(size, pos, heel_deg=0.0, density=0.5, vel=(0, 0, 0), omega=(0, 0, 0), fixed=1):
    """A cuboid body of full size (l, b, h) along (x, y, z) with its centre of
    gravity at `pos`, heeled about +x."""
    return dict(half=tuple(0.5 * s for s in size), pos=tuple(float(p) for p in pos),
                quat=heel_quat(heel_deg), vel=tuple(vel), omega=tuple(omega), density=density, fixed=fixed)


# ---------------------------------------------------------------------------
# The five workloads (sizes and parameters of the floating-box / channel tests)
# ---------------------------------------------------------------------------
def config1():
    """32^3 basin, tau 0.6, g 1e-5, liquid in the lower 16 layers, an 8x8x4
    box of density 0.5 resting at the surface (free), noise +-1e-4, 200 steps."""
    return dict(name="basin32_box8x8x4_free", steps=200, dof=0x3F,
                lattice=basin((32, 32, 32), 16.0, 0.6, 1e-5, seed=1, noise_amp=1e-4),
                bodies=[box((8, 8, 4), (16, 16, 16), 0.0, 0.5, fixed=0)])


def config2(heel=20.0, released=True, storage="fp32"):
    """128^3 basin, tau 0.55, g 5e-6, depth 64, a 32x32x16 box of density 0.5
    with G on the water plane, heeled 20 deg about x; released roll-only or
    held; 5000 steps."""
    return dict(name="basin128_box32x32x16_heel%g_%s" % (heel, "released" if released else "held"),
                steps=5000, dof=0x08,
                lattice=basin((128, 128, 128), 64.0, 0.55, 5e-6, storage=storage),
                bodies=[box((32, 32, 16), (64, 64, 64), heel, 0.5, fixed=0 if released else 1)])


def config3(heel=20.0, storage="fp16"):
    """256x192x192 basin, depth 96, a held 64x64x32 box heeled 10/20/30 deg."""
    return dict(name="basin256x192x192_box64x64x32_heel%g_held" % heel, steps=5000, dof=0,
                lattice=basin((256, 192, 192), 96.0, 0.55, 5e-6, storage=storage),
                bodies=[box((64, 64, 32), (128, 96, 96), heel, 0.5, fixed=1)])


def floating_cubes(dof=0x0C, storage="fp32", heel0=2.86):
    """Rotational equilibrium of floating cubes: a 130x40x40 basin filled to
    z = 20, tau 0.526, g 7.5e-4, three 32x16x16 boxes (the cube of side 16
    extruded along x) of density 0.75, 0.5 and 0.25, released with their
    centre at the upright equilibrium draft and heeled heel0 deg about x;
    they roll (and heave) towards the stable heel of a square section:
    26.565 deg for densities 1/4 and 3/4, 45 deg for 1/2."""
    H, s = 20.0, 16
    bodies = []
    for k, rs in enumerate((0.75, 0.5, 0.25)):
        gz = H + s / 2 - rs * s
        bodies.append(box((2 * s, s, s), (21.0 + 44.0 * k, 20.0, gz), heel0, rs, fixed=0))
    return dict(name="floating_cubes_130x40x40", dof=dof, lattice=basin((130, 40, 40), H, 1.0 / 1.9, 7.5e-4,
                                                                       storage=storage), bodies=bodies)


def splitmix64_stream(seed):
    """Plain SplitMix64 sequence (Steele, Lea & Flood 2014) for drawing
    workload parameters (not used by the method itself)."""
    state = seed & 0xFFFFFFFFFFFFFFFF
    M = 0xFFFFFFFFFFFFFFFF
    while True:
        state = (state + 0x9E3779B97F4A7C15) & M
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        yield z ^ (z >> 31)


def config4(n_inst=48, seed=4, storage="fp32"):
    """Batched heel sweep: uneven lattices 64^3 .. 160x128x128, heel uniform in
    [0, 60] deg, density ratios {0.3, 0.5, 0.7}; box b = ny/4, l = b, h = b/2;
    G placed at the upright equilibrium draft below the surface; held."""
    rnd = splitmix64_stream(seed)

    def U():
        return (next(rnd) >> 11) * (1.0 / 9007199254740992.0)

    insts = []
    for k in range(n_inst):
        nx = 64 + 16 * int(U() * 7)
        ny = nz = 64 + 16 * int(U() * 5)
        heel = 60.0 * U()
        rs = (0.3, 0.5, 0.7)[k % 3]
        b = ny // 4
        l, h = b, b // 2
        H = nz / 2
        Gz = H + h / 2 - rs * h  # upright waterline at draft rs*h
        insts.append(dict(lattice=basin((nx, ny, nz), H, 0.55, 5e-6, storage=storage),
                          bodies=[box((l, b, h), (nx / 2, ny / 2, Gz), heel, rs, fixed=1)]))
    return dict(name="batch48_heel_sweep", steps=3000, instances=insts)


def config5(storage="fp32"):
    """512x256x256 channel, periodic x and y, wall at z = 0 and the top, depth
    128, tau 0.8, g 1e-5, body-force drive a_x = 2 nu u_s / H^2 for a surface
    speed u_s = 0.05 (half-Poiseuille start), a free 48x24x24 box of density 0.6
    advected along x; 20000 steps."""
    tau, H, us = 0.8, 128.0, 0.05
    nu = (tau - 0.5) / 3.0
    ax = 2.0 * nu * us / (H * H)
    return dict(name="channel512x256x256_box48x24x24_free", steps=20000, dof=0x3F,
                lattice=basin((512, 256, 256), H, tau, 1e-5, periodic=3, u_surface=us, accel_x=ax,
                              storage=storage),
                bodies=[box((48, 24, 24), (128, 128, 125.6), 0.0, 0.6, vel=(us, 0, 0), fixed=0)])


def sphere(radius, pos, density=0.5, vel=(0, 0, 0), omega=(0, 0, 0), fixed=1):
    """A spherical body of the given radius centred at `pos`."""
    r = float(radius)
    return dict(half=(r, r, r), pos=tuple(float(p) for p in pos), quat=(1.0, 0.0, 0.0, 0.0), vel=tuple(vel),
                omega=tuple(omega), density=density, fixed=fixed, shape=1)


# The free advection test (Sec. 3.2, Table tab:velocities): relaxation times
# and wall speeds of the paper's sweep.
FREE_ADVECTION_TAUS = (0.62, 0.8, 1.1, 1.7)
FREE_ADVECTION_SPEEDS = (1e-4, 5e-5, 2.5e-5, 1e-5)


def free_advection(tau, u, storage="fp32"):
    """The paper's free advection channel: 60x40x30 cells, periodic along x,
    the long sides moving no-slip walls at u along x, g 1e-5, a planar free
    surface at z = 19.5, and a free sphere of diameter 12 and density 0.5 at
    the centre of the channel (the liquid starts at rest; the walls drive
    it)."""
    return dict(name="free_advection_60x40x30", dof=0x3F,
                lattice=dict(basin((60, 40, 30), 19.5, tau, 1e-5, periodic=1, storage=storage),
                             wall_vel=(float(u), 0.0, 0.0)),
                bodies=[sphere(6.0, (30.0, 20.0, 19.5), density=0.5, fixed=0)])


# ---------------------------------------------------------------------------
# Random injected states for phase-isolated parity tests.  Values are rounded
# to float32 so both sides see identical numbers.
# ---------------------------------------------------------------------------
def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def wavy_surface_types(n, H, amp, seed, periodic=0):
    """Cell types of a wavy liquid surface z = H + amp*sin(...) with a closed
    interface layer: cells below the surface are liquid, above gas, and every
    liquid cell with a gas cell among its 18 lattice neighbours is interface."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    p1, p2 = rng.uniform(0, 2 * np.pi, 2)
    x = np.arange(nx)[None, None, :] + 0.5
    y = np.arange(ny)[None, :, None] + 0.5
    z = np.arange(nz)[:, None, None] + 0.5
    surf = H + amp * np.sin(2 * np.pi * x / max(nx, 2) + p1) * np.cos(2 * np.pi * y / max(ny, 2) + p2)
    t = np.where(z < surf, LIQ, GAS).astype(np.uint8)
    liq = t == LIQ
    touch = np.zeros_like(liq)
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                if abs(dx) + abs(dy) + abs(dz) not in (1, 2):
                    continue
                g = t == GAS
                sh = np.roll(g, (-dz, -dy, -dx), axis=(0, 1, 2))
                # a neighbour across a non-periodic face is a wall, not gas
                if not periodic & 1:
                    if dx == 1:
                        sh[:, :, -1] = False
                    if dx == -1:
                        sh[:, :, 0] = False
                if not periodic & 2:
                    if dy == 1:
                        sh[:, -1, :] = False
                    if dy == -1:
                        sh[:, 0, :] = False
                if not periodic & 4:
                    if dz == 1:
                        sh[-1, :, :] = False
                    if dz == -1:
                        sh[0, :, :] = False
                touch |= sh
    t[liq & touch] = IF
    return t


def droplet(n, radius, centre, liquid_inside=True, axes=3, sub=8):
    """Cell types and fill levels of a liquid sphere in gas (axes=3), or of a
    liquid cylinder along z (axes=2), on a periodic lattice; the complement
    (a gas bubble in liquid) with liquid_inside=False.  The fill of a cell is
    the fraction of sub^3 sample points inside the shape, with the distance
    to the centre taken across the periodic faces.  Cells with fill 1 are
    liquid, fill 0 gas, the rest interface; a gas cell among the 18 lattice
    neighbours of a liquid cell is turned into an interface cell of fill 0,
    so that the interface layer is closed.  Returns (types u8, phi f64),
    both [nz, ny, nx]."""
    nx, ny, nz = n
    s = (np.arange(sub) + 0.5) / sub
    inside = np.zeros((nz, ny, nx))
    dims = (nx, ny, nz)
    for a in s:
        for b in s:
            for c in s:
                d2 = 0.0
                for k, (o, g) in enumerate(zip((a, b, c), dims)):
                    if k >= axes:
                        continue
                    q = np.arange(g) + o - centre[k]
                    q = q - g * np.round(q / g)
                    sh = [1, 1, 1]
                    sh[2 - k] = g
                    d2 = d2 + (q * q).reshape(sh)
                inside += d2 <= radius * radius
    phi = inside / sub ** 3
    if not liquid_inside:
        phi = 1.0 - phi
    t = np.full((nz, ny, nx), IF, np.uint8)
    t[phi >= 1.0] = LIQ
    t[phi <= 0.0] = GAS
    liq = t == LIQ
    near = np.zeros_like(liq)
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                if abs(dx) + abs(dy) + abs(dz) in (1, 2):
                    near |= np.roll(liq, (dz, dy, dx), axis=(0, 1, 2))
    t[(t == GAS) & near] = IF
    phi = np.where(t == LIQ, 1.0, np.where(t == GAS, 0.0, phi))
    return t, phi


def random_state(n, types, seed, fill_lo=0.05, fill_hi=0.95, f_spread=0.1, threshold_frac=0.0, eps=1e-2):
    """Random populations (positive, about 1/19 each), fill levels and masses for
    the given cell types.  Interface fill levels are uniform in
    [fill_lo, fill_hi]; a fraction `threshold_frac` of interface cells is pushed
    past the conversion thresholds (to exactly +-(eps + 0.01) beyond them).
    Gas and obstacle cells get zero populations."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    fluid = (types == LIQ) | (types == IF)
    f = _f32(rng.uniform(1.0 - f_spread, 1.0 + f_spread, size=(19, nz, ny, nx)) / 19.0)
    f[:, ~fluid] = 0.0
    phi = np.zeros((nz, ny, nx))
    phi[types == LIQ] = 1.0
    iface = types == IF
    phi[iface] = rng.uniform(fill_lo, fill_hi, size=int(iface.sum()))
    if threshold_frac > 0:
        pick = iface & (rng.uniform(size=iface.shape) < threshold_frac)
        up = rng.uniform(size=iface.shape) < 0.5
        phi[pick & up] = 1.0 + eps + 0.01 + rng.uniform(0, 0.05, size=int((pick & up).sum()))
        phi[pick & ~up] = -eps - 0.01 - rng.uniform(0, 0.05, size=int((pick & ~up).sum()))
    phi = _f32(phi)
    m = _f32(phi * rng.uniform(0.97, 1.03, size=phi.shape))
    m[~iface] = 0.0
    return f, phi, m
