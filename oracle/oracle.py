"""ctypes wrapper around the FP64 CPU oracle (``lgs_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg.  It shares nothing with the GPU library.

Field layouts match the library's host-side field export so tests can compare
arrays directly: populations ``[19, nz, ny, nx]`` (D3Q19 in the order of the
paper's Fig. d3q19 caption), scalars ``[nz, ny, nx]``, flags one byte per cell
(bits 0-1 type 0 gas / 1 liquid / 2 interface / 3 obstacle, bits 2-5 body).
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None
Q = 19
GAS, LIQ, IF, OBS = 0, 1, 2, 3
PH_REMAP, PH_SWEEP, PH_CONVERT, PH_ALL = 1, 2, 4, 7

_dp = C.POINTER(C.c_double)
_u8p = C.POINTER(C.c_uint8)


def _arr(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = C.CDLL(path)
        L.ob_create.restype = C.c_void_p
        L.ob_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, _dp, C.c_double, C.c_double,
                                C.c_int, C.c_int]
        L.ob_destroy.argtypes = [C.c_void_p]
        L.ob_set_threads.argtypes = [C.c_void_p, C.c_int]
        L.ob_set_stranded_rule.argtypes = [C.c_void_p, C.c_int]
        L.ob_init_basin.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_uint64, C.c_double]
        L.ob_set_body.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp, _dp, _dp, C.c_double, C.c_int]
        L.ob_set_body_shape.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.ob_set_wall_velocity.argtypes = [C.c_void_p, _dp]
        L.ob_set_surface_tension.argtypes = [C.c_void_p, C.c_double]
        L.ob_curvature.argtypes = [C.c_void_p, _dp]
        L.ob_get_body.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp, _dp]
        L.ob_step.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.ob_body_forces.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
        L.ob_mass_total.restype = C.c_double
        L.ob_mass_total.argtypes = [C.c_void_p, _dp]
        L.ob_liq_gas_contacts.restype = C.c_long
        L.ob_liq_gas_contacts.argtypes = [C.c_void_p]
        L.ob_last_conversions.argtypes = [C.c_void_p, C.POINTER(C.c_long)]
        L.ob_step_coupled.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int)]
        L.ob_step_coupled.restype = C.c_int
        for nm in ("ob_get_f", "ob_set_f", "ob_get_mass", "ob_set_mass", "ob_get_phi", "ob_set_phi"):
            getattr(L, nm).argtypes = [C.c_void_p, _dp]
        L.ob_get_flags.argtypes = [C.c_void_p, _u8p]
        L.ob_set_flags.argtypes = [C.c_void_p, _u8p]
        L.ob_set_ledger.argtypes = [C.c_void_p, C.c_double]
        L.ob_mark_mapped.argtypes = [C.c_void_p]
        L.ob_lattice.argtypes = [C.POINTER(C.c_int), _dp, C.POINTER(C.c_int)]
        L.ob_feq.argtypes = [C.c_double, _dp, _dp]
        L.ob_force.argtypes = [C.c_double, _dp, _dp, _dp]
        L.ob_integrate_body.restype = C.c_int
        L.ob_integrate_body.argtypes = [_dp, _dp, _dp, _dp, _dp, C.c_double, _dp, _dp, _dp, C.c_int,
                                        _dp, _dp, _dp, _dp, C.c_int]
        _lib = L
    return _lib


def lattice():
    """(c [19,3] int, w [19], opp [19]) as the oracle defines them."""
    c = (C.c_int * (Q * 3))()
    w = np.zeros(Q)
    o = (C.c_int * Q)()
    lib().ob_lattice(c, w.ctypes.data_as(_dp), o)
    return np.array(list(c), dtype=np.int64).reshape(Q, 3), w, np.array(list(o))


def feq(rho, u):
    out = np.zeros(Q)
    u, up = _arr(u)
    lib().ob_feq(float(rho), up, out.ctypes.data_as(_dp))
    return out


def force_term(rho, u, a):
    out = np.zeros(Q)
    u, up = _arr(u)
    a, ap = _arr(a)
    lib().ob_force(float(rho), up, ap, out.ctypes.data_as(_dp))
    return out


CUBOID, SPHERE = 0, 1


def integrate_body(half, pos, quat, vel, omega, density, F, T, accel, dof_mask, shape=CUBOID):
    outs = [np.zeros(3), np.zeros(4), np.zeros(3), np.zeros(3)]
    args = [_arr(v) for v in (half, pos, quat, vel, omega)]
    fa = [_arr(v) for v in (F, T, accel)]
    rc = lib().ob_integrate_body(args[0][1], args[1][1], args[2][1], args[3][1], args[4][1], float(density),
                                 fa[0][1], fa[1][1], fa[2][1], int(dof_mask),
                                 *[o.ctypes.data_as(_dp) for o in outs], int(shape))
    if rc != 0:
        raise ValueError("integrate_body: invalid body")
    return dict(pos=outs[0], quat=outs[1], vel=outs[2], omega=outs[3])


class Oracle:
    """One lattice instance of the FP64 reference."""

    def __init__(self, nx, ny, nz, tau, accel=(0.0, 0.0, 0.0), rho_gas=1.0, eps=1e-2, periodic=0,
                 recon_mode=0, threads=None):
        a, ap = _arr(accel)
        self.shape = (nz, ny, nx)
        self.nx, self.ny, self.nz = nx, ny, nz
        self.periodic = periodic
        self._h = lib().ob_create(nx, ny, nz, float(tau), ap, float(rho_gas), float(eps), int(periodic),
                                  int(recon_mode))
        if not self._h:
            raise MemoryError("oracle allocation failed")
        if threads is None:
            threads = int(os.environ.get("ORACLE_THREADS", "1"))
        self.threads = max(1, int(threads))
        lib().ob_set_threads(self._h, self.threads)

    def close(self):
        if self._h:
            lib().ob_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def ncells(self):
        return self.nx * self.ny * self.nz

    def init_basin(self, fill_height, u_surface=0.0, seed=0, noise_amp=0.0):
        lib().ob_init_basin(self._h, float(fill_height), float(u_surface), C.c_uint64(int(seed)),
                            float(noise_amp))

    def set_body(self, k, half, pos, quat=(1.0, 0.0, 0.0, 0.0), vel=(0, 0, 0), omega=(0, 0, 0),
                 density=1.0, fixed=1, shape=None):
        """Pose and motion of body k; `shape` (CUBOID, or SPHERE of radius
        half[0]) is kept by later calls that leave it None."""
        arrs = [_arr(v) for v in (half, pos, quat, vel, omega)]
        rc = lib().ob_set_body(self._h, int(k), *[p for _, p in arrs], float(density), int(fixed))
        if rc != 0:
            raise ValueError("bad body index")
        if shape is not None and lib().ob_set_body_shape(self._h, int(k), int(shape)) != 0:
            raise ValueError("bad body shape")

    def set_stranded_rule(self, on):
        """Interface cells with no liquid neighbour empty at the conversions
        (on by default); off keeps only the fill-level thresholds."""
        lib().ob_set_stranded_rule(self._h, int(bool(on)))

    def set_wall_velocity(self, u):
        """Velocity of the non-periodic faces (moving no-slip walls)."""
        a, p = _arr(u)
        lib().ob_set_wall_velocity(self._h, p)

    def set_surface_tension(self, sigma):
        """Surface tension: interface cells rebuild with rho_G + 2 sigma kappa / cs^2."""
        lib().ob_set_surface_tension(self._h, float(sigma))

    def curvature(self):
        """Mean curvature kappa of every interface cell, [nz, ny, nx] (0 elsewhere)."""
        out = np.zeros(self.shape)
        lib().ob_curvature(self._h, out.ctypes.data_as(_dp))
        return out

    def get_body(self, k):
        outs = [np.zeros(3), np.zeros(4), np.zeros(3), np.zeros(3)]
        rc = lib().ob_get_body(self._h, int(k), *[o.ctypes.data_as(_dp) for o in outs])
        if rc != 0:
            raise ValueError("no such body")
        return dict(pos=outs[0], quat=outs[1], vel=outs[2], omega=outs[3])

    def step(self, n=1, phases=PH_ALL):
        lib().ob_step(self._h, int(n), int(phases))

    def step_coupled(self, n, dof_masks):
        """n full steps; bodies with a non-zero DOF mask are advanced after
        every step by the host update fed with the mean of the current and the
        previous step's force and torque."""
        m = (C.c_int * 16)(*([int(v) for v in dof_masks] + [0] * (16 - len(dof_masks))))
        if lib().ob_step_coupled(self._h, int(n), m) != 0:
            raise ValueError("step_coupled: invalid body")

    def body_forces(self, k=0):
        F, T = np.zeros(3), np.zeros(3)
        lib().ob_body_forces(self._h, int(k), F.ctypes.data_as(_dp), T.ctypes.data_as(_dp))
        return F, T

    def mass_total(self):
        led = C.c_double(0.0)
        M = lib().ob_mass_total(self._h, C.byref(led))
        return M, led.value

    def liq_gas_contacts(self):
        return int(lib().ob_liq_gas_contacts(self._h))

    def last_conversions(self):
        out = (C.c_long * 4)()
        lib().ob_last_conversions(self._h, out)
        return dict(filled=out[0], emptied=out[1], new_from_gas=out[2], new_from_liquid=out[3])

    # ---- fields -----------------------------------------------------------
    def get_f(self):
        out = np.zeros((Q,) + self.shape)
        lib().ob_get_f(self._h, out.ctypes.data_as(_dp))
        return out

    def set_f(self, f):
        f, p = _arr(f)
        assert f.size == Q * self.ncells
        lib().ob_set_f(self._h, p)

    def get_mass(self):
        out = np.zeros(self.shape)
        lib().ob_get_mass(self._h, out.ctypes.data_as(_dp))
        return out

    def set_mass(self, m):
        m, p = _arr(m)
        assert m.size == self.ncells
        lib().ob_set_mass(self._h, p)

    def get_phi(self):
        out = np.zeros(self.shape)
        lib().ob_get_phi(self._h, out.ctypes.data_as(_dp))
        return out

    def set_phi(self, v):
        v, p = _arr(v)
        assert v.size == self.ncells
        lib().ob_set_phi(self._h, p)

    def get_flags(self):
        out = np.zeros(self.shape, dtype=np.uint8)
        lib().ob_get_flags(self._h, out.ctypes.data_as(_u8p))
        return out

    def set_flags(self, fl):
        fl = np.ascontiguousarray(fl, dtype=np.uint8)
        assert fl.size == self.ncells
        lib().ob_set_flags(self._h, fl.ctypes.data_as(_u8p))

    def set_ledger(self, v):
        lib().ob_set_ledger(self._h, float(v))

    def mark_mapped(self):
        lib().ob_mark_mapped(self._h)

    def types(self):
        return self.get_flags() & 3

    def rho(self):
        return self.get_f().sum(axis=0)
