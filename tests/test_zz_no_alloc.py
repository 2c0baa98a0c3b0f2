"""The allocation-free liquid-mass total (lbm_mass_total_noalloc) against the
workspace variant (lbm_mass_total): same kernels and the same fixed summation
order, so the two agree bit for bit.  Two lattices in a row, the second
smaller, so the static scratch is reused with fewer partial sums than the
call before left in it."""
import ctypes as C

import numpy as np
import pytest

from paper_1201_0351_amd import lbm
from paper_1201_0351_amd import workloads as W

pytestmark = pytest.mark.gpu


def _abi_mass(L, fn):
    M, led = C.c_double(), C.c_double()
    rc = getattr(lbm.library(), fn)(L._h, 0, C.byref(M), C.byref(led))
    return rc, M.value, led.value


def _host_mass(L):
    t = L.types()
    rho = L.read(lbm.FIELD_RHO)
    return float(rho[t == W.LIQ].sum() + L.mass()[t == W.IF].sum())


def test_noalloc_mass_total_matches_the_workspace_variant():
    big = lbm.Lattice(dict(W.basin((96, 80, 64), 32.0, 0.6, 1e-5, seed=3, noise_amp=1e-4), max_bodies=1))
    big.set_body(0, W.box((16, 16, 8), (48, 40, 32), 10.0, 0.5))
    big.step(20)
    small = lbm.Lattice(dict(W.basin((40, 24, 20), 10.0, 0.6, 1e-5, seed=5, noise_amp=1e-4, storage="fp16"),
                             max_bodies=1))
    small.step(7)
    for L in (big, small):
        rc0, m0, l0 = _abi_mass(L, "lbm_mass_total")
        rc1, m1, l1 = _abi_mass(L, "lbm_mass_total_noalloc")
        assert rc0 == 0 and rc1 == 0, lbm.library().lbm_last_error()
        assert m1 == m0 and l1 == l0  # bit for bit
        # the value itself, summed on the host from the read fields
        assert abs(m1 - _host_mass(L)) <= 1e-9 * abs(m1)
    # the first lattice again: nothing of the second call is left over
    assert _abi_mass(big, "lbm_mass_total_noalloc")[1] == _abi_mass(big, "lbm_mass_total")[1]
    big.close()
    small.close()


def test_noalloc_mass_total_rejects_more_partials_than_its_scratch_holds():
    # 16390 x 64 x 64 = 67,133,440 cells: 16,390 partial sums of 4096 cells,
    # more than the 16,384 the static scratch holds
    L = lbm.Lattice(dict(W.basin((16390, 64, 64), 32.0, 0.6, 0.0, storage="fp16"), max_bodies=0))
    rc, _, _ = _abi_mass(L, "lbm_mass_total_noalloc")
    assert rc == -1  # LBM_ERR_INVALID
    assert "cells" in lbm.library().lbm_last_error().decode()
    rc, m, _ = _abi_mass(L, "lbm_mass_total")
    assert rc == 0 and m > 0
    L.close()
