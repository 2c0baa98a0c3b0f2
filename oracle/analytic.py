"""Closed-form floating-body results used to pin the oracle (test infrastructure).

Sec. 3.3 of the paper (floating stability):
  * Archimedes: buoyancy F_B = rho g V_immersed.
  * righting moment m_s = F_B * GM * sin(alpha) with, for wall-sided bodies,
    the Scribanti formula B0M = (I/V)(1 + tan(alpha)^2 / 2); for a cuboid
    I/V = b^2 / (12 d), d = rho_s h, and GM = KB0 + B0M - KG.
  * the centre of buoyancy B is the centroid of the immersed cross-section
    (the trapezoid construction of Fig. cubeStability); here the exact
    immersed polygon of the heeled rectangle is clipped and its centroid taken,
    which also covers heel angles past the wall-sided range.
  * stable heel of a floating 2-D cube: 45 deg for rho_s = 1/2 and 26.565 deg
    for rho_s = 1/4 and 3/4.

Conventions: heel alpha is a rotation about +x (the box's long axis) through
the centre of gravity G; the immersed side dips towards -y.  m_s > 0 means
restoring.  The fluid torque about G has x-component T_x = -m_s.
"""
import math

import numpy as np


def hydrostatic_rho(z, H, g, rho_gas=1.0):
    """Linear hydrostatic density (p = rho / 3, dp/dz = -rho g), about rho_G."""
    return rho_gas + 3.0 * g * (H - np.asarray(z, dtype=float))


def archimedes(volume, g, rho=1.0):
    return rho * g * volume


def _rect(b, h, alpha):
    """Corners of the b x h cross-section (width along y, height along z),
    rotated by alpha about +x, relative to G, counter-clockwise in (y, z)."""
    pts = np.array([[-b / 2, -h / 2], [b / 2, -h / 2], [b / 2, h / 2], [-b / 2, h / 2]])
    c, s = math.cos(alpha), math.sin(alpha)
    y = pts[:, 0] * c - pts[:, 1] * s
    z = pts[:, 0] * s + pts[:, 1] * c
    return np.stack([y, z], axis=1)


def _clip_below(poly, zw):
    """Sutherland-Hodgman clip of a convex polygon to the half plane z <= zw."""
    out = []
    n = len(poly)
    for k in range(n):
        p, q = poly[k], poly[(k + 1) % n]
        pin, qin = p[1] <= zw, q[1] <= zw
        if pin:
            out.append(p)
        if pin != qin:
            t = (zw - p[1]) / (q[1] - p[1])
            out.append(p + t * (q - p))
    return np.array(out) if out else np.zeros((0, 2))


def _area_centroid(poly):
    if len(poly) < 3:
        return 0.0, np.zeros(2)
    y, z = poly[:, 0], poly[:, 1]
    y1, z1 = np.roll(y, -1), np.roll(z, -1)
    cr = y * z1 - y1 * z
    A = 0.5 * cr.sum()
    if abs(A) < 1e-300:
        return 0.0, np.zeros(2)
    cy = ((y + y1) * cr).sum() / (6 * A)
    cz = ((z + z1) * cr).sum() / (6 * A)
    return abs(A), np.array([cy, cz])


def immersed_section(b, h, alpha, zw):
    """Area and centroid (y, z relative to G) of the part of the heeled
    rectangle below the water plane z = zw (relative to G)."""
    return _area_centroid(_clip_below(_rect(b, h, alpha), zw))


def waterline_for_density(b, h, alpha, rho_s):
    """Water-plane height (relative to G) at which the immersed area of the
    heeled section equals rho_s * b * h (bisection; area is monotone in zw)."""
    target = rho_s * b * h
    r = 0.5 * math.hypot(b, h)
    lo, hi = -r, r
    for _ in range(64):
        mid = 0.5 * (lo + hi)
        if immersed_section(b, h, alpha, mid)[0] < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def righting_moment_polygon(b, h, l, alpha, g, rho_s=0.5, zw=None, rho=1.0):
    """Exact righting moment m_s = -F_B (B_y - G_y) of a heeled cuboid (long axis
    l along x).  With zw=None the water plane is placed so that the immersed
    volume balances the weight (free floating at fixed heel); pass zw=0 for a
    body held with G on the water plane."""
    if zw is None:
        zw = waterline_for_density(b, h, alpha, rho_s)
    A, c = immersed_section(b, h, alpha, zw)
    FB = rho * g * A * l
    return -FB * c[0]


def scribanti_GM(b, h, alpha, rho_s=0.5):
    d = rho_s * h
    B0M = b * b / (12.0 * d) * (1.0 + 0.5 * math.tan(alpha) ** 2)
    return d / 2.0 + B0M - h / 2.0


def righting_moment_scribanti(b, h, l, alpha, g, rho_s=0.5, rho=1.0):
    FB = rho * g * rho_s * b * h * l
    return FB * scribanti_GM(b, h, alpha, rho_s) * math.sin(alpha)


def wall_sided_limit(b, h, rho_s=0.5):
    """Largest heel (radians) for which neither deck edge nor keel edge crosses
    the water plane, i.e. the range where the Scribanti formula is exact."""
    d = rho_s * h
    return math.atan(min(2 * d, 2 * (h - d)) / b)


def stable_heel_angles(b, h, rho_s, n=180, zw=None):
    """Heel angles in [0, 90) degrees at which a b x h section of density
    rho_s is in stable rotational equilibrium (m_s changes sign from negative
    to positive with increasing alpha).  zw=None: free floating (the water
    plane moves so that buoyancy balances the weight at every heel); a number:
    the centre of gravity is held at that depth below the water plane (the box
    may only turn about its long axis)."""
    al = np.linspace(0.0, math.pi / 2, n + 1)
    ms = np.array([righting_moment_polygon(b, h, 1.0, a, 1.0, rho_s, zw=zw) for a in al])
    out = []
    for k in range(n):
        if ms[k] <= 0.0 < ms[k + 1] or (ms[k] < 0.0 <= ms[k + 1]):
            lo, hi = al[k], al[k + 1]
            for _ in range(50):
                mid = 0.5 * (lo + hi)
                if righting_moment_polygon(b, h, 1.0, mid, 1.0, rho_s, zw=zw) < 0.0:
                    lo = mid
                else:
                    hi = mid
            out.append(math.degrees(0.5 * (lo + hi)))
    return out


def cuboid_inertia(half, density):
    """Mass and principal moments (body frame) of a homogeneous cuboid."""
    hx, hy, hz = half
    M = density * 8.0 * hx * hy * hz
    return M, np.array([M / 3 * (hy * hy + hz * hz), M / 3 * (hx * hx + hz * hz), M / 3 * (hx * hx + hy * hy)])
