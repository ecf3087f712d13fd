"""Physics the method must reproduce, at sizes only the GPU path reaches in a test's
time (the GPU path itself is checked element by element against the oracle in
test_gpu_parity.py):

* the Laplace pressure jump 2 sigma / R of a resting 3D droplet (Sec. 2.1: the
  surface-tension force of a diffuse interface of width xi);
* thermocapillary migration in a uniform temperature gradient against the
  Young-Goldstein-Block velocity, at the migration set-up of 128 x 256 x 128 cells
  (unit property ratios; Ma = 1 with each thermal scheme, and Ma = 10);
* the equilibrium shape of a sessile droplet on a wetting wall over the range of
  contact angles of the paper's 3D capture study (45 to 135 degrees).
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_2401_03041_amd import workloads as W
from tests.helpers import gpu_domain

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("radius", [12.0, 16.0])
def test_laplace_pressure_jump_3d(radius):
    """Droplet at rest in a periodic 64^3 box (density ratio 10, sigma = 1e-3,
    xi = 5), 6000 steps in FP64: p_inside - p_outside within 10 % of 2 sigma / R."""
    n, sigma = 64, 1e-3
    c = (n - 1) / 2.0
    cfg = W.make(shape=(n, n, n), precision="fp64", rho_h=1.0, rho_l=0.1, nu_h=0.1, nu_l=0.1, xi=5.0,
                 sigma_ref=sigma, droplets=[(c, c, c, radius)])
    d = gpu_domain(cfg)
    d.step(6000)
    p = d.get_field("p")
    z, y, x = np.meshgrid(*(np.arange(n, dtype=np.float64),) * 3, indexing="ij")
    dist = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2)
    inside = p[dist < radius / 2].mean()
    outside = p[dist > radius + 15.0].mean()
    jump = inside - outside
    ratio = jump / (2 * sigma / radius)
    print(f"R = {radius}: jump {jump:.4e}, 2 sigma / R = {2 * sigma / radius:.4e}, ratio {ratio:.4f}")
    assert abs(ratio - 1.0) < 0.10
    d.close()


@pytest.mark.parametrize("thermal,q", [("lb", 7), ("lb", 15), ("lb", 19), ("lb", 27), ("rk2", 7), ("rk4", 7)])
def test_ygb_migration_velocity(thermal, q):
    """Droplet R = 16 in a channel 128 x 256 x 128 between walls at T = 0 and 1
    (G = 1/256), sigma_T = -1.6e-3, unit ratios, Ma = 1, each thermal scheme.  It
    moves towards the hot wall; its centroid speed over steps 4000-6000 is within
    0.6-1.05 of V_YGB = 2 |sigma_T| G R / (15 mu) (wall confinement R/H = 1/16,
    finite Re and the diffuse interface all slow it)."""
    cfg = W.migration(precision="fp64", thermal=thermal, q_thermal=q)
    R, G, mu = 16.0, 1.0 / cfg["shape"][1], cfg["nu_h"] * cfg["rho_h"]
    v_ygb = 2 * abs(cfg["sigma_t"]) * G * R / (15 * mu)
    d = gpu_domain(cfg)
    d.step(4000)
    m0, c0 = d.reduce()
    d.step(2000)
    m1, c1 = d.reduce()
    v = (c1[1] - c0[1]) / 2000.0
    print(f"{thermal}{q}: centroid speed {v:.4e}, V_YGB {v_ygb:.4e}, ratio {v / v_ygb:.4f}, "
          f"drift x {c1[0] - c0[0]:.2e} z {c1[2] - c0[2]:.2e}, mass change {(m1 - m0) / m0:.2e}")
    assert 0.6 < v / v_ygb < 1.05
    assert abs(c1[0] - c0[0]) < 1e-3 and abs(c1[2] - c0[2]) < 1e-3
    assert abs(m1 - m0) < 1e-9 * m0
    d.close()


def test_ygb_migration_higher_marangoni():
    """Ma = 10 (thermal diffusivity ten times smaller).  Over 6000 steps the
    isotherms have moved by a fraction of a cell (thermal time R^2/kappa is about
    2.7e5 steps), so the droplet still migrates towards the hot wall at close to
    the Ma = 1 speed; the ratio to V_YGB is reported."""
    cfg = W.migration(precision="fp64", marangoni=10.0)
    v_ygb = 2 * abs(cfg["sigma_t"]) * (1.0 / cfg["shape"][1]) * 16.0 / (15 * cfg["nu_h"])
    d = gpu_domain(cfg)
    d.step(4000)
    _, c0 = d.reduce()
    d.step(2000)
    _, c1 = d.reduce()
    ratio = (c1[1] - c0[1]) / 2000.0 / v_ygb
    print(f"Ma = 10: speed / V_YGB = {ratio:.4f}")
    assert 0.5 < ratio < 1.05
    d.close()


def _sphere_angle(phi):
    """Sphere fitted (least squares) to the phi = 1/2 crossings of a cap phi[z, y, x]
    on the wall y = -1/2: contact angle through the heavy phase (degrees) and radius."""
    pts = []
    for axis in range(3):
        a = np.moveaxis(phi, axis, 0)
        lo, hi = a[:-1] - 0.5, a[1:] - 0.5
        k, i, j = np.nonzero(lo * hi < 0)
        t = lo[k, i, j] / (lo[k, i, j] - hi[k, i, j])
        c = np.stack([k + t, i.astype(float), j.astype(float)], axis=1)
        # back to (z, y, x) order
        order = {0: (0, 1, 2), 1: (1, 0, 2), 2: (1, 2, 0)}[axis]
        pts.append(c[:, order])
    P = np.concatenate(pts)[:, ::-1]  # (x, y, z)
    A = np.c_[2 * P, np.ones(len(P))]
    cx, cy, cz, c = np.linalg.lstsq(A, (P ** 2).sum(1), rcond=None)[0]
    R = float(np.sqrt(c + cx * cx + cy * cy + cz * cz))
    return float(np.degrees(np.arccos(-(cy + 0.5) / R))), R


def _sessile_cap(theta, R=16.0):
    """Fitted contact angle after 40000 (R / 16)^2 steps and 5000 (R / 16)^2 more
    (FP64), of a hemisphere of radius R in a (6R, 3R, 6R) box."""
    s = R / 16.0
    n = (int(96 * s), int(48 * s), int(96 * s))
    cfg = W.make(shape=n, periodic_y=False, rho_h=1.0, rho_l=1.0, nu_h=1 / 6, nu_l=1 / 6, mobility=0.1,
                 xi=4.0, sigma_ref=5e-3, contact_angle_bot=theta,
                 droplets=[(n[0] / 2 - 0.3, -0.5, n[2] / 2 + 0.2, R)])
    d = gpu_domain(cfg)
    d.step(int(35000 * s * s))
    a1, _ = _sphere_angle(d.get_field("phi"))
    d.step(int(5000 * s * s))
    a2, _ = _sphere_angle(d.get_field("phi"))
    d.close()
    return a1, a2


@pytest.mark.parametrize("theta", [45.0, 135.0])
def test_sessile_contact_angle_offset_is_not_resolution(theta):
    """The offset of the extreme angles (45 degrees about -2.4, 135 degrees about
    +4) is a property of the wetting condition, not of the cap's resolution:
    a cap of radius 24 (R / xi = 6) lands within one degree of the radius-16
    one, on the same side of theta (measured: 42.61 / 42.42 and 139.89 /
    139.13; at R = 32, 42.36 and 138.75)."""
    _, a16 = _sessile_cap(theta, 16.0)
    _, a24 = _sessile_cap(theta, 24.0)
    print(f"theta {theta}: R 16 -> {a16:.2f}, R 24 -> {a24:.2f}")
    assert abs(a24 - a16) < 1.0
    assert (a16 - theta) * (a24 - theta) > 0 and abs(a24 - theta) > 1.5


@pytest.mark.parametrize("theta,tol", [(45.0, 4.0), (60.0, 2.0), (120.0, 2.5), (135.0, 6.5)])
def test_sessile_droplet_contact_angle(theta, tol):
    """Hemisphere R = 16 on the bottom wall of a 96 x 48 x 96 box (unit ratios,
    xi = 4, sigma = 5e-3) with the wall's contact angle set to theta: after 40000
    steps the cap fitted to the phi = 1/2 surface has stopped moving (under 0.5
    degrees over the last 5000 steps), meets the wall within tol of theta, and the
    volume is that of the start.  Measured: 42.5, 59.2, 121.4 and 140.0 degrees;
    the one-sided wall condition errs most at the extreme angles, and by about
    as much at radius 24 and 32 as at 16
    (test_sessile_contact_angle_offset_is_not_resolution), so the tolerances of
    the extreme angles cover that offset rather than a resolution error."""
    n = (96, 48, 96)
    cfg = W.make(shape=n, periodic_y=False, rho_h=1.0, rho_l=1.0, nu_h=1 / 6, nu_l=1 / 6, mobility=0.1,
                 xi=4.0, sigma_ref=5e-3, contact_angle_bot=theta,
                 droplets=[(n[0] / 2 - 0.3, -0.5, n[2] / 2 + 0.2, 16.0)])
    d = gpu_domain(cfg)
    m0, _ = d.reduce()
    d.step(35000)
    a1, _ = _sphere_angle(d.get_field("phi"))
    d.step(5000)
    a2, R = _sphere_angle(d.get_field("phi"))
    m1, _ = d.reduce()
    print(f"theta {theta}: fitted {a1:.2f} -> {a2:.2f} degrees, R {R:.2f}, mass change {(m1 - m0) / m0:.1e}")
    assert abs(a2 - theta) < tol
    assert abs(a2 - a1) < 0.5
    assert abs(m1 - m0) < 1e-9 * m0
    d.close()
