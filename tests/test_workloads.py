"""Host-side input generators and the benchmark's sample selection (no GPU)."""
from __future__ import annotations

import itertools

import numpy as np
import pytest

from paper_2401_03041_amd import workloads as W


def _periodic_gap(a, b, n):
    d = np.asarray(a[:3]) - np.asarray(b[:3])
    d -= n * np.round(d / n)
    return float(np.linalg.norm(d))


def test_droplet_block_is_seeded_and_non_overlapping():
    """64 droplets with radii in [10, 24], centres in the box, every pair apart by
    at least r_i + r_j + 2 xi across the periodic boundaries; the same seed gives
    the same block, another seed a different one."""
    cfg = W.droplet_block(n=512)
    drops = cfg["droplets"]
    assert len(drops) == 64
    for (x, y, z, r) in drops:
        assert 10.0 <= r <= 24.0
        assert all(0.0 <= c < 512.0 for c in (x, y, z))
    for a, b in itertools.combinations(drops, 2):
        assert _periodic_gap(a, b, 512.0) >= a[3] + b[3] + 2 * cfg["xi"]
    assert W.droplet_block(n=512)["droplets"] == drops
    assert W.droplet_block(n=512, seed=1)["droplets"] != drops
    assert cfg["rho_h"] / cfg["rho_l"] == pytest.approx(100.0)


def test_droplet_block_temperature_is_periodic_and_bounded():
    """Eight Gaussians of amplitude 0.5 with minimum-image distances: the field is
    periodic (a window straddling the seam equals the wrapped one) and within
    [0, 4]."""
    cfg = W.droplet_block(n=64, ndrop=2, radius=(6.0, 8.0), sigma_range=(6.0, 16.0))
    T = W.temperature(cfg)
    assert T.min() >= 0.0 and T.max() <= 8 * 0.5
    shifted = W.temperature(cfg, origin=(60, 0, 0), dims=(8, 64, 64))
    assert np.allclose(shifted[:, :, :4], T[:, :, 60:64])
    assert np.allclose(shifted[:, :, 4:], T[:, :, 0:4])


def test_capture_parameters_follow_the_dimensionless_groups():
    """The capture channel reproduces Ma = 0.01, Ca = 0.16, Re = 0.08 and
    sigma_T / sigma_ref = 0.04 with U = gamma R, gamma = lid speed / height."""
    cfg = W.capture()
    nx, ny, nz = cfg["shape"]
    R = cfg["droplets"][0][3]
    U = 0.02 / ny * R
    nu = cfg["nu_h"]
    assert U * R / nu == pytest.approx(0.08)
    assert U * nu / cfg["sigma_ref"] == pytest.approx(0.16)
    assert U * R / cfg["kappa_h"] == pytest.approx(0.01)
    assert cfg["sigma_t"] / cfg["sigma_ref"] == pytest.approx(0.04)
    assert cfg["heat_sources"][0][0] == 0.8 and cfg["u_wall_top"][0] == 0.02


def test_migration_kappa_from_marangoni_number():
    """kappa = U R / Ma with U = |sigma_T| G R / mu (Young-Goldstein-Block scale)."""
    for ma in (1.0, 10.0):
        cfg = W.migration(marangoni=ma)
        G = 1.0 / cfg["shape"][1]
        U = abs(cfg["sigma_t"]) * G * 16.0 / cfg["nu_h"]
        assert cfg["kappa_h"] == pytest.approx(U * 16.0 / ma)


def test_benchmark_oracle_window_cuts_no_droplet():
    """The CPU baseline's 64^3 window: every droplet of the block lies wholly
    inside it (clear of the faces by two interface widths) or wholly outside."""
    import bench
    cfg = W.droplet_block(n=512)
    (ox, oy, oz), inside = bench._clean_window(cfg, 64)
    assert inside >= 1
    n, box, m = 512.0, 64, 2 * cfg["xi"]
    count = 0
    for (x, y, z, r) in cfg["droplets"]:
        rel = np.mod(np.array([x, y, z]) - np.array([ox, oy, oz]), n)
        if np.all(rel >= r + m) and np.all(rel <= box - 1 - r - m):
            count += 1
            continue
        # outside: every periodic image of the centre is farther than r + 2 xi
        # from the window box [0, box - 1]^3
        best = np.inf
        for k in itertools.product((-1, 0, 1), repeat=3):
            c = rel + n * np.array(k)
            nearest = np.clip(c, 0.0, box - 1.0)
            best = min(best, float(np.linalg.norm(c - nearest)))
        assert best > r + m
    assert count == inside
