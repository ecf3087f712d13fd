"""Shared test helpers: build oracle domains and compare fields."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O
from paper_2401_03041_amd import workloads as W

FIELDS = ("phi", "ux", "uy", "uz", "p", "T")


def oracle_domain(cfg: dict, phi=None, T=None, u=None, origin=(0, 0, 0), gdim=None) -> O.OracleDomain:
    """Oracle domain initialised from a workload description (or explicit fields)."""
    d = O.OracleDomain(cfg)
    dims = cfg["shape"]
    if phi is not None:
        d.set_field("phi", phi)
    elif cfg["droplets"]:
        d.set_droplets(cfg["droplets"], gdim=gdim, origin=origin,
                       periodic=None if gdim is None else cfg.get("_global_periodic"))
    else:
        d.set_field("phi", np.zeros((dims[2], dims[1], dims[0])))
    if T is None:
        T = W.temperature(cfg) if gdim is None else None
    if T is not None:
        d.set_field("T", T)
    uu = W.velocity(cfg) if u is None else u
    for a, name in enumerate(("ux", "uy", "uz")):
        d.set_field(name, uu[a])
    if cfg["heat_sources"]:
        d.set_heat_sources(cfg["heat_sources"])
    d.initialize()
    return d


def rel_err(a: np.ndarray, b: np.ndarray, floor: float = 0.0) -> float:
    """max|a - b| / max(max|b|, floor) (absolute if both vanish)."""
    den = max(float(np.max(np.abs(b))), floor)
    num = float(np.max(np.abs(a - b)))
    return num / den if den > 0 else num


def gpu_domain(cfg: dict, phi=None, T=None, u=None):
    """GPU domain initialised from a workload description (or explicit fields)."""
    from paper_2401_03041_amd import tcplb
    d = tcplb.Domain(cfg)
    if phi is not None:
        d.set_field("phi", phi)
    elif cfg["droplets"]:
        d.set_droplets(cfg["droplets"])
    d.set_field("T", W.temperature(cfg) if T is None else T)
    uu = W.velocity(cfg) if u is None else u
    for a, name in enumerate(("ux", "uy", "uz")):
        d.set_field(name, uu[a])
    if cfg["heat_sources"]:
        d.set_heat_sources(cfg["heat_sources"])
    d.initialize()
    return d


def compare(gpu, ora, names=FIELDS, floor: float = 0.0) -> dict:
    """Per-field max|gpu - oracle| / max(max|oracle|, floor)."""
    return {k: rel_err(gpu.get_field(k), ora.get_field(k), floor) for k in names}
