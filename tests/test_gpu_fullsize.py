"""Full-size check in the configurations bench.py times: the 512^3 droplet block in
FP32, FP64 and FP16-PDF storage.  The oracle cannot run 134 M cells, but one step only couples a cell
to its 27 neighbours (every stencil and pull has radius one and the hydrodynamic
update reads phi^n), so after k steps a cell depends only on the initial state
within radius k.  The oracle therefore builds its own initial state on small
periodic patches (droplet list and temperature Gaussians of the full block, in
global coordinates), advances them k steps, and the cells at least k away from
the patch edge must match the GPU's cells at the same global positions.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from paper_2401_03041_amd import workloads as W

pytestmark = pytest.mark.gpu

N = 512
STEPS = 3
HALF = STEPS + 3  # patch half-width


def _samples(cfg):
    """Patch centres: points on droplet interfaces (one per octant), a cell near the
    periodic corner and one in the far field."""
    pts = []
    for (x, y, z, r) in cfg["droplets"][:6]:
        pts.append((int(round(x + r)) % N, int(round(y)) % N, int(round(z)) % N))
    pts.append((0, N - 1, 1))
    pts.append((N // 2, 3, N - 2))
    return pts


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("fp64", 1e-11), ("fp16", 1e-3)])
def test_droplet_block_512_sampled_against_oracle(precision, tol):
    import torch

    from paper_2401_03041_amd import tcplb
    cfg = W.droplet_block(n=N, precision=precision)
    g = tcplb.domain_from_workload(cfg)
    m0, _ = g.reduce()
    g.step(STEPS)
    m1, _ = g.reduce()
    assert abs(m1 - m0) < 1e-6 * m0
    names = ("phi", "ux", "uy", "uz", "p", "T")
    gpu = {}
    for k in names:
        t = torch.empty((N, N, N), dtype=torch.float64, device="cuda")
        g.get_field(k, out=t)
        gpu[k] = t
    torch.cuda.synchronize()
    scale = {k: float(gpu[k].abs().max()) for k in names}
    print("field scales", scale)
    side = 2 * HALF + 1
    inner = HALF - STEPS
    worst = {k: 0.0 for k in names}
    for (cx, cy, cz) in _samples(cfg):
        org = (cx - HALF, cy - HALF, cz - HALF)
        sub = dict(cfg, shape=(side, side, side))
        o = O.OracleDomain(sub)
        o.set_droplets(cfg["droplets"], gdim=(N, N, N), origin=org, periodic=(1, 1, 1))
        o.set_field("T", W.temperature(cfg, origin=org, dims=(side, side, side)))
        o.initialize()
        o.step(STEPS)
        sl = slice(HALF - inner, HALF + inner + 1)
        iz, iy, ix = (torch.as_tensor(np.arange(c - inner, c + inner + 1) % N, device="cuda")
                      for c in (cz, cy, cx))
        for k in names:
            ref = o.get_field(k)[sl, sl, sl]
            got = gpu[k].index_select(0, iz).index_select(1, iy).index_select(2, ix).cpu().numpy()
            err = float(np.max(np.abs(got - ref))) / scale[k]
            worst[k] = max(worst[k], err)
        o.close()
    print(precision, "worst relative errors", worst)
    for k in names:
        assert worst[k] < tol, (k, worst[k])
    g.close()
    del gpu
    torch.cuda.empty_cache()


@pytest.mark.parametrize("thermal", ["lb", "rk2", "rk4"])
def test_paper_block_sampled_against_oracle(thermal):
    """The paper's per-GPU benchmark shape as bench.py's paper_block runs it:
    512 x 256 x 256 capture channel (walls in y, moving lid, heater of width 32
    on the bottom wall, hemisphere of radius 24), D3Q27 phase field and
    hydrodynamics, FP64, with the fused thermal LB step or the RK2 / RK4
    stages.  One LB step couples a cell to its neighbours; one RK step to cells
    as far away as it has stages (each a 27-point stencil).  After 3 steps,
    patches spanning the whole channel height (so both walls are exact) and,
    in x and z, the 7 compared cells plus 3 (LB), 6 (RK2) or 12 (RK4) on each
    side, built by the
    oracle from the same inputs in global coordinates, must match within 1e-11
    of each field's magnitude."""
    import torch

    from paper_2401_03041_amd import tcplb
    nx, ny, nz = 512, 256, 256
    cfg = dict(W.capture(shape=(nx, ny, nz), precision="fp64"), q_pf=27, thermal=thermal, q_thermal=7,
               kappa_h=0.2, kappa_l=0.2)
    g = tcplb.domain_from_workload(cfg)
    g.step(STEPS)
    names = ("phi", "ux", "uy", "uz", "p", "T")
    gpu = {}
    for k in names:
        t = torch.empty((nz, ny, nx), dtype=torch.float64, device="cuda")
        g.get_field(k, out=t)
        gpu[k] = t
    torch.cuda.synchronize()
    scale = {k: float(gpu[k].abs().max()) for k in names}
    (dx, dy, dz, r), = cfg["droplets"]
    (q, hx, hy, hz, w, dc), = cfg["heat_sources"]
    # droplet interface along x and along z, heater centre, periodic corner
    centres = [(int(dx + r), int(dz)), (int(dx), int(dz + r)), (int(hx), int(hz)), (0, nz - 1)]
    inner = 3
    half = inner + {"lb": 1, "rk2": 2, "rk4": 4}[thermal] * STEPS
    side = 2 * half + 1
    worst = {k: 0.0 for k in names}
    for (cx, cz) in centres:
        ox, oz = cx - half, cz - half
        o = O.OracleDomain(dict(cfg, shape=(side, ny, side)))
        o.set_droplets(cfg["droplets"], gdim=(nx, ny, nz), origin=(ox, 0, oz), periodic=(1, 0, 1))
        o.set_field("T", np.zeros((side, ny, side)))
        o.set_heat_sources([(q, hx - ox, hy, hz - oz, w, dc)])
        o.initialize()
        o.step(STEPS)
        sl = slice(half - inner, half + inner + 1)
        iz, ix = (torch.as_tensor(np.arange(c - inner, c + inner + 1) % n, device="cuda")
                  for c, n in ((cz, nz), (cx, nx)))
        for k in names:
            ref = o.get_field(k)[sl, :, sl]
            got = gpu[k].index_select(0, iz).index_select(2, ix).cpu().numpy()
            worst[k] = max(worst[k], float(np.max(np.abs(got - ref))) / max(scale[k], 1e-300))
        o.close()
    print(thermal, "worst relative errors", worst, "scales", scale, flush=True)
    for k in names:
        assert worst[k] < 1e-11, (k, worst[k])
    g.close()
    del gpu
