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
