"""The allocation-free read-back (tcp_get_field_noalloc) through the C
interface, against tcp_get_field: every field of a stepped domain, then a
second domain with fewer cells read through the same staging array, then the
first again, and the size limit."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2401_03041_amd import tcplb
from paper_2401_03041_amd import workloads as W
from tests.helpers import gpu_domain

pytestmark = pytest.mark.gpu

NAMES = ("phi", "ux", "uy", "uz", "T", "p", "pstar", "rho")


def _stepped(shape, precision, steps):
    nx, ny, nz = shape
    cfg = W.make(shape=shape, periodic_y=False, precision=precision, rho_l=0.5, sigma_ref=2e-3, sigma_t=-1e-4,
                 u_wall_top=(0.02, 0.0, 0.0), t_wall_top=1.0,
                 droplets=[(nx / 2.0, ny / 3.0, nz / 2.0, min(shape) / 4.0)],
                 heat_sources=[(0.01, nx / 3.0, 1.0, nz / 2.0, 3.0, 0.0)])
    d = gpu_domain(cfg)
    d.step(steps)
    return d


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_readback_matches_get_field(precision):
    big = _stepped((70, 30, 22), precision, 12)
    small = _stepped((33, 17, 9), precision, 5)
    for d in (big, small, big):
        for name in NAMES:
            ref = d.get_field(name)
            got = d.get_field_noalloc(name)
            assert got.shape == ref.shape
            assert np.array_equal(got, ref), name
    big.close()
    small.close()


def test_noalloc_readback_size_limit():
    cfg = W.make(shape=(256, 128, 130))  # 4259840 cells > 4194304
    d = tcplb.Domain(cfg)
    with pytest.raises(tcplb.TcpError, match="4194304 cells"):
        d.get_field_noalloc("phi")
    d.close()
