"""The paper's own verification case at its full size (Sec. 3.1, App. A): the 2D
planar heated channel, 512 x 256 cells, thermal LB (D3Q7), k* = 1, 4e5 steps in
FP64, against the closed form.  The paper prints l2 errors of 1.1164e-3
(temperature) and 9.2165e-2 (velocity) for this case."""
from __future__ import annotations

import os

import pytest

from tests.appA_channel import load_table, run

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "appA_planar_channel.txt")


def test_planar_heated_channel_full_size_lb():
    paper_T, paper_u = load_table(GOLDEN)[("2D", "LB", 1.0)]
    eT, eu = run(thermal="lb", q_thermal=7, k_star=1.0, nz=1, precision="fp64")
    print(f"l2 temperature {eT:.4e} (paper {paper_T:.4e}), l2 velocity {eu:.4e} (paper {paper_u:.4e})")
    assert eT < 2.0 * paper_T
    assert eu < 2.0 * paper_u
