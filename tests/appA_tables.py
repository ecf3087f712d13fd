"""Reproduce the App. A verification tables of Sec. 3.1 on the GPU.

    python tests/appA_tables.py [--only 2D|3D] [--kstar K] [--precision fp64|fp32] [--steps N]

Runs the 2D channel with the thermal LB (D3Q7), RK2 and RK4 schemes and the
pseudo-3D channel (10 cells in z) with the D3Q7/15/19/27 thermal LB, for the
conductivity ratios k* = 1 and 1/5, and prints each relative l2 error next to
the value the paper prints (tests/golden/appA_planar_channel.txt).
"""
from __future__ import annotations

import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from tests.appA_channel import load_table, run  # noqa: E402

CASES = {"LB": ("lb", 7), "RK2": ("rk2", 7), "RK4": ("rk4", 7),
         "Q7": ("lb", 7), "Q15": ("lb", 15), "Q19": ("lb", 19), "Q27": ("lb", 27)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", choices=("2D", "3D"), default=None)
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--steps", type=int, default=400_000)
    ap.add_argument("--kstar", type=float, default=None, help="only this conductivity ratio")
    args = ap.parse_args()
    table = load_table(os.path.join(ROOT, "tests", "golden", "appA_planar_channel.txt"))
    print("| table | case | k* | l2 T | paper | l2 |u| | paper | s |")
    print("|---|---|---|---|---|---|---|---|")
    for (tab, case, ks), (pT, pu) in table.items():
        if (args.only and tab != args.only) or (args.kstar is not None and ks != args.kstar):
            continue
        thermal, q = CASES[case]
        t0 = time.perf_counter()
        eT, eu = run(thermal=thermal, q_thermal=q, k_star=ks, nz=1 if tab == "2D" else 10,
                     precision=args.precision, steps=args.steps)
        print(f"| {tab} | {case} | {ks:g} | {eT:.4e} | {pT:.4e} | {eu:.4e} | {pu:.4e} | "
              f"{time.perf_counter() - t0:.0f} |", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
