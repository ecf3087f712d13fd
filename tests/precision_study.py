"""FP32 and FP16-PDF storage against FP64 on the same GPU, at full size and over
long runs (the oracle matches the FP64 path to 1e-11 on smaller cases but
cannot run these sizes).

    python tests/precision_study.py [--block-steps 500] [--capture-steps 5000]

Workloads: the 512^3 droplet block (density ratio 100) and the 256 x 128 x 96
capture channel (walls, moving lid, heater).  The three precisions run in
lockstep; every `--every` steps each field's error is printed as
max|F - F_fp64| / max|F_fp64| (the velocity as one vector against the flow
speed), one JSON line per checkpoint.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _fields(d, n):
    import torch
    out = {}
    for k in ("phi", "ux", "uy", "uz", "p", "T"):
        t = torch.empty(n, dtype=torch.float64, device="cuda")
        d.get_field(k, out=t)
        out[k] = t
    return out


def _errors(f, ref):
    import torch
    e = {k: float((f[k] - ref[k]).abs().max() / ref[k].abs().max()) for k in ("phi", "p", "T")}
    speed = float(torch.sqrt(ref["ux"] ** 2 + ref["uy"] ** 2 + ref["uz"] ** 2).max())
    e["u"] = max(float((f[k] - ref[k]).abs().max()) for k in ("ux", "uy", "uz")) / speed
    return {k: float(f"{v:.3e}") for k, v in e.items()}


def study(name, cfg, steps, every):
    import torch

    from paper_2401_03041_amd import tcplb
    doms = {p: tcplb.domain_from_workload(dict(cfg, precision=p)) for p in ("fp64", "fp32", "fp16")}
    n = tuple(cfg["shape"][::-1])
    done = 0
    while done < steps:
        k = min(every, steps - done)
        for d in doms.values():
            d.step(k)
        done += k
        ref = _fields(doms["fp64"], n)
        row = {"workload": name, "step": done}
        for p in ("fp32", "fp16"):
            f = _fields(doms[p], n)
            row[p] = _errors(f, ref)
            del f
        mass = {p: d.reduce()[0] for p, d in doms.items()}
        row["mass_rel_to_fp64"] = {p: float(f"{(mass[p] - mass['fp64']) / mass['fp64']:.3e}") for p in ("fp32", "fp16")}
        print(json.dumps(row), flush=True)
        del ref
        torch.cuda.empty_cache()
    for d in doms.values():
        d.close()
    torch.cuda.empty_cache()


def main() -> int:
    from paper_2401_03041_amd import workloads as W
    ap = argparse.ArgumentParser()
    ap.add_argument("--block-steps", type=int, default=500)
    ap.add_argument("--capture-steps", type=int, default=5000)
    ap.add_argument("--every", type=int, default=500)
    args = ap.parse_args()
    if args.capture_steps:
        study("capture 256x128x96", W.capture(), args.capture_steps, args.every)
    if args.block_steps:
        study("droplet block 512^3", W.droplet_block(n=512), args.block_steps, min(args.every, args.block_steps))
    return 0


if __name__ == "__main__":
    sys.exit(main())
