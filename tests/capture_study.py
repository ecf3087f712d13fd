"""Droplet capture by local laser heating: centroid trajectories against the
dimensionless time t* = gamma t (Sec. 3.2 in 2D, Sec. 3.3 and App. C in 3D).

    python tests/capture_study.py --dim 2 --angles 15 30 45 90 135 --q 0.2 --tstar 40
    python tests/capture_study.py --dim 3 --R 16 --heaters pair --shift 0.6667 --q 1.0 --tstar 60

Each case: the domain of workloads.laser_capture, the temperature initialised by
the thermal solver alone (phi and u at rest) until its per-update change is below
--warm-tol, then coupled steps; one JSON line per checkpoint (t*, centroid), and a
summary line per case: whether the centroid got past the heater (x_c > x_s + R,
the centroid followed continuously across the periodic x boundary) and the
largest transverse excursion |z_c - z_0|.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _circular_mean(w, n):
    """Centre of mass of the weights w[0..n) on a periodic axis of length n."""
    a = 2.0 * np.pi * np.arange(n) / n
    return float(np.arctan2((w * np.sin(a)).sum(), (w * np.cos(a)).sum()) * n / (2.0 * np.pi)) % n


def _unwrap(v, prev, n):
    return prev + ((v - prev + 0.5 * n) % n - 0.5 * n)


def centroid(d, prev=None):
    """Droplet centroid from the phase field, continuous across the periodic x
    and z boundaries (prev: the previous centroid)."""
    phi = d.get_field("phi")
    nz, ny, nx = phi.shape
    x = _circular_mean(phi.sum(axis=(0, 1)), nx)
    z = _circular_mean(phi.sum(axis=(1, 2)), nz) if nz > 1 else 0.0
    y = float((phi.sum(axis=(0, 2)) * np.arange(ny)).sum() / phi.sum())
    if prev is not None:
        x, z = _unwrap(x, prev[0], nx), _unwrap(z, prev[2], nz)
    return (x, y, z)


def run_case(cfg, tstar, every, warm_max, warm_tol, verbose=True):
    from paper_2401_03041_amd import tcplb
    d = tcplb.domain_from_workload(cfg)
    t0 = time.time()
    nwarm, change = d.warm_temperature(warm_max, warm_tol, 500)
    t_max = float(d.get_field("T").max())
    gamma = cfg["gamma"]
    xs = cfg["heat_sources"][0][1]
    c0 = c = centroid(d)
    steps_per = max(1, int(round(every / gamma)))
    nchk = int(round(tstar / every))
    traj = []
    for k in range(1, nchk + 1):
        d.step(steps_per)
        c = centroid(d, c)
        traj.append((k * steps_per * gamma, float(c[0]), float(c[1]), float(c[2])))
        if verbose:
            print(json.dumps({"case": cfg["name"], "tstar": round(traj[-1][0], 3), "x": round(c[0], 3),
                              "y": round(c[1], 3), "z": round(c[2], 3)}), flush=True)
    d.close()
    xmax = max(t[1] for t in traj)
    zdev = max(abs(t[3] - c0[2]) for t in traj)
    out = {"case": cfg["name"], "summary": True, "warm_steps": nwarm, "warm_change": change, "t_max": round(t_max, 4),
           "x0": round(float(c0[0]), 3), "x_end": round(traj[-1][1], 3), "x_heater": xs,
           "passed": bool(xmax > xs + cfg["droplets"][0][3]), "z_excursion": round(zdev, 3),
           "steps": steps_per * nchk, "seconds": round(time.time() - t0, 1)}
    print(json.dumps(out), flush=True)
    return out, traj


def main() -> int:
    from paper_2401_03041_amd import workloads as W
    ap = argparse.ArgumentParser()
    ap.add_argument("--dim", type=int, default=2)
    ap.add_argument("--R", type=float, default=32.0)
    ap.add_argument("--angles", type=float, nargs="+", default=[90.0])
    ap.add_argument("--q", type=float, nargs="+", default=[0.2])
    ap.add_argument("--heaters", default="single")
    ap.add_argument("--shift", type=float, default=0.5)
    ap.add_argument("--tstar", type=float, default=40.0)
    ap.add_argument("--every", type=float, default=2.0)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--sigma-t", type=float, default=None, help="override sigma_T")
    ap.add_argument("--warm-max", type=int, default=200000)
    ap.add_argument("--warm-tol", type=float, default=None,
                    help="per-update change of T that ends the warm-up (default 1e-9 in FP64, 1e-6 max(1, 5 q_s) otherwise)")
    args = ap.parse_args()
    for q in args.q:
        for a in args.angles:
            cfg = W.laser_capture(dim=args.dim, R=args.R, contact_angle=a, q_s=q, heaters=args.heaters,
                                  shift=args.shift, precision=args.precision)
            if args.sigma_t is not None:
                cfg["sigma_t"] = args.sigma_t
                cfg["name"] += f"_sigmaT{args.sigma_t:g}"
            # FP32 resolves T to about 6e-8 T_max, and T_max is about 5 q_s here
            tol = args.warm_tol if args.warm_tol is not None else (
                1e-9 if args.precision == "fp64" else 1e-6 * max(1.0, 5.0 * q))
            run_case(cfg, args.tstar, args.every, args.warm_max, tol)
    return 0


if __name__ == "__main__":
    sys.exit(main())
