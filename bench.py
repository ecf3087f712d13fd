#!/usr/bin/env python3
"""Throughput of the coupled thermocapillary sweep on one MI355X.

One step = phase-field LB (D3Q15) + hydrodynamic LB (D3Q27, all forces) +
thermal LB (D3Q7) over the whole grid.  Default workload: the single-GPU
droplet block, 512^3 periodic cells, 64 droplets (radii uniform in [10, 24],
density ratio 100) in a smooth random temperature field, shifted-FP32
storage; the same block in FP64, and with FP16 phase-field and thermal
PDFs, is timed after it.  Inputs are resident in
HBM before the timed region; the timed region is `steps` calls of the whole
step bracketed by device synchronisations.

Prints one JSON line (metric, value in MLUPS, roofline of the dominant kernel
from HIP events on the library's stream, and the FP64 oracle timed on the host
cores over a bounded sample of the same workload).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS & % HBM roofline per coupled step, FP32 vs FP64; adjoint/forward cost"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_step_droplet_block_512.md")


def _log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


KERNEL_SOURCES = ("kernels_step.hip", "cell_pf.hpp", "cell_hydro.hpp", "cell_thermal.hpp", "lattice.hpp",
                  "kernels.hpp")


def _kernel_sha() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2401_03041_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _traffic(precision: str):
    """Measured HBM bytes per launch of the fused step kernel (rocprofv3
    FETCH_SIZE + WRITE_SIZE, scaled by a copy kernel), if taken on the current
    kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        line = line.strip().strip("`")
        if line.startswith("traffic_") and "=" in line:
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("traffic_kernel_sha") != _kernel_sha():
        return None
    key = f"traffic_bytes_per_launch_{precision}"
    return float(vals[key]) if key in vals else None


def run_gpu(cfg: dict, steps: int, warmup: int, precision: str, fuse: bool = True) -> dict:
    import torch

    from paper_2401_03041_amd import tcplb
    cfg = dict(cfg, precision=precision)
    t0 = time.perf_counter()
    d = tcplb.domain_from_workload(cfg)
    d.set_fusion(fuse)
    torch.cuda.synchronize()
    _log(f"{precision}: set-up {time.perf_counter() - t0:.1f} s")
    d.step(warmup)
    d.synchronize()
    d.set_profiling(True)
    d.kernel_times()  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d.step(steps)
    d.synchronize()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    times = d.kernel_times()
    d.set_profiling(False)
    mass, _ = d.reduce()
    ncell = d.ncell
    bpc = d.algorithmic_bytes()
    kernels = {}
    step_bytes = 0.0
    for k, (ms, n) in times.items():
        if n == 0:
            continue
        avg = ms / n
        # the byte model counts a whole step; the RK stages share it
        per_launch = bpc[k] * ncell / (n / steps if k == "rk" else 1)
        kernels[k] = {"avg_ms": avg, "launches": n, "algorithmic_bytes_per_launch": per_launch,
                      "achieved_GBs": per_launch / (avg * 1e-3) / 1e9}
        step_bytes += per_launch * n / steps
    d.close()
    del d
    torch.cuda.empty_cache()
    mlups = ncell * steps / elapsed / 1e6
    _log(f"{precision}: {mlups:.1f} MLUPS, {1e3 * elapsed / steps:.3f} ms/step, mass {mass:.6e}")
    return {"mlups": mlups, "ms_per_step": 1e3 * elapsed / steps, "kernels": kernels,
            "step_bytes_per_cell": step_bytes / ncell, "ncell": ncell, "mass": mass,
            "effective_GBs": step_bytes * steps / elapsed / 1e9}


def adjoint_cost(cfg: dict, updates: int, precision: str) -> dict:
    """Thermal update with phi and u held (the temperature warm-up: the LB kernel,
    or the RK stages) against its adjoint (tcp_thermal_adjoint), per update, from
    per-kernel HIP-event times on the same domain."""
    import numpy as np
    import torch

    from paper_2401_03041_amd import tcplb
    d = tcplb.domain_from_workload(dict(cfg, precision=precision))
    m = np.ones(d.shape3)
    d.warm_temperature(2, 0.0, 10)
    d.thermal_adjoint(2, m)
    d.set_profiling(True)
    d.kernel_times()
    d.warm_temperature(updates, 0.0, updates + 1)
    fkey = "thermal" if cfg.get("thermal", "lb") == "lb" else "rk"
    fwd = d.kernel_times()[fkey]
    d.thermal_adjoint(updates, m)
    adj = d.kernel_times()["adjoint"]
    d.set_profiling(False)
    bpc = d.algorithmic_bytes()
    ncell = d.ncell
    d.close()
    del d
    torch.cuda.empty_cache()
    # per update: the byte model counts a whole update, except an RK adjoint
    # stage, which it counts per launch
    f_ms, a_ms = fwd[0] / updates, adj[0] / updates
    a_bytes = bpc["adjoint"] * (adj[1] / updates if fkey == "rk" else 1.0)
    scheme = "thermal LB D3Q%d" % cfg.get("q_thermal", 7) if fkey == "thermal" else cfg["thermal"].upper()
    _log(f"{precision} {scheme}: update {f_ms:.3f} ms, adjoint update {a_ms:.3f} ms")
    return {"kind": f"{scheme} with phi and u held (temperature warm-up) and its adjoint",
            "updates": updates, "forward_ms_per_update": round(f_ms, 4), "adjoint_ms_per_update": round(a_ms, 4),
            "adjoint_over_forward": round(a_ms / f_ms, 3),
            "forward_GBs": round(bpc[fkey] * ncell / (f_ms * 1e-3) / 1e9, 1),
            "adjoint_GBs": round(a_bytes * ncell / (a_ms * 1e-3) / 1e9, 1),
            "adjoint_bytes_per_cell_update": a_bytes}


def coupled_adjoint_cost(precision: str, steps: int = 2000, segment: int = 0) -> dict:
    """Adjoint of the coupled step on the heater-design channel (96 x 64 x 64,
    walls, moving lid, heater, hemisphere; D3Q15 phase field + D3Q27 hydro +
    D3Q7 thermal LB): the gradient of the final centroid's squared distance to
    a target with respect to the heater (Q, x, y, z) and the wall
    temperatures.  Times the plain forward run of `steps` steps, the taped run
    (checkpoints every `segment` steps, 0: ceil(sqrt(steps)); 1 stores every
    state) and the reverse sweep (segment recomputation plus the reverse
    kernels); cost = (taped + reverse) / plain.
    Inputs are resident in HBM; the tape is allocated by an untimed warm-up."""
    import numpy as np
    import torch

    from paper_2401_03041_amd import tcplb
    from paper_2401_03041_amd import workloads as W
    cfg = W.capture_design(precision=precision, steps=steps)
    d = tcplb.domain_from_workload(cfg)
    c0 = d.reduce()[1]
    target = np.array([44.0, c0[1], c0[2]])
    st = d.save_state()
    d.step_taped(steps, segment)  # warm-up: allocates the tape, builds the step graphs
    d.tape_adjoint(np.zeros(3))

    def timed(fn):
        d.load_state(st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        d.synchronize()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, out

    # each part timed twice, the faster kept (the first timed run of a part is
    # a few per cent slower on some boxes)
    t_fwd = min(timed(lambda: d.step(steps))[0] for _ in range(2))
    t_tape = min(timed(lambda: d.step_taped(steps, segment))[0] for _ in range(2))
    c = d.reduce()[1]
    t_rev = None
    for _ in range(2):
        d.synchronize()
        t0 = time.perf_counter()
        g = d.tape_adjoint(2.0 * (c - target))
        t = time.perf_counter() - t0
        t_rev = t if t_rev is None else min(t_rev, t)
    d.set_profiling(True)
    d.kernel_times()
    d.load_state(st)
    d.step_taped(steps, segment)
    d.tape_adjoint(2.0 * (c - target))
    kt = d.kernel_times()
    d.set_profiling(False)
    bpc = d.algorithmic_bytes()
    ncell = d.ncell
    d.close()
    del d
    torch.cuda.empty_cache()
    rev_ms, rev_n = kt["coupled_adjoint"]
    fwd_ms, fwd_n = kt["step"]
    rev_avg, fwd_avg = rev_ms / rev_n, fwd_ms / fwd_n
    cost = (t_tape + t_rev) / t_fwd
    _log(f"{precision} coupled adjoint: forward {1e3 * t_fwd:.1f} ms, taped {1e3 * t_tape:.1f} ms, "
         f"reverse {1e3 * t_rev:.1f} ms ({steps} steps): cost {cost:.2f}x")
    return {"workload": "heater-design channel 96x64x64 (walls, lid 0.02, heater Q=0.8 w=8, hemisphere R=8), "
                        "D3Q15 phase field + D3Q27 hydro + D3Q7 thermal LB; loss |centroid(phi^N) - target|^2; "
                        "gradients w.r.t. heater Q, x, y, z and both wall-temperature fields",
            "precision": precision, "steps": steps, "segment": segment if segment > 0 else int(np.ceil(np.sqrt(steps))),
            "forward_ms": round(1e3 * t_fwd, 2), "taped_forward_ms": round(1e3 * t_tape, 2),
            "reverse_ms": round(1e3 * t_rev, 2), "adjoint_over_forward": round(cost, 3),
            "reverse_step_kernels_avg_ms": round(rev_avg, 5), "forward_step_kernel_avg_ms": round(fwd_avg, 5),
            "reverse_step_over_forward_step": round(rev_avg / fwd_avg, 3),
            "reverse_step_bytes_per_cell": bpc["coupled_adjoint"],
            "reverse_step_algorithmic_GBs": round(bpc["coupled_adjoint"] * ncell / (rev_avg * 1e-3) / 1e9, 1),
            "dL_dsource": [round(float(v), 9) for v in g[0][0]]}


# Algorithmic bytes per cell update of the coupled step (D3Q15 phase field,
# D3Q27 hydrodynamics, D3Q7 thermal LB) as the three kernels of Algorithm 1
# move them: each kernel reads and writes its PDFs once and reads or writes
# five fields once.  The fused step kernel needs fewer (it reads phi^n, u and
# phi^{n+1} once for all three updates: FP64 864, FP32 432, FP16 PDFs 344 B);
# that figure is reported beside the headline one.
STEP_MODEL_BYTES = {"fp64": 904.0, "fp32": 452.0, "fp16": 364.0}


def roofline(res: dict, precision: str) -> dict:
    k = res["kernels"]["step"]
    per_launch = STEP_MODEL_BYTES[precision] * res["ncell"]
    achieved = per_launch / (k["avg_ms"] * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": "step (phase field D3Q15 + hydrodynamics D3Q27 + thermal D3Q7, fused)",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": _traffic(precision),
            "algorithmic_bytes_per_launch": per_launch, "algorithmic_bytes_per_cell": STEP_MODEL_BYTES[precision],
            "avg_launch_ms": k["avg_ms"],
            "fused_kernel_min_bytes_per_cell": res["step_bytes_per_cell"],
            "fused_kernel_min_frac": round(k["achieved_GBs"] / HBM_PEAK_GBS, 4)}


def _clean_window(cfg: dict, box: int, stride: int = 16):
    """Origin of a box^3 window of the periodic grid whose faces cross no droplet:
    every droplet lies inside it or clear of it by two interface widths (the
    oracle wraps the window periodically, so a cut droplet would leave a jump in
    phi at the seam).  Among such windows, the one holding the most droplets."""
    import numpy as np
    n = np.array(cfg["shape"], dtype=np.float64)
    drops = np.asarray(cfg["droplets"], dtype=np.float64).reshape(-1, 4)
    margin = 2.0 * cfg["xi"]
    best, best_in = None, 0
    for ox in range(0, int(n[0]), stride):
        for oy in range(0, int(n[1]), stride):
            for oz in range(0, int(n[2]), stride):
                o = np.array([ox, oy, oz], dtype=np.float64)
                rel = np.mod(drops[:, :3] - o, n)          # centre in window coordinates, in [0, n)
                r = drops[:, 3] + margin
                inside = np.all((rel >= r[:, None]) & (rel <= box - 1 - r[:, None]), axis=1)
                # distance from the centre to the window along each axis (periodic)
                lo = np.minimum(np.abs(rel), np.abs(rel - n))
                hi = np.minimum(np.abs(rel - (box - 1)), np.abs(rel - (box - 1) + n))
                inwin = rel <= box - 1
                gap = np.where(inwin, 0.0, np.minimum(lo, hi))
                outside = np.sqrt(np.sum(gap ** 2, axis=1)) > r
                if np.all(inside | outside) and inside.sum() > best_in:
                    best, best_in = (ox, oy, oz), int(inside.sum())
    return best, best_in


def cpu_baseline(cfg: dict, box: int, steps: int) -> dict:
    """The FP64 oracle on a box x box x box window of the same workload (its own
    initialisation from the droplet list and temperature Gaussians in global
    coordinates, periodic wrap on the window), placed so that no droplet crosses
    the window's faces."""
    from oracle import oracle as O
    from paper_2401_03041_amd import workloads as W
    origin, ninside = _clean_window(cfg, box)
    if origin is None:
        raise RuntimeError(f"no {box}^3 window of the workload is free of cut droplets")
    sub = dict(cfg, shape=(box, box, box))
    d = O.OracleDomain(sub)
    d.set_droplets(cfg["droplets"], gdim=cfg["shape"], origin=origin, periodic=(1, 1, 1))
    d.set_field("T", W.temperature(cfg, origin=origin, dims=(box, box, box)))
    d.initialize()
    t0 = time.perf_counter()
    d.step(steps)
    el = time.perf_counter() - t0
    mlups = box ** 3 * steps / el / 1e6
    threads = O.num_threads()
    _log(f"oracle: {mlups:.3f} MLUPS on {threads} threads ({el:.1f} s)")
    # the same code on one thread, continuing the same run for a tenth of the steps
    steps1 = max(1, steps // 10)
    O.set_num_threads(1)
    t0 = time.perf_counter()
    d.step(steps1)
    el1 = time.perf_counter() - t0
    O.set_num_threads(threads)
    mlups1 = box ** 3 * steps1 / el1 / 1e6
    _log(f"oracle: {mlups1:.3f} MLUPS on 1 thread ({el1:.1f} s)")
    d.close()
    return {"value": round(mlups, 4), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{box}^3 window at {origin} of the {cfg['shape'][0]}^3 droplet block ({ninside} whole "
                      f"droplets, its temperature field, no droplet cut by the faces), {steps} steps, FP64, "
                      f"{el:.1f} s",
            "single_thread": {"value": round(mlups1, 4), "steps": steps1, "seconds": round(el1, 1)},
            "host_cpu": _cpu_model(), "host_logical_cpus": os.cpu_count()}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# The paper's own per-GPU figures for its coupled FP64 step on a 512 x 256 x 256
# block (D3Q27 phase field and hydrodynamics; one node of four GPUs in the weak
# scaling figures of Sec. 4.3, MLUPS per GPU, an MI250 "GPU" being the module) and
# for the thermal sub-step alone (Sec. 4.2 comparison of the thermal schemes, GLUPS).
PAPER_COUPLED_MLUPS = {"A100": {"lb_d3q7": 1189.6, "rk2": 1190.9, "rk4": 1030.8},
                       "MI250": {"lb_d3q7": 1626.7, "rk2": 1472.5, "rk4": 1244.7}}
PAPER_THERMAL_GLUPS = {"A100": {"lb_d3q7": 9.058, "lb_d3q15": 4.785, "lb_d3q19": 3.949, "lb_d3q27": 2.859,
                                "rk2": 7.781, "rk4": 3.573},
                       "MI250": {"lb_d3q7": 13.544, "lb_d3q15": 7.352, "lb_d3q19": 5.850, "lb_d3q27": 3.712,
                                 "rk2": 8.308, "rk4": 4.060}}


def paper_block(steps: int, warmup: int) -> dict:
    """The paper's per-GPU benchmark shape: 512 x 256 x 256 cells, FP64, D3Q27 phase
    field + D3Q27 hydrodynamics + each thermal scheme (capture-channel workload:
    walls, moving lid, heater, droplet; kappa = 0.2 so that the RK schemes are
    stable).  Coupled-step MLUPS (the thermal LB step fused into one kernel, the
    phase-field and hydrodynamic updates fused with the RK schemes; also with
    every kernel apart) and the thermal sub-step alone in GLUPS (timed with the
    kernels apart)."""
    from paper_2401_03041_amd import workloads as W
    coupled, split, thermal, kernel_gbs = {}, {}, {}, {}
    n = 512 * 256 * 256
    for name, th, q in (("lb_d3q7", "lb", 7), ("lb_d3q15", "lb", 15), ("lb_d3q19", "lb", 19),
                        ("lb_d3q27", "lb", 27), ("rk2", "rk2", 7), ("rk4", "rk4", 7)):
        cfg = dict(W.capture(shape=(512, 256, 256), precision="fp64"), q_pf=27, thermal=th, q_thermal=q,
                   kappa_h=0.2, kappa_l=0.2)
        if name in ("lb_d3q7", "rk2", "rk4"):
            coupled[name] = round(run_gpu(cfg, steps, warmup, "fp64")["mlups"], 1)
        res = run_gpu(cfg, steps, warmup, "fp64", fuse=False)
        if name in ("lb_d3q7", "rk2", "rk4"):
            split[name] = round(res["mlups"], 1)
        kernel_gbs[name] = {kk: round(v["achieved_GBs"], 1) for kk, v in res["kernels"].items()}
        k = res["kernels"]["thermal" if th == "lb" else "rk"]
        per_step_ms = k["avg_ms"] * k["launches"] / steps
        thermal[name] = round(n / (per_step_ms * 1e-3) / 1e9, 3)
    return {"grid": [512, 256, 256], "dtype": "f64", "steps": steps,
            "workload": "capture channel (walls, moving lid, heater, droplet), D3Q27 phase field + D3Q27 "
                        "hydrodynamics + thermal scheme",
            "coupled_MLUPS": coupled, "coupled_MLUPS_kernels_apart": split, "thermal_substep_GLUPS": thermal,
            "split_kernels_algorithmic_GBs": kernel_gbs,
            "paper_coupled_MLUPS_per_gpu": PAPER_COUPLED_MLUPS, "paper_thermal_substep_GLUPS": PAPER_THERMAL_GLUPS}


def copy_calibration(gib: float = 4.0, reps: int = 3) -> None:
    """The library's streaming copy kernel on a buffer of known size, for
    scaling the HBM byte counters: every dispatch reads and writes `gib` GiB;
    then the 27-component blocked copy (the step kernel's access pattern) on
    512^3 cells, every dispatch reading and writing 14.5 GB."""
    from paper_2401_03041_amd import tcplb
    nbytes = int(gib * (1 << 30))
    gbs = tcplb.bandwidth_probe(nbytes, reps)
    _log(f"copy calibration: {reps + 1} dispatches, each reading and writing {nbytes} bytes; best {gbs:.0f} GB/s")
    cells = 1 << 27
    gbs = tcplb.pdf_copy_probe(cells, reps)
    _log(f"blocked 27-component copy: {reps + 1} dispatches, each reading and writing {cells * 27 * 4} bytes; "
         f"best {gbs:.0f} GB/s")


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=512, help="edge of the cubic droplet block")
    ap.add_argument("--fp64-steps", type=int, default=None, help="timed FP64 steps (default: steps/2; 0 skips)")
    ap.add_argument("--fp16-steps", type=int, default=None,
                    help="timed steps with FP16 phase-field/thermal PDFs (default: steps/2; 0 skips)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-paper-block", action="store_true",
                    help="skip the FP64 runs on the paper's 512 x 256 x 256 benchmark shape")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint-cost legs")
    ap.add_argument("--oracle-box", type=int, default=64)
    ap.add_argument("--oracle-steps", type=int, default=200)
    ap.add_argument("--copy-calibration", action="store_true", help="only run the copy kernel")
    ap.add_argument("--placement", type=int, default=0,
                    help="only create this many FP32 blocks in turn (each freed before the next) and print "
                         "the step kernel's time on each (spread between physical placements)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the single-GPU block is the unit it "
              "measures (--gpus 1)", file=sys.stderr)
        return 2
    if args.copy_calibration:
        copy_calibration()
        return 0
    if args.placement > 0:
        from paper_2401_03041_amd import workloads as W
        cfg = W.droplet_block(n=args.n, precision="fp32")
        for k in range(args.placement):
            res = run_gpu(cfg, 6, 2, "fp32")
            print(json.dumps({"domain": k, "step_ms": round(res["kernels"]["step"]["avg_ms"], 3)}), flush=True)
        return 0

    from paper_2401_03041_amd import tcplb
    from paper_2401_03041_amd import workloads as W
    copy_gbs = tcplb.bandwidth_probe()
    _log(f"streaming copy probe: {copy_gbs:.0f} GB/s")
    pdf_copy_gbs = tcplb.pdf_copy_probe(args.n ** 3 if args.n % 4 == 0 else 1 << 27)
    _log(f"blocked 27-component copy probe: {pdf_copy_gbs:.0f} GB/s")
    cfg = W.droplet_block(n=args.n, precision="fp32")
    fp32 = run_gpu(cfg, args.steps, args.warmup, "fp32")
    fp64_steps = args.steps // 2 if args.fp64_steps is None else args.fp64_steps
    fp64 = run_gpu(cfg, fp64_steps, max(2, args.warmup // 4), "fp64") if fp64_steps > 0 else None
    fp16_steps = args.steps // 2 if args.fp16_steps is None else args.fp16_steps
    fp16 = run_gpu(cfg, fp16_steps, max(2, args.warmup // 4), "fp16") if fp16_steps > 0 else None
    adjoint = None
    if not args.no_adjoint:
        adjoint = {"coupled": coupled_adjoint_cost("fp32"), "coupled_fp64": coupled_adjoint_cost("fp64"),
                   "coupled_every_state": coupled_adjoint_cost("fp32", segment=1)}
        thermal = adjoint_cost(cfg, 20, "fp32")
        thermal["adjoint_update_over_coupled_step"] = round(thermal["adjoint_ms_per_update"] / fp32["ms_per_step"],
                                                            3)
        adjoint["thermal_lb"] = thermal
        adjoint["thermal_rk4"] = adjoint_cost(dict(cfg, thermal="rk4"), 10, "fp32")
    pblock = None if args.no_paper_block else paper_block(10, 2)
    base = None if args.no_cpu_baseline else cpu_baseline(cfg, args.oracle_box, args.oracle_steps)

    line = {
        "metric": METRIC,
        "value": round(fp32["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(fp32["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"droplet block {args.n}^3 periodic, 64 droplets r~U[10,24], density ratio 100, "
                               "D3Q15 phase field + D3Q27 hydro + D3Q7 thermal LB, shifted-FP32 storage",
                   "grid": [args.n] * 3, "precision": "fp32", "parallelism": "single GPU"},
        "roofline": roofline(fp32, "fp32"),
        "copy_probe_GBs": round(copy_gbs, 1),
        "step_kernel_frac_of_copy": round(fp32["kernels"]["step"]["achieved_GBs"] / copy_gbs, 4),
        "pdf_copy_probe_GBs": round(pdf_copy_gbs, 1),
        "step_kernel_frac_of_pdf_copy": round(fp32["kernels"]["step"]["achieved_GBs"] / pdf_copy_gbs, 4),
        "cpu_baseline": base,
        "step_bytes_per_cell": fp32["step_bytes_per_cell"],
        "effective_GBs": round(fp32["effective_GBs"], 1),
        "kernels": {k: {kk: round(vv, 5) if isinstance(vv, float) else vv for kk, vv in v.items()}
                    for k, v in fp32["kernels"].items()},
    }
    if fp64 is not None:
        line["fp64"] = {"value": round(fp64["mlups"], 2), "unit": "MLUPS", "steps": fp64_steps,
                        "ms_per_step": round(fp64["ms_per_step"], 4), "dtype": "f64",
                        "roofline": roofline(fp64, "fp64"), "effective_GBs": round(fp64["effective_GBs"], 1),
                        "step_bytes_per_cell": fp64["step_bytes_per_cell"]}
    if adjoint is not None:
        line["adjoint"] = adjoint
    if pblock is not None:
        line["paper_block"] = pblock
    if fp16 is not None:
        line["fp16"] = {"value": round(fp16["mlups"], 2), "unit": "MLUPS", "steps": fp16_steps,
                        "ms_per_step": round(fp16["ms_per_step"], 4),
                        "dtype": "f32 arithmetic; f16 phase-field and thermal PDFs, f32 hydrodynamic PDFs",
                        "roofline": roofline(fp16, "fp16"),
                        "effective_GBs": round(fp16["effective_GBs"], 1),
                        "step_bytes_per_cell": fp16["step_bytes_per_cell"],
                        "kernels": {k: {kk: round(vv, 5) if isinstance(vv, float) else vv for kk, vv in v.items()}
                                    for k, v in fp16["kernels"].items()}}
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
