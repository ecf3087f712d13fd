"""The planar heated two-layer channel of Sec. 3.1 on the GPU, against the App. A
closed form (shared by the GPU test and the table reproduction script).

Set-up as printed in Sec. 3.1: 512 x 256 cells (L = 256, a = b = 128), walls in y,
periodic in x (and z for the pseudo-3D channel), lower wall at
T_h + T_0 cos(omega x) with omega = 2 pi / L, upper wall at T_c, the heavy phase
(phi = 1, conductivity kappa_A) in the upper layer.  Readings where the section
is silent: unit density ratio, interface width xi = 4, initial state the flat
tanh interface with the conduction temperature profile and the fluid at rest.
"""
from __future__ import annotations

import numpy as np

from paper_2401_03041_amd import workloads as W
from tests.appA_reference import l2, planar_channel

L = 256
NX, NY = 2 * L, L
A = B = NY / 2
OMEGA = 2 * np.pi / L
T_H, T_C, T_0 = 20.0, 10.0, 4.0
SIGMA_T, SIGMA_REF, NU, KAPPA_B, MOBILITY, XI = -5e-4, 2.5e-2, 0.2, 0.2, 5e-2, 4.0


def load_table(path):
    rows = {}
    for line in open(path):
        line = line.split("#")[0].split()
        if line:
            rows[(line[0], line[1], float(line[2]))] = (float(line[3]), float(line[4]))
    return rows


def setup(thermal="lb", q_thermal=7, k_star=1.0, nz=1, precision="fp64", xi=XI):
    """Create and initialise the channel on the current torch stream; returns
    (domain, reference fields (u, v, T) of the closed form)."""
    from paper_2401_03041_amd import tcplb
    cfg = W.make(shape=(NX, NY, nz), periodic_y=False, thermal=thermal, q_thermal=q_thermal,
                 precision=precision, nu_h=NU, nu_l=NU, kappa_h=KAPPA_B * k_star, kappa_l=KAPPA_B,
                 mobility=MOBILITY, xi=xi, sigma_ref=SIGMA_REF, sigma_t=SIGMA_T, t_ref=0.0,
                 t_wall_top=T_C)
    x = np.arange(NX, dtype=np.float64)
    yc = np.arange(NY, dtype=np.float64) + 0.5 - B
    Y, X = np.meshgrid(yc, x, indexing="ij")
    ref = planar_channel(X, Y, A, B, OMEGA, T_H, T_C, T_0, SIGMA_T, NU, k_r=k_star)
    _, _, T_lin = planar_channel(X, Y, A, B, OMEGA, T_H, T_C, 0.0, SIGMA_T, NU, k_r=k_star)
    d = tcplb.Domain(cfg)
    d.set_field("phi", np.broadcast_to(0.5 + 0.5 * np.tanh(2 * Y / xi), (nz, NY, NX)).copy())
    d.set_field("T", np.broadcast_to(T_lin, (nz, NY, NX)).copy())
    d.set_wall_temperature(0, np.broadcast_to(T_H + T_0 * np.cos(OMEGA * x), (nz, NX)).copy())
    d.initialize()
    return d, ref


def finish(d, ref, fields=False):
    """(l2 temperature, l2 velocity magnitude) on the plane z = nz // 2 (or, with
    fields=True, phi, T, u_x, u_y, u_z on that plane); closes the domain."""
    k = d.nz // 2
    if fields:
        out = {name: d.get_field(name)[k] for name in ("phi", "T", "ux", "uy", "uz")}
        d.close()
        return out
    u_ref, v_ref, T_ref = ref
    T = d.get_field("T")[k]
    u, v = d.get_field("ux")[k], d.get_field("uy")[k]
    d.close()
    return l2(T, T_ref), l2(np.hypot(u, v), np.hypot(u_ref, v_ref))


def run(steps=400_000, fields=False, **kw):
    """One channel (keyword arguments of setup) for `steps` steps."""
    d, ref = setup(**kw)
    d.step(steps)
    return finish(d, ref, fields)


def run_many(cases, steps=400_000, chunk=4_000):
    """Several channels at once, each on a HIP stream of its own (default
    priority), stepped in turns of `chunk` steps: a 512 x 256 channel leaves
    most of the GPU idle, so independent channels run side by side."""
    import torch
    doms = []
    for kw in cases:
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            doms.append(setup(**kw))
    done = 0
    while done < steps:
        n = min(chunk, steps - done)
        for d, _ in doms:
            d.step(n)
        done += n
        if done % 100_000 == 0:
            doms[0][0].synchronize()
            print(f"  {len(doms)} channels: {done} steps", flush=True)
    for d, _ in doms:
        d.synchronize()
    return [finish(d, ref) for d, ref in doms]
