"""Adjoint of the temperature warm-up (thermal LB or RK, phi and u held) through the
C interface, against gradients the oracle gives by definition: the warm-up is
linear in the source amplitudes and the wall temperatures once the initial T is
zero, so dL/dQ_k is L with Q = e_k (all else zero) and dL/dT_w at one column is
L with a unit wall temperature there."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from paper_2401_03041_amd import workloads as W
from tests.helpers import gpu_domain

pytestmark = pytest.mark.gpu


def _case(q, precision, thermal="lb", nx=12, ny=10, nz=6, periodic_y=False):
    """Inputs generated here and given to both sides: a smooth phase field in
    [0.05, 0.95], a held velocity field and random loss weights."""
    rng = np.random.default_rng(7)
    cfg = W.make(shape=(nx, ny, nz), periodic_y=periodic_y, precision=precision, q_thermal=q, thermal=thermal,
                 rho_l=0.5, xi=3.0, contact_angle_bot=70.0,
                 kappa_h=0.25, kappa_l=0.1, t_wall_bot=0.3, t_wall_top=0.8,
                 heat_sources=[(0.02, 4.0, 2.0, 3.0, 3.0, 0.0), (0.01, 9.5, 7.0, 1.0, 2.0, 3.7)])
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    phi = 0.5 + 0.45 * np.sin(2 * np.pi * x / nx) * np.cos(np.pi * (y + 0.5) / ny) * np.cos(2 * np.pi * z / nz)
    u = [0.02 * np.sin(2 * np.pi * (x / nx + 0.3 * k)) * np.cos(np.pi * (y + 0.5) / ny) for k in range(3)]
    m = rng.uniform(-1.0, 1.0, (nz, ny, nx))
    return cfg, phi, u, m


def _oracle_loss(cfg, phi, u, m, steps, sources, tw_bot, tw_top):
    d = O.OracleDomain(dict(cfg, t_wall_bot=0.0, t_wall_top=0.0))
    d.set_field("phi", phi)
    for name, comp in zip(("ux", "uy", "uz"), u):
        d.set_field(name, comp)
    d.set_field("T", np.zeros_like(m))
    d.set_heat_sources(sources)
    d.set_wall_temperature(0, tw_bot)
    d.set_wall_temperature(1, tw_top)
    d.initialize()
    d.warm_temperature(steps, 0.0, steps + 1)
    L = float(np.sum(m * d.get_field("T")))
    d.close()
    return L


def _oracle_gradient(cfg, phi, u, m, steps, h=1e-4):
    """dL/dQ_k and dL/dT_w exactly (the loss at unit inputs), dL/d(x, y, z)_k by
    central differences of Q_k L(unit amplitude k) in the source position (no
    lattice cell lies within h of a cut-off sphere here)."""
    nx, ny, nz = cfg["shape"]
    zero = np.zeros((nz, nx))
    src = [list(s) for s in cfg["heat_sources"]]
    dq = []
    for k in range(len(src)):
        unit = [[1.0 if j == k else 0.0] + s[1:] for j, s in enumerate(src)]
        row = [_oracle_loss(cfg, phi, u, m, steps, unit, zero, zero)]
        for ax in range(3):
            lp, lm = [list(s) for s in unit], [list(s) for s in unit]
            lp[k][1 + ax] += h
            lm[k][1 + ax] -= h
            dl = _oracle_loss(cfg, phi, u, m, steps, lp, zero, zero) - \
                _oracle_loss(cfg, phi, u, m, steps, lm, zero, zero)
            row.append(src[k][0] * dl / (2 * h))
        dq.append(row)
    off = [[0.0] + s[1:] for s in src]
    tw = [np.zeros((nz, nx)), np.zeros((nz, nx))]
    for wall in (0, 1):
        for iz in range(nz):
            for ix in range(nx):
                e = np.zeros((nz, nx))
                e[iz, ix] = 1.0
                args = (e, zero) if wall == 0 else (zero, e)
                tw[wall][iz, ix] = _oracle_loss(cfg, phi, u, m, steps, off, *args)
    return np.array(dq), tw[0], tw[1]


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("precision,q,thermal", [("fp64", 7, "lb"), ("fp64", 19, "lb"), ("fp32", 7, "lb"),
                                                 ("fp32", 27, "lb"), ("fp64", 7, "rk2"), ("fp64", 7, "rk4"),
                                                 ("fp32", 7, "rk4"), ("fp16", 15, "lb")])
def test_thermal_adjoint_matches_oracle_gradient(precision, q, thermal):
    """Walls (70-degree bottom wall), two heaters (one cut off), conductivity
    ratio 2.5 over a smooth phase field, a held velocity field, random loss weights, 25
    updates of the LB or RK scheme: dL/dQ and dL/dT_w
    of both walls within 1e-11 (FP64) or 1e-5 (FP32) of the oracle's, and the
    source-position gradients within 1e-7 (FP64; the oracle's are central
    differences) or 1e-5 (FP32)."""
    steps = 25
    cfg, phi, u, m = _case(q, precision, thermal)
    g = gpu_domain(cfg, phi=phi, u=u, T=np.full(m.shape, 0.4))
    phi_before = g.get_field("phi")
    dq, tb, tt = g.thermal_adjoint(steps, m)
    oq, ob, ot = _oracle_gradient(cfg, phi, u, m, steps)
    tol = 1e-11 if precision == "fp64" else 1e-5  # FP16 PDFs: the adjoint itself runs in FP32
    errs = {"Q": _rel(dq[:, 0], oq[:, 0]), "Tw_bot": _rel(tb, ob), "Tw_top": _rel(tt, ot)}
    pos = _rel(dq[:, 1:], oq[:, 1:])
    print(precision, q, thermal, errs, "position", pos, dq, oq)
    assert all(v < tol for v in errs.values()), errs
    assert pos < (1e-7 if precision == "fp64" else 1e-5), pos
    # the state is untouched and a second call gives the same gradients
    dq2, tb2, tt2 = g.thermal_adjoint(steps, m)
    assert np.array_equal(dq, dq2) and np.array_equal(tb, tb2) and np.array_equal(tt, tt2)
    assert np.array_equal(g.get_field("phi"), phi_before)


@pytest.mark.parametrize("thermal,shape,periodic", [("lb", (12, 10, 6), True), ("rk4", (12, 10, 6), True),
                                                    ("lb", (8, 2, 4), False), ("rk2", (8, 2, 4), False),
                                                    ("rk4", (9, 7, 1), False)])
def test_thermal_adjoint_periodic_and_two_rows(thermal, shape, periodic):
    """Periodic y (no wall gradients: exactly zero), a two-row channel, the
    smallest with walls (every cell next to a wall), and a channel one plane
    thick (z wraps onto itself), FP64, against the oracle's unit-input
    gradients."""
    steps = 20
    cfg, phi, u, m = _case(7, "fp64", thermal, *shape, periodic_y=periodic)
    g = gpu_domain(cfg, phi=phi, u=u)
    dq, tb, tt = g.thermal_adjoint(steps, m)
    oq, ob, ot = _oracle_gradient(cfg, phi, u, m, steps)
    def close(a, b):
        return np.max(np.abs(a - b)) <= 1e-11 * np.max(np.abs(b))

    assert close(dq[:, 0], oq[:, 0]), (dq, oq)
    if periodic:
        assert not tb.any() and not tt.any()
    else:
        assert close(tb, ob) and close(tt, ot), (tb, ob, tt, ot)


@pytest.mark.parametrize("thermal", ["lb", "rk4"])
def test_thermal_adjoint_against_gpu_forward(thermal):
    """On a ragged 70 x 22 x 37 channel (two tiles in x, several in y and z, each
    with a ragged end) over 200 updates the adjoint's dL/dQ equals the loss of
    the GPU's own warm-up at unit source amplitude from T = 0 (the map is
    linear), in FP64; and the wall gradients sum to the loss of a unit
    temperature on the whole wall."""
    nx, ny, nz = 70, 22, 37
    cfg = W.make(shape=(nx, ny, nz), periodic_y=False, q_thermal=15, thermal=thermal, kappa_h=0.2, kappa_l=0.1,
                 rho_l=0.5,
                 xi=4.0, droplets=[(30.3, 6.7, 4.1, 4.5)],
                 heat_sources=[(0.02, 40.0, 6.0, 7.0, 6.0, 8.0), (0.01, 12.0, 15.0, 2.0, 3.0, 0.0)])
    rng = np.random.default_rng(3)
    m = rng.uniform(0.0, 1.0, (nz, ny, nx))
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    u = [0.01 * np.cos(2 * np.pi * x / nx), 0.0 * x, 0.01 * np.sin(2 * np.pi * z / nz)]
    g = gpu_domain(cfg, u=u)
    dq, tb, tt = g.thermal_adjoint(200, m)

    def loss(sources, wall_bot, wall_top):
        c = dict(cfg, heat_sources=sources, t_wall_bot=wall_bot, t_wall_top=wall_top)
        d = gpu_domain(c, u=u, T=np.zeros_like(m))
        d.warm_temperature(200, 0.0, 1000)
        return float(np.sum(m * d.get_field("T")))

    src = [list(s) for s in cfg["heat_sources"]]
    for k in range(2):
        unit = [[1.0 if j == k else 0.0] + s[1:] for j, s in enumerate(src)]
        ref = loss(unit, 0.0, 0.0)
        assert abs(dq[k, 0] - ref) <= 1e-11 * abs(ref), (k, dq[k, 0], ref)
    off = [[0.0] + s[1:] for s in src]
    for wall, grad in ((0, tb), (1, tt)):
        ref = loss(off, 1.0 if wall == 0 else 0.0, 1.0 if wall == 1 else 0.0)
        assert abs(grad.sum() - ref) <= 1e-11 * abs(ref), (wall, grad.sum(), ref)


def test_thermal_warmup_autograd():
    """The torch wrapper: backward through a scalar loss gives the adjoint's
    gradients, and a central difference of the wrapped forward in the first
    source's x agrees with its x gradient (FP64)."""
    import torch

    from paper_2401_03041_amd import tcplb
    nx, ny, nz = 16, 12, 8
    cfg = W.make(shape=(nx, ny, nz), periodic_y=False, q_thermal=7, kappa_h=0.2, kappa_l=0.1, rho_l=0.5,
                 xi=3.0, droplets=[(7.3, 4.2, 3.7, 3.0)], t_wall_top=0.5,
                 heat_sources=[(0.03, 6.0, 3.0, 4.0, 3.0, 0.0)])
    g = gpu_domain(cfg)
    f = tcplb.thermal_warmup(g, 40)
    m = torch.from_numpy(np.random.default_rng(5).uniform(0.0, 1.0, (nz, ny, nx)))
    src = torch.tensor([[0.03, 6.0, 3.0, 4.0, 3.0, 0.0]], dtype=torch.float64, requires_grad=True)
    twb = torch.zeros((nz, nx), dtype=torch.float64, requires_grad=True)
    twt = torch.full((nz, nx), 0.5, dtype=torch.float64, requires_grad=True)
    loss = (f(src, twb, twt) * m).sum()
    loss.backward()
    dsrc, dbot, dtop = g.thermal_adjoint(40, m.numpy())
    assert np.array_equal(src.grad[:, :4].numpy(), dsrc)
    assert np.array_equal(twb.grad.numpy(), dbot) and np.array_equal(twt.grad.numpy(), dtop)
    h = 1e-4
    with torch.no_grad():
        sp, sm = src.clone(), src.clone()
        sp[0, 1] += h
        sm[0, 1] -= h
        fd = float(((f(sp, twb, twt) - f(sm, twb, twt)) * m).sum()) / (2 * h)
    assert abs(fd - float(src.grad[0, 1])) <= 1e-6 * abs(fd), (fd, float(src.grad[0, 1]))


def test_thermal_warmup_backward_uses_its_own_inputs():
    """Two forward calls with different heaters (one source, then two) before
    the backward pass of the first: its gradients are those of its own inputs,
    not of the heaters the domain holds when backward runs."""
    import torch

    from paper_2401_03041_amd import tcplb
    nx, ny, nz = 16, 12, 8
    cfg = W.make(shape=(nx, ny, nz), periodic_y=False, q_thermal=7, kappa_h=0.2, kappa_l=0.1, rho_l=0.5,
                 xi=3.0, droplets=[(7.3, 4.2, 3.7, 3.0)], heat_sources=[])
    g = gpu_domain(cfg)
    f = tcplb.thermal_warmup(g, 30)
    m = torch.from_numpy(np.random.default_rng(11).uniform(0.0, 1.0, (nz, ny, nx)))
    twb = torch.zeros((nz, nx), dtype=torch.float64, requires_grad=True)
    twt = torch.full((nz, nx), 0.5, dtype=torch.float64, requires_grad=True)
    s1 = torch.tensor([[0.03, 6.0, 3.0, 4.0, 3.0, 0.0]], dtype=torch.float64, requires_grad=True)
    s2 = torch.tensor([[0.05, 11.0, 6.0, 2.0, 2.5, 0.0], [0.02, 3.0, 8.0, 5.0, 3.5, 0.0]], dtype=torch.float64,
                      requires_grad=True)
    l1 = (f(s1, twb, twt) * m).sum()
    l2 = (f(s2, twb * 0.5, twt) * m).sum()
    l1.backward()
    g1 = s1.grad.clone()
    l2.backward()
    g2 = s2.grad.clone()
    # references: the adjoint called directly on each call's own heaters (phi and
    # u are the held fields of the snapshot both calls start from)
    for src, grad in ((s1, g1), (s2, g2)):
        g.set_heat_sources(src.detach().numpy().tolist())
        dsrc, _, _ = g.thermal_adjoint(30, m.numpy())
        assert np.array_equal(grad[:, :4].numpy(), dsrc), (grad, dsrc)


def test_adjoint_gradient_step_moves_heater_towards_target():
    """The gradients drive a design search: L = sum (T - T*)^2 over a probe
    region, T* the warm-up temperature of a heater at x = 20.  Starting from
    x = 14 and stepping against the sign of dL/dx (the step halved whenever that
    sign flips), the heater's x ends within a quarter cell of 20."""
    import torch

    from paper_2401_03041_amd import tcplb
    nx, ny, nz = 32, 12, 8
    cfg = W.make(shape=(nx, ny, nz), periodic_y=False, thermal="lb", kappa_h=0.2, kappa_l=0.2,
                 heat_sources=[(0.05, 14.0, 5.0, 4.0, 3.0, 0.0)])
    g = gpu_domain(cfg)
    f = tcplb.thermal_warmup(g, 150)
    twb = torch.zeros((nz, nx), dtype=torch.float64)
    twt = torch.zeros((nz, nx), dtype=torch.float64)
    with torch.no_grad():
        target = f(torch.tensor([[0.05, 20.0, 5.0, 4.0, 3.0, 0.0]], dtype=torch.float64), twb, twt).clone()
    mask = torch.zeros((nz, ny, nx), dtype=torch.float64)
    mask[:, 2:9, 12:28] = 1.0
    src = torch.tensor([[0.05, 14.0, 5.0, 4.0, 3.0, 0.0]], dtype=torch.float64, requires_grad=True)
    step, last_sign = 2.0, 0.0
    for it in range(30):
        loss = (((f(src, twb, twt) - target) * mask) ** 2).sum()
        src.grad = None
        loss.backward()
        sign = float(np.sign(float(src.grad[0, 1])))
        if last_sign and sign != last_sign:
            step *= 0.5
        last_sign = sign
        with torch.no_grad():
            src[0, 1] -= sign * step
    x = float(src.detach()[0, 1])
    print("heater x", x, "loss", float(loss.detach()))
    assert abs(x - 20.0) < 0.25


@pytest.mark.parametrize("thermal", ["lb", "rk4"])
def test_thermal_adjoint_full_size(thermal):
    """The 512^3 droplet block in FP32, as bench.py's thermal-adjoint legs run it,
    with a heater of width 32 at its centre: after 10 updates the adjoint's
    dL/dQ for random loss weights equals the loss of the GPU's own warm-up at
    unit amplitude from T = 0 (the map is linear) within the FP32 bar 1e-5."""
    import torch

    n = 512
    cfg = dict(W.droplet_block(n=n, precision="fp32"), thermal=thermal,
               heat_sources=[(1.0, 256.0, 256.0, 256.0, 32.0, 0.0)])
    m = np.random.default_rng(5).uniform(0.0, 1.0, (n, n, n))
    g = gpu_domain(cfg)
    dq, _, _ = g.thermal_adjoint(10, m)
    g.close()
    del g
    torch.cuda.empty_cache()
    f = gpu_domain(cfg, T=np.zeros((n, n, n)))
    f.warm_temperature(10, 0.0, 11)
    loss = float(np.sum(m * f.get_field("T")))
    f.close()
    print(thermal, "dL/dQ", dq[0, 0], "loss at unit amplitude", loss, flush=True)
    assert loss > 1e5  # the heater adds (pi w^2 / 2)^(3/2) = 6.4e4 to sum T per update
    assert abs(dq[0, 0] - loss) <= 1e-5 * abs(loss)
