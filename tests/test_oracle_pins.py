"""Pins of the FP64 oracle against what the paper and the mathematics fix.

These run on the CPU.  Each test names the passage it follows.  Together they
are chosen so that a dropped term, a wrong sign, a wrong index or a
transposed operand anywhere in the oracle's per-cell building blocks fails at
least one of them.
"""
from __future__ import annotations

import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2401_03041_amd import workloads as W
from tests.helpers import oracle_domain

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "appB_stencils.txt")
CS2 = 1.0 / 3.0


def _golden_stencils():
    out = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        name, i, ex, ey, ez, num, den = line.split()
        q = int(name[3:])
        out.setdefault(q, []).append((int(i), (int(ex), int(ey), int(ez)), int(num) / int(den)))
    return out


# ---------------------------------------------------------------------------------------
# Stencils (App. B)
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("q", [7, 15, 19, 27])
def test_stencil_matches_appendix_b(q):
    e, w, opp = O.stencil(q)
    gold = _golden_stencils()[q]
    assert len(gold) == q
    for i, vel, wt in gold:
        assert tuple(e[i]) == vel
        assert w[i] == pytest.approx(wt, abs=1e-15)
    for i in range(q):
        assert tuple(e[opp[i]]) == tuple(-e[i])


@pytest.mark.parametrize("q", [7, 15, 19, 27])
def test_stencil_lattice_moments(q):
    """sum w = 1, sum w e = 0, sum w e e = c_s^2 delta (c_s^2 = 1/3 on all four sets),
    odd moments vanish; fourth-order isotropy holds for Q >= 15 and fails for D3Q7."""
    e, w, _ = O.stencil(q)
    e = e.astype(float)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose((w[:, None] * e).sum(0), 0.0, atol=1e-16)
    M2 = np.einsum("i,ia,ib->ab", w, e, e)
    assert np.allclose(M2, CS2 * np.eye(3), atol=1e-15)
    M3 = np.einsum("i,ia,ib,ic->abc", w, e, e, e)
    assert np.allclose(M3, 0.0, atol=1e-16)
    M4 = np.einsum("i,ia,ib,ic,id->abcd", w, e, e, e, e)
    d = np.eye(3)
    iso = CS2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                      + np.einsum("ad,bc->abcd", d, d))
    if q >= 15:
        assert np.allclose(M4, iso, atol=1e-15)
    else:
        assert not np.allclose(M4, iso, atol=1e-3)


# ---------------------------------------------------------------------------------------
# Equilibria (Sec. 2.2, Eq. lb_thermal)
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("q", [7, 15, 19, 27])
def test_scalar_equilibrium_moments(q):
    """sum h_eq = phi and sum h_eq e = phi u for the phase-field and thermal equilibria."""
    e, w, _ = O.stencil(q)
    rng = np.random.default_rng(q)
    for _ in range(5):
        u = rng.uniform(-0.1, 0.1, 3)
        phi = rng.uniform(0.0, 1.0)
        heq = O.equilibrium(q, 0, phi, u)
        assert heq.sum() == pytest.approx(phi, abs=1e-15)
        assert np.allclose((heq[:, None] * e).sum(0), phi * u, atol=1e-15)


def test_hydro_equilibrium_moments():
    """Incompressible g_eq: sum = p*, first moment = u, second = p* c_s^2 delta + u u."""
    e, w, _ = O.stencil(27)
    rng = np.random.default_rng(3)
    for _ in range(5):
        u = rng.uniform(-0.1, 0.1, 3)
        ps = rng.uniform(-1e-3, 1e-3)
        geq = O.equilibrium(27, 1, ps, u)
        assert geq.sum() == pytest.approx(ps, abs=1e-16)
        assert np.allclose((geq[:, None] * e).sum(0), u, atol=1e-16)
        M2 = np.einsum("i,ia,ib->ab", geq, e, e)
        assert np.allclose(M2, ps * CS2 * np.eye(3) + np.outer(u, u), atol=1e-16)


def test_guo_source_moments():
    """Guo's source in velocity form is defined by its moments: zero mass, first
    moment a, second moment u a + a u (so its second central moments vanish)."""
    e, w, _ = O.stencil(27)
    rng = np.random.default_rng(7)
    for _ in range(5):
        u = rng.uniform(-0.1, 0.1, 3)
        a = rng.uniform(-1e-3, 1e-3, 3)
        S = O.guo_source(u, a)
        assert abs(S.sum()) < 1e-17
        assert np.allclose((S[:, None] * e).sum(0), a, atol=1e-17)
        M2 = np.einsum("i,ia,ib->ab", S, e, e)
        assert np.allclose(M2, np.outer(u, a) + np.outer(a, u), atol=1e-17)


# ---------------------------------------------------------------------------------------
# Central-moment collision (readings R13-R15)
# ---------------------------------------------------------------------------------------
BASES = [(7, 0), (15, 0), (19, 0), (27, 0), (27, 1)]


@pytest.mark.parametrize("q,kind", BASES)
def test_moment_matrix_invertible(q, kind):
    """T(u) stays well conditioned for |u| <= 0.15; at u = 0 its rows are the raw
    lattice moments (row 0 sums, rows 1-3 are the velocity components)."""
    e, _, _ = O.stencil(q)
    rng = np.random.default_rng(q + kind)
    for _ in range(20):
        u = rng.uniform(-1, 1, 3)
        u *= 0.15 / np.linalg.norm(u)
        T, order, tag = O.moment_matrix(q, u, kind)
        assert np.linalg.cond(T) < 1e3
    T0, order, tag = O.moment_matrix(q, np.zeros(3), kind)
    assert np.allclose(T0[0], 1.0)
    assert sorted(order.tolist()).count(1) == 3
    rows1 = [T0[j] for j in range(q) if order[j] == 1]
    for r in rows1:
        assert any(np.array_equal(r, e[:, a]) for a in range(3))


@pytest.mark.parametrize("q,kind", BASES)
def test_equal_rates_reduce_to_bgk_guo(q, kind):
    """All moment rates equal to omega: the central-moment operator is exactly the
    single-relaxation-time operator with the (1 - omega/2) source correction."""
    rng = np.random.default_rng(10 * q + kind)
    for _ in range(10):
        u = rng.uniform(-0.08, 0.08, 3)
        f = rng.uniform(0.0, 0.1, q)
        feq = rng.uniform(0.0, 0.1, q)
        S = rng.uniform(-1e-3, 1e-3, q)
        om = rng.uniform(0.2, 1.9)
        out = O.cm_collide(q, kind, np.full(q, om), u, f, feq, S)
        ref = (1.0 - om) * f + om * feq + (1.0 - 0.5 * om) * S
        assert np.allclose(out, ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("q,kind", BASES)
def test_equilibrium_is_fixed_point(q, kind):
    """f = f_eq and no source stays unchanged for arbitrary, unequal rates."""
    rng = np.random.default_rng(q * 7 + kind)
    u = rng.uniform(-0.08, 0.08, 3)
    feq = O.equilibrium(q, kind, 0.4, u)
    rates = rng.uniform(0.3, 1.9, q)
    out = O.cm_collide(q, kind, rates, u, feq, feq, np.zeros(q))
    assert np.allclose(out, feq, atol=1e-15)


@pytest.mark.parametrize("q,kind", BASES)
def test_rate_of_one_projects_moment_onto_equilibrium(q, kind):
    """With every rate equal to one the post-collision state is f_eq + S/2 whatever f is."""
    rng = np.random.default_rng(q * 11 + kind)
    u = rng.uniform(-0.08, 0.08, 3)
    f = rng.uniform(0.0, 0.1, q)
    feq = rng.uniform(0.0, 0.1, q)
    S = rng.uniform(-1e-3, 1e-3, q)
    out = O.cm_collide(q, kind, np.ones(q), u, f, feq, S)
    assert np.allclose(out, feq + 0.5 * S, atol=1e-15)


def test_hydro_rates_separate_shear_and_bulk():
    """Hydrodynamic basis: the trace x^2+y^2+z^2 and the shear moments are separate rows,
    so changing only the shear rate leaves the trace of the central second moment
    exactly at its rate-one value, and changing only the bulk rate leaves the
    deviatoric part there."""
    rng = np.random.default_rng(5)
    e, w, _ = O.stencil(27)
    u = rng.uniform(-0.05, 0.05, 3)
    f = rng.uniform(0.0, 0.1, 27)
    feq = rng.uniform(0.0, 0.1, 27)
    S = np.zeros(27)
    T, order, tag = O.moment_matrix(27, u, 1)
    c = e - u

    def second(v):
        return np.einsum("i,ia,ib->ab", v, c, c)

    base = O.cm_collide(27, 1, np.ones(27), u, f, feq, S)
    shear = np.where((tag == 2) | (tag == 3), 1.4, 1.0)
    out = O.cm_collide(27, 1, shear, u, f, feq, S)
    assert np.trace(second(out)) == pytest.approx(np.trace(second(base)), abs=1e-15)
    dev = second(out) - second(base)
    pre = second(f) - second(feq)
    # deviatoric part relaxed with rate 1.4 instead of 1: difference = (1 - 1.4) * dev(pre)
    dpre = pre - np.trace(pre) / 3 * np.eye(3)
    assert np.allclose(dev, -0.4 * dpre, atol=1e-14)
    bulk = np.where(tag == 1, 1.6, 1.0)
    out = O.cm_collide(27, 1, bulk, u, f, feq, S)
    dd = second(out) - second(base)
    assert np.allclose(dd, -0.6 * np.trace(pre) / 3 * np.eye(3), atol=1e-14)


# ---------------------------------------------------------------------------------------
# Isotropic finite differences (reading R17)
# ---------------------------------------------------------------------------------------
def test_isotropic_stencils_exact_on_polynomials():
    """Gradient exact on linear fields, Laplacian exact on quadratics (interior cells)."""
    cfg = W.make(shape=(9, 9, 9))
    d = O.OracleDomain(cfg)
    z, y, x = np.meshgrid(np.arange(9.0), np.arange(9.0), np.arange(9.0), indexing="ij")
    lin = 0.3 * x - 1.7 * y + 2.2 * z + 5.0
    g, l = d.iso_grad_lap(lin, 4, 4, 4)
    assert np.allclose(g, [0.3, -1.7, 2.2], atol=1e-13)
    assert l == pytest.approx(0.0, abs=1e-13)
    quad = 0.5 * x * x + 2.0 * y * y - 0.25 * z * z + 0.7 * x * y - 0.1 * y * z
    g, l = d.iso_grad_lap(quad, 4, 5, 3)
    assert np.allclose(g, [4 + 0.7 * 5, 2 * 2 * 5 + 0.7 * 4 - 0.1 * 3, -0.5 * 3 - 0.1 * 5], atol=1e-12)
    assert l == pytest.approx(1.0 + 4.0 - 0.5, abs=1e-12)


def test_wall_ghosts_are_method_of_images():
    """At a wall row the stencils see the field continued across the wall plane
    y = -1/2: evenly for phi (mirror, zero normal derivative) and oddly about T_w for
    the temperature (Dirichlet).  Compare with the same stencils on the explicitly
    continued field in a periodic box of twice the height."""
    nx, ny, nz = 5, 6, 4
    rng = np.random.default_rng(3)
    f = rng.uniform(0, 1, (nz, ny, nx))
    tw_b, tw_t = 0.3, 0.8
    walls = O.OracleDomain(W.make(shape=(nx, ny, nz), periodic_y=False, t_wall_bot=tw_b, t_wall_top=tw_t))
    per = O.OracleDomain(W.make(shape=(nx, 2 * ny, nz)))
    even = np.concatenate([f, f[:, ::-1, :]], axis=1)            # rows ny..2ny-1 mirror the fluid rows
    odd_b = np.concatenate([f, 2 * tw_b - f[:, ::-1, :]], axis=1)  # continuation below the bottom wall
    odd_t = np.concatenate([f, 2 * tw_t - f[:, ::-1, :]], axis=1)  # continuation above the top wall
    for x, z in ((0, 0), (2, 3), (4, 1)):
        for y in (0, ny - 1):
            g1, l1 = walls.iso_grad_lap(f, x, y, z, "mirror")
            g2, l2 = per.iso_grad_lap(even, x, y, z, "mirror")
            assert np.allclose(g1, g2, atol=1e-14) and l1 == pytest.approx(l2, abs=1e-13)
            g1, l1 = walls.iso_grad_lap(f, x, y, z, "dirichlet")
            g2, l2 = per.iso_grad_lap(odd_b if y == 0 else odd_t, x, y, z, "mirror")
            assert np.allclose(g1, g2, atol=1e-13) and l1 == pytest.approx(l2, abs=1e-12)


# ---------------------------------------------------------------------------------------
# Heat source (Eq. HeatSource, reading R10)
# ---------------------------------------------------------------------------------------
def test_heat_source_integral_and_cutoff():
    """The lattice sum of the Gaussian source equals its integral Q (pi w^2/2)^(3/2)
    (Poisson summation: exact up to exp(-pi^2 w^2/2)); the source is Q at its centre
    (so the cut-off keeps the inside, not the outside) and zero beyond d_s."""
    cfg = W.make(shape=(4, 4, 4))
    d = O.OracleDomain(cfg)
    Q, w = 0.8, 6.0
    d.set_heat_sources([(Q, 0.3, -0.2, 0.1, w, 0.0)])
    r = np.arange(-40, 41)
    tot = 0.0
    for zz in r:
        for yy in r:
            tot += sum(d.heat_source(xx, yy, zz) for xx in r)
    assert tot == pytest.approx(Q * (np.pi * w * w / 2) ** 1.5, rel=1e-12)
    d.set_heat_sources([(Q, 0.0, 0.0, 0.0, w, 5.0)])
    assert d.heat_source(0.0, 0.0, 0.0) == pytest.approx(Q, rel=1e-15)
    assert d.heat_source(5.01, 0.0, 0.0) == 0.0
    assert d.heat_source(0.0, 4.99, 0.0) > 0.0


# ---------------------------------------------------------------------------------------
# Thermal LB special cases (Eq. lb_thermal, Eq. thlbm-tau, readings R1, R11)
# ---------------------------------------------------------------------------------------
def _uniform_phase(cfg):
    nx, ny, nz = cfg["shape"]
    return np.ones((nz, ny, nx))


@pytest.mark.parametrize("q", [7, 15, 19, 27])
def test_thermal_unit_rate_is_weighted_neighbour_average(q):
    """kappa = c_s^2/2 gives omega_T = 1, so at rest the new temperature is the
    weighted average sum_i w_i T(x - e_i); for D3Q7 the mean of the six neighbours."""
    cfg = W.make(shape=(6, 5, 4), q_thermal=q, kappa_h=1.0 / 6.0, kappa_l=1.0 / 6.0)
    rng = np.random.default_rng(q)
    T0 = rng.uniform(0, 1, (4, 5, 6))
    d = oracle_domain(cfg, phi=_uniform_phase(cfg), T=T0)
    e, w, _ = O.stencil(q)
    for _ in range(2):
        d.step(1)
        T1 = d.get_field("T")
        ref = np.zeros_like(T0)
        for i in range(q):
            ref += w[i] * np.roll(T0, shift=(e[i, 2], e[i, 1], e[i, 0]), axis=(0, 1, 2))
        assert np.allclose(T1, ref, atol=1e-15)
        T0 = T1
    if q == 7:
        nb = sum(np.roll(T0, s, ax) for ax in range(3) for s in (1, -1)) / 6.0
        d.step(1)
        assert np.allclose(d.get_field("T"), nb, atol=1e-15)


@pytest.mark.parametrize("thermal,q", [("lb", 7), ("lb", 27), ("rk2", 7), ("rk4", 7)])
def test_uniform_heat_source_adds_q_per_step(thermal, q):
    """A spatially uniform source raises T by exactly Q per step (sum_i w_i = 1 for
    the LB; R(T) = Q for RK)."""
    cfg = W.make(shape=(4, 4, 4), q_thermal=q, thermal=thermal, kappa_h=0.1, kappa_l=0.1)
    Q = 3e-3
    d = oracle_domain(cfg, phi=_uniform_phase(cfg), T=np.full((4, 4, 4), 0.25))
    d.set_heat_sources([(Q, 2.0, 2.0, 2.0, 1e9, 0.0)])
    prev = d.get_field("T")
    for _ in range(4):
        d.step(1)
        cur = d.get_field("T")
        if not (thermal == "lb" and _ == 0):
            assert np.allclose(cur - prev, Q, atol=1e-15)
        prev = cur


@pytest.mark.parametrize("thermal,q", [("lb", 7), ("lb", 15), ("lb", 19), ("lb", 27), ("rk2", 7), ("rk4", 7)])
def test_dirichlet_walls_keep_linear_profile(thermal, q):
    """Conduction between walls at T_b and T_t: the linear profile through the wall
    values at y = -1/2 and y = ny - 1/2 is an exact fixed point (anti-bounce-back for
    the LB, ghost 2 T_w - T for the finite differences)."""
    ny = 12
    cfg = W.make(shape=(3, ny, 2), periodic_y=False, q_thermal=q, thermal=thermal, kappa_h=0.15,
                 kappa_l=0.15, t_wall_bot=1.0, t_wall_top=3.0, t_init={"kind": "conduction"})
    d = oracle_domain(cfg, phi=_uniform_phase(cfg))
    T0 = d.get_field("T")
    d.step(60)
    assert np.allclose(d.get_field("T"), T0, atol=1e-13)
    assert np.allclose(d.get_field("ux"), 0.0, atol=1e-15)


@pytest.mark.parametrize("thermal", ["rk2", "rk4"])
def test_rk_mode_amplification_is_stability_polynomial(thermal):
    """On one Fourier mode with uniform u the stage operator R is linear with symbol
    z = kappa L(k) - i u.G(k) (L, G the symbols of the isotropic D3Q27 stencils), so one
    step multiplies the mode by 1 + z + z^2/2 (RK2, midpoint) or the degree-4 Taylor
    polynomial (RK4)."""
    n = (8, 6, 4)
    kap = 0.07
    u = np.array([0.03, -0.02, 0.01])
    cfg = W.make(shape=n, thermal=thermal, kappa_h=kap, kappa_l=kap, u_init=tuple(u))
    k = 2 * np.pi * np.array([1.0 / n[0], 2.0 / n[1], 1.0 / n[2]])
    z_, y_, x_ = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    phase = k[0] * x_ + k[1] * y_ + k[2] * z_
    T0 = np.cos(phase)
    d = oracle_domain(cfg, phi=_uniform_phase(cfg), T=T0)
    e, w, _ = O.stencil(27)
    ke = e @ k
    L = (2.0 / CS2) * np.sum(w * (np.cos(ke) - 1.0))
    G = (1.0 / CS2) * (w[:, None] * e * np.sin(ke)[:, None]).sum(0)
    z = kap * L - 1j * (u @ G)
    M = 1 + z + z * z / 2
    if thermal == "rk4":
        M += z ** 3 / 6 + z ** 4 / 24
    d.step(1)
    ref = np.real(M * np.exp(1j * phase))
    assert np.allclose(d.get_field("T"), ref, atol=1e-14)
    assert np.allclose(d.get_field("ux"), u[0], atol=1e-15)


# ---------------------------------------------------------------------------------------
# Invariants of the coupled step
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("walls", [False, True])
def test_phase_mass_and_heat_conserved(walls):
    """sum phi is conserved to 1e-12 (periodic and bounce-back walls); without
    sources and with periodic walls sum T is conserved as well."""
    cfg = W.make(shape=(16, 14, 12), periodic_y=not walls, rho_h=1.0, rho_l=0.1, nu_h=0.1, nu_l=0.02,
                 sigma_ref=2e-3, sigma_t=-2e-4, xi=4.0, droplets=[(7.0, 6.5 if not walls else 3.0, 5.5, 4.0)],
                 t_init={"kind": "linear", "axis": 0, "origin": 8.0, "slope": 0.01, "value": 0.5})
    d = oracle_domain(cfg)
    m0, _ = d.reduce()
    T0 = d.get_field("T").sum()
    d.step(30)
    m1, _ = d.reduce()
    assert abs(m1 - m0) / m0 < 1e-12
    if not walls:
        assert abs(d.get_field("T").sum() - T0) / abs(T0) < 1e-12
    f = d.fields()
    assert all(np.all(np.isfinite(v)) for v in f.values())
    assert np.max(np.abs(f["ux"])) > 0.0


def test_uniform_state_is_fixed_point():
    """Uniform phase, temperature, velocity and zero pressure stay unchanged."""
    cfg = W.make(shape=(5, 4, 3), rho_h=1.0, rho_l=0.2, sigma_ref=1e-3, sigma_t=1e-4,
                 u_init=(0.02, -0.01, 0.005), t_init={"kind": "uniform", "value": 0.3})
    d = oracle_domain(cfg, phi=np.full((3, 4, 5), 0.7))
    f0 = d.fields()
    d.step(10)
    f1 = d.fields()
    for k in f0:
        assert np.allclose(f1[k], f0[k], atol=1e-15), k


def test_centred_droplet_symmetry():
    """A droplet at the centre of a periodic cube under uniform T keeps the mirror and
    axis-permutation symmetries of the cube (catches wrong velocity indices,
    opposites or moment rows)."""
    n = 16
    c = (n - 1) / 2.0
    cfg = W.make(shape=(n, n, n), rho_h=1.0, rho_l=0.1, nu_h=0.1, nu_l=0.02, sigma_ref=2e-3,
                 xi=3.0, droplets=[(c, c, c, 4.0)], t_init={"kind": "uniform", "value": 0.0})
    d = oracle_domain(cfg)
    d.step(8)
    phi, ux, uy, uz, p = (d.get_field(k) for k in ("phi", "ux", "uy", "uz", "p"))
    # mirror x -> 15 - x, arrays are (z, y, x)
    mir = lambda a: a[:, :, ::-1]
    assert np.allclose(mir(phi), phi, atol=1e-14)
    assert np.allclose(mir(ux), -ux, atol=1e-14)
    assert np.allclose(mir(uy), uy, atol=1e-14)
    # permutation x <-> y
    assert np.allclose(np.swapaxes(phi, 1, 2), phi, atol=1e-14)
    assert np.allclose(np.swapaxes(ux, 1, 2), uy, atol=1e-14)
    assert np.allclose(np.swapaxes(p, 0, 2), p, atol=1e-14)
    assert np.max(np.abs(ux)) > 1e-9
