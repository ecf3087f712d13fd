// adjoint_math.hpp -- per-cell forward maps of the three updates of a coupled
// step and their vector-Jacobian products (reverse mode), written on plain
// arrays so that the reverse kernels can recompute a cell's update from the
// stored state and run it backwards.
//
// Each forward map takes the values the update pulls or reads (actual PDF
// values, not the deviation form they may be stored in) and returns the
// post-collision PDFs and the cell's new field value; the VJP takes the
// adjoints of those outputs and returns the adjoints of the inputs.  The maps
// are the ones the forward kernels evaluate:
//  - phase field (Eq. lb_interface with the counter-term of Eq. phasefieldforce
//    as a source, first-order central moments relaxed with omega_phi, all
//    higher ones with rate one);
//  - hydrodynamics (Sec. 2.1-2.2: forces F_s + F_b + F_p + F_mu with sigma(T),
//    Guo source, the five deviatoric second central moments relaxed with
//    omega(phi), the trace with omega_bulk, the rest with rate one);
//  - thermal LB (Eq. lb_thermal: first-order central moments relaxed with
//    omega_T(phi), source w_i q after the collision).
// In the phase-field and thermal maps the collision leaves f_eq + S/2 + D(u) v
// with v the relaxed first-order central moment of f - f_eq + S/2 and D(u)
// the inverse transform restricted to those moments (FirstOrder<Q>); D is
// linear in v and polynomial in u, and its derivative in u is taken in
// forward mode with dual numbers.  In the hydrodynamic map the inverse
// transform of the six relaxed second-order moments is a tensor product of
// 1-D columns (Axis1D); its transpose and its u-derivative are contractions
// with the same columns.
#pragma once

#include "lattice.hpp"

namespace tcp {

// ---- dual numbers (value, derivative along one direction) -------------------
template <typename R>
struct Dual {
    R v, d;
    __host__ __device__ constexpr Dual() : v(0), d(0) {}
    __host__ __device__ constexpr Dual(R a, R b) : v(a), d(b) {}
    __host__ __device__ constexpr Dual(int a) : v(R(a)), d(0) {}
    __host__ __device__ constexpr Dual(double a) : v(R(a)), d(0) {}
    __host__ __device__ constexpr Dual(float a) : v(R(a)), d(0) {}
};
template <typename R>
__host__ __device__ __forceinline__ Dual<R> operator+(Dual<R> a, Dual<R> b) { return {a.v + b.v, a.d + b.d}; }
template <typename R>
__host__ __device__ __forceinline__ Dual<R> operator-(Dual<R> a, Dual<R> b) { return {a.v - b.v, a.d - b.d}; }
template <typename R>
__host__ __device__ __forceinline__ Dual<R> operator-(Dual<R> a) { return {-a.v, -a.d}; }
template <typename R>
__host__ __device__ __forceinline__ Dual<R> operator*(Dual<R> a, Dual<R> b)
{
    return {a.v * b.v, a.d * b.v + a.v * b.d};
}

// sum_i a_i d/du_b [D(u) v]_i for b = 0, 1, 2 (v held)
template <int Q, typename R>
__host__ __device__ __forceinline__ void first_order_du(const R u[3], const R v[3], const R a[Q], R out[3])
{
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        Dual<R> ud[3], vd[3], dd[Q];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            ud[k] = Dual<R>(u[k], R(k == b ? 1 : 0));
            vd[k] = Dual<R>(v[k], R(0));
        }
        FirstOrder<Q, Dual<R>>::apply(ud, vd, dd);
        R s = R(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) s += a[i] * dd[i].d;
        out[b] = s;
    }
}

// s_b = sum_i a_i D_ib(u): the transpose of D applied to a
template <int Q, typename R>
__host__ __device__ __forceinline__ void first_order_t(const R u[3], const R a[Q], R s[3])
{
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const R unit[3] = {R(b == 0), R(b == 1), R(b == 2)};
        R d[Q];
        FirstOrder<Q, R>::apply(u, unit, d);
        R acc = R(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) acc += a[i] * d[i];
        s[b] = acc;
    }
}

// weighted moments of an adjoint vector: A0 = sum a_i w_i, A1_b = sum a_i w_i e_ib,
// A2_bc = sum a_i w_i e_ib e_ic
template <int Q, typename R>
__host__ __device__ __forceinline__ void weighted_moments(const R a[Q], R &A0, R A1[3], R A2[3][3])
{
    A0 = R(0);
    for (int b = 0; b < 3; ++b) {
        A1[b] = R(0);
        for (int c = 0; c < 3; ++c) A2[b][c] = R(0);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const R wa = R(weight<Q>(i)) * a[i];
        A0 += wa;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            if (!vel<Q>(i, b)) continue;
            A1[b] += R(vel<Q>(i, b)) * wa;
#pragma unroll
            for (int c = 0; c < 3; ++c)
                if (vel<Q>(i, c)) A2[b][c] += R(vel<Q>(i, b) * vel<Q>(i, c)) * wa;
        }
    }
}

// ============================================================================
// phase field (K1)
// ============================================================================
struct PfCoef {
    double omega_phi, inv_xi, eps2;
};

// h: pulled PDFs; G: isotropic gradient of phi^n; u: u^n.  Writes h* and
// returns phi^{n+1} = sum h.
template <int Q, typename R>
__host__ __device__ __forceinline__ R pf_forward(const PfCoef &c, const R h[Q], const R G[3], const R u[3], R hs[Q])
{
    R phi = R(0), j[3] = {R(0), R(0), R(0)};
    for (int i = 0; i < Q; ++i) {
        phi += h[i];
        for (int b = 0; b < 3; ++b)
            if (vel<Q>(i, b)) j[b] += R(vel<Q>(i, b)) * h[i];
    }
    const R inv = R(1) / sqrt(G[0] * G[0] + G[1] * G[1] + G[2] * G[2] + R(c.eps2));
    const R lam = R(4) * phi * (R(1) - phi) * R(c.inv_xi);
    const R F[3] = {lam * inv * G[0], lam * inv * G[1], lam * inv * G[2]};
    const R om1 = R(1) - R(c.omega_phi);
    R v[3];
    for (int b = 0; b < 3; ++b) v[b] = om1 * (j[b] - phi * u[b] + F[b] / R(6));
    R d[Q];
    FirstOrder<Q, R>::apply(u, v, d);
    const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        R eu = R(0), eF = R(0);
        for (int b = 0; b < 3; ++b) {
            eu += R(vel<Q>(i, b)) * u[b];
            eF += R(vel<Q>(i, b)) * F[b];
        }
        hs[i] = R(weight<Q>(i)) * (phi * (R(1) + R(3) * eu + R(4.5) * eu * eu - R(1.5) * uu) + R(0.5) * eF) + d[i];
    }
    return phi;
}

// zeroth and first moments of a pulled PDF vector
template <int Q, typename R>
__host__ __device__ __forceinline__ void moments01(const R f[Q], R &m0, R m1[3])
{
    m0 = R(0);
    for (int b = 0; b < 3; ++b) m1[b] = R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        m0 += f[i];
        for (int b = 0; b < 3; ++b)
            if (vel<Q>(i, b)) m1[b] += R(vel<Q>(i, b)) * f[i];
    }
}

// dL/df_i of a pulled PDF from the adjoints of its zeroth and first moments
template <int Q, typename R>
__host__ __device__ __forceinline__ R moment01_adjoint(R a0, const R a1[3], int i)
{
    R m = a0;
    for (int b = 0; b < 3; ++b)
        if (vel<Q>(i, b)) m += R(vel<Q>(i, b)) * a1[b];
    return m;
}

// phi, j: zeroth and first moments of the pulled h; a: adjoint of h*; aphi:
// adjoint of phi^{n+1}.  Returns the adjoints of phi and j (moment01_adjoint
// turns them into dL/dh per direction), aG = adjoint of the gradient, au =
// adjoint of u^n.
template <int Q, typename R>
__host__ __device__ __forceinline__ void pf_vjp(const PfCoef &c, R phi, const R j[3], const R G[3], const R u[3],
                                                const R a[Q], R &aphi, R aj[3], R aG[3], R au[3])
{
    const R inv = R(1) / sqrt(G[0] * G[0] + G[1] * G[1] + G[2] * G[2] + R(c.eps2));
    const R lam = R(4) * phi * (R(1) - phi) * R(c.inv_xi);
    const R F[3] = {lam * inv * G[0], lam * inv * G[1], lam * inv * G[2]};
    const R om1 = R(1) - R(c.omega_phi);
    R v[3];
    for (int b = 0; b < 3; ++b) v[b] = om1 * (j[b] - phi * u[b] + F[b] / R(6));
    const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];

    // h*_i = w_i (phi (1 + 3 e.u + 9/2 (e.u)^2 - 3/2 u.u) + e.F / 2) + [D(u) v]_i
    R A0, A1[3], A2[3][3];
    weighted_moments<Q, R>(a, A0, A1, A2);
    R A2u[3];
    for (int b = 0; b < 3; ++b) A2u[b] = A2[b][0] * u[0] + A2[b][1] * u[1] + A2[b][2] * u[2];
    R s[3];
    first_order_t<Q, R>(u, a, s);
    first_order_du<Q, R>(u, v, a, au);
    aphi += A0 * (R(1) - R(1.5) * uu) + R(3) * (A1[0] * u[0] + A1[1] * u[1] + A1[2] * u[2]) +
            R(4.5) * (u[0] * A2u[0] + u[1] * A2u[1] + u[2] * A2u[2]);
    R aF[3];
    for (int b = 0; b < 3; ++b) {
        au[b] += phi * (R(3) * A1[b] + R(9) * A2u[b] - R(3) * A0 * u[b]);
        aF[b] = R(0.5) * A1[b];
    }
    // v = (1 - omega_phi) (j - phi u + F/6)
    aphi -= om1 * (s[0] * u[0] + s[1] * u[1] + s[2] * u[2]);
    for (int b = 0; b < 3; ++b) {
        aj[b] = om1 * s[b];
        au[b] -= om1 * phi * s[b];
        aF[b] += om1 * s[b] / R(6);
    }
    // F = lam G / sqrt(|G|^2 + eps^2)
    const R p = aF[0] * G[0] + aF[1] * G[1] + aF[2] * G[2];
    const R alam = inv * p;
    for (int b = 0; b < 3; ++b) aG[b] = lam * inv * aF[b] - lam * inv * inv * inv * p * G[b];
    // lam = 4 phi (1 - phi) / xi
    aphi += alam * R(4) * R(c.inv_xi) * (R(1) - R(2) * phi);
}

// ============================================================================
// thermal LB (K3)
// ============================================================================
struct ThCoef {
    double kappa_l, dkappa;
};

// f: pulled PDFs (anti-bounce-back applied); u, phi: u^{n+1}, phi^{n+1}; q:
// heat source.  Writes f* and returns T^{n+1} = sum f.
template <int Q, typename R>
__host__ __device__ __forceinline__ R thermal_forward(const ThCoef &c, const R f[Q], const R u[3], R phi, R q, R fs[Q])
{
    R T = R(0), j[3] = {R(0), R(0), R(0)};
    for (int i = 0; i < Q; ++i) {
        T += f[i];
        for (int b = 0; b < 3; ++b)
            if (vel<Q>(i, b)) j[b] += R(vel<Q>(i, b)) * f[i];
    }
    const R phic = fmin(fmax(phi, R(0)), R(1));
    const R kap = R(c.kappa_l) + phic * R(c.dkappa);
    const R om1 = R(1) - R(1) / (R(0.5) + R(3) * kap);
    R v[3];
    for (int b = 0; b < 3; ++b) v[b] = om1 * (j[b] - T * u[b]);
    R d[Q];
    FirstOrder<Q, R>::apply(u, v, d);
    const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        R eu = R(0);
        for (int b = 0; b < 3; ++b) eu += R(vel<Q>(i, b)) * u[b];
        fs[i] = R(weight<Q>(i)) * (T * (R(1) + R(3) * eu + R(4.5) * eu * eu - R(1.5) * uu) + q) + d[i];
    }
    return T;
}

// T, j: zeroth and first moments of the pulled f; a: adjoint of f*; aT:
// adjoint of T^{n+1} on entry, of T (the zeroth moment) on return; aj:
// adjoint of j; au / aphi = adjoints of u^{n+1}, phi^{n+1}; aq = adjoint of q.
template <int Q, typename R>
__host__ __device__ __forceinline__ void thermal_vjp(const ThCoef &c, R T, const R j[3], const R u[3], R phi,
                                                     const R a[Q], R &aT, R aj[3], R au[3], R &aphi, R &aq)
{
    const R phic = fmin(fmax(phi, R(0)), R(1));
    const R kap = R(c.kappa_l) + phic * R(c.dkappa);
    const R den = R(0.5) + R(3) * kap;
    const R om1 = R(1) - R(1) / den;
    R v[3];
    for (int b = 0; b < 3; ++b) v[b] = om1 * (j[b] - T * u[b]);
    const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];

    R A0, A1[3], A2[3][3];
    weighted_moments<Q, R>(a, A0, A1, A2);
    R A2u[3];
    for (int b = 0; b < 3; ++b) A2u[b] = A2[b][0] * u[0] + A2[b][1] * u[1] + A2[b][2] * u[2];
    R s[3];
    first_order_t<Q, R>(u, a, s);
    first_order_du<Q, R>(u, v, a, au);
    aq = A0;
    aT += A0 * (R(1) - R(1.5) * uu) + R(3) * (A1[0] * u[0] + A1[1] * u[1] + A1[2] * u[2]) +
          R(4.5) * (u[0] * A2u[0] + u[1] * A2u[1] + u[2] * A2u[2]);
    aT -= om1 * (s[0] * u[0] + s[1] * u[1] + s[2] * u[2]);
    for (int b = 0; b < 3; ++b) {
        au[b] += T * (R(3) * A1[b] + R(9) * A2u[b] - R(3) * A0 * u[b]) - om1 * T * s[b];
        aj[b] = om1 * s[b];
    }
    // omega_T = 1 / (1/2 + 3 kappa(phi_c)): d(1 - omega_T)/d kappa = 3 / den^2
    const R aom1 = s[0] * (j[0] - T * u[0]) + s[1] * (j[1] - T * u[1]) + s[2] * (j[2] - T * u[2]);
    const R akap = aom1 * R(3) / (den * den);
    aphi = (phi > R(0) && phi < R(1)) ? R(c.dkappa) * akap : R(0);
}

// ============================================================================
// hydrodynamics (K2)
// ============================================================================
struct HyCoef {
    double rho_l, drho, tau_l, dtau, sigma_ref, sigma_t, t_ref, xi, g[3], omega_bulk;
};

// Stencil inputs of one cell: phi^n, its isotropic gradient and Laplacian;
// T^n and its gradient.
template <typename R>
struct HyIn {
    R phi, gp[3], lap, T, gT[3];
};

// Forward intermediates of the hydrodynamic update of one cell.
template <typename R>
struct HyFwd {
    R ps, u0[3], m[6];  // p*, momentum, raw second moments xx yy zz xy xz yz
    R rho, omega, nu, beta, kap, mu, gp2, gTgp;
    R b[6];             // strain brackets m - p*/3 delta - u0 u0
    R sfac, s[6];       // strain rate -3 omega b
    R Sgp[3], pfac, vfac, F[3], acc[3], u[3];
    R p[6];             // second central moments of g - g_eq + S/2 about u
    R om1, c[6];        // relaxed moments
};

// second-moment slot -> axes
__host__ __device__ constexpr int mom_a(int k) { return k < 3 ? k : (k == 5 ? 1 : 0); }
__host__ __device__ constexpr int mom_b(int k) { return k < 3 ? k : (k == 3 ? 1 : 2); }

// Raw moments of the pulled g the update depends on: p* = sum g, u0 = sum g e,
// m = sum g e e (slots xx yy zz xy xz yz).
template <typename R>
struct HyMom {
    R ps, u0[3], m[6];
};

template <typename R>
__host__ __device__ __forceinline__ HyMom<R> hydro_moments(const R g[27])
{
    HyMom<R> M;
    M.ps = R(0);
    for (int a = 0; a < 3; ++a) M.u0[a] = R(0);
    for (int k = 0; k < 6; ++k) M.m[k] = R(0);
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        M.ps += g[i];
        for (int a = 0; a < 3; ++a)
            if (vel27(i, a)) M.u0[a] += R(vel27(i, a)) * g[i];
        for (int k = 0; k < 6; ++k) {
            const int e = vel27(i, mom_a(k)) * vel27(i, mom_b(k));
            if (e) M.m[k] += R(e) * g[i];
        }
    }
    return M;
}

// dL/dg_i of the pulled PDFs from the adjoints of their raw moments
template <typename R>
__host__ __device__ __forceinline__ R hydro_moment_adjoint(const HyMom<R> &A, int i)
{
    R m = A.ps;
    for (int b = 0; b < 3; ++b)
        if (vel27(i, b)) m += R(vel27(i, b)) * A.u0[b];
    for (int k = 0; k < 6; ++k) {
        const int e = vel27(i, mom_a(k)) * vel27(i, mom_b(k));
        if (e) m += R(e) * A.m[k];
    }
    return m;
}

template <typename R>
__host__ __device__ __forceinline__ void hydro_intermediates(const HyCoef &c, const HyMom<R> &M, const HyIn<R> &in,
                                                             HyFwd<R> &f)
{
    f.ps = M.ps;
    for (int a = 0; a < 3; ++a) f.u0[a] = M.u0[a];
    for (int k = 0; k < 6; ++k) f.m[k] = M.m[k];
    const R third = R(1.0 / 3.0);
    const R phic = fmin(fmax(in.phi, R(0)), R(1));
    f.rho = R(c.rho_l) + phic * R(c.drho);
    const R tau = R(c.tau_l) + phic * R(c.dtau);
    f.omega = R(1) / (tau + R(0.5));
    f.nu = tau * third;
    const R sig = R(c.sigma_ref) + R(c.sigma_t) * (in.T - R(c.t_ref));
    f.beta = R(12) / R(c.xi) * sig;
    f.kap = R(1.5) * sig * R(c.xi);
    const R phi = in.phi;
    f.mu = R(4) * f.beta * phi * (phi - R(1)) * (phi - R(0.5)) - f.kap * in.lap;
    f.gp2 = in.gp[0] * in.gp[0] + in.gp[1] * in.gp[1] + in.gp[2] * in.gp[2];
    f.gTgp = in.gT[0] * in.gp[0] + in.gT[1] * in.gp[1] + in.gT[2] * in.gp[2];
    for (int k = 0; k < 6; ++k)
        f.b[k] = f.m[k] - (k < 3 ? f.ps * third : R(0)) - f.u0[mom_a(k)] * f.u0[mom_b(k)];
    f.sfac = R(-3) * f.omega;
    for (int k = 0; k < 6; ++k) f.s[k] = f.sfac * f.b[k];
    // S gp with S symmetric: slots xx yy zz xy xz yz
    f.Sgp[0] = f.s[0] * in.gp[0] + f.s[3] * in.gp[1] + f.s[4] * in.gp[2];
    f.Sgp[1] = f.s[3] * in.gp[0] + f.s[1] * in.gp[1] + f.s[5] * in.gp[2];
    f.Sgp[2] = f.s[4] * in.gp[0] + f.s[5] * in.gp[1] + f.s[2] * in.gp[2];
    const R mar = R(1.5) * R(c.xi) * R(c.sigma_t);
    f.pfac = -f.ps * third * R(c.drho);
    f.vfac = f.nu * R(c.drho);
    for (int a = 0; a < 3; ++a) {
        f.F[a] = f.mu * in.gp[a] + mar * (f.gp2 * in.gT[a] - f.gTgp * in.gp[a]) + f.rho * R(c.g[a]) +
                 f.pfac * in.gp[a] + f.vfac * f.Sgp[a];
        f.acc[a] = f.F[a] / f.rho;
        f.u[a] = f.u0[a] + R(0.5) * f.acc[a];
    }
    for (int k = 0; k < 6; ++k) {
        const int a = mom_a(k), b = mom_b(k);
        f.p[k] = f.m[k] - (k < 3 ? f.ps * third : R(0)) - f.u[a] * f.u[b] +
                 R(0.5) * (f.u[a] * f.acc[b] + f.acc[a] * f.u[b]);
    }
    f.om1 = R(1) - f.omega;
    const R tr = (R(1) - R(c.omega_bulk)) * (f.p[0] + f.p[1] + f.p[2]);
    const R d1 = f.om1 * (f.p[0] - f.p[1]), d2 = f.om1 * (f.p[0] - f.p[2]);
    f.c[0] = third * (tr + d1 + d2);
    f.c[1] = f.c[0] - d1;
    f.c[2] = f.c[0] - d2;
    for (int k = 3; k < 6; ++k) f.c[k] = f.om1 * f.p[k];
}

// 1-D inverse-transform columns m_p(c) (Axis1D) and their u-derivatives
template <typename R>
struct Cols1D {
    R m[3][3], dm[3][3]; // [p][c + 1]
    __host__ __device__ __forceinline__ explicit Cols1D(R u)
    {
        const Axis1D<R> A(u);
        for (int k = 0; k < 3; ++k) {
            m[0][k] = A.m0[k];
            m[1][k] = A.m1[k];
            m[2][k] = A.m2[k];
        }
        dm[0][0] = u - R(0.5);
        dm[0][1] = R(-2) * u;
        dm[0][2] = u + R(0.5);
        dm[1][0] = R(1);
        dm[1][1] = R(-2);
        dm[1][2] = R(1);
        for (int k = 0; k < 3; ++k) dm[2][k] = R(0);
    }
};

// exponents (p, q, r) of the six relaxed second-order moments, slot order xx yy zz xy xz yz
__host__ __device__ constexpr int mom_exp(int k, int axis)
{
    return (k < 3) ? (axis == k ? 2 : 0) : (axis == mom_a(k) || axis == mom_b(k) ? 1 : 0);
}

// For an adjoint vector a over the D3Q27 directions and the six relaxed
// moments k (exponents p, q, r): ac[k] = sum_i a_i X_p Y_q Z_r (the transpose
// of the inverse transform) and du[axis] = sum_k c_k sum_i a_i d/du_axis
// (X_p Y_q Z_r) (its u-derivative), contracted one axis at a time (z, then y,
// then x), about a fifth of the work of contracting each product separately.
template <typename R>
__host__ __device__ __forceinline__ void transform_adjoint(const R a[27], const Cols1D<R> &X, const Cols1D<R> &Y,
                                                           const Cols1D<R> &Z, const R c[6], R ac[6], R du[3])
{
    // z: P[r][xa][ya] with the columns and Pd[r][xa][ya] with their derivatives
    R P[3][3][3], Pd[2][3][3];
    for (int r = 0; r < 3; ++r)
        for (int xa = 0; xa < 3; ++xa)
            for (int ya = 0; ya < 3; ++ya) {
                P[r][xa][ya] = R(0);
                if (r < 2) Pd[r][xa][ya] = R(0);
            }
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const int xa = vel27(i, 0) + 1, ya = vel27(i, 1) + 1, za = vel27(i, 2) + 1;
        for (int r = 0; r < 3; ++r) P[r][xa][ya] += a[i] * Z.m[r][za];
        for (int r = 0; r < 2; ++r) Pd[r][xa][ya] += a[i] * Z.dm[r][za];
    }
    for (int b = 0; b < 3; ++b) du[b] = R(0);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int p = mom_exp(k, 0), q = mom_exp(k, 1), r = mom_exp(k, 2);
        // y: the three x-slices for this (q, r), and with Y' or Z'
        R s[3], sy[3], sz[3];
        for (int xa = 0; xa < 3; ++xa) {
            s[xa] = sy[xa] = sz[xa] = R(0);
            for (int ya = 0; ya < 3; ++ya) {
                s[xa] += P[r][xa][ya] * Y.m[q][ya];
                if (q < 2) sy[xa] += P[r][xa][ya] * Y.dm[q][ya];
                if (r < 2) sz[xa] += Pd[r < 2 ? r : 0][xa][ya] * Y.m[q][ya];
            }
        }
        R v = R(0), vx = R(0), vy = R(0), vz = R(0);
        for (int xa = 0; xa < 3; ++xa) {
            v += s[xa] * X.m[p][xa];
            if (p < 2) vx += s[xa] * X.dm[p][xa];
            if (q < 2) vy += sy[xa] * X.m[p][xa];
            if (r < 2) vz += sz[xa] * X.m[p][xa];
        }
        ac[k] = v;
        du[0] += c[k] * vx;
        du[1] += c[k] * vy;
        du[2] += c[k] * vz;
    }
}

template <typename R>
__host__ __device__ __forceinline__ void hydro_forward(const HyCoef &c, const R g[27], const HyIn<R> &in, R gs[27],
                                                       R u[3])
{
    HyFwd<R> f;
    hydro_intermediates(c, hydro_moments(g), in, f);
    const Cols1D<R> X(f.u[0]), Y(f.u[1]), Z(f.u[2]);
    const R uu = f.u[0] * f.u[0] + f.u[1] * f.u[1] + f.u[2] * f.u[2];
    const R ua = f.u[0] * f.acc[0] + f.u[1] * f.acc[1] + f.u[2] * f.acc[2];
    const R C = f.ps - R(1.5) * (uu + ua);
    for (int i = 0; i < 27; ++i) {
        const int e[3] = {vel27(i, 0), vel27(i, 1), vel27(i, 2)};
        R eu = R(0), ea = R(0);
        for (int a = 0; a < 3; ++a) {
            eu += R(e[a]) * f.u[a];
            ea += R(e[a]) * f.acc[a];
        }
        R corr = R(0);
        for (int k = 0; k < 6; ++k)
            corr += f.c[k] * X.m[mom_exp(k, 0)][e[0] + 1] * Y.m[mom_exp(k, 1)][e[1] + 1] * Z.m[mom_exp(k, 2)][e[2] + 1];
        gs[i] = R(weight<27>(i)) * (C + R(3) * eu + R(1.5) * ea + R(4.5) * eu * (eu + ea)) + corr;
    }
    for (int a = 0; a < 3; ++a) u[a] = f.u[a];
}

// Adjoint of the stencil inputs of one cell.
template <typename R>
struct HyAdj {
    R phi, gp[3], lap, T, gT[3];
};

// M: raw moments of the pulled g; a: adjoint of g*; au_out: adjoint of
// u^{n+1}.  Writes the adjoints of the raw moments (hydro_moment_adjoint turns
// them into dL/dg per direction) and of the stencil inputs.
template <typename R>
__host__ __device__ __forceinline__ void hydro_vjp(const HyCoef &c, const HyMom<R> &M, const HyIn<R> &in,
                                                   const R a[27], const R au_out[3], HyMom<R> &am, HyAdj<R> &ad)
{
    HyFwd<R> f;
    hydro_intermediates(c, M, in, f);
    const R third = R(1.0 / 3.0);
    const Cols1D<R> X(f.u[0]), Y(f.u[1]), Z(f.u[2]);

    // output layer: g*_i = w_i [C + 3 e.u + 3/2 e.a + 9/2 e.u (e.u + e.a)] + corr_i(u, c)
    R A0, A1[3], A2[3][3];
    weighted_moments<27, R>(a, A0, A1, A2);
    R A2u[3], A2a[3];
    for (int b = 0; b < 3; ++b) {
        A2u[b] = A2[b][0] * f.u[0] + A2[b][1] * f.u[1] + A2[b][2] * f.u[2];
        A2a[b] = A2[b][0] * f.acc[0] + A2[b][1] * f.acc[1] + A2[b][2] * f.acc[2];
    }
    R a_ps = A0, a_u[3], a_acc[3], a_c[6];
    for (int b = 0; b < 3; ++b) {
        a_u[b] = au_out[b] - R(1.5) * A0 * (R(2) * f.u[b] + f.acc[b]) + R(3) * A1[b] + R(9) * A2u[b] + R(4.5) * A2a[b];
        a_acc[b] = R(-1.5) * A0 * f.u[b] + R(1.5) * A1[b] + R(4.5) * A2u[b];
    }
    // corr_i = sum_k c_k X_p[e_x] Y_q[e_y] Z_r[e_z]
    {
        R du[3];
        transform_adjoint(a, X, Y, Z, f.c, a_c, du);
        for (int b = 0; b < 3; ++b) a_u[b] += du[b];
    }
    // relaxation: c_xx = (tr + d1 + d2)/3, c_yy = c_xx - d1, c_zz = c_xx - d2, c_off = om1 p_off
    const R sc = (a_c[0] + a_c[1] + a_c[2]) * third;
    const R a_tr = sc, a_d1 = sc - a_c[1], a_d2 = sc - a_c[2];
    const R ob = R(1) - R(c.omega_bulk);
    R a_p[6];
    a_p[0] = ob * a_tr + f.om1 * (a_d1 + a_d2);
    a_p[1] = ob * a_tr - f.om1 * a_d1;
    a_p[2] = ob * a_tr - f.om1 * a_d2;
    for (int k = 3; k < 6; ++k) a_p[k] = f.om1 * a_c[k];
    R a_om1 = a_d1 * (f.p[0] - f.p[1]) + a_d2 * (f.p[0] - f.p[2]);
    for (int k = 3; k < 6; ++k) a_om1 += a_c[k] * f.p[k];
    R a_omega = -a_om1;
    // p_ab = m_ab - p*/3 delta - u_a u_b + (u_a acc_b + acc_a u_b)/2
    R a_m[6];
    for (int k = 0; k < 6; ++k) {
        const int x = mom_a(k), y = mom_b(k);
        a_m[k] = a_p[k];
        if (k < 3) {
            a_ps -= a_p[k] * third;
            a_u[x] += a_p[k] * (R(-2) * f.u[x] + f.acc[x]);
            a_acc[x] += a_p[k] * f.u[x];
        } else {
            a_u[x] += a_p[k] * (-f.u[y] + R(0.5) * f.acc[y]);
            a_u[y] += a_p[k] * (-f.u[x] + R(0.5) * f.acc[x]);
            a_acc[x] += R(0.5) * a_p[k] * f.u[y];
            a_acc[y] += R(0.5) * a_p[k] * f.u[x];
        }
    }
    // u = u0 + acc/2
    R a_u0[3];
    for (int b = 0; b < 3; ++b) {
        a_u0[b] = a_u[b];
        a_acc[b] += R(0.5) * a_u[b];
    }
    // acc = F / rho
    R a_F[3];
    R a_rho = R(0);
    for (int b = 0; b < 3; ++b) {
        a_F[b] = a_acc[b] / f.rho;
        a_rho -= a_acc[b] * f.acc[b] / f.rho;
    }
    // F = mu gp + mar (|gp|^2 gT - (gT.gp) gp) + rho g + pfac gp + vfac S gp
    const R mar = R(1.5) * R(c.xi) * R(c.sigma_t);
    const R aFgp = a_F[0] * in.gp[0] + a_F[1] * in.gp[1] + a_F[2] * in.gp[2];
    const R aFgT = a_F[0] * in.gT[0] + a_F[1] * in.gT[1] + a_F[2] * in.gT[2];
    const R a_mu = aFgp;
    const R a_gp2 = mar * aFgT;
    const R a_gTgp = -mar * aFgp;
    const R a_pfac = aFgp;
    const R a_vfac = a_F[0] * f.Sgp[0] + a_F[1] * f.Sgp[1] + a_F[2] * f.Sgp[2];
    a_rho += a_F[0] * R(c.g[0]) + a_F[1] * R(c.g[1]) + a_F[2] * R(c.g[2]);
    R a_Sgp[3];
    for (int b = 0; b < 3; ++b) {
        ad.gp[b] = (f.mu - mar * f.gTgp + f.pfac) * a_F[b];
        ad.gT[b] = mar * f.gp2 * a_F[b];
        a_Sgp[b] = f.vfac * a_F[b];
    }
    // S gp
    R a_s[6];
    a_s[0] = a_Sgp[0] * in.gp[0];
    a_s[1] = a_Sgp[1] * in.gp[1];
    a_s[2] = a_Sgp[2] * in.gp[2];
    a_s[3] = a_Sgp[0] * in.gp[1] + a_Sgp[1] * in.gp[0];
    a_s[4] = a_Sgp[0] * in.gp[2] + a_Sgp[2] * in.gp[0];
    a_s[5] = a_Sgp[1] * in.gp[2] + a_Sgp[2] * in.gp[1];
    ad.gp[0] += f.s[0] * a_Sgp[0] + f.s[3] * a_Sgp[1] + f.s[4] * a_Sgp[2];
    ad.gp[1] += f.s[3] * a_Sgp[0] + f.s[1] * a_Sgp[1] + f.s[5] * a_Sgp[2];
    ad.gp[2] += f.s[4] * a_Sgp[0] + f.s[5] * a_Sgp[1] + f.s[2] * a_Sgp[2];
    // |gp|^2 and gT.gp
    for (int b = 0; b < 3; ++b) {
        ad.gp[b] += R(2) * a_gp2 * in.gp[b] + a_gTgp * in.gT[b];
        ad.gT[b] += a_gTgp * in.gp[b];
    }
    // pfac = -p* drho / 3, vfac = nu drho
    a_ps -= R(c.drho) * third * a_pfac;
    const R a_nu = R(c.drho) * a_vfac;
    // strain s = -3 omega b, b = m - p*/3 delta - u0 u0
    R a_sfac = R(0);
    for (int k = 0; k < 6; ++k) {
        a_sfac += a_s[k] * f.b[k];
        const R ab = f.sfac * a_s[k];
        const int x = mom_a(k), y = mom_b(k);
        a_m[k] += ab;
        if (k < 3) {
            a_ps -= ab * third;
            a_u0[x] -= R(2) * ab * f.u0[x];
        } else {
            a_u0[x] -= ab * f.u0[y];
            a_u0[y] -= ab * f.u0[x];
        }
    }
    a_omega += R(-3) * a_sfac;
    // mu = 4 beta phi (phi - 1)(phi - 1/2) - kap lap
    const R phi = in.phi;
    const R P3 = phi * (phi - R(1)) * (phi - R(0.5));
    const R dP3 = R(3) * phi * phi - R(3) * phi + R(0.5);
    const R a_beta = R(4) * P3 * a_mu;
    ad.phi = R(4) * f.beta * dP3 * a_mu;
    const R a_kap = -in.lap * a_mu;
    ad.lap = -f.kap * a_mu;
    const R a_sig = R(12) / R(c.xi) * a_beta + R(1.5) * R(c.xi) * a_kap;
    ad.T = R(c.sigma_t) * a_sig;
    // omega = 1/(tau + 1/2), nu = tau/3, rho and tau linear in phi_c
    const R a_tau = -f.omega * f.omega * a_omega + a_nu * third;
    const R a_phic = R(c.drho) * a_rho + R(c.dtau) * a_tau;
    if (phi > R(0) && phi < R(1)) ad.phi += a_phic;
    am.ps = a_ps;
    for (int b = 0; b < 3; ++b) am.u0[b] = a_u0[b];
    for (int k = 0; k < 6; ++k) am.m[k] = a_m[k];
}

} // namespace tcp
