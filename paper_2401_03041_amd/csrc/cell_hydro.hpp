// cell_hydro.hpp -- K2: velocity-based D3Q27 central-moment hydrodynamic
// LB step with the force of Sec. 2.2: F = F_s + F_b + F_p + F_mu, where
//   F_s  = mu_phi grad phi + 3/2 xi sigma_T (|grad phi|^2 grad T - (grad T . grad phi) grad phi)
//   F_b  = rho g,   F_p = -p* c_s^2 (rho_H - rho_L) grad phi,
//   F_mu = nu (rho_H - rho_L) [grad u + grad u^T] . grad phi,
// mu_phi = 4 beta phi (phi-1)(phi-1/2) - k lap phi, beta = 12 sigma/xi,
// k = 3 sigma xi / 2, sigma(T) = sigma_ref + sigma_T (T - T_ref), and the strain
// rate taken from the non-equilibrium second moment of the pulled PDFs.
// Gradients and the Laplacian use the isotropic D3Q27 stencil on phi^n (contact-angle
// ghost at walls) and on T^n (ghost 2 T_w - T).
//
// Collision: central moments about u, the five deviatoric second-order
// moments relax with omega(phi), the trace with omega_bulk, everything else
// with rate one, Guo source in velocity form.  Moments of rate one land on
// g_eq + S/2, so the kernel adds to g_eq + S/2 only the inverse transform of
// the six relaxed second-order central moments of g - g_eq + S/2; the D3Q27
// moment matrix is a tensor product of 1-D matrices, so that inverse is a
// product of 1-D columns (Axis1D).
#pragma once

#include "kernels.hpp"

namespace tcp {

// Update of one cell.  Writes g* and u^{n+1}, and returns u^{n+1}.  With
// GIVEN the phi^n stencil quantities come from the phase-field update of the
// same cell (fused step) instead of being loaded.  With QT > 0, tsrc[i]
// returns T^n at x - e_i for the QT directions of the thermal stencil (the
// values the thermal pull needs with deviation storage).
template <typename S, typename R, bool WALL, bool GIVEN = false, int QT = 0>
__device__ __forceinline__ void hydro_cell(const HydroArgs &a, const Nbr &nb, R (&u)[3],
                                           const PhiStencil<R> &given = PhiStencil<R>{}, R *tsrc = nullptr,
                                           const Staged<R> *stagedT = nullptr)
{
    const S *gs = static_cast<const S *>(a.g_src);
    const PdfLanes<27> pl(nb);

    // pull; halfway bounce-back, plus 2 w_i (e_i . u_w)/c_s^2 from a moving wall
    R g[27];
    __builtin_amdgcn_s_setprio(kPullPriority);
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const int ex = vel27(i, 0), ey = vel27(i, 1), ez = vel27(i, 2);
        if (WALL && nb.ghost(-ey)) {
            const double *uw = ey > 0 ? a.uw_bot : a.uw_top;
            const double eu = ex * uw[0] + ey * uw[1] + ez * uw[2];
            g[i] = ld<R>(elem(pdf_row<27>(gs, a.geo, nb.yr[1], nb.zi[1], opposite<27>(i)), pl.xq[1])) +
                   R(6.0 * weight<27>(i) * eu);
        } else {
            g[i] = ld<R>(elem(pdf_row<27>(gs, a.geo, nb.yr[1 - ey], nb.zi[1 - ez], i), pl.xq[1 - ex]));
        }
    }
    __builtin_amdgcn_s_setprio(0);
    // zeroth, first and second raw moments from sums and differences of opposite pairs
    R ps = g[0], u0[3] = {R(0), R(0), R(0)};
    R mxx = R(0), myy = R(0), mzz = R(0), mxy = R(0), mxz = R(0), myz = R(0);
#pragma unroll
    for (int i = 1; i < 27; ++i) {
        if (opposite<27>(i) < i) continue;
        const int o = opposite<27>(i);
        const int ex = vel27(i, 0), ey = vel27(i, 1), ez = vel27(i, 2);
        const R sm = g[i] + g[o], df = g[i] - g[o];
        ps += sm;
        if (ex) u0[0] += R(ex) * df;
        if (ey) u0[1] += R(ey) * df;
        if (ez) u0[2] += R(ez) * df;
        if (ex) mxx += sm;
        if (ey) myy += sm;
        if (ez) mzz += sm;
        if (ex * ey) mxy += R(ex * ey) * sm;
        if (ex * ez) mxz += R(ex * ez) * sm;
        if (ey * ez) myz += R(ey * ez) * sm;
    }

    // phi^n: value, gradient, Laplacian; T^n: value, gradient
    const S *pp = static_cast<const S *>(a.phi);
    const S *tp = static_cast<const S *>(a.T);
    PhiStencil<R> sten;
    R gT[3] = {R(0), R(0), R(0)};
    __builtin_amdgcn_s_setprio(kPullPriority);
    if constexpr (GIVEN) {
        sten = given;
    } else {
        R pn[27];
        nb.stencil27(pp, pn);
#pragma unroll
        for (int i = 0; i < 27; ++i)
            if (WALL && nb.ghost(vel27(i, 1))) pn[i] = nb.phi_ghost(pn[i], vel27(i, 1), a.wet);
        phi_stencil(pn, sten);
    }
    R tn[27];
    if (stagedT) stagedT->stencil27(tn); // T^n staged in LDS by the fused step
    else nb.stencil27(tp, tn);
    const R T = tn[0];
    if constexpr (QT > 0) {
#pragma unroll
        for (int i = 0; i < QT; ++i) {
            const int j = index27<QT>(i);
            tsrc[i] = tn[index_of(-vel27(j, 0), -vel27(j, 1), -vel27(j, 2))];
        }
    }
#pragma unroll
    for (int i = 1; i < 27; ++i) {
        const int ex = vel27(i, 0), ey = vel27(i, 1), ez = vel27(i, 2);
        const R w = R(weight<27>(i));
        R tv = tn[i];
        if (WALL && nb.ghost(ey)) {
            const double *tw = ey < 0 ? a.twb : a.twt;
            tv = R(2) * R(tw[nb.col(ex, ez, a.geo)]) - tv;
        }
        if (ex) gT[0] += R(ex) * w * tv;
        if (ey) gT[1] += R(ey) * w * tv;
        if (ez) gT[2] += R(ez) * w * tv;
    }
    __builtin_amdgcn_s_setprio(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) gT[k] *= R(3);
    const R phi = sten.phi;
    const R(&gp)[3] = sten.gp;
    const R lap = sten.lap;

    // material laws
    const R phic = fmin(fmax(phi, R(0)), R(1));
    const R drho = R(a.drho);
    const R rho = R(a.rho_l) + phic * drho;
    const R tau = R(a.tau_l) + phic * R(a.dtau);
    const R omega = R(1) / (tau + R(0.5));
    const R nu = tau * R(1.0 / 3.0);
    const R sig = R(a.sigma_ref) + R(a.sigma_t) * (T - R(a.t_ref));
    const R xi = R(a.xi);
    const R beta = R(a.twelve_inv_xi) * sig, kap = R(1.5) * sig * xi;
    const R mu = R(4) * beta * phi * (phi - R(1)) * (phi - R(0.5)) - kap * lap;
    const R gp2 = gp[0] * gp[0] + gp[1] * gp[1] + gp[2] * gp[2];
    const R gTgp = gT[0] * gp[0] + gT[1] * gp[1] + gT[2] * gp[2];

    // strain rate from the non-equilibrium second moment about g_eq(p*, u0)
    const R third = R(1.0 / 3.0);
    const R sfac = R(-3) * omega;
    const R sxx = sfac * (mxx - ps * third - u0[0] * u0[0]);
    const R syy = sfac * (myy - ps * third - u0[1] * u0[1]);
    const R szz = sfac * (mzz - ps * third - u0[2] * u0[2]);
    const R sxy = sfac * (mxy - u0[0] * u0[1]);
    const R sxz = sfac * (mxz - u0[0] * u0[2]);
    const R syz = sfac * (myz - u0[1] * u0[2]);
    const R Sgp[3] = {sxx * gp[0] + sxy * gp[1] + sxz * gp[2], sxy * gp[0] + syy * gp[1] + syz * gp[2],
                      sxz * gp[0] + syz * gp[1] + szz * gp[2]};

    const R mar = R(1.5) * xi * R(a.sigma_t);
    const R pfac = -ps * third * drho;
    const R vfac = nu * drho;
    R acc[3];
    const R inv_rho = R(1) / rho;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const R Fs = mu * gp[k] + mar * (gp2 * gT[k] - gTgp * gp[k]);
        const R F = Fs + rho * R(a.g[k]) + pfac * gp[k] + vfac * Sgp[k];
        acc[k] = F * inv_rho;
        u[k] = u0[k] + R(0.5) * acc[k];
    }

    // second-order central moments of g - g_eq + S/2 about u (D3Q27 closed form)
    const R pxx = mxx - ps * third - u[0] * u[0] + u[0] * acc[0];
    const R pyy = myy - ps * third - u[1] * u[1] + u[1] * acc[1];
    const R pzz = mzz - ps * third - u[2] * u[2] + u[2] * acc[2];
    const R pxy = mxy - u[0] * u[1] + R(0.5) * (u[0] * acc[1] + acc[0] * u[1]);
    const R pxz = mxz - u[0] * u[2] + R(0.5) * (u[0] * acc[2] + acc[0] * u[2]);
    const R pyz = myz - u[1] * u[2] + R(0.5) * (u[1] * acc[2] + acc[1] * u[2]);
    const R om1 = R(1) - omega;
    const R tr = (R(1) - R(a.omega_bulk)) * (pxx + pyy + pzz);
    const R d1 = om1 * (pxx - pyy), d2 = om1 * (pxx - pzz);
    const R cxx = third * (tr + d1 + d2), cyy = cxx - d1, czz = cxx - d2;
    const R cxy = om1 * pxy, cxz = om1 * pxz, cyz = om1 * pyz;

    // inverse transform of the relaxed second-order moments: the correction of PDF
    // (a, b, c) is sum_k Z.m_k[c] A_k[a][b]
    const Axis1D<R> X(u[0]), Y(u[1]), Z(u[2]);
    R A0[3][3], A1[3][3], A2[3][3];
#pragma unroll
    for (int ia = 0; ia < 3; ++ia)
#pragma unroll
        for (int ib = 0; ib < 3; ++ib) {
            A0[ia][ib] = cxx * X.m2[ia] * Y.m0[ib] + cyy * X.m0[ia] * Y.m2[ib] + cxy * X.m1[ia] * Y.m1[ib];
            A1[ia][ib] = cxz * X.m1[ia] * Y.m0[ib] + cyz * X.m0[ia] * Y.m1[ib];
            A2[ia][ib] = czz * X.m0[ia] * Y.m0[ib];
        }

    // g_eq + S/2 = w [C + 3 e.u + 3/2 e.a + 9/2 e.u (e.u + e.a)]: opposite directions share
    // the even part and flip the odd one
    const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const R ua = u[0] * acc[0] + u[1] * acc[1] + u[2] * acc[2];
    const R C = ps - R(1.5) * (uu + ua);
    S *gd = static_cast<S *>(a.g_dst);
    {
        const R corr = Z.m0[1] * A0[1][1] + Z.m1[1] * A1[1][1] + Z.m2[1] * A2[1][1];
        st_pdf(elem(pdf_row<27>(gd, a.geo, nb.yr[1], nb.zi[1], 0), pl.xq[1]), R(weight<27>(0)) * C + corr);
    }
#pragma unroll
    for (int i = 1; i < 27; ++i) {
        if (opposite<27>(i) < i) continue;
        const int o = opposite<27>(i);
        const int ex = vel27(i, 0), ey = vel27(i, 1), ez = vel27(i, 2);
        const R w = R(weight<27>(i));
        R eu = R(0), ea = R(0);
        if (ex) { eu += R(ex) * u[0]; ea += R(ex) * acc[0]; }
        if (ey) { eu += R(ey) * u[1]; ea += R(ey) * acc[1]; }
        if (ez) { eu += R(ez) * u[2]; ea += R(ez) * acc[2]; }
        const R even = w * C + R(4.5) * w * (eu * (eu + ea));
        const R odd = R(3) * w * eu + R(1.5) * w * ea;
        const int ia = ex + 1, ib = ey + 1, ic = ez + 1;
        const int oa = 1 - ex, ob = 1 - ey, oc = 1 - ez;
        const R ci = Z.m0[ic] * A0[ia][ib] + Z.m1[ic] * A1[ia][ib] + Z.m2[ic] * A2[ia][ib];
        const R co = Z.m0[oc] * A0[oa][ob] + Z.m1[oc] * A1[oa][ob] + Z.m2[oc] * A2[oa][ob];
        st_pdf(elem(pdf_row<27>(gd, a.geo, nb.yr[1], nb.zi[1], i), pl.xq[1]), even + odd + ci);
        st_pdf(elem(pdf_row<27>(gd, a.geo, nb.yr[1], nb.zi[1], o), pl.xq[1]), even - odd + co);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) st(elem(static_cast<S *>(a.u[k]), nb.c), u[k]);
}

} // namespace tcp
