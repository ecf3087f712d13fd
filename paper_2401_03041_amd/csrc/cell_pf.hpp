// cell_pf.hpp -- K1: conservative Allen-Cahn phase-field LB step
// (Eq. lb_interface with the counter-term of Eq. phasefieldforce applied as a
// source in collision space).  One thread per cell, pull streaming from the
// post-collision PDFs of the previous step, halfway bounce-back at y walls.
//
// Collision: central moments about u^n on the moment basis of the stencil,
// first-order moments relaxed with omega_phi, all higher ones with rate one.
// Because the higher moments relax fully, the post-collision state is
// h_eq + S/2 plus the inverse transform of the relaxed first-order moments
// (FirstOrder<Q>), which is what the kernel evaluates.
//
// Storage in type P: as is (FP64), or (FP32, FP16) as the deviation
// h*_i - w_i phi(x) from the rest equilibrium of the cell (deviation_storage);
// the pull then works with h_i - w_i phi^n(own), rebuilt from the stored value
// and phi^n of the source and own cells, which the kernel loads anyway for the
// gradient of phi^n.
#pragma once

#include "kernels.hpp"

namespace tcp {

// Update of one cell; returns phi^{n+1} and, in sten, phi^n at the cell with
// its isotropic gradient and Laplacian.
template <int Q, typename P, typename S, typename R, bool WALL>
__device__ __forceinline__ R phase_field_cell(const PfArgs &a, const Nbr &nb, PhiStencil<R> &sten,
                                              const Staged<R> *staged = nullptr)
{
    constexpr bool dev = deviation_storage<P>();
    const P *hs = static_cast<const P *>(a.h_src);
    const PdfLanes<Q> pl(nb);

    // phi^n on the 3x3x3 neighbourhood (contact-angle ghosts across walls);
    // the wave issues these loads and the PDF pull at raised priority
    // (kPullPriority)
    const S *po = static_cast<const S *>(a.phi_old);
    __builtin_amdgcn_s_setprio(kPullPriority);
    R pn[27];
    if (staged) staged->stencil27(pn); // phi^n staged in LDS by the fused step
    else nb.stencil27(po, pn);
#pragma unroll
    for (int k = 0; k < 27; ++k)
        if (WALL && nb.ghost(vel27(k, 1))) pn[k] = nb.phi_ghost(pn[k], vel27(k, 1), a.wet);

    // pull; a link that crosses a wall returns the cell's own opposite PDF
    R h[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int ex = vel<Q>(i, 0), ey = vel<Q>(i, 1), ez = vel<Q>(i, 2);
        const bool wall = WALL && nb.ghost(-ey);
        h[i] = wall ? ld<R>(elem(pdf_row<Q>(hs, a.geo, nb.yr[1], nb.zi[1], opposite<Q>(i)), pl.xq[1]))
                    : ld<R>(elem(pdf_row<Q>(hs, a.geo, nb.yr[1 - ey], nb.zi[1 - ez], i), pl.xq[1 - ex]));
        // deviation storage: h - w phi^n(own) = stored + w (phi^n(source) - phi^n(own)),
        // which is exactly zero in a uniform region at rest
        if constexpr (dev) {
            if (!wall) h[i] += R(weight<Q>(i)) * (pn[opposite<27>(index27<Q>(i))] - pn[0]);
        }
    }
    __builtin_amdgcn_s_setprio(0);
    // zeroth and first moments from sums and differences of opposite pairs
    // (with deviation storage h[] holds h - w phi^n(own): sum_i w_i = 1 adds
    // phi^n(own) to the zeroth moment, sum_i w_i e_i = 0 leaves the first)
    R phi = h[0], j[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        if (opposite<Q>(i) < i) continue;
        const int o = opposite<Q>(i);
        const R df = h[i] - h[o];
        phi += h[i] + h[o];
        if (vel<Q>(i, 0)) j[0] += R(vel<Q>(i, 0)) * df;
        if (vel<Q>(i, 1)) j[1] += R(vel<Q>(i, 1)) * df;
        if (vel<Q>(i, 2)) j[2] += R(vel<Q>(i, 2)) * df;
    }
    if constexpr (dev) phi += pn[0];

    // interface normal from the isotropic gradient of phi^n
    phi_stencil(pn, sten);
    const R(&gr)[3] = sten.gp;
    const R inv = R(1) / sqrt(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2] + R(a.eps2));
    const R lam = R(4) * phi * (R(1) - phi) * R(a.inv_xi);
    const R F[3] = {lam * gr[0] * inv, lam * gr[1] * inv, lam * gr[2] * inv};

    R u[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) u[k] = ld<R>(elem(static_cast<const S *>(a.u[k]), nb.c));

    // relaxed first-order central moment of h - h_eq + S/2
    const R om1 = R(1) - R(a.omega_phi);
    const R sixth = R(1.0 / 6.0);
    const R v[3] = {om1 * (j[0] - phi * u[0] + sixth * F[0]), om1 * (j[1] - phi * u[1] + sixth * F[1]),
                    om1 * (j[2] - phi * u[2] + sixth * F[2])};
    R d[Q];
    FirstOrder<Q, R>::apply(u, v, d);

    // h* = w (phi (1 + zeta) + e.F / 2) + d with zeta = 3 e.u + 9/2 (e.u)^2 - 3/2 u.u
    // (minus w phi when stored as a deviation).  Opposite directions share the
    // even part phi (1 - 3/2 u.u + 9/2 (e.u)^2) and flip the odd part
    // 3 phi e.u + e.F / 2.
    const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const R base = phi * ((dev ? R(0) : R(1)) - R(1.5) * uu);
    P *hd = static_cast<P *>(a.h_dst);
    st_pdf(elem(pdf_row<Q>(hd, a.geo, nb.yr[1], nb.zi[1], 0), pl.xq[1]), R(weight<Q>(0)) * base + d[0]);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        if (opposite<Q>(i) < i) continue;
        const int o = opposite<Q>(i);
        const int ex = vel<Q>(i, 0), ey = vel<Q>(i, 1), ez = vel<Q>(i, 2);
        const R w = R(weight<Q>(i));
        R eu = R(0), eF = R(0);
        if (ex) { eu += R(ex) * u[0]; eF += R(ex) * F[0]; }
        if (ey) { eu += R(ey) * u[1]; eF += R(ey) * F[1]; }
        if (ez) { eu += R(ez) * u[2]; eF += R(ez) * F[2]; }
        const R even = base + R(4.5) * phi * eu * eu;
        const R odd = R(3) * phi * eu + R(0.5) * eF;
        st_pdf(elem(pdf_row<Q>(hd, a.geo, nb.yr[1], nb.zi[1], i), pl.xq[1]), w * (even + odd) + d[i]);
        st_pdf(elem(pdf_row<Q>(hd, a.geo, nb.yr[1], nb.zi[1], o), pl.xq[1]), w * (even - odd) + d[o]);
    }
    st(elem(static_cast<S *>(a.phi_new), nb.c), phi);
    return phi;
}

} // namespace tcp
