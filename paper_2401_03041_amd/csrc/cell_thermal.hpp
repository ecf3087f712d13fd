// cell_thermal.hpp -- K3, passive-scalar LB (Eq. lb_thermal): pull with
// anti-bounce-back f_i = -f*_opp + 2 w_i T_w at the y walls, T = sum_i f_i,
// central-moment collision about u^{n+1} with the first-order moments relaxed
// by omega_T = 1/(1/2 + kappa(phi)/c_s^2) and all higher ones with rate one,
// then the source w_i q_T (Eq. HeatSource).  Storage in type P: f_i - w_i t_shift
// (FP64), or (FP32, FP16) the deviation f*_i - w_i T(x) from the rest
// equilibrium of the cell, rebuilt in the pull around T^n of the own cell.  T is double
// buffered (T^n read, T^{n+1} written).
#pragma once

#include "kernels.hpp"

namespace tcp {

// Update of one cell at (x, y, z) given the cell's phi^{n+1} and u^{n+1}.  With
// GIVEN_T (deviation storage), tsrc[i] holds T^n at x - e_i, handed over by the
// hydrodynamic update of the same cell, instead of being loaded.
template <int Q, typename P, typename S, typename R, bool WALL, bool GIVEN_T = false>
__device__ __forceinline__ void thermal_cell(const ThermalArgs &a, const Nbr &nb, int x, int y, int z, R phi,
                                             const R (&u)[3], const R *tsrc = nullptr)
{
    constexpr bool dev = deviation_storage<P>();
    const P *fs = static_cast<const P *>(a.f_src);
    const PdfLanes<Q> pl(nb);
    const S *to = static_cast<const S *>(a.T_old);
    const R ts = dev ? R(0) : R(a.t_shift);
    R t_own = R(0);
    if constexpr (dev) t_own = GIVEN_T ? tsrc[0] : ld<R>(elem(to, nb.c));

    // f[] holds f - w ts (constant shift) or f - w T^n(own) (deviation storage:
    // stored + w (T^n(source) - T^n(own)), exactly zero in a uniform region at rest)
    R f[Q];
    __builtin_amdgcn_s_setprio(kPullPriority);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int ex = vel<Q>(i, 0), ey = vel<Q>(i, 1), ez = vel<Q>(i, 2);
        const R w = R(weight<Q>(i));
        if (WALL && nb.ghost(-ey)) {
            // anti-bounce-back f_i = 2 w T_w - f*_opp(x)
            const double *tw = ey > 0 ? a.twb : a.twt;
            f[i] = R(2) * w * (R(tw[nb.col(0, 0, a.geo)]) - (dev ? t_own : ts)) -
                   ld<R>(elem(pdf_row<Q>(fs, a.geo, nb.yr[1], nb.zi[1], opposite<Q>(i)), pl.xq[1]));
        } else {
            f[i] = ld<R>(elem(pdf_row<Q>(fs, a.geo, nb.yr[1 - ey], nb.zi[1 - ez], i), pl.xq[1 - ex]));
            if constexpr (dev) {
                if (i != 0) f[i] += w * ((GIVEN_T ? tsrc[i] : ld<R>(nb.ptr(to, -ex, -ey, -ez))) - t_own);
            }
        }
    }
    __builtin_amdgcn_s_setprio(0);
    // zeroth and first moments from sums and differences of opposite pairs
    R Tp = f[0], j[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        if (opposite<Q>(i) < i) continue;
        const int o = opposite<Q>(i);
        const R df = f[i] - f[o];
        Tp += f[i] + f[o];
        if (vel<Q>(i, 0)) j[0] += R(vel<Q>(i, 0)) * df;
        if (vel<Q>(i, 1)) j[1] += R(vel<Q>(i, 1)) * df;
        if (vel<Q>(i, 2)) j[2] += R(vel<Q>(i, 2)) * df;
    }
    const R T = Tp + (dev ? t_own : ts);
    const R phic = fmin(fmax(phi, R(0)), R(1));
    const R kap = R(a.kappa_l) + phic * R(a.dkappa);
    const R om1 = R(1) - R(1) / (R(0.5) + R(3) * kap);
    const R v[3] = {om1 * (j[0] - T * u[0]), om1 * (j[1] - T * u[1]), om1 * (j[2] - T * u[2])};
    R d[Q];
    FirstOrder<Q, R>::apply(u, v, d);
    const R q = heat_source<R>(a.src, x, y, z);
    // f* - w c = w (T (1 + zeta) - c + q) + d with c = ts (constant shift) or T
    // (deviation storage), zeta = 3 e.u + 9/2 (e.u)^2 - 3/2 u.u: opposite
    // directions share the even part and flip 3 T e.u
    const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const R base = (dev ? R(0) : Tp) - R(1.5) * T * uu + q;
    P *fd = static_cast<P *>(a.f_dst);
    st_pdf(elem(pdf_row<Q>(fd, a.geo, nb.yr[1], nb.zi[1], 0), pl.xq[1]), R(weight<Q>(0)) * base + d[0]);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        if (opposite<Q>(i) < i) continue;
        const int o = opposite<Q>(i);
        const int ex = vel<Q>(i, 0), ey = vel<Q>(i, 1), ez = vel<Q>(i, 2);
        const R w = R(weight<Q>(i));
        R eu = R(0);
        if (ex) eu += R(ex) * u[0];
        if (ey) eu += R(ey) * u[1];
        if (ez) eu += R(ez) * u[2];
        const R even = base + R(4.5) * T * eu * eu;
        const R odd = R(3) * T * eu;
        st_pdf(elem(pdf_row<Q>(fd, a.geo, nb.yr[1], nb.zi[1], i), pl.xq[1]), w * (even + odd) + d[i]);
        st_pdf(elem(pdf_row<Q>(fd, a.geo, nb.yr[1], nb.zi[1], o), pl.xq[1]), w * (even - odd) + d[o]);
    }
    st(elem(static_cast<S *>(a.T), nb.c), T);
}

} // namespace tcp
