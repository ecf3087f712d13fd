// kernels_thermal.hip -- the thermal field.
//
// K3, passive-scalar LB (Eq. lb_thermal): pull with anti-bounce-back
// f_i = -f*_opp + 2 w_i T_w at the y walls, T = sum_i f_i, central-moment
// collision about u^{n+1} with the first-order moments relaxed by
// omega_T = 1/(1/2 + kappa(phi)/c_s^2) and all higher ones with rate one, then
// the source w_i q_T (Eq. HeatSource).  Storage in type P: f_i - w_i t_shift
// (FP64), or (FP32, FP16) the deviation f*_i - w_i T(x) from the rest
// equilibrium of the cell, rebuilt in the pull around T^n of the own cell.  T is double
// buffered (T^n read, T^{n+1} written).
//
// RK stages (Eq. rk2 as the midpoint rule, Eq. rk4): each stage evaluates
//   R(theta) = -u . grad theta + (kappa_H - kappa_L) grad phi . grad theta
//              + kappa(phi) lap theta + q_T
// with the isotropic D3Q27 stencils, ghost 2 T_w - theta at walls and the
// contact-angle ghost for phi.  Everything but theta is constant within a
// step, so a coefficient pass per step evaluates the phi stencil and the
// heat source once, and the stages read the result.
#include "cell_thermal.hpp"

namespace tcp {

// One thread per cell; rows next to a wall take the anti-bounce-back path.
template <int Q, typename P, typename S, typename R>
__global__ void __launch_bounds__(kTX *kTY) k_thermal(const ThermalArgs a, const Tiling t)
{
    int x, y, z;
    if (!cell_of_thread(t, a.geo, x, y, z)) return;
    const Nbr nb(a.geo, x, y, z);
    const R phi = ld<R>(elem(static_cast<const S *>(a.phi), nb.c));
    R u[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) u[k] = ld<R>(elem(static_cast<const S *>(a.u[k]), nb.c));
    if (nb.below || nb.above)
        thermal_cell<Q, P, S, R, true>(a, nb, x, y, z, phi, u);
    else
        thermal_cell<Q, P, S, R, false>(a, nb, x, y, z, phi, u);
}

template <int Q, typename P, typename S, typename R>
void launch_thermal(const ThermalArgs &a, hipStream_t s)
{
    const Tiling t = make_tiling(a.geo);
    hipLaunchKernelGGL((k_thermal<Q, P, S, R>), tiling_grid(t), tiling_block(), 0, s, a, t);
}

// Coefficients of the right-hand side, constant within a step (phi^{n+1},
// u^{n+1} and the sources are held while the stages run):
//   R(theta) = a . grad theta + kappa lap theta + q,  a = -u + (kappa_H - kappa_L) grad phi,
// written once per step as five fields (a_x, a_y, a_z, kappa, q); the stages
// then read a and kappa only with a conductivity ratio (gk) and q only with
// heat sources (hq), and otherwise take a = -u^{n+1} and kappa = kappa_L.
template <typename S, typename R, bool WALL>
__device__ __forceinline__ void rk_coef_cell(const RkArgs &a, const Nbr &nb, int x, int y, int z)
{
    S *co = static_cast<S *>(a.coef);
    const int64_t N = a.geo.N;
    if (a.gk) {
        const S *pp = static_cast<const S *>(a.phi);
        R gp[3] = {R(0), R(0), R(0)};
#pragma unroll
        for (int i = 1; i < 27; ++i) {
            const int ex = vel27(i, 0), ey = vel27(i, 1), ez = vel27(i, 2);
            const R w = R(weight<27>(i));
            R pv = ld<R>(nb.ptr(pp, ex, ey, ez));
            if (WALL && nb.ghost(ey)) pv = nb.phi_ghost(pv, ey, a.wet);
            gp[0] += R(ex) * w * pv;
            gp[1] += R(ey) * w * pv;
            gp[2] += R(ez) * w * pv;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k)
            st(elem(co + k * N, nb.c), -ld<R>(elem(static_cast<const S *>(a.u[k]), nb.c)) + R(3) * R(a.dkappa) * gp[k]);
        const R phic = fmin(fmax(ld<R>(elem(pp, nb.c)), R(0)), R(1));
        st(elem(co + 3 * N, nb.c), R(a.kappa_l) + phic * R(a.dkappa));
    }
    if (a.hq) st(elem(co + 4 * N, nb.c), heat_source<R>(a.src, x, y, z));
}

template <typename S, typename R>
__global__ void __launch_bounds__(kTX *kTY) k_rk_coef(const RkArgs a, const Tiling t)
{
    int x, y, z;
    if (!cell_of_thread(t, a.geo, x, y, z)) return;
    const Nbr nb(a.geo, x, y, z);
    if (nb.below || nb.above)
        rk_coef_cell<S, R, true>(a, nb, x, y, z);
    else
        rk_coef_cell<S, R, false>(a, nb, x, y, z);
}

template <typename S, typename R, bool WALL, bool GK, bool HQ>
__device__ __forceinline__ void rk_cell(const RkArgs &a, const Nbr &nb)
{
    const S *th = static_cast<const S *>(a.theta_in);
    const S *co = static_cast<const S *>(a.coef);
    const int64_t N = a.geo.N;
    const R tc = ld<R>(elem(th, nb.c));
    R gt[3] = {R(0), R(0), R(0)}, lap = R(0);
#pragma unroll
    for (int i = 1; i < 27; ++i) {
        const int ex = vel27(i, 0), ey = vel27(i, 1), ez = vel27(i, 2);
        const R w = R(weight<27>(i));
        R tv = ld<R>(nb.ptr(th, ex, ey, ez));
        if (WALL && nb.ghost(ey)) {
            const double *tw = ey < 0 ? a.twb : a.twt;
            tv = R(2) * R(tw[nb.col(ex, ez, a.geo)]) - tv;
        }
        if (ex) gt[0] += R(ex) * w * tv;
        if (ey) gt[1] += R(ey) * w * tv;
        if (ez) gt[2] += R(ez) * w * tv;
        lap += w * tv;
    }
    lap = R(6) * (lap - R(1.0 - weight<27>(0)) * tc);
    R av[3], kap;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        av[k] = GK ? ld<R>(elem(co + k * N, nb.c)) : -ld<R>(elem(static_cast<const S *>(a.u[k]), nb.c));
    kap = GK ? ld<R>(elem(co + 3 * N, nb.c)) : R(a.kappa_l);
    R k = R(3) * (av[0] * gt[0] + av[1] * gt[1] + av[2] * gt[2]) + kap * lap;
    if (HQ) k += ld<R>(elem(co + 4 * N, nb.c));
    S *ap = static_cast<S *>(a.acc);
    const R T = ld<R>(elem(static_cast<const S *>(a.T), nb.c));
    const R acc = (a.first ? R(0) : ld<R>(elem(ap, nb.c))) + R(a.w_acc) * k;
    if (a.last) {
        st(elem(static_cast<S *>(a.T_new), nb.c), T + acc);
    } else {
        if (ap) st(elem(ap, nb.c), acc);
        st(elem(static_cast<S *>(a.theta_out), nb.c), T + R(a.a_next) * k);
    }
}

template <typename S, typename R, bool GK, bool HQ>
__global__ void __launch_bounds__(kTX *kTY) k_rk_stage(const RkArgs a, const Tiling t)
{
    int x, y, z;
    if (!cell_of_thread(t, a.geo, x, y, z)) return;
    const Nbr nb(a.geo, x, y, z);
    if (nb.below || nb.above)
        rk_cell<S, R, true, GK, HQ>(a, nb);
    else
        rk_cell<S, R, false, GK, HQ>(a, nb);
}

template <typename S, typename R>
void launch_rk_coef(const RkArgs &a, hipStream_t s)
{
    if (!a.gk && !a.hq) return;
    const Tiling t = make_tiling(a.geo);
    hipLaunchKernelGGL((k_rk_coef<S, R>), tiling_grid(t), tiling_block(), 0, s, a, t);
}

template <typename S, typename R>
void launch_rk(const RkArgs &a, hipStream_t s)
{
    const Tiling t = make_tiling(a.geo);
    if (a.gk && a.hq) hipLaunchKernelGGL((k_rk_stage<S, R, true, true>), tiling_grid(t), tiling_block(), 0, s, a, t);
    else if (a.gk) hipLaunchKernelGGL((k_rk_stage<S, R, true, false>), tiling_grid(t), tiling_block(), 0, s, a, t);
    else if (a.hq) hipLaunchKernelGGL((k_rk_stage<S, R, false, true>), tiling_grid(t), tiling_block(), 0, s, a, t);
    else hipLaunchKernelGGL((k_rk_stage<S, R, false, false>), tiling_grid(t), tiling_block(), 0, s, a, t);
}

#define TCP_THERMAL_INST(Q)                                                                                  \
    template void launch_thermal<Q, double, double, double>(const ThermalArgs &, hipStream_t);             \
    template void launch_thermal<Q, float, float, float>(const ThermalArgs &, hipStream_t);                \
    template void launch_thermal<Q, _Float16, float, float>(const ThermalArgs &, hipStream_t);
TCP_THERMAL_INST(7)
TCP_THERMAL_INST(15)
TCP_THERMAL_INST(19)
TCP_THERMAL_INST(27)
#undef TCP_THERMAL_INST
template void launch_rk<double, double>(const RkArgs &, hipStream_t);
template void launch_rk<float, float>(const RkArgs &, hipStream_t);
template void launch_rk_coef<double, double>(const RkArgs &, hipStream_t);
template void launch_rk_coef<float, float>(const RkArgs &, hipStream_t);

} // namespace tcp
