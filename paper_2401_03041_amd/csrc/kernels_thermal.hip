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

// What the stage reads at its own cell besides the stencil: a (or -u),
// kappa, q, T^n and the accumulator.
template <typename R>
struct RkOwn {
    R av[3], kap, q, T, acc;
};

template <typename S, typename R, bool GK, bool HQ>
__device__ __forceinline__ void rk_own(const RkArgs &a, uint32_t c, RkOwn<R> &o)
{
    const S *co = static_cast<const S *>(a.coef);
    const int64_t N = a.geo.N;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        o.av[k] = GK ? ld<R>(elem(co + k * N, c)) : -ld<R>(elem(static_cast<const S *>(a.u[k]), c));
    o.kap = GK ? ld<R>(elem(co + 3 * N, c)) : R(a.kappa_l);
    o.q = HQ ? ld<R>(elem(co + 4 * N, c)) : R(0);
    o.T = ld<R>(elem(static_cast<const S *>(a.T), c));
    o.acc = a.first ? R(0) : ld<R>(elem(static_cast<const S *>(a.acc), c));
}

// The stage at cell c from the stencil sums of its argument theta: gt (the
// isotropic gradient without its factor 3) and lap (the Laplacian).
template <typename S, typename R, bool HQ>
__device__ __forceinline__ void rk_tail(const RkArgs &a, uint32_t c, const RkOwn<R> &o, const R (&gt)[3], R lap)
{
    R k = R(3) * (o.av[0] * gt[0] + o.av[1] * gt[1] + o.av[2] * gt[2]) + o.kap * lap;
    if (HQ) k += o.q;
    S *ap = static_cast<S *>(a.acc);
    const R acc = o.acc + R(a.w_acc) * k;
    if (a.last) {
        st(elem(static_cast<S *>(a.T_new), c), o.T + acc);
    } else {
        if (ap) st(elem(ap, c), acc);
        st(elem(static_cast<S *>(a.theta_out), c), o.T + R(a.a_next) * k);
    }
}

// One RK stage (Eq. rk2 / rk4 with the right-hand side of the energy
// equation): the argument theta is staged plane by plane in LDS for a 64 x 4
// tile and its halo while the work-group marches up kMarchZ planes (three
// planes held at a time), so its 27-point stencil costs about 1.55 loads per
// cell instead of 27.  The loads run one plane ahead: while plane z is
// computed, plane z + 2 of theta (for the LDS) and the own-cell values of
// plane z + 1 are already in flight into registers.  A neighbour across a
// wall is the ghost 2 T_w - theta of the mirror cell in the own row.
template <typename S, typename R, bool GK, bool HQ>
__global__ void __launch_bounds__(kTX *kTY) k_rk_stage(const RkArgs a, const March m)
{
    __shared__ R lds[3][kHalo];
    const Geometry &g = a.geo;
    int x0, y0, z0, z1;
    if (!march_tile(m, g, x0, y0, z0, z1)) return;
    const int lx = threadIdx.x, ly = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const int tid = lx + kTX * ly;
    const int x = x0 + lx, y = y0 + ly;
    const bool live = x < g.nx && y < g.ny;
    const bool below = g.walls && y == 0, above = g.walls && y == g.ny - 1;
    const S *th = static_cast<const S *>(a.theta_in);
    const HaloSlots hs(g, x0, y0, tid);
    const uint32_t plane = (uint32_t)g.plane;
    const uint32_t c0 = (uint32_t)x + (uint32_t)y * (uint32_t)g.nx; // own cell within a plane
    R nxt[kHaloPer];
    auto load = [&](int zz) {
#pragma unroll
        for (int j = 0; j < kHaloPer; ++j)
            nxt[j] = hs.in[j] ? ld<R>(elem(th, hs.off[j] + (uint32_t)zz * plane)) : R(0);
    };
    auto put = [&](int slot) {
#pragma unroll
        for (int j = 0; j < kHaloPer; ++j)
            if (hs.own[j]) lds[slot][tid + j * kTX * kTY] = nxt[j];
    };
    load(wrap(z0 - 1, g.nz));
    put(0);
    load(z0);
    put(1);
    load(wrap(z0 + 1, g.nz));
    RkOwn<R> cur{}, ahead{};
    if (live) rk_own<S, R, GK, HQ>(a, c0 + (uint32_t)z0 * plane, cur);
    for (int z = z0; z < z1; ++z) {
        const int k = z - z0;
        const int sl[3] = {k % 3, (k + 1) % 3, (k + 2) % 3}; // planes z - 1, z, z + 1
        put(sl[2]);                                          // plane z + 1, loaded one plane ago
        __syncthreads();
        if (z + 1 < z1) {
            load(wrap(z + 2, g.nz));
            if (live) rk_own<S, R, GK, HQ>(a, c0 + (uint32_t)(z + 1) * plane, ahead);
        }
        if (live) {
            auto at = [&](int dx, int dy, int dz) -> R { return lds[sl[dz + 1]][(ly + 1 + dy) * kHX + (lx + 1 + dx)]; };
            const R tc = at(0, 0, 0);
            R gt[3] = {R(0), R(0), R(0)}, lap = R(0);
#pragma unroll
            for (int i = 1; i < 27; ++i) {
                const int ex = vel27(i, 0), ey = vel27(i, 1), ez = vel27(i, 2);
                const R w = R(weight<27>(i));
                R tv;
                if ((ey < 0 && below) || (ey > 0 && above)) {
                    const double *tw = ey < 0 ? a.twb : a.twt;
                    const uint32_t col = (uint32_t)wrap(x + ex, g.nx) + (uint32_t)wrap(z + ez, g.nz) * (uint32_t)g.nx;
                    tv = R(2) * R(tw[col]) - at(ex, 0, ez);
                } else {
                    tv = at(ex, ey, ez);
                }
                if (ex) gt[0] += R(ex) * w * tv;
                if (ey) gt[1] += R(ey) * w * tv;
                if (ez) gt[2] += R(ez) * w * tv;
                lap += w * tv;
            }
            lap = R(6) * (lap - R(1.0 - weight<27>(0)) * tc);
            rk_tail<S, R, HQ>(a, c0 + (uint32_t)z * plane, cur, gt, lap);
        }
        cur = ahead;
        __syncthreads(); // the next plane's put overwrites the slot of plane z - 1
    }
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
    const March m = make_march(a.geo);
    const dim3 gr = march_grid(m), bl = tiling_block();
    if (a.gk && a.hq) hipLaunchKernelGGL((k_rk_stage<S, R, true, true>), gr, bl, 0, s, a, m);
    else if (a.gk) hipLaunchKernelGGL((k_rk_stage<S, R, true, false>), gr, bl, 0, s, a, m);
    else if (a.hq) hipLaunchKernelGGL((k_rk_stage<S, R, false, true>), gr, bl, 0, s, a, m);
    else hipLaunchKernelGGL((k_rk_stage<S, R, false, false>), gr, bl, 0, s, a, m);
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
