// kernels_adjoint.hip -- adjoint of the thermal LB update with the flow held.
//
// With phi and u fixed, one update of the thermal LB (Eq. lb_thermal with the
// anti-bounce-back walls and the source of Eq. HeatSource) is affine in the
// PDFs, the source amplitudes Q_k and the wall temperatures:
//   pull        fp_i(x) = f_i(x - e_i), or -f_opp(x) + 2 w_i T_w across a wall
//   T(x)      = sum_i fp_i
//   collision f*_i = w_i (1 + zeta_i(u)) T + sum_a D_ia(u) v_a + w_i q(x),
//               v_a = (1 - omega_T) (j_a - T u_a),  j_a = sum_i e_ia fp_i,
// where D(u) is the linear map FirstOrder<Q>::apply.  For a loss
// L = sum_x m(x) T(x) after N updates, the adjoint runs the updates
// backwards.  The state kept between adjoint updates is mu = dL/dfp (one value
// per link, stored like the PDFs):
//   lambda_i(x) = dL/df_i(x) = mu_i(x + e_i), or -mu_opp(x) where x + e_i
//                 lies across a wall (the link that reflected f_i(x));
//   mu_j(x)     = s0 + (1 - omega_T) sum_a (e_ja - u_a) s_a,
//                 s0 = sum_i lambda_i w_i (1 + zeta_i),  s_a = sum_i lambda_i D_ia;
// the source gets sum_i w_i lambda_i(x) per update, a wall column
// 2 w_opp mu_opp(x) per reflected link.  The last update's T seeds mu = m.
#include "kernels.hpp"

namespace tcp {

namespace {

constexpr int kThreads = 256;

// mu of the last update: dL/dfp_j = m(x) for every link
template <int Q, typename S>
__global__ void __launch_bounds__(kTX *kTY) k_adj_seed(const Geometry g, const Tiling t, const double *m, S *mu)
{
    int x, y, z;
    if (!cell_of_thread(t, g, x, y, z)) return;
    const Nbr nb(g, x, y, z);
    const PdfLanes<Q> pl(nb);
    const S v = static_cast<S>(m[nb.c]);
#pragma unroll
    for (int i = 0; i < Q; ++i) st(elem(pdf_row<Q>(mu, g, nb.yr[1], nb.zi[1], i), pl.xq[1]), v);
}

template <int Q, typename S, typename R, bool WALL>
__device__ __forceinline__ void adjoint_cell(const ThermalAdjointArgs &a, const Nbr &nb)
{
    const S *mi = static_cast<const S *>(a.mu_src);
    const PdfLanes<Q> pl(nb);
    // lambda = dL/df of the previous update's output
    R lam[Q];
    R wall_grad[2] = {R(0), R(0)}; // bottom, top
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int ex = vel<Q>(i, 0), ey = vel<Q>(i, 1), ez = vel<Q>(i, 2);
        if (WALL && nb.ghost(ey)) {
            const int o = opposite<Q>(i);
            const R m_o = ld<R>(elem(pdf_row<Q>(mi, a.geo, nb.yr[1], nb.zi[1], o), pl.xq[1]));
            lam[i] = -m_o;
            wall_grad[ey > 0] += R(2) * R(weight<Q>(o)) * m_o;
        } else {
            lam[i] = ld<R>(elem(pdf_row<Q>(mi, a.geo, nb.yr[1 + ey], nb.zi[1 + ez], i), pl.xq[1 + ex]));
        }
    }
    if (WALL) {
        // one wall-adjacent cell per column and wall: it owns the column's sums
        const uint32_t col = nb.col(0, 0, a.geo);
        if (nb.below) a.grad_twb[col] += static_cast<double>(wall_grad[0]);
        if (nb.above) a.grad_twt[col] += static_cast<double>(wall_grad[1]);
    }
    if (!a.last) {
        // the previous update's source term w_i q(x)
        R sq = R(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) sq += R(weight<Q>(i)) * lam[i];
        a.grad_q[nb.c] += static_cast<double>(sq);

        R u[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) u[k] = ld<R>(elem(static_cast<const S *>(a.u[k]), nb.c));
        const R phic = fmin(fmax(ld<R>(elem(static_cast<const S *>(a.phi), nb.c)), R(0)), R(1));
        const R kap = R(a.kappa_l) + phic * R(a.dkappa);
        const R om1 = R(1) - R(1) / (R(0.5) + R(3) * kap);
        const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        // s0 = sum_i lambda_i w_i (1 + zeta_i)
        R s0 = R(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const R eu = R(vel<Q>(i, 0)) * u[0] + R(vel<Q>(i, 1)) * u[1] + R(vel<Q>(i, 2)) * u[2];
            s0 += R(weight<Q>(i)) * (R(1) + R(3) * eu + R(4.5) * eu * eu - R(1.5) * uu) * lam[i];
        }
        // s_a = sum_i lambda_i D_ia: D applied to the unit vectors
        R s[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const R unit[3] = {R(ax == 0), R(ax == 1), R(ax == 2)};
            R d[Q];
            FirstOrder<Q, R>::apply(u, unit, d);
            R acc = R(0);
#pragma unroll
            for (int i = 0; i < Q; ++i) acc += d[i] * lam[i];
            s[ax] = om1 * acc;
        }
        const R base = s0 - (u[0] * s[0] + u[1] * s[1] + u[2] * s[2]);
        S *mo = static_cast<S *>(a.mu_dst);
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            R v = base;
            if (vel<Q>(j, 0)) v += R(vel<Q>(j, 0)) * s[0];
            if (vel<Q>(j, 1)) v += R(vel<Q>(j, 1)) * s[1];
            if (vel<Q>(j, 2)) v += R(vel<Q>(j, 2)) * s[2];
            st(elem(pdf_row<Q>(mo, a.geo, nb.yr[1], nb.zi[1], j), pl.xq[1]), v);
        }
    }
}

template <int Q, typename S, typename R>
__global__ void __launch_bounds__(kTX *kTY) k_adj_step(const ThermalAdjointArgs a, const Tiling t)
{
    int x, y, z;
    if (!cell_of_thread(t, a.geo, x, y, z)) return;
    const Nbr nb(a.geo, x, y, z);
    if (nb.below || nb.above)
        adjoint_cell<Q, S, R, true>(a, nb);
    else
        adjoint_cell<Q, S, R, false>(a, nb);
}

// Source gradients from the accumulated source adjoint G: with the profile
// g_k(x) = exp(-2 |x - x_k|^2 / w_k^2) (inside the cut-off), q = sum_k Q_k g_k
// and dg_k/dx_k = 4 (x - x_k) g_k / w_k^2, so
//   dL/dQ_k = sum_x G g_k,   dL/dx_k = Q_k sum_x G g_k 4 (x - x_k) / w_k^2
// (the cut-off sphere moves with the source; its rim is a set of measure zero
// and contributes nothing).  Four sums per source: partial sums per
// work-group, then one work-group.
__global__ void __launch_bounds__(kThreads) k_source_grad_partial(const Geometry g, const HeatSources hs,
                                                                  const double *G, double *partial)
{
    __shared__ double sh[4][kThreads];
    for (int k = 0; k < hs.n; ++k) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x; c < g.N; c += (int64_t)gridDim.x * kThreads) {
            const int x = (int)(c % g.nx), y = (int)((c / g.nx) % g.ny), z = (int)(c / g.plane);
            const double dx = x - hs.x[k], dy = y - hs.y[k], dz = z - hs.z[k];
            const double d2 = dx * dx + dy * dy + dz * dz;
            if (hs.dcut2[k] > 0.0 && d2 > hs.dcut2[k]) continue;
            const double v = G[c] * exp(-2.0 * d2 * hs.inv_w2[k]);
            const double s = 4.0 * hs.inv_w2[k] * v;
            acc[0] += v;
            acc[1] += s * dx;
            acc[2] += s * dy;
            acc[3] += s * dz;
        }
        for (int j = 0; j < 4; ++j) sh[j][threadIdx.x] = acc[j];
        __syncthreads();
        for (int s = kThreads / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s)
                for (int j = 0; j < 4; ++j) sh[j][threadIdx.x] += sh[j][threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0)
            for (int j = 0; j < 4; ++j) partial[4 * (kMaxSources * blockIdx.x + k) + j] = sh[j][0];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kThreads) k_source_grad_final(const double *partial, int nblocks,
                                                                const HeatSources hs, double *out)
{
    __shared__ double sh[kThreads];
    for (int k = 0; k < hs.n; ++k) {
        for (int j = 0; j < 4; ++j) {
            double acc = 0.0;
            for (int b = threadIdx.x; b < nblocks; b += kThreads) acc += partial[4 * (kMaxSources * b + k) + j];
            sh[threadIdx.x] = acc;
            __syncthreads();
            for (int s = kThreads / 2; s > 0; s >>= 1) {
                if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
                __syncthreads();
            }
            if (threadIdx.x == 0) out[4 * k + j] = j == 0 ? sh[0] : hs.Q[k] * sh[0];
            __syncthreads();
        }
    }
}

} // namespace

template <int Q, typename S>
void launch_adjoint_seed(const Geometry &g, const double *m, void *mu, hipStream_t s)
{
    const Tiling t = make_tiling(g);
    hipLaunchKernelGGL((k_adj_seed<Q, S>), tiling_grid(t), tiling_block(), 0, s, g, t, m, static_cast<S *>(mu));
}

template <int Q, typename S, typename R>
void launch_adjoint_step(const ThermalAdjointArgs &a, hipStream_t s)
{
    const Tiling t = make_tiling(a.geo);
    hipLaunchKernelGGL((k_adj_step<Q, S, R>), tiling_grid(t), tiling_block(), 0, s, a, t);
}

void launch_source_grad(const Geometry &g, const HeatSources &hs, const double *G, double *partial, double *out,
                        hipStream_t s)
{
    hipLaunchKernelGGL(k_source_grad_partial, dim3(kSourceGradBlocks), dim3(kThreads), 0, s, g, hs, G, partial);
    hipLaunchKernelGGL(k_source_grad_final, dim3(1), dim3(kThreads), 0, s, partial, kSourceGradBlocks, hs, out);
}

#define TCP_ADJ_INST(Q)                                                                                      \
    template void launch_adjoint_seed<Q, double>(const Geometry &, const double *, void *, hipStream_t);    \
    template void launch_adjoint_seed<Q, float>(const Geometry &, const double *, void *, hipStream_t);     \
    template void launch_adjoint_step<Q, double, double>(const ThermalAdjointArgs &, hipStream_t);          \
    template void launch_adjoint_step<Q, float, float>(const ThermalAdjointArgs &, hipStream_t);
TCP_ADJ_INST(7)
TCP_ADJ_INST(15)
TCP_ADJ_INST(19)
TCP_ADJ_INST(27)
#undef TCP_ADJ_INST

} // namespace tcp
