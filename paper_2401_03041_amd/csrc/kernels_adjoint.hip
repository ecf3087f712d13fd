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
//
// RK2 / RK4 with the flow held: R(theta) = A theta + b is affine, with
//   (A theta)(c) = sum_k C_k(c) theta(c + e_k) - 6 kappa(c) (1 - w_0) theta(c),
//   C_k(c) = w_k (3 a(c) . e_k + 6 kappa(c)),  a = -u + (kappa_H - kappa_L) grad phi,
// the D3Q27 weights w_k, a neighbour across a wall replaced by its ghost
// 2 T_w - theta(mirror cell), and b = q plus the ghosts' 2 C_k T_w.  For
// T' = T + sum_s w_s K_s, K_s = R(theta_s), theta_1 = T, theta_{s+1} = T + a_s K_s
// the reverse sweep over the stages is
//   kappa_s = w_s lambda' + a_s A^T kappa_{s+1}   (s = S .. 1),
//   lambda  = lambda' + sum_s A^T kappa_s,
// with dL/dq(x) += kappa_s(x) and dL/dT_w += 2 C_k kappa_s over the ghost links.
// A^T is applied as a gather: cell x collects C_k(x - e_k) kappa(x - e_k) over
// the links that reach it, minus C_k(c) kappa(c) over the ghost links whose
// mirror cell it is (c in its own row, shifted by -e_k in x and z).  The
// stage kernel stages C_k(c) kappa(c) = w_k (e_k . B(c) + D(c)) as four values
// per cell in LDS, so the gather reads four values per link from LDS and
// every input from memory once.
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

// a = -u + (kappa_H - kappa_L) grad phi and kappa(phi) per cell (phi and u
// held), the coefficients of the RK right-hand side; grad phi with the
// contact-angle ghosts as in the forward stages
template <typename S, typename R>
__global__ void __launch_bounds__(kTX *kTY) k_rk_adj_coeff(const RkAdjointArgs a, const Tiling t)
{
    int x, y, z;
    if (!cell_of_thread(t, a.geo, x, y, z)) return;
    const Nbr nb(a.geo, x, y, z);
    const S *pp = static_cast<const S *>(a.phi);
    R gp[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int i = 1; i < 27; ++i) {
        const int ex = vel27(i, 0), ey = vel27(i, 1), ez = vel27(i, 2);
        const R w = R(weight<27>(i));
        R pv = ld<R>(nb.ptr(pp, ex, ey, ez));
        if (nb.ghost(ey)) pv = nb.phi_ghost(pv, ey, a.wet);
        gp[0] += R(ex) * w * pv;
        gp[1] += R(ey) * w * pv;
        gp[2] += R(ez) * w * pv;
    }
    S *co = static_cast<S *>(a.coeff);
    const int64_t N = a.geo.N;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const R u = ld<R>(elem(static_cast<const S *>(a.u[k]), nb.c));
        st(elem(co + k * N, nb.c), -u + R(a.dkappa) * R(3) * gp[k]);
    }
    const R phic = fmin(fmax(ld<R>(elem(pp, nb.c)), R(0)), R(1));
    st(elem(co + 3 * N, nb.c), R(a.kappa_l) + phic * R(a.dkappa));
}

// One reverse RK stage in one pass.  A work-group owns a 64 x 4 tile of cells
// and marches up kMarchZ planes of it.  For every plane it stages, for the tile
// and a one-cell halo in x and y, the packed link sources of the stage,
//   kappa = w_s lambda' + a_s theta_in,  B = 3 kappa a,  D = 6 kappa kappa(phi),
// so that C_k(c) kappa(c) = w_k (e_k . B(c) + D(c)), in LDS; three planes
// (z - 1, z, z + 1) are held at a time, each read from memory once per
// column.  Each cell then gathers theta_out = A^T kappa from LDS, adds it to
// acc (which starts from lambda' in the last stage) and collects the source
// and wall gradients of the stage.

// The loads run one plane ahead, as in the forward stage: while plane z is
// gathered, the inputs of plane z + 2's packed sources (for the LDS) and the
// own-cell values of plane z + 1 are already in flight into registers.
template <typename S, typename R>
__global__ void __launch_bounds__(kTX *kTY) k_rk_adj_march(const RkAdjointArgs a, const March m)
{
    __shared__ R lds[3][4][kHalo];
    const Geometry &g = a.geo;
    int x0, y0, z0, z1;
    if (!march_tile(m, g, x0, y0, z0, z1)) return;
    const int lx = threadIdx.x, ly = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const int tid = lx + kTX * ly;
    const int x = x0 + lx, y = y0 + ly;
    const bool live = x < g.nx && y < g.ny;
    const bool below = g.walls && y == 0, above = g.walls && y == g.ny - 1;
    const S *lam = static_cast<const S *>(a.lam);
    const S *thi = static_cast<const S *>(a.theta_in);
    const S *co = static_cast<const S *>(a.coeff);
    const uint32_t N = (uint32_t)g.N, plane = (uint32_t)g.plane;
    const uint32_t c0 = (uint32_t)x + (uint32_t)y * (uint32_t)g.nx; // own cell within a plane
    const HaloSlots hs(g, x0, y0, tid);

    // inputs of the packed sources of the staged entries: lambda', theta_in, a, kappa
    R pl[kHaloPer], pt[kHaloPer], pc[kHaloPer][4];
    auto load = [&](int zz) {
#pragma unroll
        for (int j = 0; j < kHaloPer; ++j) {
            const uint32_t c = hs.off[j] + (uint32_t)zz * plane;
            pl[j] = hs.in[j] ? ld<R>(elem(lam, c)) : R(0);
            pt[j] = hs.in[j] && thi ? ld<R>(elem(thi, c)) : R(0);
#pragma unroll
            for (int q = 0; q < 4; ++q) pc[j][q] = hs.in[j] ? ld<R>(elem(co + q * N, c)) : R(0);
        }
    };
    // packed sources kappa = w_s lambda' + a_s theta_in, B = 3 kappa a,
    // D = 6 kappa kappa(phi); entries in rows beyond a wall are never gathered
    // from and hold zeros
    auto put = [&](int slot) {
#pragma unroll
        for (int j = 0; j < kHaloPer; ++j) {
            if (!hs.own[j]) continue;
            R k = R(a.w_s) * pl[j];
            if (thi) k += R(a.a_s) * pt[j];
            const int i = tid + j * kTX * kTY;
#pragma unroll
            for (int q = 0; q < 3; ++q) lds[slot][q][i] = R(3) * k * pc[j][q];
            lds[slot][3][i] = R(6) * k * pc[j][3];
        }
    };
    // own-cell values: lambda', theta_in, acc
    struct Own {
        R l, t, acc;
    } cur{}, ahead{};
    auto own = [&](int zz, Own &o) {
        const uint32_t c = c0 + (uint32_t)zz * plane;
        o.l = ld<R>(elem(lam, c));
        o.t = thi ? ld<R>(elem(thi, c)) : R(0);
        o.acc = a.first ? R(0) : ld<R>(elem(static_cast<const S *>(a.acc), c));
    };

    load(wrap(z0 - 1, g.nz));
    put(0);
    load(z0);
    put(1);
    load(wrap(z0 + 1, g.nz));
    if (live) own(z0, cur);
    for (int z = z0; z < z1; ++z) {
        const int k = z - z0;
        // slots of planes z - 1, z, z + 1
        const int sl[3] = {k % 3, (k + 1) % 3, (k + 2) % 3};
        put(sl[2]); // plane z + 1, loaded one plane ago
        __syncthreads();
        if (z + 1 < z1) {
            load(wrap(z + 2, g.nz));
            if (live) own(z + 1, ahead);
        }
        if (live) {
            // LDS element of the cell at offset (dx, dy, dz), component j
            auto at = [&](int j, int dx, int dy, int dz) -> R {
                return lds[sl[dz + 1]][j][(ly + 1 + dy) * kHX + (lx + 1 + dx)];
            };
            R out = -R(1.0 - 8.0 / 27.0) * at(3, 0, 0, 0);
            R refl[2] = {R(0), R(0)}; // ghost links mirrored onto this cell: bottom, top
#pragma unroll
            for (int i = 1; i < 27; ++i) {
                const int ex = vel27(i, 0), ey = vel27(i, 1), ez = vel27(i, 2);
                const R wi = R(weight<27>(i));
                if (!((ey > 0 && below) || (ey < 0 && above))) {
                    // the link from c = x - e_i reaches this cell
                    R v = at(3, -ex, -ey, -ez);
                    if (ex) v += R(ex) * at(0, -ex, -ey, -ez);
                    if (ey) v += R(ey) * at(1, -ex, -ey, -ez);
                    if (ez) v += R(ez) * at(2, -ex, -ey, -ez);
                    out += wi * v;
                }
                if ((ey < 0 && below) || (ey > 0 && above)) {
                    // the link from c = x - (e_x, 0, e_z) in this row leaves through
                    // the wall; its ghost mirrors onto this cell
                    R v = at(3, -ex, 0, -ez);
                    if (ex) v += R(ex) * at(0, -ex, 0, -ez);
                    v += R(ey) * at(1, -ex, 0, -ez);
                    if (ez) v += R(ez) * at(2, -ex, 0, -ez);
                    refl[ey > 0] += wi * v;
                }
            }
            out -= refl[0] + refl[1];
            const uint32_t c = c0 + (uint32_t)z * plane;
            st(elem(static_cast<S *>(a.theta_out), c), out);
            st(elem(static_cast<S *>(a.acc), c), (a.first ? cur.l : cur.acc) + out);
            R kc = R(a.w_s) * cur.l;
            if (thi) kc += R(a.a_s) * cur.t;
            a.grad_q[c] += static_cast<double>(kc);
            if (below || above) {
                const uint32_t col = (uint32_t)x + (uint32_t)z * (uint32_t)g.nx;
                if (below) a.grad_twb[col] += 2.0 * static_cast<double>(refl[0]);
                if (above) a.grad_twt[col] += 2.0 * static_cast<double>(refl[1]);
            }
        }
        cur = ahead;
        __syncthreads(); // the next plane's put overwrites the slot of plane z - 1
    }
}

} // namespace

template <typename S, typename R>
void launch_rk_adjoint_coeff(const RkAdjointArgs &a, hipStream_t s)
{
    const Tiling t = make_tiling(a.geo);
    hipLaunchKernelGGL((k_rk_adj_coeff<S, R>), tiling_grid(t), tiling_block(), 0, s, a, t);
}

template <typename S, typename R>
void launch_rk_adjoint_stage(const RkAdjointArgs &a, hipStream_t s)
{
    const March m = make_march(a.geo);
    hipLaunchKernelGGL((k_rk_adj_march<S, R>), march_grid(m), tiling_block(), 0, s, a, m);
}

template void launch_rk_adjoint_coeff<double, double>(const RkAdjointArgs &, hipStream_t);
template void launch_rk_adjoint_coeff<float, float>(const RkAdjointArgs &, hipStream_t);
template void launch_rk_adjoint_stage<double, double>(const RkAdjointArgs &, hipStream_t);
template void launch_rk_adjoint_stage<float, float>(const RkAdjointArgs &, hipStream_t);

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
