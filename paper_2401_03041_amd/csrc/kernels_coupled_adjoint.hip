// kernels_coupled_adjoint.hip -- reverse (adjoint) kernels of one coupled
// time step with the thermal LB: phase field (K1), hydrodynamics (K2) and
// thermal LB (K3) of Algorithm 1, run backwards K3 -> K2 -> K1.
//
// Notation for step n -> n+1 (time levels of the forward kernels): K1 reads
// the pulled h, the stencil of phi^n and u^n(x) and writes h*, phi^{n+1};
// K2 reads the pulled g and the stencils of phi^n and T^n and writes g*,
// u^{n+1}; K3 reads the pulled f, u^{n+1}(x), phi^{n+1}(x) and writes f*,
// T^{n+1}.  The adjoint carried from step n+1 back to step n is, per cell:
//   mu_h, mu_g, mu_f  dL/d(pulled PDFs) of step n+1 (blocked like the PDFs);
//   sphi = (Gamma_x, Gamma_y, Gamma_z, Lambda, Pi): dL/d of the isotropic
//          gradient and Laplacian of phi^{n+1} at the cell and dL/d of the
//          cell's own phi^{n+1} as K2 of step n+1 reads it;
//   sT   = (GammaT_x, GammaT_y, GammaT_z, PiT): the same for T^{n+1};
//   lu1  = dL/du^{n+1} from K1 of step n+1.
// Reverse step n, one thread per cell, three phases in turn:
//   R3 gathers dL/df*^{n+1}(x, i) = mu_f(x + e_i, i) (or -mu_f(x, opp i)
//      across a wall: anti-bounce-back) and dL/dT^{n+1}(x) from sT (the
//      transpose of the gradient stencil, with the wall ghosts 2 T_w - T),
//      recomputes K3 of step n at x and runs it backwards: mu_f, the local
//      adjoints of u^{n+1} and phi^{n+1}, the heat-source adjoint
//      sum_i w_i dL/df*_i and the wall-temperature adjoints of the reflected
//      links and of the ghosts;
//   R2 gathers dL/dg*^{n+1} (bounce-back across walls), adds lu1 and R3's
//      adjoint for u^{n+1}, recomputes K2 and writes mu_g and sT of step n;
//   R1 gathers dL/dh*^{n+1} and dL/dphi^{n+1} (transposed gradient and
//      Laplacian of sphi, with the derivative of the contact-angle ghost,
//      plus R3's adjoint), recomputes K1, writes mu_h and lu1, and writes
//      sphi of step n (R2's stencil adjoints plus K1's gradient adjoint).
// Every gather reads values the neighbours wrote in the previous reverse
// step (the src buffers), so there are no atomics, the result does not
// depend on scheduling, and the three phases could run in one kernel; they
// run in two, R3 and R2 then R1, each needing fewer registers.
#include "adjoint_math.hpp"
#include "kernels.hpp"

namespace tcp {

namespace {

template <int Q, typename A>
__device__ __forceinline__ A *mu_at(A *base, const Geometry &g, const Nbr &nb, const PdfLanes<Q> &pl, int i, int dx,
                                    int dy, int dz)
{
    return elem(pdf_row<Q>(base, g, nb.yr[1 + dy], nb.zi[1 + dz], i), pl.xq[1 + dx]);
}

// dL/d(post-collision PDF i at this cell) from the link adjoints of the next
// step: the link leads to x + e_i, or back into the cell's own opposite
// direction where x + e_i lies across a wall (sign -1 for anti-bounce-back)
template <int Q, typename A, typename R, bool WALL>
__device__ __forceinline__ void gather_links(const A *mu, const Geometry &g, const Nbr &nb, R sign_wall, R a[Q])
{
    const PdfLanes<Q> pl(nb);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int ex = vel<Q>(i, 0), ey = vel<Q>(i, 1), ez = vel<Q>(i, 2);
        if (WALL && nb.ghost(ey))
            a[i] = sign_wall * ld<R>(mu_at<Q>(mu, g, nb, pl, opposite<Q>(i), 0, 0, 0));
        else
            a[i] = ld<R>(mu_at<Q>(mu, g, nb, pl, i, ex, ey, ez));
    }
}

// A copy of the neighbour offsets that the compiler cannot prove equal to the
// original, so that it does not keep the offsets the three phases share live
// from the first phase to the last.
__device__ __forceinline__ Nbr opaque(const Nbr &nb)
{
    Nbr o = nb;
#pragma unroll
    for (int k = 0; k < 3; ++k) asm volatile("" : "+v"(o.xo[k]));
    return o;
}

// ---------------------------------------------------------------------------
// R3: thermal LB.  Returns K3's local adjoints of u^{n+1} and phi^{n+1}.
// ---------------------------------------------------------------------------
template <int Q, typename P, typename S, typename R, bool WALL>
__device__ __forceinline__ void adj_thermal_cell(const CoupledAdjointArgs &a, const Nbr &nb, R (&au)[3], R &aphi)
{
    constexpr bool dev = deviation_storage<P>();
    const Geometry &g = a.geo;
    const int64_t N = g.N;
    const uint32_t col = nb.col(0, 0, g);

    // recompute K3 of step n: moments of the pulled f (actual values,
    // anti-bounce-back), u^{n+1}, phi^{n+1}
    R T0, j[3];
    {
        const P *fs = static_cast<const P *>(a.s0.f);
        const S *to = static_cast<const S *>(a.s0.T);
        const PdfLanes<Q> pl(nb);
        const R t_own = dev ? ld<R>(elem(to, nb.c)) : R(0);
        R f[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int ex = vel<Q>(i, 0), ey = vel<Q>(i, 1), ez = vel<Q>(i, 2);
            const R w = R(weight<Q>(i));
            if (WALL && nb.ghost(-ey)) {
                const double *tw = ey > 0 ? a.twb : a.twt;
                const R fo = ld<R>(elem(pdf_row<Q>(fs, g, nb.yr[1], nb.zi[1], opposite<Q>(i)), pl.xq[1])) +
                             w * (dev ? t_own : R(a.t_shift));
                f[i] = R(2) * w * R(tw[col]) - fo;
            } else {
                f[i] = ld<R>(elem(pdf_row<Q>(fs, g, nb.yr[1 - ey], nb.zi[1 - ez], i), pl.xq[1 - ex]));
                f[i] += w * (dev ? ld<R>(nb.ptr(to, -ex, -ey, -ez)) : R(a.t_shift));
            }
        }
        moments01<Q, R>(f, T0, j);
    }
    R u[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) u[k] = ld<R>(elem(static_cast<const S *>(a.s1.u[k]), nb.c));
    const R phi = ld<R>(elem(static_cast<const S *>(a.s1.phi), nb.c));

    // dL/dT^{n+1}: own PiT plus the transposed gradient stencil of K2 of step n+1
    const S *sT = static_cast<const S *>(a.sT_src);
    R aT = ld<R>(elem(sT + 3 * N, nb.c));
    R ghost_sum[2] = {R(0), R(0)};
#pragma unroll
    for (int k = 1; k < 27; ++k) {
        const int ex = vel27(k, 0), ey = vel27(k, 1), ez = vel27(k, 2);
        const R w3 = R(3.0 * weight<27>(k));
        if (!(WALL && nb.ghost(-ey))) {
            R v = R(0);
            if (ex) v += R(ex) * ld<R>(nb.ptr(sT, -ex, -ey, -ez));
            if (ey) v += R(ey) * ld<R>(nb.ptr(sT + N, -ex, -ey, -ez));
            if (ez) v += R(ez) * ld<R>(nb.ptr(sT + 2 * N, -ex, -ey, -ez));
            aT += w3 * v;
        }
        if (WALL && nb.ghost(ey)) {
            // the link of the cell x - (e_x, 0, e_z) that leaves through the wall
            // reads the ghost 2 T_w - T of this cell
            R v = R(0);
            if (ex) v += R(ex) * ld<R>(nb.ptr(sT, -ex, 0, -ez));
            v += R(ey) * ld<R>(nb.ptr(sT + N, -ex, 0, -ez));
            if (ez) v += R(ez) * ld<R>(nb.ptr(sT + 2 * N, -ex, 0, -ez));
            ghost_sum[ey > 0] += w3 * v;
        }
    }
    double gtw[2] = {0.0, 0.0};
    if (WALL) {
        aT -= ghost_sum[0] + ghost_sum[1];
        gtw[0] = 2.0 * (double)ghost_sum[0];
        gtw[1] = 2.0 * (double)ghost_sum[1];
    }

    // dL/df*^{n+1}
    R lam[Q];
    gather_links<Q, S, R, WALL>(static_cast<const S *>(a.mu_src[2]), g, nb, R(-1), lam);
    R aj[3], aq;
    au[0] = au[1] = au[2] = R(0);
    thermal_vjp<Q, R>(a.th, T0, j, u, phi, lam, aT, aj, au, aphi, aq);
    {
        S *mu = static_cast<S *>(a.mu_dst[2]);
        const PdfLanes<Q> pl(nb);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const R m = moment01_adjoint<Q, R>(aT, aj, i);
            st(mu_at<Q>(mu, g, nb, pl, i, 0, 0, 0), m);
            // anti-bounce-back links of step n: f_i = 2 w_i T_w - f*_opp
            if (WALL && nb.ghost(-vel<Q>(i, 1))) gtw[vel<Q>(i, 1) < 0] += 2.0 * weight<Q>(i) * (double)m;
        }
    }
    a.grad_q[nb.c] += (double)aq;
    if (WALL) {
        if (nb.below) a.grad_twb[col] += gtw[0];
        if (nb.above) a.grad_twt[col] += gtw[1];
    }
}

// ---------------------------------------------------------------------------
// R2: hydrodynamics.  au3: K3's adjoint of u^{n+1}; returns the adjoints of
// the phi^n stencil reads (gradient, Laplacian, own value).
// ---------------------------------------------------------------------------
template <typename S, typename R, bool WALL>
__device__ __forceinline__ void adj_hydro_cell(const CoupledAdjointArgs &a, const Nbr &nb, const R (&au3)[3],
                                               R (&sp)[5])
{
    const Geometry &g = a.geo;
    const int64_t N = g.N;

    // recompute K2 of step n: raw moments of the pulled g (bounce-back, moving wall)
    HyMom<R> M;
    {
        const S *gs = static_cast<const S *>(a.s0.g);
        const PdfLanes<27> pl(nb);
        R gp[27];
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            const int ex = vel27(i, 0), ey = vel27(i, 1), ez = vel27(i, 2);
            if (WALL && nb.ghost(-ey)) {
                const double *uw = ey > 0 ? a.uw_bot : a.uw_top;
                const double eu = ex * uw[0] + ey * uw[1] + ez * uw[2];
                gp[i] = ld<R>(elem(pdf_row<27>(gs, g, nb.yr[1], nb.zi[1], opposite<27>(i)), pl.xq[1])) +
                        R(6.0 * weight<27>(i) * eu);
            } else {
                gp[i] = ld<R>(elem(pdf_row<27>(gs, g, nb.yr[1 - ey], nb.zi[1 - ez], i), pl.xq[1 - ex]));
            }
        }
        M = hydro_moments<R>(gp);
    }
    // stencils of phi^n and T^n (wall ghosts as in the forward kernel)
    HyIn<R> in;
    {
        const S *pp = static_cast<const S *>(a.s0.phi);
        const S *tp = static_cast<const S *>(a.s0.T);
        in.phi = ld<R>(elem(pp, nb.c));
        in.T = ld<R>(elem(tp, nb.c));
        R lap = R(0);
        for (int k = 0; k < 3; ++k) in.gp[k] = in.gT[k] = R(0);
#pragma unroll
        for (int i = 1; i < 27; ++i) {
            const int ex = vel27(i, 0), ey = vel27(i, 1), ez = vel27(i, 2);
            const R w = R(weight<27>(i));
            R pv = ld<R>(nb.ptr(pp, ex, ey, ez));
            R tv = ld<R>(nb.ptr(tp, ex, ey, ez));
            if (WALL && nb.ghost(ey)) {
                pv = nb.phi_ghost(pv, ey, a.wet);
                const double *tw = ey < 0 ? a.twb : a.twt;
                tv = R(2) * R(tw[nb.col(ex, ez, g)]) - tv;
            }
            if (ex) { in.gp[0] += R(ex) * w * pv; in.gT[0] += R(ex) * w * tv; }
            if (ey) { in.gp[1] += R(ey) * w * pv; in.gT[1] += R(ey) * w * tv; }
            if (ez) { in.gp[2] += R(ez) * w * pv; in.gT[2] += R(ez) * w * tv; }
            lap += w * pv;
        }
        for (int k = 0; k < 3; ++k) {
            in.gp[k] *= R(3);
            in.gT[k] *= R(3);
        }
        in.lap = R(6) * (lap - R(1.0 - weight<27>(0)) * in.phi);
    }
    // dL/dg*^{n+1} and dL/du^{n+1}
    R lam[27];
    gather_links<27, S, R, WALL>(static_cast<const S *>(a.mu_src[1]), g, nb, R(1), lam);
    R au[3];
    const S *lu1 = static_cast<const S *>(a.lu1);
#pragma unroll
    for (int k = 0; k < 3; ++k) au[k] = ld<R>(elem(lu1 + k * N, nb.c)) + au3[k];

    HyMom<R> am;
    HyAdj<R> ad;
    hydro_vjp<R>(a.hy, M, in, lam, au, am, ad);
    {
        S *mu = static_cast<S *>(a.mu_dst[1]);
        const PdfLanes<27> pl(nb);
#pragma unroll
        for (int i = 0; i < 27; ++i) st(mu_at<27>(mu, g, nb, pl, i, 0, 0, 0), hydro_moment_adjoint<R>(am, i));
    }
    S *sT = static_cast<S *>(a.sT_dst);
#pragma unroll
    for (int k = 0; k < 3; ++k) st(elem(sT + k * N, nb.c), ad.gT[k]);
    st(elem(sT + 3 * N, nb.c), ad.T);
    for (int k = 0; k < 3; ++k) sp[k] = ad.gp[k];
    sp[3] = ad.lap;
    sp[4] = ad.phi;
}

// ---------------------------------------------------------------------------
// R1: phase field.  aphi3: K3's adjoint of phi^{n+1}; K2's adjoints of the
// phi^n stencil reads, stored at the cell by the first half of the reverse
// step, are completed here with K1's gradient adjoint.
// ---------------------------------------------------------------------------
template <int Q, typename P, typename S, typename R, bool WALL>
__device__ __forceinline__ void adj_pf_cell(const CoupledAdjointArgs &a, const Nbr &nb, R aphi3)
{
    constexpr bool dev = deviation_storage<P>();
    const Geometry &g = a.geo;
    const int64_t N = g.N;

    // recompute K1 of step n: phi^n stencil, moments of the pulled h (actual values)
    R G[3] = {R(0), R(0), R(0)}, phi1, j[3];
    {
        const S *po = static_cast<const S *>(a.s0.phi);
        R pn[27];
#pragma unroll
        for (int k = 0; k < 27; ++k) {
            pn[k] = ld<R>(nb.ptr(po, vel27(k, 0), vel27(k, 1), vel27(k, 2)));
            if (WALL && nb.ghost(vel27(k, 1))) pn[k] = nb.phi_ghost(pn[k], vel27(k, 1), a.wet);
        }
        const P *hs = static_cast<const P *>(a.s0.h);
        const PdfLanes<Q> pl(nb);
        R h[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int ex = vel<Q>(i, 0), ey = vel<Q>(i, 1), ez = vel<Q>(i, 2);
            const R w = R(weight<Q>(i));
            if (WALL && nb.ghost(-ey)) {
                h[i] = ld<R>(elem(pdf_row<Q>(hs, g, nb.yr[1], nb.zi[1], opposite<Q>(i)), pl.xq[1]));
                if (dev) h[i] += w * pn[0];
            } else {
                h[i] = ld<R>(elem(pdf_row<Q>(hs, g, nb.yr[1 - ey], nb.zi[1 - ez], i), pl.xq[1 - ex]));
                if (dev) h[i] += w * pn[opposite<27>(index27<Q>(i))];
            }
        }
        moments01<Q, R>(h, phi1, j);
#pragma unroll
        for (int k = 1; k < 27; ++k) {
            const R v = R(weight<27>(k)) * pn[k];
            G[0] += R(vel27(k, 0)) * v;
            G[1] += R(vel27(k, 1)) * v;
            G[2] += R(vel27(k, 2)) * v;
        }
        for (int k = 0; k < 3; ++k) G[k] *= R(3);
    }
    R u[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) u[k] = ld<R>(elem(static_cast<const S *>(a.s0.u[k]), nb.c));

    // dL/dphi^{n+1}: the transposed gradient and Laplacian of step n+1 (K1 and
    // K2 read the same stencil), the cell's own Pi, and K3's local adjoint
    const S *spn = static_cast<const S *>(a.sphi_src);
    R aphi = ld<R>(elem(spn + 4 * N, nb.c)) - R(6.0 * (1.0 - weight<27>(0))) * ld<R>(elem(spn + 3 * N, nb.c)) + aphi3;
    R ghost_sum[2] = {R(0), R(0)};
#pragma unroll
    for (int k = 1; k < 27; ++k) {
        const int ex = vel27(k, 0), ey = vel27(k, 1), ez = vel27(k, 2);
        const R w = R(weight<27>(k));
        if (!(WALL && nb.ghost(-ey))) {
            R v = R(6) * ld<R>(nb.ptr(spn + 3 * N, -ex, -ey, -ez));
            if (ex) v += R(3 * ex) * ld<R>(nb.ptr(spn, -ex, -ey, -ez));
            if (ey) v += R(3 * ey) * ld<R>(nb.ptr(spn + N, -ex, -ey, -ez));
            if (ez) v += R(3 * ez) * ld<R>(nb.ptr(spn + 2 * N, -ex, -ey, -ez));
            aphi += w * v;
        }
        if (WALL && nb.ghost(ey)) {
            R v = R(6) * ld<R>(nb.ptr(spn + 3 * N, -ex, 0, -ez));
            if (ex) v += R(3 * ex) * ld<R>(nb.ptr(spn, -ex, 0, -ez));
            v += R(3 * ey) * ld<R>(nb.ptr(spn + N, -ex, 0, -ez));
            if (ez) v += R(3 * ez) * ld<R>(nb.ptr(spn + 2 * N, -ex, 0, -ez));
            ghost_sum[ey > 0] += w * v;
        }
    }
    if (WALL) {
        // d ghost / d phi = 1 + wet (1 - 2 phi) for the contact-angle ghost of this cell
        const R p1 = ld<R>(elem(static_cast<const S *>(a.s1.phi), nb.c));
        aphi += ghost_sum[0] * (R(1) + R(a.wet[0]) * (R(1) - R(2) * p1)) +
                ghost_sum[1] * (R(1) + R(a.wet[1]) * (R(1) - R(2) * p1));
    }

    R lam[Q];
    gather_links<Q, S, R, WALL>(static_cast<const S *>(a.mu_src[0]), g, nb, R(1), lam);
    R aj[3], aG[3], au[3];
    pf_vjp<Q, R>(a.pf, phi1, j, G, u, lam, aphi, aj, aG, au);
    {
        S *mu = static_cast<S *>(a.mu_dst[0]);
        const PdfLanes<Q> pl(nb);
#pragma unroll
        for (int i = 0; i < Q; ++i) st(mu_at<Q>(mu, g, nb, pl, i, 0, 0, 0), moment01_adjoint<Q, R>(aphi, aj, i));
    }
    S *sd = static_cast<S *>(a.sphi_dst);
    S *lu1 = static_cast<S *>(a.lu1);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        // the hydrodynamic half has stored its part of the stencil adjoint
        st(elem(sd + k * N, nb.c), ld<R>(elem(sd + k * N, nb.c)) + aG[k]);
        st(elem(lu1 + k * N, nb.c), au[k]);
    }
}

// One reverse step undoes the three updates of a cell in reverse order in two
// launches: PART 1 K3 and K2, PART 2 K1.  Every value a thread reads from
// another cell comes from the previous reverse step's buffers.  The first
// half stores its part of the phi^n stencil adjoint where the step's own
// result goes, and K3's adjoint of phi^{n+1} in a scratch field; the second
// reads both back at the same cell.  Each half needs fewer registers than the
// whole update in one thread: in FP32 164 and 125 (three and four wavefronts
// per SIMD where the whole update, 188, runs two), in FP64 two wavefronts per
// SIMD with a few spills where the whole update runs one.
template <int QH, int QF, typename P, typename S, typename R, bool WALL, int PART>
__device__ __forceinline__ void adj_step_cell(const CoupledAdjointArgs &a, const Nbr &nb)
{
    if constexpr (PART == 1) {
        R au3[3], aphi3, sp[5];
        adj_thermal_cell<QF, P, S, R, WALL>(a, opaque(nb), au3, aphi3);
        __builtin_amdgcn_sched_barrier(0);
        adj_hydro_cell<S, R, WALL>(a, opaque(nb), au3, sp);
        const int64_t N = a.geo.N;
        S *sd = static_cast<S *>(a.sphi_dst);
#pragma unroll
        for (int k = 0; k < 5; ++k) st(elem(sd + k * N, nb.c), sp[k]);
        st(elem(static_cast<S *>(a.xphi), nb.c), aphi3);
    } else {
        const R aphi3 = ld<R>(elem(static_cast<const S *>(a.xphi), nb.c));
        adj_pf_cell<QH, P, S, R, WALL>(a, opaque(nb), aphi3);
    }
}

template <int QH, int QF, typename P, typename S, typename R, int PART>
__global__ void __launch_bounds__(kTX *kTY) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 8 ? 2 : 1)))
k_adj_step(const CoupledAdjointArgs a, const Tiling t)
{
    int x, y, z;
    if (!cell_of_thread(t, a.geo, x, y, z)) return;
    const Nbr nb(a.geo, x, y, z);
    if (nb.below || nb.above)
        adj_step_cell<QH, QF, P, S, R, true, PART>(a, nb);
    else
        adj_step_cell<QH, QF, P, S, R, false, PART>(a, nb);
}

// ---------------------------------------------------------------------------
// seed and the last wall-temperature pass
// ---------------------------------------------------------------------------
// sphi of the final step: Pi = dL/dphi^N for the loss through the centroid
// c = sum phi x / sum phi (sums in out4: M, sum phi x, sum phi y, sum phi z)
// plus an optional per-cell term; Gamma = Lambda = 0
template <typename S>
__global__ void __launch_bounds__(kTX *kTY) k_adj_seed_phi(const Geometry g, const Tiling t, const double *out4,
                                                           double gcx, double gcy, double gcz, const double *dphi,
                                                           S *sphi)
{
    int x, y, z;
    if (!cell_of_thread(t, g, x, y, z)) return;
    const uint32_t c = (uint32_t)x + (uint32_t)y * (uint32_t)g.nx + (uint32_t)z * (uint32_t)g.plane;
    const double M = out4[0];
    const double cx = out4[1] / M, cy = out4[2] / M, cz = out4[3] / M;
    double s = (gcx * (x - cx) + gcy * (y - cy) + gcz * (z - cz)) / M;
    if (dphi) s += dphi[c];
    const int64_t N = g.N;
    for (int k = 0; k < 4; ++k) st(elem(sphi + k * N, c), 0.0);
    st(elem(sphi + 4 * N, c), s);
}

// wall-temperature adjoint of the ghosts read by K2 of the first step (sT of step 0)
template <typename S, typename R>
__global__ void __launch_bounds__(kTX *kTY) k_adj_tw_ghosts(const Geometry g, const Tiling t, const S *sT,
                                                            double *grad_twb, double *grad_twt)
{
    int x, y, z;
    if (!cell_of_thread(t, g, x, y, z)) return;
    const Nbr nb(g, x, y, z);
    if (!nb.below && !nb.above) return;
    const int64_t N = g.N;
    R ghost_sum[2] = {R(0), R(0)};
#pragma unroll
    for (int k = 1; k < 27; ++k) {
        const int ex = vel27(k, 0), ey = vel27(k, 1), ez = vel27(k, 2);
        if (!nb.ghost(ey)) continue;
        R v = R(0);
        if (ex) v += R(ex) * ld<R>(nb.ptr(sT, -ex, 0, -ez));
        v += R(ey) * ld<R>(nb.ptr(sT + N, -ex, 0, -ez));
        if (ez) v += R(ez) * ld<R>(nb.ptr(sT + 2 * N, -ex, 0, -ez));
        ghost_sum[ey > 0] += R(3.0 * weight<27>(k)) * v;
    }
    const uint32_t col = nb.col(0, 0, g);
    if (nb.below) grad_twb[col] += 2.0 * (double)ghost_sum[0];
    if (nb.above) grad_twt[col] += 2.0 * (double)ghost_sum[1];
}

} // namespace

template <int QH, int QF, typename P, typename S, typename R>
void launch_coupled_adjoint_step(const CoupledAdjointArgs &a, hipStream_t s)
{
    const Tiling t = make_tiling(a.geo);
    hipLaunchKernelGGL((k_adj_step<QH, QF, P, S, R, 1>), tiling_grid(t), tiling_block(), 0, s, a, t);
    hipLaunchKernelGGL((k_adj_step<QH, QF, P, S, R, 2>), tiling_grid(t), tiling_block(), 0, s, a, t);
}

template <typename S>
void launch_coupled_adjoint_seed(const Geometry &g, const double *out4, const double gc[3], const double *dphi,
                                 void *sphi, hipStream_t s)
{
    const Tiling t = make_tiling(g);
    hipLaunchKernelGGL((k_adj_seed_phi<S>), tiling_grid(t), tiling_block(), 0, s, g, t, out4, gc[0], gc[1], gc[2],
                       dphi, static_cast<S *>(sphi));
}

template <typename S>
void launch_coupled_adjoint_tw(const Geometry &g, const void *sT, double *grad_twb, double *grad_twt, hipStream_t s)
{
    const Tiling t = make_tiling(g);
    hipLaunchKernelGGL((k_adj_tw_ghosts<S, S>), tiling_grid(t), tiling_block(), 0, s, g, t,
                       static_cast<const S *>(sT), grad_twb, grad_twt);
}

#define TCP_CADJ_INST(QH, QF)                                                                                \
    template void launch_coupled_adjoint_step<QH, QF, double, double, double>(const CoupledAdjointArgs &,    \
                                                                             hipStream_t);                   \
    template void launch_coupled_adjoint_step<QH, QF, float, float, float>(const CoupledAdjointArgs &,       \
                                                                          hipStream_t);                      \
    template void launch_coupled_adjoint_step<QH, QF, _Float16, float, float>(const CoupledAdjointArgs &,    \
                                                                             hipStream_t);
TCP_CADJ_INST(15, 7)
TCP_CADJ_INST(15, 15)
TCP_CADJ_INST(15, 19)
TCP_CADJ_INST(15, 27)
TCP_CADJ_INST(27, 7)
TCP_CADJ_INST(27, 15)
TCP_CADJ_INST(27, 19)
TCP_CADJ_INST(27, 27)
#undef TCP_CADJ_INST

template void launch_coupled_adjoint_seed<double>(const Geometry &, const double *, const double[3], const double *,
                                                  void *, hipStream_t);
template void launch_coupled_adjoint_seed<float>(const Geometry &, const double *, const double[3], const double *,
                                                 void *, hipStream_t);
template void launch_coupled_adjoint_tw<double>(const Geometry &, const void *, double *, double *, hipStream_t);
template void launch_coupled_adjoint_tw<float>(const Geometry &, const void *, double *, double *, hipStream_t);

} // namespace tcp
