// kernels_hydro.hip -- K2: velocity-based D3Q27 central-moment hydrodynamic
// LB step with the force of Sec. 2.2: F = F_s + F_b + F_p + F_mu, where
//   F_s  = mu_phi grad phi + 3/2 xi sigma_T (|grad phi|^2 grad T - (grad T . grad phi) grad phi)
//   F_b  = rho g,   F_p = -p* c_s^2 (rho_H - rho_L) grad phi,
//   F_mu = nu (rho_H - rho_L) [grad u + grad u^T] . grad phi,
// mu_phi = 4 beta phi (phi-1)(phi-1/2) - k lap phi, beta = 12 sigma/xi,
// k = 3 sigma xi / 2, sigma(T) = sigma_ref + sigma_T (T - T_ref), and the strain
// rate taken from the non-equilibrium second moment of the pulled PDFs.
// Gradients and the Laplacian use the isotropic D3Q27 stencil on phi^n (mirror
// ghost at walls) and on T^n (ghost 2 T_w - T).
//
// Collision: central moments about u, the five deviatoric second-order
// moments relax with omega(phi), the trace with omega_bulk, everything else
// with rate one, Guo source in velocity form.  Moments of rate one land on
// g_eq + S/2, so the kernel adds to g_eq + S/2 only the inverse transform of
// the six relaxed second-order central moments of g - g_eq + S/2; the D3Q27
// moment matrix is a tensor product of 1-D matrices, so that inverse is a
// product of 1-D columns (Axis1D).
#include "kernels.hpp"

namespace tcp {

template <typename S, typename R>
__global__ void __launch_bounds__(kBX *kBY) k_hydro(const HydroArgs a)
{
    const int x = blockIdx.x * kBX + threadIdx.x;
    const int y = blockIdx.y * kBY + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= a.geo.nx || y >= a.geo.ny) return;
    const Nbr nb(a.geo, x, y, z);
    const int64_t N = a.geo.N;
    const S *gs = static_cast<const S *>(a.g_src);

    // pull; halfway bounce-back, plus 2 w_i (e_i . u_w)/c_s^2 from a moving wall
    R g[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const int ex = vel27(i, 0), ey = vel27(i, 1), ez = vel27(i, 2);
        if (nb.ghost(-ey)) {
            const double *uw = ey > 0 ? a.uw_bot : a.uw_top;
            const R eu = R(ex) * R(uw[0]) + R(ey) * R(uw[1]) + R(ez) * R(uw[2]);
            g[i] = ld<R>(gs + opposite<27>(i) * N + nb.c) + R(6.0 * weight<27>(i)) * eu;
        } else {
            g[i] = ld<R>(gs + i * N + nb.at(-ex, -ey, -ez));
        }
    }
    // zeroth, first and second raw moments
    R ps = R(0), u0[3] = {R(0), R(0), R(0)};
    R mxx = R(0), myy = R(0), mzz = R(0), mxy = R(0), mxz = R(0), myz = R(0);
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const int ex = vel27(i, 0), ey = vel27(i, 1), ez = vel27(i, 2);
        ps += g[i];
        u0[0] += R(ex) * g[i];
        u0[1] += R(ey) * g[i];
        u0[2] += R(ez) * g[i];
        mxx += R(ex * ex) * g[i];
        myy += R(ey * ey) * g[i];
        mzz += R(ez * ez) * g[i];
        mxy += R(ex * ey) * g[i];
        mxz += R(ex * ez) * g[i];
        myz += R(ey * ez) * g[i];
    }

    // phi^n: value, gradient, Laplacian; T^n: value, gradient
    const S *pp = static_cast<const S *>(a.phi);
    const S *tp = static_cast<const S *>(a.T);
    const R phi = ld<R>(pp + nb.c);
    const R T = ld<R>(tp + nb.c);
    R gp[3] = {R(0), R(0), R(0)}, gT[3] = {R(0), R(0), R(0)}, lap = R(0);
#pragma unroll
    for (int i = 1; i < 27; ++i) {
        const int ex = vel27(i, 0), ey = vel27(i, 1), ez = vel27(i, 2);
        const R w = R(weight<27>(i));
        const int64_t at = nb.at(ex, ey, ez);
        const R pv = ld<R>(pp + at);
        R tv = ld<R>(tp + at);
        if (nb.ghost(ey)) {
            const double *tw = ey < 0 ? a.twb : a.twt;
            tv = R(2) * R(tw[nb.col(ex, ez, a.geo)]) - tv;
        }
        gp[0] += R(ex) * w * pv;
        gp[1] += R(ey) * w * pv;
        gp[2] += R(ez) * w * pv;
        lap += w * (pv - phi);
        gT[0] += R(ex) * w * tv;
        gT[1] += R(ey) * w * tv;
        gT[2] += R(ez) * w * tv;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        gp[k] *= R(3);
        gT[k] *= R(3);
    }
    lap *= R(6);

    // material laws
    const R phic = fmin(fmax(phi, R(0)), R(1));
    const R drho = R(a.drho);
    const R rho = R(a.rho_l) + phic * drho;
    const R tau = R(a.tau_l) + phic * R(a.dtau);
    const R omega = R(1) / (tau + R(0.5));
    const R nu = tau * R(1.0 / 3.0);
    const R sig = R(a.sigma_ref) + R(a.sigma_t) * (T - R(a.t_ref));
    const R xi = R(a.xi);
    const R beta = R(12) * sig / xi, kap = R(1.5) * sig * xi;
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
    R acc[3], u[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const R Fs = mu * gp[k] + mar * (gp2 * gT[k] - gTgp * gp[k]);
        const R F = Fs + rho * R(a.g[k]) + pfac * gp[k] + vfac * Sgp[k];
        acc[k] = F / rho;
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

    const Axis1D<R> X(u[0]), Y(u[1]), Z(u[2]);
    const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const R ua = u[0] * acc[0] + u[1] * acc[1] + u[2] * acc[2];
    S *gd = static_cast<S *>(a.g_dst);
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const int ex = vel27(i, 0), ey = vel27(i, 1), ez = vel27(i, 2);
        const int ia = ex + 1, ib = ey + 1, ic = ez + 1;
        const R w = R(weight<27>(i));
        const R eu = R(ex) * u[0] + R(ey) * u[1] + R(ez) * u[2];
        const R ea = R(ex) * acc[0] + R(ey) * acc[1] + R(ez) * acc[2];
        const R geq = w * (ps + R(3) * eu + R(4.5) * eu * eu - R(1.5) * uu);
        const R src = w * (R(3) * (ea - ua) + R(9) * eu * ea);
        const R dz0 = Z.m0[ic], dz1 = Z.m1[ic], dz2 = Z.m2[ic];
        const R corr = dz0 * (cxx * X.m2[ia] * Y.m0[ib] + cyy * X.m0[ia] * Y.m2[ib] + cxy * X.m1[ia] * Y.m1[ib]) +
                       dz1 * (cxz * X.m1[ia] * Y.m0[ib] + cyz * X.m0[ia] * Y.m1[ib]) +
                       dz2 * (czz * X.m0[ia] * Y.m0[ib]);
        st(gd + i * N + nb.c, geq + R(0.5) * src + corr);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) st(static_cast<S *>(a.u[k]) + nb.c, u[k]);
}

template <typename S, typename R>
void launch_hydro(const HydroArgs &a, hipStream_t s)
{
    dim3 block(kBX, kBY, 1);
    dim3 grid((a.geo.nx + kBX - 1) / kBX, (a.geo.ny + kBY - 1) / kBY, a.geo.nz);
    hipLaunchKernelGGL((k_hydro<S, R>), grid, block, 0, s, a);
}

template void launch_hydro<double, double>(const HydroArgs &, hipStream_t);
template void launch_hydro<float, float>(const HydroArgs &, hipStream_t);

} // namespace tcp
