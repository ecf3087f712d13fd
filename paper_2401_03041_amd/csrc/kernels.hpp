// kernels.hpp -- argument blocks and host-side launchers of the gfx950
// kernels (internal to the library; the public interface is tcplb.h).
#pragma once

#include "adjoint_math.hpp"
#include "lattice.hpp"

namespace tcp {

// K1: conservative Allen-Cahn LB (Eq. lb_interface, Eq. phasefieldforce)
struct PfArgs {
    Geometry geo;
    const void *h_src;
    void *h_dst;
    const void *phi_old; // phi^n (stencil for the interface normal)
    void *phi_new;       // phi^{n+1} = sum_i h_i (output)
    const void *u[3];    // u^n
    double omega_phi;    // 1 / (1/2 + M / c_s^2)
    double inv_xi;
    double eps2;         // normal_eps^2
    double wet[2];       // (4/xi) cos(contact angle) of the bottom and top wall
};

// K2: velocity-based D3Q27 central-moment hydrodynamics with forces (Sec. 2.1-2.2)
struct HydroArgs {
    Geometry geo;
    const void *g_src;
    void *g_dst;
    const void *phi;   // phi^n (stencil)
    const void *T;     // T^n (stencil)
    const double *twb; // wall temperatures, nx*nz (walls only)
    const double *twt;
    void *u[3];        // u^{n+1} (output)
    double rho_l, drho;  // rho(phi) = rho_l + phi_c drho
    double tau_l, dtau;  // tau(phi) = tau_l + phi_c dtau, tau = nu / c_s^2
    double sigma_ref, sigma_t, t_ref, xi;
    double twelve_inv_xi; // 12 / xi (beta = 12 sigma / xi)
    double g[3];
    double omega_bulk;
    double uw_bot[3], uw_top[3];
    double wet[2];       // (4/xi) cos(contact angle) of the bottom and top wall
};

// K3: passive-scalar thermal LB (Eq. lb_thermal)
struct ThermalArgs {
    Geometry geo;
    const void *f_src;
    void *f_dst;
    const void *phi;   // phi^{n+1} (local)
    const void *u[3];  // u^{n+1} (local)
    const void *T_old; // T^n (pull sources; FP32/FP16 deviation storage)
    void *T;           // T^{n+1} (output)
    const double *twb;
    const double *twt;
    double kappa_l, dkappa;
    double t_shift;    // f is stored as f_i - w_i t_shift
    HeatSources src;
};

// RK stage of the energy equation (Eq. rk2, Eq. rk4):
//   k = R(theta_in);  acc = (first ? 0 : acc) + w_acc k;
//   last ? T_new = T + acc : theta_out = T + a_next k
struct RkArgs {
    Geometry geo;
    const void *theta_in; // stage argument (stencil)
    void *theta_out;
    const void *T;        // T^n
    void *T_new;          // T^{n+1} (last stage)
    void *acc;
    const void *phi;      // phi^{n+1} (stencil, grad kappa)
    const void *u[3];     // u^{n+1}
    const double *twb;
    const double *twt;
    double kappa_l, dkappa;
    double a_next, w_acc;
    double wet[2];        // (4/xi) cos(contact angle) of the bottom and top wall
    int first, last;
    HeatSources src;
    void *coef;           // per-step coefficients a_x, a_y, a_z, kappa, q (five fields)
    int gk;               // kappa_H != kappa_L: a and kappa come from coef
    int hq;               // heat sources present: q comes from coef
};

// phi^n at a cell, its isotropic gradient and Laplacian (the D3Q27 stencils
// of the updates, contact-angle ghosts applied): the phase-field update
// computes them for its interface normal and hands them to the hydrodynamic
// update of the same cell in the fused step, which then loads no phi stencil
template <typename R>
struct PhiStencil {
    R phi, gp[3], lap;
};

// A field staged in LDS for a work-group's 64 x 4 tile with a one-cell halo in
// x and y, three planes (z - 1, z, z + 1; kHalo values each): the FP64 fused
// step stages phi^n and T^n so that their 27-point stencils come from LDS.
template <typename R>
struct Staged {
    const R *pl[3]; // planes z - 1, z, z + 1
    int o;          // the thread's cell within a plane: (ly + 1) kHX + lx + 1
    bool below, above;
    // the 3x3x3 neighbourhood in D3Q27 order, rows beyond a wall replaced by
    // the own row (as Nbr::stencil27 reads them)
    __device__ __forceinline__ void stencil27(R (&v)[27]) const
    {
#pragma unroll
        for (int k = 0; k < 27; ++k) {
            int dy = vel27(k, 1);
            if ((dy < 0 && below) || (dy > 0 && above)) dy = 0;
            v[k] = pl[vel27(k, 2) + 1][o + dy * kHX + vel27(k, 0)];
        }
    }
};

// pn: phi^n on the 27-point neighbourhood in D3Q27 order (ghosts applied)
template <typename R>
__device__ __forceinline__ void phi_stencil(const R (&pn)[27], PhiStencil<R> &s)
{
    R gp[3] = {R(0), R(0), R(0)}, lap = R(0);
#pragma unroll
    for (int k = 1; k < 27; ++k) {
        const int ex = vel27(k, 0), ey = vel27(k, 1), ez = vel27(k, 2);
        const R w = R(weight<27>(k));
        if (ex) gp[0] += R(ex) * w * pn[k];
        if (ey) gp[1] += R(ey) * w * pn[k];
        if (ez) gp[2] += R(ez) * w * pn[k];
        lap += w * pn[k];
    }
    for (int a = 0; a < 3; ++a) s.gp[a] = R(3) * gp[a];
    s.phi = pn[0];
    // sum over the 26 neighbours of w (psi_nb - psi) = sum w psi_nb - (1 - w_0) psi
    s.lap = R(6) * (lap - R(1.0 - weight<27>(0)) * pn[0]);
}

// Wave priority (s_setprio) while a cell update issues its PDF pull and its
// stencil loads of phi and T: a wave that is loading goes ahead of waves that
// are computing, which keeps more loads in flight (measured +2 to +2.5 % on
// the fused FP32 step at 512^3).
constexpr int kPullPriority = 2;

// Template parameters: P storage type of the phase-field / thermal PDFs, S
// storage type of the hydrodynamic PDFs and of every field, R arithmetic type.
//
// With FP32 or FP16 PDFs each phase-field and thermal PDF is stored as its
// deviation from the rest equilibrium of its own cell, h*_i - w_i phi(x) and
// f*_i - w_i T(x), where phi and T are the cell's new zeroth moments (stored
// as fields).  The pull rebuilds h_i - w_i phi^n(own) as the stored value plus
// w_i (phi^n(source) - phi^n(own)), and the zeroth moment as phi^n(own) plus
// the sum of those: in a uniform region at rest every term is exactly zero,
// so rounding leaves phi and T unchanged there instead of drifting by
// sum_i fl(w_i phi) - phi every step (measured: the FP32 mass drift against
// FP64 fell from 7e-9 to 2e-11 per step).  FP64 PDFs are stored as they are
// (thermal PDFs as f_i - w_i t_shift).
template <typename P>
constexpr bool deviation_storage() { return sizeof(P) <= 4; }

template <int Q, typename P, typename S, typename R>
void launch_pf(const PfArgs &a, hipStream_t s);
template <typename S, typename R>
void launch_hydro(const HydroArgs &a, hipStream_t s);
template <int Q, typename P, typename S, typename R>
void launch_thermal(const ThermalArgs &a, hipStream_t s);
template <typename S, typename R>
void launch_rk(const RkArgs &a, hipStream_t s);
// once per step before the stages: the coefficient fields the stages read
template <typename S, typename R>
void launch_rk_coef(const RkArgs &a, hipStream_t s);

// K1 + K2 + K3 (thermal LB) of one step fused into one kernel (kernels_step.hip)
struct StepArgs {
    PfArgs pf;
    HydroArgs hy;
    ThermalArgs th;
};
template <int QH, int QF, typename P, typename S, typename R>
void launch_step(const StepArgs &a, hipStream_t s);

// ---- set-up, read-back and diagnostics (kernels_aux.hip) -------------------
struct Droplets {
    int n;
    const double *xyzr; // device, n x 4
    double inv_xi;
    int periodic[3];
};
template <typename S>
void launch_droplets(const Geometry &g, const Droplets &d, void *phi, hipStream_t s);
template <typename S>
void launch_from_f64(const double *src, void *dst, int64_t n, hipStream_t s);

struct InitArgs {
    Geometry geo;
    int q_pf, q_th;
    const void *phi;
    const void *u[3];
    const void *T;
    void *h, *g, *f;
    void *phi_other;
    double t_shift;
};
template <typename S, typename P>
void launch_init(const InitArgs &a, hipStream_t s);

// which: 0 phi, 1..3 u, 4 T, 5 p, 6 p*, 7 rho
struct ReadArgs {
    Geometry geo;
    int which;
    const void *phi, *T, *g;
    const void *u[3];
    double rho_l, drho;
    double *out;
};
template <typename S>
void launch_read(const ReadArgs &a, hipStream_t s);
// PDFs of storage type P (blocked layout), stored as f_i - w_i (shift + field(x))
// (field of type F, may be null), to unshifted component-major FP64
template <typename P, typename F>
void launch_read_pdfs(const void *src, int q, const Geometry &g, double shift, const void *field, double *out,
                      hipStream_t s);

// FP64 sums of phi, phi x, phi y, phi z in fixed order: partial sums per
// work-group (wavefronts over whole x-rows, wave64 butterflies), then one
// work-group adds them up.
constexpr int kReduceBlocks = 1024;
template <typename S>
void launch_reduce(const Geometry &g, const void *phi, double *partial, double *out4, hipStream_t s);

// max |a_c - b_c| over n values (NaN if any difference is NaN), in FP64: partial
// maxima per work-group (kReduceBlocks of them), then one work-group
template <typename S>
void launch_maxdiff(int64_t n, const void *a, const void *b, double *partial, double *out, hipStream_t s);

// Adjoint of the thermal LB update with phi and u held (one launch per update,
// last to first).  mu_src holds dL/d(pulled PDFs) of the update being undone,
// mu_dst receives that of the update before it; grad_q (one value per cell)
// and grad_twb / grad_twt (one per wall column) accumulate in FP64.
struct ThermalAdjointArgs {
    Geometry geo;
    const void *mu_src;
    void *mu_dst;
    const void *u[3];
    const void *phi;
    double kappa_l, dkappa;
    double *grad_q;
    double *grad_twb, *grad_twt;
    int last; // the first forward update: no earlier output to propagate to
};

// Adjoint of the RK2 / RK4 update with phi and u held: coeff holds a (three
// fields) and kappa (one field) of the right-hand side; one stage launch per
// reverse stage, reading lambda' (lam) and A^T kappa of the stage after it
// (theta_in, null for the last stage), writing theta_out and acc.
struct RkAdjointArgs {
    Geometry geo;
    const void *phi;
    const void *u[3];
    void *coeff;
    const void *lam;
    const void *theta_in;
    void *theta_out;
    void *acc;
    double kappa_l, dkappa;
    double wet[2];
    double w_s, a_s; // kappa = w_s lambda' + a_s theta_in
    int first;       // acc starts from lambda'
    double *grad_q;
    double *grad_twb, *grad_twt;
};
template <typename S, typename R>
void launch_rk_adjoint_coeff(const RkAdjointArgs &a, hipStream_t s);
template <typename S, typename R>
void launch_rk_adjoint_stage(const RkAdjointArgs &a, hipStream_t s);

// mu of the last update: dL/dfp_j(x) = m(x) for the loss sum_x m(x) T(x)
template <int Q, typename S>
void launch_adjoint_seed(const Geometry &g, const double *m, void *mu, hipStream_t s);
template <int Q, typename S, typename R>
void launch_adjoint_step(const ThermalAdjointArgs &a, hipStream_t s);

// For every heat source, dL/dQ_k = sum_x g_k(x) grad_q(x) (g_k: the source's
// profile at unit amplitude) and dL/d(x_k, y_k, z_k), written as four values
// per source; partial sums per work-group in `partial` (4 kMaxSources
// kSourceGradBlocks values), then one work-group
constexpr int kSourceGradBlocks = 64;
static_assert(4 * kMaxSources * kSourceGradBlocks <= 4 * kReduceBlocks, "shares the reduction's partial buffer");
void launch_source_grad(const Geometry &g, const HeatSources &hs, const double *grad_q, double *partial,
                        double *out, hipStream_t s);

// ---- adjoint of the coupled step (kernels_coupled_adjoint.hip) -------------
// One stored state of the coupled step (time level n): the three PDF fields
// (storage layout of the domain), phi^n, T^n and u^n.
struct StateSlot {
    void *h, *g, *f, *phi, *T;
    void *u[3];
};

// Reverse of step n -> n+1.  s0 holds state n, s1 state n+1.  The carried
// adjoint (type S): link adjoints mu of h, g, f (blocked like the PDFs; src
// from step n+1, dst for step n), sphi (five fields: dL/d grad phi (3),
// dL/d lap phi, dL/d phi at the cell) and sT (four fields: dL/d grad T (3),
// dL/d T at the cell) of the stencil reads of K1/K2, lu1 = dL/du from K1 (in
// place).  grad_q (per cell) and the wall-column adjoints accumulate in FP64.
struct CoupledAdjointArgs {
    Geometry geo;
    StateSlot s0, s1;
    const void *mu_src[3];
    void *mu_dst[3];
    const void *sphi_src;
    void *sphi_dst;
    const void *sT_src;
    void *sT_dst;
    void *lu1;
    void *xphi; // one field: K3's phi^{n+1} adjoint between the two halves of a split reverse step
    const double *twb, *twt;
    double uw_bot[3], uw_top[3];
    double wet[2];
    double t_shift;
    PfCoef pf;
    HyCoef hy;
    ThCoef th;
    double *grad_q, *grad_twb, *grad_twt;
};
template <int QH, int QF, typename P, typename S, typename R>
void launch_coupled_adjoint_step(const CoupledAdjointArgs &a, hipStream_t s);
// sphi of the last step from the centroid gradient dL/dc (gc) and an optional
// per-cell dL/dphi (dphi, FP64 device array or null); out4 holds the FP64
// sums of launch_reduce for the final phi
template <typename S>
void launch_coupled_adjoint_seed(const Geometry &g, const double *out4, const double gc[3], const double *dphi,
                                 void *sphi, hipStream_t s);
// wall-temperature adjoint of the T ghosts read in the first step (sT of step 0)
template <typename S>
void launch_coupled_adjoint_tw(const Geometry &g, const void *sT, double *grad_twb, double *grad_twt, hipStream_t s);

// streaming copy of n16 16-byte words (bandwidth probe)
void launch_copy16(const void *src, void *dst, int64_t n16, hipStream_t s);
// copy of a 27-component FP32 field in the blocked PDF layout, ncells a
// multiple of 64 (bandwidth probe of the step kernel's access pattern)
void launch_copy_blocked27(const void *src, void *dst, int64_t ncells, hipStream_t s);

} // namespace tcp
