// tcplb_api.hip -- host implementation of the C interface in include/tcplb.h:
// parameter validation, buffer ownership, the per-step schedule of
// Algorithm 1 (phase field -> hydrodynamics -> thermal LB) and Algorithm 2
// (... -> RK stages), read-back, diagnostics and per-kernel event timing.
#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/tcplb.h"
#include "kernels.hpp"
#include "kernels_io.hpp"

using namespace tcp;

struct TimingRecord {
    int kind;
    hipEvent_t start, stop;
};

struct tcp_domain {
    tcp_params P{};
    Geometry geo{};
    tcp_allocator A{};
    bool own_alloc = true;
    hipStream_t stream = nullptr;
    int device = 0; // the device current at creation
    size_t sb = 8; // bytes per stored field value and hydrodynamic PDF
    size_t pb = 8; // bytes per stored phase-field or thermal PDF

    void *h[2]{}, *g[2]{}, *f[2]{}, *phi[2]{}, *u[3]{}, *T[2]{}; // [cur]: time level n
    void *rk[3]{}; // theta_a, theta_b, acc
    void *rkc = nullptr; // RK right-hand side coefficients: a_x, a_y, a_z, kappa, q
    bool rkq_ready = false; // q in rkc holds the current heat sources
    double *twb = nullptr, *twt = nullptr;
    double *partial = nullptr, *out4 = nullptr;
    HeatSources src{};
    int cur = 0;
    bool initialized = false;

    double omega_phi = 1.0, tau_h = 0.5, tau_l = 0.5;
    std::string err;

    // step graphs: kGraphSteps steps captured once per parity of `cur` and
    // replayed with one launch (graph_mode: 0 never, 1 small domains, 2 always)
    int graph_mode = 1;
    bool fuse = true; // thermal LB: one fused kernel per step (tcp_set_fusion)
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec[2]{};

    // thermal adjoint workspace, allocated on first use: link adjoints (two
    // parities), loss weights, the per-cell source adjoint, the wall-column
    // adjoints (bottom then top) and the per-source gradients
    void *adj_mu[2]{};
    double *adj_m = nullptr, *adj_g = nullptr, *adj_tw = nullptr, *adj_q = nullptr;
    // RK schemes instead of adj_mu: lambda', acc, two stage fields, and the
    // right-hand side's coefficients (a_x, a_y, a_z, kappa), N values each
    void *adj_rk = nullptr;

    // tape of a coupled run for its adjoint (tcp_step_taped / tcp_tape_adjoint):
    // the states at the start of every segment of `seg` steps and the final
    // state (nseg + 1 checkpoints), one or two rings of seg - 1 states for the
    // inner states of a segment (ring_seg: the segment a ring holds, -1 none;
    // with two, the reverse sweep of one segment overlaps the recomputation of
    // the next on a second stream), the heat sources and wall temperatures in
    // force, and the reverse sweep's workspace
    struct Tape {
        bool valid = false;
        int64_t nsteps = 0, seg = 0, nseg = 0, ring_seg[2] = {-1, -1};
        int nrings = 1;
        void *mem = nullptr;
        size_t mem_bytes = 0;
        std::vector<StateSlot> ckpt, ring[2];
        hipStream_t side = nullptr;                  // recomputation stream (default priority)
        hipEvent_t ready[2] = {}, freed[2] = {}, start = nullptr;
        HeatSources src{};
        double *twb = nullptr, *twt = nullptr;
        void *mu[3][2]{}, *sphi[2]{}, *sT[2]{}, *lu1 = nullptr;
        double *grad_q = nullptr, *grad_tw = nullptr, *gsrc = nullptr, *dphi = nullptr;
    } tape;

    bool prof = false;
    std::vector<TimingRecord> records;
    std::vector<hipEvent_t> pool;
    std::vector<void *> owned;
};

namespace {

thread_local std::string g_create_error;

int fail(tcp_domain *d, int code, const std::string &msg)
{
    if (d) d->err = msg;
    else g_create_error = msg;
    return code;
}

int hip_fail(tcp_domain *d, const char *what, hipError_t e)
{
    return fail(d, TCP_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define TCP_HIP(d, call)                                                                                     \
    do {                                                                                                      \
        hipError_t e_ = (call);                                                                               \
        if (e_ != hipSuccess) return hip_fail((d), #call, e_);                                                \
    } while (0)

void *dev_alloc(tcp_domain *d, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (d->own_alloc) {
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError(); // do not leave the failure for a later launch check to find
            return nullptr;
        }
    } else {
        p = d->A.alloc(bytes, d->A.ctx);
    }
    return p;
}

void dev_free(tcp_domain *d, void *p)
{
    if (!p) return;
    if (d->own_alloc) (void)hipFree(p);
    else d->A.free(p, d->A.ctx);
}

// allocation owned by the domain until tcp_destroy
void *own(tcp_domain *d, size_t bytes)
{
    void *p = dev_alloc(d, bytes);
    if (p) d->owned.push_back(p);
    return p;
}

// Scratch device buffer released (after a stream synchronisation) when it goes out of scope.
struct Scratch {
    tcp_domain *d;
    void *p;
    Scratch(tcp_domain *dd, size_t bytes) : d(dd), p(dev_alloc(dd, bytes)) {}
    ~Scratch()
    {
        if (p) {
            (void)hipStreamSynchronize(d->stream);
            dev_free(d, p);
        }
    }
};

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// (4/xi) cos(theta) for a contact angle theta in degrees (exactly 0 at 90)
double wetting(double degrees, double xi)
{
    return degrees == 90.0 ? 0.0 : 4.0 / xi * std::cos(degrees * (3.14159265358979323846 / 180.0));
}

constexpr size_t kArenaAlign = (size_t)2 << 20;
constexpr size_t kArenaStagger = 0;

// ---- timing ---------------------------------------------------------------
struct KernelTimer {
    tcp_domain *d;
    int kind;
    hipEvent_t a = nullptr, b = nullptr;
    hipEvent_t take()
    {
        hipEvent_t e = nullptr;
        if (!d->pool.empty()) {
            e = d->pool.back();
            d->pool.pop_back();
        } else if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
        }
        return e;
    }
    KernelTimer(tcp_domain *dd, int k) : d(dd), kind(k)
    {
        if (!d->prof) return;
        a = take();
        b = take();
        if (a) (void)hipEventRecord(a, d->stream);
    }
    ~KernelTimer()
    {
        if (!d->prof || !a || !b) return;
        (void)hipEventRecord(b, d->stream);
        d->records.push_back({kind, a, b});
    }
};

// ---- per-step schedule ------------------------------------------------------
PfArgs pf_args(const tcp_domain *d)
{
    PfArgs a{};
    a.geo = d->geo;
    a.h_src = d->h[d->cur];
    a.h_dst = d->h[1 - d->cur];
    a.phi_old = d->phi[d->cur];
    a.phi_new = d->phi[1 - d->cur];
    for (int k = 0; k < 3; ++k) a.u[k] = d->u[k];
    a.omega_phi = d->omega_phi;
    a.inv_xi = 1.0 / d->P.xi;
    a.eps2 = d->P.normal_eps * d->P.normal_eps;
    a.wet[0] = wetting(d->P.contact_angle_bot, d->P.xi);
    a.wet[1] = wetting(d->P.contact_angle_top, d->P.xi);
    return a;
}

template <typename S, typename Pdf>
void phase_step(tcp_domain *d)
{
    const PfArgs a = pf_args(d);
    KernelTimer t(d, TCP_K_PHASE);
    if (d->P.q_pf == 15) launch_pf<15, Pdf, S, S>(a, d->stream);
    else launch_pf<27, Pdf, S, S>(a, d->stream);
}

HydroArgs hydro_args(const tcp_domain *d)
{
    const tcp_params &P = d->P;
    HydroArgs a{};
    a.geo = d->geo;
    a.g_src = d->g[d->cur];
    a.g_dst = d->g[1 - d->cur];
    a.phi = d->phi[d->cur];
    a.T = d->T[d->cur];
    a.twb = d->twb;
    a.twt = d->twt;
    for (int k = 0; k < 3; ++k) a.u[k] = d->u[k];
    a.rho_l = P.rho_l;
    a.drho = P.rho_h - P.rho_l;
    a.tau_l = d->tau_l;
    a.dtau = d->tau_h - d->tau_l;
    a.sigma_ref = P.sigma_ref;
    a.sigma_t = P.sigma_t;
    a.t_ref = P.t_ref;
    a.xi = P.xi;
    a.twelve_inv_xi = 12.0 / P.xi;
    for (int k = 0; k < 3; ++k) {
        a.g[k] = P.g[k];
        a.uw_bot[k] = P.u_wall_bot[k];
        a.uw_top[k] = P.u_wall_top[k];
    }
    a.omega_bulk = P.omega_bulk;
    a.wet[0] = wetting(P.contact_angle_bot, P.xi);
    a.wet[1] = wetting(P.contact_angle_top, P.xi);
    return a;
}

template <typename S>
void hydro_step(tcp_domain *d)
{
    const HydroArgs a = hydro_args(d);
    KernelTimer t(d, TCP_K_HYDRO);
    launch_hydro<S, S>(a, d->stream);
}

ThermalArgs thermal_args(const tcp_domain *d)
{
    const tcp_params &P = d->P;
    ThermalArgs a{};
    a.geo = d->geo;
    a.f_src = d->f[d->cur];
    a.f_dst = d->f[1 - d->cur];
    a.phi = d->phi[1 - d->cur];
    for (int k = 0; k < 3; ++k) a.u[k] = d->u[k];
    a.T_old = d->T[d->cur];
    a.T = d->T[1 - d->cur];
    a.twb = d->twb;
    a.twt = d->twt;
    a.kappa_l = P.kappa_l;
    a.dkappa = P.kappa_h - P.kappa_l;
    a.t_shift = P.t_shift;
    a.src = d->src;
    return a;
}

template <typename S, typename Pdf>
void thermal_step(tcp_domain *d)
{
    const tcp_params &P = d->P;
    if (P.thermal == TCP_THERMAL_LB) {
        const ThermalArgs a = thermal_args(d);
        KernelTimer t(d, TCP_K_THERMAL);
        switch (P.q_thermal) {
        case 7: launch_thermal<7, Pdf, S, S>(a, d->stream); break;
        case 15: launch_thermal<15, Pdf, S, S>(a, d->stream); break;
        case 19: launch_thermal<19, Pdf, S, S>(a, d->stream); break;
        default: launch_thermal<27, Pdf, S, S>(a, d->stream); break;
        }
        return;
    }
    RkArgs a{};
    a.geo = d->geo;
    a.wet[0] = wetting(P.contact_angle_bot, P.xi);
    a.wet[1] = wetting(P.contact_angle_top, P.xi);
    a.T = d->T[d->cur];
    a.T_new = d->T[1 - d->cur];
    a.phi = d->phi[1 - d->cur];
    for (int k = 0; k < 3; ++k) a.u[k] = d->u[k];
    a.twb = d->twb;
    a.twt = d->twt;
    a.kappa_l = P.kappa_l;
    a.dkappa = P.kappa_h - P.kappa_l;
    a.src = d->src;
    a.coef = d->rkc;
    a.gk = P.kappa_h != P.kappa_l;
    a.hq = d->src.n > 0;
    // a and kappa change every step with a conductivity ratio; q depends on
    // the sources alone, so without one the pass runs once after each change
    // of the sources (in a captured graph: in its first step)
    const bool coef = a.gk || (a.hq && !d->rkq_ready);
    if (coef) d->rkq_ready = true;
    if (P.thermal == TCP_THERMAL_RK2) {
        // theta = T + k1/2; T_new = T + R(theta)
        a.theta_in = d->T[d->cur];
        a.theta_out = d->rk[0];
        a.acc = nullptr;
        a.first = 1;
        a.last = 0;
        a.a_next = 0.5;
        a.w_acc = 0.0;
        {
            // the per-step coefficient pass is timed with the first stage
            KernelTimer t(d, TCP_K_RK);
            if (coef) launch_rk_coef<S, S>(a, d->stream);
            launch_rk<S, S>(a, d->stream);
        }
        a.theta_in = d->rk[0];
        a.first = 1;
        a.last = 1;
        a.w_acc = 1.0;
        KernelTimer t(d, TCP_K_RK);
        launch_rk<S, S>(a, d->stream);
        return;
    }
    // RK4: K1..K4, stage arguments T + K1/2, T + K2/2, T + K3
    const void *in[4] = {d->T[d->cur], d->rk[0], d->rk[1], d->rk[0]};
    void *out[4] = {d->rk[0], d->rk[1], d->rk[0], nullptr};
    const double wacc[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    const double anext[4] = {0.5, 0.5, 1.0, 0.0};
    a.acc = d->rk[2];
    for (int s = 0; s < 4; ++s) {
        a.theta_in = in[s];
        a.theta_out = out[s];
        a.first = s == 0;
        a.last = s == 3;
        a.w_acc = wacc[s];
        a.a_next = anext[s];
        KernelTimer t(d, TCP_K_RK);
        if (s == 0 && coef) launch_rk_coef<S, S>(a, d->stream);
        launch_rk<S, S>(a, d->stream);
    }
}

// K1 + K2 + K3 (thermal LB) in one kernel
template <int QH, typename S, typename Pdf>
void fused_step_q(tcp_domain *d, const StepArgs &a)
{
    switch (d->P.q_thermal) {
    case 7: launch_step<QH, 7, Pdf, S, S>(a, d->stream); break;
    case 15: launch_step<QH, 15, Pdf, S, S>(a, d->stream); break;
    case 19: launch_step<QH, 19, Pdf, S, S>(a, d->stream); break;
    default: launch_step<QH, 27, Pdf, S, S>(a, d->stream); break;
    }
}

template <typename S, typename Pdf>
void fused_step(tcp_domain *d)
{
    const StepArgs a{pf_args(d), hydro_args(d), thermal_args(d)};
    KernelTimer t(d, TCP_K_STEP);
    if (d->P.q_pf == 15) fused_step_q<15, S, Pdf>(d, a);
    else fused_step_q<27, S, Pdf>(d, a);
}

// K1 + K2 in one kernel (RK schemes: the stages follow)
template <typename S, typename Pdf>
void fused_pf_hydro(tcp_domain *d)
{
    const StepArgs a{pf_args(d), hydro_args(d), ThermalArgs{}};
    KernelTimer t(d, TCP_K_STEP);
    if (d->P.q_pf == 15) launch_step<15, 0, Pdf, S, S>(a, d->stream);
    else launch_step<27, 0, Pdf, S, S>(a, d->stream);
}

// S: hydrodynamic PDFs and fields (also the arithmetic type); Pdf: phase-field
// and thermal PDFs
template <typename S, typename Pdf>
void one_step(tcp_domain *d)
{
    if (d->fuse && d->P.thermal == TCP_THERMAL_LB) {
        fused_step<S, Pdf>(d);
    } else if (d->fuse) {
        fused_pf_hydro<S, Pdf>(d);
        thermal_step<S, Pdf>(d);
    } else {
        phase_step<S, Pdf>(d);
        hydro_step<S>(d);
        thermal_step<S, Pdf>(d);
    }
    d->cur = 1 - d->cur;
}

// thermal update alone (phase field and velocity held): the buffers of both
// parities hold the same phi, so K3 sees it as phi^{n+1}
template <typename S, typename Pdf>
void thermal_only_step(tcp_domain *d)
{
    thermal_step<S, Pdf>(d);
    d->cur = 1 - d->cur;
}

void run_thermal_steps(tcp_domain *d, int64_t nsteps)
{
    for (int64_t n = 0; n < nsteps; ++n) {
        switch (d->P.precision) {
        case TCP_FP64: thermal_only_step<double, double>(d); break;
        case TCP_FP32: thermal_only_step<float, float>(d); break;
        default: thermal_only_step<float, _Float16>(d); break;
        }
    }
}

void run_steps(tcp_domain *d, int64_t nsteps)
{
    for (int64_t n = 0; n < nsteps; ++n) {
        switch (d->P.precision) {
        case TCP_FP64: one_step<double, double>(d); break;
        case TCP_FP32: one_step<float, float>(d); break;
        default: one_step<float, _Float16>(d); break;
        }
    }
}

// ---- step graphs ------------------------------------------------------------
// A step is 3-6 kernel launches; on small grids each kernel runs for a few
// microseconds and the host-side launch cost dominates.  kGraphSteps steps are
// then captured into one HIP graph and replayed with a single launch.  The
// count is even, so a replay leaves the buffer parity `cur` where it found
// it; one graph is kept per parity.  Kernel arguments are captured by value:
// the graphs are dropped when the heat sources change.
constexpr int kGraphSteps = 16;
constexpr int64_t kGraphMaxCells = (int64_t)1 << 21;
static_assert(kGraphSteps % 2 == 0, "a replay must leave the buffer parity unchanged");

void drop_graphs(tcp_domain *d)
{
    for (auto &g : d->gexec) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
}

bool use_graphs(const tcp_domain *d, int64_t nsteps)
{
    if (d->prof || nsteps < kGraphSteps || d->graph_mode == 0) return false;
    return d->graph_mode == 2 || d->geo.N <= kGraphMaxCells;
}

int build_graph(tcp_domain *d)
{
    if (!d->cap_stream) TCP_HIP(d, hipStreamCreateWithFlags(&d->cap_stream, hipStreamNonBlocking));
    // capture on a stream of our own (the caller's may be the legacy default
    // stream, which cannot be captured); the replay goes to the caller's stream
    TCP_HIP(d, hipStreamBeginCapture(d->cap_stream, hipStreamCaptureModeThreadLocal));
    const hipStream_t user = d->stream;
    const int cur = d->cur;
    // what the recorded steps take as done only happens when the graph runs
    const bool rkq_ready = d->rkq_ready;
    d->stream = d->cap_stream;
    run_steps(d, kGraphSteps); // an even number of buffer swaps: cur is unchanged
    d->stream = user;
    hipGraph_t graph = nullptr;
    const hipError_t e_launch = hipGetLastError();
    const hipError_t e_end = hipStreamEndCapture(d->cap_stream, &graph);
    if (e_launch != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        d->rkq_ready = rkq_ready;
        return hip_fail(d, "kernel launch during graph capture", e_launch);
    }
    if (e_end != hipSuccess) {
        d->rkq_ready = rkq_ready;
        return hip_fail(d, "hipStreamEndCapture", e_end);
    }
    const hipError_t e_inst = hipGraphInstantiate(&d->gexec[cur], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e_inst != hipSuccess) {
        d->gexec[cur] = nullptr;
        d->rkq_ready = rkq_ready;
        return hip_fail(d, "hipGraphInstantiate", e_inst);
    }
    return TCP_OK;
}

int validate(const tcp_params *p, std::string &why)
{
    char buf[256];
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) { why = "grid dimensions must be >= 1"; return TCP_ERR_ARG; }
    {
        // kernels address each field array with 32-bit byte offsets (PDF rows are
        // addressed from wave-uniform 64-bit row pointers)
        const int64_t ncell = (int64_t)p->nx * p->ny * p->nz;
        const int64_t bytes = ncell * (p->precision == TCP_FP64 ? 8 : 4);
        if (bytes >= ((int64_t)1 << 32)) {
            why = "grid too large: one field array would exceed 4 GiB";
            return TCP_ERR_UNSUPPORTED;
        }
    }
    if (p->walls_y != 0 && p->walls_y != 1) { why = "walls_y must be 0 or 1"; return TCP_ERR_ARG; }
    if (p->walls_y && p->ny < 2) { why = "walls need ny >= 2"; return TCP_ERR_ARG; }
    if (p->q_pf != 15 && p->q_pf != 27) { why = "q_pf must be 15 or 27"; return TCP_ERR_ARG; }
    if (p->q_thermal != 7 && p->q_thermal != 15 && p->q_thermal != 19 && p->q_thermal != 27) {
        why = "q_thermal must be 7, 15, 19 or 27"; return TCP_ERR_ARG;
    }
    if (p->thermal < 0 || p->thermal > 2) { why = "thermal must be LB, RK2 or RK4"; return TCP_ERR_ARG; }
    if (p->precision != TCP_FP64 && p->precision != TCP_FP32 && p->precision != TCP_FP16) {
        why = "precision must be TCP_FP64, TCP_FP32 or TCP_FP16"; return TCP_ERR_ARG;
    }
    const double vals[] = {p->rho_h, p->rho_l, p->nu_h, p->nu_l, p->mobility, p->xi, p->kappa_h, p->kappa_l, p->omega_bulk};
    const char *names[] = {"rho_h", "rho_l", "nu_h", "nu_l", "mobility", "xi", "kappa_h", "kappa_l", "omega_bulk"};
    for (int k = 0; k < 9; ++k)
        if (!finite_pos(vals[k])) {
            std::snprintf(buf, sizeof buf, "%s must be finite and > 0", names[k]);
            why = buf;
            return TCP_ERR_ARG;
        }
    const double others[] = {p->sigma_ref, p->sigma_t, p->t_ref, p->g[0], p->g[1], p->g[2], p->normal_eps,
                             p->u_wall_bot[0], p->u_wall_bot[1], p->u_wall_bot[2], p->u_wall_top[0],
                             p->u_wall_top[1], p->u_wall_top[2], p->t_wall_bot, p->t_wall_top, p->t_shift};
    for (double v : others)
        if (!std::isfinite(v)) { why = "parameters must be finite"; return TCP_ERR_ARG; }
    if (p->omega_bulk >= 2.0) { why = "omega_bulk must lie in (0, 2)"; return TCP_ERR_ARG; }
    for (double a : {p->contact_angle_bot, p->contact_angle_top})
        if (!(a > 0.0 && a < 180.0)) { why = "contact angles must lie in (0, 180) degrees"; return TCP_ERR_ARG; }
    for (const double *uw : {p->u_wall_bot, p->u_wall_top})
        if (std::sqrt(uw[0] * uw[0] + uw[1] * uw[1] + uw[2] * uw[2]) >= 0.1) {
            why = "wall speed must stay below 0.1"; return TCP_ERR_ARG;
        }
    if (p->thermal != TCP_THERMAL_LB) {
        // real-axis stability of RK2 / RK4 against the most negative symbol of the
        // isotropic Laplacian, -6 * 208/216 at k = (pi, pi, pi)
        const double lmin = 6.0 * 208.0 / 216.0;
        const double bound = (p->thermal == TCP_THERMAL_RK2 ? 2.0 : 2.785) / lmin;
        const double kmax = p->kappa_h > p->kappa_l ? p->kappa_h : p->kappa_l;
        if (kmax > bound) {
            std::snprintf(buf, sizeof buf, "kappa %.4g exceeds the RK stability bound %.4g", kmax, bound);
            why = buf;
            return TCP_ERR_ARG;
        }
    }
    return TCP_OK;
}

template <typename F>
int guarded(tcp_domain *d, F &&fn)
{
    try {
        return fn();
    } catch (const std::bad_alloc &) {
        return fail(d, TCP_ERR_OOM, "host allocation failed");
    } catch (...) {
        return fail(d, TCP_ERR_HIP, "unexpected exception");
    }
}

int check_launch(tcp_domain *d)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(d, "kernel launch", e);
    return TCP_OK;
}

} // namespace

namespace {
struct Piece {
    void *p;
    size_t bytes;
};
std::vector<Piece> state_pieces(const tcp_domain *d)
{
    const size_t N = (size_t)d->geo.N, sb = d->sb, pb = d->pb;
    std::vector<Piece> v;
    v.push_back({d->h[d->cur], (size_t)pdf_elems(d->geo, d->P.q_pf) * pb});
    v.push_back({d->g[d->cur], (size_t)pdf_elems(d->geo, 27) * sb});
    if (d->P.thermal == TCP_THERMAL_LB) v.push_back({d->f[d->cur], (size_t)pdf_elems(d->geo, d->P.q_thermal) * pb});
    v.push_back({d->phi[d->cur], N * sb});
    for (int k = 0; k < 3; ++k) v.push_back({d->u[k], N * sb});
    v.push_back({d->T[d->cur], N * sb});
    return v;
}
} // namespace

namespace {

template <int Q, typename S>
void run_thermal_adjoint(tcp_domain *d, int64_t nsteps)
{
    launch_adjoint_seed<Q, S>(d->geo, d->adj_m, d->adj_mu[0], d->stream);
    ThermalAdjointArgs a{};
    a.geo = d->geo;
    for (int k = 0; k < 3; ++k) a.u[k] = d->u[k];
    a.phi = d->phi[d->cur];
    a.kappa_l = d->P.kappa_l;
    a.dkappa = d->P.kappa_h - d->P.kappa_l;
    a.grad_q = d->adj_g;
    a.grad_twb = d->adj_tw;
    a.grad_twt = d->adj_tw + (size_t)d->P.nx * d->P.nz;
    int b = 0;
    for (int64_t n = nsteps; n >= 1; --n) {
        a.mu_src = d->adj_mu[b];
        a.mu_dst = d->adj_mu[1 - b];
        a.last = n == 1;
        KernelTimer t(d, TCP_K_ADJOINT);
        launch_adjoint_step<Q, S, S>(a, d->stream);
        b = 1 - b;
    }
}

template <typename S>
void run_rk_adjoint(tcp_domain *d, int64_t nsteps)
{
    const size_t N = (size_t)d->geo.N;
    S *base = static_cast<S *>(d->adj_rk);
    S *lam = base, *acc = base + N, *th[2] = {base + 2 * N, base + 3 * N};
    // base + 4N .. 8N: coefficients
    RkAdjointArgs a{};
    a.geo = d->geo;
    a.phi = d->phi[d->cur];
    for (int k = 0; k < 3; ++k) a.u[k] = d->u[k];
    a.coeff = base + 4 * N;
    a.kappa_l = d->P.kappa_l;
    a.dkappa = d->P.kappa_h - d->P.kappa_l;
    a.wet[0] = wetting(d->P.contact_angle_bot, d->P.xi);
    a.wet[1] = wetting(d->P.contact_angle_top, d->P.xi);
    a.grad_q = d->adj_g;
    a.grad_twb = d->adj_tw;
    a.grad_twt = d->adj_tw + (size_t)d->P.nx * d->P.nz;
    launch_rk_adjoint_coeff<S, S>(a, d->stream);
    launch_from_f64<S>(d->adj_m, lam, (int64_t)N, d->stream);
    // forward: T' = T + sum_s w_s K_s, K_s = R(theta_s), theta_{s+1} = T + a_s K_s
    const bool rk4 = d->P.thermal == TCP_THERMAL_RK4;
    const int ns = rk4 ? 4 : 2;
    const double w4[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0}, a4[3] = {0.5, 0.5, 1.0};
    const double w2[2] = {0.0, 1.0}, a2[1] = {0.5};
    const double *w = rk4 ? w4 : w2, *an = rk4 ? a4 : a2;
    for (int64_t n = 0; n < nsteps; ++n) {
        a.lam = lam;
        a.acc = acc;
        int b = 0;
        for (int st = ns - 1; st >= 0; --st) {
            a.w_s = w[st];
            a.a_s = st + 1 < ns ? an[st] : 0.0;
            a.theta_in = st + 1 < ns ? th[1 - b] : nullptr;
            a.theta_out = th[b];
            a.first = st == ns - 1;
            KernelTimer t(d, TCP_K_ADJOINT);
            launch_rk_adjoint_stage<S, S>(a, d->stream);
            b = 1 - b;
        }
        std::swap(lam, acc); // lambda of the update before
    }
}

} // namespace

// ---- read-back without allocation ---------------------------------------------
// Staging array of tcp_get_field_noalloc: FP64 values of one field, one array
// per GPU (each device holds its own copy), held until the process ends.
constexpr size_t kNoAllocCells = (size_t)1 << 22; // 4 Mi values, 32 MiB
static __device__ __align__(256) double scratch[kNoAllocCells];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev, which must be current: looked up
// once per device with hipGetSymbolAddress (the array's name is only a host
// stand-in and must never be passed to a kernel or a copy).
int scratch_address(tcp_domain *d, int dev, void **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        TCP_HIP(d, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(d, TCP_ERR_HIP, "hipGetSymbolAddress returned no address for the staging array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return TCP_OK;
}

// read-kernel arguments for field `which` of the current state
ReadArgs read_args(const tcp_domain *d, int which)
{
    ReadArgs a{};
    a.geo = d->geo;
    a.which = which; // TCP_PHI..TCP_RHO use the read-kernel codes 0..7
    a.phi = d->phi[d->cur];
    a.T = d->T[d->cur];
    a.g = d->g[d->cur];
    for (int k = 0; k < 3; ++k) a.u[k] = d->u[k];
    a.rho_l = d->P.rho_l;
    a.drho = d->P.rho_h - d->P.rho_l;
    return a;
}

// read field `which` of the current state into dev_out (FP64, N values)
int read_field(tcp_domain *d, int which, double *dev_out)
{
    ReadArgs a = read_args(d, which);
    a.out = dev_out;
    if (d->sb == 8) launch_read<double>(a, d->stream);
    else launch_read<float>(a, d->stream);
    return check_launch(d);
}

// storage of a field the caller may set (phi^n, u, T^n), or nullptr
void *settable_field(tcp_domain *d, int which)
{
    switch (which) {
    case TCP_PHI: return d->phi[d->cur];
    case TCP_UX: case TCP_UY: case TCP_UZ: return d->u[which - TCP_UX];
    case TCP_T: return d->T[d->cur];
    default: return nullptr;
    }
}

} // namespace

namespace {

// advance nsteps coupled steps from the current state (step graphs on small grids)
int advance(tcp_domain *d, int64_t nsteps)
{
    int64_t left = nsteps;
    if (use_graphs(d, nsteps)) {
        for (; left >= kGraphSteps; left -= kGraphSteps) {
            if (!d->gexec[d->cur]) {
                const int rc = build_graph(d);
                if (rc != TCP_OK) return rc;
            }
            TCP_HIP(d, hipGraphLaunch(d->gexec[d->cur], d->stream));
        }
    }
    run_steps(d, left);
    return check_launch(d);
}

// ---- tape of a coupled run ---------------------------------------------------
StateSlot domain_slot(const tcp_domain *d)
{
    StateSlot s{};
    s.h = d->h[d->cur];
    s.g = d->g[d->cur];
    s.f = d->f[d->cur];
    s.phi = d->phi[d->cur];
    s.T = d->T[d->cur];
    for (int k = 0; k < 3; ++k) s.u[k] = d->u[k];
    return s;
}

constexpr int kSlotPieces = 8; // h, g, f, phi, T, u_x, u_y, u_z

void *&slot_piece(StateSlot &s, int k)
{
    switch (k) {
    case 0: return s.h;
    case 1: return s.g;
    case 2: return s.f;
    case 3: return s.phi;
    case 4: return s.T;
    default: return s.u[k - 5];
    }
}

void slot_sizes(const tcp_domain *d, size_t sz[kSlotPieces])
{
    const size_t N = (size_t)d->geo.N;
    sz[0] = (size_t)pdf_elems(d->geo, d->P.q_pf) * d->pb;
    sz[1] = (size_t)pdf_elems(d->geo, 27) * d->sb;
    sz[2] = (size_t)pdf_elems(d->geo, d->P.q_thermal) * d->pb;
    for (int k = 3; k < kSlotPieces; ++k) sz[k] = N * d->sb;
}

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

int copy_slot(tcp_domain *d, StateSlot dst, StateSlot src)
{
    size_t sz[kSlotPieces];
    slot_sizes(d, sz);
    for (int k = 0; k < kSlotPieces; ++k)
        TCP_HIP(d, hipMemcpyAsync(slot_piece(dst, k), slot_piece(src, k), sz[k], hipMemcpyDeviceToDevice, d->stream));
    return TCP_OK;
}

// One allocation holds nseg + 1 checkpoints, seg - 1 ring states, the taped
// wall temperatures and the reverse sweep's workspace.
int ensure_tape(tcp_domain *d, int64_t nseg, int64_t seg)
{
    auto &tp = d->tape;
    const size_t N = (size_t)d->geo.N, ncol = (size_t)d->P.nx * d->P.nz, sb = d->sb;
    size_t sz[kSlotPieces];
    slot_sizes(d, sz);
    size_t slot = 0;
    for (int k = 0; k < kSlotPieces; ++k) slot += round256(sz[k]);
    const size_t qb[3] = {(size_t)pdf_elems(d->geo, d->P.q_pf) * sb, (size_t)pdf_elems(d->geo, 27) * sb,
                          (size_t)pdf_elems(d->geo, d->P.q_thermal) * sb};
    std::vector<size_t> work;
    for (int k = 0; k < 3; ++k) work.insert(work.end(), {qb[k], qb[k]});          // mu[k][0..1]
    work.insert(work.end(), {5 * N * sb, 5 * N * sb, 4 * N * sb, 4 * N * sb}); // sphi, sT
    work.push_back(4 * N * sb);                                               // lu1, xphi
    work.insert(work.end(), {N * sizeof(double), 2 * ncol * sizeof(double), 4 * kMaxSources * sizeof(double),
                             N * sizeof(double), ncol * sizeof(double), ncol * sizeof(double)});
    const size_t nckpt = (size_t)nseg + 1, nring = (size_t)seg - 1;
    size_t wtotal = 0;
    for (size_t w : work) wtotal += round256(w);
    // a second ring when there is more than one segment to recompute and it
    // fits; otherwise one ring and no overlap (an allocation already made for
    // one ring of these sizes is kept rather than tried again with two)
    int nrings = nseg > 1 && nring > 0 ? 2 : 1;
    if (nrings == 2 && tp.mem && tp.mem_bytes == (nckpt + nring) * slot + wtotal) nrings = 1;
    for (; nrings >= 1; --nrings) {
        const size_t total = (nckpt + nrings * nring) * slot + wtotal;
        if (tp.mem && tp.mem_bytes == total) break;
        if (tp.mem) {
            (void)hipStreamSynchronize(d->stream);
            dev_free(d, tp.mem);
            tp.mem = nullptr;
        }
        tp.mem = dev_alloc(d, total);
        if (tp.mem) {
            tp.mem_bytes = total;
            break;
        }
    }
    if (!tp.mem) return fail(d, TCP_ERR_OOM, "device allocation failed (tape of the coupled run)");
    tp.nrings = nrings;
    if (nrings == 2 && !tp.side) {
        TCP_HIP(d, hipStreamCreateWithFlags(&tp.side, hipStreamNonBlocking));
        for (int r = 0; r < 2; ++r) {
            TCP_HIP(d, hipEventCreateWithFlags(&tp.ready[r], hipEventDisableTiming));
            TCP_HIP(d, hipEventCreateWithFlags(&tp.freed[r], hipEventDisableTiming));
        }
        TCP_HIP(d, hipEventCreateWithFlags(&tp.start, hipEventDisableTiming));
    }
    const size_t nslots = nckpt + nrings * nring;
    char *p = static_cast<char *>(tp.mem);
    tp.ckpt.assign(nckpt, StateSlot{});
    for (int r = 0; r < 2; ++r) {
        tp.ring[r].assign(r < nrings ? nring : 0, StateSlot{});
        tp.ring_seg[r] = -1;
    }
    for (size_t j = 0; j < nslots; ++j) {
        StateSlot &st = j < nckpt ? tp.ckpt[j] : tp.ring[(j - nckpt) / nring][(j - nckpt) % nring];
        for (int k = 0; k < kSlotPieces; ++k) {
            slot_piece(st, k) = p;
            p += round256(sz[k]);
        }
    }
    void **dst[] = {&tp.mu[0][0], &tp.mu[0][1], &tp.mu[1][0], &tp.mu[1][1], &tp.mu[2][0], &tp.mu[2][1],
                    &tp.sphi[0], &tp.sphi[1], &tp.sT[0], &tp.sT[1], &tp.lu1};
    size_t k = 0;
    for (; k < 11; ++k) {
        *dst[k] = p;
        p += round256(work[k]);
    }
    double **dd[] = {&tp.grad_q, &tp.grad_tw, &tp.gsrc, &tp.dphi, &tp.twb, &tp.twt};
    for (int m = 0; m < 6; ++m, ++k) {
        *dd[m] = reinterpret_cast<double *>(p);
        p += round256(work[k]);
    }
    return TCP_OK;
}

// one coupled step (fused kernel) from ring state `from` to `to`, with the
// taped heat sources and wall temperatures
template <typename S, typename Pdf>
void slot_step(tcp_domain *d, const StateSlot &from, const StateSlot &to)
{
    StepArgs a{pf_args(d), hydro_args(d), thermal_args(d)};
    a.pf.h_src = from.h;
    a.pf.h_dst = to.h;
    a.pf.phi_old = from.phi;
    a.pf.phi_new = to.phi;
    a.hy.g_src = from.g;
    a.hy.g_dst = to.g;
    a.hy.phi = from.phi;
    a.hy.T = from.T;
    a.hy.twb = a.th.twb = d->tape.twb;
    a.hy.twt = a.th.twt = d->tape.twt;
    a.th.f_src = from.f;
    a.th.f_dst = to.f;
    a.th.phi = to.phi;
    a.th.T_old = from.T;
    a.th.T = to.T;
    a.th.src = d->tape.src;
    for (int k = 0; k < 3; ++k) {
        a.pf.u[k] = from.u[k];
        a.hy.u[k] = to.u[k];
        a.th.u[k] = to.u[k];
    }
    KernelTimer t(d, TCP_K_STEP);
    if (d->P.q_pf == 15) fused_step_q<15, S, Pdf>(d, a);
    else fused_step_q<27, S, Pdf>(d, a);
}

template <int QH, typename S, typename Pdf>
void reverse_step_q(tcp_domain *d, const CoupledAdjointArgs &a)
{
    switch (d->P.q_thermal) {
    case 7: launch_coupled_adjoint_step<QH, 7, Pdf, S, S>(a, d->stream); break;
    case 15: launch_coupled_adjoint_step<QH, 15, Pdf, S, S>(a, d->stream); break;
    case 19: launch_coupled_adjoint_step<QH, 19, Pdf, S, S>(a, d->stream); break;
    default: launch_coupled_adjoint_step<QH, 27, Pdf, S, S>(a, d->stream); break;
    }
}

// reverse of the step from ring state s0 to s1; the carried adjoint is read
// from parity b and written to 1 - b
template <typename S, typename Pdf>
void reverse_step(tcp_domain *d, const StateSlot &s0, const StateSlot &s1, int b)
{
    auto &tp = d->tape;
    const tcp_params &P = d->P;
    CoupledAdjointArgs a{};
    a.geo = d->geo;
    a.s0 = s0;
    a.s1 = s1;
    for (int k = 0; k < 3; ++k) {
        a.mu_src[k] = tp.mu[k][b];
        a.mu_dst[k] = tp.mu[k][1 - b];
        a.uw_bot[k] = P.u_wall_bot[k];
        a.uw_top[k] = P.u_wall_top[k];
    }
    a.sphi_src = tp.sphi[b];
    a.sphi_dst = tp.sphi[1 - b];
    a.sT_src = tp.sT[b];
    a.sT_dst = tp.sT[1 - b];
    a.lu1 = tp.lu1;
    a.xphi = static_cast<char *>(tp.lu1) + 3 * (size_t)d->geo.N * d->sb;
    a.twb = tp.twb;
    a.twt = tp.twt;
    a.wet[0] = wetting(P.contact_angle_bot, P.xi);
    a.wet[1] = wetting(P.contact_angle_top, P.xi);
    a.t_shift = P.t_shift;
    a.pf = PfCoef{d->omega_phi, 1.0 / P.xi, P.normal_eps * P.normal_eps};
    a.hy = HyCoef{P.rho_l, P.rho_h - P.rho_l, d->tau_l, d->tau_h - d->tau_l, P.sigma_ref, P.sigma_t, P.t_ref, P.xi,
                  {P.g[0], P.g[1], P.g[2]}, P.omega_bulk};
    a.th = ThCoef{P.kappa_l, P.kappa_h - P.kappa_l};
    a.grad_q = tp.grad_q;
    a.grad_twb = tp.grad_tw;
    a.grad_twt = tp.grad_tw + (size_t)P.nx * P.nz;
    KernelTimer t(d, TCP_K_COUPLED_ADJOINT);
    if (P.q_pf == 15) reverse_step_q<15, S, Pdf>(d, a);
    else reverse_step_q<27, S, Pdf>(d, a);
}

// State s (0 .. k_j) of segment j: its first and last are checkpoints, the
// inner ones live in ring r.
const StateSlot &seg_state(const tcp_domain *d, int64_t j, int64_t s, int64_t kj, int r)
{
    const auto &tp = d->tape;
    if (s == 0) return tp.ckpt[(size_t)j];
    if (s == kj) return tp.ckpt[(size_t)j + 1];
    return tp.ring[r][(size_t)s - 1];
}

// the steps of segment j from its checkpoint: the inner states into ring r,
// the last into the next checkpoint (if `last`)
template <typename S, typename Pdf>
void run_segment(tcp_domain *d, int64_t j, int64_t kj, bool last, int r)
{
    for (int64_t s = 0; s < (last ? kj : kj - 1); ++s)
        slot_step<S, Pdf>(d, seg_state(d, j, s, kj, r), seg_state(d, j, s + 1, kj, r));
    d->tape.ring_seg[r] = j;
}

// Launches of the calling scope go to stream s (kernel timers included).
struct OnStream {
    tcp_domain *d;
    hipStream_t saved;
    OnStream(tcp_domain *dd, hipStream_t s) : d(dd), saved(dd->stream) { d->stream = s; }
    ~OnStream() { d->stream = saved; }
};

// The taped run: the domain's state becomes checkpoint 0, every segment runs
// from its checkpoint into the ring and the next checkpoint, and the final
// checkpoint is copied back into the domain.
template <typename S, typename Pdf>
int run_taped(tcp_domain *d)
{
    auto &tp = d->tape;
    int rc = copy_slot(d, tp.ckpt[0], domain_slot(d));
    if (rc != TCP_OK) return rc;
    for (int64_t j = 0; j < tp.nseg; ++j) run_segment<S, Pdf>(d, j, std::min(tp.seg, tp.nsteps - j * tp.seg), true, 0);
    rc = copy_slot(d, domain_slot(d), tp.ckpt[(size_t)tp.nseg]);
    if (rc != TCP_OK) return rc;
    return check_launch(d);
}

// The recomputation of taped steps runs with the heat sources and wall
// temperatures of the taped run, whatever the domain holds by then; the
// domain's own are restored at the end of the scope.
struct TapedInputs {
    tcp_domain *d;
    HeatSources src;
    double *twb, *twt;
    explicit TapedInputs(tcp_domain *dd) : d(dd), src(dd->src), twb(dd->twb), twt(dd->twt)
    {
        d->src = d->tape.src;
        d->twb = d->tape.twb;
        d->twt = d->tape.twt;
    }
    ~TapedInputs()
    {
        d->src = src;
        d->twb = twb;
        d->twt = twt;
    }
};

// Reverse sweep over the taped steps, last segment first: recompute the inner
// states of a segment from its checkpoint (unless a ring holds them already),
// then undo its steps last to first.  With two rings the recomputation of
// segment j - 1 runs on the side stream into one ring while the reverse steps
// of segment j read the other: the side stream waits until the reverse sweep
// that last read its ring is done (`freed`), the main stream until the ring
// it is about to read is filled (`ready`).  The loss enters through the final
// phase field (seeded before the first reverse step).
template <typename S, typename Pdf>
int run_tape_adjoint(tcp_domain *d, const double gc[3], const double *dphi)
{
    auto &tp = d->tape;
    const size_t ncol = (size_t)d->P.nx * d->P.nz;
    launch_reduce<S>(d->geo, tp.ckpt[(size_t)tp.nseg].phi, d->partial, d->out4, d->stream);
    launch_coupled_adjoint_seed<S>(d->geo, d->out4, gc, dphi, tp.sphi[0], d->stream);
    const bool overlap = tp.nrings == 2;
    if (overlap) {
        // the side stream starts after everything queued so far; both rings
        // count as released at the start (every event waited on is recorded)
        TCP_HIP(d, hipEventRecord(tp.start, d->stream));
        TCP_HIP(d, hipStreamWaitEvent(tp.side, tp.start, 0));
        for (int k = 0; k < 2; ++k) TCP_HIP(d, hipEventRecord(tp.freed[k], d->stream));
    }
    auto kseg = [&](int64_t j) { return std::min(tp.seg, tp.nsteps - j * tp.seg); };
    int b = 0;
    int r = 0; // ring of segment j (the taped run leaves the last segment in ring 0)
    for (int64_t j = tp.nseg - 1; j >= 0; --j) {
        const int64_t kj = kseg(j);
        if (tp.ring_seg[r] != j) run_segment<S, Pdf>(d, j, kj, false, r);
        if (overlap && j > 0) {
            // recompute segment j - 1 into the other ring meanwhile
            const int o = 1 - r;
            TCP_HIP(d, hipStreamWaitEvent(tp.side, tp.freed[o], 0));
            {
                OnStream on(d, tp.side);
                run_segment<S, Pdf>(d, j - 1, kseg(j - 1), false, o);
            }
            TCP_HIP(d, hipEventRecord(tp.ready[o], tp.side));
        }
        for (int64_t s = kj - 1; s >= 0; --s) {
            reverse_step<S, Pdf>(d, seg_state(d, j, s, kj, r), seg_state(d, j, s + 1, kj, r), b);
            b = 1 - b;
        }
        if (overlap && j > 0) {
            TCP_HIP(d, hipEventRecord(tp.freed[r], d->stream));
            r = 1 - r;
            TCP_HIP(d, hipStreamWaitEvent(d->stream, tp.ready[r], 0));
        }
        const int rc = check_launch(d);
        if (rc != TCP_OK) return rc;
    }
    launch_coupled_adjoint_tw<S>(d->geo, tp.sT[b], tp.grad_tw, tp.grad_tw + ncol, d->stream);
    return check_launch(d);
}

// best rate (read + write bytes per second, GB/s) of reps launches of a copy
// between two fresh device buffers of `bytes` each (one untimed warm-up)
template <typename Launch>
int copy_probe(size_t bytes, int reps, double *gbs, Launch launch)
{
    void *a = nullptr, *b = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = TCP_OK;
    if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) {
        (void)hipGetLastError();
        rc = fail(nullptr, TCP_ERR_OOM, "probe allocation failed");
    } else if (hipMemset(a, 0, bytes) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
               hipEventCreate(&e1) != hipSuccess) {
        rc = fail(nullptr, TCP_ERR_HIP, "probe set-up failed");
    } else {
        double best = 0.0;
        launch(a, b); // warm-up
        for (int r = 0; r < reps && rc == TCP_OK; ++r) {
            float ms = 0.0f;
            if (hipEventRecord(e0, nullptr) != hipSuccess) rc = TCP_ERR_HIP;
            launch(a, b);
            if (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                rc = TCP_ERR_HIP;
            if (rc == TCP_OK && ms > 0.0f) best = std::max(best, 2.0 * (double)bytes / (ms * 1e-3) / 1e9);
        }
        if (rc != TCP_OK) fail(nullptr, rc, "probe timing failed");
        *gbs = best;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    return rc;
}
} // namespace

extern "C" {

int tcp_params_default(tcp_params *p)
{
    if (!p) return TCP_ERR_ARG;
    std::memset(p, 0, sizeof *p);
    p->nx = p->ny = p->nz = 32;
    p->q_pf = 15;
    p->q_thermal = 7;
    p->thermal = TCP_THERMAL_LB;
    p->precision = TCP_FP64;
    p->rho_h = p->rho_l = 1.0;
    p->nu_h = p->nu_l = 1.0 / 6.0;
    p->mobility = 0.05;
    p->xi = 5.0;
    p->kappa_h = p->kappa_l = 0.2;
    p->omega_bulk = 1.0;
    p->normal_eps = 1e-6;
    p->contact_angle_bot = p->contact_angle_top = 90.0;
    return TCP_OK;
}

int tcp_create(const tcp_params *p, const tcp_allocator *alloc, void *stream, tcp_domain **out)
{
    if (!p || !out) return fail(nullptr, TCP_ERR_ARG, "null argument");
    *out = nullptr;
    std::string why;
    int rc = validate(p, why);
    if (rc != TCP_OK) return fail(nullptr, rc, why);
    if (alloc && (!alloc->alloc || !alloc->free)) return fail(nullptr, TCP_ERR_ARG, "allocator needs alloc and free");
    tcp_domain *d = new (std::nothrow) tcp_domain();
    if (!d) return fail(nullptr, TCP_ERR_OOM, "host allocation failed");
    d->P = *p;
    if (alloc) {
        d->A = *alloc;
        d->own_alloc = false;
    }
    d->stream = static_cast<hipStream_t>(stream);
    if (hipGetDevice(&d->device) != hipSuccess) {
        delete d;
        return fail(nullptr, TCP_ERR_HIP, "hipGetDevice failed");
    }
    d->sb = p->precision == TCP_FP64 ? 8 : 4;
    d->pb = p->precision == TCP_FP64 ? 8 : (p->precision == TCP_FP32 ? 4 : 2);
    d->geo.nx = p->nx;
    d->geo.ny = p->ny;
    d->geo.nz = p->nz;
    d->geo.walls = p->walls_y;
    d->geo.nbx = (p->nx + 63) / 64;
    d->geo.plane = (int64_t)p->nx * p->ny;
    d->geo.N = d->geo.plane * p->nz;
    d->omega_phi = 1.0 / (0.5 + 3.0 * p->mobility);
    d->tau_h = 3.0 * p->nu_h;
    d->tau_l = 3.0 * p->nu_l;
    const size_t N = (size_t)d->geo.N, sb = d->sb, pb = d->pb;
    const size_t ncol = (size_t)p->nx * p->nz;
    // All device state lives in one allocation, every buffer starting on a
    // kArenaAlign boundary (plus kArenaStagger bytes per buffer index).
    std::vector<std::pair<void **, size_t>> req;
    for (int b = 0; b < 2; ++b) {
        req.push_back({&d->h[b], (size_t)pdf_elems(d->geo, p->q_pf) * pb});
        req.push_back({&d->g[b], (size_t)pdf_elems(d->geo, 27) * sb});
        if (p->thermal == TCP_THERMAL_LB) req.push_back({&d->f[b], (size_t)pdf_elems(d->geo, p->q_thermal) * pb});
        req.push_back({&d->phi[b], N * sb});
        req.push_back({&d->T[b], N * sb});
    }
    for (int k = 0; k < 3; ++k) req.push_back({&d->u[k], N * sb});
    if (p->thermal != TCP_THERMAL_LB)
        for (int k = 0; k < (p->thermal == TCP_THERMAL_RK2 ? 1 : 3); ++k) req.push_back({&d->rk[k], N * sb});
    if (p->thermal != TCP_THERMAL_LB) req.push_back({&d->rkc, 5 * N * sb});
    void *twb = nullptr, *twt = nullptr, *partial = nullptr, *out4 = nullptr;
    req.push_back({&twb, ncol * sizeof(double)});
    req.push_back({&twt, ncol * sizeof(double)});
    req.push_back({&partial, 4 * kReduceBlocks * sizeof(double)});
    req.push_back({&out4, 4 * sizeof(double)});
    size_t total = 0;
    std::vector<size_t> offset;
    for (size_t k = 0; k < req.size(); ++k) {
        offset.push_back(total + k * kArenaStagger);
        total += (req[k].second + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
    }
    total += req.size() * kArenaStagger;
    char *arena = static_cast<char *>(own(d, total));
    bool ok = arena != nullptr;
    if (ok) {
        for (size_t k = 0; k < req.size(); ++k) *req[k].first = arena + offset[k];
        d->twb = static_cast<double *>(twb);
        d->twt = static_cast<double *>(twt);
        d->partial = static_cast<double *>(partial);
        d->out4 = static_cast<double *>(out4);
    }
    if (!ok) {
        tcp_destroy(d);
        return fail(nullptr, TCP_ERR_OOM, "device allocation failed");
    }
    std::vector<double> col(ncol, p->t_wall_bot);
    hipError_t e = hipMemcpyAsync(d->twb, col.data(), ncol * sizeof(double), hipMemcpyHostToDevice, d->stream);
    if (e == hipSuccess) {
        std::fill(col.begin(), col.end(), p->t_wall_top);
        e = hipMemcpyAsync(d->twt, col.data(), ncol * sizeof(double), hipMemcpyHostToDevice, d->stream);
    }
    // zero the fields so that an uninitialised read is well defined
    for (int k = 0; k < 3 && e == hipSuccess; ++k) e = hipMemsetAsync(d->u[k], 0, N * sb, d->stream);
    for (int b = 0; b < 2 && e == hipSuccess; ++b) e = hipMemsetAsync(d->T[b], 0, N * sb, d->stream);
    for (int b = 0; b < 2 && e == hipSuccess; ++b) e = hipMemsetAsync(d->phi[b], 0, N * sb, d->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(d->stream);
    if (e != hipSuccess) {
        std::string msg = std::string("set-up: ") + hipGetErrorString(e);
        tcp_destroy(d);
        return fail(nullptr, TCP_ERR_HIP, msg);
    }
    *out = d;
    return TCP_OK;
}

int tcp_destroy(tcp_domain *d)
{
    if (!d) return TCP_ERR_ARG;
    (void)hipStreamSynchronize(d->stream);
    drop_graphs(d);
    if (d->cap_stream) (void)hipStreamDestroy(d->cap_stream);
    if (d->tape.side) {
        (void)hipStreamSynchronize(d->tape.side);
        (void)hipStreamDestroy(d->tape.side);
    }
    for (hipEvent_t e : {d->tape.ready[0], d->tape.ready[1], d->tape.freed[0], d->tape.freed[1], d->tape.start})
        if (e) (void)hipEventDestroy(e);
    for (auto &r : d->records) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    for (auto e : d->pool) (void)hipEventDestroy(e);
    if (d->tape.mem) dev_free(d, d->tape.mem);
    for (void *p : d->owned) dev_free(d, p);
    delete d;
    return TCP_OK;
}

int tcp_set_field(tcp_domain *d, int which, const double *host, const void *dev)
{
    if (!d) return TCP_ERR_ARG;
    if ((host == nullptr) == (dev == nullptr)) return fail(d, TCP_ERR_ARG, "give exactly one of host or dev");
    void *dst = settable_field(d, which);
    if (!dst) return fail(d, TCP_ERR_ARG, "field cannot be set");
    return guarded(d, [&]() -> int {
        const int64_t N = d->geo.N;
        const double *src = static_cast<const double *>(dev);
        Scratch tmp(d, host ? (size_t)N * sizeof(double) : 0);
        if (host) {
            if (!tmp.p) return fail(d, TCP_ERR_OOM, "staging allocation failed");
            TCP_HIP(d, hipMemcpyAsync(tmp.p, host, (size_t)N * sizeof(double), hipMemcpyHostToDevice, d->stream));
            src = static_cast<const double *>(tmp.p);
        }
        if (d->sb == 8) launch_from_f64<double>(src, dst, N, d->stream);
        else launch_from_f64<float>(src, dst, N, d->stream);
        d->initialized = false;
        return check_launch(d);
    });
}

int tcp_set_field_f32(tcp_domain *d, int which, const float *dev)
{
    if (!d) return TCP_ERR_ARG;
    if (!dev) return fail(d, TCP_ERR_ARG, "a device source array is required");
    void *dst = settable_field(d, which);
    if (!dst) return fail(d, TCP_ERR_ARG, "field cannot be set");
    return guarded(d, [&]() -> int {
        if (d->sb == 8) launch_from_f32<double>(dev, dst, d->geo.N, d->stream);
        else launch_from_f32<float>(dev, dst, d->geo.N, d->stream);
        d->initialized = false;
        return check_launch(d);
    });
}

int tcp_set_droplets(tcp_domain *d, const tcp_droplet *drops, int n)
{
    if (!d || n < 0 || (n > 0 && !drops)) return fail(d, TCP_ERR_ARG, "bad droplet list");
    return guarded(d, [&]() -> int {
        Scratch tmp(d, (size_t)(n > 0 ? n : 1) * 4 * sizeof(double));
        if (!tmp.p) return fail(d, TCP_ERR_OOM, "staging allocation failed");
        std::vector<double> xyzr((size_t)n * 4);
        for (int k = 0; k < n; ++k) {
            xyzr[4 * k + 0] = drops[k].x;
            xyzr[4 * k + 1] = drops[k].y;
            xyzr[4 * k + 2] = drops[k].z;
            xyzr[4 * k + 3] = drops[k].r;
        }
        if (n > 0)
            TCP_HIP(d, hipMemcpyAsync(tmp.p, xyzr.data(), xyzr.size() * sizeof(double), hipMemcpyHostToDevice, d->stream));
        Droplets dl{};
        dl.n = n;
        dl.xyzr = static_cast<const double *>(tmp.p);
        dl.inv_xi = 1.0 / d->P.xi;
        dl.periodic[0] = 1;
        dl.periodic[1] = d->P.walls_y ? 0 : 1;
        dl.periodic[2] = 1;
        if (d->sb == 8) launch_droplets<double>(d->geo, dl, d->phi[d->cur], d->stream);
        else launch_droplets<float>(d->geo, dl, d->phi[d->cur], d->stream);
        d->initialized = false;
        return check_launch(d);
    });
}

int tcp_set_heat_sources(tcp_domain *d, const tcp_heat_source *s, int n)
{
    if (!d) return TCP_ERR_ARG;
    if (n < 0 || n > kMaxSources || (n > 0 && !s)) return fail(d, TCP_ERR_ARG, "at most 16 heat sources");
    HeatSources hs{};
    hs.n = n;
    for (int k = 0; k < n; ++k) {
        if (!std::isfinite(s[k].Q) || !finite_pos(s[k].w) || !std::isfinite(s[k].x) || !std::isfinite(s[k].y) ||
            !std::isfinite(s[k].z) || !std::isfinite(s[k].d_cut))
            return fail(d, TCP_ERR_ARG, "heat source needs finite values and w > 0");
        hs.Q[k] = s[k].Q;
        hs.x[k] = s[k].x;
        hs.y[k] = s[k].y;
        hs.z[k] = s[k].z;
        hs.inv_w2[k] = 1.0 / (s[k].w * s[k].w);
        hs.dcut2[k] = s[k].d_cut > 0.0 ? s[k].d_cut * s[k].d_cut : 0.0;
    }
    d->src = hs;
    d->rkq_ready = false; // the RK heat-source field is evaluated again
    drop_graphs(d); // captured launches hold the previous sources by value
    return TCP_OK;
}

int tcp_set_wall_temperature(tcp_domain *d, int wall, const double *Tw)
{
    if (!d) return TCP_ERR_ARG;
    if ((wall != 0 && wall != 1) || !Tw) return fail(d, TCP_ERR_ARG, "wall must be 0 or 1, Tw non-NULL");
    double *dst = wall == 0 ? d->twb : d->twt;
    TCP_HIP(d, hipMemcpyAsync(dst, Tw, (size_t)d->P.nx * d->P.nz * sizeof(double), hipMemcpyHostToDevice, d->stream));
    TCP_HIP(d, hipStreamSynchronize(d->stream));
    return TCP_OK;
}

int tcp_initialize(tcp_domain *d)
{
    if (!d) return TCP_ERR_ARG;
    InitArgs a{};
    a.geo = d->geo;
    a.q_pf = d->P.q_pf;
    a.q_th = d->P.q_thermal;
    a.phi = d->phi[d->cur];
    for (int k = 0; k < 3; ++k) a.u[k] = d->u[k];
    a.T = d->T[d->cur];
    a.h = d->h[d->cur];
    a.g = d->g[d->cur];
    a.f = d->P.thermal == TCP_THERMAL_LB ? d->f[d->cur] : nullptr;
    a.phi_other = d->phi[1 - d->cur];
    a.t_shift = d->P.t_shift;
    switch (d->P.precision) {
    case TCP_FP64: launch_init<double, double>(a, d->stream); break;
    case TCP_FP32: launch_init<float, float>(a, d->stream); break;
    default: launch_init<float, _Float16>(a, d->stream); break;
    }
    int rc = check_launch(d);
    if (rc == TCP_OK) d->initialized = true;
    return rc;
}

int tcp_step(tcp_domain *d, int64_t nsteps)
{
    if (!d) return TCP_ERR_ARG;
    if (nsteps < 0) return fail(d, TCP_ERR_ARG, "nsteps must be >= 0");
    if (!d->initialized) return fail(d, TCP_ERR_STATE, "tcp_initialize must precede tcp_step");
    return guarded(d, [&]() -> int { return advance(d, nsteps); });
}

int tcp_step_taped(tcp_domain *d, int64_t nsteps, int64_t segment)
{
    if (!d) return TCP_ERR_ARG;
    if (nsteps < 1) return fail(d, TCP_ERR_ARG, "nsteps must be >= 1");
    if (!d->initialized) return fail(d, TCP_ERR_STATE, "tcp_initialize must precede tcp_step_taped");
    if (d->P.thermal != TCP_THERMAL_LB)
        return fail(d, TCP_ERR_UNSUPPORTED, "the adjoint of the coupled step is built for the thermal LB only");
    return guarded(d, [&]() -> int {
        auto &tp = d->tape;
        tp.valid = false;
        const int64_t seg = segment > 0 ? std::min(segment, nsteps)
                                        : std::max<int64_t>(1, (int64_t)std::ceil(std::sqrt((double)nsteps)));
        const int64_t nseg = (nsteps + seg - 1) / seg;
        int rc = ensure_tape(d, nseg, seg);
        if (rc != TCP_OK) return rc;
        tp.src = d->src;
        const size_t ncol = (size_t)d->P.nx * d->P.nz;
        TCP_HIP(d, hipMemcpyAsync(tp.twb, d->twb, ncol * sizeof(double), hipMemcpyDeviceToDevice, d->stream));
        TCP_HIP(d, hipMemcpyAsync(tp.twt, d->twt, ncol * sizeof(double), hipMemcpyDeviceToDevice, d->stream));
        tp.nsteps = nsteps;
        tp.seg = seg;
        tp.nseg = nseg;
        switch (d->P.precision) {
        case TCP_FP64: rc = run_taped<double, double>(d); break;
        case TCP_FP32: rc = run_taped<float, float>(d); break;
        default: rc = run_taped<float, _Float16>(d); break;
        }
        if (rc != TCP_OK) return rc;
        tp.valid = true;
        return TCP_OK;
    });
}

int tcp_tape_adjoint(tcp_domain *d, const double dL_dcentroid[3], const double *dL_dphi, double *dL_dsource,
                     double *dL_dTw_bot, double *dL_dTw_top)
{
    if (!d || !dL_dcentroid) return fail(d, TCP_ERR_ARG, "dL_dcentroid is required");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(dL_dcentroid[k])) return fail(d, TCP_ERR_ARG, "dL_dcentroid must be finite");
    if (!d->tape.valid) return fail(d, TCP_ERR_STATE, "no taped run: tcp_step_taped must precede tcp_tape_adjoint");
    return guarded(d, [&]() -> int {
        auto &tp = d->tape;
        const size_t N = (size_t)d->geo.N, ncol = (size_t)d->P.nx * d->P.nz, sb = d->sb;
        const size_t qb[3] = {(size_t)pdf_elems(d->geo, d->P.q_pf) * sb, (size_t)pdf_elems(d->geo, 27) * sb,
                              (size_t)pdf_elems(d->geo, d->P.q_thermal) * sb};
        for (int k = 0; k < 3; ++k) TCP_HIP(d, hipMemsetAsync(tp.mu[k][0], 0, qb[k], d->stream));
        TCP_HIP(d, hipMemsetAsync(tp.sT[0], 0, 4 * N * sb, d->stream));
        TCP_HIP(d, hipMemsetAsync(tp.lu1, 0, 3 * N * sb, d->stream));
        TCP_HIP(d, hipMemsetAsync(tp.grad_q, 0, N * sizeof(double), d->stream));
        TCP_HIP(d, hipMemsetAsync(tp.grad_tw, 0, 2 * ncol * sizeof(double), d->stream));
        if (dL_dphi)
            TCP_HIP(d, hipMemcpyAsync(tp.dphi, dL_dphi, N * sizeof(double), hipMemcpyHostToDevice, d->stream));
        const double *dphi = dL_dphi ? tp.dphi : nullptr;
        int rc;
        {
            TapedInputs taped(d);
            switch (d->P.precision) {
            case TCP_FP64: rc = run_tape_adjoint<double, double>(d, dL_dcentroid, dphi); break;
            case TCP_FP32: rc = run_tape_adjoint<float, float>(d, dL_dcentroid, dphi); break;
            default: rc = run_tape_adjoint<float, _Float16>(d, dL_dcentroid, dphi); break;
            }
        }
        if (rc != TCP_OK) return rc;
        const int ns = tp.src.n;
        if (ns > 0) launch_source_grad(d->geo, tp.src, tp.grad_q, d->partial, tp.gsrc, d->stream);
        rc = check_launch(d);
        if (rc != TCP_OK) return rc;
        if (dL_dsource && ns > 0)
            TCP_HIP(d, hipMemcpyAsync(dL_dsource, tp.gsrc, 4 * ns * sizeof(double), hipMemcpyDeviceToHost, d->stream));
        if (dL_dTw_bot)
            TCP_HIP(d, hipMemcpyAsync(dL_dTw_bot, tp.grad_tw, ncol * sizeof(double), hipMemcpyDeviceToHost, d->stream));
        if (dL_dTw_top)
            TCP_HIP(d, hipMemcpyAsync(dL_dTw_top, tp.grad_tw + ncol, ncol * sizeof(double), hipMemcpyDeviceToHost,
                                      d->stream));
        TCP_HIP(d, hipStreamSynchronize(d->stream));
        return TCP_OK;
    });
}

int tcp_warm_temperature(tcp_domain *d, int64_t max_steps, double tol, int64_t check_every, int64_t *steps_done,
                         double *change)
{
    if (!d) return TCP_ERR_ARG;
    if (max_steps < 0) return fail(d, TCP_ERR_ARG, "max_steps must be >= 0");
    if (check_every < 1) return fail(d, TCP_ERR_ARG, "check_every must be >= 1");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(d, TCP_ERR_ARG, "tol must be finite and >= 0");
    if (!d->initialized) return fail(d, TCP_ERR_STATE, "tcp_initialize must precede tcp_warm_temperature");
    return guarded(d, [&]() -> int {
        const size_t nb = (size_t)d->geo.N * d->sb;
        const int start = d->cur;
        TCP_HIP(d, hipMemcpyAsync(d->phi[1 - start], d->phi[start], nb, hipMemcpyDeviceToDevice, d->stream));
        int64_t done = 0;
        double last = 0.0;
        bool measured = false;
        while (done < max_steps) {
            const int64_t k = std::min(check_every - done % check_every, max_steps - done);
            run_thermal_steps(d, k);
            done += k;
            if (done % check_every != 0 && done != max_steps) continue;
            // T of the last two time levels sit in the two parities
            if (d->sb == 8) launch_maxdiff<double>(d->geo.N, d->T[0], d->T[1], d->partial, d->out4, d->stream);
            else launch_maxdiff<float>(d->geo.N, d->T[0], d->T[1], d->partial, d->out4, d->stream);
            const int rc = check_launch(d);
            if (rc != TCP_OK) return rc;
            TCP_HIP(d, hipMemcpyAsync(&last, d->out4, sizeof last, hipMemcpyDeviceToHost, d->stream));
            TCP_HIP(d, hipStreamSynchronize(d->stream));
            measured = true;
            if (!std::isfinite(last)) return fail(d, TCP_ERR_NONFINITE, "temperature holds NaN or Inf");
            if (last <= tol) break;
        }
        // an odd count leaves the new thermal state in the other parity than the
        // phase-field and hydrodynamic PDFs: move it back
        if (d->cur != start) {
            if (d->P.thermal == TCP_THERMAL_LB) {
                const size_t fb = (size_t)pdf_elems(d->geo, d->P.q_thermal) * d->pb;
                TCP_HIP(d, hipMemcpyAsync(d->f[start], d->f[d->cur], fb, hipMemcpyDeviceToDevice, d->stream));
            }
            TCP_HIP(d, hipMemcpyAsync(d->T[start], d->T[d->cur], nb, hipMemcpyDeviceToDevice, d->stream));
            d->cur = start;
        }
        if (steps_done) *steps_done = done;
        if (change) *change = measured ? last : 0.0;
        return check_launch(d);
    });
}

int tcp_thermal_adjoint(tcp_domain *d, int64_t nsteps, const double *dL_dT, double *dL_dsource,
                        double *dL_dTw_bot, double *dL_dTw_top)
{
    if (!d) return TCP_ERR_ARG;
    if (nsteps < 0) return fail(d, TCP_ERR_ARG, "nsteps must be >= 0");
    if (!dL_dT) return fail(d, TCP_ERR_ARG, "dL_dT (one value per cell) is required");
    if (!d->initialized) return fail(d, TCP_ERR_STATE, "tcp_initialize must precede tcp_thermal_adjoint");
    return guarded(d, [&]() -> int {
        const size_t N = (size_t)d->geo.N, ncol = (size_t)d->P.nx * d->P.nz;
        const bool lb = d->P.thermal == TCP_THERMAL_LB;
        if (!d->adj_m) {
            // link adjoints (LB) or eight fields (RK: lambda', acc, two stage fields,
            // four coefficients), then the FP64 buffers
            const size_t mb = lb ? (size_t)pdf_elems(d->geo, d->P.q_thermal) * d->sb : 8 * N * d->sb;
            void *p[6] = {own(d, mb), lb ? own(d, mb) : nullptr, own(d, N * sizeof(double)),
                          own(d, N * sizeof(double)), own(d, 2 * ncol * sizeof(double)),
                          own(d, 4 * kMaxSources * sizeof(double))};
            for (int k = 0; k < 6; ++k)
                if (!p[k] && (k != 1 || lb)) return fail(d, TCP_ERR_OOM, "device allocation failed (adjoint workspace)");
            if (lb) {
                d->adj_mu[0] = p[0];
                d->adj_mu[1] = p[1];
            } else {
                d->adj_rk = p[0];
            }
            d->adj_m = static_cast<double *>(p[2]);
            d->adj_g = static_cast<double *>(p[3]);
            d->adj_tw = static_cast<double *>(p[4]);
            d->adj_q = static_cast<double *>(p[5]);
        }
        TCP_HIP(d, hipMemcpyAsync(d->adj_m, dL_dT, N * sizeof(double), hipMemcpyHostToDevice, d->stream));
        TCP_HIP(d, hipMemsetAsync(d->adj_g, 0, N * sizeof(double), d->stream));
        TCP_HIP(d, hipMemsetAsync(d->adj_tw, 0, 2 * ncol * sizeof(double), d->stream));
        const bool f64 = d->sb == 8;
        if (!lb) {
            if (f64) run_rk_adjoint<double>(d, nsteps);
            else run_rk_adjoint<float>(d, nsteps);
        } else switch (d->P.q_thermal) {
        case 7: f64 ? run_thermal_adjoint<7, double>(d, nsteps) : run_thermal_adjoint<7, float>(d, nsteps); break;
        case 15: f64 ? run_thermal_adjoint<15, double>(d, nsteps) : run_thermal_adjoint<15, float>(d, nsteps); break;
        case 19: f64 ? run_thermal_adjoint<19, double>(d, nsteps) : run_thermal_adjoint<19, float>(d, nsteps); break;
        default: f64 ? run_thermal_adjoint<27, double>(d, nsteps) : run_thermal_adjoint<27, float>(d, nsteps); break;
        }
        const int ns = d->src.n;
        if (ns > 0) launch_source_grad(d->geo, d->src, d->adj_g, d->partial, d->adj_q, d->stream);
        int rc = check_launch(d);
        if (rc != TCP_OK) return rc;
        if (dL_dsource && ns > 0)
            TCP_HIP(d, hipMemcpyAsync(dL_dsource, d->adj_q, 4 * ns * sizeof(double), hipMemcpyDeviceToHost,
                                      d->stream));
        if (dL_dTw_bot)
            TCP_HIP(d, hipMemcpyAsync(dL_dTw_bot, d->adj_tw, ncol * sizeof(double), hipMemcpyDeviceToHost, d->stream));
        if (dL_dTw_top)
            TCP_HIP(d, hipMemcpyAsync(dL_dTw_top, d->adj_tw + ncol, ncol * sizeof(double), hipMemcpyDeviceToHost,
                                      d->stream));
        TCP_HIP(d, hipStreamSynchronize(d->stream));
        return TCP_OK;
    });
}

int tcp_get_field(tcp_domain *d, int which, double *host, void *dev)
{
    if (!d) return TCP_ERR_ARG;
    if ((host == nullptr) == (dev == nullptr)) return fail(d, TCP_ERR_ARG, "give exactly one of host or dev");
    if (which < TCP_PHI || which > TCP_RHO) return fail(d, TCP_ERR_ARG, "unknown field");
    return guarded(d, [&]() -> int {
        const int64_t N = d->geo.N;
        Scratch tmp(d, host ? (size_t)N * sizeof(double) : 0);
        if (host && !tmp.p) return fail(d, TCP_ERR_OOM, "staging allocation failed");
        ReadArgs a = read_args(d, which);
        a.out = host ? static_cast<double *>(tmp.p) : static_cast<double *>(dev);
        if (d->sb == 8) launch_read<double>(a, d->stream);
        else launch_read<float>(a, d->stream);
        int rc = check_launch(d);
        if (rc != TCP_OK) return rc;
        if (host) {
            TCP_HIP(d, hipMemcpyAsync(host, tmp.p, (size_t)N * sizeof(double), hipMemcpyDeviceToHost, d->stream));
            TCP_HIP(d, hipStreamSynchronize(d->stream));
        }
        return TCP_OK;
    });
}

int tcp_get_field_f32(tcp_domain *d, int which, float *dev)
{
    if (!d) return TCP_ERR_ARG;
    if (!dev) return fail(d, TCP_ERR_ARG, "a device destination array is required");
    if (which < TCP_PHI || which > TCP_RHO) return fail(d, TCP_ERR_ARG, "unknown field");
    return guarded(d, [&]() -> int {
        const ReadArgs a = read_args(d, which);
        if (d->sb == 8) launch_read_f32<double>(a, dev, d->stream);
        else launch_read_f32<float>(a, dev, d->stream);
        return check_launch(d);
    });
}

int tcp_get_field_noalloc(tcp_domain *d, int which, double *host)
{
    if (!d || !host) return fail(d, TCP_ERR_ARG, "a domain and a host destination are required");
    if (which < TCP_PHI || which > TCP_RHO) return fail(d, TCP_ERR_ARG, "unknown field");
    const size_t N = (size_t)d->geo.N;
    if (N > kNoAllocCells)
        return fail(d, TCP_ERR_UNSUPPORTED,
                    "tcp_get_field_noalloc reads at most 4194304 cells (its 32 MiB staging array); use tcp_get_field");
    if (d->device < 0 || d->device >= kMaxDevices) return fail(d, TCP_ERR_UNSUPPORTED, "device index out of range");
    int prev = 0;
    TCP_HIP(d, hipGetDevice(&prev));
    if (prev != d->device) TCP_HIP(d, hipSetDevice(d->device));
    const int rc = guarded(d, [&]() -> int {
        void *ptr = nullptr;
        int r = scratch_address(d, d->device, &ptr);
        if (r != TCP_OK) return r;
        r = read_field(d, which, static_cast<double *>(ptr));
        if (r != TCP_OK) return r;
        TCP_HIP(d, hipMemcpyAsync(host, ptr, N * sizeof(double), hipMemcpyDeviceToHost, d->stream));
        TCP_HIP(d, hipStreamSynchronize(d->stream));
        return TCP_OK;
    });
    if (prev != d->device) (void)hipSetDevice(prev);
    return rc;
}

int tcp_get_pdfs(tcp_domain *d, int which, double *host_out)
{
    if (!d || !host_out) return TCP_ERR_ARG;
    const void *src = nullptr;
    int q = 0;
    size_t bytes = d->pb;
    double shift = 0.0;
    const void *field = nullptr; // FP32/FP16 PDFs are stored relative to w_i phi(x) or w_i T(x)
    if (which == TCP_PDF_H) {
        src = d->h[d->cur];
        q = d->P.q_pf;
        if (d->pb <= 4) field = d->phi[d->cur];
    } else if (which == TCP_PDF_G) {
        src = d->g[d->cur];
        q = 27;
        bytes = d->sb;
    } else if (which == TCP_PDF_F && d->P.thermal == TCP_THERMAL_LB) {
        src = d->f[d->cur];
        q = d->P.q_thermal;
        if (d->pb <= 4) field = d->T[d->cur];
        else shift = d->P.t_shift;
    } else {
        return fail(d, TCP_ERR_ARG, "unknown PDF field for this configuration");
    }
    return guarded(d, [&]() -> int {
        const int64_t N = d->geo.N;
        Scratch tmp(d, (size_t)N * q * sizeof(double));
        if (!tmp.p) return fail(d, TCP_ERR_OOM, "staging allocation failed");
        double *o = static_cast<double *>(tmp.p);
        if (bytes == 8) launch_read_pdfs<double, double>(src, q, d->geo, shift, field, o, d->stream);
        else if (bytes == 4) launch_read_pdfs<float, float>(src, q, d->geo, shift, field, o, d->stream);
        else launch_read_pdfs<_Float16, float>(src, q, d->geo, shift, field, o, d->stream);
        int rc = check_launch(d);
        if (rc != TCP_OK) return rc;
        TCP_HIP(d, hipMemcpyAsync(host_out, tmp.p, (size_t)N * q * sizeof(double), hipMemcpyDeviceToHost, d->stream));
        TCP_HIP(d, hipStreamSynchronize(d->stream));
        return TCP_OK;
    });
}

int tcp_reduce(tcp_domain *d, double *mass, double centroid[3])
{
    if (!d || !mass || !centroid) return TCP_ERR_ARG;
    if (d->sb == 8) launch_reduce<double>(d->geo, d->phi[d->cur], d->partial, d->out4, d->stream);
    else launch_reduce<float>(d->geo, d->phi[d->cur], d->partial, d->out4, d->stream);
    int rc = check_launch(d);
    if (rc != TCP_OK) return rc;
    double h4[4];
    TCP_HIP(d, hipMemcpyAsync(h4, d->out4, sizeof h4, hipMemcpyDeviceToHost, d->stream));
    TCP_HIP(d, hipStreamSynchronize(d->stream));
    *mass = h4[0];
    for (int k = 0; k < 3; ++k) centroid[k] = h4[k + 1] / h4[0];
    for (double v : h4)
        if (!std::isfinite(v)) return fail(d, TCP_ERR_NONFINITE, "phase field holds NaN or Inf");
    return TCP_OK;
}


int tcp_state_bytes(const tcp_domain *d, size_t *bytes)
{
    if (!d || !bytes) return TCP_ERR_ARG;
    size_t s = 0;
    for (auto &p : state_pieces(d)) s += p.bytes;
    *bytes = s;
    return TCP_OK;
}

int tcp_save_state(tcp_domain *d, void *host)
{
    if (!d || !host) return TCP_ERR_ARG;
    if (!d->initialized) return fail(d, TCP_ERR_STATE, "nothing to save before tcp_initialize");
    char *dst = static_cast<char *>(host);
    for (auto &p : state_pieces(d)) {
        TCP_HIP(d, hipMemcpyAsync(dst, p.p, p.bytes, hipMemcpyDeviceToHost, d->stream));
        dst += p.bytes;
    }
    TCP_HIP(d, hipStreamSynchronize(d->stream));
    return TCP_OK;
}

int tcp_load_state(tcp_domain *d, const void *host)
{
    if (!d || !host) return TCP_ERR_ARG;
    const char *src = static_cast<const char *>(host);
    for (auto &p : state_pieces(d)) {
        TCP_HIP(d, hipMemcpyAsync(p.p, src, p.bytes, hipMemcpyHostToDevice, d->stream));
        src += p.bytes;
    }
    TCP_HIP(d, hipStreamSynchronize(d->stream));
    d->initialized = true;
    return TCP_OK;
}

int tcp_synchronize(tcp_domain *d)
{
    if (!d) return TCP_ERR_ARG;
    TCP_HIP(d, hipStreamSynchronize(d->stream));
    return TCP_OK;
}

int tcp_set_profiling(tcp_domain *d, int enabled)
{
    if (!d) return TCP_ERR_ARG;
    d->prof = enabled != 0;
    return TCP_OK;
}

int tcp_set_fusion(tcp_domain *d, int enabled)
{
    if (!d) return TCP_ERR_ARG;
    d->fuse = enabled != 0;
    drop_graphs(d); // captured steps hold the launch sequence
    return TCP_OK;
}

int tcp_set_graphs(tcp_domain *d, int mode)
{
    if (!d) return TCP_ERR_ARG;
    if (mode < 0 || mode > 2) return fail(d, TCP_ERR_ARG, "graph mode must be 0, 1 or 2");
    d->graph_mode = mode;
    return TCP_OK;
}

int tcp_kernel_times(tcp_domain *d, double *ms, int64_t *launches)
{
    if (!d || !ms || !launches) return TCP_ERR_ARG;
    TCP_HIP(d, hipStreamSynchronize(d->stream));
    for (int k = 0; k < TCP_K_COUNT; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    for (auto &r : d->records) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, r.start, r.stop) == hipSuccess) {
            ms[r.kind] += t;
            launches[r.kind] += 1;
        }
        d->pool.push_back(r.start);
        d->pool.push_back(r.stop);
    }
    d->records.clear();
    return TCP_OK;
}

int tcp_algorithmic_bytes(const tcp_domain *d, double *b)
{
    if (!d || !b) return TCP_ERR_ARG;
    const double sb = (double)d->sb, pb = (double)d->pb;
    b[TCP_K_PHASE] = 2.0 * d->P.q_pf * pb + 5.0 * sb; // h in/out, phi^n in, phi^{n+1} out, u in
    b[TCP_K_HYDRO] = (54.0 + 5.0) * sb;                // g in/out, phi^n, T^n in, u out
    // f in/out, u and phi^{n+1} in, T out; FP32/FP16 deviation storage also reads T^n
    b[TCP_K_THERMAL] = d->P.thermal == TCP_THERMAL_LB ? 2.0 * d->P.q_thermal * pb + (d->pb <= 4 ? 6.0 : 5.0) * sb : 0.0;
    {
        // whole step of RK stages: each stage reads theta, a (or u), T and the
        // accumulator, kappa with a conductivity ratio and q with heat sources,
        // and writes the next argument / accumulator (stage 1 reads T once as
        // theta and T); with a conductivity ratio a coefficient pass per step
        // reads phi and u and writes a and kappa (and q with heat sources);
        // without one, q is written once per change of the sources, not per step
        const double gk = d->P.kappa_h != d->P.kappa_l ? 1.0 : 0.0, hq = d->src.n > 0 ? 1.0 : 0.0;
        if (d->P.thermal == TCP_THERMAL_RK2)
            b[TCP_K_RK] = (11.0 + 2.0 * (gk + hq) + 8.0 * gk + gk * hq) * sb;
        else if (d->P.thermal == TCP_THERMAL_RK4)
            b[TCP_K_RK] = (29.0 + 4.0 * (gk + hq) + 8.0 * gk + gk * hq) * sb;
        else
            b[TCP_K_RK] = 0.0;
    }
    // fused step: all PDFs in/out; phi^n, T^n, u^n in; phi^{n+1}, u^{n+1}, T^{n+1}
    // out (RK schemes: K1 and K2 only, the phase-field and hydrodynamic PDFs,
    // no T^{n+1})
    b[TCP_K_STEP] = d->P.thermal == TCP_THERMAL_LB
                        ? 2.0 * (d->P.q_pf + d->P.q_thermal) * pb + 54.0 * sb + 10.0 * sb
                        : 2.0 * d->P.q_pf * pb + 54.0 * sb + 9.0 * sb;
    // per launch.  LB update: link adjoints in/out, u and phi in, the FP64
    // source adjoint read and written.  RK stage (one pass): lambda', the next
    // stage's field, the four coefficients and acc read, acc and the stage
    // field written, the FP64 source adjoint read and written.
    b[TCP_K_ADJOINT] = d->P.thermal == TCP_THERMAL_LB ? 2.0 * d->P.q_thermal * sb + 4.0 * sb + 16.0 : 9.0 * sb + 16.0;
    // reverse step of the coupled adjoint (its algorithmic minimum: the scratch
    // field between its two launches and their shared sphi fields are not
    // counted; link and field adjoints in the arithmetic type, sb bytes):
    // reads the link adjoints of h, g, f,
    // sphi, sT and lu1, the PDFs h, g, f of step n, phi^n, T^n, u^n, and
    // phi^{n+1}, u^{n+1}; writes the link adjoints, sphi, sT and lu1; the FP64
    // source adjoint is read and written
    if (d->P.thermal == TCP_THERMAL_LB) {
        const double q = d->P.q_thermal + d->P.q_pf;
        b[TCP_K_COUPLED_ADJOINT] = (2.0 * q + 2.0 * 39.0 + 27.0 + 9.0) * sb + q * pb + 16.0;
    } else {
        b[TCP_K_COUPLED_ADJOINT] = 0.0;
    }
    return TCP_OK;
}

int tcp_bandwidth_probe(size_t bytes, int reps, double *gbs)
{
    if (!gbs || bytes < 16 || reps < 1) return fail(nullptr, TCP_ERR_ARG, "bandwidth probe needs bytes >= 16, reps >= 1");
    const int64_t n16 = (int64_t)(bytes / 16);
    return copy_probe((size_t)n16 * 16, reps, gbs,
                      [n16](void *a, void *b) { launch_copy16(a, b, n16, nullptr); });
}

int tcp_pdf_copy_probe(int64_t ncells, int reps, double *gbs)
{
    if (!gbs || ncells < 64 || ncells % 64 != 0 || reps < 1)
        return fail(nullptr, TCP_ERR_ARG, "PDF copy probe needs ncells a positive multiple of 64, reps >= 1");
    return copy_probe((size_t)ncells * 27 * sizeof(float), reps, gbs,
                      [ncells](void *a, void *b) { launch_copy_blocked27(a, b, ncells, nullptr); });
}

const char *tcp_error_string(int code)
{
    switch (code) {
    case TCP_OK: return "ok";
    case TCP_ERR_ARG: return "invalid argument";
    case TCP_ERR_UNSUPPORTED: return "unsupported";
    case TCP_ERR_HIP: return "HIP runtime error";
    case TCP_ERR_OOM: return "out of memory";
    case TCP_ERR_NONFINITE: return "non-finite values";
    case TCP_ERR_STATE: return "call out of order";
    default: return "unknown error";
    }
}

const char *tcp_last_error(const tcp_domain *d)
{
    return d ? d->err.c_str() : g_create_error.c_str();
}

} // extern "C"
