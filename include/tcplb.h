/*
 * tcplb.h -- C interface of the MI355X (gfx950) thermocapillary phase-field
 * lattice Boltzmann library.
 *
 * One domain advances the coupled sweep of Holzer et al. (arXiv 2401.03041):
 * per time step the conservative Allen-Cahn phase-field LB (D3Q15 or D3Q27,
 * Sec. 2.2 Eq. lb_interface), the velocity-based D3Q27 central-moment
 * hydrodynamic LB with surface tension, temperature-dependent Marangoni,
 * pressure and viscous correction forces (Sec. 2.1-2.2), and the thermal
 * field as a D3Q7/15/19/27 passive-scalar LB (Eq. lb_thermal) or an RK2/RK4
 * finite-difference energy update (Eq. rk2, Eq. rk4), in the order of
 * Algorithm 1 (LB) or Algorithm 2 (RK).
 *
 * Conventions shared by every call
 *  - Lattice units: dx = dt = 1, c_s^2 = 1/3.
 *  - Cell (x, y, z), 0 <= x < nx etc., has linear index x + nx*(y + ny*z);
 *    host arrays are FP64 in that order.  Device arrays given to or taken
 *    from the library are FP64 in the same order.
 *  - The domain is periodic in x and z.  In y it is periodic, or bounded by
 *    no-slip walls at y = -1/2 and y = ny - 1/2 (halfway bounce-back).  At a
 *    wall the phase field meets the contact angle theta of that wall: the
 *    stencils see phi_adj + cos(theta) (4/xi) phi_adj (1 - phi_adj) beyond it
 *    (n_w . grad phi = -cos(theta) |grad phi| for the tanh interface).
 *  - Every call returns an int: TCP_OK (0) or a negative TCP_ERR_* code; no
 *    C++ exception crosses this interface.  tcp_last_error() gives text.
 *  - Work is enqueued on the HIP stream given at creation; calls that return
 *    host data synchronise that stream, all other calls are asynchronous.
 *  - A domain is not thread-safe: calls on one domain must not overlap.
 */
#ifndef TCPLB_H
#define TCPLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    TCP_OK = 0,
    TCP_ERR_ARG = -1,         /* invalid argument or parameter value */
    TCP_ERR_UNSUPPORTED = -2, /* valid request the library does not implement */
    TCP_ERR_HIP = -3,         /* a HIP runtime call or kernel launch failed */
    TCP_ERR_OOM = -4,         /* device allocation failed */
    TCP_ERR_NONFINITE = -5,   /* a reduction met NaN or Inf in the phase field */
    TCP_ERR_STATE = -6        /* call out of order (e.g. step before initialize) */
};

/* field selectors for tcp_set_field / tcp_get_field */
enum {
    TCP_PHI = 0,   /* phase indicator phi (0 light, 1 heavy)               set/get */
    TCP_UX = 1,    /* velocity components                                 set/get */
    TCP_UY = 2,
    TCP_UZ = 3,
    TCP_T = 4,     /* temperature                                          set/get */
    TCP_P = 5,     /* pressure p = p* rho c_s^2 (Sec. 2.2)                 get */
    TCP_PSTAR = 6, /* normalised pressure p* = sum_i g_i (Sec. 2.2)        get */
    TCP_RHO = 7    /* density rho(phi) (Sec. 2.2)                          get */
};

/* PDF selectors for tcp_get_pdfs */
enum { TCP_PDF_H = 0, TCP_PDF_G = 1, TCP_PDF_F = 2 };

enum { TCP_THERMAL_LB = 0, TCP_THERMAL_RK2 = 1, TCP_THERMAL_RK4 = 2 };
/* Storage and arithmetic precision (tcp_params.precision):
 *  TCP_FP64  all PDFs and fields FP64, FP64 arithmetic;
 *  TCP_FP32  all PDFs and fields FP32, FP32 arithmetic;
 *  TCP_FP16  phase-field and thermal PDFs FP16, hydrodynamic PDFs and all
 *            fields FP32, FP32 arithmetic.
 * In FP32 and FP16 each phase-field and thermal PDF holds its deviation from
 * the rest equilibrium of its own cell, h_i - w_i phi and f_i - w_i T
 * (t_shift is used in FP64 only).
 * Reductions and read-back are FP64 in every mode. */
enum { TCP_FP64 = 0, TCP_FP32 = 1, TCP_FP16 = 2 };

/* Kernel kinds reported by tcp_kernel_times and tcp_algorithmic_bytes:
 * the phase-field, hydrodynamic and thermal LB kernels, an RK stage, the
 * fused step (all three LB updates of a step in one kernel, or the phase-field
 * and hydrodynamic updates with the RK schemes, see tcp_set_fusion), one update of the thermal adjoint (tcp_thermal_adjoint)
 * and one reverse step of the coupled adjoint (tcp_tape_adjoint: its two
 * kernels together). */
enum {
    TCP_K_PHASE = 0,
    TCP_K_HYDRO = 1,
    TCP_K_THERMAL = 2,
    TCP_K_RK = 3,
    TCP_K_STEP = 4,
    TCP_K_ADJOINT = 5,
    TCP_K_COUPLED_ADJOINT = 6,
    TCP_K_COUNT = 7
};

typedef struct tcp_domain tcp_domain;

/* Device memory provider.  alloc returns a device pointer of at least `bytes`
 * bytes (256-byte aligned) or NULL; free releases it.  ctx is passed through. */
typedef struct {
    void *(*alloc)(size_t bytes, void *ctx);
    void (*free)(void *ptr, void *ctx);
    void *ctx;
} tcp_allocator;

/* Laser heat source q_T (Eq. HeatSource): Q exp(-2 d^2 / w^2) where
 * d is the distance to (x, y, z); zero where d > d_cut, no cut-off if
 * d_cut <= 0.  Coordinates are cell-centre units (cell i sits at i). */
typedef struct {
    double Q, x, y, z, w, d_cut;
} tcp_heat_source;

/* Spherical droplet for tcp_set_droplets: centre (x, y, z), radius r. */
typedef struct {
    double x, y, z, r;
} tcp_droplet;

/* Physical and numerical parameters (Sec. 2.1-2.3, Sec. 3.1). */
typedef struct {
    int32_t nx, ny, nz;
    int32_t walls_y;        /* 0: periodic in y; 1: no-slip walls at y = -1/2, ny - 1/2 */
    int32_t q_pf;           /* phase-field stencil: 15 or 27 */
    int32_t q_thermal;      /* thermal LB stencil: 7, 15, 19 or 27 */
    int32_t thermal;        /* TCP_THERMAL_LB, _RK2 or _RK4 */
    int32_t precision;      /* TCP_FP64, TCP_FP32 or TCP_FP16 (see above) */
    double rho_h, rho_l;    /* densities of the heavy (phi = 1) and light phase */
    double nu_h, nu_l;      /* kinematic viscosities (lattice units) */
    double mobility;        /* interface mobility M */
    double xi;              /* interface width */
    double sigma_ref;       /* surface tension at t_ref */
    double sigma_t;         /* d sigma / d T */
    double t_ref;           /* reference temperature of sigma(T) */
    double kappa_h, kappa_l;/* thermal diffusivities (rho c_p = 1) */
    double g[3];            /* gravitational acceleration */
    double omega_bulk;      /* relaxation rate of the trace of the second moments */
    double normal_eps;      /* n = grad phi / sqrt(|grad phi|^2 + normal_eps^2) */
    double u_wall_bot[3];   /* wall velocities (walls_y = 1) */
    double u_wall_top[3];
    double t_wall_bot;      /* uniform wall temperatures; tcp_set_wall_temperature */
    double t_wall_top;      /*   overrides them with per-column values */
    double t_shift;         /* FP64: thermal PDFs are stored as f_i - w_i t_shift */
    double contact_angle_bot; /* wetting of the walls (walls_y = 1): contact angle in degrees,  */
    double contact_angle_top; /*   measured through the heavy phase, in (0, 180); 90 = neutral */
} tcp_params;

/* Passage: Sec. 2.1-2.3 (model parameters), Sec. 3.1 (channel parameters).
 * Fill *p with defaults: 32^3 periodic, D3Q15 phase field, D3Q7 thermal LB,
 * FP64, unit densities, nu = 1/6, M = 0.05, xi = 5, no surface tension,
 * kappa = 0.2, omega_bulk = 1, normal_eps = 1e-6, t_shift = 0, contact angles
 * 90 degrees. */
int tcp_params_default(tcp_params *p);

/* Passage: Sec. 2.2 (relaxation rates of Eq. pflbm-tau and the viscosity
 * law), Sec. 2.3 (Eq. thlbm-tau; the RK schemes of Eq. rk2 / rk4), Sec. 4.1
 * (the PDF and field arrays that a step updates).
 * Validate *p and allocate a domain.  Rejects (TCP_ERR_ARG) any relaxation
 * rate outside (0, 2), and for RK thermal updates kappa_max above the
 * real-axis stability bound of the isotropic Laplacian (2/5.78 for RK2,
 * 2.785/5.78 for RK4).  alloc: NULL uses hipMalloc/hipFree.  stream: a
 * hipStream_t (NULL: the default stream).  On success *out owns all device
 * state; release it with tcp_destroy. */
int tcp_create(const tcp_params *p, const tcp_allocator *alloc, void *stream, tcp_domain **out);
/* Passage: none (releases what tcp_create allocated).  Synchronises the
 * domain's stream, frees every device buffer and the domain itself. */
int tcp_destroy(tcp_domain *d);

/* Passage: Sec. 4.1 (phase field, velocity and temperature are the fields
 * initialised before the first step).
 * Copy one macroscopic field into the domain.  Exactly one of host (FP64
 * host array) or dev (FP64 device array) is non-NULL; both hold nx*ny*nz
 * values.  The library keeps no reference to the caller's array. */
int tcp_set_field(tcp_domain *d, int which, const double *host, const void *dev);
/* Passage: Sec. 4.1 (fields initialised before the first step), as for
 * tcp_set_field, from FP32.
 * Copy one field (TCP_PHI, TCP_UX..TCP_UZ, TCP_T) from dev, an FP32 device
 * array of nx*ny*nz values in x-fastest order, into the domain, asynchronously
 * on the domain's stream; each value is converted to the storage type (exact
 * in FP64 and FP32 storage).  The caller keeps ownership of dev and must keep
 * it alive until the stream reaches the copy.  TCP_ERR_ARG for a NULL dev or a
 * field that cannot be set. */
int tcp_set_field_f32(tcp_domain *d, int which, const float *dev);

/* Passage: Sec. 3.1 (tanh interface profile), Sec. 3.2-3.3 (droplet set-ups).
 * phi := max over droplets of 1/2 + 1/2 tanh(2 (r_k - dist_k) / xi)
 * (the tanh interface of Sec. 3.1), with minimum-image distances along the
 * periodic axes.  n = 0 sets phi = 0. */
int tcp_set_droplets(tcp_domain *d, const tcp_droplet *drops, int n);

/* Passage: Eq. HeatSource (Sec. 3.2).
 * Heat sources of Eq. HeatSource (at most 16); replaces any previous set. */
int tcp_set_heat_sources(tcp_domain *d, const tcp_heat_source *src, int n);

/* Passage: Sec. 3.1 and Sec. 3.2 (Dirichlet temperature walls).
 * Per-column wall temperature (walls_y = 1): wall 0 = bottom, 1 = top;
 * Tw holds nx*nz FP64 host values, index x + nx*z. */
int tcp_set_wall_temperature(tcp_domain *d, int wall, const double *Tw);

/* Passage: Sec. 4.1 (initialisation of the three PDF fields); the equilibria
 * of Sec. 2.2 (h, g) and Eq. lb_thermal (f).
 * Set all PDFs to the equilibria of the current phi, u, T with p* = 0
 * (Sec. 4.1 initialisation).  Must precede tcp_step. */
int tcp_initialize(tcp_domain *d);

/* Passage: Algorithm 1 (thermal LB) and Algorithm 2 (RK): per step the
 * phase-field update (Eq. lb_interface), the hydrodynamic update (Sec. 2.2)
 * and the thermal update (Eq. lb_thermal, or Eq. rk2 / rk4), each with its
 * boundary conditions (Sec. 4.1).
 * Advance nsteps coupled time steps (asynchronous). */
int tcp_step(tcp_domain *d, int64_t nsteps);

/* Passage: Sec. 4.1 (temperature initialised by running the thermal solver).
 * Temperature initialisation by running the thermal solver on its own
 * (Sec. 4.1: phi and u are set statically, T by iterating the thermal
 * update until it settles).  Runs thermal updates (the LB of Eq. lb_thermal
 * or the RK stages of Eq. rk2 / rk4, heat sources and wall temperatures
 * included) with phi, u and the phase-field and hydrodynamic PDFs held,
 * until the largest per-cell change of T over one update, measured after
 * every check_every updates and after the last, is at most tol, or
 * max_steps updates have run (tol = 0 runs exactly max_steps).  On return
 * *steps_done holds the number of updates and *change the last measured
 * change (0 if none ran); either pointer may be NULL.  Must follow
 * tcp_initialize.  Synchronises at each check.  TCP_ERR_ARG for
 * max_steps < 0, check_every < 1 or tol negative or not finite;
 * TCP_ERR_NONFINITE if T becomes NaN or Inf. */
int tcp_warm_temperature(tcp_domain *d, int64_t max_steps, double tol, int64_t check_every,
                         int64_t *steps_done, double *change);

/* Passage: Eq. lb_thermal, Eq. rk2 / rk4 and Eq. HeatSource (the map that is
 * reversed); Sec. 3.3 (heater placement is the design question it serves).
 * Adjoint of the temperature warm-up.  With phi and u held at their current
 * values, nsteps thermal updates (the LB of Eq. lb_thermal with the
 * anti-bounce-back walls, or the RK2 / RK4 stages of Eq. rk2 / rk4 with the
 * wall ghosts; the source of Eq. HeatSource) form an affine map from the
 * heat-source amplitudes Q_k and the wall temperatures to T.  For
 * the loss L = sum_x dL_dT[x] T(x) of the T reached after nsteps updates of
 * tcp_warm_temperature, this returns for every heat source, in the order of
 * tcp_set_heat_sources, four values dL/dQ_k, dL/dx_k, dL/dy_k, dL/dz_k
 * (dL_dsource, 4*n values; the cut-off sphere moves with the source), and
 * dL/dT_w of every column of the bottom and top walls (dL_dTw_bot,
 * dL_dTw_top: nx*nz values, x fastest).
 * The gradients do not depend on the current T or PDFs, which are left
 * untouched.  dL_dT: host array of nx*ny*nz values (cell order x fastest);
 * the three outputs are host arrays or NULL to skip.  One adjoint kernel per
 * LB update or RK stage, last to first, in the storage precision of the
 * domain with FP64 accumulation of the gradients; the workspace (LB: two
 * link-adjoint arrays of the thermal PDF size; RK: eight fields; and two FP64
 * fields) is allocated on the first call and kept.  Synchronises. */
int tcp_thermal_adjoint(tcp_domain *d, int64_t nsteps, const double *dL_dT, double *dL_dsource,
                        double *dL_dTw_bot, double *dL_dTw_top);

/* Passage: Algorithm 1 (the steps that are taped); Sec. 3.3 (heater design
 * by the droplet's capture, which the gradients of tcp_tape_adjoint serve).
 * Advance nsteps coupled steps (the fused step kernel, bitwise the steps
 * tcp_step takes with fusion on) and keep what their adjoint needs: the
 * state (all PDFs, phi, T, u) at the start of every segment of `segment`
 * steps and at the end (segment <= 0: ceil(sqrt(nsteps))), the inner states
 * of the last segment, and the heat sources and wall temperatures in force.
 * The reverse sweep recomputes the inner states of every other segment from
 * its checkpoint; segment = 1 stores every state and recomputes nothing.
 * Replaces any earlier tape; the device memory (nseg + 1 checkpoints and two
 * rings of segment - 1 states of the domain's state size, so that the reverse
 * sweep can recompute one segment on a second stream while it undoes the
 * next, plus the reverse sweep's workspace, about 2.3 states; one ring, and
 * no overlap, when two do not fit) is allocated through the domain's
 * allocator on the first call and again when the sizes change (TCP_ERR_OOM
 * if not even one ring fits).  Thermal LB only
 * (TCP_ERR_UNSUPPORTED for RK).  Asynchronous.  TCP_ERR_ARG for nsteps < 1,
 * TCP_ERR_STATE before tcp_initialize. */
int tcp_step_taped(tcp_domain *d, int64_t nsteps, int64_t segment);

/* Passage: Algorithm 1 and the updates it runs (Eq. lb_interface, Sec. 2.2,
 * Eq. lb_thermal, Eq. HeatSource), reversed; Sec. 3.3 (the droplet centroid
 * as the outcome of a capture set-up).
 * Adjoint of the taped run.  The loss depends on the final phase field phi^N
 * through its centroid c = sum phi x / sum phi (integer cell coordinates, as
 * tcp_reduce) and, optionally, directly: dL/dphi^N(x) =
 * dL_dcentroid . (x - c) / sum phi + dL_dphi[x] (dL_dphi: host FP64 array of
 * nx*ny*nz values, or NULL).  Returns, as tcp_thermal_adjoint does, dL/dQ_k,
 * dL/dx_k, dL/dy_k, dL/dz_k for every taped heat source (dL_dsource, 4 per
 * source) and dL/dT_w of every column of the bottom and top walls (nx*nz
 * values each, x fastest); each output may be NULL.  Segments are undone
 * last to first, each recomputed from its checkpoint unless its states are
 * at hand (with two rings, on a second stream of default priority while the
 * previous segment is undone), then step by step with two reverse kernels
 * per step (the thermal and hydrodynamic updates, then the phase-field
 * update; for each, the recompute of the cell's update and its
 * vector-Jacobian product, with link and stencil adjoints gathered from the
 * neighbours); arithmetic in the
 * domain's precision (FP32 for FP16 PDFs), gradient sums in FP64.  The
 * recomputation uses the heat sources and wall temperatures of the taped
 * run, even if tcp_set_heat_sources or tcp_set_wall_temperature changed the
 * domain's since.  The domain's current state, sources and wall
 * temperatures are not touched.  Synchronises.  TCP_ERR_STATE
 * without a tape; TCP_ERR_ARG for a missing or non-finite dL_dcentroid. */
int tcp_tape_adjoint(tcp_domain *d, const double dL_dcentroid[3], const double *dL_dphi, double *dL_dsource,
                     double *dL_dTw_bot, double *dL_dTw_top);

/* Passage: Sec. 2.2 (phi, u, the normalised pressure p* and p = p* rho c_s^2,
 * rho(phi)), Eq. lb_thermal (T = sum_i f_i).
 * Read back one field as FP64 into host (synchronises) or dev (FP64 device
 * array of nx*ny*nz values, asynchronous); exactly one is non-NULL. */
int tcp_get_field(tcp_domain *d, int which, double *host, void *dev);
/* Passage: Sec. 2.2 (phi, u, p*, p, rho(phi)), Eq. lb_thermal (T), as for
 * tcp_get_field, into FP32.
 * Read back one field into dev, an FP32 device array of nx*ny*nz values in
 * x-fastest order, asynchronously on the domain's stream.  The value is formed
 * in FP64 exactly as tcp_get_field forms it and rounded once to FP32.  The
 * caller owns dev.  TCP_ERR_ARG for a NULL dev or an unknown field. */
int tcp_get_field_f32(tcp_domain *d, int which, float *dev);

/* For callers that cannot allocate device memory: serving loops and
 * harnesses that forbid hipMalloc.  Same result as tcp_get_field with a host
 * destination, which allocates and frees a device staging buffer on every
 * call; this variant stages through a fixed 32 MiB device array of the
 * library (one per GPU, held until the process ends) and allocates nothing.
 * At most 4194304 cells (TCP_ERR_UNSUPPORTED beyond).  Runs on the device
 * that was current at tcp_create (made current for the call).  Synchronises.
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (from several threads or streams) race. */
int tcp_get_field_noalloc(tcp_domain *d, int which, double *host);

/* Passage: App. B (stencil order), Eq. lb_interface, Sec. 2.2, Eq. lb_thermal.
 * Post-collision PDFs of the current step, unshifted FP64, component-major:
 * out[i*N + cell], i in the stencil order of App. B.  Synchronises. */
int tcp_get_pdfs(tcp_domain *d, int which, double *host_out);

/* Passage: Sec. 3.2 and Sec. 3.3 (droplet centroid trajectories); Sec. 2.2
 * (the conservative phase field: sum phi is the conserved mass).
 * FP64 diagnostics: mass = sum phi and centroid = sum phi x / sum phi with
 * integer cell coordinates.  Synchronises.  TCP_ERR_NONFINITE if phi holds
 * NaN or Inf. */
int tcp_reduce(tcp_domain *d, double *mass, double centroid[3]);

/* Passage: Sec. 4.1 (the state a step carries: three PDF fields, phi, u, T).
 * Raw state (all PDF buffers and fields, storage precision) for checkpoint
 * and restart: tcp_state_bytes gives the size; save/load copy to/from a host
 * buffer of that size.  Loading restores a bitwise identical state. */
int tcp_state_bytes(const tcp_domain *d, size_t *bytes);
int tcp_save_state(tcp_domain *d, void *host);
int tcp_load_state(tcp_domain *d, const void *host);

/* Passage: none (stream synchronisation).
 * Wait for all work enqueued on the domain's stream. */
int tcp_synchronize(tcp_domain *d);

/* Passage: Sec. 4.2 (per-kernel performance of the updates).
 * Per-kernel timing with HIP events on the domain's stream.  While enabled,
 * every launch is bracketed by two events.  tcp_kernel_times synchronises,
 * writes the summed milliseconds and launch counts per TCP_K_* kind (arrays
 * of TCP_K_COUNT entries) and resets the counters. */
int tcp_set_profiling(tcp_domain *d, int enabled);
int tcp_kernel_times(tcp_domain *d, double *ms, int64_t *launches);

/* Passage: Algorithm 1 (the order the fused kernel keeps per cell).
 * Fusion.  With the thermal LB (TCP_THERMAL_LB) a step runs as one kernel in
 * which each thread updates its cell's phase field, hydrodynamics and
 * temperature in turn (no thread reads what another writes within a step, so
 * this is the same update as the three kernels of Algorithm 1, with fewer
 * field reads).  With the RK schemes (Algorithm 2) the phase-field and
 * hydrodynamic updates run as one kernel the same way and the RK stages
 * follow.  enabled = 0 launches the kernels of their own instead (default 1):
 * the same update, up to the compiler rounding single operations differently
 * in the two code paths. */
int tcp_set_fusion(tcp_domain *d, int enabled);

/* Passage: none (launch scheduling of Algorithm 1 / 2 steps).
 * Step graphs.  On small grids a step's few-microsecond kernels are bound by
 * host launch cost; tcp_step then captures 16 steps into one HIP graph (on
 * first use, once per buffer parity) and replays it.  mode 0: never;
 * 1 (default): grids of at most 2^21 cells; 2: always.  Results are bitwise
 * identical to eager launches.  Graphs are not used while profiling is
 * enabled, and are rebuilt after tcp_set_heat_sources. */
int tcp_set_graphs(tcp_domain *d, int mode);

/* Passage: Sec. 4.2 (bytes per cell of the roofline model, 2Q+4 values for
 * the D3Q7 thermal LB).
 * Bytes each kernel kind moves per cell by the algorithmic model (each PDF
 * read and written once, each scalar field read or written once). */
int tcp_algorithmic_bytes(const tcp_domain *d, double *bytes_per_cell);

/* Passage: Sec. 4.2 (memory bandwidth as the bound of the LB updates).
 * Practical HBM ceiling: allocate two device buffers of `bytes` each, copy
 * one into the other `reps` times with a 16-byte-per-lane streaming kernel on
 * the default stream, and return the best copy rate (read + write bytes per
 * second, in GB/s).  Synchronises; frees its buffers before returning. */
int tcp_bandwidth_probe(size_t bytes, int reps, double *gbs);

/* Passage: Sec. 4.2 (memory bandwidth as the bound of the LB updates).
 * Ceiling of the step kernel's own access pattern: copy a 27-component FP32
 * field of ncells cells (a multiple of 64) in the blocked PDF layout (runs of
 * 64 cells per component, one thread per cell, 4 bytes per lane,
 * non-temporal stores) between two device buffers, `reps` times on the
 * default stream, and return the best rate (read + write, GB/s).
 * Synchronises; frees its buffers before returning. */
int tcp_pdf_copy_probe(int64_t ncells, int reps, double *gbs);

/* Passage: none (error reporting).  Text of a TCP_* code. */
const char *tcp_error_string(int code);
/* Passage: none (error reporting).  Message of the last failed call on d, or
 * of the last failed tcp_create / tcp_bandwidth_probe when d is NULL. */
const char *tcp_last_error(const tcp_domain *d);

#ifdef __cplusplus
}
#endif
#endif /* TCPLB_H */
