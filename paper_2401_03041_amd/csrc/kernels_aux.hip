// kernels_aux.hip -- set-up, read-back and FP64 diagnostics.
//
//  - droplets: phi = max_k 1/2 + 1/2 tanh(2 (r_k - d_k)/xi), the tanh interface
//    of Sec. 3.1, minimum-image distances along periodic axes (FP64).
//  - init: every PDF at the equilibrium of the current fields with p* = 0.
//  - read: storage -> FP64 (or FP32) fields, p = p* rho(phi) c_s^2 with
//    p* = sum_i g_i.
//  - reduce: FP64 sums of phi and phi x in a fixed order (deterministic).
#include "kernels.hpp"
#include "kernels_io.hpp"

namespace tcp {

namespace {

constexpr int kThreads = 256;

template <typename S>
__global__ void __launch_bounds__(kThreads) k_droplets(const Geometry g, const Droplets d, S *phi)
{
    const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (c >= g.N) return;
    const int x = (int)(c % g.nx);
    const int y = (int)((c / g.nx) % g.ny);
    const int z = (int)(c / g.plane);
    const double L[3] = {(double)g.nx, (double)g.ny, (double)g.nz};
    const double p[3] = {(double)x, (double)y, (double)z};
    double best = 0.0;
    for (int k = 0; k < d.n; ++k) {
        double r2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            double dd = p[a] - d.xyzr[4 * k + a];
            if (d.periodic[a]) {
                dd = fmod(dd, L[a]);
                if (dd > 0.5 * L[a]) dd -= L[a];
                if (dd < -0.5 * L[a]) dd += L[a];
            }
            r2 += dd * dd;
        }
        const double v = 0.5 + 0.5 * tanh(2.0 * (d.xyzr[4 * k + 3] - sqrt(r2)) * d.inv_xi);
        best = (k == 0 || v > best) ? v : best;
    }
    phi[c] = static_cast<S>(best);
}

template <typename S>
__global__ void __launch_bounds__(kThreads) k_from_f64(const double *src, S *dst, int64_t n)
{
    const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (c < n) dst[c] = static_cast<S>(src[c]);
}

template <typename S>
__global__ void __launch_bounds__(kThreads) k_from_f32(const float *src, S *dst, int64_t n)
{
    const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (c < n) dst[c] = static_cast<S>(src[c]);
}

// equilibria with runtime stencil choice (set-up only), stored in type P as
// f_eq - w shift, or as the deviation f_eq - w psi (deviation_storage)
template <int Q, typename P>
__device__ void store_scalar_eq(P *dst, const Geometry &g, int x, int y, int z, double psi, double shift,
                                const double u[3])
{
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        const double eu = vel<Q>(i, 0) * u[0] + vel<Q>(i, 1) * u[1] + vel<Q>(i, 2) * u[2];
        const double w = weight<Q>(i);
        const double zeta = 3.0 * eu + 4.5 * eu * eu - 1.5 * uu;
        dst[pdf_index<Q>(g, x, y, z, i)] =
            static_cast<P>(deviation_storage<P>() ? psi * w * zeta : psi * w * (1.0 + zeta) - w * shift);
    }
}

// S: hydrodynamic PDFs and fields; P: phase-field and thermal PDFs
template <typename S, typename P>
__global__ void __launch_bounds__(kThreads) k_init(const InitArgs a)
{
    const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const Geometry &G = a.geo;
    if (c >= G.N) return;
    const int x = (int)(c % G.nx), y = (int)((c / G.nx) % G.ny), z = (int)(c / G.plane);
    const double phi = static_cast<double>(static_cast<const S *>(a.phi)[c]);
    const double T = static_cast<double>(static_cast<const S *>(a.T)[c]);
    double u[3];
    for (int k = 0; k < 3; ++k) u[k] = static_cast<double>(static_cast<const S *>(a.u[k])[c]);
    P *h = static_cast<P *>(a.h), *f = static_cast<P *>(a.f);
    S *g = static_cast<S *>(a.g);
    if (a.q_pf == 15) store_scalar_eq<15>(h, G, x, y, z, phi, 0.0, u);
    else store_scalar_eq<27>(h, G, x, y, z, phi, 0.0, u);
    // incompressible g_eq with p* = 0
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < 27; ++i) {
        const double eu = vel27(i, 0) * u[0] + vel27(i, 1) * u[1] + vel27(i, 2) * u[2];
        g[pdf_index<27>(G, x, y, z, i)] = static_cast<S>(weight<27>(i) * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu));
    }
    if (f) {
        switch (a.q_th) {
        case 7: store_scalar_eq<7>(f, G, x, y, z, T, a.t_shift, u); break;
        case 15: store_scalar_eq<15>(f, G, x, y, z, T, a.t_shift, u); break;
        case 19: store_scalar_eq<19>(f, G, x, y, z, T, a.t_shift, u); break;
        default: store_scalar_eq<27>(f, G, x, y, z, T, a.t_shift, u); break;
        }
    }
    static_cast<S *>(a.phi_other)[c] = static_cast<S>(phi);
}

template <typename S, typename O>
__global__ void __launch_bounds__(kThreads) k_read(const ReadArgs a, O *out)
{
    const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const Geometry &G = a.geo;
    if (c >= G.N) return;
    double v = 0.0;
    if (a.which == 0) v = static_cast<const S *>(a.phi)[c];
    else if (a.which >= 1 && a.which <= 3) v = static_cast<const S *>(a.u[a.which - 1])[c];
    else if (a.which == 4) v = static_cast<const S *>(a.T)[c];
    else {
        double ps = 0.0;
        if (a.which == 5 || a.which == 6) {
            const int x = (int)(c % G.nx), y = (int)((c / G.nx) % G.ny), z = (int)(c / G.plane);
            for (int i = 0; i < 27; ++i)
                ps += static_cast<double>(static_cast<const S *>(a.g)[pdf_index<27>(G, x, y, z, i)]);
        }
        const double phi = static_cast<const S *>(a.phi)[c];
        const double phic = phi < 0.0 ? 0.0 : (phi > 1.0 ? 1.0 : phi);
        const double rho = a.rho_l + phic * a.drho;
        v = a.which == 5 ? ps * rho / 3.0 : (a.which == 6 ? ps : rho);
    }
    out[c] = static_cast<O>(v);
}

// blocked PDF layout -> component-major FP64 out[i*N + c]
template <int Q, typename P, typename F>
__global__ void __launch_bounds__(kThreads) k_read_pdfs(const P *src, const Geometry g, double shift, const F *field,
                                                        double *out)
{
    const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (c >= g.N) return;
    const int x = (int)(c % g.nx), y = (int)((c / g.nx) % g.ny), z = (int)(c / g.plane);
    const double sh = shift + (field ? static_cast<double>(field[c]) : 0.0);
    for (int i = 0; i < Q; ++i)
        out[i * g.N + c] = static_cast<double>(src[pdf_index<Q>(g, x, y, z, i)]) + weight<Q>(i) * sh;
}

// Sum over the 64 lanes of a wavefront: a butterfly of cross-lane exchanges,
// after which every lane holds the total (the same order on every call).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

constexpr int kWaves = kThreads / 64;

// the four sums of the wavefronts of this work-group, added in LDS, to out[0..3]
__device__ __forceinline__ void block_sum4(double (&acc)[4], double *out)
{
    __shared__ double sh[kWaves][4];
    const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = wave_sum(acc[k]);
    if (lane == 0)
        for (int k = 0; k < 4; ++k) sh[wv][k] = acc[k];
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = 0.0;
        for (int w = 0; w < kWaves; ++w) t += sh[w][threadIdx.x];
        out[threadIdx.x] = t;
    }
}

// Sums of phi, phi x, phi y, phi z.  Each wavefront takes whole x-rows (rows
// dealt round-robin over the wavefronts of the grid), so y and z are uniform
// across it and no cell needs a division: per row the lanes add phi and
// phi x, and the row total is weighted by y and z once.
template <typename S>
__global__ void __launch_bounds__(kThreads) k_reduce_partial(const Geometry g, const S *phi, double *partial)
{
    const int lane = threadIdx.x % 64;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
    const int rows = g.ny * g.nz;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int r = (int)blockIdx.x * kWaves + wv; r < rows; r += (int)gridDim.x * kWaves) {
        const S *row = phi + (int64_t)r * g.nx;
        double rm = 0.0, rx = 0.0;
        for (int x = lane; x < g.nx; x += 64) {
            const double p = static_cast<double>(row[x]);
            rm += p;
            rx += p * x;
        }
        acc[0] += rm;
        acc[1] += rx;
        acc[2] += rm * (r % g.ny);
        acc[3] += rm * (r / g.ny);
    }
    block_sum4(acc, partial + 4 * blockIdx.x);
}

__global__ void __launch_bounds__(kThreads) k_reduce_final(const double *partial, int nblocks, double *out4)
{
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += kThreads)
        for (int k = 0; k < 4; ++k) acc[k] += partial[4 * b + k];
    block_sum4(acc, out4);
}

// max |a - b| over the grid; a NaN anywhere makes the result NaN
__device__ __forceinline__ double max_nan(double m, double v) { return (v > m || v != v) ? v : m; }

template <typename S>
__global__ void __launch_bounds__(kThreads) k_maxdiff_partial(int64_t n, const S *a, const S *b, double *partial)
{
    __shared__ double sh[kThreads];
    double m = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x; c < n; c += (int64_t)gridDim.x * kThreads)
        m = max_nan(m, fabs(static_cast<double>(a[c]) - static_cast<double>(b[c])));
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = max_nan(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(kThreads) k_max_final(const double *partial, int nblocks, double *out)
{
    __shared__ double sh[kThreads];
    double m = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kThreads) m = max_nan(m, partial[b]);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = max_nan(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// One 16-byte word per thread with non-temporal hints: the fastest plain copy
// measured on MI355X (6.3-6.6 TB/s for 4 GiB; a grid-stride loop reaches 4.9).
typedef float f32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(kThreads) k_copy16(const f32x4 *__restrict__ src, f32x4 *__restrict__ dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

} // namespace

template <typename S>
void launch_droplets(const Geometry &g, const Droplets &d, void *phi, hipStream_t s)
{
    hipLaunchKernelGGL((k_droplets<S>), dim3(blocks_for(g.N)), dim3(kThreads), 0, s, g, d, static_cast<S *>(phi));
}

template <typename S>
void launch_from_f64(const double *src, void *dst, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL((k_from_f64<S>), dim3(blocks_for(n)), dim3(kThreads), 0, s, src, static_cast<S *>(dst), n);
}

template <typename S>
void launch_from_f32(const float *src, void *dst, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL((k_from_f32<S>), dim3(blocks_for(n)), dim3(kThreads), 0, s, src, static_cast<S *>(dst), n);
}

template <typename S, typename P>
void launch_init(const InitArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL((k_init<S, P>), dim3(blocks_for(a.geo.N)), dim3(kThreads), 0, s, a);
}

template <typename S>
void launch_read(const ReadArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL((k_read<S, double>), dim3(blocks_for(a.geo.N)), dim3(kThreads), 0, s, a, a.out);
}

template <typename S>
void launch_read_f32(const ReadArgs &a, float *out, hipStream_t s)
{
    hipLaunchKernelGGL((k_read<S, float>), dim3(blocks_for(a.geo.N)), dim3(kThreads), 0, s, a, out);
}

template <typename P, typename F>
void launch_read_pdfs(const void *src, int q, const Geometry &g, double shift, const void *field, double *out,
                      hipStream_t s)
{
    const P *p = static_cast<const P *>(src);
    const F *fl = static_cast<const F *>(field);
    const dim3 gr(blocks_for(g.N)), bl(kThreads);
    switch (q) {
    case 7: hipLaunchKernelGGL((k_read_pdfs<7, P, F>), gr, bl, 0, s, p, g, shift, fl, out); break;
    case 15: hipLaunchKernelGGL((k_read_pdfs<15, P, F>), gr, bl, 0, s, p, g, shift, fl, out); break;
    case 19: hipLaunchKernelGGL((k_read_pdfs<19, P, F>), gr, bl, 0, s, p, g, shift, fl, out); break;
    default: hipLaunchKernelGGL((k_read_pdfs<27, P, F>), gr, bl, 0, s, p, g, shift, fl, out); break;
    }
}

template <typename S>
void launch_reduce(const Geometry &g, const void *phi, double *partial, double *out4, hipStream_t s)
{
    hipLaunchKernelGGL((k_reduce_partial<S>), dim3(kReduceBlocks), dim3(kThreads), 0, s, g,
                       static_cast<const S *>(phi), partial);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kThreads), 0, s, partial, kReduceBlocks, out4);
}

template <typename S>
void launch_maxdiff(int64_t n, const void *a, const void *b, double *partial, double *out, hipStream_t s)
{
    hipLaunchKernelGGL((k_maxdiff_partial<S>), dim3(kReduceBlocks), dim3(kThreads), 0, s, n,
                       static_cast<const S *>(a), static_cast<const S *>(b), partial);
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(kThreads), 0, s, partial, kReduceBlocks, out);
}

// Copy of a Q-component FP32 field in the blocked PDF layout (runs of 64 cells
// per component): one thread per cell loads its Q values, 4 bytes per lane
// from Q runs of one block, then stores them with the non-temporal hint, the
// access pattern of the step kernel's PDF pull and store without the
// neighbour offsets.
template <int Q>
__global__ void __launch_bounds__(kThreads) k_copy_blocked(const float *__restrict__ src, float *__restrict__ dst,
                                                            int64_t ncells)
{
    const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (c >= ncells) return;
    const int64_t base = (c >> 6) * (64 * Q) + (c & 63);
    float v[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] = src[base + 64 * i];
#pragma unroll
    for (int i = 0; i < Q; ++i) __builtin_nontemporal_store(v[i], dst + base + 64 * i);
}

void launch_copy_blocked27(const void *src, void *dst, int64_t ncells, hipStream_t s)
{
    hipLaunchKernelGGL((k_copy_blocked<27>), dim3(blocks_for(ncells)), dim3(kThreads), 0, s,
                       static_cast<const float *>(src), static_cast<float *>(dst), ncells);
}

void launch_copy16(const void *src, void *dst, int64_t n16, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy16, dim3(blocks_for(n16)), dim3(kThreads), 0, s, static_cast<const f32x4 *>(src),
                       static_cast<f32x4 *>(dst), n16);
}

#define TCP_AUX_INST(S)                                                                                      \
    template void launch_droplets<S>(const Geometry &, const Droplets &, void *, hipStream_t);              \
    template void launch_from_f64<S>(const double *, void *, int64_t, hipStream_t);                         \
    template void launch_from_f32<S>(const float *, void *, int64_t, hipStream_t);                          \
    template void launch_init<S, S>(const InitArgs &, hipStream_t);                                         \
    template void launch_read<S>(const ReadArgs &, hipStream_t);                                            \
    template void launch_read_f32<S>(const ReadArgs &, float *, hipStream_t);                               \
    template void launch_read_pdfs<S, S>(const void *, int, const Geometry &, double, const void *, double *, hipStream_t); \
    template void launch_reduce<S>(const Geometry &, const void *, double *, double *, hipStream_t);          \
    template void launch_maxdiff<S>(int64_t, const void *, const void *, double *, double *, hipStream_t);
TCP_AUX_INST(double)
TCP_AUX_INST(float)
#undef TCP_AUX_INST
template void launch_init<float, _Float16>(const InitArgs &, hipStream_t);
template void launch_read_pdfs<_Float16, float>(const void *, int, const Geometry &, double, const void *, double *,
                                                hipStream_t);

} // namespace tcp
