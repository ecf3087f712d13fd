// kernels_step.hip -- one coupled time step with the thermal LB as a single
// kernel: K1 (phase field), K2 (hydrodynamics) and K3 (thermal LB) of one cell
// run back to back in one thread, in the order of Algorithm 1.  With the RK
// schemes (Algorithm 2) the same kernel runs K1 and K2 only (QF = 0) and the
// RK stages follow it.
//
// This is the same update as the three kernels of their own, arithmetic
// included.  It is legal because, with the time levels used here, no thread
// reads what another thread of the same step writes: K1 and K2 read phi^n, T^n
// and the PDFs of step n, which live in buffers apart from the ones written
// (phi^{n+1}, T^{n+1}, the new PDFs); the velocity is read (u^n by K1) and then
// written (u^{n+1} by K2) only at the thread's own cell; and K3 needs
// phi^{n+1} and u^{n+1} only at its own cell, where this thread has just
// computed them.  Fusing saves the second read of the phi^n stencil (K1 hands
// phi^n at the cell, its gradient and Laplacian to K2), the T^n values the
// thermal pull needs with deviation storage (K2 has them from its stencil),
// the re-reads of u and phi^{n+1} by K3 (field traffic 10 instead of 15 values
// per cell) and two launches per step.
#include "cell_hydro.hpp"
#include "cell_pf.hpp"
#include "cell_thermal.hpp"

namespace tcp {

// A copy of the neighbour offsets that the compiler cannot prove equal to the
// original: otherwise it keeps the 26 neighbour offsets (and the PDF lane
// offsets) the phases have in common live from the first phase to the last.
__device__ __forceinline__ Nbr opaque(const Nbr &nb)
{
    Nbr o = nb;
#pragma unroll
    for (int k = 0; k < 3; ++k) asm volatile("" : "+v"(o.xo[k]));
    return o;
}

template <int QH, int QF, typename P, typename S, typename R, bool WALL>
__device__ __forceinline__ void step_cell(const StepArgs &a, const Nbr &nb, int x, int y, int z,
                                          const Staged<R> *sphi = nullptr, const Staged<R> *sT = nullptr)
{
    PhiStencil<R> ps;
    const R phi_new = phase_field_cell<QH, P, S, R, WALL>(a.pf, opaque(nb), ps, sphi);
    // keep the phases apart: hoisting one phase's loads into the previous one
    // holds both phases' PDFs in registers at once and costs occupancy
    __builtin_amdgcn_sched_barrier(0);
    R u[3];
    // with deviation storage the thermal pull needs T^n at x - e_i: the
    // hydrodynamic update has it from its T^n stencil
    constexpr bool dev = QF > 0 && deviation_storage<P>();
    R tsrc[QF > 0 ? QF : 1];
    hydro_cell<S, R, WALL, true, dev ? QF : 0>(a.hy, opaque(nb), u, ps, tsrc, sT);
    if constexpr (QF > 0) {
        __builtin_amdgcn_sched_barrier(0);
        thermal_cell<QF, P, S, R, WALL, dev>(a.th, opaque(nb), x, y, z, phi_new, u, tsrc);
    } else {
        (void)phi_new;
    }
}

// FP64 needs 174 registers per lane; capping it at 168 lets three wavefronts
// share a SIMD instead of two, at the cost of a few spills (measured 4 % faster).
template <int QH, int QF, typename P, typename S, typename R>
__global__ void __launch_bounds__(kTX *kTY) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 8 ? 3 : 1)))
k_step(const StepArgs a, const Tiling t)
{
    if constexpr (sizeof(R) == 8) {
        // FP64: the work-group first stages phi^n and T^n of its tile, a
        // one-cell halo in x and y and the planes z - 1, z, z + 1 in LDS, so that
        // the 27-point stencils of K1 and K2 read LDS instead of memory
        __shared__ R lphi[3][kHalo], lT[3][kHalo];
        const Geometry &g = a.pf.geo;
        int x0, y0, z;
        if (!tile_of_block(t, g, x0, y0, z)) return;
        const int lx = threadIdx.x, ly = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
        {
            const S *po = static_cast<const S *>(a.pf.phi_old);
            const S *to = static_cast<const S *>(a.hy.T);
            const int tid = lx + kTX * ly;
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                const int zz = wrap(z - 1 + p, g.nz);
                for (int i = tid; i < kHalo; i += kTX * kTY) {
                    uint32_t c;
                    const bool in = halo_cell(g, x0, y0, zz, i, c);
                    lphi[p][i] = in ? ld<R>(elem(po, c)) : R(0);
                    lT[p][i] = in ? ld<R>(elem(to, c)) : R(0);
                }
            }
        }
        __syncthreads();
        const int x = x0 + lx, y = y0 + ly;
        if (x >= g.nx || y >= g.ny) return;
        const Nbr nb(g, x, y, z);
        const int o = (ly + 1) * kHX + lx + 1;
        const Staged<R> sphi{{lphi[0], lphi[1], lphi[2]}, o, nb.below, nb.above};
        const Staged<R> sT{{lT[0], lT[1], lT[2]}, o, nb.below, nb.above};
        if (nb.below || nb.above)
            step_cell<QH, QF, P, S, R, true>(a, nb, x, y, z, &sphi, &sT);
        else
            step_cell<QH, QF, P, S, R, false>(a, nb, x, y, z, &sphi, &sT);
    } else {
        int x, y, z;
        if (!cell_of_thread(t, a.pf.geo, x, y, z)) return;
        const Nbr nb(a.pf.geo, x, y, z);
        if (nb.below || nb.above)
            step_cell<QH, QF, P, S, R, true>(a, nb, x, y, z);
        else
            step_cell<QH, QF, P, S, R, false>(a, nb, x, y, z);
    }
}

template <int QH, int QF, typename P, typename S, typename R>
void launch_step(const StepArgs &a, hipStream_t s)
{
    const Tiling t = make_tiling(a.pf.geo);
    hipLaunchKernelGGL((k_step<QH, QF, P, S, R>), tiling_grid(t), tiling_block(), 0, s, a, t);
}

#define TCP_STEP_INST(QH, QF)                                                                                \
    template void launch_step<QH, QF, double, double, double>(const StepArgs &, hipStream_t);              \
    template void launch_step<QH, QF, float, float, float>(const StepArgs &, hipStream_t);                 \
    template void launch_step<QH, QF, _Float16, float, float>(const StepArgs &, hipStream_t);
TCP_STEP_INST(15, 7)
TCP_STEP_INST(15, 15)
TCP_STEP_INST(15, 19)
TCP_STEP_INST(15, 27)
TCP_STEP_INST(27, 7)
TCP_STEP_INST(27, 15)
TCP_STEP_INST(27, 19)
TCP_STEP_INST(27, 27)
TCP_STEP_INST(15, 0)
TCP_STEP_INST(27, 0)
#undef TCP_STEP_INST

} // namespace tcp
