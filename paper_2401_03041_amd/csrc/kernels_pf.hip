// kernels_pf.hip -- K1 as a kernel of its own (used with the RK thermal
// schemes; the LB thermal path runs the fused step of kernels_step.hip).
#include "cell_pf.hpp"

namespace tcp {

// One thread per cell; rows next to a wall take the bounce-back path (a
// wavefront is one x-row, so the choice is uniform across it).
template <int Q, typename P, typename S, typename R>
__global__ void __launch_bounds__(kTX *kTY) k_phase_field(const PfArgs a, const Tiling t)
{
    int x, y, z;
    if (!cell_of_thread(t, a.geo, x, y, z)) return;
    const Nbr nb(a.geo, x, y, z);
    PhiStencil<R> ps;
    if (nb.below || nb.above)
        phase_field_cell<Q, P, S, R, true>(a, nb, ps);
    else
        phase_field_cell<Q, P, S, R, false>(a, nb, ps);
}

template <int Q, typename P, typename S, typename R>
void launch_pf(const PfArgs &a, hipStream_t s)
{
    const Tiling t = make_tiling(a.geo);
    hipLaunchKernelGGL((k_phase_field<Q, P, S, R>), tiling_grid(t), tiling_block(), 0, s, a, t);
}

#define TCP_PF_INST(Q)                                                                                       \
    template void launch_pf<Q, double, double, double>(const PfArgs &, hipStream_t);                        \
    template void launch_pf<Q, float, float, float>(const PfArgs &, hipStream_t);                           \
    template void launch_pf<Q, _Float16, float, float>(const PfArgs &, hipStream_t);
TCP_PF_INST(15)
TCP_PF_INST(27)
#undef TCP_PF_INST

} // namespace tcp
