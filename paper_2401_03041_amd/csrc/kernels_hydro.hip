// kernels_hydro.hip -- K2 as a kernel of its own (used with the RK thermal
// schemes; the LB thermal path runs the fused step of kernels_step.hip).
#include "cell_hydro.hpp"

namespace tcp {

// One thread per cell; rows next to a wall take the bounce-back and ghost paths
// (a wavefront is one x-row, so the choice is uniform across it).
template <typename S, typename R>
__global__ void __launch_bounds__(kTX *kTY) k_hydro(const HydroArgs a, const Tiling t)
{
    int x, y, z;
    if (!cell_of_thread(t, a.geo, x, y, z)) return;
    const Nbr nb(a.geo, x, y, z);
    R u[3];
    if (nb.below || nb.above)
        hydro_cell<S, R, true>(a, nb, u);
    else
        hydro_cell<S, R, false>(a, nb, u);
}

template <typename S, typename R>
void launch_hydro(const HydroArgs &a, hipStream_t s)
{
    const Tiling t = make_tiling(a.geo);
    hipLaunchKernelGGL((k_hydro<S, R>), tiling_grid(t), tiling_block(), 0, s, a, t);
}

template void launch_hydro<double, double>(const HydroArgs &, hipStream_t);
template void launch_hydro<float, float>(const HydroArgs &, hipStream_t);

} // namespace tcp
