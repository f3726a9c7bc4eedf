// Sweep kernels for the L1 and L2 inertia norms (Sec. 3, "The lazy PCA": inertia
// q|x_i - w_i|^p; Sec. 5.2 names p = 1 and 2 as alternatives to the indicator).  Same
// thread layout as the indicator kernels; the data factor is not shared between chains
// here because each chain's exponent also holds its own inertia term.
#include "pca_sweep.h"

namespace pcak {
namespace {

template <int G, int NBR, int SUB>
__global__ __launch_bounds__(kBlock, kMinWaves<SUB>) void sweep_kernel_inertia(SweepArgs a)
{
    __shared__ float ptab[kMaxNeighbourStat + 1];
    __shared__ uint4 vtab[kStatEntries];
    const SweepConsts kc = sweep_prologue(a, NBR, ptab, vtab);
    int pix, r, c, grp;
    if (!sweep_thread_site(a, a.Cp / G, pix, r, c, grp)) return;
    sweep_site<G, NBR, SUB, 16, 1, true>(a, ptab, vtab, kc, pix, r, c, grp, 0);
}

template <int G, int NBR>
hipError_t launch_g(const SweepArgs &a0, hipStream_t s)
{
    const SweepLayout lay = sweep_layout(a0.H, a0.W, a0.Cp / G, a0.L > 16);
    SweepArgs a = a0;
    a.patch = lay.patch;
    a.tiles_w = lay.tiles_w;
    for (a.blk0 = 0; a.blk0 < lay.blocks; a.blk0 += kMaxLaunchBlocks) {
        const unsigned grid = (unsigned)std::min<int64_t>(lay.blocks - a.blk0, kMaxLaunchBlocks);
        if (a.L <= 16)
            hipLaunchKernelGGL((sweep_kernel_inertia<G, NBR, 1>), dim3(grid), dim3(kBlock), 0, s, a);
        else
            hipLaunchKernelGGL((sweep_kernel_inertia<G, NBR, 16>), dim3(grid), dim3(kBlock), 0, s, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int G, int TILED>
hipError_t launch_batch_gt(const BatchLaunch &b, int blocks, int nbr, hipStream_t s)
{
    if (nbr == 8)
        hipLaunchKernelGGL((batch_sweep_kernel<G, 1, TILED, 8, true>), dim3(blocks), dim3(kBlock), 0, s, b);
    else
        hipLaunchKernelGGL((batch_sweep_kernel<G, 1, TILED, 4, true>), dim3(blocks), dim3(kBlock), 0, s, b);
    return hipGetLastError();
}

template <int G>
hipError_t launch_batch_g(const BatchLaunch &b, int blocks, int tiled, int nbr, hipStream_t s)
{
    return tiled ? launch_batch_gt<G, 1>(b, blocks, nbr, s) : launch_batch_gt<G, 0>(b, blocks, nbr, s);
}

}  // namespace

hipError_t launch_sweep_inertia(const SweepArgs &a, int G, int nbr, hipStream_t s)
{
    if (a.inertia != 1 && a.inertia != 2) return hipErrorInvalidValue;
    if (nbr == 4) {
        if (G == 4) return launch_g<4, 4>(a, s);
        if (G == 2) return launch_g<2, 4>(a, s);
        return launch_g<1, 4>(a, s);
    }
    if (G == 4) return launch_g<4, 8>(a, s);
    if (G == 2) return launch_g<2, 8>(a, s);
    return launch_g<1, 8>(a, s);
}

hipError_t launch_batch_sweep_inertia(const BatchLaunch &b, int blocks, int G, int tiled, int nbr, hipStream_t s)
{
    if (G == 4) return launch_batch_g<4>(b, blocks, tiled, nbr, s);
    if (G == 2) return launch_batch_g<2>(b, blocks, tiled, nbr, s);
    return launch_batch_g<1>(b, blocks, tiled, nbr, s);
}

}  // namespace pcak
