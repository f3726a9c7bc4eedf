// Batched sweeps: one launch advances every lattice of a batch by one sweep
// (batch_sweep_kernel in pca_sweep.h), plus the device-side sweep counter update.
#include "pca_sweep.h"

namespace pcak {
namespace {

__global__ void advance_kernel(ImageDesc *imgs, int n_imgs, uint32_t n)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n_imgs) return;
    const uint32_t t = imgs[i].t;
    const uint32_t room = imgs[i].t_end > t ? imgs[i].t_end - t : 0u;
    imgs[i].t = t + (n < room ? n : room);
}


template <int G, int SHARE, int TILED>
hipError_t launch_batch_gst(const BatchLaunch &b, int blocks, int nbr, hipStream_t s)
{
    if (nbr == 8)
        hipLaunchKernelGGL((batch_sweep_kernel<G, SHARE, TILED, 8>), dim3(blocks), dim3(kBlock), 0, s, b);
    else
        hipLaunchKernelGGL((batch_sweep_kernel<G, SHARE, TILED, 4>), dim3(blocks), dim3(kBlock), 0, s, b);
    return hipGetLastError();
}

template <int G, int SHARE>
hipError_t launch_batch_gs(const BatchLaunch &b, int blocks, int tiled, int nbr, hipStream_t s)
{
    return tiled ? launch_batch_gst<G, SHARE, 1>(b, blocks, nbr, s) : launch_batch_gst<G, SHARE, 0>(b, blocks, nbr, s);
}

hipError_t launch_batch_part(const BatchLaunch &b, int total_blocks, int G, int share, int tiled, int nbr,
                             hipStream_t s)
{
    if (G == 4) {
        if (share == 4) return launch_batch_gs<4, 4>(b, total_blocks, tiled, nbr, s);
        if (share == 2) return launch_batch_gs<4, 2>(b, total_blocks, tiled, nbr, s);
        return launch_batch_gs<4, 1>(b, total_blocks, tiled, nbr, s);
    }
    if (G == 2) {
        if (share == 2) return launch_batch_gs<2, 2>(b, total_blocks, tiled, nbr, s);
        return launch_batch_gs<2, 1>(b, total_blocks, tiled, nbr, s);
    }
    if (share == 4) return launch_batch_gs<1, 4>(b, total_blocks, tiled, nbr, s);
    if (share == 2) return launch_batch_gs<1, 2>(b, total_blocks, tiled, nbr, s);
    return launch_batch_gs<1, 1>(b, total_blocks, tiled, nbr, s);
}

}  // namespace

hipError_t launch_batch_sweep(const BatchLaunch &b0, int total_blocks, int G, int share, int tiled, int nbr, bool inr,
                              hipStream_t s)
{
    BatchLaunch b = b0;
    for (int64_t first = 0; first < total_blocks; first += kMaxLaunchBlocks) {
        b.block0 = (int)first;
        const int blocks = (int)std::min<int64_t>(total_blocks - first, kMaxLaunchBlocks);
        const hipError_t e = inr ? launch_batch_sweep_inertia(b, blocks, G, tiled, nbr, s)
                                 : launch_batch_part(b, blocks, G, share, tiled, nbr, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_advance(ImageDesc *imgs, int n_imgs, uint32_t n, hipStream_t s)
{
    hipLaunchKernelGGL(advance_kernel, dim3((unsigned)((n_imgs + 63) / 64)), dim3(64), 0, s, imgs, n_imgs, n);
    return hipGetLastError();
}
}  // namespace pcak
