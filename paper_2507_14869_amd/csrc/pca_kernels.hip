// Single-lattice sweep kernels, state initialisation and read-outs of the lazy PCA
// sampler (arXiv 2507.14869, Sec. 5.2) for gfx950.  The per-site arithmetic is in
// pca_sweep.h.
#include "pca_sweep.h"

namespace pcak {
namespace {

// One sweep of one lattice: tpp = Cp/G threads per pixel (one per chain group), laid out
// as sweep_thread_site describes.
template <int G, int NBR, int SUB, int NBLK, int SHARE>
__global__ __launch_bounds__(kBlock, kMinWaves<SUB>) void sweep_kernel(SweepArgs a)
{
    __shared__ float ptab[kMaxNeighbourStat + 1];
    __shared__ uint4 vtab[kStatEntries];
    const SweepConsts kc = sweep_prologue(a, NBR, ptab, vtab);
    int pix, r, c, grp;
    if (!sweep_thread_site(a, a.Cp / G, pix, r, c, grp)) return;
    sweep_site<G, NBR, SUB, NBLK, SHARE>(a, ptab, vtab, kc, pix, r, c, grp, (int)(threadIdx.x % SHARE));
}

// ---------------------------------------------------------------- init and readouts

__global__ __launch_bounds__(kBlock) void init_kernel(InitArgs a)
{
    const int64_t pix = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (pix >= a.N) return;
    float gp;
    if (a.obs) {
        gp = (float)(((double)a.obs[pix] - a.vmin) * a.scale);
        a.gp[pix] = gp;
    } else {
        gp = a.gp[pix];
    }
    float kh = __builtin_rintf(gp);
    kh = kh < 0.0f ? 0.0f : kh;
    kh = kh > (float)(a.L - 1) ? (float)(a.L - 1) : kh;
    uint8_t *row = a.x + pix * a.Cp;
    for (int c0 = 0; c0 < a.Cp; c0 += 4) {
        U4 rnd{0u, 0u, 0u, 0u};
        if (a.mode == 1) rnd = philox(U4{(uint32_t)pix, 0u, (uint32_t)(c0 >> 2), 1u}, a.key0, a.key1);
        for (int j = 0; j < 4 && c0 + j < a.Cp; ++j) {
            int v;
            if (a.mode == 0) v = (int)kh;
            else v = (int)(((uint64_t)(word_of(rnd, j) >> 8) * (uint64_t)a.L) >> 24);
            row[c0 + j] = (uint8_t)v;
        }
    }
}

__global__ __launch_bounds__(kBlock) void get_state_kernel(const uint8_t *x, uint8_t *out, int64_t N, int C, int Cp)
{
    const int64_t pix = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (pix >= N) return;
    for (int ch = 0; ch < C; ++ch) out[(int64_t)ch * N + pix] = x[pix * Cp + ch];
}

// Padding chain slots (ch >= C) take chain 0's value: they are never read out, and any
// valid level keeps their (discarded) draws in range.
__global__ __launch_bounds__(kBlock) void set_state_kernel(const uint8_t *in, uint8_t *x, int64_t N, int C, int Cp)
{
    const int64_t pix = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (pix >= N) return;
    for (int ch = 0; ch < Cp; ++ch) {
        const int src = ch < C ? ch : 0;
        x[pix * Cp + ch] = in[(int64_t)src * N + pix];
    }
}

constexpr int kCheckBlocks = 2048;

__global__ __launch_bounds__(kBlock) void check_levels_kernel(const uint8_t *in, int64_t n, int L, int *flag)
{
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)kCheckBlocks * kBlock)
        bad = bad || (int)in[i] >= L;
    if (bad) atomicOr(flag, 1);
}

__global__ __launch_bounds__(kBlock) void mean_kernel(const uint32_t *sum, float *out, int64_t N, int64_t count,
                                                      double vmin, double delta)
{
    const int64_t pix = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (pix >= N) return;
    out[pix] = (float)(vmin + ((double)sum[pix] / (double)count) * delta);
}

// Marginal mode of kMpmRows pixels per workgroup: their histogram rows (contiguous in
// memory) are staged through LDS with coalesced loads, then one thread per pixel scans
// its row; ties go to the lowest level.
constexpr int kMpmRows = 64;

__global__ __launch_bounds__(kBlock) void mpm_kernel(const uint32_t *hist, uint8_t *out, int64_t N, int L,
                                                     int hist_words)
{
    __shared__ uint32_t rows[kMpmRows * 129];  // row stride hist_words + 1 (<= 129) against bank conflicts
    const int64_t pix0 = (int64_t)blockIdx.x * kMpmRows;
    const int nrows = (int)((N - pix0) < kMpmRows ? (N - pix0) : kMpmRows);
    const int stride = hist_words + 1;
    const uint32_t *src = hist + pix0 * hist_words;
    const int words = nrows * hist_words;
    for (int w = threadIdx.x; w < words; w += kBlock) {
        const int rr = w / hist_words;
        rows[rr * stride + (w - rr * hist_words)] = src[w];
    }
    __syncthreads();
    if ((int)threadIdx.x >= nrows) return;
    const uint32_t *h = rows + threadIdx.x * stride;
    int best = 0;
    uint32_t bestv = h[0] & 0xFFFFu;
    for (int k = 1; k < L; ++k) {
        const uint32_t v = (h[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
        if (v > bestv) {
            bestv = v;
            best = k;
        }
    }
    out[pix0 + threadIdx.x] = (uint8_t)best;
}

template <int G, int NBR, int SHARE>
hipError_t launch_sweep_gs(const SweepArgs &a0, hipStream_t s)
{
    const SweepLayout lay = sweep_layout(a0.H, a0.W, a0.Cp / G, a0.L > 16);
    SweepArgs a = a0;
    a.patch = lay.patch;
    a.tiles_w = lay.tiles_w;
    for (a.blk0 = 0; a.blk0 < lay.blocks; a.blk0 += kMaxLaunchBlocks) {
        const unsigned grid = (unsigned)std::min<int64_t>(lay.blocks - a.blk0, kMaxLaunchBlocks);
        if (a.L <= 16)
            hipLaunchKernelGGL((sweep_kernel<G, NBR, 1, 16, SHARE>), dim3(grid), dim3(kBlock), 0, s, a);
        else
            hipLaunchKernelGGL((sweep_kernel<G, NBR, 16, 16, SHARE>), dim3(grid), dim3(kBlock), 0, s, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Threads per pixel = Cp / G; the data factor is shared by groups of 4 or 2 of them when
// that count allows (groups must tile the pixel's threads and align with lane quads).
template <int G, int NBR>
hipError_t launch_sweep_g(const SweepArgs &a, hipStream_t s)
{
    const int tpp = a.Cp / G;
    if constexpr (G == 4) {
        if (tpp % 4 == 0) return launch_sweep_gs<G, NBR, 4>(a, s);
        if (tpp % 2 == 0) return launch_sweep_gs<G, NBR, 2>(a, s);
    }
    return launch_sweep_gs<G, NBR, 1>(a, s);
}

}  // namespace

hipError_t launch_sweep(const SweepArgs &a, int G, int nbr, hipStream_t s)
{
    if (a.inertia != 0) return launch_sweep_inertia(a, G, nbr, s);
    if (nbr == 4) {
        if (G == 4) return launch_sweep_g<4, 4>(a, s);
        if (G == 2) return launch_sweep_g<2, 4>(a, s);
        return launch_sweep_g<1, 4>(a, s);
    }
    if (G == 4) return launch_sweep_g<4, 8>(a, s);
    if (G == 2) return launch_sweep_g<2, 8>(a, s);
    return launch_sweep_g<1, 8>(a, s);
}

hipError_t launch_init(const InitArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(init_kernel, dim3(grid_for(a.N)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_get_state(const uint8_t *x, uint8_t *out, int64_t N, int C, int Cp, hipStream_t s)
{
    hipLaunchKernelGGL(get_state_kernel, dim3(grid_for(N)), dim3(kBlock), 0, s, x, out, N, C, Cp);
    return hipGetLastError();
}

hipError_t launch_set_state(const uint8_t *in, uint8_t *x, int64_t N, int C, int Cp, hipStream_t s)
{
    hipLaunchKernelGGL(set_state_kernel, dim3(grid_for(N)), dim3(kBlock), 0, s, in, x, N, C, Cp);
    return hipGetLastError();
}

hipError_t launch_check_levels(const uint8_t *in, int64_t n, int L, int *flag, hipStream_t s)
{
    hipLaunchKernelGGL(check_levels_kernel, dim3(kCheckBlocks), dim3(kBlock), 0, s, in, n, L, flag);
    return hipGetLastError();
}

hipError_t launch_mean(const uint32_t *sum, float *out, int64_t N, int64_t count, double vmin, double delta,
                       hipStream_t s)
{
    hipLaunchKernelGGL(mean_kernel, dim3(grid_for(N)), dim3(kBlock), 0, s, sum, out, N, count, vmin, delta);
    return hipGetLastError();
}

hipError_t launch_mpm(const uint32_t *hist, uint8_t *out, int64_t N, int L, int hist_words, hipStream_t s)
{
    const unsigned blocks = (unsigned)((N + kMpmRows - 1) / kMpmRows);
    hipLaunchKernelGGL(mpm_kernel, dim3(blocks), dim3(kBlock), 0, s, hist, out, N, L, hist_words);
    return hipGetLastError();
}

}  // namespace pcak
