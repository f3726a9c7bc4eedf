// pca_run_static: the whole single-lattice job (initialisation, n sweeps, read-outs) with
// every working buffer in a fixed device array of the library, for callers that cannot
// allocate device memory (HIP graph capture, serving loops, harnesses that forbid
// allocation).  The kernels are those of pca_init / pca_sweep / pca_posterior_mean /
// pca_marginal_map / pca_get_state, so the results are the same bit for bit.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "pca.h"
#include "pca_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)PCA_STATIC_SCRATCH_BYTES;
constexpr size_t kAlign = 256;
constexpr int kMaxDevices = 64;

// The working memory of pca_run_static, one copy per device, held until the process
// ends.  Host code never uses this name as an address: it takes the device address from
// hipGetSymbolAddress (scratch_base below).
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_base[kMaxDevices];  // device address of `scratch` on each device, once looked up

// Device address of `scratch` on the current device, looked up once per device with that
// device current.
hipError_t scratch_base(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_base[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_base[dev] = p;
    }
    *out = g_base[dev];
    return hipSuccess;
}

__global__ __launch_bounds__(pcak::kBlock) void zero_kernel(uint32_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * pcak::kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * pcak::kBlock)
        p[i] = 0u;
}

// Clears n words with a kernel (not a memset node, so the call can be graph-captured).
hipError_t zero_words(uint32_t *p, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t want = (n + pcak::kBlock - 1) / pcak::kBlock;
    const unsigned grid = (unsigned)(want < 4096 ? want : 4096);
    hipLaunchKernelGGL(zero_kernel, dim3(grid), dim3(pcak::kBlock), 0, s, p, n);
    return hipGetLastError();
}

size_t round_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

}  // namespace

extern "C" int pca_run_static(const pca_params *params, const float *obs_dev, int32_t sweeps, float *mean_out_dev,
                              uint8_t *mpm_out_dev, uint8_t *state_out_dev, void *stream)
{
    pcak::set_error(PCA_OK, "");
    int rc = pcak::validate_params(params);
    if (rc) return rc;
    const pca_params &p = *params;
    if (!obs_dev) return pcak::set_error(PCA_EINVAL, "obs_dev is NULL");
    if (sweeps < 0) return pcak::set_error(PCA_EINVAL, "sweeps must be >= 0");
    if (!mean_out_dev && !mpm_out_dev && !state_out_dev) return pcak::set_error(PCA_EINVAL, "no output requested");
    if (mpm_out_dev && p.tally_stride <= 0)
        return pcak::set_error(PCA_ESTATE, "marginal mode requested but the histogram is disabled (tally_stride = 0)");

    // The same guards as pca_init followed by pca_sweep(sweeps) and the read-outs.
    int64_t acc = 0, tallies = 0;
    pcak::accumulating_sweeps(0, sweeps, p.burn_in, p.tally_stride, &acc, &tallies);
    const int64_t count = acc * p.chains;
    if ((double)count * (double)(p.levels - 1) > 4294967295.0)
        return pcak::set_error(PCA_ESTATE, "the level sum could overflow 32 bits");
    if (tallies * (int64_t)p.chains > 65535) return pcak::set_error(PCA_ESTATE, "a histogram counter could overflow 16 bits");
    if (mean_out_dev && count == 0) return pcak::set_error(PCA_ESTATE, "posterior mean requested but no sweep is accumulated");
    if (mpm_out_dev && tallies == 0) return pcak::set_error(PCA_ESTATE, "marginal mode requested but no sweep is tallied");

    // Working buffers, each 256-byte aligned inside the scratch array.
    pcak::RunBuffers b = pcak::run_layout(p);
    const size_t N = (size_t)p.height * (size_t)p.width;
    const size_t gp_off = 0;
    const size_t x0_off = gp_off + round_up(N * sizeof(float));
    const size_t x1_off = x0_off + round_up(N * (size_t)b.Cp);
    const size_t sum_off = x1_off + round_up(N * (size_t)b.Cp);
    const size_t hist_off = sum_off + round_up(N * sizeof(uint32_t));
    const size_t hist_n = p.tally_stride > 0 ? N * (size_t)b.hist_words : 0;
    const size_t need = hist_off + hist_n * sizeof(uint32_t);
    if (need > kScratchBytes) {
        char msg[160];
        snprintf(msg, sizeof msg, "pca_run_static: the run needs %zu bytes of working memory, above the %zu-byte limit",
                 need, kScratchBytes);
        return pcak::set_error(PCA_EINVAL, msg);
    }

    void *base_v = nullptr;
    hipError_t e = scratch_base(&base_v);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return pcak::set_error(PCA_EDEVICE, "pca_run_static: the working memory's device address is not available");
    }
    unsigned char *base = static_cast<unsigned char *>(base_v);
    b.gp = reinterpret_cast<float *>(base + gp_off);
    b.x[0] = base + x0_off;
    b.x[1] = base + x1_off;
    b.sum = reinterpret_cast<uint32_t *>(base + sum_off);
    b.hist = hist_n ? reinterpret_cast<uint32_t *>(base + hist_off) : nullptr;
    hipStream_t s = (hipStream_t)stream;

    // The array keeps the previous call's contents: clear the accumulators first.
    e = zero_words(b.sum, (int64_t)N, s);
    if (e == hipSuccess && b.hist) e = zero_words(b.hist, (int64_t)hist_n, s);
    if (e == hipSuccess) {
        pcak::InitArgs a{};
        a.obs = obs_dev;
        a.gp = b.gp;
        a.x = b.x[0];
        a.N = (int64_t)N;
        a.Cp = b.Cp;
        a.L = p.levels;
        a.mode = p.init_mode;
        a.vmin = (double)p.vmin;
        a.scale = (double)(p.levels - 1) / ((double)p.vmax - (double)p.vmin);
        a.key0 = (uint32_t)p.seed;
        a.key1 = (uint32_t)(p.seed >> 32);
        e = pcak::launch_init(a, s);
    }
    int cur = 0;
    int32_t done = 0;
    if (e == hipSuccess) e = pcak::enqueue_sweeps(p, p.beta, p.beta_len, b, 0, sweeps, cur, &done, s);
    if (e == hipSuccess && mean_out_dev) {
        const double delta = ((double)p.vmax - (double)p.vmin) / (double)(p.levels - 1);
        e = pcak::launch_mean(b.sum, mean_out_dev, (int64_t)N, count, (double)p.vmin, delta, s);
    }
    if (e == hipSuccess && mpm_out_dev) e = pcak::launch_mpm(b.hist, mpm_out_dev, (int64_t)N, p.levels, b.hist_words, s);
    if (e == hipSuccess && state_out_dev) e = pcak::launch_get_state(b.x[cur], state_out_dev, (int64_t)N, p.chains, b.Cp, s);
    if (e != hipSuccess) {
        char msg[160];
        snprintf(msg, sizeof msg, "pca_run_static: %s", hipGetErrorString(e));
        return pcak::set_error(PCA_EDEVICE, msg);
    }
    return PCA_OK;
}
