// C ABI of the lazy PCA sampler (declared in include/pca.h): parameter validation,
// device memory, sweep bookkeeping (beta schedule, burn-in, tally sweeps) and error
// reporting.  Every step of the sampler itself runs in the HIP kernels (pca_kernels*.hip,
// per-site arithmetic in pca_sweep.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "pca.h"
#include "pca_internal.h"

struct pca_ctx {
    pca_params p{};
    std::vector<float> beta;
    int G = 1, Cp = 1, T = 1;
    int64_t N = 0;
    int hist_words = 0;
    float *gp = nullptr;
    uint8_t *x[2] = {nullptr, nullptr};  // double-buffered chain states; x[cur] is current
    int cur = 0;
    uint32_t *sum = nullptr;
    uint32_t *hist = nullptr;
    int *flag = nullptr;  // device word for pca_set_state's level check
    int64_t t = 0, count = 0, tallies = 0;
    hipStream_t last = nullptr;
};

namespace {

// The calling thread's last error message: a fixed buffer, so that reporting an error
// allocates nothing.
thread_local char g_err[512];

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(PCA_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

int validate(const pca_params *p)
{
    if (!p) return fail(PCA_EINVAL, "params is NULL");
    if (p->height < 1 || p->width < 1) return fail(PCA_EINVAL, "height and width must be >= 1");
    if ((int64_t)p->height * p->width >= ((int64_t)1 << 31)) return fail(PCA_EINVAL, "lattice too large");
    if (p->levels < 2 || p->levels > 256) return fail(PCA_EINVAL, "levels must be in [2, 256]");
    if (p->chains < 1 || p->chains > 1024) return fail(PCA_EINVAL, "chains must be in [1, 1024]");
    if (p->neighbourhood != 4 && p->neighbourhood != 8) return fail(PCA_EINVAL, "neighbourhood must be 4 or 8");
    if (p->prior != PCA_PRIOR_POTTS && p->prior != PCA_PRIOR_TRUNC_LINEAR) return fail(PCA_EINVAL, "unknown prior");
    if (p->prior == PCA_PRIOR_TRUNC_LINEAR && p->trunc < 1) return fail(PCA_EINVAL, "trunc must be >= 1");
    if (!(p->J >= 0.0f) || !std::isfinite(p->J)) return fail(PCA_EINVAL, "J must be finite and >= 0");
    if (!(p->q >= 0.0f) || !std::isfinite(p->q)) return fail(PCA_EINVAL, "q must be finite and >= 0");
    if (!(p->sigma > 0.0f) || !std::isfinite(p->sigma)) return fail(PCA_EINVAL, "sigma must be finite and > 0");
    if (!std::isfinite(p->vmin) || !std::isfinite(p->vmax) || !(p->vmax > p->vmin))
        return fail(PCA_EINVAL, "need finite vmin < vmax");
    if (p->beta_len < 0 || (p->beta_len > 0 && !p->beta)) return fail(PCA_EINVAL, "bad beta array");
    const double log2e = pcak::kLog2e;
    for (int i = 0; i < p->beta_len; ++i) {
        if (!(p->beta[i] > 0.0f) || !std::isfinite(p->beta[i])) return fail(PCA_EINVAL, "beta[%d] must be > 0", i);
        if ((double)p->beta[i] * (double)p->q * log2e > 100.0) return fail(PCA_EINVAL, "beta*q too large");
    }
    if (p->beta_len == 0 && (double)p->q * log2e > 100.0) return fail(PCA_EINVAL, "q too large");
    if (p->init_mode != 0 && p->init_mode != 1) return fail(PCA_EINVAL, "init_mode must be 0 or 1");
    if (p->burn_in < 0 || p->tally_stride < 0) return fail(PCA_EINVAL, "burn_in and tally_stride must be >= 0");
    if (p->inertia < 0 || p->inertia > 2) return fail(PCA_EINVAL, "inertia must be 0, 1 or 2");
    return PCA_OK;
}

double level_scale(const pca_params &p) { return (double)(p.levels - 1) / ((double)p.vmax - (double)p.vmin); }

void release(pca_ctx *ctx)
{
    (void)hipFree(ctx->gp);
    (void)hipFree(ctx->x[0]);
    (void)hipFree(ctx->x[1]);
    (void)hipFree(ctx->sum);
    (void)hipFree(ctx->hist);
    (void)hipFree(ctx->flag);
    delete ctx;
}

pcak::RunBuffers run_buffers(const pca_ctx *ctx)
{
    pcak::RunBuffers b{};
    b.gp = ctx->gp;
    b.x[0] = ctx->x[0];
    b.x[1] = ctx->x[1];
    b.sum = ctx->sum;
    b.hist = ctx->hist;
    b.G = ctx->G;
    b.Cp = ctx->Cp;
    b.T = ctx->T;
    b.hist_words = ctx->hist_words;
    return b;
}

}  // namespace

pcak::RunBuffers pcak::run_layout(const pca_params &p)
{
    RunBuffers b{};
    b.G = chain_group(p.chains);
    b.Cp = (p.chains + b.G - 1) / b.G * b.G;
    b.T = p.prior == PCA_PRIOR_POTTS ? 1 : (p.trunc < p.levels - 1 ? p.trunc : p.levels - 1);
    b.hist_words = (p.levels + 1) / 2;
    return b;
}

hipError_t pcak::enqueue_sweeps(const pca_params &p, const float *beta, int beta_len, const RunBuffers &b, int64_t t0,
                                int32_t n, int &cur, int32_t *done, hipStream_t s)
{
    SweepArgs a{};
    a.gp = b.gp;
    a.H = p.height;
    a.W = p.width;
    a.L = p.levels;
    a.C = p.chains;
    a.Cp = b.Cp;
    a.T = b.T;
    a.hist_words = b.hist_words;
    a.J = (double)p.J;
    a.q = (double)p.q;
    a.kappa = p.prior == PCA_PRIOR_POTTS ? 2.0 : 1.0;
    a.inertia = p.inertia;
    a.sigma_s = (double)p.sigma * level_scale(p);
    a.key0 = (uint32_t)p.seed;
    a.key1 = (uint32_t)(p.seed >> 32);
    *done = 0;
    const TbPlan pl = tb_plan(p.height, p.width, p.levels, b.Cp, p.neighbourhood, b.T, p.inertia);
    if (pl.S > 0) {
        // several sweeps per launch from LDS tiles (lattices with few levels)
        TbArgs tb{};
        tb.a = a;
        tb.nbr = p.neighbourhood;
        tb.TH = pl.TH;
        tb.TW = pl.TW;
        tb.tiles_w = pl.tiles_w;
        tb.tiles = pl.tiles;
        tb.ptab_n = p.neighbourhood * b.T + 1;
        for (int32_t i = 0; i < n;) {
            const int S = (int)std::min<int64_t>(pl.S, n - i);
            tb.S = S;
            tb.acc_mask = tb.tally_mask = tb.beta_mask = 0u;
            for (int j = 0; j < S; ++j) {
                const int64_t t = t0 + i + j;
                const bool acc = t >= p.burn_in;
                const bool tally = acc && p.tally_stride > 0 && (t - p.burn_in) % p.tally_stride == 0;
                tb.acc_mask |= (uint32_t)acc << j;
                tb.tally_mask |= (uint32_t)tally << j;
                tb.beta[j] = beta_len == 0 ? 1.0 : (double)beta[t < beta_len ? t : beta_len - 1];
                if (j > 0 && tb.beta[j] != tb.beta[j - 1]) tb.beta_mask |= 1u << j;
            }
            tb.a.t = (uint32_t)(t0 + i);
            tb.a.xin = b.x[cur];
            tb.a.xout = b.x[cur ^ 1];
            tb.a.sum = tb.acc_mask ? b.sum : nullptr;
            tb.a.hist = tb.tally_mask ? b.hist : nullptr;
            const hipError_t e = launch_tb_sweeps(tb, s);
            if (e != hipSuccess) return e;
            cur ^= 1;
            i += S;
            *done = i;
        }
        return hipSuccess;
    }
    for (int32_t i = 0; i < n; ++i) {
        const int64_t t = t0 + i;
        const bool acc = t >= p.burn_in;
        const bool tally = acc && p.tally_stride > 0 && (t - p.burn_in) % p.tally_stride == 0;
        a.xin = b.x[cur];
        a.xout = b.x[cur ^ 1];
        a.sum = acc ? b.sum : nullptr;
        a.hist = tally ? b.hist : nullptr;
        a.beta = beta_len == 0 ? 1.0 : (double)beta[t < beta_len ? t : beta_len - 1];
        a.t = (uint32_t)t;
        const hipError_t e = launch_sweep(a, b.G, p.neighbourhood, s);
        if (e != hipSuccess) return e;
        cur ^= 1;
        *done = i + 1;
    }
    return hipSuccess;
}

namespace {

int check_ctx(const pca_ctx *ctx)
{
    if (!ctx) return fail(PCA_EINVAL, "ctx is NULL");
    return PCA_OK;
}

}  // namespace

int pcak::validate_params(const pca_params *p) { return validate(p); }

int pcak::set_error(int code, const char *message)
{
    if (message != g_err) snprintf(g_err, sizeof g_err, "%s", message);
    return code;
}

bool pcak::fault_injected(const char *site, int64_t id)
{
    const char *spec = std::getenv("PCA_FAULT_INJECT");
    if (!spec || !*spec) return false;
    const size_t n = std::strlen(site);
    for (const char *p = spec; *p;) {
        const char *end = std::strchr(p, ',');
        if (!end) end = p + std::strlen(p);
        if ((size_t)(end - p) >= n && std::strncmp(p, site, n) == 0) {
            const char *rest = p + n;
            if (rest == end) return true;  // every call at this site
            if (*rest == ':') {
                char *stop = nullptr;
                const long long want = std::strtoll(rest + 1, &stop, 10);
                if (stop == end && want == (long long)id) return true;
            }
        }
        p = *end ? end + 1 : end;
    }
    return false;
}

extern "C" {

const char *pca_last_error(void) { return g_err; }

int pca_init(const pca_params *params, const float *obs_dev, void *stream, pca_ctx **out)
{
    g_err[0] = 0;
    if (!out) return fail(PCA_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(params);
    if (rc) return rc;
    if (!obs_dev) return fail(PCA_EINVAL, "obs_dev is NULL");
    hipStream_t s = (hipStream_t)stream;

    pca_ctx *ctx = new (std::nothrow) pca_ctx();
    if (!ctx) return fail(PCA_ENOMEM, "host allocation failed");
    ctx->p = *params;
    try {
        if (params->beta_len > 0) ctx->beta.assign(params->beta, params->beta + params->beta_len);
    } catch (const std::bad_alloc &) {
        release(ctx);
        return fail(PCA_ENOMEM, "host allocation failed");
    }
    ctx->p.beta = nullptr;
    const pcak::RunBuffers lay = pcak::run_layout(*params);
    ctx->G = lay.G;
    ctx->Cp = lay.Cp;
    ctx->T = lay.T;
    ctx->hist_words = lay.hist_words;
    ctx->N = (int64_t)params->height * params->width;
    ctx->last = s;

    const size_t N = (size_t)ctx->N;
    hipError_t e = pcak::fault_injected("init", 0) ? hipErrorOutOfMemory : hipMalloc(&ctx->gp, N * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&ctx->flag, sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&ctx->x[0], N * ctx->Cp);
    if (e == hipSuccess) e = hipMalloc(&ctx->x[1], N * ctx->Cp);
    if (e == hipSuccess) e = hipMalloc(&ctx->sum, N * sizeof(uint32_t));
    if (e == hipSuccess && params->tally_stride > 0) e = hipMalloc(&ctx->hist, N * ctx->hist_words * sizeof(uint32_t));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        release(ctx);
        return fail(PCA_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
    }
    e = hipMemsetAsync(ctx->sum, 0, N * sizeof(uint32_t), s);
    if (e == hipSuccess && ctx->hist) e = hipMemsetAsync(ctx->hist, 0, N * ctx->hist_words * sizeof(uint32_t), s);
    if (e == hipSuccess) {
        pcak::InitArgs a{};
        a.obs = obs_dev;
        a.gp = ctx->gp;
        a.x = ctx->x[0];
        a.N = ctx->N;
        a.Cp = ctx->Cp;
        a.L = params->levels;
        a.mode = params->init_mode;
        a.vmin = (double)params->vmin;
        a.scale = level_scale(*params);
        a.key0 = (uint32_t)params->seed;
        a.key1 = (uint32_t)(params->seed >> 32);
        e = pcak::launch_init(a, s);
    }
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(s);
        release(ctx);
        return hip_fail(e, "pca_init");
    }
    *out = ctx;
    return PCA_OK;
}

int pca_sweep(pca_ctx *ctx, int32_t n, void *stream)
{
    g_err[0] = 0;
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (n < 0) return fail(PCA_EINVAL, "n must be >= 0");
    if (n == 0) return PCA_OK;
    const pca_params &p = ctx->p;
    // the sweep index is a 32-bit Philox counter word: beyond it the draws would repeat
    if (ctx->t + n > 0xFFFFFFFFll) return fail(PCA_ESTATE, "the sweep index would pass 2^32 - 1");
    // Overflow guards: the uint32 level sum and the uint16 histogram counters.
    int64_t add_sweeps = 0, add_tallies = 0;
    pcak::accumulating_sweeps(ctx->t, n, p.burn_in, p.tally_stride, &add_sweeps, &add_tallies);
    const int64_t add_count = add_sweeps * p.chains;
    if ((double)(ctx->count + add_count) * (double)(p.levels - 1) > 4294967295.0)
        return fail(PCA_ESTATE, "the level sum could overflow 32 bits");
    if ((ctx->tallies + add_tallies) * (int64_t)p.chains > 65535)
        return fail(PCA_ESTATE, "a histogram counter could overflow 16 bits");

    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    const pcak::RunBuffers b = run_buffers(ctx);
    int32_t done = 0;
    const hipError_t e = pcak::enqueue_sweeps(p, ctx->beta.empty() ? nullptr : ctx->beta.data(), (int)ctx->beta.size(),
                                              b, ctx->t, n, ctx->cur, &done, s);
    // the sweeps enqueued before a failed launch still count
    pcak::accumulating_sweeps(ctx->t, done, p.burn_in, p.tally_stride, &add_sweeps, &add_tallies);
    ctx->t += done;
    ctx->count += add_sweeps * p.chains;
    ctx->tallies += add_tallies;
    return e == hipSuccess ? PCA_OK : hip_fail(e, "pca_sweep");
}

int pca_posterior_mean(pca_ctx *ctx, float *out_dev, void *stream)
{
    g_err[0] = 0;
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!out_dev) return fail(PCA_EINVAL, "out_dev is NULL");
    if (ctx->count <= 0) return fail(PCA_ESTATE, "no accumulated sweeps");
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    const pca_params &p = ctx->p;
    const double delta = ((double)p.vmax - (double)p.vmin) / (double)(p.levels - 1);
    hipError_t e = pcak::launch_mean(ctx->sum, out_dev, ctx->N, ctx->count, (double)p.vmin, delta, s);
    return e == hipSuccess ? PCA_OK : hip_fail(e, "pca_posterior_mean");
}

int pca_marginal_map(pca_ctx *ctx, uint8_t *out_dev, void *stream)
{
    g_err[0] = 0;
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!out_dev) return fail(PCA_EINVAL, "out_dev is NULL");
    if (!ctx->hist) return fail(PCA_ESTATE, "histogram disabled (tally_stride = 0)");
    if (ctx->tallies <= 0) return fail(PCA_ESTATE, "no tally sweeps yet");
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    hipError_t e = pcak::launch_mpm(ctx->hist, out_dev, ctx->N, ctx->p.levels, ctx->hist_words, s);
    return e == hipSuccess ? PCA_OK : hip_fail(e, "pca_marginal_map");
}

int pca_get_state(pca_ctx *ctx, uint8_t *out_dev, void *stream)
{
    g_err[0] = 0;
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!out_dev) return fail(PCA_EINVAL, "out_dev is NULL");
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    hipError_t e = pcak::launch_get_state(ctx->x[ctx->cur], out_dev, ctx->N, ctx->p.chains, ctx->Cp, s);
    return e == hipSuccess ? PCA_OK : hip_fail(e, "pca_get_state");
}

int pca_set_state(pca_ctx *ctx, const uint8_t *in_dev, int64_t t, void *stream)
{
    g_err[0] = 0;
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!in_dev) return fail(PCA_EINVAL, "in_dev is NULL");
    if (t < 0 || t > 0xFFFFFFFFll) return fail(PCA_EINVAL, "t out of range");
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    // every value must be a level index: checked on the device, then read back
    int bad = 0;
    hipError_t e = hipMemsetAsync(ctx->flag, 0, sizeof(int), s);
    if (e == hipSuccess) e = pcak::launch_check_levels(in_dev, ctx->N * ctx->p.chains, ctx->p.levels, ctx->flag, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, ctx->flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "pca_set_state");
    if (bad) return fail(PCA_EINVAL, "pca_set_state: a state value is not below levels (%d)", ctx->p.levels);
    e = pcak::launch_set_state(in_dev, ctx->x[ctx->cur], ctx->N, ctx->p.chains, ctx->Cp, s);
    if (e != hipSuccess) return hip_fail(e, "pca_set_state");
    ctx->t = t;
    return PCA_OK;
}

int pca_get_accumulators(pca_ctx *ctx, uint32_t *sum_dev, uint16_t *hist_dev, void *stream)
{
    g_err[0] = 0;
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!sum_dev) return fail(PCA_EINVAL, "sum_dev is NULL");
    if (hist_dev && !ctx->hist) return fail(PCA_EINVAL, "this run keeps no histogram");
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    const size_t L = (size_t)ctx->p.levels;
    hipError_t e = hipMemcpyAsync(sum_dev, ctx->sum, (size_t)ctx->N * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
    // the histogram row of a pixel is hist_words words of two uint16 counters (level 2w in
    // the low half), i.e. 2*hist_words uint16 counters in level order on this little-endian
    // device; the copy drops the unused counter of an odd level count
    if (e == hipSuccess && hist_dev)
        e = hipMemcpy2DAsync(hist_dev, L * sizeof(uint16_t), ctx->hist, (size_t)ctx->hist_words * sizeof(uint32_t),
                             L * sizeof(uint16_t), (size_t)ctx->N, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? PCA_OK : hip_fail(e, "pca_get_accumulators");
}

int pca_set_accumulators(pca_ctx *ctx, const uint32_t *sum_dev, const uint16_t *hist_dev, int64_t count,
                         int64_t tallies, void *stream)
{
    g_err[0] = 0;
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!sum_dev) return fail(PCA_EINVAL, "sum_dev is NULL");
    if (hist_dev && !ctx->hist) return fail(PCA_EINVAL, "this run keeps no histogram");
    if (!hist_dev && ctx->hist) return fail(PCA_EINVAL, "hist_dev is NULL but this run keeps a histogram");
    if (count < 0 || tallies < 0) return fail(PCA_EINVAL, "counts must be >= 0");
    if ((double)count * (double)(ctx->p.levels - 1) > 4294967295.0)
        return fail(PCA_EINVAL, "count too large for the 32-bit level sum");
    if (tallies * (int64_t)ctx->p.chains > 65535) return fail(PCA_EINVAL, "tallies too large for 16-bit counters");
    hipStream_t s = (hipStream_t)stream;
    ctx->last = s;
    const size_t L = (size_t)ctx->p.levels;
    hipError_t e = hipMemcpyAsync(ctx->sum, sum_dev, (size_t)ctx->N * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && hist_dev)
        e = hipMemcpy2DAsync(ctx->hist, (size_t)ctx->hist_words * sizeof(uint32_t), hist_dev, L * sizeof(uint16_t),
                             L * sizeof(uint16_t), (size_t)ctx->N, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "pca_set_accumulators");
    ctx->count = count;
    ctx->tallies = tallies;
    return PCA_OK;
}

int pca_stats(const pca_ctx *ctx, int64_t *sweep, int64_t *count, int64_t *tallies)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (sweep) *sweep = ctx->t;
    if (count) *count = ctx->count;
    if (tallies) *tallies = ctx->tallies;
    return PCA_OK;
}

int pca_sweeps_per_launch(const pca_ctx *ctx, int32_t *out)
{
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (!out) return pcak::set_error(PCA_EINVAL, "out is NULL");
    const pcak::TbPlan pl =
        pcak::tb_plan(ctx->p.height, ctx->p.width, ctx->p.levels, ctx->Cp, ctx->p.neighbourhood, ctx->T, ctx->p.inertia);
    *out = pl.S > 0 ? pl.S : 1;
    return PCA_OK;
}

int pca_sync(pca_ctx *ctx)
{
    g_err[0] = 0;
    int rc = check_ctx(ctx);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(ctx->last);
    if (e == hipSuccess) e = hipGetLastError();
    return e == hipSuccess ? PCA_OK : hip_fail(e, "pca_sync");
}

int pca_destroy(pca_ctx *ctx)
{
    g_err[0] = 0;
    if (!ctx) return PCA_OK;
    hipError_t e = hipStreamSynchronize(ctx->last);
    release(ctx);
    return e == hipSuccess ? PCA_OK : hip_fail(e, "pca_destroy");
}

}  // extern "C"
