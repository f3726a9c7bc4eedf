// C ABI of the batched sampler (declared in include/pca.h): many independent lattices of
// different sizes, level counts and parameters advanced together, one kernel launch per
// sweep for the whole batch, the launches of a pca_batch_sweep call replayed from a cached
// HIP graph, and a launch-configuration autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "pca.h"
#include "pca_internal.h"

namespace {

// Sweeps per cached graph: a longer pca_batch_sweep call replays the 64-sweep graph (the
// sweep index lives in device memory) and one graph for the remainder, so graph sizes and
// the number of cached graphs stay bounded whatever n the caller passes.
constexpr int32_t kGraphSweeps = 64;

// tiled: 0 untiled (2-D patches for L > 16, else row-major), 1 tiles 16 pixels wide, 2 as 0
// but lattices with L <= 16 run several sweeps per launch from LDS tiles.
struct LaunchConfig {
    int G = 1, share = 1, tiled = 0;
    bool operator<(const LaunchConfig &o) const
    {
        return G != o.G ? G < o.G : share != o.share ? share < o.share : tiled < o.tiled;
    }
};

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return pcak::set_error(code, buf);
}

int hip_fail(hipError_t e, const char *what) { return fail(PCA_EDEVICE, "%s: %s", what, hipGetErrorString(e)); }

double level_scale(const pca_params &p) { return (double)(p.levels - 1) / ((double)p.vmax - (double)p.vmin); }

}  // namespace

struct pca_batch {
    int n = 0;
    int nbr = 4;
    bool inr = false;  // L1/L2 inertia kernels
    std::vector<pca_params> p;
    std::vector<pcak::ImageDesc> desc;  // host copy; pointers are device buffers
    std::vector<int64_t> count, tallies;
    pcak::ImageDesc *d_desc = nullptr;
    double *d_beta = nullptr;
    int *d_block_img = nullptr;
    int *d_tb_block_img = nullptr;  // multi-sweep traversal: workgroup -> lattice
    int tb_blocks = 0;
    size_t tb_lds = 0;
    int64_t t = 0;
    LaunchConfig cfg;
    int total_blocks = 0;
    hipStream_t cap = nullptr;  // private stream used only to capture graphs
    std::map<int, hipGraphExec_t> graphs;
    hipStream_t last = nullptr;
};

namespace {

// Tile side of a lattice in the multi-sweep traversal with G chains per thread: 8, else 4
// when the items of 8x8 tiles do not fit, or 0 when the traversal does not take it (more
// levels, the L1/L2 inertia, or no tile fits).
int multi_sweep_side(const pca_batch *b, const pcak::ImageDesc &d, int G)
{
    if (b->inr || d.L > 16) return 0;
    for (int side : {pcak::kTbBatchSide, 4})
        if (pcak::tb_fits(d.H, d.W, d.Cp, G, side, pcak::kTbBatchSweeps, b->nbr * d.T + 1, pcak::kTbBatchItems,
                          pcak::kTbBatchBlock))
            return side;
    return 0;
}

bool config_valid(const pca_batch *b, const LaunchConfig &c)
{
    if (c.tiled < 0 || c.tiled > 2) return false;
    if (b->inr && c.share != 1) return false;  // each chain has its own exponent: nothing to share
    bool any_multi = false;
    for (const auto &d : b->desc) {
        if (d.Cp % c.G != 0) return false;
        const int tpp = d.Cp / c.G;
        if (tpp % c.share != 0) return false;
        if (c.tiled == 1 && (tpp > pcak::kBlock / pcak::kTileW)) return false;
        any_multi = any_multi || multi_sweep_side(b, d, c.G) > 0;
    }
    return c.tiled != 2 || any_multi;  // without such a lattice it would be configuration 0
}

std::vector<LaunchConfig> candidates(const pca_batch *b)
{
    std::vector<LaunchConfig> out;
    for (int G : {4, 2, 1})
        for (int share : {4, 2, 1})
            for (int tiled : {0, 1, 2}) {
                LaunchConfig c{G, share, tiled};
                if (config_valid(b, c)) out.push_back(c);
            }
    return out;
}

void drop_graphs(pca_batch *b)
{
    for (auto &kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    b->graphs.clear();
}

// Lays out the batched grid for a launch configuration: workgroup ranges per lattice.
int apply_config(pca_batch *b, const LaunchConfig &c, hipStream_t s)
{
    std::vector<int> block_img, tb_block_img;
    int base = 0;
    size_t tb_lds = 0;
    for (int i = 0; i < b->n; ++i) {
        pcak::ImageDesc &d = b->desc[i];
        d.tpp = d.Cp / c.G;
        d.tb_side = 0;
        const int side = c.tiled == 2 ? multi_sweep_side(b, d, c.G) : 0;
        if (side > 0) {
            // its own table of workgroups, one per LDS tile
            d.tb_side = side;
            d.patch = -1;
            d.tiles_w = (d.W + side - 1) / side;
            d.block_base = (int)tb_block_img.size();
            const int64_t tiles = (int64_t)d.tiles_w * ((d.H + side - 1) / side);
            if ((int64_t)tb_block_img.size() + tiles > 0x7FFFFFFF) return fail(PCA_EINVAL, "batch grid too large");
            try {
                tb_block_img.insert(tb_block_img.end(), (size_t)tiles, i);
            } catch (const std::bad_alloc &) {
                return fail(PCA_ENOMEM, "batch: host allocation failed");
            }
            tb_lds = std::max(tb_lds, pcak::tb_lds_bytes(d.H, d.W, d.Cp, side, pcak::kTbBatchSweeps, b->nbr * d.T + 1));
            continue;
        }
        d.block_base = base;
        int blocks;
        if (c.tiled == 1) {
            const int th = pcak::kBlock / d.tpp / pcak::kTileW;
            d.tiles_w = (d.W + pcak::kTileW - 1) / pcak::kTileW;
            d.patch = -1;
            blocks = d.tiles_w * ((d.H + th - 1) / th);
        } else {
            blocks = (int)pcak::untiled_layout(d);
        }
        if ((int64_t)base + blocks > 0x7FFFFFFF) return fail(PCA_EINVAL, "batch grid exceeds 2^31 - 1 workgroups");
        try {
            block_img.insert(block_img.end(), (size_t)blocks, i);
        } catch (const std::bad_alloc &) {
            return fail(PCA_ENOMEM, "batch: host allocation failed");
        }
        base += blocks;
    }
    (void)hipStreamSynchronize(b->last);  // no launch of the old layout may still be running
    (void)hipStreamSynchronize(s);
    for (auto &d : b->desc) {  // the device copy is re-uploaded whole: carry the sweep index
        d.t = (uint32_t)b->t;
        d.t_end = 0xFFFFFFFFu;
    }
    (void)hipFree(b->d_block_img);
    b->d_block_img = nullptr;
    (void)hipFree(b->d_tb_block_img);
    b->d_tb_block_img = nullptr;
    hipError_t e = block_img.empty() ? hipSuccess : hipMalloc(&b->d_block_img, block_img.size() * sizeof(int));
    if (e == hipSuccess && !tb_block_img.empty()) e = hipMalloc(&b->d_tb_block_img, tb_block_img.size() * sizeof(int));
    if (e != hipSuccess) return fail(PCA_ENOMEM, "batch: allocation failed");
    if (!block_img.empty())
        e = hipMemcpyAsync(b->d_block_img, block_img.data(), block_img.size() * sizeof(int), hipMemcpyHostToDevice,
                           s);
    if (e == hipSuccess && !tb_block_img.empty())
        e = hipMemcpyAsync(b->d_tb_block_img, tb_block_img.data(), tb_block_img.size() * sizeof(int),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_desc, b->desc.data(), b->desc.size() * sizeof(pcak::ImageDesc), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(s);  // the first copy reads block_img, freed on return
        return hip_fail(e, "batch: configuration upload");
    }
    b->cfg = c;
    b->total_blocks = base;
    b->tb_blocks = (int)tb_block_img.size();
    b->tb_lds = tb_lds;
    drop_graphs(b);
    return PCA_OK;
}

// Initial states from the level-unit observations, zeroed accumulators, sweep index 0.
int reset_run(pca_batch *b, const float *const *obs, hipStream_t s)
{
    for (int i = 0; i < b->n; ++i) {
        const pca_params &p = b->p[i];
        pcak::ImageDesc &d = b->desc[i];
        const size_t N = (size_t)d.H * d.W;
        hipError_t e = hipMemsetAsync(d.sum, 0, N * sizeof(uint32_t), s);
        if (e == hipSuccess && d.hist) e = hipMemsetAsync(d.hist, 0, N * d.hist_words * sizeof(uint32_t), s);
        if (e == hipSuccess) {
            pcak::InitArgs a{};
            a.obs = obs ? obs[i] : nullptr;
            a.gp = const_cast<float *>(d.gp);
            a.x = d.x0;
            a.N = (int64_t)N;
            a.Cp = d.Cp;
            a.L = p.levels;
            a.mode = p.init_mode;
            a.vmin = (double)p.vmin;
            a.scale = level_scale(p);
            a.key0 = d.key0;
            a.key1 = d.key1;
            e = pcak::launch_init(a, s);
        }
        if (e != hipSuccess) return hip_fail(e, "batch: initialisation");
        b->count[i] = 0;
        b->tallies[i] = 0;
        d.t = 0;
        d.t_end = 0xFFFFFFFFu;
    }
    hipError_t e = hipMemcpyAsync(b->d_desc, b->desc.data(), b->desc.size() * sizeof(pcak::ImageDesc),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "batch: initialisation");
    b->t = 0;
    return PCA_OK;
}

void release(pca_batch *b)
{
    drop_graphs(b);
    for (auto &d : b->desc) {
        (void)hipFree(const_cast<float *>(d.gp));
        (void)hipFree(d.x0);
        (void)hipFree(d.x1);
        (void)hipFree(d.sum);
        (void)hipFree(d.hist);
    }
    (void)hipFree(b->d_desc);
    (void)hipFree(b->d_beta);
    (void)hipFree(b->d_block_img);
    (void)hipFree(b->d_tb_block_img);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
}

int check_guards(const pca_batch *b, int32_t n, std::vector<int64_t> *add_count, std::vector<int64_t> *add_tally)
{
    add_count->assign(b->n, 0);
    add_tally->assign(b->n, 0);
    for (int i = 0; i < b->n; ++i) {
        const pca_params &p = b->p[i];
        int64_t sweeps = 0;
        pcak::accumulating_sweeps(b->t, n, p.burn_in, p.tally_stride, &sweeps, &(*add_tally)[i]);
        (*add_count)[i] = sweeps * p.chains;
        if ((double)(b->count[i] + (*add_count)[i]) * (double)(p.levels - 1) > 4294967295.0)
            return fail(PCA_ESTATE, "lattice %d: the level sum could overflow 32 bits", i);
        if ((b->tallies[i] + (*add_tally)[i]) * (int64_t)p.chains > 65535)
            return fail(PCA_ESTATE, "lattice %d: a histogram counter could overflow 16 bits", i);
    }
    if (b->t + n > 0xFFFFFFFFll) return fail(PCA_ESTATE, "sweep index overflow");
    return PCA_OK;
}

int enqueue_eager(pca_batch *b, int32_t n, hipStream_t s)
{
    for (int32_t i = 0; i < n;) {
        // the multi-sweep lattices advance an odd number of sweeps per launch: 7, or what
        // is left split into odd parts
        const int32_t left = n - i;
        const int32_t S = b->tb_blocks == 0 ? 1 : left >= pcak::kTbBatchSweeps ? pcak::kTbBatchSweeps
                                                              : (left & 1) ? left : left - 1;
        if (b->tb_blocks > 0) {
            pcak::TbBatchLaunch tl{b->d_desc, b->d_tb_block_img, (uint32_t)i, S};
            const hipError_t e = pcak::launch_tb_batch(tl, b->tb_blocks, b->cfg.G, b->nbr, b->tb_lds, s);
            if (e != hipSuccess) return hip_fail(e, "batch sweep");
        }
        for (int32_t j = i; j < i + S && b->total_blocks > 0; ++j) {
            pcak::BatchLaunch bl{b->d_desc, b->d_block_img, (uint32_t)j};
            const hipError_t e = pcak::launch_batch_sweep(bl, b->total_blocks, b->cfg.G, b->cfg.share,
                                                          b->cfg.tiled == 1 ? 1 : 0, b->nbr, b->inr, s);
            if (e != hipSuccess) return hip_fail(e, "batch sweep");
        }
        i += S;
    }
    hipError_t e = pcak::launch_advance(b->d_desc, b->n, (uint32_t)n, s);
    return e == hipSuccess ? PCA_OK : hip_fail(e, "batch sweep");
}

// Device sweep index of every lattice for an autotuner trial: 0 (burn-in sweeps) or its
// burn-in length (accumulating sweeps, with tallies).  The run is re-initialised afterwards.
int set_trial_index(pca_batch *b, bool accumulating, hipStream_t s)
{
    for (int i = 0; i < b->n; ++i) {
        b->desc[i].t = accumulating ? (uint32_t)b->p[i].burn_in : 0u;
        b->desc[i].t_end = 0xFFFFFFFFu;
    }
    hipError_t e = hipMemcpyAsync(b->d_desc, b->desc.data(), b->desc.size() * sizeof(pcak::ImageDesc),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? PCA_OK : hip_fail(e, "batch autotune: trial set-up");
}

hipGraphExec_t graph_for(pca_batch *b, int32_t n, int *rc)
{
    auto it = b->graphs.find(n);
    if (it != b->graphs.end()) return it->second;
    hipGraph_t g = nullptr;
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        *rc = hip_fail(e, "batch: graph capture");
        return nullptr;
    }
    int erc = enqueue_eager(b, n, b->cap);
    e = hipStreamEndCapture(b->cap, &g);
    if (erc != PCA_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        *rc = erc != PCA_OK ? erc : hip_fail(e, "batch: graph capture");
        return nullptr;
    }
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        *rc = hip_fail(e, "batch: graph instantiation");
        return nullptr;
    }
    b->graphs[n] = ex;
    return ex;
}

}  // namespace

extern "C" {

int pca_batch_init(const pca_params *params, const float *const *obs_dev, int32_t n, void *stream, pca_batch **out)
{
    if (!out) return fail(PCA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!params || !obs_dev || n < 1) return fail(PCA_EINVAL, "need n >= 1 parameter sets and observations");
    for (int i = 0; i < n; ++i) {
        int rc = pcak::validate_params(&params[i]);
        if (rc) return rc;
        if (!obs_dev[i]) return fail(PCA_EINVAL, "obs_dev[%d] is NULL", i);
        if (params[i].neighbourhood != params[0].neighbourhood)
            return fail(PCA_EINVAL, "all lattices of a batch must use the same neighbourhood");
        if ((params[i].inertia != 0) != (params[0].inertia != 0))
            return fail(PCA_EINVAL, "a batch cannot mix the indicator inertia with the L1/L2 norms");
    }
    hipStream_t s = (hipStream_t)stream;
    pca_batch *b = new (std::nothrow) pca_batch();
    if (!b) return fail(PCA_ENOMEM, "batch: host allocation failed");
    b->n = n;
    b->nbr = params[0].neighbourhood;
    b->inr = params[0].inertia != 0;
    b->last = s;
    std::vector<double> betas;
    std::vector<size_t> beta_off;
    try {
        b->p.assign(params, params + n);
        b->count.assign(n, 0);
        b->tallies.assign(n, 0);
        b->desc.resize(n);
        beta_off.resize(n);
        for (int i = 0; i < n; ++i) {
            beta_off[i] = betas.size();
            for (int j = 0; j < params[i].beta_len; ++j) betas.push_back((double)params[i].beta[j]);
            b->p[i].beta = nullptr;
        }
    } catch (const std::bad_alloc &) {
        release(b);
        return fail(PCA_ENOMEM, "batch: host allocation failed");
    }
    hipError_t e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&b->d_desc, n * sizeof(pcak::ImageDesc));
    if (e == hipSuccess && !betas.empty()) e = hipMalloc(&b->d_beta, betas.size() * sizeof(double));
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        const pca_params &p = params[i];
        pcak::ImageDesc &d = b->desc[i];
        d.H = p.height;
        d.W = p.width;
        d.L = p.levels;
        d.C = p.chains;
        d.Cp = pcak::chain_slots(p.chains);
        d.T = p.prior == PCA_PRIOR_POTTS ? 1 : (p.trunc < p.levels - 1 ? p.trunc : p.levels - 1);
        d.hist_words = (p.levels + 1) / 2;
        d.burn_in = p.burn_in;
        d.tally_stride = p.tally_stride;
        d.J = (double)p.J;
        d.q = (double)p.q;
        d.kappa = p.prior == PCA_PRIOR_POTTS ? 2.0 : 1.0;
        d.inertia = p.inertia;
        d.sigma_s = (double)p.sigma * level_scale(p);
        d.key0 = (uint32_t)p.seed;
        d.key1 = (uint32_t)(p.seed >> 32);
        d.beta_len = p.beta_len;
        d.beta = p.beta_len > 0 ? b->d_beta + beta_off[i] : nullptr;
        const size_t N = (size_t)d.H * d.W;
        float *gp = nullptr;
        e = hipMalloc(&gp, N * sizeof(float));
        d.gp = gp;
        if (e == hipSuccess) e = hipMalloc(&d.x0, N * d.Cp);
        if (e == hipSuccess) e = hipMalloc(&d.x1, N * d.Cp);
        if (e == hipSuccess) e = hipMalloc(&d.sum, N * sizeof(uint32_t));
        if (e == hipSuccess && p.tally_stride > 0) e = hipMalloc(&d.hist, N * d.hist_words * sizeof(uint32_t));
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        release(b);
        return fail(PCA_ENOMEM, "batch: device allocation failed");
    }
    if (!betas.empty()) {
        e = hipMemcpyAsync(b->d_beta, betas.data(), betas.size() * sizeof(double), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(s);  // the copy reads betas, freed on return
            release(b);
            return hip_fail(e, "batch: upload");
        }
    }
    LaunchConfig c{1, 1, 0};
    for (const auto &cand : candidates(b)) {  // largest chain group and sharing first
        c = cand;
        break;
    }
    int rc = apply_config(b, c, s);
    if (rc == PCA_OK) rc = reset_run(b, obs_dev, s);
    if (rc != PCA_OK) {
        (void)hipStreamSynchronize(s);
        release(b);
        return rc;
    }
    *out = b;
    return PCA_OK;
}

int pca_batch_autotune(pca_batch *b, int32_t trial_sweeps, void *stream, float *best_ms)
{
    if (!b) return fail(PCA_EINVAL, "batch is NULL");
    if (trial_sweeps < 1 || trial_sweeps > 64) return fail(PCA_EINVAL, "trial_sweeps must be in [1, 64]");
    hipStream_t s = (hipStream_t)stream;
    b->last = s;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(PCA_EDEVICE, "batch autotune: event creation failed");
    }
    const std::vector<LaunchConfig> cands = candidates(b);
    std::vector<float> score(cands.size(), 1e30f);
    int rc = PCA_OK;
    // two rounds over the candidates, each timing burn-in and accumulating sweeps; a
    // candidate keeps its best round
    for (int round = 0; round < 2 && rc == PCA_OK; ++round) {
        for (size_t ci = 0; ci < cands.size() && rc == PCA_OK; ++ci) {
            rc = apply_config(b, cands[ci], s);
            float total = 0.0f;
            for (int phase = 0; phase < 2 && rc == PCA_OK; ++phase) {
                rc = set_trial_index(b, phase == 1, s);
                if (rc == PCA_OK) rc = enqueue_eager(b, 1, s);  // warm-up
                if (rc) break;
                (void)hipEventRecord(e0, s);
                rc = enqueue_eager(b, trial_sweeps, s);
                (void)hipEventRecord(e1, s);
                if (rc) break;
                float ms = 0.0f;
                if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                    rc = fail(PCA_EDEVICE, "batch autotune: timing failed");
                total += ms;
            }
            if (rc == PCA_OK) score[ci] = std::min(score[ci], total);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    size_t best = 0;
    for (size_t ci = 1; ci < cands.size(); ++ci)
        if (score[ci] < score[best]) best = ci;
    if (rc == PCA_OK) rc = apply_config(b, cands[best], s);
    if (rc == PCA_OK) rc = reset_run(b, nullptr, s);
    if (rc == PCA_OK && hipStreamSynchronize(s) != hipSuccess) rc = fail(PCA_EDEVICE, "batch autotune: reset failed");
    if (best_ms) *best_ms = score[best] / (float)(2 * trial_sweeps);
    return rc;
}

int pca_batch_config(const pca_batch *b, int32_t *chains_per_thread, int32_t *share, int32_t *tiled)
{
    if (!b) return fail(PCA_EINVAL, "batch is NULL");
    if (chains_per_thread) *chains_per_thread = b->cfg.G;
    if (share) *share = b->cfg.share;
    if (tiled) *tiled = b->cfg.tiled;
    return PCA_OK;
}

int pca_batch_set_config(pca_batch *b, int32_t chains_per_thread, int32_t share, int32_t tiled, void *stream)
{
    if (!b) return fail(PCA_EINVAL, "batch is NULL");
    LaunchConfig c{chains_per_thread, share, tiled};
    if ((c.G != 1 && c.G != 2 && c.G != 4) || (c.share != 1 && c.share != 2 && c.share != 4) || !config_valid(b, c))
        return fail(PCA_EINVAL, "launch configuration not valid for this batch");
    b->last = (hipStream_t)stream;
    return apply_config(b, c, (hipStream_t)stream);
}

int pca_batch_sweep(pca_batch *b, int32_t n, void *stream)
{
    if (!b) return fail(PCA_EINVAL, "batch is NULL");
    if (n < 0) return fail(PCA_EINVAL, "n must be >= 0");
    if (n == 0) return PCA_OK;
    std::vector<int64_t> add_count, add_tally;
    int rc = check_guards(b, n, &add_count, &add_tally);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    b->last = s;
    const int32_t full = n / kGraphSweeps, rest = n % kGraphSweeps;
    hipGraphExec_t ex_full = full > 0 ? graph_for(b, kGraphSweeps, &rc) : nullptr;
    if (full > 0 && !ex_full) return rc;
    hipGraphExec_t ex_rest = rest > 0 ? graph_for(b, rest, &rc) : nullptr;
    if (rest > 0 && !ex_rest) return rc;
    int32_t swept = 0;  // sweeps of the graphs launched (each advances the device sweep index)
    hipError_t e = hipSuccess;
    for (int32_t i = 0; i <= full; ++i) {
        hipGraphExec_t ex = i < full ? ex_full : ex_rest;
        if (!ex) break;
        e = hipGraphLaunch(ex, s);
        if (e != hipSuccess) break;
        swept += i < full ? kGraphSweeps : rest;
    }
    if (swept < n) {  // a launch failed: the graphs before it still count
        for (int i = 0; i < b->n; ++i) {
            const pca_params &p = b->p[i];
            int64_t sweeps = 0, tallies = 0;
            pcak::accumulating_sweeps(b->t, swept, p.burn_in, p.tally_stride, &sweeps, &tallies);
            b->count[i] += sweeps * p.chains;
            b->tallies[i] += tallies;
        }
        b->t += swept;
        return hip_fail(e, "batch sweep: graph launch");
    }
    b->t += n;
    for (int i = 0; i < b->n; ++i) {
        b->count[i] += add_count[i];
        b->tallies[i] += add_tally[i];
    }
    return PCA_OK;
}

int pca_batch_posterior_mean(pca_batch *b, int32_t i, float *out_dev, void *stream)
{
    if (!b || i < 0 || i >= b->n || !out_dev) return fail(PCA_EINVAL, "bad batch, index or output");
    if (b->count[i] <= 0) return fail(PCA_ESTATE, "no accumulated sweeps");
    const pca_params &p = b->p[i];
    const pcak::ImageDesc &d = b->desc[i];
    const double delta = ((double)p.vmax - (double)p.vmin) / (double)(p.levels - 1);
    b->last = (hipStream_t)stream;
    hipError_t e = pcak::launch_mean(d.sum, out_dev, (int64_t)d.H * d.W, b->count[i], (double)p.vmin, delta,
                                     (hipStream_t)stream);
    return e == hipSuccess ? PCA_OK : hip_fail(e, "batch posterior mean");
}

int pca_batch_marginal_map(pca_batch *b, int32_t i, uint8_t *out_dev, void *stream)
{
    if (!b || i < 0 || i >= b->n || !out_dev) return fail(PCA_EINVAL, "bad batch, index or output");
    const pcak::ImageDesc &d = b->desc[i];
    if (!d.hist) return fail(PCA_ESTATE, "histogram disabled (tally_stride = 0)");
    if (b->tallies[i] <= 0) return fail(PCA_ESTATE, "no tally sweeps yet");
    b->last = (hipStream_t)stream;
    hipError_t e = pcak::launch_mpm(d.hist, out_dev, (int64_t)d.H * d.W, d.L, d.hist_words, (hipStream_t)stream);
    return e == hipSuccess ? PCA_OK : hip_fail(e, "batch marginal map");
}

int pca_batch_get_state(pca_batch *b, int32_t i, uint8_t *out_dev, void *stream)
{
    if (!b || i < 0 || i >= b->n || !out_dev) return fail(PCA_EINVAL, "bad batch, index or output");
    const pcak::ImageDesc &d = b->desc[i];
    b->last = (hipStream_t)stream;
    hipError_t e = pcak::launch_get_state((b->t & 1) ? d.x1 : d.x0, out_dev, (int64_t)d.H * d.W, d.C, d.Cp,
                                          (hipStream_t)stream);
    return e == hipSuccess ? PCA_OK : hip_fail(e, "batch get state");
}

int pca_batch_stats(const pca_batch *b, int32_t i, int64_t *sweep, int64_t *count, int64_t *tallies)
{
    if (!b || i < 0 || i >= b->n) return fail(PCA_EINVAL, "bad batch or index");
    if (sweep) *sweep = b->t;
    if (count) *count = b->count[i];
    if (tallies) *tallies = b->tallies[i];
    return PCA_OK;
}

int pca_batch_sync(pca_batch *b)
{
    if (!b) return fail(PCA_EINVAL, "batch is NULL");
    hipError_t e = hipStreamSynchronize(b->last);
    if (e == hipSuccess) e = hipGetLastError();
    return e == hipSuccess ? PCA_OK : hip_fail(e, "pca_batch_sync");
}

int pca_batch_destroy(pca_batch *b)
{
    if (!b) return PCA_OK;
    hipError_t e = hipStreamSynchronize(b->last);
    release(b);
    return e == hipSuccess ? PCA_OK : hip_fail(e, "pca_batch_destroy");
}

}  // extern "C"
