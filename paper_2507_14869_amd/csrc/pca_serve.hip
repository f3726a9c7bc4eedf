// C ABI of the request server (declared in include/pca.h): continuous batching of
// denoising requests.  Requests wait in a FIFO queue until their device footprint fits
// the memory budget and a slot is free; admitted requests keep their chain states on the
// device.  A step gives every admitted request at least one sweep and spends the rest of
// a GPU-time budget half on the requests with the least remaining work and half on the
// oldest ones; the sweeps run as
// batched kernel launches, launch i covering every request that still advances at i,
// each at its own sweep index.  A finished request is read out (posterior mean, marginal
// mode, last states) to host memory and its device memory is released at once, so queued
// requests can be admitted at the next step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "pca.h"
#include "pca_internal.h"

namespace {

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

enum { QUEUED = 0, ACTIVE = 1, DONE = 2, FAILED = 3 };

struct Request {
    int64_t id = 0;
    pca_params p{};
    std::vector<float> beta;
    std::vector<float> obs;      // host copy until the step that admits it has finished
    std::vector<double> beta_d;  // beta in double, staged for the upload at admission
    int32_t sweeps = 0;
    size_t footprint = 0;
    pcak::ImageDesc d{};
    double *d_beta = nullptr;
    float *d_obs = nullptr;
    int64_t t = 0, count = 0, tallies = 0;
    int status = QUEUED;
    int err_code = PCA_OK;  // FAILED: the error that ended the request, and its message
    std::string err_msg;
    std::vector<float> mean;
    std::vector<uint8_t> mpm, state;
};

// Work of one sweep of a request, in level evaluations (plus a per-site allowance).
double units_per_sweep(const pca_params &p)
{
    return (double)p.height * p.width * pcak::chain_slots(p.chains) * (p.levels + 16);
}

size_t footprint_of(const pca_params &p)
{
    const size_t N = (size_t)p.height * p.width;
    const size_t Cp = (size_t)pcak::chain_slots(p.chains);
    size_t b = N * 4 /* gp */ + 2 * N * Cp /* states */ + N * 4 /* sum */ + N * 4 /* obs staging */;
    if (p.tally_stride > 0) b += N * (size_t)((p.levels + 1) / 2) * 4;
    return b + (size_t)p.beta_len * 8 + 4096;
}

}  // namespace

struct pca_server {
    size_t budget = 0, used = 0;
    int max_active = 0, sweeps_per_step = 0;
    double step_ms = 20.0;        // GPU time a step aims at
    double ns_per_unit = 2.5e-4;  // measured cost of one unit of work (a level evaluation)
    int64_t next_id = 1;
    std::deque<Request *> queue;
    std::vector<Request *> active;
    std::map<int64_t, Request *> all;
    std::vector<int64_t> completed;
    pcak::ImageDesc *d_desc = nullptr;
    int *d_block_img = nullptr;
    size_t block_cap = 0;
    int64_t steps = 0, sweeps_launched = 0;
    double max_backlog_s = 0.0;  // shedding limit on the predicted wait; 0 = none
    int64_t shed = 0;            // submissions refused by it
    hipStream_t last = nullptr;
};

namespace {

void free_device(Request *r)
{
    (void)hipFree(const_cast<float *>(r->d.gp));
    (void)hipFree(r->d.x0);
    (void)hipFree(r->d.x1);
    (void)hipFree(r->d.sum);
    (void)hipFree(r->d.hist);
    (void)hipFree(r->d_beta);
    (void)hipFree(r->d_obs);
    r->d.gp = nullptr;
    r->d.x0 = r->d.x1 = nullptr;
    r->d.sum = r->d.hist = nullptr;
    r->d_beta = nullptr;
    r->d_obs = nullptr;
}

// Allocates the request's device buffers, uploads its observation and initialises it.
int admit(pca_server *sv, Request *r, hipStream_t s)
{
    const pca_params &p = r->p;
    pcak::ImageDesc &d = r->d;
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
    d.beta_len = (int)r->beta.size();
    const size_t N = (size_t)d.H * d.W;
    float *gp = nullptr;
    hipError_t e = pcak::fault_injected("admit", r->id) ? hipErrorOutOfMemory : hipMalloc(&gp, N * sizeof(float));
    d.gp = gp;
    if (e == hipSuccess) e = hipMalloc(&r->d_obs, N * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&d.x0, N * d.Cp);
    if (e == hipSuccess) e = hipMalloc(&d.x1, N * d.Cp);
    if (e == hipSuccess) e = hipMalloc(&d.sum, N * sizeof(uint32_t));
    if (e == hipSuccess && p.tally_stride > 0) e = hipMalloc(&d.hist, N * d.hist_words * sizeof(uint32_t));
    if (e == hipSuccess && !r->beta.empty()) e = hipMalloc(&r->d_beta, r->beta.size() * sizeof(double));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_device(r);
        return fail(PCA_ENOMEM, "server: device allocation failed for request %lld", (long long)r->id);
    }
    r->beta_d.assign(r->beta.begin(), r->beta.end());
    d.beta = r->d_beta;
    e = hipMemcpyAsync(r->d_obs, r->obs.data(), N * sizeof(float), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !r->beta_d.empty())
        e = hipMemcpyAsync(r->d_beta, r->beta_d.data(), r->beta_d.size() * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(d.sum, 0, N * sizeof(uint32_t), s);
    if (e == hipSuccess && d.hist) e = hipMemsetAsync(d.hist, 0, N * d.hist_words * sizeof(uint32_t), s);
    if (e == hipSuccess) {
        pcak::InitArgs a{};
        a.obs = r->d_obs;
        a.gp = gp;
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
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(s);
        free_device(r);
        return hip_fail(e, "server: admission");
    }
    // the host copies and the device staging of the observation stay until the step that
    // admitted the request has synchronised (release_staging)
    r->status = ACTIVE;
    sv->used += r->footprint;
    return PCA_OK;
}

// Posterior mean, marginal mode and last states to host memory (stream-ordered).
int read_out(Request *r, hipStream_t s)
{
    const pcak::ImageDesc &d = r->d;
    const int64_t N = (int64_t)d.H * d.W;
    const pca_params &p = r->p;
    if (pcak::fault_injected("readout", r->id))
        return fail(PCA_ENOMEM, "server: host allocation for the results of request %lld failed", (long long)r->id);
    try {
        r->mean.resize((size_t)N);
        r->state.resize((size_t)N * d.C);
        if (d.hist && r->tallies > 0) r->mpm.resize((size_t)N);
    } catch (const std::bad_alloc &) {
        return fail(PCA_ENOMEM, "server: host allocation for the results failed");
    }
    uint8_t *cur = (r->t & 1) ? d.x1 : d.x0;
    uint8_t *spare = (r->t & 1) ? d.x0 : d.x1;  // free now: holds [C][N] or [N] scratch
    float *mean_dev = const_cast<float *>(d.gp);  // the observation is no longer needed
    hipError_t e = hipSuccess;
    if (r->count > 0) {
        const double delta = ((double)p.vmax - (double)p.vmin) / (double)(p.levels - 1);
        e = pcak::launch_mean(d.sum, mean_dev, N, r->count, (double)p.vmin, delta, s);
        if (e == hipSuccess) e = hipMemcpyAsync(r->mean.data(), mean_dev, N * sizeof(float), hipMemcpyDeviceToHost, s);
    } else {
        std::fill(r->mean.begin(), r->mean.end(), 0.0f);
    }
    if (e == hipSuccess) e = pcak::launch_get_state(cur, spare, N, d.C, d.Cp, s);
    if (e == hipSuccess) e = hipMemcpyAsync(r->state.data(), spare, (size_t)N * d.C, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && d.hist && r->tallies > 0) {
        e = pcak::launch_mpm(d.hist, spare, N, d.L, d.hist_words, s);
        if (e == hipSuccess) e = hipMemcpyAsync(r->mpm.data(), spare, (size_t)N, hipMemcpyDeviceToHost, s);
    }
    return e == hipSuccess ? PCA_OK : hip_fail(e, "server: read-out");
}

// After the admitting step's synchronisation: the uploads and the init kernel are done.
void release_staging(Request *r)
{
    std::vector<float>().swap(r->obs);
    std::vector<double>().swap(r->beta_d);
    (void)hipFree(r->d_obs);
    r->d_obs = nullptr;
}

// Ends a request with an error: its device memory (if any) is released, its host copies
// dropped, and it is reported among the completed requests with status FAILED;
// pca_server_result then returns the error.
void fail_request(pca_server *sv, Request *r, int code, const char *msg);

// Remaining work of the accepted requests (admitted and queued), in cost-model units.
double backlog_units(const pca_server *sv)
{
    double u = 0.0;
    for (const auto *r : sv->active) u += (double)(r->sweeps - r->t) * units_per_sweep(r->p);
    for (const auto *r : sv->queue) u += (double)(r->sweeps - r->t) * units_per_sweep(r->p);
    return u;
}

// The two timing events of a step, destroyed on every return path.
// Waits for the stream when a step returns, on every path, so that no copy the step
// enqueued from host memory (its own vectors, the staging of admitted requests) is still
// pending once the call has returned.
struct StreamDrain {
    hipStream_t s;
    ~StreamDrain() { (void)hipStreamSynchronize(s); }
};

// Releases the staging copies of the requests a step admitted, on every return path; declared
// before the step's StreamDrain, so it runs after the drain has waited for their uploads.
struct StagingRelease {
    const std::vector<Request *> &admitted;
    ~StagingRelease()
    {
        for (auto *r : admitted) release_staging(r);
    }
};

struct StepEvents {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool ok = false;
    StepEvents() { ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess; }
    ~StepEvents()
    {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

void fail_request(pca_server *sv, Request *r, int code, const char *msg)
{
    free_device(r);
    if (r->status == ACTIVE) sv->used -= r->footprint;
    r->status = FAILED;
    r->err_code = code;
    try {
        r->err_msg = msg;
    } catch (const std::bad_alloc &) {
    }
    std::vector<float>().swap(r->obs);
    std::vector<double>().swap(r->beta_d);
    std::vector<float>().swap(r->mean);
    std::vector<uint8_t>().swap(r->mpm);
    std::vector<uint8_t>().swap(r->state);
    try {
        sv->completed.push_back(r->id);
    } catch (const std::bad_alloc &) {
    }
}

int ensure_capacity(pca_server *sv, size_t blocks)
{
    if (blocks <= sv->block_cap) return PCA_OK;
    (void)hipFree(sv->d_block_img);
    sv->d_block_img = nullptr;
    size_t cap = blocks + blocks / 2 + 1024;
    if (hipMalloc(&sv->d_block_img, cap * sizeof(int)) != hipSuccess) {
        sv->block_cap = 0;
        return fail(PCA_ENOMEM, "server: allocation failed");
    }
    sv->block_cap = cap;
    return PCA_OK;
}

}  // namespace

extern "C" {

int pca_server_create(uint64_t hbm_budget_bytes, int32_t max_active, int32_t sweeps_per_step, float step_ms,
                      pca_server **out)
{
    if (!out) return fail(PCA_EINVAL, "out is NULL");
    *out = nullptr;
    if (hbm_budget_bytes == 0 || max_active < 1 || max_active > 4096 || sweeps_per_step < 1 || !(step_ms > 0.0f))
        return fail(PCA_EINVAL, "need a positive budget, 1..4096 active requests, sweeps_per_step >= 1 and "
                                "step_ms > 0");
    pca_server *sv = new (std::nothrow) pca_server();
    if (!sv) return fail(PCA_ENOMEM, "server: host allocation failed");
    sv->budget = (size_t)hbm_budget_bytes;
    sv->max_active = max_active;
    sv->sweeps_per_step = sweeps_per_step;
    sv->step_ms = step_ms;
    if (hipMalloc(&sv->d_desc, (size_t)max_active * sizeof(pcak::ImageDesc)) != hipSuccess) {
        delete sv;
        return fail(PCA_ENOMEM, "server: allocation failed");
    }
    *out = sv;
    return PCA_OK;
}

int pca_server_submit(pca_server *sv, const pca_params *params, const float *obs_host, int32_t sweeps,
                      int64_t *request_id)
{
    if (!sv || !params || !obs_host || !request_id) return fail(PCA_EINVAL, "NULL argument");
    int rc = pcak::validate_params(params);
    if (rc) return rc;
    if (sweeps < 1) return fail(PCA_EINVAL, "sweeps must be >= 1");
    const pca_params &p = *params;
    const int64_t acc = sweeps > p.burn_in ? sweeps - p.burn_in : 0;
    if ((double)acc * p.chains * (double)(p.levels - 1) > 4294967295.0)
        return fail(PCA_EINVAL, "the level sum of this request could overflow 32 bits");
    if (p.tally_stride > 0 && ((acc + p.tally_stride - 1) / p.tally_stride) * (int64_t)p.chains > 65535)
        return fail(PCA_EINVAL, "a histogram counter of this request could overflow 16 bits");
    if (footprint_of(p) > sv->budget) return fail(PCA_EINVAL, "request needs more device memory than the whole budget");
    if (sv->max_backlog_s > 0.0) {  // load shedding: the wait predicted by the cost model
        const double wait_s = backlog_units(sv) * sv->ns_per_unit * 1e-9;
        if (wait_s > sv->max_backlog_s) {
            sv->shed += 1;
            return fail(PCA_EBUSY, "server: predicted wait %.3f s exceeds the shedding limit %.3f s", wait_s,
                        sv->max_backlog_s);
        }
    }
    Request *r = new (std::nothrow) Request();
    if (!r) return fail(PCA_ENOMEM, "server: host allocation failed");
    r->p = p;
    r->p.beta = nullptr;
    r->sweeps = sweeps;
    r->footprint = footprint_of(p);
    r->id = sv->next_id;
    try {
        if (p.beta_len > 0) r->beta.assign(p.beta, p.beta + p.beta_len);
        r->obs.assign(obs_host, obs_host + (size_t)p.height * p.width);
        sv->all[r->id] = r;
        try {
            sv->queue.push_back(r);
        } catch (const std::bad_alloc &) {
            sv->all.erase(r->id);
            throw;
        }
    } catch (const std::bad_alloc &) {
        delete r;
        return fail(PCA_ENOMEM, "server: host allocation failed");
    }
    sv->next_id += 1;
    *request_id = r->id;
    return PCA_OK;
}

int pca_server_set_shedding(pca_server *sv, double max_backlog_s)
{
    if (!sv) return fail(PCA_EINVAL, "server is NULL");
    if (!(max_backlog_s >= 0.0)) return fail(PCA_EINVAL, "max_backlog_s must be >= 0");
    sv->max_backlog_s = max_backlog_s;
    return PCA_OK;
}

int pca_server_shed_count(const pca_server *sv, int64_t *shed)
{
    if (!sv || !shed) return fail(PCA_EINVAL, "NULL argument");
    *shed = sv->shed;
    return PCA_OK;
}

int pca_server_step(pca_server *sv, void *stream, int32_t *n_completed)
{
    if (!sv) return fail(PCA_EINVAL, "server is NULL");
    hipStream_t s = (hipStream_t)stream;
    sv->last = s;
    if (n_completed) *n_completed = 0;
    std::vector<pcak::ImageDesc> desc;
    std::vector<int> block_img;
    std::vector<int> blocks_upto;  // blocks of the first j requests
    std::vector<Request *> admitted;
    const StagingRelease staging{admitted};  // runs after the drain below
    const StreamDrain drain{s};    // declared after the vectors: runs before they are freed
    // 1. admission, first come first served, by device footprint and free slots (no
    //    synchronisation here: the uploads and initialisations are stream-ordered before
    //    the step's sweeps).  The budget is the caller's; the device may hold less.  If a
    //    request's allocation fails while others hold device memory, it stays at the head
    //    of the queue until they finish; if it fails with nothing else admitted, waiting
    //    cannot help and the request fails.  Either way the admitted requests advance.
    while (!sv->queue.empty() && (int)sv->active.size() < sv->max_active &&
           sv->used + sv->queue.front()->footprint <= sv->budget) {
        Request *r = sv->queue.front();
        int rc = admit(sv, r, s);
        if (rc != PCA_OK) {
            if (!sv->active.empty()) break;
            sv->queue.pop_front();
            fail_request(sv, r, rc, pca_last_error());
            continue;
        }
        sv->queue.pop_front();
        sv->active.push_back(r);
        admitted.push_back(r);
    }
    // a request that reached its sweep count in a step that then failed (a device error
    // before its results were safely on the host) cannot be read out again
    for (size_t i = 0; i < sv->active.size();) {
        Request *r = sv->active[i];
        if (r->t < r->sweeps) {
            ++i;
            continue;
        }
        sv->active.erase(sv->active.begin() + (std::ptrdiff_t)i);
        fail_request(sv, r, PCA_EDEVICE, "an earlier step failed before this request's results were read out");
    }
    if (sv->active.empty()) return PCA_OK;
    // 2. sweeps per request this step: at least one each, then the rest of the step's
    //    GPU-time budget (below).
    // one launch runs one kernel: the requests sharing the oldest one's neighbourhood and
    // inertia form advance now, the others in a later step
    const int nbr = sv->active.front()->p.neighbourhood;
    const bool inr = sv->active.front()->p.inertia != 0;
    std::vector<Request *> cand;
    for (auto *r : sv->active)  // an active request has sweeps left: it finishes in the step that ends them
        if (r->p.neighbourhood == nbr && (r->p.inertia != 0) == inr && r->t < r->sweeps) cand.push_back(r);
    if (cand.empty()) return PCA_OK;
    if (cand.size() < sv->active.size())
        std::rotate(sv->active.begin(), sv->active.begin() + 1, sv->active.end());
    std::map<Request *, int64_t> k;
    double budget = sv->step_ms * 1e6 / sv->ns_per_unit;
    for (auto *r : cand) {
        k[r] = 1;
        budget -= units_per_sweep(r->p);
    }
    // half of what is left goes by least remaining work (short requests finish in one
    // step), the other half by age (the oldest request keeps a fixed share, so large
    // requests are not starved by a stream of small ones)
    auto grant = [&](std::vector<Request *> order, double share) {
        for (auto *r : order) {
            const double u = units_per_sweep(r->p);
            int64_t extra = std::min<int64_t>(r->sweeps - r->t, sv->sweeps_per_step) - k[r];
            extra = share > 0.0 ? std::min<int64_t>(extra, (int64_t)(share / u)) : 0;
            if (extra > 0) {
                k[r] += extra;
                share -= extra * u;
            }
        }
        return share > 0.0 ? share : 0.0;
    };
    std::vector<Request *> by_work(cand), by_age(cand);
    std::sort(by_work.begin(), by_work.end(), [](Request *a, Request *b) {
        const double ra = (a->sweeps - a->t) * units_per_sweep(a->p), rb = (b->sweeps - b->t) * units_per_sweep(b->p);
        return ra != rb ? ra < rb : a->id < b->id;
    });
    std::sort(by_age.begin(), by_age.end(), [](Request *a, Request *b) { return a->id < b->id; });
    if (budget > 0.0) {
        const double left = grant(by_work, budget / 2) + budget / 2;
        grant(by_age, left);
    }
    // launch configuration valid for every request of the step; row-major traversal (on the
    // serving trace it kept the GPU busy 2% less than 16-pixel-wide tiles)
    int G = 1, share = 1;
    for (int g : {4, 2}) {
        bool ok = true;
        for (auto *r : cand) ok = ok && r->d.Cp % g == 0;
        if (ok) {
            G = g;
            break;
        }
    }
    for (int sh : {4, 2}) {
        bool ok = true;
        for (auto *r : cand) ok = ok && (r->d.Cp / G) % sh == 0;
        if (ok) {
            share = sh;
            break;
        }
    }
    // lay the requests out by decreasing sweep count, so launch i covers a prefix of the grid
    std::vector<Request *> launched(cand);
    std::stable_sort(launched.begin(), launched.end(), [&](Request *a, Request *b) { return k[a] > k[b]; });
    double units = 0.0;
    for (auto *r : launched) {
        pcak::ImageDesc d = r->d;
        d.tpp = d.Cp / G;
        d.block_base = (int)block_img.size();
        const int64_t blocks = pcak::untiled_layout(d);
        d.t = (uint32_t)r->t;
        d.t_end = (uint32_t)(r->t + k[r]);
        if ((int64_t)block_img.size() + blocks > 0x7FFFFFFF) return fail(PCA_EINVAL, "server: step grid too large");
        block_img.insert(block_img.end(), (size_t)blocks, (int)desc.size());
        blocks_upto.push_back((int)block_img.size());
        desc.push_back(d);
        units += k[r] * units_per_sweep(r->p);
    }
    int rc = ensure_capacity(sv, block_img.size());
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(sv->d_desc, desc.data(), desc.size() * sizeof(pcak::ImageDesc),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(sv->d_block_img, block_img.data(), block_img.size() * sizeof(int), hipMemcpyHostToDevice, s);
    const int K = (int)k[launched.front()];
    StepEvents ev;
    if (ev.ok) (void)hipEventRecord(ev.e0, s);
    size_t j = launched.size();
    int enqueued = 0;  // launches enqueued (each advanced the requests it covered by one sweep)
    for (int i = 0; i < K && e == hipSuccess; ++i) {
        while (j > 0 && k[launched[j - 1]] <= i) --j;  // requests still advancing at launch i
        pcak::BatchLaunch bl{sv->d_desc, sv->d_block_img, (uint32_t)i};
        e = pcak::launch_batch_sweep(bl, blocks_upto[j - 1], G, share, 0, nbr, inr, s);
        if (e == hipSuccess) enqueued = i + 1;
    }
    if (ev.ok) (void)hipEventRecord(ev.e1, s);
    if (e != hipSuccess) {
        // the sweeps enqueued before the failure still count, so each request's sweep index
        // keeps matching its device state
        for (auto *r : launched) {
            const int64_t adv = std::min<int64_t>(k[r], enqueued);
            int64_t sweeps = 0, tallies = 0;
            pcak::accumulating_sweeps(r->t, adv, r->p.burn_in, r->p.tally_stride, &sweeps, &tallies);
            r->count += sweeps * r->p.chains;
            r->tallies += tallies;
            r->t += adv;
        }
        return hip_fail(e, "server: sweep launch");
    }
    sv->steps += 1;
    sv->sweeps_launched += K;
    // 3. bookkeeping of the sweeps each request took, read-out of finished requests; a
    //    request whose read-out fails ends with that error (its device memory is released
    //    after the step's synchronisation, like a finished request's)
    std::vector<Request *> finished;
    std::vector<std::pair<Request *, std::pair<int, std::string>>> broken;
    for (auto *r : launched) {
        const int64_t adv = k[r];
        int64_t sweeps = 0, tallies = 0;
        pcak::accumulating_sweeps(r->t, adv, r->p.burn_in, r->p.tally_stride, &sweeps, &tallies);
        r->count += sweeps * r->p.chains;
        r->tallies += tallies;
        r->t += adv;
        if (r->t >= r->sweeps) {
            rc = read_out(r, s);
            try {
                if (rc == PCA_OK) finished.push_back(r);
                else broken.push_back({r, {rc, std::string(pca_last_error())}});
            } catch (const std::bad_alloc &) {
                return fail(PCA_ENOMEM, "server: host allocation failed");
            }
        }
    }
    // the host vectors above are filled by asynchronous copies; the descriptor and block
    // uploads came from host vectors local to this call
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "server: step");
    if (ev.ok) {  // refine the cost model from the measured step
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ev.e0, ev.e1) == hipSuccess && units > 0.0 && ms > 0.0f)
            sv->ns_per_unit = 0.7 * sv->ns_per_unit + 0.3 * (ms * 1e6 / units);
    }
    for (auto *r : finished) {
        free_device(r);
        r->status = DONE;
        sv->used -= r->footprint;
        sv->active.erase(std::find(sv->active.begin(), sv->active.end(), r));
        sv->completed.push_back(r->id);
    }
    for (auto &b : broken) {
        sv->active.erase(std::find(sv->active.begin(), sv->active.end(), b.first));
        fail_request(sv, b.first, b.second.first, b.second.second.c_str());
    }
    if (n_completed) *n_completed = (int32_t)(finished.size() + broken.size());
    return PCA_OK;
}

int pca_server_completed(pca_server *sv, int64_t *ids, int32_t capacity, int32_t *n)
{
    if (!sv || !n || (capacity > 0 && !ids)) return fail(PCA_EINVAL, "NULL argument");
    const int32_t k = std::min<int32_t>(capacity, (int32_t)sv->completed.size());
    for (int32_t i = 0; i < k; ++i) ids[i] = sv->completed[i];
    sv->completed.erase(sv->completed.begin(), sv->completed.begin() + k);
    *n = k;
    return PCA_OK;
}

int pca_server_status(const pca_server *sv, int64_t id, int32_t *status, int64_t *sweep)
{
    if (!sv) return fail(PCA_EINVAL, "server is NULL");
    auto it = sv->all.find(id);
    if (it == sv->all.end()) return fail(PCA_EINVAL, "unknown request %lld", (long long)id);
    if (status) *status = it->second->status;
    if (sweep) *sweep = it->second->t;
    return PCA_OK;
}

int pca_server_result(pca_server *sv, int64_t id, float *mean_host, uint8_t *mpm_host, uint8_t *state_host)
{
    if (!sv) return fail(PCA_EINVAL, "server is NULL");
    auto it = sv->all.find(id);
    if (it == sv->all.end()) return fail(PCA_EINVAL, "unknown request %lld", (long long)id);
    Request *r = it->second;
    if (r->status == FAILED)
        return fail(r->err_code, "request %lld failed: %s", (long long)id, r->err_msg.c_str());
    if (r->status != DONE) return fail(PCA_ESTATE, "request %lld has not finished", (long long)id);
    if (mean_host && r->count <= 0) return fail(PCA_ESTATE, "request %lld accumulated no sweeps", (long long)id);
    if (mpm_host && r->mpm.empty()) return fail(PCA_ESTATE, "request %lld has no histogram", (long long)id);
    if (mean_host) std::copy(r->mean.begin(), r->mean.end(), mean_host);
    if (mpm_host) std::copy(r->mpm.begin(), r->mpm.end(), mpm_host);
    if (state_host) std::copy(r->state.begin(), r->state.end(), state_host);
    return PCA_OK;
}

int pca_server_release(pca_server *sv, int64_t id)
{
    if (!sv) return fail(PCA_EINVAL, "server is NULL");
    auto it = sv->all.find(id);
    if (it == sv->all.end()) return fail(PCA_EINVAL, "unknown request %lld", (long long)id);
    if (it->second->status != DONE && it->second->status != FAILED)
        return fail(PCA_ESTATE, "request %lld has not finished", (long long)id);
    delete it->second;
    sv->all.erase(it);
    return PCA_OK;
}

int pca_server_stats(const pca_server *sv, int32_t *queued, int32_t *active, uint64_t *used_bytes, int64_t *steps,
                     int64_t *sweeps_launched)
{
    if (!sv) return fail(PCA_EINVAL, "server is NULL");
    if (queued) *queued = (int32_t)sv->queue.size();
    if (active) *active = (int32_t)sv->active.size();
    if (used_bytes) *used_bytes = sv->used;
    if (steps) *steps = sv->steps;
    if (sweeps_launched) *sweeps_launched = sv->sweeps_launched;
    return PCA_OK;
}

int pca_server_destroy(pca_server *sv)
{
    if (!sv) return PCA_OK;
    hipError_t e = hipStreamSynchronize(sv->last);
    for (auto &kv : sv->all) {
        free_device(kv.second);
        delete kv.second;
    }
    (void)hipFree(sv->d_desc);
    (void)hipFree(sv->d_block_img);
    delete sv;
    return e == hipSuccess ? PCA_OK : hip_fail(e, "pca_server_destroy");
}

}  // extern "C"
