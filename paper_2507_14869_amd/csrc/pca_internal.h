// Internal interface between the host side of the C ABI (pca_api.hip, pca_batch.hip,
// pca_serve.hip) and the gfx950 kernels (pca_kernels*.hip, per-site code in pca_sweep.h).
// Not part of the public boundary; see include/pca.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pca.h"

namespace pcak {

constexpr int kBlock = 256;                 // threads per workgroup (4 wave64)
// A dispatch counts its grid in 32-bit work-items, so a sweep with more threads than this
// is split into launches of at most this many (a multiple of kBlock: every wave and lane
// quad then holds the same threads as in a single launch).
constexpr int64_t kMaxLaunchThreads = (int64_t)1 << 31;
constexpr int kMaxLaunchBlocks = (int)(kMaxLaunchThreads / kBlock);
constexpr int kMaxNeighbourStat = 8 * 255;  // largest S = sum_j min(|k-x_j|, T) over 8 neighbours
constexpr double kLog2e = 1.4426950408889634;
constexpr double kLn2 = 0.6931471805599453;

// Scalars of one sweep launch.  Doubles are the run parameters; the kernel derives its
// FP32 constants from them with a fixed operation order.
struct SweepArgs {
    const float *gp;      // [N] observation in level units
    const uint8_t *xin;   // [N][Cp] state at sweep t (chain-interleaved)
    uint8_t *xout;        // [N][Cp] state at sweep t+1
    uint32_t *sum;        // [N] level sums over chains and sweeps, or nullptr (not accumulated)
    uint32_t *hist;       // [N][hist_words] packed uint16 level counters, or nullptr
    int H, W, L, C, Cp;   // Cp = chains rounded up to the per-thread chain group
    int T;                // effective truncation (1 for Potts, min(trunc, L-1) otherwise)
    int hist_words;       // (L + 1) / 2
    double beta, J, q, kappa, sigma_s;  // kappa = 2 (Potts) or 1; sigma_s = sigma in level units
    uint32_t key0, key1;  // Philox key (seed split)
    uint32_t t;           // sweep index
    int inertia;          // inertia norm exponent: 0 (indicator, stay weight), 1 or 2
    int64_t blk0;         // global index of the launch's first workgroup (split sweeps)
    int patch;            // log2 of threads per pixel if pixels are laid out in 2-D patches, else -1
    int tiles_w;          // workgroup tiles per lattice row (patch layout)
};

// Thread layout of a single-lattice sweep.  With `patches` and 1, 2, 4, 8 or 16 threads
// per pixel the pixels of a wave form a near-square patch (8x8, 4x8, 4x4, 2x4 or 2x2) and
// the four waves of a workgroup a 2x2 arrangement of patches: the chains of nearby pixels
// have similar neighbour levels, so more 16-level blocks pass the wave-wide far test
// (measured on 2048x2048, L = 256, 16 chains: 2.76 against 2.94 ms per sweep).  Without
// that test (L <= 16) row-major order was as fast or faster, and it is the only order for
// other thread counts.
struct SweepLayout {
    int patch;       // log2(threads per pixel), or -1 for row-major
    int tiles_w;     // tiles per row (patch layout)
    int64_t blocks;  // workgroups of one sweep (fewer than 2^31)
};

inline SweepLayout sweep_layout(int H, int W, int tpp, bool patches)
{
    SweepLayout l{-1, 0, 0};
    for (int lg = 0; lg <= 4 && patches; ++lg) {
        if (tpp == (1 << lg)) l.patch = lg;
    }
    if (l.patch < 0) {
        l.blocks = ((int64_t)H * W * tpp + kBlock - 1) / kBlock;
        return l;
    }
    const int lp = 6 - l.patch, lr = lp >> 1, lc = lp - lr;  // wave patch 2^lr x 2^lc pixels
    const int th = 2 << lr, tw = 2 << lc;                     // workgroup tile
    l.tiles_w = (W + tw - 1) / tw;
    l.blocks = (int64_t)l.tiles_w * ((H + th - 1) / th);
    return l;
}

struct InitArgs {
    const float *obs;  // [N] value units, or nullptr to re-initialise from gp
    float *gp;         // [N] level units
    uint8_t *x;        // [N][Cp]
    int64_t N;
    int Cp, L, mode;
    double vmin, scale;
    uint32_t key0, key1;
};

// Sweeps t0 .. t0+n-1 of a run with the given burn-in and tally stride: how many of them
// accumulate into the mean (t >= burn_in) and how many also tally the histogram
// ((t - burn_in) % stride == 0; none if stride <= 0).
inline void accumulating_sweeps(int64_t t0, int64_t n, int64_t burn_in, int64_t stride, int64_t *acc,
                                int64_t *tallies)
{
    const int64_t a = t0 > burn_in ? t0 : burn_in, b = t0 + n;  // accumulating sweeps: [a, b)
    *acc = b > a ? b - a : 0;
    *tallies = 0;
    if (stride > 0 && b > a) {
        // multiples of stride in [0, x) for x >= 0
        auto upto = [stride](int64_t x) { return x <= 0 ? (int64_t)0 : (x - 1) / stride + 1; };
        *tallies = upto(b - burn_in) - upto(a - burn_in);
    }
}

// Chains handled by one thread: 4 (one Philox call feeds four chains) unless fewer exist.
inline int chain_group(int chains) { return chains >= 3 ? 4 : chains; }
// Chain slots in the interleaved state: chains rounded up to a multiple of 4 (1 or 2 stay).
inline int chain_slots(int chains) { return chains <= 2 ? chains : (chains + 3) / 4 * 4; }

// One lattice of a batch, resident in device memory; read by every workgroup of it.
struct ImageDesc {
    const float *gp;
    uint8_t *x0, *x1;     // state buffers: sweep t reads x[t & 1] and writes the other
    uint32_t *sum, *hist;
    const double *beta;   // per-sweep beta (device), beta_len entries; none => 1
    int beta_len;
    int H, W, L, C, Cp, T, hist_words, burn_in, tally_stride;
    int inertia;          // 0, 1 or 2; every lattice of one launch has inertia 0 or none has
    double J, q, kappa, sigma_s;
    uint32_t key0, key1;
    int tpp;              // threads per pixel (Cp / G) in the launch configuration in use
    int block_base;       // first workgroup of this lattice in the batched grid
    int tiles_w;          // tiled traversal: tiles per tile row; patch traversal: tiles per row
    int patch;            // untiled traversal: log2(tpp) if the pixels form 2-D patches, else -1
    int tb_side;          // multi-sweep traversal: side of the lattice's square LDS tiles, else 0
    uint32_t t;           // sweep index before the current replay; advanced on the device
    uint32_t t_end;       // the lattice stops advancing at this sweep index
};

struct BatchLaunch {
    const ImageDesc *imgs;
    const int *block_img;  // workgroup -> lattice
    uint32_t toff;         // sweep offset of this launch within the replay
    int block0;            // first workgroup of this launch in the batch's grid (split grids)
};

constexpr int kTileW = 16;  // tiled traversal: tiles 16 pixels wide, kBlock / tpp pixels each

// Traversal of one lattice in an untiled batched launch, as in the single-lattice sweep:
// 2-D pixel patches for L > 16 (when tpp allows), row-major otherwise.  Sets d.patch and
// d.tiles_w from d.H, d.W, d.L and d.tpp; returns the lattice's workgroups.
inline int64_t untiled_layout(ImageDesc &d)
{
    const SweepLayout l = sweep_layout(d.H, d.W, d.tpp, d.L > 16);
    d.patch = l.patch;
    d.tiles_w = l.tiles_w;
    return l.blocks;
}

// inr: the lattices use the L1/L2 inertia form (share is then ignored).  Grids of more
// than kMaxLaunchBlocks workgroups are issued as several launches (BatchLaunch.block0).
hipError_t launch_batch_sweep(const BatchLaunch &b, int total_blocks, int G, int share, int tiled, int nbr, bool inr,
                              hipStream_t s);
hipError_t launch_advance(ImageDesc *imgs, int n_imgs, uint32_t n, hipStream_t s);
// The L1/L2 inertia kernels (pca_kernels_inertia.hip); the two launchers above hand over
// to these when the sweep (or every lattice of the batch) has inertia 1 or 2.
hipError_t launch_sweep_inertia(const SweepArgs &a, int G, int nbr, hipStream_t s);
hipError_t launch_batch_sweep_inertia(const BatchLaunch &b, int blocks, int G, int tiled, int nbr, hipStream_t s);

// Several sweeps in one launch for lattices with L <= 16 (pca_kernels_tb.hip): each
// workgroup advances one tile of the lattice S sweeps from an LDS copy of the tile and a
// halo S sites deep.
constexpr int kTbMaxSweeps = 16;
constexpr int kTbBlock = 512;          // threads per workgroup (two waves per SIMD)
constexpr int kTbItems = 2;            // items of the first sweep per thread, at most
constexpr int kTbMaxLds = 64 * 1024;  // LDS bytes a workgroup may use
constexpr int64_t kTbMaxThreads = 4 * 256 * 4 * 64;  // most single-sweep threads for which it is used

struct TbArgs {
    SweepArgs a;      // a.t: first sweep; a.xin: state at a.t; a.xout: receives the state at
                      // a.t + S; a.sum / a.hist: accumulators of the sweeps the masks select
    int S;            // sweeps of this launch, 1..kTbMaxSweeps
    int nbr;          // neighbourhood, 4 or 8
    int TH, TW;       // tile shape in pixels (square)
    int tiles_w;      // tiles per lattice row
    int tiles;        // tiles (workgroups) in all
    int ptab_n;       // prior table entries, nbr * T + 1
    uint32_t acc_mask, tally_mask;  // bit s: sweep a.t + s adds to the sum / to the histogram
    uint32_t beta_mask;             // bit s (s >= 1): beta of sweep a.t + s differs from the one before
    double beta[kTbMaxSweeps];      // beta of sweep a.t + s
};

// Launch plan of the multi-sweep kernel: S == 0 when it does not apply (L > 16, inertia
// 1 or 2, a lattice large enough to fill the GPU with one sweep, or no tile whose halo
// and items fit).
struct TbPlan {
    int TH, TW, S, tiles_w, tiles;
};

TbPlan tb_plan(int H, int W, int L, int Cp, int nbr, int T, int inertia);
hipError_t launch_tb_sweeps(const TbArgs &b, hipStream_t s);

// Whether square tiles of `side` advancing S sweeps per launch fit an H x W lattice with
// Cp chain slots, G chains per thread, in workgroups of `block` threads: the tile's own
// (site, chain group) items one per thread, the items of the first sweep `imax` per
// thread, and the LDS limit.
bool tb_fits(int H, int W, int Cp, int G, int side, int S, int ptab_n, int imax, int block);
size_t tb_lds_bytes(int H, int W, int Cp, int side, int S, int ptab_n);

// The same for the lattices of a batch that use the multi-sweep traversal (one launch for
// all of them, S odd so that the state stays in the buffer of its sweep index's parity).
constexpr int kTbBatchSweeps = 7;  // sweeps per launch (odd)
constexpr int kTbBatchSide = 8;    // tile side (4 where the items of 8x8 tiles do not fit)
constexpr int kTbBatchItems = 4;   // items of the first sweep per thread, at most
constexpr int kTbBatchBlock = 256; // threads per workgroup
struct TbBatchLaunch {
    const ImageDesc *imgs;
    const int *block_img;  // workgroup -> lattice (each lattice's tiles consecutive from its block_base)
    uint32_t toff;         // first sweep of the launch, relative to each lattice's sweep index
    int S;                 // sweeps (odd), fewer for a lattice that reaches its end
};
hipError_t launch_tb_batch(const TbBatchLaunch &L, int blocks, int G, int nbr, size_t lds_bytes, hipStream_t s);

// Device buffers of one single-lattice run and the chain layout that goes with them.
struct RunBuffers {
    float *gp;           // [N] observation in level units
    uint8_t *x[2];       // [N][Cp] double-buffered chain states
    uint32_t *sum;       // [N] level sums
    uint32_t *hist;      // [N][hist_words] packed uint16 counters, or nullptr (no histogram)
    int G, Cp, T, hist_words;
};

// Chain grouping, truncation and histogram row length of a run (buffers left null).
RunBuffers run_layout(const pca_params &p);

// Enqueues sweeps t0 .. t0+n-1 of a run on `b`: sweep t reads b.x[cur] and writes the other
// buffer, and cur flips once per sweep enqueued.  beta: host array of beta_len per-sweep
// values (none: beta = 1).  Returns the first launch error; *done receives the number of
// sweeps enqueued before it (n on success).
hipError_t enqueue_sweeps(const pca_params &p, const float *beta, int beta_len, const RunBuffers &b, int64_t t0,
                          int32_t n, int &cur, int32_t *done, hipStream_t s);

// Shared by the single-lattice and batch entry points (pca_api.hip).
int validate_params(const pca_params *p);     // PCA_OK or PCA_EINVAL with the error message set
int set_error(int code, const char *message);  // records the calling thread's last error, returns code

// Failure-handling hook for tests: the environment variable PCA_FAULT_INJECT holds a
// comma-separated list of allocation sites, each optionally with a request id
// ("init", "admit:3", "readout:7").  A listed site fails as if its allocation had been
// refused: "init" the device buffers of pca_init, "admit" a server request's device
// buffers at admission, "readout" the host buffers of a finished request's results.
// The variable is read at every call, so a test can set and clear it between calls.
bool fault_injected(const char *site, int64_t id);

hipError_t launch_init(const InitArgs &a, hipStream_t s);
hipError_t launch_sweep(const SweepArgs &a, int G, int nbr, hipStream_t s);
hipError_t launch_get_state(const uint8_t *x, uint8_t *out, int64_t N, int C, int Cp, hipStream_t s);
hipError_t launch_set_state(const uint8_t *in, uint8_t *x, int64_t N, int C, int Cp, hipStream_t s);
// Sets *flag (device int, zeroed by the caller) to 1 if any of the n bytes at in is >= L.
hipError_t launch_check_levels(const uint8_t *in, int64_t n, int L, int *flag, hipStream_t s);
hipError_t launch_mean(const uint32_t *sum, float *out, int64_t N, int64_t count, double vmin, double delta,
                       hipStream_t s);
hipError_t launch_mpm(const uint32_t *hist, uint8_t *out, int64_t N, int L, int hist_words, hipStream_t s);

}  // namespace pcak
