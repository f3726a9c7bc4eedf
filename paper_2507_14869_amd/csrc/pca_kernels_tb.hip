// Multi-sweep kernel for lattices with few levels (L <= 16): each workgroup keeps a tile
// of the chain states, with a halo as deep as the number of sweeps it runs, in LDS and
// advances it S sweeps without leaving the kernel.
//
// Why this is exact: a site's new level depends only on the previous states of the site
// and its neighbours (Sec. 5.2: every pixel is drawn independently given the previous
// configuration) and on its own random word, keyed by (seed, chain, sweep, pixel).  A tile
// loaded with a halo of depth S at sweep t0 therefore holds enough of the lattice to
// compute sweep t0 + s on the tile grown by S - 1 - s, for s = 0 .. S-1: after S sweeps
// the tile itself is at t0 + S, identical to S single-sweep launches.  Halo sites are
// computed by more than one workgroup (each gets the same value); only the tile's own
// sites are written back and counted in the statistics.
//
// What it saves on such lattices, where a sweep is short: S - 1 of every S kernel
// launches and the state's trips through memory between them, and the level sums, which
// are accumulated in LDS and added to memory once per launch.
#include <algorithm>

#include "pca_sweep.h"

namespace pcak {
namespace {

// LDS layout of one workgroup (byte offsets; see tb_lds_layout).
struct TbLayout {
    int ptab, gp, xa, xb, sum, bytes;
};

__host__ __device__ inline int tb_round16(int x) { return (x + 15) & ~15; }

__host__ __device__ inline TbLayout tb_lds_layout(int region_pixels, int Cp, int tile_pixels, int ptab_n, bool sums)
{
    TbLayout l;
    l.ptab = 0;
    l.gp = tb_round16(ptab_n * 4);
    l.xa = l.gp + tb_round16(region_pixels * 4);
    l.xb = l.xa + tb_round16(region_pixels * Cp);
    l.sum = l.xb + tb_round16(region_pixels * Cp);
    l.bytes = l.sum + (sums ? tb_round16(tile_pixels * 4) : 0);
    return l;
}

// Copies `rows` rows of `row_bytes` bytes between two row-strided byte arrays, by dwords
// when every row start and length is a multiple of 4.
__device__ __forceinline__ void copy_rows(uint8_t *dst, int64_t dst_stride, const uint8_t *src, int64_t src_stride,
                                          int rows, int row_bytes, bool dwords, int tid, int nthreads)
{
    if (dwords) {
        const int rw = row_bytes >> 2;
        const int n = rows * rw;
        for (int i = tid; i < n; i += nthreads) {
            const int r = i / rw, c = i - r * rw;
            reinterpret_cast<uint32_t *>(dst + r * dst_stride)[c] =
                reinterpret_cast<const uint32_t *>(src + r * src_stride)[c];
        }
    } else {
        const int n = rows * row_bytes;
        for (int i = tid; i < n; i += nthreads) {
            const int r = i / row_bytes, c = i - r * row_bytes;
            dst[r * dst_stride + c] = src[r * src_stride + c];
        }
    }
}

// n / d for 0 <= n < 2^22 and 1 <= d, from a float reciprocal and one correction (the
// float quotient is within one of the exact one).
__device__ __forceinline__ int small_div(int n, int d, float inv_d)
{
    int q = (int)((float)n * inv_d);
    const int r = n - q * d;
    q += r >= d ? 1 : 0;
    q -= r < 0 ? 1 : 0;
    return q;
}

// The sweeps of one tile: `a` holds the lattice (a.t the first sweep, a.xin / a.xout the
// state before and after, a.sum / a.hist the accumulators), tile `tile` of a grid of
// tiles_w tiles per row, each TH x TW; sch gives each sweep's beta and whether it adds to
// the level sum (acc) and to the histogram (tally).
template <int G, int NBR, int SHARE, int BLK, class Schedule>
__device__ __forceinline__ void tb_tile(SweepArgs a, int tile, int TH, int TW, int tiles_w, int S, int ptab_n,
                                        const Schedule &sch, unsigned char *lds)
{
    const int tid = (int)threadIdx.x;
    const int Cp = a.Cp, tpp = Cp / G, H = a.H, W = a.W;

    // The tile [r0, r1) x [c0, c1) and the loaded region: the tile grown by S, clipped.
    const int tr = tile / tiles_w, tc = tile - tr * tiles_w;
    const int r0 = tr * TH, c0 = tc * TW;
    const int r1 = min(H, r0 + TH), c1 = min(W, c0 + TW);
    const int gr0 = max(0, r0 - S), gc0 = max(0, c0 - S), gr1 = min(H, r1 + S), gc1 = min(W, c1 + S);
    const int w0 = gc1 - gc0, h0 = gr1 - gr0;
    const bool sums = sch.any_acc();
    const TbLayout lay = tb_lds_layout(w0 * h0, Cp, TH * TW, ptab_n, sums);
    float *ptab = reinterpret_cast<float *>(lds + lay.ptab);
    float *gpl = reinterpret_cast<float *>(lds + lay.gp);
    uint8_t *xa = lds + lay.xa;
    uint8_t *xb = lds + lay.xb;
    uint32_t *suml = reinterpret_cast<uint32_t *>(lds + lay.sum);

    // Load the region's observation and state at sweep t0; clear the tile's sums.
    for (int i = tid; i < w0 * h0; i += BLK) {
        const int rr = i / w0, cc = i - rr * w0;
        gpl[i] = a.gp[(gr0 + rr) * W + gc0 + cc];
    }
    const bool dwords = (Cp & 3) == 0;
    copy_rows(xa, (int64_t)w0 * Cp, a.xin + ((int64_t)gr0 * W + gc0) * Cp, (int64_t)W * Cp, h0, w0 * Cp, dwords, tid,
              BLK);
    if (sums)
        for (int i = tid; i < TH * TW; i += BLK) suml[i] = 0u;

    const float inv_tpp = 1.0f / (float)tpp;
    const uint32_t t0 = a.t;
    SweepConsts kc{};
    double beta_prev = 0.0;
    for (int s = 0; s < S; ++s) {
        a.t = t0 + (uint32_t)s;
        a.beta = sch.beta(s);
        if (s == 0 || a.beta != beta_prev) {
            __syncthreads();  // the previous sweep's table reads are done
            fill_prior_table(a, NBR, ptab, tid, BLK);
            kc = sweep_constants(a);
            beta_prev = a.beta;
        }
        __syncthreads();  // table, and the state of sweep t0 + s, complete
        const uint8_t *in = (s & 1) ? xb : xa;
        uint8_t *out = (s & 1) ? xa : xb;
        const bool acc = sch.acc(s), tally = sch.tally(s);

        // Sites of sweep s: the tile grown by e = S - 1 - s, clipped to the lattice.
        const int e = S - 1 - s;
        const int sr0 = max(0, r0 - e), sc0 = max(0, c0 - e), sr1 = min(H, r1 + e), sc1 = min(W, c1 + e);
        const int rw = sc1 - sc0;
        const int items = (sr1 - sr0) * rw * tpp;
        const float inv_rw = 1.0f / (float)rw;
        for (int idx = tid; idx < items; idx += BLK) {
            const int p = small_div(idx, tpp, inv_tpp), grp = idx - p * tpp;
            const int pr = small_div(p, rw, inv_rw);
            const int r = sr0 + pr, c = sc0 + (p - pr * rw);
            const int li = (r - gr0) * w0 + (c - gc0);
            SiteInputs<NBR> si;
            si.gp = gpl[li];
            si.own = load_group<G>(in + li * Cp + grp * G);
#pragma unroll
            for (int j = 0; j < NBR; ++j) {
                const int rr = r + kNbrDr[j], cc = c + kNbrDc[j];
                si.present[j] = rr >= 0 && rr < H && cc >= 0 && cc < W;
                si.nbw[j] = si.present[j] ? load_group<G>(in + (li + kNbrDr[j] * w0 + kNbrDc[j]) * Cp + grp * G) : 0u;
            }
            const int pix = r * W + c;
            int knew[G];
            const uint32_t packed = site_draw<G, NBR, 1, 16, SHARE>(a, ptab, kc, si, pix, grp, grp % SHARE, knew);
            store_group<G>(out + li * Cp + grp * G, packed);
            if ((acc || tally) && r >= r0 && r < r1 && c >= c0 && c < c1) {
                // the tile's own sites: level sums into LDS, tallies into the histogram
                site_stats<G, 1>(acc ? suml + (r - r0) * TW + (c - c0) : nullptr,
                                 tally ? a.hist + (int64_t)pix * a.hist_words : nullptr, a.hist_words, a.C, tpp, grp,
                                 knew);
            }
        }
    }
    __syncthreads();

    // The tile's state at t0 + S (written by sweep S-1) and its level sums go to memory.
    const uint8_t *fin = ((S - 1) & 1) ? xa : xb;
    copy_rows(a.xout + ((int64_t)r0 * W + c0) * Cp, (int64_t)W * Cp, fin + ((r0 - gr0) * w0 + (c0 - gc0)) * Cp,
              (int64_t)w0 * Cp, r1 - r0, (c1 - c0) * Cp, dwords, tid, BLK);
    if (sums) {
        const int tw = c1 - c0, n = (r1 - r0) * tw;
        for (int i = tid; i < n; i += BLK) {
            const int rr = i / tw, cc = i - rr * tw;
            a.sum[(int64_t)(r0 + rr) * W + c0 + cc] += suml[rr * TW + cc];
        }
    }
}

// Schedule of a single-lattice launch: from the host-filled arguments.
struct ArgSchedule {
    const TbArgs &b;
    __device__ double beta(int s) const { return b.beta[s]; }
    __device__ bool acc(int s) const { return (b.acc_mask >> s) & 1u; }
    __device__ bool tally(int s) const { return (b.tally_mask >> s) & 1u; }
    __device__ bool any_acc() const { return b.acc_mask != 0u; }
};

template <int G, int NBR, int SHARE, int BLK>
__global__ __launch_bounds__(BLK) void tb_sweep_kernel(TbArgs b)
{
    extern __shared__ __align__(16) unsigned char lds[];
    tb_tile<G, NBR, SHARE, BLK>(b.a, (int)blockIdx.x, b.TH, b.TW, b.tiles_w, b.S, b.ptab_n, ArgSchedule{b}, lds);
}

// Schedule of a lattice in a batched launch: from its descriptor, sweeps t0 .. t0+S-1.
struct DescSchedule {
    const ImageDesc &d;
    uint32_t t0;
    __device__ double beta(int s) const
    {
        const uint32_t t = t0 + (uint32_t)s;
        return d.beta_len == 0 ? 1.0 : d.beta[t < (uint32_t)d.beta_len ? t : (uint32_t)(d.beta_len - 1)];
    }
    __device__ bool acc(int s) const { return (int64_t)(t0 + (uint32_t)s) >= d.burn_in; }
    __device__ bool tally(int s) const
    {
        const int64_t t = (int64_t)(t0 + (uint32_t)s);
        return t >= d.burn_in && d.tally_stride > 0 && (t - d.burn_in) % d.tally_stride == 0;
    }
    __device__ bool any_acc() const { return acc(S - 1); }
    int S;
};

// Several sweeps of every lattice a batch runs from LDS tiles (the batch's "multi-sweep"
// traversal): workgroup -> lattice by a table, each lattice's tiles consecutive.  S is odd,
// so a lattice's state after the launch is in the buffer of its new sweep index's parity,
// as the one-sweep launches keep it.
template <int G, int NBR, int SHARE, int BLK>
__global__ __launch_bounds__(BLK) void tb_batch_kernel(TbBatchLaunch L)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const int img = L.block_img[blockIdx.x];
    const ImageDesc &d = L.imgs[img];
    const uint32_t t0 = d.t + L.toff;
    if (t0 >= d.t_end) return;  // this lattice has finished (uniform over the workgroup)
    const int S = (int)min((uint32_t)L.S, d.t_end - t0);
    SweepArgs a;
    a.gp = d.gp;
    a.xin = (t0 & 1u) ? d.x1 : d.x0;
    a.xout = (t0 & 1u) ? d.x0 : d.x1;
    a.sum = d.sum;
    a.hist = d.hist;
    a.H = d.H;
    a.W = d.W;
    a.L = d.L;
    a.C = d.C;
    a.Cp = d.Cp;
    a.T = d.T;
    a.hist_words = d.hist_words;
    a.beta = 1.0;
    a.J = d.J;
    a.q = d.q;
    a.kappa = d.kappa;
    a.sigma_s = d.sigma_s;
    a.key0 = d.key0;
    a.key1 = d.key1;
    a.t = t0;
    a.inertia = 0;
    a.blk0 = 0;
    a.patch = -1;
    a.tiles_w = 0;
    tb_tile<G, NBR, SHARE, BLK>(a, (int)blockIdx.x - d.block_base, d.tb_side, d.tb_side, d.tiles_w, S,
                                NBR * d.T + 1, DescSchedule{d, t0, S}, lds);
}

template <int G, int NBR, int SHARE>
hipError_t launch_tb_gs(const TbArgs &b, size_t lds_bytes, hipStream_t s)
{
    hipLaunchKernelGGL((tb_sweep_kernel<G, NBR, SHARE, kTbBlock>), dim3((unsigned)b.tiles), dim3(kTbBlock), lds_bytes,
                       s, b);
    return hipGetLastError();
}

template <int G, int NBR>
hipError_t launch_tb_g(const TbArgs &b, size_t lds_bytes, hipStream_t s)
{
    const int tpp = b.a.Cp / G;
    if constexpr (G == 4) {
        if (tpp % 4 == 0) return launch_tb_gs<G, NBR, 4>(b, lds_bytes, s);
        if (tpp % 2 == 0) return launch_tb_gs<G, NBR, 2>(b, lds_bytes, s);
    }
    return launch_tb_gs<G, NBR, 1>(b, lds_bytes, s);
}

template <int G, int NBR, int SHARE>
hipError_t launch_tb_batch_gs(const TbBatchLaunch &L, int blocks, size_t lds_bytes, hipStream_t s)
{
    hipLaunchKernelGGL((tb_batch_kernel<G, NBR, SHARE, kTbBlock>), dim3((unsigned)blocks), dim3(kTbBlock), lds_bytes,
                       s, L);
    return hipGetLastError();
}

template <int G, int NBR>
hipError_t launch_tb_batch_g(const TbBatchLaunch &L, int blocks, int share, size_t lds_bytes, hipStream_t s)
{
    if constexpr (G == 4) {
        if (share == 4) return launch_tb_batch_gs<G, NBR, 4>(L, blocks, lds_bytes, s);
        if (share == 2) return launch_tb_batch_gs<G, NBR, 2>(L, blocks, lds_bytes, s);
    }
    return launch_tb_batch_gs<G, NBR, 1>(L, blocks, lds_bytes, s);
}

}  // namespace

size_t tb_batch_lds_bytes(int H, int W, int Cp, int side, int S, int ptab_n)
{
    const int rh = std::min(H, side + 2 * S), rw = std::min(W, side + 2 * S);
    return (size_t)tb_lds_layout(rh * rw, Cp, side * side, ptab_n, true).bytes;
}

hipError_t launch_tb_batch(const TbBatchLaunch &L, int blocks, int G, int share, int nbr, size_t lds_bytes,
                           hipStream_t s)
{
    if (nbr == 8) {
        if (G == 4) return launch_tb_batch_g<4, 8>(L, blocks, share, lds_bytes, s);
        if (G == 2) return launch_tb_batch_g<2, 8>(L, blocks, share, lds_bytes, s);
        return launch_tb_batch_g<1, 8>(L, blocks, share, lds_bytes, s);
    }
    if (G == 4) return launch_tb_batch_g<4, 4>(L, blocks, share, lds_bytes, s);
    if (G == 2) return launch_tb_batch_g<2, 4>(L, blocks, share, lds_bytes, s);
    return launch_tb_batch_g<1, 4>(L, blocks, share, lds_bytes, s);
}

TbPlan tb_plan(int H, int W, int L, int Cp, int nbr, int T, int inertia)
{
    TbPlan pl{};
    if (L > 16 || inertia != 0) return pl;
    // Only lattices whose single-sweep launch has fewer threads than the GPU has lanes
    // (256 CUs x 4 SIMDs x 64): there a sweep costs a launch and one site's latency, which
    // several sweeps per launch amortise.  On larger ones the halo's extra work and the
    // barriers cost more than they save (measured on 512x512, L = 16, 8 chains: 23.7
    // against 19.3 us per sweep).
    const int G = chain_group(Cp);
    if ((int64_t)H * W * (Cp / G) >= kTbMaxThreads) return pl;
    // Tiles as large as keep every compute unit busy (about one workgroup each), down to
    // 4x4; 8 sweeps per launch.  Measured on 64x64, 1 chain, L = 2 (us per sweep): one
    // launch per sweep 3.41; 8x8 tiles with 8 sweeps 3.06, with 16 sweeps 4.45; 16x16 tiles
    // with 8 sweeps 4.81; 4x4 tiles with 8 sweeps 2.69, with 4 sweeps 3.14.
    static const int kSides[3] = {16, 8, 4};
    for (int i = 0; i < 3; ++i) {
        const int side = kSides[i];
        const int64_t tiles = (int64_t)((H + side - 1) / side) * ((W + side - 1) / side);
        if (tiles < 240 && side > 4) continue;
        const int S = 8;
        const int rh = std::min(H, side + 2 * S), rw = std::min(W, side + 2 * S);
        const TbLayout lay = tb_lds_layout(rh * rw, Cp, side * side, nbr * T + 1, true);
        if (lay.bytes > kTbMaxLds) return pl;
        pl.TH = pl.TW = side;
        pl.S = S;
        pl.tiles_w = (W + side - 1) / side;
        pl.tiles = (int)tiles;
        return pl;
    }
    return pl;
}

static size_t tb_lds_bytes(const TbArgs &b)
{
    const int rh = std::min(b.a.H, b.TH + 2 * b.S), rw = std::min(b.a.W, b.TW + 2 * b.S);
    return (size_t)tb_lds_layout(rh * rw, b.a.Cp, b.TH * b.TW, b.ptab_n, b.acc_mask != 0u).bytes;
}

hipError_t launch_tb_sweeps(const TbArgs &b, hipStream_t s)
{
    const size_t lds = tb_lds_bytes(b);
    const int G = chain_group(b.a.C);
    if (b.nbr == 8) {
        if (G == 4) return launch_tb_g<4, 8>(b, lds, s);
        if (G == 2) return launch_tb_g<2, 8>(b, lds, s);
        return launch_tb_g<1, 8>(b, lds, s);
    }
    if (G == 4) return launch_tb_g<4, 4>(b, lds, s);
    if (G == 2) return launch_tb_g<2, 4>(b, lds, s);
    return launch_tb_g<1, 4>(b, lds, s);
}

}  // namespace pcak
