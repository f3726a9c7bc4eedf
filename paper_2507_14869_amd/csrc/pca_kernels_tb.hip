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
// launches and the state's trips through memory between them.  A sweep here costs about
// one site's latency (a workgroup has two waves per SIMD), so the per-site code is laid out
// for a short dependent chain: every thread owns the same sites for the whole launch,
// with their LDS addresses, neighbour presence and data factors (which depend on neither
// the state nor beta) computed once; the level loop runs to a compile-time bound with no
// branch; absent neighbours read a border of zeros; with 8 or more levels the neighbour
// statistics come from the statistic table of the one-sweep kernels; and the level sums and
// tallies of the tile's sites stay in registers until the launch ends.
#include <algorithm>

#include "pca_sweep.h"

namespace pcak {
namespace {

// Level bound the per-site code is compiled for: L rounded up to a power of two.  The data
// factor of every level past L - 1 is 0, which leaves the running sums unchanged.
__host__ __device__ inline int tb_levels(int L) { return L <= 2 ? 2 : L <= 4 ? 4 : L <= 8 ? 8 : 16; }

// LDS layout of one workgroup (byte offsets): the prior table and the two state buffers of
// the loaded region, each with a border of zeros one site wide.
struct TbLayout {
    int ptab, vtab, xa, xb, bytes;
};

__host__ __device__ inline int tb_round16(int x) { return (x + 15) & ~15; }

// rh x rw: the loaded region.
__host__ __device__ inline TbLayout tb_lds_layout(int rh, int rw, int Cp, int ptab_n)
{
    TbLayout l;
    const int buf = tb_round16((rh + 2) * (rw + 2) * Cp);
    l.ptab = 0;
    l.vtab = tb_round16(ptab_n * 4);
    l.xa = l.vtab + kStatEntries * 16;
    l.xb = l.xa + buf;
    l.bytes = l.xb + buf;
    return l;
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

// One (site, chain group) pair that a thread updates in every sweep of the launch that
// reaches it.
template <int NW, int LB>
struct TbItem {
    int off;          // byte offset of the chain group in a state buffer
    int pix;          // lattice index r * W + c
    int last;         // last sweep of the launch that updates it (-1: no item)
    int grp;          // chain group
    bool own;         // a site of the tile itself
    uint32_t tm[NW];  // T in the byte of each present neighbour
    float D[LB];      // data factors of levels 0 .. LB-1 (0 past L - 1)
    float gp, m;      // observation in level units, data-term shift
};

// v[x] for x < N (N = 2 or 4) by selects on values (selects of loads from one array
// would be folded into an indexed load, which puts the array in scratch memory).
template <int N>
__device__ __forceinline__ float pick(const float (&v)[N], int x)
{
    const float v0 = v[0], v1 = v[1];
    if constexpr (N == 2) {
        return x ? v1 : v0;
    } else {
        const float v2 = v[2], v3 = v[3];
        const float lo = (x & 1) ? v1 : v0;
        const float hi = (x & 1) ? v3 : v2;
        return (x & 2) ? hi : lo;
    }
}

// New levels of one item's chains, from the state buffer `in`.  The arithmetic of
// site_draw for L <= 16: stay weight (D_x P(S_x)) R, running sums fma(D_k, P(S_k), .)
// over the levels, the threshold rounded down from u Z, and the first running sum above
// it (found by counting the sums at or below it: they are nondecreasing).
// The uniforms of the G chains of an item for sweep t (Sec. 5.2's draw, keyed by pixel,
// sweep and chain as in site_draw).
template <int G>
__device__ __forceinline__ void item_uniforms(int pix, int grp, uint32_t t, uint32_t key0, uint32_t key1, float (&u)[G])
{
    const int chain0 = grp * G;
    U4 rnd = philox<true>(U4{(uint32_t)pix, t, (uint32_t)(chain0 >> 2), 0u}, key0, key1);
    // all four words in registers before the selects below (otherwise the last round is
    // split into branches per word)
    asm volatile("" : "+v"(rnd.x), "+v"(rnd.y), "+v"(rnd.z), "+v"(rnd.w));
#pragma unroll
    for (int ch = 0; ch < G; ++ch) {
        const int wi = (chain0 & 3) + ch;
        const uint32_t w01 = (wi & 1) ? rnd.y : rnd.x, w23 = (wi & 1) ? rnd.w : rnd.z;
        const uint32_t w = (wi & 2) ? w23 : w01;
        u[ch] = (float)(w >> 8) * 0x1p-24f;
    }
}

// The state words an item's update reads: its own chain group and each neighbour's.
template <int NBR>
struct TbWords {
    uint32_t own, nbw[NBR];
};

template <int G, int NBR, int NW, int LB>
__device__ __forceinline__ TbWords<NBR> tb_load(const TbItem<NW, LB> &it, const uint8_t *in, const int (&nofs)[NBR])
{
    TbWords<NBR> v;
    const uint8_t *p = in + it.off;
    v.own = load_group<G>(p);
#pragma unroll
    for (int j = 0; j < NBR; ++j) v.nbw[j] = load_group<G>(p + nofs[j]);
    return v;
}

// pix: the item's pixel (the counter of its random words).
template <int G, int NBR, int LB>
__device__ __forceinline__ uint32_t tb_draw(const TbItem<NBR / 4, LB> &it, const TbWords<NBR> &v, int pix,
                                            const float *ptab, const uint4 *vtab, float R, float a2, uint32_t t,
                                            uint32_t key0, uint32_t key1, int (&knew)[G])
{
    constexpr int NW = NBR / 4;
    // with 8 or more levels the statistics come from the statistic table (see
    // fill_stat_table); byte k of a chain's sum is 4 S_k (4 neighbours) or S_k (8)
    constexpr bool TSTAT = LB >= 8;
    constexpr int kOffShift = NBR == 4 ? 0 : 2;
    const uint32_t own = v.own;
    const uint32_t(&nbw)[NBR] = v.nbw;
    float u[G];
    item_uniforms<G>(pix, it.grp, t, key0, key1, u);

    uint32_t sv[G][4];
    if constexpr (TSTAT) {
#pragma unroll
        for (int ch = 0; ch < G; ++ch)
#pragma unroll
            for (int d = 0; d < 4; ++d) sv[ch][d] = 0u;
#pragma unroll
        for (int j = 0; j < NBR; ++j) {
            const bool present = ((it.tm[j / 4] >> (8 * (j % 4))) & 0xFFu) != 0u;
            const uint32_t wj = present ? nbw[j] : 0x10101010u;  // absent: entry 16
#pragma unroll
            for (int ch = 0; ch < G; ++ch) {
                const uint4 e = vtab[(wj >> (8 * ch)) & 0xFFu];
                sv[ch][0] += e.x;
                sv[ch][1] += e.y;
                sv[ch][2] += e.z;
                sv[ch][3] += e.w;
            }
        }
    }

    // Neighbour packs of each chain (see NbrPack); absent neighbours are 0 with T = 0.
    NbrPack<NW> nb[G];
#pragma unroll
    for (int w = 0; w < NW && !TSTAT; ++w) {
        uint32_t X[G];
        transpose_group<G>(nbw[4 * w], nbw[4 * w + 1], nbw[4 * w + 2], nbw[4 * w + 3], X);
#pragma unroll
        for (int ch = 0; ch < G; ++ch) {
            const uint32_t hi = X[ch] + it.tm[w];
            const uint32_t d = (X[ch] | 0x80808080u) - it.tm[w];  // byte: x - T + 128, no borrows
            const uint32_t hb = d & 0x80808080u;                   // byte: 0x80 where x >= T
            const uint32_t lo = (d ^ 0x80808080u) & (hb | (hb - (hb >> 7)));
            nb[ch].x[w] = X[ch];
            nb[ch].lo[w] = lo;
            nb[ch].hi[w] = hi;
            nb[ch].cb = (int)__builtin_amdgcn_sad_u8(hi, lo, w == 0 ? 0u : (uint32_t)nb[ch].cb);
        }
    }
#pragma unroll
    for (int ch = 0; ch < G && !TSTAT; ++ch) nb[ch].cb *= 2;

    const char *pt = reinterpret_cast<const char *>(ptab);
    float P[LB][G];
    uint32_t kk = 0u;
#pragma unroll
    for (int k = 0; k < LB; ++k) {
#pragma unroll
        for (int ch = 0; ch < G; ++ch) {
            if constexpr (TSTAT)
                P[k][ch] = *reinterpret_cast<const float *>(pt + (((sv[ch][k >> 2] >> (8 * (k & 3))) & 0xFFu) << kOffShift));
            else
                P[k][ch] = prior_lookup<NW>(pt, nb[ch], kk);
        }
        kk += 0x01010101u;
    }

    uint32_t packed = 0u;
#pragma unroll
    for (int ch = 0; ch < G; ++ch) {
        const int x = (int)((own >> (8 * ch)) & 0xFFu);
        float Dx, Px;
        if constexpr (LB <= 4) {
            float Pc[LB];
#pragma unroll
            for (int k = 0; k < LB; ++k) Pc[k] = P[k][ch];
            Dx = pick<LB>(it.D, x);
            Px = pick<LB>(Pc, x);
        } else {
            const float ex = it.gp - (float)x;
            Dx = exp2s(__builtin_fmaf(-a2, ex * ex, it.m));
            if constexpr (TSTAT) {
                uint32_t s0 = sv[ch][0], s1 = sv[ch][1], s2 = sv[ch][2], s3 = sv[ch][3];
                asm("" : "+v"(s0), "+v"(s1), "+v"(s2), "+v"(s3));
                const uint32_t w01 = (x & 4) ? s1 : s0, w23 = (x & 4) ? s3 : s2;
                const uint32_t w = (x & 8) ? w23 : w01;
                Px = *reinterpret_cast<const float *>(pt + (((w >> (8 * (x & 3))) & 0xFFu) << kOffShift));
            } else {
                Px = prior_lookup<NW>(pt, nb[ch], (uint32_t)x * 0x01010101u);
            }
        }
        const float stay = (Dx * Px) * R;
        float acc = stay;
        float part[LB];
#pragma unroll
        for (int k = 0; k < LB; ++k) {
            acc = __builtin_fmaf(it.D[k], P[k][ch], acc);
            part[k] = acc;
        }
        const float tf = threshold_rd(u[ch], acc);
        int below = 0;  // part[LB-1] = Z > tf whenever Z > 0
#pragma unroll
        for (int k = 0; k < LB - 1; ++k) below += part[k] <= tf ? 1 : 0;
        const int k = (acc != 0.0f && !(stay > tf)) ? below : x;
        knew[ch] = k;
        packed |= (uint32_t)k << (8 * ch);
    }
    return packed;
}

// Site of item rank q in ring order around a TS x TS tile at (r0, c0): ring 0 is the tile
// (row-major), ring e >= 1 the border of the tile grown by e (its top row, bottom row, left
// column, right column), which follows the (TS + 2(e-1))^2 sites of the rings inside it.
// Returns the ring; sites outside the lattice are the caller's to reject.
__device__ __forceinline__ int ring_site(int q, int TS, int r0, int c0, int S, int &r, int &c)
{
    int e = 0;
    for (int k = 1; k < S; ++k) e += q >= (TS + 2 * (k - 1)) * (TS + 2 * (k - 1)) ? 1 : 0;
    if (e == 0) {
        const int rr = q / TS;
        r = r0 + rr;
        c = c0 + (q - rr * TS);
        return 0;
    }
    const int n = TS + 2 * e, i = q - (n - 2) * (n - 2);
    if (i < n) {
        r = r0 - e;
        c = c0 - e + i;
    } else if (i < 2 * n) {
        r = r0 + TS - 1 + e;
        c = c0 - e + (i - n);
    } else if (i < 3 * n - 2) {
        r = r0 - e + 1 + (i - 2 * n);
        c = c0 - e;
    } else {
        r = r0 - e + 1 + (i - (3 * n - 2));
        c = c0 + TS - 1 + e;
    }
    return e;
}

// The sweeps of one tile: `a` holds the lattice (a.t the first sweep, a.xin / a.xout the
// state before and after, a.sum / a.hist the accumulators), tile `tile` of a grid of
// tiles_w square tiles of side TS per row; sch gives each sweep's beta and whether it adds
// to the level sum (acc) and to the histogram (tally).  The launch guarantees that the
// (TS + 2(S-1))^2 * tpp items of sweep 0 fit IMAX per thread and the TS^2 * tpp items of
// the tile itself one per thread.
template <int G, int NBR, int LB, int IMAX, int BLK, class Schedule>
__device__ __forceinline__ void tb_tile(SweepArgs a, int tile, int TS, int tiles_w, int S, int ptab_n,
                                        const Schedule &sch, unsigned char *lds)
{
    constexpr int NW = NBR / 4;
    const int tid = (int)threadIdx.x;
    const int Cp = a.Cp, tpp = Cp / G, H = a.H, W = a.W;

    // The tile [r0, r1) x [c0, c1) and the loaded region, the tile grown by S (clipped).
    const int tr = tile / tiles_w, tc = tile - tr * tiles_w;
    const int r0 = tr * TS, c0 = tc * TS;
    const int r1 = min(H, r0 + TS), c1 = min(W, c0 + TS);
    const int gr0 = max(0, r0 - S), gc0 = max(0, c0 - S), gr1 = min(H, r1 + S), gc1 = min(W, c1 + S);
    const int h0 = gr1 - gr0, w0 = gc1 - gc0, wp = w0 + 2;
    const TbLayout lay = tb_lds_layout(h0, w0, Cp, ptab_n);
    float *ptab = reinterpret_cast<float *>(lds + lay.ptab);
    uint4 *vtab = reinterpret_cast<uint4 *>(lds + lay.vtab);
    uint8_t *xa = lds + lay.xa;
    uint8_t *xb = lds + lay.xb;

    // The region's state at sweep t0 goes to xa and zeros to xb, both with the border.  The
    // first KL * BLK units (bytes, or dwords when Cp is a multiple of 4) are requested before
    // anything else, so that their latency covers the item set-up and the prior table, and
    // stored after them; any further units are loaded and stored in rounds.
    const bool dwords = (Cp & 3) == 0;
    const int unit = dwords ? 4 : 1, per_site = Cp / unit, per_row = wp * per_site;
    const int nunits = (h0 + 2) * per_row;
    const float inv_row = 1.0f / (float)per_row, inv_site = 1.0f / (float)per_site;
    auto load_unit = [&](int i) -> uint32_t {
        if (i >= nunits) return 0u;
        const int pr = small_div(i, per_row, inv_row), rem = i - pr * per_row;
        const int pc = small_div(rem, per_site, inv_site), bi = rem - pc * per_site;
        if (pr < 1 || pr > h0 || pc < 1 || pc > w0) return 0u;
        const int64_t src = ((int64_t)(gr0 + pr - 1) * W + (gc0 + pc - 1)) * Cp + bi * unit;
        return dwords ? *reinterpret_cast<const uint32_t *>(a.xin + src) : (uint32_t)a.xin[src];
    };
    auto store_unit = [&](int i, uint32_t v) {
        if (i >= nunits) return;
        if (dwords) {
            reinterpret_cast<uint32_t *>(xa)[i] = v;
            reinterpret_cast<uint32_t *>(xb)[i] = 0u;
        } else {
            xa[i] = (uint8_t)v;
            xb[i] = 0;
        }
    };
    constexpr int KL = 4;
    uint32_t v0[KL];
#pragma unroll
    for (int q = 0; q < KL; ++q) v0[q] = load_unit(tid + q * BLK);

    // The thread's items: item j = (site of rank j / tpp in ring order, chain group j % tpp);
    // items whose site is outside the lattice (or past the area) take the tile's first
    // site and are never stored.  Their observations, and the accumulator words of the
    // tile's own sites, are requested now so that one memory latency covers them all.
    const bool pre_sum = sch.any_acc() && a.sum != nullptr;
    const bool pre_hist = sch.any_tally() && a.hist != nullptr;
    const bool quad = tpp == 1 || tpp == 2 || tpp == 4;  // DPP sums, else global atomics
    const int span = TS + 2 * (S - 1), nitems = span * span * tpp;
    TbItem<NW, LB> it[IMAX];
    float gpv[IMAX];
    uint32_t osum = 0u, orow[8];
    {
        const float inv_tpp = 1.0f / (float)tpp;
#pragma unroll
        for (int k = 0; k < IMAX; ++k) {
            const int j = tid + k * BLK;
            const int rank = small_div(j, tpp, inv_tpp);
            int r, c;
            const int ring = ring_site(rank, TS, r0, c0, S, r, c);
            const bool valid = j < nitems && r >= 0 && r < H && c >= 0 && c < W;
            const int grp = valid ? j - rank * tpp : 0;
            if (!valid) {
                r = r0;
                c = c0;
            }
            it[k].off = ((r - gr0 + 1) * wp + (c - gc0 + 1)) * Cp + grp * G;
            it[k].pix = r * W + c;
            it[k].last = valid ? S - 1 - ring : -1;
            it[k].grp = grp;
            it[k].own = valid && ring == 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) it[k].tm[w] = 0u;
#pragma unroll
            for (int q = 0; q < NBR; ++q) {
                const int rq = r + kNbrDr[q], cq = c + kNbrDc[q];
                if (rq >= 0 && rq < H && cq >= 0 && cq < W) it[k].tm[q / 4] |= (uint32_t)a.T << (8 * (q % 4));
            }
            gpv[k] = a.gp[it[k].pix];
        }
        const TbItem<NW, LB> &o = it[0];
#pragma unroll
        for (int w = 0; w < 8; ++w) orow[w] = 0u;
        if (o.own && quad) {
            if (pre_sum && o.grp == 0) osum = a.sum[o.pix];
            if (pre_hist) {
                const uint32_t *hrow = a.hist + (int64_t)o.pix * a.hist_words;
#pragma unroll
                for (int w = 0; w < 8; ++w)
                    if (w < a.hist_words && (w & (tpp - 1)) == o.grp) orow[w] = hrow[w];
            }
        }
    }

    // Sweep 0's prior table and constants.
    a.beta = sch.beta(0);
    fill_prior_table(a, NBR, ptab, tid, BLK);
    if constexpr (LB >= 8) fill_stat_table(a, NBR, reinterpret_cast<uint32_t *>(vtab), tid, BLK);
    SweepConsts kc = sweep_constants(a);
    double beta_prev = a.beta;

#pragma unroll
    for (int q = 0; q < KL; ++q) store_unit(tid + q * BLK, v0[q]);
    for (int base = KL * BLK; base < nunits; base += KL * BLK) {
        uint32_t v[KL];
#pragma unroll
        for (int q = 0; q < KL; ++q) v[q] = load_unit(base + tid + q * BLK);
#pragma unroll
        for (int q = 0; q < KL; ++q) store_unit(base + tid + q * BLK, v[q]);
    }

    // The items' data factors, as site_draw evaluates them.
#pragma unroll
    for (int k = 0; k < IMAX; ++k) {
        const float gp = gpv[k];
        float khat = __builtin_rintf(gp);
        khat = khat < 0.0f ? 0.0f : khat;
        khat = khat > (float)(a.L - 1) ? (float)(a.L - 1) : khat;
        const float e0 = gp - khat;
        const float m = kc.a2 * (e0 * e0);
        it[k].gp = gp;
        it[k].m = m;
#pragma unroll
        for (int q = 0; q < LB; ++q) {
            const float e = gp - (float)q;
            it[k].D[q] = q < a.L ? exp2s(__builtin_fmaf(-kc.a2, e * e, m)) : 0.0f;
        }
    }

    int nofs[NBR];
#pragma unroll
    for (int q = 0; q < NBR; ++q) nofs[q] = (kNbrDr[q] * wp + kNbrDc[q]) * Cp;

    // Statistics of the thread's own site (slot 0): level sum, and 8-bit counters of
    // levels 4w .. 4w+3 in cnt8[w] (at most S * G < 256 per thread and launch).
    uint32_t lsum = 0u, cnt8[4] = {0u, 0u, 0u, 0u};
    const uint32_t t0 = a.t;
    for (int s = 0; s < S; ++s) {
        if (s > 0 && sch.beta_changes(s, beta_prev)) {
            __syncthreads();  // the previous sweep's table reads are done
            a.beta = sch.beta(s);
            fill_prior_table(a, NBR, ptab, tid, BLK);
            kc = sweep_constants(a);
            beta_prev = a.beta;
        }
        __syncthreads();  // table, and the state of sweep t0 + s, complete
        const uint8_t *in = (s & 1) ? xb : xa;
        uint8_t *out = (s & 1) ? xa : xb;
        const bool acc = sch.acc(s), tally = sch.tally(s);
        const uint32_t t = t0 + (uint32_t)s;
        auto tally_own = [&](const int (&knew)[G]) {
#pragma unroll
            for (int ch = 0; ch < G; ++ch) {
                if (it[0].grp * G + ch < a.C) {
                    if (acc) lsum += (uint32_t)knew[ch];
                    if (tally) {
                        const uint32_t inc = 1u << (8 * (knew[ch] & 3));
#pragma unroll
                        for (int w = 0; w < 4; ++w) cnt8[w] += (knew[ch] >> 2) == w ? inc : 0u;
                    }
                }
            }
        };
#pragma unroll
        for (int k = 0; k < IMAX; ++k) {
            const bool act = s <= it[k].last;
            if (__any(act)) {
                const TbWords<NBR> v = tb_load<G>(it[k], in, nofs);
                int knew[G];
                const uint32_t packed =
                    tb_draw<G, NBR, LB>(it[k], v, it[k].pix, ptab, vtab, kc.R, kc.a2, t, a.key0, a.key1, knew);
                if (act) store_group<G>(out + it[k].off, packed);
                if (k == 0 && it[0].own) tally_own(knew);
            }
        }
    }
    __syncthreads();

    // The tile's state at t0 + S (written by sweep S-1) to memory.
    {
        const uint8_t *fin = ((S - 1) & 1) ? xa : xb;
        const int rows = r1 - r0, row_bytes = (c1 - c0) * Cp;
        const bool dwords = (Cp & 3) == 0;
        const int unit = dwords ? 4 : 1, per_row = row_bytes / unit, n = rows * per_row;
        const float inv_row = 1.0f / (float)per_row;
        for (int i = tid; i < n; i += BLK) {
            const int rr = small_div(i, per_row, inv_row), b = (i - rr * per_row) * unit;
            const int src = ((r0 + rr - gr0 + 1) * wp + (c0 - gc0 + 1)) * Cp + b;
            const int64_t dst = ((int64_t)(r0 + rr) * W + c0) * Cp + b;
            if (dwords) *reinterpret_cast<uint32_t *>(a.xout + dst) = *reinterpret_cast<const uint32_t *>(fin + src);
            else a.xout[dst] = fin[src];
        }
    }

    // The tile's level sums and tallies of the launch, added once.  The tpp lanes of a site
    // are consecutive (aligned pairs or quads when tpp is 2 or 4) and all run this code;
    // each accumulator word has one owner lane, which read it at the start.
    const TbItem<NW, LB> &o = it[0];
    if (pre_sum) {
        uint32_t v = lsum;
        if (tpp == 2 || tpp == 4) {
            v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);                  // [1,0,3,2]
            if (tpp == 4) v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);  // [2,3,0,1]
        }
        if (o.own) {
            if (quad) {
                if (o.grp == 0) a.sum[o.pix] = osum + v;
            } else {
                atomicAdd(a.sum + o.pix, lsum);
            }
        }
    }
    if (pre_hist) {
        // uint16 counter pairs: word w holds levels 2w and 2w+1
        uint32_t row[8];
#pragma unroll
        for (int w = 0; w < 8; ++w) {
            const uint32_t two = (cnt8[w >> 1] >> (16 * (w & 1))) & 0xFFFFu;
            row[w] = (two & 0xFFu) | ((two >> 8) << 16);
        }
        if (tpp == 2 || tpp == 4) {
#pragma unroll
            for (int w = 0; w < 8; ++w) {
                row[w] += (uint32_t)__builtin_amdgcn_mov_dpp((int)row[w], 0xB1, 0xF, 0xF, false);
                if (tpp == 4) row[w] += (uint32_t)__builtin_amdgcn_mov_dpp((int)row[w], 0x4E, 0xF, 0xF, false);
            }
        }
        if (o.own) {
            uint32_t *hrow = a.hist + (int64_t)o.pix * a.hist_words;
#pragma unroll
            for (int w = 0; w < 8; ++w) {
                if (w < a.hist_words && row[w] != 0u) {
                    if (quad) {
                        if ((w & (tpp - 1)) == o.grp) hrow[w] = orow[w] + row[w];
                    } else {
                        atomicAdd(hrow + w, row[w]);
                    }
                }
            }
        }
    }
}

// Schedule of a single-lattice launch: from the host-filled arguments.
struct ArgSchedule {
    const TbArgs &b;
    __device__ double beta(int s) const { return b.beta[s]; }
    // (from a mask in the arguments: no per-sweep load of beta while it stays the same)
    __device__ bool beta_changes(int s, double) const { return (b.beta_mask >> s) & 1u; }
    __device__ bool acc(int s) const { return (b.acc_mask >> s) & 1u; }
    __device__ bool tally(int s) const { return (b.tally_mask >> s) & 1u; }
    __device__ bool any_acc() const { return b.acc_mask != 0u; }
    __device__ bool any_tally() const { return b.tally_mask != 0u; }
};

template <int G, int NBR, int LB, int IMAX, int BLK>
__global__ __launch_bounds__(BLK) void tb_sweep_kernel(TbArgs b)
{
    extern __shared__ __align__(16) unsigned char lds[];
    tb_tile<G, NBR, LB, IMAX, BLK>(b.a, (int)blockIdx.x, b.TH, b.tiles_w, b.S, b.ptab_n, ArgSchedule{b}, lds);
}

// Schedule of a lattice in a batched launch: from its descriptor, sweeps t0 .. t0+S-1.
struct DescSchedule {
    const ImageDesc &d;
    uint32_t t0;
    int S;
    __device__ double beta(int s) const
    {
        const uint32_t t = t0 + (uint32_t)s;
        return d.beta_len == 0 ? 1.0 : d.beta[t < (uint32_t)d.beta_len ? t : (uint32_t)(d.beta_len - 1)];
    }
    __device__ bool beta_changes(int s, double prev) const { return d.beta_len > 0 && beta(s) != prev; }
    __device__ bool acc(int s) const { return (int64_t)(t0 + (uint32_t)s) >= d.burn_in; }
    __device__ bool tally(int s) const
    {
        const int64_t t = (int64_t)(t0 + (uint32_t)s);
        return t >= d.burn_in && d.tally_stride > 0 && (t - d.burn_in) % d.tally_stride == 0;
    }
    __device__ bool any_acc() const { return acc(S - 1); }
    __device__ bool any_tally() const
    {
        bool any = false;
        for (int s = 0; s < S; ++s) any = any || tally(s);
        return any;
    }
};

// Several sweeps of every lattice a batch runs from LDS tiles (the batch's "multi-sweep"
// traversal): workgroup -> lattice by a table, each lattice's tiles consecutive.  S is odd,
// so a lattice's state after the launch is in the buffer of its new sweep index's parity,
// as the one-sweep launches keep it.  The level bound is chosen per lattice.
template <int G, int NBR, int BLK>
__global__ __launch_bounds__(BLK) void tb_batch_kernel(TbBatchLaunch L)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const int img = L.block_img[blockIdx.x];
    const ImageDesc &d = L.imgs[img];
    const uint32_t t0 = d.t + L.toff;
    // A batch's lattices run to the same sweep index (t_end is 2^32 - 1, and the host keeps
    // t0 + S below it), so S is the launch's odd count; only the request server ends lattices
    // early, and it does not use this traversal.
    if (t0 >= d.t_end) return;
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
    const int tile = (int)blockIdx.x - d.block_base;
    const int side = d.tb_side, pn = NBR * d.T + 1;
    const DescSchedule sch{d, t0, S};
    switch (tb_levels(d.L)) {
    case 2: tb_tile<G, NBR, 2, kTbBatchItems, BLK>(a, tile, side, d.tiles_w, S, pn, sch, lds); break;
    case 4: tb_tile<G, NBR, 4, kTbBatchItems, BLK>(a, tile, side, d.tiles_w, S, pn, sch, lds); break;
    case 8: tb_tile<G, NBR, 8, kTbBatchItems, BLK>(a, tile, side, d.tiles_w, S, pn, sch, lds); break;
    default: tb_tile<G, NBR, 16, kTbBatchItems, BLK>(a, tile, side, d.tiles_w, S, pn, sch, lds); break;
    }
}

template <int G, int NBR, int LB>
hipError_t launch_tb_l(const TbArgs &b, size_t lds_bytes, hipStream_t s)
{
    hipLaunchKernelGGL((tb_sweep_kernel<G, NBR, LB, kTbItems, kTbBlock>), dim3((unsigned)b.tiles), dim3(kTbBlock),
                       lds_bytes, s, b);
    return hipGetLastError();
}

template <int G, int NBR>
hipError_t launch_tb_g(const TbArgs &b, size_t lds_bytes, hipStream_t s)
{
    switch (tb_levels(b.a.L)) {
    case 2: return launch_tb_l<G, NBR, 2>(b, lds_bytes, s);
    case 4: return launch_tb_l<G, NBR, 4>(b, lds_bytes, s);
    case 8: return launch_tb_l<G, NBR, 8>(b, lds_bytes, s);
    default: return launch_tb_l<G, NBR, 16>(b, lds_bytes, s);
    }
}

template <int G, int NBR>
hipError_t launch_tb_batch_g(const TbBatchLaunch &L, int blocks, size_t lds_bytes, hipStream_t s)
{
    hipLaunchKernelGGL((tb_batch_kernel<G, NBR, kTbBatchBlock>), dim3((unsigned)blocks), dim3(kTbBatchBlock), lds_bytes,
                       s, L);
    return hipGetLastError();
}

// Loaded region along one axis (upper bound over the tiles) and the items of sweep 0.
int tb_region(int n, int side, int S) { return std::min(n, side + 2 * S); }
int64_t tb_items(int side, int S, int tpp) { return (int64_t)(side + 2 * (S - 1)) * (side + 2 * (S - 1)) * tpp; }

}  // namespace

bool tb_fits(int H, int W, int Cp, int G, int side, int S, int ptab_n, int imax, int block)
{
    const int64_t tpp = Cp / G;
    if ((int64_t)side * side * tpp > block) return false;  // the tile's own items in slot 0
    if (tb_items(side, S, (int)tpp) > (int64_t)imax * block) return false;
    return tb_lds_bytes(H, W, Cp, side, S, ptab_n) <= (size_t)kTbMaxLds;
}

size_t tb_lds_bytes(int H, int W, int Cp, int side, int S, int ptab_n)
{
    return (size_t)tb_lds_layout(tb_region(H, side, S), tb_region(W, side, S), Cp, ptab_n).bytes;
}

hipError_t launch_tb_batch(const TbBatchLaunch &L, int blocks, int G, int nbr, size_t lds_bytes, hipStream_t s)
{
    if (nbr == 8) {
        if (G == 4) return launch_tb_batch_g<4, 8>(L, blocks, lds_bytes, s);
        if (G == 2) return launch_tb_batch_g<2, 8>(L, blocks, lds_bytes, s);
        return launch_tb_batch_g<1, 8>(L, blocks, lds_bytes, s);
    }
    if (G == 4) return launch_tb_batch_g<4, 4>(L, blocks, lds_bytes, s);
    if (G == 2) return launch_tb_batch_g<2, 4>(L, blocks, lds_bytes, s);
    return launch_tb_batch_g<1, 4>(L, blocks, lds_bytes, s);
}

TbPlan tb_plan(int H, int W, int L, int Cp, int nbr, int T, int inertia)
{
    TbPlan pl{};
    if (L > 16 || inertia != 0) return pl;
    // Only lattices whose single-sweep launch has at most four threads per lane of the GPU
    // (256 CUs x 4 SIMDs x 64, four waves per SIMD): there a sweep costs a launch and little
    // more than one site's latency, which several sweeps per launch amortise.  Measured (us
    // per sweep, several against one sweep per launch, results identical): 256 x 256, one
    // chain, 5 levels, 8 neighbours 1.97 / 4.47; 384 x 384, one chain, 16 levels 4.44 / 5.90;
    // 256 x 256, 8 chains, 16 levels 5.88 / 6.66; 512 x 512, one chain, 9 levels, 8 neighbours
    // 6.35 / 7.15, 16 levels 5.71 / 7.46, 2 levels 3.44 / 5.40.  Beyond that the halo's extra
    // work and the barriers cost more than they save (512 x 512, 8 chains, 16 levels: 22.2
    // against 16.1).
    const int G = chain_group(Cp);
    if ((int64_t)H * W * (Cp / G) > kTbMaxThreads) return pl;
    // Tiles as large as keep every compute unit busy (about one workgroup each), down to
    // 4x4; the most sweeps per launch (12, else 10, 8, 4 or 2) whose items fit two per
    // thread.  Measured on 64x64, 1 chain, L = 2, 4x4 tiles (us per sweep): 512 threads per
    // workgroup, 10 sweeps per launch 1.03, 12 1.02, 14 1.05, 16 1.25; 256 threads, 8 sweeps
    // 1.15, 10 1.10, 12 1.30; 1024 threads, 12 to 20 sweeps 1.11 to 1.19; 8x8 tiles with
    // 512 threads and 10 or 12 sweeps 1.07, 1.08.
    static const int kSides[3] = {16, 8, 4};
    static const int kSweeps[5] = {12, 10, 8, 4, 2};
    for (int i = 0; i < 3; ++i) {
        const int side = kSides[i];
        const int64_t tiles = (int64_t)((H + side - 1) / side) * ((W + side - 1) / side);
        if (tiles < 240 && side > 4) continue;
        for (int j = 0; j < 5; ++j) {
            const int S = kSweeps[j];
            if (!tb_fits(H, W, Cp, G, side, S, nbr * T + 1, kTbItems, kTbBlock)) continue;
            pl.TH = pl.TW = side;
            pl.S = S;
            pl.tiles_w = (W + side - 1) / side;
            pl.tiles = (int)tiles;
            return pl;
        }
        return pl;
    }
    return pl;
}

hipError_t launch_tb_sweeps(const TbArgs &b, hipStream_t s)
{
    const int G = chain_group(b.a.C);
    const size_t lds = tb_lds_bytes(b.a.H, b.a.W, b.a.Cp, b.TH, b.S, b.ptab_n);
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
