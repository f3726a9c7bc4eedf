// Device code shared by the gfx950 kernels of the lazy PCA sampler (Costarelli, Piconi, Troiani, arXiv 2507.14869,
// Sec. 5.2).  The path is bound by vector ALU work (L level evaluations per site
// update), so the kernels are written for VALU throughput: no MFMA (there is no dense
// contraction), one thread per (pixel, group of up to four chains), chain-interleaved
// uint8 state so one dword load brings a pixel's four chain values, the neighbour
// statistic from byte-wise sums of absolute differences, and the per-sweep prior
// factor table in LDS.
//
// Arithmetic of one site update (identical, operation for operation, to the written
// convention the CPU reference follows; FP32, round to nearest even, no implicit
// contraction - the file is built with -ffp-contract=off):
//   exp2s(y)  = 0 if y < -125, else ldexp(p(f), n) with n = rint(y), f = y - n and p the
//               degree-6 Taylor polynomial of 2^f (coefficients (float)(ln2^k / k!), the
//               double values built as t_k = (t_{k-1} * ln2) / k), evaluated by fma Horner.
//   D_k       = exp2s(fma(-a2, e_k*e_k, m)), e_k = g' - k, m = a2*(e0*e0), e0 = g' - khat,
//               khat = clamp(rint(g'), 0, L-1), a2 = (float)(log2e / ((2 s) s)), s = sigma
//               in level units: the Gaussian data term of Sec. 4, not scaled by beta.
//   P(S)      = exp2s(-(c2 * S)), c2 = (float)(((beta*J)*kappa)*log2e), S = sum over
//               in-lattice neighbours of min(|k - x_j|, T): the pair prior (Potts counts
//               disagreeing neighbours with kappa = 2, T = 1).
//   R         = exp2s((float)((beta*q)*log2e)) - 1: the inertia of Sec. 5.2 written as an
//               extra "stay" weight, P(k|x) ~ D_k P(S_k) + [k = x] D_x P(S_x) R.
//   acc_{-1}  = (D_x * P(S_x)) * R, acc_k = fma(D_k, P(S_k), acc_{k-1}), Z = acc_{L-1}.
//   draw      = x if acc_{-1} > u Z, else the least k with acc_k > u Z (exact comparison,
//               done as acc > RD(u Z)); x if Z == 0.  u = (r >> 8) 2^-24, r the chain's
//               Philox4x32-10 word for counter {pixel, t, chain/4, 0}.
// Inertia q|k - x|^p with p = 1 or 2 (Sec. 3, "The lazy PCA"; the L1/L2 norms of Sec. 5.2)
// replaces the stay weight by one exponent per (chain, level) that holds both the data
// and the inertia term, shifted by its maximum over the levels:
//   F_k = fma(-a2, e_k*e_k, -(q2 * d^p)), d = |k - x|, q2 = (float)((beta*q)*log2e),
//   acc_{-1} = 0, acc_k = fma(exp2s(F_k - Fmax), P(S_k), acc_{k-1}),
//   Fmax = max(F_k1, F_k2), k1 = clamp(floor(kc), 0, L-1), k2 = min(k1+1, L-1), kc the
//   real maximiser: clamp(x, g' - h, g' + h) with h = q2/(2 a2) for p = 1,
//   (a2 g' + q2 x)/(a2 + q2) for p = 2.
#pragma once

#include "pca_internal.h"

namespace pcak {
namespace {


// ---------------------------------------------------------------- exp2s

constexpr double taylor_coeff(int k)
{
    double t = 1.0;
    for (int i = 1; i <= k; ++i) t = (t * kLn2) / (double)i;
    return t;
}

constexpr float kP0 = (float)taylor_coeff(0);
constexpr float kP1 = (float)taylor_coeff(1);
constexpr float kP2 = (float)taylor_coeff(2);
constexpr float kP3 = (float)taylor_coeff(3);
constexpr float kP4 = (float)taylor_coeff(4);
constexpr float kP5 = (float)taylor_coeff(5);
constexpr float kP6 = (float)taylor_coeff(6);

__device__ __forceinline__ float exp2s(float y)
{
    const float n = __builtin_rintf(y);
    const float f = y - n;
    float p = kP6;
    p = __builtin_fmaf(p, f, kP5);
    p = __builtin_fmaf(p, f, kP4);
    p = __builtin_fmaf(p, f, kP3);
    p = __builtin_fmaf(p, f, kP2);
    p = __builtin_fmaf(p, f, kP1);
    p = __builtin_fmaf(p, f, kP0);
    const float r = __builtin_amdgcn_ldexpf(p, (int)n);
    return y < -125.0f ? 0.0f : r;
}

// ---------------------------------------------------------------- Philox4x32-10

struct U4 {
    uint32_t x, y, z, w;
};

// WIDE: each 32x32-bit product as one 64-bit multiply (v_mad_u64_u32, cheaper than a low
// and a high multiply; used where registers are not scarce: the kernels for L <= 16 spill
// nothing, while in the 16-level-block kernels the register pairs cost extra spills).
template <bool WIDE = false>
__device__ __forceinline__ U4 philox(U4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint32_t lo0, hi0, lo1, hi1;
        if constexpr (WIDE) {
            const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
            const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
            lo0 = (uint32_t)p0;
            hi0 = (uint32_t)(p0 >> 32);
            lo1 = (uint32_t)p1;
            hi1 = (uint32_t)(p1 >> 32);
        } else {
            lo0 = 0xD2511F53u * c.x;
            hi0 = __umulhi(0xD2511F53u, c.x);
            lo1 = 0xCD9E8D57u * c.z;
            hi1 = __umulhi(0xCD9E8D57u, c.z);
        }
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    }
    return c;
}

__device__ __forceinline__ uint32_t word_of(const U4 &r, int i)
{
    return i == 0 ? r.x : i == 1 ? r.y : i == 2 ? r.z : r.w;
}

// Round-down of the exact product u*Z (both FP32, exact in double).
__device__ __forceinline__ float threshold_rd(float u, float Z)
{
    const double t = (double)u * (double)Z;
    float f = (float)t;
    if ((double)f > t) f = __uint_as_float(__float_as_uint(f) - 1u);  // f > t >= 0
    return f;
}

template <int G>
__device__ __forceinline__ uint32_t load_group(const uint8_t *p)
{
    if constexpr (G == 4) return *reinterpret_cast<const uint32_t *>(p);
    else if constexpr (G == 2) return *reinterpret_cast<const uint16_t *>(p);
    else return *p;
}

template <int G>
__device__ __forceinline__ void store_group(uint8_t *p, uint32_t v)
{
    if constexpr (G == 4) *reinterpret_cast<uint32_t *>(p) = v;
    else if constexpr (G == 2) *reinterpret_cast<uint16_t *>(p) = (uint16_t)v;
    else *p = (uint8_t)v;
}

// ---------------------------------------------------------------- sweep

// Byte transpose of four state words (byte ch of word j = chain ch's level at neighbour j)
// into X[ch] = the chain's four neighbour levels (byte j = neighbour j), for the G chains.
template <int G>
__device__ __forceinline__ void transpose_group(uint32_t A, uint32_t B, uint32_t C, uint32_t D, uint32_t (&X)[G])
{
    // v_perm_b32 picks bytes of {src0:src1}: selector 0-3 = src1's bytes, 4-7 = src0's
    const uint32_t ab01 = __builtin_amdgcn_perm(B, A, 0x05010400u);  // A0 B0 A1 B1
    const uint32_t cd01 = __builtin_amdgcn_perm(D, C, 0x05010400u);  // C0 D0 C1 D1
    X[0] = __builtin_amdgcn_perm(cd01, ab01, 0x05040100u);           // A0 B0 C0 D0
    if constexpr (G >= 2) X[1] = __builtin_amdgcn_perm(cd01, ab01, 0x07060302u);  // A1 B1 C1 D1
    if constexpr (G == 4) {
        const uint32_t ab23 = __builtin_amdgcn_perm(B, A, 0x07030602u);  // A2 B2 A3 B3
        const uint32_t cd23 = __builtin_amdgcn_perm(D, C, 0x07030602u);  // C2 D2 C3 D3
        X[2] = __builtin_amdgcn_perm(cd23, ab23, 0x05040100u);
        X[3] = __builtin_amdgcn_perm(cd23, ab23, 0x07060302u);
    }
}

// Per-chain neighbour data for the byte-wise statistic.  With lo_j = max(x_j - T_j, 0),
// hi_j = min(x_j + T_j, 255) and T_j = 0 for absent neighbours, for every k in [0, 255]
//   2 min(|k - x_j|, T_j) = 2|k - x_j| - |k - hi_j| - |k - lo_j| + (hi_j - lo_j),
// so 2S_k = 2 SAD(k, x) - SAD(k, hi) - SAD(k, lo) + sum_j (hi_j - lo_j), each SAD one
// v_sad_u8 over four neighbours packed in a dword.
template <int NW>
struct NbrPack {
    uint32_t x[NW], lo[NW], hi[NW];
    int cb;  // 2 * sum_j (hi_j - lo_j): byte offset term of the table address
};

template <int NW>
__device__ __forceinline__ float prior_lookup(const char *ptab, const NbrPack<NW> &nb, uint32_t kk)
{
    uint32_t u = 0, v = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        u = __builtin_amdgcn_sad_u8(kk, nb.x[w], u);
        v = __builtin_amdgcn_sad_u8(kk, nb.lo[w], v);
        v = __builtin_amdgcn_sad_u8(kk, nb.hi[w], v);
    }
    // byte offset 4 S = 4u - 2v + 2 sum(hi - lo), as one shift-add and one 24-bit mad
    int off;
    asm("v_lshl_add_u32 %0, %1, 2, %2\n\tv_mad_i32_i24 %0, %3, -2, %0" : "=&v"(off) : "v"(u), "v"(nb.cb), "v"(v));
    return *reinterpret_cast<const float *>(ptab + off);
}

// Broadcast lane J of each group of SHARE consecutive lanes to the whole group (DPP
// quad permutation; groups never straddle a quad).
template <int SHARE, int J>
__device__ __forceinline__ float group_bcast(float v)
{
    if constexpr (SHARE == 1) {
        return v;
    } else {
        constexpr int ctrl = SHARE == 4 ? (J | (J << 2) | (J << 4) | (J << 6))
                                        : (J | (J << 2) | ((2 + J) << 4) | ((2 + J) << 6));
        return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), ctrl, 0xF, 0xF, false));
    }
}

// GROUPED issues all G table reads before the first is consumed, so their LDS latencies
// overlap (used in the 16-level blocks; the L <= 16 path measured faster without).
template <int G, int NW, bool GROUPED = true>
__device__ __forceinline__ void level_update(const char *pt, const NbrPack<NW> (&nb)[G], float (&acc)[G], float D,
                                             uint32_t kk)
{
    if constexpr (GROUPED) {
        float P[G];
#pragma unroll
        for (int ch = 0; ch < G; ++ch) P[ch] = prior_lookup<NW>(pt, nb[ch], kk);
#pragma unroll
        for (int ch = 0; ch < G; ++ch) acc[ch] = __builtin_fmaf(D, P[ch], acc[ch]);
    } else {
#pragma unroll
        for (int ch = 0; ch < G; ++ch) acc[ch] = __builtin_fmaf(D, prior_lookup<NW>(pt, nb[ch], kk), acc[ch]);
    }
}

// Levels J.. of a group of SHARE consecutive levels; only the first nlev exist.
template <int SHARE, int J, int G, int NW>
__device__ __forceinline__ void group_levels(const char *pt, const NbrPack<NW> (&nb)[G], float (&acc)[G], float Dmine,
                                             uint32_t &kk, int nlev)
{
    if constexpr (J < SHARE) {
        if (J < nlev) {
            level_update<G, NW>(pt, nb, acc, group_bcast<SHARE, J>(Dmine), kk);
            kk += 0x01010101u;
            group_levels<SHARE, J + 1, G, NW>(pt, nb, acc, Dmine, kk, nlev);
        }
    }
}

// All SHARE levels of a group.
template <int SHARE, int J, int G, int NW>
__device__ __forceinline__ void group_full(const char *pt, const NbrPack<NW> (&nb)[G], float (&acc)[G], float Dmine,
                                           uint32_t &kk)
{
    if constexpr (J < SHARE) {
        level_update<G, NW>(pt, nb, acc, group_bcast<SHARE, J>(Dmine), kk);
        kk += 0x01010101u;
        group_full<SHARE, J + 1, G, NW>(pt, nb, acc, Dmine, kk);
    }
}

// Levels J.. of a group of SHARE consecutive levels where every chain's neighbour
// statistic is at its maximum: the prior factor is the same table entry for all of them.
template <int SHARE, int J, int G>
__device__ __forceinline__ void group_far(float (&acc)[G], float Dmine, float pfar)
{
    if constexpr (J < SHARE) {
        const float D = group_bcast<SHARE, J>(Dmine);
#pragma unroll
        for (int ch = 0; ch < G; ++ch) acc[ch] = __builtin_fmaf(D, pfar, acc[ch]);
        group_far<SHARE, J + 1, G>(acc, Dmine, pfar);
    }
}

// Per-sweep scalars shared by a workgroup, and the prior factor table P(S), S = 0..nbr*T,
// in LDS.  Every thread of the workgroup must call this (it ends with a barrier).
struct SweepConsts {
    float R, a2, q2;
};

// FP32 constants of a sweep from the run parameters and the sweep's beta (fixed operation
// order, identical in every kernel).
__device__ __forceinline__ SweepConsts sweep_constants(const SweepArgs &a)
{
    const float q2 = (float)((a.beta * a.q) * kLog2e);
    SweepConsts k;
    k.R = exp2s(q2) - 1.0f;
    k.q2 = q2;
    k.a2 = (float)(kLog2e / ((2.0 * a.sigma_s) * a.sigma_s));
    return k;
}

// Entries s = first, first + stride, ... of the prior factor table P(S) = exp2s(-(c2 S)),
// S = 0..nbr*T.
__device__ __forceinline__ void fill_prior_table(const SweepArgs &a, int nbr, float *ptab, int first, int stride)
{
    const float c2 = (float)(((a.beta * a.J) * a.kappa) * kLog2e);
    const int nP = nbr * a.T + 1;
    for (int s = first; s < nP; s += stride) ptab[s] = exp2s(-(c2 * (float)s));
}

// Statistic table of the few-level kernels (L <= 16): entry x (a neighbour's level, 0..15)
// holds, in byte k of its 16 bytes, one neighbour's term of the statistic S_k: with four
// neighbours 4 min(|k - x|, T), its share of the byte offset 4 S_k of P(S_k) in the prior
// table, with eight min(|k - x|, T); entry 16 (an absent neighbour) is 0.  A chain's 16
// statistics are then the bytewise sum of its neighbours' entries (at most 4 * 4 * 15 or
// 8 * 15, below 256: no carries between bytes).
constexpr int kStatEntries = 17;

__device__ __forceinline__ void fill_stat_table(const SweepArgs &a, int nbr, uint32_t *vtab, int first, int stride)
{
    const int scale = nbr == 4 ? 4 : 1;
    for (int i = first; i < kStatEntries * 4; i += stride) {
        const int x = i >> 2;
        uint32_t w = 0u;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int k = 4 * (i & 3) + b;
            const int d = k > x ? k - x : x - k;
            const int v = x < 16 ? scale * (d < a.T ? d : a.T) : 0;
            w |= (uint32_t)v << (8 * b);
        }
        vtab[i] = w;
    }
}

// vtab: the statistic table, filled for the few-level path (may be null).
__device__ __forceinline__ SweepConsts sweep_prologue(const SweepArgs &a, int nbr, float *ptab, uint4 *vtab = nullptr)
{
    const SweepConsts k = sweep_constants(a);
    fill_prior_table(a, nbr, ptab, threadIdx.x, blockDim.x);
    if (vtab && a.L <= 16) fill_stat_table(a, nbr, reinterpret_cast<uint32_t *>(vtab), threadIdx.x, blockDim.x);
    __syncthreads();
    return k;
}

// Exponent F_k of the L1/L2 inertia form: data term plus q2 |k - x|^p (log2 units).
__device__ __forceinline__ float inertia_exponent(float ee, int k, int x, int p, float a2, float q2)
{
    const int d = k > x ? k - x : x - k;
    const int dp = p == 1 ? d : d * d;
    return __builtin_fmaf(-a2, ee, -(q2 * (float)dp));
}

// Maximum of F_k over the levels: F is concave in k, so it is attained next to the
// maximiser kc of the real-valued form.
__device__ __forceinline__ float inertia_fmax(float gp, int x, int L, int p, float a2, float q2)
{
    float kc;
    if (p == 1) {
        const float h = q2 / (2.0f * a2);
        kc = fminf(fmaxf((float)x, gp - h), gp + h);
    } else {
        kc = (a2 * gp + q2 * (float)x) / (a2 + q2);
    }
    const int k1 = (int)fminf(fmaxf(floorf(kc), 0.0f), (float)(L - 1));
    const int k2 = k1 + 1 < L ? k1 + 1 : k1;
    const float e1 = gp - (float)k1, e2 = gp - (float)k2;
    const float F1 = inertia_exponent(e1 * e1, k1, x, p, a2, q2);
    const float F2 = inertia_exponent(e2 * e2, k2, x, p, a2, q2);
    return F1 > F2 ? F1 : F2;
}

// First index b in [0, 16) with part[b][ch] > tf, given that part[.][ch] is nondecreasing
// and part[15][ch] > tf: a branch-free binary search (halving the candidates four times).
template <int G>
__device__ __forceinline__ int first_above(const float (&part)[16][G], int ch, float tf)
{
    float v8[8], v4[4], v2[2];
    const bool c8 = part[7][ch] > tf;
#pragma unroll
    for (int i = 0; i < 8; ++i) v8[i] = c8 ? part[i][ch] : part[8 + i][ch];
    int base = c8 ? 0 : 8;
    const bool c4 = v8[3] > tf;
#pragma unroll
    for (int i = 0; i < 4; ++i) v4[i] = c4 ? v8[i] : v8[4 + i];
    base += c4 ? 0 : 4;
    const bool c2 = v4[1] > tf;
#pragma unroll
    for (int i = 0; i < 2; ++i) v2[i] = c2 ? v4[i] : v4[2 + i];
    base += c2 ? 0 : 2;
    return base + (v2[0] > tf ? 0 : 1);
}

// What one thread's site updates read: the observation, its chain group's current levels
// and those of each neighbour, however the caller holds the state (global memory or an
// LDS tile).
template <int NBR>
struct SiteInputs {
    float gp;            // observation in level units
    uint32_t own;        // byte ch: level of chain grp*G + ch at this pixel
    uint32_t nbw[NBR];   // the same for each neighbour (0 if absent)
    bool present[NBR];   // neighbour inside the lattice
};

// Neighbour offsets (row, column); the first four are the 4-neighbourhood.
__device__ constexpr int kNbrDr[8] = {-1, 1, 0, 0, -1, -1, 1, 1};
__device__ constexpr int kNbrDc[8] = {0, 0, -1, 1, -1, 1, -1, 1};

// One thread's site updates: pixel `pix`, chains grp*G .. grp*G+G-1, from the inputs `in`.
// `q` is the thread's position in its group of SHARE lanes serving the same pixel.  Returns
// the new levels packed one per byte and also in knew.
// INR selects the L1/L2 inertia form (a.inertia = 1 or 2; SHARE must then be 1).
template <int G, int NBR, int SUB, int NBLK, int SHARE, bool INR = false>
__device__ __forceinline__ uint32_t site_draw(const SweepArgs &a, const float *ptab, const uint4 *vtab, SweepConsts kc,
                                              const SiteInputs<NBR> &in, int pix, int grp, int q, int (&knew)[G])
{
    constexpr int NW = NBR / 4;
    // the few-level path (indicator inertia) reads its neighbour statistics from the
    // statistic table; byte k of a chain's sum is 4 S_k (4 neighbours) or S_k (8)
    constexpr bool STAT = SUB == 1 && !INR;
    constexpr int kOffShift = NBR == 4 ? 0 : 2;
    const float R = kc.R;
    const float a2 = kc.a2;
    const int cofs = grp * G;
    const int L = a.L;

    // Observation and the data-term shift.
    const float gp = in.gp;
    float khat = __builtin_rintf(gp);
    khat = khat < 0.0f ? 0.0f : khat;
    khat = khat > (float)(L - 1) ? (float)(L - 1) : khat;
    const float e0 = gp - khat;
    const float m = a2 * (e0 * e0);

    const uint32_t own = in.own;
    uint32_t nbw[NBR];
    bool present[NBR];
#pragma unroll
    for (int j = 0; j < NBR; ++j) {
        nbw[j] = in.nbw[j];
        present[j] = in.present[j];
    }

    const char *pt = reinterpret_cast<const char *>(ptab);
    NbrPack<NW> nb[G];
    int xs[G];
    float stay[G], acc[G], fmx[G];
    // Levels outside [nlo, nhi] are at least T away from every present neighbour of every
    // chain of this thread, so their statistic is npres*T.
    int nlo = 1 << 20, nhi = -(1 << 20), npres = 0;
#pragma unroll
    for (int j = 0; j < NBR; ++j) npres += present[j] ? 1 : 0;
    uint32_t sv[G][4];  // STAT: byte k of sv[ch][k / 4] is S_k of chain ch, times 4 with 4 neighbours
    if constexpr (STAT) {
#pragma unroll
        for (int ch = 0; ch < G; ++ch)
#pragma unroll
            for (int d = 0; d < 4; ++d) sv[ch][d] = 0u;
#pragma unroll
        for (int j = 0; j < NBR; ++j) {
            const uint32_t wj = present[j] ? nbw[j] : 0x10101010u;  // absent: entry 16
#pragma unroll
            for (int ch = 0; ch < G; ++ch) {
                const uint4 v = vtab[(wj >> (8 * ch)) & 0xFFu];
                sv[ch][0] += v.x;
                sv[ch][1] += v.y;
                sv[ch][2] += v.z;
                sv[ch][3] += v.w;
            }
        }
    } else if constexpr (SUB == 1) {
        // L <= 16, so every level and T are below 16: the four neighbours of a chain are
        // handled as the bytes of one dword (the state words transposed so that each
        // dword holds one chain's neighbours), hi = x + T needs no clamp and lo = max(x - T, 0)
        // is a bytewise saturating subtraction.  Absent neighbours have x = lo = hi = 0.
        uint32_t tm[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) tm[w] = 0u;
#pragma unroll
        for (int j = 0; j < NBR; ++j)
            if (present[j]) tm[j / 4] |= (uint32_t)a.T << (8 * (j % 4));
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            uint32_t X[G];
            transpose_group<G>(nbw[4 * w], nbw[4 * w + 1], nbw[4 * w + 2], nbw[4 * w + 3], X);
#pragma unroll
            for (int ch = 0; ch < G; ++ch) {
                const uint32_t hi = X[ch] + tm[w];
                const uint32_t d = (X[ch] | 0x80808080u) - tm[w];  // byte: x - T + 128, no borrows
                const uint32_t ge = (d & 0x80808080u) >> 7;         // byte: 1 where x >= T
                const uint32_t lo = (d ^ 0x80808080u) & (ge * 0xFFu);
                nb[ch].x[w] = X[ch];
                nb[ch].lo[w] = lo;
                nb[ch].hi[w] = hi;
                // sum_j (hi_j - lo_j) over this dword's neighbours, twice
                nb[ch].cb = __builtin_amdgcn_sad_u8(hi, lo, w == 0 ? 0u : (uint32_t)nb[ch].cb);
            }
        }
#pragma unroll
        for (int ch = 0; ch < G; ++ch) nb[ch].cb *= 2;
    }
#pragma unroll
    for (int ch = 0; ch < G; ++ch) {
        xs[ch] = (int)((own >> (8 * ch)) & 0xFFu);
        int csum = 0;
#pragma unroll
        for (int w = 0; w < NW && SUB > 1; ++w) {
            nb[ch].x[w] = nb[ch].lo[w] = nb[ch].hi[w] = 0u;
        }
#pragma unroll
        for (int j = 0; j < NBR && SUB > 1; ++j) {
            const int xj = (int)((nbw[j] >> (8 * ch)) & 0xFFu);
            const int Tj = present[j] ? a.T : 0;
            const int lo = xj > Tj ? xj - Tj : 0;
            const int hi = xj + Tj < 255 ? xj + Tj : 255;
            csum += hi - lo;
            if (present[j]) {
                nlo = xj - a.T + 1 < nlo ? xj - a.T + 1 : nlo;
                nhi = xj + a.T - 1 > nhi ? xj + a.T - 1 : nhi;
            }
            nb[ch].x[j / 4] |= (uint32_t)xj << (8 * (j % 4));
            nb[ch].lo[j / 4] |= (uint32_t)lo << (8 * (j % 4));
            nb[ch].hi[j / 4] |= (uint32_t)hi << (8 * (j % 4));
        }
        if constexpr (SUB > 1) nb[ch].cb = 2 * csum;
        if constexpr (INR) {
            fmx[ch] = inertia_fmax(gp, xs[ch], L, a.inertia, a2, kc.q2);
            stay[ch] = 0.0f;
        } else {
            // Stay weight of the lazy conditional.
            const float ex = gp - (float)xs[ch];
            const float Dx = exp2s(__builtin_fmaf(-a2, ex * ex, m));
            float Px;
            if constexpr (STAT) {
                const int x = xs[ch];
                // selects of opaque values (selects of the array's elements would be folded
                // into an indexed load, which puts the array in scratch memory)
                uint32_t s0 = sv[ch][0], s1 = sv[ch][1], s2 = sv[ch][2], s3 = sv[ch][3];
                asm("" : "+v"(s0), "+v"(s1), "+v"(s2), "+v"(s3));
                const uint32_t w01 = (x & 4) ? s1 : s0, w23 = (x & 4) ? s3 : s2;
                const uint32_t w = (x & 8) ? w23 : w01;
                Px = *reinterpret_cast<const float *>(pt + (((w >> (8 * (x & 3))) & 0xFFu) << kOffShift));
            } else {
                Px = prior_lookup<NW>(pt, nb[ch], (uint32_t)xs[ch] * 0x01010101u);
            }
            stay[ch] = (Dx * Px) * R;
        }
        acc[ch] = stay[ch];
    }

    // Levels below flo are below nlo for every lane of the wave, levels above fhi above
    // every lane's nhi: there every chain's statistic is npres*T (the lane's own npres), so
    // the prior factor is the table entry pfar.  Both bounds are wave-uniform, found by
    // binary search with wave votes over the active lanes (the predicates are monotone).
    int flo = 0, fhi = L - 1;
    if constexpr (SUB > 1) {
#pragma unroll
        for (int step = 256; step >= 1; step >>= 1) {
            if (flo + step <= L && __all(flo + step <= nlo)) flo += step;
            if (fhi - step >= -1 && __all(nhi <= fhi - step)) fhi -= step;
        }
    }
    const float pfar = ptab[npres * a.T];

    // Main pass over levels, keeping the running sum at the end of every block.  The
    // SHARE lanes serving one pixel each compute the data factor of every SHARE-th level
    // and broadcast it, so a pixel's chains share one evaluation per level.
    float part[NBLK][G];
    const int nblk = (L + SUB - 1) / SUB;
    uint32_t kk = 0u;
    float kq = (float)q;  // level whose data factor this lane evaluates next
    if constexpr (INR) {
        // L1/L2 inertia: every (chain, level) has its own exponent; nothing is shared.
#pragma unroll
        for (int b = 0; b < NBLK; ++b) {
            if (b < nblk) {
                const int kend = (L - b * SUB) < SUB ? (L - b * SUB) : SUB;
                // whole blocks only: a test per level in this loop measured slower
                if (b * SUB + kend - 1 < flo || b * SUB > fhi) {  // wave-uniform: block far
                    for (int i = 0; i < kend; ++i) {
                        const int k = b * SUB + i;
                        const float e = gp - (float)k;
                        const float ee = e * e;
#pragma unroll
                        for (int ch = 0; ch < G; ++ch) {
                            const float E = exp2s(inertia_exponent(ee, k, xs[ch], a.inertia, a2, kc.q2) - fmx[ch]);
                            acc[ch] = __builtin_fmaf(E, pfar, acc[ch]);
                        }
                    }
                    kk += (uint32_t)kend * 0x01010101u;
                } else {
                    for (int i = 0; i < kend; ++i) {
                        const int k = b * SUB + i;
                        const float e = gp - (float)k;
                        const float ee = e * e;
#pragma unroll
                        for (int ch = 0; ch < G; ++ch) {
                            const float E = exp2s(inertia_exponent(ee, k, xs[ch], a.inertia, a2, kc.q2) - fmx[ch]);
                            acc[ch] = __builtin_fmaf(E, prior_lookup<NW>(pt, nb[ch], kk), acc[ch]);
                        }
                        kk += 0x01010101u;
                    }
                }
            }
            // (slots past the last level keep Z, which the L <= 16 draw's search relies on)
#pragma unroll
            for (int ch = 0; ch < G; ++ch) part[b][ch] = acc[ch];
        }
    } else if constexpr (SUB == 1) {
#pragma unroll
        for (int k0 = 0; k0 < NBLK; k0 += SHARE) {
            if (k0 < L) {
                const float e = gp - kq;
                const float Dm = exp2s(__builtin_fmaf(-a2, e * e, m));
                kq += (float)SHARE;
#pragma unroll
                for (int j = 0; j < SHARE; ++j) {
                    if (k0 + j < L) {
                        float D;
                        if (j == 0) D = group_bcast<SHARE, 0>(Dm);
                        else if (j == 1) D = group_bcast<SHARE, (SHARE > 1 ? 1 : 0)>(Dm);
                        else if (j == 2) D = group_bcast<SHARE, (SHARE > 2 ? 2 : 0)>(Dm);
                        else D = group_bcast<SHARE, (SHARE > 3 ? 3 : 0)>(Dm);
                        if constexpr (STAT) {
                            const int k = k0 + j;
#pragma unroll
                            for (int ch = 0; ch < G; ++ch) {
                                const uint32_t off = ((sv[ch][k >> 2] >> (8 * (k & 3))) & 0xFFu) << kOffShift;
                                acc[ch] = __builtin_fmaf(D, *reinterpret_cast<const float *>(pt + off), acc[ch]);
                            }
                        } else {
                            level_update<G, NW, false>(pt, nb, acc, D, kk);
                        }
                        kk += 0x01010101u;
                    }
                    // past the last level acc stays at Z, which the draw's search relies on
#pragma unroll
                    for (int ch = 0; ch < G; ++ch) part[k0 + j][ch] = acc[ch];
                }
            } else {
#pragma unroll
                for (int j = 0; j < SHARE; ++j)
#pragma unroll
                    for (int ch = 0; ch < G; ++ch) part[k0 + j][ch] = acc[ch];
            }
        }
    } else {
#pragma unroll
        for (int b = 0; b < NBLK; ++b) {
            if (b < nblk) {
                const int kend = (L - b * SUB) < SUB ? (L - b * SUB) : SUB;
                if (kend == SUB && SHARE == 4) {
                    // groups of 4 levels tested against the wave-uniform far bounds
#pragma unroll 2
                    for (int i = 0; i < SUB; i += SHARE) {
                        const int k = b * SUB + i;
                        const float e = gp - kq;
                        const float Dm = exp2s(__builtin_fmaf(-a2, e * e, m));
                        kq += (float)SHARE;
                        if (k + SHARE - 1 < flo || k > fhi) {
                            group_far<SHARE, 0, G>(acc, Dm, pfar);
                            kk += (uint32_t)SHARE * 0x01010101u;
                        } else {
                            group_full<SHARE, 0, G, NW>(pt, nb, acc, Dm, kk);
                        }
                    }
                } else if (kend == SUB && (b * SUB + SUB - 1 < flo || b * SUB > fhi)) {
                    // with fewer levels per group, whole blocks (a test per level or pair of
                    // levels measured slower)
#pragma unroll 2
                    for (int i = 0; i < SUB; i += SHARE) {
                        const float e = gp - kq;
                        const float Dm = exp2s(__builtin_fmaf(-a2, e * e, m));
                        kq += (float)SHARE;
                        group_far<SHARE, 0, G>(acc, Dm, pfar);
                    }
                    kk += (uint32_t)SUB * 0x01010101u;
                } else if (kend == SUB) {
#pragma unroll 2
                    for (int i = 0; i < SUB; i += SHARE) {
                        const float e = gp - kq;
                        const float Dm = exp2s(__builtin_fmaf(-a2, e * e, m));
                        kq += (float)SHARE;
                        group_full<SHARE, 0, G, NW>(pt, nb, acc, Dm, kk);
                    }
                } else {
                    for (int i = 0; i < kend; i += SHARE) {
                        const float e = gp - kq;
                        const float Dm = exp2s(__builtin_fmaf(-a2, e * e, m));
                        kq += (float)SHARE;
                        group_levels<SHARE, 0, G, NW>(pt, nb, acc, Dm, kk, kend - i);
                    }
                }
#pragma unroll
                for (int ch = 0; ch < G; ++ch) part[b][ch] = acc[ch];
            }
        }
    }

    // Inverse-CDF draw for each chain.
    const int chain0 = cofs;
    const U4 rnd = philox<SUB == 1>(U4{(uint32_t)pix, a.t, (uint32_t)(chain0 >> 2), 0u}, a.key0, a.key1);
    uint32_t packed = 0u;
#pragma unroll
    for (int ch = 0; ch < G; ++ch) {
        const uint32_t w = word_of(rnd, (chain0 & 3) + ch);
        const float u = (float)(w >> 8) * 0x1p-24f;
        const float Z = acc[ch];
        int k = xs[ch];
        if (Z != 0.0f) {
            const float tf = threshold_rd(u, Z);
            if (!(stay[ch] > tf)) {
                if constexpr (SUB == 1) {
                    // the running sums are nondecreasing and every slot past the last level
                    // holds Z > tf: binary search for the first one above tf
                    k = first_above(part, ch, tf);
                } else {
                    int bsel = nblk - 1;
                    float start = 0.0f;
#pragma unroll
                    for (int b = NBLK - 1; b >= 0; --b) {
                        if (b < nblk && part[b][ch] > tf) {
                            bsel = b;
                            start = b == 0 ? stay[ch] : part[b > 0 ? b - 1 : 0][ch];
                        }
                    }
                    // Re-run the sums of the selected block; they reproduce the main pass exactly.
                    // (A branch-free form evaluating all 16 levels measured 2% slower per sweep
                    // on 2048x2048, L = 256, 16 chains: more spills and no early exit.)
                    const int k0 = bsel * SUB;
                    const int kend = (L - k0) < SUB ? (L - k0) : SUB;
                    float s = start;
                    k = k0 + kend - 1;
                    uint32_t kk2 = (uint32_t)k0 * 0x01010101u;
                    for (int i = 0; i < kend; ++i) {
                        float D;
                        if constexpr (INR) {
                            const float e = gp - (float)(k0 + i);
                            D = exp2s(inertia_exponent(e * e, k0 + i, xs[ch], a.inertia, a2, kc.q2) - fmx[ch]);
                        } else {
                            const float e = gp - (float)(k0 + i);
                            D = exp2s(__builtin_fmaf(-a2, e * e, m));
                        }
                        const float P = prior_lookup<NW>(pt, nb[ch], kk2);
                        s = __builtin_fmaf(D, P, s);
                        if (s > tf) {
                            k = k0 + i;
                            break;
                        }
                        kk2 += 0x01010101u;
                    }
                }
            }
        }
        knew[ch] = k;
        packed |= (uint32_t)k << (8 * ch);
    }
    return packed;
}

// Tally of one thread's new levels: the level sum of its chains into sum[0] (a pixel's
// word), its chains' uint16 counters into the pixel's histogram row hrow (either may be
// null).  The tpp threads of a pixel are consecutive lanes; chains >= C (padding) count
// nothing.
// Words a thread updates, loaded before the level loop so their load latency overlaps it
// (valid = false: site_stats loads them itself).  Safe because no other thread of the
// launch writes them: each counter word and each pixel's sum has one owner.
struct StatsPrefetch {
    bool valid;
    uint32_t sum;      // the pixel's level sum (when this lane updates it)
    uint32_t row[8];   // the lane's histogram words, indexed by word (L <= 16 row path)
    uint4 q0, q1;      // full rows (row_in_quads): the lane's words 4 grp .. 4 grp + 3, and 4 .. 7
};

// A full histogram row (8 words: L = 15 or 16) with at most 15 chains and one or two lanes
// per pixel: each lane then owns a contiguous, 16-byte aligned run of the row (all 8 words,
// or words 4 grp .. 4 grp + 3) and moves it with 16-byte loads and stores instead of one
// access per word.
__device__ __forceinline__ bool row_in_quads(int hist_words, int C, int tpp)
{
    return hist_words == 8 && C <= 15 && (tpp == 1 || tpp == 2);
}

template <int G, int SUB>
__device__ __forceinline__ void site_stats(uint32_t *sum, uint32_t *hrow, int hist_words, int C, int tpp, int grp,
                                           const int (&knew)[G], const StatsPrefetch &pf = StatsPrefetch{false, 0u, {}, {}, {}})
{
    const int chain0 = grp * G;
    if (sum) {
        uint32_t lsum = 0u;
#pragma unroll
        for (int ch = 0; ch < G; ++ch)
            if (chain0 + ch < C) lsum += (uint32_t)knew[ch];
        // Lanes of a pixel sit in aligned pairs or quads when tpp is 2 or 4: add their sums
        // with DPP and let the first lane update the word, instead of one atomic per lane
        // (global atomics are performed past L2, one memory write each).
        if (tpp == 1) {
            *sum = (pf.valid ? pf.sum : *sum) + lsum;
        } else if (tpp == 2 || tpp == 4) {
            uint32_t s = lsum + (uint32_t)__builtin_amdgcn_mov_dpp((int)lsum, 0xB1, 0xF, 0xF, false);  // [1,0,3,2]
            if (tpp == 4) s += (uint32_t)__builtin_amdgcn_mov_dpp((int)s, 0x4E, 0xF, 0xF, false);      // [2,3,0,1]
            if (grp == 0) *sum = (pf.valid ? pf.sum : *sum) + s;
        } else {
            atomicAdd(sum, lsum);
        }
    }
    if (hrow) {
        if (SUB == 1 && row_in_quads(hist_words, C, tpp)) {
            // 4-bit counters as below; lane grp adds levels 8 grp .. 8 grp + 7 (tpp = 2) or
            // all 16 (tpp = 1) as uint16 pairs.
            uint32_t n0 = 0u, n1 = 0u;
#pragma unroll
            for (int ch = 0; ch < G; ++ch) {
                const uint32_t inc = chain0 + ch < C ? 1u << (4 * (knew[ch] & 7)) : 0u;
                if (knew[ch] < 8) n0 += inc;
                else n1 += inc;
            }
            auto widen = [](uint32_t b) { return (b & 0xFu) | ((b >> 4) << 16); };
            uint32_t *q = hrow + 4 * grp;
            if (tpp == 2) {
                n0 += (uint32_t)__builtin_amdgcn_mov_dpp((int)n0, 0xB1, 0xF, 0xF, false);
                n1 += (uint32_t)__builtin_amdgcn_mov_dpp((int)n1, 0xB1, 0xF, 0xF, false);
                n0 = grp ? n1 : n0;
            }
            if (n0 != 0u) {
                uint4 v = pf.valid ? pf.q0 : *reinterpret_cast<const uint4 *>(q);
                v.x += widen(n0 & 0xFFu);
                v.y += widen((n0 >> 8) & 0xFFu);
                v.z += widen((n0 >> 16) & 0xFFu);
                v.w += widen(n0 >> 24);
                *reinterpret_cast<uint4 *>(q) = v;
            }
            if (tpp == 1 && n1 != 0u) {
                uint4 v = pf.valid ? pf.q1 : *reinterpret_cast<const uint4 *>(hrow + 4);
                v.x += widen(n1 & 0xFFu);
                v.y += widen((n1 >> 8) & 0xFFu);
                v.z += widen((n1 >> 16) & 0xFFu);
                v.w += widen(n1 >> 24);
                *reinterpret_cast<uint4 *>(hrow + 4) = v;
            }
        } else if (SUB == 1 && C <= 15 && (tpp == 1 || tpp == 2 || tpp == 4)) {
            // L <= 16 and at most 15 chains: a pixel's 16 counters fit one 64-bit word of
            // 4-bit counters (no count reaches 16), built by shifts, summed across the
            // pixel's lanes with DPP and widened to the uint16 row, each lane adding its
            // words with plain read-modify-writes.
            uint32_t n0 = 0u, n1 = 0u;  // counters of levels 0-7 and 8-15
#pragma unroll
            for (int ch = 0; ch < G; ++ch) {
                const uint32_t inc = chain0 + ch < C ? 1u << (4 * (knew[ch] & 7)) : 0u;
                if (knew[ch] < 8) n0 += inc;
                else n1 += inc;
            }
            if (tpp >= 2) {
                n0 += (uint32_t)__builtin_amdgcn_mov_dpp((int)n0, 0xB1, 0xF, 0xF, false);
                n1 += (uint32_t)__builtin_amdgcn_mov_dpp((int)n1, 0xB1, 0xF, 0xF, false);
            }
            if (tpp == 4) {
                n0 += (uint32_t)__builtin_amdgcn_mov_dpp((int)n0, 0x4E, 0xF, 0xF, false);
                n1 += (uint32_t)__builtin_amdgcn_mov_dpp((int)n1, 0x4E, 0xF, 0xF, false);
            }
#pragma unroll
            for (int w = 0; w < 8; ++w) {
                if (w < hist_words && (w & (tpp - 1)) == grp) {
                    const uint32_t byte = ((w < 4 ? n0 : n1) >> (8 * (w & 3))) & 0xFFu;  // levels 2w, 2w+1
                    const uint32_t v = (byte & 0xFu) | ((byte >> 4) << 16);
                    if (v != 0u) hrow[w] = (pf.valid ? pf.row[w] : hrow[w]) + v;
                }
            }
        } else if (SUB == 1 && (tpp == 1 || tpp == 2 || tpp == 4)) {
            // L <= 16, more chains: the pixel's whole counter row (at most 8 words) is built in registers,
            // summed across the pixel's lanes with DPP and added to memory by plain
            // read-modify-writes, one word per lane: no global atomics, which are performed
            // beyond the L2 here and would dominate a sweep with so few levels.
            const int nw = hist_words;
            uint32_t row[8];
#pragma unroll
            for (int w = 0; w < 8; ++w) row[w] = 0u;
#pragma unroll
            for (int ch = 0; ch < G; ++ch) {
                const int wi = chain0 + ch < C ? knew[ch] >> 1 : -1;
                const uint32_t inc = (knew[ch] & 1) ? 0x10000u : 1u;
#pragma unroll
                for (int w = 0; w < 8; ++w)
                    if (w < nw) row[w] += wi == w ? inc : 0u;
            }
            if (tpp >= 2) {
#pragma unroll
                for (int w = 0; w < 8; ++w)
                    if (w < nw) row[w] += (uint32_t)__builtin_amdgcn_mov_dpp((int)row[w], 0xB1, 0xF, 0xF, false);
            }
            if (tpp == 4) {
#pragma unroll
                for (int w = 0; w < 8; ++w)
                    if (w < nw) row[w] += (uint32_t)__builtin_amdgcn_mov_dpp((int)row[w], 0x4E, 0xF, 0xF, false);
            }
#pragma unroll
            for (int w = 0; w < 8; ++w)
                if (w < nw && (w & (tpp - 1)) == grp && row[w] != 0u) hrow[w] = (pf.valid ? pf.row[w] : hrow[w]) + row[w];
        } else {
#pragma unroll
            for (int ch = 0; ch < G; ++ch) {
                if (chain0 + ch < C) atomicAdd(hrow + (knew[ch] >> 1), 1u << (16 * (knew[ch] & 1)));
            }
        }
    }
}

// One thread's site updates of a sweep over state in global memory: pixel (r, c) = pix,
// chains grp*G .. grp*G+G-1 (see site_draw).
template <int G, int NBR, int SUB, int NBLK, int SHARE, bool INR = false>
__device__ __forceinline__ void sweep_site(const SweepArgs &a, const float *ptab, const uint4 *vtab, SweepConsts kc,
                                           int pix, int r, int c, int grp, int q)
{
    const int cofs = grp * G;
    SiteInputs<NBR> in;
    in.gp = a.gp[pix];
    const uint8_t *xin = a.xin;
    in.own = load_group<G>(xin + (int64_t)pix * a.Cp + cofs);
#pragma unroll
    for (int j = 0; j < NBR; ++j) {
        const int rr = r + kNbrDr[j], cc = c + kNbrDc[j];
        in.present[j] = rr >= 0 && rr < a.H && cc >= 0 && cc < a.W;
        in.nbw[j] = in.present[j] ? load_group<G>(xin + ((int64_t)rr * a.W + cc) * a.Cp + cofs) : 0u;
    }
    // with few levels (a short level loop), the accumulator words this lane will update
    // are loaded now (see StatsPrefetch); the 16-level-block kernels would spill them
    const int tpp = a.Cp / G;
    StatsPrefetch pf{SUB == 1, 0u, {}, {}, {}};
    if constexpr (SUB == 1) {
        if (a.sum && (tpp == 1 || ((tpp == 2 || tpp == 4) && grp == 0))) pf.sum = a.sum[pix];
        if (a.hist && row_in_quads(a.hist_words, a.C, tpp)) {
            const uint32_t *hrow = a.hist + (int64_t)pix * 8;
            pf.q0 = *reinterpret_cast<const uint4 *>(hrow + 4 * grp);
            if (tpp == 1) pf.q1 = *reinterpret_cast<const uint4 *>(hrow + 4);
        } else if (a.hist && (tpp == 1 || tpp == 2 || tpp == 4)) {
            const uint32_t *hrow = a.hist + (int64_t)pix * a.hist_words;
#pragma unroll
            for (int w = 0; w < 8; ++w)
                if (w < a.hist_words && (w & (tpp - 1)) == grp) pf.row[w] = hrow[w];
        }
    }
    int knew[G];
    const uint32_t packed = site_draw<G, NBR, SUB, NBLK, SHARE, INR>(a, ptab, vtab, kc, in, pix, grp, q, knew);
    store_group<G>(a.xout + (int64_t)pix * a.Cp + cofs, packed);
    site_stats<G, SUB>(a.sum ? a.sum + pix : nullptr, a.hist ? a.hist + (int64_t)pix * a.hist_words : nullptr,
                       a.hist_words, a.C, tpp, grp, knew, pf);
}

inline unsigned grid_for(int64_t threads) { return (unsigned)((threads + kBlock - 1) / kBlock); }

// Site of this thread in a single-lattice sweep (layout of SweepLayout); false if the
// thread has none (past the last pixel, or outside the lattice in an edge tile).  All
// threads of a pixel are consecutive lanes starting at a multiple of tpp.
__device__ __forceinline__ bool sweep_thread_site(const SweepArgs &a, int tpp, int &pix, int &r, int &c, int &grp)
{
    const int64_t blk = a.blk0 + blockIdx.x;
    const int t = (int)threadIdx.x;
    if (a.patch >= 0) {
        const int lp = 6 - a.patch, lr = lp >> 1, lc = lp - lr;
        const int b = (int)blk;  // fewer than 2^31 workgroups
        const int tr = b / a.tiles_w, tc = b - tr * a.tiles_w;
        const int w = t >> 6;               // wave of the workgroup: 2x2 patches
        const int p = (t & 63) >> a.patch;  // pixel within the wave's patch
        grp = t & (tpp - 1);
        r = (((tr << 1) + (w >> 1)) << lr) + (p >> lc);
        c = (((tc << 1) + (w & 1)) << lc) + (p & ((1 << lc) - 1));
        if (r >= a.H || c >= a.W) return false;
        pix = r * a.W + c;
        return true;
    }
    const int64_t gid = blk * kBlock + t;
    if (gid >= (int64_t)a.H * a.W * tpp) return false;
    pix = (int)(gid / tpp);
    grp = (int)(gid - (int64_t)pix * tpp);
    r = pix / a.W;
    c = pix - r * a.W;
    return true;
}

// ---------------------------------------------------------------- batched sweep

// One sweep of every lattice of a batch in one launch.  Each workgroup belongs to one
// lattice (its descriptor is read once, uniformly); lattices may differ in size, level
// count, chains, parameters, seed and sweep index.  The sweep index lives in the
// descriptor in device memory, so a captured graph of n launches can be replayed for the
// next n sweeps; a lattice whose index reached its end is skipped.
template <int G, int SHARE, int TILED, int NBR, bool INR = false>
__global__ __launch_bounds__(kBlock) void batch_sweep_kernel(BatchLaunch b)
{
    __shared__ float ptab[kMaxNeighbourStat + 1];
    __shared__ uint4 vtab[kStatEntries];
    const int blk = (int)blockIdx.x + b.block0;
    const int img = b.block_img[blk];
    const ImageDesc &d = b.imgs[img];
    const uint32_t t = d.t + b.toff;
    if (t >= d.t_end) return;  // this lattice has finished (uniform over the workgroup)
    SweepArgs a;
    a.gp = d.gp;
    a.xin = (t & 1u) ? d.x1 : d.x0;
    a.xout = (t & 1u) ? d.x0 : d.x1;
    const bool acc = (int64_t)t >= d.burn_in;
    const bool tally = acc && d.tally_stride > 0 && ((int64_t)t - d.burn_in) % d.tally_stride == 0;
    a.sum = acc ? d.sum : nullptr;
    a.hist = tally ? d.hist : nullptr;
    a.H = d.H;
    a.W = d.W;
    a.L = d.L;
    a.C = d.C;
    a.Cp = d.Cp;
    a.T = d.T;
    a.hist_words = d.hist_words;
    a.beta = d.beta_len == 0 ? 1.0 : d.beta[t < (uint32_t)d.beta_len ? t : (uint32_t)(d.beta_len - 1)];
    a.J = d.J;
    a.q = d.q;
    a.kappa = d.kappa;
    a.sigma_s = d.sigma_s;
    a.key0 = d.key0;
    a.key1 = d.key1;
    a.t = t;
    a.inertia = d.inertia;
    a.blk0 = 0;
    a.patch = -1;
    a.tiles_w = 0;
    const SweepConsts kc = sweep_prologue(a, NBR, ptab, vtab);

    const int tpp = d.tpp;
    const int local = blk - d.block_base;
    int pix, r, c, grp;
    if constexpr (TILED == 0) {
        // row-major, or 2-D pixel patches for L > 16, laid out as in a single-lattice sweep
        a.patch = d.patch;
        a.tiles_w = d.tiles_w;
        a.blk0 = (int64_t)local - (int64_t)blockIdx.x;
        if (!sweep_thread_site(a, tpp, pix, r, c, grp)) return;
    } else {
        const int th = kBlock / tpp / kTileW;  // tile height in pixels
        const int tr = local / d.tiles_w, tc = local - (local / d.tiles_w) * d.tiles_w;
        const int lp = (int)threadIdx.x / tpp;
        // when tpp does not divide kBlock / kTileW, the last threads of the workgroup have
        // no pixel in its tile (they would land in the next tile row)
        if (lp >= th * kTileW) return;
        grp = (int)threadIdx.x - lp * tpp;
        r = tr * th + lp / kTileW;
        c = tc * kTileW + lp % kTileW;
        if (r >= d.H || c >= d.W) return;
        pix = r * d.W + c;
    }
    const int q = (int)(threadIdx.x % SHARE);
    if (a.L <= 16) sweep_site<G, NBR, 1, 16, SHARE, INR>(a, ptab, vtab, kc, pix, r, c, grp, q);
    else sweep_site<G, NBR, 16, 16, SHARE, INR>(a, ptab, vtab, kc, pix, r, c, grp, q);
}

// Waves per SIMD the single-lattice sweep kernels are compiled for.  With 16-level blocks
// (L > 16) the register allocator would otherwise settle at 127 VGPRs and 4 waves; at 5
// waves (96 VGPRs) the LDS and DPP latencies of the level loop are better hidden although
// about 19 values, mostly block partial sums, then go to scratch.  Measured on 2048x2048,
// L = 256, 16 chains with the grouped table reads: 4 waves 3.06 ms per sweep, 5 waves 2.93,
// 6 waves 2.90 with 2.5x the scratch write traffic, 7 and 8 waves slower.
template <int SUB>
constexpr int kMinWaves = SUB > 1 ? 5 : 1;

}  // namespace
}  // namespace pcak
