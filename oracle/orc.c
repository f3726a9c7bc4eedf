/*
 * CPU oracle for the lazy Probabilistic Cellular Automaton (PCA) sampler and for the
 * sequential single-site Gibbs sampler it is compared against.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no code, header, table or
 * constant generator with the HIP path: every quantity below is computed here, from
 * the paper's definitions and from the arithmetic convention written out in this
 * header.  Plain, slow, scalar C; every loop follows the definition it cites.
 *
 * Paper: Costarelli, Piconi, Troiani, "Bayesian Inversion via Probabilistic Cellular
 * Automata: an application to image denoising" (arXiv 2507.14869).
 *
 *  - Posterior Hamiltonian with Gaussian noise, beta not scaling the data term:
 *    Sec. 2 eq. (posterior_hamiltonian), Sec. 4 eq. (denoising_posterior_Hamiltonian).
 *  - Pair prior: Potts V(z,w) = -J if z = w else +J, eq. (prior_pair_potential);
 *    neighbourhood eq. (neighborhood) (8 sites; 4 sites also offered).
 *  - Gibbs single-site conditional: Sec. 5.1 eq. (gibbs_sampler_elementary_step);
 *    sweeps in a fixed order, updated in place.
 *  - Lazy PCA: pair Hamiltonian eq. (denoising_pair_posterior_Hamiltonian) and the
 *    product transition of Sec. 5.2; the inertia indicator compares the new value
 *    with the site's OWN previous value x_i (the printed x_j is read as a typo).
 *
 * Readings where the paper is silent (each listed in the design notes):
 *  - Potts log-weight is written as -2*beta*J*#(disagreeing neighbours); it differs
 *    from the paper's +2*beta*J*#(agreeing) by a per-site constant, which cancels.
 *    Truncated-linear prior: -beta*J*sum_j min(|k-x_j|, T).  Both are
 *    -c * S_k with S_k = sum_j min(|k - x_j|, T) and (c,T) = (2 beta J, 1) for Potts.
 *  - Free boundary: absent neighbours contribute nothing.
 *  - Levels are indices 0..L-1 (value vmin + k*(vmax-vmin)/(L-1)); observations and
 *    sigma are rescaled to level units once.
 *
 * Arithmetic convention (what "the same result" means between this oracle and any
 * other implementation; FP32 unless stated, IEEE round-to-nearest-even, no
 * contraction of a*b+c unless fmaf is written):
 *  C1  scalars in double, rounded once to float:
 *        s   = (L-1)/(vmax-vmin)                      (double)
 *        g'  = (float)(((double)g - vmin) * s)         per pixel
 *        a2  = (float)(LOG2E / ((2*sigma_s)*sigma_s)),  sigma_s = sigma*s
 *        c2  = (float)(((beta*J)*kappa)*LOG2E),  kappa = 2 (Potts) or 1
 *        q2  = (float)((beta*q)*LOG2E)
 *  C2  exp2s(y): 0 if y < -125; else n = rint(y), f = y - n,
 *        p = Horner(fmaf) of c_6..c_0 at f, c_k = (float)t_k, t_0 = 1,
 *        t_k = (t_{k-1}*LN2)/k in double;  result ldexp(p, n).
 *  C3  data factor  D_k = exp2s(fmaf(-a2, e_k*e_k, m)),  e_k = g' - (float)k,
 *        m = a2*(e0*e0), e0 = g' - khat, khat = clamp(rint(g'), 0, L-1).
 *      prior factor P(S) = exp2s(-(c2*(float)S)).
 *      stay factor  R = exp2s(q2) - 1.
 *  C4  The lazy conditional  P(k|x) prop. to  D_k P(S_k) exp(-beta q [k != x])  is
 *      drawn as the equivalent mixture  "stay at x" with weight D_x P(S_x)(e^{beta q}-1)
 *      followed by every level k with weight D_k P(S_k) (both scaled by e^{beta q}):
 *        acc_{-1} = (D_x * P(S_x)) * R,
 *        acc_k    = fmaf(D_k, P(S_k), acc_{k-1}),  k = 0..L-1,   Z = acc_{L-1}.
 *  C5  u = (r >> 8) * 2^-24 with r the chain's Philox4x32-10 word; the new value is
 *      x if acc_{-1} > u*Z, else the least k with acc_k > u*Z (products and
 *      comparisons exact); x if Z == 0.
 *  C6  Philox4x32-10 (Salmon et al., SC'11): counter {pixel, sweep, chain>>2, stream},
 *      key {seed lo, seed hi}, word chain&3; stream 0 = updates, 1 = random init.
 *  C7  Gibbs uses the same C1-C6 with R = 0, reading the partially updated state.
 *  C8  Inertia norms (Sec. 3, "The lazy PCA": the inertia q|x_i - w_i|^p, with 0^0 = 0;
 *      L1 and L2 offered at the end of Sec. 5.2).  p = 0 is C4.  For p = 1 or 2 the data
 *      and inertia terms share one exponent, shifted by its maximum over the levels so
 *      that the product cannot underflow where both terms are large:
 *        F_k = fmaf(-a2, e_k*e_k, -(q2 * (float)d_k^p)),  d_k = |k - x|,
 *        E_k = exp2s(F_k - Fmax),  acc_{-1} = 0,  acc_k = fmaf(E_k, P(S_k), acc_{k-1}),
 *      drawn as in C5 (the stay branch never fires).  F is concave in k, so Fmax is the
 *      larger of F at k1 = clamp(floor(kc), 0, L-1) and k2 = min(k1 + 1, L-1), where kc
 *      maximises the real-valued form: for p = 1, kc = min(max(x, g' - h), g' + h) with
 *      h = q2 / (2*a2); for p = 2, kc = (a2*g' + q2*x) / (a2 + q2).  Gibbs has no
 *      inertia at any p.
 *
 * What pins this code (the CPU tests): the per-site conditionals against closed forms and
 * float64 evaluations, the whole samplers' laws against exactly enumerated transition
 * matrices and closed-form stationary laws, exp2s against its error bound, Philox against
 * an independent library implementation of the same published generator, the draw rule
 * on constructed sums.  The bit-level choices of C1-C6 (rounding order, the Philox
 * counter layout, the exact threshold comparison) are conventions the paper does not fix:
 * parity unpinned by the paper beyond those laws and bounds; a frozen fixture guards them
 * against unintended change.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_LOG2E 1.4426950408889634
#define ORC_LN2 0.6931471805599453

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2
#define ORC_ESTATE -4

typedef struct {
    int32_t height, width, levels, chains, neighbourhood, prior, trunc;
    float J, q, sigma, vmin, vmax;
    const float *beta; /* per-sweep inverse temperature, NULL => 1 */
    int32_t beta_len;  /* sweeps past the end reuse the last value */
    uint64_t seed;
    int32_t init_mode, burn_in, tally_stride;
    int32_t inertia;   /* exponent p of the inertia norm: 0 (indicator), 1 or 2 */
} orc_params;

/* ------------------------------------------------------------------ Philox (C6) */

/* One 32x32 -> 64 bit product split into high and low words. */
static void mulhilo32(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo)
{
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

/* Philox4x32 with 10 rounds: each round multiplies words 0 and 2 by the two
 * published multipliers, and the key advances by the two Weyl increments between
 * rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint32_t hi0, lo0, hi1, lo1;
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        mulhilo32(0xD2511F53u, x0, &hi0, &lo0);
        mulhilo32(0xCD9E8D57u, x2, &hi1, &lo1);
        uint32_t n0 = hi1 ^ x1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ x3 ^ k1;
        uint32_t n3 = lo0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static uint32_t chain_word(uint64_t seed, uint32_t pixel, uint32_t sweep, int chain, uint32_t stream)
{
    uint32_t ctr[4] = {pixel, sweep, (uint32_t)chain >> 2, stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[chain & 3];
}

float orc_uniform(uint32_t r) { return (float)(r >> 8) * 0x1p-24f; }

/* ---------------------------------------------------------------- exp2s (C2) */

static float exp2s_coeff[7];
static int exp2s_ready = 0;

static void exp2s_setup(void)
{
    double t = 1.0;
    exp2s_coeff[0] = 1.0f;
    for (int k = 1; k <= 6; ++k) {
        t = (t * ORC_LN2) / (double)k;
        exp2s_coeff[k] = (float)t;
    }
    exp2s_ready = 1;
}

float orc_exp2s(float y)
{
    if (!exp2s_ready) exp2s_setup();
    if (y < -125.0f) return 0.0f;
    float n = rintf(y);
    float f = y - n;
    float p = exp2s_coeff[6];
    for (int k = 5; k >= 0; --k) p = fmaf(p, f, exp2s_coeff[k]);
    return ldexpf(p, (int)n);
}

/* ------------------------------------------------------------ parameters (C1) */

typedef struct {
    int H, W, L, C, nbr, T;
    double scale; /* (L-1)/(vmax-vmin) */
    float a2;
} orc_run_consts;

typedef struct {
    float c2, q2, R;
    int p; /* inertia exponent; 0 also for Gibbs */
} orc_sweep_consts;

static int check_params(const orc_params *p)
{
    if (!p) return ORC_EINVAL;
    if (p->height < 1 || p->width < 1) return ORC_EINVAL;
    if (p->levels < 2 || p->levels > 256) return ORC_EINVAL;
    if (p->chains < 1) return ORC_EINVAL;
    if (p->neighbourhood != 4 && p->neighbourhood != 8) return ORC_EINVAL;
    if (p->prior != 0 && p->prior != 1) return ORC_EINVAL;
    if (p->prior == 1 && p->trunc < 1) return ORC_EINVAL;
    if (!(p->J >= 0.0f) || !(p->q >= 0.0f) || !(p->sigma > 0.0f)) return ORC_EINVAL;
    if (!(p->vmax > p->vmin)) return ORC_EINVAL;
    if (p->beta_len < 0 || (p->beta_len > 0 && !p->beta)) return ORC_EINVAL;
    for (int i = 0; i < p->beta_len; ++i) {
        if (!(p->beta[i] > 0.0f)) return ORC_EINVAL;
        if ((double)p->beta[i] * (double)p->q * ORC_LOG2E > 100.0) return ORC_EINVAL;
    }
    if (p->beta_len == 0 && (double)p->q * ORC_LOG2E > 100.0) return ORC_EINVAL;
    if (p->init_mode != 0 && p->init_mode != 1) return ORC_EINVAL;
    if (p->burn_in < 0 || p->tally_stride < 0) return ORC_EINVAL;
    if (p->inertia < 0 || p->inertia > 2) return ORC_EINVAL;
    return ORC_OK;
}

static orc_run_consts run_consts(const orc_params *p)
{
    orc_run_consts rc;
    rc.H = p->height;
    rc.W = p->width;
    rc.L = p->levels;
    rc.C = p->chains;
    rc.nbr = p->neighbourhood;
    rc.T = p->prior == 0 ? 1 : (p->trunc < p->levels - 1 ? p->trunc : p->levels - 1);
    rc.scale = (double)(p->levels - 1) / ((double)p->vmax - (double)p->vmin);
    double sigma_s = (double)p->sigma * rc.scale;
    rc.a2 = (float)(ORC_LOG2E / ((2.0 * sigma_s) * sigma_s));
    return rc;
}

static double beta_at(const orc_params *p, int64_t t)
{
    if (p->beta_len == 0) return 1.0;
    if (t >= p->beta_len) return (double)p->beta[p->beta_len - 1];
    return (double)p->beta[t];
}

static orc_sweep_consts sweep_consts(const orc_params *p, int64_t t, int gibbs)
{
    orc_sweep_consts sc;
    double beta = beta_at(p, t);
    double kappa = p->prior == 0 ? 2.0 : 1.0;
    sc.c2 = (float)(((beta * (double)p->J) * kappa) * ORC_LOG2E);
    sc.q2 = (float)((beta * (double)p->q) * ORC_LOG2E);
    sc.p = gibbs ? 0 : p->inertia;
    sc.R = gibbs ? 0.0f : orc_exp2s(sc.q2) - 1.0f;
    return sc;
}

float orc_level_obs(const orc_params *p, float g)
{
    orc_run_consts rc = run_consts(p);
    return (float)(((double)g - (double)p->vmin) * rc.scale);
}

/* --------------------------------------------------- per-site weights (C3, C4) */

static float data_factor(float gp, int k, int L, float a2)
{
    float khat = rintf(gp);
    if (khat < 0.0f) khat = 0.0f;
    if (khat > (float)(L - 1)) khat = (float)(L - 1);
    float e0 = gp - khat;
    float m = a2 * (e0 * e0);
    float e = gp - (float)k;
    return orc_exp2s(fmaf(-a2, e * e, m));
}

static float prior_factor(int S, float c2) { return orc_exp2s(-(c2 * (float)S)); }

/* F_k of C8: data exponent plus inertia exponent q2 |k - x|^p, in log2 units. */
static float inertia_exponent(float gp, int k, int x, int p, float a2, float q2)
{
    int d = abs(k - x);
    int dp = p == 1 ? d : d * d;
    float e = gp - (float)k;
    return fmaf(-a2, e * e, -(q2 * (float)dp));
}

/* Shift of the C8 exponents: their maximum over the levels, found in O(1).  F_k is a
 * concave function of k (a downward parabola in k plus -q2|k - x|^p, p >= 1), so its
 * maximum over the integers lies at one of the two integers around the maximiser kc of
 * the real-valued form: kc = clamp(x, g' - h, g' + h) with h = q2/(2 a2) for p = 1, the
 * weighted mean (a2 g' + q2 x)/(a2 + q2) for p = 2. */
static float inertia_fmax(const orc_run_consts *rc, const orc_sweep_consts *sc, float gp, int x)
{
    float kc;
    if (sc->p == 1) {
        float h = sc->q2 / (2.0f * rc->a2);
        kc = fminf(fmaxf((float)x, gp - h), gp + h);
    } else {
        kc = (rc->a2 * gp + sc->q2 * (float)x) / (rc->a2 + sc->q2);
    }
    int k1 = (int)fminf(fmaxf(floorf(kc), 0.0f), (float)(rc->L - 1));
    int k2 = k1 + 1 < rc->L ? k1 + 1 : k1;
    float F1 = inertia_exponent(gp, k1, x, sc->p, rc->a2, sc->q2);
    float F2 = inertia_exponent(gp, k2, x, sc->p, rc->a2, sc->q2);
    return F1 > F2 ? F1 : F2;
}

/* S_k = sum over in-lattice neighbours j of min(|k - x_j|, T); `plane` is one chain's
 * [H][W] state. */
static int neighbour_stat(const orc_run_consts *rc, const uint8_t *plane, int r, int c, int k)
{
    static const int dr4[4] = {-1, 1, 0, 0}, dc4[4] = {0, 0, -1, 1};
    static const int dr8[8] = {-1, 1, 0, 0, -1, -1, 1, 1}, dc8[8] = {0, 0, -1, 1, -1, 1, -1, 1};
    const int *dr = rc->nbr == 4 ? dr4 : dr8;
    const int *dc = rc->nbr == 4 ? dc4 : dc8;
    int S = 0;
    for (int j = 0; j < rc->nbr; ++j) {
        int rr = r + dr[j], cc = c + dc[j];
        if (rr < 0 || rr >= rc->H || cc < 0 || cc >= rc->W) continue; /* free boundary */
        int d = abs(k - (int)plane[(size_t)rr * rc->W + cc]);
        S += d < rc->T ? d : rc->T;
    }
    return S;
}

/* Running sums acc[0] = acc_{-1} (stay), acc[1+k] = acc_k, for one site of one chain. */
static void site_acc(const orc_run_consts *rc, const orc_sweep_consts *sc, const uint8_t *plane,
                     int r, int c, float gp, float *acc)
{
    int x = plane[(size_t)r * rc->W + c];
    if (sc->p > 0) { /* C8: data and inertia in one shifted exponent, no stay branch */
        float Fmax = inertia_fmax(rc, sc, gp, x);
        float a = 0.0f;
        acc[0] = a;
        for (int k = 0; k < rc->L; ++k) {
            float Ek = orc_exp2s(inertia_exponent(gp, k, x, sc->p, rc->a2, sc->q2) - Fmax);
            float Pk = prior_factor(neighbour_stat(rc, plane, r, c, k), sc->c2);
            a = fmaf(Ek, Pk, a);
            acc[1 + k] = a;
        }
        return;
    }
    float Dx = data_factor(gp, x, rc->L, rc->a2);
    float Px = prior_factor(neighbour_stat(rc, plane, r, c, x), sc->c2);
    float a = (Dx * Px) * sc->R;
    acc[0] = a;
    for (int k = 0; k < rc->L; ++k) {
        float Dk = data_factor(gp, k, rc->L, rc->a2);
        float Pk = prior_factor(neighbour_stat(rc, plane, r, c, k), sc->c2);
        a = fmaf(Dk, Pk, a);
        acc[1 + k] = a;
    }
}

static int draw_from_acc(const float *acc, int L, int x, uint32_t rword)
{
    float Z = acc[L];
    if (Z == 0.0f) return x;
    double t = (double)orc_uniform(rword) * (double)Z; /* exact: 24 x 24 bit product */
    if ((double)acc[0] > t) return x;
    for (int k = 0; k < L; ++k)
        if ((double)acc[1 + k] > t) return k;
    return x; /* not reached: acc[L] = Z > t because u < 1 */
}

static int site_update(const orc_run_consts *rc, const orc_sweep_consts *sc, const orc_params *p,
                       const uint8_t *plane, const float *gp, int chain, int r, int c, int64_t t,
                       float *scratch)
{
    uint32_t pixel = (uint32_t)((size_t)r * rc->W + c);
    site_acc(rc, sc, plane, r, c, gp[pixel], scratch);
    uint32_t w = chain_word(p->seed, pixel, (uint32_t)t, chain, 0);
    return draw_from_acc(scratch, rc->L, plane[pixel], w);
}

/* ---------------------------------------------------------------- public API */

static int level_obs_all(const orc_params *p, const float *obs, float *gp)
{
    orc_run_consts rc = run_consts(p);
    size_t N = (size_t)rc.H * rc.W;
    for (size_t i = 0; i < N; ++i) gp[i] = (float)(((double)obs[i] - (double)p->vmin) * rc.scale);
    return ORC_OK;
}

/* Initial state [C][H][W]: nearest level to the observation (mode 0) or a Philox
 * uniform level from stream 1 (mode 1). */
int orc_init_state(const orc_params *p, const float *obs, uint8_t *state)
{
    int rcode = check_params(p);
    if (rcode) return rcode;
    orc_run_consts rc = run_consts(p);
    size_t N = (size_t)rc.H * rc.W;
    for (int ch = 0; ch < rc.C; ++ch) {
        for (size_t i = 0; i < N; ++i) {
            int v;
            if (p->init_mode == 0) {
                float gp = (float)(((double)obs[i] - (double)p->vmin) * rc.scale);
                float kh = rintf(gp);
                if (kh < 0.0f) kh = 0.0f;
                if (kh > (float)(rc.L - 1)) kh = (float)(rc.L - 1);
                v = (int)kh;
            } else {
                uint32_t w = chain_word(p->seed, (uint32_t)i, 0, ch, 1);
                v = (int)(((uint64_t)(w >> 8) * (uint64_t)rc.L) >> 24);
            }
            state[(size_t)ch * N + i] = (uint8_t)v;
        }
    }
    return ORC_OK;
}

static void accumulate(const orc_params *p, const orc_run_consts *rc, const uint8_t *state, int64_t t,
                       uint32_t *sum, int64_t *count, uint16_t *hist)
{
    if (t < p->burn_in) return;
    size_t N = (size_t)rc->H * rc->W;
    if (sum) {
        for (int ch = 0; ch < rc->C; ++ch)
            for (size_t i = 0; i < N; ++i) sum[i] += state[(size_t)ch * N + i];
        if (count) *count += rc->C;
    }
    if (hist && p->tally_stride > 0 && ((t - p->burn_in) % p->tally_stride) == 0) {
        for (int ch = 0; ch < rc->C; ++ch)
            for (size_t i = 0; i < N; ++i) hist[i * rc->L + state[(size_t)ch * N + i]] += 1;
    }
}

/* Runs sweeps t0 .. t0+n-1 on `state` ([C][H][W], in/out).  gibbs = 0: lazy PCA, every
 * site of a chain reads only the previous state.  gibbs = 1: systematic single-site
 * Gibbs in row-major order, in place, no inertia.  sum/count/hist may be NULL. */
int orc_run(const orc_params *p, const float *obs, uint8_t *state, int64_t t0, int32_t n,
            uint32_t *sum, int64_t *count, uint16_t *hist, int32_t gibbs)
{
    int rcode = check_params(p);
    if (rcode) return rcode;
    if (n < 0 || t0 < 0 || !obs || !state) return ORC_EINVAL;
    orc_run_consts rc = run_consts(p);
    size_t N = (size_t)rc.H * rc.W;
    float *gp = (float *)malloc(N * sizeof(float));
    float *scratch = (float *)malloc((size_t)(rc.L + 1) * sizeof(float));
    uint8_t *next = gibbs ? NULL : (uint8_t *)malloc(N);
    if (!gp || !scratch || (!gibbs && !next)) {
        free(gp); free(scratch); free(next);
        return ORC_ENOMEM;
    }
    level_obs_all(p, obs, gp);
    for (int64_t t = t0; t < t0 + n; ++t) {
        orc_sweep_consts sc = sweep_consts(p, t, gibbs);
        for (int ch = 0; ch < rc.C; ++ch) {
            uint8_t *plane = state + (size_t)ch * N;
            for (int r = 0; r < rc.H; ++r) {
                for (int c = 0; c < rc.W; ++c) {
                    int v = site_update(&rc, &sc, p, plane, gp, ch, r, c, t, scratch);
                    if (gibbs) plane[(size_t)r * rc.W + c] = (uint8_t)v;
                    else next[(size_t)r * rc.W + c] = (uint8_t)v;
                }
            }
            if (!gibbs) memcpy(plane, next, N);
        }
        accumulate(p, &rc, state, t, sum, count, hist);
    }
    free(gp); free(scratch); free(next);
    return ORC_OK;
}

/* New PCA values at selected sites after sweep t from the full previous state
 * ([C][H][W]); used to check large lattices one site at a time. */
int orc_update_sites(const orc_params *p, const float *obs, const uint8_t *state, int64_t t,
                     int64_t n_sites, const int32_t *chains, const int64_t *pixels, uint8_t *out)
{
    int rcode = check_params(p);
    if (rcode) return rcode;
    orc_run_consts rc = run_consts(p);
    size_t N = (size_t)rc.H * rc.W;
    float *scratch = (float *)malloc((size_t)(rc.L + 1) * sizeof(float));
    if (!scratch) return ORC_ENOMEM;
    orc_sweep_consts sc = sweep_consts(p, t, 0);
    for (int64_t s = 0; s < n_sites; ++s) {
        int ch = chains[s];
        int64_t pix = pixels[s];
        if (ch < 0 || ch >= rc.C || pix < 0 || (size_t)pix >= N) { free(scratch); return ORC_EINVAL; }
        int r = (int)(pix / rc.W), c = (int)(pix % rc.W);
        const uint8_t *plane = state + (size_t)ch * N;
        float gp = (float)(((double)obs[pix] - (double)p->vmin) * rc.scale);
        site_acc(&rc, &sc, plane, r, c, gp, scratch);
        uint32_t w = chain_word(p->seed, (uint32_t)pix, (uint32_t)t, ch, 0);
        out[s] = (uint8_t)draw_from_acc(scratch, rc.L, plane[pix], w);
    }
    free(scratch);
    return ORC_OK;
}

/* New PCA values of one chain after sweep t, for rows r0 .. r1-1 of the lattice, from the
 * full previous state ([C][H][W]); out is [r1-r0][W].  Row bands of one sweep can be
 * computed independently (each reads only the previous state), so a whole sweep of a
 * large lattice can be checked band by band, in several host threads. */
int orc_pca_rows(const orc_params *p, const float *obs, const uint8_t *state, int64_t t, int32_t chain,
                 int32_t r0, int32_t r1, uint8_t *out)
{
    int rcode = check_params(p);
    if (rcode) return rcode;
    orc_run_consts rc = run_consts(p);
    if (chain < 0 || chain >= rc.C || r0 < 0 || r1 > rc.H || r0 > r1 || t < 0) return ORC_EINVAL;
    size_t N = (size_t)rc.H * rc.W;
    float *scratch = (float *)malloc((size_t)(rc.L + 1) * sizeof(float));
    if (!scratch) return ORC_ENOMEM;
    orc_sweep_consts sc = sweep_consts(p, t, 0);
    const uint8_t *plane = state + (size_t)chain * N;
    for (int r = r0; r < r1; ++r) {
        for (int c = 0; c < rc.W; ++c) {
            size_t pix = (size_t)r * rc.W + c;
            float gp = (float)(((double)obs[pix] - (double)p->vmin) * rc.scale);
            site_acc(&rc, &sc, plane, r, c, gp, scratch);
            uint32_t w = chain_word(p->seed, (uint32_t)pix, (uint32_t)t, chain, 0);
            out[(size_t)(r - r0) * rc.W + c] = (uint8_t)draw_from_acc(scratch, rc.L, plane[pix], w);
        }
    }
    free(scratch);
    return ORC_OK;
}

/* The C8 exponents F_0 .. F_{L-1} of one site (unshifted) and the O(1) shift Fmax the
 * sampler uses, for tests that compare the shift with the plain maximum over the levels. */
int orc_inertia_exponents(const orc_params *p, const float *obs, const uint8_t *state, int32_t chain,
                          int32_t r, int32_t c, int64_t t, float *F, float *Fmax)
{
    int rcode = check_params(p);
    if (rcode) return rcode;
    if (p->inertia < 1) return ORC_EINVAL;
    orc_run_consts rc = run_consts(p);
    if (chain < 0 || chain >= rc.C || r < 0 || r >= rc.H || c < 0 || c >= rc.W) return ORC_EINVAL;
    size_t N = (size_t)rc.H * rc.W;
    orc_sweep_consts sc = sweep_consts(p, t, 0);
    size_t pix = (size_t)r * rc.W + c;
    float gp = (float)(((double)obs[pix] - (double)p->vmin) * rc.scale);
    int x = state[(size_t)chain * N + pix];
    for (int k = 0; k < rc.L; ++k) F[k] = inertia_exponent(gp, k, x, sc.p, rc.a2, sc.q2);
    *Fmax = inertia_fmax(&rc, &sc, gp, x);
    return ORC_OK;
}

/* The draw of C5 from running sums acc[0..L] (acc[0] the stay weight), current level x
 * and Philox word rword; for tests of the rule itself. */
int32_t orc_draw(const float *acc, int32_t L, int32_t x, uint32_t rword)
{
    if (!acc || L < 1) return -1;
    return draw_from_acc(acc, L, x, rword);
}

/* The running sums acc[0..L] of one site (see C4), for inspection by tests. */
int orc_site_acc(const orc_params *p, const float *obs, const uint8_t *state, int32_t chain,
                 int32_t r, int32_t c, int64_t t, int32_t gibbs, float *acc)
{
    int rcode = check_params(p);
    if (rcode) return rcode;
    orc_run_consts rc = run_consts(p);
    if (chain < 0 || chain >= rc.C || r < 0 || r >= rc.H || c < 0 || c >= rc.W) return ORC_EINVAL;
    size_t N = (size_t)rc.H * rc.W;
    orc_sweep_consts sc = sweep_consts(p, t, gibbs);
    size_t pix = (size_t)r * rc.W + c;
    float gp = (float)(((double)obs[pix] - (double)p->vmin) * rc.scale);
    site_acc(&rc, &sc, state + (size_t)chain * N, r, c, gp, acc);
    return ORC_OK;
}

/* Posterior mean in value units: vmin + (sum/count) * (vmax-vmin)/(L-1), in double,
 * rounded once. */
int orc_posterior_mean(const orc_params *p, const uint32_t *sum, int64_t count, float *out)
{
    int rcode = check_params(p);
    if (rcode) return rcode;
    if (count <= 0) return ORC_ESTATE;
    size_t N = (size_t)p->height * p->width;
    double delta = ((double)p->vmax - (double)p->vmin) / (double)(p->levels - 1);
    for (size_t i = 0; i < N; ++i)
        out[i] = (float)((double)p->vmin + ((double)sum[i] / (double)count) * delta);
    return ORC_OK;
}

/* Marginal posterior mode: per pixel the level with the largest tally, ties to the
 * lowest level. */
int orc_marginal_map(const orc_params *p, const uint16_t *hist, uint8_t *out)
{
    int rcode = check_params(p);
    if (rcode) return rcode;
    size_t N = (size_t)p->height * p->width;
    int L = p->levels;
    for (size_t i = 0; i < N; ++i) {
        int best = 0;
        for (int k = 1; k < L; ++k)
            if (hist[i * L + k] > hist[i * L + best]) best = k;
        out[i] = (uint8_t)best;
    }
    return ORC_OK;
}

/* Per-sweep constants, for inspection by tests: c2, R and a2 as defined in C1-C3. */
int orc_constants(const orc_params *p, int64_t t, int32_t gibbs, float *out3)
{
    int rcode = check_params(p);
    if (rcode) return rcode;
    orc_run_consts rc = run_consts(p);
    orc_sweep_consts sc = sweep_consts(p, t, gibbs);
    out3[0] = sc.c2;
    out3[1] = sc.R;
    out3[2] = rc.a2;
    return ORC_OK;
}
