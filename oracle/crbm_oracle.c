/*
 * crbm_oracle.c -- plain, slow, single-threaded CPU oracle for block Gibbs
 * sampling of the convolutional RBM that encodes the classical
 * Shastry-Sutherland (SS) Ising lattice.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call this
 * file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code (kernels, headers, helpers, tables) with
 * the HIP library: every formula below is written out again from the paper
 * and from the conventions stated here.
 *
 * What it follows (paper: Brahma et al., "Hardware Acceleration of Frustrated
 * Lattice Systems using Convolutional Restricted Boltzmann Machine"):
 *   - SS Ising Hamiltonian, Sec. I Eq. (1), with the field sign read so that
 *     h > 0 favours up spins (H = J1 sum_sq s s + J2 sum_dimer s s - h sum s):
 *     this is the reading under which the paper's h = 3 state is the 1/3
 *     plateau and its h = 7 state is ferromagnetic (Sec. III.A).
 *   - one hidden unit per bond, Sec. II.A Eqs. (4)-(8): for a bond with
 *     coupling K = -J/T the hidden unit has weight w = arccosh(exp(2|K|))/2 on
 *     its first spin and sgn(K) w on its second spin; the marginal over the
 *     hidden unit reproduces exp(K s_a s_b) up to a constant.
 *   - convolutional weight sharing with 10 filters over the 3x3 unit-cell
 *     window and stride 2, Sec. II.A Eqs. (9)-(10) and Sec. II.B.
 *   - block Gibbs: all hidden units given the spins, Eq. (11); then all spins
 *     given the hidden units, Eq. (12), with the visible bias of App. A
 *     (accumulator).  Units are +-1; P(unit = +1) = sigmoid(2 x) where x is
 *     the unit's field (the factor 2 comes from +-1 units, Eqs. (5)-(6)).
 *   - sigmoid by table lookup with the closest value (App. A, sigmoid
 *     module) and a comparison against a uniform random number (App. A, LFSR
 *     module).  Here: 32-bit thresholds and 32-bit uniforms from Philox4x32-10
 *     (Salmon et al., SC'11) instead of the paper's 16-bit LUT and LFSR.
 *
 * Conventions (the contract both implementations obey, bit for bit):
 *   spins      s(r,c) in {-1,+1}, 0 <= r,c < L, L even, periodic.
 *   cells      (i,j), 0 <= i,j < L/2, window origin (2i,2j).
 *   bonds      10 per cell (filters k = 0..9), endpoints a and b given as
 *              offsets in the 3x3 window, coordinates taken mod L:
 *                k0 J1 (0,0)-(0,1)   k1 J1 (0,1)-(0,2)
 *                k2 J1 (1,0)-(1,1)   k3 J1 (1,1)-(1,2)
 *                k4 J1 (0,0)-(1,0)   k5 J1 (1,0)-(2,0)
 *                k6 J1 (0,1)-(1,1)   k7 J1 (1,1)-(2,1)
 *                k8 J2 (0,0)-(1,1)   k9 J2 (1,2)-(2,1)
 *   quantise   Jq = llround(J * 2^16) for J1, J2, h (16.16 fixed point).
 *   schedule   T_s, s = 0..S-1: const T0; linear T0 + (T1-T0)*(s/(S-1));
 *              geometric T0 * pow(T1/T0, s/(S-1)); explicit list.
 *   weights    per sweep and bond type t: K = -(Jq/2^16)/T_s,
 *              sig_t = (K < 0) ? -1 : +1,
 *              w = |K| + log1p(sqrt(-expm1(-4|K|)))/2   (= arccosh(e^{2|K|})/2),
 *              wq_t = llround(w * 2^16);  visible bias aq = llround(hq / T_s).
 *   fields     hidden unit of bond (a,b) of type t: x = wq_t (s_a + sig_t s_b);
 *              spin at a site: x = aq + sum over its 5 bonds of
 *              wq_t * coef * h_bond, coef = 1 at endpoint a, sig_t at b.
 *   threshold  t(y) for an integer field magnitude y >= 0:
 *              p = 1/(1 + exp(-2 y / 2^16)),
 *              t = min(2^32 - 1, floor(p * 2^32 + 0.5))   (closest value).
 *   update     s = (x >= 0) ? +1 : -1; the unit becomes s if U < t(|x|),
 *              else -s, where U is the unit's 32-bit uniform.
 *   Philox     out = Philox4x32-10(ctr = (c0, sweep, chain, (id << 3) | stream),
 *                                  key = (seed & 0xffffffff, seed >> 32)).
 *              Streams: 0 init, 1 hidden, 3 visible primary, 4 visible
 *              refinement, 5 MH, 6 AR proposals.
 *   column words: word w covers columns 32w .. 32w + m_w - 1,
 *              m_w = min(32, L - 32 w), and cells 16w .. 16w + m_w/2 - 1;
 *              W = ceil(L/32).
 *   hidden uniform (bit-sliced): hidden unit (k,i,j), w = j/16, n = m_w/2,
 *              u = 2 n (k/2) + 2 (j - 16 w) + (k % 2), pw = u/32.  Bit b of U
 *              (b = 0 most significant) is bit u%32 of out[b & 3] of the block
 *              c0 = ((i W + w) << 8) | (pw << 3) | (b >> 2), stream 1.
 *   spin uniform: U = (P << 16) | Q with P, Q the 16-bit slot q of the blocks
 *              c0 = ((i W + w) << 5) | (q >> 3) of streams 3 and 4, for spin
 *              (r,c), i = r/2, w = c/32, q = (r - 2i) m_w + (c - 32 w); slot q
 *              of a block is (out[(q & 7) >> 1] >> (16 (q & 1))) & 0xffff.
 *   init       s(r,c) = +1 iff bit b = (rL + c) & 127 of the block
 *              Philox(ctr = ((rL + c) >> 7, 0, chain, id << 3 | 0)) is set,
 *              bit b being bit (b & 31) of out[b >> 5].
 *   counts     M = sum s, B1 = sum over J1 bonds s_a s_b, B2 = same over dimers;
 *              energy E_q = J1q B1 + J2q B2 - hq M (exact, 2^16 units).
 */
#include "crbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ Philox */

/* Philox4x32 with 10 rounds, written from the description in Salmon, Moraes,
 * Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11):
 * each round multiplies counter words 0 and 2 by the two round multipliers,
 * swaps the halves across and xors in the other counter words and the round
 * key; the key is advanced by the two Weyl increments between rounds. */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* 16-bit slot q (0..7) of the block with counter word c0. */
static uint32_t slot16(uint64_t seed, uint32_t id, uint32_t stream, uint32_t chain,
                       uint32_t sweep, uint32_t c0, int q)
{
    uint32_t ctr[4] = { c0, sweep, chain, (id << 3) | stream };
    uint32_t key[2] = { (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    return (out[(q & 7) >> 1] >> (16 * (q & 1))) & 0xffffu;
}

/* The unit's 32-bit uniform: primary 16 bits on top, refinement below. */
static uint32_t unit_uniform(uint64_t seed, uint32_t id, uint32_t stream_primary,
                             uint32_t chain, uint32_t sweep, uint32_t c0, int q)
{
    uint32_t p = slot16(seed, id, stream_primary, chain, sweep, c0, q);
    uint32_t r = slot16(seed, id, stream_primary + 1u, chain, sweep, c0, q);
    return (p << 16) | r;
}

uint32_t oracle_uniform_hidden(uint64_t seed, uint32_t id, uint32_t chain, uint32_t sweep,
                               int L, int k, int i, int j)
{
    /* Bit-sliced draw: the hidden units of (cell row i, column word w) are
     * numbered u = 2 n (k / 2) + 2 (j - 16 w) + (k % 2), n = cells in the
     * word, and packed 32 to a word (pw = u / 32, bit u % 32).  Bit b of the
     * unit's uniform (b = 0 the most significant) is bit (u % 32) of random
     * word b & 3 of the Philox block with counter word
     * ((i W + w) << 8) | (pw << 3) | (b >> 2), stream 1. */
    int W = (L + 31) / 32;
    int w = j / 16;
    int m = (L - 32 * w) < 32 ? (L - 32 * w) : 32;
    int n = m / 2;
    int u = 2 * n * (k / 2) + 2 * (j - 16 * w) + (k % 2);
    int pw = u / 32, bit = u % 32;
    uint32_t key[2] = { (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    uint32_t U = 0;
    for (int b = 0; b < 32; ++b) {
        uint32_t ctr[4] = { ((uint32_t)(i * W + w) << 8) | ((uint32_t)pw << 3) | (uint32_t)(b >> 2),
                            sweep, chain, (id << 3) | 1u };
        uint32_t out[4];
        oracle_philox4x32_10(ctr, key, out);
        U |= ((out[b & 3] >> bit) & 1u) << (31 - b);
    }
    return U;
}

uint32_t oracle_uniform_visible(uint64_t seed, uint32_t id, uint32_t chain, uint32_t sweep,
                                int L, int r, int c)
{
    int W = (L + 31) / 32;
    int i = r / 2;
    int w = c / 32;
    int m = (L - 32 * w) < 32 ? (L - 32 * w) : 32;
    int q = (r - 2 * i) * m + (c - 32 * w);
    uint32_t c0 = ((uint32_t)(i * W + w) << 5) | (uint32_t)(q >> 3);
    return unit_uniform(seed, id, 3u, chain, sweep, c0, q);
}

/* ------------------------------------------------------- quantisation etc. */

int64_t oracle_quantise(double J)
{
    return llround(J * 65536.0);
}

double oracle_schedule_T(int kind, double T0, double T1, const double* T_explicit,
                         int64_t S, int64_t s)
{
    switch (kind) {
    case 0: /* constant */
        return T0;
    case 1: /* linear, inclusive end points */
        if (S <= 1) return T0;
        return T0 + (T1 - T0) * ((double)s / (double)(S - 1));
    case 2: /* geometric, inclusive end points */
        if (S <= 1) return T0;
        return T0 * pow(T1 / T0, (double)s / (double)(S - 1));
    case 3:
        return T_explicit[s];
    default:
        return NAN;
    }
}

/* Hidden-unit weight magnitude and sign for a bond of quantised coupling Jq at
 * temperature T (Eqs. (6)-(7) with K = -J/T; the stable form of
 * arccosh(exp(2|K|))/2 is |K| + log1p(sqrt(1 - exp(-4|K|)))/2). */
void oracle_bond_weight(int64_t Jq, double T, int64_t* wq, int* sig)
{
    double K = -((double)Jq / 65536.0) / T;
    double a = fabs(K);
    double w = a + 0.5 * log1p(sqrt(-expm1(-4.0 * a)));
    *wq = llround(w * 65536.0);
    *sig = (K < 0.0) ? -1 : +1;
}

int64_t oracle_visible_bias(int64_t hq, double T)
{
    return llround((double)hq / T);
}

uint32_t oracle_threshold(int64_t y)
{
    double z = 2.0 * ldexp((double)y, -16);
    double p = 1.0 / (1.0 + exp(-z));
    double t = floor(p * 4294967296.0 + 0.5);
    if (t > 4294967295.0) t = 4294967295.0;
    return (uint32_t)t;
}

/* ---------------------------------------------- hardware precision mode */

/* App. A Dimension and Precision: the convolution uses 10-bit signed fixed
 * point with 4 fraction bits (steps of 1/16, magnitude at most 511/16, read
 * here as saturating), the accumulator 2 more integer bits (2047/16); App. A
 * Sigmoid and LFSR-Forward: the sigmoid is the closest 16-bit value and is
 * compared with a 16-bit uniform.  Values in 2^-16 units. */
#define Q54_STEP 4096
#define Q54_MAX (511 * Q54_STEP)
#define ACC_MAX (2047 * Q54_STEP)

int64_t oracle_q54(double v)
{
    long m = lround(fabs(v) * 16.0);
    if (m > 511) m = 511;
    return (int64_t)(v < 0.0 ? -m : m) * Q54_STEP;
}

static int64_t clamp_abs(int64_t x, int64_t lim)
{
    return x > lim ? lim : (x < -lim ? -lim : x);
}

/* closest 16-bit value of sigmoid(2 y 2^-16), capped at 65535 */
uint32_t oracle_sigmoid16(int64_t y)
{
    double p = 1.0 / (1.0 + exp(-2.0 * ldexp((double)y, -16)));
    double t = floor(p * 65536.0 + 0.5);
    return t > 65535.0 ? 65535u : (uint32_t)t;
}

void oracle_bond_weight_q54(int64_t Jq, double T, int64_t* wq, int* sig)
{
    double K = -((double)Jq / 65536.0) / T;
    double a = fabs(K);
    *wq = oracle_q54(a + 0.5 * log1p(sqrt(-expm1(-4.0 * a))));
    *sig = (K < 0.0) ? -1 : +1;
}

/* ------------------------------------------------------------------- bonds */

/* Window offsets (dr_a, dc_a, dr_b, dc_b) and coupling type (1 = J1, 2 = J2)
 * of the 10 filters. */
static const int BOND[10][5] = {
    { 0, 0, 0, 1, 1 }, { 0, 1, 0, 2, 1 }, { 1, 0, 1, 1, 1 }, { 1, 1, 1, 2, 1 },
    { 0, 0, 1, 0, 1 }, { 1, 0, 2, 0, 1 }, { 0, 1, 1, 1, 1 }, { 1, 1, 2, 1, 1 },
    { 0, 0, 1, 1, 2 }, { 1, 2, 2, 1, 2 },
};

void oracle_bond_sites(int L, int k, int i, int j, int* ra, int* ca, int* rb, int* cb, int* type)
{
    *ra = (2 * i + BOND[k][0]) % L;
    *ca = (2 * j + BOND[k][1]) % L;
    *rb = (2 * i + BOND[k][2]) % L;
    *cb = (2 * j + BOND[k][3]) % L;
    *type = BOND[k][4];
}

/* ---------------------------------------------------------------- counts */

void oracle_counts(int L, const int8_t* s, int64_t* M, int64_t* B1, int64_t* B2)
{
    int64_t m = 0, b1 = 0, b2 = 0;
    int C = L / 2;
    for (int r = 0; r < L; ++r)
        for (int c = 0; c < L; ++c) m += s[r * L + c];
    for (int i = 0; i < C; ++i)
        for (int j = 0; j < C; ++j)
            for (int k = 0; k < 10; ++k) {
                int ra, ca, rb, cb, type;
                oracle_bond_sites(L, k, i, j, &ra, &ca, &rb, &cb, &type);
                int prod = s[ra * L + ca] * s[rb * L + cb];
                if (type == 1) b1 += prod; else b2 += prod;
            }
    *M = m; *B1 = b1; *B2 = b2;
}

/* Staggered (Neel) magnetisation sum_{r,c} (-1)^(r+c) s(r,c): +-N in the two
 * Neel states of the square-lattice bonds (the antiferromagnetic phase of
 * Sec. III.A, whose S(q) peaks at (pi, pi) in Sec. III.B). */
int64_t oracle_staggered(int L, const int8_t* s)
{
    int64_t ms = 0;
    for (int r = 0; r < L; ++r)
        for (int c = 0; c < L; ++c) ms += ((r + c) % 2 == 0) ? s[r * L + c] : -s[r * L + c];
    return ms;
}

void oracle_corr(int L, const int8_t* s, int64_t* corr)
{
    /* corr[dr * L + dc] += sum_{r,c} s(r,c) s(r+dr, c+dc) */
    for (int dr = 0; dr < L; ++dr)
        for (int dc = 0; dc < L; ++dc) {
            int64_t acc = 0;
            for (int r = 0; r < L; ++r)
                for (int c = 0; c < L; ++c)
                    acc += s[r * L + c] * s[((r + dr) % L) * L + (c + dc) % L];
            corr[dr * L + dc] += acc;
        }
}

/* Plateau structure factor (Sec. III.B Eq. (13) at the 1/3-plateau wave
 * vectors): out[1] = |sum_{r,c} s(r,c) exp(i (pi r + 2 pi c / 3))|^2,
 * out[2] = |sum s(r,c) exp(i (2 pi r / 3 + pi c))|^2, out[0] = max of the two.
 * The true values are integers (the sums lie in Z[e^{2 pi i/3}]); they are
 * evaluated here with cos/sin in double and rounded. */
void oracle_order(int L, const int8_t* s, int64_t out[3])
{
    const double pi = 3.14159265358979323846;
    double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
    for (int r = 0; r < L; ++r)
        for (int c = 0; c < L; ++c) {
            const double v = s[r * L + c];
            const double pa = pi * r + 2.0 * pi * c / 3.0, pb = 2.0 * pi * r / 3.0 + pi * c;
            ar += v * cos(pa);
            ai += v * sin(pa);
            br += v * cos(pb);
            bi += v * sin(pb);
        }
    out[1] = llround(ar * ar + ai * ai);
    out[2] = llround(br * br + bi * bi);
    out[0] = out[1] > out[2] ? out[1] : out[2];
}

/* ------------------------------------------------------------- one chain */

static int sweep_params(const oracle_instance* in, int64_t S, int64_t s,
                        int64_t* wq1, int* sg1, int64_t* wq2, int* sg2, int64_t* aq)
{
    double T = oracle_schedule_T(in->sched_kind, in->T0, in->T1, in->T_explicit, S, s);
    if (!(T > 0.0) || !isfinite(T)) return -1;
    int64_t J1q = oracle_quantise(in->J1), J2q = oracle_quantise(in->J2), hq = oracle_quantise(in->h);
    if (in->precision == 1) {
        oracle_bond_weight_q54(J1q, T, wq1, sg1);
        oracle_bond_weight_q54(J2q, T, wq2, sg2);
        *aq = oracle_q54(((double)hq / 65536.0) / T);
        return 0;
    }
    oracle_bond_weight(J1q, T, wq1, sg1);
    oracle_bond_weight(J2q, T, wq2, sg2);
    *aq = oracle_visible_bias(hq, T);
    return 0;
}

void oracle_init_spins(const oracle_instance* in, uint64_t seed, uint32_t chain, int8_t* s)
{
    int L = in->L;
    uint32_t key[2] = { (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    for (int r = 0; r < L; ++r)
        for (int c = 0; c < L; ++c) {
            uint32_t site = (uint32_t)(r * L + c);
            uint32_t ctr[4] = { site >> 7, 0u, chain, (in->id << 3) | 0u };
            uint32_t out[4];
            oracle_philox4x32_10(ctr, key, out);
            uint32_t b = site & 127u;
            int bit = (out[b >> 5] >> (b & 31u)) & 1u;
            s[r * L + c] = bit ? +1 : -1;
        }
}

static int8_t gibbs_unit(int64_t x, uint32_t U)
{
    int8_t sgn = (x >= 0) ? +1 : -1;
    int64_t y = (x >= 0) ? x : -x;
    return (U < oracle_threshold(y)) ? sgn : (int8_t)(-sgn);
}

/* hardware precision: field saturated to lim, 16-bit sigmoid against the top
 * 16 bits of the unit's uniform */
static int8_t gibbs_unit16(int64_t x, int64_t lim, uint32_t U)
{
    x = clamp_abs(x, lim);
    int8_t sgn = (x >= 0) ? +1 : -1;
    int64_t y = (x >= 0) ? x : -x;
    return ((U >> 16) < oracle_sigmoid16(y)) ? sgn : (int8_t)(-sgn);
}

int oracle_run_chain(const oracle_instance* in, int64_t S, uint64_t seed, uint32_t chain,
                     int64_t sweep_begin, int64_t sweep_end, int8_t* s,
                     int32_t* trace, int32_t measure_every, int64_t burn_in, int64_t* acc,
                     int64_t* corr_acc)
{
    int L = in->L;
    int C = L / 2;
    int8_t* hid = (int8_t*)malloc((size_t)10 * C * C);
    int64_t* field = (int64_t*)malloc(sizeof(int64_t) * (size_t)L * L);
    if (!hid || !field) { free(hid); free(field); return -3; }
    for (int64_t sw = sweep_begin; sw < sweep_end; ++sw) {
        int64_t wq1, wq2, aq;
        int sg1, sg2;
        if (sweep_params(in, S, sw, &wq1, &sg1, &wq2, &sg2, &aq) != 0) {
            free(hid);
            free(field);
            return -1;
        }
        uint32_t sweep = (uint32_t)sw;
        /* hidden half-step, Eq. (11): every hidden unit from the old spins */
        for (int k = 0; k < 10; ++k)
            for (int i = 0; i < C; ++i)
                for (int j = 0; j < C; ++j) {
                    int ra, ca, rb, cb, type;
                    oracle_bond_sites(L, k, i, j, &ra, &ca, &rb, &cb, &type);
                    int64_t wq = (type == 1) ? wq1 : wq2;
                    int sg = (type == 1) ? sg1 : sg2;
                    int64_t x = wq * (int64_t)(s[ra * L + ca] + sg * s[rb * L + cb]);
                    uint32_t U = oracle_uniform_hidden(seed, in->id, chain, sweep, L, k, i, j);
                    hid[(k * C + i) * C + j] = in->precision == 1 ? gibbs_unit16(x, Q54_MAX, U) : gibbs_unit(x, U);
                }
        /* visible half-step, Eq. (12) plus the visible bias: every spin from
         * the hidden units just drawn.  Accumulate fields bond by bond. */
        for (int q = 0; q < L * L; ++q) field[q] = aq;
        for (int k = 0; k < 10; ++k)
            for (int i = 0; i < C; ++i)
                for (int j = 0; j < C; ++j) {
                    int ra, ca, rb, cb, type;
                    oracle_bond_sites(L, k, i, j, &ra, &ca, &rb, &cb, &type);
                    int64_t wq = (type == 1) ? wq1 : wq2;
                    int sg = (type == 1) ? sg1 : sg2;
                    int64_t hv = hid[(k * C + i) * C + j];
                    field[ra * L + ca] += wq * hv;
                    field[rb * L + cb] += wq * sg * hv;
                }
        for (int r = 0; r < L; ++r)
            for (int c = 0; c < L; ++c) {
                uint32_t U = oracle_uniform_visible(seed, in->id, chain, sweep, L, r, c);
                s[r * L + c] = in->precision == 1 ? gibbs_unit16(field[r * L + c], ACC_MAX, U)
                                                  : gibbs_unit(field[r * L + c], U);
            }
        const int measured = measure_every > 0 && sw >= burn_in && (sw - burn_in) % measure_every == 0;
        if (trace || acc) {
            int64_t M, B1, B2;
            oracle_counts(L, s, &M, &B1, &B2);
            if (trace) {
                int32_t* t = trace + 3 * (sw - sweep_begin);
                t[0] = (int32_t)M; t[1] = (int32_t)B1; t[2] = (int32_t)B2;
            }
            if (acc && measured) {
                int64_t ms = oracle_staggered(L, s);
                acc[0] += 1;
                acc[1] += M; acc[2] += B1; acc[3] += B2;
                acc[4] += M * M; acc[5] += B1 * B1; acc[6] += B2 * B2;
                acc[7] += M * B1; acc[8] += M * B2; acc[9] += B1 * B2;
                acc[10] += (M < 0) ? -M : M;
                acc[11] += ms; acc[12] += ms * ms; acc[13] += (ms < 0) ? -ms : ms;
            }
        }
        if (corr_acc && measured) oracle_corr(L, s, corr_acc);  /* Sec. III.B Eq. (13): summed C(dr, dc) */
    }
    free(hid);
    free(field);
    return 0;
}

/* ------------------------------------------------- CRBM marginal (checks) */

/* log of sum over all hidden units of exp(sum_b w_b h_b (s_a + sig_b s_b) + a sum s),
 * with the real-valued weights w = wq/2^16, a = aq/2^16 of sweep s: each hidden
 * unit sums out to 2 cosh(w (s_a + sig s_b)), Eq. (4). */
double oracle_log_marginal(const oracle_instance* in, int64_t S, int64_t sweep, const int8_t* s)
{
    int64_t wq1, wq2, aq;
    int sg1, sg2;
    if (sweep_params(in, S, sweep, &wq1, &sg1, &wq2, &sg2, &aq) != 0) return NAN;
    int L = in->L, C = L / 2;
    double acc = 0.0;
    int64_t M = 0;
    for (int q = 0; q < L * L; ++q) M += s[q];
    acc += ldexp((double)aq, -16) * (double)M;
    for (int k = 0; k < 10; ++k)
        for (int i = 0; i < C; ++i)
            for (int j = 0; j < C; ++j) {
                int ra, ca, rb, cb, type;
                oracle_bond_sites(L, k, i, j, &ra, &ca, &rb, &cb, &type);
                double w = ldexp((double)((type == 1) ? wq1 : wq2), -16);
                int sg = (type == 1) ? sg1 : sg2;
                double x = w * (double)(s[ra * L + ca] + sg * s[rb * L + cb]);
                acc += log(2.0 * cosh(x));
            }
    return acc;
}

/* ==================================================================== */
/* General lattices: open or periodic axes, rectangular Lr x Lc, one      */
/* coupling per filter, a field per column parity.                        */
/* ==================================================================== */
/*
 * What it follows:
 *   - App. A Wrapper Module: per axis, the lattice either wraps (the first
 *     columns / rows are copied past the last ones) or is padded with zeros.
 *     Reading: on an open axis a bond whose endpoint falls past the last row
 *     (column) does not exist: no hidden unit is drawn for it and no field
 *     reaches its remaining spin.  (A hidden unit coupled to a padded zero
 *     would see one spin only; summed out it gives the constant 2 cosh(w),
 *     so the marginal law of the spins is the same either way; leaving the
 *     bond out also leaves no stray noise in the dynamics.)
 *   - App. A Hidden Node Registers: floor((L+1)/2) cells per axis; for the
 *     even sizes taken here that is L/2.
 *   - App. A Convoluter-Reverse: every filter has its own weights (raw
 *     filters), so each of the 10 filters k carries its own coupling J_k
 *     (the SS lattice is J_k = J1 for k < 8, J2 for k = 8, 9).
 *   - App. A Accumulator: separate visible biases for even and odd columns.
 *
 * Conventions (beyond those at the top of this file, which they reduce to
 * for a periodic square lattice with J_k = (J1 x 8, J2 x 2), h_even = h_odd):
 *   spins      s(r,c), 0 <= r < Lr, 0 <= c < Lc, Lr and Lc even.
 *   cells      (i,j), 0 <= i < Lr/2, 0 <= j < Lc/2; bond k of cell (i,j) joins
 *              (2i + dr_a, 2j + dc_a) and (2i + dr_b, 2j + dc_b) (the table
 *              above); a coordinate equal to Lr (Lc) wraps to 0 on a periodic
 *              axis and makes the bond absent on an open one.
 *   weights    per sweep and filter k: K_k = -(Jq_k / 2^16) / T_s, sig_k, wq_k
 *              as above; visible bias aq_p = llround(hq_p / T_s) for column
 *              parity p = c mod 2.
 *   uniforms   the hidden and spin uniforms of the square lattice with the
 *              column layout of Lc (W = ceil(Lc/32) words per row, i the cell
 *              row); init: site index r Lc + c.
 *   counts     M_e, M_o = spin sums over even / odd columns; B_k = sum over the
 *              present bonds of filter k of s_a s_b; energy
 *              E_q = sum_k Jq_k B_k - hq_e M_e - hq_o M_o (exact, 2^16 units).
 *   corr       Cn(dr, dc) = sum over sites with (r + dr, c + dc) inside the
 *              lattice of s(r,c) s(r+dr, c+dc), 0 <= dr < Lr, -Lc < dc < Lc,
 *              no wrapping, stored [dr][dc + Lc - 1]: for every wave vector q,
 *              |sum_r s_r e^{i q.r}|^2 = sum over all displacements of
 *              Cn(d) e^{i q.d} (Eq. (13)), with Cn(-d) = Cn(d).
 */


/* Sites of bond k of cell (i,j); returns 1 if the bond exists. */
int oracle_lattice_bond(const oracle_lattice* in, int k, int i, int j, int* ra, int* ca, int* rb, int* cb)
{
    int r0 = 2 * i + BOND[k][0], c0 = 2 * j + BOND[k][1];
    int r1 = 2 * i + BOND[k][2], c1 = 2 * j + BOND[k][3];
    if (r0 >= in->Lr || r1 >= in->Lr) {
        if (in->open_r) return 0;
        r0 %= in->Lr;
        r1 %= in->Lr;
    }
    if (c0 >= in->Lc || c1 >= in->Lc) {
        if (in->open_c) return 0;
        c0 %= in->Lc;
        c1 %= in->Lc;
    }
    *ra = r0; *ca = c0; *rb = r1; *cb = c1;
    return 1;
}

void oracle_lattice_counts(const oracle_lattice* in, const int8_t* s, int64_t out[12])
{
    int Lr = in->Lr, Lc = in->Lc;
    for (int q = 0; q < 12; ++q) out[q] = 0;
    for (int r = 0; r < Lr; ++r)
        for (int c = 0; c < Lc; ++c) out[c % 2] += s[r * Lc + c];
    for (int k = 0; k < 10; ++k)
        for (int i = 0; i < Lr / 2; ++i)
            for (int j = 0; j < Lc / 2; ++j) {
                int ra, ca, rb, cb;
                if (oracle_lattice_bond(in, k, i, j, &ra, &ca, &rb, &cb))
                    out[2 + k] += s[ra * Lc + ca] * s[rb * Lc + cb];
            }
}

void oracle_lattice_corr(int Lr, int Lc, const int8_t* s, int64_t* corr)
{
    /* corr[dr][dc + Lc - 1] += sum of s(r,c) s(r+dr, c+dc) over pairs inside the lattice */
    for (int dr = 0; dr < Lr; ++dr)
        for (int dc = -(Lc - 1); dc < Lc; ++dc) {
            int64_t acc = 0;
            for (int r = 0; r + dr < Lr; ++r)
                for (int c = 0; c < Lc; ++c) {
                    int c2 = c + dc;
                    if (c2 < 0 || c2 >= Lc) continue;
                    acc += s[r * Lc + c] * s[(r + dr) * Lc + c2];
                }
            corr[dr * (2 * Lc - 1) + dc + Lc - 1] += acc;
        }
}

void oracle_lattice_init_spins(const oracle_lattice* in, uint64_t seed, uint32_t chain, int8_t* s)
{
    uint32_t key[2] = { (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    for (int r = 0; r < in->Lr; ++r)
        for (int c = 0; c < in->Lc; ++c) {
            uint32_t site = (uint32_t)(r * in->Lc + c);
            uint32_t ctr[4] = { site >> 7, 0u, chain, (in->id << 3) | 0u };
            uint32_t out[4];
            oracle_philox4x32_10(ctr, key, out);
            uint32_t b = site & 127u;
            s[r * in->Lc + c] = ((out[b >> 5] >> (b & 31u)) & 1u) ? +1 : -1;
        }
}

/* Per-sweep weights of a general lattice: wq[k], sig[k] per filter, aq[p] per column parity. */
static int lattice_params(const oracle_lattice* in, int64_t S, int64_t s, int64_t wq[10], int sig[10],
                          int64_t aq[2])
{
    double T = oracle_schedule_T(in->sched_kind, in->T0, in->T1, in->T_explicit, S, s);
    if (!(T > 0.0) || !isfinite(T)) return -1;
    for (int k = 0; k < 10; ++k) oracle_bond_weight(oracle_quantise(in->J[k]), T, &wq[k], &sig[k]);
    aq[0] = oracle_visible_bias(oracle_quantise(in->h_even), T);
    aq[1] = oracle_visible_bias(oracle_quantise(in->h_odd), T);
    return 0;
}

int oracle_lattice_run_chain(const oracle_lattice* in, int64_t S, uint64_t seed, uint32_t chain,
                             int64_t sweep_begin, int64_t sweep_end, int8_t* s, int32_t* trace,
                             int32_t measure_every, int64_t burn_in, int64_t* acc, int64_t* corr_acc)
{
    int Lr = in->Lr, Lc = in->Lc, Cr = Lr / 2, Cc = Lc / 2;
    int8_t* hid = (int8_t*)malloc((size_t)10 * Cr * Cc);
    int64_t* field = (int64_t*)malloc(sizeof(int64_t) * (size_t)Lr * Lc);
    if (!hid || !field) { free(hid); free(field); return -3; }
    for (int64_t sw = sweep_begin; sw < sweep_end; ++sw) {
        int64_t wq[10], aq[2];
        int sig[10];
        if (lattice_params(in, S, sw, wq, sig, aq) != 0) {
            free(hid);
            free(field);
            return -1;
        }
        uint32_t sweep = (uint32_t)sw;
        /* hidden half-step, Eq. (11): every present bond's unit from the old spins */
        for (int k = 0; k < 10; ++k)
            for (int i = 0; i < Cr; ++i)
                for (int j = 0; j < Cc; ++j) {
                    int ra, ca, rb, cb;
                    int8_t* h = &hid[(k * Cr + i) * Cc + j];
                    if (!oracle_lattice_bond(in, k, i, j, &ra, &ca, &rb, &cb)) {
                        *h = 0;
                        continue;
                    }
                    int64_t x = wq[k] * (int64_t)(s[ra * Lc + ca] + sig[k] * s[rb * Lc + cb]);
                    *h = gibbs_unit(x, oracle_uniform_hidden(seed, in->id, chain, sweep, Lc, k, i, j));
                }
        /* visible half-step, Eq. (12), with the column-parity bias of App. A Accumulator */
        for (int r = 0; r < Lr; ++r)
            for (int c = 0; c < Lc; ++c) field[r * Lc + c] = aq[c % 2];
        for (int k = 0; k < 10; ++k)
            for (int i = 0; i < Cr; ++i)
                for (int j = 0; j < Cc; ++j) {
                    int ra, ca, rb, cb;
                    if (!oracle_lattice_bond(in, k, i, j, &ra, &ca, &rb, &cb)) continue;
                    int64_t hv = hid[(k * Cr + i) * Cc + j];
                    field[ra * Lc + ca] += wq[k] * hv;
                    field[rb * Lc + cb] += wq[k] * sig[k] * hv;
                }
        for (int r = 0; r < Lr; ++r)
            for (int c = 0; c < Lc; ++c)
                s[r * Lc + c] = gibbs_unit(field[r * Lc + c],
                                           oracle_uniform_visible(seed, in->id, chain, sweep, Lc, r, c));
        const int measured = measure_every > 0 && sw >= burn_in && (sw - burn_in) % measure_every == 0;
        if (trace || (acc && measured)) {
            int64_t cnt[12];
            oracle_lattice_counts(in, s, cnt);
            if (trace)
                for (int q = 0; q < 12; ++q) trace[12 * (sw - sweep_begin) + q] = (int32_t)cnt[q];
            if (acc && measured) {
                int64_t M = cnt[0] + cnt[1], ms = 0;
                for (int r = 0; r < Lr; ++r)
                    for (int c = 0; c < Lc; ++c) ms += ((r + c) % 2 == 0) ? s[r * Lc + c] : -s[r * Lc + c];
                acc[0] += 1;
                for (int q = 0; q < 12; ++q) acc[1 + q] += cnt[q];
                acc[13] += M * M;
                acc[14] += M < 0 ? -M : M;
                acc[15] += ms;
                acc[16] += ms * ms;
                acc[17] += ms < 0 ? -ms : ms;
            }
        }
        if (corr_acc && measured) oracle_lattice_corr(Lr, Lc, s, corr_acc);
    }
    free(hid);
    free(field);
    return 0;
}

/* log of the sum over the hidden units of exp(sum_b w_b h_b (s_a + sig_b s_b) + sum_c a_{c%2} s),
 * real-valued weights of sweep s (Eq. (4) on a general lattice: present bonds only). */
double oracle_lattice_log_marginal(const oracle_lattice* in, int64_t S, int64_t sweep, const int8_t* s)
{
    int64_t wq[10], aq[2];
    int sig[10];
    if (lattice_params(in, S, sweep, wq, sig, aq) != 0) return NAN;
    int Lr = in->Lr, Lc = in->Lc;
    double acc = 0.0;
    for (int r = 0; r < Lr; ++r)
        for (int c = 0; c < Lc; ++c) acc += ldexp((double)aq[c % 2], -16) * (double)s[r * Lc + c];
    for (int k = 0; k < 10; ++k)
        for (int i = 0; i < Lr / 2; ++i)
            for (int j = 0; j < Lc / 2; ++j) {
                int ra, ca, rb, cb;
                if (!oracle_lattice_bond(in, k, i, j, &ra, &ca, &rb, &cb)) continue;
                double x = ldexp((double)wq[k], -16) * (double)(s[ra * Lc + ca] + sig[k] * s[rb * Lc + cb]);
                acc += log(2.0 * cosh(x));
            }
    return acc;
}
