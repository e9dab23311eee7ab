// gibbs_kernel.h -- gfx950 device code for block Gibbs sampling of the CRBM
// that encodes the classical Shastry-Sutherland Ising lattice
// (Brahma et al., arXiv 2511.20911, Sec. II.A-II.B, App. A).
//
// Layout and mapping
//   * A chain's spins are bit rows of W = ceil(L/32) words (bit c of word w =
//     column 32w + c, 1 = up).
//   * A chain is handled by G = (L/2)/R lanes of one wavefront; lane g owns the
//     band of cell rows g*R .. g*R+R-1 (spin rows 2gR .. 2gR+2R-1) and keeps it
//     in registers for the whole launch.  64/G chains share a wavefront; all
//     chains of a wavefront belong to one instance, so the per-sweep weights
//     and thresholds are wavefront-uniform.
//   * Hidden units are never stored: a cell row's 10 hidden planes (one bit per
//     cell, at the cell's even column) are drawn from the old spins and consumed
//     at once by the visible update of the rows that need them.  The first row
//     of a band also needs the last hidden row of the band above; it is updated
//     last, after a lane shuffle (the periodic copy of App. A Zero Padder).
//
// Hidden half-step (Eq. (11)), bit-sliced: a bond "agrees" if s_a == sig s_b,
// giving field 2 wq s_a, else field 0.  The unit takes the field's sign with
// probability t(|x|)/2^32.  All agreeing J1 (resp. J2) bonds share one
// threshold T1 (T2), disagreeing ones have 2^31, so the comparison U < t runs
// over 32 packed units at a time: random words are consumed as bit planes of U,
// most significant first, against the threshold's bits, until no unit of the
// wavefront is still tied (usually 12-16 planes).
//
// Visible half-step (Eq. (12)): field = aq + wq1 (2n - 4) + wq2 (2d - 1) with n
// the number of +1 J1 terms and d the dimer term; n is summed bit-sliced over a
// row, the threshold is looked up per spin by (n, d) from a 10-entry table held
// one entry per lane.  U = (P << 16) | Q with P, Q 16-bit Philox slots; Q is
// drawn only when P equals the threshold's top half (probability 2^-16).
// With tc = ceil(t / 2^16), P >= tc decides U >= t except where P = tc - 1,
// which holds every such tie (and, when 2^16 divides t, P = t/2^16 - 1,
// which the exact path then decides as well).  The table entry carries the
// field's sign as 2^31 added to tc where the field is negative, so the sign
// bit of P - entry is the new spin itself (1 = up): P < tc for a field >= 0,
// P >= tc for a negative one; a tie leaves 0xffff in the low half either way.
#pragma once
#include "crbm_internal.h"

namespace crbmlib {
namespace gk {

constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;  // Philox round multipliers
constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;  // Philox key increments

struct P4 {
    uint32_t v[4];
};

// a ^ b ^ k in one VALU op (gfx950 three-input bitwise op, xor3 truth table).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t k) {
    return __builtin_amdgcn_bitop3_b32(a, b, k, 0x96);
}

// Philox4x32-10 (Salmon et al., SC'11).  c1 and c3 enter as wavefront-uniform
// words (sweep index, stream word); the key schedule is scalar.  Each round is
// two 32x32->64 multiplies (v_mad_u64_u32) and two three-input xors.
__device__ __forceinline__ P4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                     uint32_t k1) {
    uint64_t p0 = (uint64_t)kM0 * c0;
    uint64_t p1 = (uint64_t)kM1 * c2;
    uint32_t x0 = (uint32_t)(p1 >> 32) ^ (c1 ^ k0);
    // one VALU op with the uniform c3 ^ k1 as its scalar operand (an ordinary
    // xor chain is reassociated into two vector xors)
    uint32_t x2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3 ^ k1, 0u, 0xF0 ^ 0xCC);
    uint32_t x1 = (uint32_t)p1, x3 = (uint32_t)p0;
#pragma unroll
    for (int r = 1; r < 10; ++r) {
        k0 += kW0;
        k1 += kW1;
        p0 = (uint64_t)kM0 * x0;
        p1 = (uint64_t)kM1 * x2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), x1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), x3, k1);
        x1 = (uint32_t)p1;
        x3 = (uint32_t)p0;
        x0 = n0;
        x2 = n2;
    }
    return P4{{x0, x1, x2, x3}};
}

__device__ __forceinline__ uint32_t slot16(const P4& p, int s) {
    const uint32_t w = p.v[s >> 1];
    return (s & 1) ? (w >> 16) : (w & 0xffffu);
}

template <int L>
struct Geo {
    static constexpr int W = (L + 31) / 32;   // words per row
    static constexpr int C = L / 2;           // cells per cell row
    static constexpr int ML = L - 32 * (W - 1);  // columns in the last word
    __host__ __device__ static constexpr int m(int w) { return w == W - 1 ? ML : 32; }
    __host__ __device__ static constexpr int n(int w) { return m(w) / 2; }
    __host__ __device__ static constexpr uint32_t full(int w) {
        return m(w) == 32 ? 0xffffffffu : ((1u << m(w)) - 1u);
    }
    __host__ __device__ static constexpr uint32_t even(int w) { return 0x55555555u & full(w); }
    // columns 32 w + b with (32 w + b) mod 3 == k
    __host__ __device__ static constexpr uint32_t mod3(int w, int k) {
        uint32_t m = 0u;
        for (int b = 0; b < 32; ++b)
            if ((32 * w + b) % 3 == k) m |= 1u << b;
        return m & full(w);
    }
    __host__ __device__ static constexpr int cnt3(int k) { return (L - k + 2) / 3; }  // columns c < L, c % 3 == k
};

// bit c of word w <- column 32w + c + S (mod L), S in {1, 2}
template <int L, int S>
__device__ __forceinline__ uint32_t rsh(const uint32_t (&x)[Geo<L>::W], int w) {
    using G = Geo<L>;
    if (w < G::W - 1) return (x[w] >> S) | (x[w + 1] << (32 - S));
    const uint32_t wrap = x[0] & ((1u << S) - 1u);
    return ((x[w] >> S) | (wrap << (G::ML - S))) & G::full(G::W - 1);
}

// bit c of word w <- column 32w + c - 2 (mod L)
template <int L>
__device__ __forceinline__ uint32_t lsh2(const uint32_t (&x)[Geo<L>::W], int w) {
    using G = Geo<L>;
    if (w > 0) return ((x[w] << 2) | (x[w - 1] >> 30)) & G::full(w);
    const uint32_t top = (x[G::W - 1] >> (G::ML - 2)) & 3u;
    return ((x[0] << 2) | top) & G::full(0);
}

// Wavefront-uniform constants of one sweep, plus the per-lane visible table.
struct SweepK {
    uint32_t T[2];     // hidden agree thresholds (J1, J2), >= 2^31
    uint32_t neg[2];   // all ones if sig_t < 0
    uint32_t en[2];    // all ones if wq_t != 0
    uint32_t kge[2];   // spin field >= 0 iff n >= kge[d]
    uint32_t tabv;     // lane l < 10: ceil(t / 2^16) of visible entry l (0 .. 2^16), plus 2^31
                       // where the entry's field is negative
    uint32_t tfull;    // lane l < 10: full visible threshold t of entry l
};

__device__ __forceinline__ SweepK load_sweep(const uint32_t* tb, int lane) {
    SweepK K;
    const uint32_t fl = tb[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        K.T[t] = tb[t];
        K.neg[t] = (fl & (1u << t)) ? 0xffffffffu : 0u;
        K.en[t] = (fl & (4u << t)) ? 0xffffffffu : 0u;
        K.kge[t] = (fl >> (8 + 4 * t)) & 15u;
    }
    const int l = lane < 10 ? lane : 9;  // entry l: dimer term d = l & 1, J1 count n = l >> 1
    const uint32_t tv = tb[3 + l];
    K.tfull = tv;
    const uint32_t kge = (l & 1) ? K.kge[1] : K.kge[0];  // a select: no runtime index into K
    // tc - 1 with tc = ceil(t / 2^16) >= 2^15 (t >= 2^31: the threshold of |x|), so bit 31 is the sign alone
    K.tabv = (tv >> 16) + ((tv & 0xffffu) != 0u) - 1u + (((uint32_t)(l >> 1) >= kge) ? 0u : 0x80000000u);
    return K;
}

// a[k] and a[k] = v for a runtime k, as bit masks over constant indices: a
// select between array elements would be folded into an indexed load, which
// keeps the whole array in memory (scratch or LDS) instead of registers
template <int N>
__device__ __forceinline__ uint32_t pick(const uint32_t (&a)[N], int k) {
    uint32_t v = 0u;
#pragma unroll
    for (int x = 0; x < N; ++x) v |= a[x] & (0u - (uint32_t)(k == x));
    return v;
}
template <int N>
__device__ __forceinline__ void put(uint32_t (&a)[N], int k, uint32_t v) {
#pragma unroll
    for (int x = 0; x < N; ++x) {
        const uint32_t msk = 0u - (uint32_t)(k == x);
        a[x] = (a[x] & ~msk) | (v & msk);
    }
}

struct Rng {
    uint32_t sweep, chain, k0, k1;
};

// Mask of bits [lo, hi) of a 32-bit word (0 <= lo <= hi <= 32).
__host__ __device__ constexpr uint32_t bits_between(int lo, int hi) {
    return (hi <= lo) ? 0u : ((hi - lo == 32) ? 0xffffffffu : (((1u << (hi - lo)) - 1u) << lo));
}

// Truth tables of the three-input bit operation, written as functions of the
// operand patterns a = 0xF0, b = 0xCC, c = 0xAA.
constexpr int kLutAndNotAnd = 0xF0 & ~0xCC & 0xAA;      // a & ~b & c
constexpr int kLutKeepEqual = 0xF0 & ~(0xCC ^ 0xAA) & 0xFF;  // a & ~(b ^ c)
constexpr int kLutSelectC = ((0xF0 & ~0xAA) | (0xCC & 0xAA)) & 0xFF;  // c ? b : a

// All ones where bit (31 - b) of the wavefront-uniform word x is set.
__device__ __forceinline__ uint32_t plane_mask(uint32_t x, int b) {
    return (uint32_t)((int32_t)(x << b) >> 31);
}

// One plane of the bit-sliced compare: t holds the thresholds' bit of this
// plane for every unit (wavefront-uniform), p the random bits.  Units still
// tied (eq) with random bit 0 against threshold bit 1 fall below it (lt).
__device__ __forceinline__ void compare_plane(uint32_t& lt, uint32_t& eq, uint32_t p, uint32_t t) {
    lt |= __builtin_amdgcn_bitop3_b32(eq, p, t, kLutAndNotAnd);
    eq = __builtin_amdgcn_bitop3_b32(eq, p, t, kLutKeepEqual);
}

// Threshold plane b for 32 units whose dimer-type units are the bits of j2.
__device__ __forceinline__ uint32_t threshold_plane(const SweepK& K, int b, uint32_t j2) {
    return __builtin_amdgcn_bitop3_b32(plane_mask(K.T[0], b), plane_mask(K.T[1], b), j2, kLutSelectC);
}

// First two Philox blocks (planes 0-7) of the bit-sliced comparison U < T
// over 32 packed hidden units.  val: units that exist; ag: agreeing units
// (threshold T1 or T2 by type); j2: units of dimer type.  Leaves in lt the
// units already known to fall below their threshold and in eq those still
// tied.  The threshold plane is uniform over the wavefront: a scalar operand
// of the two bit operations per plane.
__device__ __forceinline__ void hidden_compare_head(uint32_t val, uint32_t ag, uint32_t j2, const SweepK& K,
                                                    uint32_t cb, uint32_t c3, const Rng& rg, uint32_t& lt,
                                                    uint32_t& eq) {
    // only bits of units that exist matter (eq is confined to them)
    const bool only1 = j2 == 0u, only2 = (j2 & val) == val;
    auto tplane = [&](int b) -> uint32_t {
        const uint32_t m0 = plane_mask(K.T[0], b), m1 = plane_mask(K.T[1], b);
        return only1 ? m0 : (only2 ? m1 : (m0 & ~j2) | (m1 & j2));
    };
    P4 p = philox(cb, rg.sweep, rg.chain, c3, rg.k0, rg.k1);
    // plane 0: every threshold has its top bit set (T >= 2^31); disagreeing
    // units (threshold exactly 2^31) are decided here
    lt = val & ~p.v[0];
    eq = ag & p.v[0];
#pragma unroll
    for (int b = 1; b < 4; ++b) compare_plane(lt, eq, p.v[b], tplane(b));
    if (!__any(eq != 0u)) return;
    p = philox(cb | 1u, rg.sweep, rg.chain, c3, rg.k0, rg.k1);
#pragma unroll
    for (int s = 0; s < 4; ++s) compare_plane(lt, eq, p.v[s], tplane(4 + s));
}

// The rest of the comparison (planes 8-31) for the NPW words of one row word
// whose units are still tied.  A unit is tied after 8 planes with probability
// 2^-8, so only about one word in ten has such a unit; continuing every word
// in place would run each further block on all 64 lanes while any lane of the
// wavefront is tied.  Instead the tied words of the wavefront are ranked
// (ballot and prefix count) and moved through this wavefront's 5 x 64 word
// LDS buffer onto consecutive lanes, up to cap at a time, which draw their
// remaining blocks together and hand each word's result back; words ranked
// beyond cap wait for the next round.  cap is 64 in sampling (a test hook
// lowers it to force several rounds); ranks start at 64 - cap, so that the
// test against the buffer's end stays a constant.  Every unit still consumes
// exactly its own planes, in order, so the decisions are those of the full
// 32-bit comparison.  A unit equal to its threshold in all 32
// planes is not below it.
__device__ __forceinline__ void hidden_compare_tail(int NPW, uint32_t (&lt)[5], uint32_t (&eq)[5],
                                                    const uint32_t (&j2)[5], uint32_t cbw, uint32_t cap, const SweepK& K, uint32_t c3, const Rng& rg,
                                                    uint32_t* buf, int lane) {
    const uint32_t first = 64u - cap;  // buffer entries below first stay unused
    uint32_t* const b_eq = buf;
    uint32_t* const b_lt = buf + 64;
    uint32_t* const b_cb = buf + 128;
    uint32_t* const b_ch = buf + 192;
    uint32_t* const b_j2 = buf + 256;
    for (;;) {
        int slot[5] = {-1, -1, -1, -1, -1};
        uint32_t n = first;  // next buffer entry: first + tied words ranked so far (wavefront-uniform)
#pragma unroll
        for (int pw = 0; pw < 5; ++pw) {
            if (pw >= NPW) continue;
            const bool tied = eq[pw] != 0u;
            const uint64_t bal = __ballot(tied);
            const uint32_t r = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)bal, n));
            slot[pw] = (tied && r < 64u) ? (int)r : -1;
            if (slot[pw] >= 0) {
                b_eq[r] = eq[pw];
                b_lt[r] = lt[pw];
                b_cb[r] = cbw | ((uint32_t)pw << 3);
                b_ch[r] = rg.chain;
                b_j2[r] = j2[pw];
            }
            n += (uint32_t)__popcll(bal);
        }
        if (n == first) return;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const bool mine = (uint32_t)lane - first < n - first;  // first <= lane < n
        uint32_t e = 0u, l = 0u, cb = 0u, ch = 0u, jm = 0u;
        if (mine) {
            e = b_eq[lane];
            l = b_lt[lane];
            cb = b_cb[lane];
            ch = b_ch[lane];
            jm = b_j2[lane];
        }
#pragma unroll 1
        for (int c = 2; c < 8; ++c) {
            if (!__any(e != 0u)) break;
            const P4 p = philox(cb | (uint32_t)c, rg.sweep, ch, c3, rg.k0, rg.k1);
#pragma unroll
            for (int s = 0; s < 4; ++s) compare_plane(l, e, p.v[s], threshold_plane(K, 4 * c + s, jm));
        }
        if (mine) b_lt[lane] = l;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int pw = 0; pw < 5; ++pw) {
            if (pw < NPW && slot[pw] >= 0) {
                lt[pw] = b_lt[slot[pw]];
                eq[pw] = 0u;
            }
        }
        if (n <= 64u) return;
    }
}

// Hidden half-step of one cell row i: 10 hidden planes (bits at the cells' even
// columns) from the old spin rows top = 2i, mid = 2i+1, bot = 2i+2.
template <int L>
__device__ __forceinline__ void hidden_row(const uint32_t (&top)[Geo<L>::W], const uint32_t (&mid)[Geo<L>::W],
                                           const uint32_t (&bot)[Geo<L>::W], const SweepK& K, uint32_t i,
                                           uint32_t c3, const Rng& rg, uint32_t* tailbuf, uint32_t tail_cap,
                                           int lane, uint32_t (&H)[10][Geo<L>::W]) {
    using G = Geo<L>;
#pragma unroll
    for (int w = 0; w < G::W; ++w) {
        const int n = G::n(w);
        const uint32_t E = G::even(w);
        const uint32_t t1 = rsh<L, 1>(top, w), t2 = rsh<L, 2>(top, w);
        const uint32_t m1 = rsh<L, 1>(mid, w), m2 = rsh<L, 2>(mid, w);
        const uint32_t b1 = rsh<L, 1>(bot, w);
        // endpoint a and endpoint b of each filter, aligned on the cell's even column
        const uint32_t ea[10] = {top[w], t1, mid[w], m1, top[w], mid[w], t1, m1, top[w], m2};
        const uint32_t eb[10] = {t1, t2, m1, m2, mid[w], bot[w], m1, b1, m1, b1};
        uint32_t A[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            const int ty = k >= 8;
            A[k] = ~(ea[k] ^ eb[k] ^ K.neg[ty]) & K.en[ty] & E;
        }
        // pack: unit u = 2n (k/2) + 2 jl + k%2 -> word u/32, bit u%32
        constexpr int NPWMAX = 5;
        uint32_t PA[NPWMAX] = {0u, 0u, 0u, 0u, 0u};
#pragma unroll
        for (int p = 0; p < 5; ++p) {
            const uint32_t pair = A[2 * p] | (A[2 * p + 1] << 1);
            const int off = 2 * n * p;
            PA[off >> 5] |= pair << (off & 31);
            if ((off & 31) + 2 * n > 32) PA[(off >> 5) + 1] |= pair >> (32 - (off & 31));
        }
        const int NQ = 10 * n;
        const int NPW = (NQ + 31) / 32;
        uint32_t LT[NPWMAX] = {0u, 0u, 0u, 0u, 0u}, EQ[NPWMAX] = {0u, 0u, 0u, 0u, 0u};
        uint32_t J2[NPWMAX] = {0u, 0u, 0u, 0u, 0u}, VAL[NPWMAX] = {0u, 0u, 0u, 0u, 0u};
        const uint32_t cbw = (uint32_t)(i * G::W + w) << 8;
#pragma unroll
        for (int pw = 0; pw < NPWMAX; ++pw) {
            if (pw < NPW) {
                const int lo = 32 * pw;
                VAL[pw] = bits_between(0, (NQ - lo) < 32 ? (NQ - lo) : 32);
                const int j2lo = 8 * n - lo;
                J2[pw] = bits_between(j2lo < 0 ? 0 : (j2lo > 32 ? 32 : j2lo), (NQ - lo) < 32 ? (NQ - lo) : 32);
                hidden_compare_head(VAL[pw], PA[pw], J2[pw], K, cbw | ((uint32_t)pw << 3), c3, rg, LT[pw], EQ[pw]);
            }
        }
        hidden_compare_tail(NPW, LT, EQ, J2, cbw, tail_cap, K, c3, rg, tailbuf, lane);
        uint32_t DP[NPWMAX] = {0u, 0u, 0u, 0u, 0u};  // units at or above their threshold
#pragma unroll
        for (int pw = 0; pw < NPWMAX; ++pw) DP[pw] = VAL[pw] & ~LT[pw];
#pragma unroll
        for (int p = 0; p < 5; ++p) {
            const int off = 2 * n * p;
            uint32_t pair = DP[off >> 5] >> (off & 31);
            if ((off & 31) + 2 * n > 32) pair |= DP[(off >> 5) + 1] << (32 - (off & 31));
            // sign of the field (s_a for agreeing bonds, +1 for a zero field),
            // flipped where the unit went against it.  Only the cells' even
            // columns are meaningful: the other bits are left as they fall,
            // because every consumer of H masks with the even-column mask and
            // column shifts move bits by even amounts.
            H[2 * p][w] = (ea[2 * p] | ~A[2 * p]) ^ pair;
            H[2 * p + 1][w] = (ea[2 * p + 1] | ~A[2 * p + 1]) ^ (pair >> 1);
        }
    }
}

// Minimum of the low 16 bits of three registers (v_min3_u16 reads the low
// halves; only the low half of the result is meaningful).  Written out
// because the compiler packs 16-bit minima into pairs with byte permutes,
// which costs more than the two inputs per instruction this takes.
__device__ __forceinline__ uint32_t min3_u16(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t d;
    asm("v_min3_u16 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

// Visible half-step of the two rows of cell row i (Eq. (12)).  H: hidden
// planes of this cell row; Hp5/Hp7/Hp9: planes 5, 7, 9 of the cell row above.
// Classes: 0 top even, 1 top odd, 2 mid even, 3 mid odd columns.
// A row that is not updated in this call is skipped slot by slot.  When the
// two rows of a cell row are updated in two calls (mid only, later top only),
// the Philox block that holds slots of both rows (word width not a multiple
// of 8) is drawn once: the mid-only call stores it in `straddle`, the
// top-only call reuses it.
template <int L>
__device__ __forceinline__ void visible_row(const uint32_t (&H)[10][Geo<L>::W], const uint32_t (&Hp5)[Geo<L>::W],
                                            const uint32_t (&Hp7)[Geo<L>::W], const uint32_t (&Hp9)[Geo<L>::W],
                                            const SweepK& K, bool do_top, bool do_mid, uint32_t i, uint32_t c3p,
                                            const Rng& rg, uint32_t (&ntop)[Geo<L>::W],
                                            uint32_t (&nmid)[Geo<L>::W], P4 (&straddle)[Geo<L>::W]) {
    using G = Geo<L>;
#pragma unroll
    for (int w = 0; w < G::W; ++w) {
        const int m = G::m(w);
        const uint32_t E = G::even(w);
        const uint32_t n1 = K.neg[0], n2 = K.neg[1];
        const uint32_t h1l = lsh2<L>(H[1], w), h3l = lsh2<L>(H[3], w), h9l = lsh2<L>(H[9], w);
        // the 4 J1 terms and the dimer term of every spin (1 = +1)
        const uint32_t term[4][5] = {
            {H[0][w], H[4][w], h1l ^ n1, Hp5[w] ^ n1, H[8][w]},           // (0,0): k0a k4a k1b(j-1) k5b(i-1) | k8a
            {H[0][w] ^ n1, H[1][w], H[6][w], Hp7[w] ^ n1, Hp9[w] ^ n2},  // (0,1): k0b k1a k6a k7b(i-1) | k9b(i-1)
            {H[2][w], H[4][w] ^ n1, H[5][w], h3l ^ n1, h9l},              // (1,0): k2a k4b k5a k3b(j-1) | k9a(j-1)
            {H[2][w] ^ n1, H[3][w], H[6][w] ^ n1, H[7][w], H[8][w] ^ n2}, // (1,1): k2b k3a k6b k7a | k8b
        };
        uint32_t Pa[4], Pb[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint32_t s1 = term[c][0] ^ term[c][1], c1 = term[c][0] & term[c][1];
            const uint32_t s2 = term[c][2] ^ term[c][3], c2 = term[c][2] & term[c][3];
            const uint32_t b0 = (s1 ^ s2) & E, cc = s1 & s2;
            const uint32_t b1 = (c1 ^ c2 ^ cc) & E, b2 = (c1 & c2) & E;
            const uint32_t dd = term[c][4] & E;
            Pa[c] = dd | (b0 << 1);
            Pb[c] = b1 | (b2 << 1);
        }
        // Byte offsets of the table lookups: byte k of By[4c + j] is 4 idx, with
        // idx = dd + 2 b0 + 4 b1 + 8 b2, of the class-c spin at even column
        // 2 (j + 4k), so that each lookup address is one byte of a register.
        // ds_bpermute reads its source lane from address bits 2-7 only (lane
        // index modulo 64), so By >> 8k is the address of byte k as it stands.
        uint32_t By[16];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint32_t xe = (Pa[c] & 0x33333333u) | ((Pb[c] & 0x33333333u) << 2);  // columns 4u
            const uint32_t xo = ((Pa[c] >> 2) & 0x33333333u) | (Pb[c] & 0xccccccccu);  // columns 4u + 2
            By[4 * c + 0] = (xe & 0x0f0f0f0fu) << 2;
            By[4 * c + 1] = (xo & 0x0f0f0f0fu) << 2;
            By[4 * c + 2] = (xe >> 2) & 0x3c3c3c3cu;
            By[4 * c + 3] = (xo >> 2) & 0x3c3c3c3cu;
        }
        const int NQ = 2 * m;
        const int NB = (NQ + 7) / 8;
        const uint32_t cbase = (uint32_t)(i * G::W + w) << 5;
        // NS[row]: bit c = the new spin at column c (1 = up), shifted in from
        // the highest column down: slots are taken from the last block and the
        // last slot backwards, so each row's spins arrive in descending column
        // order
        uint32_t NS[2] = {0u, 0u};
        uint32_t tieblk = 0u;
#pragma unroll
        for (int blk = 7; blk >= 0; --blk) {
            if (blk >= NB) continue;
            const bool has_top = blk * 8 < m, has_mid = blk * 8 + 7 >= m;
            if (!((do_top && has_top) || (do_mid && has_mid))) continue;
            const bool shared = has_top && has_mid;  // the straddling block (m % 8 != 0)
            P4 p;
            if (shared && do_top && !do_mid) {
                p = straddle[w];
            } else {
                p = philox(cbase | (uint32_t)blk, rg.sweep, rg.chain, c3p, rg.k0, rg.k1);
                if (shared && do_mid && !do_top) straddle[w] = p;
            }
            // r of each slot (0xffff where a slot is absent or its row not
            // updated): a tie is a zero low half, found by a 16-bit minimum
            // over the block, two slots per instruction
            uint32_t rv[8];
#pragma unroll
            for (int s = 0; s < 8; ++s) rv[s] = 0xffffu;
#pragma unroll
            for (int s = 7; s >= 0; --s) {
                const int q = blk * 8 + s;
                if (q < NQ) {
                    const int row = q / m, col = q % m, cls = 2 * row + (col & 1);
                    if (!(row == 0 ? do_top : do_mid)) continue;
                    const int si = col >> 1;
                    const uint32_t addr = By[4 * cls + (si & 3)] >> (8 * (si >> 2));
                    const uint32_t v = (uint32_t)__builtin_amdgcn_ds_bpermute((int)addr, (int)K.tabv);
                    const uint32_t r = slot16(p, s) - v;  // sign bit: the new spin
                    NS[row] = __builtin_amdgcn_alignbit(NS[row], r, 31);
                    rv[s] = r;
                }
            }
            const int ns = NQ - blk * 8 < 8 ? NQ - blk * 8 : 8;  // slots of this block (compile time)
            uint32_t low = ns > 1 ? min3_u16(rv[ns - 1], rv[ns - 1], rv[ns - 2]) : rv[0];
#pragma unroll
            for (int s = ns - 3; s >= 0; s -= 2) low = min3_u16(low, rv[s], rv[s > 0 ? s - 1 : 0]);
            if (__ballot((uint16_t)low == 0u)) tieblk |= 1u << blk;
        }
        // Rare path: a primary slot P = tc - 1; redo the affected blocks with
        // the refinement stream and exact 32-bit compares (the new spin is
        // U < t for a field >= 0, U >= t for a negative one).
        while (tieblk) {
            const int blk = __builtin_ctz(tieblk);
            tieblk &= tieblk - 1u;
            const P4 p = philox(cbase | (uint32_t)blk, rg.sweep, rg.chain, c3p, rg.k0, rg.k1);
            const P4 r = philox(cbase | (uint32_t)blk, rg.sweep, rg.chain, c3p + 1u, rg.k0, rg.k1);
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int q = blk * 8 + s;
                if (q < NQ) {
                    const int row = q / m, col = q % m, cls = 2 * row + (col & 1);
                    if (!(row == 0 ? do_top : do_mid)) continue;
                    const uint32_t U = (slot16(p, s) << 16) | slot16(r, s);
                    const int si = col >> 1;
                    const int addr = (int)(pick(By, 4 * cls + (si & 3)) >> (8 * (si >> 2)));
                    const uint32_t t = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)K.tfull);
                    const uint32_t neg = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)K.tabv) >> 31;
                    const uint32_t bit = 1u << col, f = ((U < t) ^ neg) ? bit : 0u;
                    if (row == 0)
                        NS[0] = (NS[0] & ~bit) | f;
                    else
                        NS[1] = (NS[1] & ~bit) | f;
                }
            }
        }
        ntop[w] = NS[0] & G::full(w);
        nmid[w] = NS[1] & G::full(w);
    }
}

// One work item: up to 64/G chains of one instance, all sweeps [s0, s1).
// CAP: the tail takes a.tail_cap words per round (else the constant 64).
template <int L, int R, bool CAP>
__device__ __forceinline__ void gibbs_item(const GibbsArgs& a, const Item& it, int lane, uint32_t* tailbuf) {
    using Gm = Geo<L>;
    constexpr int W = Gm::W;
    constexpr int C = L / 2;
    constexpr int G = C / R;
    constexpr int NR = 2 * R;
    constexpr int N = L * L;
    static_assert(C % R == 0, "R must divide L/2");
    static_assert(G <= 64, "a chain must fit in one wavefront");

    const int cl = lane / G, g = lane - cl * G;
    const bool active = cl < (int)it.nchains;
    const uint32_t chain = it.chain0 + (active ? (uint32_t)cl : 0u);
    const uint64_t gch = it.gbase + (active ? (uint64_t)cl : 0u);
    const int nxt = cl * G + (g + 1 == G ? 0 : g + 1);
    const int prv = cl * G + (g == 0 ? G - 1 : g - 1);

    uint32_t Q[NR + 1][W];
    {
        const uint32_t* st = a.state + it.state_off + ((uint64_t)(active ? cl : 0) * L + (uint64_t)g * NR) * W;
#pragma unroll
        for (int x = 0; x < NR; ++x)
#pragma unroll
            for (int w = 0; w < W; ++w) Q[x][w] = st[x * W + w];
#pragma unroll
        for (int w = 0; w < W; ++w) Q[NR][w] = 0u;
    }
    const uint32_t c3h = (it.id << 3) | 1u, c3v = (it.id << 3) | 3u;
    // The item's table base and stride, read once into scalar registers: the
    // loop's stores could alias the item in memory, so the compiler would
    // otherwise reload it every sweep and form the address per lane.
    // readfirstlane returns a signed int: widen each half through uint32_t.
    const uint64_t toff = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(it.tab_off >> 32)) << 32) |
                          (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)it.tab_off);
    const uint32_t tstride = (uint32_t)__builtin_amdgcn_readfirstlane((int)it.tab_stride);
    const uint32_t* const tb0 = a.tables + toff;

    for (int64_t s = a.s0; s < a.s1; ++s) {
        const uint32_t* tb = tb0 + (uint64_t)tstride * (uint64_t)s;
        const SweepK K = load_sweep(tb, lane);
        const Rng rg{(uint32_t)s, chain, (uint32_t)a.seed, (uint32_t)(a.seed >> 32)};
#pragma unroll
        for (int w = 0; w < W; ++w) Q[NR][w] = __shfl(Q[0][w], nxt);  // old first row of the next band
        uint32_t Hf0[W], Hf1[W], Hf4[W], Hf6[W], Hf8[W], Hp5[W], Hp7[W], Hp9[W];
        P4 straddle[W];  // Philox block shared by the two rows of the band's first cell row
#pragma unroll
        for (int w = 0; w < W; ++w) {
            Hf0[w] = Hf1[w] = Hf4[w] = Hf6[w] = Hf8[w] = 0u;
            Hp5[w] = Hp7[w] = Hp9[w] = 0u;
        }
#pragma unroll 1
        for (int m = 0; m < R; ++m) {
            const uint32_t i = (uint32_t)(g * R + m);
            uint32_t H[10][W];
            hidden_row<L>(Q[0], Q[1], Q[2], K, i, c3h, rg, tailbuf, CAP ? a.tail_cap : 64u, lane, H);
            uint32_t nt[W], nm[W];
            visible_row<L>(H, Hp5, Hp7, Hp9, K, m > 0, true, i, c3v, rg, nt, nm, straddle);
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const uint32_t old_top = Q[0][w];
#pragma unroll
                for (int x = 0; x + 2 <= NR; ++x) Q[x][w] = Q[x + 2][w];
                Q[NR - 1][w] = (m == 0) ? old_top : nt[w];
                Q[NR][w] = nm[w];
                if (m == 0) {
                    Hf0[w] = H[0][w]; Hf1[w] = H[1][w]; Hf4[w] = H[4][w]; Hf6[w] = H[6][w]; Hf8[w] = H[8][w];
                }
                Hp5[w] = H[5][w]; Hp7[w] = H[7][w]; Hp9[w] = H[9][w];
            }
        }
        // first row of the band: needs the last hidden row of the band above
#pragma unroll
        for (int w = 0; w < W; ++w) {
            Hp5[w] = __shfl(Hp5[w], prv);
            Hp7[w] = __shfl(Hp7[w], prv);
            Hp9[w] = __shfl(Hp9[w], prv);
        }
        {
            uint32_t Hd[10][W];
#pragma unroll
            for (int w = 0; w < W; ++w) {
                Hd[0][w] = Hf0[w]; Hd[1][w] = Hf1[w]; Hd[4][w] = Hf4[w]; Hd[6][w] = Hf6[w]; Hd[8][w] = Hf8[w];
                Hd[2][w] = Hd[3][w] = Hd[5][w] = Hd[7][w] = Hd[9][w] = 0u;
            }
            uint32_t nt[W], nm[W];
            visible_row<L>(Hd, Hp5, Hp7, Hp9, K, true, false, (uint32_t)(g * R), c3v, rg, nt, nm, straddle);
#pragma unroll
            for (int w = 0; w < W; ++w) Q[1][w] = nt[w];
        }
#pragma unroll
        for (int x = 0; x < NR; ++x)
#pragma unroll
            for (int w = 0; w < W; ++w) Q[x][w] = Q[x + 1][w];

        const bool meas = a.measure_every > 0 && s >= a.burn_in && ((s - a.burn_in) % a.measure_every) == 0;
        const bool rec = a.trace != nullptr && ((s - a.trace_s0 + 1) % a.trace_every) == 0;
        if (meas || rec) {
            uint32_t nb[W];
#pragma unroll
            for (int w = 0; w < W; ++w) nb[w] = __shfl(Q[0][w], nxt);  // new first row of the next band
            int pop = 0, dis1 = 0, dis2 = 0;
#pragma unroll
            for (int x = 0; x < NR; ++x)
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const uint32_t below = (x + 1 < NR) ? Q[x + 1][w] : nb[w];
                    pop += __popc(Q[x][w]);
                    dis1 += __popc(Q[x][w] ^ rsh<L, 1>(Q[x], w)) + __popc(Q[x][w] ^ below);
                }
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const uint32_t(&tp)[W] = Q[2 * m];
                const uint32_t(&md)[W] = Q[2 * m + 1];
                const uint32_t(&bt)[W] = (2 * m + 2 < NR) ? Q[2 * m + 2] : nb;
#pragma unroll
                for (int w = 0; w < W; ++w)
                    dis2 += __popc((tp[w] ^ rsh<L, 1>(md, w)) & Gm::even(w)) +
                            __popc((rsh<L, 2>(md, w) ^ rsh<L, 1>(bt, w)) & Gm::even(w));
            }
            // staggered magnetisation sum (-1)^(r+c) s = sum over rows of (-1)^r 2 (up at even
            // columns - up at odd columns) (L even: as many even as odd columns)
            int stag = 0;
            if (meas) {
#pragma unroll
                for (int x = 0; x < NR; ++x) {
                    int pe = 0, po = 0;
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        pe += __popc(Q[x][w] & Gm::even(w));
                        po += __popc(Q[x][w] & ~Gm::even(w) & Gm::full(w));
                    }
                    stag += (x & 1) ? 2 * (po - pe) : 2 * (pe - po);  // band rows start at an even row
                }
            }
            // plateau structure factor sums: A_k = sum (-1)^r s over columns = k (mod 3),
            // B_k = sum (-1)^c s over rows = k (mod 3)
            const bool want_order = rec && a.order != nullptr;
            int oa[3] = {0, 0, 0}, ob[3] = {0, 0, 0};
            if (want_order) {
#pragma unroll
                for (int x = 0; x < NR; ++x) {
                    const int row = g * NR + x;
                    int pk[3] = {0, 0, 0}, pe = 0, po = 0;
#pragma unroll
                    for (int w = 0; w < W; ++w) {
#pragma unroll
                        for (int k = 0; k < 3; ++k) pk[k] += __popc(Q[x][w] & Gm::mod3(w, k));
                        pe += __popc(Q[x][w] & Gm::even(w));
                        po += __popc(Q[x][w] & ~Gm::even(w) & Gm::full(w));
                    }
                    const int sg = (row & 1) ? -1 : 1;
#pragma unroll
                    for (int k = 0; k < 3; ++k) oa[k] += sg * (2 * pk[k] - Gm::cnt3(k));
                    const int rm = row % 3, e = 2 * (pe - po);
                    ob[0] += (rm == 0) ? e : 0;
                    ob[1] += (rm == 1) ? e : 0;
                    ob[2] += (rm == 2) ? e : 0;
                }
            }
            int tp = pop, t1 = dis1, t2 = dis2, ts = stag;
            int sa3[3] = {oa[0], oa[1], oa[2]}, sb3[3] = {ob[0], ob[1], ob[2]};  // chain totals
            if (want_order) {
#pragma unroll
                for (int d = 1; d < G; ++d) {
                    const int src = cl * G + (g + d) % G;
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        sa3[k] += __shfl(oa[k], src);  // the other lanes' own partial sums
                        sb3[k] += __shfl(ob[k], src);
                    }
                }
            }
#pragma unroll
            for (int d = 1; d < G; ++d) {
                const int src = cl * G + (g + d) % G;
                tp += __shfl(pop, src);
                t1 += __shfl(dis1, src);
                t2 += __shfl(dis2, src);
                if (meas) ts += __shfl(stag, src);
            }
            const int64_t M = 2 * tp - N, B1 = 2 * N - 2 * t1, B2 = N / 2 - 2 * t2;
            if (rec && g == 0 && active) {
                const uint64_t rix = ((uint64_t)((s - a.trace_s0) / a.trace_every) * (uint64_t)a.total_chains + gch) * 3;
                int32_t* tr = a.trace + rix;
                tr[0] = (int32_t)M;
                tr[1] = (int32_t)B1;
                tr[2] = (int32_t)B2;
                if (want_order) {
                    // |A0 + A1 w + A2 w^2|^2 with w = exp(2 pi i / 3)
                    auto sq3 = [](const int (&v)[3]) {
                        const int64_t x = v[0], y = v[1], z = v[2];
                        return x * x + y * y + z * z - x * y - y * z - z * x;
                    };
                    const int64_t sa = sq3(sa3), sb = sq3(sb3);
                    int32_t* od = a.order + rix;
                    od[0] = (int32_t)(sa > sb ? sa : sb);
                    od[1] = (int32_t)sa;
                    od[2] = (int32_t)sb;
                }
            }
            if (meas && g == 0 && active) {  // the chain's accumulators live in memory: no registers held
                int64_t* ac = a.acc + gch * CRBM_N_ACC;
                const int64_t Ms = ts;
                ac[0] += 1;
                ac[1] += M; ac[2] += B1; ac[3] += B2;
                ac[4] += M * M; ac[5] += B1 * B1; ac[6] += B2 * B2;
                ac[7] += M * B1; ac[8] += M * B2; ac[9] += B1 * B2;
                ac[10] += M < 0 ? -M : M;
                ac[11] += Ms; ac[12] += Ms * Ms; ac[13] += Ms < 0 ? -Ms : Ms;
            }
        }
    }
    if (!active) return;  // returns from this item only
    {
        uint32_t* st = a.state + it.state_off + ((uint64_t)cl * L + (uint64_t)g * NR) * W;
#pragma unroll
        for (int x = 0; x < NR; ++x)
#pragma unroll
            for (int w = 0; w < W; ++w) st[x * W + w] = Q[x][w];
    }
    if (a.spins_out) {
        int8_t* out = a.spins_out + it.spin_off + ((uint64_t)cl * L + (uint64_t)g * NR) * L;
        for (int x = 0; x < NR; ++x)
            for (int c = 0; c < L; ++c) out[x * L + c] = ((Q[x][c >> 5] >> (c & 31)) & 1u) ? 1 : -1;
    }
}

// Direct mode: wavefront w of the grid takes item w.  Persistent mode
// (a.queue != nullptr): each wavefront pops items from a device counter until
// the list is exhausted, so a grid sized to the machine drains any number of
// items and concurrent kernels share the CUs as their queues empty.
// Rows of three words (L > 64) would otherwise take more than 256 registers
// per lane and one wavefront per SIMD; asking for two trades a few spilled
// values for the latency hiding of a second wavefront (measured: 96x96 runs
// 1.6x faster, 72x72 1.5x).
template <int L, int R, bool CAP>
__global__ void __launch_bounds__(256, (Geo<L>::W >= 3 ? 2 : 1)) gibbs_kernel(GibbsArgs a) {
    const int lane = threadIdx.x & 63;
    // per wavefront: the tied hidden words of the comparison's tail (5 x 64 words)
    __shared__ uint32_t tail_lds[4][5 * 64];
    uint32_t* const tailbuf = tail_lds[threadIdx.x >> 6];
    if (a.queue == nullptr) {
        const int wv = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
        if (wv >= a.n_items) return;
        gibbs_item<L, R, CAP>(a, a.items[wv], lane, tailbuf);
        return;
    }
    for (;;) {
        uint32_t next = 0u;
        if (lane == 0) next = atomicAdd(a.queue, 1u);
        next = __builtin_amdgcn_readfirstlane(next);
        if (next >= (uint32_t)a.n_items) return;
        gibbs_item<L, R, CAP>(a, a.items[next], lane, tailbuf);
    }
}

template <int L, int R>
hipError_t launch_tile(const GibbsArgs& a, hipStream_t st) {
    const int wpb = a.waves_per_block > 0 ? a.waves_per_block : 4;
    int blocks = (a.n_items + wpb - 1) / wpb;
    if (a.queue != nullptr && a.grid_blocks > 0 && a.grid_blocks < blocks) blocks = a.grid_blocks;
    if (blocks == 0) return hipSuccess;
    if (a.tail_cap < 64u)
        hipLaunchKernelGGL((gibbs_kernel<L, R, true>), dim3(blocks), dim3(64 * wpb), 0, st, a);
    else
        hipLaunchKernelGGL((gibbs_kernel<L, R, false>), dim3(blocks), dim3(64 * wpb), 0, st, a);
    return hipGetLastError();
}

// Kernel function pointer, for explicit graph nodes (the variant that the
// current tail cap selects).
template <int L, int R>
const void* kernel_ptr() {
    if (tail_cap() < 64u) return reinterpret_cast<const void*>(&gibbs_kernel<L, R, true>);
    return reinterpret_cast<const void*>(&gibbs_kernel<L, R, false>);
}

}  // namespace gk
}  // namespace crbmlib
