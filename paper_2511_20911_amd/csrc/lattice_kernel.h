// lattice_kernel.h -- gfx950 device code of block Gibbs sampling of the CRBM
// on general lattices (Brahma et al., arXiv 2511.20911, Sec. II.A-II.B,
// III.A; App. A Wrapper Module, Zero Padder, Convoluter-Reverse,
// Accumulator): Lr x Lc spins, each axis periodic or open, one coupling per
// filter, separate visible biases on even and odd columns.  Same arithmetic
// and random-number conventions as the square-lattice sampler, so a periodic
// square SS lattice gives the same trajectories in both.
//
// Reading of the open boundary: a bond whose endpoint would lie past the last
// row (column) of an open axis does not exist.  Its hidden unit is not drawn
// and no field reaches its remaining spin.
//
// Mapping: one lane per chain, 64 chains of one instance per wavefront (one
// wavefront per workgroup).  The kernel is compiled for each even column
// count Lc (a template argument: every bit position is a compile-time
// constant, as in the square-lattice kernel); the row count and the open or
// periodic axes are runtime values, uniform over the wavefront.  A chain's bit
// rows (W = ceil(Lc/32) words) live in LDS for the whole launch,
// lane-interleaved ([row][word][lane]: every access of a wavefront hits 64
// consecutive words), because the row loop runs at run time.
//
// Per sweep and cell row i (rows 2i, 2i+1): the 10 hidden planes of the cell
// row from the old spins (bit-sliced compare against per-filter thresholds,
// with the tied words compacted across the wavefront after two Philox
// blocks, as in the square-lattice sampler), then the new spins of rows 2i+1
// and (for i > 0) 2i; row 0 is updated last, after the last cell row's hidden
// units (which read the old row 0 on a periodic axis).  A spin's threshold
// and field sign come from a 512-entry table by (sublattice class, edge
// flags, 5-bit pattern of its incident hidden units); absent terms are zero
// bits of the pattern and the table entry of that edge type leaves them out.
// Each class's patterns are regrouped once per row word into bytes that hold
// the entry's LDS byte offset (4 x pattern, plus 128 on an open row edge), so
// a spin's lookup address is one byte of a register.
#pragma once
#include "crbm.h"
#include "crbm_internal.h"
#include "gibbs_kernel.h"

namespace crbmlib {
namespace lat {

using gk::P4;
using gk::philox;

// Per-sweep table of one instance (words), as the host builds it:
//   [0..9]    agree threshold t(2 wq_k) of filter k (2^31 if wq_k == 0)
//   [10]      bit k: sig_k < 0;  [11] bit k: wq_k != 0;  [12..15] zero
//   [16 + e]  visible entry e (e = type * 32 + pattern, type = (cls * 2 + row edge) * 2 + column edge):
//             min(tceil16, 0xffff) | thi16 << 16
//   [528 + e] full 32-bit threshold of entry e
//   [1040 + e / 32] bit e % 32: the field of entry e is >= 0
constexpr int kHead = 16;
constexpr int kEntries = 512;
constexpr int kLatTabWords = kHead + 2 * kEntries + kEntries / 32;

struct LatItem {
    uint32_t id;          // random-number id of the instance
    uint32_t chain0;      // first chain (within the instance)
    uint32_t nchains;     // <= 64
    uint32_t tab_stride;  // kLatTabWords, or 0 for a constant schedule
    uint64_t gbase;       // global index of chain0
    uint64_t state_off;   // word offset of chain0's rows ([chain][Lr][W])
    uint64_t spin_off;    // byte offset of chain0's int8 spins ([chain][Lr][Lc])
    uint64_t tab_off;     // word offset of the instance's first table
    int64_t corr_off;     // offset of the instance's Cn sums, or -1
    int32_t Lr, Lc, open_r, open_c;
    int32_t np[10];       // present bonds of each filter
};

struct LatArgs {
    uint32_t* state;
    const uint32_t* tables;
    const LatItem* items;
    int32_t n_items;
    int32_t measure_every;
    int64_t s0, s1, burn_in;
    uint64_t seed;
    int64_t* acc;               // [global chain][CRBM_LAT_N_ACC]
    int32_t* trace;             // [(s1 - trace_s0) / trace_every][total_chains][12] or nullptr
    int32_t trace_every;
    int64_t trace_s0;
    int64_t total_chains;
    int8_t* spins_out;
    unsigned long long* corr;   // Cn sums of every instance, or nullptr
    uint32_t tail_cap;          // lanes per round of the hidden comparison's compacted tail (1..64)
};

// Visible terms of each sublattice class (0: even row even col, 1: even row
// odd col, 2: odd row even col, 3: odd row odd col) and which of them vanish
// at a row edge (class 0, 1: row 0; class 2, 3: the last row) or a column edge
// (class 0, 2: column 0; class 1, 3: the last column) of an open axis.
//   0: k0a k4a k1b(j-1) k5b(i-1) k8a      1: k0b k1a k6a k7b(i-1) k9b(i-1)
//   2: k2a k4b k5a k3b(j-1) k9a(j-1)      3: k2b k3a k6b k7a k8b
__host__ __device__ constexpr int term_filter(int cls, int t) {
    return cls == 0 ? (t == 0 ? 0 : t == 1 ? 4 : t == 2 ? 1 : t == 3 ? 5 : 8)
         : cls == 1 ? (t == 0 ? 0 : t == 1 ? 1 : t == 2 ? 6 : t == 3 ? 7 : 9)
         : cls == 2 ? (t == 0 ? 2 : t == 1 ? 4 : t == 2 ? 5 : t == 3 ? 3 : 9)
                    : (t == 0 ? 2 : t == 1 ? 3 : t == 2 ? 6 : t == 3 ? 7 : 8);
}
// endpoint b of its bond (the coupling sign applies)
__host__ __device__ constexpr bool term_is_b(int cls, int t) {
    return cls == 0 ? (t == 2 || t == 3)
         : cls == 1 ? (t == 0 || t == 3 || t == 4)
         : cls == 2 ? (t == 1 || t == 3)
                    : (t == 0 || t == 2 || t == 4);
}
__host__ __device__ constexpr uint32_t row_edge_terms(int cls) {
    return cls == 0 ? 0x08u : cls == 1 ? 0x18u : cls == 2 ? 0x14u : 0x08u;
}
__host__ __device__ constexpr uint32_t col_edge_terms(int cls) {
    return cls == 0 ? 0x04u : cls == 1 ? 0x12u : cls == 2 ? 0x18u : 0x02u;
}

// LDS of a workgroup (words; small enough that 16 workgroups of an 18 x 18
// lattice fit a compute unit, as many as its registers allow):
//   [kVis, +512)       visible entry of kernel index x = ((cls * 2 + column edge) * 2 + row edge) * 32
//                      + pattern: ceil(t / 2^16), plus 2^31 where the entry's field is negative
//   [kTail, +256)      tied hidden words of the comparison's tail (4 x 64)
//   [kPlanes, +160 W)  threshold planes of the hidden words, [w][pw][b] (5 words pw of 32 planes b
//                      per row word w), from the sweep's filter thresholds
//   [spins(W), ...)    bit rows [Lr][W][64]
// The full thresholds, needed only by the rare exact path, stay in the global table.
constexpr int kVis = 0, kTail = 512, kPlanes = 768;
__host__ __device__ constexpr int lat_spins_word(int W) { return kPlanes + 160 * W; }
__host__ __device__ constexpr int lat_lds_bytes(int Lr, int W) { return (lat_spins_word(W) + Lr * W * 64) * 4; }

template <int LC>
struct LGeo {
    static constexpr int W = (LC + 31) / 32;
    static constexpr int ML = LC - 32 * (W - 1);  // columns in the last word
    __host__ __device__ static constexpr int m(int w) { return w == W - 1 ? ML : 32; }
    __host__ __device__ static constexpr int n(int w) { return m(w) / 2; }
    __host__ __device__ static constexpr uint32_t full(int w) {
        return m(w) == 32 ? 0xffffffffu : ((1u << m(w)) - 1u);
    }
    __host__ __device__ static constexpr uint32_t even(int w) { return 0x55555555u & full(w); }
    // even-column bit of the last cell, in the last word (a column-edge site of classes 1, 3)
    __host__ __device__ static constexpr uint32_t last_cell(int w) { return w == W - 1 ? (1u << (ML - 2)) : 0u; }
};

// bit c of word w <- column 32w + c + S (S = 1, 2); past the last column the
// first columns on a periodic axis, zero on an open one
template <int LC, int S>
__device__ __forceinline__ uint32_t rsh(const uint32_t (&x)[LGeo<LC>::W], int w, bool open_c) {
    using G = LGeo<LC>;
    if (w < G::W - 1) return (x[w] >> S) | (x[w + 1] << (32 - S));
    const uint32_t wrap = open_c ? 0u : (x[0] & ((1u << S) - 1u));
    return ((x[w] >> S) | (wrap << (G::ML - S))) & G::full(w);
}
// bit c of word w <- column 32w + c - 2 (the last columns on a periodic axis)
template <int LC>
__device__ __forceinline__ uint32_t lsh2(const uint32_t (&x)[LGeo<LC>::W], int w, bool open_c) {
    using G = LGeo<LC>;
    if (w > 0) return ((x[w] << 2) | (x[w - 1] >> 30)) & G::full(w);
    const uint32_t top = open_c ? 0u : ((x[G::W - 1] >> (G::ML - 2)) & 3u);
    return ((x[0] << 2) | top) & G::full(0);
}

struct LSweep {
    uint32_t neg[10];  // all ones if sig_k < 0
    uint32_t en[10];   // all ones if wq_k != 0
};

// Threshold plane b of hidden word pw of a row word with n cells: units
// 32 pw .. 32 pw + 31; unit u belongs to filter 2 (u div 2n) + (u mod 2).
// T: the ten filter thresholds.  Built once per table into LDS (kPlanes).
__device__ __forceinline__ uint32_t filter_plane(const uint32_t* T, int n, int pw, int b) {
    uint32_t t = 0u;
#pragma unroll
    for (int p = 0; p < 5; ++p) {
        const int lo = 2 * n * p - 32 * pw, hi = 2 * n * (p + 1) - 32 * pw;
        if (hi <= 0 || lo >= 32) continue;
        const uint32_t run = gk::bits_between(lo < 0 ? 0 : lo, hi > 32 ? 32 : hi);
        t |= run & ((gk::plane_mask(T[2 * p], b) & 0x55555555u) | (gk::plane_mask(T[2 * p + 1], b) & 0xAAAAAAAAu));
    }
    return t;
}

// First two Philox blocks (planes 0-7) of the comparison U < t over the 32
// units of hidden word pw: val, units that exist; ag, agreeing units.  Every
// threshold has its top bit set (t >= 2^31), so plane 0 decides the units of
// threshold exactly 2^31 (disagreeing bonds, zero fields).
// pl: the word's 32 threshold planes in LDS (the same for every lane).
__device__ __forceinline__ void hidden_head(uint32_t val, uint32_t ag, const uint32_t* pl, uint32_t cb, uint32_t c3,
                                            uint32_t sweep, uint32_t chain, uint32_t k0, uint32_t k1, uint32_t& lt,
                                            uint32_t& eq) {
    P4 p = philox(cb, sweep, chain, c3, k0, k1);
    lt = val & ~p.v[0];
    eq = ag & p.v[0];
    const uint4 t0 = *reinterpret_cast<const uint4*>(pl);
    gk::compare_plane(lt, eq, p.v[1], t0.y);
    gk::compare_plane(lt, eq, p.v[2], t0.z);
    gk::compare_plane(lt, eq, p.v[3], t0.w);
    if (!__any(eq != 0u)) return;
    p = philox(cb | 1u, sweep, chain, c3, k0, k1);
    const uint4 t1 = *reinterpret_cast<const uint4*>(pl + 4);
    gk::compare_plane(lt, eq, p.v[0], t1.x);
    gk::compare_plane(lt, eq, p.v[1], t1.y);
    gk::compare_plane(lt, eq, p.v[2], t1.z);
    gk::compare_plane(lt, eq, p.v[3], t1.w);
}

// The rest of the comparison (planes 8-31) for the NPW hidden words of one
// row word whose units are still tied: the tied words of the wavefront are
// ranked (ballot and prefix count) and moved through this wavefront's 4 x 64
// word LDS buffer onto consecutive lanes, up to cap at a time, which draw
// their remaining blocks together and hand each word's result back; words
// ranked beyond cap wait for the next round.  cap is 64 in sampling (a test
// hook lowers it to force several rounds); ranks start at 64 - cap, so that
// the test against the buffer's end stays a constant.  Each unit
// consumes exactly its own planes, in order, so the decisions are those of
// the full 32-bit comparison; a unit equal to its threshold in all 32 planes
// is not below it.  A compacted lane reads the threshold planes of its own
// word from LDS (planes: the row word's [pw][32] planes).
__device__ __forceinline__ void hidden_tail(int NPW, uint32_t (&lt)[5], uint32_t (&eq)[5], uint32_t cbw,
                                            uint32_t cap, const uint32_t* planes, uint32_t c3, uint32_t sweep,
                                            uint32_t chain, uint32_t k0, uint32_t k1, uint32_t* buf, int lane) {
    const uint32_t first = 64u - cap;  // buffer entries below first stay unused
    uint32_t* const b_eq = buf;
    uint32_t* const b_lt = buf + 64;
    uint32_t* const b_cb = buf + 128;
    uint32_t* const b_ch = buf + 192;
    for (;;) {
        int slot[5] = {-1, -1, -1, -1, -1};
        uint32_t cnt = first;  // next buffer entry: first + tied words ranked so far (wavefront-uniform)
#pragma unroll
        for (int pw = 0; pw < 5; ++pw) {
            if (pw >= NPW) continue;
            const bool tied = eq[pw] != 0u;
            const uint64_t bal = __ballot(tied);
            const uint32_t r = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)bal, cnt));
            slot[pw] = (tied && r < 64u) ? (int)r : -1;
            if (slot[pw] >= 0) {
                b_eq[r] = eq[pw];
                b_lt[r] = lt[pw];
                b_cb[r] = cbw | ((uint32_t)pw << 3);
                b_ch[r] = chain;
            }
            cnt += (uint32_t)__popcll(bal);
        }
        if (cnt == first) return;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const bool mine = (uint32_t)lane - first < cnt - first;  // first <= lane < cnt
        uint32_t e = 0u, l = 0u, cb = 0u, ch = 0u;
        if (mine) {
            e = b_eq[lane];
            l = b_lt[lane];
            cb = b_cb[lane];
            ch = b_ch[lane];
        }
        const uint32_t* const wpl = planes + 32 * ((cb >> 3) & 7u);
#pragma unroll 1
        for (int c = 2; c < 8; ++c) {
            if (!__any(e != 0u)) break;
            const P4 p = philox(cb | (uint32_t)c, sweep, ch, c3, k0, k1);
            const uint4 t = *reinterpret_cast<const uint4*>(wpl + 4 * c);
            gk::compare_plane(l, e, p.v[0], t.x);
            gk::compare_plane(l, e, p.v[1], t.y);
            gk::compare_plane(l, e, p.v[2], t.z);
            gk::compare_plane(l, e, p.v[3], t.w);
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
        if (cnt <= 64u) return;
    }
}

// Hidden half-step of cell row i: H[k][w] holds the unit of bond k of every
// cell at the cell's even column (other bits undefined: every consumer masks
// with the even-column mask, and column shifts move bits by even amounts).
template <int LC>
__device__ __forceinline__ void hidden_row(const uint32_t (&top)[LGeo<LC>::W], const uint32_t (&mid)[LGeo<LC>::W],
                                           const uint32_t (&bot)[LGeo<LC>::W], bool open_c, bool last_row_open,
                                           const LSweep& K, const uint32_t* planes, int i, uint32_t c3,
                                           uint32_t sweep, uint32_t chain, uint32_t k0, uint32_t k1,
                                           uint32_t* tailbuf, uint32_t tail_cap, int lane,
                                           uint32_t (&H)[10][LGeo<LC>::W]) {
    using G = LGeo<LC>;
#pragma unroll
    for (int w = 0; w < G::W; ++w) {
        const int n = G::n(w);
        const uint32_t E = G::even(w);
        const uint32_t t1 = rsh<LC, 1>(top, w, open_c), t2 = rsh<LC, 2>(top, w, open_c);
        const uint32_t m1 = rsh<LC, 1>(mid, w, open_c), m2 = rsh<LC, 2>(mid, w, open_c);
        const uint32_t b1 = rsh<LC, 1>(bot, w, open_c);
        const uint32_t ea[10] = {top[w], t1, mid[w], m1, top[w], mid[w], t1, m1, top[w], m2};
        const uint32_t eb[10] = {t1, t2, m1, m2, mid[w], bot[w], m1, b1, m1, b1};
        // bonds present at this cell row: k1, k3, k9 lose the last cell on an open
        // column axis; k5, k7, k9 lose the last cell row on an open row axis
        const uint32_t pc = open_c ? ~G::last_cell(w) : 0xffffffffu;
        const uint32_t pr = last_row_open ? 0u : 0xffffffffu;
        uint32_t P[10], A[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            uint32_t pm = E;
            if (k == 1 || k == 3 || k == 9) pm &= pc;
            if (k == 5 || k == 7 || k == 9) pm &= pr;
            P[k] = pm;
            A[k] = ~(ea[k] ^ eb[k] ^ K.neg[k]) & K.en[k] & pm;
        }
        // pack: unit u = 2n (k/2) + 2 jl + k%2 -> word u/32, bit u%32
        uint32_t PA[5] = {0u, 0u, 0u, 0u, 0u}, PP[5] = {0u, 0u, 0u, 0u, 0u};
#pragma unroll
        for (int p = 0; p < 5; ++p) {
            const uint32_t pa = A[2 * p] | (A[2 * p + 1] << 1);
            const uint32_t pp = P[2 * p] | (P[2 * p + 1] << 1);
            const int off = 2 * n * p;
            PA[off >> 5] |= pa << (off & 31);
            PP[off >> 5] |= pp << (off & 31);
            if ((off & 31) + 2 * n > 32) {
                PA[(off >> 5) + 1] |= pa >> (32 - (off & 31));
                PP[(off >> 5) + 1] |= pp >> (32 - (off & 31));
            }
        }
        const int NPW = (10 * n + 31) / 32;
        const uint32_t cbw = (uint32_t)(i * G::W + w) << 8;
        uint32_t LT[5] = {0u, 0u, 0u, 0u, 0u}, EQ[5] = {0u, 0u, 0u, 0u, 0u};
        const uint32_t* const wpl = planes + 160 * w;
#pragma unroll
        for (int pw = 0; pw < 5; ++pw)
            if (pw < NPW)
                hidden_head(PP[pw], PA[pw], wpl + 32 * pw, cbw | ((uint32_t)pw << 3), c3, sweep, chain, k0, k1,
                            LT[pw], EQ[pw]);
        hidden_tail(NPW, LT, EQ, cbw, tail_cap, wpl, c3, sweep, chain, k0, k1, tailbuf, lane);
#pragma unroll
        for (int p = 0; p < 5; ++p) {
            const int off = 2 * n * p;
            // units at or above their threshold go against their field
            uint32_t pair = (PP[off >> 5] & ~LT[off >> 5]) >> (off & 31);
            if ((off & 31) + 2 * n > 32) pair |= (PP[(off >> 5) + 1] & ~LT[(off >> 5) + 1]) << (32 - (off & 31));
            // the sign of the field (s_a for an agreeing bond, +1 for a zero field),
            // flipped where the unit went against it
            H[2 * p][w] = (ea[2 * p] | ~A[2 * p]) ^ pair;
            H[2 * p + 1][w] = (ea[2 * p + 1] | ~A[2 * p + 1]) ^ (pair >> 1);
        }
    }
}

// Byte offsets of the table lookups of one class: byte k of By[j] is
// 4 pattern (+ 128 on an open row edge) of the class's spin at even column
// 2 (j + 4k) of the word; pattern bit t is term t of the spin.
__device__ __forceinline__ void regroup(const uint32_t (&tp)[5], uint32_t redge_bits, uint32_t (&By)[4]) {
    const uint32_t Pa = tp[0] | (tp[1] << 1), Pb = tp[2] | (tp[3] << 1);
    const uint32_t xe = (Pa & 0x33333333u) | ((Pb & 0x33333333u) << 2);  // columns 4u
    const uint32_t xo = ((Pa >> 2) & 0x33333333u) | (Pb & 0xccccccccu);  // columns 4u + 2
    By[0] = ((xe & 0x0f0f0f0fu) << 2) | ((tp[4] << 6) & 0x40404040u) | redge_bits;
    By[1] = ((xo & 0x0f0f0f0fu) << 2) | ((tp[4] << 4) & 0x40404040u) | redge_bits;
    By[2] = ((xe >> 2) & 0x3c3c3c3cu) | ((tp[4] << 2) & 0x40404040u) | redge_bits;
    By[3] = ((xo >> 2) & 0x3c3c3c3cu) | (tp[4] & 0x40404040u) | redge_bits;
}

template <int N>
__device__ __forceinline__ uint32_t pick(const uint32_t (&a)[N], int k) {
    uint32_t v = 0u;
#pragma unroll
    for (int x = 0; x < N; ++x) v |= a[x] & (0u - (uint32_t)(k == x));
    return v;
}

// Visible half-step of the rows of cell row i: the mid row 2i+1 when DO_MID,
// the top row 2i when do_top.  H: hidden planes of cell row i; Hp5/7/9: of
// cell row i - 1.  Slots are taken from the last block and the last slot
// backwards, so each row's new spins are shifted in from the highest column
// down.  The Philox block holding slots of both rows (when Lc is not a
// multiple of 8) of cell row 0 is drawn once: the first call (mid row only,
// save) stores it in `straddle`, the last (top row only) reuses it.
template <int LC, bool DO_MID>
__device__ __forceinline__ void visible_rows(const uint32_t (&H)[10][LGeo<LC>::W], const uint32_t (&Hp5)[LGeo<LC>::W],
                                             const uint32_t (&Hp7)[LGeo<LC>::W], const uint32_t (&Hp9)[LGeo<LC>::W],
                                             bool open_c, bool redge_top, bool redge_mid, const LSweep& K,
                                             const uint32_t* lds, const uint32_t* __restrict__ gtab, int i,
                                             bool do_top, bool save, uint32_t c3,
                                             uint32_t sweep, uint32_t chain, uint32_t k0, uint32_t k1,
                                             uint32_t (&nt)[LGeo<LC>::W], uint32_t (&nm)[LGeo<LC>::W],
                                             P4 (&straddle)[LGeo<LC>::W]) {
    using G = LGeo<LC>;
    const char* const tb = reinterpret_cast<const char*>(lds);
    const uint32_t cedge_off = open_c ? 256u : 0u;  // the column-edge entries of a class
#pragma unroll
    for (int w = 0; w < G::W; ++w) {
        const int m = G::m(w);
        const uint32_t E = G::even(w);
        uint32_t ByT[8], ByM[8];  // classes 0, 1 (top row) and 2, 3 (mid row)
        {
            const uint32_t h1l = lsh2<LC>(H[1], w, open_c), h3l = lsh2<LC>(H[3], w, open_c),
                           h9l = lsh2<LC>(H[9], w, open_c);
            const uint32_t src[4][5] = {
                {H[0][w], H[4][w], h1l, Hp5[w], H[8][w]},
                {H[0][w], H[1][w], H[6][w], Hp7[w], Hp9[w]},
                {H[2][w], H[4][w], H[5][w], h3l, h9l},
                {H[2][w], H[3][w], H[6][w], H[7][w], H[8][w]},
            };
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (c >= 2 && !DO_MID) continue;
                const bool redge = (c < 2) ? redge_top : redge_mid;
                // column-edge cell: column 0 (classes 0, 2) or the last cell (classes 1, 3)
                const uint32_t cedge = !open_c ? 0u : ((c == 0 || c == 2) ? (w == 0 ? 1u : 0u) : G::last_cell(w));
                uint32_t tp[5];
#pragma unroll
                for (int t = 0; t < 5; ++t) {
                    uint32_t v = src[c][t];
                    if (term_is_b(c, t)) v ^= K.neg[term_filter(c, t)];
                    if ((row_edge_terms(c) >> t) & 1u) v = redge ? 0u : v;
                    if ((col_edge_terms(c) >> t) & 1u) v &= ~cedge;
                    tp[t] = v & E;
                }
                uint32_t By[4];
                regroup(tp, redge ? 0x80808080u : 0u, By);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (c < 2) ByT[4 * (c & 1) + j] = By[j];
                    else ByM[4 * (c & 1) + j] = By[j];
                }
            }
        }
        const int NQ = 2 * m;
        const int NB = (NQ + 7) / 8;
        const uint32_t cbase = (uint32_t)(i * G::W + w) << 5;
        uint32_t NS[2] = {0u, 0u};
        uint32_t tieblk = 0u;
        // one slot: outside a tie the new spin is the sign bit of P - entry;
        // a tie (P = tc - 1) leaves a zero low half, kept in rv[s] for the
        // block's 16-bit minimum
        auto spin = [&](const P4& p, int s, int q, uint32_t (&rv)[8]) {
            const int row = q / m, col = q % m, cls = 2 * row + (col & 1);
            const int si = col >> 1;
            const uint32_t by = (row == 0 ? ByT[4 * (cls & 1) + (si & 3)] : ByM[4 * (cls & 1) + (si & 3)]);
            uint32_t addr = (by >> (8 * (si >> 2))) & 0xffu;
            const bool edge = (cls & 1) ? (w == G::W - 1 && col == m - 1) : (w == 0 && col == 0);
            if (edge) addr += cedge_off;
            const uint32_t v = *reinterpret_cast<const uint32_t*>(tb + 4 * kVis + 512 * cls + addr);
            const uint32_t r = gk::slot16(p, s) - v;
            NS[row] = __builtin_amdgcn_alignbit(NS[row], r, 31);
            rv[s] = r;
        };
#pragma unroll
        for (int blk = 7; blk >= 0; --blk) {
            if (blk >= NB) continue;
            const bool has_top = blk * 8 < m, has_mid = blk * 8 + 7 >= m;
            const bool shared = has_top && has_mid;
            if (!(has_mid && DO_MID) && !(has_top && do_top)) continue;
            P4 p;
            if (shared && !DO_MID) {
                p = straddle[w];
            } else {
                p = philox(cbase | (uint32_t)blk, sweep, chain, c3, k0, k1);
                if (shared && save) straddle[w] = p;
            }
            uint32_t rv[8];  // 0xffff where a slot is absent or its row not updated
#pragma unroll
            for (int s = 0; s < 8; ++s) rv[s] = 0xffffu;
            if (DO_MID) {
#pragma unroll
                for (int s = 7; s >= 0; --s) {
                    const int q = blk * 8 + s;
                    if (q < NQ && q >= m) spin(p, s, q, rv);
                }
            }
            if (has_top && do_top) {
#pragma unroll
                for (int s = 7; s >= 0; --s) {
                    const int q = blk * 8 + s;
                    if (q < m) spin(p, s, q, rv);
                }
            }
            const int ns = NQ - blk * 8 < 8 ? NQ - blk * 8 : 8;  // slots of this block (compile time)
            uint32_t low = ns > 1 ? gk::min3_u16(rv[ns - 1], rv[ns - 1], rv[ns - 2]) : rv[0];
#pragma unroll
            for (int s = ns - 3; s >= 0; s -= 2) low = gk::min3_u16(low, rv[s], rv[s > 0 ? s - 1 : 0]);
            if (__ballot((uint16_t)low == 0u)) tieblk |= 1u << blk;
        }
        // Rare path: a primary slot P = tc - 1; redo the affected blocks with
        // the refinement stream and exact 32-bit compares (the new spin is
        // U < t for a field >= 0, U >= t for a negative one).
        while (tieblk) {
            const int blk = __builtin_ctz(tieblk);
            tieblk &= tieblk - 1u;
            const P4 p = philox(cbase | (uint32_t)blk, sweep, chain, c3, k0, k1);
            const P4 r = philox(cbase | (uint32_t)blk, sweep, chain, c3 + 1u, k0, k1);
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int q = blk * 8 + s;
                if (q >= NQ) continue;
                const int row = q >= m ? 1 : 0;
                if (row == 1 && !DO_MID) continue;
                if (row == 0 && !do_top) continue;
                const int col = q - row * m, cls = 2 * row + (col & 1), si = col >> 1;
                const int k = 4 * (cls & 1) + (si & 3);
                uint32_t addr = ((row == 0 ? pick(ByT, k) : pick(ByM, k)) >> (8 * (si >> 2))) & 0xffu;
                const bool edge = (cls & 1) ? (w == G::W - 1 && col == m - 1) : (w == 0 && col == 0);
                if (edge) addr += cedge_off;
                const uint32_t off = 512u * (uint32_t)cls + addr;
                const uint32_t v = *reinterpret_cast<const uint32_t*>(tb + 4 * kVis + off);
                // the host's entry index ((cls * 2 + row edge) * 2 + column edge) * 32 + pattern
                const uint32_t x = off >> 2, pat = x & 31u, redge = (x >> 5) & 1u, cedge = (x >> 6) & 1u;
                const uint32_t t = gtab[kHead + kEntries + ((((uint32_t)cls * 2u + redge) * 2u + cedge) << 5) + pat];
                const uint32_t U = (gk::slot16(p, s) << 16) | gk::slot16(r, s);
                const uint32_t bit = 1u << col, f = ((U < t) ^ (v >> 31)) ? bit : 0u;
                if (row == 0)
                    NS[0] = (NS[0] & ~bit) | f;
                else
                    NS[1] = (NS[1] & ~bit) | f;
            }
        }
        nt[w] = NS[0];
        nm[w] = NS[1];
    }
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// CAP: the hidden tail takes a.tail_cap words per round (else the constant 64).
template <int LC, bool CAP>
__global__ void __launch_bounds__(64) lattice_kernel(LatArgs a) {
    using G = LGeo<LC>;
    constexpr int W = G::W;
    extern __shared__ uint32_t lds[];
    const LatItem it = a.items[blockIdx.x];
    const int lane = threadIdx.x;
    const int Lr = it.Lr, Cr = it.Lr / 2;
    const bool open_r = it.open_r != 0, open_c = it.open_c != 0;
    uint32_t* const S = lds + lat_spins_word(W);  // [Lr][W][64]
    uint32_t* const tailbuf = lds + kTail;
    const bool active = lane < (int)it.nchains;
    const uint32_t chain = it.chain0 + (active ? (uint32_t)lane : 0u);
    const uint64_t gch = it.gbase + (active ? (uint64_t)lane : 0u);
    {
        const uint32_t* st = a.state + it.state_off + (uint64_t)(active ? lane : 0) * Lr * W;
        for (int x = 0; x < Lr * W; ++x) S[x * 64 + lane] = st[x];
    }
    const uint32_t c3h = (it.id << 3) | 1u, c3v = (it.id << 3) | 3u;
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    int64_t tab_loaded = -1;
    for (int64_t s = a.s0; s < a.s1; ++s) {
        const int64_t ts = it.tab_stride ? s : 0;
        const uint32_t* tb = a.tables + it.tab_off + (uint64_t)it.tab_stride * (uint64_t)s;
        if (ts != tab_loaded) {
            // the visible entries in the kernel's order, each with its field's sign
            __syncthreads();
            for (int x = lane; x < kEntries; x += 64) {
                const int pat = x & 31, cedge = (x >> 5) & 1, redge = (x >> 6) & 1, cls = x >> 7;
                const uint32_t t = tb[kHead + kEntries + x];
                const bool nonneg = ((tb[kHead + 2 * kEntries + (x >> 5)] >> (x & 31)) & 1u) != 0u;
                const int kx = ((cls * 2 + cedge) * 2 + redge) * 32 + pat;
                // tc - 1, tc = ceil(t / 2^16) >= 2^15 (t: the threshold of |x|), then the sign in bit 31
                lds[kVis + kx] = (t >> 16) + ((t & 0xffffu) != 0u) - 1u + (nonneg ? 0u : 0x80000000u);
            }
            // the hidden words' threshold planes
            uint32_t T[10];
#pragma unroll
            for (int k = 0; k < 10; ++k) T[k] = tb[k];
            for (int x = lane; x < W * 160; x += 64) {
                const int w = x / 160, pw = (x / 32) % 5, b = x % 32;
                lds[kPlanes + x] = filter_plane(T, w == W - 1 ? G::ML / 2 : 16, pw, b);
            }
            __syncthreads();
            tab_loaded = ts;
        }
        LSweep K;
        const uint32_t fneg = tb[10], fen = tb[11];
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            K.neg[k] = ((fneg >> k) & 1u) ? 0xffffffffu : 0u;
            K.en[k] = ((fen >> k) & 1u) ? 0xffffffffu : 0u;
        }
        const uint32_t sweep = (uint32_t)s;
        uint32_t Hf0[W], Hf1[W], Hf4[W], Hf6[W], Hf8[W], Hp5[W], Hp7[W], Hp9[W];
        P4 straddle[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            Hf0[w] = Hf1[w] = Hf4[w] = Hf6[w] = Hf8[w] = Hp5[w] = Hp7[w] = Hp9[w] = 0u;
            straddle[w] = P4{{0u, 0u, 0u, 0u}};
        }
        for (int i = 0; i < Cr; ++i) {
            uint32_t top[W], mid[W], bot[W];
            const int rb = (2 * i + 2 < Lr) ? 2 * i + 2 : 0;  // the old row 0 on a periodic axis
#pragma unroll
            for (int w = 0; w < W; ++w) {
                top[w] = S[((2 * i) * W + w) * 64 + lane];
                mid[w] = S[((2 * i + 1) * W + w) * 64 + lane];
                bot[w] = S[(rb * W + w) * 64 + lane];
            }
            uint32_t H[10][W];
            hidden_row<LC>(top, mid, bot, open_c, open_r && i == Cr - 1, K, lds + kPlanes, i, c3h, sweep, chain, k0,
                           k1, tailbuf, CAP ? a.tail_cap : 64u, lane, H);
            uint32_t nt[W], nm[W];
            visible_rows<LC, true>(H, Hp5, Hp7, Hp9, open_c, false, open_r && i == Cr - 1, K, lds, tb, i, i > 0,
                                   i == 0, c3v, sweep, chain, k0, k1, nt, nm, straddle);
#pragma unroll
            for (int w = 0; w < W; ++w) {
                if (i > 0) S[((2 * i) * W + w) * 64 + lane] = nt[w];
                S[((2 * i + 1) * W + w) * 64 + lane] = nm[w];
                if (i == 0) {
                    Hf0[w] = H[0][w]; Hf1[w] = H[1][w]; Hf4[w] = H[4][w]; Hf6[w] = H[6][w]; Hf8[w] = H[8][w];
                }
                Hp5[w] = H[5][w]; Hp7[w] = H[7][w]; Hp9[w] = H[9][w];
            }
        }
        {   // row 0: its terms from the cell row above are those of the last cell row
            uint32_t Hd[10][W], nt[W], nm[W];
#pragma unroll
            for (int w = 0; w < W; ++w) {
                Hd[0][w] = Hf0[w]; Hd[1][w] = Hf1[w]; Hd[4][w] = Hf4[w]; Hd[6][w] = Hf6[w]; Hd[8][w] = Hf8[w];
                Hd[2][w] = Hd[3][w] = Hd[5][w] = Hd[7][w] = Hd[9][w] = 0u;
            }
            visible_rows<LC, false>(Hd, Hp5, Hp7, Hp9, open_c, open_r, false, K, lds, tb, 0, true, false, c3v,
                                    sweep, chain, k0, k1, nt, nm, straddle);
#pragma unroll
            for (int w = 0; w < W; ++w) S[w * 64 + lane] = nt[w];
        }

        const bool meas = a.measure_every > 0 && s >= a.burn_in && ((s - a.burn_in) % a.measure_every) == 0;
        const bool rec = a.trace != nullptr && ((s - a.trace_s0 + 1) % a.trace_every) == 0;
        if (meas || rec) {
            // counts: M_even, M_odd, B_k = present_k - 2 (disagreeing bonds of filter k)
            int me = 0, mo = 0, stag = 0, dis[10];
#pragma unroll
            for (int k = 0; k < 10; ++k) dis[k] = 0;
            for (int i = 0; i < Cr; ++i) {
                uint32_t top[W], mid[W], bot[W];
                const int rb = (2 * i + 2 < Lr) ? 2 * i + 2 : 0;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    top[w] = S[((2 * i) * W + w) * 64 + lane];
                    mid[w] = S[((2 * i + 1) * W + w) * 64 + lane];
                    bot[w] = S[(rb * W + w) * 64 + lane];
                }
                const bool last_row_open = open_r && i == Cr - 1;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const uint32_t E = G::even(w), O = G::full(w) & ~E;
                    const int pe = __popc(top[w] & E) + __popc(mid[w] & E);
                    const int po = __popc(top[w] & O) + __popc(mid[w] & O);
                    me += pe;
                    mo += po;
                    stag += 2 * ((__popc(top[w] & E) - __popc(top[w] & O)) - (__popc(mid[w] & E) - __popc(mid[w] & O)));
                    const uint32_t t1 = rsh<LC, 1>(top, w, open_c), t2 = rsh<LC, 2>(top, w, open_c);
                    const uint32_t m1 = rsh<LC, 1>(mid, w, open_c), m2 = rsh<LC, 2>(mid, w, open_c);
                    const uint32_t b1 = rsh<LC, 1>(bot, w, open_c);
                    const uint32_t ea[10] = {top[w], t1, mid[w], m1, top[w], mid[w], t1, m1, top[w], m2};
                    const uint32_t eb[10] = {t1, t2, m1, m2, mid[w], bot[w], m1, b1, m1, b1};
                    const uint32_t pc = open_c ? ~G::last_cell(w) : 0xffffffffu;
                    const uint32_t pr = last_row_open ? 0u : 0xffffffffu;
#pragma unroll
                    for (int k = 0; k < 10; ++k) {
                        uint32_t pm = E;
                        if (k == 1 || k == 3 || k == 9) pm &= pc;
                        if (k == 5 || k == 7 || k == 9) pm &= pr;
                        dis[k] += __popc((ea[k] ^ eb[k]) & pm);
                    }
                }
            }
            const int half = (Lr * LC) / 2;  // sites per column parity
            int cnt[12];
            cnt[0] = 2 * me - half;
            cnt[1] = 2 * mo - half;
#pragma unroll
            for (int k = 0; k < 10; ++k) cnt[2 + k] = it.np[k] - 2 * dis[k];
            if (rec && active) {
                int32_t* tr = a.trace + ((uint64_t)((s - a.trace_s0) / a.trace_every) * (uint64_t)a.total_chains + gch) * 12;
#pragma unroll
                for (int q = 0; q < 12; ++q) tr[q] = cnt[q];
            }
            if (meas && active) {
                int64_t* ac = a.acc + gch * CRBM_LAT_N_ACC;
                const int64_t M = (int64_t)cnt[0] + cnt[1], Ms = stag;
                ac[0] += 1;
#pragma unroll
                for (int q = 0; q < 12; ++q) ac[1 + q] += cnt[q];
                ac[13] += M * M;
                ac[14] += M < 0 ? -M : M;
                ac[15] += Ms;
                ac[16] += Ms * Ms;
                ac[17] += Ms < 0 ? -Ms : Ms;
            }
            if (meas && a.corr != nullptr && it.corr_off >= 0) {
                // Cn(dr, dc): pairs inside the lattice (no wrap); rows as 64-bit words
                constexpr uint64_t fullrow = LC == 64 ? ~0ull : ((1ull << LC) - 1ull);
                unsigned long long* cn = a.corr + it.corr_off;
                for (int dr = 0; dr < Lr; ++dr)
                    for (int dc = -(LC - 1); dc < LC; ++dc) {
                        const uint64_t ov = dc >= 0 ? (fullrow >> dc) : ((fullrow << (-dc)) & fullrow);
                        const int nov = LC - (dc < 0 ? -dc : dc);
                        int dsum = 0;
                        for (int r = 0; r + dr < Lr; ++r) {
                            uint64_t x = 0ull, y = 0ull;
#pragma unroll
                            for (int w = 0; w < W; ++w) {
                                x |= (uint64_t)S[(r * W + w) * 64 + lane] << (32 * w);
                                y |= (uint64_t)S[((r + dr) * W + w) * 64 + lane] << (32 * w);
                            }
                            const uint64_t ys = dc >= 0 ? (y >> dc) : (y << (-dc));
                            dsum += __popcll((x ^ ys) & ov);
                        }
                        int v = active ? (nov * (Lr - dr) - 2 * dsum) : 0;
                        v = wave_sum(v);
                        if (lane == 0)
                            atomicAdd(&cn[dr * (2 * LC - 1) + dc + LC - 1], (unsigned long long)(int64_t)v);
                    }
            }
        }
    }
    if (!active) return;
    {
        uint32_t* st = a.state + it.state_off + (uint64_t)lane * Lr * W;
        for (int x = 0; x < Lr * W; ++x) st[x] = S[x * 64 + lane];
    }
    if (a.spins_out) {
        int8_t* out = a.spins_out + it.spin_off + (uint64_t)lane * Lr * LC;
        for (int r = 0; r < Lr; ++r)
            for (int c = 0; c < LC; ++c) out[r * LC + c] = ((S[(r * W + (c >> 5)) * 64 + lane] >> (c & 31)) & 1u) ? 1 : -1;
    }
}

// Launch the kernel of column count LC over a.n_items workgroups of one
// wavefront with `lds` bytes of dynamic LDS.
template <int LC>
hipError_t launch_width(const LatArgs& a, int lds, hipStream_t st) {
    if (a.tail_cap < 64u)
        hipLaunchKernelGGL((lattice_kernel<LC, true>), dim3((unsigned)a.n_items), dim3(64), lds, st, a);
    else
        hipLaunchKernelGGL((lattice_kernel<LC, false>), dim3((unsigned)a.n_items), dim3(64), lds, st, a);
    return hipGetLastError();
}

// Compiled column counts, split over translation units: each returns false
// if Lc is not one of its own, else launches and sets *err.
bool widths_a(int Lc, const LatArgs& a, int lds, hipStream_t st, hipError_t* err);
bool widths_b(int Lc, const LatArgs& a, int lds, hipStream_t st, hipError_t* err);
bool widths_c(int Lc, const LatArgs& a, int lds, hipStream_t st, hipError_t* err);
bool widths_d(int Lc, const LatArgs& a, int lds, hipStream_t st, hipError_t* err);

}  // namespace lat
}  // namespace crbmlib
