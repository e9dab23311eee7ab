// lattice.hip -- block Gibbs sampling of the CRBM on general lattices:
// Lr x Lc, each axis periodic or open (App. A Wrapper Module: columns and
// rows past the edge are copies or zeros), one coupling per filter (App. A
// Convoluter-Reverse: the host writes every filter's weights), and separate
// visible biases for even and odd columns (App. A Accumulator).  Same
// arithmetic and random-number conventions as the square-lattice sampler, so
// a periodic square SS lattice gives the same trajectories in both.
//
// Reading of the open boundary: a bond whose endpoint would lie past the last
// row (column) of an open axis does not exist.  Its hidden unit is not drawn
// and no field reaches its remaining spin.
//
// Mapping: one lane per chain, 64 chains of one instance per wavefront (one
// wavefront per workgroup).  A chain's bit rows (W = ceil(Lc/32) <= 2 words)
// live in LDS for the whole launch, lane-interleaved ([row][word][lane]: every
// access of a wavefront hits 64 consecutive words), because the geometry is a
// runtime value and registers cannot be indexed at run time.  All geometry,
// weights and thresholds are wavefront-uniform (scalar registers); only spins,
// hidden bits and random bits are per lane.
//
// Per sweep and cell row i (rows 2i, 2i+1): the 10 hidden planes of the cell
// row from the old spins (bit-sliced compare against per-filter thresholds,
// as in the square-lattice sampler), then the new spins of rows 2i+1 and (for
// i > 0) 2i; row 0 is updated last, after the last cell row's hidden units
// (which read the old row 0 on a periodic axis).  A spin's threshold and sign
// come from a 512-entry table by (sublattice, edge flags, 5-bit pattern of its
// incident hidden units); absent terms are zero bits of the pattern and the
// table entry of that edge type leaves them out.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "crbm.h"
#include "crbm_internal.h"
#include "gibbs_kernel.h"

namespace crbmlib {
namespace lat {

using gk::P4;
using gk::philox;

// Per-sweep table of one instance (words):
//   [0..9]    agree threshold t(2 wq_k) of filter k (2^31 if wq_k == 0)
//   [10]      bit k: sig_k < 0;  [11] bit k: wq_k != 0;  [12..15] zero
//   [16 + e]  visible entry e (e = type * 32 + pattern): min(tceil16, 0xffff) | thi16 << 16
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

// ------------------------------------------------------------ device code

struct Geo {
    int Lr, Lc, W, Cr, ML;   // ML: columns in the last word
    bool open_r, open_c;
    __device__ int m(int w) const { return w == W - 1 ? ML : 32; }
    __device__ uint32_t full(int w) const { return m(w) == 32 ? 0xffffffffu : ((1u << m(w)) - 1u); }
    __device__ uint32_t even(int w) const { return 0x55555555u & full(w); }
    // even-column bit of the last cell, in the last word (a column-edge site of classes 1, 3)
    __device__ uint32_t last_cell(int w) const { return w == W - 1 ? (1u << (ML - 2)) : 0u; }
};

template <int W>
__device__ __forceinline__ uint32_t rsh1(const uint32_t (&x)[W], int w, const Geo& g) {
    if (w < W - 1) return (x[w] >> 1) | (x[w + 1] << 31);
    const uint32_t wrap = g.open_c ? 0u : (x[0] & 1u);
    return ((x[w] >> 1) | (wrap << (g.ML - 1))) & g.full(w);
}
template <int W>
__device__ __forceinline__ uint32_t rsh2(const uint32_t (&x)[W], int w, const Geo& g) {
    if (w < W - 1) return (x[w] >> 2) | (x[w + 1] << 30);
    const uint32_t wrap = g.open_c ? 0u : (x[0] & 3u);
    return ((x[w] >> 2) | (wrap << (g.ML - 2))) & g.full(w);
}
template <int W>
__device__ __forceinline__ uint32_t lsh2(const uint32_t (&x)[W], int w, const Geo& g) {
    if (w > 0) return ((x[w] << 2) | (x[w - 1] >> 30)) & g.full(w);
    const uint32_t top = g.open_c ? 0u : ((x[W - 1] >> (g.ML - 2)) & 3u);
    return ((x[0] << 2) | top) & g.full(0);
}

__device__ __forceinline__ uint32_t bits_between(int lo, int hi) {
    if (hi <= lo) return 0u;
    const uint32_t top = hi >= 32 ? 0xffffffffu : ((1u << hi) - 1u);
    return top & ~((1u << lo) - 1u);
}

struct Sweep {
    uint32_t T[10];    // agree thresholds
    uint32_t neg[10];  // all ones if sig_k < 0
    uint32_t en[10];   // all ones if wq_k != 0
};

// Bit-sliced U < t over 32 packed hidden units of word pw (units u = 32 pw +
// bit; unit u belongs to filter 2 (u div 2n) + (u mod 2)); val: units that
// exist; ag: agreeing units.  Returns the units that go against their field.
__device__ __forceinline__ uint32_t hidden_compare(uint32_t val, uint32_t ag, int n, int pw, const Sweep& K, uint32_t cb,
                                   uint32_t c3, uint32_t sweep, uint32_t chain, uint32_t k0, uint32_t k1) {
    const int lo = 32 * pw, span = 2 * n;
    const int p0 = lo / span, p1 = min((lo + 31) / span, 4);
    auto tplane = [&](int b) -> uint32_t {
        uint32_t t = 0u;
#pragma unroll
        for (int p = 0; p < 5; ++p) {  // constant indices: K stays in scalar registers
            if (p < p0 || p > p1) continue;
            const uint32_t run = bits_between(max(span * p - lo, 0), min(span * (p + 1) - lo, 32));
            const uint32_t pl = (gk::plane_mask(K.T[2 * p], b) & 0x55555555u) |
                                (gk::plane_mask(K.T[2 * p + 1], b) & 0xAAAAAAAAu);
            t |= run & pl;
        }
        return t;
    };
    P4 p = philox(cb, sweep, chain, c3, k0, k1);
    uint32_t lt = val & ~p.v[0];
    uint32_t eq = ag & p.v[0];
    for (int b = 1; b < 4; ++b) gk::compare_plane(lt, eq, p.v[b], tplane(b));
    for (int c = 1; c < 8; ++c) {
        if (!__any(eq != 0u)) break;
        p = philox(cb | (uint32_t)c, sweep, chain, c3, k0, k1);
        for (int s = 0; s < 4; ++s) gk::compare_plane(lt, eq, p.v[s], tplane(4 * c + s));
    }
    return val & ~lt;
}

// Hidden half-step of cell row i: H[k][w] holds the unit of bond k of every
// cell at the cell's even column (other bits undefined).
template <int W>
__device__ __forceinline__ void hidden_row(const uint32_t (&top)[W], const uint32_t (&mid)[W], const uint32_t (&bot)[W],
                           const Geo& g, const Sweep& K, int i, uint32_t c3, uint32_t sweep, uint32_t chain,
                           uint32_t k0, uint32_t k1, uint32_t (&H)[10][W]) {
    const bool last_row_open = g.open_r && i == g.Cr - 1;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const int n = g.m(w) / 2;
        const uint32_t E = g.even(w);
        const uint32_t t1 = rsh1<W>(top, w, g), t2 = rsh2<W>(top, w, g);
        const uint32_t m1 = rsh1<W>(mid, w, g), m2 = rsh2<W>(mid, w, g);
        const uint32_t b1 = rsh1<W>(bot, w, g);
        const uint32_t ea[10] = {top[w], t1, mid[w], m1, top[w], mid[w], t1, m1, top[w], m2};
        const uint32_t eb[10] = {t1, t2, m1, m2, mid[w], bot[w], m1, b1, m1, b1};
        // bonds present at this cell row: k1, k3, k9 lose the last cell on an open
        // column axis; k5, k7, k9 lose the last cell row on an open row axis
        const uint32_t pc = g.open_c ? ~g.last_cell(w) : 0xffffffffu;
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
        uint32_t PA[5] = {0u, 0u, 0u, 0u, 0u}, PP[5] = {0u, 0u, 0u, 0u, 0u};
#pragma unroll
        for (int p = 0; p < 5; ++p) {
            const uint32_t pa = A[2 * p] | (A[2 * p + 1] << 1);
            const uint32_t pp = P[2 * p] | (P[2 * p + 1] << 1);
            const int off = 2 * n * p, wd = off >> 5, sh = off & 31;
#pragma unroll
            for (int x = 0; x < 5; ++x) {
                if (x == wd) {
                    PA[x] |= pa << sh;
                    PP[x] |= pp << sh;
                }
                if (x == wd + 1 && sh + 2 * n > 32) {
                    PA[x] |= pa >> (32 - sh);
                    PP[x] |= pp >> (32 - sh);
                }
            }
        }
        const int NPW = (10 * n + 31) / 32;
        uint32_t DP[5] = {0u, 0u, 0u, 0u, 0u};
        const uint32_t cbw = (uint32_t)(i * W + w) << 8;
#pragma unroll
        for (int pw = 0; pw < 5; ++pw)
            if (pw < NPW)
                DP[pw] = hidden_compare(PP[pw], PA[pw], n, pw, K, cbw | ((uint32_t)pw << 3), c3, sweep, chain,
                                        k0, k1);
#pragma unroll
        for (int p = 0; p < 5; ++p) {
            const int off = 2 * n * p, wd = off >> 5, sh = off & 31;
            uint32_t pair = 0u;
#pragma unroll
            for (int x = 0; x < 5; ++x) {
                if (x == wd) pair |= DP[x] >> sh;
                if (x == wd + 1 && sh + 2 * n > 32) pair |= DP[x] << (32 - sh);
            }
            // the sign of the field (s_a for an agreeing bond, +1 for a zero field),
            // flipped where the unit went against it
            H[2 * p][w] = (ea[2 * p] | ~A[2 * p]) ^ pair;
            H[2 * p + 1][w] = (ea[2 * p + 1] | ~A[2 * p + 1]) ^ (pair >> 1);
        }
    }
}

// Visible half-step of the rows of cell row i (top = 2i if do_top, mid = 2i+1
// if do_mid).  H: hidden planes of cell row i; Hp5/7/9: of cell row i - 1.
template <int W>
__device__ __forceinline__ void visible_rows(const uint32_t (&H)[10][W], const uint32_t (&Hp5)[W], const uint32_t (&Hp7)[W],
                             const uint32_t (&Hp9)[W], const Geo& g, const Sweep& K, const uint32_t* tab, int i,
                             bool do_top, bool do_mid, uint32_t c3, uint32_t sweep, uint32_t chain, uint32_t k0,
                             uint32_t k1, uint32_t (&nt)[W], uint32_t (&nm)[W]) {
    const bool redge_top = g.open_r && i == 0, redge_mid = g.open_r && i == g.Cr - 1;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const int m = g.m(w);
        const uint32_t E = g.even(w);
        uint32_t trm[4][5];
        {
            const uint32_t h1l = lsh2<W>(H[1], w, g), h3l = lsh2<W>(H[3], w, g), h9l = lsh2<W>(H[9], w, g);
            const uint32_t src[4][5] = {
                {H[0][w], H[4][w], h1l, Hp5[w], H[8][w]},
                {H[0][w], H[1][w], H[6][w], Hp7[w], Hp9[w]},
                {H[2][w], H[4][w], H[5][w], h3l, h9l},
                {H[2][w], H[3][w], H[6][w], H[7][w], H[8][w]},
            };
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const bool redge = (c < 2) ? redge_top : redge_mid;
                // column-edge cell: column 0 (classes 0, 2) or the last cell (classes 1, 3)
                const uint32_t cedge = !g.open_c ? 0u : ((c == 0 || c == 2) ? (w == 0 ? 1u : 0u) : g.last_cell(w));
#pragma unroll
                for (int t = 0; t < 5; ++t) {
                    uint32_t v = src[c][t];
                    if (term_is_b(c, t)) v ^= K.neg[term_filter(c, t)];
                    if (redge && ((row_edge_terms(c) >> t) & 1u)) v = 0u;
                    if ((col_edge_terms(c) >> t) & 1u) v &= ~cedge;
                    trm[c][t] = v & E;
                }
            }
        }
        const int NQ = 2 * m;
        const int NB = (NQ + 7) / 8;
        const uint32_t cbase = (uint32_t)(i * W + w) << 5;
        uint32_t top_new = 0u, mid_new = 0u;
        for (int blk = 0; blk < NB; ++blk) {
            const bool has_top = blk * 8 < m, has_mid = blk * 8 + 7 >= m;
            if (!((do_top && has_top) || (do_mid && has_mid))) continue;
            const P4 p = philox(cbase | (uint32_t)blk, sweep, chain, c3, k0, k1);
            for (int s = 0; s < 8; ++s) {
                const int q = blk * 8 + s;
                if (q >= NQ) break;
                const int row = q >= m ? 1 : 0;
                if (!(row == 0 ? do_top : do_mid)) continue;
                const int col = q - row * m;
                const int cls = 2 * row + (col & 1);
                const int pos = col & ~1;
                uint32_t pat = 0u;
#pragma unroll
                for (int t = 0; t < 5; ++t) {
                    const uint32_t v = cls == 0 ? trm[0][t] : cls == 1 ? trm[1][t] : cls == 2 ? trm[2][t] : trm[3][t];
                    pat |= ((v >> pos) & 1u) << t;
                }
                const bool redge = row == 0 ? redge_top : redge_mid;
                const bool cedge = g.open_c && ((cls & 1) ? (w == g.W - 1 && col == m - 1) : (w == 0 && col == 0));
                const uint32_t e = (uint32_t)((((cls * 2 + (redge ? 1 : 0)) * 2 + (cedge ? 1 : 0)) << 5) | pat);
                const uint32_t tv = tab[kHead + e];
                const uint32_t sg = (tab[kHead + 2 * kEntries + (e >> 5)] >> (e & 31u)) & 1u;
                const uint32_t p16 = gk::slot16(p, s);
                uint32_t d = p16 >= (tv & 0xffffu) ? 1u : 0u;
                if (p16 == (tv >> 16)) {  // primary slot ties with the threshold's top half: exact 32-bit compare
                    const P4 r = philox(cbase | (uint32_t)blk, sweep, chain, c3 + 1u, k0, k1);
                    const uint32_t U = (p16 << 16) | gk::slot16(r, s);
                    d = U >= tab[kHead + kEntries + e] ? 1u : 0u;
                }
                const uint32_t bit = (sg ^ d) << col;
                if (row == 0) top_new |= bit; else mid_new |= bit;
            }
        }
        nt[w] = top_new;
        nm[w] = mid_new;
    }
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <int W>
__global__ void __launch_bounds__(64) lattice_kernel(LatArgs a) {
    extern __shared__ uint32_t lds[];
    const LatItem it = a.items[blockIdx.x];
    const int lane = threadIdx.x;
    Geo g;
    g.Lr = it.Lr;
    g.Lc = it.Lc;
    g.W = W;
    g.Cr = it.Lr / 2;
    g.ML = it.Lc - 32 * (W - 1);
    g.open_r = it.open_r != 0;
    g.open_c = it.open_c != 0;
    const int Lr = g.Lr;
    uint32_t* S = lds;                            // [Lr][W][64]
    uint32_t* tab = lds + (size_t)Lr * W * 64;    // one sweep's table
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
            __syncthreads();
            for (int x = lane; x < kLatTabWords; x += 64) tab[x] = tb[x];
            __syncthreads();
            tab_loaded = ts;
        }
        Sweep K;
        const uint32_t fneg = tb[10], fen = tb[11];
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            K.T[k] = tb[k];
            K.neg[k] = ((fneg >> k) & 1u) ? 0xffffffffu : 0u;
            K.en[k] = ((fen >> k) & 1u) ? 0xffffffffu : 0u;
        }
        const uint32_t sweep = (uint32_t)s;
        uint32_t Hf0[W], Hf1[W], Hf4[W], Hf6[W], Hf8[W], Hp5[W], Hp7[W], Hp9[W];
#pragma unroll
        for (int w = 0; w < W; ++w) Hf0[w] = Hf1[w] = Hf4[w] = Hf6[w] = Hf8[w] = Hp5[w] = Hp7[w] = Hp9[w] = 0u;
        for (int i = 0; i < g.Cr; ++i) {
            uint32_t top[W], mid[W], bot[W];
            const int rb = (2 * i + 2 < Lr) ? 2 * i + 2 : 0;  // the old row 0 on a periodic axis
#pragma unroll
            for (int w = 0; w < W; ++w) {
                top[w] = S[((2 * i) * W + w) * 64 + lane];
                mid[w] = S[((2 * i + 1) * W + w) * 64 + lane];
                bot[w] = S[(rb * W + w) * 64 + lane];
            }
            uint32_t H[10][W];
            hidden_row<W>(top, mid, bot, g, K, i, c3h, sweep, chain, k0, k1, H);
            uint32_t nt[W], nm[W];
            visible_rows<W>(H, Hp5, Hp7, Hp9, g, K, tab, i, i > 0, true, c3v, sweep, chain, k0, k1, nt, nm);
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
            visible_rows<W>(Hd, Hp5, Hp7, Hp9, g, K, tab, 0, true, false, c3v, sweep, chain, k0, k1, nt, nm);
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
            for (int i = 0; i < g.Cr; ++i) {
                uint32_t top[W], mid[W], bot[W];
                const int rb = (2 * i + 2 < Lr) ? 2 * i + 2 : 0;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    top[w] = S[((2 * i) * W + w) * 64 + lane];
                    mid[w] = S[((2 * i + 1) * W + w) * 64 + lane];
                    bot[w] = S[(rb * W + w) * 64 + lane];
                }
                const bool last_row_open = g.open_r && i == g.Cr - 1;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const uint32_t E = g.even(w), O = g.full(w) & ~E;
                    const int pe = __popc(top[w] & E) + __popc(mid[w] & E);
                    const int po = __popc(top[w] & O) + __popc(mid[w] & O);
                    me += pe;
                    mo += po;
                    stag += 2 * ((__popc(top[w] & E) - __popc(top[w] & O)) - (__popc(mid[w] & E) - __popc(mid[w] & O)));
                    const uint32_t t1 = rsh1<W>(top, w, g), t2 = rsh2<W>(top, w, g);
                    const uint32_t m1 = rsh1<W>(mid, w, g), m2 = rsh2<W>(mid, w, g);
                    const uint32_t b1 = rsh1<W>(bot, w, g);
                    const uint32_t ea[10] = {top[w], t1, mid[w], m1, top[w], mid[w], t1, m1, top[w], m2};
                    const uint32_t eb[10] = {t1, t2, m1, m2, mid[w], bot[w], m1, b1, m1, b1};
                    const uint32_t pc = g.open_c ? ~g.last_cell(w) : 0xffffffffu;
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
            const int half = (Lr * g.Lc) / 2;  // sites per column parity
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
                const int Lc = g.Lc;
                const uint64_t fullrow = Lc == 64 ? ~0ull : ((1ull << Lc) - 1ull);
                unsigned long long* cn = a.corr + it.corr_off;
                for (int dr = 0; dr < Lr; ++dr)
                    for (int dc = -(Lc - 1); dc < Lc; ++dc) {
                        const uint64_t ov = dc >= 0 ? (fullrow >> dc) : ((fullrow << (-dc)) & fullrow);
                        const int nov = Lc - (dc < 0 ? -dc : dc);
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
                            atomicAdd(&cn[dr * (2 * Lc - 1) + dc + Lc - 1], (unsigned long long)(int64_t)v);
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
        const int Lc = g.Lc;
        int8_t* out = a.spins_out + it.spin_off + (uint64_t)lane * Lr * Lc;
        for (int r = 0; r < Lr; ++r)
            for (int c = 0; c < Lc; ++c) out[r * Lc + c] = ((S[(r * W + (c >> 5)) * 64 + lane] >> (c & 31)) & 1u) ? 1 : -1;
    }
}

// Seeded start (stream 0): spin (r, c) is up iff bit (r Lc + c) & 127 of the
// Philox block with counter word (r Lc + c) >> 7 is set.  One thread per row.
__global__ void lat_init_kernel(uint32_t* state, const LatItem* items, int n_items, uint64_t seed) {
    const LatItem it = items[blockIdx.x];
    const int W = (it.Lc + 31) / 32;
    for (int t = threadIdx.x; t < (int)it.nchains * it.Lr; t += blockDim.x) {
        const int ch = t / it.Lr, r = t - ch * it.Lr;
        const uint32_t chain = it.chain0 + ch;
        uint32_t* row = state + it.state_off + ((uint64_t)ch * it.Lr + r) * W;
        for (int w = 0; w < W; ++w) {
            const int m = min(32, it.Lc - 32 * w);
            uint32_t word = 0u;
            for (int c = 0; c < m; ++c) {
                const uint32_t site = (uint32_t)(r * it.Lc + 32 * w + c);
                const P4 p = philox(site >> 7, 0u, chain, it.id << 3, (uint32_t)seed, (uint32_t)(seed >> 32));
                const uint32_t b = site & 127u;
                word |= ((p.v[b >> 5] >> (b & 31u)) & 1u) << c;
            }
            row[w] = word;
        }
    }
}

// int8 [chains][Lr][Lc] <-> bit rows, one thread per row of one instance.
__global__ void lat_pack_kernel(uint32_t* state, const int8_t* spins, int64_t nrows, int Lc) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrows) return;
    const int W = (Lc + 31) / 32;
    for (int w = 0; w < W; ++w) {
        uint32_t word = 0u;
        for (int c = 0; c < min(32, Lc - 32 * w); ++c) word |= (spins[t * Lc + 32 * w + c] > 0 ? 1u : 0u) << c;
        state[t * W + w] = word;
    }
}
__global__ void lat_unpack_kernel(const uint32_t* state, int8_t* spins, int64_t nrows, int Lc) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrows) return;
    const int W = (Lc + 31) / 32;
    for (int c = 0; c < Lc; ++c) spins[t * Lc + c] = ((state[t * W + (c >> 5)] >> (c & 31)) & 1u) ? 1 : -1;
}

// ------------------------------------------------------------- host code

int64_t q16(double x) { return llround(x * 65536.0); }

// One sweep's table at temperature T (layout above).  Returns CRBM_ERANGE if a
// field could leave int32.
int build_lattice_table(const crbm_lattice& I, double T, uint32_t* out) {
    int64_t wq[10];
    int sg[10];
    for (int k = 0; k < 10; ++k) map_hidden_weight(q16(I.J[k]), T, &wq[k], &sg[k]);
    const int64_t aq[2] = {llround((double)q16(I.h_even) / T), llround((double)q16(I.h_odd) / T)};
    // every field must stay inside int32: a hidden unit's 2 wq_k, and a spin's
    // bias plus its five incident weights
    const int64_t lim = (int64_t)1 << 31;
    for (int k = 0; k < 10; ++k)
        if (2 * wq[k] >= lim) return CRBM_ERANGE;
    for (int cls = 0; cls < 4; ++cls) {
        int64_t s5 = 0;
        for (int t = 0; t < 5; ++t) s5 += wq[term_filter(cls, t)];
        const int64_t a = aq[cls & 1] < 0 ? -aq[cls & 1] : aq[cls & 1];
        if (a + s5 >= lim) return CRBM_ERANGE;
    }
    std::memset(out, 0, sizeof(uint32_t) * kLatTabWords);
    for (int k = 0; k < 10; ++k) {
        out[k] = wq[k] != 0 ? map_threshold(2 * wq[k]) : 0x80000000u;
        if (sg[k] < 0) out[10] |= 1u << k;
        if (wq[k] != 0) out[11] |= 1u << k;
    }
    for (int cls = 0; cls < 4; ++cls)
        for (int redge = 0; redge < 2; ++redge)
            for (int cedge = 0; cedge < 2; ++cedge) {
                uint32_t absent = 0u;
                if (redge) absent |= row_edge_terms(cls);
                if (cedge) absent |= col_edge_terms(cls);
                for (int pat = 0; pat < 32; ++pat) {
                    int64_t x = aq[cls & 1];
                    for (int t = 0; t < 5; ++t) {
                        if ((absent >> t) & 1u) continue;
                        const int64_t w = wq[term_filter(cls, t)];
                        x += ((pat >> t) & 1) ? w : -w;
                    }
                    const int e = ((cls * 2 + redge) * 2 + cedge) * 32 + pat;
                    const uint32_t t = map_threshold(x < 0 ? -x : x);
                    uint32_t tc = (t >> 16) + ((t & 0xffffu) != 0u);
                    tc = tc > 0xffffu ? 0xffffu : tc;
                    out[kHead + e] = tc | (t & 0xffff0000u);
                    out[kHead + kEntries + e] = t;
                    if (x >= 0) out[kHead + 2 * kEntries + e / 32] |= 1u << (e % 32);
                }
            }
    return CRBM_OK;
}

// bonds of filter k that exist on the lattice (App. A Hidden Node Registers:
// Lr/2 x Lc/2 cells, minus those crossing an open edge)
int present_bonds(const crbm_lattice& I, int k) {
    const int Cr = I.rows / 2, Cc = I.cols / 2;
    const bool lose_c = I.open_cols && (k == 1 || k == 3 || k == 9);
    const bool lose_r = I.open_rows && (k == 5 || k == 7 || k == 9);
    return (Cr - (lose_r ? 1 : 0)) * (Cc - (lose_c ? 1 : 0));
}

}  // namespace lat
}  // namespace crbmlib

using namespace crbmlib;
using namespace crbmlib::lat;

struct crbm_lat_s {
    std::vector<crbm_lattice> inst;
    std::vector<std::vector<double>> Texp;
    crbm_config cfg{};
    hipStream_t stream = nullptr;
    int64_t S = 0, cur = 0, total_chains = 0;
    std::vector<int64_t> state_off, spin_off, chain_off, corr_off;
    std::vector<LatItem> items[2];      // by words per row (1, 2)
    LatItem* d_items[2] = {nullptr, nullptr};
    int lds_bytes[2] = {0, 0};
    uint32_t* d_state = nullptr;
    uint32_t* d_tables = nullptr;
    int64_t* d_acc = nullptr;
    unsigned long long* d_corr = nullptr;
    int64_t corr_words = 0;
    ~crbm_lat_s() {
        if (d_state) (void)hipFree(d_state);
        if (d_tables) (void)hipFree(d_tables);
        if (d_acc) (void)hipFree(d_acc);
        if (d_corr) (void)hipFree(d_corr);
        for (int x = 0; x < 2; ++x)
            if (d_items[x]) (void)hipFree(d_items[x]);
    }
};

namespace {

int lfail(int code, const std::string& msg) { return set_error(code, msg.c_str()); }

#define LAT_HIP(expr, what)                                                                   \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return lfail(CRBM_EHIP, std::string(what) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define LAT_ALLOC(expr, what)                                                                 \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return lfail(e_ == hipErrorOutOfMemory ? CRBM_ENOMEM : CRBM_EHIP,                 \
                         std::string(what) + ": " + hipGetErrorString(e_));                   \
    } while (0)

LatArgs lat_args(const crbm_lat_s* h, int x, int64_t s0, int64_t s1, int8_t* spins_out, int32_t* trace,
                 int32_t trace_every) {
    LatArgs a{};
    a.state = h->d_state;
    a.tables = h->d_tables;
    a.items = h->d_items[x];
    a.n_items = (int32_t)h->items[x].size();
    a.measure_every = h->cfg.measure_every;
    a.s0 = s0;
    a.s1 = s1;
    a.burn_in = h->cfg.burn_in;
    a.seed = h->cfg.seed;
    a.acc = h->d_acc;
    a.trace = trace;
    a.trace_every = trace_every;
    a.trace_s0 = s0;
    a.total_chains = h->total_chains;
    a.spins_out = spins_out;
    a.corr = h->d_corr;
    return a;
}

}  // namespace

extern "C" {

int crbm_lattice_create(const crbm_lattice* insts, int32_t n_inst, const crbm_config* cfg, crbm_lat_t** out) {
    set_error(CRBM_OK, "");
    if (!out) return lfail(CRBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!insts || n_inst < 1 || !cfg) return lfail(CRBM_EINVAL, "need at least one instance and a config");
    if (cfg->n_sweeps < 1) return lfail(CRBM_EINVAL, "n_sweeps must be >= 1");
    if (cfg->measure_every < 0 || cfg->burn_in < 0) return lfail(CRBM_EINVAL, "measure_every and burn_in must be >= 0");
    if (cfg->precision != CRBM_PRECISION_Q16) return lfail(CRBM_EUNSUPPORTED, "general lattices use the 16.16 arithmetic");
    if (cfg->n_sweeps > 0xffffffffll) return lfail(CRBM_ERANGE, "n_sweeps must fit the 32-bit sweep counter");
    auto h = std::make_unique<crbm_lat_s>();
    h->cfg = *cfg;
    h->stream = (hipStream_t)cfg->stream;
    h->S = cfg->n_sweeps;
    std::vector<uint32_t> tables;
    std::vector<uint64_t> tab_off(n_inst);
    std::vector<uint32_t> tab_stride(n_inst);
    int64_t words = 0, spins = 0, chains = 0;
    for (int i = 0; i < n_inst; ++i) {
        crbm_lattice I = insts[i];
        const std::string tag = "instance " + std::to_string(i) + ": ";
        if (I.rows < 4 || I.cols < 4 || (I.rows & 1) || (I.cols & 1) || I.rows > CRBM_LAT_MAX_SIDE ||
            I.cols > CRBM_LAT_MAX_SIDE)
            return lfail(CRBM_EINVAL, tag + "rows and cols must be even, 4 .. 64");
        if ((I.open_rows != 0 && I.open_rows != 1) || (I.open_cols != 0 && I.open_cols != 1))
            return lfail(CRBM_EINVAL, tag + "open_rows / open_cols must be 0 or 1");
        if (I.n_chains < 1) return lfail(CRBM_EINVAL, tag + "n_chains must be >= 1");
        if (I.id >= (1u << 29)) return lfail(CRBM_EINVAL, tag + "id must be < 2^29");
        for (int k = 0; k < 10; ++k)
            if (!std::isfinite(I.J[k]) || fabs(I.J[k]) * 65536.0 >= 2147483648.0)
                return lfail(CRBM_EINVAL, tag + "couplings must be finite with |J| 2^16 < 2^31");
        if (!std::isfinite(I.h_even) || !std::isfinite(I.h_odd) || fabs(I.h_even) * 65536.0 >= 2147483648.0 ||
            fabs(I.h_odd) * 65536.0 >= 2147483648.0)
            return lfail(CRBM_EINVAL, tag + "fields must be finite with |h| 2^16 < 2^31");
        if (I.sched_kind < CRBM_SCHED_CONST || I.sched_kind > CRBM_SCHED_EXPLICIT)
            return lfail(CRBM_EINVAL, tag + "unknown schedule");
        std::vector<double> te;
        if (I.sched_kind == CRBM_SCHED_EXPLICIT) {
            if (!I.T_explicit) return lfail(CRBM_EINVAL, tag + "T_explicit is NULL");
            te.assign(I.T_explicit, I.T_explicit + h->S);
            I.T_explicit = nullptr;
        }
        const int64_t n_tab = I.sched_kind == CRBM_SCHED_CONST ? 1 : h->S;
        tab_off[i] = tables.size();
        tab_stride[i] = I.sched_kind == CRBM_SCHED_CONST ? 0u : (uint32_t)kLatTabWords;
        tables.resize(tables.size() + (size_t)n_tab * kLatTabWords);
        for (int64_t s = 0; s < n_tab; ++s) {
            const double T = map_schedule_T(I.sched_kind, I.T0, I.T1, te.empty() ? nullptr : te.data(), h->S, s);
            if (!(T > 0.0) || !std::isfinite(T)) return lfail(CRBM_EINVAL, tag + "temperatures must be finite and > 0");
            if (build_lattice_table(I, T, tables.data() + tab_off[i] + (size_t)s * kLatTabWords) != CRBM_OK)
                return lfail(CRBM_ERANGE, tag + "a field leaves the int32 range at sweep " + std::to_string(s));
        }
        const int W = (I.cols + 31) / 32;
        h->state_off.push_back(words);
        h->spin_off.push_back(spins);
        h->chain_off.push_back(chains);
        for (int64_t c0 = 0; c0 < I.n_chains; c0 += 64) {
            LatItem it{};
            it.id = I.id;
            it.chain0 = (uint32_t)c0;
            it.nchains = (uint32_t)std::min<int64_t>(64, I.n_chains - c0);
            it.tab_stride = tab_stride[i];
            it.gbase = (uint64_t)(chains + c0);
            it.state_off = (uint64_t)(words + c0 * I.rows * W);
            it.spin_off = (uint64_t)(spins + c0 * I.rows * I.cols);
            it.tab_off = tab_off[i];
            it.corr_off = -1;
            it.Lr = I.rows;
            it.Lc = I.cols;
            it.open_r = I.open_rows;
            it.open_c = I.open_cols;
            for (int k = 0; k < 10; ++k) it.np[k] = present_bonds(I, k);
            h->items[W - 1].push_back(it);
        }
        if (cfg->flags & CRBM_F_CORR) {
            h->corr_off.push_back(h->corr_words);
            for (auto& it : h->items[W - 1])
                if (it.gbase >= (uint64_t)chains) it.corr_off = h->corr_words;
            h->corr_words += (int64_t)I.rows * (2 * I.cols - 1);
        }
        words += (int64_t)I.n_chains * I.rows * W;
        spins += (int64_t)I.n_chains * I.rows * I.cols;
        chains += I.n_chains;
        h->lds_bytes[W - 1] = std::max(h->lds_bytes[W - 1], (int)((I.rows * W * 64 + kLatTabWords) * 4));
        h->inst.push_back(I);
        h->Texp.push_back(std::move(te));
    }
    h->total_chains = chains;
    LAT_ALLOC(dev_alloc(&h->d_state, sizeof(uint32_t) * (size_t)words), "hipMalloc state");
    LAT_ALLOC(dev_alloc(&h->d_tables, sizeof(uint32_t) * tables.size()), "hipMalloc tables");
    LAT_ALLOC(dev_alloc(&h->d_acc, sizeof(int64_t) * (size_t)chains * CRBM_LAT_N_ACC), "hipMalloc accumulators");
    LAT_HIP(hipMemcpyAsync(h->d_tables, tables.data(), sizeof(uint32_t) * tables.size(), hipMemcpyHostToDevice,
                           h->stream), "copy tables");
    LAT_HIP(hipMemsetAsync(h->d_acc, 0, sizeof(int64_t) * (size_t)chains * CRBM_LAT_N_ACC, h->stream), "clear accumulators");
    if (h->corr_words > 0) {
        LAT_ALLOC(dev_alloc(&h->d_corr, sizeof(unsigned long long) * (size_t)h->corr_words), "hipMalloc corr");
        LAT_HIP(hipMemsetAsync(h->d_corr, 0, sizeof(unsigned long long) * (size_t)h->corr_words, h->stream), "clear corr");
    }
    for (int x = 0; x < 2; ++x) {
        if (h->items[x].empty()) continue;
        LAT_ALLOC(dev_alloc(&h->d_items[x], sizeof(LatItem) * h->items[x].size()), "hipMalloc items");
        LAT_HIP(hipMemcpyAsync(h->d_items[x], h->items[x].data(), sizeof(LatItem) * h->items[x].size(),
                               hipMemcpyHostToDevice, h->stream), "copy items");
        hipLaunchKernelGGL(lat_init_kernel, dim3((unsigned)h->items[x].size()), dim3(256), 0, h->stream, h->d_state,
                           h->d_items[x], (int)h->items[x].size(), cfg->seed);
        LAT_HIP(hipGetLastError(), "init kernel");
    }
    // the host vectors copied above must outlive the copies
    LAT_HIP(hipStreamSynchronize(h->stream), "create");
    *out = h.release();
    return CRBM_OK;
}

int crbm_lattice_sample(crbm_lat_t* h, int64_t n_sweeps, int8_t* spins_out, int32_t* counts_trace,
                        int32_t trace_every) {
    set_error(CRBM_OK, "");
    if (!h) return lfail(CRBM_EINVAL, "handle is NULL");
    if (n_sweeps < 0) return lfail(CRBM_EINVAL, "n_sweeps must be >= 0");
    if (trace_every < 1 || n_sweeps % trace_every != 0)
        return lfail(CRBM_EINVAL, "trace_every must be >= 1 and divide n_sweeps");
    if (h->cur + n_sweeps > h->S) return lfail(CRBM_ESTATE, "sampling past the end of the schedule");
    for (int x = 0; x < 2; ++x) {
        if (h->items[x].empty()) continue;
        const LatArgs a = lat_args(h, x, h->cur, h->cur + n_sweeps, spins_out, counts_trace, trace_every);
        if (x == 0)
            hipLaunchKernelGGL(lattice_kernel<1>, dim3((unsigned)a.n_items), dim3(64), h->lds_bytes[x], h->stream, a);
        else
            hipLaunchKernelGGL(lattice_kernel<2>, dim3((unsigned)a.n_items), dim3(64), h->lds_bytes[x], h->stream, a);
        LAT_HIP(hipGetLastError(), "lattice kernel");
    }
    h->cur += n_sweeps;
    return CRBM_OK;
}

int crbm_lattice_observables(crbm_lat_t* h, int64_t* acc_out, int64_t* corr_out) {
    set_error(CRBM_OK, "");
    if (!h || !acc_out) return lfail(CRBM_EINVAL, "handle and acc_out must not be NULL");
    if (corr_out && !h->d_corr) return lfail(CRBM_EINVAL, "corr_out needs a handle created with CRBM_F_CORR");
    std::vector<int64_t> acc((size_t)h->total_chains * CRBM_LAT_N_ACC);
    LAT_HIP(hipMemcpyAsync(acc.data(), h->d_acc, sizeof(int64_t) * acc.size(), hipMemcpyDeviceToHost, h->stream),
            "copy accumulators");
    std::vector<unsigned long long> cn((size_t)h->corr_words);
    if (corr_out)
        LAT_HIP(hipMemcpyAsync(cn.data(), h->d_corr, sizeof(unsigned long long) * cn.size(), hipMemcpyDeviceToHost,
                               h->stream), "copy corr");
    LAT_HIP(hipStreamSynchronize(h->stream), "observables");
    for (size_t i = 0; i < h->inst.size(); ++i) {
        int64_t* o = acc_out + i * CRBM_LAT_N_ACC;
        for (int q = 0; q < CRBM_LAT_N_ACC; ++q) o[q] = 0;
        for (int64_t c = 0; c < h->inst[i].n_chains; ++c)
            for (int q = 0; q < CRBM_LAT_N_ACC; ++q) o[q] += acc[(size_t)(h->chain_off[i] + c) * CRBM_LAT_N_ACC + q];
    }
    if (corr_out)
        for (int64_t x = 0; x < h->corr_words; ++x) corr_out[x] = (int64_t)cn[x];
    return CRBM_OK;
}

int crbm_lattice_reset_observables(crbm_lat_t* h) {
    set_error(CRBM_OK, "");
    if (!h) return lfail(CRBM_EINVAL, "handle is NULL");
    LAT_HIP(hipMemsetAsync(h->d_acc, 0, sizeof(int64_t) * (size_t)h->total_chains * CRBM_LAT_N_ACC, h->stream),
            "clear accumulators");
    if (h->d_corr)
        LAT_HIP(hipMemsetAsync(h->d_corr, 0, sizeof(unsigned long long) * (size_t)h->corr_words, h->stream),
                "clear corr");
    return CRBM_OK;
}

int crbm_lattice_get_state(crbm_lat_t* h, int8_t* spins_dev, int64_t* sweep_index) {
    set_error(CRBM_OK, "");
    if (!h) return lfail(CRBM_EINVAL, "handle is NULL");
    if (spins_dev)
        for (size_t i = 0; i < h->inst.size(); ++i) {
            const crbm_lattice& I = h->inst[i];
            const int64_t nrows = (int64_t)I.n_chains * I.rows;
            hipLaunchKernelGGL(lat_unpack_kernel, dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0, h->stream,
                               h->d_state + h->state_off[i], spins_dev + h->spin_off[i], nrows, I.cols);
            LAT_HIP(hipGetLastError(), "unpack kernel");
        }
    LAT_HIP(hipStreamSynchronize(h->stream), "get_state");
    if (sweep_index) *sweep_index = h->cur;
    return CRBM_OK;
}

int crbm_lattice_set_state(crbm_lat_t* h, const int8_t* spins_dev, int64_t sweep_index) {
    set_error(CRBM_OK, "");
    if (!h) return lfail(CRBM_EINVAL, "handle is NULL");
    if (sweep_index < 0 || sweep_index > h->S) return lfail(CRBM_EINVAL, "sweep_index outside the schedule");
    if (spins_dev)
        for (size_t i = 0; i < h->inst.size(); ++i) {
            const crbm_lattice& I = h->inst[i];
            const int64_t nrows = (int64_t)I.n_chains * I.rows;
            hipLaunchKernelGGL(lat_pack_kernel, dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0, h->stream,
                               h->d_state + h->state_off[i], spins_dev + h->spin_off[i], nrows, I.cols);
            LAT_HIP(hipGetLastError(), "pack kernel");
        }
    h->cur = sweep_index;
    return CRBM_OK;
}

int64_t crbm_lattice_total_chains(const crbm_lat_t* h) { return h ? h->total_chains : 0; }

void crbm_lattice_destroy(crbm_lat_t* h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    delete h;
}

int crbm_lattice_table(const crbm_lattice* inst, double T, uint32_t* out) {
    set_error(CRBM_OK, "");
    if (!inst || !out) return lfail(CRBM_EINVAL, "inst and out must not be NULL");
    if (!(T > 0.0) || !std::isfinite(T)) return lfail(CRBM_EINVAL, "T must be finite and > 0");
    if (build_lattice_table(*inst, T, out) != CRBM_OK) return lfail(CRBM_ERANGE, "a field leaves the int32 range");
    return CRBM_OK;
}

}  // extern "C"
