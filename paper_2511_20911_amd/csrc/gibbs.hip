// gibbs.hip -- gfx950 kernels for block Gibbs sampling of the CRBM that
// encodes the classical Shastry-Sutherland Ising lattice
// (Brahma et al., arXiv 2511.20911, Sec. II.A-II.B, App. A).
//
// Layout and mapping
//   * A chain's spins are bit rows: one 32-bit word per lattice row
//     (bit c = column c, 1 = up), L <= 32.
//   * A chain is handled by G = (L/2)/R lanes of one wavefront; lane g owns the
//     band of cell rows g*R .. g*R+R-1 (visible rows 2gR .. 2gR+2R-1) and keeps
//     it in registers for the whole launch.  64/G chains share a wavefront;
//     all chains of a wavefront belong to one instance, so the per-sweep
//     weight/threshold table is wavefront-uniform.
//   * Hidden units are never stored: a cell row's 10 hidden planes (one bit per
//     cell, at even bit positions) are drawn from the old spins and consumed
//     at once by the visible update of the rows that need them.  The first
//     row of a band also needs the previous lane's last hidden row; it is
//     updated last, after a lane shuffle (App. A Zero Padder: the periodic
//     copy of the last hidden row).
//
// Per unit (Sec. II.B Eqs. (11)-(12) with +-1 units):
//   hidden: the bond "agrees" if s_a == sig_t s_b; then its field is
//           2 wq s_a, otherwise 0.  The unit takes the field's sign s with
//           probability t(|x|)/2^32: h = s unless U >= t.
//   spin:   field = aq + wq1 (2n - 4) + wq2 (2d - 1), with n the number of J1
//           terms (coef * h) equal to +1 and d the dimer term; n is summed
//           bit-sliced over a whole row, the threshold is looked up by
//           (n, d) from a 10-entry table held one entry per lane.
//   U = (P << 16) | Q with P, Q 16-bit Philox4x32-10 slots.  The kernel
//   compares P against the threshold's top half and only draws Q when P
//   equals it (probability 2^-16): the decision equals the full 32-bit one.
#include "crbm_internal.h"

namespace crbmlib {
namespace {

constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;  // Philox round multipliers
constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;  // Philox key increments

struct P4 {
    uint32_t v[4];
};

// Philox4x32-10 (Salmon et al., SC'11).
__device__ __forceinline__ P4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)kM0 * c0;
        const uint64_t p1 = (uint64_t)kM1 * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += kW0;
        k1 += kW1;
    }
    return P4{{c0, c1, c2, c3}};
}

// 16-bit slot s (0..7) of a Philox block.
__device__ __forceinline__ uint32_t slot16(const P4& p, int s) {
    const uint32_t w = p.v[s >> 1];
    return (s & 1) ? (w >> 16) : (w & 0xffffu);
}

template <int L>
struct Lat {
    static constexpr int C = L / 2;
    static constexpr uint32_t FULL = (L == 32) ? 0xffffffffu : ((1u << L) - 1u);
    static constexpr uint32_t EVEN = 0x55555555u & FULL;
    // bit c <- column c + n (mod L)
    __device__ static __forceinline__ uint32_t r1(uint32_t x) { return ((x >> 1) | (x << (L - 1))) & FULL; }
    __device__ static __forceinline__ uint32_t r2(uint32_t x) { return ((x >> 2) | (x << (L - 2))) & FULL; }
    // bit c <- column c - 2 (mod L)
    __device__ static __forceinline__ uint32_t l2(uint32_t x) { return ((x << 2) | (x >> (L - 2))) & FULL; }
};

// Wavefront-uniform constants of one sweep, plus the per-lane visible table.
struct SweepK {
    uint32_t T[2];      // hidden agree thresholds (J1, J2)
    uint32_t tceil[2];  // P >= tceil <=> U >= T, unless P == thi
    uint32_t thi[2];    // top half of T, or 0x10000 when the bottom half is 0 (no tie possible)
    uint32_t neg[2];    // EVEN if sig_t < 0
    uint32_t en[2];     // EVEN if wq_t != 0
    uint32_t kge[2];    // spin field >= 0 iff n >= kge[d]
    uint32_t tabv;      // lane l < 10: min(tceil,0xffff) | thi << 16 of visible entry l
    uint32_t tfull;     // lane l < 10: full visible threshold of entry l
};

template <int L>
__device__ __forceinline__ SweepK load_sweep(const uint32_t* tb, int lane) {
    using Lt = Lat<L>;
    SweepK K;
    const uint32_t fl = tb[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const uint32_t T = tb[t];
        K.T[t] = T;
        K.tceil[t] = (T >> 16) + ((T & 0xffffu) != 0u);
        K.thi[t] = (T & 0xffffu) ? (T >> 16) : 0x10000u;
        K.neg[t] = (fl & (1u << t)) ? Lt::EVEN : 0u;
        K.en[t] = (fl & (4u << t)) ? Lt::EVEN : 0u;
        K.kge[t] = (fl >> (8 + 4 * t)) & 15u;
    }
    const uint32_t tv = tb[3 + (lane < 10 ? lane : 9)];
    uint32_t tc = (tv >> 16) + ((tv & 0xffffu) != 0u);
    tc = tc > 0xffffu ? 0xffffu : tc;
    K.tfull = tv;
    K.tabv = tc | (tv & 0xffff0000u);
    return K;
}

// Uniform select / update of one of N registers by a wavefront-uniform index.
template <int N>
__device__ __forceinline__ uint32_t pick(const uint32_t (&a)[N], int k) {
    uint32_t v = a[0];
#pragma unroll
    for (int x = 1; x < N; ++x) v = (k == x) ? a[x] : v;
    return v;
}
template <int N>
__device__ __forceinline__ void put(uint32_t (&a)[N], int k, uint32_t v) {
#pragma unroll
    for (int x = 0; x < N; ++x) a[x] = (k == x) ? v : a[x];
}

struct Rng {
    uint32_t sweep, chain, k0, k1;
};

// Hidden half-step of one cell row (Eq. (11)): 10 hidden planes from the old
// spin rows top = 2i, mid = 2i+1, bot = 2i+2.
template <int L>
__device__ __forceinline__ void hidden_row(uint32_t top, uint32_t mid, uint32_t bot, const SweepK& K,
                                           uint32_t cbase, uint32_t c3p, const Rng& rg,
                                           uint32_t (&H)[10]) {
    using Lt = Lat<L>;
    constexpr int C = Lt::C;
    constexpr int NQ = 10 * C;
    constexpr int NB = (NQ + 7) / 8;
    const uint32_t t1 = Lt::r1(top), t2 = Lt::r2(top), m1 = Lt::r1(mid), m2 = Lt::r2(mid), b1 = Lt::r1(bot);
    // endpoint a and endpoint b of each filter, aligned on the cell's even column
    const uint32_t ea[10] = {top, t1, mid, m1, top, mid, t1, m1, top, m2};
    const uint32_t eb[10] = {t1, t2, m1, m2, mid, bot, m1, b1, m1, b1};
    uint32_t A[10], D[10], CA[10], CT[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        const int ty = k >= 8;
        A[k] = ~(ea[k] ^ eb[k] ^ K.neg[ty]) & K.en[ty];
        CA[k] = 0u;
        CT[k] = 0u;
    }
    uint32_t tieblk = 0u;
#pragma unroll
    for (int blk = 0; blk < NB; ++blk) {
        const P4 p = philox(cbase | (uint32_t)blk, rg.sweep, rg.chain, c3p, rg.k0, rg.k1);
        uint64_t tie = 0;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int q = blk * 8 + s;
            if (q < NQ) {
                const int k = q / C, pos = 2 * (q % C), ty = k >= 8;
                const uint32_t p16 = slot16(p, s);
                CA[k] |= (uint32_t)(p16 >= K.tceil[ty]) << pos;
                CT[k] |= (p16 >> 15) << pos;
                tie |= __ballot(p16 == K.thi[ty]);
            }
        }
        if (tie) tieblk |= 1u << blk;
    }
#pragma unroll
    for (int k = 0; k < 10; ++k) D[k] = (CA[k] & A[k]) | (CT[k] & ~A[k]);
    // Rare path: a primary slot equal to the threshold's top half; redo the
    // affected blocks with the refinement stream and exact 32-bit compares.
    while (tieblk) {
        const int blk = __builtin_ctz(tieblk);
        tieblk &= tieblk - 1u;
        const P4 p = philox(cbase | (uint32_t)blk, rg.sweep, rg.chain, c3p, rg.k0, rg.k1);
        const P4 r = philox(cbase | (uint32_t)blk, rg.sweep, rg.chain, c3p + 1u, rg.k0, rg.k1);
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int q = blk * 8 + s;
            if (q < NQ) {
                const int k = q / C, pos = 2 * (q % C), ty = k >= 8;
                const uint32_t U = (slot16(p, s) << 16) | slot16(r, s);
                const uint32_t ag = (pick(A, k) >> pos) & 1u;
                const uint32_t th = ag ? K.T[ty] : 0x80000000u;
                const uint32_t d = U >= th;
                const uint32_t Dk = (pick(D, k) & ~(1u << pos)) | (d << pos);
                put(D, k, Dk);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        const int ty = k >= 8;
        const uint32_t S = ((ea[k] & A[k]) | ~A[k]) & Lt::EVEN;  // field sign (+1 when the field is 0)
        H[k] = S ^ D[k];
        (void)ty;
    }
}

// n >= k for a bit-sliced count n = n0 + 2 n1 + 4 n2 in 0..4 and uniform k.
__device__ __forceinline__ uint32_t count_ge(uint32_t n0, uint32_t n1, uint32_t n2, uint32_t k) {
    switch (k) {
        case 0: return 0xffffffffu;
        case 1: return n0 | n1 | n2;
        case 2: return n1 | n2;
        case 3: return n2 | (n1 & n0);
        case 4: return n2;
        default: return 0u;
    }
}

// Visible half-step of the two rows of one cell row (Eq. (12)).
// H: hidden planes of this cell row; Hp5/Hp7/Hp9: planes 5, 7, 9 of the cell
// row above.  Classes: 0 top even, 1 top odd, 2 mid even, 3 mid odd columns.
template <int L>
__device__ __forceinline__ void visible_row(const uint32_t (&H)[10], uint32_t Hp5, uint32_t Hp7, uint32_t Hp9,
                                            const SweepK& K, bool do_top, bool do_mid, uint32_t cbase,
                                            uint32_t c3p, const Rng& rg, uint32_t& ntop, uint32_t& nmid) {
    using Lt = Lat<L>;
    constexpr int NQ = 2 * L;
    constexpr int NB = (NQ + 7) / 8;
    const uint32_t n1 = K.neg[0], n2 = K.neg[1], E = Lt::EVEN;
    // the 4 J1 terms and the dimer term of every site (1 = +1), cf. the bond table
    const uint32_t term[4][5] = {
        {H[0], H[4], Lt::l2(H[1]) ^ n1, Hp5 ^ n1, H[8]},          // (0,0): k0a k4a k1b(j-1) k5b(i-1) | k8a
        {H[0] ^ n1, H[1], H[6], Hp7 ^ n1, Hp9 ^ n2},             // (0,1): k0b k1a k6a k7b(i-1) | k9b(i-1)
        {H[2], H[4] ^ n1, H[5], Lt::l2(H[3]) ^ n1, Lt::l2(H[9])}, // (1,0): k2a k4b k5a k3b(j-1) | k9a(j-1)
        {H[2] ^ n1, H[3], H[6] ^ n1, H[7], H[8] ^ n2},            // (1,1): k2b k3a k6b k7a | k8b
    };
    uint32_t Pa[4], Pb[4], Sg[4], D[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const uint32_t s1 = term[c][0] ^ term[c][1], c1 = term[c][0] & term[c][1];
        const uint32_t s2 = term[c][2] ^ term[c][3], c2 = term[c][2] & term[c][3];
        const uint32_t b0 = (s1 ^ s2) & E, cc = s1 & s2;
        const uint32_t b1 = (c1 ^ c2 ^ cc) & E, b2 = (c1 & c2) & E;
        const uint32_t dd = term[c][4] & E;
        Pa[c] = dd | (b0 << 1);
        Pb[c] = b1 | (b2 << 1);
        Sg[c] = ((dd & count_ge(b0, b1, b2, K.kge[1])) | (~dd & count_ge(b0, b1, b2, K.kge[0]))) & E;
        D[c] = 0u;
    }
    uint32_t tieblk = 0u;
#pragma unroll
    for (int blk = 0; blk < NB; ++blk) {
        const bool has_top = blk * 8 < L, has_mid = blk * 8 + 7 >= L;
        if (!((do_top && has_top) || (do_mid && has_mid))) continue;
        const P4 p = philox(cbase | (uint32_t)blk, rg.sweep, rg.chain, c3p, rg.k0, rg.k1);
        uint64_t tie = 0;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int q = blk * 8 + s;
            if (q < NQ) {
                const int row = q / L, col = q % L, cls = 2 * row + (col & 1), pos = col & ~1;
                const uint32_t p16 = slot16(p, s);
                const uint32_t idx = ((Pa[cls] >> pos) & 3u) | (((Pb[cls] >> pos) & 3u) << 2);
                const uint32_t e = __shfl(K.tabv, (int)idx);
                D[cls] |= (uint32_t)(p16 >= (e & 0xffffu)) << pos;
                tie |= __ballot(p16 == (e >> 16));
            }
        }
        if (tie) tieblk |= 1u << blk;
    }
    while (tieblk) {
        const int blk = __builtin_ctz(tieblk);
        tieblk &= tieblk - 1u;
        const P4 p = philox(cbase | (uint32_t)blk, rg.sweep, rg.chain, c3p, rg.k0, rg.k1);
        const P4 r = philox(cbase | (uint32_t)blk, rg.sweep, rg.chain, c3p + 1u, rg.k0, rg.k1);
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int q = blk * 8 + s;
            if (q < NQ) {
                const int row = q / L, col = q % L, cls = 2 * row + (col & 1), pos = col & ~1;
                const uint32_t U = (slot16(p, s) << 16) | slot16(r, s);
                const uint32_t idx = ((pick(Pa, cls) >> pos) & 3u) | (((pick(Pb, cls) >> pos) & 3u) << 2);
                const uint32_t t = __shfl(K.tfull, (int)idx);
                const uint32_t d = U >= t;
                put(D, cls, (pick(D, cls) & ~(1u << pos)) | (d << pos));
            }
        }
    }
    ntop = (Sg[0] ^ D[0]) | ((Sg[1] ^ D[1]) << 1);
    nmid = (Sg[2] ^ D[2]) | ((Sg[3] ^ D[3]) << 1);
}

template <int L, int R>
__global__ void __launch_bounds__(256) gibbs_kernel(GibbsArgs a) {
    using Lt = Lat<L>;
    constexpr int C = L / 2;
    constexpr int G = C / R;
    constexpr int NR = 2 * R;
    constexpr int N = L * L;
    static_assert(C % R == 0, "R must divide L/2");
    static_assert(G <= 64, "a chain must fit in one wavefront");

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    if (wv >= a.n_items) return;
    const Item it = a.items[wv];
    const int cl = lane / G, g = lane - cl * G;
    const bool active = cl < (int)it.nchains;
    const uint32_t chain = it.chain0 + (active ? (uint32_t)cl : 0u);
    const uint64_t gch = it.gbase + (active ? (uint64_t)cl : 0u);
    const int nxt = cl * G + (g + 1 == G ? 0 : g + 1);
    const int prv = cl * G + (g == 0 ? G - 1 : g - 1);

    uint32_t Q[NR + 1];
    {
        const uint32_t* st = a.state + it.state_off + (uint64_t)(active ? cl : 0) * L + (uint64_t)g * NR;
#pragma unroll
        for (int x = 0; x < NR; ++x) Q[x] = st[x];
        Q[NR] = 0u;
    }
    const uint32_t c3h = (it.id << 3) | 1u, c3v = (it.id << 3) | 3u;
    int64_t acc[11];
#pragma unroll
    for (int x = 0; x < 11; ++x) acc[x] = 0;

    for (int64_t s = a.s0; s < a.s1; ++s) {
        const uint32_t* tb = a.tables + it.tab_off + (uint64_t)it.tab_stride * (uint64_t)s;
        const SweepK K = load_sweep<L>(tb, lane);
        const Rng rg{(uint32_t)s, chain, (uint32_t)a.seed, (uint32_t)(a.seed >> 32)};
        Q[NR] = __shfl(Q[0], nxt);  // old first row of the next band
        uint32_t Hf0 = 0, Hf1 = 0, Hf4 = 0, Hf6 = 0, Hf8 = 0, Hp5 = 0, Hp7 = 0, Hp9 = 0;
#pragma unroll 1
        for (int m = 0; m < R; ++m) {
            const uint32_t cbase = (uint32_t)(g * R + m) << 5;
            uint32_t H[10];
            hidden_row<L>(Q[0], Q[1], Q[2], K, cbase, c3h, rg, H);
            uint32_t nt, nm;
            visible_row<L>(H, Hp5, Hp7, Hp9, K, m > 0, true, cbase, c3v, rg, nt, nm);
            const uint32_t old_top = Q[0];
#pragma unroll
            for (int x = 0; x + 2 <= NR; ++x) Q[x] = Q[x + 2];
            Q[NR - 1] = (m == 0) ? old_top : nt;
            Q[NR] = nm;
            if (m == 0) {
                Hf0 = H[0]; Hf1 = H[1]; Hf4 = H[4]; Hf6 = H[6]; Hf8 = H[8];
            }
            Hp5 = H[5]; Hp7 = H[7]; Hp9 = H[9];
        }
        // first row of the band: needs the last hidden row of the previous band
        Hp5 = __shfl(Hp5, prv);
        Hp7 = __shfl(Hp7, prv);
        Hp9 = __shfl(Hp9, prv);
        {
            const uint32_t Hd[10] = {Hf0, Hf1, 0u, 0u, Hf4, 0u, Hf6, 0u, Hf8, 0u};
            uint32_t nt, nm;
            visible_row<L>(Hd, Hp5, Hp7, Hp9, K, true, false, (uint32_t)(g * R) << 5, c3v, rg, nt, nm);
            Q[1] = nt;
        }
#pragma unroll
        for (int x = 0; x < NR; ++x) Q[x] = Q[x + 1];

        const bool meas = a.measure_every > 0 && s >= a.burn_in && ((s - a.burn_in) % a.measure_every) == 0;
        if (meas || a.trace) {
            const uint32_t nb = __shfl(Q[0], nxt);  // new first row of the next band
            int pop = 0, dis1 = 0, dis2 = 0;
#pragma unroll
            for (int x = 0; x < NR; ++x) {
                const uint32_t r = Q[x], below = (x + 1 < NR) ? Q[x + 1] : nb;
                pop += __popc(r);
                dis1 += __popc(r ^ Lt::r1(r)) + __popc(r ^ below);
            }
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const uint32_t top = Q[2 * m], mid = Q[2 * m + 1], bot = (2 * m + 2 < NR) ? Q[2 * m + 2] : nb;
                dis2 += __popc((top ^ Lt::r1(mid)) & Lt::EVEN) + __popc((Lt::r2(mid) ^ Lt::r1(bot)) & Lt::EVEN);
            }
            int tp = pop, t1 = dis1, t2 = dis2;
#pragma unroll
            for (int d = 1; d < G; ++d) {
                const int src = cl * G + (g + d) % G;
                tp += __shfl(pop, src);
                t1 += __shfl(dis1, src);
                t2 += __shfl(dis2, src);
            }
            const int64_t M = 2 * tp - N, B1 = 2 * N - 2 * t1, B2 = N / 2 - 2 * t2;
            if (a.trace && g == 0 && active) {
                int32_t* tr = a.trace + ((uint64_t)(s - a.s0) * (uint64_t)a.total_chains + gch) * 3;
                tr[0] = (int32_t)M;
                tr[1] = (int32_t)B1;
                tr[2] = (int32_t)B2;
            }
            if (meas) {
                acc[0] += 1;
                acc[1] += M; acc[2] += B1; acc[3] += B2;
                acc[4] += M * M; acc[5] += B1 * B1; acc[6] += B2 * B2;
                acc[7] += M * B1; acc[8] += M * B2; acc[9] += B1 * B2;
                acc[10] += M < 0 ? -M : M;
            }
        }
    }
    if (!active) return;
    {
        uint32_t* st = a.state + it.state_off + (uint64_t)cl * L + (uint64_t)g * NR;
#pragma unroll
        for (int x = 0; x < NR; ++x) st[x] = Q[x];
    }
    if (g == 0 && a.measure_every > 0) {
        int64_t* ac = a.acc + gch * 11;
#pragma unroll
        for (int x = 0; x < 11; ++x) ac[x] += acc[x];
    }
    if (a.spins_out) {
        int8_t* out = a.spins_out + it.spin_off + ((uint64_t)cl * L + (uint64_t)g * NR) * L;
        for (int x = 0; x < NR; ++x)
            for (int c = 0; c < L; ++c) out[x * L + c] = ((Q[x] >> c) & 1u) ? 1 : -1;
    }
}

// Seeded initial state (stream 0): spin (r,c) is up iff bit (rL+c) & 127 of
// the Philox block with counter word (rL+c) >> 7 is set.
__global__ void init_kernel(uint32_t* state, const Item* items, int n_items, int L, int cpw, uint64_t seed) {
    const int lane = threadIdx.x & 63;
    const int wv = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (wv >= n_items) return;
    const Item it = items[wv];
    if (lane >= (int)it.nchains) return;
    const uint32_t chain = it.chain0 + lane;
    uint32_t* rows = state + it.state_off + (uint64_t)lane * L;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    uint32_t cur = 0xffffffffu;
    P4 p{};
    for (int r = 0; r < L; ++r) {
        uint32_t row = 0u;
        for (int c = 0; c < L; ++c) {
            const uint32_t site = (uint32_t)(r * L + c);
            if ((site >> 7) != cur) {
                cur = site >> 7;
                p = philox(cur, 0u, chain, it.id << 3, k0, k1);
            }
            const uint32_t b = site & 127u;
            row |= ((p.v[b >> 5] >> (b & 31u)) & 1u) << c;
        }
        rows[r] = row;
    }
    (void)cpw;
}

__global__ void pack_kernel(uint32_t* state, const int8_t* spins, int64_t nrows, int L) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrows) return;
    const int8_t* s = spins + t * L;
    uint32_t row = 0u;
    for (int c = 0; c < L; ++c) row |= (s[c] > 0 ? 1u : 0u) << c;
    state[t] = row;
}

__global__ void unpack_kernel(const uint32_t* state, int8_t* spins, int64_t nrows, int L) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrows) return;
    const uint32_t row = state[t];
    int8_t* s = spins + t * L;
    for (int c = 0; c < L; ++c) s[c] = ((row >> c) & 1u) ? 1 : -1;
}

// C(dr, dc) = sum_{r,c} s(r,c) s(r+dr, c+dc) summed over a block of chains of
// one instance in LDS, then added to the instance's int64 total.
__global__ void __launch_bounds__(256) corr_kernel(const uint32_t* state, int64_t nchains, int L,
                                                   unsigned long long* corr) {
    __shared__ int part[32 * 32];
    const int N = L * L;
    for (int x = threadIdx.x; x < N; x += blockDim.x) part[x] = 0;
    __syncthreads();
    const int64_t ch = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (ch < nchains) {
        const uint32_t* rows = state + ch * L;
        const uint32_t full = (L == 32) ? 0xffffffffu : ((1u << L) - 1u);
        for (int dr = 0; dr < L; ++dr)
            for (int dc = 0; dc < L; ++dc) {
                int dis = 0;
                for (int r = 0; r < L; ++r) {
                    const uint32_t x = rows[r];
                    uint32_t y = rows[(r + dr) % L];
                    if (dc) y = ((y >> dc) | (y << (L - dc))) & full;
                    dis += __popc(x ^ y);
                }
                atomicAdd(&part[dr * L + dc], N - 2 * dis);
            }
    }
    __syncthreads();
    for (int x = threadIdx.x; x < N; x += blockDim.x)
        atomicAdd(&corr[x], (unsigned long long)(long long)part[x]);
}

template <int L, int R>
hipError_t launch_one(const GibbsArgs& a, hipStream_t st) {
    const int waves_per_block = 4;
    const int blocks = (a.n_items + waves_per_block - 1) / waves_per_block;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL((gibbs_kernel<L, R>), dim3(blocks), dim3(64 * waves_per_block), 0, st, a);
    return hipGetLastError();
}

}  // namespace

// (L, R) pairs with a compiled kernel: R cell rows per lane, R | L/2.
#define CRBM_FOR_EACH_TILE(X) \
    X(4, 1) X(4, 2) X(6, 1) X(6, 3) X(8, 1) X(8, 2) X(8, 4) X(10, 1) X(10, 5) X(12, 1) X(12, 2) X(12, 3) \
    X(12, 6) X(14, 1) X(14, 7) X(16, 1) X(16, 2) X(16, 4) X(16, 8) X(18, 1) X(18, 3) X(18, 9) X(20, 1) \
    X(20, 2) X(20, 5) X(20, 10) X(22, 1) X(22, 11) X(24, 1) X(24, 2) X(24, 3) X(24, 4) X(24, 6) X(24, 12) \
    X(26, 1) X(26, 13) X(28, 1) X(28, 2) X(28, 7) X(28, 14) X(30, 1) X(30, 3) X(30, 5) X(30, 15) X(32, 1) \
    X(32, 2) X(32, 4) X(32, 8) X(32, 16)

bool gibbs_supported(int L, int R) {
#define CRBM_CASE(l, r) if (L == l && R == r) return true;
    CRBM_FOR_EACH_TILE(CRBM_CASE)
#undef CRBM_CASE
    return false;
}

hipError_t launch_gibbs(int L, int R, const GibbsArgs& a, hipStream_t st) {
#define CRBM_CASE(l, r) if (L == l && R == r) return launch_one<l, r>(a, st);
    CRBM_FOR_EACH_TILE(CRBM_CASE)
#undef CRBM_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_init(uint32_t* state, const Item* items, int n_items, int L, int R, uint64_t seed,
                       hipStream_t st) {
    const int blocks = (n_items + 3) / 4;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(init_kernel, dim3(blocks), dim3(256), 0, st, state, items, n_items, L,
                       chains_per_wave(L, R), seed);
    return hipGetLastError();
}

hipError_t launch_pack(uint32_t* state, const int8_t* spins, int64_t nchains, int L, hipStream_t st) {
    const int64_t nrows = nchains * L;
    if (nrows == 0) return hipSuccess;
    hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0, st, state, spins,
                       nrows, L);
    return hipGetLastError();
}

hipError_t launch_unpack(const uint32_t* state, int8_t* spins, int64_t nchains, int L, hipStream_t st) {
    const int64_t nrows = nchains * L;
    if (nrows == 0) return hipSuccess;
    hipLaunchKernelGGL(unpack_kernel, dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0, st, state,
                       spins, nrows, L);
    return hipGetLastError();
}

hipError_t launch_corr(const uint32_t* state, int64_t nchains, int L, unsigned long long* corr,
                       hipStream_t st) {
    if (nchains == 0) return hipSuccess;
    hipLaunchKernelGGL(corr_kernel, dim3((unsigned)((nchains + 255) / 256)), dim3(256), 0, st, state,
                       nchains, L, corr);
    return hipGetLastError();
}

}  // namespace crbmlib
