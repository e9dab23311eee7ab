// ar.hip -- learned proposal for independent Metropolis-Hastings: a masked-
// convolution autoregressive network over the spins in raster order, with
// bf16 matrix-core (MFMA) kernels accumulating in fp32 for training and for
// sequential sampling / scoring, and the MH accept step on exact integer
// energies so the chain keeps the CRBM's stationary law.  (The paper samples
// its CRBM by Gibbs only, Sec. II.B; this proposal is an addition on top.)
//
// Network: C = 32 channels, 12 layers of 3x3 masked convolutions, zero
// padding.  Layer 1 uses mask A (the 4 sites before the centre in raster
// order), layers 2-12 mask B (plus the centre).  Layers 2-11 are residual,
// h_l = bf16(h_{l-1} + relu(z_l)); layer 12 gives one logit per site.
// Training fits log sigmoid(s_i logit_i) per site.  The proposal draws each
// spin by an integer compare whose probability is exactly representable: with
// t(x) = clamp(rint(2^32 sigmoid(-|x|)), 1, 2^31) the probability of the
// value against the sign of the logit x (the minority value; +1 counts as the
// sign of 0), the spin is +1 iff a 32-bit uniform u < t_up(x), t_up = 2^32 - t
// for x >= 0 and t for x < 0 (monotone in x), so P(minority) = t / 2^32
// exactly, and log q(s) sums the logs of exactly these probabilities.  The Metropolis-Hastings ratio then uses the probability of
// the proposal that was really drawn, at every logit, however confident.
//
// Layouts: activations [pixel][32] bf16 (pixel = (b L + r) L + c), channel
// dimension padded to 32 for the 1-channel input and output; weights per layer
// and tap as 32x32 bf16 blocks, "fwd" [tap][cout][cin] (matrix-core B operand
// for the forward conv) and "bwd" [tap][cin][cout] (for the data gradient).
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "crbm.h"
#include "crbm_internal.h"
#include "gibbs_kernel.h"

namespace crbmlib {
namespace ar {

constexpr int C = 32;
constexpr int NL = 12;
constexpr int NT = 5;  // taps per layer (mask A uses the first 4)
// conditioning MLP: features -> hidden (tanh) -> one bias offset per layer and channel
constexpr int kCondF = 3, kCondH = 32, kCondOut = NL * C;
constexpr int kCondMaxPoints = 128;

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

struct Taps {
    int n;
    int dr[NT], dc[NT];
};

// Mask A / B taps; "mirrored" taps (negated) give the adjoint convolution.
inline Taps taps_for(int layer, bool mirrored) {
    const int dr[NT] = {-1, -1, -1, 0, 0};
    const int dc[NT] = {-1, 0, 1, -1, 0};
    Taps t{};
    t.n = (layer == 0) ? 4 : 5;
    for (int k = 0; k < t.n; ++k) {
        t.dr[k] = mirrored ? -dr[k] : dr[k];
        t.dc[k] = mirrored ? -dc[k] : dc[k];
    }
    return t;
}

__device__ __forceinline__ Taps taps_for_dev(int layer) {
    Taps t;
    t.n = (layer == 0) ? 4 : 5;
    t.dr[0] = -1; t.dc[0] = -1;
    t.dr[1] = -1; t.dc[1] = 0;
    t.dr[2] = -1; t.dc[2] = 1;
    t.dr[3] = 0;  t.dc[3] = -1;
    t.dr[4] = 0;  t.dc[4] = 0;
    return t;
}

__device__ __forceinline__ float bf2f(__bf16 x) { return (float)x; }
__device__ __forceinline__ __bf16 f2bf(float x) { return (__bf16)x; }  // round to nearest even

__device__ __forceinline__ bf16x8 load8(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }
__device__ __forceinline__ bf16x8 zero8() {
    bf16x8 z;
#pragma unroll
    for (int e = 0; e < 8; ++e) z[e] = (__bf16)0.0f;
    return z;
}

// Which neighbours pixel p (p < 2^31, checked on the host) of a batch of
// L x L lattices has inside its own lattice: bit 0 the row above, bit 1 the
// row below, bit 2 the column to the left, bit 3 the column to the right.
// Two 32-bit divisions, once per pixel; only this one word stays live.
__device__ __forceinline__ uint32_t edge_flags(int64_t p, int L) {
    const uint32_t pu = (uint32_t)p, LL = (uint32_t)(L * L);
    const uint32_t rc = pu - (pu / LL) * LL, r = rc / (uint32_t)L, c = rc - r * (uint32_t)L;
    const uint32_t last = (uint32_t)L - 1u;
    return (uint32_t)(r > 0u) | ((uint32_t)(r < last) << 1) | ((uint32_t)(c > 0u) << 2) | ((uint32_t)(c < last) << 3);
}

// Neighbour of pixel p shifted by (dr, dc), |dr|, |dc| <= 1 (3 x 3 taps),
// inside the same lattice, or -1; f = edge_flags(p, L).
__device__ __forceinline__ int64_t shift_pix(int64_t p, uint32_t f, int dr, int dc, int L) {
    const uint32_t need = (dr < 0 ? 1u : 0u) | (dr > 0 ? 2u : 0u) | (dc < 0 ? 4u : 0u) | (dc > 0 ? 8u : 0u);
    return (f & need) == need ? p + (int64_t)(dr * L + dc) : -1;
}

// Minority threshold of a site with logit x (fp32 arithmetic): the value
// against the sign of x has probability t / 2^32, t = clamp(rint(2^32
// sigmoid(-|x|)), 1, 2^31).  p 2^32 is exact (a power-of-two scale), so the
// rounding is the only one after the sigmoid.  NaN gives t = 1.
__device__ __forceinline__ uint32_t minority_threshold(float x) {
    const float e = expf(-fabsf(x));
    const float p = e / (1.0f + e);
    const float t = fminf(fmaxf(rintf(p * 4294967296.0f), 1.0f), 2147483648.0f);
    return (uint32_t)t;
}

// The spin is +1 iff its 32-bit uniform is below this: 2^32 - t for x >= 0,
// t for x < 0 (monotone in x, 2^31 at x = 0 from both sides).
__device__ __forceinline__ uint32_t up_threshold(float x) {
    const uint32_t t = minority_threshold(x);
    return x >= 0.0f ? 0u - t : t;
}

// log of the probability with which the proposal drew spin s (+-1) at a site
// with logit x: log(t / 2^32) for the minority value, log(1 - t / 2^32) for
// the sign of x, in fp64.
__device__ __forceinline__ double site_logq(float x, float s) {
    const double t = (double)minority_threshold(x) * 0x1p-32;
    const bool majority = (x >= 0.0f) == (s > 0.0f);
    return majority ? log1p(-t) : log(t);
}

// A point index clamped to the points that exist.
__device__ __forceinline__ int clamp_point(int q, int npts) { return q < 0 ? 0 : (q >= npts ? npts - 1 : q); }

// Orders this wavefront's LDS writes before its later LDS reads of other
// lanes' data: a wavefront's LDS accesses execute in issue order, so only the
// compiler has to be kept from moving them (no workgroup barrier: the
// wavefronts of a workgroup loop over different numbers of tiles).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kOutRow = 33;  // LDS row stride (floats) of a staged output tile: the two lane halves hit different banks

// Epilogue modes of the generic conv kernel.
enum { EP_RELU = 0, EP_RESID = 1, EP_LOGIT = 2, EP_DGRAD = 3, EP_DGRAD_RESID = 4 };

// out tile of 32 pixels x 32 channels per wavefront:
//   acc[p][j] = sum_t sum_k in[p + tap_t][k] * Wop[t][j][k]
// with the matrix-core layout: A row i = pixel, B column j = out channel,
// k = 16-element chunks of the 32 input channels of each tap.
// bias: layer biases [C] (pt == nullptr), or layer row of a per-point table
// with rows kCondOut apart, the row of pixel p being that of its sample's
// point pt[p / L^2] (clamped to [0, npts))
// out_mask (ReLU modes, may be NULL): one word per pixel, bit j set where
// channel j's pre-activation is positive
// gate (data-gradient modes, may be NULL): the ReLU mask of the layer below;
// then gz also receives the gated gradient in bf16 (out_f where the mask bit
// is set, else 0), and gbias[wave][C] each wavefront's fp32 sum of it over its
// pixels (fixed order: its tiles in turn, then a butterfly over its lanes)
__global__ void __launch_bounds__(256) conv32_kernel(const __bf16* __restrict__ in, const __bf16* __restrict__ Wop,
                                                     const float* __restrict__ bias, const int32_t* __restrict__ pt,
                                                     int npts, Taps taps, int L, int64_t P, int mode,
                                                     const __bf16* __restrict__ resid_bf,
                                                     const float* __restrict__ resid_f, __bf16* out_bf,
                                                     uint32_t* out_mask, float* out_f, const uint32_t* __restrict__ gate,
                                                     __bf16* __restrict__ gz, float* __restrict__ gbias) {
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t w0 = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int li = lane & 31, half = lane >> 5;
    __shared__ float tile_out[4][32 * kOutRow];  // one output tile per wavefront (4 per workgroup)
    float* T = tile_out[threadIdx.x >> 6];
    // B fragments stay in registers for the whole launch
    bf16x8 Bf[NT][2];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int kh = 0; kh < 2; ++kh)
            Bf[t][kh] = (t < taps.n) ? load8(Wop + ((int64_t)t * C + li) * C + kh * 16 + half * 8) : zero8();
    const bool dgrad = mode == EP_DGRAD || mode == EP_DGRAD_RESID;
    const float bj = dgrad ? 0.f : bias[li];
    const int64_t LL = (int64_t)L * L;
    const int64_t ntiles = (P + 31) / 32;
    // A tile's operands are loaded while the previous tile's epilogue runs.
    bf16x8 A[NT][2];
    auto gather = [&](int64_t tl) {
        const int64_t pp = tl * 32 + li;
        const uint32_t ef = edge_flags(pp < P ? pp : 0, L);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int64_t q = (t < taps.n && pp < P) ? shift_pix(pp, ef, taps.dr[t], taps.dc[t], L) : -1;
#pragma unroll
            for (int kh = 0; kh < 2; ++kh) A[t][kh] = (q >= 0) ? load8(in + q * C + kh * 16 + half * 8) : zero8();
        }
    };
    float gsum[16];  // gated-gradient sums of this lane's 16 channels (gate only)
#pragma unroll
    for (int k = 0; k < 16; ++k) gsum[k] = 0.f;
    if (w0 < ntiles) gather(w0);
    for (int64_t tile = w0; tile < ntiles; tile += nw) {
        f32x16 acc;
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[v] = 0.f;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (t >= taps.n) break;
#pragma unroll
            for (int kh = 0; kh < 2; ++kh) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[t][kh], Bf[t][kh], acc, 0, 0, 0);
        }
        // the epilogue's residual is loaded before the next tile's operands, so
        // that waiting for it does not wait for them
        const int64_t pi = tile * 32 + (lane >> 1);
        const int c0 = (lane & 1) * 16;
        bf16x8 rb[2];
        float4 rf[4];
        if (mode == EP_RESID && pi < P) {
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) rb[hh] = load8(resid_bf + pi * C + c0 + 8 * hh);
        }
        if (mode == EP_DGRAD_RESID && pi < P) {
#pragma unroll
            for (int k = 0; k < 4; ++k) rf[k] = *reinterpret_cast<const float4*>(resid_f + pi * C + c0 + 4 * k);
        }
        const uint32_t gm = (gate && pi < P) ? gate[pi] >> c0 : 0u;
        if (tile + nw < ntiles) gather(tile + nw);
        if (mode == EP_LOGIT) {
            // D[i][j]: j = lane & 31, i = 8 (v / 4) + 4 half + (v % 4); only channel 0 is the logit
            if (li == 0)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int i = 8 * (v >> 2) + 4 * half + (v & 3);
                    const int64_t pi = tile * 32 + i;
                    if (pi >= P) continue;
                    float bv = bj;
                    if (pt) bv = bias[(int64_t)clamp_point(pt[pi / LL], npts) * kCondOut];
                    out_f[pi] = acc[v] + bv;
                }
            continue;
        }
        // The tile's 32 pixels x 32 channels are one contiguous block of the
        // pixel-major output: pass the accumulators through this wavefront's
        // LDS rows so that each lane then owns 16 consecutive elements (one
        // pixel, half its channels) and moves them with 16-byte accesses.
#pragma unroll
        for (int v = 0; v < 16; ++v) T[(8 * (v >> 2) + 4 * half + (v & 3)) * kOutRow + li] = acc[v];
        wave_sync();
        if (pi < P) {
            const float* br = dgrad ? nullptr : (pt ? bias + (int64_t)clamp_point(pt[pi / LL], npts) * kCondOut : bias);
            uint32_t mbits = 0u;  // ReLU mask of this lane's 16 channels
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {  // two runs of 8 channels keep fewer values live
                const int cb = c0 + 8 * hh;
                float z[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) z[e] = T[(lane >> 1) * kOutRow + cb + e] + (dgrad ? 0.f : br[cb + e]);
                const int64_t o = pi * C + cb;
                if (mode == EP_RELU || mode == EP_RESID) {
                    const bf16x8 r = mode == EP_RESID ? rb[hh] : zero8();
                    bf16x8 ob;
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const float y = z[e] > 0.f ? z[e] : 0.f;
                        ob[e] = f2bf(mode == EP_RESID ? bf2f(r[e]) + y : y);
                        mbits |= (uint32_t)(z[e] > 0.f) << (8 * hh + e);
                    }
                    *reinterpret_cast<bf16x8*>(out_bf + o) = ob;
                } else {  // EP_DGRAD, EP_DGRAD_RESID
                    float dv[8];
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        float4 d = make_float4(z[4 * q], z[4 * q + 1], z[4 * q + 2], z[4 * q + 3]);
                        if (mode == EP_DGRAD_RESID) {
                            const float4 r = rf[2 * hh + q];
                            d.x += r.x;
                            d.y += r.y;
                            d.z += r.z;
                            d.w += r.w;
                        }
                        *reinterpret_cast<float4*>(out_f + o + 4 * q) = d;
                        dv[4 * q] = d.x;
                        dv[4 * q + 1] = d.y;
                        dv[4 * q + 2] = d.z;
                        dv[4 * q + 3] = d.w;
                    }
                    if (gate) {
                        bf16x8 zb;
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            const float v = ((gm >> (8 * hh + e)) & 1u) ? dv[e] : 0.f;
                            zb[e] = f2bf(v);
                            gsum[8 * hh + e] += v;
                        }
                        *reinterpret_cast<bf16x8*>(gz + o) = zb;
                    }
                }
            }
            // one 32-bit word per pixel, bit j = channel j; each lane stores its half
            if (out_mask) reinterpret_cast<uint16_t*>(out_mask)[2 * pi + (lane & 1)] = (uint16_t)mbits;
        }
        wave_sync();  // the rows are rewritten by the next tile
    }
    if (gate) {
        // lanes of equal parity hold the same 16 channels (pixel = lane / 2)
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            float v = gsum[k];
#pragma unroll
            for (int m = 2; m < 64; m <<= 1) v += __shfl_xor(v, m);
            gsum[k] = v;
        }
        if (lane < 2)
#pragma unroll
            for (int k = 0; k < 16; ++k) gbias[w0 * C + (lane & 1) * 16 + k] = gsum[k];
    }
}

// Fused training forward for L <= kFwdMaxL: one workgroup of four wavefronts
// per configuration runs all 12 layers with the layer input and output in
// LDS, and writes what the backward reads (every layer's input h_l in the
// pixel-major layout [NL][P][C], the ReLU masks, the logits).  Per 32-pixel
// tile it runs exactly the arithmetic of conv32_kernel: the same
// 32x32x16 instructions with the same operands in the same order, the
// accumulators from zero, the bias added in the same epilogue, so its
// activations, masks and logits equal the layered path's bit for bit; only
// the operands come from LDS instead of the caches.  The LDS grid carries a
// zero border (one row above, one column on each side) so that every tap
// reads a valid address and out-of-lattice taps read zeros, as the layered
// path's edge tests give; a pixel's four 16-byte channel chunks are XOR
// swizzled by (pixel / 4) mod 4, so eight lanes reading one chunk of eight
// consecutive pixels hit distinct banks.
constexpr int kFwdMaxL = 30;
__host__ __device__ constexpr int fwd_pixels(int L) { return (L + 1) * (L + 2); }
__host__ __device__ constexpr int fwd_lds_bytes(int L) {
    return 2 * fwd_pixels(L) * C * 2 + 4 * 32 * kOutRow * 4;
}

__device__ __forceinline__ int fwd_off(int pix, int chunk) {  // bf16 offset of a 16-byte chunk
    return pix * C + ((chunk ^ ((pix >> 2) & 3)) << 3);
}

__global__ void __launch_bounds__(256) train_fwd_kernel(int64_t B, int L, const int8_t* __restrict__ spins,
                                                        const __bf16* __restrict__ wf,
                                                        const float* __restrict__ bias_tab,
                                                        const int32_t* __restrict__ pt, int npts,
                                                        __bf16* __restrict__ hs, uint32_t* __restrict__ mask,
                                                        float* __restrict__ logit) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = L * L, W2 = L + 2, PP = fwd_pixels(L);
    __bf16* bufs = reinterpret_cast<__bf16*>(smem);                       // [2][PP][C]
    float* T = reinterpret_cast<float*>(smem + (size_t)2 * PP * C * 2) + (threadIdx.x >> 6) * 32 * kOutRow;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int li = lane & 31, half = lane >> 5;
    const int64_t b = blockIdx.x;
    if (b >= B) return;  // uniform per workgroup
    const int64_t P = B * N, LSZ = P * C;
    const int8_t* sp = spins + b * N;
    const float* brow = bias_tab + (pt ? (int64_t)clamp_point(pt[b], npts) * kCondOut : 0);  // [NL][C]
    for (int g = tid; g < 2 * PP * (C / 8); g += blockDim.x)
        *reinterpret_cast<bf16x8*>(bufs + (int64_t)g * 8) = zero8();
    __syncthreads();
    // h_0: the spin in channel 0 (the embedding of the layered path), in LDS and in HBM
    for (int g = tid; g < N * (C / 8); g += blockDim.x) {
        const int p = g >> 2, ch = g & 3;
        bf16x8 v = zero8();
        if (ch == 0) v[0] = f2bf((float)sp[p]);
        *reinterpret_cast<bf16x8*>(hs + (b * N + p) * C + ch * 8) = v;
        const int r = p / L, c = p - r * L;
        if (ch == 0) *reinterpret_cast<bf16x8*>(bufs + fwd_off((r + 1) * W2 + c + 1, 0)) = v;
    }
    __syncthreads();
    const int ntiles = (N + 31) / 32;
    int in_b = 0;
    for (int l = 0; l < NL; ++l) {
        const int nt = (l == 0) ? 4 : 5;
        const int mode = (l == NL - 1) ? EP_LOGIT : (l == 0 ? EP_RELU : EP_RESID);
        const __bf16* Wop = wf + (int64_t)l * NT * C * C;
        bf16x8 Bf[NT][2];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int kh = 0; kh < 2; ++kh)
                Bf[t][kh] = (t < nt) ? load8(Wop + ((int64_t)t * C + li) * C + kh * 16 + half * 8) : zero8();
        const float* br = brow + l * C;
        const __bf16* bin = bufs + (size_t)in_b * PP * C;
        __bf16* bout = bufs + (size_t)(1 - in_b) * PP * C;
        const int toff[NT] = {-W2 - 1, -W2, -W2 + 1, -1, 0};
        for (int tile = w; tile < ntiles; tile += 4) {
            const int pp = tile * 32 + li;
            bf16x8 A[NT][2];
            if (pp < N) {
                const int r = pp / L, c = pp - r * L, pidx = (r + 1) * W2 + c + 1;
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int kh = 0; kh < 2; ++kh)
                        A[t][kh] = (t < nt) ? *reinterpret_cast<const bf16x8*>(bin + fwd_off(pidx + toff[t], 2 * kh + half))
                                            : zero8();
            } else {
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int kh = 0; kh < 2; ++kh) A[t][kh] = zero8();
            }
            f32x16 acc;
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[v] = 0.f;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                if (t >= nt) break;
#pragma unroll
                for (int kh = 0; kh < 2; ++kh) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[t][kh], Bf[t][kh], acc, 0, 0, 0);
            }
            if (mode == EP_LOGIT) {
                if (li == 0)
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        const int i = 8 * (v >> 2) + 4 * half + (v & 3);
                        const int p = tile * 32 + i;
                        if (p < N) logit[b * N + p] = acc[v] + br[0];
                    }
                continue;
            }
#pragma unroll
            for (int v = 0; v < 16; ++v) T[(8 * (v >> 2) + 4 * half + (v & 3)) * kOutRow + li] = acc[v];
            wave_sync();
            const int pi = tile * 32 + (lane >> 1), c0 = (lane & 1) * 16;
            if (pi < N) {
                const int r = pi / L, c = pi - r * L, pidx = (r + 1) * W2 + c + 1;
                uint32_t mbits = 0u;
#pragma unroll
                for (int hh = 0; hh < 2; ++hh) {
                    const int cb = c0 + 8 * hh;
                    const bf16x8 rr = mode == EP_RESID ? *reinterpret_cast<const bf16x8*>(bin + fwd_off(pidx, cb >> 3))
                                                       : zero8();
                    bf16x8 ob;
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const float z = T[(lane >> 1) * kOutRow + cb + e] + br[cb + e];
                        const float y = z > 0.f ? z : 0.f;
                        ob[e] = f2bf(mode == EP_RESID ? bf2f(rr[e]) + y : y);
                        mbits |= (uint32_t)(z > 0.f) << (8 * hh + e);
                    }
                    *reinterpret_cast<bf16x8*>(bout + fwd_off(pidx, cb >> 3)) = ob;
                    *reinterpret_cast<bf16x8*>(hs + (int64_t)(l + 1) * LSZ + (b * N + pi) * C + cb) = ob;
                }
                reinterpret_cast<uint16_t*>(mask + (int64_t)l * P)[2 * (b * N + pi) + (lane & 1)] = (uint16_t)mbits;
            }
            wave_sync();  // the rows are rewritten by the next tile
        }
        __syncthreads();  // the layer's output is complete before it is read as input
        in_b = 1 - in_b;
    }
}

// Fused data-gradient chain for L <= kBwdMaxL: one workgroup of four
// wavefronts per configuration runs the transposed convolutions of layers
// 11 .. 1 with the gated gradient dz in LDS (double-buffered, zero border
// below and on both sides for the mirrored taps) and the fp32 gradient of the
// residual stream dh in registers (each wavefront keeps its tiles, at most
// MAXT of 32 pixels, for the whole chain).  Per tile it runs conv32_kernel's
// data-gradient arithmetic exactly (same instructions, operands and order;
// dh_{l-1} = conv^T(dz_l) + dh_l; dz_{l-1} = bf16 of dh_{l-1} where layer
// l-1's ReLU was open, else 0), so every dz equals the layered path's bit for
// bit.  Outputs: dz_l of layers 10 .. 0 (pixel-major, the weight gradient's
// operand), and per configuration and layer the sum of dz over its pixels in
// fp32 (the bias-gradient partials, bpl[NL][B][C]; layer 11's is the sum of
// the logit gradient, [B]); with gs != nullptr the same sums are the
// per-sample bias gradients of a conditional network.
constexpr int kBwdMaxL = 24;
__host__ __device__ constexpr int bwd_lds_bytes(int L) {
    return 2 * (L + 1) * (L + 2) * C * 2 + 4 * 32 * kOutRow * 4 + 4 * 32 * 4;
}

template <int MAXT>
__global__ void __launch_bounds__(256) train_bwd_kernel(int64_t B, int L, const __bf16* __restrict__ g,
                                                        const float* __restrict__ g32,
                                                        const __bf16* __restrict__ wb,
                                                        const uint32_t* __restrict__ mask, __bf16* __restrict__ dzs,
                                                        float* __restrict__ bpl, float* __restrict__ gs) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = L * L, W2 = L + 2, PP = (L + 1) * (L + 2);
    __bf16* bufs = reinterpret_cast<__bf16*>(smem);  // [2][PP][C]
    float* Tall = reinterpret_cast<float*>(smem + (size_t)2 * PP * C * 2);
    float* red = Tall + 4 * 32 * kOutRow;           // [4 wavefronts][C]
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    float* T = Tall + w * 32 * kOutRow;
    const int li = lane & 31, half = lane >> 5;
    const int64_t b = blockIdx.x;
    if (b >= B) return;  // uniform per workgroup
    const int64_t P = B * N, LSZ = P * C;
    for (int q = tid; q < 2 * PP * (C / 8); q += blockDim.x)
        *reinterpret_cast<bf16x8*>(bufs + (int64_t)q * 8) = zero8();
    __syncthreads();
    // dz of the logit layer: the loss gradient (channel 0), and its sum over the pixels
    float gsum0 = 0.f;
    for (int q = tid; q < N * (C / 8); q += blockDim.x) {
        const int p = q >> 2, ch = q & 3;
        const int r = p / L, c = p - r * L;
        *reinterpret_cast<bf16x8*>(bufs + fwd_off(r * W2 + c + 1, ch)) =
            *reinterpret_cast<const bf16x8*>(g + (b * N + p) * C + ch * 8);
    }
    for (int p = tid; p < N; p += blockDim.x) gsum0 += g32[b * N + p];
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) gsum0 += __shfl_xor(gsum0, m);
    if (lane == 0) red[w * C] = gsum0;
    __syncthreads();
    if (tid == 0) {
        const float t0 = ((red[0] + red[C]) + red[2 * C]) + red[3 * C];
        bpl[(int64_t)(NL - 1) * B * C + b] = t0;
        if (gs) {
            gs[(b * NL + (NL - 1)) * C] = t0;
            for (int c = 1; c < C; ++c) gs[(b * NL + (NL - 1)) * C + c] = 0.f;
        }
    }
    const int ntiles = (N + 31) / 32;
    const int mtoff[NT] = {W2 + 1, W2, W2 - 1, 1, 0};  // the mirrored taps (1,1) (1,0) (1,-1) (0,1) (0,0)
    float dh[MAXT][16];
#pragma unroll
    for (int k = 0; k < MAXT; ++k)
#pragma unroll
        for (int e = 0; e < 16; ++e) dh[k][e] = 0.f;
    int in_b = 0;
    for (int l = NL - 1; l >= 1; --l) {
        const __bf16* Wop = wb + (int64_t)l * NT * C * C;
        bf16x8 Bf[NT][2];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int kh = 0; kh < 2; ++kh) Bf[t][kh] = load8(Wop + ((int64_t)t * C + li) * C + kh * 16 + half * 8);
        const __bf16* bin = bufs + (size_t)in_b * PP * C;
        __bf16* bout = bufs + (size_t)(1 - in_b) * PP * C;
        const uint32_t* gate = mask + (int64_t)(l - 1) * P;
        __bf16* dzo = dzs + (int64_t)(l - 1) * LSZ;
        float gsum[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) gsum[e] = 0.f;
#pragma unroll
        for (int k = 0; k < MAXT; ++k) {
            const int tile = w + 4 * k;
            if (tile >= ntiles) break;
            const int pp = tile * 32 + li;
            bf16x8 A[NT][2];
            if (pp < N) {
                const int r = pp / L, c = pp - r * L, pidx = r * W2 + c + 1;
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int kh = 0; kh < 2; ++kh)
                        A[t][kh] = *reinterpret_cast<const bf16x8*>(bin + fwd_off(pidx + mtoff[t], 2 * kh + half));
            } else {
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int kh = 0; kh < 2; ++kh) A[t][kh] = zero8();
            }
            f32x16 acc;
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[v] = 0.f;
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int kh = 0; kh < 2; ++kh) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[t][kh], Bf[t][kh], acc, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 16; ++v) T[(8 * (v >> 2) + 4 * half + (v & 3)) * kOutRow + li] = acc[v];
            wave_sync();
            const int pi = tile * 32 + (lane >> 1), c0 = (lane & 1) * 16;
            if (pi < N) {
                const int r = pi / L, c = pi - r * L, pidx = r * W2 + c + 1;
                const uint32_t gm = gate[b * N + pi] >> c0;
#pragma unroll
                for (int hh = 0; hh < 2; ++hh) {
                    bf16x8 zb;
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const float z = T[(lane >> 1) * kOutRow + c0 + 8 * hh + e];
                        const float d = (l == NL - 1) ? z : z + dh[k][8 * hh + e];
                        dh[k][8 * hh + e] = d;
                        const float v = ((gm >> (8 * hh + e)) & 1u) ? d : 0.f;
                        zb[e] = f2bf(v);
                        gsum[8 * hh + e] += v;
                    }
                    *reinterpret_cast<bf16x8*>(bout + fwd_off(pidx, (c0 >> 3) + hh)) = zb;
                    *reinterpret_cast<bf16x8*>(dzo + (b * N + pi) * C + c0 + 8 * hh) = zb;
                }
            }
            wave_sync();  // the rows are rewritten by the next tile
        }
        // per-configuration sums of dz_{l-1}: lanes of equal parity hold the same 16 channels
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            float v = gsum[e];
#pragma unroll
            for (int m = 2; m < 64; m <<= 1) v += __shfl_xor(v, m);
            gsum[e] = v;
        }
        if (lane < 2)
#pragma unroll
            for (int e = 0; e < 16; ++e) red[w * C + lane * 16 + e] = gsum[e];
        __syncthreads();  // dz_{l-1} and the sums are complete
        if (tid < C) {
            const float t0 = ((red[tid] + red[C + tid]) + red[2 * C + tid]) + red[3 * C + tid];
            bpl[((int64_t)(l - 1) * B + b) * C + tid] = t0;
            if (gs) gs[(b * NL + (l - 1)) * C + tid] = t0;
        }
        __syncthreads();  // red is rewritten by the next layer
        in_b = 1 - in_b;
    }
}

// Partial weight gradients, one chunk of kWChunk pixels each, all taps at once
// (they share the gradient operand):
//   part[chunk][t][i][j] = sum_{p in chunk} in[p + tap_t][i] dz[p][j]
// (A row i = input channel, k = pixel; B column j = output channel).
constexpr int kWChunk = 512;
constexpr int kWWaves = 2;  // wavefronts per chunk, kWChunk / kWWaves pixels each

// Each wavefront of a chunk's workgroup stages 32-pixel tiles of the
// pixel-major layer input, shifted by each tap (zero outside the lattice), and
// of the gradient through LDS in channel-major form (the matrix-core operands
// need consecutive pixels per channel) and contracts them on the matrix cores.
// No channel-major copy goes through HBM.  The wavefronts' sums are added in
// LDS (wavefront 0's plus wavefront 1's), so a chunk writes one partial.
constexpr int kFT = 32;           // pixels per staged tile (two 16-pixel k-steps)
constexpr int kFRow = kFT + 8;    // LDS row stride in elements (80 bytes: 16-byte aligned rows)

// Weight-gradient jobs of one launch (blockIdx.y picks the job): the layer's
// input, its gated gradient, its partial-sum buffer and its layer index.
struct WgradJobs {
    const __bf16* in[NL];
    const __bf16* dz[NL];
    float* part[NL];
    int layer[NL];
};

__global__ void __launch_bounds__(64 * kWWaves) wgrad_fused_kernel(WgradJobs jobs, int L, int64_t P) {
    const int job = blockIdx.y;
    const __bf16* __restrict__ in = jobs.in[job];
    const __bf16* __restrict__ dz = jobs.dz[job];
    float* __restrict__ part = jobs.part[job];
    const Taps taps = taps_for_dev(jobs.layer[job]);
    constexpr int kSlot = (NT + 1) * C * kFRow;  // one wavefront's tiles: slots 0..NT-1 taps, slot NT the gradient
    __shared__ __align__(16) __bf16 tls[kWWaves * kSlot];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __bf16* tl = tls + wv * kSlot;
    const int li = lane & 31, half = lane >> 5;
    const int px = lane >> 1, hc = lane & 1;  // staging: pixel of the tile, channel half
    const int64_t chunk = blockIdx.x;
    const int64_t c_begin = chunk * kWChunk;
    const int64_t k_begin = c_begin + wv * (kWChunk / kWWaves);
    const int64_t k_end = (k_begin + kWChunk / kWWaves < P) ? k_begin + kWChunk / kWWaves : P;
    f32x16 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[t][v] = 0.f;
    // Global loads of the next tile are issued before the current tile's
    // matrix-core work and land in registers; they are written to LDS after it.
    bf16x8 G[2], X[NT][2];
    auto fetch = [&](int64_t p0) {
        const int64_t p = p0 + px;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) G[hh] = (p < P) ? load8(dz + p * C + hc * 16 + hh * 8) : zero8();
        const uint32_t ef = edge_flags(p < P ? p : 0, L);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int64_t q = (t < taps.n && p < P) ? shift_pix(p, ef, taps.dr[t], taps.dc[t], L) : -1;
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) X[t][hh] = (q >= 0) ? load8(in + q * C + hc * 16 + hh * 8) : zero8();
        }
    };
    if (k_begin < k_end) fetch(k_begin);
    for (int64_t p0 = k_begin; p0 < k_end; p0 += kFT) {
#pragma unroll
        for (int hh = 0; hh < 2; ++hh)
#pragma unroll
            for (int e = 0; e < 8; ++e) tl[(NT * C + hc * 16 + hh * 8 + e) * kFRow + px] = G[hh][e];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (t >= taps.n) break;
#pragma unroll
            for (int hh = 0; hh < 2; ++hh)
#pragma unroll
                for (int e = 0; e < 8; ++e) tl[(t * C + hc * 16 + hh * 8 + e) * kFRow + px] = X[t][hh][e];
        }
        wave_sync();  // this wavefront's own tiles: no workgroup barrier
        if (p0 + kFT < k_end) fetch(p0 + kFT);
#pragma unroll
        for (int ks = 0; ks < kFT / 16; ++ks) {
            const int col = ks * 16 + half * 8;
            const bf16x8 b = *reinterpret_cast<const bf16x8*>(tl + (NT * C + li) * kFRow + col);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                if (t >= taps.n) break;
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(tl + (t * C + li) * kFRow + col);
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[t], 0, 0, 0);
            }
        }
        wave_sync();  // this wavefront's own tiles: no workgroup barrier
    }
    // every wavefront reaches this point (no barrier inside the loops above)
    float* red = reinterpret_cast<float*>(tls);  // NT * 16 * 64 floats fit in the tiles' space
    static_assert(kWWaves == 2 && NT * 16 * 64 * sizeof(float) <= kWWaves * kSlot * sizeof(__bf16), "reduction buffer");
    __syncthreads();
    if (wv == 1)
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 16; ++v) red[(t * 16 + v) * 64 + lane] = acc[t][v];
    __syncthreads();
    if (wv == 0)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (t >= taps.n) break;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int i = 8 * (v >> 2) + 4 * half + (v & 3);
                part[((chunk * NT + t) * C + i) * C + li] = acc[t][v] + red[(t * 16 + v) * 64 + lane];
            }
        }
}

// Two-stage deterministic sum over chunks: stage 1 (block = 256 entries x one
// of S slices) sums chunks s, s + S, ... in fp64; stage 2 sums the S slices.
constexpr int kRedSlices = 16;

// blockIdx.z picks one of several partial-sum sets, part_stride / part2_stride apart
__global__ void __launch_bounds__(256) reduce_slices_kernel(const float* __restrict__ part, int nchunks, int n,
                                                            double* __restrict__ part2, int64_t part_stride,
                                                            int64_t part2_stride) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int sl = blockIdx.y;
    part += (int64_t)blockIdx.z * part_stride;
    part2 += (int64_t)blockIdx.z * part2_stride;
    if (x >= n) return;
    double s = 0.0;
#pragma unroll 8  // loads in flight; the sum keeps its order
    for (int c = sl; c < nchunks; c += kRedSlices) s += part[(int64_t)c * n + x];
    part2[(int64_t)sl * n + x] = s;
}


// spins int8 [P] -> bf16 [P][32] with the spin in channel 0; a thread writes
// 8 channels (16 bytes) of one pixel
__global__ void embed_kernel(const int8_t* spins, int64_t P, __bf16* h0) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P * (C / 8)) return;
    bf16x8 v = zero8();
    if ((i & 3) == 0) v[0] = f2bf((float)spins[i >> 2]);
    *reinterpret_cast<bf16x8*>(h0 + i * 8) = v;
}

// loss: per sample log q (fp64) and the logit gradient of -mean log q
// (bf16, channel 0 of a [P][32] buffer)
__global__ void __launch_bounds__(256) loss_kernel(const float* logit, const int8_t* spins, int L, float inv_batch,
                                                   double* logq, __bf16* g, float* g32) {
    const int b = blockIdx.x;
    const int N = L * L;
    double s = 0.0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const int64_t p = (int64_t)b * N + i;
        const float sg = (float)spins[p];
        const float x = sg * logit[p];
        s += -log1p(exp(-(double)x));
        const float gi = -sg * (1.f / (1.f + expf(x))) * inv_batch;
        g[p * C] = f2bf(gi);
        g32[p] = gi;
        for (int c = 1; c < C; ++c) g[p * C + c] = (__bf16)0.0f;
    }
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) logq[b] = red[0];
}

// log q per chain from per-site logits: the sum over sites of site_logq, the
// log-probability with which the sampler's integer rule draws that spin, in
// fp64.  One wavefront per chain: lane k sums the sites k, k + 64, ... in
// order, then a fixed butterfly over the 64 lane sums.  The sampler and the
// scorer both reduce their logits with this kernel, so equal logits give
// bit-identical log q.
__global__ void __launch_bounds__(256) logq_kernel(const float* __restrict__ logit, const int8_t* __restrict__ spins,
                                                   int64_t n, int N, double* __restrict__ logq) {
    const int lane = threadIdx.x & 63;
    const int64_t ch = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (ch >= n) return;  // uniform per wavefront
    double s = 0.0;
    for (int i = lane; i < N; i += 64) {
        s += site_logq(logit[ch * N + i], (float)spins[ch * N + i]);
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) s += __shfl_xor(s, d);
    if (lane == 0) logq[ch] = s;
}

// bias gradient of the logit layer: sum over pixels of the fp32 logit gradient
__global__ void __launch_bounds__(256) colsum0_kernel(const float* g32, int64_t P, float* part) {
    float s = 0.f;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x)
        s += g32[p];
    __shared__ float red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// ------------------------------------------------------------------------
// Conditioning.  A point's features x (kCondF values) shift the biases of
// every layer by g(x) = W2^T tanh(W1^T x + b1); MLP parameters (fp32) are
// W1 [kCondF][kCondH], b1 [kCondH], W2 [kCondH][NL][C].  The inference and
// training kernels read the per-point table cb[p][l][c] = bias[l][c] + g(x_p).


// one workgroup (kCondOut threads) per point
__global__ void __launch_bounds__(kCondOut) cond_bias_kernel(const float* __restrict__ mlp,
                                                             const float* __restrict__ feats,
                                                             const float* __restrict__ bias, float* __restrict__ cb) {
    __shared__ float hsh[kCondH];
    const int p = blockIdx.x, j = threadIdx.x;
    const float* W1 = mlp;
    const float* b1 = W1 + kCondF * kCondH;
    const float* W2 = b1 + kCondH;
    if (j < kCondH) {
        float z = b1[j];
#pragma unroll
        for (int f = 0; f < kCondF; ++f) z += feats[p * kCondF + f] * W1[f * kCondH + j];
        hsh[j] = tanhf(z);
    }
    __syncthreads();
    float g = 0.f;
#pragma unroll 8
    for (int k = 0; k < kCondH; ++k) g += hsh[k] * W2[k * kCondOut + j];
    cb[(int64_t)p * kCondOut + j] = bias[j] + g;
}

// gradient of the loss with respect to each sample's biases of layer l: the
// sum over the sample's pixels of the pre-activation gradient (masked dh, or
// the logit gradient g32 in the logit layer), in a fixed order; one
// workgroup per sample, 8 pixel slices x 32 channels
__global__ void __launch_bounds__(256) sample_bias_grad_kernel(const float* __restrict__ dh,
                                                               const uint32_t* __restrict__ mask,
                                                               const float* __restrict__ g32, int N, int l,
                                                               float* __restrict__ gs) {
    const int64_t b = blockIdx.x;
    const int c = threadIdx.x & 31, slot = threadIdx.x >> 5;
    float s = 0.f;
    if (g32) {
        if (c == 0)
            for (int i = slot; i < N; i += 8) s += g32[b * N + i];
    } else {
        for (int i = slot; i < N; i += 8) {
            const int64_t px = b * N + i;
            s += ((mask[px] >> c) & 1u) ? dh[px * C + c] : 0.f;
        }
    }
    __shared__ float red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    if (slot == 0) {
        float t = 0.f;
        for (int k = 0; k < 8; ++k) t += red[k * 32 + c];
        gs[(b * NL + l) * C + c] = t;
    }
}

// per point: the sum of its samples' bias gradients, samples in index order
__global__ void point_grad_kernel(const float* __restrict__ gs, const int32_t* __restrict__ pt, int64_t B, int npts,
                                  float* __restrict__ gp) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (int64_t)npts * kCondOut) return;
    const int p = (int)(x / kCondOut), j = (int)(x % kCondOut);
    double s = 0.0;
    for (int64_t b = 0; b < B; ++b)
        if ((pt ? clamp_point(pt[b], npts) : 0) == p) s += gs[b * kCondOut + j];
    gp[x] = (float)s;
}

// MLP backward from the per-point bias gradients gp [npts][kCondOut] into
// gmlp (the MLP part of the gradient vector); one workgroup
__global__ void __launch_bounds__(kCondOut) cond_backward_kernel(const float* __restrict__ mlp,
                                                                 const float* __restrict__ feats, int npts,
                                                                 const float* __restrict__ gp,
                                                                 float* __restrict__ gmlp) {
    __shared__ float hsh[kCondMaxPoints * kCondH];
    __shared__ float dpre[kCondMaxPoints * kCondH];
    const int j = threadIdx.x;
    const float* W1 = mlp;
    const float* b1 = W1 + kCondF * kCondH;
    const float* W2 = b1 + kCondH;
    for (int x = j; x < npts * kCondH; x += blockDim.x) {
        const int p = x / kCondH, k = x % kCondH;
        float z = b1[k];
#pragma unroll
        for (int f = 0; f < kCondF; ++f) z += feats[p * kCondF + f] * W1[f * kCondH + k];
        hsh[x] = tanhf(z);
    }
    __syncthreads();
    // dW2[k][j] = sum_p h[p][k] gp[p][j]
    for (int k = 0; k < kCondH; ++k) {
        float s = 0.f;
        for (int p = 0; p < npts; ++p) s += hsh[p * kCondH + k] * gp[(int64_t)p * kCondOut + j];
        gmlp[kCondF * kCondH + kCondH + k * kCondOut + j] = s;
    }
    // dpre[p][k] = (1 - h^2) sum_j W2[k][j] gp[p][j]
    for (int x = j; x < npts * kCondH; x += blockDim.x) {
        const int p = x / kCondH, k = x % kCondH;
        float s = 0.f;
        for (int jj = 0; jj < kCondOut; ++jj) s += W2[k * kCondOut + jj] * gp[(int64_t)p * kCondOut + jj];
        const float hv = hsh[x];
        dpre[x] = s * (1.f - hv * hv);
    }
    __syncthreads();
    if (j < kCondF * kCondH) {  // dW1[f][k] = sum_p x[p][f] dpre[p][k]
        const int f = j / kCondH, k = j % kCondH;
        float s = 0.f;
        for (int p = 0; p < npts; ++p) s += feats[p * kCondF + f] * dpre[p * kCondH + k];
        gmlp[j] = s;
    } else if (j < kCondF * kCondH + kCondH) {  // db1[k] = sum_p dpre[p][k]
        const int k = j - kCondF * kCondH;
        float s = 0.f;
        for (int p = 0; p < npts; ++p) s += dpre[p * kCondH + k];
        gmlp[j] = s;
    }
}

// Adam on the fp32 master parameters (Kingma & Ba, 2015)
__global__ void adam_kernel(float* th, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// master fp32 parameters -> padded bf16 operand blocks and padded biases
__global__ void pack_kernel(const float* th, __bf16* wf, __bf16* wb, float* bias) {
    // one thread per (layer, tap, a, b) with a, b in 0..31
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= NL * NT * C * C) return;
    const int b = x % C, a = (x / C) % C, t = (x / (C * C)) % NT, l = x / (NT * C * C);
    int64_t off = 0;
    for (int k = 0; k < l; ++k) {
        const int T = (k == 0) ? 4 : 5, ci = (k == 0) ? 1 : C, co = (k == NL - 1) ? 1 : C;
        off += (int64_t)T * ci * co + co;
    }
    const int T = (l == 0) ? 4 : 5, ci = (l == 0) ? 1 : C, co = (l == NL - 1) ? 1 : C;
    // wf[l][t][cout=a][cin=b], wb[l][t][cin=a][cout=b]
    float vf = 0.f, vb = 0.f;
    if (t < T) {
        if (a < co && b < ci) vf = th[off + ((int64_t)t * ci + b) * co + a];
        if (a < ci && b < co) vb = th[off + ((int64_t)t * ci + a) * co + b];
    }
    const int64_t o = (((int64_t)l * NT + t) * C + a) * C + b;
    wf[o] = f2bf(vf);
    wb[o] = f2bf(vb);
    if (t == 0 && b == 0) bias[l * C + a] = (a < co) ? th[off + (int64_t)T * ci * co + a] : 0.f;
}

// ------------------------------------------------------------------------
// Sampling and scoring share one per-element arithmetic: for every output
// (configuration, site, channel) the five taps are accumulated in order
// (-1,-1), (-1,0), (-1,1), (0,-1), (0,0) by one 16x16x32 bf16 matrix-core
// instruction each (all 32 input channels at once), starting from the bias;
// then ReLU and the residual add in fp32 and one rounding to bf16.  The
// logits of both paths are therefore bit-identical, and so is log q, which
// logq_kernel sums from them.

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ f32x4 mfma16(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// max(z, +0) as an integer max of the bit pattern: equal to (z > 0 ? z : +0)
// for every non-NaN z (negative values and -0 give +0), in one instruction
__device__ __forceinline__ float relu(float z) { return __int_as_float(max(__float_as_int(z), 0)); }

// hidden activation of one element from its pre-activation z (bias
// included): relu(z) for layer 1, h + relu(z) after
__device__ __forceinline__ __bf16 hidden_out(bool first, float z, __bf16 resid) {
    const float rz = relu(z);
    return f2bf(first ? rz : bf2f(resid) + rz);
}

typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
typedef unsigned int uint4v __attribute__((ext_vector_type(4)));  // a buffer store's 128-bit data

// four consecutive output channels of one pixel / chain (the D layout below)
__device__ __forceinline__ bf16x4 hidden_out4(bool first, f32x4 z, bf16x4 resid) {
    bf16x4 h;
#pragma unroll
    for (int v = 0; v < 4; ++v) h[v] = hidden_out(first, z[v], resid[v]);
    return h;
}

// the same element arithmetic with the residual input already widened to fp32
__device__ __forceinline__ bf16x4 hidden_out4f(bool first, f32x4 z, f32x4 resid) {
    bf16x4 h;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const float rz = relu(z[v]);
        h[v] = f2bf(first ? rz : resid[v] + rz);
    }
    return h;
}

// four bf16 values widened to fp32 exactly (a bf16 is the top half of its fp32)
__device__ __forceinline__ f32x4 widen4(bf16x4 h) {
    const uint2 b = __builtin_bit_cast(uint2, h);
    return f32x4{__uint_as_float(b.x << 16), __uint_as_float(b.x & 0xffff0000u), __uint_as_float(b.y << 16),
                 __uint_as_float(b.y & 0xffff0000u)};
}

// D layout -> B fragment inside a wavefront.  Lane (j, g) (j = lane % 16,
// g = lane / 16) holds channels 4g..4g+3 (h0) and 16+4g..16+4g+3 (h1) of
// column j; the B operand wants channels 8g..8g+7 of the same column, i.e.
// half g / 2 of the lanes in rows 2 (g % 2) and 2 (g % 2) + 1.  Per packed
// dword, a 32-lane swap (rows 2,3 of h0 <-> rows 0,1 of h1) followed by a
// 16-lane swap (odd rows of the first <-> even rows of the second) leaves
// the first four channels in the first register and the last four in the
// second.
__device__ __forceinline__ bf16x8 regroup(bf16x4 h0, bf16x4 h1) {
    const uint2 a = __builtin_bit_cast(uint2, h0), b = __builtin_bit_cast(uint2, h1);
    const auto s0 = __builtin_amdgcn_permlane32_swap(a.x, b.x, false, false);
    const auto t0 = __builtin_amdgcn_permlane16_swap(s0[0], s0[1], false, false);
    const auto s1 = __builtin_amdgcn_permlane32_swap(a.y, b.y, false, false);
    const auto t1 = __builtin_amdgcn_permlane16_swap(s1[0], s1[1], false, false);
    const uint4 o = {t0[0], t1[0], t0[1], t1[1]};
    return __builtin_bit_cast(bf16x8, o);
}

// B fragment -> D layout: the inverse of regroup (each swap is its own inverse)
__device__ __forceinline__ void ungroup(bf16x8 x, bf16x4& h0, bf16x4& h1) {
    const uint4 o = __builtin_bit_cast(uint4, x);
    const auto s0 = __builtin_amdgcn_permlane16_swap(o.x, o.z, false, false);
    const auto t0 = __builtin_amdgcn_permlane32_swap(s0[0], s0[1], false, false);
    const auto s1 = __builtin_amdgcn_permlane16_swap(o.y, o.w, false, false);
    const auto t1 = __builtin_amdgcn_permlane32_swap(s1[0], s1[1], false, false);
    h0 = __builtin_bit_cast(bf16x4, uint2{t0[0], t1[0]});
    h1 = __builtin_bit_cast(bf16x4, uint2{t0[1], t1[1]});
}

__device__ __forceinline__ bf16x4 zero4() {
    bf16x4 z;
#pragma unroll
    for (int v = 0; v < 4; ++v) z[v] = (__bf16)0.0f;
    return z;
}

// Scorer layer: one wavefront per 16 pixels x 32 output channels.
// 16x16x32 operand layout: A row = lane % 16, k = 8 (lane / 16) + e; B column
// = lane % 16, same k; D column lane % 16, rows 4 (lane / 16) + v.  The
// weights are the A operand (rows = output channels of a 16-block) and the
// activations the B operand (columns = pixels), so a lane's D values are four
// consecutive output channels of its own pixel.
// bias: this layer's row of the bias table (rows kCondOut apart; the row of
// pixel p is that of its configuration's point pt[p / L^2], or row 0 if pt is
// nullptr)
__global__ void __launch_bounds__(256) conv16_kernel(const __bf16* __restrict__ in, const __bf16* __restrict__ Wl,
                                                     const float* __restrict__ bias, const int32_t* __restrict__ pt,
                                                     int npts, int layer, int L, int64_t P,
                                                     __bf16* __restrict__ out, float* __restrict__ logit) {
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15, kg = lane >> 4;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t w0 = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const bool first = layer == 0, last = layer == NL - 1;
    const Taps taps = taps_for_dev(layer);
    bf16x8 Wa[NT][2];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
            Wa[t][cb] = (t < taps.n) ? load8(Wl + ((int64_t)t * C + 16 * cb + r16) * C + kg * 8) : zero8();
    const int64_t ntiles = (P + 15) / 16;
    const uint32_t LL = (uint32_t)(L * L);  // pixel indices fit 32 bits
    for (int64_t tile = w0; tile < ntiles; tile += nw) {
        const int64_t p = tile * 16 + r16;
        const float* brow = bias + (pt ? (int64_t)clamp_point(pt[(uint32_t)(p < P ? p : P - 1) / LL], npts) * kCondOut : 0);
        const f32x4 bj0 = *reinterpret_cast<const f32x4*>(brow + 4 * kg);
        const f32x4 bj1 = *reinterpret_cast<const f32x4*>(brow + 16 + 4 * kg);
        f32x4 acc0 = bj0, acc1 = bj1;
        const uint32_t ef = edge_flags(p < P ? p : 0, L);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (t >= taps.n) break;
            const int64_t q = (p < P) ? shift_pix(p, ef, taps.dr[t], taps.dc[t], L) : -1;
            const bf16x8 a = (q >= 0) ? load8(in + q * C + kg * 8) : zero8();
            acc0 = mfma16(Wa[t][0], a, acc0);
            if (!last) acc1 = mfma16(Wa[t][1], a, acc1);
        }
        if (p >= P) continue;
        if (last) {
            if (kg == 0) logit[p] = acc0[0];
        } else {
            const int64_t o0 = p * C + 4 * kg, o1 = o0 + 16;
            const bf16x4 r0 = first ? zero4() : *reinterpret_cast<const bf16x4*>(in + o0);
            const bf16x4 r1 = first ? zero4() : *reinterpret_cast<const bf16x4*>(in + o1);
            *reinterpret_cast<bf16x4*>(out + o0) = hidden_out4(first, acc0, r0);
            *reinterpret_cast<bf16x4*>(out + o1) = hidden_out4(first, acc1, r1);
        }
    }
}

// LDS rows of 32 bf16 channels (64 bytes) with their four 16-byte groups
// XOR-swizzled by bits 1-2 of the row index.  A 16-byte read is served eight
// lanes at a time over 32 four-byte banks; eight consecutive rows at one
// group then land on eight distinct bank quads (row parity picks the half,
// the swizzle the quad within it), so the reads of consecutive rows or
// output channels are free of bank conflicts.
__device__ __forceinline__ int swz(int row, int grp) { return row * C + ((grp ^ ((row >> 1) & 3)) << 3); }
__device__ __forceinline__ int swz_el(int row, int ch) { return swz(row, ch >> 3) + (ch & 7); }

// Fused scorer: one workgroup of four wavefronts per configuration, all 12
// layers with the activations of the whole lattice in LDS, so only the spins
// are read and the logits written.  Both activation buffers carry a zero
// border (one row above, one column on each side: (L+1) x (L+2) pixels of 32
// bf16 channels, rows XOR-swizzled), so every tap reads a valid address and
// out-of-lattice taps read zeros, as in the sampler.  Wavefront w takes the
// 16-pixel tiles w, w + 4, ... of each layer; per tile it runs the same five
// 16x16x32 instructions per 16-channel block, in the same order and with the
// same epilogue as conv16_kernel and the sampler.  Used for L <= kFuseMaxL.
constexpr int kFuseMaxL = 32;

// padded pixels per buffer, a multiple of 8 so that both buffers start on a
// 512-byte boundary (the address arithmetic below relies on it)
__host__ __device__ constexpr int fused_pixels(int L) { return ((L + 1) * (L + 2) + 7) / 8 * 8; }

__global__ void __launch_bounds__(256) score_fused_kernel(int64_t n, int L, const int8_t* __restrict__ spins,
                                                          const __bf16* __restrict__ wf,
                                                          const float* __restrict__ bias_tab,
                                                          const int32_t* __restrict__ pt, int npts,
                                                          float* __restrict__ logit) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = L * L, W2 = L + 2, PP = fused_pixels(L);
    __bf16* buf0 = reinterpret_cast<__bf16*>(smem);  // two buffers of PP pixels: layer input and output
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int r16 = lane & 15, kg = lane >> 4;
    const int64_t b = blockIdx.x;
    if (b >= n) return;  // uniform per workgroup
    const int8_t* sp = spins + b * N;
    const float* bias = bias_tab + (pt ? (int64_t)clamp_point(pt[b], npts) * kCondOut : 0);  // [NL][C]
    // both buffers: zeros everywhere (the border stays zero), then the spins
    for (int g = tid; g < 2 * PP * 4; g += blockDim.x) *reinterpret_cast<bf16x8*>(buf0 + g * 8) = zero8();
    __syncthreads();
    for (int p = tid; p < N; p += blockDim.x) {
        const int r = p / L, c = p - (p / L) * L;
        buf0[swz_el((r + 1) * W2 + c + 1, 0)] = f2bf((float)sp[p]);
    }
    const int ntiles = (N + 15) / 16;
    // this lane's B-column pixel in its wavefront's first tile, and the step to
    // the next tile (64 pixels on) in rows and columns
    const int p0 = w * 16 + r16, r0 = p0 / L, c0 = p0 - r0 * L;
    const int dr64 = 64 / L, dc64 = 64 - dr64 * L;
    const int plast = (L + 1) * W2 - 2;  // padded index of pixel N - 1 (row L-1, column L-1)
    const int toff[NT] = {-W2 - 1, -W2, -W2 + 1, -1, 0};
    // Byte address of (row, group kg) in a buffer at byte offset `base` (a
    // multiple of 512): with u = base / 8 + 8 row it is swz(row, kg) * 2 + base
    // = 8 u | ((u ^ 16 kg) & 0x30), because bits 4-5 of u are bits 1-2 of row.
    const uint32_t kg16 = 16u * kg;
    auto lds_at = [&](uint32_t u) -> uint32_t { return (u << 3) | ((u ^ kg16) & 0x30u); };
    __syncthreads();
    uint32_t in_u = 0, out_u = (uint32_t)PP * C * 2 / 8;  // buffer base / 8
    // A fragments and biases of a layer; the next layer's are loaded before
    // the barrier that ends the current one
    bf16x8 Wa[NT][2], Wn[NT][2];
    f32x4 bj0, bj1, bn0, bn1;
    auto load_w = [&](int l, bf16x8 (&W)[NT][2], f32x4& b0, f32x4& b1) {
        const __bf16* Wl = wf + (int64_t)l * NT * C * C;
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) W[t][cb] = load8(Wl + ((int64_t)t * C + 16 * cb + r16) * C + kg * 8);
        b0 = *reinterpret_cast<const f32x4*>(bias + l * C + 4 * kg);
        b1 = *reinterpret_cast<const f32x4*>(bias + l * C + 16 + 4 * kg);
    };
    load_w(0, Wa, bj0, bj1);
    // one layer over this wavefront's tiles; K = 0 first layer (four taps, no
    // residual), 1 hidden layer, 2 last layer (the logit only)
    auto pass = [&](auto kind) {
        constexpr int K = decltype(kind)::value;
        constexpr bool first = K == 0, last = K == 2;
        constexpr int nt = first ? 4 : 5;
        int r = r0, c = c0;
#pragma unroll 1
        for (int tile = w; tile < ntiles; tile += 4) {
            // the ragged tail reads a valid pixel; its outputs are dropped
            const bool live = tile * 16 + r16 < N;
            const int pid = live ? (r + 1) * W2 + c + 1 : plast;
            bf16x8 a[NT];
            const uint32_t u = in_u + 8u * (uint32_t)pid;
#pragma unroll
            for (int t = 0; t < nt; ++t)
                a[t] = *reinterpret_cast<const bf16x8*>(smem + lds_at(u + 8 * toff[t]));
            f32x4 acc0 = bj0, acc1 = bj1;
#pragma unroll
            for (int t = 0; t < nt; ++t) {
                acc0 = mfma16(Wa[t][0], a[t], acc0);
                if (!last) acc1 = mfma16(Wa[t][1], a[t], acc1);
            }
            if (last) {
                if (live && kg == 0) logit[b * N + tile * 16 + r16] = acc0[0];
            } else {
                // the residual inputs are the centre tap's operand in the D layout
                f32x4 rf0 = {0.f, 0.f, 0.f, 0.f}, rf1 = rf0;
                if (!first) {
                    bf16x4 h0, h1;
                    ungroup(a[4], h0, h1);
                    rf0 = widen4(h0);
                    rf1 = widen4(h1);
                }
                const bf16x8 o = regroup(hidden_out4f(first, acc0, rf0), hidden_out4f(first, acc1, rf1));
                if (live) *reinterpret_cast<bf16x8*>(smem + lds_at(out_u + 8u * (uint32_t)pid)) = o;
            }
            r += dr64;
            c += dc64;
            if (c >= L) {
                c -= L;
                ++r;
            }
        }
    };
    for (int l = 0; l < NL; ++l) {
        if (l == 0)
            pass(std::integral_constant<int, 0>{});
        else if (l < NL - 1)
            pass(std::integral_constant<int, 1>{});
        else
            pass(std::integral_constant<int, 2>{});
        if (l + 1 < NL) load_w(l + 1, Wn, bn0, bn1);
        __syncthreads();
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            Wa[t][0] = Wn[t][0];
            Wa[t][1] = Wn[t][1];
        }
        bj0 = bn0;
        bj1 = bn1;
        const uint32_t t_ = in_u;
        in_u = out_u;
        out_u = t_;
    }
}

// Ancestral sampler.  Each wavefront draws 16 configurations site by site in
// raster order and computes every layer and all 32 channels of its own
// chains, so the wavefronts of a workgroup (1, 2 or 4 of them, sharing the
// packed weights in LDS) never wait for each other inside the site loop.  Per
// layer the weights are the A operand (rows = output channels, two halves of
// 16) and the activations the B operand (columns = chains): a lane ends the
// layer with four consecutive channels of each half for its chain, and two
// lane swaps per register regroup them into the next layer's B fragment.
// The operand of the (0,-1) tap is the fragment each lane used at the
// previous site; the taps of the row above come from a one-row ring in global
// memory, each element read once into a window that slides along the row.
// Ring accesses are buffer loads and stores: a wavefront-uniform descriptor
// (this wavefront's slot of a layer and column, or a zero block of the same
// shape outside the lattice) plus the lane's fixed byte offset, so no address
// arithmetic runs per access.  Each lane reads the weights from LDS at two
// base addresses (layers 0-5 and 6-11) plus immediate offsets.
// The weights of the next layer are loaded while a layer finishes.  Spin i is
// +1 iff u < up_threshold(logit), u = word 0 of Philox (ctr = (site, step,
// chain, id << 3 | 6)), decided by the lane that holds the logit at the end of
// the last layer; the logits go to logit_out for the log q sum.
// Up to 4 wavefronts per workgroup: one per SIMD.  (The kernel needs about
// 290 registers per lane; capped at 256 so that two wavefronts share a SIMD
// it spills inside the layer loop and runs slower: 32768 proposals at 18x18
// took 7.5 ms against 4.7 ms in two rounds of one wavefront per SIMD.)
constexpr int kSeqMaxWaves = 4;
// MH: proposals of several cycles per sampler launch, up to this many chains
// (1024 wavefronts of 16 chains: one per SIMD) and this many cycles
constexpr int64_t kMhBatchChains = 16384, kMhMaxBatch = 8;
constexpr int kSeqPad = 16 * kSeqMaxWaves;  // the ring's chain count is a multiple of this
constexpr int kSeqLdsBytes = NL * NT * C * C * 2 + NL * C * 4;  // weights, then the shared biases

// bias_tab: the bias table (rows kCondOut apart).  PER_CHAIN: chain i reads
// row pt[i] (clamped to [0, npts)) from global memory; else every chain reads
// row 0, staged in LDS with the weights (a global read in each layer's
// dependency chain would add its latency to every layer step).
template <bool PER_CHAIN>
__global__ void __launch_bounds__(256) seq_kernel(int64_t n, int64_t npad, int L, const __bf16* __restrict__ wf,
                                                  const float* __restrict__ bias_tab, const int32_t* __restrict__ pt,
                                                  int npts, __bf16* __restrict__ ring,
                                                  const __bf16* __restrict__ zpad, int8_t* __restrict__ spins,
                                                  float* __restrict__ logit_out, uint64_t seed, uint32_t step,
                                                  uint32_t id, int64_t n_step) {
    extern __shared__ __align__(16) unsigned char smem[];
    __bf16* wl = reinterpret_cast<__bf16*>(smem);                 // [NL][NT][C][C], rows swizzled
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int r16 = lane & 15, kg = lane >> 4;
    float* bsh = reinterpret_cast<float*>(wl + NL * NT * C * C);  // [NL][C] shared biases (not PER_CHAIN)
    for (int g = tid; g < NL * NT * C * 4; g += blockDim.x) {
        const int row = g >> 2, grp = g & 3;
        *reinterpret_cast<bf16x8*>(wl + swz(row, grp)) = load8(wf + (int64_t)row * C + grp * 8);
    }
    if (!PER_CHAIN)
        for (int g = tid; g < NL * C; g += blockDim.x) bsh[g] = bias_tab[g];
    __syncthreads();
    // wavefront-uniform by construction; readfirstlane lets the compiler keep it (and the ring base) scalar
    const int64_t wbase = (int64_t)blockIdx.x * (blockDim.x >> 2) + 16 * __builtin_amdgcn_readfirstlane(w);
    if (wbase >= n) return;  // no further workgroup barrier below
    // Operand roles: A row = output channel 16 h + r16 (h = half), B / D column
    // = chain r16 of this wavefront; a lane's D values of half h are channels
    // 16 h + 4 kg .. + 3 of its chain.
    const int64_t gca = wbase + r16;  // the ring has npad >= grid size chains: padding rows have their own slots
    // proposal gca of the launch is chain gca % n_step of batch gca / n_step:
    // its random stream, and its point, are those of a launch of that batch alone
    const int64_t gcr = gca % n_step;
    const uint32_t stepr = step + (uint32_t)(gca / n_step);
    const int N = L * L;
    // this lane's chain's bias rows (padding chains read the last chain's)
    const float* bl =
        PER_CHAIN ? bias_tab + (int64_t)clamp_point(pt[gca < n ? gcr : (n - 1) % n_step], npts) * kCondOut : bsh;
    // Ring element (layer, chain, column, channel): [NL][npad][L][C], one row
    // per chain and layer.  Site (r, c) writes column c after the row above's
    // column c was last read (as the (-1,+1) tap of site (r, c - 1)), so the
    // slots of a row hold row r at columns < c and row r - 1 from c on.
    // Addresses are a wavefront-uniform part (this wavefront's first chain,
    // layer, column) plus a per-lane 32-bit byte offset (chain within the
    // wavefront, channel group) fixed for the whole kernel.
    const int64_t chain_stride = (int64_t)L * C;
    const int64_t ring_layer = npad * chain_stride;
    const __bf16* ring_w = ring + wbase * chain_stride;
    const uint32_t rd_off = (uint32_t)(r16 * chain_stride + kg * 8) * 2;  // bytes: B fragment of the lane
    auto slot = [&](int l, int c) -> int64_t { return (int64_t)l * ring_layer + (int64_t)c * C; };  // uniform
    // buffer descriptor of a wavefront-uniform base covering 16 chains' rows (nrec bytes)
    const int nrec = (int)(16 * chain_stride * 2);
    auto rsrc = [&](const __bf16* base) {
        // readfirstlane returns a signed int: widen each half through uint32_t,
        // or a low half with bit 31 set would fill the high half with ones
        const uint64_t v = reinterpret_cast<uint64_t>(base);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
        const uint64_t u = ((uint64_t)hi << 32) | (uint64_t)lo;
        return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(u), (short)0, nrec, 0x00020000);
    };
    auto fetch = [&](int l, bool inside, int c) -> bf16x8 {  // `inside` is wavefront-uniform
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(rsrc(inside ? ring_w + slot(l, c) : zpad), rd_off, 0, 0);
        return __builtin_bit_cast(bf16x8, v);
    };
    // A fragments of layer l for both halves (the centre tap is masked in the first layer, the last
    // layer has one output channel)
    bf16x8 bw0[NT], bw1[NT];
    f32x4 bj0, bj1;  // biases of the lane's output channels: the accumulators' initial values
    // this lane's A fragments at two bases, so that every load is a base plus an
    // immediate offset below 64 KiB (row 16 + r16 is 16 rows after row r16: the
    // swizzle depends on the row's low bits only)
    const char* const wb_lo = reinterpret_cast<const char*>(wl + swz(r16, kg));
    uint32_t hi_off = 2u * 6u * NT * C * C;
    asm volatile("" : "+v"(hi_off));  // keeps the second base a register of its own
    const char* const wb_hi = wb_lo + hi_off;
    auto load_w = [&](int l) {
        const char* Wl = l < 6 ? wb_lo + 2 * l * NT * C * C : wb_hi + 2 * (l - 6) * NT * C * C;
        bj0 = *reinterpret_cast<const f32x4*>(bl + l * C + 4 * kg);
        bj1 = *reinterpret_cast<const f32x4*>(bl + l * C + 16 + 4 * kg);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const bool used = t < 4 || l > 0;
            bw0[t] = used ? *reinterpret_cast<const bf16x8*>(Wl + 2 * t * C * C) : zero8();
            bw1[t] = (used && l < NL - 1) ? *reinterpret_cast<const bf16x8*>(Wl + 2 * (t * C * C + 16 * C)) : zero8();
        }
    };
    // B fragments per layer l: the row above at columns c - 1 and c (a
    // window that slides by one column per site and is refilled at a row
    // end), at column c + 1 (prefetched three layers ahead into slot l % 3),
    // and h_l at the previous site (l = 0: its spin; zero at a row start).
    constexpr int kAhead = 3;
    bf16x8 up0[NL], up1[NL], left[NL], pr[kAhead], sv[NL];
    // ring fragment of layer m at column c: an even column's waits in sv for the odd one
    auto store_pair = [&](int m, int c, const bf16x8& f, auto par) {
        if (decltype(par)::value == 0) {
            sv[m] = f;
        } else {
            const auto rw = rsrc(ring_w + slot(m, c - 1));
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(uint4v, sv[m]), rw, rd_off, 0, 0);
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(uint4v, f), rw, rd_off + 2u * C, 0, 0);
        }
    };
#pragma unroll
    for (int l = 0; l < NL; ++l) up0[l] = up1[l] = zero8();
#pragma unroll
    for (int l = 0; l < kAhead; ++l) pr[l] = zero8();  // row 0 has no row above
    f32x4 hp0 = {0.f, 0.f, 0.f, 0.f}, hp1 = hp0;  // h_l of this lane's outputs as floats: the residual inputs
    bf16x8 hb = zero8();                           // h_l as this lane's B fragment: the centre tap's operand
    load_w(0);
    // One site; PAR = its column's parity.  L is even, so the sites of a row
    // pair up: an even site keeps its layers' ring fragments (sv) and the odd
    // site after it stores both columns together, each chain's 128-byte line
    // whole (a column alone left half-written lines, which cost memory-side
    // reads).  A column is first read a row later, so the delay is safe.
    auto do_site = [&](int site, auto par) {
        constexpr int PAR = decltype(par)::value;
        const int r = site / L, c = site - r * L;
        const int sn = site + 1, rn = sn / L, cn = sn - rn * L;
        const bool more = sn < N;
        // PER_CHAIN: an empty statement that marks the bias row pointer as
        // modified, so the bias loads stay in the loop (vector-memory reads
        // that hit the cache) instead of being hoisted into registers that
        // every layer must copy
        if (PER_CHAIN) asm volatile("" : "+v"(bl));
        if (c == 0) {  // a row start: no left neighbour; the row above at columns -1 (outside) and 0
#pragma unroll
            for (int l = 0; l < NL; ++l) left[l] = zero8();
            if (r > 0) {
#pragma unroll
                for (int l = 0; l < NL; ++l) {
                    up0[l] = zero8();
                    up1[l] = fetch(l, true, 0);
                }
            }
        }
        const gk::P4 q = gk::philox((uint32_t)site, stepr, (uint32_t)gcr, (id << 3) | 6u, (uint32_t)seed,
                                    (uint32_t)(seed >> 32));
        const uint32_t u = q.v[0];
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const bool last = l == NL - 1;
            const bf16x8 op[4] = {up0[l], up1[l], pr[l % kAhead], left[l]};
            f32x4 acc0 = bj0, acc1 = bj1;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                acc0 = mfma16(bw0[t], op[t], acc0);
                if (!last) acc1 = mfma16(bw1[t], op[t], acc1);
            }
            if (l > 0) {
                acc0 = mfma16(bw0[4], hb, acc0);
                if (!last) acc1 = mfma16(bw1[4], hb, acc1);
                left[l] = hb;
            }
            // the next layer's weights (of this site or the next) load while this one finishes
            if (l + 1 < NL)
                load_w(l + 1);
            else if (more)
                load_w(0);
            // slide the window (a row start refills it)
            up0[l] = up1[l];
            up1[l] = pr[l % kAhead];
            if (!last) {
                const bf16x4 h0 = hidden_out4f(l == 0, acc0, hp0);
                const bf16x4 h1 = hidden_out4f(l == 0, acc1, hp1);
                hb = regroup(h0, h1);
                // the ring keeps the B fragment: 16 bytes per lane, 64 per chain and column
                store_pair(l + 1, c, hb, par);
                hp0 = widen4(h0);
                hp1 = widen4(h1);
            } else {
                // the logit is output channel 0: element 0 of the lanes with kg == 0
                const float x = acc0[0];
                const bool up = u < up_threshold(x);
                const __bf16 sg = f2bf(up ? 1.f : -1.f);
                bf16x8 s8 = zero8();
                if (kg == 0) {
                    s8[0] = sg;  // the first layer's input fragment: channel 0 is the spin, the rest 0
                    if (gca < n) {
                        spins[gca * N + site] = (int8_t)bf2f(sg);
                        logit_out[gca * N + site] = x;
                    }
                }
                store_pair(0, c, s8, par);
                left[0] = s8;
            }
            wave_sync();  // this layer's ring stores precede every later ring load
            // refill this prefetch slot: column c + 1 of the row above for layer l + 3 of this site, or of
            // the next site
            if (l + kAhead < NL)
                pr[l % kAhead] = fetch(l + kAhead, r > 0 && c + 1 < L, c + 1);
            else if (more)
                pr[l % kAhead] = fetch(l + kAhead - NL, rn > 0 && cn + 1 < L, cn + 1);
        }
    };
    for (int site = 0; site < N; site += 2) {
        do_site(site, std::integral_constant<int, 0>{});
        do_site(site + 1, std::integral_constant<int, 1>{});
    }
}

// Minibatch of a training run: sample b of step `step` is training sample
// idx = floor(u64 n / 2^64) with u64 = (out[0] << 32 | out[1]) of Philox
// (ctr = (b, step, 0, 7), key = seed), moved by a lattice symmetry of the
// periodic Shastry-Sutherland lattice: rolled by (dr, dc) = (2 (out[2] mod
// L/2), 2 ((out[3] >> 1) mod L/2)) sites (even translations map the dimer
// pattern onto itself), then transposed if out[3] is odd (the transpose maps
// both dimer orientations onto themselves).  out[r][c] = in[(r - dr) mod L]
// [(c - dc) mod L] before the transpose.  One workgroup per sample.
__global__ void __launch_bounds__(256) gather_batch_kernel(const int8_t* __restrict__ samples,
                                                           const int32_t* __restrict__ pts_in, int64_t n, int L,
                                                           uint64_t seed, uint32_t step, int augment,
                                                           int8_t* __restrict__ out, int32_t* __restrict__ pts_out,
                                                           int64_t* __restrict__ idx_out) {
    const int64_t b = blockIdx.x;
    const gk::P4 q = gk::philox((uint32_t)b, step, 0u, 7u, (uint32_t)seed, (uint32_t)(seed >> 32));
    const uint64_t u = ((uint64_t)q.v[0] << 32) | q.v[1];
    const int64_t idx = (int64_t)__umul64hi(u, (uint64_t)n);
    const int half = L / 2;
    const int dr = augment ? 2 * (int)(q.v[2] % (uint32_t)half) : 0;
    const int dc = augment ? 2 * (int)((q.v[3] >> 1) % (uint32_t)half) : 0;
    const bool tr = augment && (q.v[3] & 1u);
    const int N = L * L;
    const int8_t* src = samples + idx * N;
    int8_t* dst = out + b * N;
    for (int p = threadIdx.x; p < N; p += blockDim.x) {
        int r = p / L, c = p - (p / L) * L;
        if (tr) {
            const int t = r;
            r = c;
            c = t;
        }
        int rs = r - dr, cs = c - dc;
        rs += rs < 0 ? L : 0;
        cs += cs < 0 ? L : 0;
        dst[p] = src[rs * L + cs];
    }
    if (threadIdx.x == 0) {
        if (pts_out) pts_out[b] = pts_in ? pts_in[idx] : 0;
        if (idx_out) idx_out[b] = idx;
    }
}

}  // namespace ar
}  // namespace crbmlib

// ---------------------------------------------------------------- host side

namespace crbmlib {
namespace ar {

// Exact integer (M, B1, B2) of int8 configurations, one wavefront per chain;
// with ord != nullptr also the plateau structure factor record
// (max, |S_A|^2, |S_B|^2) from A_k = sum (-1)^r s over columns = k (mod 3) and
// B_k = sum (-1)^c s over rows = k (mod 3).
__global__ void __launch_bounds__(256) counts_int8_kernel(const int8_t* s, int64_t n, int L, int32_t* out,
                                                          int32_t* ord) {
    const int lane = threadIdx.x & 63;
    const int64_t ch = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (ch >= n) return;  // uniform per wavefront
    const int8_t* x = s + ch * L * L;
    int M = 0, B1 = 0, B2 = 0;
    int A[3] = {0, 0, 0}, B[3] = {0, 0, 0};
    for (int i = lane; i < L * L; i += 64) {
        const int r = i / L, c = i - (i / L) * L;
        const int v = x[i];
        const int va = (r & 1) ? -v : v, vb = (c & 1) ? -v : v, cm = c % 3, rm = r % 3;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            A[k] += (cm == k) ? va : 0;
            B[k] += (rm == k) ? vb : 0;
        }
        M += v;
        B1 += v * x[r * L + (c + 1) % L] + v * x[((r + 1) % L) * L + c];
        if ((r & 1) == 0 && (c & 1) == 0) B2 += v * x[(r + 1) * L + c + 1];          // '\\' dimer
        if ((r & 1) == 1 && (c & 1) == 0) B2 += v * x[((r + 1) % L) * L + (c + L - 1) % L];  // '/' dimer
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        M += __shfl_xor(M, d);
        B1 += __shfl_xor(B1, d);
        B2 += __shfl_xor(B2, d);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            A[k] += __shfl_xor(A[k], d);
            B[k] += __shfl_xor(B[k], d);
        }
    }
    if (lane == 0) {
        out[ch * 3] = M;
        out[ch * 3 + 1] = B1;
        out[ch * 3 + 2] = B2;
        if (ord) {
            auto sq3 = [](const int (&v)[3]) {
                const int64_t p = v[0], q = v[1], t = v[2];
                return p * p + q * q + t * t - p * q - q * t - t * p;
            };
            const int64_t sa = sq3(A), sb = sq3(B);
            ord[ch * 3] = (int32_t)(sa > sb ? sa : sb);
            ord[ch * 3 + 1] = (int32_t)sa;
            ord[ch * 3 + 2] = (int32_t)sb;
        }
    }
}

// Independent MH (one thread per chain): log alpha = [log pi' - log pi] +
// [log q - log q'], log pi from the exact integer counts; accept iff
// log u < log alpha with u from Philox stream 5.
// the MH target of one instance: log pi = a M + c1 n1 + c2 n2 (+ const)
struct MhTarget {
    double a, c1, c2;
    int32_t sg1, sg2;
};

// chain ch belongs to instance ci[ch] with target tg[ci[ch]]
// One wavefront per chain: lane 0 takes the accept decision on the exact
// integer log pi_q (R16) and the two log q; on acceptance the wavefront copies
// the proposal (L^2 bytes, a multiple of 4) as 32-bit words, strided over its
// lanes, with the counts and log q.
__global__ void __launch_bounds__(256) mh_kernel(int64_t n, int L, int8_t* cur, const int8_t* prop,
                                                 int32_t* cnt_cur, const int32_t* cnt_prop, double* lq_cur,
                                                 const double* lq_prop, const MhTarget* tg, const int32_t* ci,
                                                 uint64_t seed, uint32_t step, uint32_t id,
                                                 unsigned long long* n_acc) {
    const int64_t ch = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (ch >= n) return;
    const int64_t N = (int64_t)L * L;
    int acc = 0;
    if (lane == 0) {
        const MhTarget t = tg[ci[ch]];
        auto logpi = [&](const int32_t* k) {
            const int64_t M = k[0], B1 = k[1], B2 = k[2];
            const int64_t n1 = t.sg1 < 0 ? (2 * N - B1) / 2 : (2 * N + B1) / 2;
            const int64_t n2 = t.sg2 < 0 ? (N / 2 - B2) / 2 : (N / 2 + B2) / 2;
            return t.a * (double)M + t.c1 * (double)n1 + t.c2 * (double)n2;
        };
        const double la = (logpi(cnt_prop + ch * 3) - logpi(cnt_cur + ch * 3)) + (lq_cur[ch] - lq_prop[ch]);
        const gk::P4 r = gk::philox(0u, step, (uint32_t)ch, (id << 3) | 5u, (uint32_t)seed, (uint32_t)(seed >> 32));
        const double u = ((double)(((uint64_t)r.v[0] << 21) ^ (r.v[1] >> 11)) + 0.5) * (1.0 / 9007199254740992.0);
        acc = log(u) < la ? 1 : 0;
    }
    acc = __shfl(acc, 0);
    if (!acc) return;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(prop + ch * N);
    uint32_t* dst = reinterpret_cast<uint32_t*>(cur + ch * N);
    for (int64_t w = lane; w < N / 4; w += 64) dst[w] = src[w];
    if (lane < 3) cnt_cur[ch * 3 + lane] = cnt_prop[ch * 3 + lane];
    if (lane == 0) {
        lq_cur[ch] = lq_prop[ch];
        atomicAdd(n_acc, 1ull);
    }
}

// Offset of layer l's weights in the parameter layout (each layer: its
// [T][ci][co] weights, then its co biases).
__device__ __forceinline__ int64_t layer_offset(int l) {
    int64_t off = 0;
    for (int k = 0; k < l; ++k) {
        const int Tk = (k == 0) ? 4 : 5, cik = (k == 0) ? 1 : C, cok = (k == NL - 1) ? 1 : C;
        off += (int64_t)Tk * cik * cok + cok;
    }
    return off;
}

// Layer l's gradient in the parameter layout, one launch:
// - the first wblocks workgroups: weight entry (t, i, o) is the fp64 sum of
//   the kRedSlices slices of part2 [slice][NT][C][C] (taps, input and output
//   channels beyond the layer's own are padding and skipped);
// - then one workgroup per output channel j: bias j is the sum of the nparts
//   partial sums bpart[p][j] (the last layer: bpart[p]), 256 threads each
//   adding a strided share, then a fixed-order tree in LDS (fp64).
// layer l = l0 + blockIdx.y; its slices at part2 + blockIdx.y part2_stride,
// its bias partials at bpart + blockIdx.y bpart_stride; blocks beyond the
// layer's weight blocks and bias channels return
__global__ void __launch_bounds__(256) finish_layer_grad_kernel(const double* __restrict__ part2,
                                                                int64_t part2_stride,
                                                                const float* __restrict__ bpart,
                                                                int64_t bpart_stride, int nparts, int l0,
                                                                float* __restrict__ grad) {
    const int l = l0 + (int)blockIdx.y;
    part2 += (int64_t)blockIdx.y * part2_stride;
    bpart += (int64_t)blockIdx.y * bpart_stride;
    const int T = (l == 0) ? 4 : 5, ci = (l == 0) ? 1 : C, co = (l == NL - 1) ? 1 : C;
    const int wblocks = (T * ci * co + 255) / 256;
    if ((int)blockIdx.x >= wblocks + co) return;
    const int64_t off = layer_offset(l);
    if ((int)blockIdx.x < wblocks) {
        const int x = blockIdx.x * blockDim.x + threadIdx.x;
        if (x >= T * ci * co) return;
        const int o = x % co, i = (x / co) % ci, t = x / (co * ci);
        const int64_t n = (int64_t)NT * C * C, src = ((int64_t)t * C + i) * C + o;
        double sum = 0.0;
#pragma unroll 4
        for (int k = 0; k < kRedSlices; ++k) sum += part2[k * n + src];
        grad[off + x] = (float)sum;
        return;
    }
    // the whole workgroup takes this branch (blockIdx is uniform)
    const int j = (int)blockIdx.x - wblocks;
    const int stride = (co == 1) ? 1 : C;
    double s = 0.0;
    for (int p = threadIdx.x; p < nparts; p += blockDim.x) s += bpart[(int64_t)p * stride + j];
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) grad[off + (int64_t)T * ci * co + j] = (float)red[0];
}

int64_t n_params() {
    int64_t n = 0;
    for (int l = 0; l < NL; ++l) {
        const int T = (l == 0) ? 4 : 5, ci = (l == 0) ? 1 : C, co = (l == NL - 1) ? 1 : C;
        n += (int64_t)T * ci * co + co;
    }
    return n;
}

}  // namespace ar
}  // namespace crbmlib

using namespace crbmlib;
using namespace crbmlib::ar;

struct crbm_ar_s {
    int L = 0;
    int conv_wg = 512;     // convolution workgroups that are resident at once on the device
    uint64_t seed = 0;
    hipStream_t stream = nullptr;
    int64_t np = 0;        // parameters: the network's, then (conditional) the MLP's
    int64_t np_base = 0;   // the network's
    int cond = 0;          // conditional: capacity in points (0 = unconditional)
    int npts = 0;          // points set by crbm_ar_set_points
    float* feats = nullptr;  // [cond][kCondF]
    float* cb = nullptr;     // [cond][NL][C]: per-point bias table
    float *gs = nullptr, *gp = nullptr;  // training: per-sample [B][NL][C] and per-point [cond][NL][C] bias gradients
    int64_t t_adam = 0;
    uint64_t mh_step = 0;  // MH cycles run so far: the counter word of their random streams
    float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr, *bias = nullptr;
    __bf16 *wf = nullptr, *wb = nullptr;
    // training buffers (capacity in samples)
    int64_t tcap = 0;
    __bf16* hs = nullptr;       // [NL][P][C]
    uint32_t* mask = nullptr;   // [NL-1][P]: bit j of a pixel's word = channel j of its ReLU is open
    float* logit = nullptr;     // [P]
    float* g32 = nullptr;       // [P]
    float *dh0 = nullptr, *dh1 = nullptr;  // [P][C]
    __bf16 *dz = nullptr, *g = nullptr;    // [P][C]
    double* logq = nullptr;     // [B]
    float *part = nullptr, *bpart = nullptr;
    double* part2 = nullptr;                // [kRedSlices][NT][C][C]
    int8_t* spins_copy = nullptr;
    __bf16* dzs = nullptr;      // fused backward: dz of layers 0 .. NL-2, [NL-1][P][C]
    float* bpl = nullptr;       // fused backward: per-configuration bias partials, [NL][B][C]
    // sequential sampler buffers (capacity in chains)
    int64_t scap = 0;
    __bf16* ring = nullptr;     // [NL][n][2][L][C]: activations of the last two rows
    float* slogit = nullptr;    // [n][N]
    __bf16* zpad = nullptr;     // [16][L][C] zeros: the sampler's row-above operand outside the lattice
    // scoring buffers (capacity in chains): ping-pong activations and logits
    int64_t icap = 0;
    __bf16 *ih0 = nullptr, *ih1 = nullptr;  // [n N][C]
    float* ilogit = nullptr;                // [n N]
    // MH buffers
    int64_t mcap = 0;
    int32_t* mh_ci = nullptr;   // [chains]: instance (= point) of each chain
    MhTarget* mh_tg = nullptr;  // [kCondMaxPoints or instances]: per-instance targets
    int mh_tgcap = 0;
    int8_t* cur = nullptr;
    int32_t *ccur = nullptr, *cprop = nullptr;
    double* lqc = nullptr;
    unsigned long long* nacc = nullptr;
    // proposals of up to mh_kcap cycles of mh_kn chains: [cycle][chain][N] and [cycle][chain],
    // two sets: the sampler fills one on its own stream while MH consumes the other
    int64_t mh_kcap = 0, mh_kn = 0;
    int8_t* mh_prop = nullptr;
    double* mh_lqp = nullptr;
    int8_t* mh_prop2 = nullptr;
    double* mh_lqp2 = nullptr;
    hipStream_t side = nullptr;  // MH's sampler stream (default priority), created on first use
    hipEvent_t ev_in = nullptr, ev_ready[2] = {nullptr, nullptr}, ev_free[2] = {nullptr, nullptr};
    // crbm_ar_train: the current minibatch and its points (capacity in samples)
    int64_t bcap = 0;
    int8_t* bspins = nullptr;
    int32_t* bpts = nullptr;
    ~crbm_ar_s() {
        void* ps[] = {theta, grad, m, v, bias, wf, wb, hs, mask, logit, g32, dh0, dh1, dz, g, logq, part, bpart,
                      part2, dzs, bpl,
                      spins_copy, ring, slogit, zpad, ih0, ih1, ilogit, cur, ccur, cprop, lqc, nacc,
                      feats, cb, gs, gp, mh_ci, mh_tg, mh_prop, mh_lqp, mh_prop2, mh_lqp2, bspins, bpts};
        for (void* p : ps)
            if (p) (void)hipFree(p);
        hipEvent_t evs[] = {ev_in, ev_ready[0], ev_ready[1], ev_free[0], ev_free[1]};
        for (hipEvent_t e : evs)
            if (e) (void)hipEventDestroy(e);
        if (side) (void)hipStreamDestroy(side);
    }
};

namespace {

int fail_ar(int code, const char* msg) { return set_error(code, msg); }

#define AR_TRY(expr, what)                                                              \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) return fail_ar(CRBM_EHIP, (std::string(what) + ": " + hipGetErrorString(e_)).c_str()); \
    } while (0)

template <class T>
hipError_t alloc(T** p, int64_t n) {
    return dev_alloc(p, sizeof(T) * (size_t)(n > 0 ? n : 1));
}

// weight-gradient chunks of a batch of P pixels
int64_t wgrad_chunks(int64_t P) { return (P + kWChunk - 1) / kWChunk; }

// The convolution kernels index pixels in 32 bits.
constexpr int64_t kMaxPixels = (int64_t)1 << 31;

int ensure_train(crbm_ar_t* a, int64_t B) {
    if (B <= a->tcap) return CRBM_OK;
    if (B > (kMaxPixels - 1) / ((int64_t)a->L * a->L)) return fail_ar(CRBM_EINVAL, "batch too large (samples x L^2 must be below 2^31)");
    void* ps[] = {a->hs, a->mask, a->logit, a->g32, a->dh0, a->dh1, a->dz, a->g, a->logq, a->part, a->bpart,
                  a->spins_copy, a->part2, a->gs, a->dzs, a->bpl};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    // every pointer is cleared: an allocation that fails part-way leaves the
    // rest null, so neither a later call nor the destructor frees them twice
    a->hs = nullptr;
    a->mask = nullptr;
    a->logit = a->g32 = nullptr;
    a->dh0 = a->dh1 = nullptr;
    a->dz = a->g = nullptr;
    a->logq = nullptr;
    a->part = a->bpart = nullptr;
    a->spins_copy = nullptr;
    a->part2 = nullptr;
    a->gs = nullptr;
    a->dzs = nullptr;
    a->bpl = nullptr;
    a->tcap = 0;
    const int64_t P = B * a->L * a->L;
    const int64_t nch = wgrad_chunks(P);
    if (alloc(&a->hs, (int64_t)NL * P * C) || alloc(&a->mask, (int64_t)(NL - 1) * P) || alloc(&a->logit, P) ||
        alloc(&a->g32, P) || alloc(&a->dh0, P * C) || alloc(&a->dh1, P * C) || alloc(&a->dz, P * C) ||
        alloc(&a->g, P * C) || alloc(&a->logq, B) ||
        alloc(&a->part, (a->L <= kBwdMaxL ? NL : 1) * nch * NT * C * C) ||
        alloc(&a->bpart, (int64_t)std::max<int64_t>(4096, 4 * (int64_t)a->conv_wg) * C) || alloc(&a->spins_copy, P) ||
        alloc(&a->part2, (int64_t)(a->L <= kBwdMaxL ? NL : 1) * kRedSlices * NT * C * C) || (a->cond > 0 && alloc(&a->gs, B * kCondOut)) ||
        (a->L <= kBwdMaxL && (alloc(&a->dzs, (int64_t)(NL - 1) * P * C) || alloc(&a->bpl, (int64_t)NL * B * C)))) {
        a->tcap = 0;
        return fail_ar(CRBM_ENOMEM, "training buffers");
    }
    a->tcap = B;
    return CRBM_OK;
}

int ensure_seq(crbm_ar_t* a, int64_t n) {
    if (n <= a->scap) return CRBM_OK;
    if (a->ring) (void)hipFree(a->ring);
    if (a->slogit) (void)hipFree(a->slogit);
    a->ring = nullptr;
    a->slogit = nullptr;
    const int64_t npad = (n + kSeqPad - 1) / kSeqPad * kSeqPad;
    if (alloc(&a->ring, (int64_t)NL * npad * a->L * C) || alloc(&a->slogit, n * a->L * a->L)) {
        a->scap = 0;
        return fail_ar(CRBM_ENOMEM, "sampler buffers");
    }
    a->scap = n;
    return CRBM_OK;
}

int pack(crbm_ar_t* a) {
    hipLaunchKernelGGL(pack_kernel, dim3((NL * NT * C * C + 255) / 256), dim3(256), 0, a->stream, a->theta, a->wf, a->wb,
                       a->bias);
    if (a->cond > 0 && a->npts > 0)
        hipLaunchKernelGGL(cond_bias_kernel, dim3((unsigned)a->npts), dim3(kCondOut), 0, a->stream,
                           a->theta + a->np_base, a->feats, a->bias, a->cb);
    AR_TRY(hipGetLastError(), "pack");
    return CRBM_OK;
}

// the bias table the kernels read, the point map they use, and its size:
// the per-point table of a conditional network, else the layer biases
struct BiasSel {
    const float* tab;
    const int32_t* pt;
    int npts;
};
BiasSel bias_sel(const crbm_ar_t* a, const int32_t* pt) {
    if (a->cond > 0) return {a->cb, pt, a->npts};
    return {a->bias, nullptr, 1};
}

// Workgroups of the forward / data-gradient convolution: as many as are
// resident at once (cap: compute units x the kernel's occupancy in
// workgroups), each wavefront looping over 32-pixel tiles with its weight
// fragments loaded once and the next tile's operands loading during the
// current tile's epilogue.  At 1024-sample batches this beats one tile per
// wavefront, and also half or 1.5x the resident count.
int conv_blocks(int64_t P, int cap) {
    const int64_t tiles = (P + 31) / 32;
    const int64_t b = (tiles + 3) / 4;
    return (int)(b < cap ? (b > 0 ? b : 1) : cap);
}

// forward + loss + backward into a->grad; per-sample log q into a->logq.
// pt: point of each sample (conditional network), or nullptr (point 0)
int grad_pass(crbm_ar_t* a, const int8_t* spins, int64_t B, const int32_t* pt) {
    const BiasSel bs = bias_sel(a, pt);
    const int L = a->L;
    const int64_t P = B * L * L;
    const size_t LSZ = (size_t)P * C;
    hipStream_t st = a->stream;
    if (L <= kFwdMaxL) {
        // the whole forward per configuration in LDS, bit for bit the layered path's
        const int lds = fwd_lds_bytes(L);
        AR_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&train_fwd_kernel),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lds),
               "training forward LDS size");
        hipLaunchKernelGGL(train_fwd_kernel, dim3((unsigned)B), dim3(256), lds, st, B, L, spins, a->wf, bs.tab, bs.pt,
                           bs.npts, a->hs, a->mask, a->logit);
    } else {
    hipLaunchKernelGGL(embed_kernel, dim3((unsigned)((P * (C / 8) + 255) / 256)), dim3(256), 0, st, spins, P, a->hs);
    for (int l = 0; l < NL; ++l) {
        const Taps tp = taps_for(l, false);
        const __bf16* W = a->wf + (size_t)l * NT * C * C;
        const int mode = (l == NL - 1) ? EP_LOGIT : (l == 0 ? EP_RELU : EP_RESID);
        __bf16* out = (l < NL - 1) ? a->hs + (size_t)(l + 1) * LSZ : nullptr;
        uint32_t* mk = (l < NL - 1) ? a->mask + (size_t)l * P : nullptr;
        hipLaunchKernelGGL(conv32_kernel, dim3(conv_blocks(P, a->conv_wg)), dim3(256), 0, st, a->hs + (size_t)l * LSZ, W,
                           bs.tab + l * C, bs.pt, bs.npts, tp, L, P, mode, a->hs + (size_t)l * LSZ,
                           (const float*)nullptr, out, mk, a->logit, (const uint32_t*)nullptr, (__bf16*)nullptr,
                           (float*)nullptr);
    }
    }
    hipLaunchKernelGGL(loss_kernel, dim3((unsigned)B), dim3(256), 0, st, a->logit, spins, L, 1.0f / (float)B, a->logq,
                       a->g, a->g32);
    const int nch = (int)wgrad_chunks(P);
    if (L <= kBwdMaxL) {
        // the whole data-gradient chain per configuration, then the weight
        // gradients of all layers from the stored dz (bit for bit the layered
        // path's; the bias sums come per configuration instead of per
        // wavefront of the layered launch, so their fp32 grouping differs)
        const int lds = bwd_lds_bytes(L);
        const bool small = (L * L + 31) / 32 <= 12;
        const void* fn = small ? reinterpret_cast<const void*>(&train_bwd_kernel<3>)
                               : reinterpret_cast<const void*>(&train_bwd_kernel<5>);
        AR_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds), "training backward LDS size");
        float* gs = a->cond > 0 ? a->gs : nullptr;
        if (small)
            hipLaunchKernelGGL(train_bwd_kernel<3>, dim3((unsigned)B), dim3(256), lds, st, B, L, a->g, a->g32, a->wb,
                               a->mask, a->dzs, a->bpl, gs);
        else
            hipLaunchKernelGGL(train_bwd_kernel<5>, dim3((unsigned)B), dim3(256), lds, st, B, L, a->g, a->g32, a->wb,
                               a->mask, a->dzs, a->bpl, gs);
        // the weight gradients of all layers in one launch each of the
        // partial sums, their slice fold and the finish
        WgradJobs jobs{};
        const int64_t pst = (int64_t)nch * NT * C * C, p2st = (int64_t)kRedSlices * NT * C * C;
        for (int l = 0; l < NL; ++l) {
            jobs.in[l] = a->hs + (size_t)l * LSZ;
            jobs.dz[l] = (l == NL - 1) ? a->g : a->dzs + (size_t)l * LSZ;
            jobs.part[l] = a->part + l * pst;
            jobs.layer[l] = l;
        }
        hipLaunchKernelGGL(wgrad_fused_kernel, dim3((unsigned)nch, NL), dim3(64 * kWWaves), 0, st, jobs, L, P);
        hipLaunchKernelGGL(reduce_slices_kernel, dim3((NT * C * C + 255) / 256, kRedSlices, NL), dim3(256), 0, st,
                           a->part, nch, NT * C * C, a->part2, pst, p2st);
        hipLaunchKernelGGL(finish_layer_grad_kernel, dim3((NT * C * C + 255) / 256 + C, NL), dim3(256), 0, st, a->part2,
                           p2st, a->bpl, (int64_t)B * C, (int)B, 0, a->grad);
    } else {
    float* dh = a->dh0;
    float* dh_alt = a->dh1;
    // The data-gradient convolution of layer l also applies the ReLU mask of
    // layer l - 1 and sums the result per channel, so layer l - 1 starts with
    // its gated gradient (bf16, alternating between dz and the logit-gradient
    // buffer, which is free after the top layer) and its bias partial sums.
    __bf16* dz_next = nullptr;
    int nbp_next = 0;
    for (int l = NL - 1; l >= 0; --l) {
        const Taps tm = taps_for(l, true);
        const __bf16* dzl;
        int nbp;
        if (l == NL - 1) {
            dzl = a->g;
            nbp = 256;
            hipLaunchKernelGGL(colsum0_kernel, dim3(nbp), dim3(256), 0, st, a->g32, P, a->bpart);
        } else {
            dzl = dz_next;
            nbp = nbp_next;
        }
        if (a->cond > 0)  // each sample's share, for the conditioning MLP
            hipLaunchKernelGGL(sample_bias_grad_kernel, dim3((unsigned)B), dim3(256), 0, st, dh,
                               a->mask + (size_t)(l < NL - 1 ? l : 0) * P, l == NL - 1 ? a->g32 : nullptr, L * L,
                               l, a->gs);
        WgradJobs job1{};
        job1.in[0] = a->hs + (size_t)l * LSZ;
        job1.dz[0] = dzl;
        job1.part[0] = a->part;
        job1.layer[0] = l;
        hipLaunchKernelGGL(wgrad_fused_kernel, dim3((unsigned)nch, 1), dim3(64 * kWWaves), 0, st, job1, L, P);
        hipLaunchKernelGGL(reduce_slices_kernel, dim3((NT * C * C + 255) / 256, kRedSlices, 1), dim3(256), 0, st,
                           a->part, nch, NT * C * C, a->part2, (int64_t)0, (int64_t)0);
        const int T = (l == 0) ? 4 : 5, ci = (l == 0) ? 1 : C, co = (l == NL - 1) ? 1 : C;
        const int wblocks = (T * ci * co + 255) / 256;
        hipLaunchKernelGGL(finish_layer_grad_kernel, dim3(wblocks + co, 1), dim3(256), 0, st, a->part2, (int64_t)0,
                           a->bpart, (int64_t)0, nbp, l, a->grad);
        if (l > 0) {
            const __bf16* Wb = a->wb + (size_t)l * NT * C * C;
            const int mode = (l == NL - 1) ? EP_DGRAD : EP_DGRAD_RESID;
            const int nb = conv_blocks(P, a->conv_wg);
            dz_next = (dzl == a->dz) ? a->g : a->dz;
            nbp_next = 4 * nb;
            hipLaunchKernelGGL(conv32_kernel, dim3(nb), dim3(256), 0, st, dzl, Wb, a->bias, (const int32_t*)nullptr, 1,
                               tm, L, P, mode, (const __bf16*)nullptr, (const float*)dh, (__bf16*)nullptr,
                               (uint32_t*)nullptr, dh_alt, (const uint32_t*)(a->mask + (size_t)(l - 1) * P), dz_next,
                               a->bpart);
            std::swap(dh, dh_alt);
        }
    }
    }
    if (a->cond > 0) {
        hipLaunchKernelGGL(point_grad_kernel, dim3((unsigned)((a->npts * kCondOut + 255) / 256)), dim3(256), 0, st,
                           a->gs, pt, B, a->npts, a->gp);
        hipLaunchKernelGGL(cond_backward_kernel, dim3(1), dim3(kCondOut), 0, st, a->theta + a->np_base, a->feats,
                           a->npts, a->gp, a->grad + a->np_base);
    }
    AR_TRY(hipGetLastError(), "training kernels");
    return CRBM_OK;
}

// ancestral sampling of n configurations (spins and their log q)
// n proposals in batches of n_step (n a multiple of n_step): batch k is keyed
// as step + k and is conditioned on pt[0 .. n_step)
int run_seq(crbm_ar_t* a, int64_t n, int8_t* spins, double* logq, uint64_t seed, uint32_t step, uint32_t id,
            const int32_t* pt, int64_t n_step, hipStream_t st) {
    const BiasSel bs = bias_sel(a, pt);
    int rc = ensure_seq(a, n);
    if (rc != CRBM_OK) return rc;
    const int L = a->L;
    // st: the stream of every step (the sampler buffers are used in stream order)
    // the first layer's ring rows: channels 1..31 stay zero, channel 0 receives the spins
    const int64_t npad = (n + kSeqPad - 1) / kSeqPad * kSeqPad;
    AR_TRY(hipMemsetAsync(a->ring, 0, sizeof(__bf16) * (size_t)npad * L * C, st), "clear sampler input");
    // one wavefront per 16 chains; as many per workgroup as keep one workgroup per compute unit busy
    const int waves = n <= 16 * 256 ? 1 : n <= 32 * 256 ? 2 : kSeqMaxWaves;
    const int per_wg = 16 * waves;
    const dim3 grid((unsigned)((n + per_wg - 1) / per_wg)), block(64 * waves);
    auto launch = [&](auto kernel) -> int {
        AR_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                   kSeqLdsBytes),
               "sampler LDS size");
        hipLaunchKernelGGL(kernel, grid, block, kSeqLdsBytes, st, n, npad, L, a->wf, bs.tab, bs.pt, bs.npts, a->ring,
                           a->zpad, spins, a->slogit, seed, step, id, n_step);
        return CRBM_OK;
    };
    rc = bs.pt ? launch(seq_kernel<true>) : launch(seq_kernel<false>);
    if (rc != CRBM_OK) return rc;
    hipLaunchKernelGGL(logq_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, a->slogit, spins, n, L * L,
                       logq);
    AR_TRY(hipGetLastError(), "sampler kernels");
    return CRBM_OK;
}

int ensure_infer(crbm_ar_t* a, int64_t n) {
    if (n <= a->icap) return CRBM_OK;
    if (n > (kMaxPixels - 1) / ((int64_t)a->L * a->L)) return fail_ar(CRBM_EINVAL, "batch too large (samples x L^2 must be below 2^31)");
    void* ps[] = {a->ih0, a->ih1, a->ilogit};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    a->ih0 = a->ih1 = nullptr;
    a->ilogit = nullptr;
    const int64_t P = n * a->L * a->L;
    const bool layered = a->L > kFuseMaxL;  // the fused scorer needs only the logits
    if ((layered && (alloc(&a->ih0, P * C) || alloc(&a->ih1, P * C))) || alloc(&a->ilogit, P)) {
        a->icap = 0;
        return fail_ar(CRBM_ENOMEM, "scoring buffers");
    }
    a->icap = n;
    return CRBM_OK;
}

// log q of n given configurations by one full forward pass over all sites
int run_score(crbm_ar_t* a, int64_t n, const int8_t* spins, double* logq, const int32_t* pt) {
    const BiasSel bs = bias_sel(a, pt);
    int rc = ensure_infer(a, n);
    if (rc != CRBM_OK) return rc;
    const int L = a->L;
    const int64_t P = n * L * L;
    hipStream_t st = a->stream;
    if (L <= kFuseMaxL) {
        const int lds = 2 * fused_pixels(L) * C * (int)sizeof(__bf16);
        AR_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&score_fused_kernel),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lds),
               "scorer LDS size");
        hipLaunchKernelGGL(score_fused_kernel, dim3((unsigned)n), dim3(256), lds, st, n, L, spins, a->wf, bs.tab,
                           bs.pt, bs.npts, a->ilogit);
        hipLaunchKernelGGL(logq_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, a->ilogit, spins, n,
                           L * L, logq);
        AR_TRY(hipGetLastError(), "scoring kernels");
        return CRBM_OK;
    }
    hipLaunchKernelGGL(embed_kernel, dim3((unsigned)((P * (C / 8) + 255) / 256)), dim3(256), 0, st, spins, P, a->ih0);
    __bf16* in = a->ih0;
    __bf16* out = a->ih1;
    const int64_t tiles = (P + 15) / 16;
    const int blocks = (int)std::min<int64_t>(4096, (tiles + 3) / 4);
    for (int l = 0; l < NL; ++l) {
        hipLaunchKernelGGL(conv16_kernel, dim3(blocks), dim3(256), 0, st, in, a->wf + (size_t)l * NT * C * C,
                           bs.tab + l * C, bs.pt, bs.npts, l, L, P, out, a->ilogit);
        std::swap(in, out);
    }
    hipLaunchKernelGGL(logq_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, a->ilogit, spins, n, L * L,
                       logq);
    AR_TRY(hipGetLastError(), "scoring kernels");
    return CRBM_OK;
}

}  // namespace

extern "C" {

int64_t crbm_ar_num_params(const crbm_ar_t* a) { return a ? a->np : 0; }

int crbm_ar_create(const crbm_ar_config* c, crbm_ar_t** out) {
    if (!c || !out) return fail_ar(CRBM_EINVAL, "NULL argument");
    *out = nullptr;
    if (c->L < 4 || c->L > CRBM_MAX_L || (c->L & 1)) return fail_ar(CRBM_EINVAL, "bad L");
    if (c->channels != C || c->layers != NL) return fail_ar(CRBM_EUNSUPPORTED, "kernels are built for 32 channels, 12 layers");
    if (c->cond_points < 0 || c->cond_points > kCondMaxPoints) return fail_ar(CRBM_EINVAL, "cond_points must be 0..128");
    crbm_ar_s* a = new (std::nothrow) crbm_ar_s();
    if (!a) return fail_ar(CRBM_ENOMEM, "host allocation");
    a->L = c->L;
    a->seed = c->seed;
    {
        int dev = 0, n = 0, per_cu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0 &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, conv32_kernel, 256, 0) == hipSuccess && per_cu > 0)
            a->conv_wg = n * per_cu;
    }
    a->stream = (hipStream_t)c->stream;
    a->cond = c->cond_points;
    a->np_base = n_params();
    a->np = a->np_base + (a->cond > 0 ? (int64_t)kCondF * kCondH + kCondH + (int64_t)kCondH * kCondOut : 0);
    if (alloc(&a->theta, a->np) || alloc(&a->grad, a->np) || alloc(&a->m, a->np) || alloc(&a->v, a->np) ||
        alloc(&a->bias, NL * C) || alloc(&a->wf, (int64_t)NL * NT * C * C) || alloc(&a->wb, (int64_t)NL * NT * C * C) ||
        alloc(&a->zpad, (int64_t)16 * c->L * C) ||
        (a->cond > 0 && (alloc(&a->feats, (int64_t)a->cond * kCondF) || alloc(&a->cb, (int64_t)a->cond * kCondOut) ||
                         alloc(&a->gp, (int64_t)a->cond * kCondOut)))) {
        delete a;
        return fail_ar(CRBM_ENOMEM, "parameter buffers");
    }
    int rc = CRBM_OK;
    if (hipMemsetAsync(a->zpad, 0, sizeof(__bf16) * 16 * c->L * C, a->stream) != hipSuccess ||
        hipMemsetAsync(a->theta, 0, sizeof(float) * a->np, a->stream) != hipSuccess ||
        hipMemsetAsync(a->m, 0, sizeof(float) * a->np, a->stream) != hipSuccess ||
        hipMemsetAsync(a->v, 0, sizeof(float) * a->np, a->stream) != hipSuccess ||
        hipMemsetAsync(a->grad, 0, sizeof(float) * a->np, a->stream) != hipSuccess)
        rc = fail_ar(CRBM_EHIP, "zeroing the parameter buffers");
    if (rc == CRBM_OK) rc = pack(a);
    if (rc == CRBM_OK && hipStreamSynchronize(a->stream) != hipSuccess) rc = fail_ar(CRBM_EHIP, "synchronize");
    if (rc != CRBM_OK) {
        delete a;
        return rc;
    }
    *out = a;
    return CRBM_OK;
}

int crbm_ar_set_points(crbm_ar_t* a, int32_t n_points, const double* feats_host) {
    if (!a || !feats_host) return fail_ar(CRBM_EINVAL, "NULL argument");
    if (a->cond == 0) return fail_ar(CRBM_EINVAL, "the network is not conditional");
    if (n_points < 1 || n_points > a->cond) return fail_ar(CRBM_EINVAL, "n_points must be 1..cond_points");
    std::vector<float> f((size_t)n_points * kCondF);
    for (size_t i = 0; i < f.size(); ++i) {
        if (!std::isfinite(feats_host[i])) return fail_ar(CRBM_EINVAL, "features must be finite");
        f[i] = (float)feats_host[i];
    }
    AR_TRY(hipMemcpyAsync(a->feats, f.data(), sizeof(float) * f.size(), hipMemcpyHostToDevice, a->stream), "copy features");
    a->npts = n_points;
    int rc = pack(a);
    if (rc != CRBM_OK) return rc;
    AR_TRY(hipStreamSynchronize(a->stream), "synchronize");
    return CRBM_OK;
}

int crbm_ar_set_params(crbm_ar_t* a, const float* host, int64_t n) {
    if (!a || !host || n != a->np) return fail_ar(CRBM_EINVAL, "parameter count mismatch");
    AR_TRY(hipMemcpyAsync(a->theta, host, sizeof(float) * n, hipMemcpyHostToDevice, a->stream), "copy params");
    AR_TRY(hipMemsetAsync(a->m, 0, sizeof(float) * a->np, a->stream), "clear Adam moments");
    AR_TRY(hipMemsetAsync(a->v, 0, sizeof(float) * a->np, a->stream), "clear Adam moments");
    a->t_adam = 0;
    int rc = pack(a);
    if (rc != CRBM_OK) return rc;
    AR_TRY(hipStreamSynchronize(a->stream), "synchronize");
    return CRBM_OK;
}

int crbm_ar_init_params(crbm_ar_t* a, uint64_t seed, double scale) {
    if (!a || !(scale >= 0.0)) return fail_ar(CRBM_EINVAL, "bad arguments");
    // N(0, std^2) by SplitMix64 + Box-Muller; std = scale sqrt(2 / fan-in),
    // times 0.1 for the logit layer; biases zero.  Conditioning MLP: W1 with
    // std sqrt(1 / features), b1 and W2 zero (a fresh conditional network is
    // its unconditional part)
    std::vector<float> th((size_t)a->np, 0.f);
    uint64_t x = seed;
    auto next = [&]() {
        x += 0x9E3779B97F4A7C15ull;
        uint64_t z = x;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    auto normal = [&]() {
        const double u1 = ((next() >> 11) + 1.0) * (1.0 / 9007199254740992.0);
        const double u2 = (next() >> 11) * (1.0 / 9007199254740992.0);
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
    };
    size_t off = 0;
    for (int l = 0; l < NL; ++l) {
        const int T = (l == 0) ? 4 : 5, ci = (l == 0) ? 1 : C, co = (l == NL - 1) ? 1 : C;
        const double sd = scale * std::sqrt(2.0 / (T * ci)) * (l == NL - 1 ? 0.1 : 1.0);
        for (int k = 0; k < T * ci * co; ++k) th[off + k] = (float)(sd * normal());
        off += (size_t)T * ci * co + co;
    }
    if (a->cond > 0)
        for (int k = 0; k < kCondF * kCondH; ++k) th[off + k] = (float)(std::sqrt(1.0 / kCondF) * normal());
    return crbm_ar_set_params(a, th.data(), a->np);
}

int crbm_ar_get_params(crbm_ar_t* a, float* host, int64_t n) {
    if (!a || !host || n != a->np) return fail_ar(CRBM_EINVAL, "parameter count mismatch");
    AR_TRY(hipMemcpyAsync(host, a->theta, sizeof(float) * n, hipMemcpyDeviceToHost, a->stream), "copy params");
    AR_TRY(hipStreamSynchronize(a->stream), "synchronize");
    return CRBM_OK;
}

static int need_points(const crbm_ar_t* a) {
    if (a->cond > 0 && a->npts == 0) return fail_ar(CRBM_ESTATE, "conditional network: call crbm_ar_set_points first");
    return CRBM_OK;
}

static int mean_loss(crbm_ar_t* a, int64_t batch, double* loss_out) {
    std::vector<double> lq(batch);
    AR_TRY(hipMemcpyAsync(lq.data(), a->logq, sizeof(double) * batch, hipMemcpyDeviceToHost, a->stream), "copy logq");
    AR_TRY(hipStreamSynchronize(a->stream), "synchronize");
    double s = 0.0;
    for (double x : lq) s += x;
    *loss_out = -s / (double)batch;
    return CRBM_OK;
}

int crbm_ar_grad_cond(crbm_ar_t* a, const int8_t* samples_dev, const int32_t* points_dev, int64_t batch,
                      float* grad_host, double* loss_out) {
    if (!a || !samples_dev || batch < 1) return fail_ar(CRBM_EINVAL, "bad arguments");
    int rc = need_points(a);
    if (rc != CRBM_OK) return rc;
    rc = ensure_train(a, batch);
    if (rc != CRBM_OK) return rc;
    rc = grad_pass(a, samples_dev, batch, points_dev);
    if (rc != CRBM_OK) return rc;
    if (grad_host)
        AR_TRY(hipMemcpyAsync(grad_host, a->grad, sizeof(float) * a->np, hipMemcpyDeviceToHost, a->stream), "copy grad");
    if (loss_out) {
        rc = mean_loss(a, batch, loss_out);
        if (rc != CRBM_OK) return rc;
    }
    AR_TRY(hipStreamSynchronize(a->stream), "synchronize");
    return CRBM_OK;
}

int crbm_ar_grad(crbm_ar_t* a, const int8_t* samples_dev, int64_t batch, float* grad_host, double* loss_out) {
    return crbm_ar_grad_cond(a, samples_dev, nullptr, batch, grad_host, loss_out);
}

int crbm_ar_train_step_cond(crbm_ar_t* a, const int8_t* samples_dev, const int32_t* points_dev, int64_t batch,
                            float lr, double* loss_out) {
    if (!a || !samples_dev || batch < 1 || !(lr > 0.f)) return fail_ar(CRBM_EINVAL, "bad arguments");
    int rc = need_points(a);
    if (rc != CRBM_OK) return rc;
    rc = ensure_train(a, batch);
    if (rc != CRBM_OK) return rc;
    rc = grad_pass(a, samples_dev, batch, points_dev);
    if (rc != CRBM_OK) return rc;
    a->t_adam += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)a->t_adam), c2 = 1.f - powf(b2, (float)a->t_adam);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((a->np + 255) / 256)), dim3(256), 0, a->stream, a->theta, a->grad,
                       a->m, a->v, a->np, lr, b1, b2, 1e-8f, c1, c2);
    rc = pack(a);
    if (rc != CRBM_OK) return rc;
    if (loss_out) return mean_loss(a, batch, loss_out);
    return CRBM_OK;
}

int crbm_ar_train_step(crbm_ar_t* a, const int8_t* samples_dev, int64_t batch, float lr, double* loss_out) {
    return crbm_ar_train_step_cond(a, samples_dev, nullptr, batch, lr, loss_out);
}

int crbm_ar_batch(const int8_t* samples_dev, const int32_t* points_dev, int64_t n, int32_t L, int64_t batch,
                  uint64_t seed, int64_t step, int32_t augment, int8_t* out_dev, int32_t* points_out_dev,
                  int64_t* index_out_dev, void* stream) {
    if (!samples_dev || !out_dev || n < 1 || batch < 1 || L < 4 || L > CRBM_MAX_L || (L & 1) || step < 0 ||
        step > 0xffffffffLL || batch > 0x7fffffffLL)
        return fail_ar(CRBM_EINVAL, "crbm_ar_batch: bad arguments");
    hipLaunchKernelGGL(gather_batch_kernel, dim3((unsigned)batch), dim3(256), 0, (hipStream_t)stream, samples_dev,
                       points_dev, n, L, seed, (uint32_t)step, augment ? 1 : 0, out_dev, points_out_dev,
                       index_out_dev);
    AR_TRY(hipGetLastError(), "crbm_ar_batch");
    return CRBM_OK;
}

int crbm_ar_train(crbm_ar_t* a, const int8_t* samples_dev, const int32_t* points_dev, int64_t n,
                  const crbm_train_opts* o, double* loss_out) {
    if (!a || !samples_dev || !o || n < 1 || o->steps < 0 || o->batch < 1 || !(o->lr > 0.f) ||
        !(o->lr_late > 0.f) || !(o->late_from >= 0.0) || o->step0 < 0 || o->step0 + o->steps > 0xffffffffLL)
        return fail_ar(CRBM_EINVAL, "crbm_ar_train: bad arguments");
    int rc = need_points(a);
    if (rc != CRBM_OK) return rc;
    if (o->batch > a->bcap) {
        if (a->bspins) (void)hipFree(a->bspins);
        if (a->bpts) (void)hipFree(a->bpts);
        a->bspins = nullptr;
        a->bpts = nullptr;
        a->bcap = 0;
        if (alloc(&a->bspins, o->batch * a->L * a->L) || alloc(&a->bpts, o->batch))
            return fail_ar(CRBM_ENOMEM, "crbm_ar_train: batch buffers");
        a->bcap = o->batch;
    }
    const bool cond = a->cond > 0 && points_dev != nullptr;
    for (int64_t k = 0; k < o->steps; ++k) {
        rc = crbm_ar_batch(samples_dev, cond ? points_dev : nullptr, n, a->L, o->batch, o->seed, o->step0 + k,
                           o->augment, a->bspins, cond ? a->bpts : nullptr, nullptr, a->stream);
        if (rc != CRBM_OK) return rc;
        const float lr = (double)k < o->late_from * (double)o->steps ? o->lr : o->lr_late;
        rc = crbm_ar_train_step_cond(a, a->bspins, cond ? a->bpts : nullptr, o->batch, lr,
                                     (loss_out && k + 1 == o->steps) ? loss_out : nullptr);
        if (rc != CRBM_OK) return rc;
    }
    if (loss_out && o->steps == 0) *loss_out = 0.0;
    return CRBM_OK;
}

int crbm_ar_logq_cond(crbm_ar_t* a, const int8_t* spins_dev, const int32_t* points_dev, int64_t n, double* logq_dev) {
    if (!a || !spins_dev || !logq_dev || n < 1) return fail_ar(CRBM_EINVAL, "bad arguments");
    const int rc = need_points(a);
    if (rc != CRBM_OK) return rc;
    return run_score(a, n, spins_dev, logq_dev, points_dev);
}

int crbm_ar_logq(crbm_ar_t* a, const int8_t* spins_dev, int64_t n, double* logq_dev) {
    return crbm_ar_logq_cond(a, spins_dev, nullptr, n, logq_dev);
}

int crbm_ar_sample_cond(crbm_ar_t* a, int64_t n, uint64_t seed, int64_t step, uint32_t id, const int32_t* points_dev,
                        int8_t* spins_dev, double* logq_dev) {
    if (!a || !spins_dev || !logq_dev || n < 1) return fail_ar(CRBM_EINVAL, "bad arguments");
    const int rc = need_points(a);
    if (rc != CRBM_OK) return rc;
    return run_seq(a, n, spins_dev, logq_dev, seed, (uint32_t)step, id, points_dev, n, a->stream);
}

int crbm_ar_sample(crbm_ar_t* a, int64_t n, uint64_t seed, int64_t step, uint32_t id, int8_t* spins_dev,
                   double* logq_dev) {
    return crbm_ar_sample_cond(a, n, seed, step, id, nullptr, spins_dev, logq_dev);
}

int crbm_ar_sample_steps(crbm_ar_t* a, int64_t n, int32_t n_steps, uint64_t seed, int64_t step0, uint32_t id,
                         const int32_t* points_dev, int8_t* spins_dev, double* logq_dev) {
    if (!a || !spins_dev || !logq_dev || n < 1 || n_steps < 1 || n > ((int64_t)1 << 31) / n_steps)
        return fail_ar(CRBM_EINVAL, "bad arguments");
    const int rc = need_points(a);
    if (rc != CRBM_OK) return rc;
    return run_seq(a, n * n_steps, spins_dev, logq_dev, seed, (uint32_t)step0, id, points_dev, n, a->stream);
}

void crbm_ar_destroy(crbm_ar_t* a) {
    if (!a) return;
    (void)hipStreamSynchronize(a->stream);
    if (a->side) (void)hipStreamSynchronize(a->side);
    delete a;
}

int crbm_sample_mh(crbm_t* h, crbm_ar_t* a, int64_t n_cycles, int32_t gibbs_per_mh, int32_t* counts_trace,
                   int32_t* order_trace, int64_t* n_accepted) {
    if (!h || !a || n_cycles < 0 || gibbs_per_mh < 0) return fail_ar(CRBM_EINVAL, "bad arguments");
    HandleView v{};
    if (handle_view(h, &v, 0) != CRBM_OK) return fail_ar(CRBM_EINVAL, "bad handle");
    if (v.L != a->L) return fail_ar(CRBM_EINVAL, "lattice size of the network and the handle differ");
    if (v.stream != a->stream) return fail_ar(CRBM_EINVAL, "handle and network must use the same stream");
    if (v.precision != CRBM_PRECISION_Q16)
        return fail_ar(CRBM_EUNSUPPORTED, "MH needs the default precision (the acceptance uses the exact CRBM marginal)");
    const int n_inst = v.n_inst;
    if (a->cond > 0 && n_inst > a->npts)
        return fail_ar(CRBM_EINVAL, "conditional network: instance i uses point i, set at least one point per instance");
    // every instance: same L, constant temperature, its chains right after the previous instance's
    const int64_t N = (int64_t)v.L * v.L, words = (int64_t)v.L * ((v.L + 31) / 32);
    std::vector<MhTarget> tg((size_t)n_inst);
    int64_t n = 0;
    for (int i = 0; i < n_inst; ++i) {
        HandleView vi{};
        if (handle_view(h, &vi, i) != CRBM_OK) return fail_ar(CRBM_EINVAL, "bad handle");
        if (vi.L != v.L || vi.sched_kind != CRBM_SCHED_CONST)
            return fail_ar(CRBM_EUNSUPPORTED, "MH needs instances of one lattice size, each at a constant temperature");
        if (vi.state != v.state + n * words) return fail_ar(CRBM_EUNSUPPORTED, "instances are not contiguous");
        tg[(size_t)i] = MhTarget{vi.a, vi.c1, vi.c2, vi.sg1, vi.sg2};
        n += vi.n_chains;
    }
    hipStream_t st = a->stream;
    if (n > a->mcap) {
        void* ps[] = {a->cur, a->ccur, a->cprop, a->lqc, a->nacc, a->mh_ci};
        for (void* p : ps)
            if (p) (void)hipFree(p);
        a->cur = nullptr;
        a->ccur = a->cprop = nullptr;
        a->lqc = nullptr;
        a->nacc = nullptr;
        a->mh_ci = nullptr;
        a->mcap = 0;
        if (alloc(&a->cur, n * N) || alloc(&a->ccur, n * 3) || alloc(&a->cprop, n * 3) || alloc(&a->lqc, n) ||
            alloc(&a->nacc, 1) || alloc(&a->mh_ci, n)) {
            a->mcap = 0;
            return fail_ar(CRBM_ENOMEM, "MH buffers");
        }
        a->mcap = n;
    }
    if (n_inst > a->mh_tgcap) {
        if (a->mh_tg) (void)hipFree(a->mh_tg);
        a->mh_tg = nullptr;
        if (alloc(&a->mh_tg, n_inst)) {
            a->mh_tgcap = 0;
            return fail_ar(CRBM_ENOMEM, "MH targets");
        }
        a->mh_tgcap = n_inst;
    }
    {
        std::vector<int32_t> ci((size_t)n);
        int64_t c0 = 0;
        for (int i = 0; i < n_inst; ++i) {
            HandleView vi{};
            (void)handle_view(h, &vi, i);
            for (int64_t k = 0; k < vi.n_chains; ++k) ci[(size_t)(c0 + k)] = i;
            c0 += vi.n_chains;
        }
        AR_TRY(hipMemcpyAsync(a->mh_ci, ci.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st), "copy chain map");
        AR_TRY(hipMemcpyAsync(a->mh_tg, tg.data(), sizeof(MhTarget) * n_inst, hipMemcpyHostToDevice, st),
               "copy targets");
        AR_TRY(hipStreamSynchronize(st), "synchronize");  // the host vectors go out of scope
    }
    const int32_t* pts = a->cond > 0 ? a->mh_ci : nullptr;  // chain i of instance k is conditioned on point k
    AR_TRY(hipMemsetAsync(a->nacc, 0, sizeof(unsigned long long), st), "zero counter");
    // Proposals do not depend on the chains, so the sampler draws those of
    // up to kb cycles in one launch: enough wavefronts (16 chains each) for
    // one per SIMD, where one cycle's alone would leave SIMDs idle.  Each
    // cycle's proposals keep their own step in the random stream, so the
    // results do not depend on kb.  The sampler runs ahead on a stream of its
    // own into two buffer sets: batch b goes to set b % 2 once MH has
    // consumed batch b - 2, so the sweeps, counts and MH steps of one batch
    // overlap the drawing of the next (the scorer cannot: its LDS and the
    // sampler's do not fit one compute unit together).
    const int64_t kb = std::max<int64_t>(1, std::min<int64_t>(kMhBatchChains / n, kMhMaxBatch));
    if (kb > a->mh_kcap || n > a->mh_kn) {
        void* pb[] = {a->mh_prop, a->mh_lqp, a->mh_prop2, a->mh_lqp2};
        for (void* p : pb)
            if (p) (void)hipFree(p);
        a->mh_prop = a->mh_prop2 = nullptr;
        a->mh_lqp = a->mh_lqp2 = nullptr;
        if (alloc(&a->mh_prop, kb * n * N) || alloc(&a->mh_lqp, kb * n) || alloc(&a->mh_prop2, kb * n * N) ||
            alloc(&a->mh_lqp2, kb * n)) {
            a->mh_kcap = a->mh_kn = 0;
            return fail_ar(CRBM_ENOMEM, "MH proposal buffers");
        }
        a->mh_kcap = kb;
        a->mh_kn = n;
    }
    if (!a->side) {
        AR_TRY(hipStreamCreateWithFlags(&a->side, hipStreamNonBlocking), "MH sampler stream");
        hipEvent_t* evs[] = {&a->ev_in, &a->ev_ready[0], &a->ev_ready[1], &a->ev_free[0], &a->ev_free[1]};
        for (hipEvent_t* e : evs) AR_TRY(hipEventCreateWithFlags(e, hipEventDisableTiming), "MH events");
    }
    {
        const int rc0 = ensure_seq(a, kb * n);  // before any launch: no reallocation while the sampler runs
        if (rc0 != CRBM_OK) return rc0;
    }
    int8_t* const bprop[2] = {a->mh_prop, a->mh_prop2};
    double* const blqp[2] = {a->mh_lqp, a->mh_lqp2};
    const uint64_t step0 = a->mh_step;
    const int64_t nb = (n_cycles + kb - 1) / kb;
    // the sampler reads the weights, biases and point map written on the main stream
    AR_TRY(hipEventRecord(a->ev_in, st), "MH start event");
    AR_TRY(hipStreamWaitEvent(a->side, a->ev_in, 0), "MH sampler wait");
    auto draw = [&](int64_t b) -> int {
        const int j = (int)(b & 1);
        if (b >= 2) AR_TRY(hipStreamWaitEvent(a->side, a->ev_free[j], 0), "MH buffer wait");
        const int64_t len = std::min<int64_t>(kb, n_cycles - b * kb);
        const int rcs = run_seq(a, len * n, bprop[j], blqp[j], v.seed, (uint32_t)(step0 + (uint64_t)(b * kb)), v.id,
                                pts, n, a->side);
        if (rcs != CRBM_OK) return rcs;
        AR_TRY(hipEventRecord(a->ev_ready[j], a->side), "MH batch event");
        return CRBM_OK;
    };
    for (int64_t b = 0; b < std::min<int64_t>(nb, 2); ++b) {
        const int rcd = draw(b);
        if (rcd != CRBM_OK) return rcd;
    }
    for (int64_t cyc = 0; cyc < n_cycles; ++cyc) {
        if (gibbs_per_mh > 0) {
            const int rc = crbm_sample(h, gibbs_per_mh, nullptr, nullptr);
            if (rc != CRBM_OK) return rc;
        }
        int rc = CRBM_OK;
        // the current state changes only by MH itself when no Gibbs sweeps
        // are interleaved; then its counts and log q carry over
        if (cyc == 0 || gibbs_per_mh > 0) {
            AR_TRY(launch_unpack(v.state, a->cur, n, v.L, st), "unpack state");
            hipLaunchKernelGGL(counts_int8_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, a->cur, n, v.L, a->ccur,
                               (int32_t*)nullptr);
            rc = run_score(a, n, a->cur, a->lqc, pts);
            if (rc != CRBM_OK) return rc;
        }
        const int64_t b = cyc / kb, in_b = cyc - b * kb;
        const int j = (int)(b & 1);
        if (in_b == 0) AR_TRY(hipStreamWaitEvent(st, a->ev_ready[j], 0), "MH proposal wait");
        const uint32_t step = (uint32_t)(a->mh_step++);
        int8_t* prop = bprop[j] + in_b * n * N;
        double* lqp = blqp[j] + in_b * n;
        hipLaunchKernelGGL(counts_int8_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, prop, n, v.L, a->cprop,
                           (int32_t*)nullptr);
        hipLaunchKernelGGL(mh_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, n, v.L, a->cur, prop, a->ccur,
                           a->cprop, a->lqc, lqp, a->mh_tg, a->mh_ci, v.seed, step, v.id, a->nacc);
        AR_TRY(launch_pack(v.state, a->cur, n, v.L, st), "pack state");
        if (order_trace)  // recounts the current states (same counts) with the structure factor
            hipLaunchKernelGGL(counts_int8_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, a->cur, n, v.L,
                               a->ccur, order_trace + cyc * n * 3);
        if (counts_trace)
            AR_TRY(hipMemcpyAsync(counts_trace + cyc * n * 3, a->ccur, sizeof(int32_t) * n * 3, hipMemcpyDeviceToDevice, st),
                   "trace");
        AR_TRY(hipGetLastError(), "MH kernels");
        if (in_b == kb - 1 || cyc == n_cycles - 1) {  // batch b consumed: its set takes batch b + 2
            AR_TRY(hipEventRecord(a->ev_free[j], st), "MH buffer event");
            if (b + 2 < nb) {
                const int rcd = draw(b + 2);
                if (rcd != CRBM_OK) return rcd;
            }
        }
    }
    if (n_accepted) {
        unsigned long long acc = 0;
        AR_TRY(hipMemcpyAsync(&acc, a->nacc, sizeof(acc), hipMemcpyDeviceToHost, st), "copy counter");
        AR_TRY(hipStreamSynchronize(st), "synchronize");
        *n_accepted = (int64_t)acc;
    }
    return CRBM_OK;
}

}  // extern "C"
