// gibbs_aux.hip -- initial state, int8 <-> bit-row conversion, the summed
// spin-spin correlation C(dr, dc) behind the structure factor (Sec. III.B
// Eq. (13)), and the dispatch over the compiled Gibbs variants.
#include "gibbs_kernel.h"

namespace crbmlib {

bool tiles_a(int L, int R, const GibbsArgs* a, hipStream_t st, hipError_t* err, const void** fn);
bool tiles_b(int L, int R, const GibbsArgs* a, hipStream_t st, hipError_t* err, const void** fn);
bool tiles_c(int L, int R, const GibbsArgs* a, hipStream_t st, hipError_t* err, const void** fn);
bool tiles_d(int L, int R, const GibbsArgs* a, hipStream_t st, hipError_t* err, const void** fn);
bool tiles_e(int L, int R, const GibbsArgs* a, hipStream_t st, hipError_t* err, const void** fn);
bool tiles_f(int L, int R, const GibbsArgs* a, hipStream_t st, hipError_t* err, const void** fn);

namespace {

using gk::P4;
using gk::philox;

__host__ __device__ inline int words_per_row(int L) { return (L + 31) / 32; }

// Seeded initial state (stream 0): spin (r,c) is up iff bit (rL+c) & 127 of
// the Philox block with counter word (rL+c) >> 7 is set.
__global__ void init_kernel(uint32_t* state, const Item* items, int n_items, int L, uint64_t seed) {
    const int lane = threadIdx.x & 63;
    const int wv = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (wv >= n_items) return;
    const Item it = items[wv];
    if (lane >= (int)it.nchains) return;
    const int W = words_per_row(L);
    const uint32_t chain = it.chain0 + lane;
    uint32_t* rows = state + it.state_off + (uint64_t)lane * L * W;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    uint32_t cur = 0xffffffffu;
    P4 p{};
    for (int r = 0; r < L; ++r)
        for (int w = 0; w < W; ++w) {
            uint32_t word = 0u;
            const int m = (L - 32 * w) < 32 ? (L - 32 * w) : 32;
            for (int c = 0; c < m; ++c) {
                const uint32_t site = (uint32_t)(r * L + 32 * w + c);
                if ((site >> 7) != cur) {
                    cur = site >> 7;
                    p = philox(cur, 0u, chain, it.id << 3, k0, k1);
                }
                const uint32_t b = site & 127u;
                word |= ((p.v[b >> 5] >> (b & 31u)) & 1u) << c;
            }
            rows[r * W + w] = word;
        }
}

__global__ void pack_kernel(uint32_t* state, const int8_t* spins, int64_t nrows, int L) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrows) return;
    const int W = words_per_row(L);
    const int8_t* s = spins + t * L;
    for (int w = 0; w < W; ++w) {
        uint32_t word = 0u;
        const int m = (L - 32 * w) < 32 ? (L - 32 * w) : 32;
        for (int c = 0; c < m; ++c) word |= (s[32 * w + c] > 0 ? 1u : 0u) << c;
        state[t * W + w] = word;
    }
}

__global__ void unpack_kernel(const uint32_t* state, int8_t* spins, int64_t nrows, int L) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrows) return;
    const int W = words_per_row(L);
    int8_t* s = spins + t * L;
    for (int c = 0; c < L; ++c) s[c] = ((state[t * W + (c >> 5)] >> (c & 31)) & 1u) ? 1 : -1;
}

// C(dr, dc) = sum_{r,c} s(r,c) s(r+dr, c+dc), summed over the chains of one
// instance: one thread per (chain, dr); for each row pair the partner row is
// rotated one column at a time, so all L column offsets cost W popcounts each.
template <int L>
__global__ void __launch_bounds__(256) corr_kernel(const uint32_t* state, int64_t nchains,
                                                   unsigned long long* corr) {
    using G = gk::Geo<L>;
    constexpr int W = G::W;
    constexpr int N = L * L;
    __shared__ int part[N];
    for (int x = threadIdx.x; x < N; x += blockDim.x) part[x] = 0;
    __syncthreads();
    const int64_t chains_per_block = blockDim.x / L;
    const int64_t base = (int64_t)blockIdx.x * chains_per_block;
    const int64_t item = threadIdx.x;
    const int64_t ch = base + item / L;
    const int dr = (int)(item % L);
    if (item < chains_per_block * L && ch < nchains) {
        const uint32_t* rows = state + ch * L * W;
        int dis[L];
#pragma unroll
        for (int dc = 0; dc < L; ++dc) dis[dc] = 0;
        for (int r = 0; r < L; ++r) {
            uint32_t x[W], z[W];
#pragma unroll
            for (int w = 0; w < W; ++w) {
                x[w] = rows[r * W + w];
                z[w] = rows[((r + dr) % L) * W + w];
            }
#pragma unroll
            for (int dc = 0; dc < L; ++dc) {
#pragma unroll
                for (int w = 0; w < W; ++w) dis[dc] += __popc(x[w] ^ z[w]);
                uint32_t y[W];
#pragma unroll
                for (int w = 0; w < W; ++w) y[w] = gk::rsh<L, 1>(z, w);
#pragma unroll
                for (int w = 0; w < W; ++w) z[w] = y[w];
            }
        }
#pragma unroll
        for (int dc = 0; dc < L; ++dc) atomicAdd(&part[dr * L + dc], N - 2 * dis[dc]);
    }
    __syncthreads();
    for (int x = threadIdx.x; x < N; x += blockDim.x)
        atomicAdd(&corr[x], (unsigned long long)(long long)part[x]);
}

template <int L>
hipError_t launch_corr_t(const uint32_t* state, int64_t nchains, unsigned long long* corr, hipStream_t st) {
    const int threads = 256;
    const int64_t cpb = threads / L;
    const int64_t blocks = (nchains + cpb - 1) / cpb;
    hipLaunchKernelGGL((corr_kernel<L>), dim3((unsigned)blocks), dim3(threads), 0, st, state, nchains, corr);
    return hipGetLastError();
}

}  // namespace

static bool tiles(int L, int R, const GibbsArgs* a, hipStream_t st, hipError_t* e, const void** fn) {
    return tiles_a(L, R, a, st, e, fn) || tiles_b(L, R, a, st, e, fn) || tiles_c(L, R, a, st, e, fn) ||
           tiles_d(L, R, a, st, e, fn) || tiles_e(L, R, a, st, e, fn) || tiles_f(L, R, a, st, e, fn);
}

bool gibbs_supported(int L, int R) { return tiles(L, R, nullptr, nullptr, nullptr, nullptr); }

hipError_t launch_gibbs(int L, int R, const GibbsArgs& a, hipStream_t st) {
    hipError_t e = hipErrorInvalidValue;
    if (tiles(L, R, &a, st, &e, nullptr)) return e;
    return hipErrorInvalidValue;
}

const void* gibbs_kernel_fn(int L, int R) {
    const void* fn = nullptr;
    tiles(L, R, nullptr, nullptr, nullptr, &fn);
    return fn;
}

namespace {
__global__ void zero_u32_kernel(uint32_t* p, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0u;
}
}  // namespace

hipError_t launch_zero_u32(uint32_t* p, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_u32_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

const void* zero_u32_fn() { return reinterpret_cast<const void*>(&zero_u32_kernel); }

namespace {
// Workgroup i adds the accumulator rows (CRBM_N_ACC int64 per chain) of
// chains [ranges[2i], ranges[2i] + ranges[2i+1]) into sums[i]: integer
// sums, so the order of the additions does not change the result.
__global__ void __launch_bounds__(256) acc_sum_kernel(const int64_t* acc, const int64_t* ranges, int64_t* sums) {
    constexpr int NA = CRBM_N_ACC;
    __shared__ int64_t part[NA * 256];
    const int tid = threadIdx.x;
    const int64_t c0 = ranges[2 * blockIdx.x], c1 = c0 + ranges[2 * blockIdx.x + 1];
    int64_t s[NA];
#pragma unroll
    for (int x = 0; x < NA; ++x) s[x] = 0;
    for (int64_t c = c0 + tid; c < c1; c += 256) {
#pragma unroll
        for (int x = 0; x < NA; ++x) s[x] += acc[c * NA + x];
    }
#pragma unroll
    for (int x = 0; x < NA; ++x) part[x * 256 + tid] = s[x];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
#pragma unroll
            for (int x = 0; x < NA; ++x) part[x * 256 + tid] += part[x * 256 + tid + w];
        }
        __syncthreads();
    }
    if (tid < NA) sums[(int64_t)blockIdx.x * NA + tid] = part[tid * 256];
}
}  // namespace

hipError_t launch_acc_sum(const int64_t* acc, const int64_t* ranges, int n_inst, int64_t* sums, hipStream_t st) {
    if (n_inst <= 0) return hipSuccess;
    hipLaunchKernelGGL(acc_sum_kernel, dim3((unsigned)n_inst), dim3(256), 0, st, acc, ranges, sums);
    return hipGetLastError();
}

hipError_t launch_init(uint32_t* state, const Item* items, int n_items, int L, int R, uint64_t seed,
                       hipStream_t st) {
    (void)R;
    const int blocks = (n_items + 3) / 4;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(init_kernel, dim3(blocks), dim3(256), 0, st, state, items, n_items, L, seed);
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
    switch (L) {
#define CORR_CASE(l) \
    case l: return launch_corr_t<l>(state, nchains, corr, st);
        CORR_CASE(4) CORR_CASE(6) CORR_CASE(8) CORR_CASE(10) CORR_CASE(12) CORR_CASE(14) CORR_CASE(16)
        CORR_CASE(18) CORR_CASE(20) CORR_CASE(22) CORR_CASE(24) CORR_CASE(26) CORR_CASE(28) CORR_CASE(30)
        CORR_CASE(32) CORR_CASE(36) CORR_CASE(40) CORR_CASE(48) CORR_CASE(64) CORR_CASE(72) CORR_CASE(96)
#undef CORR_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace crbmlib
