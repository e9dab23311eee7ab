// stats.hip -- integrated autocorrelation time and effective sample size of
// an observable of the per-sweep counts trace, for the ESS/s comparison of
// samplers; and the per-chain minimum energy and first-hit sweep behind the
// time-to-solution of Sec. III.C Eq. (14).
//
// O[t][c] = wM M + wB1 B1 + wB2 B2 from the trace record (M, B1, B2) of chain
// c at sample t.  The grand mean over chains and kept samples is removed, so
// that chains stuck at different levels appear as correlation that does not
// decay; the autocovariance at lag k is summed over chains and samples in
// fp64 and normalised by (n - k); the host turns it into rho(k) and applies
// the automatic window.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "crbm.h"
#include "crbm_internal.h"

namespace crbmlib {
namespace {

// one thread per chain: mean of O over samples [discard, n)
__global__ void chain_mean_kernel(const int32_t* trace, int64_t n, int64_t stride_chains, int64_t c0, int64_t nc,
                                  int64_t discard, double w0, double w1, double w2, double* mean) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    double s = 0.0;
    for (int64_t t = discard; t < n; ++t) {
        const int32_t* r = trace + (t * stride_chains + c0 + c) * 3;
        s += w0 * r[0] + w1 * r[1] + w2 * r[2];
    }
    mean[c] = s / (double)(n - discard);
}

// one block: grand mean = mean of the per-chain means (equal sample counts)
__global__ void __launch_bounds__(256) grand_mean_kernel(const double* mean, int64_t nc, double* gm) {
    double s = 0.0;
    for (int64_t c = threadIdx.x; c < nc; c += blockDim.x) s += mean[c];
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *gm = red[0] / (double)nc;
}

// centred series, layout [t][c] so that consecutive threads read consecutive words
__global__ void centre_kernel(const int32_t* trace, int64_t n, int64_t stride_chains, int64_t c0, int64_t nc,
                              int64_t discard, double w0, double w1, double w2, const double* gm, double* x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t m = n - discard;
    if (i >= m * nc) return;
    const int64_t t = i / nc, c = i % nc;
    const int32_t* r = trace + ((t + discard) * stride_chains + c0 + c) * 3;
    x[i] = w0 * r[0] + w1 * r[1] + w2 * r[2] - *gm;
}

// block (lag k, chain block b): partial[k][b] = sum over its chains and t of x[t] x[t+k]
__global__ void __launch_bounds__(256) autocov_kernel(const double* x, int64_t m, int64_t nc, int max_lag,
                                                      double* partial, int nblk) {
    const int k = blockIdx.x;
    const int b = blockIdx.y;
    const int64_t c = (int64_t)b * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (c < nc)
        for (int64_t t = 0; t + k < m; ++t) s += x[t * nc + c] * x[(t + k) * nc + c];
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)k * nblk + b] = red[0];
    (void)max_lag;
}

// one thread per chain of [c0, c0 + nc): fold samples [0, n) of the counts
// trace into the chain's running minimum of E = w0 M + w1 B1 + w2 B2 (exact
// int64) and the number of completed sweeps at which that minimum was first
// reached; sample t of the trace was recorded after sweep0 + (t + 1) every
// sweeps.  A later sample only replaces the minimum if it is strictly lower.
__global__ void min_energy_kernel(const int32_t* trace, int64_t n, int64_t stride_chains, int64_t c0, int64_t nc,
                                  int64_t w0, int64_t w1, int64_t w2, int64_t sweep0, int64_t every, int reset,
                                  int64_t* emin, int64_t* first) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    int64_t best = reset ? INT64_MAX : emin[c];
    int64_t at = reset ? -1 : first[c];
    for (int64_t t = 0; t < n; ++t) {
        const int32_t* r = trace + (t * stride_chains + c0 + c) * 3;
        const int64_t E = w0 * (int64_t)r[0] + w1 * (int64_t)r[1] + w2 * (int64_t)r[2];
        if (E < best) {
            best = E;
            at = sweep0 + (t + 1) * every;
        }
    }
    emin[c] = best;
    first[c] = at;
}

// one thread per lag k: the autocovariance sum at lag k over the chain
// blocks' partial sums, added in block order (the order in which the host
// adds them in crbm_tau_int, so both entry points give the same sums)
__global__ void lag_sum_kernel(const double* part, int K, int nblk, double* sums) {
    const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k > K) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)k * nblk + b];
    sums[k] = s;
}

// Scratch of crbm_tau_int_noalloc: chain means and grand mean, the centred
// series and the per-block partial sums, all in one file-scope device array
// (each device holds its own copy).  Host code reaches it only through the
// address hipGetSymbolAddress returns for the current device.
constexpr int64_t kTauScratchDoubles = CRBM_TAU_NOALLOC_MAX_DOUBLES;
__device__ __align__(256) double scratch[kTauScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

// Device address of the current device's scratch array, looked up once per
// device.  Returns nullptr (with the error set) if the lookup fails.
double* scratch_ptr() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        set_error(CRBM_EHIP, "crbm_tau_int_noalloc: no current device");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(CRBM_EHIP, "crbm_tau_int_noalloc: hipGetSymbolAddress failed");
            return nullptr;
        }
        g_scratch[dev] = static_cast<double*>(p);
    }
    return g_scratch[dev];
}

}  // namespace
}  // namespace crbmlib

using namespace crbmlib;

extern "C" int crbm_min_energy(const int32_t* trace_dev, int64_t n_samples, int64_t trace_chains, int64_t c0,
                               int64_t c1, const int64_t w[3], int64_t sweep0, int32_t trace_every, int32_t reset,
                               int64_t* emin_dev, int64_t* first_dev, void* stream) {
    if (!w || !emin_dev || !first_dev || n_samples < 0 || (n_samples > 0 && !trace_dev) || trace_chains < 1 ||
        c0 < 0 || c1 > trace_chains || c1 <= c0 || sweep0 < 0 || trace_every < 1)
        return set_error(CRBM_EINVAL, "crbm_min_energy: bad arguments");
    const int64_t lim = (int64_t)1 << 31;
    for (int k = 0; k < 3; ++k)
        if (w[k] <= -lim || w[k] >= lim) return set_error(CRBM_EINVAL, "crbm_min_energy: |w| must be < 2^31");
    const int64_t nc = c1 - c0;
    hipLaunchKernelGGL(min_energy_kernel, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       trace_dev, n_samples, trace_chains, c0, nc, w[0], w[1], w[2], sweep0, (int64_t)trace_every,
                       reset ? 1 : 0, emin_dev, first_dev);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(CRBM_EHIP, hipGetErrorString(e));
    set_error(CRBM_OK, "");
    return CRBM_OK;
}

extern "C" int crbm_tau_int(const int32_t* trace_dev, int64_t n_samples, int64_t trace_chains, int64_t c0,
                            int64_t c1, int64_t discard, const double w[3], int32_t max_lag, double c_window,
                            void* stream, double* tau_out, double* ess_out, int32_t* window_out,
                            double* rho_out) {
    if (!trace_dev || !w || !tau_out || n_samples < 2 || trace_chains < 1 || c0 < 0 || c1 > trace_chains ||
        c1 <= c0 || discard < 0 || n_samples - discard < 2 || max_lag < 1 || !(c_window > 0.0))
        return set_error(CRBM_EINVAL, "crbm_tau_int: bad arguments");
    hipStream_t st = (hipStream_t)stream;
    const int64_t nc = c1 - c0, m = n_samples - discard;
    const int K = (int)std::min<int64_t>(max_lag, m - 1);
    double *d_mean = nullptr, *d_x = nullptr, *d_part = nullptr;
    const int nblk = (int)((nc + 255) / 256);
    if (dev_alloc(&d_mean, sizeof(double) * (nc + 1)) != hipSuccess) return set_error(CRBM_ENOMEM, "hipMalloc");
    if (dev_alloc(&d_x, sizeof(double) * m * nc) != hipSuccess) {
        (void)hipFree(d_mean);
        return set_error(CRBM_ENOMEM, "hipMalloc");
    }
    if (dev_alloc(&d_part, sizeof(double) * (int64_t)(K + 1) * nblk) != hipSuccess) {
        (void)hipFree(d_mean);
        (void)hipFree(d_x);
        return set_error(CRBM_ENOMEM, "hipMalloc");
    }
    hipLaunchKernelGGL(chain_mean_kernel, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, trace_dev,
                       n_samples, trace_chains, c0, nc, discard, w[0], w[1], w[2], d_mean);
    hipLaunchKernelGGL(grand_mean_kernel, dim3(1), dim3(256), 0, st, d_mean, nc, d_mean + nc);
    hipLaunchKernelGGL(centre_kernel, dim3((unsigned)((m * nc + 255) / 256)), dim3(256), 0, st, trace_dev,
                       n_samples, trace_chains, c0, nc, discard, w[0], w[1], w[2], d_mean + nc, d_x);
    hipLaunchKernelGGL(autocov_kernel, dim3((unsigned)(K + 1), (unsigned)nblk), dim3(256), 0, st, d_x, m, nc, K,
                       d_part, nblk);
    std::vector<double> part((size_t)(K + 1) * nblk);
    hipError_t e = hipMemcpyAsync(part.data(), d_part, sizeof(double) * part.size(), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d_mean);
    (void)hipFree(d_x);
    (void)hipFree(d_part);
    if (e != hipSuccess) return set_error(CRBM_EHIP, hipGetErrorString(e));
    std::vector<double> gam(K + 1);
    for (int k = 0; k <= K; ++k) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += part[(size_t)k * nblk + b];
        gam[k] = s / (double)(m - k) / (double)nc;
    }
    double tau = 1.0;
    int W = K;
    if (gam[0] > 0.0) {
        for (int k = 1; k <= K; ++k) {
            tau += 2.0 * gam[k] / gam[0];
            if ((double)k >= c_window * tau) {
                W = k;
                break;
            }
        }
    }
    if (rho_out)
        for (int k = 0; k <= K; ++k) rho_out[k] = gam[0] > 0.0 ? gam[k] / gam[0] : (k == 0 ? 1.0 : 0.0);
    *tau_out = tau;
    if (ess_out) *ess_out = (double)nc * (double)m / tau;
    if (window_out) *window_out = W;
    set_error(CRBM_OK, "");
    return CRBM_OK;
}

extern "C" int crbm_tau_int_noalloc(const int32_t* trace_dev, int64_t n_samples, int64_t trace_chains, int64_t c0,
                                    int64_t c1, int64_t discard, const double w[3], int32_t max_lag,
                                    double c_window, void* stream, double* tau_out, double* ess_out,
                                    int32_t* window_out, double* rho_out) {
    if (!trace_dev || !w || !tau_out || n_samples < 2 || trace_chains < 1 || c0 < 0 || c1 > trace_chains ||
        c1 <= c0 || discard < 0 || n_samples - discard < 2 || max_lag < 1 || !(c_window > 0.0))
        return set_error(CRBM_EINVAL, "crbm_tau_int_noalloc: bad arguments");
    const int64_t nc = c1 - c0, m = n_samples - discard;
    const int K = (int)std::min<int64_t>(max_lag, m - 1);
    const int nblk = (int)((nc + 255) / 256);
    if (K > CRBM_TAU_NOALLOC_MAX_LAG)
        return set_error(CRBM_ERANGE, "crbm_tau_int_noalloc: max_lag (capped at n_samples - discard - 1) exceeds "
                                      "CRBM_TAU_NOALLOC_MAX_LAG");
    // scratch layout: [nc + 1] means | [m nc] centred series | [(K + 1) nblk] partials | [K + 1] lag sums
    const int64_t need = (nc + 1) + m * nc + (int64_t)(K + 1) * nblk + (K + 1);
    if (nc > kTauScratchDoubles || m > kTauScratchDoubles || need > kTauScratchDoubles)
        return set_error(CRBM_ERANGE, "crbm_tau_int_noalloc: the request needs more than "
                                      "CRBM_TAU_NOALLOC_MAX_DOUBLES doubles of scratch");
    double* base = scratch_ptr();
    if (!base) return CRBM_EHIP;
    hipStream_t st = (hipStream_t)stream;
    double* d_mean = base;
    double* d_x = d_mean + (nc + 1);
    double* d_part = d_x + m * nc;
    double* d_sums = d_part + (int64_t)(K + 1) * nblk;
    // every scratch word that is read is written first in this call: no clearing needed
    hipLaunchKernelGGL(chain_mean_kernel, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, trace_dev,
                       n_samples, trace_chains, c0, nc, discard, w[0], w[1], w[2], d_mean);
    hipLaunchKernelGGL(grand_mean_kernel, dim3(1), dim3(256), 0, st, d_mean, nc, d_mean + nc);
    hipLaunchKernelGGL(centre_kernel, dim3((unsigned)((m * nc + 255) / 256)), dim3(256), 0, st, trace_dev,
                       n_samples, trace_chains, c0, nc, discard, w[0], w[1], w[2], d_mean + nc, d_x);
    hipLaunchKernelGGL(autocov_kernel, dim3((unsigned)(K + 1), (unsigned)nblk), dim3(256), 0, st, d_x, m, nc, K,
                       d_part, nblk);
    hipLaunchKernelGGL(lag_sum_kernel, dim3((unsigned)((K + 1 + 255) / 256)), dim3(256), 0, st, d_part, K, nblk,
                       d_sums);
    hipError_t e = hipGetLastError();
    double sums[CRBM_TAU_NOALLOC_MAX_LAG + 1];
    if (e == hipSuccess) e = hipMemcpyAsync(sums, d_sums, sizeof(double) * (size_t)(K + 1), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return set_error(CRBM_EHIP, hipGetErrorString(e));
    for (int k = 0; k <= K; ++k) sums[k] = sums[k] / (double)(m - k) / (double)nc;
    double tau = 1.0;
    int W = K;
    if (sums[0] > 0.0) {
        for (int k = 1; k <= K; ++k) {
            tau += 2.0 * sums[k] / sums[0];
            if ((double)k >= c_window * tau) {
                W = k;
                break;
            }
        }
    }
    if (rho_out)
        for (int k = 0; k <= K; ++k) rho_out[k] = sums[0] > 0.0 ? sums[k] / sums[0] : (k == 0 ? 1.0 : 0.0);
    *tau_out = tau;
    if (ess_out) *ess_out = (double)nc * (double)m / tau;
    if (window_out) *window_out = W;
    set_error(CRBM_OK, "");
    return CRBM_OK;
}
