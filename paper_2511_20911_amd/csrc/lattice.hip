// lattice.hip -- host side of the general-lattice sampler (Lr x Lc, each
// axis periodic or open, one coupling per filter, even/odd column biases):
// tables, handles, launches by column count, and the start-state, pack and
// unpack kernels.  The sampling kernel is in lattice_kernel.h.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "crbm.h"
#include "crbm_internal.h"
#include "lattice_kernel.h"

namespace crbmlib {
namespace lat {

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
    static constexpr int kGroups = CRBM_LAT_MAX_SIDE / 2 + 1;
    std::vector<LatItem> items[kGroups];  // by column count / 2
    LatItem* d_items[kGroups] = {};
    int lds_bytes[kGroups] = {};
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
        for (int x = 0; x < kGroups; ++x)
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
    a.tail_cap = tail_cap();
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
            h->items[I.cols / 2].push_back(it);
        }
        if (cfg->flags & CRBM_F_CORR) {
            h->corr_off.push_back(h->corr_words);
            for (auto& it : h->items[I.cols / 2])
                if (it.gbase >= (uint64_t)chains) it.corr_off = h->corr_words;
            h->corr_words += (int64_t)I.rows * (2 * I.cols - 1);
        }
        words += (int64_t)I.n_chains * I.rows * W;
        spins += (int64_t)I.n_chains * I.rows * I.cols;
        chains += I.n_chains;
        h->lds_bytes[I.cols / 2] = std::max(h->lds_bytes[I.cols / 2], lat_lds_bytes(I.rows, W));
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
    for (int x = 0; x < crbm_lat_s::kGroups; ++x) {
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
    for (int x = 0; x < crbm_lat_s::kGroups; ++x) {
        if (h->items[x].empty()) continue;
        const LatArgs a = lat_args(h, x, h->cur, h->cur + n_sweeps, spins_out, counts_trace, trace_every);
        const int Lc = 2 * x, lds = h->lds_bytes[x];
        hipError_t e = hipSuccess;
        const bool found = widths_a(Lc, a, lds, h->stream, &e) || widths_b(Lc, a, lds, h->stream, &e) ||
                           widths_c(Lc, a, lds, h->stream, &e) || widths_d(Lc, a, lds, h->stream, &e);
        if (!found) return lfail(CRBM_EUNSUPPORTED, "no lattice kernel compiled for " + std::to_string(Lc) + " columns");
        LAT_HIP(e, "lattice kernel");
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
