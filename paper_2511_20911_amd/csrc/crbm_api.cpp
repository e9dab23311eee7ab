// crbm_api.cpp -- host side of the C ABI declared in include/crbm.h.
//
// The host maps each Hamiltonian point to the CRBM (Sec. II.A Eqs. (4)-(10)):
// per sweep of the temperature schedule it computes the fixed-point hidden
// weights and visible bias and tabulates the 32-bit sigmoid thresholds the
// device compares against (App. A Sigmoid module: closest value).  The paper's
// host does the same mapping before writing the FPGA registers (App. A I/O).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <atomic>
#include <mutex>
#include <vector>

#include "crbm.h"
#include "crbm_internal.h"

using namespace crbmlib;

namespace {
thread_local std::string g_err;
}

namespace {
// allocations to let through before the armed failure; -1 = not armed
std::atomic<int64_t> g_alloc_countdown{-1};
}

hipError_t crbmlib::dev_alloc_bytes(void** p, size_t bytes) {
    int64_t c = g_alloc_countdown.load();
    while (c >= 0) {
        if (g_alloc_countdown.compare_exchange_weak(c, c - 1)) {
            if (c == 0) {
                *p = nullptr;
                return hipErrorOutOfMemory;
            }
            break;
        }
    }
    return hipMalloc(p, bytes);
}

extern "C" int crbm_debug_fail_alloc(int32_t n) {
    g_alloc_countdown.store(n < 0 ? -1 : (int64_t)n);
    return CRBM_OK;
}

namespace {
std::atomic<uint32_t> g_tail_cap{64u};
}

uint32_t crbmlib::tail_cap() { return g_tail_cap.load(); }

extern "C" int crbm_debug_tail_cap(int32_t cap) {
    if (cap < 1 || cap > 64) return crbmlib::set_error(CRBM_EINVAL, "the tail cap must be 1 .. 64");
    g_tail_cap.store((uint32_t)cap);
    return CRBM_OK;
}

int crbmlib::set_error(int code, const char* msg) {
    g_err = msg ? msg : "";
    return code;
}

namespace {

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr, what)                                                                  \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(CRBM_EHIP, std::string(what) + ": " + hipGetErrorString(e_));         \
    } while (0)

// ---- the mapping (library's own implementation of the conventions) ----

int64_t q16(double x) { return llround(x * 65536.0); }

double schedule_T(int kind, double T0, double T1, const double* Te, int64_t S, int64_t s) {
    switch (kind) {
        case CRBM_SCHED_CONST: return T0;
        case CRBM_SCHED_LINEAR: return S <= 1 ? T0 : T0 + (T1 - T0) * ((double)s / (double)(S - 1));
        case CRBM_SCHED_GEOMETRIC: return S <= 1 ? T0 : T0 * pow(T1 / T0, (double)s / (double)(S - 1));
        case CRBM_SCHED_EXPLICIT: return Te[s];
        default: return NAN;
    }
}

// Hidden weight for coupling Jq at temperature T: K = -J/T,
// w = arccosh(exp(2|K|))/2 = |K| + log1p(sqrt(1 - exp(-4|K|)))/2 (Eqs. (6)-(7)).
void hidden_weight(int64_t Jq, double T, int64_t* wq, int* sig) {
    const double K = -((double)Jq / 65536.0) / T;
    const double k = fabs(K);
    const double w = k + 0.5 * log1p(sqrt(-expm1(-4.0 * k)));
    *wq = llround(w * 65536.0);
    *sig = K < 0.0 ? -1 : 1;
}

uint32_t threshold(int64_t y) {
    const double p = 1.0 / (1.0 + exp(-(2.0 * ldexp((double)y, -16))));
    double t = floor(p * 4294967296.0 + 0.5);
    if (t > 4294967295.0) t = 4294967295.0;
    return (uint32_t)t;
}

// The paper's hardware precision (App. A Dimension and Precision; Sigmoid and
// LFSR-Forward), in 16.16 units: signed Q5.4 values are multiples of 2^12
// with magnitude at most 511 steps (saturating); the visible accumulator has
// two more integer bits (2047 steps); the sigmoid is the closest 16-bit value,
// so the 32-bit threshold is that value shifted up by 16 bits and the compare
// with a 32-bit uniform decides on its top 16 bits alone.
constexpr int64_t kQ54Step = 4096, kQ54Max = 511 * kQ54Step, kAccMax = 2047 * kQ54Step;

int64_t q54(double v) {
    double m = floor(fabs(v) * 16.0 + 0.5);
    if (m > 511.0) m = 511.0;
    return (v < 0.0 ? -(int64_t)m : (int64_t)m) * kQ54Step;
}

int64_t saturate(int64_t x, int64_t lim) { return x > lim ? lim : (x < -lim ? -lim : x); }

uint32_t threshold16(int64_t y) {
    const double p = 1.0 / (1.0 + exp(-(2.0 * ldexp((double)y, -16))));
    double t = floor(p * 65536.0 + 0.5);
    if (t > 65535.0) t = 65535.0;
    return (uint32_t)t << 16;
}

// One sweep's 16-word device table (layout in crbm_internal.h).
int build_table(int64_t J1q, int64_t J2q, int64_t hq, double T, int precision, uint32_t* out) {
    int64_t wq1, wq2;
    int s1, s2;
    hidden_weight(J1q, T, &wq1, &s1);
    hidden_weight(J2q, T, &wq2, &s2);
    int64_t aq = llround((double)hq / T);
    const bool fpga = precision == CRBM_PRECISION_FPGA;
    if (fpga) {
        // re-round the exact weights and bias to Q5.4 (the 16.16 values above
        // are only used for the range check of the default path)
        const double K1 = fabs(((double)J1q / 65536.0) / T), K2 = fabs(((double)J2q / 65536.0) / T);
        wq1 = q54(K1 + 0.5 * log1p(sqrt(-expm1(-4.0 * K1))));
        wq2 = q54(K2 + 0.5 * log1p(sqrt(-expm1(-4.0 * K2))));
        aq = q54(((double)hq / 65536.0) / T);
    }
    const int64_t lim = (int64_t)1 << 31;
    if (wq1 >= lim || wq2 >= lim || aq >= lim || aq <= -lim) return CRBM_ERANGE;
    auto thr = [&](int64_t y) { return fpga ? threshold16(y) : threshold(y); };
    std::memset(out, 0, sizeof(uint32_t) * kTabWords);
    out[0] = thr(fpga ? saturate(2 * wq1, kQ54Max) : 2 * wq1);
    out[1] = thr(fpga ? saturate(2 * wq2, kQ54Max) : 2 * wq2);
    uint32_t kge[2] = {5u, 5u};
    for (int d = 0; d < 2; ++d)
        for (int n = 4; n >= 0; --n) {
            int64_t x = aq + wq1 * (2 * n - 4) + wq2 * (2 * d - 1);
            if (fpga) x = saturate(x, kAccMax);
            out[3 + 2 * n + d] = thr(x < 0 ? -x : x);
            if (x >= 0) kge[d] = (uint32_t)n;
        }
    out[2] = (s1 < 0 ? 1u : 0u) | (s2 < 0 ? 2u : 0u) | (wq1 != 0 ? 4u : 0u) | (wq2 != 0 ? 8u : 0u) |
             (kge[0] << 8) | (kge[1] << 12);
    return CRBM_OK;
}

}  // namespace

double crbmlib::map_schedule_T(int kind, double T0, double T1, const double* Te, int64_t S, int64_t s) {
    return schedule_T(kind, T0, T1, Te, S, s);
}
void crbmlib::map_hidden_weight(int64_t Jq, double T, int64_t* wq, int* sig) { hidden_weight(Jq, T, wq, sig); }
uint32_t crbmlib::map_threshold(int64_t y) { return threshold(y); }

namespace {

// Default cell rows per lane, used until the autotuner or the caller sets
// one: the compiled tiling nearest to what the autotuner picks on this GPU
// (one cell row per lane up to L = 22, two up to 40, three above: fewer rows
// keep each lane's share of a sweep short, more keep the registers of the
// multi-word rows in bounds), the smaller on a tie.
int default_rows(int L) {
    const int C = L / 2;
    const int want = L <= 22 ? 1 : (L <= 40 ? 2 : 3);
    int best = 0;
    for (int R = 1; R <= C; ++R) {
        if (C % R != 0 || !gibbs_supported(L, R) || C / R > 64) continue;
        if (best == 0 || std::abs(R - want) < std::abs(best - want)) best = R;
    }
    return best;
}

bool lattice_supported(int L) { return default_rows(L) > 0; }

// Process-wide tiling choice per lattice side (set by the autotuner or by hand).
struct Tiling {
    int rows = 0, wpb = 0;
};
std::mutex g_tiling_mu;
Tiling g_tiling[CRBM_MAX_L + 1];

Tiling tiling_for(int L) {
    std::lock_guard<std::mutex> lk(g_tiling_mu);
    Tiling t = g_tiling[L];
    if (t.rows == 0) t.rows = default_rows(L);
    if (t.wpb == 0) t.wpb = 4;
    return t;
}

struct Group {
    int L = 0, R = 0, wpb = 4, grid_blocks = 0;
    std::vector<Item> items;
    Item* d_items = nullptr;
    hipGraphNode_t node = nullptr;
    const void* fn = nullptr;  // the kernel of the graph node (per-call updates keep it)
};

}  // namespace

struct crbm_s {
    std::vector<crbm_instance> inst;
    std::vector<std::vector<double>> Texp;
    std::vector<int64_t> Jq[3];
    std::vector<int64_t> gbase, state_off, spin_off;
    std::vector<uint64_t> tab_off;
    std::vector<uint32_t> tab_stride;
    std::vector<uint32_t> h_tables;
    crbm_config cfg{};
    hipStream_t stream = nullptr;
    int64_t total_chains = 0, total_words = 0, total_spins = 0;
    int64_t S = 0, cur = 0;
    uint32_t* d_state = nullptr;
    uint32_t* d_tables = nullptr;
    int64_t* d_acc = nullptr;
    int64_t* d_ranges = nullptr;  // per instance: first global chain, chain count
    int64_t* d_sums = nullptr;    // per instance: the accumulators summed over its chains
    uint32_t* d_queue = nullptr;  // one work counter per group (graph mode)
    unsigned long long* d_corr = nullptr;  // CRBM_F_CORR: summed C(dr, dc), [sum over instances of L^2]
    std::vector<int64_t> corr_off;         // offset of each instance's C block
    std::vector<Group> groups;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~crbm_s() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (d_state) (void)hipFree(d_state);
        if (d_tables) (void)hipFree(d_tables);
        if (d_acc) (void)hipFree(d_acc);
        if (d_ranges) (void)hipFree(d_ranges);
        if (d_sums) (void)hipFree(d_sums);
        if (d_queue) (void)hipFree(d_queue);
        if (d_corr) (void)hipFree(d_corr);
        for (auto& g : groups)
            if (g.d_items) (void)hipFree(g.d_items);
    }
};

namespace crbmlib {
// sums[i][x] = sum of acc[c][x] over the chains c of instance i, whose first
// chain and count are ranges[2i] and ranges[2i+1] (device arrays); in gibbs_aux.hip.
hipError_t launch_acc_sum(const int64_t* acc, const int64_t* ranges, int n_inst, int64_t* sums, hipStream_t st);
}  // namespace crbmlib

namespace {

GibbsArgs make_args(const crbm_s* h, const Group& g, size_t gi, int64_t s0, int64_t s1, int8_t* spins_out,
                    int32_t* trace, int32_t trace_every = 1, int32_t* order = nullptr, int64_t trace_s0 = -1,
                    bool direct = false) {
    GibbsArgs a{};
    a.trace_s0 = trace_s0 < 0 ? s0 : trace_s0;
    a.state = h->d_state;
    a.tables = h->d_tables;
    a.items = g.d_items;
    a.n_items = (int32_t)g.items.size();
    a.measure_every = h->cfg.measure_every;
    a.s0 = s0;
    a.s1 = s1;
    a.burn_in = h->cfg.burn_in;
    a.seed = h->cfg.seed;
    a.acc = h->d_acc;
    a.trace = trace;
    a.trace_every = trace_every;
    a.order = order;
    a.total_chains = h->total_chains;
    a.spins_out = spins_out;
    a.queue = (h->cfg.launch_mode == CRBM_LAUNCH_GRAPH && !direct) ? h->d_queue + gi : nullptr;
    a.waves_per_block = g.wpb;
    a.grid_blocks = g.grid_blocks;
    a.tail_cap = tail_cap();
    return a;
}

// Graph: [reset the work counters] -> one persistent Gibbs kernel per lattice
// size, all depending only on the reset node (parallel branches).
int build_graph(crbm_s* h) {
    HIP_TRY(hipGraphCreate(&h->graph, 0), "hipGraphCreate");
    hipGraphNode_t reset = nullptr;
    {
        int n = (int)h->groups.size();
        uint32_t* q = h->d_queue;
        void* args[] = {&q, &n};
        hipKernelNodeParams p{};
        p.func = const_cast<void*>(zero_u32_fn());
        p.gridDim = dim3((unsigned)((n + 255) / 256));
        p.blockDim = dim3(256);
        p.sharedMemBytes = 0;
        p.kernelParams = args;
        p.extra = nullptr;
        HIP_TRY(hipGraphAddKernelNode(&reset, h->graph, nullptr, 0, &p), "graph reset node");
    }
    // Nodes in decreasing order of work (chains x L^2): the process has a few
    // hardware queues (four by default), so only that many nodes run at once
    // and the largest sizes start together.  A later node waits for a node
    // that was added before it, not for the first queue to free up: in the
    // traces of the six-size batch, the fifth and sixth nodes started when the
    // first and second ended.
    std::vector<size_t> order(h->groups.size());
    std::vector<double> work(h->groups.size(), 0.0);
    for (size_t gi = 0; gi < h->groups.size(); ++gi) {
        order[gi] = gi;
        for (const Item& it : h->groups[gi].items) work[gi] += (double)it.nchains * it.L * it.L;
    }
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return work[x] > work[y]; });
    for (const size_t gi : order) {
        Group& g = h->groups[gi];
        GibbsArgs a = make_args(h, g, gi, 0, 0, nullptr, nullptr);
        void* args[] = {&a};
        hipKernelNodeParams p{};
        g.fn = gibbs_kernel_fn(g.L, g.R);
        p.func = const_cast<void*>(g.fn);
        const int items_blocks = (int)((g.items.size() + g.wpb - 1) / g.wpb);
        p.gridDim = dim3((unsigned)std::max(1, std::min(items_blocks, g.grid_blocks)));
        p.blockDim = dim3((unsigned)(64 * g.wpb));
        p.sharedMemBytes = 0;
        p.kernelParams = args;
        p.extra = nullptr;
        HIP_TRY(hipGraphAddKernelNode(&g.node, h->graph, &reset, 1, &p), "graph Gibbs node");
    }
    HIP_TRY(hipGraphInstantiate(&h->exec, h->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    return CRBM_OK;
}

}  // namespace

int crbmlib::handle_view(crbm_t* h, HandleView* v, int i) {
    if (!h || !v || i < 0 || i >= (int)h->inst.size()) return CRBM_EINVAL;
    const crbm_instance& I = h->inst[(size_t)i];
    v->state = h->d_state + h->state_off[(size_t)i];
    v->L = I.L;
    v->n_chains = I.n_chains;
    v->id = I.id;
    v->seed = h->cfg.seed;
    v->n_inst = (int)h->inst.size();
    v->sched_kind = I.sched_kind;
    v->T0 = I.T0;
    v->cur = h->cur;
    v->S = h->S;
    v->stream = h->stream;
    v->precision = h->cfg.precision;
    int64_t wq1, wq2;
    hidden_weight(h->Jq[0][(size_t)i], I.T0, &wq1, &v->sg1);
    hidden_weight(h->Jq[1][(size_t)i], I.T0, &wq2, &v->sg2);
    v->a = (double)llround((double)h->Jq[2][(size_t)i] / I.T0) / 65536.0;
    v->c1 = log(cosh(2.0 * (double)wq1 / 65536.0));
    v->c2 = log(cosh(2.0 * (double)wq2 / 65536.0));
    return CRBM_OK;
}

extern "C" {

const char* crbm_last_error(void) { return g_err.c_str(); }

uint32_t crbm_threshold(int64_t y) { return threshold(y < 0 ? -y : y); }

int64_t crbm_total_chains(const crbm_t* h) { return h ? h->total_chains : 0; }

int crbm_create(const crbm_instance* inst, int32_t n_inst, const crbm_config* cfg, crbm_t** out) {
    g_err.clear();
    if (!out) return fail(CRBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!inst || n_inst < 1) return fail(CRBM_EINVAL, "need at least one instance");
    if (!cfg) return fail(CRBM_EINVAL, "cfg is NULL");
    if (cfg->n_sweeps < 1) return fail(CRBM_EINVAL, "n_sweeps must be >= 1");
    if (cfg->measure_every < 0 || cfg->burn_in < 0) return fail(CRBM_EINVAL, "measure_every and burn_in must be >= 0");
    if (cfg->launch_mode != CRBM_LAUNCH_DIRECT && cfg->launch_mode != CRBM_LAUNCH_GRAPH)
        return fail(CRBM_EINVAL, "unknown launch_mode");
    if (cfg->waves_per_block < 0 || cfg->waves_per_block > 4) return fail(CRBM_EINVAL, "waves_per_block must be 0..4");
    if (cfg->precision != CRBM_PRECISION_Q16 && cfg->precision != CRBM_PRECISION_FPGA)
        return fail(CRBM_EINVAL, "unknown precision");
    if (cfg->flags & ~CRBM_F_CORR) return fail(CRBM_EINVAL, "unknown flags");
    const double lim = 2147483647.0 / 65536.0;
    for (int i = 0; i < n_inst; ++i) {
        const crbm_instance& I = inst[i];
        const std::string tag = "instance " + std::to_string(i) + ": ";
        if (I.L < 4 || (I.L & 1)) return fail(CRBM_EINVAL, tag + "L must be even and >= 4");
        if (I.L > CRBM_MAX_L || !lattice_supported(I.L))
            return fail(CRBM_EUNSUPPORTED, tag + "no compiled kernel for this L");
        if (I.periodic != 1) return fail(CRBM_EUNSUPPORTED, tag + "only periodic lattices are supported");
        if (!std::isfinite(I.J1) || !std::isfinite(I.J2) || !std::isfinite(I.h))
            return fail(CRBM_EINVAL, tag + "J1, J2, h must be finite");
        if (fabs(I.J1) >= lim || fabs(I.J2) >= lim || fabs(I.h) >= lim)
            return fail(CRBM_ERANGE, tag + "|J| * 2^16 must fit in int32");
        if (I.n_chains < 1) return fail(CRBM_EINVAL, tag + "n_chains must be >= 1");
        if (I.id >= (1u << 29)) return fail(CRBM_EINVAL, tag + "id must be < 2^29");
        if (I.sched_kind < 0 || I.sched_kind > 3) return fail(CRBM_EINVAL, tag + "unknown schedule");
        if (I.sched_kind == CRBM_SCHED_EXPLICIT) {
            if (!I.T_explicit) return fail(CRBM_EINVAL, tag + "T_explicit is NULL");
            for (int64_t s = 0; s < cfg->n_sweeps; ++s)
                if (!(I.T_explicit[s] > 0.0) || !std::isfinite(I.T_explicit[s]))
                    return fail(CRBM_EINVAL, tag + "temperatures must be finite and > 0");
        } else {
            if (!(I.T0 > 0.0) || !std::isfinite(I.T0)) return fail(CRBM_EINVAL, tag + "T0 must be finite and > 0");
            if (I.sched_kind != CRBM_SCHED_CONST && (!(I.T1 > 0.0) || !std::isfinite(I.T1)))
                return fail(CRBM_EINVAL, tag + "T1 must be finite and > 0");
        }
        if (cfg->tile_rows != 0 && (((I.L / 2) % cfg->tile_rows) != 0 || !gibbs_supported(I.L, cfg->tile_rows)))
            return fail(CRBM_EUNSUPPORTED, tag + "tile_rows must divide L/2 (and have a compiled kernel)");
    }

    crbm_s* h = new (std::nothrow) crbm_s();
    if (!h) return fail(CRBM_ENOMEM, "host allocation failed");
    h->cfg = *cfg;
    h->stream = (hipStream_t)cfg->stream;
    h->S = cfg->n_sweeps;
    h->inst.assign(inst, inst + n_inst);
    h->Texp.resize(n_inst);
    for (int k = 0; k < 3; ++k) h->Jq[k].resize(n_inst);
    h->gbase.resize(n_inst);
    h->state_off.resize(n_inst);
    h->spin_off.resize(n_inst);
    h->tab_off.resize(n_inst);
    h->tab_stride.resize(n_inst);

    // per-sweep tables
    for (int i = 0; i < n_inst; ++i) {
        crbm_instance& I = h->inst[i];
        if (I.sched_kind == CRBM_SCHED_EXPLICIT) {
            h->Texp[i].assign(I.T_explicit, I.T_explicit + cfg->n_sweeps);
            I.T_explicit = h->Texp[i].data();
        } else {
            I.T_explicit = nullptr;
        }
        h->Jq[0][i] = q16(I.J1);
        h->Jq[1][i] = q16(I.J2);
        h->Jq[2][i] = q16(I.h);
        const int64_t ntab = (I.sched_kind == CRBM_SCHED_CONST) ? 1 : h->S;
        h->tab_off[i] = h->h_tables.size();
        h->tab_stride[i] = (I.sched_kind == CRBM_SCHED_CONST) ? 0u : (uint32_t)kTabWords;
        h->h_tables.resize(h->h_tables.size() + (size_t)ntab * kTabWords);
        for (int64_t s = 0; s < ntab; ++s) {
            const double T = schedule_T(I.sched_kind, I.T0, I.T1, I.T_explicit, h->S, s);
            const int rc = build_table(h->Jq[0][i], h->Jq[1][i], h->Jq[2][i], T, cfg->precision,
                                       h->h_tables.data() + h->tab_off[i] + (size_t)s * kTabWords);
            if (rc != CRBM_OK) {
                delete h;
                return fail(rc, "instance " + std::to_string(i) + ": fixed-point weight or bias overflows int32 at sweep " +
                                    std::to_string(s));
            }
        }
        h->gbase[i] = h->total_chains;
        h->state_off[i] = h->total_words;
        h->spin_off[i] = h->total_spins;
        h->total_chains += I.n_chains;
        h->total_words += (int64_t)I.n_chains * I.L * ((I.L + 31) / 32);
        h->total_spins += (int64_t)I.n_chains * I.L * I.L;
    }

    // work items, grouped by (L, R)
    for (int i = 0; i < n_inst; ++i) {
        const crbm_instance& I = h->inst[i];
        const Tiling tl = tiling_for(I.L);
        const int R = cfg->tile_rows ? cfg->tile_rows : tl.rows;
        const int wpb = cfg->waves_per_block ? cfg->waves_per_block : tl.wpb;
        Group* grp = nullptr;
        for (auto& g : h->groups)
            if (g.L == I.L && g.R == R && g.wpb == wpb) grp = &g;
        if (!grp) {
            h->groups.push_back(Group{});
            grp = &h->groups.back();
            grp->L = I.L;
            grp->R = R;
            grp->wpb = wpb;
        }
        const int cpw = chains_per_wave(I.L, R);
        for (int c0 = 0; c0 < I.n_chains; c0 += cpw) {
            Item it{};
            it.inst = (uint32_t)i;
            it.id = I.id;
            it.chain0 = (uint32_t)c0;
            it.nchains = (uint32_t)std::min(cpw, I.n_chains - c0);
            it.gbase = (uint64_t)(h->gbase[i] + c0);
            it.state_off = (uint64_t)(h->state_off[i] + (int64_t)c0 * I.L * ((I.L + 31) / 32));
            it.spin_off = (uint64_t)(h->spin_off[i] + (int64_t)c0 * I.L * I.L);
            it.tab_off = h->tab_off[i];
            it.tab_stride = h->tab_stride[i];
            it.L = (uint32_t)I.L;
            grp->items.push_back(it);
        }
    }

    // device state
    hipError_t e;
    if ((e = dev_alloc(&h->d_state, sizeof(uint32_t) * (size_t)h->total_words)) != hipSuccess ||
        (e = dev_alloc(&h->d_tables, sizeof(uint32_t) * h->h_tables.size())) != hipSuccess ||
        (e = dev_alloc(&h->d_acc, sizeof(int64_t) * CRBM_N_ACC * (size_t)h->total_chains)) != hipSuccess ||
        (e = dev_alloc(&h->d_ranges, sizeof(int64_t) * 2 * (size_t)n_inst)) != hipSuccess ||
        (e = dev_alloc(&h->d_sums, sizeof(int64_t) * CRBM_N_ACC * (size_t)n_inst)) != hipSuccess) {
        delete h;
        return fail(e == hipErrorOutOfMemory ? CRBM_ENOMEM : CRBM_EHIP, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    for (auto& g : h->groups) {
        if ((e = dev_alloc(&g.d_items, sizeof(Item) * g.items.size())) != hipSuccess) {
            delete h;
            return fail(CRBM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
    }
    if (cfg->flags & CRBM_F_CORR) {
        int64_t tot = 0;
        for (int i = 0; i < n_inst; ++i) {
            h->corr_off.push_back(tot);
            tot += (int64_t)h->inst[i].L * h->inst[i].L;
        }
        if ((e = dev_alloc(&h->d_corr, sizeof(unsigned long long) * (size_t)tot)) != hipSuccess) {
            delete h;
            return fail(CRBM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
    }
    if (cfg->launch_mode == CRBM_LAUNCH_GRAPH) {
        if ((e = dev_alloc(&h->d_queue, sizeof(uint32_t) * h->groups.size())) != hipSuccess) {
            delete h;
            return fail(CRBM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        int dev = 0, cus = 0;
        if ((e = hipGetDevice(&dev)) != hipSuccess ||
            (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) {
            delete h;
            return fail(CRBM_EHIP, std::string("device query: ") + hipGetErrorString(e));
        }
        for (auto& g : h->groups) {
            int per_cu = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, gibbs_kernel_fn(g.L, g.R), 64 * g.wpb, 0) !=
                    hipSuccess || per_cu < 1)
                per_cu = 1;
            g.grid_blocks = std::max(1, cus) * per_cu;
        }
    }
    int rc = CRBM_OK;
    auto chk = [&](hipError_t x, const char* what) {
        if (x != hipSuccess && rc == CRBM_OK) rc = fail(CRBM_EHIP, std::string(what) + ": " + hipGetErrorString(x));
    };
    chk(hipMemcpyAsync(h->d_tables, h->h_tables.data(), sizeof(uint32_t) * h->h_tables.size(), hipMemcpyHostToDevice,
                       h->stream), "copy tables");
    chk(hipMemsetAsync(h->d_acc, 0, sizeof(int64_t) * CRBM_N_ACC * (size_t)h->total_chains, h->stream), "zero acc");
    std::vector<int64_t> ranges(2 * (size_t)n_inst);
    for (int i = 0; i < n_inst; ++i) {
        ranges[2 * (size_t)i] = h->gbase[(size_t)i];
        ranges[2 * (size_t)i + 1] = h->inst[(size_t)i].n_chains;
    }
    chk(hipMemcpyAsync(h->d_ranges, ranges.data(), sizeof(int64_t) * ranges.size(), hipMemcpyHostToDevice, h->stream),
        "copy chain ranges");
    if (h->d_corr)
        chk(hipMemsetAsync(h->d_corr, 0, sizeof(unsigned long long) * (size_t)(h->corr_off.back() +
                                                                               (int64_t)h->inst.back().L * h->inst.back().L),
                           h->stream),
            "zero corr");
    for (auto& g : h->groups) {
        chk(hipMemcpyAsync(g.d_items, g.items.data(), sizeof(Item) * g.items.size(), hipMemcpyHostToDevice, h->stream),
            "copy items");
        chk(launch_init(h->d_state, g.d_items, (int)g.items.size(), g.L, g.R, cfg->seed, h->stream), "init kernel");
    }
    // the host vectors must outlive the async copies
    chk(hipStreamSynchronize(h->stream), "synchronize");
    if (rc == CRBM_OK && cfg->launch_mode == CRBM_LAUNCH_GRAPH) rc = build_graph(h);
    if (rc != CRBM_OK) {
        delete h;
        return rc;
    }
    *out = h;
    return CRBM_OK;
}

int crbm_sample(crbm_t* h, int64_t n_sweeps, int8_t* spins_out, int32_t* counts_trace) {
    return crbm_sample_thinned(h, n_sweeps, spins_out, counts_trace, nullptr, 1);
}

int crbm_sample_thinned(crbm_t* h, int64_t n_sweeps, int8_t* spins_out, int32_t* counts_trace,
                        int32_t* order_trace, int32_t trace_every) {
    g_err.clear();
    if (!h) return fail(CRBM_EINVAL, "handle is NULL");
    if (n_sweeps < 0) return fail(CRBM_EINVAL, "n_sweeps must be >= 0");
    if (trace_every < 1 || n_sweeps % trace_every != 0)
        return fail(CRBM_EINVAL, "trace_every must be >= 1 and divide n_sweeps");
    if (order_trace && !counts_trace) return fail(CRBM_EINVAL, "order_trace needs counts_trace");
    if (h->cur + n_sweeps > h->S) return fail(CRBM_ESTATE, "sampling past the end of the schedule");
    if (h->d_corr && h->cfg.measure_every > 0) {
        // one direct launch per measured sweep, then that sweep's C(dr, dc) added to the sums
        const int64_t call0 = h->cur, end = h->cur + n_sweeps, me = h->cfg.measure_every, b = h->cfg.burn_in;
        int64_t s = h->cur;
        while (s < end) {
            int64_t m = s < b ? b : s;  // next measured sweep >= s
            if ((m - b) % me) m += me - (m - b) % me;
            const int64_t stop = m < end ? m + 1 : end;
            for (size_t gi = 0; gi < h->groups.size(); ++gi) {
                const GibbsArgs a = make_args(h, h->groups[gi], gi, s, stop, stop == end ? spins_out : nullptr,
                                              counts_trace, trace_every, order_trace, call0, true);
                HIP_TRY(launch_gibbs(h->groups[gi].L, h->groups[gi].R, a, h->stream), "gibbs kernel");
            }
            if (m < end)
                for (size_t i = 0; i < h->inst.size(); ++i)
                    HIP_TRY(launch_corr(h->d_state + h->state_off[i], h->inst[i].n_chains, h->inst[i].L,
                                        h->d_corr + h->corr_off[i], h->stream),
                            "correlation kernel");
            s = stop;
        }
        h->cur = end;
        return CRBM_OK;
    }
    if (h->cfg.launch_mode == CRBM_LAUNCH_GRAPH) {
        for (size_t gi = 0; gi < h->groups.size(); ++gi) {
            Group& g = h->groups[gi];
            GibbsArgs a =
                make_args(h, g, gi, h->cur, h->cur + n_sweeps, spins_out, counts_trace, trace_every, order_trace);
            void* args[] = {&a};
            hipKernelNodeParams p{};
            p.func = const_cast<void*>(g.fn);
            const int items_blocks = (int)((g.items.size() + g.wpb - 1) / g.wpb);
            p.gridDim = dim3((unsigned)std::max(1, std::min(items_blocks, g.grid_blocks)));
            p.blockDim = dim3((unsigned)(64 * g.wpb));
            p.sharedMemBytes = 0;
            p.kernelParams = args;
            p.extra = nullptr;
            HIP_TRY(hipGraphExecKernelNodeSetParams(h->exec, g.node, &p), "update graph node");
        }
        HIP_TRY(hipGraphLaunch(h->exec, h->stream), "hipGraphLaunch");
    } else {
        for (size_t gi = 0; gi < h->groups.size(); ++gi) {
            const GibbsArgs a = make_args(h, h->groups[gi], gi, h->cur, h->cur + n_sweeps, spins_out, counts_trace,
                                          trace_every, order_trace);
            HIP_TRY(launch_gibbs(h->groups[gi].L, h->groups[gi].R, a, h->stream), "gibbs kernel");
        }
    }
    h->cur += n_sweeps;
    return CRBM_OK;
}

int crbm_set_tiling(int32_t L, int32_t rows, int32_t waves_per_block) {
    g_err.clear();
    if (L < 4 || L > CRBM_MAX_L || (L & 1)) return fail(CRBM_EINVAL, "bad L");
    if (rows < 1 || (L / 2) % rows != 0 || !gibbs_supported(L, rows)) return fail(CRBM_EUNSUPPORTED, "no such tiling");
    if (waves_per_block < 1 || waves_per_block > 4) return fail(CRBM_EINVAL, "waves_per_block must be 1..4");
    std::lock_guard<std::mutex> lk(g_tiling_mu);
    g_tiling[L].rows = rows;
    g_tiling[L].wpb = waves_per_block;
    return CRBM_OK;
}

int crbm_get_tiling(int32_t L, int32_t* rows, int32_t* waves_per_block) {
    g_err.clear();
    if (L < 4 || L > CRBM_MAX_L || (L & 1) || !lattice_supported(L)) return fail(CRBM_EUNSUPPORTED, "bad L");
    const Tiling t = tiling_for(L);
    if (rows) *rows = t.rows;
    if (waves_per_block) *waves_per_block = t.wpb;
    return CRBM_OK;
}

int crbm_autotune(int32_t L, int32_t n_chains, int32_t n_sweeps, void* stream, int32_t* best_rows,
                  int32_t* best_waves_per_block, double* best_rate) {
    g_err.clear();
    if (L < 4 || L > CRBM_MAX_L || (L & 1) || !lattice_supported(L)) return fail(CRBM_EUNSUPPORTED, "bad L");
    if (n_chains < 1 || n_sweeps < 1) return fail(CRBM_EINVAL, "n_chains and n_sweeps must be >= 1");
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
    HIP_TRY(hipEventCreate(&e1), "hipEventCreate");
    double best = -1.0;
    int bR = 0, bW = 0;
    const int wpbs[] = {1, 2, 4};
    for (int R = 1; R <= L / 2; ++R) {
        if ((L / 2) % R != 0 || !gibbs_supported(L, R) || (L / 2) / R > 64) continue;
        for (int wpb : wpbs) {
            crbm_instance I{};
            I.L = L;
            I.periodic = 1;
            I.J1 = 1.0;
            I.J2 = 1.0;
            I.h = 1.0;
            I.n_chains = n_chains;
            I.sched_kind = CRBM_SCHED_CONST;
            I.T0 = 1.0;
            crbm_config c{};
            c.seed = 1;
            c.n_sweeps = 2 * (int64_t)n_sweeps + 2;
            c.stream = stream;
            c.tile_rows = R;
            c.waves_per_block = wpb;
            crbm_t* t = nullptr;
            int rc = crbm_create(&I, 1, &c, &t);
            if (rc != CRBM_OK) {
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                return rc;
            }
            rc = crbm_sample(t, 2, nullptr, nullptr);  // warm-up
            if (rc == CRBM_OK && hipEventRecord(e0, st) != hipSuccess) rc = fail(CRBM_EHIP, "autotune: event record");
            if (rc == CRBM_OK) rc = crbm_sample(t, n_sweeps, nullptr, nullptr);
            float ms = 0.f;
            if (rc == CRBM_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                  hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = fail(CRBM_EHIP, "autotune: event timing");
            crbm_destroy(t);
            if (rc != CRBM_OK) {
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                return rc;
            }
            const double rate = (double)n_chains * n_sweeps * L * L / (ms * 1e-3);
            if (rate > best) {
                best = rate;
                bR = R;
                bW = wpb;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (bR == 0) return fail(CRBM_EUNSUPPORTED, "no tiling for this L");
    {
        std::lock_guard<std::mutex> lk(g_tiling_mu);
        g_tiling[L].rows = bR;
        g_tiling[L].wpb = bW;
    }
    if (best_rows) *best_rows = bR;
    if (best_waves_per_block) *best_waves_per_block = bW;
    if (best_rate) *best_rate = best;
    g_err.clear();
    return CRBM_OK;
}

int crbm_observables(crbm_t* h, crbm_obs* out, int64_t* corr_out) {
    g_err.clear();
    if (!h || !out) return fail(CRBM_EINVAL, "NULL argument");
    const int n = (int)h->inst.size();
    // summed over each instance's chains on the device; only the sums cross to the host
    std::vector<int64_t> sums((size_t)CRBM_N_ACC * n);
    HIP_TRY(launch_acc_sum(h->d_acc, h->d_ranges, n, h->d_sums, h->stream), "accumulator sums");
    HIP_TRY(hipMemcpyAsync(sums.data(), h->d_sums, sizeof(int64_t) * sums.size(), hipMemcpyDeviceToHost, h->stream),
            "copy accumulator sums");
    HIP_TRY(hipStreamSynchronize(h->stream), "synchronize");
    for (int i = 0; i < n; ++i) {
        const crbm_instance& I = h->inst[i];
        const int64_t* s = sums.data() + (size_t)i * CRBM_N_ACC;
        crbm_obs& o = out[i];
        std::memset(&o, 0, sizeof(o));
        o.n_samples = s[0];
        o.sum_M = s[1]; o.sum_B1 = s[2]; o.sum_B2 = s[3];
        o.sum_MM = s[4]; o.sum_B1B1 = s[5]; o.sum_B2B2 = s[6];
        o.sum_MB1 = s[7]; o.sum_MB2 = s[8]; o.sum_B1B2 = s[9];
        o.sum_absM = s[10];
        o.sum_Ms = s[11]; o.sum_MsMs = s[12]; o.sum_absMs = s[13];
        if (s[0] > 0) {
            const double N = (double)I.L * I.L, ns = (double)s[0];
            const double a = (double)h->Jq[0][i] / 65536.0, b = (double)h->Jq[1][i] / 65536.0,
                         c = (double)h->Jq[2][i] / 65536.0;
            const double mE = (a * s[2] + b * s[3] - c * s[1]) / ns;
            const double mE2 = (a * a * s[5] + b * b * s[6] + c * c * s[4] + 2 * a * b * s[9] - 2 * a * c * s[7] -
                                2 * b * c * s[8]) / ns;
            o.E_per_spin = mE / N;
            o.m = (double)s[1] / ns / N;
            o.abs_m = (double)s[10] / ns / N;
            o.dimer = -((double)s[3] / ns) / (N / 2.0);
            o.E_var_per_spin = (mE2 - mE * mE) / N;
            o.abs_stag_m = (double)s[13] / ns / N;
        }
    }
    if (corr_out && h->d_corr) {
        const int64_t tot = h->corr_off.back() + (int64_t)h->inst.back().L * h->inst.back().L;
        HIP_TRY(hipMemcpyAsync(corr_out, h->d_corr, sizeof(int64_t) * (size_t)tot, hipMemcpyDeviceToHost, h->stream),
                "copy correlation sums");
        HIP_TRY(hipStreamSynchronize(h->stream), "synchronize");
    } else if (corr_out) {
        int64_t tot = 0;
        for (int i = 0; i < n; ++i) tot += (int64_t)h->inst[i].L * h->inst[i].L;
        unsigned long long* d = nullptr;
        if (dev_alloc(&d, sizeof(unsigned long long) * (size_t)tot) != hipSuccess)
            return fail(CRBM_ENOMEM, "hipMalloc corr");
        int rc = CRBM_OK;
        int64_t off = 0;
        hipError_t e = hipMemsetAsync(d, 0, sizeof(unsigned long long) * (size_t)tot, h->stream);
        for (int i = 0; i < n && e == hipSuccess; ++i) {
            const crbm_instance& I = h->inst[i];
            e = launch_corr(h->d_state + h->state_off[i], I.n_chains, I.L, d + off, h->stream);
            off += (int64_t)I.L * I.L;
        }
        if (e == hipSuccess) e = hipMemcpyAsync(corr_out, d, sizeof(int64_t) * (size_t)tot, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) rc = fail(CRBM_EHIP, std::string("structure factor: ") + hipGetErrorString(e));
        (void)hipFree(d);
        if (rc != CRBM_OK) return rc;
    }
    return CRBM_OK;
}

int crbm_reset_observables(crbm_t* h) {
    g_err.clear();
    if (!h) return fail(CRBM_EINVAL, "handle is NULL");
    HIP_TRY(hipMemsetAsync(h->d_acc, 0, sizeof(int64_t) * CRBM_N_ACC * (size_t)h->total_chains, h->stream),
            "zero accumulators");
    if (h->d_corr)
        HIP_TRY(hipMemsetAsync(h->d_corr, 0,
                               sizeof(unsigned long long) *
                                   (size_t)(h->corr_off.back() + (int64_t)h->inst.back().L * h->inst.back().L),
                               h->stream),
                "zero correlation sums");
    return CRBM_OK;
}

int crbm_get_state(crbm_t* h, int8_t* spins_dev, int64_t* sweep_index) {
    g_err.clear();
    if (!h) return fail(CRBM_EINVAL, "handle is NULL");
    if (spins_dev) {
        for (size_t i = 0; i < h->inst.size(); ++i)
            HIP_TRY(launch_unpack(h->d_state + h->state_off[i], spins_dev + h->spin_off[i], h->inst[i].n_chains,
                                  h->inst[i].L, h->stream),
                    "unpack kernel");
        HIP_TRY(hipStreamSynchronize(h->stream), "synchronize");
    }
    if (sweep_index) *sweep_index = h->cur;
    return CRBM_OK;
}

int crbm_set_state(crbm_t* h, const int8_t* spins_dev, int64_t sweep_index) {
    g_err.clear();
    if (!h) return fail(CRBM_EINVAL, "handle is NULL");
    if (sweep_index < 0 || sweep_index > h->S) return fail(CRBM_EINVAL, "sweep_index out of the schedule");
    if (spins_dev)
        for (size_t i = 0; i < h->inst.size(); ++i)
            HIP_TRY(launch_pack(h->d_state + h->state_off[i], spins_dev + h->spin_off[i], h->inst[i].n_chains,
                                h->inst[i].L, h->stream),
                    "pack kernel");
    h->cur = sweep_index;
    return CRBM_OK;
}

int crbm_sweep_table(const crbm_t* h, int32_t i, int64_t s, uint32_t out[16]) {
    g_err.clear();
    if (!h || !out || i < 0 || i >= (int32_t)h->inst.size() || s < 0 || s >= h->S)
        return fail(CRBM_EINVAL, "bad arguments");
    const uint32_t* src = h->h_tables.data() + h->tab_off[i] + (size_t)h->tab_stride[i] * (size_t)s;
    std::memcpy(out, src, sizeof(uint32_t) * kTabWords);
    return CRBM_OK;
}

int crbm_table_for(double J1, double J2, double h, double T, uint32_t out[16]) {
    g_err.clear();
    const double lim = 2147483647.0 / 65536.0;
    if (!out || !(T > 0.0) || !std::isfinite(T) || !std::isfinite(J1) || !std::isfinite(J2) || !std::isfinite(h))
        return fail(CRBM_EINVAL, "bad arguments");
    if (fabs(J1) >= lim || fabs(J2) >= lim || fabs(h) >= lim) return fail(CRBM_ERANGE, "|J| * 2^16 must fit in int32");
    const int rc = build_table(q16(J1), q16(J2), q16(h), T, CRBM_PRECISION_Q16, out);
    if (rc != CRBM_OK) return fail(rc, "fixed-point weight or bias overflows int32");
    return CRBM_OK;
}

int crbm_table_for_precision(double J1, double J2, double h, double T, int32_t precision, uint32_t* out) {
    g_err.clear();
    const double lim = 2147483647.0 / 65536.0;
    if (!out || !(T > 0.0) || !std::isfinite(T) || !std::isfinite(J1) || !std::isfinite(J2) || !std::isfinite(h) ||
        (precision != CRBM_PRECISION_Q16 && precision != CRBM_PRECISION_FPGA))
        return fail(CRBM_EINVAL, "bad arguments");
    if (fabs(J1) >= lim || fabs(J2) >= lim || fabs(h) >= lim) return fail(CRBM_ERANGE, "|J| * 2^16 must fit in int32");
    const int rc = build_table(q16(J1), q16(J2), q16(h), T, precision, out);
    if (rc != CRBM_OK) return fail(rc, "fixed-point weight or bias overflows int32");
    return CRBM_OK;
}

void crbm_destroy(crbm_t* h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    delete h;
}

}  // extern "C"
