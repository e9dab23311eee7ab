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
#include <cstring>
#include <string>
#include <vector>

#include "crbm.h"
#include "crbm_internal.h"

using namespace crbmlib;

namespace {

thread_local std::string g_err;

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

// One sweep's 16-word device table (layout in crbm_internal.h).
int build_table(int64_t J1q, int64_t J2q, int64_t hq, double T, uint32_t* out) {
    int64_t wq1, wq2;
    int s1, s2;
    hidden_weight(J1q, T, &wq1, &s1);
    hidden_weight(J2q, T, &wq2, &s2);
    const int64_t aq = llround((double)hq / T);
    const int64_t lim = (int64_t)1 << 31;
    if (wq1 >= lim || wq2 >= lim || aq >= lim || aq <= -lim) return CRBM_ERANGE;
    std::memset(out, 0, sizeof(uint32_t) * kTabWords);
    out[0] = threshold(2 * wq1);
    out[1] = threshold(2 * wq2);
    uint32_t kge[2] = {5u, 5u};
    for (int d = 0; d < 2; ++d)
        for (int n = 4; n >= 0; --n) {
            const int64_t x = aq + wq1 * (2 * n - 4) + wq2 * (2 * d - 1);
            out[3 + 2 * n + d] = threshold(x < 0 ? -x : x);
            if (x >= 0) kge[d] = (uint32_t)n;
        }
    out[2] = (s1 < 0 ? 1u : 0u) | (s2 < 0 ? 2u : 0u) | (wq1 != 0 ? 4u : 0u) | (wq2 != 0 ? 8u : 0u) |
             (kge[0] << 8) | (kge[1] << 12);
    return CRBM_OK;
}

int default_rows(int L) {
    const int C = L / 2;
    for (int R = 3; R >= 1; --R)
        if (C % R == 0 && gibbs_supported(L, R)) return R;
    return 1;
}

struct Group {
    int L = 0, R = 0;
    std::vector<Item> items;
    Item* d_items = nullptr;
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
    int64_t total_chains = 0, total_rows = 0, total_spins = 0;
    int64_t S = 0, cur = 0;
    uint32_t* d_state = nullptr;
    uint32_t* d_tables = nullptr;
    int64_t* d_acc = nullptr;
    std::vector<Group> groups;
    ~crbm_s() {
        if (d_state) (void)hipFree(d_state);
        if (d_tables) (void)hipFree(d_tables);
        if (d_acc) (void)hipFree(d_acc);
        for (auto& g : groups)
            if (g.d_items) (void)hipFree(g.d_items);
    }
};

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
    const double lim = 2147483647.0 / 65536.0;
    for (int i = 0; i < n_inst; ++i) {
        const crbm_instance& I = inst[i];
        const std::string tag = "instance " + std::to_string(i) + ": ";
        if (I.L < 4 || (I.L & 1)) return fail(CRBM_EINVAL, tag + "L must be even and >= 4");
        if (I.L > CRBM_MAX_L) return fail(CRBM_EUNSUPPORTED, tag + "L > CRBM_MAX_L");
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
            const int rc = build_table(h->Jq[0][i], h->Jq[1][i], h->Jq[2][i], T,
                                       h->h_tables.data() + h->tab_off[i] + (size_t)s * kTabWords);
            if (rc != CRBM_OK) {
                delete h;
                return fail(rc, "instance " + std::to_string(i) + ": fixed-point weight or bias overflows int32 at sweep " +
                                    std::to_string(s));
            }
        }
        h->gbase[i] = h->total_chains;
        h->state_off[i] = h->total_rows;
        h->spin_off[i] = h->total_spins;
        h->total_chains += I.n_chains;
        h->total_rows += (int64_t)I.n_chains * I.L;
        h->total_spins += (int64_t)I.n_chains * I.L * I.L;
    }

    // work items, grouped by (L, R)
    for (int i = 0; i < n_inst; ++i) {
        const crbm_instance& I = h->inst[i];
        const int R = cfg->tile_rows ? cfg->tile_rows : default_rows(I.L);
        Group* grp = nullptr;
        for (auto& g : h->groups)
            if (g.L == I.L && g.R == R) grp = &g;
        if (!grp) {
            h->groups.push_back(Group{});
            grp = &h->groups.back();
            grp->L = I.L;
            grp->R = R;
        }
        const int cpw = chains_per_wave(I.L, R);
        for (int c0 = 0; c0 < I.n_chains; c0 += cpw) {
            Item it{};
            it.inst = (uint32_t)i;
            it.id = I.id;
            it.chain0 = (uint32_t)c0;
            it.nchains = (uint32_t)std::min(cpw, I.n_chains - c0);
            it.gbase = (uint64_t)(h->gbase[i] + c0);
            it.state_off = (uint64_t)(h->state_off[i] + (int64_t)c0 * I.L);
            it.spin_off = (uint64_t)(h->spin_off[i] + (int64_t)c0 * I.L * I.L);
            it.tab_off = h->tab_off[i];
            it.tab_stride = h->tab_stride[i];
            it.L = (uint32_t)I.L;
            grp->items.push_back(it);
        }
    }

    // device state
    hipError_t e;
    if ((e = hipMalloc(&h->d_state, sizeof(uint32_t) * (size_t)h->total_rows)) != hipSuccess ||
        (e = hipMalloc(&h->d_tables, sizeof(uint32_t) * h->h_tables.size())) != hipSuccess ||
        (e = hipMalloc(&h->d_acc, sizeof(int64_t) * CRBM_N_ACC * (size_t)h->total_chains)) != hipSuccess) {
        delete h;
        return fail(e == hipErrorOutOfMemory ? CRBM_ENOMEM : CRBM_EHIP, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    for (auto& g : h->groups) {
        if ((e = hipMalloc(&g.d_items, sizeof(Item) * g.items.size())) != hipSuccess) {
            delete h;
            return fail(CRBM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
    }
    int rc = CRBM_OK;
    auto chk = [&](hipError_t x, const char* what) {
        if (x != hipSuccess && rc == CRBM_OK) rc = fail(CRBM_EHIP, std::string(what) + ": " + hipGetErrorString(x));
    };
    chk(hipMemcpyAsync(h->d_tables, h->h_tables.data(), sizeof(uint32_t) * h->h_tables.size(), hipMemcpyHostToDevice,
                       h->stream), "copy tables");
    chk(hipMemsetAsync(h->d_acc, 0, sizeof(int64_t) * CRBM_N_ACC * (size_t)h->total_chains, h->stream), "zero acc");
    for (auto& g : h->groups) {
        chk(hipMemcpyAsync(g.d_items, g.items.data(), sizeof(Item) * g.items.size(), hipMemcpyHostToDevice, h->stream),
            "copy items");
        chk(launch_init(h->d_state, g.d_items, (int)g.items.size(), g.L, g.R, cfg->seed, h->stream), "init kernel");
    }
    // the host vectors must outlive the async copies
    chk(hipStreamSynchronize(h->stream), "synchronize");
    if (rc != CRBM_OK) {
        delete h;
        return rc;
    }
    *out = h;
    return CRBM_OK;
}

int crbm_sample(crbm_t* h, int64_t n_sweeps, int8_t* spins_out, int32_t* counts_trace) {
    g_err.clear();
    if (!h) return fail(CRBM_EINVAL, "handle is NULL");
    if (n_sweeps < 0) return fail(CRBM_EINVAL, "n_sweeps must be >= 0");
    if (h->cur + n_sweeps > h->S) return fail(CRBM_ESTATE, "sampling past the end of the schedule");
    for (auto& g : h->groups) {
        GibbsArgs a{};
        a.state = h->d_state;
        a.tables = h->d_tables;
        a.items = g.d_items;
        a.n_items = (int32_t)g.items.size();
        a.measure_every = h->cfg.measure_every;
        a.s0 = h->cur;
        a.s1 = h->cur + n_sweeps;
        a.burn_in = h->cfg.burn_in;
        a.seed = h->cfg.seed;
        a.acc = h->d_acc;
        a.trace = counts_trace;
        a.total_chains = h->total_chains;
        a.spins_out = spins_out;
        HIP_TRY(launch_gibbs(g.L, g.R, a, h->stream), "gibbs kernel");
    }
    h->cur += n_sweeps;
    return CRBM_OK;
}

int crbm_observables(crbm_t* h, crbm_obs* out, int64_t* corr_out) {
    g_err.clear();
    if (!h || !out) return fail(CRBM_EINVAL, "NULL argument");
    const int n = (int)h->inst.size();
    std::vector<int64_t> acc((size_t)CRBM_N_ACC * h->total_chains);
    HIP_TRY(hipMemcpyAsync(acc.data(), h->d_acc, sizeof(int64_t) * acc.size(), hipMemcpyDeviceToHost, h->stream),
            "copy accumulators");
    HIP_TRY(hipStreamSynchronize(h->stream), "synchronize");
    for (int i = 0; i < n; ++i) {
        const crbm_instance& I = h->inst[i];
        int64_t s[CRBM_N_ACC] = {0};
        for (int64_t c = 0; c < I.n_chains; ++c)
            for (int x = 0; x < CRBM_N_ACC; ++x) s[x] += acc[(size_t)(h->gbase[i] + c) * CRBM_N_ACC + x];
        crbm_obs& o = out[i];
        std::memset(&o, 0, sizeof(o));
        o.n_samples = s[0];
        o.sum_M = s[1]; o.sum_B1 = s[2]; o.sum_B2 = s[3];
        o.sum_MM = s[4]; o.sum_B1B1 = s[5]; o.sum_B2B2 = s[6];
        o.sum_MB1 = s[7]; o.sum_MB2 = s[8]; o.sum_B1B2 = s[9];
        o.sum_absM = s[10];
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
        }
    }
    if (corr_out) {
        int64_t tot = 0;
        for (int i = 0; i < n; ++i) tot += (int64_t)h->inst[i].L * h->inst[i].L;
        unsigned long long* d = nullptr;
        HIP_TRY(hipMalloc(&d, sizeof(unsigned long long) * (size_t)tot), "hipMalloc corr");
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
    const int rc = build_table(q16(J1), q16(J2), q16(h), T, out);
    if (rc != CRBM_OK) return fail(rc, "fixed-point weight or bias overflows int32");
    return CRBM_OK;
}

void crbm_destroy(crbm_t* h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    delete h;
}

}  // extern "C"
