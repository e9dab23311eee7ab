// crbm_internal.h -- declarations shared by the library's own translation
// units (host API and device kernels).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "crbm.h"

namespace crbmlib {

// Words per sweep in the device table of one instance:
//   [0] T1   32-bit threshold t(2 wq1) for an agreeing J1 hidden unit
//   [1] T2   same for a dimer (J2) hidden unit
//   [2] flags: bit0 sig1 < 0, bit1 sig2 < 0, bit2 wq1 != 0, bit3 wq2 != 0,
//              bits 8..11 kge0, bits 12..15 kge1: a spin with n positive J1
//              terms and dimer term d (0/1) has field >= 0 iff n >= kge_d
//   [3 + 2n + d]  t(|x|) of that spin's field x, n = 0..4, d = 0..1
//   [13..15] zero
constexpr int kTabWords = 16;

struct Item {
    uint32_t inst;        // index of the instance in the create() list
    uint32_t id;          // instance id used in the random-number counter
    uint32_t chain0;      // first chain of this item, within the instance
    uint32_t nchains;     // chains in this item (at most 64 / lanes-per-chain)
    uint64_t gbase;       // global chain index of chain0 (instances concatenated)
    uint64_t state_off;   // word offset of chain0's first row in the state buffer ([chain][L][W])
    uint64_t spin_off;    // byte offset of chain0's spins in a [chain][L][L] int8 buffer
    uint64_t tab_off;     // word offset of the instance's first table
    uint32_t tab_stride;  // kTabWords for per-sweep tables, 0 for a constant schedule
    uint32_t L;
};

struct GibbsArgs {
    uint32_t* state;          // bit rows, ceil(L/32) words per row, chains at Item::state_off
    const uint32_t* tables;   // per-instance tables, see above
    const Item* items;        // one item per wavefront
    int32_t n_items;
    int32_t measure_every;    // 0 = no accumulation
    int64_t s0, s1;           // sweeps [s0, s1) of the schedule
    int64_t burn_in;
    uint64_t seed;
    int64_t* acc;             // [global chain][CRBM_N_ACC] int64 accumulators
    int32_t* trace;           // [(s1 - trace_s0) / trace_every][total_chains][3] or nullptr
    int32_t trace_every;      // record after every trace_every-th sweep of the call
    int64_t trace_s0;         // first sweep of the crbm_sample call (a call may take several launches)
    int32_t* order;           // plateau structure factor trace, same layout as trace, or nullptr
    int64_t total_chains;
    int8_t* spins_out;        // int8 spins at Item::spin_off, or nullptr
    uint32_t* queue;          // persistent mode: work counter (zeroed before launch); nullptr = direct
    int32_t waves_per_block;  // 1..4 (0 = 4)
    int32_t grid_blocks;      // persistent mode: blocks in the grid
    uint32_t tail_cap;        // lanes per round of the hidden comparison's compacted tail (1..64)
};

// What the learned-proposal code needs from a Gibbs handle.
struct HandleView {
    uint32_t* state;   // bit rows of the instance
    int L;
    int64_t n_chains;
    uint32_t id;
    uint64_t seed;
    int n_inst;
    int sched_kind;
    double T0;
    int64_t cur, S;
    hipStream_t stream;
    // MH target: log pi = a M + c1 n1 + c2 n2 (+ const) at the constant temperature
    double a, c1, c2;
    int sg1, sg2;
    int precision;     // CRBM_PRECISION_* of the handle's tables
};
// the view of instance i (0 <= i < number of instances)
int handle_view(crbm_t* h, HandleView* v, int i);

// The host mapping of the conventions (crbm_api.cpp), shared with the
// general-lattice sampler: schedule temperature of sweep s, hidden weight and
// coupling sign of a quantised coupling at T, and the 32-bit sigmoid threshold
// of a field magnitude y (2^-16 units).
double map_schedule_T(int kind, double T0, double T1, const double* Te, int64_t S, int64_t s);
void map_hidden_weight(int64_t Jq, double T, int64_t* wq, int* sig);
uint32_t map_threshold(int64_t y);

// Lanes per round of the compacted tail of the hidden comparison (64; fewer
// only when crbm_debug_tail_cap has set them, to exercise the multi-round path).
uint32_t tail_cap();

// Every device allocation of the library goes through dev_alloc, which fails
// with hipErrorOutOfMemory when crbm_debug_fail_alloc has armed it (tests of
// the error paths), and otherwise calls hipMalloc.
hipError_t dev_alloc_bytes(void** p, size_t bytes);
template <class T>
inline hipError_t dev_alloc(T** p, size_t bytes) {
    return dev_alloc_bytes(reinterpret_cast<void**>(p), bytes);
}

// Records the message returned by crbm_last_error() on this thread; returns code.
int set_error(int code, const char* msg);

// Lanes per chain for a lattice side and a number of cell rows per lane.
inline int lanes_per_chain(int L, int R) { return (L / 2) / R; }
inline int chains_per_wave(int L, int R) { return 64 / lanes_per_chain(L, R); }

// Returns false if no kernel was compiled for (L, R).
bool gibbs_supported(int L, int R);
hipError_t launch_gibbs(int L, int R, const GibbsArgs& a, hipStream_t st);
const void* gibbs_kernel_fn(int L, int R);   // for explicit graph kernel nodes
hipError_t launch_zero_u32(uint32_t* p, int n, hipStream_t st);
const void* zero_u32_fn();
hipError_t launch_init(uint32_t* state, const Item* items, int n_items, int L, int R,
                       uint64_t seed, hipStream_t st);
// state: first row of the instance's first chain; spins: its first spin.
hipError_t launch_pack(uint32_t* state, const int8_t* spins, int64_t nchains, int L, hipStream_t st);
hipError_t launch_unpack(const uint32_t* state, int8_t* spins, int64_t nchains, int L, hipStream_t st);
hipError_t launch_corr(const uint32_t* state, int64_t nchains, int L, unsigned long long* corr,
                       hipStream_t st);

}  // namespace crbmlib
