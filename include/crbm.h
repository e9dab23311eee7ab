/*
 * crbm.h -- C ABI of the MI355X (gfx950) CRBM Gibbs sampler for the classical
 * Shastry-Sutherland (SS) Ising lattice.
 *
 * The operation (Brahma et al., arXiv 2511.20911):
 *   - the lattice Hamiltonian of Sec. I Eq. (1), read with the field
 *     favouring up spins:  H = J1 sum_sq s s + J2 sum_dimer s s - h sum s;
 *   - its exact CRBM encoding, Sec. II.A Eqs. (4)-(10): one hidden unit per
 *     bond, 10 filters on the 3x3 unit-cell window, stride 2;
 *   - block Gibbs sampling, Sec. II.B Eqs. (11)-(12): all hidden units from
 *     the spins, then all spins from the hidden units (zero-inserted hidden
 *     planes, flipped filters, accumulated over the 10 filters plus the
 *     visible bias, App. A Zero Padder / Convoluter-Reverse / Accumulator);
 *   - the sigmoid as a table of closest values compared against a uniform
 *     random number (App. A Sigmoid and LFSR), here 32-bit thresholds and
 *     counter-based Philox4x32-10 uniforms;
 *   - host-side energies of the sampled states (App. A I/O Programming Logic)
 *     and the static structure factor of Sec. III.B Eq. (13).
 *
 * Every unit update is an integer compare; couplings, weights and the visible
 * bias are 16.16 fixed point; all counts are exact integers.  The random
 * stream of a unit depends only on (seed, instance id, chain, sweep, unit), so
 * results do not depend on tiling, launch shape or batch composition.
 *
 * Errors: every function returns CRBM_OK (0) or a negative code and never
 * throws; crbm_last_error() returns a message for the calling thread.
 * Threading: a handle may be used from one thread at a time.
 * Streams: work is enqueued on the hipStream_t given in crbm_config.stream
 * (NULL = the default stream).  Functions that return host data synchronise
 * that stream first.
 */
#ifndef CRBM_H
#define CRBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CRBM_OK = 0,
    CRBM_EINVAL = -1,      /* invalid argument (odd L, T <= 0, NULL pointer, ...) */
    CRBM_ERANGE = -2,      /* a fixed-point weight or bias does not fit in int32 */
    CRBM_ENOMEM = -3,      /* device or host allocation failed */
    CRBM_EHIP = -4,        /* a HIP runtime call failed */
    CRBM_EUNSUPPORTED = -5,/* valid request this library does not implement (open boundaries, an L without a compiled kernel) */
    CRBM_ESTATE = -6       /* misuse of a handle (e.g. sampling past the end of the schedule) */
};

enum {
    CRBM_SCHED_CONST = 0,     /* T_s = T0 */
    CRBM_SCHED_LINEAR = 1,    /* T_s = T0 + (T1 - T0) * (s / (S - 1)) */
    CRBM_SCHED_GEOMETRIC = 2, /* T_s = T0 * pow(T1 / T0, s / (S - 1)) */
    CRBM_SCHED_EXPLICIT = 3   /* T_s = T_explicit[s] */
};

#define CRBM_MAX_L 96      /* largest lattice side supported by this library */
#define CRBM_N_ACC 14      /* per-chain accumulator words, see crbm_obs */

/* One Hamiltonian point (one "instance").  Host memory, copied at create. */
typedef struct {
    int32_t L;                 /* lattice side: even, 4 <= L <= 32, or 36, 40, 48, 64, 72, 96 */
    int32_t periodic;          /* must be 1 (periodic in both directions); open axes: crbm_lattice_create */
    double J1, J2, h;          /* couplings and field; |J| * 2^16 < 2^31 */
    int32_t n_chains;          /* independent chains, >= 1 */
    int32_t sched_kind;        /* CRBM_SCHED_* */
    double T0, T1;             /* temperatures, finite and > 0 */
    const double* T_explicit;  /* host array of n_sweeps temperatures (EXPLICIT only) */
    uint32_t id;               /* instance id in the random-number counter, < 2^29 */
} crbm_instance;

typedef struct {
    uint64_t seed;             /* Philox key */
    int64_t n_sweeps;          /* schedule length S; crbm_sample may run at most S sweeps in total */
    int32_t measure_every;     /* 0 = accumulate nothing; k > 0 = accumulate every k-th sweep at or after burn_in */
    int64_t burn_in;           /* first sweep that may be accumulated */
    void* stream;              /* hipStream_t (NULL = default stream) */
    int32_t tile_rows;         /* cell rows per lane: 0 = tuned/default choice, else must divide L/2 */
    int32_t launch_mode;       /* CRBM_LAUNCH_DIRECT or CRBM_LAUNCH_GRAPH */
    int32_t waves_per_block;   /* 1..4 wavefronts per workgroup; 0 = tuned/default choice */
    int32_t precision;         /* CRBM_PRECISION_* (0 = the default 16.16 / 32-bit path) */
    uint32_t flags;            /* CRBM_F_* */
} crbm_config;

/* crbm_config.flags.  CRBM_F_CORR: accumulate the spin-spin correlation
 * C(dr, dc) = sum_{r,c} s(r,c) s(r+dr, c+dc) of every chain after every
 * measured sweep (the sweeps crbm_obs accumulates), exactly in int64, for the
 * static structure factor S(q) of Sec. III.B Eq. (13); crbm_observables
 * returns the sums.  A measured sweep then ends a kernel launch, so sampling
 * runs one launch per measured sweep (direct launches, also for
 * CRBM_LAUNCH_GRAPH handles). */
#define CRBM_F_CORR 1u

/* Arithmetic of the per-sweep weights, fields and sigmoid thresholds.
 * CRBM_PRECISION_Q16: 16.16 weights and bias, 32-bit thresholds and uniforms.
 * CRBM_PRECISION_FPGA: the paper's hardware precision (App. A Dimension and
 *   Precision; Sigmoid and LFSR-Forward), for studying its effect on sampling:
 *   weights w and visible bias a = h/T rounded to signed Q5.4 (steps of 1/16,
 *   |.| <= 511/16, saturating); the hidden convolution output (0 or +-2w) in
 *   the same 10 bits and the visible accumulator (bias plus the 5 incident
 *   +-w) in 12 bits (|.| <= 2047/16), both saturating; the sigmoid as the
 *   closest 16-bit value, min(65535, round(65536 sigmoid(2|x|))), compared
 *   with a 16-bit uniform (the top half of the unit's 32-bit Philox uniform).
 *   Handles in this mode are refused by crbm_sample_mh: their stationary law
 *   is not the exact CRBM marginal the acceptance uses. */
enum { CRBM_PRECISION_Q16 = 0, CRBM_PRECISION_FPGA = 1 };

enum {
    CRBM_LAUNCH_DIRECT = 0, /* one grid launch per lattice size, one wavefront per work item */
    CRBM_LAUNCH_GRAPH = 1   /* one hipGraph launch: a queue-reset node, then one persistent kernel per
                               lattice size on parallel branches, each draining a work queue */
};

/* Per-instance observables, host memory, filled by crbm_observables.
 * Sums run over chains and accumulated sweeps.  Counts of one state:
 *   M  = sum of spins,  B1 = sum over J1 bonds of s_a s_b,  B2 = same over dimers.
 * Energy per spin E/N = (J1q B1 + J2q B2 - hq M) / (2^16 N) with Jq = llround(J 2^16). */
typedef struct {
    int64_t n_samples;                        /* chains x accumulated sweeps */
    int64_t sum_M, sum_B1, sum_B2;
    int64_t sum_MM, sum_B1B1, sum_B2B2, sum_MB1, sum_MB2, sum_B1B2;
    int64_t sum_absM;
    int64_t sum_Ms, sum_MsMs, sum_absMs;      /* staggered magnetisation Ms = sum (-1)^(r+c) s(r,c) */
    double E_per_spin;                        /* <E>/N from the exact sums */
    double m;                                 /* <M>/N */
    double abs_m;                             /* <|M|>/N */
    double dimer;                             /* -<B2>/(N/2): +1 for antiparallel dimers */
    double E_var_per_spin;                    /* (<E^2> - <E>^2)/N from the exact second moments */
    double abs_stag_m;                        /* <|Ms|>/N: 1 in a Neel state (Sec. III.A AFM phase) */
} crbm_obs;

typedef struct crbm_s crbm_t;

/* Create a sampler for n_inst instances (each with its own L, couplings,
 * schedule and chain count) sharing one config.  Quantises the couplings,
 * builds the per-sweep weight and threshold tables on the host, allocates the
 * device state (bit-packed spins, tables, accumulators) and enqueues the
 * seeded initialisation of every chain on cfg->stream.
 * Returns CRBM_EINVAL for invalid parameters, CRBM_ERANGE for fixed-point
 * overflow, CRBM_EUNSUPPORTED for open boundaries or L > CRBM_MAX_L. */
int crbm_create(const crbm_instance* inst, int32_t n_inst, const crbm_config* cfg, crbm_t** out);

/* Run the next n_sweeps sweeps of the schedule (asynchronous on the stream).
 * spins_out: device pointer or NULL; if given, receives the final state as
 *   int8 +-1 values, layout [chain][L][L] with chains of all instances
 *   concatenated in instance order (sizes may differ per instance).
 * counts_trace: device pointer or NULL; if given, receives int32 (M, B1, B2)
 *   after every sweep of this call, layout [sweep][chain][3] with the chains
 *   of all instances concatenated.
 * Returns CRBM_ESTATE if the schedule would be exceeded. */
int crbm_sample(crbm_t* h, int64_t n_sweeps, int8_t* spins_out, int32_t* counts_trace);

/* As crbm_sample, with the counts trace thinned: (M, B1, B2) is recorded
 * after every trace_every-th sweep of this call only, layout
 * [n_sweeps / trace_every][chain][3] (for autocorrelation estimates over long
 * runs).  order_trace (device, may be NULL; needs counts_trace): at the same
 * sweeps, the 1/3-plateau structure factor of Sec. III.B Eq. (13) as exact
 * integers (max, |S_A|^2, |S_B|^2) with S_A = sum s(r,c) e^{i(pi r + 2 pi c/3)}
 * and S_B = sum s(r,c) e^{i(2 pi r/3 + pi c)}, same layout; O_1/3 = max / N^2.
 * trace_every must be >= 1 and divide n_sweeps, else CRBM_EINVAL.
 * crbm_sample is the case trace_every = 1, no order trace. */
int crbm_sample_thinned(crbm_t* h, int64_t n_sweeps, int8_t* spins_out, int32_t* counts_trace,
                        int32_t* order_trace, int32_t trace_every);

/* Synchronise the stream and fill out[n_inst] from the exact int64
 * accumulators.  corr_out: host pointer or NULL; if given, receives for each
 * instance, int64 [L][L] per instance, instances concatenated, the sum of
 * C(dr,dc) = sum_{r,c} s(r,c) s(r+dr,c+dc):
 *   - handles created with CRBM_F_CORR: over its chains and all measured
 *     sweeps since creation or the last crbm_reset_observables (the same
 *     samples as out[i].n_samples, so C/n_samples is the sample average);
 *   - other handles: over its chains in the current state only.
 * S(q) of Eq. (13) is the 2-D Fourier transform of the average. */
int crbm_observables(crbm_t* h, crbm_obs* out, int64_t* corr_out);

/* Checkpoint / resume.  spins: device pointer, int8 +-1, same layout as
 * crbm_sample's spins_out.  sweep_index: global index of the next sweep. */
int crbm_get_state(crbm_t* h, int8_t* spins_dev, int64_t* sweep_index);
int crbm_set_state(crbm_t* h, const int8_t* spins_dev, int64_t sweep_index);

/* Total number of chains over all instances. */
int64_t crbm_total_chains(const crbm_t* h);

/* Zero the accumulators (e.g. after a burn-in phase). */
int crbm_reset_observables(crbm_t* h);

/* Autotuner (batched launches): time every compiled tiling of lattice side L
 * (cell rows per lane x wavefronts per workgroup) on the current device with
 * n_chains chains for n_sweeps sweeps, keep the fastest as the process-wide
 * choice for L and return it.  Enqueues work on `stream` and synchronises it.
 * best_rate: visible spin-updates/s of the winner (may be NULL). */
int crbm_autotune(int32_t L, int32_t n_chains, int32_t n_sweeps, void* stream, int32_t* best_rows,
                  int32_t* best_waves_per_block, double* best_rate);

/* Process-wide tiling choice for lattice side L (used by crbm_create when the
 * config leaves tile_rows / waves_per_block at 0).  set: rows must divide L/2
 * and have a compiled kernel; waves_per_block in 1..4. */
int crbm_set_tiling(int32_t L, int32_t rows, int32_t waves_per_block);
int crbm_get_tiling(int32_t L, int32_t* rows, int32_t* waves_per_block);

/* Integrated autocorrelation time and effective sample size of the
 * observable O = w[0] M + w[1] B1 + w[2] B2 (e.g. the energy with
 * w = (-hq, J1q, J2q)) over a counts trace written by crbm_sample
 * (trace_dev: device, int32 [n_samples][trace_chains][3]), for chains
 * [c0, c1), after dropping the first `discard` samples.  With the grand mean
 * over all kept samples removed (chains stuck at different levels then count
 * as correlated, not as independent), Gamma(k) = sum over chains and t of
 * x_t x_{t+k} / ((n - k) n_chains), rho(k) = Gamma(k)/Gamma(0),
 * tau_int = 1 + 2 sum_{k=1}^{W} rho(k) with the automatic window
 * W = min{W : W >= c_window tau_int(W)} (Sokal), else the largest lag, and
 * ESS = n_chains (n_samples - discard) / tau_int.  rho_out (host, may be NULL)
 * receives rho(0..min(max_lag, n-discard-1)).  Synchronises `stream`. */
int crbm_tau_int(const int32_t* trace_dev, int64_t n_samples, int64_t trace_chains, int64_t c0, int64_t c1,
                 int64_t discard, const double w[3], int32_t max_lag, double c_window, void* stream,
                 double* tau_out, double* ess_out, int32_t* window_out, double* rho_out);

/* crbm_tau_int without device allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, arithmetic and results as
 * crbm_tau_int (bit for bit).  Its scratch (chain means, the centred series,
 * per-block and per-lag sums) is one file-scope device array of
 * CRBM_TAU_NOALLOC_MAX_DOUBLES doubles (64 MiB) per device, held until the
 * process ends; a request needs (c1 - c0) (n_samples - discard + 1) + 1 +
 * (K + 1) (ceil((c1 - c0) / 256) + 1) doubles with K = min(max_lag,
 * n_samples - discard - 1), and K <= CRBM_TAU_NOALLOC_MAX_LAG; larger
 * requests return CRBM_ERANGE before any work is enqueued.  Every scratch
 * word the call reads it has written first, so nothing needs clearing.  All
 * calls on one device share that device's array: calls that overlap in time
 * on one device (several streams or host threads) race and must be
 * serialised by the caller.  Synchronises `stream`. */
#define CRBM_TAU_NOALLOC_MAX_DOUBLES (8 * 1024 * 1024)
#define CRBM_TAU_NOALLOC_MAX_LAG 4096
int crbm_tau_int_noalloc(const int32_t* trace_dev, int64_t n_samples, int64_t trace_chains, int64_t c0, int64_t c1,
                         int64_t discard, const double w[3], int32_t max_lag, double c_window, void* stream,
                         double* tau_out, double* ess_out, int32_t* window_out, double* rho_out);

/* Ground-state search behind the time-to-solution of Sec. III.C Eq. (14)
 * (the host picks the lowest-energy states it has sampled, App. A I/O
 * Programming Logic): fold a counts trace written by crbm_sample /
 * crbm_sample_thinned (trace_dev: device, int32 [n_samples][trace_chains][3])
 * into per-chain running minima of E = w[0] M + w[1] B1 + w[2] B2, exact in
 * int64 (with w = (-hq, J1q, J2q), E is H in 2^-16 units).  For chain c0 + i,
 * i < c1 - c0: emin_dev[i] (device int64) is the lowest E seen and
 * first_dev[i] (device int64) the number of completed sweeps of the chain when
 * that value was first reached, sample t of the trace counting as sweep0 +
 * (t + 1) * trace_every (sweep0 = the handle's sweep index before the
 * crbm_sample call that wrote the trace).  Only a strictly lower energy
 * replaces a minimum, so folding consecutive traces of one run gives the
 * first hit over the whole run.  reset != 0 starts from emin = INT64_MAX,
 * first = -1 instead of the arrays' contents.  n_samples = 0 with reset = 0 is
 * a no-op.  Asynchronous on `stream`.  CRBM_EINVAL for NULL outputs, an empty
 * or out-of-range chain range, trace_every < 1, sweep0 < 0 or |w[k]| >= 2^31. */
int crbm_min_energy(const int32_t* trace_dev, int64_t n_samples, int64_t trace_chains, int64_t c0, int64_t c1,
                    const int64_t w[3], int64_t sweep0, int32_t trace_every, int32_t reset, int64_t* emin_dev,
                    int64_t* first_dev, void* stream);

/* ---------------------------------------------------------------------------
 * Learned proposal (an addition to the paper's Gibbs sampler): a masked-
 * convolution autoregressive network q(s) over the spins in raster order
 * (12 layers of 3x3 masked convolutions, 32 channels, bf16 weights and
 * activations on the matrix cores, fp32 accumulation), used as an independent
 * Metropolis-Hastings proposal.  Acceptance uses the exact integer counts of
 * the current and proposed states under the CRBM marginal the Gibbs chain
 * samples, log pi = a M + c1 n1 + c2 n2 + const (c_t = log cosh(2 w_t), n_t =
 * number of type-t bonds whose hidden unit "agrees", Sec. II.A Eq. (4) with the
 * hidden units summed out), so interleaving keeps the stationary law.
 *
 * Parameter layout (fp32, host arrays of crbm_ar_num_params() values): for
 * layers l = 0..11: weights [taps][cin][cout] then bias [cout], with 4 taps
 * (mask A: offsets (-1,-1) (-1,0) (-1,1) (0,-1)) for l = 0 and 5 taps (plus
 * (0,0)) otherwise; cin = 1 for l = 0 else 32; cout = 1 for l = 11 else 32.
 * All device pointers are caller-owned.  Calls are asynchronous on the
 * network's stream unless they return host data.
 * ------------------------------------------------------------------------- */
typedef struct crbm_ar_s crbm_ar_t;
typedef struct {
    int32_t L;          /* lattice side */
    int32_t channels;   /* must be 32 */
    int32_t layers;     /* must be 12 */
    uint64_t seed;      /* random stream of the sequential scorer (unused by training) */
    void* stream;       /* hipStream_t */
    int32_t cond_points;/* 0: unconditional; 1..128: conditional network for up to this many points */
} crbm_ar_config;

/* Conditional network (an addition for the multi-point workloads): each point
 * p has a feature vector x_p of 3 doubles chosen by the caller (for example
 * J2/J1, h/J1 and ln T of a Hamiltonian point); every layer's biases are
 * shifted by g(x_p) = W2^T tanh(W1^T x_p + b1) (32 hidden units), so one
 * network serves all points.  The MLP parameters follow the network's in the
 * parameter layout: W1 [3][32], b1 [32], W2 [32][12][32] (layer, channel; only
 * channel 0 of the logit layer is used).  crbm_ar_init_params draws W1 from
 * N(0, 1/3) and zeroes b1 and W2.  A conditional network needs its points
 * (crbm_ar_set_points) before it trains, scores or samples (else
 * CRBM_ESTATE).  The *_cond calls take a device int32 array `points_dev` with
 * one point index per configuration (values are clamped to [0, n_points));
 * NULL means point 0 for every configuration.  On an unconditional network
 * points_dev is ignored and the plain calls below are the *_cond calls with
 * NULL. */

int crbm_ar_create(const crbm_ar_config* c, crbm_ar_t** out);   /* parameters start at zero */
int64_t crbm_ar_num_params(const crbm_ar_t* a);
int crbm_ar_set_params(crbm_ar_t* a, const float* host, int64_t n); /* also resets the Adam state */
int crbm_ar_get_params(crbm_ar_t* a, float* host, int64_t n);
/* Seeded initial parameters: every weight N(0, sd^2) with sd = scale *
 * sqrt(2 / fan-in) (fan-in = taps x input channels), times 0.1 in the logit
 * layer, drawn by SplitMix64 + Box-Muller from `seed`; biases zero.  Resets
 * the Adam state.  Synchronises.  CRBM_EINVAL for scale < 0. */
int crbm_ar_init_params(crbm_ar_t* a, uint64_t seed, double scale);
/* Set the feature vectors of the points (host, [n_points][3]; copied).
 * CRBM_EINVAL if the network is unconditional, n_points is not in
 * 1..cond_points or a feature is not finite.  Synchronises. */
int crbm_ar_set_points(crbm_ar_t* a, int32_t n_points, const double* feats_host);
int crbm_ar_grad_cond(crbm_ar_t* a, const int8_t* samples_dev, const int32_t* points_dev, int64_t batch,
                      float* grad_host, double* loss_out);
int crbm_ar_train_step_cond(crbm_ar_t* a, const int8_t* samples_dev, const int32_t* points_dev, int64_t batch,
                            float lr, double* loss_out);
int crbm_ar_logq_cond(crbm_ar_t* a, const int8_t* spins_dev, const int32_t* points_dev, int64_t n, double* logq_dev);
int crbm_ar_sample_cond(crbm_ar_t* a, int64_t n, uint64_t seed, int64_t step, uint32_t id, const int32_t* points_dev,
                        int8_t* spins_dev, double* logq_dev);
/* Gradient of the mean negative log-likelihood over a batch of samples
 * (device int8 +-1 [batch][L][L]); grad_host (may be NULL) receives it in the
 * parameter layout, loss_out (may be NULL) the loss.  Synchronises.
 * Training and scoring batches hold fewer than 2^31 pixels (batch x L^2: the
 * convolution kernels index pixels in 32 bits); larger ones get CRBM_EINVAL. */
int crbm_ar_grad(crbm_ar_t* a, const int8_t* samples_dev, int64_t batch, float* grad_host, double* loss_out);
/* One Adam step (beta = 0.9, 0.999, eps = 1e-8) at learning rate lr on a batch. */
int crbm_ar_train_step(crbm_ar_t* a, const int8_t* samples_dev, int64_t batch, float lr, double* loss_out);
/* A whole training run in the library (Sec. II.B's sampler supplies the
 * data; the training itself is an addition): `steps` Adam steps, each on a
 * minibatch drawn on the device from `n` training configurations
 * (samples_dev, device int8 [n][L][L]; points_dev, device int32 [n] point
 * indices of a conditional network, or NULL) as crbm_ar_batch draws it
 * with step = step0 + k for the k-th step; learning rate lr for the steps
 * k < late_from * steps, lr_late after.  loss_out (host, may be NULL): the
 * mean negative log-likelihood per configuration of the last step's batch.
 * Equals `steps` calls of crbm_ar_train_step_cond on those batches, bit for
 * bit.  CRBM_EINVAL for bad options (steps < 0, batch < 1, lr <= 0,
 * step0 + steps > 2^32 - 1), CRBM_ESTATE for a conditional network without
 * points.  Synchronises only to return the loss. */
typedef struct {
    int64_t steps;       /* Adam steps */
    int64_t batch;       /* configurations per step */
    float lr, lr_late;   /* learning rates */
    double late_from;    /* fraction of the steps after which lr_late applies */
    uint64_t seed;       /* key of the minibatch stream */
    int64_t step0;       /* counter of the first step's minibatch */
    int32_t augment;     /* nonzero: random lattice symmetries (see crbm_ar_batch) */
} crbm_train_opts;
int crbm_ar_train(crbm_ar_t* a, const int8_t* samples_dev, const int32_t* points_dev, int64_t n,
                  const crbm_train_opts* opts, double* loss_out);
/* The minibatch of training step `step` (no network needed; asynchronous on
 * `stream`): configuration b of out_dev (device int8 [batch][L][L]) is
 * training configuration idx_b = floor(u n / 2^64), u = out[0] 2^32 + out[1]
 * of Philox (ctr = (b, step, 0, 7), key = seed); with augment, rolled by
 * (2 (out[2] mod L/2), 2 ((out[3] >> 1) mod L/2)) sites along (rows,
 * columns), out[r][c] = in[(r - dr) mod L][(c - dc) mod L], then transposed
 * if out[3] is odd: symmetries of the periodic Shastry-Sutherland lattice
 * (the dimer layout of Sec. I Fig. 1 maps onto itself), so every
 * configuration keeps its energy.  points_out_dev (may be NULL): the point
 * of each drawn configuration (points_dev[idx_b], 0 if points_dev is NULL);
 * index_out_dev (may be NULL): idx_b. */
int crbm_ar_batch(const int8_t* samples_dev, const int32_t* points_dev, int64_t n, int32_t L, int64_t batch,
                  uint64_t seed, int64_t step, int32_t augment, int8_t* out_dev, int32_t* points_out_dev,
                  int64_t* index_out_dev, void* stream);
/* log q of n configurations (device int8 [n][L][L]) into logq_dev (device fp64 [n])
 * by one forward pass over all sites, under the proposal law of
 * crbm_ar_sample (per site log(t / 2^32) or log(1 - t / 2^32)).  The per-site arithmetic, and the fp64 sum
 * over sites in raster order, are those of crbm_ar_sample, so a proposal scored
 * here gets the log q its sampler returned, bit for bit.  Asynchronous. */
int crbm_ar_logq(crbm_ar_t* a, const int8_t* spins_dev, int64_t n, double* logq_dev);
/* n independent proposals by ancestral sampling in raster order into
 * spins_dev (int8 [n][L][L]) with their log q into logq_dev (fp64 [n]).
 * With t(x) = clamp(rint(2^32 sigmoid(-|x|)), 1, 2^31) (fp32 sigmoid) for
 * the logit x of site i, the spin is +1 iff u < 2^32 - t (x >= 0) or u < t
 * (x < 0), with u word 0 of Philox (ctr = (site, step, chain, id << 3 | 6),
 * key = seed): the value against the sign of x has probability exactly
 * t / 2^32, and log q sums log(t / 2^32) or log(1 - t / 2^32) over the sites,
 * the exact probability of the drawn proposal (for the Metropolis-Hastings
 * ratio), at any logit. */
int crbm_ar_sample(crbm_ar_t* a, int64_t n, uint64_t seed, int64_t step, uint32_t id, int8_t* spins_dev,
                   double* logq_dev);
/* n_steps batches of n proposals in one launch (for an independent-MH
 * proposal stream, whose draws do not depend on the chains): batch k, written
 * at spins_dev + k n L^2 and logq_dev + k n (device int8 [n_steps][n][L][L],
 * fp64 [n_steps][n]), equals crbm_ar_sample_cond(a, n, seed, step0 + k, id,
 * points_dev, ...) bit for bit; points_dev (device int32 [n], or NULL for an
 * unconditional network) is shared by all batches.  One launch of n n_steps
 * chains keeps more SIMDs busy than n_steps launches of n.  CRBM_EINVAL for
 * n < 1, n_steps < 1, n n_steps > 2^31 or NULL outputs. */
int crbm_ar_sample_steps(crbm_ar_t* a, int64_t n, int32_t n_steps, uint64_t seed, int64_t step0, uint32_t id,
                         const int32_t* points_dev, int8_t* spins_dev, double* logq_dev);
/* n_cycles of: gibbs_per_mh Gibbs sweeps of h (crbm_sample), then one
 * independent MH step per chain with a's proposals; every instance of h must
 * have the network's L and a constant temperature, and h and a must use the
 * same stream.  Each chain's acceptance uses its own instance's target.  A
 * conditional network draws the proposals of instance i's chains at point i
 * (CRBM_EINVAL if fewer points are set than h has instances).  Cycle k of the
 * network's life draws its proposals with step = k and its MH uniforms from
 * Philox (ctr = (0, k, chain, id << 3 | 5)); chain is the index over all
 * instances' chains and id the first instance's id.  counts_trace
 * (device, may be NULL): int32 (M, B1, B2) after each cycle, [n_cycles][chains][3].
 * order_trace (device, may be NULL): the plateau structure factor record of
 * crbm_sample_thinned after each cycle, same layout.
 * n_accepted (host, may be NULL): accepted moves (synchronises).
 * The proposals of up to 8 cycles (at most 16384 proposals) are drawn in one
 * sampler launch, as by crbm_ar_sample_steps; results do not depend on how
 * cycles are grouped, or on how they are split over calls.  The sampler runs
 * ahead on a stream the network handle owns (created on first use, default
 * priority), two batches at most, ordered by events: the call is asynchronous
 * on the handles' stream, whose work after it waits for every proposal it
 * uses, and the sampler waits for the stream's earlier work (the weights).
 * CRBM_EUNSUPPORTED for a handle created with CRBM_PRECISION_FPGA. */
int crbm_sample_mh(crbm_t* h, crbm_ar_t* a, int64_t n_cycles, int32_t gibbs_per_mh, int32_t* counts_trace,
                   int32_t* order_trace, int64_t* n_accepted);
void crbm_ar_destroy(crbm_ar_t* a);

/* Free everything the handle owns.  NULL is allowed. */
void crbm_destroy(crbm_t* h);

/* Message of the last error on this thread ("" if none). */
const char* crbm_last_error(void);

/* Failure injection for tests of the error paths (process-wide, not
 * thread-safe against concurrent creates): with n >= 0, the library's n-th
 * device allocation from now on (0 = the next) fails as if the device were out
 * of memory, once; n < 0 disarms it.  Every entry point that allocates must
 * then return CRBM_ENOMEM with a message, free what it had taken, and work
 * normally on the next call.  Returns CRBM_OK. */
int crbm_debug_fail_alloc(int32_t n);

/* Test hook (process-wide): the hidden comparison of the Gibbs samplers
 * (crbm_sample, crbm_lattice_sample) finishes the words still tied after two
 * random blocks on at most `cap` lanes per round, 64 by default; a smaller cap
 * makes the launches from now on take several rounds, a path that 64 lanes
 * almost never need (direct launches, and the graph of a handle created in
 * graph mode after the call: a graph keeps the kernel it was built with).
 * Trajectories do not depend on it.  CRBM_EINVAL unless 1 <= cap <= 64. */
int crbm_debug_tail_cap(int32_t cap);

/* Host-side helpers that expose the library's own tables (used by tests to
 * check them against the oracle).
 * crbm_threshold: the 32-bit sigmoid threshold t(y) for an integer field
 *   magnitude y >= 0 in 2^16 units (App. A sigmoid module, closest value).
 * crbm_sweep_table: the 16-word table the device reads for sweep s of
 *   instance i (see the kernel source for the layout). */
uint32_t crbm_threshold(int64_t y);
int crbm_sweep_table(const crbm_t* h, int32_t i, int64_t s, uint32_t out[16]);

/* Host only, no device needed: the 16-word table for couplings (J1, J2, h) at
 * temperature T, exactly as crbm_create builds it.  Returns CRBM_EINVAL for
 * T <= 0 or non-finite input, CRBM_ERANGE on fixed-point overflow. */
int crbm_table_for(double J1, double J2, double h, double T, uint32_t out[16]);

/* The 16-word device table of one sweep for (J1, J2, h) at temperature T in
 * the given precision (CRBM_PRECISION_*), built on the host exactly as
 * crbm_create builds it (layout: the library's internal table; for tests).
 * CRBM_ERANGE if a 16.16 value overflows int32, CRBM_EINVAL for a bad T,
 * precision or NULL out. */
int crbm_table_for_precision(double J1, double J2, double h, double T, int32_t precision, uint32_t* out);

/* ------------------------------------------------------------------------
 * General lattices: open or periodic axes, one coupling per filter, a field
 * per column parity.
 *
 * App. A Wrapper Module: each axis of the lattice either wraps around or is
 * padded with zeros (open boundary; Sec. III.A uses it for the laterally
 * confined lattices of width 12).  Here a bond whose endpoint falls past the
 * last row (column) of an open axis does not exist: no hidden unit is drawn
 * for it and no field reaches its other spin.  App. A Hidden Node Registers:
 * (rows/2) x (cols/2) cells of 10 filters.  App. A Convoluter-Reverse: the
 * host writes every filter, so each filter k carries its own coupling J_k
 * (k0-k3: horizontal square edges (0,0)-(0,1), (0,1)-(0,2), (1,0)-(1,1),
 * (1,1)-(1,2) of the cell window; k4-k7: vertical edges (0,0)-(1,0),
 * (1,0)-(2,0), (0,1)-(1,1), (1,1)-(2,1); k8: the dimer (0,0)-(1,1); k9: the
 * dimer (1,2)-(2,1)); the Shastry-Sutherland lattice is J_k = J1 for k < 8
 * and J2 for k = 8, 9.  App. A Accumulator: separate visible biases for even
 * and odd columns.  H = sum_k J_k sum_{bonds of k} s_a s_b - h_even sum_{even c} s
 * - h_odd sum_{odd c} s.
 *
 * Arithmetic and random numbers follow the square-lattice sampler (16.16
 * couplings, 32-bit thresholds, the same Philox counters with the column
 * layout of `cols`), so a periodic square lattice with the SS couplings gives
 * the trajectories of crbm_create / crbm_sample bit for bit.
 *
 * Counts of one state (int32, exact): c[0] = M_even, c[1] = M_odd (spin sums
 * over even / odd columns), c[2 + k] = B_k = sum over the bonds of filter k of
 * s_a s_b; E = sum_k Jq_k B_k - hq_even M_even - hq_odd M_odd in 2^-16 units
 * (Jq = llround(J 2^16)).
 * ------------------------------------------------------------------------ */
#define CRBM_LAT_MAX_SIDE 64
#define CRBM_LAT_N_COUNTS 12
/* accumulator words per instance: n, sums of the 12 counts, sum M^2, sum |M|,
 * sum Ms, sum Ms^2, sum |Ms| (M = M_even + M_odd, Ms = sum (-1)^(r+c) s) */
#define CRBM_LAT_N_ACC 18

typedef struct {
    int32_t rows, cols;            /* even, 4 <= rows, cols <= CRBM_LAT_MAX_SIDE */
    int32_t open_rows, open_cols;  /* 1: that axis is open, 0: periodic */
    double J[10];                  /* coupling of filter k; |J| 2^16 < 2^31 */
    double h_even, h_odd;          /* field on even / odd columns */
    int32_t n_chains;              /* >= 1 */
    int32_t sched_kind;            /* CRBM_SCHED_* */
    double T0, T1;
    const double* T_explicit;      /* host array of n_sweeps temperatures (EXPLICIT only), copied */
    uint32_t id;                   /* instance id in the random-number counter, < 2^29 */
} crbm_lattice;

typedef struct crbm_lat_s crbm_lat_t;

/* Create a sampler for n_inst general lattices sharing cfg (seed, n_sweeps,
 * measure_every, burn_in, stream, flags; CRBM_F_CORR accumulates the
 * displacement correlation below).  tile_rows, launch_mode and
 * waves_per_block are ignored; precision must be CRBM_PRECISION_Q16.
 * Builds the per-sweep tables on the host, allocates the device state and
 * initialises every chain from the seed (stream 0, site index r cols + c);
 * returns after the set-up has finished on cfg->stream.  Errors:
 * CRBM_EINVAL (odd or out-of-range sides, non-finite couplings or fields,
 * T <= 0, n_chains < 1, NULL pointers), CRBM_ERANGE (a field leaves int32 at
 * some sweep), CRBM_EUNSUPPORTED (another precision), CRBM_EHIP. */
int crbm_lattice_create(const crbm_lattice* inst, int32_t n_inst, const crbm_config* cfg, crbm_lat_t** out);

/* Enqueue the next n_sweeps sweeps on cfg->stream (asynchronous).
 * spins_out: device int8 [sum of chains x rows x cols] (+-1, instances
 *   concatenated, chains row-major) or NULL.
 * counts_trace: device int32 [n_sweeps / trace_every][total chains][12], the
 *   counts after every trace_every-th sweep of this call, or NULL.
 * Errors: CRBM_EINVAL (trace_every < 1 or not dividing n_sweeps),
 * CRBM_ESTATE (past the end of the schedule), CRBM_EHIP. */
int crbm_lattice_sample(crbm_lat_t* h, int64_t n_sweeps, int8_t* spins_out, int32_t* counts_trace,
                        int32_t trace_every);

/* Synchronise the stream and return, per instance, the CRBM_LAT_N_ACC
 * accumulator sums over chains and measured sweeps (host int64
 * [n_inst][CRBM_LAT_N_ACC]).  corr_out (host int64, or NULL; needs
 * CRBM_F_CORR): per instance [rows][2 cols - 1] sums over chains and measured
 * sweeps of Cn(dr, dc) = sum of s(r,c) s(r+dr, c+dc) over the pairs inside the
 * lattice (no wrapping), 0 <= dr < rows, -cols < dc < cols at index
 * [dr][dc + cols - 1]: the static structure factor of Sec. III.B Eq. (13) at
 * any wave vector q is sum over all displacements d of Cn(d) e^{i q.d}
 * (Cn(-d) = Cn(d)), on open and periodic lattices alike. */
int crbm_lattice_observables(crbm_lat_t* h, int64_t* acc_out, int64_t* corr_out);

/* Zero the accumulators and correlation sums (asynchronous). */
int crbm_lattice_reset_observables(crbm_lat_t* h);

/* Checkpoint / resume: int8 spins (device, layout of spins_out) and the
 * sweep index.  get_state synchronises; set_state is asynchronous.
 * CRBM_EINVAL for a sweep index outside [0, n_sweeps]. */
int crbm_lattice_get_state(crbm_lat_t* h, int8_t* spins_dev, int64_t* sweep_index);
int crbm_lattice_set_state(crbm_lat_t* h, const int8_t* spins_dev, int64_t sweep_index);

int64_t crbm_lattice_total_chains(const crbm_lat_t* h);

/* Free everything the handle owns (after its stream has finished).  NULL is allowed. */
void crbm_lattice_destroy(crbm_lat_t* h);

/* Host only: the device table of one sweep at temperature T for a lattice
 * (1056 words: per-filter hidden thresholds and flags, then 512 visible
 * entries by sublattice, edge type and incident-unit pattern; layout in the
 * kernel source).  For tests.  CRBM_EINVAL, CRBM_ERANGE as crbm_lattice_create. */
int crbm_lattice_table(const crbm_lattice* inst, double T, uint32_t* out);

#ifdef __cplusplus
}
#endif
#endif /* CRBM_H */
