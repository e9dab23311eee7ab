/*
 * crbm_oracle.h -- interface of the CPU oracle (test infrastructure only).
 * Not included by, and not sharing anything with, the HIP library.
 * All conventions are stated at the top of crbm_oracle.c.
 */
#ifndef CRBM_ORACLE_H
#define CRBM_ORACLE_H
#include <stdint.h>

typedef struct {
    int32_t L;             /* even lattice side */
    double J1, J2, h;      /* H = J1 sum_sq s s + J2 sum_dimer s s - h sum s */
    int32_t sched_kind;    /* 0 const, 1 linear, 2 geometric, 3 explicit */
    double T0, T1;
    const double* T_explicit;
    uint32_t id;           /* instance id in the random-number counter */
    int32_t precision;     /* 0: 16.16 weights, 32-bit sigmoid; 1: the hardware's Q5.4 / 16-bit precision */
} oracle_instance;

void     oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
uint32_t oracle_uniform_hidden(uint64_t seed, uint32_t id, uint32_t chain, uint32_t sweep,
                               int L, int k, int i, int j);
uint32_t oracle_uniform_visible(uint64_t seed, uint32_t id, uint32_t chain, uint32_t sweep,
                                int L, int r, int c);
int64_t  oracle_quantise(double J);
int64_t  oracle_q54(double v);
uint32_t oracle_sigmoid16(int64_t y);
void     oracle_bond_weight_q54(int64_t Jq, double T, int64_t* wq, int* sig);
double   oracle_schedule_T(int kind, double T0, double T1, const double* T_explicit,
                           int64_t S, int64_t s);
void     oracle_bond_weight(int64_t Jq, double T, int64_t* wq, int* sig);
int64_t  oracle_visible_bias(int64_t hq, double T);
uint32_t oracle_threshold(int64_t y);
void     oracle_bond_sites(int L, int k, int i, int j, int* ra, int* ca, int* rb, int* cb, int* type);
void     oracle_counts(int L, const int8_t* s, int64_t* M, int64_t* B1, int64_t* B2);
void     oracle_corr(int L, const int8_t* s, int64_t* corr);
int64_t  oracle_staggered(int L, const int8_t* s);
void     oracle_order(int L, const int8_t* s, int64_t out[3]);
void     oracle_init_spins(const oracle_instance* in, uint64_t seed, uint32_t chain, int8_t* s);
int      oracle_run_chain(const oracle_instance* in, int64_t S, uint64_t seed, uint32_t chain,
                          int64_t sweep_begin, int64_t sweep_end, int8_t* s,
                          int32_t* trace, int32_t measure_every, int64_t burn_in, int64_t* acc,
                          int64_t* corr_acc);
double   oracle_log_marginal(const oracle_instance* in, int64_t S, int64_t sweep, const int8_t* s);

/* General lattices (open or periodic axes, one coupling per filter, a field
 * per column parity); conventions in crbm_oracle.c. */
typedef struct {
    int32_t Lr, Lc;        /* rows, columns: even */
    int32_t open_r, open_c;/* 1: that axis is open (bonds past the edge absent), 0: periodic */
    double J[10];          /* coupling of filter k */
    double h_even, h_odd;  /* field on even / odd columns */
    int32_t sched_kind;
    double T0, T1;
    const double* T_explicit;
    uint32_t id;
} oracle_lattice;

#define ORACLE_LATTICE_N_ACC 18  /* n, M_e, M_o, B_0..B_9, sum M^2, sum |M|, sum Ms, sum Ms^2, sum |Ms| */

int      oracle_lattice_bond(const oracle_lattice* in, int k, int i, int j, int* ra, int* ca, int* rb, int* cb);
void     oracle_lattice_counts(const oracle_lattice* in, const int8_t* s, int64_t out[12]);
void     oracle_lattice_corr(int Lr, int Lc, const int8_t* s, int64_t* corr);
void     oracle_lattice_init_spins(const oracle_lattice* in, uint64_t seed, uint32_t chain, int8_t* s);
int      oracle_lattice_run_chain(const oracle_lattice* in, int64_t S, uint64_t seed, uint32_t chain,
                                  int64_t sweep_begin, int64_t sweep_end, int8_t* s, int32_t* trace,
                                  int32_t measure_every, int64_t burn_in, int64_t* acc, int64_t* corr_acc);
double   oracle_lattice_log_marginal(const oracle_lattice* in, int64_t S, int64_t sweep, const int8_t* s);

#endif
