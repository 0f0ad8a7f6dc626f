/*
 * kadabra_oracle.h -- interface of the plain CPU oracle (test infrastructure
 * only; never linked into the product library).  See kadabra_oracle.c for
 * what each function computes and the paper passage it follows.
 */
#ifndef KADABRA_ORACLE_H
#define KADABRA_ORACLE_H
#include <stdint.h>

typedef struct {
    int64_t tau;           /* samples drawn when the loop stopped */
    int64_t omega;         /* maximal number of samples */
    int64_t vd;            /* vertex-diameter bound */
    int64_t epochs;        /* number of check boundaries reached */
    int64_t v_exp;         /* frontier vertices expanded */
    int64_t e_scan;        /* arcs scanned by expansions (sum of frontier degrees) */
    int64_t v_new;         /* vertices newly reached */
    int64_t e_pred;        /* predecessor arcs summed into sigma */
    int64_t e_bt;          /* arcs scanned while backtracking */
    int64_t path_interior; /* counter increments */
    int64_t disconnected;  /* samples whose endpoints lie in different components */
    int64_t rescaled_levels; /* BFS levels whose sigma had to be divided by 2^sh */
    double L;              /* log(1 / delta_L) (uniform) */
    int64_t first_samples; /* balancing: first-phase samples (0 = uniform constants) */
    int64_t plan_tau;      /* balancing: planned sample count t* (0 = no plan) */
    int64_t first_v_exp;   /* work counters of the first phase */
    int64_t first_e_scan;
    int64_t first_e_bt;
    int64_t first_path_interior;
    int64_t first_disconnected;
} oracle_stats;

typedef struct {
    int32_t s, t;
    int32_t d;             /* distance, -1 if disconnected */
    int32_t meet_size;     /* size of the meeting set */
    int32_t meet_vertex;   /* chosen meeting vertex */
    int32_t meet_shift;    /* shift applied to the meeting weights */
    uint64_t meet_total;   /* sum of the quantised meeting weights */
    uint64_t sigma_w[4];   /* sum over the meeting set of m_s m_t (256-bit, little endian) */
    int32_t side_x_last;   /* side expanded at the meeting level (0 = s) */
    int32_t sigma_scale;   /* sigma_st ~= sigma_w * 2^sigma_scale (exact if 0) */
} oracle_sample_info;

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
uint64_t oracle_uniform64(uint64_t seed, uint64_t i, uint32_t j);
void oracle_pair(uint64_t seed, uint64_t i, int32_t n, int32_t *s, int32_t *t);
void oracle_pairs(uint64_t seed, uint64_t i0, int64_t count, int32_t n, int32_t *s, int32_t *t);
int32_t oracle_components(int32_t n, const int32_t *row_ptr, const int32_t *col, int32_t *comp);
int32_t oracle_vd_bound(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *comp,
                        int32_t ncomp);
int64_t oracle_omega(int32_t vd, double eps, double delta);
double oracle_log_inv_delta(int32_t n, double delta);
void oracle_fg(int32_t c, int64_t tau, int64_t omega, double L, double *f, double *g);
/* oracle_fg over counts[0, n) at one (tau, omega, L) into f[0, n), g[0, n). */
void oracle_fg_batch(int64_t n, const int32_t *counts, int64_t tau, int64_t omega, double L, double *f,
                     double *g);
int oracle_check_stop(int32_t n, const int32_t *counts, int64_t tau, int64_t omega, double L,
                      double eps);
int oracle_check_stop_v(int32_t n, const int32_t *counts, int64_t tau, int64_t omega,
                        const double *LL, const double *LU, double eps);
int64_t oracle_first_phase_samples(int64_t omega);
void oracle_plan_lfg(double b, int64_t t, int64_t omega, double eps, double *Lf, double *Lg);
double oracle_plan_sum(int32_t n, const int32_t *c1, int64_t m1, int64_t t, int64_t omega,
                       double eps);
int64_t oracle_plan(int32_t n, const int32_t *c1, int64_t m1, int64_t omega, double eps,
                    double delta, double L, double *LL, double *LU);
int oracle_run_balanced(int32_t n, const int32_t *row_ptr, const int32_t *col, double eps,
                        double delta, uint64_t seed, int64_t check_interval, int64_t sample_cap,
                        int64_t first_samples, int32_t *counts, oracle_stats *st,
                        int8_t *decisions, int64_t max_decisions, double *LL, double *LU,
                        int32_t *c1);
int oracle_setup(int32_t n, const int32_t *row_ptr, const int32_t *col, double eps, double delta,
                 int32_t *comp, int32_t *vd, int64_t *omega, double *L);
int oracle_run(int32_t n, const int32_t *row_ptr, const int32_t *col, double eps, double delta,
               uint64_t seed, int64_t check_interval, int64_t sample_cap, int32_t *counts,
               oracle_stats *st, int8_t *decisions, int64_t max_decisions);

/* oracle_run (uniform constants, no sample cap) on `threads` threads: each
 * epoch's samples are split by index over per-thread counter frames that are
 * added into the counters at the boundary before the check; the result equals
 * oracle_run's.  Returns 0, -1 (bad argument) or -2 (allocation or thread
 * creation failed). */
int oracle_run_threads(int32_t n, const int32_t *row_ptr, const int32_t *col, double eps, double delta,
                       uint64_t seed, int64_t check_interval, int32_t threads, int32_t *counts,
                       oracle_stats *st, int8_t *decisions, int64_t max_decisions);
int32_t oracle_sample(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *comp,
                      uint64_t seed, uint64_t i, int32_t *interior, oracle_sample_info *info);
int32_t oracle_sample_pair(int32_t n, const int32_t *row_ptr, const int32_t *col,
                           const int32_t *comp, uint64_t seed, int32_t s, int32_t t, uint64_t i0,
                           int64_t count, int32_t stride, int32_t *paths, int32_t *meet,
                           oracle_sample_info *info);
int64_t oracle_accumulate(int32_t n, const int32_t *row_ptr, const int32_t *col,
                          const int32_t *comp, uint64_t seed, uint64_t i0, uint64_t i1,
                          int64_t *acc);
void oracle_brandes(int32_t n, const int32_t *row_ptr, const int32_t *col, double *bc);
void oracle_bfs_sigma(int32_t n, const int32_t *row_ptr, const int32_t *col, int32_t s,
                      int32_t *dist, double *sigma);
#endif
