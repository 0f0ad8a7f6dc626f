/*
 * kadabra_oracle.c -- plain, slow, single-threaded CPU oracle for KADABRA
 * adaptive-sampling betweenness approximation as parallelised by
 * van der Grinten, Angriman and Meyerhenke ("Parallel Adaptive Sampling with
 * almost no Synchronization").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header, table or constant
 * generator with the HIP implementation.
 *
 * What it computes, and where each step comes from:
 *   - the generic adaptive-sampling loop: Algorithm 1 (sample, aggregate with
 *     an associative operator, check only on a consistent state);
 *   - the KADABRA sample (Section 2.3): a uniform vertex pair (s, t) and a
 *     uniformly random shortest s-t path; the estimator counts, per vertex,
 *     the sampled paths it lies on;
 *   - the stopping rule f, g <= eps for every vertex (Appendix B), with
 *     omega, delta_L and delta_U from the preprocessing of Section 2.3;
 *   - the same-component test and path reconstruction from the graph plus a
 *     distance vector (Appendix C.1);
 *   - per-sample reseeding by a sample index, which makes the result
 *     independent of the schedule (indexed-frame algorithm, Appendix D).
 *   - optionally, per-vertex delta_L(v), delta_U(v) chosen from a first,
 *     separate sampling phase (Section 2.3 requires only that their sum over
 *     all vertices stays within delta; KADABRA's own balancing is in the
 *     paper it cites, so the rule used here is a reading, derived below).
 * Readings of points on which the paper is silent (the balanced bidirectional
 * BFS rule, the omega formula, uniform delta_L/delta_U, the balancing rule,
 * exact 128-bit sigma that a level divides by a power of two only beyond
 * 2^104, the 40-bit meeting weights, the random-draw assignment) are listed
 * with the function that takes them.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared (no fast-math: the
 * stop test must evaluate the exact IEEE expression tree given below).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "kadabra_oracle.h"

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): a counter-based generator; 10 rounds of a       */
/* multiply/xor round function with a Weyl-sequence key schedule.            */
/* ------------------------------------------------------------------------ */

void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u; /* round multipliers */
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u; /* key increments */
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Draw j of sample i: Philox block with key = seed, counter = (i, j, 0).
 * Each sample owns its own stream of draws, so sample i is the same whatever
 * thread or schedule produces it (the indexed-frame idea, Appendix D). */
static void draw_block(uint64_t seed, uint64_t i, uint32_t j, uint32_t out[4])
{
    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(i >> 32), j, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, out);
}

/* 64-bit uniform word of draw j: x0 | x1 << 32. */
uint64_t oracle_uniform64(uint64_t seed, uint64_t i, uint32_t j)
{
    uint32_t x[4];
    draw_block(seed, i, j, x);
    return (uint64_t)x[0] | ((uint64_t)x[1] << 32);
}

/* floor(u * m / 2^64): maps a uniform 64-bit word onto [0, m). */
static uint64_t mulhi64(uint64_t u, uint64_t m)
{
    return (uint64_t)(((u128)u * (u128)m) >> 64);
}

/* Uniform ordered pair s != t (Section 2.3: "vertex pairs uniformly at
 * random"; ordered and distinct, as in the sum defining b(u)). */
void oracle_pair(uint64_t seed, uint64_t i, int32_t n, int32_t *s_out, int32_t *t_out)
{
    uint32_t x[4];
    draw_block(seed, i, 0u, x);
    uint64_t ua = (uint64_t)x[0] | ((uint64_t)x[1] << 32);
    uint64_t ub = (uint64_t)x[2] | ((uint64_t)x[3] << 32);
    int64_t s = (int64_t)mulhi64(ua, (uint64_t)n);
    int64_t t = (int64_t)mulhi64(ub, (uint64_t)(n - 1));
    if (t >= s) t += 1;
    *s_out = (int32_t)s;
    *t_out = (int32_t)t;
}

/* Pairs of samples i0 .. i0 + count - 1 (for the pair-law tests). */
void oracle_pairs(uint64_t seed, uint64_t i0, int64_t count, int32_t n, int32_t *s, int32_t *t)
{
    for (int64_t k = 0; k < count; ++k) oracle_pair(seed, i0 + (uint64_t)k, n, &s[k], &t[k]);
}

/* number of significant bits of x (0 for x == 0) */
static int bit_width64(uint64_t x)
{
    int w = 0;
    while (x) { ++w; x >>= 1; }
    return w;
}

static int bit_width128(u128 x)
{
    int w = 0;
    while (x) { ++w; x >>= 1; }
    return w;
}

static int64_t degree(const int32_t *row_ptr, int32_t v)
{
    return (int64_t)row_ptr[v + 1] - (int64_t)row_ptr[v];
}

/* ------------------------------------------------------------------------ */
/* Preprocessing (Section 2.3: omega and delta_L, delta_U are fixed before   */
/* sampling, mostly by bounding the diameter; Appendix C.1: components are   */
/* computed along with the diameter).                                        */
/* ------------------------------------------------------------------------ */

/* Connected components by BFS; comp[v] = index of v's component, numbered in
 * order of each component's lowest vertex.  Returns the number of components. */
int32_t oracle_components(int32_t n, const int32_t *row_ptr, const int32_t *col, int32_t *comp)
{
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int32_t v = 0; v < n; ++v) comp[v] = -1;
    int32_t ncomp = 0;
    for (int32_t r = 0; r < n; ++r) {
        if (comp[r] >= 0) continue;
        int32_t head = 0, tail = 0;
        queue[tail++] = r;
        comp[r] = ncomp;
        while (head < tail) {
            int32_t u = queue[head++];
            for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                int32_t w = col[e];
                if (comp[w] < 0) { comp[w] = ncomp; queue[tail++] = w; }
            }
        }
        ++ncomp;
    }
    free(queue);
    return ncomp;
}

/* Eccentricity of r inside its component, by plain BFS. */
static int32_t eccentricity(int32_t n, const int32_t *row_ptr, const int32_t *col, int32_t r,
                            int32_t *dist, int32_t *queue)
{
    int32_t head = 0, tail = 0, ecc = 0;
    (void)n;
    dist[r] = 0;
    queue[tail++] = r;
    while (head < tail) {
        int32_t u = queue[head++];
        if (dist[u] > ecc) ecc = dist[u];
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int32_t w = col[e];
            if (dist[w] < 0) { dist[w] = dist[u] + 1; queue[tail++] = w; }
        }
    }
    for (int32_t k = 0; k < tail; ++k) dist[queue[k]] = -1; /* leave dist all -1 */
    return ecc;
}

/* Vertex-diameter bound VD (number of vertices on a longest shortest path is
 * at most VD).  Reading: in each component c, BFS from its maximum-degree
 * vertex r_c (lowest id on ties); every shortest path in c has at most
 * 2 ecc(r_c) edges, so VD = max_c (2 ecc(r_c) + 1). */
int32_t oracle_vd_bound(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *comp,
                        int32_t ncomp)
{
    int32_t *root = (int32_t *)malloc(sizeof(int32_t) * (size_t)ncomp);
    for (int32_t c = 0; c < ncomp; ++c) root[c] = -1;
    for (int32_t v = 0; v < n; ++v) {
        int32_t c = comp[v];
        if (root[c] < 0 || degree(row_ptr, v) > degree(row_ptr, root[c])) root[c] = v;
    }
    int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int32_t v = 0; v < n; ++v) dist[v] = -1;
    int32_t vd = 1;
    for (int32_t c = 0; c < ncomp; ++c) {
        int32_t ecc = eccentricity(n, row_ptr, col, root[c], dist, queue);
        if (2 * ecc + 1 > vd) vd = 2 * ecc + 1;
    }
    free(root); free(dist); free(queue);
    return vd;
}

/* Maximal number of samples omega.  The paper only says that such a bound
 * exists (Section 2.3) and defers its formula to the original KADABRA paper.
 * Reading: omega = ceil( (0.5 / eps^2) * (floor(log2(VD - 2)) + 1 + ln(2/delta)) ),
 * the VC-dimension bound of the Riondato-Kornaropoulos / KADABRA line of work,
 * with VD - 2 clamped to at least 1 and floor(log2) taken exactly on integers. */
int64_t oracle_omega(int32_t vd, double eps, double delta)
{
    int64_t x = (int64_t)vd - 2;
    if (x < 1) x = 1;
    int k = bit_width64((uint64_t)x) - 1;
    double w = 0.5 / (eps * eps) * ((double)k + 1.0 + log(2.0 / delta));
    return (int64_t)ceil(w);
}

/* log(1/delta_L(v)) = log(1/delta_U(v)).  Reading: uniform
 * delta_L(v) = delta_U(v) = delta / (4 n), which meets the constraint of
 * Section 2.3 that sum_v delta_L(v) + delta_U(v) <= delta (it uses delta/2). */
double oracle_log_inv_delta(int32_t n, double delta)
{
    return log(4.0 * (double)n / delta);
}

/* ------------------------------------------------------------------------ */
/* The stopping condition (Appendix B).                                      */
/* f = (L/tau) (1/3 - w/tau + sqrt((1/3 - w/tau)^2 + 2 b w / L))              */
/* g = (L/tau) (1/3 + w/tau + sqrt((1/3 + w/tau)^2 + 2 b w / L))              */
/* with L = log(1/delta_{L,U}(v)), w = omega, b = c(v)/tau.  Stop iff f <= eps */
/* and g <= eps for every vertex (the explicit form of Appendix B; Section   */
/* 2.3 writes "<").  Evaluated in IEEE double in exactly this order, without  */
/* contraction.                                                              */
/* ------------------------------------------------------------------------ */

void oracle_fg(int32_t c, int64_t tau, int64_t omega, double L, double *f_out, double *g_out)
{
    double t = (double)tau;
    double w = (double)omega;
    double b = (double)c / t;
    double af = 1.0 / 3.0 - w / t;
    double ag = 1.0 / 3.0 + w / t;
    double q = 2.0 * b * w / L;
    *f_out = (L / t) * (af + sqrt(af * af + q));
    *g_out = (L / t) * (ag + sqrt(ag * ag + q));
}

/* f and g of every counts[k] (k < n) at one (tau, omega, L), as oracle_fg. */
void oracle_fg_batch(int64_t n, const int32_t *counts, int64_t tau, int64_t omega, double L, double *f,
                     double *g)
{
    for (int64_t k = 0; k < n; ++k) oracle_fg(counts[k], tau, omega, L, &f[k], &g[k]);
}

/* Returns 1 iff the stopping condition holds on (counts, tau). */
int oracle_check_stop(int32_t n, const int32_t *counts, int64_t tau, int64_t omega, double L,
                      double eps)
{
    for (int32_t v = 0; v < n; ++v) {
        double f, g;
        oracle_fg(counts[v], tau, omega, L, &f, &g);
        if (!(f <= eps) || !(g <= eps)) return 0;
    }
    return 1;
}

/* Same rule with separate constants: f uses log(1/delta_L(v)), g uses
 * log(1/delta_U(v)) (the two invariants of Section 2.3). */
int oracle_check_stop_v(int32_t n, const int32_t *counts, int64_t tau, int64_t omega,
                        const double *LL, const double *LU, double eps)
{
    for (int32_t v = 0; v < n; ++v) {
        double f, g, unused;
        oracle_fg(counts[v], tau, omega, LL[v], &f, &unused);
        oracle_fg(counts[v], tau, omega, LU[v], &unused, &g);
        if (!(f <= eps) || !(g <= eps)) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Balancing delta_L(v), delta_U(v) (the adjacent step before the adaptive   */
/* loop).  Section 2.3 fixes only sum_v delta_L(v) + delta_U(v) <= delta;    */
/* this code spends delta/2 on it (as the uniform reading does) and keeps    */
/* the other delta/2 for the omega cap.  Reading, derived from Appendix B:   */
/*                                                                           */
/*  1. A first phase draws M1 samples from a stream the adaptive loop never  */
/*     uses: first-phase sample m is sample index 2^63 + m.  c1(v) counts    */
/*     the first-phase paths through v; these samples are not part of the    */
/*     estimate, so the constants do not depend on the adaptive samples.     */
/*  2. Planning value b_p(v) = (c1(v) + 1) / M1 (add-one, so that a vertex   */
/*     no first-phase path crossed still gets a positive value).            */
/*  3. For a target sample count t, the largest L for which f(b_p, L, w, t)  */
/*     <= eps has a closed form.  With x = L / t, af = 1/3 - w/t and         */
/*     q = 2 b w / t, f = x af + sqrt(x^2 af^2 + q x) is increasing in x,   */
/*     and f = eps at x = eps^2 / (q + 2 eps af).  If q + 2 eps af <= 0,     */
/*     f stays below eps for every L (its limit is b w / (w - t/3)): then    */
/*     L_f = +inf.  For g the same with ag = 1/3 + w/t (always finite).      */
/*  4. S(t) = sum_v exp(-L_f(v, t)) + exp(-L_g(v, t)) is the failure budget  */
/*     that makes every vertex meet the rule at t if b~ = b_p.  The terms    */
/*     depend on v only through c1(v) = k, so S is evaluated over the count  */
/*     histogram h(k) = #{v : c1(v) = k}: the rows with h(k) > 0 in          */
/*     ascending k, each adding h(k) (exp(-L_f(k)) + exp(-L_g(k))), left to  */
/*     right in double.  This order is part of the definition: any           */
/*     implementation that sums in it with the same exp gets the same bits.  */
/*     t* is found by bisection on [1, omega] for S(t) <= (1 - beta)         */
/*     delta/2; if the bisection ends at omega there is no plan and the      */
/*     uniform constants are kept.                                           */
/*  5. delta_L(v) = (1 - beta) exp(-L_f(v, t*)) + beta delta / (4 n), and    */
/*     delta_U(v) likewise: a floor share beta = 1/10 of the budget, spread  */
/*     uniformly, covers vertices whose count grows past the plan.  Then    */
/*     sum_v delta_L + delta_U = (1 - beta) S(t*) + beta delta/2 <= delta/2. */
/*     The target carries a relative margin of 1e-6 for the rounding of S.  */
/* Evaluated in IEEE double in exactly the order written, no contraction.    */
/* ------------------------------------------------------------------------ */

#define BALANCE_FLOOR 0.1
#define FIRST_PHASE_BASE ((uint64_t)1 << 63)

/* First-phase sample count when none is given: ceil(omega / 20). */
int64_t oracle_first_phase_samples(int64_t omega)
{
    return (omega + 19) / 20;
}

/* L_f and L_g (step 3) for planning value b at target t. */
void oracle_plan_lfg(double b, int64_t t_, int64_t omega, double eps, double *Lf, double *Lg)
{
    double t = (double)t_;
    double w = (double)omega;
    double af = 1.0 / 3.0 - w / t;
    double ag = 1.0 / 3.0 + w / t;
    double q = 2.0 * b * w / t;
    double df = q + 2.0 * eps * af;
    double dg = q + 2.0 * eps * ag;
    double e2 = eps * eps;
    *Lf = (df > 0.0) ? t * e2 / df : INFINITY;
    *Lg = t * e2 / dg;
}

static double plan_b(int32_t c1, int64_t m1)
{
    return ((double)c1 + 1.0) / (double)m1;
}

/* S(t) of step 4: over the count histogram's nonzero rows in ascending k. */
double oracle_plan_sum(int32_t n, const int32_t *c1, int64_t m1, int64_t t, int64_t omega,
                       double eps)
{
    int64_t *h = calloc((size_t)m1 + 1, sizeof *h);
    if (!h) return NAN;
    for (int32_t v = 0; v < n; ++v)
        if (c1[v] >= 0 && (int64_t)c1[v] <= m1) h[c1[v]] += 1;
    double S = 0.0;
    for (int64_t k = 0; k <= m1; ++k) {
        if (h[k] == 0) continue;
        double Lf, Lg;
        oracle_plan_lfg(((double)k + 1.0) / (double)m1, t, omega, eps, &Lf, &Lg);
        S += (double)h[k] * (exp(-Lf) + exp(-Lg));
    }
    free(h);
    return S;
}

/* Steps 4-5: writes log(1/delta_L(v)), log(1/delta_U(v)) and returns t*
 * (0: no plan, LL = LU = L, the uniform constant). */
int64_t oracle_plan(int32_t n, const int32_t *c1, int64_t m1, int64_t omega, double eps,
                    double delta, double L, double *LL, double *LU)
{
    double beta = BALANCE_FLOOR;
    double target = (1.0 - beta) * (delta / 2.0) * (1.0 - 1e-6);
    int64_t lo = 1, hi = omega;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (oracle_plan_sum(n, c1, m1, mid, omega, eps) <= target) hi = mid;
        else lo = mid + 1;
    }
    if (lo >= omega) {
        for (int32_t v = 0; v < n; ++v) LL[v] = LU[v] = L;
        return 0;
    }
    double floor_share = beta * delta / (4.0 * (double)n);
    for (int32_t v = 0; v < n; ++v) {
        double Lf, Lg;
        oracle_plan_lfg(plan_b(c1[v], m1), lo, omega, eps, &Lf, &Lg);
        LL[v] = -log((1.0 - beta) * exp(-Lf) + floor_share);
        LU[v] = -log((1.0 - beta) * exp(-Lg) + floor_share);
    }
    return lo;
}

/* ------------------------------------------------------------------------ */
/* One KADABRA sample (Section 2.3): uniform pair, then a uniformly random   */
/* shortest path, found by a balanced bidirectional BFS that counts shortest */
/* paths (sigma) and a backtracking walk on the graph and distance vectors   */
/* (Appendix C.1: no predecessor graph is stored).                           */
/*                                                                           */
/* Readings (the paper defers the sampler to the original KADABRA paper):    */
/*  - expand the side whose frontier has the smaller degree sum, s on ties;  */
/*  - sigma of a new level is an exact 128-bit integer sum over             */
/*    predecessors; only if the level's largest sum reaches 2^104 is the     */
/*    whole level divided by a power of two (rounding up), so sigma is exact */
/*    below 2^104 (degree < 2^23 keeps every sum below 2^127);               */
/*  - the meeting vertex is drawn with probability proportional to           */
/*    sigma_s(v) sigma_t(v) over the meeting set in ascending vertex order,  */
/*    with the exact products rounded up to 40-bit integer weights;          */
/*    predecessors are drawn proportional to sigma in CSR order;             */
/*  - draw 1 picks the meeting vertex; draw 2 d + [side t] picks the         */
/*    predecessor of the path vertex at distance d from that side's root;    */
/*  - the counter is incremented on the interior path vertices only (the     */
/*    definition of b(u) excludes the endpoints).                            */
/* ------------------------------------------------------------------------ */

#define SIDE_S 0
#define SIDE_T 1
#define SIGMA_BITS 104  /* largest stored sigma mantissa: 2^104 */
#define WEIGHT_BITS 40  /* meeting weights are at most 2^40 */

/* 256-bit unsigned integer as two 128-bit halves (for sigma_s * sigma_t) */
typedef struct { u128 hi, lo; } u256;

static u256 mul128(u128 a, u128 b)
{
    const u128 M = ((u128)1 << 64) - 1;
    u128 a0 = a & M, a1 = a >> 64, b0 = b & M, b1 = b >> 64;
    u128 p00 = a0 * b0, p01 = a0 * b1, p10 = a1 * b0, p11 = a1 * b1;
    u128 mid = (p00 >> 64) + (p01 & M) + (p10 & M);
    u256 r;
    r.lo = (p00 & M) | (mid << 64);
    r.hi = p11 + (p01 >> 64) + (p10 >> 64) + (mid >> 64);
    return r;
}

static int bit_width256(u256 x)
{
    return x.hi ? 128 + bit_width128(x.hi) : bit_width128(x.lo);
}

static int less256(u256 a, u256 b)
{
    return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
}

/* ceil(x / 2^sh) for a result known to fit in 64 bits */
static uint64_t ceil_shift256(u256 x, int sh)
{
    u128 q;
    int rem;
    if (sh == 0) return (uint64_t)x.lo;
    if (sh < 128) {
        q = (x.lo >> sh) | (x.hi << (128 - sh));
        rem = (x.lo & (((u128)1 << sh) - 1)) != 0;
    } else {
        q = (sh == 128) ? x.hi : (x.hi >> (sh - 128));
        rem = x.lo != 0 || (sh > 128 && (x.hi & (((u128)1 << (sh - 128)) - 1)) != 0);
    }
    return (uint64_t)q + (uint64_t)rem;
}

/* floor(u * m / 2^64) for a 64-bit uniform u and a 128-bit total m < 2^127 */
static u128 mulhi64x128(uint64_t u, u128 m)
{
    const u128 M = ((u128)1 << 64) - 1;
    u128 lo = (u128)u * (m & M);
    u128 hi = (u128)u * (m >> 64);
    return hi + (lo >> 64);
}

struct sampler {
    int32_t n;
    const int32_t *row_ptr, *col, *comp;
    int32_t *dist[2];   /* -1 = not reached; reset through the visited lists */
    u128 *m[2];         /* sigma (scaled by 2^-shift of its level, see above) */
    int32_t *ball[2];   /* vertices reached by each side, in BFS order */
    int32_t nball[2];
    int32_t *next;      /* the level being built */
    int32_t *meet;      /* meeting set */
};

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static int sampler_init(struct sampler *S, int32_t n, const int32_t *row_ptr, const int32_t *col,
                        const int32_t *comp)
{
    memset(S, 0, sizeof(*S));
    S->n = n; S->row_ptr = row_ptr; S->col = col; S->comp = comp;
    for (int x = 0; x < 2; ++x) {
        S->dist[x] = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        S->m[x] = (u128 *)calloc((size_t)n, sizeof(u128));
        S->ball[x] = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        if (!S->dist[x] || !S->m[x] || !S->ball[x]) return -1;
        for (int32_t v = 0; v < n; ++v) S->dist[x][v] = -1;
    }
    S->next = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    S->meet = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    return (S->next && S->meet) ? 0 : -1;
}

static void sampler_free(struct sampler *S)
{
    for (int x = 0; x < 2; ++x) { free(S->dist[x]); free(S->m[x]); free(S->ball[x]); }
    free(S->next); free(S->meet);
}

/* Draws sample i.  Writes the path's interior vertices to interior[] (room
 * for n entries) and returns their number, or -1 if s and t are in different
 * components (the sample then adds nothing).  Optional outputs describe the
 * search for the tests. */
static int32_t sample_path(struct sampler *S, uint64_t seed, uint64_t i, int32_t *interior,
                           oracle_sample_info *info, oracle_stats *st, int32_t s_given,
                           int32_t t_given)
{
    const int32_t *row_ptr = S->row_ptr, *col = S->col;
    int32_t s, t;
    if (s_given >= 0) { s = s_given; t = t_given; }  /* a fixed pair (path-law tests) */
    else oracle_pair(seed, i, S->n, &s, &t);
    if (info) { memset(info, 0, sizeof(*info)); info->s = s; info->t = t; info->d = -1; }
    /* Appendix C.1: no search between different components */
    if (S->comp[s] != S->comp[t]) return -1;

    int32_t *dist_s = S->dist[SIDE_S], *dist_t = S->dist[SIDE_T];
    int32_t level[2] = {0, 0};
    int32_t front_lo[2] = {0, 0}, front_hi[2] = {1, 1};
    int64_t dsum[2];
    int32_t cumshift[2] = {0, 0}; /* true sigma of a frontier = m * 2^cumshift */
    S->ball[SIDE_S][0] = s; S->nball[SIDE_S] = 1;
    S->ball[SIDE_T][0] = t; S->nball[SIDE_T] = 1;
    dist_s[s] = 0; S->m[SIDE_S][s] = 1;
    dist_t[t] = 0; S->m[SIDE_T][t] = 1;
    dsum[SIDE_S] = degree(row_ptr, s);
    dsum[SIDE_T] = degree(row_ptr, t);

    int32_t nmeet = 0, X = SIDE_S, Y = SIDE_T, d = -1, meet_scale = 0;
    for (;;) {
        X = (dsum[SIDE_S] <= dsum[SIDE_T]) ? SIDE_S : SIDE_T;
        Y = 1 - X;
        int32_t *dx = S->dist[X], *dy = S->dist[Y];
        u128 *mx = S->m[X];
        if (st) { st->v_exp += front_hi[X] - front_lo[X]; st->e_scan += dsum[X]; }

        /* next level: unreached neighbours of the frontier */
        int32_t nnext = 0;
        for (int32_t k = front_lo[X]; k < front_hi[X]; ++k) {
            int32_t u = S->ball[X][k];
            for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                int32_t w = col[e];
                if (dx[w] < 0) {
                    dx[w] = level[X] + 1;
                    S->next[nnext++] = w;
                }
            }
        }
        if (st) st->v_new += nnext;
        if (nnext == 0) abort(); /* same component, so the balls must grow */

        /* sigma of the new level: raw(w) = sum of m_X(p) over the neighbours p
         * of w at distance level[X].  Those neighbours are exactly the
         * frontier vertices adjacent to w (the graph is undirected), so the sum
         * is taken over the frontier's arcs. */
        for (int32_t k = 0; k < nnext; ++k) mx[S->next[k]] = 0;
        for (int32_t k = front_lo[X]; k < front_hi[X]; ++k) {
            int32_t u = S->ball[X][k];
            for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                int32_t w = col[e];
                if (dx[w] == level[X] + 1) {
                    mx[w] += mx[u];
                    if (st) st->e_pred += 1;
                }
            }
        }
        u128 hmax = 0;
        for (int32_t k = 0; k < nnext; ++k)
            if (mx[S->next[k]] > hmax) hmax = mx[S->next[k]];
        int sh = bit_width128(hmax) - SIGMA_BITS;
        if (sh < 0) sh = 0;
        if (sh > 0) {
            u128 add = ((u128)1 << sh) - 1;
            for (int32_t k = 0; k < nnext; ++k) {
                int32_t w = S->next[k];
                mx[w] = (mx[w] + add) >> sh;
            }
            if (st) st->rescaled_levels += 1;
        }

        /* append the level to the ball (it is reset after the sample) */
        for (int32_t k = 0; k < nnext; ++k) S->ball[X][S->nball[X]++] = S->next[k];

        /* meeting set: new vertices already reached from the other side; all
         * of them lie on the other side's frontier (the balls were disjoint) */
        nmeet = 0;
        for (int32_t k = 0; k < nnext; ++k) {
            int32_t w = S->next[k];
            if (dy[w] >= 0) {
                if (dy[w] != level[Y]) abort();
                S->meet[nmeet++] = w;
            }
        }
        if (nmeet > 0) {
            d = level[X] + 1 + level[Y];
            meet_scale = cumshift[X] + sh + cumshift[Y];
            break;
        }
        cumshift[X] += sh;
        front_lo[X] = front_hi[X];
        front_hi[X] = S->nball[X];
        level[X] += 1;
        int64_t ds = 0;
        for (int32_t k = front_lo[X]; k < front_hi[X]; ++k) ds += degree(row_ptr, S->ball[X][k]);
        dsum[X] = ds;
    }

    /* meeting vertex: weight P(v) = m_s(v) m_t(v) (exact, 256-bit), rounded up
     * to at most 2^40 by a common power of two; ascending vertex order */
    qsort(S->meet, (size_t)nmeet, sizeof(int32_t), cmp_i32);
    u256 pmax = {0, 0};
    for (int32_t k = 0; k < nmeet; ++k) {
        int32_t v = S->meet[k];
        u256 p = mul128(S->m[SIDE_S][v], S->m[SIDE_T][v]);
        if (less256(pmax, p)) pmax = p;
    }
    int shp = bit_width256(pmax) - WEIGHT_BITS;
    if (shp < 0) shp = 0;
    uint64_t total = 0;
    for (int32_t k = 0; k < nmeet; ++k) {
        int32_t v = S->meet[k];
        total += ceil_shift256(mul128(S->m[SIDE_S][v], S->m[SIDE_T][v]), shp);
    }
    uint64_t r = mulhi64(oracle_uniform64(seed, i, 1u), total);
    int32_t v = -1;
    uint64_t acc = 0;
    for (int32_t k = 0; k < nmeet; ++k) {
        int32_t x = S->meet[k];
        acc += ceil_shift256(mul128(S->m[SIDE_S][x], S->m[SIDE_T][x]), shp);
        if (acc > r) { v = x; break; }
    }
    if (info) {
        u256 sig = {0, 0};
        for (int32_t k = 0; k < nmeet; ++k) {
            int32_t x = S->meet[k];
            u256 p = mul128(S->m[SIDE_S][x], S->m[SIDE_T][x]);
            u128 lo = sig.lo + p.lo;
            sig.hi += p.hi + (lo < sig.lo);
            sig.lo = lo;
        }
        info->d = d;
        info->meet_size = nmeet;
        info->meet_vertex = v;
        info->meet_total = total;
        info->meet_shift = shp;
        info->sigma_w[0] = (uint64_t)sig.lo;
        info->sigma_w[1] = (uint64_t)(sig.lo >> 64);
        info->sigma_w[2] = (uint64_t)sig.hi;
        info->sigma_w[3] = (uint64_t)(sig.hi >> 64);
        info->side_x_last = X;
        info->sigma_scale = meet_scale;
    }

    /* path: the meeting vertex, then backtrack towards s and towards t */
    int32_t ni = 0;
    if (dist_s[v] > 0 && dist_t[v] > 0) interior[ni++] = v;
    for (int side = SIDE_S; side <= SIDE_T; ++side) {
        int32_t *dx = S->dist[side];
        u128 *mx = S->m[side];
        int32_t x = v;
        while (dx[x] > 1) {
            int32_t want = dx[x] - 1;
            u128 sum = 0;
            if (st) st->e_bt += degree(row_ptr, x);
            for (int32_t e = row_ptr[x]; e < row_ptr[x + 1]; ++e)
                if (dx[col[e]] == want) sum += mx[col[e]];
            uint32_t j = 2u * (uint32_t)dx[x] + (uint32_t)side;
            u128 rr = mulhi64x128(oracle_uniform64(seed, i, j), sum);
            u128 a = 0;
            int32_t pick = -1;
            for (int32_t e = row_ptr[x]; e < row_ptr[x + 1]; ++e) {
                int32_t p = col[e];
                if (dx[p] != want) continue;
                a += mx[p];
                if (a > rr) { pick = p; break; }
            }
            x = pick;
            interior[ni++] = x;
        }
    }
    if (st) { st->path_interior += ni; }

    /* reset the per-sample state through the visited lists */
    for (int side = SIDE_S; side <= SIDE_T; ++side)
        for (int32_t k = 0; k < S->nball[side]; ++k) {
            int32_t w = S->ball[side][k];
            S->dist[side][w] = -1;
            S->m[side][w] = 0;
        }
    return ni;
}

/* ------------------------------------------------------------------------ */
/* The adaptive loop (Algorithm 1) with checks only at the fixed sample      */
/* counts B_k = min(k N, omega) (Appendix C.2: check every N samples; the   */
/* cap omega of Section 2.3).  Counts are checked only when they hold exactly */
/* the samples 0 .. B_k - 1: the consistency requirement of Section 2.1.     */
/* ------------------------------------------------------------------------ */

int oracle_setup(int32_t n, const int32_t *row_ptr, const int32_t *col, double eps, double delta,
                 int32_t *comp, int32_t *vd_out, int64_t *omega_out, double *L_out)
{
    if (n < 2 || !(eps > 0.0 && eps < 1.0) || !(delta > 0.0 && delta < 1.0)) return -1;
    int32_t ncomp = oracle_components(n, row_ptr, col, comp);
    int32_t vd = oracle_vd_bound(n, row_ptr, col, comp, ncomp);
    *vd_out = vd;
    *omega_out = oracle_omega(vd, eps, delta);
    *L_out = oracle_log_inv_delta(n, delta);
    return 0;
}

/* First phase (balancing step 1): c1(v) over first-phase samples 0 .. m1-1,
 * i.e. sample indices 2^63 .. 2^63 + m1 - 1.  Work counters go to st. */
static int first_phase(struct sampler *S, int32_t n, uint64_t seed, int64_t m1, int32_t *c1,
                       int32_t *interior, oracle_stats *st)
{
    for (int32_t v = 0; v < n; ++v) c1[v] = 0;
    for (int64_t m = 0; m < m1; ++m) {
        int32_t ni = sample_path(S, seed, FIRST_PHASE_BASE + (uint64_t)m, interior, NULL, st, -1, -1);
        if (ni < 0) { st->disconnected += 1; continue; }
        for (int32_t q = 0; q < ni; ++q) c1[interior[q]] += 1;
    }
    return 0;
}

/* The adaptive loop.  first_samples: 0 = uniform delta_L = delta_U (no first
 * phase); -1 = balanced with ceil(omega / 20) first-phase samples; > 0 =
 * balanced with that many.  LL, LU (optional, n each) receive the constants
 * used; c1 (optional, n) the first-phase counts. */
int oracle_run_balanced(int32_t n, const int32_t *row_ptr, const int32_t *col, double eps,
                        double delta, uint64_t seed, int64_t check_interval, int64_t sample_cap,
                        int64_t first_samples, int32_t *counts, oracle_stats *st,
                        int8_t *decisions, int64_t max_decisions, double *LL_out,
                        double *LU_out, int32_t *c1_out)
{
    if (check_interval < 1 || first_samples < -1) return -1;
    memset(st, 0, sizeof(*st));
    int32_t *comp = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *interior = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double *LL = (double *)malloc(sizeof(double) * (size_t)n);
    double *LU = (double *)malloc(sizeof(double) * (size_t)n);
    int32_t *c1 = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!comp || !interior || !LL || !LU || !c1) {
        free(comp); free(interior); free(LL); free(LU); free(c1);
        return -2;
    }
    int32_t vd;
    int64_t omega;
    double L;
    if (oracle_setup(n, row_ptr, col, eps, delta, comp, &vd, &omega, &L) != 0) {
        free(comp); free(interior); free(LL); free(LU); free(c1);
        return -1;
    }
    st->vd = vd; st->omega = omega; st->L = L;
    struct sampler S;
    if (sampler_init(&S, n, row_ptr, col, comp) != 0) {
        free(comp); free(interior); free(LL); free(LU); free(c1);
        return -2;
    }

    for (int32_t v = 0; v < n; ++v) { LL[v] = LU[v] = L; c1[v] = 0; }
    if (first_samples != 0) {
        int64_t m1 = first_samples > 0 ? first_samples : oracle_first_phase_samples(omega);
        oracle_stats fs;
        memset(&fs, 0, sizeof(fs));
        first_phase(&S, n, seed, m1, c1, interior, &fs);
        st->first_samples = m1;
        st->first_v_exp = fs.v_exp;
        st->first_e_scan = fs.e_scan;
        st->first_e_bt = fs.e_bt;
        st->first_path_interior = fs.path_interior;
        st->first_disconnected = fs.disconnected;
        st->plan_tau = oracle_plan(n, c1, m1, omega, eps, delta, L, LL, LU);
    }
    for (int32_t v = 0; v < n; ++v) counts[v] = 0;

    int64_t tau = 0, k = 0;
    for (;;) {
        ++k;
        int64_t hi = k * check_interval;
        if (hi > omega) hi = omega;
        if (sample_cap >= 0 && hi > sample_cap) hi = sample_cap;
        for (int64_t i = tau; i < hi; ++i) {
            int32_t ni = sample_path(&S, seed, (uint64_t)i, interior, NULL, st, -1, -1);
            if (ni < 0) { st->disconnected += 1; continue; }
            for (int32_t q = 0; q < ni; ++q) counts[interior[q]] += 1;
        }
        tau = hi;
        st->epochs = k;
        if (sample_cap >= 0 && tau >= sample_cap) break; /* bounded timing sample */
        if (tau == omega) {
            if (decisions && k - 1 < max_decisions) decisions[k - 1] = 2;
            break;
        }
        int stop = oracle_check_stop_v(n, counts, tau, omega, LL, LU, eps);
        if (decisions && k - 1 < max_decisions) decisions[k - 1] = (int8_t)stop;
        if (stop) break;
    }
    st->tau = tau;
    if (LL_out) memcpy(LL_out, LL, sizeof(double) * (size_t)n);
    if (LU_out) memcpy(LU_out, LU, sizeof(double) * (size_t)n);
    if (c1_out) memcpy(c1_out, c1, sizeof(int32_t) * (size_t)n);
    sampler_free(&S);
    free(comp); free(interior); free(LL); free(LU); free(c1);
    return 0;
}

int oracle_run(int32_t n, const int32_t *row_ptr, const int32_t *col, double eps, double delta,
               uint64_t seed, int64_t check_interval, int64_t sample_cap, int32_t *counts,
               oracle_stats *st, int8_t *decisions, int64_t max_decisions)
{
    return oracle_run_balanced(n, row_ptr, col, eps, delta, seed, check_interval, sample_cap, 0,
                               counts, st, decisions, max_decisions, NULL, NULL, NULL);
}

/* ------------------------------------------------------------------------ */
/* The same adaptive loop on T threads (the CPU baseline on all host cores):  */
/* the local-frame idea of Section 3 with the indexed-frame assignment of    */
/* Appendix D.2.  In each epoch [B_{k-1}, B_k), thread t draws the samples    */
/* i = B_{k-1} + t, + T, ... into its own counter frame; the frames are added */
/* into the counters at the boundary, and only then is the stopping rule      */
/* checked, on exactly the samples [0, B_k).  Sample i depends on i alone and */
/* the sums are integer, so tau and every counter equal oracle_run's.         */
/* ------------------------------------------------------------------------ */

struct thread_part {
    struct sampler S;
    int32_t *frame, *interior;
    oracle_stats st;
    uint64_t seed;
    int64_t lo, hi, stride;
};

static void *thread_epoch(void *arg)
{
    struct thread_part *P = (struct thread_part *)arg;
    for (int64_t i = P->lo; i < P->hi; i += P->stride) {
        int32_t ni = sample_path(&P->S, P->seed, (uint64_t)i, P->interior, NULL, &P->st, -1, -1);
        if (ni < 0) { P->st.disconnected += 1; continue; }
        for (int32_t q = 0; q < ni; ++q) P->frame[P->interior[q]] += 1;
    }
    return NULL;
}

int oracle_run_threads(int32_t n, const int32_t *row_ptr, const int32_t *col, double eps, double delta,
                       uint64_t seed, int64_t check_interval, int32_t threads, int32_t *counts,
                       oracle_stats *st, int8_t *decisions, int64_t max_decisions)
{
    if (check_interval < 1 || threads < 1 || threads > 1024) return -1;
    memset(st, 0, sizeof(*st));
    int32_t *comp = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    struct thread_part *P = (struct thread_part *)calloc((size_t)threads, sizeof *P);
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof *tid);
    int rc = -2;
    int32_t made = 0;
    if (!comp || !P || !tid) goto out;
    int32_t vd;
    int64_t omega;
    double L;
    if (oracle_setup(n, row_ptr, col, eps, delta, comp, &vd, &omega, &L) != 0) { rc = -1; goto out; }
    st->vd = vd; st->omega = omega; st->L = L;
    for (; made < threads; ++made) {
        struct thread_part *p = &P[made];
        p->frame = (int32_t *)calloc((size_t)n, sizeof(int32_t));
        p->interior = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        if (!p->frame || !p->interior || sampler_init(&p->S, n, row_ptr, col, comp) != 0) {
            free(p->frame); free(p->interior);
            goto out;
        }
        p->seed = seed;
        p->stride = threads;
    }
    for (int32_t v = 0; v < n; ++v) counts[v] = 0;
    int64_t tau = 0, k = 0;
    for (;;) {
        ++k;
        int64_t hi = k * check_interval;
        if (hi > omega) hi = omega;
        for (int32_t t = 0; t < threads; ++t) {
            P[t].lo = tau + t;
            P[t].hi = hi;
            if (pthread_create(&tid[t], NULL, thread_epoch, &P[t]) != 0) {
                for (int32_t u = 0; u < t; ++u) pthread_join(tid[u], NULL);
                rc = -2;
                goto out;
            }
        }
        for (int32_t t = 0; t < threads; ++t) pthread_join(tid[t], NULL);
        /* the boundary: every frame into the counters (and zeroed) */
        for (int32_t t = 0; t < threads; ++t)
            for (int32_t v = 0; v < n; ++v) {
                counts[v] += P[t].frame[v];
                P[t].frame[v] = 0;
            }
        tau = hi;
        st->epochs = k;
        if (tau == omega) {
            if (decisions && k - 1 < max_decisions) decisions[k - 1] = 2;
            break;
        }
        int stop = oracle_check_stop(n, counts, tau, omega, L, eps);
        if (decisions && k - 1 < max_decisions) decisions[k - 1] = (int8_t)stop;
        if (stop) break;
    }
    st->tau = tau;
    for (int32_t t = 0; t < threads; ++t) {
        st->v_exp += P[t].st.v_exp;
        st->e_scan += P[t].st.e_scan;
        st->v_new += P[t].st.v_new;
        st->e_pred += P[t].st.e_pred;
        st->e_bt += P[t].st.e_bt;
        st->path_interior += P[t].st.path_interior;
        st->disconnected += P[t].st.disconnected;
        st->rescaled_levels += P[t].st.rescaled_levels;
    }
    rc = 0;
out:
    for (int32_t t = 0; t < made; ++t) {
        sampler_free(&P[t].S);
        free(P[t].frame);
        free(P[t].interior);
    }
    free(P); free(tid); free(comp);
    return rc;
}

/* Single sample, for the path-law and unbiasedness tests.  Returns the number
 * of interior vertices written to interior[] (room for n), or -1 if s and t
 * lie in different components. */
int32_t oracle_sample(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *comp,
                      uint64_t seed, uint64_t i, int32_t *interior, oracle_sample_info *info)
{
    struct sampler S;
    if (sampler_init(&S, n, row_ptr, col, comp) != 0) return -2;
    int32_t r = sample_path(&S, seed, i, interior, info, NULL, -1, -1);
    sampler_free(&S);
    return r;
}

/* Samples i0 .. i0 + count - 1 with the pair (s, t) given instead of drawn
 * (s != t, one component): draw 0 is unused, draws j >= 1 of each sample pick
 * the meeting vertex and the predecessors as in any sample.  For the
 * path-law tests at one pair.  Writes sample k's interior vertices (their
 * order as in oracle_sample) to paths[k stride ...] (stride >= d - 1), its
 * meeting vertex to meet[k], and the first sample's description to *info.
 * Returns the number of interior vertices per sample (the same for every
 * sample of one pair), -1 if s and t lie in different components, -2 on a
 * failed allocation, -3 if stride is too small. */
int32_t oracle_sample_pair(int32_t n, const int32_t *row_ptr, const int32_t *col,
                           const int32_t *comp, uint64_t seed, int32_t s, int32_t t, uint64_t i0,
                           int64_t count, int32_t stride, int32_t *paths, int32_t *meet,
                           oracle_sample_info *info)
{
    struct sampler S;
    oracle_sample_info one;
    int32_t *interior = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!interior || sampler_init(&S, n, row_ptr, col, comp) != 0) { free(interior); return -2; }
    int32_t ni = 0;
    for (int64_t k = 0; k < count; ++k) {
        ni = sample_path(&S, seed, i0 + (uint64_t)k, interior, &one, NULL, s, t);
        if (k == 0 && info) *info = one;
        if (ni < 0) break;
        if (ni > stride) { ni = -3; break; }
        memcpy(paths + (size_t)k * (size_t)stride, interior, sizeof(int32_t) * (size_t)ni);
        meet[k] = one.meet_vertex;
    }
    sampler_free(&S);
    free(interior);
    return ni;
}

/* Sum of x_i(v) over samples [i0, i1) without any stopping rule (for the
 * unbiasedness test).  Returns the number of connected samples. */
int64_t oracle_accumulate(int32_t n, const int32_t *row_ptr, const int32_t *col,
                          const int32_t *comp, uint64_t seed, uint64_t i0, uint64_t i1,
                          int64_t *acc)
{
    struct sampler S;
    int32_t *interior = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!interior || sampler_init(&S, n, row_ptr, col, comp) != 0) return -2;
    int64_t connected = 0;
    for (uint64_t i = i0; i < i1; ++i) {
        int32_t ni = sample_path(&S, seed, i, interior, NULL, NULL, -1, -1);
        if (ni < 0) continue;
        ++connected;
        for (int32_t q = 0; q < ni; ++q) acc[interior[q]] += 1;
    }
    sampler_free(&S);
    free(interior);
    return connected;
}

/* ------------------------------------------------------------------------ */
/* Exact betweenness (Section 2.2: Brandes' algorithm, Theta(|V||E|) for     */
/* unweighted graphs), normalised by n(n-1) so that it is the quantity the  */
/* estimator approximates: b(v) = sum over ordered s != t, v not in {s,t},  */
/* of sigma_st(v) / sigma_st, divided by n(n-1).                            */
/* ------------------------------------------------------------------------ */

void oracle_brandes(int32_t n, const int32_t *row_ptr, const int32_t *col, double *bc)
{
    int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double *sigma = (double *)malloc(sizeof(double) * (size_t)n);
    double *delta = (double *)malloc(sizeof(double) * (size_t)n);
    for (int32_t v = 0; v < n; ++v) bc[v] = 0.0;
    for (int32_t s = 0; s < n; ++s) {
        for (int32_t v = 0; v < n; ++v) { dist[v] = -1; sigma[v] = 0.0; delta[v] = 0.0; }
        int32_t head = 0, tail = 0;
        dist[s] = 0; sigma[s] = 1.0; order[tail++] = s;
        while (head < tail) {
            int32_t u = order[head++];
            for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                int32_t w = col[e];
                if (dist[w] < 0) { dist[w] = dist[u] + 1; order[tail++] = w; }
                if (dist[w] == dist[u] + 1) sigma[w] += sigma[u];
            }
        }
        /* dependency accumulation in order of non-increasing distance */
        for (int32_t k = tail - 1; k >= 0; --k) {
            int32_t w = order[k];
            for (int32_t e = row_ptr[w]; e < row_ptr[w + 1]; ++e) {
                int32_t p = col[e];
                if (dist[p] == dist[w] - 1) delta[p] += sigma[p] / sigma[w] * (1.0 + delta[w]);
            }
            if (w != s) bc[w] += delta[w];
        }
    }
    double norm = (double)n * (double)(n - 1);
    for (int32_t v = 0; v < n; ++v) bc[v] /= norm;
    free(dist); free(order); free(sigma); free(delta);
}

/* Unidirectional BFS from s: distances (-1 if unreachable) and exact shortest
 * path counts in double (exact up to 2^53), for the sigma pins. */
void oracle_bfs_sigma(int32_t n, const int32_t *row_ptr, const int32_t *col, int32_t s,
                      int32_t *dist, double *sigma)
{
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int32_t v = 0; v < n; ++v) { dist[v] = -1; sigma[v] = 0.0; }
    int32_t head = 0, tail = 0;
    dist[s] = 0; sigma[s] = 1.0; queue[tail++] = s;
    while (head < tail) {
        int32_t u = queue[head++];
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int32_t w = col[e];
            if (dist[w] < 0) { dist[w] = dist[u] + 1; queue[tail++] = w; }
            if (dist[w] == dist[u] + 1) sigma[w] += sigma[u];
        }
    }
    free(queue);
}
