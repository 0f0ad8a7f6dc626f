// kadabra_host.cpp -- C ABI and host runtime of the gfx950 KADABRA library.
//
// Host side: input validation, the driver of the graph-only preprocessing on
// the device (components and the vertex-diameter bound, Section 2.3 /
// Appendix C.1, kernels in kadabra_prep.hip), omega and L, device
// memory, and the adaptive loop of Algorithm 1 with checks every N samples
// (Appendix C.2), driven for any number of concurrent queries:
//
//   Runner      the device engine: a pool of sample slots shared by all
//               queries, a control block per query, and the round loop.  In a
//               round the stream runs
//                 sample_kernel   the next epochs (up to epochs_per_launch
//                                 check intervals) of every active query
//                 merge_check     per boundary B_k in order: counters +=
//                                 frames, stopping rule on [0, B_k)
//                 copy            every query's control block to the host
//               and, with overlap on, the following epochs' samples are queued
//               before the host reads the flags; a query that stopped makes
//               them exit on the device (the counters checked at B_k hold
//               exactly samples [0, B_k) either way).  A query with balanced
//               delta_L(v), delta_U(v) also carries its first phase in its
//               first launch, followed by the histogram and plan kernels
//               (kadabra_balance.hip) before its first check.
//   kadabra_graph   one graph on the device, running one query at a time.
//   kadabra_batch   many queries on many graphs in the same launches.
//   kadabra_server  continuous batching: a worker thread runs the round loop
//                   and admits submitted queries at every round boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/kadabra.h"
#include "kadabra_internal.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_OR_FAIL(expr)                                                                     \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(e_ == hipErrorOutOfMemory ? KADABRA_ENOMEM : KADABRA_EDEVICE,         \
                        "%s: %s", #expr, hipGetErrorString(e_));                              \
    } while (0)

#define OK_OR_RETURN(expr)           \
    do {                             \
        const int rc_ = (expr);      \
        if (rc_ != KADABRA_OK) return rc_; \
    } while (0)

constexpr int32_t kMaxN = 1 << 23;       // n and every degree stay below 2^23
constexpr int64_t kMaxOmega = INT32_MAX; // int32 counters
constexpr int64_t kMaxFirstPhase = INT32_MAX - 1;  // int32 first-phase counters, m1 + 1 table rows

// Device allocation.  *fail_countdown is a test hook: when it is positive it
// counts allocations down and the one that brings it to zero fails with
// out-of-memory (failure paths are then testable in-process).
hipError_t dev_alloc(void **p, size_t bytes, int64_t *fail_countdown = nullptr)
{
    if (fail_countdown && *fail_countdown > 0 && --*fail_countdown == 0) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    if (bytes == 0) bytes = 8;
    return hipMalloc(p, bytes);
}

template <class T>
hipError_t alloc_n(T **p, size_t count, int64_t *fail_countdown = nullptr)
{
    return dev_alloc(reinterpret_cast<void **>(p), count * sizeof(T), fail_countdown);
}

void dev_free(void *p)
{
    if (p) (void)hipFree(p);
}

template <class T>
void dev_release(T *&p)
{
    dev_free(p);
    p = nullptr;
}


int validate_csr(int32_t n, int64_t num_arcs, const int32_t *row_ptr, const int32_t *col,
                 int32_t *max_deg_out)
{
    if (n < 2) return fail(KADABRA_EINVAL, "n must be at least 2 (got %d)", n);
    if (n >= kMaxN) return fail(KADABRA_ERANGE, "n must be below 2^23 (got %d)", n);
    if (num_arcs < 0 || num_arcs > INT32_MAX)
        return fail(num_arcs < 0 ? KADABRA_EINVAL : KADABRA_ERANGE, "bad arc count %lld",
                    (long long)num_arcs);
    if (!row_ptr || (num_arcs > 0 && !col)) return fail(KADABRA_EINVAL, "null CSR array");
    if (row_ptr[0] != 0) return fail(KADABRA_EINVAL, "row_ptr[0] must be 0");
    if ((int64_t)row_ptr[n] != num_arcs)
        return fail(KADABRA_EINVAL, "row_ptr[n] (%d) != num_arcs (%lld)", row_ptr[n],
                    (long long)num_arcs);
    // every row bound first: non-decreasing from 0, so each lies in
    // [0, num_arcs], and only then any read of col
    int32_t max_deg = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (row_ptr[v + 1] < row_ptr[v])
            return fail(KADABRA_EINVAL, "row_ptr decreases at %d", v);
        if ((int64_t)row_ptr[v + 1] > num_arcs)
            return fail(KADABRA_EINVAL, "row_ptr[%d] (%d) exceeds num_arcs (%lld)", v + 1,
                        row_ptr[v + 1], (long long)num_arcs);
        max_deg = std::max(max_deg, row_ptr[v + 1] - row_ptr[v]);
    }
    for (int32_t v = 0; v < n; ++v) {
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            const int32_t w = col[e];
            if (w < 0 || w >= n) return fail(KADABRA_EINVAL, "column %d out of range at row %d", w, v);
            if (w == v) return fail(KADABRA_EINVAL, "self-loop at vertex %d", v);
            if (e > row_ptr[v] && col[e - 1] >= w)
                return fail(KADABRA_EINVAL, "row %d not strictly ascending", v);
        }
    }
    if (max_deg >= kMaxN) return fail(KADABRA_ERANGE, "degree %d is not below 2^23", max_deg);
    // symmetry: every arc (v, w) has its reverse (w, v).  Rows are strictly
    // ascending, so a scan over v upwards meets the sources of the arcs into w
    // in the order of row w: one cursor per row must find v at each step and
    // reach the row's end (O(n + m), no search).
    std::vector<int32_t> cur(row_ptr, row_ptr + n);
    for (int32_t v = 0; v < n; ++v)
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            const int32_t w = col[e];
            const int32_t t = cur[(size_t)w]++;
            if (t >= row_ptr[w + 1] || col[t] != v)
                return fail(KADABRA_EINVAL, "arc (%d, %d) has no reverse: graph not undirected", v, w);
        }
    for (int32_t w = 0; w < n; ++w)
        if (cur[(size_t)w] != row_ptr[w + 1])
            return fail(KADABRA_EINVAL, "arc (%d, %d) has no reverse: graph not undirected", w,
                        col[cur[(size_t)w]]);
    *max_deg_out = max_deg;
    return KADABRA_OK;
}

// omega = ceil(0.5/eps^2 (floor(log2(max(VD - 2, 1))) + 1 + ln(2/delta)))
int64_t omega_of(int32_t vd, double eps, double delta)
{
    int64_t x = (int64_t)vd - 2;
    if (x < 1) x = 1;
    int k = 63;
    while (!((x >> k) & 1)) --k;  // floor(log2 x), exact
    const double w = 0.5 / (eps * eps) * ((double)k + 1.0 + std::log(2.0 / delta));
    return (int64_t)std::ceil(w);
}


int32_t code_stride_for(int64_t nstride) { return (int32_t)(((nstride + 7) / 8 + 15) / 16 * 16); }

// Bytes of one sample slot for graphs of up to nstride vertices.
size_t slot_bytes(int64_t nstride, int32_t lcap)
{
    return (size_t)code_stride_for(nstride) * 4 +
           (size_t)nstride * (2 * sizeof(kd::Sigma) + 2 * sizeof(int32_t) + sizeof(int32_t) + sizeof(uint64_t)) +
           2 * (size_t)lcap * sizeof(int32_t);
}

// Run parameters (none but check_interval changes a result).
struct Params {
    int64_t check_interval = 1024;
    int team = 0;            // 0 auto, 64, 256
    int64_t slots = 0;       // 0 auto
    int frames = 1;
    int overlap = 1;
    int epochs = 2;          // epochs (check intervals) per sampling launch, 1..4
    int64_t probe_min = -1;  // -1 auto rule
    int probe_pull = 0;      // 1: meeting probes in the pull form (256-lane teams)
    int balance = 0;         // 1: per-vertex delta_L, delta_U from a first sampling phase
    int64_t balance_samples = 0;  // first-phase samples; 0: ceil(omega / 20)
    int64_t fail_alloc = 0;  // test hook
    int32_t level_cap = 0;   // test hook: 0, or a smaller level capacity per side
    int64_t stop_after = 0;  // > 0: stop at the first round end after this many boundaries of the run
};

int set_common_param(Params &p, const char *key, int64_t value, bool *known)
{
    *known = true;
    if (!strcmp(key, "check_interval")) {
        if (value < 1 || value > INT32_MAX) return fail(KADABRA_EINVAL, "check_interval must be in [1, 2^31)");
        p.check_interval = value;
    } else if (!strcmp(key, "team")) {
        if (value != 0 && value != 64 && value != 128 && value != 256 && value != 512)
            return fail(KADABRA_EINVAL, "team must be 0, 64, 128, 256 or 512");
        p.team = (int)value;
    } else if (!strcmp(key, "slots")) {
        if (value < 0 || value > (1 << 20)) return fail(KADABRA_EINVAL, "slots must be in [0, 2^20]");
        p.slots = value;
    } else if (!strcmp(key, "frames")) {
        if (value < 1 || value > 4096) return fail(KADABRA_EINVAL, "frames must be in [1, 4096]");
        p.frames = (int)value;
    } else if (!strcmp(key, "overlap")) {
        if (value != 0 && value != 1) return fail(KADABRA_EINVAL, "overlap must be 0 or 1");
        p.overlap = (int)value;
    } else if (!strcmp(key, "epochs_per_launch")) {
        if (value < 1 || value > kd::kMaxSets / 2)
            return fail(KADABRA_EINVAL, "epochs_per_launch must be in [1, %d]", kd::kMaxSets / 2);
        p.epochs = (int)value;
    } else if (!strcmp(key, "probe_min")) {
        if (value < -1) return fail(KADABRA_EINVAL, "probe_min must be >= -1");
        p.probe_min = value;
    } else if (!strcmp(key, "probe_pull")) {
        if (value != 0 && value != 1) return fail(KADABRA_EINVAL, "probe_pull must be 0 or 1");
        p.probe_pull = (int)value;
    } else if (!strcmp(key, "balance")) {
        if (value != 0 && value != 1) return fail(KADABRA_EINVAL, "balance must be 0 or 1");
        p.balance = (int)value;
    } else if (!strcmp(key, "balance_samples")) {
        if (value < 0 || value > kMaxFirstPhase)
            return fail(KADABRA_EINVAL, "balance_samples must be in [0, %lld]", (long long)kMaxFirstPhase);
        p.balance_samples = value;
    } else if (!strcmp(key, "test_fail_alloc")) {
        if (value < 0) return fail(KADABRA_EINVAL, "test_fail_alloc must be >= 0");
        p.fail_alloc = value;
    } else if (!strcmp(key, "stop_after_epochs")) {
        if (value < 0) return fail(KADABRA_EINVAL, "stop_after_epochs must be >= 0");
        p.stop_after = value;
    } else if (!strcmp(key, "test_level_cap")) {
        if (value != 0 && (value < 3 || value > (1 << 20)))
            return fail(KADABRA_EINVAL, "test_level_cap must be 0 or in [3, 2^20]");
        p.level_cap = (int32_t)value;
    } else {
        *known = false;
    }
    return KADABRA_OK;
}

int get_common_param(const Params &p, const char *key, int64_t *value)
{
    if (!strcmp(key, "check_interval")) *value = p.check_interval;
    else if (!strcmp(key, "team")) *value = p.team;
    else if (!strcmp(key, "slots")) *value = p.slots;
    else if (!strcmp(key, "frames")) *value = p.frames;
    else if (!strcmp(key, "overlap")) *value = p.overlap;
    else if (!strcmp(key, "epochs_per_launch")) *value = p.epochs;
    else if (!strcmp(key, "probe_min")) *value = p.probe_min;
    else if (!strcmp(key, "probe_pull")) *value = p.probe_pull;
    else if (!strcmp(key, "balance")) *value = p.balance;
    else if (!strcmp(key, "balance_samples")) *value = p.balance_samples;
    else if (!strcmp(key, "test_level_cap")) *value = p.level_cap;
    else if (!strcmp(key, "stop_after_epochs")) *value = p.stop_after;
    else return 1;
    return 0;
}

// Graphs whose vertex-diameter bound reaches this are high-diameter: they are
// relabelled for locality, the sampler's automatic meeting probe asks for
// more expected hits (probe_h8_for), and a probe that meets nothing in its
// first round is given up (QueryDesc::probe_quit).
constexpr int32_t kRelabelMinVd = 64;

// The automatic meeting probe fires when D_X D_Y >= h x arcs, in eighths
// (QueryDesc::probe_h8 = 8 h).  High-diameter graphs: h = 4 (their arcs stay
// local, and the degree-proportional estimate counts hits long before the
// balls touch).  Otherwise h = 1 / kappa, kappa = n sum(d^2) / (sum d)^2 =
// E[d^2] / E[d]^2 >= 1, clamped to [1/8, 1]: the frontiers of a degree-skewed
// graph crowd onto the same hubs and meet sooner than that estimate says
// (measured on R-MAT-18: h = 1/8 is 3.5% faster than h = 1; on ER-4096,
// kappa = 1.1, h = 1/8 is 3.5% slower).
int32_t probe_h8_for(int32_t vd, int32_t n, int64_t arcs, const int32_t *row_ptr)
{
    if (vd >= kRelabelMinVd) return 32;
    if (n <= 0 || arcs <= 0) return 8;
    double s2 = 0.0;
    for (int32_t v = 0; v < n; ++v) {
        const double d = (double)(row_ptr[v + 1] - row_ptr[v]);
        s2 += d * d;
    }
    const double kappa = (double)n * s2 / ((double)arcs * (double)arcs);
    return (int32_t)std::min(8L, std::max(1L, std::lround(8.0 / kappa)));
}

// A graph resident on the device, plus what depends on the graph only.
// On a high-diameter graph the device arrays use an internal vertex order
// (relabel_for_locality); d_perm maps original to internal ids, d_iperm back,
// and d_colo holds each internal row's neighbours as original ids (the row
// order is the original one, ascending in original id).  Null: identity.
struct GraphData {
    int32_t n = 0;
    int64_t arcs = 0;
    int32_t max_deg = 0;
    int32_t vd = 1;
    int32_t ncomp = 0;
    int32_t probe_h8 = 8;  // automatic meeting-probe constant (probe_h8_for)
    int device = 0;  // the HIP device holding the arrays
    int32_t *d_row_ptr = nullptr, *d_col = nullptr, *d_comp = nullptr;
    int32_t *d_colo = nullptr, *d_perm = nullptr, *d_iperm = nullptr;
    std::vector<int32_t> h_perm;  // host copy of d_perm (empty: identity)
    ~GraphData()
    {
        dev_free(d_row_ptr);
        dev_free(d_col);
        dev_free(d_comp);
        dev_free(d_colo);
        dev_free(d_perm);
        dev_free(d_iperm);
    }
};

// Components and the vertex-diameter bound on the device (kadabra_prep.hip):
// per component, a BFS from its maximum-degree vertex (lowest id on ties)
// reaches everything within ecc levels, and every shortest path there has at
// most 2 ecc edges, so VD = max (2 ecc + 1) = 2 (deepest level of one BFS from
// all roots) + 1 (Section 2.3, Appendix C.1).  d_comp receives each vertex's
// component (its smallest vertex id).
int gpu_preprocess(GraphData &gd, hipStream_t s)
{
    const int32_t n = gd.n;
    constexpr int32_t kSmallMax = 8192;  // one workgroup runs levels up to this frontier size
    unsigned long long *key = nullptr;
    int32_t *dist = nullptr, *q0 = nullptr, *q1 = nullptr, *cnt = nullptr, *host = nullptr;
    struct Release {
        std::vector<void *> dev;
        int32_t **host;
        ~Release()
        {
            for (void *p : dev) dev_free(p);
            if (*host) (void)hipHostFree(*host);
        }
    } rel{{}, &host};
    HIP_OR_FAIL(alloc_n(&gd.d_comp, (size_t)n));
    HIP_OR_FAIL(alloc_n(&key, (size_t)n));
    rel.dev.push_back(key);
    HIP_OR_FAIL(alloc_n(&dist, (size_t)n));
    rel.dev.push_back(dist);
    HIP_OR_FAIL(alloc_n(&q0, (size_t)n));
    rel.dev.push_back(q0);
    HIP_OR_FAIL(alloc_n(&q1, (size_t)n));
    rel.dev.push_back(q1);
    HIP_OR_FAIL(alloc_n(&cnt, 8));  // [0], [1] queue sizes, [2] components, [4..6] one-workgroup state
    rel.dev.push_back(cnt);
    HIP_OR_FAIL(hipHostMalloc((void **)&host, 8 * sizeof(int32_t), hipHostMallocDefault));
    HIP_OR_FAIL(kd::launch_fill_u32((uint32_t *)key, 2 * (size_t)n, 0u, s));
    HIP_OR_FAIL(kd::launch_fill_u32((uint32_t *)cnt, 8, 0u, s));
    HIP_OR_FAIL(kd::launch_cc(gd.d_row_ptr, gd.d_col, n, gd.d_comp, s));
    HIP_OR_FAIL(kd::launch_bfs_roots(gd.d_row_ptr, gd.d_comp, n, key, dist, q0, cnt, s));
    HIP_OR_FAIL(hipMemcpyAsync(host, cnt, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    gd.ncomp = host[2];
    int32_t fn = host[0], level = 0, which = 0;
    if (fn != gd.ncomp || fn < 1)
        return fail(KADABRA_EDEVICE, "preprocessing found %d roots for %d components", fn, gd.ncomp);
    while (fn > 0) {
        if (fn <= kSmallMax) {
            host[4] = fn;
            host[5] = level;
            host[6] = which;
            HIP_OR_FAIL(hipMemcpyAsync(cnt + 4, host + 4, 3 * sizeof(int32_t), hipMemcpyHostToDevice, s));
            HIP_OR_FAIL(kd::launch_bfs_small(gd.d_row_ptr, gd.d_col, dist, q0, q1, cnt + 4, kSmallMax, s));
            HIP_OR_FAIL(hipMemcpyAsync(host + 4, cnt + 4, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            HIP_OR_FAIL(hipStreamSynchronize(s));
            fn = host[4];
            level = host[5];
            which = host[6];
        } else {
            host[which] = fn;
            host[which ^ 1] = 0;
            HIP_OR_FAIL(hipMemcpyAsync(cnt, host, 2 * sizeof(int32_t), hipMemcpyHostToDevice, s));
            HIP_OR_FAIL(kd::launch_bfs_level(gd.d_row_ptr, gd.d_col, which ? q1 : q0, cnt + which, fn, level, dist,
                                             which ? q0 : q1, cnt + (which ^ 1), s));
            HIP_OR_FAIL(hipMemcpyAsync(host, cnt, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            HIP_OR_FAIL(hipStreamSynchronize(s));
            fn = host[which ^ 1];
            level += 1;
            which ^= 1;
        }
        if (fn < 0 || fn > n || level > n) return fail(KADABRA_EDEVICE, "preprocessing BFS out of range");
    }
    // the frontier emptied after `level` expansions: the deepest level is level - 1
    gd.vd = 2 * std::max(level - 1, 0) + 1;
    return KADABRA_OK;
}

// Balanced delta_L(v), delta_U(v) (Section 2.3 bounds only their sum over the
// vertices; this library spends delta/2 on it, the omega cap the other half).
// From the first phase's count histogram h(k) = #{v : c1(v) = k}, k <= m1:
//   - planning value b(k) = (k + 1) / m1;
//   - at a target count t, the largest log(1/delta) with f <= eps (Appendix
//     B) is L_f = t eps^2 / (q + 2 eps af), af = 1/3 - w/t, q = 2 b w / t,
//     unbounded when the denominator is <= 0 (f then stays below eps for every
//     constant); L_g the same with ag = 1/3 + w/t;
//   - S(t) = sum over the rows with h(k) > 0, ascending k, of
//     h(k) (exp(-L_f) + exp(-L_g)), added left to right;
//   - t* = bisection on [1, omega] (midpoint lo + (hi - lo) / 2) for
//     S(t) <= 0.9 (delta/2) (1 - 1e-6); ending at omega means no plan;
//   - log(1/delta_L) = -log(0.9 exp(-L_f(t*)) + 0.1 delta / (4 n)), and
//     log(1/delta_U) with L_g.
// Evaluated on the host in IEEE double in the order written (no contraction)
// with the C library's exp and log, so t* and every constant follow from the
// histogram alone.  Writes lcon[2k], lcon[2k + 1] for k = 0 .. m1 (rows no
// vertex has keep L) and returns t* (0: no plan, every constant L).
constexpr double kBalanceFloor = 0.1;  // share of the budget spread evenly

void balance_lfg(double b, double t, double w, double eps, double *lf, double *lg)
{
    const double af = 1.0 / 3.0 - w / t;
    const double ag = 1.0 / 3.0 + w / t;
    const double q = 2.0 * b * w / t;
    const double df = q + 2.0 * eps * af;
    const double dg = q + 2.0 * eps * ag;
    const double e2 = eps * eps;
    *lf = (df > 0.0) ? t * e2 / df : HUGE_VAL;
    *lg = t * e2 / dg;
}

int64_t balance_plan(const int32_t *hist, int64_t m1, int64_t omega, double eps, double delta, double L, int32_t n,
                     std::vector<double> *lcon)
{
    const double beta = kBalanceFloor;
    const double target = (1.0 - beta) * (delta / 2.0) * (1.0 - 1e-6);
    const double w = (double)omega, m = (double)m1;
    std::vector<int64_t> rows;  // k with h(k) > 0, ascending
    for (int64_t k = 0; k <= m1; ++k)
        if (hist[k] > 0) rows.push_back(k);
    int64_t lo = 1, hi = omega;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        const double t = (double)mid;
        double S = 0.0;
        for (const int64_t k : rows) {
            double lf, lg;
            balance_lfg(((double)k + 1.0) / m, t, w, eps, &lf, &lg);
            S += (double)hist[k] * (std::exp(-lf) + std::exp(-lg));
        }
        if (S <= target) hi = mid;
        else lo = mid + 1;
    }
    lcon->assign(2 * ((size_t)m1 + 1), L);
    if (lo >= omega) return 0;
    const double t = (double)lo;
    const double floor_share = beta * delta / (4.0 * (double)n);
    for (const int64_t k : rows) {
        double lf, lg;
        balance_lfg(((double)k + 1.0) / m, t, w, eps, &lf, &lg);
        (*lcon)[2 * (size_t)k] = -std::log((1.0 - beta) * std::exp(-lf) + floor_share);
        (*lcon)[2 * (size_t)k + 1] = -std::log((1.0 - beta) * std::exp(-lg) + floor_share);
    }
    return lo;
}

// One adaptive run.
struct Query {
    const GraphData *gd = nullptr;
    double eps = 0, delta = 0;
    uint64_t seed = 0;
    int64_t N = 1024;
    int nframes = 1;
    int epl = 1;                // epochs per sampling launch
    int nsets = 2;              // frame sets, 2 epl: epoch e uses set e mod nsets
    int64_t probe_min = -1;
    int64_t omega = 0;
    double L = 0;
    int64_t m1 = 0;             // balanced runs: first-phase samples (0: L for every vertex)
    // device buffers
    int32_t *counts = nullptr;
    int32_t *frames = nullptr;  // [nsets][nframes][n]
    size_t frames_len = 0;
    double *scores = nullptr;
    int32_t *c1 = nullptr;      // balanced runs: first-phase counters [n]
    void *plan_buf = nullptr;   // balanced runs: lcon [2 (m1 + 1)] doubles, then hist [m1 + 1]
    size_t plan_len = 0;        // bytes of plan_buf
    int cslot = -1;             // control block index in the runner
    // progress
    int64_t k = 0;              // epochs whose samplers were launched
    int64_t merged = 0;         // epochs whose merges were launched
    int64_t merged_prev = 0;    // ... before this round's merges
    int64_t lo = 0;             // first sample of epoch k + 1
    bool spec = false;          // epoch k's sampler was queued speculatively
    bool first_launched = false;  // the first phase and its plan are queued
    bool done = false;
    int status = KADABRA_OK;
    std::vector<int8_t> decisions;
    int64_t tau = 0;
    int decision = 0;
    int64_t work[kd::ST_COUNT] = {};
    int64_t work_first[kd::ST_COUNT] = {};  // the first phase's work counters
    int64_t plan_tau = 0;       // planned sample count t* (0: no plan)
    std::vector<int32_t> h_hist;  // balanced runs: host copies of the count histogram and
    std::vector<double> h_lcon;   // the constant table (read by the copy to the device)
    double ms_kernels = 0.0;    // sampler launches that did this query's work
    int64_t launches = 0;
    // resuming from a checkpoint: the counters of samples [0, resume_tau) (host),
    // resume_k boundaries already checked, the work counters so far
    const int32_t *resume_counts = nullptr;
    int64_t resume_k = 0, resume_tau = 0;
    int64_t resume_work[kd::ST_COUNT] = {};
    bool checkpointed = false;  // stopped at a boundary with the counters of [0, tau)
    std::chrono::steady_clock::time_point t_submit, t_done;

    int64_t bound(int64_t epoch) const { return std::min<int64_t>(epoch * N, omega); }
    int32_t set_of(int64_t epoch) const { return (int32_t)(epoch % nsets); }
    size_t frames_count() const { return (size_t)nsets * (size_t)nframes * (size_t)gd->n; }
    size_t plan_bytes() const { return m1 ? (size_t)(m1 + 1) * (2 * sizeof(double) + sizeof(int32_t)) : 0; }
    double *lcon() const { return (double *)plan_buf; }
    int32_t *hist() const { return (int32_t *)((char *)plan_buf + (size_t)(m1 + 1) * 2 * sizeof(double)); }
    ~Query()
    {
        dev_free(counts);
        dev_free(frames);
        dev_free(scores);
        dev_free(c1);
        dev_free(plan_buf);
    }
};

// The device engine shared by the queries of one handle or batch.
struct Runner {
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;
    int num_cu = 0;
    // sample slot pool
    kd::SlotState st{};
    int team = 0;
    int64_t slots = 0;
    unsigned long long *d_claim = nullptr;
    uint64_t claim_next = 0;
    bool pool_dirty = true;
    // control blocks (one per concurrent query) and their pinned mirror
    kd::Control *d_ctl = nullptr;
    kd::Control *h_ctl = nullptr;
    int ctl_cap = 0;
    std::vector<int> free_cslots;
    // launch tables: a ring of device tables and pinned staging copies
    static constexpr int RING = 8;
    int table_cap = 0;
    kd::QueryDesc *d_qt[RING] = {};
    kd::QueryDesc *h_qt[RING] = {};
    kd::MergeDesc *d_mt[RING] = {};
    kd::MergeDesc *h_mt[RING] = {};
    int ring_pos = 0;
    hipEvent_t ev_round = nullptr;
    std::vector<hipEvent_t> ev_pool;   // every event created
    std::vector<hipEvent_t> ev_free;   // those not recording a launch in flight
    std::atomic<int> cancel{0};

    ~Runner()
    {
        (void)hipStreamSynchronize(stream);
        release_pool();
        dev_release(d_claim);
        dev_release(d_ctl);
        if (h_ctl) (void)hipHostFree(h_ctl);
        for (int r = 0; r < RING; ++r) {
            dev_free(d_qt[r]);
            dev_free(d_mt[r]);
            if (h_qt[r]) (void)hipHostFree(h_qt[r]);
            if (h_mt[r]) (void)hipHostFree(h_mt[r]);
        }
        if (ev_round) (void)hipEventDestroy(ev_round);
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
        if (own_stream) (void)hipStreamDestroy(own_stream);
    }

    int init()
    {
        hipError_t e;
        int dev = 0;
        if ((e = hipGetDevice(&dev)) != hipSuccess)
            return fail(KADABRA_EDEVICE, "no HIP device: %s", hipGetErrorString(e));
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) num_cu = prop.multiProcessorCount;
        HIP_OR_FAIL(hipStreamCreateWithFlags(&own_stream, hipStreamNonBlocking));
        stream = own_stream;
        // only waited for, never timed
        HIP_OR_FAIL(hipEventCreateWithFlags(&ev_round, hipEventDisableTiming));
        HIP_OR_FAIL(alloc_n(&d_claim, 1));
        // zeroed on the runner's stream and waited for: every later launch,
        // on whichever stream, sees the counter at claim_next = 0
        HIP_OR_FAIL(kd::launch_fill_u32((uint32_t *)d_claim, 2, 0u, own_stream));
        HIP_OR_FAIL(hipStreamSynchronize(own_stream));
        return KADABRA_OK;
    }

    void release_pool()
    {
        dev_release(st.code);
        dev_release(st.sigma);
        dev_release(st.ball);
        dev_release(st.meet);
        dev_release(st.meetw);
        dev_release(st.loff);
        st = kd::SlotState{};
        team = 0;
        slots = 0;
        pool_dirty = true;
    }

    // A pool of `sl` slots for graphs of up to nstride vertices and lcap levels.
    int ensure_pool(int tm, int64_t sl, int64_t nstride, int32_t lcap, int64_t *fc)
    {
        if (st.code && team == tm && slots == sl && st.nstride >= nstride && st.lcap >= lcap)
            return KADABRA_OK;
        release_pool();
        const size_t S = (size_t)sl, ns = (size_t)nstride;
        const int32_t cs = code_stride_for(nstride);
        HIP_OR_FAIL(alloc_n(&st.code, S * (size_t)cs, fc));
        HIP_OR_FAIL(alloc_n(&st.sigma, S * 2 * ns, fc));
        HIP_OR_FAIL(alloc_n(&st.ball, S * 2 * ns, fc));
        HIP_OR_FAIL(alloc_n(&st.meet, S * ns, fc));
        HIP_OR_FAIL(alloc_n(&st.meetw, S * ns, fc));
        HIP_OR_FAIL(alloc_n(&st.loff, S * 2 * (size_t)lcap, fc));
        st.nstride = nstride;
        st.lcap = lcap;
        st.code_stride = cs;
        team = tm;
        slots = sl;
        pool_dirty = true;
        return KADABRA_OK;
    }

    int clear_pool_if_dirty()
    {
        if (!pool_dirty) return KADABRA_OK;
        // code words start at zero (a sample clears the words it set); sigma
        // needs no initial value (a sample writes it before reading it)
        HIP_OR_FAIL(kd::launch_fill_u32(st.code, (size_t)slots * st.code_stride, 0u, stream));
        pool_dirty = false;
        return KADABRA_OK;
    }

    int ensure_tables(int cap, int64_t *fc)
    {
        if (cap <= table_cap && cap <= ctl_cap) return KADABRA_OK;
        HIP_OR_FAIL(hipStreamSynchronize(stream));
        const int ncap = std::max({cap, 2 * table_cap, 1});
        for (int r = 0; r < RING; ++r) {
            dev_release(d_qt[r]);
            dev_release(d_mt[r]);
            if (h_qt[r]) (void)hipHostFree(h_qt[r]);
            if (h_mt[r]) (void)hipHostFree(h_mt[r]);
            h_qt[r] = nullptr;
            h_mt[r] = nullptr;
            // a query's first phase takes a second sampling descriptor
            HIP_OR_FAIL(alloc_n(&d_qt[r], 2 * (size_t)ncap, fc));
            HIP_OR_FAIL(alloc_n(&d_mt[r], (size_t)ncap, fc));
            HIP_OR_FAIL(hipHostMalloc((void **)&h_qt[r], 2 * (size_t)ncap * sizeof(kd::QueryDesc),
                                      hipHostMallocDefault));
            HIP_OR_FAIL(hipHostMalloc((void **)&h_mt[r], (size_t)ncap * sizeof(kd::MergeDesc), hipHostMallocDefault));
        }
        table_cap = ncap;
        if (ncap > ctl_cap) {
            // control blocks move: only while no query holds one
            if (ctl_cap > 0 && (int)free_cslots.size() != ctl_cap)
                return fail(KADABRA_ESTATE, "control blocks in use");
            dev_release(d_ctl);
            if (h_ctl) (void)hipHostFree(h_ctl);
            h_ctl = nullptr;
            HIP_OR_FAIL(alloc_n(&d_ctl, (size_t)ncap, fc));
            HIP_OR_FAIL(hipHostMalloc((void **)&h_ctl, (size_t)ncap * sizeof(kd::Control), hipHostMallocDefault));
            ctl_cap = ncap;
            free_cslots.clear();
            for (int c = ncap - 1; c >= 0; --c) free_cslots.push_back(c);
        }
        return KADABRA_OK;
    }

    hipEvent_t take_event()
    {
        if (!ev_free.empty()) {
            hipEvent_t e = ev_free.back();
            ev_free.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        ev_pool.push_back(e);
        return e;
    }

    size_t pool_bytes() const { return st.code ? (size_t)slots * slot_bytes(st.nstride, st.lcap) : 0; }

    // Mapping for a set of queries (never changes a result).  The automatic
    // slot count is capped at half of the device memory that is free or held
    // by this runner's own pool, so repeated runs keep the same pool.
    void choose_mapping(const Params &p, int64_t nmax, int32_t lcap, int *tm, int64_t *sl) const
    {
        int t = p.team ? p.team : 256;
        int64_t s = p.slots;
        if (s == 0) {
            s = (int64_t)std::max(num_cu, 1) * ((t == 512) ? 2 : (t == 256) ? 4 : 8);
            size_t free_b = 0, total_b = 0;
            if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b > 0) {
                free_b += pool_bytes();
                const int64_t fit = (int64_t)((free_b / 2) / slot_bytes(nmax, lcap));
                s = std::min(s, std::max<int64_t>(fit, 1));
            }
        }
        *tm = t;
        *sl = std::max<int64_t>(s, 1);
    }

    int start_query(Query &q, int64_t *fc);
    void finish_query(Query &q);
    // admit: may append new queries at every round (continuous batching);
    // on_done: called for each query once its result is final and the runner
    // holds no further reference to it.
    int run(std::vector<Query *> &queries, const Params &p,
            const std::function<void(std::vector<Query *> &)> &admit = nullptr,
            int64_t sample_cap = -1, int64_t *fail_countdown = nullptr,
            const std::function<void(Query *)> &on_done = nullptr);

  private:
    std::vector<Query *> live_;  // queries the current run has started
    int run_rounds(std::vector<Query *> &queries, const Params &p,
                   const std::function<void(std::vector<Query *> &)> &admit, int64_t sample_cap,
                   int64_t *fail_countdown, const std::function<void(Query *)> &on_done);
};

int Runner::start_query(Query &q, int64_t *fc)
{
    q.done = false;  // from here on the runner owns the query until finish_query
    q.status = KADABRA_OK;
    const size_t n = (size_t)q.gd->n;
    if (!q.counts) HIP_OR_FAIL(alloc_n(&q.counts, n, fc));
    if (q.frames_len != q.frames_count()) {
        dev_release(q.frames);
        q.frames_len = 0;
        HIP_OR_FAIL(alloc_n(&q.frames, q.frames_count(), fc));
        q.frames_len = q.frames_count();
    }
    if (q.m1 > 0) {
        if (!q.c1) HIP_OR_FAIL(alloc_n(&q.c1, n, fc));
        if (q.plan_len != q.plan_bytes()) {
            dev_release(q.plan_buf);
            q.plan_len = 0;
            HIP_OR_FAIL(alloc_n((char **)&q.plan_buf, q.plan_bytes(), fc));
            q.plan_len = q.plan_bytes();
        }
    }
    if (free_cslots.empty()) return fail(KADABRA_ESTATE, "no free control block");
    q.cslot = free_cslots.back();
    free_cslots.pop_back();
    // counters, frames, control block (and the balancing buffers): one launch
    kd::ZeroRegions z{};
    static_assert(sizeof(kd::Control) % 4 == 0, "the control block is cleared as 32-bit words");
    static_assert(kd::kMaxZeroRegions >= 5, "counters, frames, control block, c1, histogram");
    auto zero = [&](void *p, size_t words) {
        z.ptr[z.n] = (uint32_t *)p;
        z.count[z.n] = words;
        ++z.n;
    };
    zero(q.counts, n);
    zero(q.frames, q.frames_count());
    zero(d_ctl + q.cslot, sizeof(kd::Control) / 4);
    if (q.m1 > 0) {
        zero(q.c1, n);
        zero(q.hist(), (size_t)(q.m1 + 1));
    }
    HIP_OR_FAIL(kd::launch_zero_regions(z, stream));
    q.k = q.merged = q.merged_prev = q.lo = 0;
    q.checkpointed = false;
    if (q.resume_counts) {
        // after the zero fill in stream order: the counters and work so far
        HIP_OR_FAIL(hipMemcpyAsync(q.counts, q.resume_counts, n * sizeof(int32_t), hipMemcpyHostToDevice, stream));
        HIP_OR_FAIL(hipMemcpyAsync(d_ctl[q.cslot].stats_total, q.resume_work, sizeof q.resume_work,
                                   hipMemcpyHostToDevice, stream));
        HIP_OR_FAIL(hipStreamSynchronize(stream));  // the host arrays may go away after the call
    }
    q.spec = false;
    q.first_launched = false;
    q.plan_tau = 0;
    for (auto &w : q.work_first) w = 0;
    q.done = false;
    q.status = KADABRA_OK;
    q.decisions.clear();
    q.tau = 0;
    q.decision = 0;
    q.ms_kernels = 0.0;
    q.launches = 0;
    for (auto &w : q.work) w = 0;
    if (q.resume_counts) {
        q.k = q.merged = q.merged_prev = q.resume_k;
        q.lo = q.resume_tau;
        q.tau = q.resume_tau;
        q.decisions.assign((size_t)q.resume_k, (int8_t)0);
    }
    return KADABRA_OK;
}

void Runner::finish_query(Query &q)
{
    q.done = true;
    q.t_done = std::chrono::steady_clock::now();
    if (q.cslot >= 0) {
        free_cslots.push_back(q.cslot);
        q.cslot = -1;
    }
}

// The round loop (see the file header).  `admit` may append new queries at
// every round (continuous batching); sample_cap >= 0 stops every query after
// that many samples without checks (autotuning trials).
int Runner::run(std::vector<Query *> &queries, const Params &p,
                const std::function<void(std::vector<Query *> &)> &admit, int64_t sample_cap,
                int64_t *fail_countdown, const std::function<void(Query *)> &on_done)
{
    live_.clear();
    const int rc = run_rounds(queries, p, admit, sample_cap, fail_countdown, on_done);
    // a run that ended early (a failed device call) still returns every
    // control block and marks its unfinished queries failed
    for (Query *q : live_)
        if (!q->done) {
            if (q->status == KADABRA_OK) q->status = rc != KADABRA_OK ? rc : KADABRA_EDEVICE;
            finish_query(*q);
        }
    live_.clear();
    return rc;
}

int Runner::run_rounds(std::vector<Query *> &queries, const Params &p,
                       const std::function<void(std::vector<Query *> &)> &admit, int64_t sample_cap,
                       int64_t *fail_countdown, const std::function<void(Query *)> &on_done)
{
    std::vector<Query *> active;
    auto take_new = [&](std::vector<Query *> &incoming) -> int {
        for (Query *q : incoming) {
            live_.push_back(q);
            OK_OR_RETURN(start_query(*q, fail_countdown));
            active.push_back(q);
        }
        incoming.clear();
        return KADABRA_OK;
    };
    {
        std::vector<Query *> first = queries;
        OK_OR_RETURN(take_new(first));
    }
    OK_OR_RETURN(clear_pool_if_dirty());
    // a sampler launch and the queries (with epochs) it carried, for timing
    struct Launch {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        std::vector<std::pair<Query *, int64_t>> items;
    };
    std::deque<Launch> pend;  // launched, not yet accounted
    // a finished launch's time goes to the queries whose merged epochs it carried
    auto account = [&](Launch &L) -> int {
        float ms = 0.f;
        HIP_OR_FAIL(hipEventElapsedTime(&ms, L.e0, L.e1));
        for (auto &it : L.items) {
            Query *q = it.first;
            if (q && it.second <= (int64_t)q->decisions.size()) {
                q->ms_kernels += ms / (double)L.items.size();
                q->launches += 1;
            }
        }
        ev_free.push_back(L.e0);
        ev_free.push_back(L.e1);
        return KADABRA_OK;
    };

    auto launch_sampler = [&](std::vector<Query *> &qs, bool speculative) -> int {
        if (qs.empty()) return KADABRA_OK;
        const int r = ring_pos;
        ring_pos = (ring_pos + 1) % RING;
        kd::QueryDesc *h = h_qt[r];
        int64_t total = 0;
        size_t nd = 0;
        Launch L;
        std::vector<Query *> planned;  // queries whose first phase rides in this launch
        for (size_t x = 0; x < qs.size(); ++x) {
            Query &q = *qs[x];
            int epochs_now = q.epl;
            if (q.m1 > 0 && !q.first_launched && !speculative && sample_cap < 0) {
                // a balanced query's first launch: the first phase, claimed
                // first and added into c1, then one check interval only (the
                // run is planned to stop early, so its first check should
                // come as soon as possible)
                kd::QueryDesc &d = h[nd++];
                d = kd::QueryDesc{};
                d.row_ptr = q.gd->d_row_ptr;
                d.col = q.gd->d_col;
                d.comp = q.gd->d_comp;
                d.perm = q.gd->d_perm;
                d.iperm = q.gd->d_iperm;
                d.colo = q.gd->d_colo;
                d.frames = q.c1;
                d.ctl = d_ctl + q.cslot;
                d.seed = q.seed;
                d.lo = INT64_MIN;  // sample m draws index (uint64) lo + m = kFirstPhaseBase + m
                d.hi = INT64_MIN + q.m1;
                d.epoch_len = 1;
                d.claim_begin = total;
                d.probe_min = q.probe_min;
                d.probe_h8 = q.gd->probe_h8;
                d.probe_quit = q.gd->vd >= kRelabelMinVd ? 1 : 0;
                d.num_arcs = q.gd->arcs;
                d.n = q.gd->n;
                d.nframes = 1;
                d.nsets = 1;
                d.gate = -1;
                d.stat_set = kd::kFirstSet;
                static_assert((uint64_t)INT64_MIN == kd::kFirstPhaseBase, "first-phase index base");
                total += q.m1;
                q.first_launched = true;
                planned.push_back(&q);
                epochs_now = 1;
            }
            // the next epl epochs (fewer where omega or the sample cap ends them);
            // callers pass only queries with samples left
            int64_t epoch = q.k, hi = q.lo;
            for (int j = 0; j < epochs_now && hi < q.omega && (sample_cap < 0 || hi < sample_cap); ++j) {
                // the interval cut short by omega is never joined to earlier ones:
                // it is reached only if every earlier check fails
                if (j > 0 && sample_cap < 0 && (epoch + 1) * q.N > q.omega) break;
                ++epoch;
                hi = q.bound(epoch);
                if (sample_cap >= 0) hi = std::min(hi, sample_cap);
            }
            kd::QueryDesc &d = h[nd++];
            d = kd::QueryDesc{};
            d.stat_set = -1;
            d.row_ptr = q.gd->d_row_ptr;
            d.col = q.gd->d_col;
            d.comp = q.gd->d_comp;
            d.perm = q.gd->d_perm;
            d.iperm = q.gd->d_iperm;
            d.colo = q.gd->d_colo;
            d.frames = q.frames;
            d.ctl = d_ctl + q.cslot;
            d.seed = q.seed;
            d.lo = q.lo;
            d.hi = hi;
            d.epoch_len = q.N;
            d.claim_begin = total;
            d.probe_min = q.probe_min;
            d.probe_h8 = q.gd->probe_h8;
            d.probe_quit = q.gd->vd >= kRelabelMinVd ? 1 : 0;
            d.num_arcs = q.gd->arcs;
            d.n = q.gd->n;
            d.nframes = q.nframes;
            d.nsets = q.nsets;
            d.gate = speculative ? q.set_of(q.k) : -1;
            total += hi - q.lo;
            L.items.push_back({&q, q.k + 1});  // the launch's first epoch
            q.k = epoch;
            q.lo = hi;
            q.spec = speculative;
        }
        HIP_OR_FAIL(hipMemcpyAsync(d_qt[r], h, nd * sizeof(kd::QueryDesc), hipMemcpyHostToDevice, stream));
        kd::SampleArgs sa{};
        sa.q = d_qt[r];
        sa.nq = (int32_t)nd;
        sa.gated = 1;
        for (size_t k = 0; k < nd; ++k) sa.gated &= h[k].gate >= 0 ? 1 : 0;
        sa.total = total;
        sa.claim = d_claim;
        sa.claim_base = claim_next;
        sa.st = st;
        // test hook: a smaller level capacity trips the sampler's level-bound
        // check (the level offsets of a slot then pack into a smaller stride)
        if (p.level_cap > 0 && p.level_cap < st.lcap) sa.st.lcap = p.level_cap;
        // no more workgroups than samples (a small or gated launch starts fewer)
        const int grid = (int)std::min<int64_t>(slots, std::max<int64_t>(total, 1));
        claim_next += (uint64_t)total + (uint64_t)grid;  // every workgroup makes one failing claim
        L.e0 = take_event();
        L.e1 = take_event();
        if (!L.e0 || !L.e1) return fail(KADABRA_EDEVICE, "event creation failed");
        HIP_OR_FAIL(hipEventRecord(L.e0, stream));
        bool mapped = false;
        for (Query *q : qs) mapped = mapped || q->gd->d_perm != nullptr;
        HIP_OR_FAIL(kd::launch_sample(team, grid, sa, mapped, p.probe_pull != 0, stream));
        HIP_OR_FAIL(hipEventRecord(L.e1, stream));
        pend.push_back(std::move(L));
        // the balanced constants, from the finished first phase, before any
        // check: the histograms on the device, the plans on the host (the C
        // library's exp and log)
        for (Query *q : planned) {
            HIP_OR_FAIL(kd::launch_hist(q->c1, q->gd->n, q->hist(), q->m1, d_ctl + q->cslot, stream));
            q->h_hist.resize((size_t)q->m1 + 1);
            HIP_OR_FAIL(hipMemcpyAsync(q->h_hist.data(), q->hist(), q->h_hist.size() * sizeof(int32_t),
                                       hipMemcpyDeviceToHost, stream));
        }
        if (!planned.empty()) HIP_OR_FAIL(hipStreamSynchronize(stream));
        for (Query *q : planned) {
            q->plan_tau = balance_plan(q->h_hist.data(), q->m1, q->omega, q->eps, q->delta, q->L, q->gd->n,
                                       &q->h_lcon);
            HIP_OR_FAIL(hipMemcpyAsync(q->lcon(), q->h_lcon.data(), q->h_lcon.size() * sizeof(double),
                                       hipMemcpyHostToDevice, stream));
        }
        return KADABRA_OK;
    };

    // Merges the launched epochs merged+1 .. k of every query in order: one
    // merge-and-check launch per position, each boundary gated on the one
    // before it (the first follows a boundary the host has seen continue).
    auto launch_merge = [&](std::vector<Query *> &qs) -> int {
        if (qs.empty()) return KADABRA_OK;
        int64_t depth = 0;
        for (Query *q : qs) {
            q->merged_prev = q->merged;
            depth = std::max(depth, q->k - q->merged);
        }
        for (int64_t j = 1; j <= depth; ++j) {
            const int r = ring_pos;
            ring_pos = (ring_pos + 1) % RING;
            kd::MergeDesc *h = h_mt[r];
            int32_t blocks = 0, nq = 0;
            for (Query *qp : qs) {
                Query &q = *qp;
                if (q.k - q.merged_prev < j) continue;
                const int64_t epoch = q.merged_prev + j;
                int64_t tau = q.bound(epoch);
                if (sample_cap >= 0) tau = std::min(tau, sample_cap);
                kd::MergeDesc &m = h[nq++];
                m.counts = q.counts;
                m.set = q.set_of(epoch);
                m.frames = q.frames + (size_t)m.set * q.nframes * (size_t)q.gd->n;
                m.ctl = d_ctl + q.cslot;
                m.perm = q.gd->d_perm;
                m.c1 = q.first_launched ? q.c1 : nullptr;
                m.lcon = q.first_launched ? q.lcon() : nullptr;
                m.m1 = q.first_launched ? q.m1 : 0;
                m.tau = tau;
                m.omega = q.omega;
                m.L = q.L;
                m.eps = q.eps;
                m.n = q.gd->n;
                m.nframes = q.nframes;
                m.gate = (j == 1) ? -1 : q.set_of(epoch - 1);
                m.do_check = (sample_cap < 0 && tau < q.omega) ? 1 : 0;
                m.block_begin = blocks;
                blocks += kd::merge_blocks_for(q.gd->n);
            }
            kd::MergeArgs ma{};
            if (nq == 1) {  // in the launch's arguments
                ma.m = nullptr;
                ma.one = h[0];
            } else {
                HIP_OR_FAIL(hipMemcpyAsync(d_mt[r], h, (size_t)nq * sizeof(kd::MergeDesc),
                                           hipMemcpyHostToDevice, stream));
                ma.m = d_mt[r];
            }
            ma.nq = nq;
            ma.nblocks = blocks;
            HIP_OR_FAIL(kd::launch_merge_check(ma, stream));
        }
        for (Query *q : qs) q->merged = q->k;
        return KADABRA_OK;
    };

    int status = KADABRA_OK;
    while (!active.empty()) {
        // samplers for queries whose next epoch is not queued yet
        std::vector<Query *> fresh;
        for (Query *q : active)
            if (q->merged == q->k) fresh.push_back(q);
        OK_OR_RETURN(launch_sampler(fresh, false));
        OK_OR_RETURN(launch_merge(active));
        HIP_OR_FAIL(hipMemcpyAsync(h_ctl, d_ctl, (size_t)ctl_cap * sizeof(kd::Control), hipMemcpyDeviceToHost, stream));
        HIP_OR_FAIL(hipEventRecord(ev_round, stream));
        // speculative next epoch for queries that may continue
        std::vector<Query *> spec;
        if (p.overlap)
            for (Query *q : active) {
                const bool capped = sample_cap >= 0 && q->lo >= sample_cap;
                if (q->lo < q->omega && !capped) spec.push_back(q);
            }
        OK_OR_RETURN(launch_sampler(spec, true));
        const size_t in_flight = spec.empty() ? 0 : 1;  // this round's speculative launch
        HIP_OR_FAIL(hipEventSynchronize(ev_round));
        // decisions of this round's boundaries
        std::vector<Query *> still, finished;
        for (Query *q : active) {
            const kd::Control &c = h_ctl[q->cslot];
            int dec = 0;
            if (c.err) {
                static const char *const site[] = {"?", "more BFS levels than the vertex-diameter bound",
                                                   "no predecessor on a BFS level", "empty frontier",
                                                   "a first-phase counter above the first-phase samples"};
                q->status = fail(KADABRA_EDEVICE,
                                 "device-side invariant failure in the sampler (%s) at sample %lld of the "
                                 "query with seed %llu on a graph of %d vertices",
                                 site[(c.err >= 1 && c.err <= 4) ? c.err : 0], (long long)c.err_sample,
                                 (unsigned long long)q->seed, q->gd->n);
                status = q->status;
                pool_dirty = true;
                q->tau = q->bound(q->merged);
            } else {
                // this round's boundaries in order, up to the first that stops
                for (int64_t e = q->merged_prev + 1; e <= q->merged && dec == 0; ++e) {
                    int64_t tau = q->bound(e);
                    if (sample_cap >= 0) tau = std::min(tau, sample_cap);
                    if ((sample_cap >= 0 && tau >= sample_cap) || tau == q->omega) dec = 2;
                    else if (c.viol[q->set_of(e)] == 0) dec = 1;
                    q->tau = tau;
                    q->decisions.push_back((int8_t)dec);
                }
            }
            if (dec == 0 && q->status == KADABRA_OK && p.stop_after > 0 && sample_cap < 0 && q->m1 == 0 &&
                (int64_t)q->decisions.size() - q->resume_k >= p.stop_after) {
                // stop here with a consistent state: every merged boundary was
                // decided "continue", so the counters hold exactly [0, tau)
                q->status = fail(KADABRA_ECANCELED, "stopped after %lld boundaries at %lld samples (checkpoint)",
                                 (long long)q->decisions.size(), (long long)q->tau);
                q->checkpointed = true;
            }
            if (dec || q->status != KADABRA_OK) {
                q->decision = dec;
                for (int w = 0; w < kd::ST_COUNT; ++w) q->work[w] = c.stats_total[w];
                for (int w = 0; w < kd::ST_COUNT; ++w) q->work_first[w] = c.stats[kd::kFirstSet][w];
                finished.push_back(q);
            } else {
                still.push_back(q);
            }
        }
        // account the launches that have completed (all but this round's
        // speculative one), drop finished queries from it, hand them over
        while (pend.size() > in_flight) {
            OK_OR_RETURN(account(pend.front()));
            pend.pop_front();
        }
        if (cancel.load() && status == KADABRA_OK) {
            for (Query *q : still) {
                q->status = fail(KADABRA_ECANCELED, "run canceled at %lld samples", (long long)q->tau);
                // the boundaries of this round were all decided "continue": a
                // consistent state to resume from (uniform constants only)
                const kd::Control &c = h_ctl[q->cslot];
                for (int w = 0; w < kd::ST_COUNT; ++w) q->work[w] = c.stats_total[w];
                q->checkpointed = q->m1 == 0 && sample_cap < 0;
                finished.push_back(q);
            }
            still.clear();
            status = KADABRA_ECANCELED;
        }
        if (status != KADABRA_OK)
            for (Query *q : still) {  // cut short by another query's failure
                if (q->status == KADABRA_OK) q->status = status;
                finished.push_back(q);
            }
        // a finished query leaves every list of the runner before on_done hands
        // it back: its owner may free it from then on
        for (Query *q : finished) {
            for (Launch &L : pend)
                for (auto &it : L.items)
                    if (it.first == q) it.first = nullptr;
            finish_query(*q);
        }
        if (!finished.empty())
            live_.erase(std::remove_if(live_.begin(), live_.end(), [](const Query *q) { return q->done; }),
                        live_.end());
        if (on_done)
            for (Query *q : finished) on_done(q);
        if (status != KADABRA_OK) break;
        active.swap(still);
        if (admit) {
            std::vector<Query *> incoming;
            admit(incoming);
            OK_OR_RETURN(take_new(incoming));
        }
    }
    HIP_OR_FAIL(hipStreamSynchronize(stream));
    while (!pend.empty()) {
        OK_OR_RETURN(account(pend.front()));
        pend.pop_front();
    }
    return status;
}

}  // namespace

struct kadabra_graph {
    GraphData gd;
    Params params;
    Runner runner;
    Query q;  // the last run
    bool have_result = false;
    double ms_total = 0.0;
};

struct kadabra_batch {
    Params params;
    Runner runner;
    std::vector<std::unique_ptr<Query>> queries;
    bool have_result = false;
    double ms_total = 0.0;
};

// A query submitted to a server: the run plus its ticket and budget charge.
struct Served : Query {
    int64_t ticket = 0;
    int64_t charge = 0;        // budget bytes held now
    int64_t frame_bytes = 0;   // part of the charge returned when sampling ends
    bool admitted = false;
    bool final_ = false;
    int readers = 0;           // result reads in progress (release waits for none)
    std::string err;
    std::chrono::steady_clock::time_point t_admit;
    double latency_ms = 0.0;
    int32_t graph = 0;         // index in the server's graphs
    double est_ms = 0.0;       // estimated device time of its first sampling launch
};

struct kadabra_server {
    Params params;
    Runner runner;
    std::vector<const GraphData *> graphs;
    int64_t nmax = 1;
    int32_t lcap = 3;
    int64_t budget = 0;
    int32_t max_active = 256;
    int device = 0;
    hipStream_t io = nullptr;  // result reads, beside the worker's stream
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Served *> pending;
    std::unordered_map<int64_t, std::unique_ptr<Served>> tickets;
    int64_t next_ticket = 1;
    // device buffers of finished or released queries, by size, for reuse
    std::unordered_map<size_t, std::vector<void *>> bins;
    int64_t in_use = 0, binned = 0;
    int64_t active = 0, peak_active = 0;
    int64_t submitted = 0, completed = 0, failed = 0;
    std::vector<double> lat;
    double queue_ms_sum = 0.0;
    int64_t queue_n = 0;
    bool started = false, stop = false;
    bool mapped = false;  // the pool matches params (fixed from the first run on)
    // Round work cap: queries are admitted (in submission order) only while the
    // estimated device time of the admitted queries' launches stays within
    // round_ms, except that a query is always admitted when nothing runs.  A
    // long query then runs without later arrivals in its launches (as it would
    // first come first served), and short ones are batched in short rounds.
    // Estimates come from a calibration launch per graph; they never change a
    // result.  0: no cap.
    double round_ms = 16.0;
    std::vector<double> ms_per_sample;  // per graph, from the calibration
    double active_est = 0.0;            // sum of est_ms over admitted, unfinished queries
    int broken = KADABRA_OK;
    std::string broken_err;
    std::thread worker;

    ~kadabra_server();
    // device bytes a query holds only while it samples: its frame sets and, for
    // a balanced run, the first-phase counters and the plan tables
    int64_t frame_bytes_of(const Query &q) const
    {
        const int64_t n = q.gd->n;
        int64_t b = n * 4 * 2 * params.epochs * (int64_t)params.frames;
        if (q.m1 > 0) b += n * 4 + (int64_t)q.plan_bytes();
        return b;
    }
    int64_t charge_of(const Query &q) const { return (int64_t)q.gd->n * (4 + 8) + frame_bytes_of(q); }
    void *take_bin(size_t bytes)
    {
        auto it = bins.find(bytes);
        if (it == bins.end() || it->second.empty()) return nullptr;
        void *p = it->second.back();
        it->second.pop_back();
        binned -= (int64_t)bytes;
        return p;
    }
    void put_bin(void *p, size_t bytes)
    {
        if (!p) return;
        bins[bytes].push_back(p);
        binned += (int64_t)bytes;
    }
    bool can_admit_locked() const
    {
        if (pending.empty() || active >= max_active || in_use + pending.front()->charge > budget) return false;
        return round_ms <= 0.0 || active == 0 || active_est + pending.front()->est_ms <= round_ms;
    }
    // estimated device time of a query's first sampling launch
    double estimate_ms(const Served &v) const
    {
        if ((size_t)v.graph >= ms_per_sample.size()) return 0.0;
        const int64_t first = std::min<int64_t>((int64_t)params.epochs * v.N, v.omega) + v.m1;
        return (double)first * ms_per_sample[(size_t)v.graph];
    }
    // Moves admissible queries (in submission order) to out; buffers that no
    // longer fit next to the admitted ones are handed back in to_free.
    void admit_locked(std::vector<Query *> &out, std::vector<void *> &to_free)
    {
        while (can_admit_locked()) {
            Served *v = pending.front();
            pending.pop_front();
            const size_t n = (size_t)v->gd->n;
            v->admitted = true;
            v->est_ms = estimate_ms(*v);
            active_est += v->est_ms;
            v->t_admit = std::chrono::steady_clock::now();
            queue_ms_sum += std::chrono::duration<double, std::milli>(v->t_admit - v->t_submit).count();
            queue_n += 1;
            in_use += v->charge;
            active += 1;
            peak_active = std::max(peak_active, active);
            v->counts = (int32_t *)take_bin(n * sizeof(int32_t));
            const size_t fl = v->frames_count();
            v->frames = (int32_t *)take_bin(fl * sizeof(int32_t));
            v->frames_len = v->frames ? fl : 0;
            v->scores = (double *)take_bin(n * sizeof(double));
            if (v->m1 > 0) {
                v->c1 = (int32_t *)take_bin(n * sizeof(int32_t));
                v->plan_buf = take_bin(v->plan_bytes());
                v->plan_len = v->plan_buf ? v->plan_bytes() : 0;
            }
            out.push_back(v);
        }
        for (auto &b : bins) {
            while (in_use + binned > budget && !b.second.empty()) {
                to_free.push_back(b.second.back());
                b.second.pop_back();
                binned -= (int64_t)b.first;
            }
        }
    }
};

namespace {

// First-phase samples of a query with cap omega under p (0: uniform constants).
int64_t first_phase_of(const Params &p, int64_t omega)
{
    return p.balance ? (p.balance_samples ? p.balance_samples : (omega + 19) / 20) : 0;
}

int make_query(Query &q, const GraphData &gd, const Params &p, double eps, double delta, uint64_t seed,
               int64_t N)
{
    if (!(eps > 0.0 && eps < 1.0)) return fail(KADABRA_EINVAL, "eps must be in (0, 1)");
    if (!(delta > 0.0 && delta < 1.0)) return fail(KADABRA_EINVAL, "delta must be in (0, 1)");
    if (N < 1 || N > INT32_MAX) return fail(KADABRA_EINVAL, "check_interval must be in [1, 2^31)");
    const int64_t omega = omega_of(gd.vd, eps, delta);
    if (omega > kMaxOmega || omega < 1)
        return fail(KADABRA_ERANGE, "omega = %lld samples exceeds the int32 counters", (long long)omega);
    q.gd = &gd;
    q.eps = eps;
    q.delta = delta;
    q.seed = seed;
    q.N = N;
    q.nframes = p.frames;
    q.epl = p.epochs;
    q.nsets = 2 * p.epochs;
    q.probe_min = p.probe_min;
    q.omega = omega;
    q.L = std::log(4.0 * (double)gd.n / delta);
    q.m1 = first_phase_of(p, omega);
    q.t_submit = std::chrono::steady_clock::now();
    return KADABRA_OK;
}

// Runs queries (all on graphs of up to nmax vertices) to completion.
int run_queries(Runner &R, std::vector<Query *> &qs, Params &p, int64_t sample_cap = -1)
{
    int64_t nmax = 1;
    int32_t lcap = 3;
    for (Query *q : qs) {
        nmax = std::max<int64_t>(nmax, q->gd->n);
        lcap = std::max(lcap, q->gd->vd + 2);  // a side reaches at most diameter <= VD - 1 levels
    }
    int tm;
    int64_t sl;
    R.choose_mapping(p, nmax, lcap, &tm, &sl);
    int64_t *fc = &p.fail_alloc;
    OK_OR_RETURN(R.ensure_pool(tm, sl, nmax, lcap, fc));
    OK_OR_RETURN(R.ensure_tables((int)qs.size(), fc));
    return R.run(qs, p, nullptr, sample_cap, fc);
}

void fill_stats(const Query &q, double ms_total, kadabra_stats *stats)
{
    memset(stats, 0, sizeof *stats);
    stats->tau = q.tau;
    stats->omega = q.omega;
    stats->vd_bound = q.gd->vd;
    stats->epochs = (int64_t)q.decisions.size();
    stats->decision = q.decision;
    stats->v_exp = q.work[kd::ST_VEXP];
    stats->e_scan = q.work[kd::ST_ESCAN];
    stats->e_bt = q.work[kd::ST_EBT];
    stats->path_interior = q.work[kd::ST_INTERIOR];
    stats->disconnected = q.work[kd::ST_DISCONN];
    stats->v_written = q.work[kd::ST_VMAT];
    stats->log_inv_delta = q.L;
    stats->ms_sampling = q.ms_kernels;
    stats->ms_total = ms_total;
    stats->ms_sample_kernels = q.ms_kernels;
    stats->sample_launches = q.launches;
    stats->first_samples = q.first_launched ? q.m1 : 0;
    stats->plan_tau = q.plan_tau;
    stats->first_v_exp = q.work_first[kd::ST_VEXP];
    stats->first_e_scan = q.work_first[kd::ST_ESCAN];
    stats->first_e_bt = q.work_first[kd::ST_EBT];
    stats->first_path_interior = q.work_first[kd::ST_INTERIOR];
    stats->first_disconnected = q.work_first[kd::ST_DISCONN];
}

int read_result(const Query &q, hipStream_t s, double *scores, int32_t *counts)
{
    Query &mq = const_cast<Query &>(q);
    const size_t n = (size_t)q.gd->n;
    if (scores) {
        if (!mq.scores) HIP_OR_FAIL(alloc_n(&mq.scores, n));
        HIP_OR_FAIL(kd::launch_scores(q.counts, mq.scores, q.gd->n, q.tau, s));
        HIP_OR_FAIL(hipMemcpyAsync(scores, mq.scores, n * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    if (counts) HIP_OR_FAIL(hipMemcpyAsync(counts, q.counts, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    return KADABRA_OK;
}

}  // namespace

namespace {

int ensure_graph_query(kadabra_graph *g, double eps, double delta, uint64_t seed)
{
    return make_query(g->q, g->gd, g->params, eps, delta, seed, g->params.check_interval);
}

// Trial-times mapping candidates on the first trial_samples samples of every
// query (no stop checks) and keeps the fastest in *p: the team (one, two or
// four wavefronts per sample), the samples in flight, the meeting probe on or
// off, then the epochs per launch for the best of those.  Results never depend
// on the mapping, so the choice cannot change any output.
int autotune(Runner &R, std::vector<Query *> &qs, Params &p, int64_t trial_samples)
{
    struct Cand {
        int team;
        int64_t slots_mul2;  // slots = auto * mul2 / 2
        int64_t probe;
        int epochs;          // 0: keep
    };
    const Cand cands[] = {{256, 2, -1, 0}, {256, 4, -1, 0}, {256, 1, -1, 0}, {128, 2, -1, 0}, {128, 1, -1, 0},
                          {64, 2, -1, 0},  {64, 4, -1, 0},  {256, 2, (int64_t)1 << 62, 0},
                          {64, 4, (int64_t)1 << 62, 0}};
    const Params base = p;
    double best = 1e300;
    Params best_p = p;
    int64_t nmax = 1;
    int32_t lcap = 3;
    for (Query *q : qs) {
        nmax = std::max<int64_t>(nmax, q->gd->n);
        lcap = std::max(lcap, q->gd->vd + 2);
    }
    // slots_mul2 > 0: slots = the automatic count * slots_mul2 / 2; 0: t.slots as given
    auto trial = [&](Params t, int64_t slots_mul2) -> int {
        for (Query *q : qs) {
            q->probe_min = t.probe_min;
            q->epl = t.epochs;
            q->nsets = 2 * t.epochs;
        }
        if (slots_mul2 > 0) {
            int tm;
            int64_t sl;
            t.slots = 0;
            R.choose_mapping(t, nmax, lcap, &tm, &sl);
            t.slots = std::max<int64_t>(1, sl * slots_mul2 / 2);
        }
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess &&
            (size_t)t.slots * slot_bytes(nmax, lcap) > free_b / 2)
            return KADABRA_OK;
        OK_OR_RETURN(run_queries(R, qs, t, trial_samples));  // warm-up: buffers, caches
        const auto t0 = std::chrono::steady_clock::now();
        OK_OR_RETURN(run_queries(R, qs, t, trial_samples));
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (ms < best) {
            best = ms;
            best_p = t;
        }
        return KADABRA_OK;
    };
    for (const Cand &c : cands) {
        Params t = base;
        t.team = c.team;
        t.probe_min = c.probe;
        OK_OR_RETURN(trial(t, c.slots_mul2));
    }
    // epochs per launch, on the best mapping so far (its slots are explicit)
    const int first_epochs = best_p.epochs;
    for (int e : {1, 2, 4}) {
        if (e == first_epochs) continue;
        Params t = best_p;
        t.epochs = e;
        OK_OR_RETURN(trial(t, 0));
    }
    p.team = best_p.team;
    p.slots = best_p.slots;
    p.probe_min = best_p.probe_min;
    p.epochs = best_p.epochs;
    for (Query *q : qs) {
        q->probe_min = p.probe_min;
        q->epl = p.epochs;
        q->nsets = 2 * p.epochs;
    }
    return KADABRA_OK;
}

// Device time per sample of each of the server's graphs: one launch of a
// fixed number of samples (a calibration seed, no checks) per graph, on the
// server's pool and mapping, after one warm-up launch.  Only admission uses
// it.  The estimates of pending queries are filled in.
int calibrate_server(kadabra_server *s)
{
    if (!s->mapped) {
        int tm;
        int64_t sl;
        s->runner.choose_mapping(s->params, s->nmax, s->lcap, &tm, &sl);
        OK_OR_RETURN(s->runner.ensure_pool(tm, sl, s->nmax, s->lcap, nullptr));
        s->mapped = true;
    }
    std::vector<double> ms(s->graphs.size(), 0.0);
    Params p = s->params;
    p.balance = 0;
    for (size_t g = 0; g < s->graphs.size(); ++g) {
        Query q;
        OK_OR_RETURN(make_query(q, *s->graphs[g], p, 0.01, 0.1, 0xCA11B8A7Eull, 1 << 30));
        const int64_t trial = std::min<int64_t>(2048, q.omega);
        for (int rep = 0; rep < (g == 0 ? 2 : 1); ++rep) {
            std::vector<Query *> qs{&q};
            const auto t0 = std::chrono::steady_clock::now();
            OK_OR_RETURN(s->runner.run(qs, p, nullptr, trial, nullptr, nullptr));
            ms[g] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() /
                    (double)trial;
        }
    }
    std::lock_guard<std::mutex> lk(s->mu);
    s->ms_per_sample = ms;
    return KADABRA_OK;
}

// The server's worker: waits for submissions, then runs the round loop for
// as long as any query is active, admitting new ones at every boundary.
void server_main(kadabra_server *s)
{
    (void)hipSetDevice(s->device);
    auto on_done = [s](Query *q) {
        Served *v = static_cast<Served *>(q);
        std::lock_guard<std::mutex> lk(s->mu);
        v->final_ = true;
        if (v->status != KADABRA_OK) {
            v->err = g_last_error;
            s->failed += 1;
        }
        v->latency_ms = std::chrono::duration<double, std::milli>(v->t_done - v->t_submit).count();
        s->lat.push_back(v->latency_ms);
        s->completed += 1;
        s->active -= 1;
        s->active_est = s->active > 0 ? std::max(0.0, s->active_est - v->est_ms) : 0.0;
        // the frames are free once the last merge has run (an epoch queued
        // speculatively for this query exits on the device without writing)
        s->put_bin(v->frames, v->frames_len * sizeof(int32_t));
        v->frames = nullptr;
        v->frames_len = 0;
        s->put_bin(v->c1, v->c1 ? (size_t)v->gd->n * sizeof(int32_t) : 0);
        s->put_bin(v->plan_buf, v->plan_len);
        v->c1 = nullptr;
        v->plan_buf = nullptr;
        v->plan_len = 0;
        s->in_use -= v->frame_bytes;
        v->charge -= v->frame_bytes;
        s->cv_done.notify_all();
    };
    auto admit = [s](std::vector<Query *> &incoming) {
        std::vector<void *> to_free;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (s->stop) s->runner.cancel.store(1);
            else s->admit_locked(incoming, to_free);
        }
        for (void *p : to_free) dev_free(p);
    };
    for (;;) {
        std::vector<Query *> first;
        std::vector<void *> to_free;
        if (s->ms_per_sample.empty() && s->round_ms > 0.0) {
            // wait for the first submission (parameters are fixed from then
            // on), then time a short calibration launch per graph
            {
                std::unique_lock<std::mutex> lk(s->mu);
                s->cv_work.wait(lk, [s] { return s->stop || !s->pending.empty(); });
                if (s->stop) break;
            }
            if (calibrate_server(s) != KADABRA_OK) {
                std::lock_guard<std::mutex> lk(s->mu);
                s->round_ms = 0.0;  // no estimates: admit without the cap
            }
        }
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [s] { return s->stop || s->can_admit_locked(); });
            if (s->stop) break;
            s->admit_locked(first, to_free);
        }
        for (void *p : to_free) dev_free(p);
        int rc = KADABRA_OK;
        if (!s->mapped) {
            int tm;
            int64_t sl;
            s->runner.choose_mapping(s->params, s->nmax, s->lcap, &tm, &sl);
            rc = s->runner.ensure_pool(tm, sl, s->nmax, s->lcap, nullptr);
            s->mapped = rc == KADABRA_OK;
        }
        if (rc == KADABRA_OK) rc = s->runner.run(first, s->params, admit, -1, nullptr, on_done);
        if (rc != KADABRA_OK && rc != KADABRA_ECANCELED) {
            // a device failure: every query still admitted fails with it and
            // the server accepts no more work
            std::lock_guard<std::mutex> lk(s->mu);
            s->broken = rc;
            s->broken_err = g_last_error;
            for (auto &t : s->tickets) {
                Served *v = t.second.get();
                if (v->admitted && !v->final_) {
                    v->status = rc;
                    v->err = g_last_error;
                    v->final_ = true;
                    v->t_done = std::chrono::steady_clock::now();
                    s->runner.finish_query(*v);
                    s->failed += 1;
                    s->completed += 1;
                    s->active -= 1;
                }
            }
            for (Served *v : s->pending) {
                v->status = rc;
                v->err = g_last_error;
                v->final_ = true;
                s->failed += 1;
                s->completed += 1;
            }
            s->pending.clear();
            s->cv_done.notify_all();
            break;
        }
    }
}

}  // namespace

kadabra_server::~kadabra_server()
{
    if (worker.joinable()) worker.join();
    if (io) {
        (void)hipStreamSynchronize(io);
        (void)hipStreamDestroy(io);
    }
    (void)hipStreamSynchronize(runner.stream);
    tickets.clear();
    for (auto &b : bins)
        for (void *p : b.second) dev_free(p);
}


// ---------------------------------------------------------------------------
// Run-time state in a static device array, for kadabra_run_static (callers
// that may not allocate).  The array is part of the code object, so every GPU
// the library runs on holds its own copy until the process ends.  Host code
// never uses the name `scratch` as an address: the device address of each
// GPU's copy comes from hipGetSymbolAddress, once per device.
// ---------------------------------------------------------------------------
constexpr size_t kStaticScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxStaticDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_dev[kMaxStaticDevices] = {};

// The device address of the current device's scratch array (looked up on the
// first call on that device, with it current).
int static_scratch(int dev, char **out)
{
    if (dev < 0 || dev >= kMaxStaticDevices) return fail(KADABRA_EDEVICE, "device %d beyond the static table", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(KADABRA_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_dev[dev] = (char *)p;
    }
    *out = g_scratch_dev[dev];
    return KADABRA_OK;
}

// Byte offsets of one static run's buffers in the scratch array: control
// block, claim counter, launch descriptor, two frame sets, then the slot pool.
struct StaticLayout {
    size_t ctl, claim, desc, frames, code, sigma, ball, meet, meetw, loff, end;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

StaticLayout static_layout(int64_t n, int32_t lcap, int64_t slots)
{
    const size_t S = (size_t)slots, ns = (size_t)n;
    StaticLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    L.ctl = take(sizeof(kd::Control));
    L.claim = take(sizeof(unsigned long long));
    L.desc = take(sizeof(kd::QueryDesc));
    L.frames = take(2 * ns * sizeof(int32_t));
    L.code = take(S * (size_t)code_stride_for(n) * sizeof(uint32_t));
    L.sigma = take(S * 2 * ns * sizeof(kd::Sigma));
    L.ball = take(S * 2 * ns * sizeof(int32_t));
    L.meet = take(S * ns * sizeof(int32_t));
    L.meetw = take(S * ns * sizeof(uint64_t));
    L.loff = take(S * 2 * (size_t)lcap * sizeof(int32_t));
    L.end = o;
    return L;
}

}  // namespace

namespace {


// Reverse Cuthill-McKee order: per component (in order of its smallest id), a
// BFS from a pseudo-peripheral vertex (of the deepest level of a BFS from the
// component's smallest id, the one of least degree, lowest id on ties) that
// queues each vertex's unplaced neighbours by (degree, id); the whole order is
// then reversed.  Returns order[k] = the original id of internal vertex k.
std::vector<int32_t> rcm_order(int32_t n, const int32_t *rp, const int32_t *col)
{
    auto deg = [&](int32_t v) { return rp[v + 1] - rp[v]; };
    std::vector<int32_t> order, q, nb;
    order.reserve((size_t)n);
    q.reserve((size_t)n);
    std::vector<int32_t> dist((size_t)n, -1);
    std::vector<char> placed((size_t)n, 0);
    for (int32_t seed = 0; seed < n; ++seed) {
        if (placed[(size_t)seed]) continue;
        q.clear();
        q.push_back(seed);
        dist[(size_t)seed] = 0;
        for (size_t h = 0; h < q.size(); ++h) {
            const int32_t u = q[h];
            for (int32_t e = rp[u]; e < rp[u + 1]; ++e) {
                const int32_t w = col[e];
                if (dist[(size_t)w] < 0) {
                    dist[(size_t)w] = dist[(size_t)u] + 1;
                    q.push_back(w);
                }
            }
        }
        const int32_t dmax = dist[(size_t)q.back()];
        int32_t start = -1;
        for (int32_t v : q)
            if (dist[(size_t)v] == dmax &&
                (start < 0 || deg(v) < deg(start) || (deg(v) == deg(start) && v < start)))
                start = v;
        for (int32_t v : q) dist[(size_t)v] = -1;
        const size_t base = order.size();
        order.push_back(start);
        placed[(size_t)start] = 1;
        for (size_t h = base; h < order.size(); ++h) {
            const int32_t u = order[h];
            nb.clear();
            for (int32_t e = rp[u]; e < rp[u + 1]; ++e) {
                const int32_t w = col[e];
                if (!placed[(size_t)w]) {
                    placed[(size_t)w] = 1;
                    nb.push_back(w);
                }
            }
            std::sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) {
                return deg(a) != deg(b) ? deg(a) < deg(b) : a < b;
            });
            order.insert(order.end(), nb.begin(), nb.end());
        }
    }
    std::reverse(order.begin(), order.end());
    return order;
}

// Locality order for high-diameter graphs: clusters of 128 vertices (half a
// 128-byte line of code words) grown by BFS over unplaced vertices from seeds
// taken in reverse Cuthill-McKee order, so that consecutive clusters lie near
// each other; inside each cluster, sub-clusters of 32 (four lines of sigma)
// grown the same way from the cluster's vertices in their BFS order.  A
// sample's BFS ball then covers few lines of either.  (Sizes measured on the
// 1024^2 grid: 128 and 32 beat 256 and 8 by 2.6%, and 512 or more outer
// vertices lose.)  Returns order[k] = the original id of internal vertex k.
std::vector<int32_t> cluster_order(int32_t n, const int32_t *rp, const int32_t *col)
{
    const std::vector<int32_t> seeds = rcm_order(n, rp, col);
    std::vector<uint8_t> mark((size_t)n, 0);  // 0 unplaced, 1 in the current cluster, 2 placed
    std::vector<int32_t> order, cl, sub;
    order.reserve((size_t)n);
    // BFS from seed over vertices marked `from`, marking them `to`, at most cap of them
    auto grow = [&](int32_t seed, size_t cap, uint8_t from, uint8_t to, std::vector<int32_t> &out) {
        out.clear();
        out.push_back(seed);
        mark[(size_t)seed] = to;
        for (size_t h = 0; h < out.size() && out.size() < cap; ++h) {
            const int32_t u = out[h];
            for (int32_t e = rp[u]; e < rp[u + 1] && out.size() < cap; ++e) {
                const int32_t w = col[e];
                if (mark[(size_t)w] == from) {
                    mark[(size_t)w] = to;
                    out.push_back(w);
                }
            }
        }
    };
    for (int32_t sd : seeds) {
        if (mark[(size_t)sd] != 0) continue;
        grow(sd, 128, 0, 1, cl);
        for (int32_t v : cl) {
            if (mark[(size_t)v] != 1) continue;
            grow(v, 32, 1, 2, sub);
            order.insert(order.end(), sub.begin(), sub.end());
        }
    }
    return order;
}

// Replaces the device graph by its internal order (a layout change only:
// every result is the one of the original order, see GraphData).  BFS balls
// of a high-diameter graph then fall in fewer cache lines.
int relabel_for_locality(GraphData &gd, const int32_t *row_ptr, const int32_t *col, hipStream_t s)
{
    const int32_t n = gd.n;
    const size_t m = (size_t)gd.arcs;
    std::vector<int32_t> iperm = cluster_order(n, row_ptr, col);
    std::vector<int32_t> perm((size_t)n);
    for (int32_t k = 0; k < n; ++k) perm[(size_t)iperm[(size_t)k]] = k;
    std::vector<int32_t> rp2((size_t)n + 1), col2(m), colo(m);
    rp2[0] = 0;
    for (int32_t k = 0; k < n; ++k) {
        const int32_t o = iperm[(size_t)k];
        const int32_t d = row_ptr[o + 1] - row_ptr[o];
        rp2[(size_t)k + 1] = rp2[(size_t)k] + d;
        for (int32_t j = 0; j < d; ++j) {
            const int32_t w = col[row_ptr[o] + j];
            col2[(size_t)rp2[(size_t)k] + j] = perm[(size_t)w];
            colo[(size_t)rp2[(size_t)k] + j] = w;
        }
    }
    int32_t *d_rp = nullptr, *d_c = nullptr, *d_co = nullptr, *d_p = nullptr, *d_ip = nullptr, *d_comp = nullptr;
    auto drop = [&] {
        dev_free(d_rp);
        dev_free(d_c);
        dev_free(d_co);
        dev_free(d_p);
        dev_free(d_ip);
        dev_free(d_comp);
    };
    hipError_t e = hipSuccess;
    if ((e = alloc_n(&d_rp, (size_t)n + 1)) != hipSuccess || (e = alloc_n(&d_c, m)) != hipSuccess ||
        (e = alloc_n(&d_co, m)) != hipSuccess || (e = alloc_n(&d_p, (size_t)n)) != hipSuccess ||
        (e = alloc_n(&d_ip, (size_t)n)) != hipSuccess || (e = alloc_n(&d_comp, (size_t)n)) != hipSuccess) {
        drop();
        return fail(e == hipErrorOutOfMemory ? KADABRA_ENOMEM : KADABRA_EDEVICE, "relabelling: %s",
                    hipGetErrorString(e));
    }
    if ((e = hipMemcpy(d_rp, rp2.data(), ((size_t)n + 1) * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
        (m && (e = hipMemcpy(d_c, col2.data(), m * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess) ||
        (m && (e = hipMemcpy(d_co, colo.data(), m * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess) ||
        (e = hipMemcpy(d_p, perm.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(d_ip, iperm.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = kd::launch_gather_i32(d_comp, gd.d_comp, d_ip, n, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess) {
        drop();
        return fail(KADABRA_EDEVICE, "relabelling: %s", hipGetErrorString(e));
    }
    dev_free(gd.d_row_ptr);
    dev_free(gd.d_col);
    dev_free(gd.d_comp);
    gd.d_row_ptr = d_rp;
    gd.d_col = d_c;
    gd.d_colo = d_co;
    gd.d_perm = d_p;
    gd.d_iperm = d_ip;
    gd.d_comp = d_comp;
    gd.h_perm = std::move(perm);
    return KADABRA_OK;
}

}  // namespace

extern "C" {

const char *kadabra_last_error(void) { return g_last_error.c_str(); }

int kadabra_version(void) { return 10100; }

int kadabra_create_graph(int32_t n, int64_t num_arcs, const int32_t *row_ptr, const int32_t *col_idx,
                         kadabra_graph **out)
{
    g_last_error.clear();
    if (!out) return fail(KADABRA_EINVAL, "out is NULL");
    *out = nullptr;
    int32_t max_deg = 0;
    OK_OR_RETURN(validate_csr(n, num_arcs, row_ptr, col_idx, &max_deg));
    std::unique_ptr<kadabra_graph> g(new (std::nothrow) kadabra_graph);
    if (!g) return fail(KADABRA_ENOMEM, "host allocation failed");
    GraphData &gd = g->gd;
    gd.n = n;
    gd.arcs = num_arcs;
    gd.max_deg = max_deg;
    HIP_OR_FAIL(hipGetDevice(&gd.device));
    OK_OR_RETURN(g->runner.init());
    struct {
        int32_t **dst;
        const int32_t *src;
        size_t count;
    } up[] = {{&gd.d_row_ptr, row_ptr, (size_t)n + 1}, {&gd.d_col, col_idx, (size_t)num_arcs}};
    for (auto &u : up) {
        HIP_OR_FAIL(alloc_n(u.dst, u.count));
        if (u.count) HIP_OR_FAIL(hipMemcpy(*u.dst, u.src, u.count * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    // the graph is read by kernels on non-blocking streams: the uploads land first
    HIP_OR_FAIL(hipDeviceSynchronize());
    OK_OR_RETURN(gpu_preprocess(gd, g->runner.own_stream));
    gd.probe_h8 = probe_h8_for(gd.vd, n, num_arcs, row_ptr);
    if (gd.vd >= kRelabelMinVd) OK_OR_RETURN(relabel_for_locality(gd, row_ptr, col_idx, g->runner.own_stream));
    *out = g.release();
    return KADABRA_OK;
}

int kadabra_set_param(kadabra_graph *g, const char *key, int64_t value)
{
    if (!g || !key) return fail(KADABRA_EINVAL, "null argument");
    bool known;
    OK_OR_RETURN(set_common_param(g->params, key, value, &known));
    if (!known) return fail(KADABRA_EINVAL, "unknown parameter '%s'", key);
    if (!strcmp(key, "test_fail_alloc")) g->runner.release_pool();  // the next run allocates afresh
    return KADABRA_OK;
}

int kadabra_get_param(const kadabra_graph *g, const char *key, int64_t *value)
{
    if (!g || !key || !value) return fail(KADABRA_EINVAL, "null argument");
    if (get_common_param(g->params, key, value) == 0) return KADABRA_OK;
    if (!strcmp(key, "vd_bound")) *value = g->gd.vd;
    else if (!strcmp(key, "components")) *value = g->gd.ncomp;
    else if (!strcmp(key, "max_degree")) *value = g->gd.max_deg;
    else if (!strcmp(key, "relabeled")) *value = g->gd.d_perm ? 1 : 0;
    else if (!strcmp(key, "last_team")) *value = g->runner.team;
    else if (!strcmp(key, "last_slots")) *value = g->runner.slots;
    else return fail(KADABRA_EINVAL, "unknown parameter '%s'", key);
    return KADABRA_OK;
}

int kadabra_set_stream(kadabra_graph *g, void *hip_stream)
{
    if (!g) return fail(KADABRA_EINVAL, "null handle");
    g->runner.stream = hip_stream ? (hipStream_t)hip_stream : g->runner.own_stream;
    return KADABRA_OK;
}

int kadabra_run(kadabra_graph *g, double eps, double delta, uint64_t seed)
{
    if (!g) return fail(KADABRA_EINVAL, "null handle");
    g->runner.cancel.store(0);  // a cancel from now on, setup included, stops this run
    g_last_error.clear();
    const auto t0 = std::chrono::steady_clock::now();
    g->have_result = false;
    OK_OR_RETURN(ensure_graph_query(g, eps, delta, seed));
    g->q.resume_counts = nullptr;
    g->q.resume_k = g->q.resume_tau = 0;
    std::vector<Query *> qs{&g->q};
    OK_OR_RETURN(run_queries(g->runner, qs, g->params));
    if (g->q.status != KADABRA_OK) return g->q.status;
    g->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    g->have_result = true;
    return KADABRA_OK;
}

int kadabra_get_checkpoint(const kadabra_graph *g, kadabra_checkpoint *ck, int32_t *counts)
{
    if (!g || !ck) return fail(KADABRA_EINVAL, "null argument");
    const Query &q = g->q;
    if (g->have_result || !q.checkpointed || !q.counts)
        return fail(KADABRA_ESTATE, "the last run did not stop at a boundary");
    memset(ck, 0, sizeof *ck);
    ck->n = g->gd.n;
    ck->tau = q.tau;
    ck->epochs = (int64_t)q.decisions.size();
    ck->omega = q.omega;
    ck->check_interval = q.N;
    ck->eps = q.eps;
    ck->delta = q.delta;
    ck->seed = q.seed;
    static_assert(kd::ST_COUNT == 6, "checkpoint work counters");
    for (int w = 0; w < kd::ST_COUNT; ++w) ck->work[w] = q.work[w];
    if (counts) {
        HIP_OR_FAIL(hipMemcpyAsync(counts, q.counts, (size_t)g->gd.n * sizeof(int32_t), hipMemcpyDeviceToHost,
                                   g->runner.stream));
        HIP_OR_FAIL(hipStreamSynchronize(g->runner.stream));
    }
    return KADABRA_OK;
}

int kadabra_resume(kadabra_graph *g, const kadabra_checkpoint *ck, const int32_t *counts)
{
    if (!g || !ck || !counts) return fail(KADABRA_EINVAL, "null argument");
    g->runner.cancel.store(0);
    g_last_error.clear();
    const auto t0 = std::chrono::steady_clock::now();
    g->have_result = false;
    if (g->params.balance) return fail(KADABRA_EINVAL, "a balanced run cannot be resumed (balance = 0)");
    if (ck->n != g->gd.n) return fail(KADABRA_EINVAL, "checkpoint of a graph of %lld vertices", (long long)ck->n);
    OK_OR_RETURN(make_query(g->q, g->gd, g->params, ck->eps, ck->delta, ck->seed, ck->check_interval));
    Query &q = g->q;
    if (q.omega != ck->omega) return fail(KADABRA_EINVAL, "checkpoint omega %lld, this graph gives %lld",
                                          (long long)ck->omega, (long long)q.omega);
    if (ck->epochs < 1 || ck->tau != q.bound(ck->epochs) || ck->tau >= q.omega)
        return fail(KADABRA_EINVAL, "checkpoint at %lld samples is not a boundary before omega", (long long)ck->tau);
    int64_t total = 0;
    for (int64_t v = 0; v < ck->n; ++v) {
        if (counts[v] < 0 || counts[v] > ck->tau) return fail(KADABRA_EINVAL, "counter %lld out of range", (long long)v);
        total += counts[v];
    }
    if (total != ck->work[kd::ST_INTERIOR]) return fail(KADABRA_EINVAL, "counters do not sum to the increments");
    q.resume_counts = counts;
    q.resume_k = ck->epochs;
    q.resume_tau = ck->tau;
    for (int w = 0; w < kd::ST_COUNT; ++w) q.resume_work[w] = ck->work[w];
    std::vector<Query *> qs{&q};
    const int rc = run_queries(g->runner, qs, g->params);
    q.resume_counts = nullptr;
    OK_OR_RETURN(rc);
    if (q.status != KADABRA_OK) return q.status;
    g->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    g->have_result = true;
    return KADABRA_OK;
}

int kadabra_autotune(kadabra_graph *g, double eps, double delta, int64_t trial_samples)
{
    if (!g) return fail(KADABRA_EINVAL, "null handle");
    if (trial_samples < 1) return fail(KADABRA_EINVAL, "trial_samples must be >= 1");
    g->runner.cancel.store(0);
    g_last_error.clear();
    g->have_result = false;
    OK_OR_RETURN(ensure_graph_query(g, eps, delta, 0x5EEDull));
    std::vector<Query *> qs{&g->q};
    return autotune(g->runner, qs, g->params, trial_samples);
}

int kadabra_get_scores(const kadabra_graph *g, double *scores, int32_t *counts, kadabra_stats *stats)
{
    if (!g) return fail(KADABRA_EINVAL, "null handle");
    if (!g->have_result) return fail(KADABRA_ESTATE, "no completed run");
    OK_OR_RETURN(read_result(g->q, g->runner.stream, scores, counts));
    if (stats) fill_stats(g->q, g->ms_total, stats);
    return KADABRA_OK;
}

int kadabra_get_scores_device(const kadabra_graph *g, double *scores_dev, int32_t *counts_dev)
{
    if (!g) return fail(KADABRA_EINVAL, "null handle");
    if (!g->have_result) return fail(KADABRA_ESTATE, "no completed run");
    if (scores_dev) HIP_OR_FAIL(kd::launch_scores(g->q.counts, scores_dev, g->gd.n, g->q.tau, g->runner.stream));
    if (counts_dev)
        HIP_OR_FAIL(hipMemcpyAsync(counts_dev, g->q.counts, (size_t)g->gd.n * sizeof(int32_t),
                                   hipMemcpyDeviceToDevice, g->runner.stream));
    return KADABRA_OK;
}

int kadabra_get_decisions(const kadabra_graph *g, int8_t *out, int64_t cap, int64_t *count)
{
    if (!g) return fail(KADABRA_EINVAL, "null handle");
    if (!g->have_result) return fail(KADABRA_ESTATE, "no completed run");
    const int64_t m = (int64_t)g->q.decisions.size();
    if (out)
        for (int64_t k = 0; k < std::min(cap, m); ++k) out[k] = g->q.decisions[(size_t)k];
    if (count) *count = m;
    return KADABRA_OK;
}

int kadabra_get_balance(const kadabra_graph *g, double *log_inv_delta_L, double *log_inv_delta_U,
                        int32_t *first_counts)
{
    if (!g) return fail(KADABRA_EINVAL, "null handle");
    if (!g->have_result) return fail(KADABRA_ESTATE, "no completed run");
    const Query &q = g->q;
    const size_t n = (size_t)g->gd.n;
    if (!q.first_launched) {
        for (size_t v = 0; v < n; ++v) {
            if (log_inv_delta_L) log_inv_delta_L[v] = q.L;
            if (log_inv_delta_U) log_inv_delta_U[v] = q.L;
            if (first_counts) first_counts[v] = 0;
        }
        return KADABRA_OK;
    }
    // the counters and the per-count table, then one lookup per vertex
    std::vector<int32_t> c1(n);
    std::vector<double> lcon((size_t)(q.m1 + 1) * 2);
    HIP_OR_FAIL(hipMemcpyAsync(c1.data(), q.c1, n * sizeof(int32_t), hipMemcpyDeviceToHost, g->runner.stream));
    HIP_OR_FAIL(hipMemcpyAsync(lcon.data(), q.lcon(), lcon.size() * sizeof(double), hipMemcpyDeviceToHost,
                               g->runner.stream));
    HIP_OR_FAIL(hipStreamSynchronize(g->runner.stream));
    const std::vector<int32_t> &perm = g->gd.h_perm;  // c1 is in the internal order
    for (size_t v = 0; v < n; ++v) {
        const int32_t c = c1[perm.empty() ? v : (size_t)perm[v]];
        const size_t k = (size_t)c;
        if (k > (size_t)q.m1) return fail(KADABRA_EDEVICE, "first-phase counter out of range");
        if (log_inv_delta_L) log_inv_delta_L[v] = lcon[2 * k];
        if (log_inv_delta_U) log_inv_delta_U[v] = lcon[2 * k + 1];
        if (first_counts) first_counts[v] = c;
    }
    return KADABRA_OK;
}

int kadabra_eval_stop_fg(int32_t n, const int32_t *counts, int64_t tau, int64_t omega, double L,
                         double *f, double *g)
{
    if (n < 1 || tau < 1 || !counts || !f || !g) return fail(KADABRA_EINVAL, "bad argument");
    int32_t *d_c = nullptr;
    double *d_f = nullptr, *d_g = nullptr;
    auto cleanup = [&] {
        dev_free(d_c);
        dev_free(d_f);
        dev_free(d_g);
    };
    hipError_t e;
    const size_t m = (size_t)n;
    if ((e = alloc_n(&d_c, m)) != hipSuccess || (e = alloc_n(&d_f, m)) != hipSuccess ||
        (e = alloc_n(&d_g, m)) != hipSuccess) {
        cleanup();
        return fail(e == hipErrorOutOfMemory ? KADABRA_ENOMEM : KADABRA_EDEVICE, "device allocation: %s",
                    hipGetErrorString(e));
    }
    if ((e = hipMemcpy(d_c, counts, m * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = kd::launch_eval_fg(d_c, n, tau, omega, L, d_f, d_g, nullptr)) != hipSuccess ||
        (e = hipMemcpy(f, d_f, m * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipMemcpy(g, d_g, m * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess) {
        cleanup();
        return fail(KADABRA_EDEVICE, "eval_stop_fg: %s", hipGetErrorString(e));
    }
    cleanup();
    return KADABRA_OK;
}

int kadabra_run_static(kadabra_graph *g, double eps, double delta, uint64_t seed, int32_t *counts_dev,
                       kadabra_stats *stats)
{
    if (!g || !counts_dev) return fail(KADABRA_EINVAL, "null argument");
    g_last_error.clear();
    g->runner.cancel.store(0);
    const auto t0 = std::chrono::steady_clock::now();
    const GraphData &gd = g->gd;
    const Params &p = g->params;
    if (p.balance) return fail(KADABRA_EINVAL, "kadabra_run_static runs uniform delta_L, delta_U only (balance = 0)");
    if (!(eps > 0.0 && eps < 1.0)) return fail(KADABRA_EINVAL, "eps must be in (0, 1)");
    if (!(delta > 0.0 && delta < 1.0)) return fail(KADABRA_EINVAL, "delta must be in (0, 1)");
    int dev = -1;
    HIP_OR_FAIL(hipGetDevice(&dev));
    if (dev != gd.device)
        return fail(KADABRA_EINVAL, "the graph lives on device %d, the current device is %d", gd.device, dev);
    const int64_t omega = omega_of(gd.vd, eps, delta);
    if (omega > kMaxOmega || omega < 1)
        return fail(KADABRA_ERANGE, "omega = %lld samples exceeds the int32 counters", (long long)omega);
    const double L = std::log(4.0 * (double)gd.n / delta);
    const int64_t N = p.check_interval;
    const int32_t lcap = gd.vd + 2;
    // as many samples in flight as the array holds (at most the "slots"
    // parameter, else 1024)
    int64_t slots = p.slots ? p.slots : 1024;
    if (static_layout(gd.n, lcap, 1).end > kStaticScratchBytes)
        return fail(KADABRA_ERANGE,
                    "a graph of %d vertices needs %zu bytes of run state for one sample in flight; the static "
                    "array holds %zu (use kadabra_run)",
                    gd.n, static_layout(gd.n, lcap, 1).end, kStaticScratchBytes);
    while (slots > 1 && static_layout(gd.n, lcap, slots).end > kStaticScratchBytes) {
        const size_t per = static_layout(gd.n, lcap, 2).end - static_layout(gd.n, lcap, 1).end;
        const size_t fixed = static_layout(gd.n, lcap, 1).end - per;
        slots = std::min<int64_t>(slots - 1, (int64_t)((kStaticScratchBytes - fixed) / per));
    }
    slots = std::max<int64_t>(slots, 1);
    const int team = p.team ? p.team : 256;
    char *base = nullptr;
    OK_OR_RETURN(static_scratch(dev, &base));
    const StaticLayout lay = static_layout(gd.n, lcap, slots);
    kd::Control *const ctl = (kd::Control *)(base + lay.ctl);
    unsigned long long *const claim = (unsigned long long *)(base + lay.claim);
    kd::QueryDesc *const desc = (kd::QueryDesc *)(base + lay.desc);
    int32_t *const frames = (int32_t *)(base + lay.frames);
    kd::SlotState st{};
    st.code = (uint32_t *)(base + lay.code);
    st.sigma = (kd::Sigma *)(base + lay.sigma);
    st.ball = (int32_t *)(base + lay.ball);
    st.meet = (int32_t *)(base + lay.meet);
    st.meetw = (uint64_t *)(base + lay.meetw);
    st.loff = (int32_t *)(base + lay.loff);
    st.nstride = gd.n;
    st.lcap = lcap;
    st.code_stride = code_stride_for(gd.n);
    const hipStream_t s = g->runner.stream;
    // the array keeps the last call's contents: clear what must start at zero
    // (counters, frames, control block and claim counter, code words; sigma is
    // written by a sample before it reads it)
    kd::ZeroRegions z{};
    auto zero = [&](void *ptr, size_t bytes) {
        z.ptr[z.n] = (uint32_t *)ptr;
        z.count[z.n] = bytes / 4;
        ++z.n;
    };
    zero(counts_dev, (size_t)gd.n * sizeof(int32_t));
    zero(ctl, lay.desc - lay.ctl);  // control block and claim counter
    zero(frames, 2 * (size_t)gd.n * sizeof(int32_t));
    zero(st.code, (size_t)slots * (size_t)st.code_stride * sizeof(uint32_t));
    HIP_OR_FAIL(kd::launch_zero_regions(z, s));
    // one epoch per launch, checked before the next is queued
    uint64_t claim_next = 0;
    int64_t lo = 0, epochs = 0;
    int decision = 0;
    kd::Control h{};
    while (decision == 0) {
        const int64_t k = epochs + 1, hi = std::min<int64_t>(k * N, omega);
        const int32_t set = (int32_t)(k % 2);
        kd::QueryDesc d{};
        d.row_ptr = gd.d_row_ptr;
        d.col = gd.d_col;
        d.comp = gd.d_comp;
        d.perm = gd.d_perm;
        d.iperm = gd.d_iperm;
        d.colo = gd.d_colo;
        d.frames = frames;
        d.ctl = ctl;
        d.seed = seed;
        d.lo = lo;
        d.hi = hi;
        d.epoch_len = N;
        d.claim_begin = 0;
        d.probe_min = p.probe_min;
        d.probe_h8 = gd.probe_h8;
        d.probe_quit = gd.vd >= kRelabelMinVd ? 1 : 0;
        d.num_arcs = gd.arcs;
        d.n = gd.n;
        d.nframes = 1;
        d.nsets = 2;
        d.gate = -1;
        d.stat_set = -1;
        HIP_OR_FAIL(hipMemcpyAsync(desc, &d, sizeof d, hipMemcpyHostToDevice, s));
        kd::SampleArgs sa{};
        sa.q = desc;
        sa.nq = 1;
        sa.gated = 0;
        sa.total = hi - lo;
        sa.claim = claim;
        sa.claim_base = claim_next;
        sa.st = st;
        const int grid = (int)std::min<int64_t>(slots, hi - lo);
        claim_next += (uint64_t)(hi - lo) + (uint64_t)grid;
        HIP_OR_FAIL(kd::launch_sample(team, grid, sa, gd.d_perm != nullptr, p.probe_pull != 0, s));
        kd::MergeArgs ma{};
        ma.m = nullptr;
        ma.nq = 1;
        ma.nblocks = kd::merge_blocks_for(gd.n);
        kd::MergeDesc &m = ma.one;
        m.counts = counts_dev;
        m.frames = frames + (size_t)set * (size_t)gd.n;
        m.ctl = ctl;
        m.perm = gd.d_perm;
        m.tau = hi;
        m.omega = omega;
        m.L = L;
        m.eps = eps;
        m.n = gd.n;
        m.nframes = 1;
        m.set = set;
        m.gate = -1;
        m.do_check = hi < omega ? 1 : 0;
        m.block_begin = 0;
        HIP_OR_FAIL(kd::launch_merge_check(ma, s));
        HIP_OR_FAIL(hipMemcpyAsync(&h, ctl, sizeof h, hipMemcpyDeviceToHost, s));
        HIP_OR_FAIL(hipStreamSynchronize(s));
        if (h.err)
            return fail(KADABRA_EDEVICE, "device-side invariant failure %d in the sampler at sample %lld", h.err,
                        (long long)h.err_sample);
        epochs = k;
        lo = hi;
        if (hi == omega) decision = 2;
        else if (h.viol[set] == 0) decision = 1;
        else if (g->runner.cancel.load())
            return fail(KADABRA_ECANCELED, "run canceled at %lld samples", (long long)hi);
    }
    if (stats) {
        memset(stats, 0, sizeof *stats);
        stats->tau = lo;
        stats->omega = omega;
        stats->vd_bound = gd.vd;
        stats->epochs = epochs;
        stats->decision = decision;
        stats->v_exp = h.stats_total[kd::ST_VEXP];
        stats->e_scan = h.stats_total[kd::ST_ESCAN];
        stats->e_bt = h.stats_total[kd::ST_EBT];
        stats->path_interior = h.stats_total[kd::ST_INTERIOR];
        stats->disconnected = h.stats_total[kd::ST_DISCONN];
        stats->v_written = h.stats_total[kd::ST_VMAT];
        stats->log_inv_delta = L;
        stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        stats->sample_launches = epochs;
    }
    return KADABRA_OK;
}

#ifdef KADABRA_PHASE_TIMERS
// Phase-timer builds only: sampler cycles per phase of the handle's last run
// (0 pair, 1 expansion, 2 level bookkeeping, 3 meeting draw, 4 backtracking,
// 5 clearing), summed over its control blocks.
int kadabra_debug_phase_cycles(const kadabra_graph *g, int64_t *out8)
{
    if (!g || !g->runner.d_ctl || !out8) return fail(KADABRA_EINVAL, "bad argument");
    std::vector<kd::Control> ctl((size_t)g->runner.ctl_cap);
    HIP_OR_FAIL(hipStreamSynchronize(g->runner.stream));
    HIP_OR_FAIL(hipMemcpy(ctl.data(), g->runner.d_ctl, ctl.size() * sizeof(kd::Control), hipMemcpyDeviceToHost));
    for (int k = 0; k < 8; ++k) {
        out8[k] = 0;
        for (const kd::Control &c : ctl) out8[k] += c.phase_cycles[k];
    }
    return KADABRA_OK;
}
#endif

int kadabra_cancel(kadabra_graph *g)
{
    if (!g) return fail(KADABRA_EINVAL, "null handle");
    g->runner.cancel.store(1);
    return KADABRA_OK;
}

void kadabra_destroy_graph(kadabra_graph *g) { delete g; }

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------

int kadabra_batch_create(kadabra_batch **out)
{
    g_last_error.clear();
    if (!out) return fail(KADABRA_EINVAL, "out is NULL");
    *out = nullptr;
    std::unique_ptr<kadabra_batch> b(new (std::nothrow) kadabra_batch);
    if (!b) return fail(KADABRA_ENOMEM, "host allocation failed");
    OK_OR_RETURN(b->runner.init());
    *out = b.release();
    return KADABRA_OK;
}

int kadabra_batch_set_param(kadabra_batch *b, const char *key, int64_t value)
{
    if (!b || !key) return fail(KADABRA_EINVAL, "null argument");
    if (!strcmp(key, "check_interval")) return fail(KADABRA_EINVAL, "check_interval is set per query");
    bool known;
    OK_OR_RETURN(set_common_param(b->params, key, value, &known));
    if (!known) return fail(KADABRA_EINVAL, "unknown parameter '%s'", key);
    return KADABRA_OK;
}

int kadabra_batch_get_param(const kadabra_batch *b, const char *key, int64_t *value)
{
    if (!b || !key || !value) return fail(KADABRA_EINVAL, "null argument");
    if (get_common_param(b->params, key, value) == 0) return KADABRA_OK;
    if (!strcmp(key, "last_team")) *value = b->runner.team;
    else if (!strcmp(key, "last_slots")) *value = b->runner.slots;
    else if (!strcmp(key, "queries")) *value = (int64_t)b->queries.size();
    else return fail(KADABRA_EINVAL, "unknown parameter '%s'", key);
    return KADABRA_OK;
}

int kadabra_batch_set_stream(kadabra_batch *b, void *hip_stream)
{
    if (!b) return fail(KADABRA_EINVAL, "null handle");
    b->runner.stream = hip_stream ? (hipStream_t)hip_stream : b->runner.own_stream;
    return KADABRA_OK;
}

int kadabra_batch_add(kadabra_batch *b, const kadabra_graph *g, double eps, double delta, uint64_t seed,
                      int64_t check_interval, int32_t *index)
{
    if (!b || !g) return fail(KADABRA_EINVAL, "null handle");
    std::unique_ptr<Query> q(new (std::nothrow) Query);
    if (!q) return fail(KADABRA_ENOMEM, "host allocation failed");
    OK_OR_RETURN(make_query(*q, g->gd, b->params, eps, delta, seed, check_interval));
    b->queries.push_back(std::move(q));
    b->have_result = false;
    if (index) *index = (int32_t)b->queries.size() - 1;
    return KADABRA_OK;
}

int kadabra_batch_run(kadabra_batch *b)
{
    if (!b) return fail(KADABRA_EINVAL, "null handle");
    if (b->queries.empty()) return fail(KADABRA_ESTATE, "empty batch");
    b->runner.cancel.store(0);
    g_last_error.clear();
    const auto t0 = std::chrono::steady_clock::now();
    b->have_result = false;
    std::vector<Query *> qs;
    for (auto &q : b->queries) {
        q->nframes = b->params.frames;
        q->epl = b->params.epochs;
        q->nsets = 2 * b->params.epochs;
        q->probe_min = b->params.probe_min;
        q->m1 = first_phase_of(b->params, q->omega);
        qs.push_back(q.get());
    }
    OK_OR_RETURN(run_queries(b->runner, qs, b->params));
    for (Query *q : qs)
        if (q->status != KADABRA_OK) return q->status;
    b->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    b->have_result = true;
    return KADABRA_OK;
}

int kadabra_batch_autotune(kadabra_batch *b, int64_t trial_samples)
{
    if (!b) return fail(KADABRA_EINVAL, "null handle");
    if (b->queries.empty()) return fail(KADABRA_ESTATE, "empty batch");
    if (trial_samples < 1) return fail(KADABRA_EINVAL, "trial_samples must be >= 1");
    b->runner.cancel.store(0);
    b->have_result = false;
    std::vector<Query *> qs;
    for (auto &q : b->queries) qs.push_back(q.get());
    return autotune(b->runner, qs, b->params, trial_samples);
}

int kadabra_batch_get_scores(const kadabra_batch *b, int32_t index, double *scores, int32_t *counts,
                             kadabra_stats *stats)
{
    if (!b) return fail(KADABRA_EINVAL, "null handle");
    if (index < 0 || index >= (int32_t)b->queries.size()) return fail(KADABRA_EINVAL, "bad query index");
    if (!b->have_result) return fail(KADABRA_ESTATE, "no completed run");
    const Query &q = *b->queries[(size_t)index];
    OK_OR_RETURN(read_result(q, b->runner.stream, scores, counts));
    if (stats) fill_stats(q, b->ms_total, stats);
    return KADABRA_OK;
}

int kadabra_batch_clear(kadabra_batch *b)
{
    if (!b) return fail(KADABRA_EINVAL, "null handle");
    (void)hipStreamSynchronize(b->runner.stream);
    b->queries.clear();
    b->have_result = false;
    return KADABRA_OK;
}

void kadabra_batch_destroy(kadabra_batch *b) { delete b; }

// ---------------------------------------------------------------------------
// Serving
// ---------------------------------------------------------------------------

int kadabra_server_create(const kadabra_graph *const *graphs, int32_t ngraphs, int64_t hbm_budget_bytes,
                          int32_t max_active, kadabra_server **out)
{
    g_last_error.clear();
    if (!out) return fail(KADABRA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!graphs || ngraphs < 1) return fail(KADABRA_EINVAL, "need at least one graph");
    if (hbm_budget_bytes < 0) return fail(KADABRA_EINVAL, "hbm_budget_bytes must be >= 0");
    if (max_active < 0 || max_active > 65536) return fail(KADABRA_EINVAL, "max_active must be in [0, 65536]");
    std::unique_ptr<kadabra_server> s(new (std::nothrow) kadabra_server);
    if (!s) return fail(KADABRA_ENOMEM, "host allocation failed");
    for (int32_t i = 0; i < ngraphs; ++i) {
        if (!graphs[i]) return fail(KADABRA_EINVAL, "graphs[%d] is NULL", i);
        const GraphData &gd = graphs[i]->gd;
        s->graphs.push_back(&gd);
        s->nmax = std::max<int64_t>(s->nmax, gd.n);
        s->lcap = std::max(s->lcap, gd.vd + 2);
    }
    s->max_active = max_active ? max_active : 256;
    HIP_OR_FAIL(hipGetDevice(&s->device));
    OK_OR_RETURN(s->runner.init());
    HIP_OR_FAIL(hipStreamCreateWithFlags(&s->io, hipStreamNonBlocking));
    int tm;
    int64_t sl;
    s->runner.choose_mapping(s->params, s->nmax, s->lcap, &tm, &sl);
    OK_OR_RETURN(s->runner.ensure_pool(tm, sl, s->nmax, s->lcap, nullptr));
    s->mapped = true;
    OK_OR_RETURN(s->runner.ensure_tables(s->max_active, nullptr));
    if (hbm_budget_bytes == 0) {
        size_t free_b = 0, total_b = 0;
        HIP_OR_FAIL(hipMemGetInfo(&free_b, &total_b));
        hbm_budget_bytes = (int64_t)(free_b / 2);
    }
    s->budget = hbm_budget_bytes;
    kadabra_server *raw = s.get();
    try {
        s->worker = std::thread(server_main, raw);
    } catch (...) {
        return fail(KADABRA_ENOMEM, "cannot start the worker thread");
    }
    *out = s.release();
    return KADABRA_OK;
}

int kadabra_server_set_param(kadabra_server *s, const char *key, int64_t value)
{
    if (!s || !key) return fail(KADABRA_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->started) return fail(KADABRA_ESTATE, "parameters are fixed once a query was submitted");
    if (!strcmp(key, "check_interval")) return fail(KADABRA_EINVAL, "check_interval is set per query");
    if (!strcmp(key, "test_fail_alloc")) return fail(KADABRA_EINVAL, "test_fail_alloc is not supported here");
    if (!strcmp(key, "round_us")) {
        if (value < 0 || value > (int64_t)1e9) return fail(KADABRA_EINVAL, "round_us must be in [0, 1e9]");
        s->round_ms = (double)value * 1e-3;
        return KADABRA_OK;
    }
    bool known;
    OK_OR_RETURN(set_common_param(s->params, key, value, &known));
    if (!known) return fail(KADABRA_EINVAL, "unknown parameter '%s'", key);
    s->mapped = false;
    return KADABRA_OK;
}

int kadabra_server_get_param(const kadabra_server *s, const char *key, int64_t *value)
{
    if (!s || !key || !value) return fail(KADABRA_EINVAL, "null argument");
    if (get_common_param(s->params, key, value) == 0) return KADABRA_OK;
    if (!strcmp(key, "graphs")) *value = (int64_t)s->graphs.size();
    else if (!strcmp(key, "max_active")) *value = s->max_active;
    else if (!strcmp(key, "budget")) *value = s->budget;
    else if (!strcmp(key, "round_us")) *value = (int64_t)std::llround(s->round_ms * 1e3);
    else return fail(KADABRA_EINVAL, "unknown parameter '%s'", key);
    return KADABRA_OK;
}

int kadabra_server_submit(kadabra_server *s, int32_t graph_index, double eps, double delta, uint64_t seed,
                          int64_t check_interval, int64_t *ticket)
{
    if (!s || !ticket) return fail(KADABRA_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->broken != KADABRA_OK)
        return fail(s->broken, "server stopped after a device error: %s", s->broken_err.c_str());
    if (s->stop) return fail(KADABRA_ESTATE, "server is shutting down");
    if (graph_index < 0 || graph_index >= (int32_t)s->graphs.size())
        return fail(KADABRA_EINVAL, "bad graph index %d", graph_index);
    std::unique_ptr<Served> v(new (std::nothrow) Served);
    if (!v) return fail(KADABRA_ENOMEM, "host allocation failed");
    const GraphData &gd = *s->graphs[(size_t)graph_index];
    OK_OR_RETURN(make_query(*v, gd, s->params, eps, delta, seed, check_interval));
    v->graph = graph_index;
    v->charge = s->charge_of(*v);
    v->frame_bytes = s->frame_bytes_of(*v);
    if (v->charge > s->budget)
        return fail(KADABRA_ERANGE, "query needs %lld device bytes, budget is %lld", (long long)v->charge,
                    (long long)s->budget);
    v->ticket = s->next_ticket++;
    *ticket = v->ticket;
    s->pending.push_back(v.get());
    s->tickets[v->ticket] = std::move(v);
    s->submitted += 1;
    s->started = true;
    s->cv_work.notify_one();
    return KADABRA_OK;
}

int kadabra_server_wait(kadabra_server *s, int64_t ticket, double timeout_s, int32_t *done)
{
    if (!s) return fail(KADABRA_EINVAL, "null handle");
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->tickets.find(ticket) == s->tickets.end())
        return fail(KADABRA_EINVAL, "unknown ticket %lld", (long long)ticket);
    // the ticket is looked up again at every wake-up: another thread may release it
    auto ready = [s, ticket] {
        auto it = s->tickets.find(ticket);
        return it == s->tickets.end() || it->second->final_;
    };
    if (timeout_s < 0) s->cv_done.wait(lk, ready);
    else s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return fail(KADABRA_EINVAL, "ticket %lld was released while waiting", (long long)ticket);
    if (done) *done = it->second->final_ ? 1 : 0;
    return KADABRA_OK;
}

int kadabra_server_result(kadabra_server *s, int64_t ticket, double *scores, int32_t *counts,
                          kadabra_stats *stats, double *latency_ms)
{
    if (!s) return fail(KADABRA_EINVAL, "null handle");
    Served *v;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->tickets.find(ticket);
        if (it == s->tickets.end()) return fail(KADABRA_EINVAL, "unknown ticket %lld", (long long)ticket);
        v = it->second.get();
        if (!v->final_) return fail(KADABRA_ESTATE, "ticket %lld is not final", (long long)ticket);
        if (v->status != KADABRA_OK) return fail(v->status, "%s", v->err.c_str());
        // the score buffer is made here, once, so concurrent reads share it
        if (scores && !v->scores) HIP_OR_FAIL(alloc_n(&v->scores, (size_t)v->gd->n));
        v->readers += 1;  // pinned: release refuses while a read is in progress
    }
    const int rc = read_result(*v, s->io, scores, counts);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        v->readers -= 1;
    }
    OK_OR_RETURN(rc);
    if (stats) fill_stats(*v, v->latency_ms, stats);
    if (latency_ms) *latency_ms = v->latency_ms;
    return KADABRA_OK;
}

int kadabra_server_release(kadabra_server *s, int64_t ticket)
{
    if (!s) return fail(KADABRA_EINVAL, "null handle");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return fail(KADABRA_EINVAL, "unknown ticket %lld", (long long)ticket);
    Served *v = it->second.get();
    if (!v->final_) return fail(KADABRA_ESTATE, "ticket %lld is not final", (long long)ticket);
    if (v->readers > 0) return fail(KADABRA_ESTATE, "ticket %lld has a result read in progress", (long long)ticket);
    if (v->admitted) {
        const size_t n = (size_t)v->gd->n;
        s->put_bin(v->counts, n * sizeof(int32_t));
        s->put_bin(v->scores, n * sizeof(double));
        s->put_bin(v->frames, v->frames_len * sizeof(int32_t));
        v->counts = nullptr;
        v->scores = nullptr;
        v->frames = nullptr;
        v->frames_len = 0;
        s->in_use -= v->charge;
        v->charge = 0;
    }
    s->tickets.erase(it);
    s->cv_work.notify_one();
    return KADABRA_OK;
}

int kadabra_server_info_get(kadabra_server *s, kadabra_server_info *info, int32_t reset)
{
    if (!s || !info) return fail(KADABRA_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    memset(info, 0, sizeof *info);
    info->submitted = s->submitted;
    info->completed = s->completed;
    info->failed = s->failed;
    info->active = s->active;
    info->pending = (int64_t)s->pending.size();
    info->bytes_in_use = s->in_use;
    info->budget_bytes = s->budget;
    info->peak_active = s->peak_active;
    if (!s->lat.empty()) {
        std::vector<double> l = s->lat;
        std::sort(l.begin(), l.end());
        auto rank = [&](double p) {  // nearest-rank percentile
            size_t r = (size_t)std::ceil(p * (double)l.size());
            return l[std::min(std::max<size_t>(r, 1), l.size()) - 1];
        };
        info->p50_ms = rank(0.50);
        info->p99_ms = rank(0.99);
        info->max_ms = l.back();
    }
    if (s->queue_n) info->mean_queue_ms = s->queue_ms_sum / (double)s->queue_n;
    if (reset) {
        s->lat.clear();
        s->queue_ms_sum = 0.0;
        s->queue_n = 0;
        s->peak_active = s->active;
    }
    return KADABRA_OK;
}

void kadabra_server_destroy(kadabra_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->runner.cancel.store(1);
        for (Served *v : s->pending) {
            v->status = KADABRA_ECANCELED;
            v->err = "server destroyed before the query was admitted";
            v->final_ = true;
        }
        s->pending.clear();
        s->cv_work.notify_all();
        s->cv_done.notify_all();
    }
    delete s;
}

}  // extern "C"
