// kadabra_host.cpp -- C ABI and host driver of the gfx950 KADABRA library.
//
// Host side: input validation, graph-only preprocessing (components and the
// vertex-diameter bound, Section 2.3 / Appendix C.1), omega and L, device
// memory, and the epoch loop of Algorithm 1 with checks every N samples
// (Appendix C.2).  Per epoch k the stream runs
//     sample_kernel(k)      samples [B_{k-1}, B_k) into the frames of parity k
//     merge_check_kernel(k) counters += frames; stopping rule on [0, B_k)
// and the host reads one flag.  With overlap on, sample_kernel(k+1) is queued
// before the flag of epoch k is read and is discarded if epoch k stops: the
// counters checked at B_k hold exactly samples [0, B_k) either way.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
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

constexpr int32_t kMaxN = 1 << 23;       // n and every degree stay below 2^23
constexpr int64_t kMaxOmega = INT32_MAX; // int32 counters

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

void dev_free(void *p)
{
    if (p) (void)hipFree(p);
}

}  // namespace

struct kadabra_graph {
    int32_t n = 0;
    int64_t arcs = 0;
    int32_t max_deg = 0;
    int32_t vd = 1;
    int32_t ncomp = 0;
    int device = 0;
    int num_cu = 0;
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;
    int32_t *d_row_ptr = nullptr, *d_col = nullptr, *d_comp = nullptr;

    // parameters
    int64_t check_interval = 1024;
    int team = 0;
    int64_t slots = 0;
    int frames = 1;
    int overlap = 1;
    int64_t fail_alloc = 0;  // test hook: the fail_alloc-th run-buffer allocation fails
    int64_t probe_min = -1;  // meeting-probe threshold in arcs; -1 = auto

    // run buffers (kept across runs; grown when needed)
    int rb_team = 0;
    int64_t rb_slots = 0;
    int rb_frames = 0;
    kd::SlotState st{};
    int32_t *d_counts = nullptr;
    int32_t *d_frames = nullptr;
    kd::Control *d_ctl = nullptr;
    double *d_scores = nullptr;
    int32_t *h_flags = nullptr;  // pinned: violation flags of the two parities
    bool state_dirty = true;     // slot state must be cleared before sampling
    hipEvent_t ev_start = nullptr, ev_stop = nullptr, ev_flag[2] = {nullptr, nullptr};
    hipEvent_t ev_ks[2] = {nullptr, nullptr}, ev_ke[2] = {nullptr, nullptr};  // sampling launches

    // last result
    bool have_result = false;
    int64_t tau = 0, omega = 0, epochs = 0, decision = 0;
    double L = 0.0, ms_sampling = 0.0, ms_total = 0.0, ms_kernels = 0.0;
    int64_t work[kd::ST_COUNT] = {};
    std::vector<int8_t> decisions;
    std::atomic<int> cancel{0};

    ~kadabra_graph()
    {
        release_run_buffers();
        dev_free(d_row_ptr);
        dev_free(d_col);
        dev_free(d_comp);
        dev_free(d_scores);
        if (h_flags) (void)hipHostFree(h_flags);
        for (hipEvent_t e : {ev_start, ev_stop, ev_flag[0], ev_flag[1], ev_ks[0], ev_ks[1], ev_ke[0], ev_ke[1]})
            if (e) (void)hipEventDestroy(e);
        if (own_stream) (void)hipStreamDestroy(own_stream);
    }

    void release_run_buffers()
    {
        dev_free(st.code);
        dev_free(st.sigma);
        dev_free(st.loff);
        dev_free(st.ball);
        dev_free(st.meet);
        dev_free(st.meetw);
        dev_free(d_counts);
        dev_free(d_frames);
        dev_free(d_ctl);
        st = kd::SlotState{};
        d_counts = nullptr;
        d_frames = nullptr;
        d_ctl = nullptr;
        rb_team = 0;
        rb_slots = 0;
        rb_frames = 0;
        state_dirty = true;
    }
};

namespace {

// Bytes of per-slot sampling state for a graph of n vertices.
int32_t code_stride(int32_t n) { return ((n + 7) / 8 + 15) / 16 * 16; }

size_t slot_bytes(int32_t n, int32_t lcap)
{
    return (size_t)code_stride(n) * 4 +
           (size_t)n * (2 * sizeof(kd::Sigma) + 2 * sizeof(int32_t) + sizeof(int32_t) + sizeof(uint64_t)) +
           2 * (size_t)lcap * sizeof(int32_t);
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
    int32_t max_deg = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (row_ptr[v + 1] < row_ptr[v])
            return fail(KADABRA_EINVAL, "row_ptr decreases at %d", v);
        const int32_t deg = row_ptr[v + 1] - row_ptr[v];
        max_deg = std::max(max_deg, deg);
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            const int32_t w = col[e];
            if (w < 0 || w >= n) return fail(KADABRA_EINVAL, "column %d out of range at row %d", w, v);
            if (w == v) return fail(KADABRA_EINVAL, "self-loop at vertex %d", v);
            if (e > row_ptr[v] && col[e - 1] >= w)
                return fail(KADABRA_EINVAL, "row %d not strictly ascending", v);
        }
    }
    if (max_deg >= kMaxN) return fail(KADABRA_ERANGE, "degree %d is not below 2^23", max_deg);
    // symmetry: every arc (v, w) has its reverse (w, v)
    for (int32_t v = 0; v < n; ++v)
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            const int32_t w = col[e];
            if (!std::binary_search(col + row_ptr[w], col + row_ptr[w + 1], v))
                return fail(KADABRA_EINVAL, "arc (%d, %d) has no reverse: graph not undirected", v, w);
        }
    *max_deg_out = max_deg;
    return KADABRA_OK;
}

// Components (numbered by lowest vertex) and the vertex-diameter bound: per
// component, BFS from its maximum-degree vertex (lowest id on ties); every
// shortest path there has at most 2 ecc edges, so VD = max (2 ecc + 1).
void preprocess(int32_t n, const int32_t *row_ptr, const int32_t *col, std::vector<int32_t> &comp,
                int32_t *ncomp_out, int32_t *vd_out)
{
    comp.assign(n, -1);
    std::vector<int32_t> queue(n), root;
    int32_t ncomp = 0;
    for (int32_t r = 0; r < n; ++r) {
        if (comp[r] >= 0) continue;
        size_t head = 0, tail = 0;
        queue[tail++] = r;
        comp[r] = ncomp;
        int32_t best = r;
        while (head < tail) {
            const int32_t u = queue[head++];
            const int32_t du = row_ptr[u + 1] - row_ptr[u], db = row_ptr[best + 1] - row_ptr[best];
            if (du > db || (du == db && u < best)) best = u;
            for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
                if (comp[col[e]] < 0) {
                    comp[col[e]] = ncomp;
                    queue[tail++] = col[e];
                }
        }
        root.push_back(best);
        ++ncomp;
    }
    std::vector<int32_t> dist(n, -1);
    int32_t vd = 1;
    for (int32_t c = 0; c < ncomp; ++c) {
        size_t head = 0, tail = 0;
        queue[tail++] = root[c];
        dist[root[c]] = 0;
        int32_t ecc = 0;
        while (head < tail) {
            const int32_t u = queue[head++];
            ecc = std::max(ecc, dist[u]);
            for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
                if (dist[col[e]] < 0) {
                    dist[col[e]] = dist[u] + 1;
                    queue[tail++] = col[e];
                }
        }
        vd = std::max(vd, 2 * ecc + 1);
    }
    *ncomp_out = ncomp;
    *vd_out = vd;
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

int ensure_run_buffers(kadabra_graph *g, int team, int64_t slots, int frames)
{
    if (g->rb_team == team && g->rb_slots == slots && g->rb_frames == frames && g->d_ctl)
        return KADABRA_OK;
    g->release_run_buffers();
    const size_t n = (size_t)g->n;
    const size_t S = (size_t)slots;
    const int32_t lcap = g->vd + 2;  // a side reaches at most diameter <= VD - 1 levels
    const int32_t cstride = code_stride(g->n);
    HIP_OR_FAIL(dev_alloc((void **)&g->st.code, S * (size_t)cstride * sizeof(uint32_t), &g->fail_alloc));
    HIP_OR_FAIL(dev_alloc((void **)&g->st.sigma, S * 2 * n * sizeof(kd::Sigma), &g->fail_alloc));
    HIP_OR_FAIL(dev_alloc((void **)&g->st.loff, S * 2 * (size_t)lcap * sizeof(int32_t), &g->fail_alloc));
    g->st.lcap = lcap;
    g->st.code_stride = cstride;
    HIP_OR_FAIL(dev_alloc((void **)&g->st.ball, S * 2 * n * sizeof(int32_t), &g->fail_alloc));
    HIP_OR_FAIL(dev_alloc((void **)&g->st.meet, S * n * sizeof(int32_t), &g->fail_alloc));
    HIP_OR_FAIL(dev_alloc((void **)&g->st.meetw, S * n * sizeof(uint64_t), &g->fail_alloc));
    HIP_OR_FAIL(dev_alloc((void **)&g->d_counts, n * sizeof(int32_t), &g->fail_alloc));
    HIP_OR_FAIL(dev_alloc((void **)&g->d_frames, 2 * (size_t)frames * n * sizeof(int32_t), &g->fail_alloc));
    HIP_OR_FAIL(dev_alloc((void **)&g->d_ctl, sizeof(kd::Control), &g->fail_alloc));
    g->rb_team = team;
    g->rb_slots = slots;
    g->rb_frames = frames;
    g->state_dirty = true;
    return KADABRA_OK;
}

// Mapping choices (none of them changes the result).
void choose_mapping(const kadabra_graph *g, int *team, int64_t *slots)
{
    int tm = g->team;
    if (tm == 0) tm = 256;
    int64_t sl = g->slots;
    if (sl == 0) {
        const int per_cu = (tm == 64) ? 8 : 4;
        sl = (int64_t)std::max(g->num_cu, 1) * per_cu;
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b > 0) {
            const int64_t fit = (int64_t)((free_b / 2) / slot_bytes(g->n, g->vd + 2));
            sl = std::min(sl, std::max<int64_t>(fit, 1));
        }
    }
    *team = tm;
    *slots = std::max<int64_t>(sl, 1);
}

int run_impl(kadabra_graph *g, double eps, double delta, uint64_t seed)
{
    const auto t_wall0 = std::chrono::steady_clock::now();
    g->have_result = false;
    g->cancel.store(0);
    if (!(eps > 0.0 && eps < 1.0)) return fail(KADABRA_EINVAL, "eps must be in (0, 1)");
    if (!(delta > 0.0 && delta < 1.0)) return fail(KADABRA_EINVAL, "delta must be in (0, 1)");
    const int64_t omega = omega_of(g->vd, eps, delta);
    if (omega > kMaxOmega || omega < 1)
        return fail(KADABRA_ERANGE, "omega = %lld samples exceeds the int32 counters",
                    (long long)omega);
    const double L = std::log(4.0 * (double)g->n / delta);
    const int64_t N = g->check_interval;

    int team;
    int64_t slots;
    choose_mapping(g, &team, &slots);
    if (int rc = ensure_run_buffers(g, team, slots, g->frames)) return rc;

    hipStream_t s = g->stream;
    const size_t n = (size_t)g->n;
    if (g->state_dirty) {
        HIP_OR_FAIL(kd::launch_fill_u32(g->st.code, (size_t)slots * g->st.code_stride, 0u, s));
        HIP_OR_FAIL(kd::launch_fill_u32((uint32_t *)g->st.sigma, (size_t)slots * n * 8, 0u, s));
        g->state_dirty = false;
    }
    HIP_OR_FAIL(kd::launch_fill_u32((uint32_t *)g->d_counts, n, 0u, s));
    HIP_OR_FAIL(kd::launch_fill_u32((uint32_t *)g->d_frames, 2 * (size_t)g->frames * n, 0u, s));
    HIP_OR_FAIL(kd::launch_fill_u32((uint32_t *)g->d_ctl, sizeof(kd::Control) / 4, 0u, s));

    kd::SampleArgs sa{};
    sa.row_ptr = g->d_row_ptr;
    sa.col = g->d_col;
    sa.comp = g->d_comp;
    sa.n = g->n;
    sa.nframes = g->frames;
    sa.seed = seed;
    sa.probe_min = g->probe_min;
    sa.num_arcs = g->arcs;
    sa.frames = g->d_frames;
    sa.ctl = g->d_ctl;
    sa.st = g->st;
    kd::CheckArgs ca{};
    ca.counts = g->d_counts;
    ca.frames = g->d_frames;
    ca.n = g->n;
    ca.nframes = g->frames;
    ca.omega = omega;
    ca.L = L;
    ca.eps = eps;
    ca.ctl = g->d_ctl;

    g->decisions.clear();
    HIP_OR_FAIL(hipEventRecord(g->ev_start, s));
    int64_t k = 0, lo = 0, tau = 0;
    int decision = 0;
    bool next_launched = false;
    int status = KADABRA_OK;
    double ms_kernels = 0.0;
    for (;;) {
        ++k;
        const int64_t hi = std::min<int64_t>(k * N, omega);  // k*N cannot overflow: N, k < 2^31
        const int par = (int)(k & 1);
        if (!next_launched) {
            sa.lo = lo;
            sa.hi = hi;
            sa.parity = par;
            sa.gate = -1;  // the host knows the previous boundary did not stop
            HIP_OR_FAIL(hipEventRecord(g->ev_ks[par], s));
            HIP_OR_FAIL(kd::launch_sample(team, (int)slots, sa, s));
            HIP_OR_FAIL(hipEventRecord(g->ev_ke[par], s));
        }
        ca.tau = hi;
        ca.parity = par;
        ca.do_check = hi < omega;
        HIP_OR_FAIL(kd::launch_merge_check(ca, s));
        HIP_OR_FAIL(hipMemcpyAsync(&g->h_flags[par], &g->d_ctl->viol[par], sizeof(int32_t),
                                   hipMemcpyDeviceToHost, s));
        HIP_OR_FAIL(hipEventRecord(g->ev_flag[par], s));
        next_launched = false;
        if (g->overlap && hi < omega) {
            // speculative: the next epoch's samples, discarded if this epoch stops
            sa.lo = hi;
            sa.hi = std::min<int64_t>((k + 1) * N, omega);
            sa.parity = par ^ 1;
            sa.gate = par;  // exits at once if this boundary's check stops the run
            HIP_OR_FAIL(hipEventRecord(g->ev_ks[par ^ 1], s));
            HIP_OR_FAIL(kd::launch_sample(team, (int)slots, sa, s));
            HIP_OR_FAIL(hipEventRecord(g->ev_ke[par ^ 1], s));
            next_launched = true;
        }
        HIP_OR_FAIL(hipEventSynchronize(g->ev_flag[par]));
        {
            float kms = 0.f;  // this epoch's sampling launch has finished
            HIP_OR_FAIL(hipEventElapsedTime(&kms, g->ev_ks[par], g->ev_ke[par]));
            ms_kernels += kms;
        }
        tau = hi;
        lo = hi;
        if (hi == omega) {
            decision = 2;
        } else if (g->h_flags[par] == 0) {
            decision = 1;
        }
        g->decisions.push_back((int8_t)decision);
        if (decision) break;
        if (g->cancel.load()) {
            status = fail(KADABRA_ECANCELED, "run canceled at %lld samples", (long long)tau);
            break;
        }
    }
    HIP_OR_FAIL(hipEventRecord(g->ev_stop, s));
    kd::Control ctl;
    HIP_OR_FAIL(hipMemcpyAsync(&ctl, g->d_ctl, sizeof ctl, hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    if (ctl.err) {
        g->state_dirty = true;
        return fail(KADABRA_EDEVICE, "device-side invariant failure in the sampler");
    }
    if (status != KADABRA_OK) return status;
    float ms = 0.f;
    HIP_OR_FAIL(hipEventElapsedTime(&ms, g->ev_start, g->ev_flag[(int)(k & 1)]));
    g->ms_sampling = ms;
    g->ms_kernels = ms_kernels;
    g->tau = tau;
    g->omega = omega;
    g->epochs = k;
    g->decision = decision;
    g->L = L;
    for (int q = 0; q < kd::ST_COUNT; ++q) g->work[q] = ctl.stats_total[q];
    g->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_wall0).count();
    g->have_result = true;
    return KADABRA_OK;
}

}  // namespace

extern "C" {

const char *kadabra_last_error(void) { return g_last_error.c_str(); }

int kadabra_version(void) { return 10000; }

int kadabra_create_graph(int32_t n, int64_t num_arcs, const int32_t *row_ptr, const int32_t *col_idx,
                         kadabra_graph **out)
{
    g_last_error.clear();
    if (!out) return fail(KADABRA_EINVAL, "out is NULL");
    *out = nullptr;
    int32_t max_deg = 0;
    if (int rc = validate_csr(n, num_arcs, row_ptr, col_idx, &max_deg)) return rc;
    kadabra_graph *g = new (std::nothrow) kadabra_graph;
    if (!g) return fail(KADABRA_ENOMEM, "host allocation failed");
    g->n = n;
    g->arcs = num_arcs;
    g->max_deg = max_deg;
    std::vector<int32_t> comp;
    preprocess(n, row_ptr, col_idx, comp, &g->ncomp, &g->vd);
    auto bail = [&](int rc) {
        delete g;
        return rc;
    };
    hipError_t e = hipGetDevice(&g->device);
    if (e != hipSuccess) return bail(fail(KADABRA_EDEVICE, "no HIP device: %s", hipGetErrorString(e)));
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, g->device) == hipSuccess) g->num_cu = prop.multiProcessorCount;
    if ((e = hipStreamCreateWithFlags(&g->own_stream, hipStreamNonBlocking)) != hipSuccess)
        return bail(fail(KADABRA_EDEVICE, "stream: %s", hipGetErrorString(e)));
    g->stream = g->own_stream;
    for (hipEvent_t *ev : {&g->ev_start, &g->ev_stop, &g->ev_flag[0], &g->ev_flag[1], &g->ev_ks[0],
                           &g->ev_ks[1], &g->ev_ke[0], &g->ev_ke[1]})
        if ((e = hipEventCreate(ev)) != hipSuccess)
            return bail(fail(KADABRA_EDEVICE, "event: %s", hipGetErrorString(e)));
    if ((e = hipHostMalloc((void **)&g->h_flags, 2 * sizeof(int32_t), hipHostMallocDefault)) != hipSuccess)
        return bail(fail(KADABRA_ENOMEM, "pinned host memory: %s", hipGetErrorString(e)));
    struct {
        int32_t **dst;
        const int32_t *src;
        size_t count;
    } up[] = {{&g->d_row_ptr, row_ptr, (size_t)n + 1},
              {&g->d_col, col_idx, (size_t)num_arcs},
              {&g->d_comp, comp.data(), (size_t)n}};
    for (auto &u : up) {
        if ((e = dev_alloc((void **)u.dst, u.count * sizeof(int32_t))) != hipSuccess)
            return bail(fail(e == hipErrorOutOfMemory ? KADABRA_ENOMEM : KADABRA_EDEVICE,
                             "device allocation: %s", hipGetErrorString(e)));
        if (u.count &&
            (e = hipMemcpy(*u.dst, u.src, u.count * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess)
            return bail(fail(KADABRA_EDEVICE, "upload: %s", hipGetErrorString(e)));
    }
    *out = g;
    return KADABRA_OK;
}

int kadabra_set_param(kadabra_graph *g, const char *key, int64_t value)
{
    if (!g || !key) return fail(KADABRA_EINVAL, "null argument");
    if (!strcmp(key, "check_interval")) {
        if (value < 1 || value > INT32_MAX) return fail(KADABRA_EINVAL, "check_interval must be in [1, 2^31)");
        g->check_interval = value;
    } else if (!strcmp(key, "team")) {
        if (value != 0 && value != 64 && value != 256) return fail(KADABRA_EINVAL, "team must be 0, 64 or 256");
        g->team = (int)value;
    } else if (!strcmp(key, "slots")) {
        if (value < 0 || value > (1 << 20)) return fail(KADABRA_EINVAL, "slots must be in [0, 2^20]");
        g->slots = value;
    } else if (!strcmp(key, "frames")) {
        if (value < 1 || value > 4096) return fail(KADABRA_EINVAL, "frames must be in [1, 4096]");
        g->frames = (int)value;
    } else if (!strcmp(key, "overlap")) {
        if (value != 0 && value != 1) return fail(KADABRA_EINVAL, "overlap must be 0 or 1");
        g->overlap = (int)value;
    } else if (!strcmp(key, "probe_min")) {
        if (value < -1) return fail(KADABRA_EINVAL, "probe_min must be >= -1");
        g->probe_min = value;
    } else if (!strcmp(key, "test_fail_alloc")) {
        if (value < 0) return fail(KADABRA_EINVAL, "test_fail_alloc must be >= 0");
        g->fail_alloc = value;
        g->release_run_buffers();  // the next run allocates afresh
    } else {
        return fail(KADABRA_EINVAL, "unknown parameter '%s'", key);
    }
    return KADABRA_OK;
}

int kadabra_get_param(const kadabra_graph *g, const char *key, int64_t *value)
{
    if (!g || !key || !value) return fail(KADABRA_EINVAL, "null argument");
    if (!strcmp(key, "check_interval")) *value = g->check_interval;
    else if (!strcmp(key, "team")) *value = g->team;
    else if (!strcmp(key, "slots")) *value = g->slots;
    else if (!strcmp(key, "frames")) *value = g->frames;
    else if (!strcmp(key, "overlap")) *value = g->overlap;
    else if (!strcmp(key, "probe_min")) *value = g->probe_min;
    else if (!strcmp(key, "vd_bound")) *value = g->vd;
    else if (!strcmp(key, "components")) *value = g->ncomp;
    else if (!strcmp(key, "max_degree")) *value = g->max_deg;
    else if (!strcmp(key, "last_team")) *value = g->rb_team;
    else if (!strcmp(key, "last_slots")) *value = g->rb_slots;
    else return fail(KADABRA_EINVAL, "unknown parameter '%s'", key);
    return KADABRA_OK;
}

int kadabra_set_stream(kadabra_graph *g, void *hip_stream)
{
    if (!g) return fail(KADABRA_EINVAL, "null handle");
    g->stream = hip_stream ? (hipStream_t)hip_stream : g->own_stream;
    return KADABRA_OK;
}

int kadabra_run(kadabra_graph *g, double eps, double delta, uint64_t seed)
{
    if (!g) return fail(KADABRA_EINVAL, "null handle");
    g_last_error.clear();
    return run_impl(g, eps, delta, seed);
}

int kadabra_get_scores(const kadabra_graph *g, double *scores, int32_t *counts, kadabra_stats *stats)
{
    if (!g) return fail(KADABRA_EINVAL, "null handle");
    if (!g->have_result) return fail(KADABRA_ESTATE, "no completed run");
    kadabra_graph *mg = const_cast<kadabra_graph *>(g);
    const size_t n = (size_t)g->n;
    if (scores) {
        if (!mg->d_scores) HIP_OR_FAIL(dev_alloc((void **)&mg->d_scores, n * sizeof(double)));
        HIP_OR_FAIL(kd::launch_scores(g->d_counts, mg->d_scores, g->n, g->tau, g->stream));
        HIP_OR_FAIL(hipMemcpyAsync(scores, mg->d_scores, n * sizeof(double), hipMemcpyDeviceToHost, g->stream));
    }
    if (counts)
        HIP_OR_FAIL(hipMemcpyAsync(counts, g->d_counts, n * sizeof(int32_t), hipMemcpyDeviceToHost, g->stream));
    HIP_OR_FAIL(hipStreamSynchronize(g->stream));
    if (stats) {
        memset(stats, 0, sizeof *stats);
        stats->tau = g->tau;
        stats->omega = g->omega;
        stats->vd_bound = g->vd;
        stats->epochs = g->epochs;
        stats->decision = g->decision;
        stats->v_exp = g->work[kd::ST_VEXP];
        stats->e_scan = g->work[kd::ST_ESCAN];
        stats->e_bt = g->work[kd::ST_EBT];
        stats->path_interior = g->work[kd::ST_INTERIOR];
        stats->disconnected = g->work[kd::ST_DISCONN];
        stats->log_inv_delta = g->L;
        stats->ms_sampling = g->ms_sampling;
        stats->ms_total = g->ms_total;
        stats->ms_sample_kernels = g->ms_kernels;
        stats->sample_launches = g->epochs;
    }
    return KADABRA_OK;
}

int kadabra_get_scores_device(const kadabra_graph *g, double *scores_dev, int32_t *counts_dev)
{
    if (!g) return fail(KADABRA_EINVAL, "null handle");
    if (!g->have_result) return fail(KADABRA_ESTATE, "no completed run");
    if (scores_dev) HIP_OR_FAIL(kd::launch_scores(g->d_counts, scores_dev, g->n, g->tau, g->stream));
    if (counts_dev)
        HIP_OR_FAIL(hipMemcpyAsync(counts_dev, g->d_counts, (size_t)g->n * sizeof(int32_t),
                                   hipMemcpyDeviceToDevice, g->stream));
    return KADABRA_OK;
}

int kadabra_get_decisions(const kadabra_graph *g, int8_t *out, int64_t cap, int64_t *count)
{
    if (!g) return fail(KADABRA_EINVAL, "null handle");
    if (!g->have_result) return fail(KADABRA_ESTATE, "no completed run");
    const int64_t m = (int64_t)g->decisions.size();
    if (out)
        for (int64_t q = 0; q < std::min(cap, m); ++q) out[q] = g->decisions[(size_t)q];
    if (count) *count = m;
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
    if ((e = dev_alloc((void **)&d_c, m * sizeof(int32_t))) != hipSuccess ||
        (e = dev_alloc((void **)&d_f, m * sizeof(double))) != hipSuccess ||
        (e = dev_alloc((void **)&d_g, m * sizeof(double))) != hipSuccess) {
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

#ifdef KADABRA_PHASE_TIMERS
// Phase-timer builds only: cycles per sampler phase summed over all launches
// of the last run (0 pair, 1 expansion, 2 level bookkeeping, 3 meeting draw,
// 4 backtracking, 5 clearing).
int kadabra_debug_phase_cycles(const kadabra_graph *g, int64_t *out8)
{
    if (!g || !g->d_ctl || !out8) return fail(KADABRA_EINVAL, "bad argument");
    kd::Control ctl;
    HIP_OR_FAIL(hipMemcpy(&ctl, g->d_ctl, sizeof ctl, hipMemcpyDeviceToHost));
    for (int k = 0; k < 8; ++k) out8[k] = ctl.phase_cycles[k];
    return KADABRA_OK;
}
#endif

int kadabra_cancel(kadabra_graph *g)
{
    if (!g) return fail(KADABRA_EINVAL, "null handle");
    g->cancel.store(1);
    return KADABRA_OK;
}

void kadabra_destroy_graph(kadabra_graph *g)
{
    if (!g) return;
    (void)hipStreamSynchronize(g->stream);
    delete g;
}

}  // extern "C"
