// kadabra_balance.hip -- per-vertex failure probabilities delta_L(v),
// delta_U(v) for the stopping rule, chosen before the adaptive loop.
//
// Section 2.3 bounds only their sum over the vertices (at most delta); this
// code spends delta/2 on it (the omega cap takes the other half) and splits it
// by a rule derived from the f and g of Appendix B:
//   - a first phase of m1 samples (sample indices 2^63 + m: the adaptive loop
//     never draws them) counts c1(v); planning value b_p = (c1 + 1) / m1;
//   - at a target sample count t, the largest log(1/delta) with f <= eps is
//     t eps^2 / (q + 2 eps af), af = 1/3 - w/t, q = 2 b_p w / t (unbounded
//     when the denominator is <= 0, since f then stays below eps for every
//     constant), and for g the same with ag = 1/3 + w/t;
//   - S(t) = sum_v exp(-L_f) + exp(-L_g); t* = bisection on [1, omega] for
//     S(t) <= 0.9 (delta/2) (1 - 1e-6) (the factor covers the rounding of
//     S); a bisection that ends at omega leaves the uniform constant L;
//   - delta_L(v) = 0.9 exp(-L_f(v, t*)) + 0.1 delta / (4 n), delta_U(v) with
//     L_g, so the floor share 0.1 (delta/2) is spread evenly.
// The constants depend on v only through c1(v): they are computed once per
// count k = 0 .. m1, and the stopping check looks them up.  S(t) is summed over
// the count histogram, hist[k] (exp(-L_f(k)) + exp(-L_g(k))), in a fixed
// order inside one workgroup, so t* does not depend on the schedule.  The
// file is compiled without floating-point contraction; every expression is
// evaluated in the order written.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kadabra_internal.h"

namespace kd {

constexpr double kBalanceFloor = 0.1;  // share of the budget spread evenly
constexpr int HIST_BLOCK = 256;
constexpr int HIST_GRID = 256;   // one workgroup per CU: few global atomics per bin
constexpr int HIST_BINS = 256;   // counts below this are binned in LDS first
constexpr int PLAN_BLOCK = 1024;
constexpr int PLAN_CACHE = 4096; // nonzero histogram rows kept in LDS during the search

// hist[k] += 1 for every vertex with c1 = k.  Most vertices have c1 = 0 and
// the counts are small: a workgroup bins counts below HIST_BINS in LDS (a
// wavefront adds its zeros with one LDS atomic) and adds each nonzero bin to
// hist once.
__global__ __launch_bounds__(HIST_BLOCK) void hist_kernel(const int32_t *c1, int32_t n, int32_t *hist,
                                                          int64_t m1, Control *ctl)
{
    __shared__ int32_t bins[HIST_BINS];
    for (int k = threadIdx.x; k < HIST_BINS; k += HIST_BLOCK) bins[k] = 0;
    __syncthreads();
    const size_t stride = (size_t)gridDim.x * HIST_BLOCK;
    const int lane = threadIdx.x & 63;
    // every lane of a wavefront runs the same iterations (the ballot needs them all)
    for (size_t base = (size_t)blockIdx.x * HIST_BLOCK; base < (size_t)n; base += stride) {
        const size_t v = base + threadIdx.x;
        const int32_t k = v < (size_t)n ? c1[v] : -1;
        const uint64_t zeros = __ballot(v < (size_t)n && k == 0);
        if (lane == 0 && zeros) atomicAdd(&bins[0], (int32_t)__popcll(zeros));
        if (v < (size_t)n && k != 0) {
            if (k < 0 || (int64_t)k > m1) {
                if (atomicCAS(&ctl->err, 0, 4) == 0)
                    atomicExch((unsigned long long *)&ctl->err_sample, (unsigned long long)v);
            } else if (k < HIST_BINS) {
                atomicAdd(&bins[k], 1);
            } else {
                atomicAdd(&hist[k], 1);
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < HIST_BINS; k += HIST_BLOCK)
        if (bins[k]) atomicAdd(&hist[k], bins[k]);  // a nonzero bin has k <= m1
}

__device__ __forceinline__ void plan_lfg(double b, double t, double w, double eps, double *lf, double *lg)
{
    const double af = 1.0 / 3.0 - w / t;
    const double ag = 1.0 / 3.0 + w / t;
    const double q = 2.0 * b * w / t;
    const double df = q + 2.0 * eps * af;
    const double dg = q + 2.0 * eps * ag;
    const double e2 = eps * eps;
    *lf = (df > 0.0) ? t * e2 / df : __builtin_inf();
    *lg = t * e2 / dg;
}

// Sum over the workgroup; every thread returns the same value.
__device__ __forceinline__ double plan_block_sum(double x, double *red)
{
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    __syncthreads();  // the previous sum's reads of red are done
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < PLAN_BLOCK / 64; ++k) s += red[k];
    return s;
}

__global__ __launch_bounds__(PLAN_BLOCK) void plan_kernel(PlanArgs a)
{
    __shared__ double red[PLAN_BLOCK / 64];
    __shared__ double cb[PLAN_CACHE];   // planning values b_p of the nonzero rows, ascending k
    __shared__ int32_t ch[PLAN_CACHE];  // their vertex counts
    __shared__ int32_t wsum[PLAN_BLOCK / 64];
    const double beta = kBalanceFloor;
    const double target = (1.0 - beta) * (a.delta / 2.0) * (1.0 - 1e-6);
    const double w = (double)a.omega;
    const double m1 = (double)a.m1;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;

    // the nonzero rows of the histogram, in ascending k, into LDS (all of
    // them if they fit; otherwise the search reads the histogram itself)
    int32_t rows = 0;
    for (int64_t base = 0; base <= a.m1; base += PLAN_BLOCK) {
        const int64_t k = base + threadIdx.x;
        const int32_t h = k <= a.m1 ? a.hist[k] : 0;
        const uint64_t nz = __ballot(h != 0);
        __syncthreads();  // the previous chunk's reads of wsum are done
        if (lane == 0) wsum[wv] = (int32_t)__popcll(nz);
        __syncthreads();
        int32_t before = 0, chunk = 0;
        for (int j = 0; j < PLAN_BLOCK / 64; ++j) {
            before += j < wv ? wsum[j] : 0;
            chunk += wsum[j];
        }
        const int32_t pos = rows + before + (int32_t)__popcll(nz & ((1ull << lane) - 1));
        if (h != 0 && pos < PLAN_CACHE) {
            cb[pos] = ((double)k + 1.0) / m1;
            ch[pos] = h;
        }
        rows += chunk;
    }
    const bool cached = rows <= (a.cache_rows > 0 ? a.cache_rows : PLAN_CACHE);
    __syncthreads();

    // bisection for t*: S(t) is the same value in every thread, so every
    // thread takes the same branch and runs the same number of rounds
    int64_t lo = 1, hi = a.omega;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        const double t = (double)mid;
        double part = 0.0;
        if (cached) {
            for (int32_t j = threadIdx.x; j < rows; j += PLAN_BLOCK) {
                double lf, lg;
                plan_lfg(cb[j], t, w, a.eps, &lf, &lg);
                part += (double)ch[j] * (exp(-lf) + exp(-lg));
            }
        } else {
            for (int64_t k = threadIdx.x; k <= a.m1; k += PLAN_BLOCK) {
                const int32_t h = a.hist[k];
                if (h == 0) continue;
                double lf, lg;
                plan_lfg(((double)k + 1.0) / m1, t, w, a.eps, &lf, &lg);
                part += (double)h * (exp(-lf) + exp(-lg));
            }
        }
        if (plan_block_sum(part, red) <= target) hi = mid;
        else lo = mid + 1;
    }
    const bool found = lo < a.omega;
    const double t = (double)lo;
    const double floor_share = beta * a.delta / (4.0 * (double)a.n);
    for (int64_t k = threadIdx.x; k <= a.m1; k += PLAN_BLOCK) {
        double LL = a.L, LU = a.L;
        if (found) {
            double lf, lg;
            plan_lfg(((double)k + 1.0) / m1, t, w, a.eps, &lf, &lg);
            LL = -log((1.0 - beta) * exp(-lf) + floor_share);
            LU = -log((1.0 - beta) * exp(-lg) + floor_share);
        }
        a.lcon[2 * k] = LL;
        a.lcon[2 * k + 1] = LU;
    }
    if (threadIdx.x == 0) a.ctl->plan_tau = found ? lo : 0;
}

hipError_t launch_hist(const int32_t *c1, int32_t n, int32_t *hist, int64_t m1, Control *ctl, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    size_t g = ((size_t)n + HIST_BLOCK - 1) / HIST_BLOCK;
    if (g > HIST_GRID) g = HIST_GRID;
    hipLaunchKernelGGL(hist_kernel, dim3((unsigned)g), dim3(HIST_BLOCK), 0, s, c1, n, hist, m1, ctl);
    return hipGetLastError();
}

hipError_t launch_plan(const PlanArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(PLAN_BLOCK), 0, s, a);
    return hipGetLastError();
}

}  // namespace kd
