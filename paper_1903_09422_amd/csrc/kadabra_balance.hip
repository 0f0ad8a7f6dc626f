// kadabra_balance.hip -- the device part of choosing per-vertex failure
// probabilities delta_L(v), delta_U(v) before the adaptive loop.
//
// Section 2.3 bounds only their sum over the vertices.  A first sampling phase
// (sample indices 2^63 + m, which the adaptive loop never draws) counts c1(v)
// for every vertex; the constants depend on v only through c1(v).  This
// kernel reduces c1 to its histogram hist[k] = #{v : c1(v) = k}, k <= m1;
// the host plans the target sample count t* and the constant per count from
// it (balance_plan in kadabra_host.cpp), and the stopping check looks the
// constants up by c1(v).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kadabra_internal.h"

namespace kd {

constexpr int HIST_BLOCK = 256;
constexpr int HIST_GRID = 256;   // one workgroup per CU: few global atomics per bin
constexpr int HIST_BINS = 256;   // counts below this are binned in LDS first

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

hipError_t launch_hist(const int32_t *c1, int32_t n, int32_t *hist, int64_t m1, Control *ctl, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    size_t g = ((size_t)n + HIST_BLOCK - 1) / HIST_BLOCK;
    if (g > HIST_GRID) g = HIST_GRID;
    hipLaunchKernelGGL(hist_kernel, dim3((unsigned)g), dim3(HIST_BLOCK), 0, s, c1, n, hist, m1, ctl);
    return hipGetLastError();
}


}  // namespace kd
