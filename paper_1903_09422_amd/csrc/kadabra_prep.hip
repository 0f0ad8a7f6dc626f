// kadabra_prep.hip -- graph-only preprocessing on the device (gfx950).
//
// What the adaptive loop needs from the graph alone (Section 2.3, Appendix
// C.1): a component id per vertex (a pair in different components is counted
// without a search) and the vertex-diameter bound VD.  Per component, a BFS
// from its maximum-degree vertex (lowest id on ties) reaches every vertex
// within ecc levels, and any shortest path there has at most 2 ecc edges, so
// VD = max over components of 2 ecc + 1.  As VD is a maximum over components,
// one BFS from all roots at once gives it: VD = 2 (deepest level) + 1.
//
//   components   union-find over the arcs: a root is hooked under a smaller
//                root by compare-and-swap, finds compress their paths; the
//                final parent of every vertex is its component's smallest id
//                (independent of the order of the hooks)
//   roots        per component, the maximum of (degree, n - 1 - id) by a
//                64-bit atomic max at the component's smallest id
//   BFS          level-synchronous from all roots; arcs of a chunk of frontier
//                vertices are spread over a workgroup's lanes (exclusive scan
//                of the degrees, owner found by binary search), so that hub
//                rows are shared; while the frontier is small one workgroup
//                runs many levels in a row (long paths, road-like graphs)
#include <hip/hip_runtime.h>

#include "kadabra_internal.h"

namespace kd {

namespace {

constexpr int PB = 256;  // threads per preprocessing block

__device__ __forceinline__ int32_t find_root(int32_t *parent, int32_t v)
{
    int32_t p = parent[v];
    while (p != v) {
        const int32_t gp = parent[p];
        if (gp != p) parent[v] = gp;  // path halving: any ancestor is a valid parent
        v = p;
        p = gp;
    }
    return v;
}

// Links the components of u and w: the larger root goes under the smaller.
__device__ void link(int32_t *parent, int32_t u, int32_t w)
{
    int32_t ru = find_root(parent, u), rw = find_root(parent, w);
    while (ru != rw) {
        const int32_t hi = ru > rw ? ru : rw, lo = ru > rw ? rw : ru;
        const int32_t old = atomicCAS(&parent[hi], hi, lo);
        if (old == hi) return;
        // hi was hooked meanwhile: continue from the roots of both sides
        ru = find_root(parent, old);
        rw = find_root(parent, lo);
    }
}

__global__ void iota_kernel(int32_t *p, int32_t n)
{
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) p[v] = v;
}

// Per block, a chunk of PB consecutive items: vertex ids (list == nullptr) or
// the entries list[base + k].  Their arcs are spread over the block's lanes.
struct ArcChunk {
    int32_t rs[PB];
    int32_t pfx[PB];
    int32_t u[PB];
    int32_t total;
};

__device__ void load_chunk(ArcChunk &c, const int32_t *row_ptr, const int32_t *list, int32_t base,
                           int32_t count)
{
    const int lane = threadIdx.x;
    const int32_t k = base + lane;
    int32_t dg = 0;
    if (k < count) {
        const int32_t u = list ? list[k] : k;
        c.u[lane] = u;
        c.rs[lane] = row_ptr[u];
        dg = row_ptr[u + 1] - c.rs[lane];
    }
    c.pfx[lane] = dg;
    __syncthreads();
    // inclusive scan (Hillis-Steele) of the degrees in LDS
    for (int o = 1; o < PB; o <<= 1) {
        const int32_t add = (lane >= o) ? c.pfx[lane - o] : 0;
        __syncthreads();
        c.pfx[lane] += add;
        __syncthreads();
    }
    if (lane == PB - 1) c.total = c.pfx[PB - 1];
    __syncthreads();
}

// owner k of the chunk's arc e: pfx[k - 1] <= e < pfx[k]
__device__ __forceinline__ int32_t chunk_owner(const ArcChunk &c, int32_t e, int32_t cnt)
{
    int32_t lo = 0, hi = cnt - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (c.pfx[mid] > e) hi = mid; else lo = mid + 1;
    }
    return lo;
}

__global__ __launch_bounds__(PB) void cc_link_kernel(const int32_t *row_ptr, const int32_t *col, int32_t n,
                                                     int32_t *parent)
{
    __shared__ ArcChunk c;
    for (int32_t base = blockIdx.x * PB; base < n; base += gridDim.x * PB) {
        load_chunk(c, row_ptr, nullptr, base, n);
        const int32_t cnt = min(PB, n - base);
        for (int32_t e = threadIdx.x; e < c.total; e += PB) {
            const int32_t k = chunk_owner(c, e, cnt);
            const int32_t u = c.u[k];
            const int32_t w = col[c.rs[k] + e - (k ? c.pfx[k - 1] : 0)];
            if (u < w) link(parent, u, w);  // each edge once
        }
        __syncthreads();
    }
}

// Every vertex points at its root.  The walk only reads: a halving write by
// one thread could otherwise replace another vertex's final root pointer by a
// non-root ancestor.  Each parent[v] is written once, by its own thread.
__global__ void cc_flatten_kernel(int32_t *parent, int32_t n)
{
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        int32_t r = parent[v];
        while (parent[r] != r) r = parent[r];
        parent[v] = r;
    }
}

// key[c] = max over the component's vertices of (degree << 32 | (n - 1 - id)).
// A wavefront whose vertices all lie in one component (the usual case: one
// large component) takes the maximum by shuffles and makes one atomic.
__global__ void root_key_kernel(const int32_t *row_ptr, const int32_t *comp, int32_t n,
                                unsigned long long *key)
{
    const int32_t stride = gridDim.x * blockDim.x;
    const int32_t start = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t span = (n + stride - 1) / stride * stride;  // same trip count for all lanes
    for (int32_t v = start; v < span; v += stride) {
        const bool in = v < n;
        const int32_t c = in ? comp[v] : -1;
        unsigned long long k = in ? (((unsigned long long)(uint32_t)(row_ptr[v + 1] - row_ptr[v]) << 32) |
                                     (unsigned long long)(uint32_t)(n - 1 - v))
                                  : 0ull;
        const int32_t c0 = __shfl(c, 0, 64);
        if (__all(!in || c == c0) && c0 >= 0) {
            for (int o = 32; o > 0; o >>= 1) {
                const unsigned long long x = __shfl_xor(k, o, 64);
                k = x > k ? x : k;
            }
            if ((threadIdx.x & 63) == 0) atomicMax(&key[c0], k);
        } else if (in) {
            atomicMax(&key[c], k);
        }
    }
}

// dist = -1 everywhere, 0 at the roots, which form the first frontier;
// counters[2] = number of components
__global__ void bfs_init_kernel(const int32_t *comp, const unsigned long long *key, int32_t n, int32_t *dist,
                                int32_t *frontier, int32_t *counters)
{
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        int32_t d = -1;
        if (comp[v] == v) atomicAdd(&counters[2], 1);
        const int32_t root = n - 1 - (int32_t)(uint32_t)(key[comp[v]] & 0xFFFFFFFFull);
        if (root == v) {
            d = 0;
            frontier[atomicAdd(&counters[0], 1)] = v;
        }
        dist[v] = d;
    }
}

// One level: the frontier's unreached neighbours get level + 1 and are
// appended to next (*next_count).
__global__ __launch_bounds__(PB) void bfs_level_kernel(const int32_t *row_ptr, const int32_t *col,
                                                       const int32_t *frontier, const int32_t *count,
                                                       int32_t level, int32_t *dist, int32_t *next,
                                                       int32_t *next_count)
{
    __shared__ ArcChunk c;
    const int32_t fn = *count;
    for (int32_t base = blockIdx.x * PB; base < fn; base += gridDim.x * PB) {
        load_chunk(c, row_ptr, frontier, base, fn);
        const int32_t cnt = min(PB, fn - base);
        for (int32_t e = threadIdx.x; e < c.total; e += PB) {
            const int32_t k = chunk_owner(c, e, cnt);
            const int32_t w = col[c.rs[k] + e - (k ? c.pfx[k - 1] : 0)];
            if (dist[w] < 0 && atomicCAS(&dist[w], -1, level + 1) == -1) next[atomicAdd(next_count, 1)] = w;
        }
        __syncthreads();
    }
}

// Runs levels in one workgroup while the frontier has at most small_max
// vertices.  Queues q0/q1 alternate; state[0] = frontier size, state[1] =
// level, state[2] = which queue holds the frontier; on exit the frontier is
// empty or larger than small_max.
__global__ __launch_bounds__(PB) void bfs_small_kernel(const int32_t *row_ptr, const int32_t *col,
                                                       int32_t *dist, int32_t *q0, int32_t *q1,
                                                       int32_t *state, int32_t small_max)
{
    __shared__ ArcChunk c;
    __shared__ int32_t nnext;
    int32_t fn = state[0], level = state[1], which = state[2];
    while (fn > 0 && fn <= small_max) {
        const int32_t *cur = which ? q1 : q0;
        int32_t *nxt = which ? q0 : q1;
        if (threadIdx.x == 0) nnext = 0;
        __syncthreads();
        for (int32_t base = 0; base < fn; base += PB) {
            load_chunk(c, row_ptr, cur, base, fn);
            const int32_t cnt = min(PB, fn - base);
            for (int32_t e = threadIdx.x; e < c.total; e += PB) {
                const int32_t k = chunk_owner(c, e, cnt);
                const int32_t w = col[c.rs[k] + e - (k ? c.pfx[k - 1] : 0)];
                if (dist[w] < 0 && atomicCAS(&dist[w], -1, level + 1) == -1) nxt[atomicAdd(&nnext, 1)] = w;
            }
            __syncthreads();
        }
        fn = nnext;
        level += 1;
        which ^= 1;
        __syncthreads();  // every thread has read nnext before it is reset
    }
    if (threadIdx.x == 0) {
        state[0] = fn;
        state[1] = level;
        state[2] = which;
    }
}

unsigned grid_of(int64_t items, unsigned block)
{
    int64_t g = (items + block - 1) / block;
    if (g > 4096) g = 4096;
    return g < 1 ? 1u : (unsigned)g;
}

}  // namespace

hipError_t launch_cc(const int32_t *row_ptr, const int32_t *col, int32_t n, int32_t *parent, hipStream_t s)
{
    hipLaunchKernelGGL(iota_kernel, dim3(grid_of(n, 256)), dim3(256), 0, s, parent, n);
    hipLaunchKernelGGL(cc_link_kernel, dim3(grid_of(n, PB)), dim3(PB), 0, s, row_ptr, col, n, parent);
    hipLaunchKernelGGL(cc_flatten_kernel, dim3(grid_of(n, 256)), dim3(256), 0, s, parent, n);
    return hipGetLastError();
}

hipError_t launch_bfs_roots(const int32_t *row_ptr, const int32_t *comp, int32_t n, unsigned long long *key,
                            int32_t *dist, int32_t *frontier, int32_t *counters, hipStream_t s)
{
    hipLaunchKernelGGL(root_key_kernel, dim3(grid_of(n, 256)), dim3(256), 0, s, row_ptr, comp, n, key);
    hipLaunchKernelGGL(bfs_init_kernel, dim3(grid_of(n, 256)), dim3(256), 0, s, comp, key, n, dist, frontier,
                       counters);
    return hipGetLastError();
}

hipError_t launch_bfs_level(const int32_t *row_ptr, const int32_t *col, const int32_t *frontier,
                            const int32_t *count, int32_t frontier_size, int32_t level, int32_t *dist,
                            int32_t *next, int32_t *next_count, hipStream_t s)
{
    hipLaunchKernelGGL(bfs_level_kernel, dim3(grid_of(frontier_size, PB)), dim3(PB), 0, s, row_ptr, col, frontier,
                       count, level, dist, next, next_count);
    return hipGetLastError();
}

hipError_t launch_bfs_small(const int32_t *row_ptr, const int32_t *col, int32_t *dist, int32_t *q0, int32_t *q1,
                            int32_t *state, int32_t small_max, hipStream_t s)
{
    hipLaunchKernelGGL(bfs_small_kernel, dim3(1), dim3(PB), 0, s, row_ptr, col, dist, q0, q1, state, small_max);
    return hipGetLastError();
}

// dst[i] = src[idx[i]] (a relabelled copy of a per-vertex array)
__global__ void gather_i32_kernel(int32_t *dst, const int32_t *src, const int32_t *idx, int32_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[idx[i]];
}

hipError_t launch_gather_i32(int32_t *dst, const int32_t *src, const int32_t *idx, int32_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    size_t g = ((size_t)n + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(gather_i32_kernel, dim3((unsigned)g), dim3(256), 0, s, dst, src, idx, n);
    return hipGetLastError();
}

// Zeroes up to kMaxZeroRegions device regions in one launch: block (x, y)
// strides over region y.
__global__ void zero_regions_kernel(ZeroRegions z)
{
    const int r = (int)blockIdx.y;
    uint32_t *const p = z.ptr[r];
    const size_t count = z.count[r];
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (size_t)gridDim.x * blockDim.x)
        p[k] = 0u;
}

hipError_t launch_zero_regions(const ZeroRegions &z, hipStream_t s)
{
    if (z.n <= 0) return hipSuccess;
    if (z.n > kMaxZeroRegions) return hipErrorInvalidValue;
    size_t most = 1;
    for (int r = 0; r < z.n; ++r) most = z.count[r] > most ? z.count[r] : most;
    size_t g = (most + 255) / 256;
    if (g > 2048) g = 2048;
    hipLaunchKernelGGL(zero_regions_kernel, dim3((unsigned)g, (unsigned)z.n), dim3(256), 0, s, z);
    return hipGetLastError();
}

}  // namespace kd
