// kadabra_kernels.hip -- gfx950 kernels of the KADABRA adaptive-sampling path.
//
//   sample_kernel      one team (one to eight wavefronts) per sample in flight;
//                      persistent over the sample indices of the launch (one or
//                      more epochs of each query, and a balanced query's first
//                      phase), claimed from a counter.  Per sample: pair draw,
//                      same-component test, balanced bidirectional BFS with
//                      128-bit path counts (small levels summed in LDS), the
//                      meeting-vertex draw, backtracking on CSR + distances,
//                      +1 on the interior vertices (Section 2.3, Appendix C.1).
//   merge_check_kernel counters += frames of the epoch (frames zeroed), then
//                      the FP64 stopping rule f, g <= eps of Appendix B for
//                      every vertex (uniform or per-vertex constants); one
//                      violation flag per epoch.
//   scores_kernel      b~(v) = c(v) / tau.
//
// All path counts and weights are integers, so sums done with atomics in any
// order give bit-identical results: the output does not depend on the
// schedule (the determinism of the indexed-frame algorithm, Appendix D).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kadabra_internal.h"

namespace kd {

typedef unsigned __int128 u128;

constexpr int SIGMA_BITS = 104;  // a level is rescaled once its largest count reaches 2^104
constexpr int WEIGHT_BITS = 40;  // meeting weights are rounded up to at most 2^40

// ---------------------------------------------------------------------------
// Counter-based random numbers: Philox4x32-10 (Salmon et al., SC'11).
// Draw j of sample i is the block at counter (i_lo, i_hi, j, 0) under key seed.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t philox_u64(uint64_t seed, uint64_t i, uint32_t j,
                                               uint64_t *second = nullptr)
{
    uint32_t c0 = (uint32_t)i, c1 = (uint32_t)(i >> 32), c2 = j, c3 = 0u;
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t a0 = 0xD2511F53u * c0, b0 = __umulhi(0xD2511F53u, c0);
        const uint32_t a1 = 0xCD9E8D57u * c2, b1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = b1 ^ c1 ^ k0;
        const uint32_t n2 = b0 ^ c3 ^ k1;
        c0 = n0;
        c1 = a1;
        c2 = n2;
        c3 = a0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    if (second) *second = (uint64_t)c2 | ((uint64_t)c3 << 32);
    return (uint64_t)c0 | ((uint64_t)c1 << 32);
}

__device__ __forceinline__ u128 to128(Sigma s) { return ((u128)s.hi << 64) | s.lo; }

__device__ __forceinline__ int bitw128(u128 x)
{
    const uint64_t hi = (uint64_t)(x >> 64), lo = (uint64_t)x;
    return hi ? 128 - __clzll((long long)hi) : (lo ? 64 - __clzll((long long)lo) : 0);
}

// Workgroup-scope atomics on a sample's private state.
__device__ __forceinline__ uint64_t wg_add_u64(uint64_t *p, uint64_t v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint32_t wg_or_u32(uint32_t *p, uint32_t v)
{
    return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Level codes.  A neighbour of a vertex on BFS level l lies on level l - 1, l
// or l + 1 (or is unreached), so (level mod 3) + 1 in two bits per side
// identifies it; 0 = unreached.  Vertex w's codes sit in word w / 8 at bit
// 4 (w mod 8) (side s) and 4 (w mod 8) + 2 (side t).
__device__ __forceinline__ uint32_t level_code(int32_t level) { return (uint32_t)(level % 3) + 1u; }
__device__ __forceinline__ int code_shift(int32_t w, int side) { return 4 * (w & 7) + 2 * side; }

// floor(u * m / 2^64) for 64-bit u and 128-bit m < 2^127
__device__ __forceinline__ u128 mulhi_64x128(uint64_t u, u128 m)
{
    const uint64_t m_lo = (uint64_t)m, m_hi = (uint64_t)(m >> 64);
    const u128 lo = (u128)u * m_lo;
    const u128 hi = (u128)u * m_hi;
    return hi + (lo >> 64);
}

// Meeting weight: ceil(a * b / 2^sh) for a, b < 2^128 with a result < 2^64.
struct U256 {
    u128 hi, lo;
};

__device__ __forceinline__ U256 mul_128x128(u128 a, u128 b)
{
    const uint64_t a0 = (uint64_t)a, a1 = (uint64_t)(a >> 64);
    const uint64_t b0 = (uint64_t)b, b1 = (uint64_t)(b >> 64);
    const u128 p00 = (u128)a0 * b0, p01 = (u128)a0 * b1, p10 = (u128)a1 * b0,
               p11 = (u128)a1 * b1;
    const u128 mid = (p00 >> 64) + (uint64_t)p01 + (uint64_t)p10;
    U256 r;
    r.lo = (u128)(uint64_t)p00 | (mid << 64);
    r.hi = p11 + (p01 >> 64) + (p10 >> 64) + (mid >> 64);
    return r;
}

__device__ __forceinline__ int bitw256(U256 x) { return x.hi ? 128 + bitw128(x.hi) : bitw128(x.lo); }

__device__ __forceinline__ uint64_t ceil_shr256(U256 x, int sh)
{
    if (sh == 0) return (uint64_t)x.lo;
    u128 q;
    bool rem;
    if (sh < 128) {
        q = (x.lo >> sh) | (x.hi << (128 - sh));
        rem = (x.lo << (128 - sh)) != 0;
    } else if (sh == 128) {
        q = x.hi;
        rem = x.lo != 0;
    } else {
        q = x.hi >> (sh - 128);
        rem = x.lo != 0 || (x.hi << (256 - sh)) != 0;
    }
    return (uint64_t)q + (rem ? 1u : 0u);
}

// ---------------------------------------------------------------------------
// Wavefront scans on the data-parallel primitives (DPP) of the vector ALU.
// dmov<CTRL, ROWS>(x) is x moved across the lanes of a wavefront by a fixed
// pattern; a lane with no source, or in a row (16 lanes) that ROWS leaves
// out, receives 0.  wave_scan is an inclusive scan in lane order for an
// associative op with identity 0 (a sum, an unsigned maximum): row_shr by 1,
// 2, 4 and 8 scans each row, then the last lane of rows 0 and 2 is combined
// into rows 1 and 3 (row_bcast:15) and the last lane of row 1 into rows 2
// and 3 (row_bcast:31).  Every lane must be active.  last_lane reads lane 63
// (the whole wavefront's result) into scalar registers.
// ---------------------------------------------------------------------------
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dmov(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dmov(uint64_t x)
{
    return (uint64_t)dmov<CTRL, ROWS>((uint32_t)x) | ((uint64_t)dmov<CTRL, ROWS>((uint32_t)(x >> 32)) << 32);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ u128 dmov(u128 x)
{
    return (u128)dmov<CTRL, ROWS>((uint64_t)x) | ((u128)dmov<CTRL, ROWS>((uint64_t)(x >> 64)) << 64);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ U256 dmov(U256 x)
{
    return U256{dmov<CTRL, ROWS>(x.hi), dmov<CTRL, ROWS>(x.lo)};
}

template <typename V, typename Op>
__device__ __forceinline__ V wave_scan(V x, Op op)
{
    x = op(x, dmov<0x111, 0xf>(x));  // row_shr:1
    x = op(x, dmov<0x112, 0xf>(x));  // row_shr:2
    x = op(x, dmov<0x114, 0xf>(x));  // row_shr:4
    x = op(x, dmov<0x118, 0xf>(x));  // row_shr:8
    x = op(x, dmov<0x142, 0xa>(x));  // row_bcast:15 into rows 1 and 3
    x = op(x, dmov<0x143, 0xc>(x));  // row_bcast:31 into rows 2 and 3
    return x;
}

__device__ __forceinline__ uint32_t last_lane(uint32_t x) { return (uint32_t)__builtin_amdgcn_readlane((int)x, 63); }
__device__ __forceinline__ uint64_t last_lane(uint64_t x)
{
    return (uint64_t)last_lane((uint32_t)x) | ((uint64_t)last_lane((uint32_t)(x >> 32)) << 32);
}
__device__ __forceinline__ u128 last_lane(u128 x)
{
    return (u128)last_lane((uint64_t)x) | ((u128)last_lane((uint64_t)(x >> 64)) << 64);
}
__device__ __forceinline__ U256 last_lane(U256 x) { return U256{last_lane(x.hi), last_lane(x.lo)}; }

struct OpAdd {
    template <typename V>
    __device__ __forceinline__ V operator()(V a, V b) const { return a + b; }
};
struct OpMax {
    template <typename V>
    __device__ __forceinline__ V operator()(V a, V b) const { return b > a ? b : a; }
    __device__ __forceinline__ U256 operator()(U256 a, U256 b) const
    {
        return (b.hi > a.hi || (b.hi == a.hi && b.lo > a.lo)) ? b : a;
    }
};

// ---------------------------------------------------------------------------
// Team primitives.  A team is the whole workgroup (TEAM == blockDim.x), one
// wavefront (64) or four (256).  A sample's state is touched by its own
// workgroup only, so workgroup scope is all the ordering it needs: sync() is
// the workgroup barrier, and the state's atomics are workgroup-scope (they
// resolve in the XCD's own L2 instead of travelling to memory).
// ---------------------------------------------------------------------------
template <int TEAM>
struct Team {
    static constexpr int WAVES = TEAM / 64;

    __device__ static __forceinline__ void sync() { __syncthreads(); }

    // Team reductions: result in every lane.  A reduction has one barrier,
    // before it reads the per-wavefront words in red; it does not wait for
    // those reads to finish, so consecutive reductions must use different red
    // buffers (the next reduction's barrier then guarantees the reads of the
    // one before it are done).  red: >= 4 WAVES words of LDS.
    //
    // sum over the team
    __device__ static uint64_t sum_u64(uint64_t v, uint64_t *red)
    {
        v = last_lane(wave_scan(v, OpAdd{}));
        if (WAVES == 1) return v;
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) red[w] = v;
        __syncthreads();
        uint64_t t = 0;
#pragma unroll
        for (int k = 0; k < WAVES; ++k) t += red[k];
        return t;
    }

    __device__ static u128 sum_u128(u128 v, uint64_t *red)
    {
        v = last_lane(wave_scan(v, OpAdd{}));
        if (WAVES == 1) return v;
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            red[2 * w] = (uint64_t)v;
            red[2 * w + 1] = (uint64_t)(v >> 64);
        }
        __syncthreads();
        u128 t = 0;
#pragma unroll
        for (int k = 0; k < WAVES; ++k) t += ((u128)red[2 * k + 1] << 64) | red[2 * k];
        return t;
    }

    // sums a 64-bit and a 128-bit value over the team with one exchange
    __device__ static void sum_u64_u128(uint64_t *a, u128 *b, uint64_t *red)
    {
        const uint64_t x = last_lane(wave_scan(*a, OpAdd{}));
        const u128 y = last_lane(wave_scan(*b, OpAdd{}));
        if (WAVES == 1) {
            *a = x;
            *b = y;
            return;
        }
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            red[3 * w] = x;
            red[3 * w + 1] = (uint64_t)y;
            red[3 * w + 2] = (uint64_t)(y >> 64);
        }
        __syncthreads();
        uint64_t tx = 0;
        u128 tb = 0;
#pragma unroll
        for (int k = 0; k < WAVES; ++k) {
            tx += red[3 * k];
            tb += ((u128)red[3 * k + 2] << 64) | red[3 * k + 1];
        }
        *a = tx;
        *b = tb;
    }

    __device__ static u128 max_u128(u128 v, uint64_t *red)
    {
        v = last_lane(wave_scan(v, OpMax{}));
        if (WAVES == 1) return v;
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            red[2 * w] = (uint64_t)v;
            red[2 * w + 1] = (uint64_t)(v >> 64);
        }
        __syncthreads();
        u128 t = 0;
#pragma unroll
        for (int k = 0; k < WAVES; ++k) {
            const u128 x = ((u128)red[2 * k + 1] << 64) | red[2 * k];
            t = x > t ? x : t;
        }
        return t;
    }

    __device__ static U256 max_u256(U256 v, uint64_t *red)
    {
        v = last_lane(wave_scan(v, OpMax{}));
        if (WAVES == 1) return v;
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            red[4 * w] = (uint64_t)v.lo;
            red[4 * w + 1] = (uint64_t)(v.lo >> 64);
            red[4 * w + 2] = (uint64_t)v.hi;
            red[4 * w + 3] = (uint64_t)(v.hi >> 64);
        }
        __syncthreads();
        U256 t{0, 0};
#pragma unroll
        for (int k = 0; k < WAVES; ++k) {
            U256 x;
            x.lo = ((u128)red[4 * k + 1] << 64) | red[4 * k];
            x.hi = ((u128)red[4 * k + 3] << 64) | red[4 * k + 2];
            if (x.hi > t.hi || (x.hi == t.hi && x.lo > t.lo)) t = x;
        }
        return t;
    }

    // exclusive prefix sum of an int over the team (lane order); *total in every lane
    __device__ static int32_t excl_scan_i32(int32_t v, int32_t *total, uint64_t *red)
    {
        const int lw = threadIdx.x & 63;
        const int32_t x = (int32_t)wave_scan((uint32_t)v, OpAdd{});
        if (WAVES == 1) {
            *total = (int32_t)last_lane((uint32_t)x);
            return x - v;
        }
        const int w = threadIdx.x >> 6;
        if (lw == 63) red[w] = (uint64_t)(uint32_t)x;
        __syncthreads();
        int32_t off = 0, tot = 0;
#pragma unroll
        for (int k = 0; k < WAVES; ++k) {
            const int32_t t = (int32_t)(uint32_t)red[k];
            off += (k < w) ? t : 0;
            tot += t;
        }
        *total = tot;
        return off + x - v;
    }

    // exclusive prefix sum of a 128-bit value over the team; *total in every lane
    __device__ static u128 excl_scan_u128(u128 v, u128 *total, uint64_t *red)
    {
        const int lw = threadIdx.x & 63;
        const u128 x = wave_scan(v, OpAdd{});
        if (WAVES == 1) {
            *total = last_lane(x);
            return x - v;
        }
        const int w = threadIdx.x >> 6;
        if (lw == 63) {
            red[2 * w] = (uint64_t)x;
            red[2 * w + 1] = (uint64_t)(x >> 64);
        }
        __syncthreads();
        u128 off = 0, tot = 0;
#pragma unroll
        for (int k = 0; k < WAVES; ++k) {
            const u128 t = ((u128)red[2 * k + 1] << 64) | red[2 * k];
            off += (k < w) ? t : (u128)0;
            tot += t;
        }
        *total = tot;
        return off + x - v;
    }
};

// A value every lane holds equally (read from LDS after a barrier), made
// scalar so that the compiler keeps what derives from it in scalar registers.
__device__ __forceinline__ int32_t uniform_i32(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform_i64(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Wave-aggregated append: every active lane with `take` receives a distinct
// slot index from the LDS counter *cnt (one LDS atomic per wavefront).
__device__ __forceinline__ int wave_append(bool take, int32_t *cnt)
{
    const uint64_t act = __ballot(take);
    if (act == 0) return -1;
    const int lw = threadIdx.x & 63;
    const int leader = __ffsll((unsigned long long)act) - 1;  // uniform
    int base = 0;
    if (lw == leader) base = atomicAdd(cnt, __popcll(act));
    base = __builtin_amdgcn_readlane(base, leader);
    // lanes of act below this one
    const int below = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(act >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u));
    return take ? base + below : -1;
}

// Optional per-phase cycle counters (compile with -DKADABRA_PHASE_TIMERS):
// lane 0 of each team adds the shader-clock cycles of each phase of a sample
// into Control::phase_cycles.  Off in the library build.
#ifdef KADABRA_PHASE_TIMERS
#define PHASE_BEGIN() uint64_t ph_t0_ = __builtin_readcyclecounter()
#define PHASE_MARK(k)                                                   \
    do {                                                                \
        const uint64_t ph_t1_ = __builtin_readcyclecounter();           \
        if (threadIdx.x == 0) ph_acc[k] += ph_t1_ - ph_t0_;             \
        ph_t0_ = ph_t1_;                                                \
    } while (0)
#else
#define PHASE_BEGIN() (void)0
#define PHASE_MARK(k) (void)0
#endif

// LDS staging capacity for the meeting set and for backtracking candidates
template <int TEAM>
struct Cap {
    static constexpr int STAGE = (TEAM == 64) ? 256 : (TEAM == 128) ? 512 : 1024;
};

template <int TEAM>
struct SampleShared {
    int32_t crs[TEAM];                // frontier chunk: first arc
    int32_t cpfx[TEAM];               // frontier chunk: exclusive prefix of degrees
    Sigma cm[TEAM];                   // frontier chunk: sigma of the vertex
    int32_t sv[Cap<TEAM>::STAGE];     // staged new level / meeting vertices / candidates
    Sigma sw[Cap<TEAM>::STAGE];       // their weights
    // per side, the frontier when it fits one chunk (filled when the level is
    // completed, read when that side expands next): first arc, degree, sigma
    int32_t frs[2][TEAM];
    int32_t fdg[2][TEAM];
    Sigma fsg[2][TEAM];
    uint64_t red[2][4 * (TEAM / 64) < 16 ? 16 : 4 * (TEAM / 64)];  // reduction scratch, used alternately
    uint64_t acc[ST_COUNT];           // work counters of the query being served (lane 0)
    int64_t claim;                    // claimed launch-wide sample index
    int32_t query;                    // its query
    int32_t nnext[2], nmeet[2];       // append counters of a level, used alternately
    int32_t pick, ncand;
};

// A const int32 in the global address space, and the cast to it.
typedef const __attribute__((address_space(1))) int32_t gint32_t;
__device__ __forceinline__ gint32_t *as_global(const int32_t *p) { return (gint32_t *)p; }

// true if key is in the sorted row[0, len): a 64-way search by the lanes of
// one wavefront (row, len and key the same in all of them).  Each round every
// lane loads the last entry of its segment and a ballot picks the first
// segment that can hold key, so a row of up to 4096 entries takes two
// dependent loads.  lw: the lane's index in its wavefront.
__device__ __forceinline__ bool wave_row_contains(gint32_t *row, int32_t len, int32_t key, int lw)
{
    int32_t lo = 0, hi = len;
    while (hi - lo > 64) {
        const int32_t seg = (hi - lo + 63) >> 6;
        const int32_t beg = lo + lw * seg;
        const int32_t end = min(beg + seg, hi);
        const int32_t last = (beg < hi) ? row[end - 1] : INT32_MAX;  // an empty segment never holds it
        const uint64_t ge = __ballot(last >= key);
        if (ge == 0) return false;  // key is above every entry
        lo += (__ffsll((unsigned long long)ge) - 1) * seg;
        hi = min(lo + seg, hi);
    }
    return __ballot(lw < hi - lo && row[lo + lw] == key) != 0;
}

// Among staged (id, weight) pairs sv/sw[0, cnt), the lane holding the
// smallest id whose inclusive prefix (ascending id) exceeds r writes it to
// *pick.  Ids are distinct; total weight > r.
template <int TEAM>
__device__ __forceinline__ void pick_by_id_prefix(const int32_t *sv, const Sigma *sw, int32_t cnt,
                                                  u128 r, int32_t *pick)
{
    for (int32_t k = threadIdx.x; k < cnt; k += TEAM) {
        const int32_t c = sv[k];
        u128 pre = 0;
        for (int32_t j = 0; j < cnt; ++j) pre += (sv[j] <= c) ? to128(sw[j]) : (u128)0;
        const u128 wk = to128(sw[k]);
        if (pre > r && pre - wk <= r) *pick = c;
    }
}

// The same for weights whose total is below 2^64 (the meeting draw's 40-bit
// weights): 64-bit prefixes, four entries per step.
template <int TEAM>
__device__ __forceinline__ void pick_by_id_prefix64(const int32_t *sv, const Sigma *sw, int32_t cnt,
                                                    uint64_t r, int32_t *pick)
{
    for (int32_t k = threadIdx.x; k < cnt; k += TEAM) {
        const int32_t c = sv[k];
        uint64_t pre = 0;
        int32_t j = 0;
        for (; j + 4 <= cnt; j += 4) {
            const int32_t v0 = sv[j], v1 = sv[j + 1], v2 = sv[j + 2], v3 = sv[j + 3];
            const uint64_t w0 = sw[j].lo, w1 = sw[j + 1].lo, w2 = sw[j + 2].lo, w3 = sw[j + 3].lo;
            pre += (v0 <= c ? w0 : 0u) + (v1 <= c ? w1 : 0u) + (v2 <= c ? w2 : 0u) + (v3 <= c ? w3 : 0u);
        }
        for (; j < cnt; ++j) pre += (sv[j] <= c) ? sw[j].lo : 0u;
        const uint64_t wk = sw[k].lo;
        if (pre > r && pre - wk <= r) *pick = c;
    }
}

// An open-addressing map in LDS from the vertices of a new level to their
// positions in it: `mask + 1` slots (a power of two), -1 = empty, linear
// probing; a slot holds a position p, whose vertex is ids[p] (the level's
// staged ids).  Filled to at most half, so every probe sequence ends.
__device__ __forceinline__ int32_t hash_slot(int32_t w, int32_t mask)
{
    return (int32_t)(((uint32_t)w * 0x9E3779B1u) >> 16) & mask;
}
__device__ __forceinline__ void pos_insert(int32_t *tab, int32_t mask, int32_t w, int32_t p)
{
    int32_t h = hash_slot(w, mask);
    while (atomicCAS(&tab[h], -1, p) != -1) h = (h + 1) & mask;
}
// w's position, or -1 if w is not in the map
__device__ __forceinline__ int32_t pos_find(const int32_t *tab, const int32_t *ids, int32_t mask, int32_t w)
{
    int32_t h = hash_slot(w, mask);
    for (;;) {
        const int32_t q = tab[h];
        if (q < 0) return -1;
        if (ids[q] == w) return q;
        h = (h + 1) & mask;
    }
}

// Zeroes the code word of every vertex in ball[0, len).  (Sigma needs no
// clearing: a sample reads it only for vertices it reached, and writes it
// first for each of them.)
template <int TEAM>
__device__ __forceinline__ void clear_ball(const int32_t *ball, int32_t len, uint32_t *code)
{
    constexpr int U = 4;
    for (int32_t k0 = threadIdx.x; k0 < len; k0 += U * TEAM) {
        int32_t w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) w[u] = (k0 + u * TEAM < len) ? ball[k0 + u * TEAM] : -1;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (w[u] >= 0) code[w[u] >> 3] = 0u;
    }
}

// Wave/workgroup-per-sample sampler.  Every lane of the team runs the same
// control flow; per-sample scalars live in registers (uniform) or LDS.
// MAPPED: some query of the launch is on a relabelled graph (its descriptor
// has the vertex maps); without it the maps are never read.  PULL: meeting
// probes take the pull form (scan the other side's frontier rows).
template <int TEAM, bool MAPPED, bool PULL>
__global__ __launch_bounds__(TEAM) __attribute__((amdgpu_waves_per_eu(4))) void sample_kernel(SampleArgs a)
{
    using T = Team<TEAM>;
#ifdef KADABRA_PHASE_TIMERS
    // The one-wavefront timer build gave a wrong result once (a backtracking
    // step found no predecessor) and its cause is not known: it is not built.
    static_assert(TEAM != 64, "phase timers are not available for 64-lane teams");
#endif
    constexpr int ARCS = (TEAM == 64) ? 4 : (TEAM == 256) ? 6 : 8;  // arcs in flight per lane in a level
                                                                   // expansion (measured per team size)
    constexpr int STAGE = Cap<TEAM>::STAGE;
    __shared__ SampleShared<TEAM> sm;
    const int lane = threadIdx.x;
    // Reduction scratch: a reduction does not wait for its reads of red to
    // finish, so a buffer is reused only after a barrier.  Each call site below
    // names its buffer so that this holds: redA where a barrier follows anyway,
    // redB for a reduction directly followed by another one.
    uint64_t *const redA = sm.red[0];
    uint64_t *const redB = sm.red[1];
    const size_t ns = (size_t)a.st.nstride;
    const size_t slot = blockIdx.x;
    uint32_t *const code = a.st.code + slot * (size_t)a.st.code_stride;
    Sigma *const sig0 = a.st.sigma + (2 * slot) * ns;
    Sigma *const sig1 = a.st.sigma + (2 * slot + 1) * ns;
    int32_t *const ball0 = a.st.ball + (2 * slot) * ns;
    int32_t *const ball1 = a.st.ball + (2 * slot + 1) * ns;
    int32_t *const meet = a.st.meet + slot * ns;
    uint64_t *const meetw = a.st.meetw + slot * ns;
    int32_t *const loff0 = a.st.loff + (2 * slot) * (size_t)a.st.lcap;
    int32_t *const loff1 = loff0 + a.st.lcap;

    // the flags of this launch's boundaries start clear (their sets were last
    // read at least one launch ago; a launch reads only the set before lo)
    if (blockIdx.x == 0)
        for (int32_t k = lane; k < a.nq; k += TEAM) {
            const QueryDesc &d = a.q[k];
            if (d.stat_set >= 0) continue;  // a first phase: no boundary
            for (int64_t e = d.lo / d.epoch_len + 1; e <= (d.hi - 1) / d.epoch_len + 1; ++e)
                d.ctl->viol[e % d.nsets] = 0;
        }

    // A speculative launch whose runs have all stopped at the previous
    // boundary draws nothing.  Those flags were written earlier in stream order
    // and do not change during the launch, so every workgroup decides alike and
    // leaves; workgroup 0 moves the claim counter by what the claims would have
    // taken (the samples, and one failing claim per workgroup).
    if (a.gated) {
        int open = 0;
        for (int32_t k = lane; k < a.nq; k += TEAM) {
            const QueryDesc &d = a.q[k];
            open |= d.ctl->viol[d.gate] != 0 ? 1 : 0;
        }
        if (!__syncthreads_or(open)) {
            if (blockIdx.x == 0 && lane == 0)
                atomicAdd(a.claim, (unsigned long long)a.total + (unsigned long long)gridDim.x);
            return;
        }
    }

#ifdef KADABRA_PHASE_TIMERS
    uint64_t ph_acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    Control *ph_ctl = nullptr;
#endif
    // work counters (lane 0) of the query being served, flushed when the
    // workgroup moves to another query and at exit
    Control *acc_ctl = nullptr;
    int32_t acc_par = 0;
    if (lane < ST_COUNT) sm.acc[lane] = 0;
    auto flush = [&]() {
        if (lane != 0 || !acc_ctl) return;
        int64_t *stp = acc_ctl->stats[acc_par];
        for (int k = 0; k < ST_COUNT; ++k) {
            if (sm.acc[k]) atomicAdd((unsigned long long *)&stp[k], sm.acc[k]);
            sm.acc[k] = 0;
        }
    };

    for (;;) {
        __syncthreads();
        if (lane == 0) {
            int64_t j;
            int32_t qi = 0;
            for (;;) {
                j = (int64_t)(atomicAdd(a.claim, 1ull) - a.claim_base);
                if (j >= a.total) break;
                int32_t lo = 0, hi = a.nq;  // the query whose range holds claim j
                while (hi - lo > 1) {
                    const int32_t mid = (lo + hi) >> 1;
                    if (a.q[mid].claim_begin <= j) lo = mid; else hi = mid;
                }
                qi = lo;
                // Launched before the host has read the previous boundary's
                // check: stream order has already run that check, so its flag
                // decides.  A stopped run's range needs no claims: the counter
                // moves past it at once (never past the launch's total, so
                // every workgroup still ends on exactly one failing claim).
                const QueryDesc &d = a.q[qi];
                if (d.gate < 0 || d.ctl->viol[d.gate] != 0) break;
                atomicMax(a.claim, (unsigned long long)(a.claim_base + (uint64_t)(d.claim_begin + (d.hi - d.lo))));
            }
            sm.claim = j;
            sm.query = qi;
        }
        T::sync();
        const int64_t jc = uniform_i64(sm.claim);
        if (jc >= a.total) break;
        // the query's fields, once, into scalar registers
        const QueryDesc *const qd = a.q + uniform_i32(sm.query);
        Control *const qctl = qd->ctl;
        const int64_t i = qd->lo + (jc - qd->claim_begin);
        const int32_t qpar = (int32_t)((i / qd->epoch_len + 1) % qd->nsets);  // the epoch's set
        const int32_t qstat = qd->stat_set >= 0 ? qd->stat_set : qpar;       // its work counters
        // graph arrays live in device global memory: say so, so that their
        // loads are global (not flat) instructions
        const gint32_t *const row_ptr = as_global(qd->row_ptr);
        const gint32_t *const col = as_global(qd->col);
        const gint32_t *const comp = as_global(qd->comp);
        const int32_t nv = qd->n;
        const uint64_t seed = qd->seed;
        const int64_t probe_min = qd->probe_min, num_arcs = qd->num_arcs, probe_h8 = qd->probe_h8;
        const bool probe_quit = qd->probe_quit != 0;
        int32_t *const frame =
            qd->frames + ((size_t)qpar * qd->nframes + (size_t)(blockIdx.x % qd->nframes)) * (size_t)nv;
        if (qctl != acc_ctl || qstat != acc_par) {
            flush();
            acc_ctl = qctl;
            acc_par = qstat;
        }
#ifdef KADABRA_PHASE_TIMERS
        ph_ctl = qctl;
#endif
        PHASE_BEGIN();

        // -- pair: ordered, s != t, uniform (64-bit multiply-high mapping) --
        uint64_t u_t;
        const uint64_t u_s = philox_u64(seed, (uint64_t)i, 0u, &u_t);
        int32_t s = (int32_t)__umul64hi(u_s, (uint64_t)nv);
        int32_t t = (int32_t)__umul64hi(u_t, (uint64_t)(nv - 1));
        t += (t >= s) ? 1 : 0;
        // a relabelled graph: ids below are internal; ties are still broken
        // by original id (meeting draw, level-list candidates).  The maps are
        // read from the descriptor where used, not held through the search.
        if (MAPPED) {
            const int32_t *const pm = qd->perm;
            const int32_t ms = pm ? pm[s] : s, mt = pm ? pm[t] : t;
            s = uniform_i32(ms);
            t = uniform_i32(mt);
        }
        // the component test and both rows' bounds, loaded together
        const int32_t cs = comp[s], ct = comp[t];
        const int32_t rs_s = row_ptr[s], re_s = row_ptr[s + 1];
        const int32_t rs_t = row_ptr[t], re_t = row_ptr[t + 1];
        if (cs != ct) {  // Appendix C.1: no search across components
            if (lane == 0) sm.acc[ST_DISCONN] += 1;
            continue;
        }
        PHASE_MARK(0);

        // -- balanced bidirectional BFS with path counts ----------------------
        if (lane == 0) {
            // every code word is zero between samples (each sample clears the
            // words it touched), so s and t are entered by stores, with no read
            const uint32_t cs0 = level_code(0) << code_shift(s, 0);
            const uint32_t ct1 = level_code(0) << code_shift(t, 1);
            if ((s >> 3) == (t >> 3)) {
                code[s >> 3] = cs0 | ct1;
            } else {
                code[s >> 3] = cs0;
                code[t >> 3] = ct1;
            }
            ball0[0] = s;
            ball1[0] = t;
            loff0[0] = 0;
            loff0[1] = 1;
            loff1[0] = 0;
            loff1[1] = 1;
            sm.nnext[0] = sm.nnext[1] = 0;
            sm.nmeet[0] = sm.nmeet[1] = 0;
        }
        // per-side BFS state (uniform across the team; side X selected by value)
        int32_t lvl0 = 0, lvl1 = 0;
        int32_t flo0 = 0, flo1 = 0, fhi0 = 1, fhi1 = 1;  // frontier = ball[flo, fhi)
        int64_t dsum0 = re_s - rs_s, dsum1 = re_t - rs_t;
        bool fc0 = true, fc1 = true;  // the side's frontier is in the LDS cache
        if (lane == 0) {
            sm.frs[0][0] = rs_s;
            sm.fdg[0][0] = (int32_t)dsum0;
            sm.fsg[0][0] = Sigma{1u, 0u};
            sm.frs[1][0] = rs_t;
            sm.fdg[1][0] = (int32_t)dsum1;
            sm.fsg[1][0] = Sigma{1u, 0u};
        }
        u128 fmass0 = 1, fmass1 = 1;  // sum of the frontier's sigma
        int X = 0, nN = 0, nM = 0;
        bool meet_staged = false;  // the meeting set is sm.sv[0, nM) (a probe level that fit)
        int fail_site = 0;
        bool ok = true, retry = false;
        int lp = 0;  // which append counters this BFS iteration uses (the other ones are zero)
        T::sync();
        for (;;) {
            X = (dsum0 <= dsum1) ? 0 : 1;  // cheaper side; s on ties
            int32_t *const ballx = X ? ball1 : ball0;
            Sigma *const sigx = X ? sig1 : sig0;
            const int32_t lvlx = X ? lvl1 : lvl0;
            const int32_t flox = X ? flo1 : flo0;
            const int32_t fhix = X ? fhi1 : fhi0;
            const int64_t dsx = X ? dsum1 : dsum0;
            if (lvlx + 3 > a.st.lcap) {  // more levels than the diameter bound allows
                ok = false;
                fail_site = 1;
                nN = 0;
                break;
            }
            // Meeting probe: on a large expansion, first claim only the new
            // vertices the other side has already reached.  If there are any,
            // they are the whole meeting set and the rest of the level is never
            // needed (sigma of a meeting vertex is the same sum either way);
            // otherwise the level is expanded in full.  The probe cannot skip a
            // rescaling: it runs only when the frontier's mass is below 2^104.
            // Auto rule (probe_min < 0): probe when the arcs leaving X's
            // frontier are expected to hit Y's frontier at least h =
            // probe_h8 / 8 times, D_X D_Y >= h x (number of arcs), an arc
            // landing on a vertex with probability proportional to its
            // degree.  The host sets a small h on low-diameter graphs and a
            // larger one on high-diameter graphs, whose arcs stay local: there
            // the estimate counts hits long before the balls touch.
            const int64_t dsy = X ? dsum0 : dsum1;
            const bool want_probe = (probe_min >= 0) ? (dsx >= probe_min)
                                                     : (dsx * dsy >= probe_h8 * num_arcs / 8);
            const bool probe = !retry && want_probe && bitw128(X ? fmass1 : fmass0) <= SIGMA_BITS;
            if (lane == 0 && !retry) {
                sm.acc[ST_VEXP] += (uint64_t)(fhix - flox);
                sm.acc[ST_ESCAN] += (uint64_t)dsx;
            }
            const uint32_t code_new = level_code(lvlx + 1);  // code of the new level
            const int32_t base_new = fhix;
            int32_t *const cnt_new = &sm.nnext[lp];
            int32_t *const cnt_meet = &sm.nmeet[lp];
            const bool fcx = X ? fc1 : fc0;  // then the frontier is one chunk
            // Full levels whose frontier mass is below 2^63 (no count of the new
            // level leaves 64 bits) sum sigma in LDS for their first STAGE new
            // vertices: the staging area's counts hold a map from vertex to
            // position (2 STAGE slots) and a 64-bit count per position.  The
            // claim's winner at position p < STAGE enters w -> p and stores its
            // own arc's count at p; after the round's barrier the other arcs
            // into w add there; each such count is stored to global memory once,
            // in the bookkeeping.  The new vertices past STAGE are summed in
            // global memory (the winner stores, the others add).  Not on probe
            // levels.
            // A vertex one arc from its root has exactly one shortest path from
            // it, and the root itself one: sigma of levels 0 and 1 is 1, never
            // stored nor read (on low-diameter graphs most new vertices lie on
            // level 1 of one side).
            const bool implicit_new = lvlx == 0;    // the new level is level 1
            const bool implicit_front = lvlx <= 1;  // the frontier's sigma is 1
            const bool low_mass = bitw128(X ? fmass1 : fmass0) <= 63;
            const bool lds_try = !probe && !implicit_new && low_mass;
            int32_t *const ptab = reinterpret_cast<int32_t *>(&sm.sw[0]);               // [2 STAGE]
            uint64_t *const pval = reinterpret_cast<uint64_t *>(&sm.sw[0]) + STAGE;     // [STAGE]
            constexpr int32_t PMASK = 2 * STAGE - 1;
            if (PULL && probe) {
                // Pull form of the meeting probe: the rows of Y's frontier are
                // scanned for neighbours on X's frontier.  Such a neighbour p
                // makes the row's vertex y a meeting vertex, and sigma_X(y) is
                // the sum of sigma_X(p) over them: the same set and the same sums
                // as the push form, because no vertex is reached by both sides
                // before the level on which they meet and every meeting vertex
                // lies on Y's frontier.  (A neighbour with X's frontier code mod 3
                // lies on X's frontier itself: one three levels closer to X's root
                // would have made y reached by X already.)
                constexpr int PA = ARCS / 2;  // arcs in flight per lane
                const int Y = X ^ 1;
                const int32_t *const bally = Y ? ball1 : ball0;
                const int32_t floy = Y ? flo1 : flo0, fhiy = Y ? fhi1 : fhi0;
                const bool fcy = Y ? fc1 : fc0;
                const uint32_t code_front = level_code(lvlx);
                for (int32_t c0 = floy; c0 < fhiy; c0 += TEAM) {
                    const int32_t idx = c0 + lane;
                    int32_t dg = 0;
                    if (idx < fhiy) {
                        const int32_t y = bally[idx];
                        if (fcy) {
                            dg = sm.fdg[Y][lane];
                            sm.crs[lane] = sm.frs[Y][lane];
                        } else {
                            const int32_t rs = row_ptr[y];
                            dg = row_ptr[y + 1] - rs;
                            sm.crs[lane] = rs;
                        }
                        sm.cm[lane].lo = (uint64_t)(uint32_t)y;  // the row's vertex
                    }
                    int32_t tot;
                    const int32_t ex = T::excl_scan_i32(dg, &tot, redA);
                    sm.cpfx[lane] = ex;
                    const int32_t cnt = min(TEAM, fhiy - c0);
                    __syncthreads();
                    int32_t own = 0;
                    auto owner_of = [&](int32_t e) {
                        int32_t step = 1;
                        while (own + step < cnt && sm.cpfx[own + step] <= e) {
                            own += step;
                            step <<= 1;
                        }
                        int32_t hi = min(own + step, cnt);
                        while (hi - own > 1) {
                            const int32_t mid = (own + hi) >> 1;
                            if (sm.cpfx[mid] <= e) own = mid; else hi = mid;
                        }
                        return own;
                    };
                    // rounds of PA * TEAM arcs, the same number in every lane: the
                    // winner of y's claim zeroes sigma_X(y), and the round's adds
                    // follow a barrier
                    const int32_t rounds = (tot + PA * TEAM - 1) / (PA * TEAM);
                    for (int32_t r = 0; r < rounds; ++r) {
                        const int32_t e = r * PA * TEAM + lane;
                        int32_t ai[PA], yv[PA], pv[PA];
                        uint32_t wd[PA], old[PA];
                        bool hit[PA], won[PA];
                        Sigma sp[PA];
#pragma unroll
                        for (int k = 0; k < PA; ++k) {
                            const int32_t ek = e + k * TEAM;
                            int32_t o = own;
                            if (ek < tot) {
                                o = owner_of(ek);
                                ai[k] = sm.crs[o] + (ek - sm.cpfx[o]);
                            } else {
                                ai[k] = 0;  // arc 0 of the graph: the load stays in bounds
                            }
                            yv[k] = (int32_t)(uint32_t)sm.cm[o].lo;
                        }
#pragma unroll
                        for (int k = 0; k < PA; ++k) pv[k] = col[ai[k]];
#pragma unroll
                        for (int k = 0; k < PA; ++k) wd[k] = code[pv[k] >> 3];
#pragma unroll
                        for (int k = 0; k < PA; ++k) {
                            hit[k] = e + k * TEAM < tot && ((wd[k] >> code_shift(pv[k], X)) & 3u) == code_front;
                            sp[k] = !hit[k] ? Sigma{0u, 0u} : (implicit_front ? Sigma{1u, 0u} : sigx[pv[k]]);
                        }
#pragma unroll
                        for (int k = 0; k < PA; ++k)
                            old[k] = hit[k] ? wg_or_u32(&code[yv[k] >> 3], code_new << code_shift(yv[k], X)) : 0u;
#pragma unroll
                        for (int k = 0; k < PA; ++k) {
                            const bool claimed = hit[k] && ((old[k] >> code_shift(yv[k], X)) & 3u) == 0u;
                            won[k] = claimed;
                            const int pp = wave_append(claimed, cnt_new);
                            if (claimed) {
                                ballx[base_new + pp] = yv[k];
                                if (pp < STAGE) sm.sv[pp] = yv[k];
                                if (!implicit_new) sigx[yv[k]] = sp[k];  // the claim's own hit
                            }
                            const int q = wave_append(claimed, cnt_meet);
                            if (claimed) meet[q] = yv[k];
                        }
                        if (implicit_new) continue;  // sigma_X(y) is 1
                        __syncthreads();
                        // sigma_X(y) += sigma_X(p)
#pragma unroll
                        for (int k = 0; k < PA; ++k) {
                            if (!hit[k] || won[k]) continue;
                            if (low_mass) {
                                (void)wg_add_u64(&sigx[yv[k]].lo, sp[k].lo);
                            } else {
                                const uint64_t o = wg_add_u64(&sigx[yv[k]].lo, sp[k].lo);
                                const uint64_t hi = sp[k].hi + ((o + sp[k].lo) < o ? 1u : 0u);
                                if (hi) wg_add_u64(&sigx[yv[k]].hi, hi);
                            }
                        }
                    }
                    __syncthreads();
                }
            } else {
                bool gave_up = false;  // a probe given up after its first round
                // (high-diameter graphs are the relabelled ones: a launch without
                // one has no probe to give up, and the test is compiled out)
                const bool quit_first = MAPPED && probe_quit && probe && dsx > (int64_t)ARCS * TEAM;
                for (int32_t c0 = flox; c0 < fhix; c0 += TEAM) {
                    const int32_t idx = c0 + lane;
                    int32_t dg = 0;
                    if (idx < fhix) {
                        if (fcx) {
                            dg = sm.fdg[X][lane];
                            sm.crs[lane] = sm.frs[X][lane];
                            sm.cm[lane] = sm.fsg[X][lane];
                        } else {
                            const int32_t u = ballx[idx];
                            const int32_t rs = row_ptr[u];
                            dg = row_ptr[u + 1] - rs;
                            sm.crs[lane] = rs;
                            sm.cm[lane] = implicit_front ? Sigma{1u, 0u} : sigx[u];
                        }
                    }
                    if (lds_try && c0 == flox) {
                        // an empty map; a position's count is written by its winner
                        // before any add
                        for (int32_t h = lane; h < 2 * STAGE; h += TEAM) ptab[h] = -1;
                    }
                    int32_t tot;
                    const int32_t ex = T::excl_scan_i32(dg, &tot, redA);
                    sm.cpfx[lane] = ex;
                    const int32_t cnt = min(TEAM, fhix - c0);
                    __syncthreads();
                    // Each lane takes arcs lane, lane + TEAM, ... ARCS at a time: all
                    // their owners, column entries and code words are fetched before
                    // any is processed.  A lane's owners only move forward, so each
                    // is found by galloping from the previous one.
                    int32_t own = 0;
                    auto owner_of = [&](int32_t e) {
                        int32_t step = 1;
                        while (own + step < cnt && sm.cpfx[own + step] <= e) {
                            own += step;
                            step <<= 1;
                        }
                        int32_t hi = min(own + step, cnt);
                        while (hi - own > 1) {
                            const int32_t mid = (own + hi) >> 1;
                            if (sm.cpfx[mid] <= e) own = mid; else hi = mid;
                        }
                        return own;
                    };
                    // One round: arcs e, e + TEAM, ... (up to ARCS) of this lane --
                    // owners, column entries, code words, claims and appends.  wv,
                    // ow and add receive the arcs and which of them enter the new level.
                    auto claim_round = [&](int32_t e, int32_t (&wv)[ARCS], int32_t (&ow)[ARCS], bool (&add)[ARCS]) {
                        // owners and arc positions (LDS only), each arc's column
                        // entry requested as soon as its position is known, so that
                        // the loads overlap the next owners' searches; an arc past
                        // the end reads arc 0 of the graph, so that every load is
                        // unconditional (the round loop is the same for every lane,
                        // so in the last round even a lane's first arc may be past it)
                        uint32_t wd[ARCS];
    #pragma unroll
                        for (int k = 0; k < ARCS; ++k) {
                            const int32_t ek = e + k * TEAM;
                            int32_t ai = 0;
                            if (ek < tot) {
                                ow[k] = owner_of(ek);
                                ai = sm.crs[ow[k]] + (ek - sm.cpfx[ow[k]]);
                            } else {
                                ow[k] = own;
                            }
                            wv[k] = col[ai];
                        }
    #pragma unroll
                        for (int k = 0; k < ARCS; ++k) wd[k] = code[wv[k] >> 3];
                        // claims: decided from the words read, and all issued before
                        // any result is awaited.  Every claim on this level writes the
                        // same code, so an OR into a field another lane (or an earlier
                        // arc of this lane) just set changes nothing.
                        uint32_t dxc[ARCS], dyc[ARCS], old[ARCS];
                        bool cand[ARCS];
    #pragma unroll
                        for (int k = 0; k < ARCS; ++k) {
                            const bool valid = e + k * TEAM < tot;
                            dxc[k] = (wd[k] >> code_shift(wv[k], X)) & 3u;
                            dyc[k] = (wd[k] >> code_shift(wv[k], X ^ 1)) & 3u;
                            cand[k] = valid && dxc[k] == 0u && (!probe || dyc[k] != 0u);
                        }
    #pragma unroll
                        for (int k = 0; k < ARCS; ++k)
                            old[k] = cand[k] ? wg_or_u32(&code[wv[k] >> 3], code_new << code_shift(wv[k], X)) : 0u;
    #pragma unroll
                        for (int k = 0; k < ARCS; ++k) {
                            const int32_t w = wv[k];
                            bool claimed = false;
                            if (cand[k]) {
                                const uint32_t o = (old[k] >> code_shift(w, X)) & 3u;
                                claimed = (o == 0u);
                                dxc[k] = claimed ? code_new : o;
                            }
                            const int p = wave_append(claimed, cnt_new);
                            if (claimed) {
                                ballx[base_new + p] = w;
                                if (p < STAGE) sm.sv[p] = w;
                                // the claim's own arc is a store (in LDS or in global
                                // memory), the other arcs into w add after a barrier
                                if (lds_try && p < STAGE) {
                                    pval[p] = sm.cm[ow[k]].lo;
                                    pos_insert(ptab, PMASK, w, p);
                                } else if (!implicit_new) {
                                    sigx[w] = sm.cm[ow[k]];
                                }
                            }
                            const bool is_meet = claimed && dyc[k] != 0u;
                            const int q = wave_append(is_meet, cnt_meet);
                            if (is_meet) meet[q] = w;
                            add[k] = e + k * TEAM < tot && dxc[k] == code_new && !claimed;
                        }
                    };
                    // sigma(w) += sigma(owner) for every arc into the new level, in
                    // global memory: all low-word adds first, then the carries.  When
                    // the frontier's mass is below 2^63 no count of the new level can
                    // leave the low word, so the adds need no result and no wait.
                    auto global_adds = [&](const int32_t (&wv)[ARCS], const int32_t (&ow)[ARCS],
                                           const bool (&add)[ARCS]) {
                        if (low_mass) {
    #pragma unroll
                            for (int k = 0; k < ARCS; ++k)
                                if (add[k]) (void)wg_add_u64(&sigx[wv[k]].lo, sm.cm[ow[k]].lo);
                            return;
                        }
                        uint64_t olo[ARCS];
    #pragma unroll
                        for (int k = 0; k < ARCS; ++k) olo[k] = 0u;
    #pragma unroll
                        for (int k = 0; k < ARCS; ++k)
                            if (add[k]) olo[k] = wg_add_u64(&sigx[wv[k]].lo, sm.cm[ow[k]].lo);
    #pragma unroll
                        for (int k = 0; k < ARCS; ++k) {
                            if (!add[k]) continue;
                            const Sigma m = sm.cm[ow[k]];
                            const uint64_t hi = m.hi + ((olo[k] + m.lo) < olo[k] ? 1u : 0u);
                            if (hi) wg_add_u64(&sigx[wv[k]].hi, hi);
                        }
                    };
                    int32_t wv[ARCS], ow[ARCS];
                    bool add[ARCS];
    #pragma unroll
                    for (int k = 0; k < ARCS; ++k) add[k] = false;
                    // sigma(w) += sigma(owner) for the arcs into w that did not claim
                    // it: in LDS if w has a slot there, else in global memory
                    auto lds_adds = [&](const int32_t (&wv)[ARCS], const int32_t (&ow)[ARCS], bool (&add)[ARCS]) {
    #pragma unroll
                        for (int k = 0; k < ARCS; ++k) {
                            if (!add[k]) continue;
                            const int32_t q = pos_find(ptab, sm.sv, PMASK, wv[k]);
                            if (q < 0) continue;  // past STAGE: stays for global_adds
                            add[k] = false;
                            // no carry possible (mass below 2^63): an add without a result
                            (void)atomicAdd((unsigned long long *)&pval[q], (unsigned long long)sm.cm[ow[k]].lo);
                        }
                    };
                    // rounds of ARCS * TEAM arcs, the same number in every lane.  A
                    // vertex's sigma is written only by the sample that reaches it
                    // (nothing clears it afterwards): the winner of its claim stores
                    // its own arc's count, and the other arcs into the vertex add
                    // theirs after a barrier that follows the round's claims (most
                    // new vertices have one predecessor: a store, no atomic).
                    const int32_t rounds = (tot + ARCS * TEAM - 1) / (ARCS * TEAM);
                    for (int32_t r = 0; r < rounds; ++r) {
                        claim_round(r * ARCS * TEAM + lane, wv, ow, add);
                        if (!implicit_new) {  // else sigma 1
                            __syncthreads();
                            if (lds_try) lds_adds(wv, ow, add);
                            global_adds(wv, ow, add);
                        }
                        // On high-diameter graphs (probe_quit) a probe whose first
                        // round meets no vertex of the other side, with more of
                        // the level to scan, is given up: the level is then
                        // expanded in full (as after a probe that met nothing).
                        // There probes mostly fail; on low-diameter graphs a
                        // probe's meeting vertices often come in later rounds.
                        // The count is read after the round's barrier, so every
                        // wave decides alike.
                        if (quit_first && r == 0 && c0 == flox) {
                            if (implicit_new) __syncthreads();  // else taken above
                            if (uniform_i32(*cnt_meet) == 0) {
                                gave_up = true;
                                break;
                            }
                        }
                    }
                    __syncthreads();
                    if (gave_up) break;
                }
            }
            PHASE_MARK(1);
            nN = uniform_i32(*cnt_new);
            nM = uniform_i32(*cnt_meet);
            if (lane == 0) sm.acc[ST_VMAT] += (uint64_t)nN;
            // the next iteration counts in the other pair, last read before this
            // iteration's barriers
            if (lane == 0) {
                sm.nnext[lp ^ 1] = 0;
                sm.nmeet[lp ^ 1] = 0;
            }
            lp ^= 1;
            // LDS-summed sigma (positions below STAGE): each such new vertex's
            // count to its global slot; the bookkeeping below reads them by
            // position from LDS
            const bool lds_sig = lds_try;
            const int32_t nH = min(nN, STAGE);
            if (lds_sig) {
                for (int32_t k = lane; k < nH; k += TEAM) sigx[sm.sv[k]] = Sigma{pval[k], 0u};
                // counts read: a meeting draw may restage the area (the
                // bookkeeping below reads the counts again, the staging not)
                __syncthreads();
            }
            if (probe && nM == 0) {  // no meeting on this level: expand it in full
                retry = true;
                continue;
            }
            retry = false;
            if (nN == 0) {  // cannot happen inside one component
                ok = false;
                fail_site = 3;
                break;
            }
            // rescale the new level if its largest count may reach 2^SIGMA_BITS
            // the frontier's mass bounds every new count
            if (bitw128(X ? fmass1 : fmass0) > SIGMA_BITS) {
                u128 hm = 0;
                for (int32_t k = lane; k < nN; k += TEAM) {
                    const u128 v = to128(sigx[ballx[base_new + k]]);
                    hm = v > hm ? v : hm;
                }
                hm = T::max_u128(hm, redA);
                const int sh = bitw128(hm) - SIGMA_BITS;
                if (sh > 0) {
                    const u128 add = ((u128)1 << sh) - 1;
                    for (int32_t k = lane; k < nN; k += TEAM) {
                        const int32_t w = ballx[base_new + k];
                        const u128 v = (to128(sigx[w]) + add) >> sh;
                        sigx[w] = Sigma{(uint64_t)v, (uint64_t)(v >> 64)};
                    }
                }
                T::sync();
            }
            PHASE_MARK(2);
            if (nM > 0) {
                // on a probe level only meeting vertices were claimed, so the
                // new level (staged in LDS when it fits) is the meeting set
                meet_staged = probe && nN == nM && nN <= STAGE;
                break;
            }
            // advance side X: its frontier becomes the new level (ids staged in
            // LDS by the claims when they fit; a one-chunk level is cached)
            uint64_t ds = 0;
            u128 ms = 0;
            const bool staged_new = nN <= STAGE, cache_new = nN <= TEAM;
            // two vertices per lane and pass: both loads issued before either is used
            for (int32_t k = lane; k < nN; k += 2 * TEAM) {
                const int32_t k2 = k + TEAM;
                const bool two = k2 < nN;
                const int32_t w = staged_new ? sm.sv[k] : ballx[base_new + k];
                const int32_t w2 = two ? (staged_new ? sm.sv[k2] : ballx[base_new + k2]) : w;
                const int32_t rs = row_ptr[w], re = row_ptr[w + 1];
                const int32_t rs2 = row_ptr[w2], re2 = row_ptr[w2 + 1];
                const Sigma m = implicit_new ? Sigma{1u, 0u} : ((lds_sig && k < nH) ? Sigma{pval[k], 0u} : sigx[w]);
                const Sigma m2 = implicit_new ? Sigma{1u, 0u} : ((lds_sig && k2 < nH) ? Sigma{pval[k2], 0u} : sigx[w2]);
                const int32_t dg = re - rs;
                ds += (uint64_t)dg;
                ms += to128(m);
                if (two) {
                    ds += (uint64_t)(re2 - rs2);
                    ms += to128(m2);
                }
                if (cache_new) {  // then nN <= TEAM: k is the only vertex of the lane
                    sm.frs[X][k] = rs;
                    sm.fdg[X][k] = dg;
                    sm.fsg[X][k] = m;
                }
            }
            T::sum_u64_u128(&ds, &ms, redB);
            if (X) fc1 = cache_new; else fc0 = cache_new;
            if (lane == 0) (X ? loff1 : loff0)[lvlx + 2] = fhix + nN;
            if (X) {
                flo1 = fhi1;
                fhi1 += nN;
                lvl1 += 1;
                dsum1 = (int64_t)ds;
                fmass1 = ms;
            } else {
                flo0 = fhi0;
                fhi0 += nN;
                lvl0 += 1;
                dsum0 = (int64_t)ds;
                fmass0 = ms;
            }
            PHASE_MARK(2);
        }
        // the last level built belongs to side X's ball (it is cleared below)
        const int32_t bend0 = fhi0 + ((X == 0) ? nN : 0);
        const int32_t bend1 = fhi1 + ((X == 1) ? nN : 0);

        if (ok) {
            // -- meeting vertex: P(v) = sigma_s(v) sigma_t(v), ascending id ----
            // the meeting vertices' distances: one more than side X's frontier
            // level, side Y's level (sigma 1 on levels 0 and 1)
            const int32_t dv0 = (X == 0) ? lvl0 + 1 : lvl0;
            const int32_t dv1 = (X == 1) ? lvl1 + 1 : lvl1;
            auto sig_of = [&](const Sigma *sg, int32_t dist, int32_t w) -> u128 {
                return dist <= 1 ? (u128)1 : to128(sg[w]);
            };
            int32_t v;
            if (nM == 1) {
                v = meet_staged ? sm.sv[0] : meet[0];
            } else if (nM <= TEAM) {
                // one meeting vertex per lane: its product stays in registers
                // between the maximum and the weight
                const bool has = lane < nM;
                int32_t w = 0, wo = 0;  // internal and original id
                U256 p{0, 0};
                if (has) {
                    w = meet_staged ? sm.sv[lane] : meet[lane];
                    wo = (MAPPED && qd->iperm) ? qd->iperm[w] : w;
                    p = mul_128x128(sig_of(sig0, dv0, w), sig_of(sig1, dv1, w));
                }
                const U256 pm = T::max_u256(p, redA);
                const int shp = max(0, bitw256(pm) - WEIGHT_BITS);
                const uint64_t wt = has ? ceil_shr256(p, shp) : 0u;
                if (has) {
                    sm.sv[lane] = wo;  // ranked by original id
                    sm.sw[lane] = Sigma{wt, 0u};
                }
                const uint64_t tot = T::sum_u64(wt, redB);
                const uint64_t r = __umul64hi(philox_u64(seed, (uint64_t)i, 1u), tot);
                // rank by scanning the staged set: the element whose
                // ascending-id inclusive prefix first exceeds r
                if (lane == 0) sm.pick = -1;
                __syncthreads();  // also: the staged weights are visible
                pick_by_id_prefix64<TEAM>(sm.sv, sm.sw, nM, r, &sm.pick);
                __syncthreads();
                v = uniform_i32(sm.pick);
                if (MAPPED && qd->perm) v = qd->perm[v];
                // every wave holds v before backtracking resets sm.pick
                __syncthreads();
            } else {
                const bool staged = nM <= STAGE;
                U256 pm{0, 0};
                for (int32_t k = lane; k < nM; k += TEAM) {
                    const int32_t w = meet[k];
                    const U256 p = mul_128x128(sig_of(sig0, dv0, w), sig_of(sig1, dv1, w));
                    if (p.hi > pm.hi || (p.hi == pm.hi && p.lo > pm.lo)) pm = p;
                }
                pm = T::max_u256(pm, redA);
                const int shp = max(0, bitw256(pm) - WEIGHT_BITS);
                uint64_t tot = 0;
                int32_t vmin = nv, vmax = -1;
                for (int32_t k = lane; k < nM; k += TEAM) {
                    const int32_t w = meet[k];
                    const int32_t wo = (MAPPED && qd->iperm) ? qd->iperm[w] : w;  // ranked by original id
                    const uint64_t wt =
                        ceil_shr256(mul_128x128(sig_of(sig0, dv0, w), sig_of(sig1, dv1, w)), shp);
                    if (staged) {
                        sm.sv[k] = wo;
                        sm.sw[k] = Sigma{wt, 0u};
                    } else {
                        meet[k] = wo;
                        meetw[k] = wt;
                    }
                    tot += wt;
                    vmin = min(vmin, wo);
                    vmax = max(vmax, wo);
                }
                tot = T::sum_u64(tot, redB);
                // team min / max of the ids (as maxima of n - id and id + 1)
                uint64_t mn = (uint64_t)(uint32_t)(nv - vmin), mx = (uint64_t)(uint32_t)(vmax + 1);
                mn = last_lane(wave_scan(mn, OpMax{}));
                mx = last_lane(wave_scan(mx, OpMax{}));
                if (T::WAVES > 1) {
                    uint64_t *const rr = redA;  // then a sync
                    const int wv = lane >> 6;
                    if ((lane & 63) == 0) {
                        rr[2 * wv] = mn;
                        rr[2 * wv + 1] = mx;
                    }
                    __syncthreads();
                    for (int k = 0; k < T::WAVES; ++k) {
                        mn = max(mn, rr[2 * k]);
                        mx = max(mx, rr[2 * k + 1]);
                    }
                }
                T::sync();  // staged weights visible to the whole team
                const uint64_t r = __umul64hi(philox_u64(seed, (uint64_t)i, 1u), tot);
                // smallest id v whose inclusive prefix (ascending ids) exceeds r
                int32_t lo = nv - (int32_t)mn, hi = (int32_t)mx - 1;
                int32_t it = 0;  // consecutive sums alternate their scratch
                while (lo < hi) {
                    const int32_t mid = lo + ((hi - lo) >> 1);
                    uint64_t part = 0;
                    if (staged) {
                        for (int32_t k = lane; k < nM; k += TEAM)
                            part += (sm.sv[k] <= mid) ? sm.sw[k].lo : 0u;
                    } else {
                        for (int32_t k = lane; k < nM; k += TEAM)
                            part += (meet[k] <= mid) ? meetw[k] : 0u;
                    }
                    part = T::sum_u64(part, (it++ & 1) ? redB : redA);
                    if (part > r) hi = mid; else lo = mid + 1;
                }
                v = (MAPPED && qd->perm) ? qd->perm[lo] : lo;
            }
            PHASE_MARK(3);
            if (lane == 0 && dv0 > 0 && dv1 > 0) {
                atomicAdd(&frame[v], 1);
                sm.acc[ST_INTERIOR] += 1;
            }
            // -- backtrack towards s (side 0) and t (side 1) -------------------
            for (int side = 0; side < 2 && ok; ++side) {
                const int32_t *const balls = side ? ball1 : ball0;
                const int32_t *const loffs = side ? loff1 : loff0;
                const Sigma *const sg = side ? sig1 : sig0;
                int32_t x = v;
                for (int32_t dxv = side ? dv1 : dv0; dxv > 1; --dxv) {  // x on level dxv
                    const uint32_t want = level_code(dxv - 1);
                    const bool one = dxv - 1 <= 1;  // the candidates' sigma is 1
                    const int32_t rs = row_ptr[x], deg = row_ptr[x + 1] - rs;
                    // predecessors = x's neighbours on level dxv - 1 of this side
                    const int32_t llo = loffs[dxv - 1], lhi = loffs[dxv];
                    const uint32_t j = 2u * (uint32_t)dxv + (uint32_t)side;
                    const uint64_t U = philox_u64(seed, (uint64_t)i, j);
                    if (lane == 0) {
                        sm.pick = -1;
                        sm.ncand = 0;
                    }
                    __syncthreads();
                    bool done = false, probe_pick = false;
                    if ((int64_t)(lhi - llo) * 24 < (int64_t)deg) {
                        // short level, long row: each wavefront takes level
                        // vertices p in turn and tests p for adjacency to x by a
                        // 64-way search in the shorter of the two sorted rows (the
                        // graph is symmetric); stage the candidates with their counts
                        // (on a relabelled graph the rows are searched in original
                        // ids, and candidates are ranked by them)
                        const int wid = uniform_i32(lane >> 6), lw = lane & 63;
                        gint32_t *const colk = (MAPPED && qd->colo) ? as_global(qd->colo) : col;
                        const int32_t *const iperm = MAPPED ? qd->iperm : nullptr;
                        const int32_t xo = iperm ? iperm[x] : x;
                        for (int32_t k = llo + wid; k < lhi; k += T::WAVES) {
                            const int32_t p = uniform_i32(balls[k]);
                            const int32_t po = iperm ? iperm[p] : p;
                            const int32_t prs = row_ptr[p], pdeg = row_ptr[p + 1] - prs;
                            const bool hit = (pdeg < deg) ? wave_row_contains(colk + prs, pdeg, xo, lw)
                                                          : wave_row_contains(colk + rs, deg, po, lw);
                            if (hit && lw == 0) {
                                const int at = atomicAdd(&sm.ncand, 1);
                                if (at < STAGE) {
                                    sm.sv[at] = po;
                                    sm.sw[at] = one ? Sigma{1u, 0u} : sg[p];
                                }
                            }
                        }
                        __syncthreads();
                        const int32_t nc = sm.ncand;
                        if (nc <= STAGE) {
                            u128 part = 0;
                            for (int32_t k = lane; k < nc; k += TEAM) part += to128(sm.sw[k]);
                            const u128 tot = T::sum_u128(part, redA);
                            const u128 r = mulhi_64x128(U, tot);
                            pick_by_id_prefix<TEAM>(sm.sv, sm.sw, nc, r, &sm.pick);
                            done = probe_pick = true;
                        }
                    }
                    if (!done && deg <= TEAM) {
                        // a row of at most TEAM arcs: lane k holds arc k; the code
                        // word and sigma of its neighbour are loaded together, and
                        // the lane whose prefix interval holds r is the pick
                        const bool mine = lane < deg;
                        const int32_t p = mine ? col[rs + lane] : 0;
                        const uint32_t cw = code[p >> 3];
                        const Sigma sp = one ? Sigma{1u, 0u} : sg[p];
                        const u128 part = (mine && ((cw >> code_shift(p, side)) & 3u) == want) ? to128(sp)
                                                                                               : (u128)0;
                        u128 tot;
                        const u128 ex_pre = T::excl_scan_u128(part, &tot, redA);
                        const u128 r = mulhi_64x128(U, tot);
                        if (part != 0 && ex_pre <= r && r < ex_pre + part) sm.pick = p;
                        done = true;
                    }
                    if (!done) {
                        // scan x's row: lane owns the contiguous arc segment [e0, e1)
                        const int32_t e0 = rs + (int32_t)(((int64_t)deg * lane) / TEAM);
                        const int32_t e1 = rs + (int32_t)(((int64_t)deg * (lane + 1)) / TEAM);
                        u128 part = 0;
                        int32_t e = e0;
                        for (; e + 4 <= e1; e += 4) {  // four independent loads in flight
                            const int32_t p0 = col[e], p1 = col[e + 1], p2 = col[e + 2], p3 = col[e + 3];
                            const uint32_t c0 = (code[p0 >> 3] >> code_shift(p0, side)) & 3u;
                            const uint32_t c1 = (code[p1 >> 3] >> code_shift(p1, side)) & 3u;
                            const uint32_t c2 = (code[p2 >> 3] >> code_shift(p2, side)) & 3u;
                            const uint32_t c3 = (code[p3 >> 3] >> code_shift(p3, side)) & 3u;
                            if (c0 == want) part += one ? (u128)1 : to128(sg[p0]);
                            if (c1 == want) part += one ? (u128)1 : to128(sg[p1]);
                            if (c2 == want) part += one ? (u128)1 : to128(sg[p2]);
                            if (c3 == want) part += one ? (u128)1 : to128(sg[p3]);
                        }
                        for (; e < e1; ++e) {
                            const int32_t p = col[e];
                            if (((code[p >> 3] >> code_shift(p, side)) & 3u) == want)
                                part += one ? (u128)1 : to128(sg[p]);
                        }
                        u128 tot;
                        const u128 ex_pre = T::excl_scan_u128(part, &tot, redA);
                        const u128 r = mulhi_64x128(U, tot);
                        if (part != 0 && ex_pre <= r && r < ex_pre + part) {
                            u128 acc = ex_pre;
                            for (int32_t q = e0; q < e1; ++q) {
                                const int32_t p = col[q];
                                if (((code[p >> 3] >> code_shift(p, side)) & 3u) != want) continue;
                                acc += one ? (u128)1 : to128(sg[p]);
                                if (acc > r) {
                                    sm.pick = p;
                                    break;
                                }
                            }
                        }
                    }
                    __syncthreads();
                    x = uniform_i32(sm.pick);
                    __syncthreads();
                    // the level-list path picks an original id
                    if (MAPPED && x >= 0 && probe_pick && qd->perm) x = qd->perm[x];
                    if (x < 0) {  // no predecessor found: cannot happen on a BFS level
                        if (lane == 0 && atomicCAS(&qctl->err, 0, 2) == 0)
                            atomicExch((unsigned long long *)&qctl->err_sample, (unsigned long long)i);
                        ok = false;
                        break;
                    }
                    if (lane == 0) {
                        sm.acc[ST_EBT] += (uint64_t)deg;
                        atomicAdd(&frame[x], 1);
                        sm.acc[ST_INTERIOR] += 1;
                    }
                }
            }
        } else if (lane == 0 && atomicCAS(&qctl->err, 0, fail_site) == 0) {
            atomicExch((unsigned long long *)&qctl->err_sample, (unsigned long long)i);
        }
        PHASE_MARK(4);

        // -- clear what this sample touched ----------------------------------
        // a code word holds only codes of vertices reached by this sample, so
        // zeroing whole words restores the all-zero state; four list entries
        // are loaded before their stores
        clear_ball<TEAM>(ball0, bend0, code);
        clear_ball<TEAM>(ball1, bend1, code);
        PHASE_MARK(5);
    }
    flush();

#ifdef KADABRA_PHASE_TIMERS
    if (lane == 0 && ph_ctl)
        for (int k = 0; k < 8; ++k)
            if (ph_acc[k]) atomicAdd((unsigned long long *)&ph_ctl->phase_cycles[k], ph_acc[k]);
#endif
}

// ---------------------------------------------------------------------------
// Epoch boundary: merge the epoch's frames into the counters (zeroing them)
// and evaluate the stopping rule of Appendix B on exactly samples [0, tau):
//   f = (L/tau) (1/3 - w/tau + sqrt((1/3 - w/tau)^2 + 2 b w / L))
//   g = (L/tau) (1/3 + w/tau + sqrt((1/3 + w/tau)^2 + 2 b w / L))
// b = c / tau, w = omega, L = log(1/delta_L(v)) in f and log(1/delta_U(v))
// in g.  IEEE double in this exact order; the file is compiled without
// floating-point contraction.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void stop_fg(int32_t c, double t, double w, double LL, double LU,
                                        double *f, double *g)
{
    const double b = (double)c / t;
    const double af = 1.0 / 3.0 - w / t;
    const double ag = 1.0 / 3.0 + w / t;
    const double qf = 2.0 * b * w / LL;
    const double qg = 2.0 * b * w / LU;
    *f = (LL / t) * (af + sqrt(af * af + qf));
    *g = (LU / t) * (ag + sqrt(ag * ag + qg));
}

constexpr int32_t MERGE_BLOCK = 256;
constexpr int32_t MERGE_MAX_BLOCKS = 1024;  // per query

// blocks a query's boundary gets in a merge launch
int32_t merge_blocks_for(int32_t n)
{
    const int32_t b = (n + MERGE_BLOCK - 1) / MERGE_BLOCK;
    return b < 1 ? 1 : (b > MERGE_MAX_BLOCKS ? MERGE_MAX_BLOCKS : b);
}

__global__ __launch_bounds__(MERGE_BLOCK) void merge_check_kernel(MergeArgs a)
{
    // the query whose block range holds this block (one query travels in the
    // arguments)
    MergeDesc M;
    int32_t qb, nb;
    if (!a.m) {
        M = a.one;
        qb = (int32_t)blockIdx.x;
        nb = a.nblocks;
    } else {
        int32_t lo = 0, hi = a.nq;
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (a.m[mid].block_begin <= (int32_t)blockIdx.x) lo = mid; else hi = mid;
        }
        M = a.m[lo];
        qb = (int32_t)blockIdx.x - M.block_begin;
        nb = ((lo + 1 < a.nq) ? a.m[lo + 1].block_begin : a.nblocks) - M.block_begin;
    }
    // the run stopped at the previous boundary: leave its counters as they are
    if (M.gate >= 0 && M.ctl->viol[M.gate] == 0) return;
    const size_t n = (size_t)M.n;
    const double t = (double)M.tau, w = (double)M.omega;
    int viol = 0;
    for (size_t v = (size_t)qb * MERGE_BLOCK + threadIdx.x; v < n; v += (size_t)nb * MERGE_BLOCK) {
        // counters in the original vertex order, frames and c1 in the internal one
        const size_t iv = M.perm ? (size_t)M.perm[v] : v;
        int32_t c = M.counts[v];
        for (int f = 0; f < M.nframes; ++f) {
            c += M.frames[(size_t)f * n + iv];
            M.frames[(size_t)f * n + iv] = 0;
        }
        M.counts[v] = c;
        if (M.do_check) {
            double LL = M.L, LU = M.L;
            if (M.lcon) {  // balanced: the constants of the vertex's first-phase count
                int64_t k = M.c1[iv];
                k = k < 0 ? 0 : (k > M.m1 ? M.m1 : k);  // in range (else device error 4 is set)
                LL = M.lcon[2 * k];
                LU = M.lcon[2 * k + 1];
            }
            double fv, gv;
            stop_fg(c, t, w, LL, LU, &fv, &gv);
            if (!(fv <= M.eps) || !(gv <= M.eps)) viol = 1;
        }
    }
    if (__syncthreads_or(viol) && threadIdx.x == 0) atomicOr(&M.ctl->viol[M.set], 1);
    if (qb == 0 && threadIdx.x < ST_COUNT) {
        // fold the epoch's work counters into the run's totals
        M.ctl->stats_total[threadIdx.x] += M.ctl->stats[M.set][threadIdx.x];
        M.ctl->stats[M.set][threadIdx.x] = 0;
    }
}

__global__ void scores_kernel(const int32_t *counts, double *scores, int32_t n, int64_t tau)
{
    const double t = (double)tau;
    for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < (size_t)n;
         v += (size_t)gridDim.x * blockDim.x)
        scores[v] = (double)counts[v] / t;
}

__global__ void eval_fg_kernel(const int32_t *counts, int32_t n, int64_t tau, int64_t omega,
                               double L, double *f, double *g)
{
    for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < (size_t)n;
         v += (size_t)gridDim.x * blockDim.x)
        stop_fg(counts[v], (double)tau, (double)omega, L, L, &f[v], &g[v]);
}

__global__ void fill_u32_kernel(uint32_t *p, size_t count, uint32_t value)
{
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < count;
         k += (size_t)gridDim.x * blockDim.x)
        p[k] = value;
}

static unsigned grid_for(size_t count, unsigned block)
{
    size_t g = (count + block - 1) / block;
    if (g > 8192) g = 8192;
    return g ? (unsigned)g : 1u;
}

template <bool MAPPED>
static hipError_t launch_sample_as(int team, int slots, const SampleArgs &a, bool pull, hipStream_t s)
{
#ifndef KADABRA_PHASE_TIMERS
    if (team == 64)
        hipLaunchKernelGGL((sample_kernel<64, MAPPED, false>), dim3(slots), dim3(64), 0, s, a);
    else
#endif
    if (team == 128)
        hipLaunchKernelGGL((sample_kernel<128, MAPPED, false>), dim3(slots), dim3(128), 0, s, a);
    else if (team == 256 && pull)
        hipLaunchKernelGGL((sample_kernel<256, MAPPED, true>), dim3(slots), dim3(256), 0, s, a);
    else if (team == 256)
        hipLaunchKernelGGL((sample_kernel<256, MAPPED, false>), dim3(slots), dim3(256), 0, s, a);
    else if (team == 512)
        hipLaunchKernelGGL((sample_kernel<512, MAPPED, false>), dim3(slots), dim3(512), 0, s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_sample(int team, int slots, const SampleArgs &a, bool mapped, bool pull, hipStream_t s)
{
    return mapped ? launch_sample_as<true>(team, slots, a, pull, s) : launch_sample_as<false>(team, slots, a, pull, s);
}

hipError_t launch_merge_check(const MergeArgs &a, hipStream_t s)
{
    if (a.nq == 0) return hipSuccess;
    hipLaunchKernelGGL(merge_check_kernel, dim3(a.nblocks), dim3(MERGE_BLOCK), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_scores(const int32_t *counts, double *scores, int32_t n, int64_t tau,
                         hipStream_t s)
{
    hipLaunchKernelGGL(scores_kernel, dim3(grid_for((size_t)n, 256)), dim3(256), 0, s, counts,
                       scores, n, tau);
    return hipGetLastError();
}

hipError_t launch_eval_fg(const int32_t *counts, int32_t n, int64_t tau, int64_t omega, double L,
                          double *f, double *g, hipStream_t s)
{
    hipLaunchKernelGGL(eval_fg_kernel, dim3(grid_for((size_t)n, 256)), dim3(256), 0, s, counts, n,
                       tau, omega, L, f, g);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, size_t count, uint32_t value, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(count, 256)), dim3(256), 0, s, p, count,
                       value);
    return hipGetLastError();
}

}  // namespace kd
