// kadabra_internal.h -- device-side argument blocks and kernel launchers shared
// by the host driver (kadabra_host.cpp) and the kernels (kadabra_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kd {

// Per-vertex 128-bit path count (sigma), little-endian words.
struct Sigma {
    uint64_t lo, hi;
};

// Indices into the per-epoch work counters (int64).  Every counter but
// ST_VMAT is algorithm-defined: it does not depend on the mapping of samples
// to lanes.
enum StatIdx {
    ST_VEXP = 0,   // frontier vertices expanded
    ST_ESCAN,      // arcs scanned by expansions
    ST_EBT,        // arcs scanned while backtracking (sum of the path vertices' degrees)
    ST_INTERIOR,   // counter increments
    ST_DISCONN,    // samples with endpoints in different components
    ST_VMAT,       // new vertices written (claimed) by level expansions: every new level in
                   // full except a probed meeting level, which writes only the meeting set.
                   // The one counter that depends on the mapping (the probe threshold).
    ST_COUNT
};

// Epochs (check intervals) in flight per query are kept apart in frame sets:
// epoch e (samples [B_{e-1}, B_e)) uses set e mod nsets, nsets = 2 x (epochs
// per launch), so a launch and the speculative launch after it never share one.
constexpr int kMaxSets = 8;
constexpr int kFirstSet = kMaxSets;  // work-counter set of the balancing first phase

// First-phase sample m of a balanced run is sample index kFirstPhaseBase + m:
// a range of the random stream that the adaptive samples never reach.
constexpr uint64_t kFirstPhaseBase = 1ull << 63;

// Device control block of one adaptive run (one per query).
struct Control {
    int32_t viol[kMaxSets];          // stopping-rule violations of a boundary, by epoch set
    int32_t err;                     // device-side invariant failure (0 = none), by site:
                                     // 1 level bound, 2 no predecessor, 3 frontier empty
    int32_t pad;
    int64_t err_sample;              // sample index of the first failure
    int64_t stats[kMaxSets + 1][ST_COUNT];  // work counters of epochs in flight, by set;
                                            // [kFirstSet]: the first phase (never merged)
    int64_t stats_total[ST_COUNT];   // work counters of merged epochs
    int64_t phase_cycles[8];         // per-phase cycles (phase-timer builds only)
};

// Per-slot sampling state (a pool shared by every query of a launch; a slot
// holds one sample at a time).  Between samples every code word is zero (each
// sample clears the words it set); sigma holds stale values, and a sample
// writes the sigma of each vertex it reaches before reading it.
struct SlotState {
    uint32_t *code;     // [slots][code_stride] 2-bit level codes per side, 8 vertices a word
    Sigma *sigma;       // [slots][2][nstride] sigma_s, sigma_t
    int32_t *ball;      // [slots][2][nstride] vertices reached by each side, BFS order
    int32_t *meet;      // [slots][nstride] meeting set
    uint64_t *meetw;    // [slots][nstride] meeting weights (when the set exceeds LDS)
    int32_t *loff;      // [slots][2][lcap] start of each BFS level in ball
    int64_t nstride;    // vertex capacity of a slot (largest n of the launch)
    int32_t lcap;       // level capacity per side (largest diameter bound + 2)
    int32_t code_stride;  // words per slot (ceil(nstride / 8), rounded up to 64 bytes)
};

// One query's consecutive epochs in a sampling launch.
struct QueryDesc {
    const int32_t *row_ptr;
    const int32_t *col;
    const int32_t *comp;
    const int32_t *perm;   // original -> internal vertex id (null: the same)
    const int32_t *iperm;  // internal -> original
    const int32_t *colo;   // col as original ids (rows ascending in them)
    int32_t *frames;      // every frame set: [nsets][nframes][n]
    Control *ctl;
    uint64_t seed;
    int64_t lo, hi;       // sample indices of this launch: [lo, hi), whole epochs (the last
                          // one may end at omega)
    int64_t epoch_len;    // N: sample i belongs to epoch i / N + 1
    int64_t claim_begin;  // launch-wide claim index of sample lo
    int64_t probe_min;    // >= 0: probe expansions of at least this many arcs; -1: auto rule
    int64_t num_arcs;
    int32_t n;
    int32_t nframes;
    int32_t nsets;        // frame sets (epoch e uses set e mod nsets)
    int32_t gate;         // -1, or the set of the boundary before lo: if its check found no
                          // violation the run has stopped and this launch does no work for it
    int32_t stat_set;     // -1: work counters by epoch set; else this set (first phase)
    int32_t probe_h8;     // auto probe rule (probe_min < 0): probe when the frontiers' degree
                          // sums D_X D_Y reach probe_h8 / 8 x num_arcs
    int32_t probe_quit;   // 1: a probe whose first round meets nothing is given up
    int32_t pad;
    // A first phase is a descriptor with lo = INT64_MIN (its samples' indices
    // are then kFirstPhaseBase + m as unsigned), nsets = nframes = 1,
    // frames = c1 and stat_set = kFirstSet.
};

struct SampleArgs {
    const QueryDesc *q;   // queries of this launch, by increasing claim_begin
    int32_t nq;
    int32_t gated;        // 1: every query of the launch has a gate (a speculative launch)
    int64_t total;        // samples of this launch
    unsigned long long *claim;  // monotone claim counter
    uint64_t claim_base;  // its value when this launch starts
    SlotState st;
};

// One query's boundary in a merge-and-check launch.
struct MergeDesc {
    int32_t *counts;      // [n] counters of samples [0, tau)
    int32_t *frames;      // the epoch's frame set: [nframes][n]
    Control *ctl;
    const int32_t *perm;  // counters are in the original order, frames and c1 in the
                          // internal one: vertex v's entries are at perm[v] (null: v)
    const int32_t *c1;    // balanced runs: first-phase counters [n]; the vertex's constants
    const double *lcon;   // are lcon[2 c1[v]] (delta_L) and lcon[2 c1[v] + 1] (delta_U);
                          // null: L for every vertex
    int64_t m1;           // first-phase samples (rows of lcon: m1 + 1)
    int64_t tau, omega;
    double L, eps;
    int32_t n;
    int32_t nframes;
    int32_t set;          // the epoch's set (flag and work counters)
    int32_t gate;         // -1, or the set of the previous boundary: skip if the run stopped there
    int32_t do_check;     // 0: merge only (tau == omega)
    int32_t block_begin;  // first block of this query in the launch
};

struct MergeArgs {
    const MergeDesc *m;   // the queries' descriptors in device memory; null: the one query
    int32_t nq;           // is `one`, passed in the arguments (no copy before the launch)
    int32_t nblocks;
    MergeDesc one;
};

// Balancing of delta_L(v), delta_U(v) from the first-phase counters c1:
// hist[k] = #{v : c1[v] = k} (hist zeroed beforehand, m1 + 1 entries; a
// counter above m1 cannot occur and is reported as device error 4).  The
// host then plans t* and the constant table lcon from the histogram.

// mapped: some query of the launch is on a relabelled graph; pull: meeting
// probes in the pull form (256-lane teams; other teams push)
hipError_t launch_sample(int team, int slots, const SampleArgs &a, bool mapped, bool pull, hipStream_t s);
hipError_t launch_hist(const int32_t *c1, int32_t n, int32_t *hist, int64_t m1, Control *ctl, hipStream_t s);
hipError_t launch_merge_check(const MergeArgs &a, hipStream_t s);
int32_t merge_blocks_for(int32_t n);
hipError_t launch_scores(const int32_t *counts, double *scores, int32_t n, int64_t tau,
                         hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, size_t count, uint32_t value, hipStream_t s);
hipError_t launch_eval_fg(const int32_t *counts, int32_t n, int64_t tau, int64_t omega, double L,
                          double *f, double *g, hipStream_t s);

// Graph preprocessing (kadabra_prep.hip): components as each vertex's
// component minimum id; BFS from every component's maximum-degree vertex
// (lowest id on ties).  counters: [0] roots found (the first frontier),
// [2] components; key must start zeroed.
hipError_t launch_cc(const int32_t *row_ptr, const int32_t *col, int32_t n, int32_t *parent, hipStream_t s);
hipError_t launch_bfs_roots(const int32_t *row_ptr, const int32_t *comp, int32_t n, unsigned long long *key,
                            int32_t *dist, int32_t *frontier, int32_t *counters, hipStream_t s);
hipError_t launch_bfs_level(const int32_t *row_ptr, const int32_t *col, const int32_t *frontier,
                            const int32_t *count, int32_t frontier_size, int32_t level, int32_t *dist,
                            int32_t *next, int32_t *next_count, hipStream_t s);
hipError_t launch_gather_i32(int32_t *dst, const int32_t *src, const int32_t *idx, int32_t n, hipStream_t s);

// Several buffers zeroed by one launch (a query's counters, frames, control
// block and balancing buffers).
constexpr int kMaxZeroRegions = 5;
struct ZeroRegions {
    uint32_t *ptr[kMaxZeroRegions];
    size_t count[kMaxZeroRegions];  // 32-bit words
    int n;
};
hipError_t launch_zero_regions(const ZeroRegions &z, hipStream_t s);
hipError_t launch_bfs_small(const int32_t *row_ptr, const int32_t *col, int32_t *dist, int32_t *q0, int32_t *q1,
                            int32_t *state, int32_t small_max, hipStream_t s);

}  // namespace kd
