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

// Indices into the per-epoch work counters (int64).  Every counter is
// algorithm-defined: it does not depend on the mapping of samples to lanes.
enum StatIdx {
    ST_VEXP = 0,   // frontier vertices expanded
    ST_ESCAN,      // arcs scanned by expansions
    ST_EBT,        // arcs scanned while backtracking (sum of the path vertices' degrees)
    ST_INTERIOR,   // counter increments
    ST_DISCONN,    // samples with endpoints in different components
    ST_COUNT
};

// Device control block (one per handle).
struct Control {
    uint32_t claim[2];               // sample claim counters, by epoch parity
    int32_t viol[2];                 // stopping-rule violations, by epoch parity
    int32_t err;                     // device-side invariant failure (0 = none)
    int32_t pad;
    int64_t stats[2][ST_COUNT];      // work counters of the epoch in flight, by parity
    int64_t stats_total[ST_COUNT];   // work counters of merged epochs
    int64_t phase_cycles[8];         // per-phase cycles (phase-timer builds only)
};

// Per-slot sampling state.  Between samples every code word and every sigma
// is zero (each sample clears what it touched).
struct SlotState {
    uint32_t *code;     // [slots][code_stride] 2-bit level codes per side, 8 vertices a word
    Sigma *sigma;       // [slots][2][n] sigma_s, sigma_t
    int32_t *ball;      // [slots][2][n] vertices reached by each side, BFS order
    int32_t *meet;      // [slots][n] meeting set
    uint64_t *meetw;    // [slots][n] meeting weights (when the set exceeds LDS)
    int32_t *loff;      // [slots][2][lcap] start of each BFS level in ball
    int32_t lcap;       // entries per side (diameter bound + 2)
    int32_t code_stride;  // words per slot (ceil(n / 8), rounded up to 64 bytes)
};

struct SampleArgs {
    const int32_t *row_ptr;
    const int32_t *col;
    const int32_t *comp;
    int32_t n;
    int32_t nframes;
    uint64_t seed;
    int64_t lo, hi;   // sample indices of this epoch: [lo, hi)
    int32_t parity;   // epoch parity (selects claim counter, frames, stats)
    int64_t probe_min;  // >= 0: expansions of at least this many arcs probe for the meeting
                        // first; -1: probe when D_X * D_Y >= num_arcs
    int64_t num_arcs;
    int32_t gate;     // -1, or the parity of the previous boundary: if its check
                      // found no violation the run has stopped and this launch exits
    int32_t *frames;  // [2][nframes][n]
    Control *ctl;
    SlotState st;
};

struct CheckArgs {
    int32_t *counts;  // [n] counters of samples [0, tau)
    int32_t *frames;  // [2][nframes][n]
    int32_t n;
    int32_t nframes;
    int32_t parity;
    int32_t do_check; // 0: merge only (tau == omega)
    int64_t tau, omega;
    double L, eps;
    Control *ctl;
};

hipError_t launch_sample(int team, int slots, const SampleArgs &a, hipStream_t s);
hipError_t launch_merge_check(const CheckArgs &a, hipStream_t s);
hipError_t launch_scores(const int32_t *counts, double *scores, int32_t n, int64_t tau,
                         hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, size_t count, uint32_t value, hipStream_t s);
hipError_t launch_eval_fg(const int32_t *counts, int32_t n, int64_t tau, int64_t omega, double L,
                          double *f, double *g, hipStream_t s);

}  // namespace kd
