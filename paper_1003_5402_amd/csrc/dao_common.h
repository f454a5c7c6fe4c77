// Internal types shared by the host library and the gfx950 kernels.
#pragma once

#include <stdint.h>

namespace dao {

constexpr int WAVE = 64;              // CDNA wavefront width
constexpr int SLICE = 64;             // rows per forward-layout slice (one per wavefront)
constexpr int MAX_ROW_LEN = 64;       // one MLC row per wavefront in pricing
constexpr int MAX_APERTURES = 256;
constexpr int KS = 64;                // aperture slots per row of the aperture dose matrix
constexpr int LS_MAX_ITER = 60;       // line-search evaluations per master step
constexpr int BLOCK = 256;            // threads per block of the streaming kernels
constexpr int NPART = 6;              // doubles per block in a reduction record

// Rows of the persistent master's workgroups (forms that stream the aperture
// dose matrix): the batches of voxel rows are dealt in rounds of one batch
// per workgroup; in round lb, workgroup b of a solve on gn workgroups owns
// batch lb * gn + (b + COOP_SKEW * lb) % gn.  The rows the update pass has to
// read (voxels outside their dose window) cluster in space and, after the
// length sort, at the start of each sort window; dealing the batches spreads
// them over the workgroups, and the skew keeps a pattern that repeats with
// the round length from landing on the same workgroups every round.
// (constexpr: usable on the host and, in HIP, on the device.)
constexpr int64_t COOP_SKEW = 101;
constexpr int64_t coop_batch(int64_t lb, uint32_t b, uint32_t gn) {
    return lb * gn + (int64_t(b) + COOP_SKEW * lb) % gn;
}
// Batches of workgroup b: one per full round, and the last partial round's
// when its slot falls inside it.
constexpr int64_t coop_nbatches(int64_t nbat, uint32_t b, uint32_t gn) {
    return nbat / gn + ((nbat % gn > 0 && (int64_t(b) + COOP_SKEW * (nbat / gn)) % gn < nbat % gn) ? 1 : 0);
}

// Objective coefficients of a voxel class (eq. 9 and eq. 10): the terms of
// its first structure and, for a voxel in two overlapping structures, of its
// second (zero weights when there is none).  a and b are the structure
// weights already divided by the structure size.  Classes 0 .. n_struct - 1
// are the single structures, class n_struct is "no structure" (all zero),
// later classes are pairs of structures.
struct ObjClass {
    double a, t_under, b, t_over;
    double a2, t_under2, b2, t_over2;
};
constexpr int MAX_CLASSES = 256;

// Phases of one gradient-projection step (the master loop is a fixed
// sequence of launches; each launch runs only in its phase).
enum Phase : int {
    PH_DIR = 0,   // gradient over the pool, projection, t_max, dx = A p
    PH_Q = 1,     // q = D dx and the first line-search evaluation
    PH_LS = 2,    // further line-search evaluations
    PH_UPD = 3,   // d += t q (or d = D(A y) on refresh steps), grad F, F
    PH_TP = 4     // g = D^T grad F
};

// Device-resident master state.  Written only by single threads (a lone
// block, or the last block of a launch) and read by every block at the start
// of the next launch.
struct MasterState {
    int32_t phase;
    int32_t done;          // 1: converged / cap reached / zero direction
    int32_t steps;         // steps taken in the current master solve
    int32_t max_steps;
    int32_t K;             // pool size
    int32_t ls_iter;       // evaluations in the current line search
    int32_t hi_known;
    int32_t refresh;       // update mode: 0 d += t q, 1 d = D(A y), 2 keep d (refresh u, F only)
    int32_t refresh_every;
    int32_t stop_reason;   // 0 running, 1 kkt, 2 cap, 3 zero direction
    int64_t total_steps;
    int64_t total_ls;
    double tol;
    double kkt;
    double t;              // current trial / final step
    double lo, hi;
    double t_max;
    double gphi0;          // <grad_y, p>
    double F;              // objective at the current dose
    double F_const;        // objective of voxels no beamlet reaches (dose 0)
    double last_step;      // length of the last step
    double prev_step;      // length of the step before it
    int32_t conj;          // 1: conjugate gradient projection, 0: projected steepest descent
    int32_t cg_valid;      // the conjugate memory (CgMem, p) holds the last step of this pool
    int32_t cg_K;          // pool size when the memory was recorded
    int32_t cg_pad;
};

// Memory of the conjugate direction: projected negative gradient r and free
// set of the last step (its direction stays in the master's p array).
struct CgMem {
    double r[MAX_APERTURES];
    int32_t free[MAX_APERTURES];
};

// Work counters of the aperture master's kernels, kept by workgroup 0 of
// every launch that does work: launches that ran and their algorithmic
// bytes.  Index: 0 update pass, 1 q pass, 2 line-search pass, 3 direction.
// The persistent master also splits workgroup 0's time into phases.
constexpr int PROF_PHASES = 7;
struct ProfCounters {
    double bytes[4];
    uint64_t real[4];
    uint64_t ticks[PROF_PHASES];   // persistent master: wall-clock ticks per phase (workgroup 0)
};

// Pricing result written by the last block of the pricing launch.
struct PriceResult {
    int32_t beam;
    int32_t n_rows;
    double rc;
    double gap;
    int16_t leaves[2 * 1024];   // (L, R) per row of the chosen beam
};

}  // namespace dao
