// kmc_internal.h -- structures shared by the host runtime (kmc_api.hip) and
// the gfx950 kernels (kmc_device.hip) of libkmc.so.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kmc.h"

namespace kmc {

// Threads per block of the streaming kernels and of the three-pass scan.
constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;
// Per-step accumulators of the collision count, the digest and the recorded
// candidates: one 128-byte line each, so the per-block atomics of the search
// and the resolve spread over this many cache lines (k_advance folds them).
constexpr int kAccLanes = 1024;
// Candidates the search records per particle before the particle falls
// back to a full search.
constexpr int kSlots = 8;
// Table stride of the per-kind-pair tables (= KMC_MAX_SPECIES).
constexpr int kMaxKinds = 8;
// FP32 screen: thresholds per box for search groups of at most 64, 256, 1024
// and 4096 cells along x (a group uses the smallest class that holds it;
// wider rows are split into groups of 4096 cells).
constexpr int kSpanClasses = 4;

// Device copy of one box.  All derived scalars are computed once on the host
// (L = hi - lo, R2 = R*R) so that every kernel sees the same bits.  With
// particle kinds D2 is the largest pair value (the screen's bounds and the
// cell-size check use it); the criterion takes the pair's own value.
struct alignas(16) BoxDev {
    double lo[3], hi[3], L[3], inv_h[3];
    double D2, dt, R, R2;
    int32_t nc[3];
    int32_t periodic[3];
    int32_t absorb[3];   // absorbing faces per axis
    int32_t sphere;
    uint32_t coff;       // first global cell of the box (its nc[0]*nc[1]*nc[2] grid cells are
                         // followed by one cell for the particles absorbed so far)
    uint32_t poff;       // first global particle index of the box
    uint32_t n;          // particles in the box
    // FP32 screen constants
    float D2_32, dt_32;  // thresholds rounded to FP32
    double rmax[3];      // bound on |r_k| for any neighbour pair (2 h_k)
    // time step: dt above is this step's; dt_cap is the box's configured step
    // (the adaptive rule's upper bound), dx the smallest cell edge
    // (hi_k - lo_k) / nc_k, time the simulated time since initialisation
    double dx, dt_cap, time;
    double h[3];         // cell edges (hi_k - lo_k) / nc_k
};

// Flag on a particle id (ids stay below 2^31): the particle was absorbed by
// an absorbing face and has left the gas.
constexpr uint32_t kGone = 0x80000000u;

// Cell-sorted FP64 particle record (48 bytes, 16-byte aligned).
struct alignas(16) P64 {
    double x, y, z, vx, vy, vz;
};

struct alignas(128) StepAcc {
    unsigned long long np, dig, cand;
    unsigned long long pad_[13];
};

// Candidate list entry: one 16-byte store per posted pair.
struct alignas(16) SlotEntry {
    double key;      // c2 / g2 of the pair (the same from both sides)
    uint32_t j;      // sorted index of the other particle
    uint32_t pad_;
};

// Per-context control block in device memory.
struct Ctl {
    unsigned long long step;            // global index of the next step
    unsigned long long steps_done;      // steps completed since init
    unsigned long long rechecks_total;  // particles re-searched in full FP64 (list overflow)
    unsigned long long fallbacks_total; // steps that took the whole-step FP64 search
    unsigned long long scratch;         // target of host-requested reductions
    unsigned long long absorbed_total;  // particles absorbed by absorbing faces so far
    unsigned long long candidates_total;// pairs the search recorded, summed over steps
    unsigned int recheck_count;         // this step's recheck list length
    unsigned int overflow;              // this step's flag for the whole-step FP64 search
    unsigned int ovf_count;             // this step's overflow pair list length
    unsigned int refined_count;         // adaptive bins: bins split this step
    unsigned int pool_used;             // adaptive bins: leaf-table entries claimed this step
    unsigned int pad_;
};

// FP32 screen thresholds of one box for one step.  The bounds on the error
// of the screen's b, m2 = -b - dt g2 and m3 = (|r|^2 - D2) g2 - b^2 are affine
// in the pair's g2 (t0 + t1 g2); the g2 terms are folded into the tests'
// constants, so a pair is kept when
//   b - tb1 g2 <= tb0,  -b - kdt g2 <= tt0,  (|r|^2 - kD2) g2 - b^2 <= tc0
// with kdt >= dt + tt1 and kD2 >= D2 + tc1 plus the rounding of |r|^2 - kD2.
// tt1 and tc1 are kept for reference.
struct alignas(16) ScreenBounds {
    float tb0, tb1, tt0, kdt, tc0, kD2, tt1, tc1;
};

// Device pointers carved out of the caller's workspace plus launch scalars.
struct Plan {
    Ctl* ctl;
    BoxDev* boxes;
    unsigned long long* hist_np;   // [history]: collision count of each step (a ring)
    unsigned long long* hist_dig;  // [history]: digest of each step
    StepAcc* acc;                  // [kAccLanes]: this step's partial sums
    double* A;                     // current state, 6*N SoA (previous cell order)
    P64* B;                        // cell-sorted copy of the current state (records)
    float* vmax_part;              // per scatter block: max |v_k| of its particles this step
    unsigned int* box_vmax;        // per box: max |fl32(v_k)| this step (FP32 bits)
    ScreenBounds* box_sb;          // per box [kSpanClasses]: FP32 screen thresholds this step
    uint32_t* idA;
    uint32_t* idB;
    uint32_t* cell;                // per particle in A order: global cell (adaptive bins only;
                                   // otherwise recomputed from the position where needed)
    uint32_t* slot;                // per particle in A order: rank inside its cell
    int32_t* partner;              // per sorted particle: sorted index of partner or -1
    uint32_t* sl_cnt;              // per sorted particle: entries posted to its candidate list
    SlotEntry* sl;                 // [kSlots][N]: (FP64 key, sorted index of the other particle)
    double* fb_key;                // per sorted particle: key of its forward best (inf: none)
    int32_t* fb_j;                 // per sorted particle: its forward best (-1: none)
    uint32_t* boxidx;              // per particle: its box (null when there is one box)
    uint32_t* count;               // per cell: particles (zero between steps)
    uint32_t* start;               // per cell + 1: exclusive prefix of count
    uint32_t* partial;             // scan block sums
    uint32_t* recheck;             // sorted indices to re-search in full FP64
    uint2* ovf;                    // pairs a search lane found beyond its register slots
    unsigned long long* v2_part;   // adaptive dt: per scatter block, max |v|^2 (FP64 bits) of
                                   // its particles in the box of its first particle
    unsigned long long* box_v2;    // adaptive dt: per box, max |v|^2 of the other particles
    uint32_t N, C, nboxes, H;
    uint32_t nblk_scan;
    uint32_t recheck_cap;
    uint32_t ovf_cap;
    uint64_t seed;
    int32_t precision, kinematics, block;
    uint32_t nblk_part;            // scatter blocks (entries of vmax_part)
    float guard;                   // FP32 screen: scale of the rounding-error bounds (>= 1)
    int32_t dt_rule;               // kmc_dt_rule
    int32_t search_mode;           // kmc_search_mode
    int32_t tile;                  // tile shape of the search kernel (0, 1, 2)
    // density-adaptive bins (adapt_L == 0: the uniform grid)
    int32_t adapt_L;               // at most this many halvings of a bin
    uint32_t adapt_T;              // split while more than adapt_T * 8^level particles
    uint8_t* level;                // per cell: its split level this step
    uint8_t* mixed;                // per cell: 1 if it or one of its 26 neighbours is split
    uint32_t* pool_base;           // per split cell: first entry of its leaf table in pool
    uint32_t* refined;             // the cells split this step (ctl->refined_count)
    uint32_t* pool;                // leaf tables: per split cell 8^level counts, then their
                                   // exclusive prefix (leaf starts relative to the cell's
                                   // start) and the cell's count
    uint32_t pool_cap;             // entries of pool
    uint32_t* leaf_slot;           // per particle in A order: its rank in its leaf
    int32_t dims;                  // 3, or 2 for the planar mode
    double dt_factor;              // adaptive dt: C in dt = min(cap, C dx / v_max)
    // particle kinds (nspecies == 0: one kind, the box's D2, equal masses)
    int32_t nspecies;
    uint8_t* spA;                  // per particle in A order: its kind
    uint8_t* spB;                  // per sorted particle: its kind
    const double* sp_D2;           // [kMaxKinds][kMaxKinds]: (radius_s + radius_t)^2
    const double* sp_mass;         // [kMaxKinds]
    float* box_kD2;                // per box [kSpanClasses][kMaxKinds][kMaxKinds]: the FP32
                                   // screen's folded D2 constant of each pair of kinds this step
};

// Kernel launchers (kmc_device.hip).  `ev`, when not null, points to
// KMC_PHASE_COUNT + 2 events recorded on `s`: ev[k] at the start of phase k,
// ev[KMC_PHASE_COUNT] at the end of the step and ev[KMC_PHASE_COUNT + 1]
// right before the search kernel itself (after the screen's bound kernels).
hipError_t launch_init(const Plan& p, const double* d_state, const uint8_t* d_kind, hipStream_t s);
hipError_t launch_step(const Plan& p, hipStream_t s, hipEvent_t* ev);
hipError_t launch_read_partners(const Plan& p, int32_t* out, hipStream_t s);
hipError_t launch_read_state(const Plan& p, double* out, hipStream_t s);
hipError_t launch_count_tests(const Plan& p, unsigned long long* d_out, hipStream_t s);

}  // namespace kmc
