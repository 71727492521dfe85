/*
 * kmc.h -- C ABI of libkmc.so, an MI355X (gfx950) implementation of the
 * per-time-step collision step of the kinetic Monte-Carlo code of Howell et
 * al., "Parallelization of Kinetic Theory Simulations" (arXiv:1310.3437).
 *
 * One step (Section 1, "Initial Simulation Setup"):
 *   1. bin every particle into a uniform grid of cells (the paper's bins);
 *   2. every particle searches its own and the 26 neighbouring cells for its
 *      closest acceptable partner by distance of closest approach (DCA):
 *      with r = x_j - x_i, g = v_j - v_i the relative path r + g t comes
 *      closest at t* = -r.g/|g|^2 with squared distance |r x g|^2/|g|^2;
 *      j is acceptable if 0 <= t* <= dt and that distance is below
 *      D = sqrt(sigma/pi) (for particles of several kinds, the sum of the
 *      two effective radii); the closest acceptable partner wins, equal
 *      distances going to the smaller id;
 *   3. two particles collide only if each chose the other;
 *   4. a colliding pair moves to t*, scatters elastically and isotropically
 *      in its centre-of-mass frame (direction from Philox4x64-10 keyed by
 *      the seed, the step and the pair's smaller id; mass-weighted for
 *      particles of unequal masses), and moves on with the new velocities
 *      for dt - t*; everybody else streams freely for dt;
 *   5. boundary conditions: periodic, reflecting or absorbing box faces
 *      (Section 1 names reflective, absorptive and periodic boxes) or a
 *      reflecting sphere.
 * The exact arithmetic (rounding order, fused operations, random-number
 * layout) is the library's published definition, identical to that of the
 * independent CPU reference it is tested against.
 *
 * Conventions for every function:
 *   - all functions return a kmc_status (0 = KMC_OK, < 0 = error) and never
 *     abort; invalid arguments return KMC_EINVAL with no side effects;
 *   - "device pointer" means memory on the GPU that is current when the
 *     function is called; "host pointer" means ordinary CPU memory;
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream);
 *     all device work is enqueued on it, asynchronously unless stated;
 *   - the caller owns every device buffer (state, workspace, outputs); the
 *     library never allocates device memory.  It owns only the host-side
 *     kmc_ctx and, when graphs are enabled, one private capture stream and
 *     the captured graph, all released by kmc_destroy (and, for
 *     kmc_init_scratch, a static workspace array per device).
 */
#ifndef KMC_H
#define KMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KMC_ABI_VERSION 5

typedef enum {
    KMC_OK = 0,
    KMC_EINVAL = -1,     /* invalid argument (nothing was done)                    */
    KMC_ENOMEM = -2,     /* workspace too small, or host allocation failed          */
    KMC_EDEVICE = -3,    /* a HIP runtime call failed                               */
    KMC_EOVERFLOW = -4,  /* a size exceeds the library's index range                */
    KMC_ESTATE = -5      /* call not valid in the context's current state          */
} kmc_status;

/* KMC_FP64: the pair test in binary64.
 * KMC_FP32_SCREEN: the search tests pairs in FP32 against rigorous bounds on
 *   the rounding error and decides every pair it keeps in FP64, so the
 *   partners are those of KMC_FP64 bit for bit.  A step that breaks an
 *   assumption of the bounds takes the whole-step FP64 search instead
 *   (counted in kmc_stats.fallbacks).  That happens when a particle lies
 *   outside its box's grid, or when a box's cell edges or largest speed
 *   fall outside [2^-40, 2^40] (a speed of 0 is fine). */
typedef enum { KMC_FP64 = 0, KMC_FP32_SCREEN = 1 } kmc_precision;
typedef enum { KMC_GEOM_BOX = 0, KMC_GEOM_SPHERE = 1 } kmc_geometry;
typedef enum { KMC_BC_REFLECT = 0, KMC_BC_PERIODIC = 1, KMC_BC_ABSORB = 2 } kmc_bc;
typedef enum { KMC_KIN_AT_TSTAR = 0, KMC_KIN_VEL_ONLY = 1 } kmc_kinematics;
typedef enum { KMC_DT_FIXED = 0, KMC_DT_ADAPTIVE = 1 } kmc_dt_rule;
/* How the partner search is organised (the result is the same):
 *   KMC_SEARCH_HALF  every unordered neighbour pair is tested once and
 *                    acceptable pairs are recorded for both particles; the
 *                    partner is the minimum over the recorded pairs (fast
 *                    when particles have few acceptable partners);
 *   KMC_SEARCH_FULL  every particle scans its whole neighbourhood keeping
 *                    a running minimum (twice the pair tests, no lists; for
 *                    dense cells with many acceptable partners). */
typedef enum { KMC_SEARCH_HALF = 0, KMC_SEARCH_FULL = 1 } kmc_search_mode;

/* One independent simulation box.
 *   n         particles in the box (their state is a contiguous slice of the
 *             caller's state, boxes in order);
 *   geometry  KMC_GEOM_BOX: faces at lo/hi with per-axis bc;
 *             KMC_GEOM_SPHERE: reflecting sphere of radius sphere_r about the
 *             origin inside the cell grid lo..hi (bc must be REFLECT);
 *   bc[k]     KMC_BC_PERIODIC, KMC_BC_REFLECT or KMC_BC_ABSORB for axis k
 *             (Section 1 names reflective, absorptive and periodic boxes).
 *             Absorbing faces (geometry BOX only): a particle whose streamed
 *             position lies beyond them (x < lo or x > hi on that axis) at
 *             the end of a step leaves the gas for good: it is in no cell,
 *             never searches, collides or moves again, its partner is -1,
 *             and kmc_read_state reports the state it had when it left;
 *   ncell[k]  cells (bins) along axis k; >= 1, and >= 3 on periodic axes;
 *   lo, hi    grid (and box) bounds, hi > lo;
 *   inv_h[k]  ncell[k] / (hi[k] - lo[k]) as computed by the caller (the
 *             cell of x is clamp(floor((x - lo) * inv_h), 0, ncell - 1));
 *             the cell edge 1/inv_h must be >= sqrt(D2) on every axis;
 *   D2        squared interaction diameter sigma/pi (> 0);
 *   dt        time step (> 0); with KMC_DT_ADAPTIVE the largest step allowed.
 * Requirement (not checked): no particle moves more than one box length per
 * step. */
typedef struct kmc_box {
    uint32_t n;
    int32_t geometry;
    int32_t bc[3];
    int32_t ncell[3];
    double lo[3];
    double hi[3];
    double inv_h[3];
    double sphere_r;
    double D2;
    double dt;
} kmc_box;

/* Kinds of particles (species).  Section 1 gives every particle its own
 * mass and effective radius, and a candidate must be within the effective
 * radii of the searcher.  With species, particle i is of kind s_i:
 *   - a pair (i, j) is within each other's effective radii when its distance
 *     of closest approach is below radius[s_i] + radius[s_j]: the criterion
 *     c2 < D2_ij * g2 uses D2_ij = d * d with d = radius[s_i] + radius[s_j]
 *     in binary64, in place of the box's D2 (which is then not used in the
 *     criterion, but is still validated);
 *   - the ordering key is unchanged (the squared distance of closest
 *     approach c2 / g2);
 *   - a colliding pair with equal masses scatters as without species; with
 *     masses m_a != m_b (a the smaller id) M = m_a + m_b,
 *     v_cm,k = fma(m_a, v_a,k, m_b * v_b,k) / M, |g| = sqrt(g2), and a and b
 *     leave with v_cm + ((m_b / M) * |g|) n and v_cm - ((m_a / M) * |g|) n
 *     (momentum and kinetic energy are kept);
 *   - every box's cell edge must be >= the largest pair diameter
 *     2 * max(radius) on every axis.
 * Fields:
 *   count      kinds, 1..KMC_MAX_SPECIES;
 *   reserved   must be zero;
 *   radius[s]  effective radius of kind s (finite, > 0), s < count;
 *   mass[s]    mass of kind s (finite, > 0), s < count;
 *   d_kind     device pointer, n_total bytes in id order (box offsets as for
 *              the state): the kind of each particle, < count; read on the
 *              caller's stream during kmc_init (and during each context that
 *              kmc_autotune creates); an entry >= count makes kmc_init fail
 *              with KMC_EINVAL.
 * The structure is read during kmc_workspace_bytes, kmc_init and
 * kmc_autotune only; the context keeps a copy of count, radius and mass. */
#define KMC_MAX_SPECIES 8
typedef struct kmc_species {
    uint32_t count;
    uint32_t reserved;
    double radius[KMC_MAX_SPECIES];
    double mass[KMC_MAX_SPECIES];
    const uint8_t* d_kind;
} kmc_species;

/* Run configuration.  Zero-initialise and set what you need. */
typedef struct kmc_config {
    uint64_t seed;             /* Philox key word 0                                      */
    uint64_t step0;            /* global index of the first step (resume)                */
    int32_t precision;         /* kmc_precision                                          */
    int32_t kinematics;        /* kmc_kinematics                                         */
    uint32_t history;          /* per-step (npairs, digest) slots kept; 0 = 1024         */
    uint32_t recheck_capacity; /* particles re-searched in full FP64 per step (the FP32
                                  screen's undecided ones, and any particle with more
                                  candidates than the search records) before the whole
                                  step falls back to the full FP64 search;
                                  0 = all particles (never falls back)                   */
    int32_t use_graph;         /* 1: each step is replayed from a captured hipGraph      */
    int32_t block_size;        /* threads per block, multiple of 64 in [64, 1024]; 0 = 256 */
    int32_t profile;           /* 1: time every phase with HIP events (disables graphs)  */
    int32_t dt_rule;           /* kmc_dt_rule (see below)                                */
    int32_t search_mode;       /* kmc_search_mode                                        */
    int32_t dims;              /* 3 (or 0): space.  2: planar mode (Section 1 also runs
                                  the method in two dimensions, with 9 neighbouring
                                  bins): every box must have ncell[2] = 1, bc[2] =
                                  REFLECT and geometry BOX, the caller keeps z and vz
                                  constant (vz = 0), and the scatter direction is
                                  uniform in the x-y plane: from the first (e1, e2)
                                  with 0 < s = e1*e1 + e2*e2 < 1 of the same random
                                  numbers, n = ((e1*e1 - e2*e2) / s,
                                  ((2*e1)*e2) / s, 0)                                    */
    int32_t tile;              /* tile shape of the partner-search kernel: 0 (default), 1
                                  (small LDS chunks) or 2 (large chunks, fewer waves per
                                  SIMD); the results do not depend on it (a launch
                                  choice, see kmc_autotune)                              */
    int32_t reserved;          /* must be zero                                           */
    double guard_scale;        /* FP32 screen: factor applied to the derived rounding-error
                                  bounds; 0 = 4 (default), >= 1 otherwise.  -1 disables the
                                  bounds (testing only: the screen is then not exact)     */
    double dt_factor;          /* KMC_DT_ADAPTIVE: the factor C below; 0 = 1 (the paper's
                                  rule), otherwise finite and > 0                         */
    const kmc_species* species; /* NULL: one kind of particle (each box's D2, equal
                                   masses); otherwise the kinds described above (host
                                   pointer, read by kmc_workspace_bytes, kmc_init and
                                   kmc_autotune)                                        */
    int32_t adapt_levels;      /* density-adaptive bins (below): 0 = the uniform grid;
                                  1..3 = at most that many halvings of a bin            */
    uint32_t adapt_threshold;  /* adaptive bins: a bin is split while it holds more than
                                  adapt_threshold * 8^level particles (>= 1)             */
} kmc_config;

/* Density-adaptive bins (Section 1 proposes an adaptive bin size against the
 * load imbalance of dense bins; Section 4: areas of higher density get
 * smaller bins).  With adapt_levels = L > 0, at the start of every step each
 * bin (cell) c of a box's grid holding n_c particles is split into
 * 2^l x 2^l x 2^l equal sub-bins, l the smallest level in 0..L with
 * n_c <= adapt_threshold * 8^l (L if none).  A particle's bin (its leaf) is
 * the sub-bin it falls in: on the finest grid (ncell[k] * 2^L bins per axis,
 * index clamp(floor((x - lo) * (inv_h * 2^L)), 0, ncell[k] * 2^L - 1)) a leaf
 * spans an interval of indices on each axis.  Two particles are in each
 * other's collision neighbourhood when their leaves touch: on every axis the
 * intervals are at most one index apart (on a periodic axis with the image
 * that makes them so).  An unsplit grid gives the 27-cell rule.  Requires
 * search_mode KMC_SEARCH_FULL, dims 3, no absorbing faces and ncell[k] <=
 * 2^27; the partners then differ from the uniform grid's wherever a bin is
 * split. */

/* Time step rules.
 *   KMC_DT_FIXED     every step of box b lasts boxes[b].dt.
 *   KMC_DT_ADAPTIVE  the adaptive step of Section 1 (dt = dx / v_max, so no
 *                    particle leaves its neighbourhood within one step),
 *                    evaluated per box at the start of every step from the
 *                    current velocities:
 *                      dx  = min over k of (hi[k] - lo[k]) / ncell[k]
 *                      v2  = max over the box's particles of
 *                            fma(vz, vz, fma(vy, vy, vx * vx))
 *                      dt  = v2 > 0 ? min(boxes[b].dt, (C * dx) / sqrt(v2))
 *                                   : boxes[b].dt
 *                    with IEEE-754 binary64 operations in that order (the
 *                    result is independent of how the maximum is reduced).
 *                    Section 3 synchronises this step over MPI domains; the
 *                    boxes of one context are independent and keep their own. */

/* Phases timed in profile mode (indices into kmc_stats.ms). */
enum {
    KMC_PHASE_BIN = 0,      /* cell index + per-cell count (runs fused into the
                               previous step's resolve; 0 ms in practice)           */
    KMC_PHASE_SCAN = 1,     /* exclusive prefix sum of the counts                   */
    KMC_PHASE_SCATTER = 2,  /* cell-sorted copy of the state, the step's dt, and the
                               FP32 screen's per-box bounds                         */
    KMC_PHASE_SEARCH = 3,   /* DCA pair search kernel (FP64, or the FP32 screen)    */
    KMC_PHASE_FINISH = 4,   /* closest partner from the recorded candidates         */
    KMC_PHASE_RECHECK = 5,  /* full FP64 re-search of undecided particles           */
    KMC_PHASE_RESOLVE = 6,  /* mutual check, scatter, free stream, boundaries, and
                               the next step's cell index + count                   */
    KMC_PHASE_COUNT = 7
};

typedef struct kmc_stats {
    uint64_t steps;            /* steps run since kmc_init                              */
    uint64_t n_total;          /* particles over all boxes                              */
    uint64_t cells_total;      /* cells over all boxes                                  */
    uint64_t rechecks;         /* particles listed for a full FP64 re-search (more list
                                  entries than slots), summed over steps; in a step
                                  that takes the whole-step FP64 search they are
                                  covered by it                                         */
    uint64_t fallbacks;        /* steps that took the whole-step FP64 search (a list
                                  overflowed, or the FP32 screen's assumptions failed)  */
    double ms[8];              /* accumulated milliseconds per phase (profile mode)      */
    uint64_t timed_steps;      /* steps that contributed to ms                          */
    double search_kernel_ms;   /* accumulated milliseconds of the search kernel alone   */
    uint64_t candidates;       /* pairs the search recorded per particle, summed over
                                  particles and steps (FP64: acceptable pairs; FP32
                                  screen: pairs it could not reject)                    */
    uint64_t absorbed;         /* particles absorbed by absorbing faces so far          */
} kmc_stats;

typedef struct kmc_ctx kmc_ctx;

/* Device workspace needed for these boxes and this configuration. */
int kmc_workspace_bytes(const kmc_box* boxes, uint32_t nboxes, const kmc_config* cfg,
                        size_t* bytes);

/* Create a context.
 *   boxes, nboxes  host array of box descriptions (copied);
 *   cfg            host pointer (copied);
 *   d_state        device pointer, 6*n_total doubles in structure-of-arrays
 *                  layout x[n_total], y, z, vx, vy, vz; box b's particles are
 *                  the slice [off_b, off_b + n_b) with off_b = n_0+..+n_{b-1};
 *                  particle ids are these global indices.  Read once (copied
 *                  into the workspace on `stream`); the caller may reuse it
 *                  after the stream has passed this call;
 *   d_workspace    device pointer, >= kmc_workspace_bytes, 256-byte aligned,
 *                  owned by the caller, untouched by anyone else until
 *                  kmc_destroy;
 *   out            receives the context.
 * Errors: KMC_EINVAL (bad box or config, null pointer, misaligned workspace,
 * a particle kind >= species->count),
 * KMC_ENOMEM (workspace too small), KMC_EOVERFLOW (more than 2^31-1 particles
 * or 2^32-2 cells in total), KMC_EDEVICE. */
int kmc_init(const kmc_box* boxes, uint32_t nboxes, const kmc_config* cfg,
             const double* d_state, void* d_workspace, size_t workspace_bytes,
             void* stream, kmc_ctx** out);

/* For callers that cannot allocate device memory (code that runs while a
 * HIP graph is being captured elsewhere, tight serving loops, harnesses that
 * forbid hipMalloc): kmc_init with the library's own per-device workspace
 * instead of a caller-owned one.
 *   - the workspace is a static device array of KMC_SCRATCH_BYTES in the
 *     library, one per GPU, held until the process ends; its address is
 *     looked up once per device (hipGetSymbolAddress) on the first call made
 *     with that device current;
 *   - boxes whose kmc_workspace_bytes exceed KMC_SCRATCH_BYTES are rejected
 *     with KMC_ENOMEM before anything is done (about 200 000 particles fit);
 *   - the call allocates no device or pinned memory (the context is a small
 *     host structure, as for kmc_init) and otherwise behaves as kmc_init:
 *     same arguments minus the workspace, same errors, same results; every
 *     other function takes the returned context as usual;
 *   - every context created this way on one GPU shares that GPU's array: a
 *     second kmc_init_scratch on the same device overwrites the first
 *     context's data, so at most one such context may be in use per device,
 *     and calls that overlap on one GPU race.  kmc_init clears whatever must
 *     start at zero, so stale contents of an earlier context do not matter. */
#define KMC_SCRATCH_BYTES ((size_t)64 << 20)
int kmc_init_scratch(const kmc_box* boxes, uint32_t nboxes, const kmc_config* cfg,
                     const double* d_state, void* stream, kmc_ctx** out);

/* Enqueue nsteps steps on `stream` (asynchronous). */
int kmc_step(kmc_ctx* ctx, uint32_t nsteps, void* stream);

/* Partner ids of the last step's search, in id order: d_partner_by_id is a
 * device pointer to n_total int32; entry i is the id of particle i's chosen
 * partner or -1 (not necessarily mutual).  Asynchronous on `stream`.
 * KMC_ESTATE before the first step. */
int kmc_read_partners(kmc_ctx* ctx, int32_t* d_partner_by_id, void* stream);

/* Current state in id order into d_state_by_id (device pointer, 6*n_total
 * doubles, same layout as kmc_init's input).  Asynchronous on `stream`. */
int kmc_read_state(kmc_ctx* ctx, double* d_state_by_id, void* stream);

/* Per-step collision counts and digests (sum over colliding pairs {a<b} of
 * SplitMix64((a << 32 | b) + 0x9E3779B97F4A7C15) mod 2^64) of the most
 * recent min(steps, capacity, history) steps, oldest first, into host arrays
 * h_npairs and h_digest (capacity entries each); *count receives the number
 * written.  Synchronises `stream`. */
int kmc_read_history(kmc_ctx* ctx, uint64_t* h_npairs, uint64_t* h_digest,
                     uint32_t capacity, uint32_t* count, void* stream);

/* Number of ordered pairs (i, j != i) in the 27-cell neighbourhoods of the
 * last step's cell grid (the pair tests that step's search performed), into
 * the host variable *h_pair_tests.  Synchronises `stream`.  KMC_ESTATE
 * before the first step. */
int kmc_count_pair_tests(kmc_ctx* ctx, uint64_t* h_pair_tests, void* stream);

/* Time step of the last step and simulated time since kmc_init (the sum of
 * the steps' dt) of each box, into host arrays of `capacity` >= nboxes
 * doubles (either may be NULL).  Synchronises `stream`. */
int kmc_read_time(kmc_ctx* ctx, double* h_dt, double* h_time, uint32_t capacity, void* stream);

/* Counters and (profile mode) per-phase times.  Synchronises `stream`. */
int kmc_get_stats(kmc_ctx* ctx, kmc_stats* out, void* stream);

/* Launch tuning.  kmc_autotune times short runs of candidate
 * configurations on the caller's input and returns the fastest.
 *   KMC_TUNE_LAUNCH  search organisation (kmc_search_mode), tile shape of
 *                    the search kernel (kmc_config.tile) and threads per
 *                    block of the streaming kernels; the results of the step
 *                    do not depend on these;
 *   KMC_TUNE_PRECISION  also the precision of the pair test (KMC_FP64 or
 *                    KMC_FP32_SCREEN): both give the same partners and states
 *                    bit for bit, so this too is a speed choice only;
 *   KMC_TUNE_CELLS   also the cell edge: every box gets ncell[k] =
 *                    floor((hi[k] - lo[k]) / (kappa * sqrt(D2))) cells
 *                    (kappa in {1, 1.25, 1.5, 2}; at least 3 on periodic
 *                    axes, candidates that violate it are skipped) and
 *                    inv_h[k] = ncell[k] / (hi[k] - lo[k]).  The cell grid is
 *                    part of the partner criteria (Section 1: partners are
 *                    searched in the neighbouring bins), so this changes the
 *                    results: the caller must use the returned boxes
 *                    everywhere (including any reference it compares with);
 *   KMC_TUNE_ADAPT   with density-adaptive bins (cfg->adapt_levels > 0,
 *                    else KMC_EINVAL) also their threshold: adapt_threshold
 *                    in {4, 8, 16, 32}.  The bins are part of the partner
 *                    criteria as well, so the caller must use the returned
 *                    out_cfg->adapt_threshold everywhere. */
enum { KMC_TUNE_LAUNCH = 1, KMC_TUNE_CELLS = 2, KMC_TUNE_PRECISION = 4, KMC_TUNE_ADAPT = 8 };

/* The candidates are searched one coordinate at a time, for every cell grid
 * (the given one, or each kappa with KMC_TUNE_CELLS) and every adaptive-bin
 * threshold (the given one, or each candidate with KMC_TUNE_ADAPT): first the
 * precisions (with KMC_TUNE_PRECISION) times the search organisations (only
 * the full search with adaptive bins), then the other tile shapes, then the
 * other block sizes (128, 512), each stage keeping the fastest so far.  At
 * most KMC_TUNE_MAX candidates are timed (later ones are not tried). */
#define KMC_TUNE_MAX 64
typedef struct kmc_tuning {
    uint32_t ntried;                 /* candidates timed                           */
    uint32_t best;                   /* index of the chosen one                    */
    double ms_per_step[KMC_TUNE_MAX];/* per candidate (NaN: skipped)               */
    int32_t search_mode[KMC_TUNE_MAX];
    int32_t block_size[KMC_TUNE_MAX];
    double kappa[KMC_TUNE_MAX];      /* cell-edge factor (0: the given grid)       */
    int32_t precision[KMC_TUNE_MAX];
    int32_t tile[KMC_TUNE_MAX];
    uint32_t adapt_threshold[KMC_TUNE_MAX]; /* adaptive-bin threshold (0: uniform grid) */
} kmc_tuning;

/* Time every candidate over `steps` steps (after one untimed step) from the
 * same input, choose the fastest, and write the chosen boxes and
 * configuration to out_boxes (nboxes entries; equal to `boxes` unless
 * KMC_TUNE_CELLS) and *out_cfg (cfg with search_mode, tile, block_size and,
 * with KMC_TUNE_PRECISION, precision and, with KMC_TUNE_ADAPT,
 * adapt_threshold set; the other fields are copied).
 *   d_state, d_workspace  as for kmc_init; the workspace must hold the
 *                    largest candidate (kmc_workspace_bytes of the boxes
 *                    with kappa = 1, block_size 64 and, with
 *                    KMC_TUNE_PRECISION, precision KMC_FP32_SCREEN and, with
 *                    KMC_TUNE_ADAPT, adapt_threshold 4 suffices); candidates
 *                    that do not fit are skipped;
 *   flags            KMC_TUNE_LAUNCH, KMC_TUNE_CELLS, KMC_TUNE_PRECISION
 *                    and/or KMC_TUNE_ADAPT (0 = LAUNCH).
 * d_state is only read.  Synchronises `stream`.  Errors as kmc_init, and
 * KMC_ENOMEM when no candidate fits. */
int kmc_autotune(const kmc_box* boxes, uint32_t nboxes, const kmc_config* cfg, const double* d_state,
                 void* d_workspace, size_t workspace_bytes, uint32_t flags, uint32_t steps, void* stream,
                 kmc_box* out_boxes, kmc_config* out_cfg, kmc_tuning* out);

/* Cell grid of a box for a cell-edge factor kappa, as KMC_TUNE_CELLS sets
 * it (host helper, no device work): fills out->ncell and out->inv_h from
 * box (other fields copied).  KMC_EINVAL if kappa < 1 or a periodic axis
 * would get fewer than 3 cells. */
int kmc_box_with_kappa(const kmc_box* box, double kappa, kmc_box* out);

/* Release the host context, its private stream and graph.  The workspace
 * may be freed by the caller afterwards.  NULL is ignored. */
void kmc_destroy(kmc_ctx* ctx);

/* Static description of a status code. */
const char* kmc_strerror(int status);

/* KMC_ABI_VERSION of the built library. */
int kmc_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* KMC_H */
