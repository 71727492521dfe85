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
 *      D = sqrt(sigma/pi); the closest acceptable partner wins, equal
 *      distances going to the smaller id;
 *   3. two particles collide only if each chose the other;
 *   4. a colliding pair moves to t*, scatters elastically and isotropically
 *      in its centre-of-mass frame (direction from Philox4x64-10 keyed by
 *      the seed, the step and the pair's smaller id), and moves on with the
 *      new velocities for dt - t*; everybody else streams freely for dt;
 *   5. boundary conditions: periodic or reflecting box faces (Section 1
 *      names reflective, absorptive and periodic boxes) or a reflecting
 *      sphere.
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
 *     the captured graph, all released by kmc_destroy.
 */
#ifndef KMC_H
#define KMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KMC_ABI_VERSION 1

typedef enum {
    KMC_OK = 0,
    KMC_EINVAL = -1,     /* invalid argument (nothing was done)                    */
    KMC_ENOMEM = -2,     /* workspace too small, or host allocation failed          */
    KMC_EDEVICE = -3,    /* a HIP runtime call failed                               */
    KMC_EOVERFLOW = -4,  /* a size exceeds the library's index range                */
    KMC_ESTATE = -5      /* call not valid in the context's current state          */
} kmc_status;

typedef enum { KMC_FP64 = 0, KMC_FP32_SCREEN = 1 } kmc_precision;
typedef enum { KMC_GEOM_BOX = 0, KMC_GEOM_SPHERE = 1 } kmc_geometry;
typedef enum { KMC_BC_REFLECT = 0, KMC_BC_PERIODIC = 1 } kmc_bc;
typedef enum { KMC_KIN_AT_TSTAR = 0, KMC_KIN_VEL_ONLY = 1 } kmc_kinematics;

/* One independent simulation box.
 *   n         particles in the box (their state is a contiguous slice of the
 *             caller's state, boxes in order);
 *   geometry  KMC_GEOM_BOX: faces at lo/hi with per-axis bc;
 *             KMC_GEOM_SPHERE: reflecting sphere of radius sphere_r about the
 *             origin inside the cell grid lo..hi (bc must be REFLECT);
 *   bc[k]     KMC_BC_PERIODIC or KMC_BC_REFLECT for axis k;
 *   ncell[k]  cells (bins) along axis k; >= 1, and >= 3 on periodic axes;
 *   lo, hi    grid (and box) bounds, hi > lo;
 *   inv_h[k]  ncell[k] / (hi[k] - lo[k]) as computed by the caller (the
 *             cell of x is clamp(floor((x - lo) * inv_h), 0, ncell - 1));
 *             the cell edge 1/inv_h must be >= sqrt(D2) on every axis;
 *   D2        squared interaction diameter sigma/pi (> 0);
 *   dt        time step (> 0).
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
    int32_t reserved[5];       /* must be zero                                           */
    double guard_scale;        /* FP32 screen: factor applied to the derived rounding-error
                                  bounds; 0 = 4 (default), >= 1 otherwise.  -1 disables the
                                  bounds (testing only: the screen is then not exact)     */
} kmc_config;

/* Phases timed in profile mode (indices into kmc_stats.ms). */
enum {
    KMC_PHASE_BIN = 0,      /* cell index + per-cell count (runs fused into the
                               previous step's resolve; 0 ms in practice)           */
    KMC_PHASE_SCAN = 1,     /* exclusive prefix sum of the counts                   */
    KMC_PHASE_SCATTER = 2,  /* cell-sorted copy of the state                        */
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
    uint64_t rechecks;         /* particles re-searched in full FP64 (sum over steps)   */
    uint64_t fallbacks;        /* steps whose recheck list overflowed                   */
    double ms[8];              /* accumulated milliseconds per phase (profile mode)      */
    uint64_t timed_steps;      /* steps that contributed to ms                          */
    double search_kernel_ms;   /* accumulated milliseconds of the search kernel alone   */
    uint64_t candidates;       /* pairs the search recorded per particle, summed over
                                  particles and steps (FP64: acceptable pairs; FP32
                                  screen: pairs it could not reject)                    */
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
 * Errors: KMC_EINVAL (bad box or config, null pointer, misaligned workspace),
 * KMC_ENOMEM (workspace too small), KMC_EOVERFLOW (more than 2^31-1 particles
 * or 2^32-2 cells in total), KMC_EDEVICE. */
int kmc_init(const kmc_box* boxes, uint32_t nboxes, const kmc_config* cfg,
             const double* d_state, void* d_workspace, size_t workspace_bytes,
             void* stream, kmc_ctx** out);

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

/* Counters and (profile mode) per-phase times.  Synchronises `stream`. */
int kmc_get_stats(kmc_ctx* ctx, kmc_stats* out, void* stream);

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
