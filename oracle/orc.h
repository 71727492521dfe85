/*
 * orc.h -- CPU oracle for one time step of the distance-of-closest-approach
 * (DCA) kinetic Monte-Carlo collision step of Howell et al., "Parallelization
 * of Kinetic Theory Simulations" (arXiv:1310.3437).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, deliberately obvious
 * FP64 implementation used to check the GPU library.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header, table or constant with the GPU library.
 *
 * Paper passages followed (Section 1, "Initial Simulation Setup", unless
 * noted):
 *   - uniform grid of bins, one list of particles per bin, bin counts and
 *     box size set by the user;
 *   - each particle compares itself with the particles of its own bin and of
 *     the 26 neighbouring bins;
 *   - partner criteria: inside each other's collision neighbourhood, within
 *     the effective radii (distance of closest approach), and closest
 *     approach reached within the next time step;
 *   - the partner pointer is replaced whenever a closer partner is found;
 *   - two particles collide only if each found the other; positions and
 *     velocities are then updated and the box boundary conditions applied
 *     (reflective or periodic; the paper also names absorptive).
 * Where the paper is silent (the ordering key, the tie-break, the collision
 * kinematics, the random numbers, the rounding) the readings are the ones
 * listed next to each function below.
 *
 * State layout: one array of 6*n doubles, structure of arrays,
 *   s[0n..1n) = x, s[1n..2n) = y, s[2n..3n) = z,
 *   s[3n..4n) = vx, s[4n..5n) = vy, s[5n..6n) = vz.
 * Particle identities are given by a separate uint32 array ids[n].
 *
 * All functions return 0 on success and a negative value on invalid input.
 */
#ifndef ORC_H
#define ORC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int64_t  n;            /* particles in the box                              */
    int32_t  sphere;       /* 1: reflecting sphere |x| <= R about the origin     */
    int32_t  periodic[3];  /* per axis: 1 periodic, 0 reflecting planes lo/hi     */
    int32_t  ncell[3];     /* bins per axis                                     */
    int32_t  kinematics;   /* 0: scatter executed at t*, 1: velocity-only update */
    int32_t  dims;         /* 3 (or 0): space; 2: planar mode (one bin along z,
                              no periodic z, no sphere; isotropic scatter in the
                              x-y plane; z and vz stay as given)              */
    int32_t  absorb[3];    /* per axis: 1 absorbing faces lo/hi (not periodic,
                              no sphere): a particle whose streamed position
                              lies beyond them leaves the gas for good       */
    double   lo[3], hi[3]; /* box (and bin grid) bounds                         */
    double   inv_h[3];     /* ncell[k] / (hi[k] - lo[k]), supplied by the caller */
    double   R;            /* sphere radius (sphere == 1)                       */
    double   D2;           /* squared interaction diameter sigma/pi              */
    double   dt;           /* time step                                         */
    uint64_t seed;         /* Philox key word 0                                 */
    /* Kinds of particles (Section 1: every particle carries its own mass and
     * effective radius).  nspecies == 0: one kind, interaction diameter
     * sqrt(D2), equal masses.  1 <= nspecies <= 8: particle i is of kind
     * species[i]; a pair (s, t) is within each other's effective radii when
     * its distance of closest approach is below radius[s] + radius[t] (D2 is
     * then not used), and it scatters with masses mass[s], mass[t]. */
    int32_t  nspecies;
    int32_t  pad_;
    const uint8_t* species; /* n entries when nspecies > 0                     */
    const double*  radius;  /* nspecies entries, > 0                           */
    const double*  mass;    /* nspecies entries, > 0                           */
    /* Density-adaptive bins (Section 1 proposes an adaptive bin size against
     * the load imbalance of dense bins; Section 4: areas of higher density
     * get smaller bins).  adapt_levels == 0: the uniform grid above.
     * 1 <= adapt_levels <= 3: at the start of the step each bin c of the grid
     * holding n_c particles is split into 2^l x 2^l x 2^l equal sub-bins,
     * l the smallest level in 0..adapt_levels with n_c <= adapt_threshold *
     * 8^l (adapt_levels if none).  A particle's bin (its leaf) is the sub-bin
     * it falls in; on the finest grid (ncell[k] * 2^adapt_levels bins per
     * axis, index clamp(floor((x - lo) * (inv_h * 2^adapt_levels)), 0, ..))
     * a leaf spans an interval of finest indices per axis.  Two particles
     * are in each other's collision neighbourhood when their leaves touch
     * (their closed boxes intersect: on every axis the index intervals are at
     * most one apart, across the seam of a periodic axis with the image that
     * makes them so, which is unique with >= 3 bins per periodic axis).  On a
     * uniform grid (no bin split) this is the 27-bin rule. */
    int32_t  adapt_levels;
    int32_t  adapt_threshold;
} orc_box;

/* Quantities of one ordered pair (searcher i, candidate j). */
typedef struct {
    double r[3], g[3];     /* relative position (with periodic image) and velocity */
    double b, g2, c2;      /* r.g, |g|^2, |r x g|^2                              */
    double key;            /* c2/g2 when accepted, else +inf                     */
    int32_t acc;           /* 1 if j is an acceptable partner of i               */
} orc_pair_q;

/* Bin coordinates of a point (clamped to the grid). */
int orc_cell_coords(const orc_box* b, double x, double y, double z, int32_t c[3]);

/* Pair quantities for searcher state pi[6] and candidate state pj[6], with the
 * periodic image selector wrap[k] in {-1,0,1} (candidate shifted by wrap*L). */
int orc_pair(const orc_box* b, const double pi[6], const double pj[6],
             const int32_t wrap[3], orc_pair_q* out);

/* Cell-list partner search: partner[i] = index of i's partner or -1.
 * pair_tests (optional) receives the number of ordered (i, j != i) pairs
 * examined.  nthreads <= 0 means the OpenMP default. */
int orc_find_partners(const orc_box* b, const double* s, const uint32_t* ids,
                      int32_t* partner, int nthreads, uint64_t* pair_tests);

/* The same search by brute force over all ordered pairs, with neighbourhood
 * decided by an explicit test on bin coordinates. */
int orc_find_partners_bruteforce(const orc_box* b, const double* s,
                                 const uint32_t* ids, int32_t* partner);

/* Philox4x64-10 block function (Salmon, Moraes, Dror and Shaw, SC'11). */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Isotropic unit vector for the pair whose smaller id is a, at step `step`. */
void orc_direction(uint64_t seed, uint64_t step, uint32_t a, double n[3]);

/* Planar variant: uniformly distributed unit vector in the x-y plane. */
void orc_direction2(uint64_t seed, uint64_t step, uint32_t a, double n[3]);

/* 64-bit hash of an unordered pair (a < b), used for the per-step digest. */
uint64_t orc_pair_hash(uint32_t a, uint32_t b);

/* One full step with absorbing faces: gone[i] != 0 marks a particle that
 * has left the gas (it is in no bin, never searches or collides, and its
 * state stays as it was); particles absorbed during this step get gone[i] = 1.
 * gone may be NULL (no particle has left and none is absorbed).  Otherwise as
 * orc_step. */
int orc_step_ex(const orc_box* b, double* s, const uint32_t* ids, unsigned char* gone, uint64_t step,
                int32_t* partner, uint64_t* npairs, uint64_t* digest,
                int nthreads, uint64_t* pair_tests);

/* One full step in place: search, mutual resolve, scatter, free-stream,
 * boundary conditions.  partner (optional, n entries) receives the search
 * result (array indices); npairs/digest receive the collision count and the
 * sum of orc_pair_hash over colliding pairs (mod 2^64). */
int orc_step(const orc_box* b, double* s, const uint32_t* ids, uint64_t step,
             int32_t* partner, uint64_t* npairs, uint64_t* digest,
             int nthreads, uint64_t* pair_tests);

/* The step of orc_step evaluated at selected particles only (checks of runs
 * too large for a full oracle step): for k < nsel, partner_out[k] receives
 * the partner (index or -1) of particle sel[k] and state_out[6k .. 6k+6) its
 * x, y, z, vx, vy, vz after the step.  s is not modified. */
int orc_step_sampled(const orc_box* b, const double* s, const uint32_t* ids, uint64_t step,
                     const int64_t* sel, int64_t nsel, int32_t* partner_out,
                     double* state_out, int nthreads);

/* Adaptive time step of Section 1 (dt = dx / v_max: no particle can leave
 * its neighbourhood within one step), scaled by `factor` and capped by
 * b->dt: with dx the smallest bin width and v_max the largest particle
 * speed in s, *dt = min(b->dt, factor * dx / v_max), or b->dt when every
 * particle is at rest. */
int orc_adaptive_dt(const orc_box* b, const double* s, double factor, double* dt);

/* The same over the particles still in the gas (gone[i] == 0; gone may be
 * NULL). */
int orc_adaptive_dt_ex(const orc_box* b, const double* s, const unsigned char* gone, double factor,
                       double* dt);

/* Ordered pairs (i, j != i) examined and ordered pairs accepted by the
 * partner criteria in the current state, without choosing partners; used by
 * the collision-rate check. */
int orc_count_accepted(const orc_box* b, const double* s, const uint32_t* ids,
                       int nthreads, uint64_t* accepted, uint64_t* pair_tests);

/* Number of OpenMP threads the oracle would use for nthreads <= 0. */
int orc_max_threads(void);

#ifdef __cplusplus
}
#endif

#endif /* ORC_H */
