/*
 * orc.c -- CPU oracle for the DCA collision step (arXiv:1310.3437).
 *
 * TEST INFRASTRUCTURE ONLY: a plain, slow FP64 reference against which the
 * GPU library is checked.  Built with -ffp-contract=off so that the only
 * fused multiply-adds are the explicit fma() calls of the definition.
 *
 * The step follows Section 1 ("Initial Simulation Setup") of the paper:
 * bin the particles, let every particle search its own and the 26
 * neighbouring bins for its closest acceptable partner, let a pair collide
 * only if both chose each other, update positions and velocities, apply the
 * boundary conditions.  The readings taken where the paper is silent are
 * stated at each function.
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Parameter checks                                                          */
/* ------------------------------------------------------------------------ */

static int box_ok(const orc_box* b)
{
    if (!b || b->n < 0) return 0;
    if (!(b->dt > 0.0) || !(b->D2 > 0.0)) return 0;
    for (int k = 0; k < 3; ++k) {
        if (b->ncell[k] < 1) return 0;
        if (!(b->hi[k] > b->lo[k]) || !(b->inv_h[k] > 0.0)) return 0;
        /* a periodic axis needs three distinct bins in every stencil row */
        if (b->periodic[k] && b->ncell[k] < 3) return 0;
        if (b->sphere && b->periodic[k]) return 0;
    }
    if (b->sphere && !(b->R > 0.0)) return 0;
    if (b->dims != 0 && b->dims != 2 && b->dims != 3) return 0;
    if (b->dims == 2 && (b->ncell[2] != 1 || b->periodic[2] || b->sphere)) return 0;
    for (int k = 0; k < 3; ++k)
        if (b->absorb[k] && (b->periodic[k] || b->sphere)) return 0;
    if (b->nspecies < 0 || b->nspecies > 8) return 0;
    if (b->adapt_levels < 0 || b->adapt_levels > 3 || b->adapt_threshold < 0) return 0;
    if (b->adapt_levels > 0) {
        if (b->dims == 2) return 0;   /* bins are split in all three axes */
        for (int k = 0; k < 3; ++k)
            if (b->ncell[k] > (1 << 27)) return 0;   /* finest index fits int32 */
    }
    if (b->nspecies > 0) {
        if (!b->radius || !b->mass || (b->n > 0 && !b->species)) return 0;
        for (int s = 0; s < b->nspecies; ++s)
            if (!(b->radius[s] > 0.0) || !(b->mass[s] > 0.0) || isinf(b->radius[s]) || isinf(b->mass[s]))
                return 0;
        for (int64_t i = 0; i < b->n; ++i)
            if (b->species[i] >= b->nspecies) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Bins (Section 1: a grid of bins whose counts and extent the user sets)    */
/* ------------------------------------------------------------------------ */

/* Bin index along one axis: floor((x - lo) * inv_h), clamped to the grid.
 * The clamp is the reading for points on or beyond the upper face. */
static int32_t bin1(double x, double lo, double inv_h, int32_t n)
{
    double f = floor((x - lo) * inv_h);
    if (!(f >= 0.0)) return 0;
    if (f >= (double)n) return n - 1;
    return (int32_t)f;
}

int orc_cell_coords(const orc_box* b, double x, double y, double z, int32_t c[3])
{
    if (!b || !c) return -1;
    c[0] = bin1(x, b->lo[0], b->inv_h[0], b->ncell[0]);
    c[1] = bin1(y, b->lo[1], b->inv_h[1], b->ncell[1]);
    c[2] = bin1(z, b->lo[2], b->inv_h[2], b->ncell[2]);
    return 0;
}

static int64_t linear_cell(const orc_box* b, const int32_t c[3])
{
    return (int64_t)c[0] + (int64_t)b->ncell[0] * ((int64_t)c[1] + (int64_t)b->ncell[1] * (int64_t)c[2]);
}

/* ------------------------------------------------------------------------ */
/* Partner criteria (Section 1, the three bullet criteria)                   */
/* ------------------------------------------------------------------------ */

/* Quantities of the pair (i searching, j candidate).
 *   r = x_j - x_i (+ wrap*L on a periodic axis whose neighbour bin wrapped),
 *   g = v_j - v_i,
 *   b = r.g, g2 = |g|^2, c = r x g, c2 = |c|^2, each with the fixed fma order
 *   below (the only fused operations of the definition).
 * Closest approach of the straight relative path r + g t is at
 * t* = -b/g2 with squared distance d_min^2 = c2/g2.  The criteria that the
 * closest approach falls within the next step (0 <= t* <= dt) and inside the
 * effective radii (d_min^2 < D2 = sigma/pi) are evaluated multiplied through
 * by g2 > 0:  b <= 0, -b <= dt*g2, c2 < D2*g2.
 * The ordering key of an acceptable candidate is d_min^2 = c2/g2. */
static void pair_q(const orc_box* b, const double pi[6], const double pj[6], const int32_t wrap[3], double D2,
                   orc_pair_q* q)
{
    for (int k = 0; k < 3; ++k) {
        double r = pj[k] - pi[k];
        if (wrap[k] != 0) r = r + (double)wrap[k] * (b->hi[k] - b->lo[k]);
        q->r[k] = r;
        q->g[k] = pj[3 + k] - pi[3 + k];
    }
    const double* r = q->r;
    const double* g = q->g;
    q->b  = fma(r[2], g[2], fma(r[1], g[1], r[0] * g[0]));
    q->g2 = fma(g[2], g[2], fma(g[1], g[1], g[0] * g[0]));
    double cx = fma(r[1], g[2], -(r[2] * g[1]));
    double cy = fma(r[2], g[0], -(r[0] * g[2]));
    double cz = fma(r[0], g[1], -(r[1] * g[0]));
    q->c2 = fma(cz, cz, fma(cy, cy, cx * cx));
    q->acc = (q->g2 > 0.0) && (q->b <= 0.0) && (-q->b <= b->dt * q->g2) &&
             (q->c2 < D2 * q->g2);
    q->key = q->acc ? q->c2 / q->g2 : INFINITY;
}

int orc_pair(const orc_box* b, const double pi[6], const double pj[6],
             const int32_t wrap[3], orc_pair_q* q)
{
    if (!b || !pi || !pj || !wrap || !q) return -1;
    pair_q(b, pi, pj, wrap, b->D2, q);
    return 0;
}

/* Squared interaction diameter of the pair (i, j): D2 for one kind of
 * particle, else the square of the sum of the two effective radii (hard
 * spheres touch when their centres are that far apart). */
static double pair_D2(const orc_box* b, int64_t i, int64_t j)
{
    if (b->nspecies == 0) return b->D2;
    const double d = b->radius[b->species[i]] + b->radius[b->species[j]];
    return d * d;
}

static void load6(const double* s, int64_t n, int64_t i, double p[6])
{
    for (int k = 0; k < 6; ++k) p[k] = s[(int64_t)k * n + i];
}

/* "Closer" partner: smaller key; equal keys go to the smaller id. */
static int better(double key, uint32_t id, double best_key, uint32_t best_id)
{
    return key < best_key || (key == best_key && id < best_id);
}

/* ------------------------------------------------------------------------ */
/* Cell-list search (Section 1: loop over bins, compare with the particles   */
/* of the 27-bin neighbourhood, keep the closest partner found so far)       */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t ncells;
    int64_t* start;   /* ncells + 1 */
    int64_t* member;  /* n: particle indices grouped by bin, index order within a bin */
    /* adaptive bins only (NULL otherwise) */
    int8_t* level;    /* ncells: refinement level of each bin this step */
    int32_t* fine;    /* 3n: each particle's index on the finest grid */
} csr_t;

/* Adaptive bins: index of a point on the finest grid along one axis,
 * clamp(floor((x - lo) * (inv_h * 2^L)), 0, n 2^L - 1).  inv_h * 2^L is exact,
 * and so the bin of the uniform grid is this index >> L (the power-of-two
 * scaling commutes with the rounding of the product). */
static int32_t fine1(double x, double lo, double inv_h, int32_t n, int L)
{
    double f = floor((x - lo) * (inv_h * (double)(1 << L)));
    if (!(f >= 0.0)) return 0;
    double m = (double)n * (double)(1 << L);
    if (f >= m) return (int32_t)(m - 1.0);
    return (int32_t)f;
}

/* Refinement level of a bin holding `count` particles: the smallest l in
 * 0..L with count <= threshold * 8^l, else L. */
static int8_t bin_level(int64_t count, int32_t threshold, int L)
{
    for (int l = 0; l < L; ++l)
        if (count <= (int64_t)threshold << (3 * l)) return (int8_t)l;
    return (int8_t)L;
}

static int build_csr(const orc_box* b, const double* s, const unsigned char* gone, csr_t* t)
{
    int64_t n = b->n;
    t->level = NULL;
    t->fine = NULL;
    t->ncells = (int64_t)b->ncell[0] * b->ncell[1] * b->ncell[2];
    t->start = (int64_t*)calloc((size_t)t->ncells + 1, sizeof(int64_t));
    t->member = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t* cellof = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!t->start || !t->member || !cellof) {
        free(t->start); free(t->member); free(cellof);
        return -1;
    }
    const int L = b->adapt_levels;
    if (L > 0) {
        t->fine = (int32_t*)malloc((size_t)(n > 0 ? 3 * n : 1) * sizeof(int32_t));
        t->level = (int8_t*)malloc((size_t)t->ncells + 1);
        if (!t->fine || !t->level) {
            free(t->start); free(t->member); free(cellof); free(t->fine); free(t->level);
            return -1;
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        if (gone && gone[i]) { cellof[i] = -1; continue; }   /* in no bin */
        int32_t c[3];
        orc_cell_coords(b, s[i], s[n + i], s[2 * n + i], c);
        if (L > 0)
            for (int k = 0; k < 3; ++k) t->fine[3 * i + k] = fine1(s[(int64_t)k * n + i], b->lo[k], b->inv_h[k],
                                                                  b->ncell[k], L);
        cellof[i] = linear_cell(b, c);
        t->start[cellof[i] + 1] += 1;
    }
    if (L > 0)
        for (int64_t c = 0; c < t->ncells; ++c) t->level[c] = bin_level(t->start[c + 1], b->adapt_threshold, L);
    for (int64_t c = 0; c < t->ncells; ++c) t->start[c + 1] += t->start[c];
    int64_t* fill = (int64_t*)malloc((size_t)t->ncells * sizeof(int64_t) + 1);
    if (!fill) {
        free(t->start); free(t->member); free(cellof);
        return -1;
    }
    memcpy(fill, t->start, (size_t)t->ncells * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i)
        if (cellof[i] >= 0) t->member[fill[cellof[i]]++] = i;
    free(fill);
    free(cellof);
    return 0;
}

static void free_csr(csr_t* t)
{
    free(t->start);
    free(t->member);
    free(t->level);
    free(t->fine);
}

/* Adaptive bins: the interval [lo, hi] of finest indices that particle i's
 * leaf spans on each axis. */
static void leaf_of(const orc_box* b, const csr_t* t, int64_t i, int32_t lo[3], int32_t hi[3])
{
    const int L = b->adapt_levels;
    int32_t c[3];
    for (int k = 0; k < 3; ++k) c[k] = t->fine[3 * i + k] >> L;
    const int sh = L - t->level[linear_cell(b, c)];
    for (int k = 0; k < 3; ++k) {
        lo[k] = (t->fine[3 * i + k] >> sh) << sh;
        hi[k] = lo[k] + (1 << sh) - 1;
    }
}

/* Do two leaves touch, the second seen with the periodic image wrap? */
static int leaves_touch(const orc_box* b, const int32_t alo[3], const int32_t ahi[3], const int32_t blo[3],
                        const int32_t bhi[3], const int32_t wrap[3])
{
    for (int k = 0; k < 3; ++k) {
        const int64_t M = (int64_t)b->ncell[k] << b->adapt_levels;
        const int64_t b0 = blo[k] + wrap[k] * M, b1 = bhi[k] + wrap[k] * M;
        if (b0 > (int64_t)ahi[k] + 1 || (int64_t)alo[k] > b1 + 1) return 0;
    }
    return 1;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Closest acceptable partner of particle i (index, or -1). */
static int64_t search_one(const orc_box* b, const double* s, const uint32_t* ids,
                          const csr_t* t, int64_t i, uint64_t* tests, uint64_t* acc_count)
{
    int64_t n = b->n;
    double pi[6], pj[6];
    load6(s, n, i, pi);
    int32_t c[3];
    orc_cell_coords(b, pi[0], pi[1], pi[2], c);
    double best_key = INFINITY;
    uint32_t best_id = UINT32_MAX;
    int64_t best = -1;
    /* adaptive bins: i's leaf; every leaf it touches lies in the 27 bins */
    int32_t alo[3] = {0, 0, 0}, ahi[3] = {0, 0, 0};
    if (t->level) leaf_of(b, t, i, alo, ahi);
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int32_t d[3] = {dx, dy, dz};
                int32_t nc[3], wrap[3];
                int inside = 1;
                for (int k = 0; k < 3; ++k) {
                    nc[k] = c[k] + d[k];
                    wrap[k] = 0;
                    if (nc[k] < 0) {
                        if (b->periodic[k]) { nc[k] += b->ncell[k]; wrap[k] = -1; }
                        else inside = 0;
                    } else if (nc[k] >= b->ncell[k]) {
                        if (b->periodic[k]) { nc[k] -= b->ncell[k]; wrap[k] = 1; }
                        else inside = 0;
                    }
                }
                if (!inside) continue;
                int64_t cell = linear_cell(b, nc);
                for (int64_t q = t->start[cell]; q < t->start[cell + 1]; ++q) {
                    int64_t j = t->member[q];
                    if (j == i) continue;
                    if (t->level) {
                        int32_t blo[3], bhi[3];
                        leaf_of(b, t, j, blo, bhi);
                        if (!leaves_touch(b, alo, ahi, blo, bhi, wrap)) continue;
                    }
                    ++*tests;
                    load6(s, n, j, pj);
                    orc_pair_q pq;
                    pair_q(b, pi, pj, wrap, pair_D2(b, i, j), &pq);
                    if (!pq.acc) continue;
                    ++*acc_count;
                    if (better(pq.key, ids[j], best_key, best_id)) {
                        best_key = pq.key;
                        best_id = ids[j];
                        best = j;
                    }
                }
            }
    return best;
}

static int64_t search_with_csr(const orc_box* b, const double* s, const uint32_t* ids,
                               const unsigned char* gone, const csr_t* t, int32_t* partner,
                               int nthreads, uint64_t* pair_tests, uint64_t* accepted)
{
    int64_t n = b->n;
    uint64_t tests = 0, acc_count = 0;
#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 512) num_threads(nt) reduction(+ : tests, acc_count)
#else
    (void)nthreads;
#endif
    for (int64_t i = 0; i < n; ++i) {
        uint64_t nt_i = 0, na_i = 0;
        if (gone && gone[i]) { partner[i] = -1; continue; }
        partner[i] = (int32_t)search_one(b, s, ids, t, i, &nt_i, &na_i);
        tests += nt_i;
        acc_count += na_i;
    }
    if (pair_tests) *pair_tests = tests;
    if (accepted) *accepted = acc_count;
    return 0;
}

int orc_find_partners(const orc_box* b, const double* s, const uint32_t* ids,
                      int32_t* partner, int nthreads, uint64_t* pair_tests)
{
    if (!box_ok(b) || (b->n > 0 && (!s || !ids || !partner))) return -1;
    if (b->n > INT32_MAX) return -1;
    csr_t t;
    if (build_csr(b, s, NULL, &t) != 0) return -2;
    search_with_csr(b, s, ids, NULL, &t, partner, nthreads, pair_tests, NULL);
    free_csr(&t);
    return 0;
}

/* Ordered accepted pairs in the current state (collision-rate check). */
int orc_count_accepted(const orc_box* b, const double* s, const uint32_t* ids,
                       int nthreads, uint64_t* accepted, uint64_t* pair_tests)
{
    if (!box_ok(b) || !accepted) return -1;
    int32_t* partner = (int32_t*)malloc((size_t)(b->n > 0 ? b->n : 1) * sizeof(int32_t));
    if (!partner) return -2;
    csr_t t;
    if (build_csr(b, s, NULL, &t) != 0) { free(partner); return -2; }
    search_with_csr(b, s, ids, NULL, &t, partner, nthreads, pair_tests, accepted);
    free_csr(&t);
    free(partner);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Brute force over all ordered pairs                                        */
/* ------------------------------------------------------------------------ */

/* Neighbourhood and image along one axis from the two bin indices:
 * adjacent if the bins differ by at most one, counting across the periodic
 * seam; the candidate's image is shifted by -L (+L) when it sits in the last
 * (first) bin and the searcher in the first (last). */
static int axis_adjacent(const orc_box* b, int k, int32_t ci, int32_t cj, int32_t* wrap)
{
    int32_t d = cj - ci;
    *wrap = 0;
    if (b->periodic[k]) {
        if (d == b->ncell[k] - 1) { *wrap = -1; return 1; }
        if (d == -(b->ncell[k] - 1)) { *wrap = 1; return 1; }
    }
    return d >= -1 && d <= 1;
}

/* Adaptive bins, by brute force: the leaf interval [lo, hi] of a point on
 * each axis, given the particle counts of every bin. */
static void bf_leaf(const orc_box* b, const int64_t* count, const double p[6], int32_t lo[3], int32_t hi[3])
{
    const int L = b->adapt_levels;
    int32_t g[3], c[3];
    for (int k = 0; k < 3; ++k) {
        g[k] = fine1(p[k], b->lo[k], b->inv_h[k], b->ncell[k], L);
        c[k] = g[k] >> L;
    }
    const int sh = L - bin_level(count[linear_cell(b, c)], b->adapt_threshold, L);
    for (int k = 0; k < 3; ++k) {
        lo[k] = (g[k] >> sh) << sh;
        hi[k] = lo[k] + (1 << sh) - 1;
    }
}

/* Two leaf intervals along axis k: do they touch (closed boxes intersect)?
 * On a periodic axis of M finest bins try the images -M, 0, +M of the
 * second; *wrap receives the one that touches. */
static int bf_axis_touch(const orc_box* b, int k, int32_t alo, int32_t ahi, int32_t blo, int32_t bhi, int32_t* wrap)
{
    const int64_t M = (int64_t)b->ncell[k] << b->adapt_levels;
    for (int w = -1; w <= 1; ++w) {
        if (w != 0 && !b->periodic[k]) continue;
        const int64_t b0 = blo + w * M, b1 = bhi + w * M;
        if (b0 <= (int64_t)ahi + 1 && (int64_t)alo <= b1 + 1) {
            *wrap = w;
            return 1;
        }
    }
    return 0;
}

int orc_find_partners_bruteforce(const orc_box* b, const double* s,
                                 const uint32_t* ids, int32_t* partner)
{
    if (!box_ok(b) || (b->n > 0 && (!s || !ids || !partner))) return -1;
    int64_t n = b->n;
    int64_t* count = NULL;
    if (b->adapt_levels > 0) {
        /* particles per bin of the uniform grid, counted directly */
        const int64_t nc = (int64_t)b->ncell[0] * b->ncell[1] * b->ncell[2];
        count = (int64_t*)calloc((size_t)nc, sizeof(int64_t));
        if (!count) return -2;
        for (int64_t i = 0; i < n; ++i) {
            int32_t c[3];
            orc_cell_coords(b, s[i], s[n + i], s[2 * n + i], c);
            count[linear_cell(b, c)] += 1;
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        double pi[6], pj[6];
        load6(s, n, i, pi);
        int32_t ci[3];
        orc_cell_coords(b, pi[0], pi[1], pi[2], ci);
        double best_key = INFINITY;
        uint32_t best_id = UINT32_MAX;
        int64_t best = -1;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            load6(s, n, j, pj);
            int32_t cj[3], wrap[3];
            orc_cell_coords(b, pj[0], pj[1], pj[2], cj);
            int adj = 1;
            if (count) {
                int32_t alo[3], ahi[3], blo[3], bhi[3];
                bf_leaf(b, count, pi, alo, ahi);
                bf_leaf(b, count, pj, blo, bhi);
                for (int k = 0; k < 3; ++k) adj &= bf_axis_touch(b, k, alo[k], ahi[k], blo[k], bhi[k], &wrap[k]);
            } else {
                for (int k = 0; k < 3; ++k) adj &= axis_adjacent(b, k, ci[k], cj[k], &wrap[k]);
            }
            if (!adj) continue;
            orc_pair_q pq;
            pair_q(b, pi, pj, wrap, pair_D2(b, i, j), &pq);
            if (pq.acc && better(pq.key, ids[j], best_key, best_id)) {
                best_key = pq.key;
                best_id = ids[j];
                best = j;
            }
        }
        partner[i] = (int32_t)best;
    }
    free(count);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Random numbers: Philox4x64-10 (Salmon et al., SC'11)                      */
/* ------------------------------------------------------------------------ */

static void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    /* round multipliers and Weyl key increments of Philox4x64 */
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, c0, &hi0, &lo0);
        mulhilo64(M1, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Isotropic direction by Marsaglia's (1972) rejection method.  Reading:
 * Philox key (seed, 0); block k uses counter (k, a, step, 0) where a is the
 * smaller id of the pair; each block offers two attempts, words (0,1) and
 * (2,3); a word w maps to e = 2*((w >> 11) * 2^-53) - 1, exact in binary64.
 * Accept 0 < s < 1 with s = e1*e1 + e2*e2; then
 * n = (2 e1 sqrt(1-s), 2 e2 sqrt(1-s), 1 - 2 s).  After 32 blocks without
 * an accepted pair (probability < 1e-40) the direction is (0, 0, 1). */
void orc_direction(uint64_t seed, uint64_t step, uint32_t a, double n[3])
{
    const uint64_t key[2] = {seed, 0};
    for (uint64_t blk = 0; blk < 32; ++blk) {
        const uint64_t ctr[4] = {blk, (uint64_t)a, step, 0};
        uint64_t w[4];
        orc_philox4x64_10(ctr, key, w);
        for (int t = 0; t < 2; ++t) {
            double e1 = 2.0 * ((double)(w[2 * t] >> 11) * 0x1.0p-53) - 1.0;
            double e2 = 2.0 * ((double)(w[2 * t + 1] >> 11) * 0x1.0p-53) - 1.0;
            double s = e1 * e1 + e2 * e2;
            if (s > 0.0 && s < 1.0) {
                double f = 2.0 * sqrt(1.0 - s);
                n[0] = e1 * f;
                n[1] = e2 * f;
                n[2] = 1.0 - 2.0 * s;
                return;
            }
        }
    }
    n[0] = 0.0; n[1] = 0.0; n[2] = 1.0;
}

/* SplitMix64 output function of the packed pair (a << 32 | b). */
/* Planar mode (Section 1 also runs the method in two dimensions): a point
 * (e1, e2) uniform in the unit disk has a uniform polar angle phi, and
 * ((e1^2 - e2^2), 2 e1 e2) / (e1^2 + e2^2) = (cos 2phi, sin 2phi) is then a
 * uniform direction; same random numbers and rejection as in space. */
void orc_direction2(uint64_t seed, uint64_t step, uint32_t a, double n[3])
{
    const uint64_t key[2] = {seed, 0};
    for (uint64_t blk = 0; blk < 32; ++blk) {
        const uint64_t ctr[4] = {blk, (uint64_t)a, step, 0};
        uint64_t w[4];
        orc_philox4x64_10(ctr, key, w);
        for (int t = 0; t < 2; ++t) {
            double e1 = 2.0 * ((double)(w[2 * t] >> 11) * 0x1.0p-53) - 1.0;
            double e2 = 2.0 * ((double)(w[2 * t + 1] >> 11) * 0x1.0p-53) - 1.0;
            double a1 = e1 * e1, a2 = e2 * e2;
            double s = a1 + a2;
            if (s > 0.0 && s < 1.0) {
                n[0] = (a1 - a2) / s;
                n[1] = ((2.0 * e1) * e2) / s;
                n[2] = 0.0;
                return;
            }
        }
    }
    n[0] = 1.0; n[1] = 0.0; n[2] = 0.0;
}

uint64_t orc_pair_hash(uint32_t a, uint32_t b)
{
    uint64_t z = (((uint64_t)a << 32) | (uint64_t)b) + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* ------------------------------------------------------------------------ */
/* Boundary conditions (Section 1: reflective or periodic box; the sphere is */
/* the reflecting container of the collapse workload)                        */
/* ------------------------------------------------------------------------ */

static void apply_bc(const orc_box* b, double x[3], double v[3])
{
    if (b->sphere) {
        /* radial mirror: a point at distance rn > R goes to distance 2R - rn
         * along the same ray; the radial velocity component is reversed */
        double rr = fma(x[2], x[2], fma(x[1], x[1], x[0] * x[0]));
        if (rr > b->R * b->R) {
            double rn = sqrt(rr);
            double sc = (2.0 * b->R - rn) / rn;
            double vn = fma(v[2], x[2], fma(v[1], x[1], v[0] * x[0]));
            double cf = (2.0 * vn) / rr;
            for (int k = 0; k < 3; ++k) {
                v[k] = v[k] - cf * x[k];
                x[k] = x[k] * sc;
            }
        }
        return;
    }
    for (int k = 0; k < 3; ++k) {
        double lo = b->lo[k], hi = b->hi[k];
        if (b->absorb[k]) continue;   /* decided after streaming */
        if (b->periodic[k]) {
            double L = hi - lo;
            if (x[k] >= hi) x[k] = x[k] - L;
            else if (x[k] < lo) x[k] = x[k] + L;
        } else {
            if (x[k] < lo) { x[k] = 2.0 * lo - x[k]; v[k] = -v[k]; }
            else if (x[k] > hi) { x[k] = 2.0 * hi - x[k]; v[k] = -v[k]; }
            if (x[k] < lo) x[k] = lo;
            else if (x[k] > hi) x[k] = hi;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Adaptive time step (Section 1: the step is the bin width over the largest */
/* particle speed)                                                           */
/* ------------------------------------------------------------------------ */

int orc_adaptive_dt(const orc_box* b, const double* s, double factor, double* dt)
{
    return orc_adaptive_dt_ex(b, s, NULL, factor, dt);
}

int orc_adaptive_dt_ex(const orc_box* b, const double* s, const unsigned char* gone, double factor,
                       double* dt)
{
    if (!box_ok(b) || !dt || (b->n > 0 && !s) || !(factor > 0.0)) return -1;
    int64_t n = b->n;
    double dx = (b->hi[0] - b->lo[0]) / b->ncell[0];
    for (int k = 1; k < 3; ++k) {
        double w = (b->hi[k] - b->lo[k]) / b->ncell[k];
        if (w < dx) dx = w;
    }
    double v2max = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (gone && gone[i]) continue;
        double vx = s[3 * n + i], vy = s[4 * n + i], vz = s[5 * n + i];
        double v2 = fma(vz, vz, fma(vy, vy, vx * vx));
        if (v2 > v2max) v2max = v2;
    }
    double step = b->dt;
    if (v2max > 0.0) {
        double a = (factor * dx) / sqrt(v2max);
        if (a < step) step = a;
    }
    *dt = step;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One step (Section 1: search, mutual collisions, update, boundaries)       */
/* ------------------------------------------------------------------------ */

/* Collision of the mutual pair (a, c) with ids[a] < ids[c]: collision time
 * t* (from a's side) and the two new velocities.  Elastic, isotropic scatter
 * in the centre-of-mass frame: |g| is kept, its direction is drawn uniformly
 * with the random numbers of the pair's smaller id.  Equal masses:
 * v_cm = (v_a + v_c)/2 and each particle moves off at |g|/2 along +-n.
 * Masses m_a != m_c: v_cm = (m_a v_a + m_c v_c)/M with M = m_a + m_c;
 * a leaves with v_cm + (m_c/M)|g| n and c with v_cm - (m_a/M)|g| n, which
 * keeps the momentum and, as |v'_c - v'_a| = |g|, the kinetic energy. */
static void collide_pair(const orc_box* b, const double* s, const uint32_t* ids,
                         uint64_t step, int64_t a, int64_t c,
                         double nva[3], double nvc[3], double* tstar)
{
    int64_t n = b->n;
    double pa[6], pc[6];
    load6(s, n, a, pa);
    load6(s, n, c, pc);
    int32_t ca[3], cc[3], wrap[3];
    orc_cell_coords(b, pa[0], pa[1], pa[2], ca);
    orc_cell_coords(b, pc[0], pc[1], pc[2], cc);
    for (int k = 0; k < 3; ++k) axis_adjacent(b, k, ca[k], cc[k], &wrap[k]);
    orc_pair_q q;
    orc_pair(b, pa, pc, wrap, &q);
    *tstar = (-q.b) / q.g2;
    double nhat[3];
    if (b->dims == 2) orc_direction2(b->seed, step, ids[a], nhat);
    else orc_direction(b->seed, step, ids[a], nhat);
    double ma = 1.0, mc = 1.0;
    if (b->nspecies > 0) {
        ma = b->mass[b->species[a]];
        mc = b->mass[b->species[c]];
    }
    if (ma == mc) {
        double hg = 0.5 * sqrt(q.g2);
        for (int k = 0; k < 3; ++k) {
            double vcm = 0.5 * (pa[3 + k] + pc[3 + k]);
            nva[k] = vcm + hg * nhat[k];
            nvc[k] = vcm - hg * nhat[k];
        }
    } else {
        double M = ma + mc;
        double gm = sqrt(q.g2);
        double wa = (mc / M) * gm, wc = (ma / M) * gm;
        for (int k = 0; k < 3; ++k) {
            double vcm = fma(ma, pa[3 + k], mc * pc[3 + k]) / M;
            nva[k] = vcm + wa * nhat[k];
            nvc[k] = vcm - wc * nhat[k];
        }
    }
}

/* Free flight of one particle over the step, then the boundary conditions.
 * A collider (hit) moves to t* with its old velocity and on with the new one
 * (or, in velocity-only mode, the whole step with the new one). */
static void advance_one(const orc_box* b, double x[3], double v[3], int hit,
                        const double vn[3], double tstar)
{
    const double dt = b->dt;
    if (hit) {
        for (int k = 0; k < 3; ++k) {
            if (b->kinematics == 0) {
                double xs = x[k] + v[k] * tstar;
                x[k] = xs + vn[k] * (dt - tstar);
            } else {
                x[k] = x[k] + vn[k] * dt;
            }
            v[k] = vn[k];
        }
    } else {
        for (int k = 0; k < 3; ++k) x[k] = x[k] + v[k] * dt;
    }
    apply_bc(b, x, v);
}

int orc_step(const orc_box* b, double* s, const uint32_t* ids, uint64_t step,
             int32_t* partner_out, uint64_t* npairs, uint64_t* digest,
             int nthreads, uint64_t* pair_tests)
{
    return orc_step_ex(b, s, ids, NULL, step, partner_out, npairs, digest, nthreads, pair_tests);
}

/* A particle beyond an absorbing face after streaming leaves the gas. */
static int absorbed(const orc_box* b, const double x[3])
{
    for (int k = 0; k < 3; ++k)
        if (b->absorb[k] && (x[k] < b->lo[k] || x[k] > b->hi[k])) return 1;
    return 0;
}

int orc_step_ex(const orc_box* b, double* s, const uint32_t* ids, unsigned char* gone, uint64_t step,
                int32_t* partner_out, uint64_t* npairs, uint64_t* digest,
                int nthreads, uint64_t* pair_tests)
{
    if (!box_ok(b) || (b->n > 0 && (!s || !ids))) return -1;
    if (b->n > INT32_MAX) return -1;
    if (!gone && (b->absorb[0] || b->absorb[1] || b->absorb[2])) return -1;
    int64_t n = b->n;
    size_t nn = (size_t)(n > 0 ? n : 1);
    int32_t* partner = partner_out ? partner_out : (int32_t*)malloc(nn * sizeof(int32_t));
    double* nv = (double*)malloc(3 * nn * sizeof(double));     /* post-collision velocity */
    double* ts = (double*)malloc(nn * sizeof(double));         /* collision time t*       */
    unsigned char* hit = (unsigned char*)calloc(nn, 1);
    if (!partner || !nv || !ts || !hit) {
        if (!partner_out) free(partner);
        free(nv); free(ts); free(hit);
        return -2;
    }

    /* 1-2: bins and partner search */
    csr_t t;
    if (build_csr(b, s, gone, &t) != 0) {
        if (!partner_out) free(partner);
        free(nv); free(ts); free(hit);
        return -2;
    }
    search_with_csr(b, s, ids, gone, &t, partner, nthreads, pair_tests, NULL);
    free_csr(&t);

    /* 3: a pair collides only if each particle chose the other.  The pair is
     * handled once, from its member with the smaller id (a). */
    uint64_t pairs = 0, dig = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t p = partner[i];
        if (p < 0 || partner[p] != (int32_t)i || !(ids[i] < ids[p])) continue;
        int64_t a = i, c = p;
        double nva[3], nvc[3], tstar;
        collide_pair(b, s, ids, step, a, c, nva, nvc, &tstar);
        for (int k = 0; k < 3; ++k) {
            nv[(size_t)k * nn + (size_t)a] = nva[k];
            nv[(size_t)k * nn + (size_t)c] = nvc[k];
        }
        ts[a] = tstar;
        ts[c] = tstar;
        hit[a] = 1;
        hit[c] = 1;
        ++pairs;
        dig += orc_pair_hash(ids[a], ids[c]);
    }

    /* 4: free streaming and boundary conditions; particles that have left
     * the gas stay where they are */
    for (int64_t i = 0; i < n; ++i) {
        if (gone && gone[i]) continue;
        double x[3], v[3], vn[3];
        for (int k = 0; k < 3; ++k) {
            x[k] = s[(size_t)k * nn + (size_t)i];
            v[k] = s[(size_t)(3 + k) * nn + (size_t)i];
            vn[k] = nv[(size_t)k * nn + (size_t)i];
        }
        advance_one(b, x, v, hit[i], vn, ts[i]);
        if (gone && absorbed(b, x)) gone[i] = 1;
        for (int k = 0; k < 3; ++k) {
            s[(size_t)k * nn + (size_t)i] = x[k];
            s[(size_t)(3 + k) * nn + (size_t)i] = v[k];
        }
    }

    if (npairs) *npairs = pairs;
    if (digest) *digest = dig;
    if (!partner_out) free(partner);
    free(nv);
    free(ts);
    free(hit);
    return 0;
}

/* The same step evaluated for selected particles only: for each listed index
 * sel[k], its partner (index or -1) and its state after the step.  The bins
 * are built for all particles; the search runs for each selected particle and
 * for its partner (to decide mutuality), so large runs can be checked at
 * sampled particles. */
int orc_step_sampled(const orc_box* b, const double* s, const uint32_t* ids, uint64_t step,
                     const int64_t* sel, int64_t nsel, int32_t* partner_out,
                     double* state_out, int nthreads)
{
    if (!box_ok(b) || (b->n > 0 && (!s || !ids)) || nsel < 0 ||
        (nsel > 0 && (!sel || !partner_out || !state_out)))
        return -1;
    if (b->n > INT32_MAX) return -1;
    for (int64_t k = 0; k < nsel; ++k)
        if (sel[k] < 0 || sel[k] >= b->n) return -1;
    int64_t n = b->n;
    csr_t t;
    if (build_csr(b, s, NULL, &t) != 0) return -2;
#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt)
#else
    (void)nthreads;
#endif
    for (int64_t k = 0; k < nsel; ++k) {
        int64_t i = sel[k];
        uint64_t tests = 0, acc = 0;
        int64_t p = search_one(b, s, ids, &t, i, &tests, &acc);
        int hit = p >= 0 && search_one(b, s, ids, &t, p, &tests, &acc) == i;
        double x[3], v[3], vn[3] = {0.0, 0.0, 0.0}, tstar = 0.0;
        for (int a = 0; a < 3; ++a) {
            x[a] = s[(int64_t)a * n + i];
            v[a] = s[(int64_t)(3 + a) * n + i];
        }
        if (hit) {
            double nva[3], nvc[3];
            if (ids[i] < ids[p]) {
                collide_pair(b, s, ids, step, i, p, nva, nvc, &tstar);
                for (int a = 0; a < 3; ++a) vn[a] = nva[a];
            } else {
                collide_pair(b, s, ids, step, p, i, nva, nvc, &tstar);
                for (int a = 0; a < 3; ++a) vn[a] = nvc[a];
            }
        }
        advance_one(b, x, v, hit, vn, tstar);
        partner_out[k] = (int32_t)p;
        for (int a = 0; a < 3; ++a) {
            state_out[6 * k + a] = x[a];
            state_out[6 * k + 3 + a] = v[a];
        }
    }
    free_csr(&t);
    return 0;
}
