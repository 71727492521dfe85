// kmc_device.hip -- gfx950 kernels of the DCA collision step (arXiv:1310.3437,
// Section 1): bin, scan, cell-sorted copy, partner search, mutual resolve with
// isotropic centre-of-mass scatter, free stream and boundary conditions.
//
// Built with -ffp-contract=off: the only fused multiply-adds are the fma()
// calls written below, which are part of the step's definition.  Every
// floating-point expression that decides a result is written in the
// definition's order so that results are bit-identical to any other
// IEEE-754 binary64 implementation of the same definition.
#include "kmc_internal.h"

namespace kmc {
namespace {

// --------------------------------------------------------------------------
// Definition pieces
// --------------------------------------------------------------------------

// Cell index along one axis: clamp(floor((x - lo) * inv_h), 0, n - 1).
__device__ __forceinline__ int cell1(double x, double lo, double inv_h, int n)
{
    double f = floor((x - lo) * inv_h);
    if (!(f >= 0.0)) return 0;
    if (f >= (double)n) return n - 1;
    return (int)f;
}

// Image of a partner along one axis, from the two cell indices: the
// partner's image is shifted by -L (+L) when it sits in the last (first)
// cell of a periodic axis and the other particle in the first (last).
__device__ __forceinline__ int wrap_of(int ci, int cj, int n, int periodic)
{
    if (!periodic) return 0;
    int d = cj - ci;
    if (d == n - 1) return -1;
    if (d == -(n - 1)) return 1;
    return 0;
}

// Closest-approach quantities of the ordered pair (searcher, candidate):
// b = r.g, g2 = |g|^2, c2 = |r x g|^2 with a fixed fma order.
struct PairQ {
    double b, g2, c2;
};

__device__ __forceinline__ PairQ pair_q(double rx, double ry, double rz,
                                        double gx, double gy, double gz)
{
    PairQ q;
    q.b = fma(rz, gz, fma(ry, gy, rx * gx));
    q.g2 = fma(gz, gz, fma(gy, gy, gx * gx));
    double cx = fma(ry, gz, -(rz * gy));
    double cy = fma(rz, gx, -(rx * gz));
    double cz = fma(rx, gy, -(ry * gx));
    q.c2 = fma(cz, cz, fma(cy, cy, cx * cx));
    return q;
}

// Partner criteria multiplied through by g2 > 0: closest approach within
// [0, dt] (b <= 0, -b <= dt g2) and inside the interaction diameter
// (c2 < D2 g2, i.e. d_min^2 < sigma/pi).
__device__ __forceinline__ bool accept(const PairQ& q, double D2, double dt)
{
    return (q.g2 > 0.0) & (q.b <= 0.0) & (-q.b <= dt * q.g2) & (q.c2 < D2 * q.g2);
}

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): two 64x64->128
// multiplications per round, Weyl-sequence key schedule.
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    const uint64_t m0 = 0xD2E7470EE14C6C93ull, m1 = 0xCA5A826395121157ull;
    const uint64_t w0 = 0x9E3779B97F4A7C15ull, w1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += w0; k1 += w1; }
        uint64_t hi0 = __umul64hi(m0, c[0]), lo0 = m0 * c[0];
        uint64_t hi1 = __umul64hi(m1, c[2]), lo1 = m1 * c[2];
        uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
}

// Isotropic unit vector (Marsaglia 1972) for the pair whose smaller id is a:
// block k of Philox with key (seed, 0) and counter (k, a, step, 0) offers two
// candidate points (words 0,1 and 2,3) e = 2 (w >> 11) 2^-53 - 1 in [-1, 1);
// the first with 0 < s = e1^2 + e2^2 < 1 gives
// n = (2 e1 sqrt(1-s), 2 e2 sqrt(1-s), 1 - 2s).
__device__ void direction(uint64_t seed, uint64_t step, uint32_t a, double n[3])
{
    for (uint64_t blk = 0; blk < 32; ++blk) {
        uint64_t w[4] = {blk, (uint64_t)a, step, 0};
        philox4x64_10(w, seed, 0);
#pragma unroll
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

// SplitMix64 output of the packed pair (a << 32 | b): the digest term.
__device__ __forceinline__ uint64_t pair_hash(uint32_t a, uint32_t b)
{
    uint64_t z = (((uint64_t)a << 32) | (uint64_t)b) + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ const BoxDev& box_of(const Plan& p, uint32_t i)
{
    return p.boxes[p.boxidx ? p.boxidx[i] : 0u];
}

// Visit the 27-cell neighbourhood of cell (cx, cy, cz) as contiguous ranges
// [s, e) of the cell-sorted arrays: per neighbour row (dy, dz) the cells
// cx-1..cx+1 that exist without wrapping form one range; on a periodic x axis
// a wrapped end cell is a separate range.  f(s, e, wx, wy, wz) receives the
// image selectors of the range.
template <class F>
__device__ __forceinline__ void for_each_range(const BoxDev& B, int cx, int cy, int cz,
                                               const uint32_t* __restrict__ start, F&& f)
{
    const int NX = B.nc[0], NY = B.nc[1], NZ = B.nc[2];
    for (int dz = -1; dz <= 1; ++dz) {
        int nz = cz + dz, wz = 0;
        if (nz < 0) { if (!B.periodic[2]) continue; nz += NZ; wz = -1; }
        else if (nz >= NZ) { if (!B.periodic[2]) continue; nz -= NZ; wz = 1; }
        for (int dy = -1; dy <= 1; ++dy) {
            int ny = cy + dy, wy = 0;
            if (ny < 0) { if (!B.periodic[1]) continue; ny += NY; wy = -1; }
            else if (ny >= NY) { if (!B.periodic[1]) continue; ny -= NY; wy = 1; }
            const uint32_t row = B.coff + (uint32_t)NX * ((uint32_t)ny + (uint32_t)NY * (uint32_t)nz);
            const int x0 = cx - 1, x1 = cx + 1;
            const int m0 = x0 < 0 ? 0 : x0;
            const int m1 = x1 >= NX ? NX - 1 : x1;
            f(start[row + m0], start[row + m1 + 1], 0, wy, wz);
            if (B.periodic[0]) {
                if (x0 < 0) f(start[row + NX - 1], start[row + NX], -1, wy, wz);
                if (x1 >= NX) f(start[row], start[row + 1], 1, wy, wz);
            }
        }
    }
}

// Block-wide sum of two 64-bit values; thread 0 gets the totals.
__device__ __forceinline__ void block_sum2(uint64_t& a, uint64_t& b, uint64_t* lds /*[2*16]*/)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
    }
    if (lane == 0) { lds[wid] = a; lds[16 + wid] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < nw; ++w) { a += lds[w]; b += lds[16 + w]; }
    }
}

// --------------------------------------------------------------------------
// Initialisation and read-back
// --------------------------------------------------------------------------

__global__ void k_init_particles(Plan p, const double* __restrict__ in)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.N) return;
    const size_t N = p.N;
#pragma unroll
    for (int k = 0; k < 6; ++k) p.A[k * N + i] = in[k * N + i];
    p.idA[i] = i;
    if (p.boxidx) {
        uint32_t lo = 0, hi = p.nboxes - 1;   // last box with poff <= i
        while (lo < hi) {
            uint32_t mid = (lo + hi + 1) >> 1;
            if (p.boxes[mid].poff <= i) lo = mid; else hi = mid - 1;
        }
        p.boxidx[i] = lo;
    }
}

__global__ void k_fill_u32(uint32_t* __restrict__ a, uint32_t n, uint32_t v)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) a[i] = v;
}

__global__ void k_init_ctl(Plan p, unsigned long long step0)
{
    const uint32_t t = threadIdx.x;
    if (t == 0) {
        p.ctl->step = step0;
        p.ctl->steps_done = 0;
        p.ctl->rechecks_total = 0;
        p.ctl->fallbacks_total = 0;
        p.ctl->recheck_count = 0;
        p.ctl->overflow = 0;
        p.ctl->work_next = 0;
    }
    for (uint32_t k = t; k < (uint32_t)kHistLanes; k += blockDim.x) {
        p.hist_np[k] = 0;
        p.hist_dig[k] = 0;
    }
}

__global__ void k_read_partners(Plan p, int32_t* __restrict__ out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.N) return;
    const int32_t q = p.partner[i];
    out[p.idB[i]] = q >= 0 ? (int32_t)p.idB[q] : -1;
}

__global__ void k_read_state(Plan p, double* __restrict__ out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.N) return;
    const size_t N = p.N;
    const uint32_t id = p.idA[i];
#pragma unroll
    for (int k = 0; k < 6; ++k) out[k * N + id] = p.A[k * N + i];
}

// --------------------------------------------------------------------------
// a1: bin + count.  The rank returned by the atomic is the particle's slot
// inside its cell; the order inside a cell never affects a result.
// --------------------------------------------------------------------------

__global__ void k_bin(Plan p)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.N) return;
    const BoxDev& B = box_of(p, i);
    const size_t N = p.N;
    const int cx = cell1(p.A[i], B.lo[0], B.inv_h[0], B.nc[0]);
    const int cy = cell1(p.A[N + i], B.lo[1], B.inv_h[1], B.nc[1]);
    const int cz = cell1(p.A[2 * N + i], B.lo[2], B.inv_h[2], B.nc[2]);
    const uint32_t c = B.coff + (uint32_t)cx + (uint32_t)B.nc[0] * ((uint32_t)cy + (uint32_t)B.nc[1] * (uint32_t)cz);
    p.cell[i] = c;
    p.slot[i] = atomicAdd(&p.count[c], 1u);
}

// --------------------------------------------------------------------------
// a2: exclusive prefix sum of the cell counts (reduce, scan of block sums,
// down-sweep).  The down-sweep also clears the counts for the next step.
// --------------------------------------------------------------------------

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* lds, uint32_t& total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) lds[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int w = 0; w < nw; ++w) { uint32_t t = lds[w]; lds[w] = s; s += t; }
        lds[nw] = s;
    }
    __syncthreads();
    const uint32_t excl = lds[wid] + x - v;
    total = lds[nw];
    __syncthreads();
    return excl;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(Plan p)
{
    __shared__ uint32_t lds[kScanBlock / 64 + 1];
    const uint32_t base = blockIdx.x * (uint32_t)kScanTile + threadIdx.x * kScanItems;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const uint32_t c = base + k;
        if (c < p.C) s += p.count[c];
    }
    uint32_t total;
    block_exclusive_scan(s, lds, total);
    if (threadIdx.x == 0) p.partial[blockIdx.x] = total;
}

// One block of 1024 threads scans the block sums in place.  It also starts
// the step's device-side bookkeeping (recheck list, work queue).
__global__ __launch_bounds__(1024) void k_scan_partials(Plan p)
{
    __shared__ uint32_t lds[1024 / 64 + 1];
    uint32_t carry = 0;
    for (uint32_t base = 0; base < p.nblk_scan; base += blockDim.x) {
        const uint32_t k = base + threadIdx.x;
        const uint32_t v = k < p.nblk_scan ? p.partial[k] : 0u;
        uint32_t total;
        const uint32_t e = block_exclusive_scan(v, lds, total);
        if (k < p.nblk_scan) p.partial[k] = carry + e;
        carry += total;
    }
    if (threadIdx.x == 0) {
        p.ctl->recheck_count = 0;
        p.ctl->overflow = 0;
        p.ctl->work_next = 0;
    }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_down(Plan p)
{
    __shared__ uint32_t lds[kScanBlock / 64 + 1];
    const uint32_t base = blockIdx.x * (uint32_t)kScanTile + threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const uint32_t c = base + k;
        v[k] = c < p.C ? p.count[c] : 0u;
        s += v[k];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, lds, total) + p.partial[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const uint32_t c = base + k;
        if (c < p.C) {
            p.start[c] = run;
            p.count[c] = 0u;
        }
        run += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) p.start[p.C] = p.N;
}

// --------------------------------------------------------------------------
// a3: cell-sorted copy of the state (and, for the FP32 screen, an FP32 copy
// of positions relative to the box origin ctr32 and of velocities).
// --------------------------------------------------------------------------

template <bool F32>
__global__ void k_scatter(Plan p)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.N) return;
    const size_t N = p.N;
    const uint32_t d = p.start[p.cell[i]] + p.slot[i];
    double s[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        s[k] = p.A[k * N + i];
        p.B[k * N + d] = s[k];
    }
    p.idB[d] = p.idA[i];
    if (F32) {
        const BoxDev& B = box_of(p, i);
#pragma unroll
        for (int k = 0; k < 3; ++k) p.B32[k * N + d] = (float)(s[k] - (double)B.ctr32[k]);
#pragma unroll
        for (int k = 3; k < 6; ++k) p.B32[k * N + d] = (float)s[k];
    }
}

// --------------------------------------------------------------------------
// a4: DCA partner search in FP64, one thread per cell-sorted particle.
// --------------------------------------------------------------------------

// Search of one particle over its 27-cell neighbourhood.  Returns the
// sorted index of the closest acceptable partner ((key, id) minimum) or -1.
__device__ __forceinline__ int32_t search_one64(const Plan& p, uint32_t i)
{
    const BoxDev& B = box_of(p, i);
    const size_t N = p.N;
    const double* __restrict__ X = p.B;
    const double xi = X[i], yi = X[N + i], zi = X[2 * N + i];
    const double ui = X[3 * N + i], vi = X[4 * N + i], wi = X[5 * N + i];
    const int cx = cell1(xi, B.lo[0], B.inv_h[0], B.nc[0]);
    const int cy = cell1(yi, B.lo[1], B.inv_h[1], B.nc[1]);
    const int cz = cell1(zi, B.lo[2], B.inv_h[2], B.nc[2]);
    const double D2 = B.D2, dt = B.dt;
    double best_key = __builtin_inf();
    uint32_t best_id = 0xFFFFFFFFu;
    int32_t best = -1;
    for_each_range(B, cx, cy, cz, p.start, [&](uint32_t s, uint32_t e, int wx, int wy, int wz) {
        const bool shift = (wx | wy | wz) != 0;
        const double sx = (double)wx * B.L[0], sy = (double)wy * B.L[1], sz = (double)wz * B.L[2];
        for (uint32_t j = s; j < e; ++j) {
            if (j == i) continue;
            double rx = X[j] - xi, ry = X[N + j] - yi, rz = X[2 * N + j] - zi;
            if (shift) {
                // the image shift is added only where the range wrapped;
                // adding +0.0 elsewhere changes at most the sign of a zero
                rx = rx + sx; ry = ry + sy; rz = rz + sz;
            }
            const double gx = X[3 * N + j] - ui, gy = X[4 * N + j] - vi, gz = X[5 * N + j] - wi;
            const PairQ q = pair_q(rx, ry, rz, gx, gy, gz);
            if (accept(q, D2, dt)) {
                const double key = q.c2 / q.g2;
                const uint32_t idj = p.idB[j];
                if (key < best_key || (key == best_key && idj < best_id)) {
                    best_key = key;
                    best_id = idj;
                    best = (int32_t)j;
                }
            }
        }
    });
    return best;
}

__global__ void k_search64(Plan p)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.N) return;
    p.partner[i] = search_one64(p, i);
}

// --------------------------------------------------------------------------
// a5-a8: mutual resolve, isotropic CM scatter at t*, free stream, boundary
// conditions, per-step pair count and digest.  One thread per sorted
// particle; both members of a pair compute the pair's update identically and
// each writes only its own particle.
// --------------------------------------------------------------------------

__device__ __forceinline__ void apply_bc(const BoxDev& B, double x[3], double v[3])
{
    if (B.sphere) {
        const double rr = fma(x[2], x[2], fma(x[1], x[1], x[0] * x[0]));
        if (rr > B.R2) {
            const double rn = sqrt(rr);
            const double sc = (2.0 * B.R - rn) / rn;
            const double vn = fma(v[2], x[2], fma(v[1], x[1], v[0] * x[0]));
            const double cf = (2.0 * vn) / rr;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                v[k] = v[k] - cf * x[k];
                x[k] = x[k] * sc;
            }
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double lo = B.lo[k], hi = B.hi[k];
        if (B.periodic[k]) {
            if (x[k] >= hi) x[k] = x[k] - B.L[k];
            else if (x[k] < lo) x[k] = x[k] + B.L[k];
        } else {
            if (x[k] < lo) { x[k] = 2.0 * lo - x[k]; v[k] = -v[k]; }
            else if (x[k] > hi) { x[k] = 2.0 * hi - x[k]; v[k] = -v[k]; }
            if (x[k] < lo) x[k] = lo;
            else if (x[k] > hi) x[k] = hi;
        }
    }
}

__global__ __launch_bounds__(1024) void k_resolve(Plan p)
{
    __shared__ uint64_t lds[32];
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t my_np = 0, my_dig = 0;
    if (i < p.N) {
        const BoxDev& B = box_of(p, i);
        const size_t N = p.N;
        const double* __restrict__ X = p.B;
        double x[3], v[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) { x[k] = X[k * N + i]; v[k] = X[(3 + k) * N + i]; }
        const uint32_t id = p.idB[i];
        const int32_t q = p.partner[i];
        const double dt = B.dt;
        bool hit = false;
        if (q >= 0 && p.partner[q] == (int32_t)i) {
            hit = true;
            const uint32_t idq = p.idB[q];
            double xq[3], vq[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) { xq[k] = X[k * N + q]; vq[k] = X[(3 + k) * N + q]; }
            const bool me_a = id < idq;   // a = the member with the smaller id
            const double* xa = me_a ? x : xq;
            const double* va = me_a ? v : vq;
            const double* xb = me_a ? xq : x;
            const double* vb = me_a ? vq : v;
            const uint32_t ida = me_a ? id : idq, idb = me_a ? idq : id;
            double r[3], g[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int ca = cell1(xa[k], B.lo[k], B.inv_h[k], B.nc[k]);
                const int cb = cell1(xb[k], B.lo[k], B.inv_h[k], B.nc[k]);
                const int w = wrap_of(ca, cb, B.nc[k], B.periodic[k]);
                r[k] = xb[k] - xa[k];
                if (w != 0) r[k] = r[k] + (double)w * B.L[k];
                g[k] = vb[k] - va[k];
            }
            const PairQ pq = pair_q(r[0], r[1], r[2], g[0], g[1], g[2]);
            const double tstar = (-pq.b) / pq.g2;
            double nh[3];
            direction(p.seed, p.ctl->step, ida, nh);
            const double hg = 0.5 * sqrt(pq.g2);
            double vn[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double vcm = 0.5 * (va[k] + vb[k]);
                vn[k] = me_a ? vcm + hg * nh[k] : vcm - hg * nh[k];
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                if (p.kinematics == KMC_KIN_AT_TSTAR) {
                    const double xs = x[k] + v[k] * tstar;
                    x[k] = xs + vn[k] * (dt - tstar);
                } else {
                    x[k] = x[k] + vn[k] * dt;
                }
                v[k] = vn[k];
            }
            if (me_a) {
                my_np = 1;
                my_dig = pair_hash(ida, idb);
            }
        }
        if (!hit) {
#pragma unroll
            for (int k = 0; k < 3; ++k) x[k] = x[k] + v[k] * dt;
        }
        apply_bc(B, x, v);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            p.A[k * N + i] = x[k];
            p.A[(3 + k) * N + i] = v[k];
        }
        p.idA[i] = id;
    }
    block_sum2(my_np, my_dig, lds);
    if (threadIdx.x == 0 && my_np != 0) {
        const size_t row = (size_t)(p.ctl->steps_done % p.H) * kHistLanes + (blockIdx.x % kHistLanes);
        atomicAdd(&p.hist_np[row], (unsigned long long)my_np);
        atomicAdd(&p.hist_dig[row], (unsigned long long)my_dig);
    }
}

// End of step: advance the step counters, fold the screen statistics and
// clear the next history row.
__global__ void k_advance(Plan p)
{
    const unsigned long long next = p.ctl->steps_done + 1;
    const size_t row = (size_t)(next % p.H) * kHistLanes;
    for (uint32_t k = threadIdx.x; k < (uint32_t)kHistLanes; k += blockDim.x) {
        p.hist_np[row + k] = 0;
        p.hist_dig[row + k] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        p.ctl->rechecks_total += p.ctl->recheck_count;
        p.ctl->fallbacks_total += p.ctl->overflow ? 1ull : 0ull;
        p.ctl->steps_done = next;
        p.ctl->step += 1;
    }
}

// Pair tests of the last step: sum over sorted particles of the 27-cell
// neighbourhood population minus one.
__global__ __launch_bounds__(256) void k_count_tests(Plan p, unsigned long long* out)
{
    __shared__ uint64_t lds[32];
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t t = 0, z = 0;
    if (i < p.N) {
        const BoxDev& B = box_of(p, i);
        const size_t N = p.N;
        const int cx = cell1(p.B[i], B.lo[0], B.inv_h[0], B.nc[0]);
        const int cy = cell1(p.B[N + i], B.lo[1], B.inv_h[1], B.nc[1]);
        const int cz = cell1(p.B[2 * N + i], B.lo[2], B.inv_h[2], B.nc[2]);
        for_each_range(B, cx, cy, cz, p.start, [&](uint32_t s, uint32_t e, int, int, int) { t += e - s; });
        t -= 1;
    }
    block_sum2(t, z, lds);
    if (threadIdx.x == 0) atomicAdd(out, (unsigned long long)t);
}

inline uint32_t blocks_for(uint32_t n, uint32_t b) { return (n + b - 1) / b; }

}  // namespace

// --------------------------------------------------------------------------
// Launchers
// --------------------------------------------------------------------------

hipError_t launch_init(const Plan& p, const double* d_state, hipStream_t s)
{
    const uint32_t b = 256;
    if (p.N > 0) k_init_particles<<<blocks_for(p.N, b), b, 0, s>>>(p, d_state);
    k_fill_u32<<<blocks_for(p.C, b) < 4096 ? blocks_for(p.C, b) : 4096, b, 0, s>>>(p.count, p.C, 0u);
    k_init_ctl<<<1, 64, 0, s>>>(p, 0);
    return hipGetLastError();
}

hipError_t launch_step(const Plan& p, hipStream_t s, hipEvent_t* ev)
{
    const uint32_t b = (uint32_t)p.block;
    const uint32_t gN = blocks_for(p.N, b);
    auto mark = [&](int k) { if (ev) (void)hipEventRecord(ev[k], s); };
    mark(KMC_PHASE_BIN);
    if (p.N > 0) k_bin<<<gN, b, 0, s>>>(p);
    mark(KMC_PHASE_SCAN);
    k_scan_reduce<<<p.nblk_scan, kScanBlock, 0, s>>>(p);
    k_scan_partials<<<1, 1024, 0, s>>>(p);
    k_scan_down<<<p.nblk_scan, kScanBlock, 0, s>>>(p);
    mark(KMC_PHASE_SCATTER);
    if (p.N > 0) {
        if (p.precision == KMC_FP32_SCREEN) k_scatter<true><<<gN, b, 0, s>>>(p);
        else k_scatter<false><<<gN, b, 0, s>>>(p);
    }
    mark(KMC_PHASE_SEARCH);
    if (p.N > 0) k_search64<<<gN, b, 0, s>>>(p);
    mark(KMC_PHASE_RECHECK);
    mark(KMC_PHASE_RESOLVE);
    if (p.N > 0) k_resolve<<<gN, b, 0, s>>>(p);
    k_advance<<<1, 64, 0, s>>>(p);
    mark(KMC_PHASE_COUNT);
    return hipGetLastError();
}

hipError_t launch_read_partners(const Plan& p, int32_t* out, hipStream_t s)
{
    if (p.N > 0) k_read_partners<<<blocks_for(p.N, 256), 256, 0, s>>>(p, out);
    return hipGetLastError();
}

hipError_t launch_read_state(const Plan& p, double* out, hipStream_t s)
{
    if (p.N > 0) k_read_state<<<blocks_for(p.N, 256), 256, 0, s>>>(p, out);
    return hipGetLastError();
}

hipError_t launch_count_tests(const Plan& p, unsigned long long* d_out, hipStream_t s)
{
    if (p.N > 0) k_count_tests<<<blocks_for(p.N, 256), 256, 0, s>>>(p, d_out);
    return hipGetLastError();
}

}  // namespace kmc
