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

// Density-adaptive bins: index of a point on the finest grid (n 2^L cells)
// along one axis, clamp(floor((x - lo) * (inv_h * 2^L)), 0, n 2^L - 1).
// inv_h * 2^L is exact and the power-of-two scaling commutes with the
// rounding of the product, so the point's cell is this index >> L.
__device__ __forceinline__ int fine1(double x, double lo, double inv_h, int n, int L)
{
    const double f = floor((x - lo) * (inv_h * (double)(1 << L)));
    if (!(f >= 0.0)) return 0;
    const double m = (double)n * (double)(1 << L);
    if (f >= m) return (int)(m - 1.0);
    return (int)f;
}

// Split level of a cell holding `count` particles: the smallest l in 0..L
// with count <= T 8^l, else L.
__device__ __forceinline__ uint32_t split_level(uint32_t count, uint32_t T, int L)
{
    for (int l = 0; l < L; ++l)
        if ((uint64_t)count <= ((uint64_t)T << (3 * l))) return (uint32_t)l;
    return (uint32_t)L;
}

// Index of the sub-bin (leaf) a point falls in inside its cell split at
// level lvl: the sub-bin coordinates are bits L-lvl .. L-1 of the finest
// indices, linearised x fastest.
__device__ __forceinline__ uint32_t leaf_code(const BoxDev& B, int L, uint32_t lvl, double x, double y, double z)
{
    const int sh = L - (int)lvl;
    const uint32_t m = (1u << lvl) - 1u;
    const uint32_t sx = ((uint32_t)fine1(x, B.lo[0], B.inv_h[0], B.nc[0], L) >> sh) & m;
    const uint32_t sy = ((uint32_t)fine1(y, B.lo[1], B.inv_h[1], B.nc[1], L) >> sh) & m;
    const uint32_t sz = ((uint32_t)fine1(z, B.lo[2], B.inv_h[2], B.nc[2], L) >> sh) & m;
    return sx + (m + 1u) * (sy + (m + 1u) * sz);
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
// (c2 < D2 g2, i.e. d_min^2 < D2: sigma/pi for one kind of particle, the
// squared sum of the two radii for particles of several kinds).
__device__ __forceinline__ bool accept(const PairQ& q, double D2, double dt)
{
    return (q.g2 > 0.0) & (q.b <= 0.0) & (-q.b <= dt * q.g2) & (q.c2 < D2 * q.g2);
}

// Full 128-bit product of two 64-bit words from four 32x32 partial
// products (schoolbook); each partial product plus a 64-bit addend fits in
// 64 bits, so every step is one 32x32+64 multiply-add and the low word
// reuses the partial products instead of multiplying again.
__device__ __forceinline__ void mul_wide(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo)
{
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
    const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
    const uint64_t p00 = (uint64_t)a0 * b0;
    const uint64_t p01 = (uint64_t)a0 * b1 + (p00 >> 32);
    const uint64_t p10 = (uint64_t)a1 * b0 + (uint32_t)p01;
    hi = (uint64_t)a1 * b1 + (p01 >> 32) + (p10 >> 32);
    lo = (p10 << 32) | (uint32_t)p00;
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
        uint64_t hi0, lo0, hi1, lo1;
        mul_wide(m0, c[0], hi0, lo0);
        mul_wide(m1, c[2], hi1, lo1);
        uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
}

// Isotropic unit vector (Marsaglia 1972) for the pair whose smaller id is a:
// block k of Philox with key (seed, 0) and counter (k, a, step, 0) offers two
// candidate points (words 0,1 and 2,3) e = 2 (w >> 11) 2^-53 - 1 in [-1, 1);
// the first with 0 < s = e1^2 + e2^2 < 1 gives
// n = (2 e1 sqrt(1-s), 2 e2 sqrt(1-s), 1 - 2s).
__device__ void direction(uint64_t seed, uint64_t step, uint32_t a, double n[3], int dims)
{
    for (uint64_t blk = 0; blk < 32; ++blk) {
        uint64_t w[4] = {blk, (uint64_t)a, step, 0};
        philox4x64_10(w, seed, 0);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            double e1 = 2.0 * ((double)(w[2 * t] >> 11) * 0x1.0p-53) - 1.0;
            double e2 = 2.0 * ((double)(w[2 * t + 1] >> 11) * 0x1.0p-53) - 1.0;
            if (dims == 2) {
                // planar: (cos 2phi, sin 2phi) of a point uniform in the unit disk
                const double a1 = e1 * e1, a2 = e2 * e2;
                const double s = a1 + a2;
                if (s > 0.0 && s < 1.0) {
                    n[0] = (a1 - a2) / s;
                    n[1] = ((2.0 * e1) * e2) / s;
                    n[2] = 0.0;
                    return;
                }
            } else {
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
    }
    n[0] = dims == 2 ? 1.0 : 0.0;
    n[1] = 0.0;
    n[2] = dims == 2 ? 0.0 : 1.0;
}

// SplitMix64 output of the packed pair (a << 32 | b): the digest term.
__device__ __forceinline__ uint64_t pair_hash(uint32_t a, uint32_t b)
{
    uint64_t z = (((uint64_t)a << 32) | (uint64_t)b) + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Logical block index for kernels whose neighbouring blocks share data:
// the dispatcher hands consecutive workgroups to the 8 XCDs in turn, each
// with its own L2, so block b is mapped to a contiguous per-XCD range of
// tiles (a bijection for any grid size) and each XCD sweeps one slice of
// the cell-sorted particles.
constexpr uint32_t kXcds = 8;

__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t nb)
{
    const uint32_t x = b % kXcds, idx = b / kXcds, q = nb / kXcds, r = nb % kXcds;
    return x * q + (x < r ? x : r) + idx;
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

__global__ void k_init_particles(Plan p, const double* __restrict__ in, const uint8_t* __restrict__ kind)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.N) return;
    const size_t N = p.N;
#pragma unroll
    for (int k = 0; k < 6; ++k) p.A[k * N + i] = in[k * N + i];
    p.idA[i] = i;
    if (p.spA) {
        // an invalid kind is counted by k_check_kinds (the context is then not
        // created); it is clamped here so that no table read leaves its table
        const uint8_t k = kind[i];
        p.spA[i] = k < (uint8_t)p.nspecies ? k : (uint8_t)(p.nspecies - 1);
    }
    if (p.boxidx) {
        uint32_t lo = 0, hi = p.nboxes - 1;   // last box with poff <= i
        while (lo < hi) {
            uint32_t mid = (lo + hi + 1) >> 1;
            if (p.boxes[mid].poff <= i) lo = mid; else hi = mid - 1;
        }
        p.boxidx[i] = lo;
    }
}

__global__ void k_fill_u32(uint32_t* __restrict__ a, size_t n, uint32_t v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) a[i] = v;
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
        p.ctl->absorbed_total = 0;
        p.ctl->candidates_total = 0;
        p.ctl->scratch = 0;
    }
    for (uint32_t k = t; k < (uint32_t)kAccLanes; k += blockDim.x) {
        p.acc[k].np = 0;
        p.acc[k].dig = 0;
        p.acc[k].cand = 0;
    }
    for (uint32_t b = t; b < p.nboxes; b += blockDim.x) p.box_v2[b] = 0ull;
}

// Kinds at or beyond the number of kinds, counted into the control block's
// scratch word (kmc_init reads it back).
__global__ void k_check_kinds(Plan p, const uint8_t* __restrict__ kind)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool bad = i < p.N && kind[i] >= (uint8_t)p.nspecies;
    const uint64_t m = __ballot(bad);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(&p.ctl->scratch, (unsigned long long)__popcll(m));
}

__global__ void k_read_partners(Plan p, int32_t* __restrict__ out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.N) return;
    const int32_t q = p.partner[i];   // an absorbed particle has none, nor is it anyone's
    out[p.idB[i] & ~kGone] = q >= 0 ? (int32_t)p.idB[q] : -1;
}

__global__ void k_read_state(Plan p, double* __restrict__ out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.N) return;
    const size_t N = p.N;
    const uint32_t id = p.idA[i] & ~kGone;
#pragma unroll
    for (int k = 0; k < 6; ++k) out[k * N + id] = p.A[k * N + i];
}

// --------------------------------------------------------------------------
// a1: bin + count.  The rank returned by the atomic is the particle's slot
// inside its cell; the order inside a cell never affects a result.
// --------------------------------------------------------------------------

// Cell of particle i at position (x, y, z) and its slot: the state is in
// the previous step's cell order, so neighbouring lanes mostly share a cell
// and each run of equal cells takes its slots with one atomic issued by the
// run's first lane.  Every lane of the wave must call this.
// Global cell of a particle at (x, y, z) in box B; absorbed particles go to
// the box's extra cell after its grid.  On the uniform grid the sorted copy
// recomputes it from the same stored position instead of reading it back;
// with adaptive bins the binning stores it for the leaf count and the copy.
__device__ __forceinline__ uint32_t cell_of(const BoxDev& B, double x, double y, double z, bool gone)
{
    if (gone) return B.coff + (uint32_t)B.nc[0] * (uint32_t)B.nc[1] * (uint32_t)B.nc[2];
    const int cx = cell1(x, B.lo[0], B.inv_h[0], B.nc[0]);
    const int cy = cell1(y, B.lo[1], B.inv_h[1], B.nc[1]);
    const int cz = cell1(z, B.lo[2], B.inv_h[2], B.nc[2]);
    return B.coff + (uint32_t)cx + (uint32_t)B.nc[0] * ((uint32_t)cy + (uint32_t)B.nc[1] * (uint32_t)cz);
}

__device__ __forceinline__ void bin_particle(const Plan& p, uint32_t i, bool valid, const BoxDev& B, double x,
                                             double y, double z, bool gone)
{
    uint32_t c = 0xFFFFFFFFu;
    if (valid) {
        c = cell_of(B, x, y, z, gone);
        if (p.adapt_L > 0) p.cell[i] = c;   // the leaf count reads it back
    }
    const int lane = threadIdx.x & 63;
    const uint64_t live = __ballot(valid);
    if (live == 0) return;
    const uint32_t prev = __shfl_up(c, 1, 64);
    const bool head = valid && (lane == 0 || prev != c);
    const uint64_t H = __ballot(head);
    const uint64_t upto = (2ull << lane) - 1ull;           // lanes 0..lane
    const int my_head = 63 - __clzll((long long)(H & upto));
    const uint64_t above = H & ~upto;
    const int nvalid = __popcll(live);
    const int next = above ? __ffsll((unsigned long long)above) - 1 : nvalid;
    uint32_t base = 0;
    if (head) base = atomicAdd(&p.count[c], (unsigned int)(next - lane));
    base = (uint32_t)__shfl((int)base, my_head, 64);
    if (valid) p.slot[i] = base + (uint32_t)(lane - my_head);
}

// a1 for the state written by kmc_init (later steps bin in k_resolve).
__global__ void k_bin(Plan p)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < p.N;
    const size_t N = p.N;
    const BoxDev& B = box_of(p, valid ? i : 0u);
    bin_particle(p, i, valid, B, valid ? p.A[i] : 0.0, valid ? p.A[N + i] : 0.0, valid ? p.A[2 * N + i] : 0.0,
                 false);
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

// The eight counts of cells base..base+7 (zero beyond the last cell), with
// two 16-byte loads when all eight exist.
__device__ __forceinline__ void load_counts(const Plan& p, uint32_t base, uint32_t v[kScanItems])
{
    static_assert(kScanItems == 8, "two uint4 per thread");
    if (base + kScanItems <= p.C) {
        const uint4* cp = reinterpret_cast<const uint4*>(p.count + base);
        const uint4 a = cp[0], b = cp[1];
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) v[k] = base + k < p.C ? p.count[base + k] : 0u;
    }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(Plan p)
{
    __shared__ uint32_t lds[kScanBlock / 64 + 1];
    const uint32_t base = blockIdx.x * (uint32_t)kScanTile + threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    load_counts(p, base, v);
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) s += v[k];
    uint32_t total;
    block_exclusive_scan(s, lds, total);
    if (threadIdx.x == 0) p.partial[blockIdx.x] = total;
}

// One block of 1024 threads scans the block sums in place.  It also starts
// the step's device-side bookkeeping (recheck list, overflow pair list and
// the FP32 screen's per-box velocity bounds).
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
        p.ctl->ovf_count = 0;
        p.ctl->refined_count = 0;
        p.ctl->pool_used = 0;
    }
    for (uint32_t b = threadIdx.x; b < p.nboxes; b += blockDim.x) p.box_vmax[b] = 0u;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_down(Plan p)
{
    __shared__ uint32_t lds[kScanBlock / 64 + 1];
    const uint32_t base = blockIdx.x * (uint32_t)kScanTile + threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    load_counts(p, base, v);
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) s += v[k];
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, lds, total) + p.partial[blockIdx.x];
    uint32_t st[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        st[k] = run;
        run += v[k];
    }
    if (base + kScanItems <= p.C) {
        // 32-byte aligned runs of eight cells (the arrays are 256-byte aligned)
        uint4* sp = reinterpret_cast<uint4*>(p.start + base);
        uint4* cp = reinterpret_cast<uint4*>(p.count + base);
        sp[0] = make_uint4(st[0], st[1], st[2], st[3]);
        sp[1] = make_uint4(st[4], st[5], st[6], st[7]);
        cp[0] = make_uint4(0u, 0u, 0u, 0u);
        cp[1] = make_uint4(0u, 0u, 0u, 0u);
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            const uint32_t c = base + k;
            if (c < p.C) {
                p.start[c] = st[k];
                p.count[c] = 0u;
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) p.start[p.C] = p.N;
    if (p.adapt_L > 0) {
        // adaptive bins: this step's split level of every cell from its count;
        // split cells are listed and claim their leaf tables (one pair of
        // atomics per block, on two counters that every block shares: the
        // block's split cells take consecutive list entries and pool ranges,
        // in thread order)
        uint64_t lv = 0;
        uint32_t nsplit = 0, need = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            const uint32_t c = base + k;
            if (c < p.C) {
                const uint32_t l = split_level(v[k], p.adapt_T, p.adapt_L);
                lv |= (uint64_t)l << (8 * k);
                if (l) {
                    nsplit += 1u;
                    need += (1u << (3 * l)) + 1u;
                }
            }
        }
        const int lane = threadIdx.x & 63;
        uint32_t xs = nsplit, xn = need;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t ys = __shfl_up(xs, off, 64), yn = __shfl_up(xn, off, 64);
            if (lane >= off) {
                xs += ys;
                xn += yn;
            }
        }
        __shared__ uint32_t wsum[2][kScanBlock / 64];
        const int wid = threadIdx.x >> 6, nw = (int)(blockDim.x >> 6);
        if (lane == 63) {
            wsum[0][wid] = xs;
            wsum[1][wid] = xn;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t ts = 0, tn = 0;
            for (int w = 0; w < nw; ++w) {
                ts += wsum[0][w];
                tn += wsum[1][w];
            }
            uint32_t bs = 0, bn = 0;
            if (ts) {
                bs = atomicAdd(&p.ctl->refined_count, ts);
                bn = atomicAdd(&p.ctl->pool_used, tn);
            }
            for (int w = 0; w < nw; ++w) {   // each wave's first entry and pool offset
                const uint32_t a = wsum[0][w], b = wsum[1][w];
                wsum[0][w] = bs;
                wsum[1][w] = bn;
                bs += a;
                bn += b;
            }
        }
        __syncthreads();
        uint32_t rs = wsum[0][wid] + xs - nsplit;
        uint32_t rn = wsum[1][wid] + xn - need;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            const uint32_t l = (uint32_t)(lv >> (8 * k)) & 0xFFu;
            if (l) {
                const uint32_t c = base + k;
                p.refined[rs++] = c;
                p.pool_base[c] = rn;
                rn += (1u << (3 * l)) + 1u;
            }
        }
        if (base + kScanItems <= p.C) {
            *reinterpret_cast<uint64_t*>(p.level + base) = lv;
            *reinterpret_cast<uint64_t*>(p.mixed + base) = 0ull;
        } else {
            for (int k = 0; k < kScanItems; ++k)
                if (base + k < p.C) {
                    p.level[base + k] = (uint8_t)(lv >> (8 * k));
                    p.mixed[base + k] = 0;
                }
        }
    }
}

// Box of a global cell (the boxes' cells are consecutive, in box order).
__device__ __forceinline__ uint32_t box_of_cell(const Plan& p, uint32_t c)
{
    uint32_t lo = 0, hi = p.nboxes - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (p.boxes[mid].coff <= c) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Adaptive bins, per split cell (one wave each): clear its leaf counts and
// mark it and its 26 neighbours as cells whose particles' neighbourhoods
// are not the plain 27 cells.
__global__ __launch_bounds__(64) void k_refined_prep(Plan p)
{
    const uint32_t n = p.ctl->refined_count;
    const uint32_t lane = threadIdx.x;
    for (uint32_t k = blockIdx.x; k < n; k += gridDim.x) {
        const uint32_t c = p.refined[k];
        const uint32_t m = 1u << (3u * p.level[c]);
        const uint32_t pb = p.pool_base[c];
        for (uint32_t t = lane; t < m; t += 64u) p.pool[pb + t] = 0u;
        if (lane < 27u) {
            const BoxDev& B = p.boxes[box_of_cell(p, c)];
            const uint32_t loc = c - B.coff, NX = (uint32_t)B.nc[0], NY = (uint32_t)B.nc[1];
            int q[3] = {(int)(loc % NX), (int)((loc / NX) % NY), (int)(loc / (NX * NY))};
            const int d[3] = {(int)(lane % 3u) - 1, (int)((lane / 3u) % 3u) - 1, (int)(lane / 9u) - 1};
            bool ok = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                q[a] += d[a];
                if (q[a] < 0) { if (B.periodic[a]) q[a] += B.nc[a]; else ok = false; }
                else if (q[a] >= B.nc[a]) { if (B.periodic[a]) q[a] -= B.nc[a]; else ok = false; }
            }
            if (ok) p.mixed[B.coff + (uint32_t)q[0] + NX * ((uint32_t)q[1] + NY * (uint32_t)q[2])] = 1;
        }
    }
}

// Adaptive bins: each particle of a split cell counts itself into its leaf;
// the returned value is its rank in the leaf.  The state is in the previous
// step's leaf order, so neighbouring lanes mostly share a leaf: each run of
// equal leaves takes its ranks with one atomic issued by the run's first lane
// (as the binning does for cells).  Every lane of the wave takes part.
__global__ void k_leaf_count(Plan p)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t kNone = 0xFFFFFFFFu;
    uint32_t key = kNone;   // the particle's leaf counter in the pool (none: its cell is not split)
    if (i < p.N) {
        const uint32_t c = p.cell[i];
        const uint32_t lvl = p.level[c];
        if (lvl != 0u) {
            const size_t N = p.N;
            key = p.pool_base[c] + leaf_code(box_of(p, i), p.adapt_L, lvl, p.A[i], p.A[N + i], p.A[2 * N + i]);
        }
    }
    const int lane = threadIdx.x & 63;
    const bool counted = key != kNone;
    const uint32_t prev = __shfl_up(key, 1, 64);
    const bool cont = counted && lane > 0 && prev == key;   // same leaf as the lane before
    const uint64_t H = __ballot(counted && !cont);          // first lanes of runs
    const uint64_t E = __ballot(!cont);                     // lanes that do not continue a run
    const uint64_t upto = (2ull << lane) - 1ull;            // lanes 0..lane
    const uint64_t after = E & ~upto;
    const int next = after ? __ffsll((unsigned long long)after) - 1 : 64;
    uint32_t base = 0;
    if (counted && !cont) base = atomicAdd(&p.pool[key], (unsigned int)(next - lane));
    const int my_head = counted ? 63 - __clzll((long long)(H & upto)) : lane;
    base = (uint32_t)__shfl((int)base, my_head, 64);
    if (counted) p.leaf_slot[i] = base + (uint32_t)(lane - my_head);
}

// Adaptive bins, per split cell (one wave each): the exclusive prefix of its
// leaf counts in place (leaf starts relative to the cell's start), then the
// cell's count after the last.
__global__ __launch_bounds__(64) void k_leaf_scan(Plan p)
{
    const uint32_t n = p.ctl->refined_count;
    const int lane = threadIdx.x;
    for (uint32_t k = blockIdx.x; k < n; k += gridDim.x) {
        const uint32_t c = p.refined[k];
        const uint32_t m = 1u << (3u * p.level[c]);
        uint32_t* t = p.pool + p.pool_base[c];
        const uint32_t per = m > 64u ? m / 64u : 1u;    // entries per lane (m is 8, 64 or 512)
        const uint32_t b0 = (uint32_t)lane * per;
        uint32_t v[8];
        uint32_t sum = 0;
#pragma unroll
        for (uint32_t e = 0; e < 8u; ++e) {
            v[e] = (e < per && b0 + e < m) ? t[b0 + e] : 0u;
            sum += v[e];
        }
        uint32_t x = sum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        uint32_t run = x - sum;
#pragma unroll
        for (uint32_t e = 0; e < 8u; ++e) {
            if (e < per && b0 + e < m) t[b0 + e] = run;
            run += v[e];
        }
        if (lane == 63) t[m] = x;
    }
}

// --------------------------------------------------------------------------
// a3: cell-sorted copy of the state as 48-byte records (ids and kinds beside
// them); for the FP32 screen also the per-block bound on |fl32(v_k)| from
// which the screen's error bounds per box are made.
// --------------------------------------------------------------------------

template <bool F32>
__global__ void k_scatter(Plan p)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < p.N;
    const size_t N = p.N;
    float vm = 0.f;
    bool outside = false;
    double vx = 0.0, vy = 0.0, vz = 0.0;
    // the particle's box; one box (no per-particle index): the same for the
    // whole grid, read through scalar loads
    auto body = [&](const BoxDev& B) {
        const uint32_t id = p.idA[i];
        P64 r;
        r.x = p.A[i];
        r.y = p.A[N + i];
        r.z = p.A[2 * N + i];
        const uint32_t c = p.adapt_L > 0 ? p.cell[i] : cell_of(B, r.x, r.y, r.z, (id & kGone) != 0u);
        uint32_t d = p.start[c] + p.slot[i];
        if (p.adapt_L > 0) {
            // adaptive bins: leaf-sorted inside a split cell
            const uint32_t lvl = p.level[c];
            if (lvl) {
                const uint32_t code = leaf_code(B, p.adapt_L, lvl, r.x, r.y, r.z);
                d = p.start[c] + p.pool[p.pool_base[c] + code] + p.leaf_slot[i];
            }
        }
        r.vx = vx = p.A[3 * N + i];
        r.vy = vy = p.A[4 * N + i];
        r.vz = vz = p.A[5 * N + i];
        p.B[d] = r;
        p.idB[d] = id;
        if (p.spA) p.spB[d] = p.spA[i];
        if (id & kGone) vx = vy = vz = 0.0;   // not in the gas: no part in the adaptive step
        if (F32) {
            vm = fmaxf(fabsf((float)r.vx), fmaxf(fabsf((float)r.vy), fabsf((float)r.vz)));

            // The screen's error bounds take every particle to lie inside the
            // cell it is binned in (up to a slack of 1e-9 of a cell edge).  A
            // particle outside its box's grid (placed there, or moved more
            // than a box length in one step) is binned in an end cell; the
            // step's partners then come from the whole-step FP64 search
            // instead.  Rounding-level excursions (a sphere's mirror image
            // just past a face of a grid that fits it exactly) stay within
            // the slack and are ignored.
            if (!(id & kGone)) {
                outside = !(r.x >= B.lo[0] && r.x <= B.hi[0] && r.y >= B.lo[1] && r.y <= B.hi[1] &&
                            r.z >= B.lo[2] && r.z <= B.hi[2]);
                if (outside) {
                    const double t0 = 1e-11 * B.h[0], t1 = 1e-11 * B.h[1], t2 = 1e-11 * B.h[2];
                    outside = !(r.x >= B.lo[0] - t0 && r.x <= B.hi[0] + t0 && r.y >= B.lo[1] - t1 &&
                                r.y <= B.hi[1] + t1 && r.z >= B.lo[2] - t2 && r.z <= B.hi[2] + t2);
                }
            }
        }
    };
    if (valid) {
        if (p.boxidx) body(p.boxes[p.boxidx[i]]);
        else body(p.boxes[0]);
    }
    __shared__ float wmax[16];
    __shared__ unsigned long long wv2[16];
    if (F32) {
        if (__ballot(outside) && (threadIdx.x & 63) == 0) atomicOr(&p.ctl->overflow, 1u);
        // per-block maximum of |fl32(v_k)|; k_vmax_reduce folds the blocks of each box
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) vm = fmaxf(vm, __shfl_xor(vm, off, 64));
        if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = vm;
    }
    if (p.dt_rule == KMC_DT_ADAPTIVE) {
        // adaptive time step: max |v|^2 per box.  Non-negative doubles order
        // like their bit patterns, so the maximum is exact in any order.  The
        // block folds its particles that share the box of its first particle
        // (k_adapt_dt reads the partial); any others go to their box directly.
        const uint32_t first = blockIdx.x * blockDim.x;
        const uint32_t b0 = p.boxidx ? p.boxidx[first] : 0u;
        unsigned long long q = 0ull;
        if (valid) {
            const double v2 = fma(vz, vz, fma(vy, vy, vx * vx));
            const unsigned long long bits = (unsigned long long)__double_as_longlong(v2);
            const uint32_t bi = p.boxidx ? p.boxidx[i] : 0u;
            if (bi == b0) q = bits;
            else atomicMax(&p.box_v2[bi], bits);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_xor(q, off, 64);
            q = o > q ? o : q;
        }
        if ((threadIdx.x & 63) == 0) wv2[threadIdx.x >> 6] = q;
    }
    if (F32 || p.dt_rule == KMC_DT_ADAPTIVE) {
        __syncthreads();
        if (threadIdx.x == 0) {
            const int nw = (int)(blockDim.x >> 6);
            if (F32) {
                float m = 0.f;
                for (int w = 0; w < nw; ++w) m = fmaxf(m, wmax[w]);
                p.vmax_part[blockIdx.x] = m;
            }
            if (p.dt_rule == KMC_DT_ADAPTIVE) {
                unsigned long long m = 0ull;
                for (int w = 0; w < nw; ++w) m = wv2[w] > m ? wv2[w] : m;
                p.v2_part[blockIdx.x] = m;
            }
        }
    }
}

// This step's time step of every box (one block per box), from the maxima
// k_scatter gathered: dt = min(cap, (C dx) / sqrt(max |v|^2)) under the
// adaptive rule, the configured dt otherwise; also the simulated time.
__global__ __launch_bounds__(256) void k_adapt_dt(Plan p)
{
    __shared__ unsigned long long red[256];
    const uint32_t b = blockIdx.x;
    BoxDev& B = p.boxes[b];
    unsigned long long m = 0ull;
    if (p.dt_rule == KMC_DT_ADAPTIVE && B.n > 0) {
        // the scatter blocks whose first particle lies in this box
        const uint32_t blk = (uint32_t)p.block;
        const uint32_t k0 = (B.poff + blk - 1) / blk, k1 = (B.poff + B.n - 1) / blk;
        for (uint32_t k = k0 + threadIdx.x; k <= k1; k += blockDim.x) {
            const unsigned long long v = p.v2_part[k];
            m = v > m ? v : m;
        }
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (uint32_t w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = red[threadIdx.x + w] > red[threadIdx.x] ? red[threadIdx.x + w] : red[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (p.dt_rule == KMC_DT_ADAPTIVE) {
            const unsigned long long o = p.box_v2[b];
            const unsigned long long mm = o > red[0] ? o : red[0];
            p.box_v2[b] = 0ull;
            const double v2 = __longlong_as_double((long long)mm);
            double dt = B.dt_cap;
            if (v2 > 0.0) {
                const double a = (p.dt_factor * B.dx) / sqrt(v2);
                if (a < dt) dt = a;
            }
            B.dt = dt;
            B.dt_32 = (float)dt;
        }
        B.time = B.time + B.dt;
    }
}

// Per-box maximum of the scatter blocks' partials: kVmaxSplit blocks per
// box, one atomic each (non-negative floats order like their bit patterns).
constexpr uint32_t kVmaxSplit = 32;

__global__ __launch_bounds__(256) void k_vmax_reduce(Plan p)
{
    __shared__ float red[256];
    const uint32_t b = blockIdx.x / kVmaxSplit, part = blockIdx.x % kVmaxSplit;
    const BoxDev& B = p.boxes[b];
    float vm = 0.f;
    if (B.n > 0) {
        const uint32_t blk = (uint32_t)p.block;
        const uint32_t first = B.poff / blk, last = (B.poff + B.n - 1) / blk;
        for (uint32_t k = first + part * blockDim.x + threadIdx.x; k <= last; k += kVmaxSplit * blockDim.x)
            vm = fmaxf(vm, p.vmax_part[k]);
    }
    red[threadIdx.x] = vm;
    __syncthreads();
    for (uint32_t w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0] > 0.f) atomicMax(&p.box_vmax[b], __float_as_uint(red[0]));
}

// --------------------------------------------------------------------------
// a4: DCA partner search.
//
// The pair quantities are symmetric under exchange of the two particles
// (r, g and r x g change sign, b, g2, c2 do not), so every unordered pair is
// tested once, from the particle whose cell comes first in a half
// neighbourhood: its own row from the particle onwards through cell cx+1,
// the row y+1 (cells cx-1..cx+1) and the three rows z+1 (y-1..y+1).  A lane
// keeps the pairs that pass; at the end of the wave it decides them exactly
// in FP64, writes the best of them (its forward best) and posts each
// acceptable pair, with its key, to the other particle's candidate list.  A
// per-particle finish pass then takes the (key, id) minimum of the forward
// best and the list.
//
// One wave (= one block of 64 threads) takes 64 consecutive cell-sorted
// particles, one per lane.  Lanes whose particles share a cell row form a
// group; for each of the five half-neighbourhood rows the group's window of
// cells is a contiguous range of the sorted arrays, which the wave stages
// into LDS in chunks with coalesced loads.  Each lane then tests its own
// sub-range of the window from LDS.
// --------------------------------------------------------------------------

// Row of sorted particle i's kind in the kind-pair tables (kMaxKinds * its
// kind; 0 for one kind of particle).
__device__ __forceinline__ uint32_t kind_row(const Plan& p, uint32_t i)
{
    return p.nspecies ? (uint32_t)p.spB[i] * (uint32_t)kMaxKinds : 0u;
}

// Squared interaction diameter of the pair of sorted particles (i, j): the
// box's D2 for one kind of particle, else (radius_s + radius_t)^2 of their
// kinds.
__device__ __forceinline__ double pair_D2(const Plan& p, const BoxDev& B, uint32_t row_i, uint32_t j)
{
    return p.nspecies ? p.sp_D2[row_i + p.spB[j]] : B.D2;
}

// Relative position of candidate j seen from i in FP64 with the image fixed
// by the two cells, exactly as in the search.
__device__ __forceinline__ void rel64(const BoxDev& B, const P64& me, const P64& q, double r[3])
{
    const double xi[3] = {me.x, me.y, me.z}, xj[3] = {q.x, q.y, q.z};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int ci = cell1(xi[k], B.lo[k], B.inv_h[k], B.nc[k]);
        const int cj = cell1(xj[k], B.lo[k], B.inv_h[k], B.nc[k]);
        const int w = wrap_of(ci, cj, B.nc[k], B.periodic[k]);
        r[k] = xj[k] - xi[k];
        if (w != 0) r[k] = r[k] + (double)w * B.L[k];
    }
}

// Candidate lists: per particle a count and up to kSlots entries (sorted
// index of the other particle and the pair's FP64 key c2/g2, which is the
// same from both sides, or +inf for a pair the FP32 screen kept and the exact
// test rejected); entry k of particle i lives at [k * N + i].
__device__ __forceinline__ void post_candidate(const Plan& p, uint32_t i, uint32_t j, double key)
{
    const uint32_t k = atomicAdd(&p.sl_cnt[i], 1u);
    if (k < (uint32_t)kSlots) {
        SlotEntry e;
        e.key = key;
        e.j = j;
        e.pad_ = 0u;
        p.sl[(size_t)k * p.N + i] = e;
    }
}

// The definition's exact FP64 decision for the pair (i, j) seen from i (the
// image from the two cells), and its key when acceptable.
__device__ __forceinline__ bool exact_key(const Plan& p, const BoxDev& B, uint32_t i, const P64& me, uint32_t j,
                                          double& key)
{
    const P64 q = p.B[j];
    double r[3];
    rel64(B, me, q, r);
    const PairQ pq = pair_q(r[0], r[1], r[2], q.vx - me.vx, q.vy - me.vy, q.vz - me.vz);
    if (!accept(pq, pair_D2(p, B, kind_row(p, i), j), B.dt)) return false;
    key = pq.c2 / pq.g2;
    return true;
}

// Pairs a lane found, kept until the end of the wave's search (the sorted
// indices in LDS, the image shifts in a register: a global atomic or a
// division inside the search loop would stall the whole wave); a lane that
// finds more than kReg appends the excess to the step's overflow pair list
// (one counter, handled by k_distribute_overflow), or raises the overflow
// flag when that list is full (whole-step FP64 fallback).
constexpr int kReg = 4;

__device__ __forceinline__ uint32_t wcode(int wx, int wy, int wz)
{
    return (uint32_t)(wx + 1) | ((uint32_t)(wy + 1) << 2) | ((uint32_t)(wz + 1) << 4);
}
constexpr uint32_t kNoImage = 0x15u;   // wcode(0, 0, 0)

struct Found {
    uint32_t* sj; // this lane's kept indices in LDS: pair k at sj[64 k] (one store per pair
                  // instead of a select over register slots)
    uint32_t w;   // image shift of pair k in bits 6k..6k+5: (wx+1) | (wy+1) << 2 | (wz+1) << 4;
                  // bit 31: the overflow pair list was full, nothing more is recorded
    uint32_t sh;  // 6 n
    int n;
    __device__ __forceinline__ void add(const Plan& p, uint32_t i, uint32_t jj, uint32_t wcode)
    {
        if (n < kReg) {
            sj[64 * n] = jj;
            w |= wcode << sh;
            sh += 6u;
            ++n;
        } else if (!(w >> 31)) {
            const uint32_t idx = atomicAdd(&p.ctl->ovf_count, 1u);
            if (idx < p.ovf_cap) {
                p.ovf[idx] = make_uint2(i, jj);
            } else {
                // list full: the whole-step FP64 search decides this step, so
                // the lane records nothing more (the top bit of w, which the
                // image shifts of kReg pairs leave free, marks it)
                atomicOr(&p.ctl->overflow, 1u);
                w |= 0x80000000u;
            }
        }
    }
    // Decide the kept pairs exactly in FP64 (the FP32 screen keeps pairs it
    // could not reject), write i's best among them (its forward best) and
    // post each kept pair to the other particle's list (key +inf when the
    // exact test rejects it).  The image shift is the one the search used
    // (that of the two cells).  All lanes take the same path: list slots
    // claimed, records loaded, the arithmetic, then the list entries
    // written.  Returns the number of pairs examined (statistics).
    // BATCH records are loaded at a time; SKIP: no loads for empty slots
    // (otherwise branch-free, loading the own record for them) -- measured
    // per precision
    // K: particles of several kinds (the pair's D2 from the kind table).
    template <int BATCH, bool SKIP, bool K>
    __device__ __forceinline__ uint32_t flush(const Plan& p, uint32_t i, const P64& me, const BoxDev& B)
    {
        const uint32_t row = K ? kind_row(p, i) : 0u;
        uint32_t j[kReg];
#pragma unroll
        for (int k = 0; k < kReg; ++k) j[k] = k < n ? sj[64 * k] : 0u;
        // list slots of the kept pairs claimed first: the atomics are in
        // flight while the records load and the pairs are decided (a pair the
        // FP64 test then rejects leaves an entry with key +inf, which never
        // wins in the finish)
        uint32_t slot[kReg];
#pragma unroll
        for (int k = 0; k < kReg; ++k) slot[k] = k < n ? atomicAdd(&p.sl_cnt[j[k]], 1u) : (uint32_t)kSlots;
        double key[kReg];
        bool acc[kReg];
#pragma unroll
        for (int k = 0; k < kReg; ++k) {
            acc[k] = false;
            key[k] = __builtin_inf();
        }
#pragma unroll
        for (int h = 0; h < kReg; h += BATCH) {
            if (!SKIP || h < n) {
                P64 q[BATCH];
#pragma unroll
                for (int e = 0; e < BATCH; ++e) q[e] = p.B[h + e < n ? j[h + e] : (SKIP ? j[h] : i)];
#pragma unroll
                for (int e = 0; e < BATCH; ++e) {
                    const int k = h + e;
                    const uint32_t c = w >> (6 * k);
                    const int wx = (int)(c & 3u) - 1, wy = (int)((c >> 2) & 3u) - 1, wz = (int)((c >> 4) & 3u) - 1;
                    double rx = q[e].x - me.x, ry = q[e].y - me.y, rz = q[e].z - me.z;
                    if (wx != 0) rx = rx + (double)wx * B.L[0];
                    if (wy != 0) ry = ry + (double)wy * B.L[1];
                    if (wz != 0) rz = rz + (double)wz * B.L[2];
                    const PairQ pq = pair_q(rx, ry, rz, q[e].vx - me.vx, q[e].vy - me.vy, q[e].vz - me.vz);
                    acc[k] = k < n && accept(pq, K ? pair_D2(p, B, row, j[k]) : B.D2, B.dt);
                    key[k] = acc[k] ? pq.c2 / pq.g2 : __builtin_inf();
                }
            }
        }
        double best_key = __builtin_inf();
        int32_t best = -1;
#pragma unroll
        for (int k = 0; k < kReg; ++k) {
            if (acc[k] && (best < 0 || key[k] < best_key ||
                           (key[k] == best_key && p.idB[j[k]] < p.idB[best]))) {
                best_key = key[k];
                best = (int32_t)j[k];
            }
        }
#pragma unroll
        for (int k = 0; k < kReg; ++k) {
            if (slot[k] < (uint32_t)kSlots) {
                SlotEntry e;
                e.key = acc[k] ? key[k] : __builtin_inf();
                e.j = i;
                e.pad_ = 0u;
                p.sl[(size_t)slot[k] * p.N + j[k]] = e;
            }
        }
        p.fb_key[i] = best_key;
        p.fb_j[i] = best;
        return (uint32_t)n;
    }
};

// Per-group context of the search (the FP64 search needs none).
struct NoGroup {
};

// Running (key, id) minimum of one lane in the full-neighbourhood search.
struct Best {
    double key;
    uint32_t id;
    int32_t j;
    uint32_t accepted;   // acceptable pairs seen (statistics)
    uint32_t screened;   // FP32 screen: pairs decided in FP64
    __device__ __forceinline__ void offer(double k, uint32_t idj, uint32_t jj)
    {
        accepted += 1u;
        if (k < key || (k == key && idj < id)) {
            key = k;
            id = idj;
            j = (int32_t)jj;
        }
    }
};

// Pairs the FP32 screen keeps in the full-neighbourhood search, decided in
// FP64 once the tile's rows are done (a record gather inside the pair loop
// stalls the whole wave); a lane's pairs beyond kDefer are decided at once.
constexpr int kDefer = 4;
struct Deferred {
    uint32_t* sj;   // this lane's slots in LDS: sorted index of pair k at sj[64 k],
                    // its image shift (wcode) at sj[64 (kDefer + k)]
    int n;
};

// Tile shape of a search kernel: W records staged per LDS chunk, and the
// waves per SIMD the half- and full-neighbourhood searches are compiled for
// (fewer waves leave more registers per wave).  The launch autotuner picks
// one of three shapes per precision (kmc_config.tile); the results do not
// depend on it.
template <int W_, int HALF_WAVES, int FULL_WAVES>
struct Tile {
    static constexpr int W = W_;
    static constexpr int kWaves = HALF_WAVES;
    static constexpr int kFullWaves = FULL_WAVES;
};
// FP64: 96 records per chunk (4.5 KiB) by default
using TileF64_0 = Tile<96, 6, 5>;
using TileF64_1 = Tile<64, 6, 5>;
using TileF64_2 = Tile<160, 5, 4>;
// FP32 screen: 128 records (4 KiB) by default (measured against 96, 160,
// 192 and 256 on the headline gas)
using TileF32_0 = Tile<128, 6, 5>;
using TileF32_1 = Tile<64, 6, 5>;
using TileF32_2 = Tile<256, 5, 4>;

// K: particles of several kinds (the pair's D2 from the per-kind-pair table,
// staged in LDS with each record's kind); otherwise the box's D2.
template <bool K, class T = TileF64_0>
struct PolF64 {
    static constexpr int W = T::W;
    static constexpr bool kScreen = false;
    static constexpr bool kKinds = K;
    static constexpr int kFlushBatch = 2;
    static constexpr bool kFlushSkipEmpty = true;
    static constexpr int kWaves = T::kWaves;
    static constexpr int kFullWaves = T::kFullWaves;
    struct Lds {
        P64 rec[W];
        uint8_t kind[K ? W : 1];
        double d2[K ? kMaxKinds * kMaxKinds : 1];
    };
    struct Own {
        P64 me;
        uint32_t row;   // K: kMaxKinds * own kind
    };
    using Group = NoGroup;
    __device__ static void begin_group(const Plan&, const BoxDev&, Own&, Group&, int, int, int, int, int, uint32_t,
                                       bool) {}
    // per-group LDS tables, written before the group's first staging barrier
    __device__ static void group_lds(Lds& l, const Plan& p, uint32_t, int lane)
    {
        if (K) l.d2[lane] = p.sp_D2[lane];
    }
    __device__ static void load_own(const Plan& p, uint32_t i, Own& o, double& x, double& y, double& z)
    {
        o.me = p.B[i];
        o.row = K ? (uint32_t)p.spB[i] * (uint32_t)kMaxKinds : 0u;
        x = o.me.x; y = o.me.y; z = o.me.z;
    }
    __device__ static P64 self64(const Plan&, uint32_t, const Own& o) { return o.me; }
    __device__ static void stage(Lds& l, uint32_t t, const Plan& p, uint32_t j, const BoxDev&, const Group&,
                                 int, int, int, int, int)
    {
        l.rec[t] = p.B[j];
        if (K) l.kind[t] = p.spB[j];
    }
    template <bool SH>
    __device__ static void scan(const Plan& p, const Lds& l, uint32_t c0, uint32_t j0, uint32_t j1, uint32_t i,
                                const Own& o, const BoxDev& B, const Group&, int wx, int wy, int wz, int, int,
                                Found& f)
    {
        const double sx = (double)wx * B.L[0], sy = (double)wy * B.L[1], sz = (double)wz * B.L[2];
        const double D2 = B.D2, dt = B.dt;
        for (uint32_t j = j0; j < j1; ++j) {
            const P64 q = l.rec[j - c0];
            double rx = q.x - o.me.x, ry = q.y - o.me.y, rz = q.z - o.me.z;
            if (SH) { rx = rx + sx; ry = ry + sy; rz = rz + sz; }
            const PairQ pq = pair_q(rx, ry, rz, q.vx - o.me.vx, q.vy - o.me.vy, q.vz - o.me.vz);
            const double d2 = K ? l.d2[o.row + l.kind[j - c0]] : D2;
            if (accept(pq, d2, dt)) f.add(p, i, j, wcode(wx, wy, wz));
        }
    }
    // full neighbourhood: running (key, id) minimum over the acceptable pairs
    // (the particle itself has g2 = 0 and is never accepted)
    template <bool SH>
    __device__ static void scan_best(const Plan&, const Lds& l, const uint32_t* lid, uint32_t c0, uint32_t j0,
                                     uint32_t j1, uint32_t, const Own& o, const BoxDev& B, const Group&, int wx,
                                     int wy, int wz, int, int, Best& best, Deferred&)
    {
        const double sx = (double)wx * B.L[0], sy = (double)wy * B.L[1], sz = (double)wz * B.L[2];
        const double D2 = B.D2, dt = B.dt;
        for (uint32_t j = j0; j < j1; ++j) {
            const P64 q = l.rec[j - c0];
            double rx = q.x - o.me.x, ry = q.y - o.me.y, rz = q.z - o.me.z;
            if (SH) { rx = rx + sx; ry = ry + sy; rz = rz + sz; }
            const PairQ pq = pair_q(rx, ry, rz, q.vx - o.me.vx, q.vy - o.me.vy, q.vz - o.me.vz);
            const double d2 = K ? l.d2[o.row + l.kind[j - c0]] : D2;
            if (accept(pq, d2, dt)) best.offer(pq.c2 / pq.g2, lid[j - c0], j);
        }
    }
    // adaptive bins: the staged candidates t = u, u + kk, ... (< n) against
    // owner io; candidate t is sorted particle lj[t] seen with the periodic
    // image of code lw[t]
    __device__ static void scan_adapt(const Plan&, const Lds& l, const uint32_t* lid, const uint32_t* lj,
                                      const uint32_t* lw, uint32_t n, uint32_t u, uint32_t kk, uint32_t io,
                                      const Own& o, const BoxDev& B, const Group&, Best& best)
    {
        const double D2 = B.D2, dt = B.dt;
        for (uint32_t t = u; t < n; t += kk) {
            const uint32_t j = lj[t];
            if (j == io) continue;
            const P64 q = l.rec[t];
            double rx = q.x - o.me.x, ry = q.y - o.me.y, rz = q.z - o.me.z;
            const uint32_t w = lw[t];
            if (w != kNoImage) {
                const int wx = (int)(w & 3u) - 1, wy = (int)((w >> 2) & 3u) - 1, wz = (int)((w >> 4) & 3u) - 1;
                if (wx != 0) rx = rx + (double)wx * B.L[0];
                if (wy != 0) ry = ry + (double)wy * B.L[1];
                if (wz != 0) rz = rz + (double)wz * B.L[2];
            }
            const PairQ pq = pair_q(rx, ry, rz, q.vx - o.me.vx, q.vy - o.me.vy, q.vz - o.me.vz);
            const double d2 = K ? l.d2[o.row + l.kind[t]] : D2;
            if (accept(pq, d2, dt)) best.offer(pq.c2 / pq.g2, lid[t], j);
        }
    }
};

// FP32 screen.  Positions are rounded to FP32 relative to the centre X0 of
// the group's neighbourhood (periodic images added in FP64 first), so their
// rounding error is u times the neighbourhood size, not the box size.  The
// screen tests the Lagrange form d_min^2 g2 = |r|^2 g2 - b^2 (cheaper than the
// cross product) and drops a pair only when the FP64 definition is certain to
// reject it; every pair it keeps is decided exactly in FP64 afterwards.
//
// The bounds depend on how far a group's neighbourhood reaches along x.  A
// screened group of at most span_cells(c) cells uses the thresholds of class
// c (k_screen_bounds computes each class per box), so dense rows keep tight
// bounds while the lanes of a sparse row (under one particle per cell),
// hundreds of cells apart, share looser ones; the search splits rows wider
// than the last class.
__host__ __device__ constexpr int span_cells(int c) { return 64 << (2 * c); }
constexpr int kScreenGroupCells = span_cells(kSpanClasses - 1);

__device__ __forceinline__ uint32_t span_class(int cells)
{
    uint32_t c = 0;
    while (c + 1 < (uint32_t)kSpanClasses && cells > span_cells((int)c)) ++c;
    return c;
}

struct ScreenGroup {
    double X0[3];
    ScreenBounds t;
};

// Bounds on |screen value - FP64 definition value| for every neighbour pair
// of any search group of the box (forward error analysis, Higham 2002,
// ch. 3).  Inputs: |r_k| <= R_k = 2 h_k; FP32 position errors
// e_r,k = u (2 P_k + 2 R_k) with positions relative to the group centre X0
// (a group of class c spans at most s = span_cells(c) cells along x, so
// |x - X0| <= P_x = (s/2 + 1) h_x, P_y = 1.5 h_y, P_z = 1.5 h_z) plus the
// FP64 definition's own input rounding; velocity-difference error
// e_g = 4 u V.
// With q = sqrt(g2_hat) (kappa q bounds every |g_hat_k|):
//   |db|   <= b0 + b1 q
//   |dg2|  <= g0 + g1 q + g2c q^2
//   |dm2|  <= P0 + P1 q + P2 q^2          (m2 = -b - dt g2)
//   |dm3|  <= A0 + A1 q + A2 q^2          (m3 = (|r|^2 - D2) g2 - b^2, Lagrange form
//                                          of the definition's c2 - D2 g2)
// and q <= (q^2 / G0 + G0) / 2 for any G0 > 0 makes each bound affine in
// g2_hat.  gamma terms cover the rounding of every sum and product in both
// precisions; the guard factor scales the result.
// The bound itself, for a screen of unit roundoff u: er[k] bounds the error
// of the screen's r_k (including the FP64 definition's own input rounding),
// R[k] bounds |r_k|, eg the error of each g_k, D2 and dt are the criteria's
// constants in the screen's units, G0 > 0 the AM-GM point, f the guard
// factor.  t = {b0, b1, t0, t1, c0, c1, g0, g1} of the affine thresholds.
__device__ __forceinline__ void screen_bound(double u, const double er[3], const double Rk[3], double eg, double D2,
                                             double dt, double G0, double f, double t[8])
{
    const double u64 = 0x1.0p-53;
    const double g3 = 3.0 * u / (1.0 - 3.0 * u) + 3.0 * u64 / (1.0 - 3.0 * u64);
    const double kap = 1.0 + g3;
    double SE = 0, SRE = 0, RR = 0, Err = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        SE += er[k];
        SRE += Rk[k] + er[k];
        RR += (Rk[k] + er[k]) * (Rk[k] + er[k]);
        Err += 2.0 * Rk[k] * er[k] + er[k] * er[k];
    }
    Err += g3 * RR;
    const double Rn = sqrt(RR) * (1.0 + 1e-12);
    const double s3 = 1.7320508075688774;     // >= sqrt(3)
    const double b0 = eg * (SRE + SE), b1 = kap * (SE + g3 * SRE);
    const double g0 = 3.0 * eg * eg, g1 = 2.0 * s3 * kap * eg, g2c = g3 * kap * kap;
    const double Et = Err + u * D2 + u * (RR + D2);
    const double Tm = RR + D2 + Et;
    const double A2 = 2.0 * Rn * kap * b1 + b1 * b1 + u * RR * kap * kap * (1.0 + g3) * (1.0 + g3) + Tm * g2c +
                      Et * (1.0 + g2c) + 128.0 * u64 * (RR + D2) * kap * kap;
    const double A1 = 2.0 * Rn * (kap * b0 + s3 * eg * b1) + 2.0 * b0 * b1 + Tm * g1 + Et * g1;
    const double A0 = 2.0 * Rn * s3 * eg * b0 + b0 * b0 + Tm * g0 + Et * g0 + 384.0 * u64 * (RR + D2) * eg * eg;
    const double dtf = dt * (1.0 + 2.0 * u64);
    const double P0 = b0 + dtf * g0, P1 = b1 + dtf * g1, P2 = dtf * g2c + (u + u64) * dt;
    t[0] = f * (b0 + 0.5 * b1 * G0);
    t[1] = f * (0.5 * b1 / G0);
    t[2] = f * (P0 + 0.5 * P1 * G0);
    t[3] = f * (P2 + 0.5 * P1 / G0);
    t[4] = f * (A0 + 0.5 * A1 * G0);
    t[5] = f * (A2 + 0.5 * A1 / G0);
    t[6] = f * (g0 + 0.5 * g1 * G0);
    t[7] = f * (g2c + 0.5 * g1 / G0);
}

// Folded D2 constant of the m3 test for the criterion's FP32 D2 (see below).
__device__ __forceinline__ float fold_kD2(double D2_32, double tc1, double RRb)
{
    const double u = 0x1.0p-24;
    return tc1 > 0.0 ? (float)((D2_32 + tc1 + 2.0 * u * (RRb + D2_32 + tc1)) * (1.0 + 2e-6)) : (float)D2_32;
}

// Returns tc1 and RRb (for fold_kD2 with other D2 values of the box).  With
// particle kinds B.D2 is the largest pair value; every bound term grows with
// D2, so the bounds hold for every pair of kinds.
__device__ __forceinline__ void screen_thresholds(const BoxDev& B, const double P[3], double V, float guard,
                                                  ScreenBounds& g, double& tc1, double& RRb)
{
    const double u = 0x1.0p-24, u64 = 0x1.0p-53;
    const double eg = 4.0001 * u * V + 4.0 * u64 * V;
    double er[3], Rk[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        Rk[k] = B.rmax[k];
        er[k] = u * (2.0 * P[k] + 2.0 * Rk[k]) * (1.0 + 1e-5) + 2.0 * u64 * (Rk[k] + 2.0 * B.L[k]);
    }
    const double G0 = V > 0.0 ? 0.25 * V : 1.0;
    const double f = (double)guard * (1.0 + 1e-5) * (1.0 + 1e-6);
    double t[8];
    screen_bound(u, er, Rk, eg, B.D2, B.dt, G0, f, t);
    // thresholds rounded to FP32 stay above the bounds (f carries 1e-5 of slack)
    g.tb0 = (float)t[0];
    g.tb1 = (float)t[1];
    g.tt0 = (float)t[2];
    g.tt1 = (float)t[3];
    g.tc0 = (float)t[4];
    g.tc1 = (float)t[5];
    // Folded constants, rounded up (the factor 1 + 2e-6 exceeds every rounding
    // here).  m2: -b - kdt g2 <= -b - (dt + tt1) g2 for kdt >= dt + tt1, and the
    // screen's one rounding of the FMA is monotone.  m3: replacing the
    // subtrahend D2 of the screen's fl(|r|^2 - D2) by kD2 lowers that value by
    // at least kD2 - D2 - u (|fl(|r|^2) - kD2| + |fl(|r|^2) - D2|), which is >= tc1
    // when kD2 (1 - u) >= D2 (1 + u) + tc1 + 2 u RRb with RRb >= fl(|r|^2).
    // Without bounds (guard 0) the constants are the criteria's own.
    const double dt32 = (double)B.dt_32;
    RRb = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) RRb += (Rk[k] + er[k]) * (Rk[k] + er[k]);
    RRb *= 1.0 + 1e-5;
    tc1 = t[5];
    g.kdt = t[3] > 0.0 ? (float)((dt32 + t[3]) * (1.0 + 2e-6)) : B.dt_32;
    g.kD2 = fold_kD2((double)B.D2_32, t[5], RRb);
}

__global__ void k_screen_bounds(Plan p)
{
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= p.nboxes) return;
    const BoxDev& B = p.boxes[b];
    const double V = (double)__uint_as_float(p.box_vmax[b]) * (1.0 + 3.0 * 0x1.0p-24);
    // The bounds take FP32 arithmetic to neither overflow nor lose to
    // underflow more than a small fraction of them: cell edges in
    // [2^-40, 2^40], the largest speed 0 or in [2^-40, 2^40], the pair test's
    // largest products (|r|^2 g2 <= 144 h^2 V^2 and the folded thresholds
    // times g2 <= 12 V^2) below 2^120, every threshold finite.  Outside that
    // range this step's partners come from the whole-step FP64 search.
    const double lo_s = 0x1.0p-40, hi_s = 0x1.0p40, big = 0x1.0p120;
    bool safe = V == 0.0 || (V >= lo_s && V <= hi_s);
    double hmax = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        safe = safe && B.h[k] >= lo_s && B.h[k] <= hi_s;
        hmax = fmax(hmax, B.h[k]);
    }
    const double g2max = 12.0 * V * V;
    safe = safe && 256.0 * hmax * hmax * g2max < big;
    for (int c = 0; c < kSpanClasses; ++c) {
        // neighbourhood of a group of this class in cells (its own cells and
        // one on each side)
        const double cells[3] = {(double)(span_cells(c) + 2), 3.0, 3.0};
        double P[3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            P[k] = 0.5 * cells[k] * B.h[k] * (1.0 + 1e-9) + 1e-12 * (fabs(B.lo[k]) + fabs(B.hi[k]) + 2.0 * B.L[k]);
        double tc1, RRb;
        ScreenBounds g;
        screen_thresholds(B, P, V, p.guard, g, tc1, RRb);
        p.box_sb[(size_t)b * kSpanClasses + c] = g;
        const float th[8] = {g.tb0, g.tb1, g.tt0, g.tt1, g.tc0, g.tc1, g.kdt, g.kD2};
#pragma unroll
        for (int k = 0; k < 8; ++k) safe = safe && isfinite(th[k]) && (double)fabsf(th[k]) * g2max < big;
        if (p.nspecies > 0) {
            // the folded constant of each pair of kinds, from the pair's own D2
            // rounded to FP32 (entries of absent kinds are never read)
            float* tab = p.box_kD2 + ((size_t)b * kSpanClasses + c) * (kMaxKinds * kMaxKinds);
            for (int e = 0; e < kMaxKinds * kMaxKinds; ++e) {
                tab[e] = fold_kD2((double)(float)p.sp_D2[e], tc1, RRb);
                safe = safe && isfinite(tab[e]) && (double)tab[e] * g2max < big;
            }
        }
    }
    if (!safe) atomicOr(&p.ctl->overflow, 1u);
}



// K: particles of several kinds (the screen's folded D2 constant of each
// pair of kinds from a per-box table in LDS); otherwise the box's constant.
template <bool K, class T = TileF32_0>
struct PolF32 {
    static constexpr int W = T::W;
    static constexpr bool kScreen = true;
    static constexpr bool kKinds = K;
    static constexpr int kFlushBatch = 2;
    static constexpr bool kFlushSkipEmpty = true;
    static constexpr int kWaves = T::kWaves;
    static constexpr int kFullWaves = T::kFullWaves;
    // A staged candidate is two 16-byte halves in two arrays: a = x, y, z
    // relative to the group centre and vx; b = vy, vz, its kind (particle
    // kinds only) and its sorted index (bit patterns).  With 16-byte strides
    // consecutive records fall in distinct LDS banks (a 32-byte record would
    // use only half of them).
    struct Lds {
        float4 a[W];
        float4 b[W];
        float kd2[K ? kMaxKinds * kMaxKinds : 1];
    };
    struct Own {
        float x, y, z, vx, vy, vz;   // position relative to the current group's centre
        uint32_t row;                // K: kMaxKinds * own kind
        double X, Y, Z;              // own FP64 position (kept: reloading it per group costs more)
    };
    using Group = ScreenGroup;
    __device__ static P64 self64(const Plan& p, uint32_t i, const Own&) { return p.B[i]; }
    __device__ static void load_own(const Plan& p, uint32_t i, Own& o, double& x, double& y, double& z)
    {
        const P64 m = p.B[i];
        o.vx = (float)m.vx; o.vy = (float)m.vy; o.vz = (float)m.vz;
        o.row = K ? (uint32_t)p.spB[i] * (uint32_t)kMaxKinds : 0u;
        x = m.x; y = m.y; z = m.z;
        o.X = m.x; o.Y = m.y; o.Z = m.z;
    }
    // per-group LDS tables, written before the group's first staging barrier
    // (sbi: the group's threshold set, box * kSpanClasses + span class)
    __device__ static void group_lds(Lds& l, const Plan& p, uint32_t sbi, int lane)
    {
        if (K) l.kd2[lane] = p.box_kD2[(size_t)sbi * (kMaxKinds * kMaxKinds) + (uint32_t)lane];
    }
    // Centre and thresholds (set sbi) of the group whose cells are x in
    // [cxf, cxl] of row (gcy, gcz); its neighbourhood spans cells
    // cxf-1..cxl+1, gcy-1..gcy+1, gcz-1..gcz+1 (images included).
    __device__ static void group_ctx(const Plan& p, const BoxDev& B, Group& g, int cxf, int cxl, int gcy, int gcz,
                                     int sbi)
    {
        const int clo[3] = {cxf - 1, gcy - 1, gcz - 1}, chi[3] = {cxl + 1, gcy + 1, gcz + 1};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double h = B.h[k];
            g.X0[k] = B.lo[k] + 0.5 * (double)(clo[k] + chi[k] + 1) * h;
        }
        g.t = p.box_sb[sbi];
    }
    __device__ static void begin_group(const Plan& p, const BoxDev& B, Own& o, Group& g, int cxf, int cxl,
                                       int gcy, int gcz, int sbi, uint32_t i, bool in)
    {
        group_ctx(p, B, g, cxf, cxl, gcy, gcz, sbi);
        if (in) {
            o.x = (float)(o.X - g.X0[0]);
            o.y = (float)(o.Y - g.X0[1]);
            o.z = (float)(o.Z - g.X0[2]);
        }
    }
    // FP32 copy of a candidate: image-shifted position relative to X0 and
    // velocity, each rounded once.  Rows without an image (almost all) skip
    // the shift (the row's shift is the same for the whole wave).
    __device__ static void stage(Lds& l, uint32_t t, const Plan& p, uint32_t j, const BoxDev& B, const Group& g,
                                 int wx, int wy, int wz, int, int)
    {
        const P64 q = p.B[j];
        double x = q.x, y = q.y, z = q.z;
        if (wx | wy | wz) {
            x = x + (wx ? (double)wx * B.L[0] : 0.0);
            y = y + (wy ? (double)wy * B.L[1] : 0.0);
            z = z + (wz ? (double)wz * B.L[2] : 0.0);
        }
        l.a[t] = make_float4((float)(x - g.X0[0]), (float)(y - g.X0[1]), (float)(z - g.X0[2]), (float)q.vx);
        l.b[t] = make_float4((float)q.vy, (float)q.vz, __uint_as_float(K ? (uint32_t)p.spB[j] : 0u),
                             __uint_as_float(j));
    }
    template <bool SH>
    __device__ static void scan(const Plan& p, const Lds& l, uint32_t c0, uint32_t j0, uint32_t j1, uint32_t i,
                                const Own& o, const BoxDev& B, const Group& g, int wx, int wy, int wz, int, int,
                                Found& f)
    {
        const float tb0 = g.t.tb0, tb1 = g.t.tb1, tt0 = g.t.tt0, kdt = g.t.kdt, tc0 = g.t.tc0, kD2 = g.t.kD2;
        // the loop steps an LDS pointer only; the sorted index is read from
        // the staged record for a kept pair alone
        const float4* rp = l.a + (j0 - c0);
        const float4* const re = rp + (j1 > j0 ? j1 - j0 : 0u);
        auto test = [&](const float4& qa, const float4& qb) {
            const float rx = qa.x - o.x, ry = qa.y - o.y, rz = qa.z - o.z;
            const float gx = qa.w - o.vx, gy = qb.x - o.vy, gz = qb.y - o.vz;
            const float b = fmaf(rz, gz, fmaf(ry, gy, rx * gx));
            const float g2 = fmaf(gz, gz, fmaf(gy, gy, gx * gx));
            const float rr = fmaf(rz, rz, fmaf(ry, ry, rx * rx));
            const float kd = K ? l.kd2[o.row + __float_as_uint(qb.z)] : kD2;
            const float mb = fmaf(-tb1, g2, b);
            const float m2 = fmaf(-kdt, g2, -b);
            const float m3 = fmaf(rr - kd, g2, -(b * b));
            return (mb <= tb0) & (m2 <= tt0) & (m3 <= tc0);
        };
        // two records per iteration: one loop test and one branch on the
        // kept pairs per two pair tests, and both LDS reads in flight
        for (; rp + 1 < re; rp += 2) {
            const float4 qa0 = rp[0], qb0 = rp[W], qa1 = rp[1], qb1 = rp[W + 1];
            const bool k0 = test(qa0, qb0), k1 = test(qa1, qb1);
            if (k0 | k1) {
                if (k0) f.add(p, i, __float_as_uint(qb0.w), wcode(wx, wy, wz));
                if (k1) f.add(p, i, __float_as_uint(qb1.w), wcode(wx, wy, wz));
            }
        }
        if (rp < re) {
            const float4 qa = rp[0], qb = rp[W];
            if (test(qa, qb)) f.add(p, i, __float_as_uint(qb.w), wcode(wx, wy, wz));
        }
    }
    // full neighbourhood: every pair the screen cannot reject is decided in
    // FP64 from the sorted records, with the image shift of its cell
    template <bool SH>
    __device__ static void scan_best(const Plan& p, const Lds& l, const uint32_t* lid, uint32_t c0, uint32_t j0,
                                     uint32_t j1, uint32_t i, const Own& o, const BoxDev& B, const Group& g,
                                     int wx, int wy, int wz, int, int, Best& best, Deferred& d)
    {
        const float tb0 = g.t.tb0, tb1 = g.t.tb1, tt0 = g.t.tt0, kdt = g.t.kdt, tc0 = g.t.tc0, kD2 = g.t.kD2;
        auto test = [&](uint32_t j) {
            const float4 qa = l.a[j - c0];
            const float4 qb = l.b[j - c0];
            const float rx = qa.x - o.x, ry = qa.y - o.y, rz = qa.z - o.z;
            const float gx = qa.w - o.vx, gy = qb.x - o.vy, gz = qb.y - o.vz;
            const float b = fmaf(rz, gz, fmaf(ry, gy, rx * gx));
            const float g2 = fmaf(gz, gz, fmaf(gy, gy, gx * gx));
            const float rr = fmaf(rz, rz, fmaf(ry, ry, rx * rx));
            const float kd = K ? l.kd2[o.row + __float_as_uint(qb.z)] : kD2;
            const float mb = fmaf(-tb1, g2, b);
            const float m2 = fmaf(-kdt, g2, -b);
            const float m3 = fmaf(rr - kd, g2, -(b * b));
            return (mb <= tb0) & (m2 <= tt0) & (m3 <= tc0) & (j != i);
        };
        // a kept pair: recorded for the end of the tile, or decided at once
        auto take = [&](uint32_t j) {
            if (d.n < kDefer) {
                d.sj[64 * d.n] = j;
                d.sj[64 * (kDefer + d.n)] = wcode(wx, wy, wz);
                ++d.n;
                return;
            }
            const P64 me = p.B[i], q = p.B[j];
            double rx6 = q.x - me.x, ry6 = q.y - me.y, rz6 = q.z - me.z;
            if (SH) {
                rx6 = rx6 + (double)wx * B.L[0];
                ry6 = ry6 + (double)wy * B.L[1];
                rz6 = rz6 + (double)wz * B.L[2];
            }
            const PairQ pq = pair_q(rx6, ry6, rz6, q.vx - me.vx, q.vy - me.vy, q.vz - me.vz);
            best.screened += 1u;
            if (accept(pq, pair_D2(p, B, o.row, j), B.dt)) best.offer(pq.c2 / pq.g2, lid[j - c0], j);
        };
        uint32_t j = j0;
        for (; j + 1 < j1; j += 2) {   // two records per iteration, as in scan
            const bool k0 = test(j), k1 = test(j + 1);
            if (k0 | k1) {
                if (k0) take(j);
                if (k1) take(j + 1);
            }
        }
        if (j < j1 && test(j)) take(j);
    }
    // the deferred pairs of particle i, decided in FP64 with their image shifts
    __device__ static void decide_deferred(const Plan& p, uint32_t i, const Deferred& d, const BoxDev& B,
                                           Best& best)
    {
        if (d.n == 0) return;
        const P64 me = p.B[i];
        const uint32_t row = kind_row(p, i);
        for (int k = 0; k < d.n; ++k) {
            const uint32_t j = d.sj[64 * k];
            const uint32_t c = d.sj[64 * (kDefer + k)];
            const int wx = (int)(c & 3u) - 1, wy = (int)((c >> 2) & 3u) - 1, wz = (int)((c >> 4) & 3u) - 1;
            const P64 q = p.B[j];
            double rx = q.x - me.x, ry = q.y - me.y, rz = q.z - me.z;
            if (wx != 0) rx = rx + (double)wx * B.L[0];
            if (wy != 0) ry = ry + (double)wy * B.L[1];
            if (wz != 0) rz = rz + (double)wz * B.L[2];
            const PairQ pq = pair_q(rx, ry, rz, q.vx - me.vx, q.vy - me.vy, q.vz - me.vz);
            best.screened += 1u;
            if (accept(pq, pair_D2(p, B, row, j), B.dt)) best.offer(pq.c2 / pq.g2, p.idB[j], j);
        }
    }
};

template <class Pol>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(Pol::kWaves)))
void k_search_half(Plan p)
{
    __shared__ typename Pol::Lds lds;
    const int lane = threadIdx.x;
    const uint32_t i = xcd_tile(blockIdx.x, gridDim.x) * 64u + (uint32_t)lane;
    const bool valid = i < p.N;
    const bool alive = valid && !(p.idB[i] & kGone);   // absorbed particles do not search
    uint32_t bidx = 0, rowkey = 0xFFFFFFFFu;
    int cx = 0, cy = 0, cz = 0;
    typename Pol::Own own{};
    if (alive) {
        bidx = p.boxidx ? p.boxidx[i] : 0u;
        const BoxDev& B = p.boxes[bidx];
        double x, y, z;
        Pol::load_own(p, i, own, x, y, z);
        cx = cell1(x, B.lo[0], B.inv_h[0], B.nc[0]);
        cy = cell1(y, B.lo[1], B.inv_h[1], B.nc[1]);
        cz = cell1(z, B.lo[2], B.inv_h[2], B.nc[2]);
        rowkey = B.coff + (uint32_t)B.nc[0] * ((uint32_t)cy + (uint32_t)B.nc[1] * (uint32_t)cz);
    }
    __shared__ uint32_t found_j[kReg * 64];
    Found found;
    found.sj = found_j + lane;
    found.n = 0;
    found.w = 0u;
    found.sh = 0u;
    uint64_t remaining = __ballot(alive);
    while (remaining) {
        const int lead = __ffsll((unsigned long long)remaining) - 1;
        const uint32_t key = (uint32_t)__builtin_amdgcn_readlane((int)rowkey, lead);
        const int cxf = __builtin_amdgcn_readlane(cx, lead);
        // the row's lanes in ascending cells; a screened group ends after
        // kScreenGroupCells cells (the rest of the row forms the next one),
        // and its span picks its class of screen thresholds
        const uint64_t grp =
            __ballot(alive && rowkey == key && (!Pol::kScreen || cx - cxf < kScreenGroupCells)) & remaining;
        remaining &= ~grp;
        const bool in = (grp >> lane) & 1ull;
        const int last = 63 - __clzll((long long)grp);
        const uint32_t gb = (uint32_t)__builtin_amdgcn_readlane((int)bidx, lead);
        const BoxDev& B = p.boxes[gb];
        const int gcy = __builtin_amdgcn_readlane(cy, lead), gcz = __builtin_amdgcn_readlane(cz, lead);
        const int cxl = __builtin_amdgcn_readlane(cx, last);
        const int NX = B.nc[0], NY = B.nc[1], NZ = B.nc[2];
        typename Pol::Group gctx;
        const uint32_t sbi = gb * (uint32_t)kSpanClasses + span_class(cxl - cxf + 1);
        Pol::begin_group(p, B, own, gctx, cxf, cxl, gcy, gcz, (int)sbi, i, in);
        Pol::group_lds(lds, p, sbi, lane);
        // Cells [ca, cb] of a row seen with image shift (wx, wy, wz); each lane
        // tests the sub-range [ls, le) of it (empty when ls >= le).
        auto part = [&](uint32_t row, int ca, int cb, uint32_t ls, uint32_t le, int wx, int wy, int wz, int dy,
                        int dz) {
            const uint32_t gs = p.start[row + ca], ge = p.start[row + cb + 1];
            const bool sh = (wx | wy | wz) != 0;
            for (uint32_t c0 = gs; c0 < ge; c0 += (uint32_t)Pol::W) {
                const uint32_t n = min((uint32_t)Pol::W, ge - c0);
                for (uint32_t t = (uint32_t)lane; t < n; t += 64u)
                    Pol::stage(lds, t, p, c0 + t, B, gctx, wx, wy, wz, dy, dz);
                __syncthreads();
                const uint32_t j0 = max(ls, c0), j1 = min(le, c0 + n);
                if (sh) Pol::template scan<true>(p, lds, c0, j0, j1, i, own, B, gctx, wx, wy, wz, dy, dz, found);
                else Pol::template scan<false>(p, lds, c0, j0, j1, i, own, B, gctx, wx, wy, wz, dy, dz, found);
                __syncthreads();
            }
        };
        // a wrapped end cell of a periodic x axis, used by lanes at that end
        auto wrap_cell = [&](uint32_t row, int cell, bool use, int wx, int wy, int wz, int dy, int dz) {
            part(row, cell, cell, use ? 0u : 1u, use ? 0xFFFFFFFFu : 0u, wx, wy, wz, dy, dz);
        };
        // own row: the rest of the own cell after i, and cell cx+1
        {
            const uint32_t row = key;
            const int cb = cxl + 1 >= NX ? NX - 1 : cxl + 1;
            uint32_t ls = 0, le = 0;
            if (in) {
                ls = i + 1;
                le = p.start[row + (cx + 1 >= NX ? NX - 1 : cx + 1) + 1];
            }
            part(row, cxf, cb, ls, le, 0, 0, 0, 0, 0);
            if (B.periodic[0] && cxl + 1 >= NX) wrap_cell(row, 0, in && cx == NX - 1, 1, 0, 0, 0, 0);
        }
        // rows (dy, dz) = (+1, 0), (-1, +1), (0, +1), (+1, +1): cells cx-1..cx+1
        for (int r = 0; r < 4; ++r) {
            const int dy = r == 0 ? 1 : r - 2, dz = r == 0 ? 0 : 1;
            int nz = gcz + dz, wz = 0;
            if (nz >= NZ) { if (!B.periodic[2]) continue; nz -= NZ; wz = 1; }
            int ny = gcy + dy, wy = 0;
            if (ny < 0) { if (!B.periodic[1]) continue; ny += NY; wy = -1; }
            else if (ny >= NY) { if (!B.periodic[1]) continue; ny -= NY; wy = 1; }
            const uint32_t row = B.coff + (uint32_t)NX * ((uint32_t)ny + (uint32_t)NY * (uint32_t)nz);
            uint32_t ls = 0, le = 0;
            if (in) {
                ls = p.start[row + (cx - 1 < 0 ? 0 : cx - 1)];
                le = p.start[row + (cx + 1 >= NX ? NX - 1 : cx + 1) + 1];
            }
            part(row, cxf - 1 < 0 ? 0 : cxf - 1, cxl + 1 >= NX ? NX - 1 : cxl + 1, ls, le, 0, wy, wz, dy, dz);
            if (B.periodic[0]) {
                if (cxf - 1 < 0) wrap_cell(row, NX - 1, in && cx == 0, -1, wy, wz, dy, dz);
                if (cxl + 1 >= NX) wrap_cell(row, 0, in && cx == NX - 1, 1, wy, wz, dy, dz);
            }
        }
    }
    uint64_t c = valid ? found.template flush<Pol::kFlushBatch, Pol::kFlushSkipEmpty, Pol::kKinds>(p, i, Pol::self64(p, i, own),
                                                                                       p.boxes[bidx])
                       : 0u;
    // statistics: pairs the search kept, counted at both particles
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if (lane == 0 && c) atomicAdd(&p.acc[blockIdx.x % kAccLanes].cand, 2ull * (unsigned long long)c);
}

// Full-neighbourhood variant of the search (KMC_SEARCH_FULL): every
// particle scans its own and all 26 neighbouring cells and keeps the running
// (key, id) minimum in registers, writing its partner directly.  It tests
// every pair twice but records nothing, so it suits dense cells with many
// acceptable partners per particle, where the candidate lists of the
// half-neighbourhood search overflow.  Rows and staging as in k_search_half.
// Under the FP32 screen the kept pairs wait in LDS (Deferred) and are decided
// in FP64 after the last row.  One tile of 64 cell-sorted particles (one
// wave), writing their partners; dslots: kDefer * 2 * 64 words of LDS for
// the FP32 screen (unused in FP64); STATS: count the pairs for the statistics.
template <class Pol, bool STATS>
__device__ __forceinline__ void search_full_tile(const Plan& p, uint32_t tile, typename Pol::Lds& lds, uint32_t* lid,
                                                 uint32_t* dslots)
{
    const int lane = threadIdx.x;
    const uint32_t i = tile * 64u + (uint32_t)lane;
    const bool valid = i < p.N;
    bool alive = valid && !(p.idB[i] & kGone);   // absorbed particles do not search
    uint32_t bidx = 0, rowkey = 0xFFFFFFFFu;
    int cx = 0, cy = 0, cz = 0;
    typename Pol::Own own{};
    if (alive) {
        bidx = p.boxidx ? p.boxidx[i] : 0u;
        const BoxDev& B = p.boxes[bidx];
        double x, y, z;
        Pol::load_own(p, i, own, x, y, z);
        cx = cell1(x, B.lo[0], B.inv_h[0], B.nc[0]);
        cy = cell1(y, B.lo[1], B.inv_h[1], B.nc[1]);
        cz = cell1(z, B.lo[2], B.inv_h[2], B.nc[2]);
        rowkey = B.coff + (uint32_t)B.nc[0] * ((uint32_t)cy + (uint32_t)B.nc[1] * (uint32_t)cz);
        // adaptive bins: particles in or next to a split cell search their
        // touching leaves instead (k_search_adapt)
        if (p.adapt_L > 0 && p.mixed[rowkey + (uint32_t)cx]) alive = false;
    }
    Best best;
    best.key = __builtin_inf();
    best.id = 0xFFFFFFFFu;
    best.j = -1;
    best.accepted = 0u;
    best.screened = 0u;
    Deferred dfr;
    dfr.sj = nullptr;
    dfr.n = 0;
    if constexpr (Pol::kScreen) dfr.sj = dslots + lane;
    uint64_t remaining = __ballot(alive);
    while (remaining) {
        const int lead = __ffsll((unsigned long long)remaining) - 1;
        const uint32_t key = (uint32_t)__builtin_amdgcn_readlane((int)rowkey, lead);
        const int cxf = __builtin_amdgcn_readlane(cx, lead);
        // the row's lanes in ascending cells; a screened group ends after
        // kScreenGroupCells cells (the rest of the row forms the next one),
        // and its span picks its class of screen thresholds
        const uint64_t grp =
            __ballot(alive && rowkey == key && (!Pol::kScreen || cx - cxf < kScreenGroupCells)) & remaining;
        remaining &= ~grp;
        const bool in = (grp >> lane) & 1ull;
        const int last = 63 - __clzll((long long)grp);
        const uint32_t gb = (uint32_t)__builtin_amdgcn_readlane((int)bidx, lead);
        const BoxDev& B = p.boxes[gb];
        const int gcy = __builtin_amdgcn_readlane(cy, lead), gcz = __builtin_amdgcn_readlane(cz, lead);
        const int cxl = __builtin_amdgcn_readlane(cx, last);
        const int NX = B.nc[0], NY = B.nc[1], NZ = B.nc[2];
        typename Pol::Group gctx;
        const uint32_t sbi = gb * (uint32_t)kSpanClasses + span_class(cxl - cxf + 1);
        Pol::begin_group(p, B, own, gctx, cxf, cxl, gcy, gcz, (int)sbi, i, in);
        Pol::group_lds(lds, p, sbi, lane);
        auto part = [&](uint32_t row, int ca, int cb, uint32_t ls, uint32_t le, int wx, int wy, int wz, int dy,
                        int dz) {
            const uint32_t gs = p.start[row + ca], ge = p.start[row + cb + 1];
            const bool sh = (wx | wy | wz) != 0;
            for (uint32_t c0 = gs; c0 < ge; c0 += (uint32_t)Pol::W) {
                const uint32_t n = min((uint32_t)Pol::W, ge - c0);
                for (uint32_t t = (uint32_t)lane; t < n; t += 64u) {
                    Pol::stage(lds, t, p, c0 + t, B, gctx, wx, wy, wz, dy, dz);
                    lid[t] = p.idB[c0 + t];
                }
                __syncthreads();
                const uint32_t j0 = max(ls, c0), j1 = min(le, c0 + n);
                if (sh)
                    Pol::template scan_best<true>(p, lds, lid, c0, j0, j1, i, own, B, gctx, wx, wy, wz, dy, dz, best,
                                                  dfr);
                else
                    Pol::template scan_best<false>(p, lds, lid, c0, j0, j1, i, own, B, gctx, wx, wy, wz, dy, dz, best,
                                                   dfr);
                __syncthreads();
            }
        };
        auto wrap_cell = [&](uint32_t row, int cell, bool use, int wx, int wy, int wz, int dy, int dz) {
            part(row, cell, cell, use ? 0u : 1u, use ? 0xFFFFFFFFu : 0u, wx, wy, wz, dy, dz);
        };
        for (int r = 0; r < 9; ++r) {
            const int dy = r % 3 - 1, dz = r / 3 - 1;
            int nz = gcz + dz, wz = 0;
            if (nz < 0) { if (!B.periodic[2]) continue; nz += NZ; wz = -1; }
            else if (nz >= NZ) { if (!B.periodic[2]) continue; nz -= NZ; wz = 1; }
            int ny = gcy + dy, wy = 0;
            if (ny < 0) { if (!B.periodic[1]) continue; ny += NY; wy = -1; }
            else if (ny >= NY) { if (!B.periodic[1]) continue; ny -= NY; wy = 1; }
            const uint32_t row = B.coff + (uint32_t)NX * ((uint32_t)ny + (uint32_t)NY * (uint32_t)nz);
            uint32_t ls = 0, le = 0;
            if (in) {
                ls = p.start[row + (cx - 1 < 0 ? 0 : cx - 1)];
                le = p.start[row + (cx + 1 >= NX ? NX - 1 : cx + 1) + 1];
            }
            part(row, cxf - 1 < 0 ? 0 : cxf - 1, cxl + 1 >= NX ? NX - 1 : cxl + 1, ls, le, 0, wy, wz, dy, dz);
            if (B.periodic[0]) {
                if (cxf - 1 < 0) wrap_cell(row, NX - 1, in && cx == 0, -1, wy, wz, dy, dz);
                if (cxl + 1 >= NX) wrap_cell(row, 0, in && cx == NX - 1, 1, wy, wz, dy, dz);
            }
        }
    }
    if constexpr (Pol::kScreen) {
        if (alive) Pol::decide_deferred(p, i, dfr, p.boxes[bidx], best);
    }
    if (valid && (alive || p.adapt_L == 0)) p.partner[i] = best.j;
    if (STATS) {
        // statistics: pairs accepted (FP64) or decided in FP64 (FP32 screen)
        uint64_t c = Pol::kScreen ? best.screened : best.accepted;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
        if (lane == 0 && c) atomicAdd(&p.acc[blockIdx.x % kAccLanes].cand, (unsigned long long)c);
    }
}

template <class Pol>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(Pol::kFullWaves)))
void k_search_full(Plan p)
{
    __shared__ typename Pol::Lds lds;
    __shared__ uint32_t lid[Pol::W];
    __shared__ uint32_t dslots[Pol::kScreen ? 2 * kDefer * 64 : 1];
    search_full_tile<Pol, true>(p, xcd_tile(blockIdx.x, gridDim.x), lds, lid, dslots);
}

// Whole-step FP64 search, by the full-neighbourhood organisation, when a
// list overflowed (recheck list or overflow pair list) or, under the FP32
// screen, a particle lies outside its box's grid or a box's scales leave the
// screen's safe range.  A fixed grid of waves that exits at once unless the
// step's flag is set, and otherwise takes the tiles in turn.
constexpr uint32_t kFallbackBlocks = 4096;
// Waves that walk the list of split cells (adaptive bins).
constexpr uint32_t kAdaptPrepBlocks = 4096;

template <class Pol>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(Pol::kFullWaves)))
void k_fallback_full(Plan p)
{
    __shared__ typename Pol::Lds lds;
    __shared__ uint32_t lid[Pol::W];
    if (p.ctl->overflow == 0u) return;
    const uint32_t ntiles = (p.N + 63u) / 64u;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) search_full_tile<Pol, false>(p, t, lds, lid, nullptr);
}

// --------------------------------------------------------------------------
// Density-adaptive bins: the search of particles in or next to a split cell.
//
// Particles of one leaf share their neighbourhood: the leaves that touch
// theirs, all inside the 27 cells around their cell.  A wave takes 64
// consecutive sorted particles; the lanes of one leaf form a group (they are
// consecutive, the sort keeps leaves contiguous).  For each group the wave
// lists the sorted ranges of the touching leaves, stages their particles
// into LDS and tests every (owner, candidate) pair with all 64 lanes: each of
// the group's g owners gets 64 / g' lanes (g' the next power of two), which
// take every (64/g')-th staged candidate, and the owner's (key, id) minimum
// is reduced over its lanes.  Each pair is tested from both sides (running
// minimum, no lists).
// --------------------------------------------------------------------------

// The leaves of the neighbour cell (c + d) that touch the leaf [lo, hi]
// (finest indices per axis) of a particle in cell c, as ranges of the sorted
// arrays: f(s, e, code) once per run of touching leaves that is contiguous
// in the cell's leaf order (one range for an unsplit cell); code packs the
// periodic image (wcode) and the cell offset d.  Nothing when the neighbour
// cell does not exist or no leaf of it touches.
template <class F>
__device__ __forceinline__ void neighbour_leaves(const Plan& p, const BoxDev& B, const int c[3], const int lo[3],
                                                 const int hi[3], int dx, int dy, int dz, F&& f)
{
    const int L = p.adapt_L;
    const int d[3] = {dx, dy, dz};
    int q[3], w[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        q[a] = c[a] + d[a];
        w[a] = 0;
        if (q[a] < 0) { if (!B.periodic[a]) return; q[a] += B.nc[a]; w[a] = -1; }
        else if (q[a] >= B.nc[a]) { if (!B.periodic[a]) return; q[a] -= B.nc[a]; w[a] = 1; }
    }
    const uint32_t cell = B.coff + (uint32_t)q[0] + (uint32_t)B.nc[0] * ((uint32_t)q[1] + (uint32_t)B.nc[1] * (uint32_t)q[2]);
    const int lvl = (int)p.level[cell];
    const int sh = L - lvl, r = 1 << lvl;
    int jlo[3], jhi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        // leaf j of the neighbour spans [b0 + j 2^sh, b0 + (j + 1) 2^sh - 1]
        // (b0: its lower face, with the image); it touches [lo, hi] iff
        // (lo - b0 - 1) >> sh <= j <= (hi + 1 - b0) >> sh
        const long long b0 = ((long long)q[a] << L) + (long long)w[a] * ((long long)B.nc[a] << L);
        jlo[a] = (int)max(0ll, ((long long)lo[a] - b0 - 1) >> sh);
        jhi[a] = (int)min((long long)(r - 1), ((long long)hi[a] + 1 - b0) >> sh);
        if (jlo[a] > jhi[a]) return;
    }
    const uint32_t code = wcode(w[0], w[1], w[2]) | ((uint32_t)wcode(dx, dy, dz) << 6);
    const uint32_t s0 = p.start[cell];
    if (lvl == 0) {
        f(s0, p.start[cell + 1], code);
        return;
    }
    const uint32_t* t = p.pool + p.pool_base[cell];
    for (int jz = jlo[2]; jz <= jhi[2]; ++jz)
        for (int jy = jlo[1]; jy <= jhi[1]; ++jy) {
            const uint32_t row = (uint32_t)r * ((uint32_t)jy + (uint32_t)r * (uint32_t)jz);
            f(s0 + t[row + (uint32_t)jlo[0]], s0 + t[row + (uint32_t)jhi[0] + 1u], code);
        }
}

// The same ranges in two parts, for a wave that lists the neighbourhoods of
// several leaves of one cell in turn: the neighbour cell's data (its index,
// level, start and leaf-table offset, loaded together) kept across the
// leaves, then per leaf the touching runs, which only load leaf-table
// entries (and nothing at all when only counted).
struct NbCell {
    int32_t lvl;       // split level; -1: the neighbour cell does not exist
    int32_t qw[3];     // its cell coordinates with the periodic image (q + w n)
    uint32_t code;     // image and cell offset (as neighbour_leaves reports them)
    uint32_t s0, s1;   // start[cell], start[cell + 1]
    uint32_t pb;       // pool_base[cell] (split cells)
};

__device__ __forceinline__ void nb_cell_load(const Plan& p, const BoxDev& B, const int c[3], int dx, int dy, int dz,
                                             NbCell& nc)
{
    const int d[3] = {dx, dy, dz};
    int q[3], w[3];
    nc.lvl = -1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        q[a] = c[a] + d[a];
        w[a] = 0;
        if (q[a] < 0) { if (!B.periodic[a]) return; q[a] += B.nc[a]; w[a] = -1; }
        else if (q[a] >= B.nc[a]) { if (!B.periodic[a]) return; q[a] -= B.nc[a]; w[a] = 1; }
        nc.qw[a] = q[a] + w[a] * B.nc[a];
    }
    nc.code = wcode(w[0], w[1], w[2]) | ((uint32_t)wcode(dx, dy, dz) << 6);
    const uint32_t cell = B.coff + (uint32_t)q[0] + (uint32_t)B.nc[0] * ((uint32_t)q[1] + (uint32_t)B.nc[1] * (uint32_t)q[2]);
    nc.lvl = (int)p.level[cell];
    nc.s0 = p.start[cell];
    nc.s1 = p.start[cell + 1];
    nc.pb = p.pool_base[cell];
}

// The leaves of a cached neighbour cell that touch the leaf [lo, hi]: their
// index box jlo..jhi per axis, and the number of runs they form in the
// cell's leaf order (one per (jy, jz) row of a split cell, one for an
// unsplit cell, 0 when none touches).
__device__ __forceinline__ uint32_t nb_leaf_box(const Plan& p, const NbCell& nc, const int lo[3], const int hi[3],
                                                int jlo[3], int jhi[3])
{
    if (nc.lvl < 0) return 0u;
    const int L = p.adapt_L;
    const int sh = L - nc.lvl, r = 1 << nc.lvl;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        // the neighbour's lower face on the finest grid, with its image
        const long long b0 = (long long)nc.qw[a] << L;
        jlo[a] = (int)max(0ll, ((long long)lo[a] - b0 - 1) >> sh);
        jhi[a] = (int)min((long long)(r - 1), ((long long)hi[a] + 1 - b0) >> sh);
        if (jlo[a] > jhi[a]) return 0u;
    }
    if (nc.lvl == 0) return 1u;
    return (uint32_t)(jhi[1] - jlo[1] + 1) * (uint32_t)(jhi[2] - jlo[2] + 1);
}

// One neighbour cell of a group as the wave's lanes read it when they list
// the runs in parallel.
struct NbBox {
    int32_t jlo0, jhi0, jlo1, ny, jlo2, lvl;
    uint32_t s0, s1, pb, code;
};

// A particle's cell (c) and leaf ([lo, hi] in finest indices) under adaptive
// bins, from its position; returns the linear cell.
__device__ __forceinline__ uint32_t leaf_of(const Plan& p, const BoxDev& B, double x, double y, double z, int c[3],
                                            int lo[3], int hi[3], uint32_t& code)
{
    const int L = p.adapt_L;
    const double xs[3] = {x, y, z};
    int g[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        g[a] = fine1(xs[a], B.lo[a], B.inv_h[a], B.nc[a], L);
        c[a] = g[a] >> L;
    }
    const uint32_t cell = B.coff + (uint32_t)c[0] + (uint32_t)B.nc[0] * ((uint32_t)c[1] + (uint32_t)B.nc[1] * (uint32_t)c[2]);
    const int lvl = (int)p.level[cell];
    const int sh = L - lvl;
    const uint32_t m = (1u << lvl) - 1u;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = (g[a] >> sh) << sh;
        hi[a] = lo[a] + (1 << sh) - 1;
    }
    code = (((uint32_t)g[0] >> sh) & m) + (m + 1u) * ((((uint32_t)g[1] >> sh) & m) + (m + 1u) * (((uint32_t)g[2] >> sh) & m));
    return cell;
}

constexpr int kRangeBatch = 128;

template <int W>
struct AdaptLds {
    NbBox nb[27];                    // the group's neighbour cells (runs of touching leaves)
    uint32_t noff[27];               // exclusive prefix of their run counts
    uint32_t rs[kRangeBatch];        // range starts (sorted index)
    uint32_t rc[kRangeBatch];        // range codes (image, cell offset)
    uint32_t rp[kRangeBatch + 1];    // exclusive prefix of the range sizes
    uint32_t lid[W];                 // staged candidates' ids
    uint32_t lj[W];                  // ... sorted indices
    uint32_t lw[W];                  // ... image codes
};

// Binary search: the range r of flat candidate index f (rp[r] <= f < rp[r+1]).
__device__ __forceinline__ uint32_t range_of(const uint32_t* rp, uint32_t nr, uint32_t f)
{
    uint32_t lo = 0, hi = nr - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (rp[mid] <= f) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <class Pol, bool STATS>
__device__ __forceinline__ void search_adapt_tile(const Plan& p, uint32_t tile, typename Pol::Lds& lds,
                                                  AdaptLds<Pol::W>& al)
{
    const int lane = threadIdx.x;
    const uint32_t i = tile * 64u + (uint32_t)lane;
    bool alive = i < p.N && !(p.idB[i] & kGone);
    uint32_t bidx = 0, cell = 0xFFFFFFFFu, code = 0;
    int c[3] = {0, 0, 0}, lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    if (alive) {
        bidx = p.boxidx ? p.boxidx[i] : 0u;
        const P64 me = p.B[i];
        cell = leaf_of(p, p.boxes[bidx], me.x, me.y, me.z, c, lo, hi, code);
        alive = p.mixed[cell] != 0;
    }
    Best best;
    uint64_t nstat = 0;
    uint64_t remaining = __ballot(alive);
    // lanes 0..26: neighbour cell (lane % 3 - 1, lane / 3 % 3 - 1, lane / 9 - 1)
    // of the cell of the current group, kept while the groups stay in it
    const int ndx = lane % 3 - 1, ndy = (lane / 3) % 3 - 1, ndz = lane / 9 - 1;
    NbCell nbc;
    nbc.lvl = -1;
    uint32_t nb_of = 0xFFFFFFFFu;
    while (remaining) {
        const int lead = __ffsll((unsigned long long)remaining) - 1;
        const uint32_t gcell = (uint32_t)__builtin_amdgcn_readlane((int)cell, lead);
        const uint32_t gcode = (uint32_t)__builtin_amdgcn_readlane((int)code, lead);
        const uint64_t grp = __ballot(alive && cell == gcell && code == gcode) & remaining;
        remaining &= ~grp;
        const uint32_t g = (uint32_t)__popcll(grp);   // lanes lead .. lead + g - 1 (a leaf is contiguous)
        const uint32_t gb = (uint32_t)__builtin_amdgcn_readlane((int)bidx, lead);
        const BoxDev& B = p.boxes[gb];
        int gc[3], glo[3], ghi[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            gc[a] = __builtin_amdgcn_readlane(c[a], lead);
            glo[a] = __builtin_amdgcn_readlane(lo[a], lead);
            ghi[a] = __builtin_amdgcn_readlane(hi[a], lead);
        }
        // owners: 64 / g' lanes each (g' = g rounded up to a power of two)
        uint32_t gp = 1;
        while (gp < g) gp <<= 1;
        const uint32_t kk = 64u / gp, o = (uint32_t)lane / kk, u = (uint32_t)lane % kk;
        const bool owner = o < g;
        const uint32_t io = tile * 64u + (uint32_t)lead + (owner ? o : 0u);
        typename Pol::Own own{};
        double ox, oy, oz;
        Pol::load_own(p, io, own, ox, oy, oz);
        typename Pol::Group gctx;
        const uint32_t sbi = gb * (uint32_t)kSpanClasses;   // the neighbourhood spans 3 cells: class 0
        Pol::begin_group(p, B, own, gctx, gc[0], gc[0], gc[1], gc[2], (int)sbi, io, owner);
        Pol::group_lds(lds, p, sbi, lane);
        best.key = __builtin_inf();
        best.id = 0xFFFFFFFFu;
        best.j = -1;
        best.accepted = 0u;
        best.screened = 0u;
        // ranges of the touching leaves: lanes 0..26 take one neighbour cell each
        if (gcell != nb_of) {
            if (lane < 27) nb_cell_load(p, B, gc, ndx, ndy, ndz, nbc);
            nb_of = gcell;
        }
        // per neighbour cell the box of touching leaves and its number of
        // runs, published; then the lanes list the runs f = lane, lane + 64,
        // ... of the flat sequence (cell by cell, rows jz-major) in parallel
        int bjlo[3] = {0, 0, 0}, bjhi[3] = {0, 0, 0};
        uint32_t nr = 0;
        if (lane < 27) nr = nb_leaf_box(p, nbc, glo, ghi, bjlo, bjhi);
        uint32_t off = nr;
#pragma unroll
        for (int sft = 1; sft < 64; sft <<= 1) {
            const uint32_t y = __shfl_up(off, sft, 64);
            if (lane >= sft) off += y;
        }
        const uint32_t R = (uint32_t)__shfl((int)off, 63, 64);
        off -= nr;
        if (lane < 27) {
            NbBox& nx = al.nb[lane];
            nx.jlo0 = bjlo[0];
            nx.jhi0 = bjhi[0];
            nx.jlo1 = bjlo[1];
            nx.ny = bjhi[1] - bjlo[1] + 1;
            nx.jlo2 = bjlo[2];
            nx.lvl = nbc.lvl;
            nx.s0 = nbc.s0;
            nx.s1 = nbc.s1;
            nx.pb = nbc.pb;
            nx.code = nbc.code;
            al.noff[lane] = off;
        }
        __syncthreads();
        for (uint32_t rb = 0; rb < R; rb += (uint32_t)kRangeBatch) {
            const uint32_t nb = min((uint32_t)kRangeBatch, R - rb);
            for (uint32_t f = rb + (uint32_t)lane; f < rb + nb; f += 64u) {
                // the neighbour cell d of run f: the last with noff[d] <= f
                uint32_t d = 0;
#pragma unroll
                for (uint32_t step = 16; step > 0; step >>= 1)
                    if (d + step < 27u && al.noff[d + step] <= f) d += step;
                const NbBox& nx = al.nb[d];
                const uint32_t k = f - al.noff[d];
                uint32_t s0 = nx.s0, e0 = nx.s1;
                if (nx.lvl > 0) {
                    const uint32_t r = 1u << nx.lvl;
                    const uint32_t jy = (uint32_t)nx.jlo1 + k % (uint32_t)nx.ny;
                    const uint32_t jz = (uint32_t)nx.jlo2 + k / (uint32_t)nx.ny;
                    const uint32_t* t = p.pool + nx.pb + r * (jy + r * jz);
                    s0 = nx.s0 + t[nx.jlo0];
                    e0 = nx.s0 + t[nx.jhi0 + 1];
                }
                al.rs[f - rb] = s0;
                al.rc[f - rb] = nx.code;
                al.rp[f - rb] = e0 - s0;   // size, turned into the prefix below
            }
            __syncthreads();
            // exclusive prefix of the nb sizes: two per lane
            const uint32_t e0 = 2u * (uint32_t)lane, e1 = e0 + 1u;
            const uint32_t v0 = e0 < nb ? al.rp[e0] : 0u, v1 = e1 < nb ? al.rp[e1] : 0u;
            uint32_t x = v0 + v1;
#pragma unroll
            for (int sft = 1; sft < 64; sft <<= 1) {
                const uint32_t y = __shfl_up(x, sft, 64);
                if (lane >= sft) x += y;
            }
            __syncthreads();
            if (e0 < nb) al.rp[e0] = x - v0 - v1;
            if (e1 < nb) al.rp[e1] = x - v1;
            if (lane == 63) al.rp[nb] = x;
            __syncthreads();
            const uint32_t total = al.rp[nb];
            for (uint32_t c0 = 0; c0 < total; c0 += (uint32_t)Pol::W) {
                const uint32_t n = min((uint32_t)Pol::W, total - c0);
                for (uint32_t t = (uint32_t)lane; t < n; t += 64u) {
                    const uint32_t f = c0 + t;
                    const uint32_t r = range_of(al.rp, nb, f);
                    const uint32_t j = al.rs[r] + (f - al.rp[r]);
                    const uint32_t cd = al.rc[r];
                    const int wx = (int)(cd & 3u) - 1, wy = (int)((cd >> 2) & 3u) - 1, wz = (int)((cd >> 4) & 3u) - 1;
                    const int dy = (int)((cd >> 8) & 3u) - 1, dz = (int)((cd >> 10) & 3u) - 1;
                    Pol::stage(lds, t, p, j, B, gctx, wx, wy, wz, dy, dz);
                    al.lid[t] = p.idB[j];
                    al.lj[t] = j;
                    al.lw[t] = cd & 0x3Fu;
                }
                __syncthreads();
                if (owner) Pol::scan_adapt(p, lds, al.lid, al.lj, al.lw, n, u, kk, io, own, B, gctx, best);
                __syncthreads();
            }
            __syncthreads();   // every read of this batch's ranges is done
        }
        // each owner's (key, id) minimum over its kk lanes
        for (uint32_t sft = kk >> 1; sft > 0; sft >>= 1) {
            const double k2 = __shfl_xor(best.key, (int)sft, 64);
            const uint32_t id2 = (uint32_t)__shfl_xor((int)best.id, (int)sft, 64);
            const int32_t j2 = __shfl_xor(best.j, (int)sft, 64);
            if (k2 < best.key || (k2 == best.key && id2 < best.id)) {
                best.key = k2;
                best.id = id2;
                best.j = j2;
            }
        }
        if (owner && u == 0) p.partner[io] = best.j;
        if (owner) nstat += Pol::kScreen ? best.screened : best.accepted;
    }
    if (STATS) {
#pragma unroll
        for (int sft = 32; sft > 0; sft >>= 1) nstat += __shfl_xor(nstat, sft, 64);
        if (lane == 0 && nstat) atomicAdd(&p.acc[blockIdx.x % kAccLanes].cand, (unsigned long long)nstat);
    }
}

template <class Pol>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(Pol::kFullWaves)))
void k_search_adapt(Plan p)
{
    __shared__ typename Pol::Lds lds;
    __shared__ AdaptLds<Pol::W> al;
    search_adapt_tile<Pol, true>(p, xcd_tile(blockIdx.x, gridDim.x), lds, al);
}

// The whole-step FP64 search of the particles k_search_adapt takes (see
// k_fallback_full).
template <class Pol>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(Pol::kFullWaves)))
void k_fallback_adapt(Plan p)
{
    __shared__ typename Pol::Lds lds;
    __shared__ AdaptLds<Pol::W> al;
    if (p.ctl->overflow == 0u) return;
    const uint32_t ntiles = (p.N + 63u) / 64u;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) search_adapt_tile<Pol, false>(p, t, lds, al);
}

// Pairs beyond a search lane's register slots: decided in FP64 and posted to
// both candidate lists.
__global__ void k_distribute_overflow(Plan p)
{
    const uint32_t cnt = p.ctl->ovf_count;
    const uint32_t n = cnt < p.ovf_cap ? cnt : p.ovf_cap;
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        const uint2 e = p.ovf[k];
        const P64 me = p.B[e.x];
        double key;
        if (exact_key(p, box_of(p, e.x), e.x, me, e.y, key)) {
            post_candidate(p, e.x, e.y, key);
            post_candidate(p, e.y, e.x, key);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && n)
        atomicAdd(&p.acc[0].cand, 2ull * (unsigned long long)n);
}

// Wave-aggregated append of this lane's particle to the FP64 recheck list
// (all lanes of the wave must call it).
__device__ __forceinline__ void push_recheck(const Plan& p, uint32_t i, bool need)
{
    const uint64_t mask = __ballot(need);
    if (!mask) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(&p.ctl->recheck_count, (unsigned int)__popcll(mask));
    base = (uint32_t)__builtin_amdgcn_readlane((int)base, leader);
    if (need) {
        const uint32_t idx = base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
        if (idx < p.recheck_cap) p.recheck[idx] = i;
        else atomicOr(&p.ctl->overflow, 1u);
    }
}

// Partner of every particle: the (key, id) minimum of its forward best (the
// pairs its own search lane found) and the entries of its candidate list
// (pairs found from the other side, or through the overflow list); keys are
// exact FP64, ids are read only to break equal keys.  A particle with more
// list entries than slots is searched again in full.
__global__ __launch_bounds__(256) void k_finish(Plan p)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < p.N;
    const uint32_t cnt = valid ? p.sl_cnt[i] : 0u;
    if (cnt != 0) p.sl_cnt[i] = 0u;
    double best_key = valid ? p.fb_key[i] : 0.0;
    int32_t best = valid ? p.fb_j[i] : -1;
    if (cnt >= 1 && cnt <= (uint32_t)kSlots) {
        for (uint32_t k = 0; k < cnt; ++k) {
            const SlotEntry e = p.sl[(size_t)k * p.N + i];
            const uint32_t j = e.j;
            const double key = e.key;
            // best_key is +inf while there is no best, so an entry with key
            // +inf (a kept pair that the exact test rejected) never wins
            if (key < best_key || (key == best_key && best >= 0 && p.idB[j] < p.idB[best])) {
                best_key = key;
                best = (int32_t)j;
            }
        }
    }
    push_recheck(p, i, cnt > (uint32_t)kSlots);
    if (valid) p.partner[i] = best;
}

// The FP64 search of one particle by a whole wave: the lanes share its
// candidates and the wave takes the (key, id) minimum of their minima.  All
// lanes of the wave must call it with the same i; returns the partner in
// every lane.
__device__ int32_t search_one64_wave(const Plan& p, uint32_t i)
{
    if (p.idB[i] & kGone) return -1;
    const int lane = threadIdx.x & 63;
    const BoxDev& B = box_of(p, i);
    const P64* __restrict__ X = p.B;
    const P64 me = X[i];
    const int cx = cell1(me.x, B.lo[0], B.inv_h[0], B.nc[0]);
    const int cy = cell1(me.y, B.lo[1], B.inv_h[1], B.nc[1]);
    const int cz = cell1(me.z, B.lo[2], B.inv_h[2], B.nc[2]);
    const double dt = B.dt;
    const uint32_t row = kind_row(p, i);
    double best_key = __builtin_inf();
    uint32_t best_id = 0xFFFFFFFFu;
    int32_t best = -1;
    for_each_range(B, cx, cy, cz, p.start, [&](uint32_t s, uint32_t e, int wx, int wy, int wz) {
        const bool shift = (wx | wy | wz) != 0;
        const double sx = (double)wx * B.L[0], sy = (double)wy * B.L[1], sz = (double)wz * B.L[2];
        for (uint32_t j = s + (uint32_t)lane; j < e; j += 64u) {
            const P64 q = X[j];
            double rx = q.x - me.x, ry = q.y - me.y, rz = q.z - me.z;
            if (shift) { rx = rx + sx; ry = ry + sy; rz = rz + sz; }
            const PairQ pq = pair_q(rx, ry, rz, q.vx - me.vx, q.vy - me.vy, q.vz - me.vz);
            if (accept(pq, pair_D2(p, B, row, j), dt)) {
                const double key = pq.c2 / pq.g2;
                const uint32_t idj = p.idB[j];
                if (key < best_key || (key == best_key && idj < best_id)) {
                    best_key = key;
                    best_id = idj;
                    best = (int32_t)j;
                }
            }
        }
    });
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double k2 = __shfl_xor(best_key, off, 64);
        const uint32_t id2 = (uint32_t)__shfl_xor((int)best_id, off, 64);
        const int32_t b2 = __shfl_xor(best, off, 64);
        if (k2 < best_key || (k2 == best_key && id2 < best_id)) {
            best_key = k2;
            best_id = id2;
            best = b2;
        }
    }
    return best;
}

// FP64 re-search of the particles whose candidate lists overflowed, one
// wave per particle.
__global__ void k_recheck64(Plan p)
{
    if (p.ctl->overflow != 0u) return;   // the whole-step FP64 search follows
    const uint32_t cnt = p.ctl->recheck_count;
    const uint32_t n = cnt < p.recheck_cap ? cnt : p.recheck_cap;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t k = wave; k < n; k += nwaves) {
        const uint32_t i = p.recheck[k];
        const int32_t b = search_one64_wave(p, i);
        if ((threadIdx.x & 63) == 0) p.partner[i] = b;
    }
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
        if (B.absorb[k]) continue;   // decided by the caller after streaming
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

// K: particles of several kinds (masses from the kind table).
// One kind of particle: compiled for eight waves per SIMD.  The collision
// path is bound by the latency of its partner-record gathers, and the
// default allocation (103 SGPRs) allowed seven; the few scalar values that
// no longer fit go to vector-register lanes (measured 4.36 -> 3.92 ms at
// N = 1e8).  With kinds, eight waves would spill vector registers.
template <bool K>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(K ? 1 : 8))) void k_resolve(Plan p)
{
    __shared__ uint64_t lds[32];
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t my_np = 0, my_dig = 0;
    double nx = 0.0, ny = 0.0, nz = 0.0;
    bool gone = false, left = false;
    if (i < p.N) {
        const BoxDev& B = box_of(p, i);
        const size_t N = p.N;
        const P64 me = p.B[i];
        double x[3] = {me.x, me.y, me.z}, v[3] = {me.vx, me.vy, me.vz};
        uint32_t id = p.idB[i];
        gone = (id & kGone) != 0u;   // absorbed earlier: keeps its state
        const int32_t q = p.partner[i];
        const double dt = B.dt;
        bool hit = false;
        if (q >= 0 && p.partner[q] == (int32_t)i) {
            hit = true;
            const uint32_t idq = p.idB[q];
            const P64 o = p.B[q];
            const double xq[3] = {o.x, o.y, o.z}, vq[3] = {o.vx, o.vy, o.vz};
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
            direction(p.seed, p.ctl->step, ida, nh, p.dims);
            // masses of a and b (particle kinds), equal otherwise
            double ma = 1.0, mb = 1.0;
            if (K) {
                const uint32_t ki = p.spB[i], kq = p.spB[q];
                ma = p.sp_mass[me_a ? ki : kq];
                mb = p.sp_mass[me_a ? kq : ki];
            }
            double vn[3];
            if (ma == mb) {
                const double hg = 0.5 * sqrt(pq.g2);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const double vcm = 0.5 * (va[k] + vb[k]);
                    vn[k] = me_a ? vcm + hg * nh[k] : vcm - hg * nh[k];
                }
            } else {
                // centre-of-mass velocity, |g| shared in inverse proportion to the masses
                const double M = ma + mb, gm = sqrt(pq.g2);
                const double wa = (mb / M) * gm, wb = (ma / M) * gm;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const double vcm = fma(ma, va[k], mb * vb[k]) / M;
                    vn[k] = me_a ? vcm + wa * nh[k] : vcm - wb * nh[k];
                }
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
        if (!hit && !gone) {
#pragma unroll
            for (int k = 0; k < 3; ++k) x[k] = x[k] + v[k] * dt;
        }
        if (!gone) {
            apply_bc(B, x, v);
            // absorbing faces: beyond them the particle leaves the gas
#pragma unroll
            for (int k = 0; k < 3; ++k)
                if (B.absorb[k] && (x[k] < B.lo[k] || x[k] > B.hi[k])) left = true;
            if (left) {
                id |= kGone;
                gone = true;
            }
        }
        // streaming (non-temporal) stores: the state is read again only by
        // the next step's sorted copy (measured 4% faster than cached stores)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            __builtin_nontemporal_store(x[k], p.A + k * N + i);
            __builtin_nontemporal_store(v[k], p.A + (3 + k) * N + i);
        }
        __builtin_nontemporal_store(id, p.idA + i);
        if (K) p.spA[i] = p.spB[i];
        nx = x[0]; ny = x[1]; nz = x[2];
    }
    // a1 of the next step: cell and slot of the new position
    bin_particle(p, i, i < p.N, box_of(p, i < p.N ? i : 0u), nx, ny, nz, gone);
    const uint64_t lm = __ballot(left);
    if ((threadIdx.x & 63) == 0 && lm) atomicAdd(&p.ctl->absorbed_total, (unsigned long long)__popcll(lm));
    block_sum2(my_np, my_dig, lds);
    if (threadIdx.x == 0 && my_np != 0) {
        StepAcc& a = p.acc[blockIdx.x % kAccLanes];
        atomicAdd(&a.np, (unsigned long long)my_np);
        atomicAdd(&a.dig, (unsigned long long)my_dig);
    }
}

// End of step (one block of kAdvanceThreads): fold this step's partial sums
// into its history row and the running candidate count, clear them, and
// advance the step counters.
constexpr uint32_t kAdvanceThreads = 1024;

__global__ __launch_bounds__(kAdvanceThreads) void k_advance(Plan p)
{
    __shared__ uint64_t lds[32];
    uint64_t np = 0, dig = 0, cand = 0, z = 0;
    for (uint32_t k = threadIdx.x; k < (uint32_t)kAccLanes; k += blockDim.x) {
        StepAcc& a = p.acc[k];
        np += a.np;
        dig += a.dig;
        cand += a.cand;
        a.np = 0;
        a.dig = 0;
        a.cand = 0;
    }
    block_sum2(np, dig, lds);
    __syncthreads();
    block_sum2(cand, z, lds);
    if (threadIdx.x == 0) {
        const unsigned long long done = p.ctl->steps_done;
        p.hist_np[done % p.H] = np;
        p.hist_dig[done % p.H] = dig;
        p.ctl->candidates_total += cand;
        p.ctl->rechecks_total += p.ctl->recheck_count;
        p.ctl->fallbacks_total += p.ctl->overflow ? 1ull : 0ull;
        p.ctl->steps_done = done + 1;
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
    if (i < p.N && !(p.idB[i] & kGone)) {
        const BoxDev& B = box_of(p, i);
        const P64 me = p.B[i];
        const int cx = cell1(me.x, B.lo[0], B.inv_h[0], B.nc[0]);
        const int cy = cell1(me.y, B.lo[1], B.inv_h[1], B.nc[1]);
        const int cz = cell1(me.z, B.lo[2], B.inv_h[2], B.nc[2]);
        const uint32_t cell = B.coff + (uint32_t)cx + (uint32_t)B.nc[0] * ((uint32_t)cy + (uint32_t)B.nc[1] * (uint32_t)cz);
        if (p.adapt_L > 0 && p.mixed[cell]) {
            // adaptive bins: the particles of the touching leaves
            int c[3], lo[3], hi[3];
            uint32_t code;
            leaf_of(p, B, me.x, me.y, me.z, c, lo, hi, code);
            for (int k = 0; k < 27; ++k)
                neighbour_leaves(p, B, c, lo, hi, k % 3 - 1, (k / 3) % 3 - 1, k / 9 - 1,
                                 [&](uint32_t s, uint32_t e, uint32_t) { t += e - s; });
        } else {
            for_each_range(B, cx, cy, cz, p.start, [&](uint32_t s, uint32_t e, int, int, int) { t += e - s; });
        }
        t -= 1;
    }
    block_sum2(t, z, lds);
    if (threadIdx.x == 0) atomicAdd(out, (unsigned long long)t);
}

inline uint32_t blocks_for(uint32_t n, uint32_t b) { return (n + b - 1) / b; }

// The search kernel of one precision policy and tile shape.
template <template <bool, class> class Pol, class T>
void launch_search(bool kinds, bool full, uint32_t gW, hipStream_t s, const Plan& p)
{
    if (full) {
        if (kinds) k_search_full<Pol<true, T>><<<gW, 64, 0, s>>>(p);
        else k_search_full<Pol<false, T>><<<gW, 64, 0, s>>>(p);
    } else {
        if (kinds) k_search_half<Pol<true, T>><<<gW, 64, 0, s>>>(p);
        else k_search_half<Pol<false, T>><<<gW, 64, 0, s>>>(p);
    }
}

}  // namespace

// --------------------------------------------------------------------------
// Launchers
// --------------------------------------------------------------------------

hipError_t launch_init(const Plan& p, const double* d_state, const uint8_t* d_kind, hipStream_t s)
{
    const uint32_t b = 256;
    if (p.N > 0) k_init_particles<<<blocks_for(p.N, b), b, 0, s>>>(p, d_state, d_kind);
    k_fill_u32<<<blocks_for(p.C, b) < 4096 ? blocks_for(p.C, b) : 4096, b, 0, s>>>(p.count, p.C, 0u);
    if (p.N > 0) k_fill_u32<<<4096, b, 0, s>>>(p.sl_cnt, (size_t)p.N, 0u);
    k_init_ctl<<<1, 64, 0, s>>>(p, 0);
    if (p.N > 0 && p.nspecies > 0) k_check_kinds<<<blocks_for(p.N, b), b, 0, s>>>(p, d_kind);
    if (p.N > 0) k_bin<<<blocks_for(p.N, b), b, 0, s>>>(p);
    return hipGetLastError();
}

hipError_t launch_step(const Plan& p, hipStream_t s, hipEvent_t* ev)
{
    const uint32_t b = (uint32_t)p.block;
    const uint32_t gN = blocks_for(p.N, b);
    auto mark = [&](int k) { if (ev) (void)hipEventRecord(ev[k], s); };
    mark(KMC_PHASE_BIN);   // binning runs at the end of the previous step (k_resolve) or in kmc_init
    mark(KMC_PHASE_SCAN);
    k_scan_reduce<<<p.nblk_scan, kScanBlock, 0, s>>>(p);
    k_scan_partials<<<1, 1024, 0, s>>>(p);
    k_scan_down<<<p.nblk_scan, kScanBlock, 0, s>>>(p);
    if (p.adapt_L > 0 && p.N > 0) {
        // adaptive bins: split cells' leaf tables, then every particle's rank in its leaf
        k_refined_prep<<<kAdaptPrepBlocks, 64, 0, s>>>(p);
        k_leaf_count<<<gN, b, 0, s>>>(p);
        k_leaf_scan<<<kAdaptPrepBlocks, 64, 0, s>>>(p);
    }
    mark(KMC_PHASE_SCATTER);
    if (p.N > 0) {
        if (p.precision == KMC_FP32_SCREEN) k_scatter<true><<<gN, b, 0, s>>>(p);
        else k_scatter<false><<<gN, b, 0, s>>>(p);
    }
    k_adapt_dt<<<p.nboxes, 256, 0, s>>>(p);
    mark(KMC_PHASE_SEARCH);
    const uint32_t gW = blocks_for(p.N, 64);
    if (p.precision == KMC_FP32_SCREEN) {
        k_vmax_reduce<<<p.nboxes * kVmaxSplit, 256, 0, s>>>(p);
        k_screen_bounds<<<blocks_for(p.nboxes, 64), 64, 0, s>>>(p);
    }
    if (ev) (void)hipEventRecord(ev[KMC_PHASE_COUNT + 1], s);   // search kernel alone
    const bool full = p.search_mode == KMC_SEARCH_FULL;
    if (p.N > 0) {
        const bool kinds = p.nspecies > 0;
        if (p.precision == KMC_FP32_SCREEN) {
            if (p.tile == 1) launch_search<PolF32, TileF32_1>(kinds, full, gW, s, p);
            else if (p.tile == 2) launch_search<PolF32, TileF32_2>(kinds, full, gW, s, p);
            else launch_search<PolF32, TileF32_0>(kinds, full, gW, s, p);
        } else {
            if (p.tile == 1) launch_search<PolF64, TileF64_1>(kinds, full, gW, s, p);
            else if (p.tile == 2) launch_search<PolF64, TileF64_2>(kinds, full, gW, s, p);
            else launch_search<PolF64, TileF64_0>(kinds, full, gW, s, p);
        }
    }
    if (p.N > 0 && p.adapt_L > 0) {
        // the particles next to split cells: plain FP64 in both precisions
        // (their groups are leaves of a few particles, where the screen's
        // conversions and FP64 decisions cost more than they save)
        if (p.nspecies > 0) k_search_adapt<PolF64<true>><<<gW, 64, 0, s>>>(p);
        else k_search_adapt<PolF64<false>><<<gW, 64, 0, s>>>(p);
    }
    mark(KMC_PHASE_FINISH);
    if (p.N > 0 && !full) {
        k_distribute_overflow<<<256, 256, 0, s>>>(p);
        k_finish<<<blocks_for(p.N, 256), 256, 0, s>>>(p);
    }
    mark(KMC_PHASE_RECHECK);
    if (p.N > 0 && !full) k_recheck64<<<128, 256, 0, s>>>(p);
    // (the full search raises no overflow; the FP32 sorted copy may)
    if (p.N > 0 && (!full || p.precision == KMC_FP32_SCREEN)) {
        if (p.nspecies > 0) k_fallback_full<PolF64<true>><<<kFallbackBlocks, 64, 0, s>>>(p);
        else k_fallback_full<PolF64<false>><<<kFallbackBlocks, 64, 0, s>>>(p);
        if (p.adapt_L > 0) {
            if (p.nspecies > 0) k_fallback_adapt<PolF64<true>><<<kFallbackBlocks, 64, 0, s>>>(p);
            else k_fallback_adapt<PolF64<false>><<<kFallbackBlocks, 64, 0, s>>>(p);
        }
    }
    mark(KMC_PHASE_RESOLVE);
    if (p.N > 0) {
        if (p.nspecies > 0) k_resolve<true><<<gN, b, 0, s>>>(p);
        else k_resolve<false><<<gN, b, 0, s>>>(p);
    }
    k_advance<<<1, kAdvanceThreads, 0, s>>>(p);
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
