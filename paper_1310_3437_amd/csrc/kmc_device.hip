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
    const bool valid = i < p.N;
    uint32_t c = 0xFFFFFFFFu;
    if (valid) {
        const BoxDev& B = box_of(p, i);
        const size_t N = p.N;
        const int cx = cell1(p.A[i], B.lo[0], B.inv_h[0], B.nc[0]);
        const int cy = cell1(p.A[N + i], B.lo[1], B.inv_h[1], B.nc[1]);
        const int cz = cell1(p.A[2 * N + i], B.lo[2], B.inv_h[2], B.nc[2]);
        c = B.coff + (uint32_t)cx + (uint32_t)B.nc[0] * ((uint32_t)cy + (uint32_t)B.nc[1] * (uint32_t)cz);
        p.cell[i] = c;
    }
    // The state is still in the previous step's cell order, so neighbouring
    // lanes mostly share a cell: each run of equal cells takes its slots
    // with one atomic issued by the run's first lane.
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
    for (uint32_t b = threadIdx.x; b < p.nboxes; b += blockDim.x) p.box_vmax[b] = 0u;
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
// a3: cell-sorted copy of the state as 48-byte records; for the FP32 screen
// also an FP32 copy (positions relative to the box centre, velocities) and
// the per-box bound on |v_k| that the screen's error bounds need.
// --------------------------------------------------------------------------

template <bool F32>
__global__ void k_scatter(Plan p)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < p.N;
    const size_t N = p.N;
    float vm = 0.f;
    if (valid) {
        const uint32_t d = p.start[p.cell[i]] + p.slot[i];
        P64 r;
        r.x = p.A[i];
        r.y = p.A[N + i];
        r.z = p.A[2 * N + i];
        r.vx = p.A[3 * N + i];
        r.vy = p.A[4 * N + i];
        r.vz = p.A[5 * N + i];
        p.B[d] = r;
        p.idB[d] = p.idA[i];
        if (F32) vm = fmaxf(fabsf((float)r.vx), fmaxf(fabsf((float)r.vy), fabsf((float)r.vz)));
    }
    if (F32) {
        // per-block maximum of |fl32(v_k)|; k_vmax_reduce folds the blocks of each box
        __shared__ float wmax[16];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) vm = fmaxf(vm, __shfl_xor(vm, off, 64));
        if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = vm;
        __syncthreads();
        if (threadIdx.x == 0) {
            float m = 0.f;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = fmaxf(m, wmax[w]);
            p.vmax_part[blockIdx.x] = m;
        }
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

// Loose screen thresholds of every box for this step (FP64 arithmetic,
// rounded up).  They bound, over every neighbour pair of the box, the
// difference between the FP32 screen's b, -b - dt g2, c2 - D2 g2 and the
// FP64 definition's, from worst-case magnitudes |r_k| <= 2 h_k and
// |v_k| <= V (standard forward error analysis of sums and products,
// Higham 2002, ch. 3), times the guard factor.
__global__ void k_box_bounds(Plan p)
{
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= p.nboxes) return;
    const BoxDev& B = p.boxes[b];
    const float vm = __uint_as_float(p.box_vmax[b]);
    const double u = 0x1.0p-24, u64 = 0x1.0p-53;
    const double g3 = 3.0 * u / (1.0 - 3.0 * u) + 3.0 * u64 / (1.0 - 3.0 * u64);
    const double g2 = 2.0 * u / (1.0 - 2.0 * u) + 2.0 * u64 / (1.0 - 2.0 * u64);
    const double V = (double)vm * (1.0 + 3.0 * u);
    const double eg = 4.0001 * u * V;
    const double G = 2.0 * V;
    double R[3], er[3];
    for (int k = 0; k < 3; ++k) { R[k] = B.rmax[k]; er[k] = (double)B.er[k]; }
    double Eb = 0, Eg2 = 0, Ec2 = 0, sb = 0, sg = 0, sc = 0;
    for (int k = 0; k < 3; ++k) {
        Eb += R[k] * eg + G * er[k] + er[k] * eg;
        sb += (R[k] + er[k]) * (G + eg);
        Eg2 += 2.0 * G * eg + eg * eg;
        sg += (G + eg) * (G + eg);
    }
    Eb += g3 * sb;
    Eg2 += g3 * sg;
    for (int k = 0; k < 3; ++k) {
        const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        const double C = R[k1] * G + R[k2] * G;
        const double Ec = (R[k1] * eg + G * er[k1] + er[k1] * eg) + (R[k2] * eg + G * er[k2] + er[k2] * eg) +
                          g2 * ((R[k1] + er[k1]) * (G + eg) + (R[k2] + er[k2]) * (G + eg));
        Ec2 += 2.0 * C * Ec + Ec * Ec;
        sc += (C + Ec) * (C + Ec);
    }
    Ec2 += g3 * sc;
    const double G2max = 3.0 * (G + eg) * (G + eg);
    const double Et = Eb + B.dt * (1.0 + u) * Eg2 + 3.0 * u * B.dt * G2max;
    const double Ecc = Ec2 + B.D2 * (1.0 + u) * Eg2 + 3.0 * u * B.D2 * G2max;
    const double f = (double)p.guard * (1.0 + 1e-5);
    BoxStep st;
    st.Tb = (float)(f * Eb);
    st.Tt = (float)(f * Et);
    st.Tc = (float)(f * Ecc);
    st.vmax = (float)V;
    p.box_step[b] = st;
}

// --------------------------------------------------------------------------
// a4: DCA partner search.
//
// The pair quantities are symmetric under exchange of the two particles
// (r, g and r x g change sign, b, g2, c2 do not), so every unordered pair is
// tested once, from the particle whose cell comes first in a half
// neighbourhood: its own row from the particle onwards through cell cx+1,
// the row y+1 (cells cx-1..cx+1) and the three rows z+1 (y-1..y+1).  A pair
// that passes is recorded in the candidate lists of both particles; a
// per-particle finish pass then takes the exact FP64 (key, id) minimum, or,
// for the FP32 screen, classifies the recorded candidates.
//
// One wave (= one block of 64 threads) takes 64 consecutive cell-sorted
// particles, one per lane.  Lanes whose particles share a cell row form a
// group; for each of the five half-neighbourhood rows the group's window of
// cells is a contiguous range of the sorted arrays, which the wave stages
// into LDS in chunks with coalesced loads.  Each lane then tests its own
// sub-range of the window from LDS.
// --------------------------------------------------------------------------

// Exact FP64 search of one particle over its full 27-cell neighbourhood,
// straight from the sorted records (rechecks, list overflow, fallback).
__device__ int32_t search_one64(const Plan& p, uint32_t i)
{
    const BoxDev& B = box_of(p, i);
    const P64* __restrict__ X = p.B;
    const P64 me = X[i];
    const int cx = cell1(me.x, B.lo[0], B.inv_h[0], B.nc[0]);
    const int cy = cell1(me.y, B.lo[1], B.inv_h[1], B.nc[1]);
    const int cz = cell1(me.z, B.lo[2], B.inv_h[2], B.nc[2]);
    const double D2 = B.D2, dt = B.dt;
    double best_key = __builtin_inf();
    uint32_t best_id = 0xFFFFFFFFu;
    int32_t best = -1;
    for_each_range(B, cx, cy, cz, p.start, [&](uint32_t s, uint32_t e, int wx, int wy, int wz) {
        const bool shift = (wx | wy | wz) != 0;
        const double sx = (double)wx * B.L[0], sy = (double)wy * B.L[1], sz = (double)wz * B.L[2];
        for (uint32_t j = s; j < e; ++j) {
            const P64 q = X[j];
            double rx = q.x - me.x, ry = q.y - me.y, rz = q.z - me.z;
            if (shift) { rx = rx + sx; ry = ry + sy; rz = rz + sz; }
            const PairQ pq = pair_q(rx, ry, rz, q.vx - me.vx, q.vy - me.vy, q.vz - me.vz);
            if (accept(pq, D2, dt)) {   // the particle itself has g2 = 0 and is never accepted
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
    return best;
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

// Slot k of particle i's candidate list (slot 0 lives in a dense array: most
// particles have at most one candidate).
__device__ __forceinline__ uint32_t* slot_ptr(const Plan& p, uint32_t i, uint32_t k)
{
    return k == 0 ? p.sl_first + i : p.sl_idx + (size_t)i * (kSlots - 1) + (k - 1);
}

// Record the unordered pair {i, j} in the candidate lists of both.
__device__ __forceinline__ void record_pair(const Plan& p, uint32_t i, uint32_t j)
{
    uint32_t k = atomicAdd(&p.sl_cnt[i], 1u);
    if (k < (uint32_t)kSlots) *slot_ptr(p, i, k) = j;
    k = atomicAdd(&p.sl_cnt[j], 1u);
    if (k < (uint32_t)kSlots) *slot_ptr(p, j, k) = i;
}

// Pairs a lane found, kept in registers until the end of the wave's search
// (a global atomic inside the search loop would stall the whole wave); a
// lane that finds more records the excess at once.
constexpr int kReg = 4;

struct Found {
    uint32_t j[kReg];
    int n;
    __device__ __forceinline__ void add(const Plan& p, uint32_t i, uint32_t jj)
    {
        if (n < kReg) {
#pragma unroll
            for (int k = 0; k < kReg; ++k) j[k] = (n == k) ? jj : j[k];
            ++n;
        } else {
            record_pair(p, i, jj);
        }
    }
    // append the kept pairs to both candidate lists
    __device__ __forceinline__ void flush(const Plan& p, uint32_t i)
    {
        if (n == 0) return;
        const uint32_t base = atomicAdd(&p.sl_cnt[i], (unsigned int)n);
#pragma unroll
        for (int k = 0; k < kReg; ++k) {
            if (k < n) {
                if (base + k < (uint32_t)kSlots) *slot_ptr(p, i, base + k) = j[k];
                const uint32_t q = atomicAdd(&p.sl_cnt[j[k]], 1u);
                if (q < (uint32_t)kSlots) *slot_ptr(p, j[k], q) = i;
            }
        }
    }
};

struct PolF64 {
    static constexpr int W = 96;          // staged records per chunk (4.5 KiB)
    struct Lds {
        P64 rec[W];
    };
    struct Own {
        P64 me;
    };
    __device__ static void load_own(const Plan& p, uint32_t i, Own& o, double& x, double& y, double& z)
    {
        o.me = p.B[i];
        x = o.me.x; y = o.me.y; z = o.me.z;
    }
    __device__ static void stage(Lds& l, uint32_t t, const Plan& p, uint32_t j, const BoxDev&) { l.rec[t] = p.B[j]; }
    template <bool SH>
    __device__ static void scan(const Plan& p, const Lds& l, uint32_t c0, uint32_t j0, uint32_t j1, uint32_t i,
                                const Own& o, const BoxDev& B, const BoxStep& /*st*/, int wx, int wy, int wz,
                                Found& f)
    {
        const double sx = (double)wx * B.L[0], sy = (double)wy * B.L[1], sz = (double)wz * B.L[2];
        const double D2 = B.D2, dt = B.dt;
        for (uint32_t j = j0; j < j1; ++j) {
            const P64 q = l.rec[j - c0];
            double rx = q.x - o.me.x, ry = q.y - o.me.y, rz = q.z - o.me.z;
            if (SH) { rx = rx + sx; ry = ry + sy; rz = rz + sz; }
            const PairQ pq = pair_q(rx, ry, rz, q.vx - o.me.vx, q.vy - o.me.vy, q.vz - o.me.vz);
            if (accept(pq, D2, dt)) f.add(p, i, j);
        }
    }
};

// FP32 screen: a candidate is dropped only when the FP64 definition is
// certain to reject it (thresholds from the per-box bounds of this step).
struct PolF32 {
    static constexpr int W = 192;         // staged records per chunk (4.5 KiB)
    struct Lds {
        float4 a[W];
        float2 b[W];
    };
    struct Own {
        float x, y, z, vx, vy, vz;
    };
    __device__ static void load_own(const Plan& p, uint32_t i, Own& o, double& x, double& y, double& z)
    {
        const P64 m = p.B[i];
        const BoxDev& B = box_of(p, i);
        o.x = (float)(m.x - (double)B.ctr32[0]);
        o.y = (float)(m.y - (double)B.ctr32[1]);
        o.z = (float)(m.z - (double)B.ctr32[2]);
        o.vx = (float)m.vx; o.vy = (float)m.vy; o.vz = (float)m.vz;
        x = m.x; y = m.y; z = m.z;
    }
    // FP32 screen copy of a record: position relative to the box centre and
    // velocity, each rounded once to FP32 (the candidates staged belong to the
    // box of the staging group)
    __device__ static void stage(Lds& l, uint32_t t, const Plan& p, uint32_t j, const BoxDev& B)
    {
        const P64 q = p.B[j];
        l.a[t] = make_float4((float)(q.x - (double)B.ctr32[0]), (float)(q.y - (double)B.ctr32[1]),
                             (float)(q.z - (double)B.ctr32[2]), (float)q.vx);
        l.b[t] = make_float2((float)q.vy, (float)q.vz);
    }
    template <bool SH>
    __device__ static void scan(const Plan& p, const Lds& l, uint32_t c0, uint32_t j0, uint32_t j1, uint32_t i,
                                const Own& o, const BoxDev& B, const BoxStep& st, int wx, int wy, int wz,
                                Found& f)
    {
        const float sx = (float)wx * B.L32[0], sy = (float)wy * B.L32[1], sz = (float)wz * B.L32[2];
        const float D2 = B.D2_32, dt = B.dt_32;
        const float Tb = st.Tb, Tt = st.Tt, Tc = st.Tc;
        for (uint32_t j = j0; j < j1; ++j) {
            const float4 qa = l.a[j - c0];
            const float2 qb = l.b[j - c0];
            float rx = qa.x - o.x, ry = qa.y - o.y, rz = qa.z - o.z;
            if (SH) { rx = rx + sx; ry = ry + sy; rz = rz + sz; }
            const float gx = qa.w - o.vx, gy = qb.x - o.vy, gz = qb.y - o.vz;
            const float b = fmaf(rz, gz, fmaf(ry, gy, rx * gx));
            const float g2 = fmaf(gz, gz, fmaf(gy, gy, gx * gx));
            const float cx = fmaf(ry, gz, -(rz * gy));
            const float cy = fmaf(rz, gx, -(rx * gz));
            const float cz = fmaf(rx, gy, -(ry * gx));
            const float c2 = fmaf(cz, cz, fmaf(cy, cy, cx * cx));
            const float m2 = fmaf(-dt, g2, -b);
            const float m3 = fmaf(-D2, g2, c2);
            if ((b <= Tb) & (m2 <= Tt) & (m3 <= Tc)) f.add(p, i, j);
        }
    }
};

#ifndef KMC_SEARCH_WAVES_PER_EU
#define KMC_SEARCH_WAVES_PER_EU 5
#endif

template <class Pol>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(KMC_SEARCH_WAVES_PER_EU)))
void k_search_half(Plan p)
{
    __shared__ typename Pol::Lds lds;
    const int lane = threadIdx.x;
    const uint32_t i = blockIdx.x * 64u + (uint32_t)lane;
    const bool valid = i < p.N;
    uint32_t bidx = 0, rowkey = 0xFFFFFFFFu;
    int cx = 0, cy = 0, cz = 0;
    typename Pol::Own own;
    if (valid) {
        bidx = p.boxidx ? p.boxidx[i] : 0u;
        const BoxDev& B = p.boxes[bidx];
        double x, y, z;
        Pol::load_own(p, i, own, x, y, z);
        cx = cell1(x, B.lo[0], B.inv_h[0], B.nc[0]);
        cy = cell1(y, B.lo[1], B.inv_h[1], B.nc[1]);
        cz = cell1(z, B.lo[2], B.inv_h[2], B.nc[2]);
        rowkey = B.coff + (uint32_t)B.nc[0] * ((uint32_t)cy + (uint32_t)B.nc[1] * (uint32_t)cz);
    }
    Found found;
    found.n = 0;
#pragma unroll
    for (int k = 0; k < kReg; ++k) found.j[k] = 0;
    uint64_t remaining = __ballot(valid);
    while (remaining) {
        const int lead = __ffsll((unsigned long long)remaining) - 1;
        const uint32_t key = (uint32_t)__builtin_amdgcn_readlane((int)rowkey, lead);
        const uint64_t grp = __ballot(valid && rowkey == key) & remaining;
        remaining &= ~grp;
        const bool in = (grp >> lane) & 1ull;
        const int last = 63 - __clzll((long long)grp);
        const uint32_t gb = (uint32_t)__builtin_amdgcn_readlane((int)bidx, lead);
        const BoxDev& B = p.boxes[gb];
        const BoxStep st = p.box_step[gb];
        const int gcy = __builtin_amdgcn_readlane(cy, lead), gcz = __builtin_amdgcn_readlane(cz, lead);
        const int cxf = __builtin_amdgcn_readlane(cx, lead), cxl = __builtin_amdgcn_readlane(cx, last);
        const int NX = B.nc[0], NY = B.nc[1], NZ = B.nc[2];
        // Cells [ca, cb] of a row seen with image shift (wx, wy, wz); each lane
        // tests the sub-range [ls, le) of it (empty when ls >= le).
        auto part = [&](uint32_t row, int ca, int cb, uint32_t ls, uint32_t le, int wx, int wy, int wz) {
            const uint32_t gs = p.start[row + ca], ge = p.start[row + cb + 1];
            const bool sh = (wx | wy | wz) != 0;
            for (uint32_t c0 = gs; c0 < ge; c0 += (uint32_t)Pol::W) {
                const uint32_t n = min((uint32_t)Pol::W, ge - c0);
                for (uint32_t t = (uint32_t)lane; t < n; t += 64u) Pol::stage(lds, t, p, c0 + t, B);
                __syncthreads();
                const uint32_t j0 = max(ls, c0), j1 = min(le, c0 + n);
                if (sh) Pol::template scan<true>(p, lds, c0, j0, j1, i, own, B, st, wx, wy, wz, found);
                else Pol::template scan<false>(p, lds, c0, j0, j1, i, own, B, st, wx, wy, wz, found);
                __syncthreads();
            }
        };
        // a wrapped end cell of a periodic x axis, used by lanes at that end
        auto wrap_cell = [&](uint32_t row, int cell, bool use, int wx, int wy, int wz) {
            part(row, cell, cell, use ? 0u : 1u, use ? 0xFFFFFFFFu : 0u, wx, wy, wz);
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
            part(row, cxf, cb, ls, le, 0, 0, 0);
            if (B.periodic[0] && cxl + 1 >= NX) wrap_cell(row, 0, in && cx == NX - 1, 1, 0, 0);
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
            part(row, cxf - 1 < 0 ? 0 : cxf - 1, cxl + 1 >= NX ? NX - 1 : cxl + 1, ls, le, 0, wy, wz);
            if (B.periodic[0]) {
                if (cxf - 1 < 0) wrap_cell(row, NX - 1, in && cx == 0, -1, wy, wz);
                if (cxl + 1 >= NX) wrap_cell(row, 0, in && cx == NX - 1, 1, wy, wz);
            }
        }
    }
    if (valid) found.flush(p, i);
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

// Partner of every particle from its recorded candidates (FP64: all of
// them are acceptable; the (key, id) minimum is taken with exact keys).
__global__ __launch_bounds__(256) void k_finish64(Plan p)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < p.N;
    const uint32_t cnt = valid ? p.sl_cnt[i] : 0u;
    int32_t best = -1;
    if (cnt != 0) p.sl_cnt[i] = 0u;
    if (cnt == 1) {
        best = (int32_t)p.sl_first[i];
    } else if (cnt > 1 && cnt <= (uint32_t)kSlots) {
        const BoxDev& B = box_of(p, i);
        const P64 me = p.B[i];
        double best_key = __builtin_inf();
        uint32_t best_id = 0xFFFFFFFFu;
        for (uint32_t k = 0; k < cnt; ++k) {
            const uint32_t j = *slot_ptr(p, i, k);
            const P64 q = p.B[j];
            double r[3];
            rel64(B, me, q, r);
            const PairQ pq = pair_q(r[0], r[1], r[2], q.vx - me.vx, q.vy - me.vy, q.vz - me.vz);
            const double key = pq.c2 / pq.g2;
            const uint32_t idj = p.idB[j];
            if (key < best_key || (key == best_key && idj < best_id)) {
                best_key = key;
                best_id = idj;
                best = (int32_t)j;
            }
        }
    }
    // more candidates than slots: the particle is searched again in full
    const bool need = cnt > (uint32_t)kSlots;
    push_recheck(p, i, need);
    if (valid) p.partner[i] = best;
}

// FP32 screen finish: every recorded candidate is classified with per-pair
// rounding-error bounds (Higham 2002, ch. 3) into certainly rejected,
// certainly accepted or undecided by the FP64 definition, with an interval
// that certainly contains its FP64 key.  The partner is certain when the
// candidate with the lowest key bound is certainly accepted and its upper
// bound lies below every other candidate's lower bound; otherwise the
// particle is appended to the FP64 recheck list.
__global__ __launch_bounds__(256) void k_finish32(Plan p)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < p.N;
    bool need = false;
    int32_t best = -1;
    if (valid) {
        const uint32_t cnt = p.sl_cnt[i];
        if (cnt != 0) p.sl_cnt[i] = 0u;
        if (cnt > (uint32_t)kSlots) {
            need = true;
        } else if (cnt > 0) {
            const BoxDev& B = box_of(p, i);
            const float u = 0x1.0p-24f;
            const float g3 = 3.0f * u * 1.001f + 4e-16f;
            const float g2c = 2.0f * u * 1.001f + 3e-16f;
            const float gf = p.guard * 1.001f;
            float lo1 = __builtin_inff(), hi1 = __builtin_inff(), lo2 = __builtin_inff();
            int st1 = 0;                       // 0 none, 1 accepted, 2 undecided
            uint32_t j1 = 0;
            const P64 mi = p.B[i];
            const double xi[3] = {mi.x, mi.y, mi.z};
            const float pi[3] = {(float)(mi.x - (double)B.ctr32[0]), (float)(mi.y - (double)B.ctr32[1]),
                                 (float)(mi.z - (double)B.ctr32[2])};
            const float vi[3] = {(float)mi.vx, (float)mi.vy, (float)mi.vz};
            for (uint32_t k = 0; k < cnt; ++k) {
                const uint32_t j = *slot_ptr(p, i, k);
                const P64 qj = p.B[j];
                const double xj[3] = {qj.x, qj.y, qj.z};
                const float pj[3] = {(float)(qj.x - (double)B.ctr32[0]), (float)(qj.y - (double)B.ctr32[1]),
                                     (float)(qj.z - (double)B.ctr32[2])};
                const float vj[3] = {(float)qj.vx, (float)qj.vy, (float)qj.vz};
                float r[3], g[3], ar[3], ag[3], eg[3], er[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const int ci = cell1(xi[a], B.lo[a], B.inv_h[a], B.nc[a]);
                    const int cj = cell1(xj[a], B.lo[a], B.inv_h[a], B.nc[a]);
                    const int w = wrap_of(ci, cj, B.nc[a], B.periodic[a]);
                    r[a] = pj[a] - pi[a];
                    if (w != 0) r[a] = r[a] + (float)w * B.L32[a];
                    g[a] = vj[a] - vi[a];
                    er[a] = B.er[a];
                    eg[a] = u * 1.0001f * (fabsf(vi[a]) + fabsf(vj[a]) + fabsf(g[a]));
                    ar[a] = fabsf(r[a]) + er[a];
                    ag[a] = fabsf(g[a]) + eg[a];
                }
                const float b = fmaf(r[2], g[2], fmaf(r[1], g[1], r[0] * g[0]));
                const float gg = fmaf(g[2], g[2], fmaf(g[1], g[1], g[0] * g[0]));
                float c[3];
                c[0] = fmaf(r[1], g[2], -(r[2] * g[1]));
                c[1] = fmaf(r[2], g[0], -(r[0] * g[2]));
                c[2] = fmaf(r[0], g[1], -(r[1] * g[0]));
                const float cc = fmaf(c[2], c[2], fmaf(c[1], c[1], c[0] * c[0]));
                const float m2 = fmaf(-B.dt_32, gg, -b);
                const float m3 = fmaf(-B.D2_32, gg, cc);
                float Eb = 0.f, Eg = 0.f, sb = 0.f, sg = 0.f, Ecc = 0.f, scc = 0.f;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    Eb += ar[a] * eg[a] + ag[a] * er[a];
                    sb += ar[a] * ag[a];
                    Eg += 2.0f * ag[a] * eg[a];
                    sg += ag[a] * ag[a];
                }
                Eb += g3 * sb;
                Eg += g3 * sg;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
                    const float Ec = ar[a1] * eg[a2] + ag[a2] * er[a1] + ar[a2] * eg[a1] + ag[a1] * er[a2] +
                                     g2c * (ar[a1] * ag[a2] + ar[a2] * ag[a1]);
                    const float ac = fabsf(c[a]) + Ec;
                    Ecc += 2.0f * ac * Ec;
                    scc += ac * ac;
                }
                Ecc += g3 * scc;
                Eb *= gf;
                Eg *= gf;
                Ecc *= gf;
                const float Et = Eb + B.dt_32 * (1.0f + 2.0f * u) * Eg +
                                 gf * (3.0f * u * B.dt_32 * (gg + Eg) + 2.0f * u * fabsf(m2));
                const float Ec3 = Ecc + B.D2_32 * (1.0f + 2.0f * u) * Eg +
                                  gf * (3.0f * u * B.D2_32 * (gg + Eg) + 2.0f * u * fabsf(m3));
                const bool rej = (b > Eb) | (m2 > Et) | (m3 > Ec3);
                if (rej) continue;
                const bool acc = (b < -Eb) & (m2 < -Et) & (m3 < -Ec3) & (gg > Eg);
                const float kl = fmaxf(cc - Ecc, 0.0f) / (gg + Eg) * (1.0f - 4.0f * u);
                const float kh = gg > Eg ? (cc + Ecc) / (gg - Eg) * (1.0f + 4.0f * u) : __builtin_inff();
                if (kl < lo1) {
                    lo2 = lo1;
                    lo1 = kl;
                    hi1 = kh;
                    st1 = acc ? 1 : 2;
                    j1 = j;
                } else if (kl < lo2) {
                    lo2 = kl;
                }
            }
            if (st1 == 0) best = -1;
            else if (st1 == 1 && hi1 < lo2) best = (int32_t)j1;
            else need = true;
        }
    }
    // undecided particles go to the FP64 recheck
    push_recheck(p, i, need);
    if (valid) p.partner[i] = need ? -1 : best;
}

// FP64 re-search of the particles the screen left undecided.
__global__ void k_recheck64(Plan p)
{
    const uint32_t cnt = p.ctl->recheck_count;
    const uint32_t n = cnt < p.recheck_cap ? cnt : p.recheck_cap;
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        const uint32_t i = p.recheck[k];
        p.partner[i] = search_one64(p, i);
    }
}

// Whole-step FP64 search when the recheck list overflowed (exits at once
// otherwise).
__global__ void k_fallback64(Plan p)
{
    if (p.ctl->overflow == 0u) return;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < p.N; i += gridDim.x * blockDim.x)
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
        const P64 me = p.B[i];
        double x[3] = {me.x, me.y, me.z}, v[3] = {me.vx, me.vy, me.vz};
        const uint32_t id = p.idB[i];
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
        const P64 me = p.B[i];
        const int cx = cell1(me.x, B.lo[0], B.inv_h[0], B.nc[0]);
        const int cy = cell1(me.y, B.lo[1], B.inv_h[1], B.nc[1]);
        const int cz = cell1(me.z, B.lo[2], B.inv_h[2], B.nc[2]);
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
    if (p.N > 0) k_fill_u32<<<4096, b, 0, s>>>(p.sl_cnt, (size_t)p.N, 0u);
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
    const uint32_t gW = blocks_for(p.N, 64);
    if (p.precision == KMC_FP32_SCREEN) {
        k_vmax_reduce<<<p.nboxes * kVmaxSplit, 256, 0, s>>>(p);
        k_box_bounds<<<blocks_for(p.nboxes, 64), 64, 0, s>>>(p);
        if (p.N > 0) {
            k_search_half<PolF32><<<gW, 64, 0, s>>>(p);
            k_finish32<<<blocks_for(p.N, 256), 256, 0, s>>>(p);
        }
    } else if (p.N > 0) {
        k_search_half<PolF64><<<gW, 64, 0, s>>>(p);
        k_finish64<<<blocks_for(p.N, 256), 256, 0, s>>>(p);
    }
    mark(KMC_PHASE_RECHECK);
    if (p.N > 0) {
        k_recheck64<<<512, 256, 0, s>>>(p);
        k_fallback64<<<2048, 256, 0, s>>>(p);
    }
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
