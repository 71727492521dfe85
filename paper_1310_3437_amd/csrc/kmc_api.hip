// kmc_api.hip -- host runtime of libkmc.so: the C ABI declared in kmc.h.
//
// Parameter validation, workspace layout, kernel launch plan, optional
// hipGraph capture of one step, read-back, statistics.  The library never
// allocates device memory: everything lives in the caller's workspace, or,
// for kmc_init_scratch, in a static per-device array of the library.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "kmc_internal.h"

using namespace kmc;

static_assert(sizeof(kmc_box) == 128, "kmc_box layout");
static_assert(sizeof(kmc_config) == 96, "kmc_config layout");
static_assert(sizeof(kmc_species) == 144, "kmc_species layout");
static_assert(KMC_MAX_SPECIES == kMaxKinds, "kind table stride");

struct kmc_ctx {
    Plan plan{};
    kmc_config cfg{};
    kmc_species species{};   // copy of the caller's kinds (cfg.species points here)
    std::vector<kmc_box> boxes;
    int device = 0;
    bool stepped = false;
    // graph replay
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // profile mode: one set of phase events per step, folded in get_stats
    std::vector<hipEvent_t> ev_free;
    std::vector<std::vector<hipEvent_t>> ev_pending;
    double ms[8] = {0};
    double search_kernel_ms = 0;
    uint64_t timed_steps = 0;
};

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

int check_box(const kmc_box& b)
{
    if (b.geometry != KMC_GEOM_BOX && b.geometry != KMC_GEOM_SPHERE) return KMC_EINVAL;
    if (!finite_pos(b.D2) || !finite_pos(b.dt)) return KMC_EINVAL;
    const double D = std::sqrt(b.D2);
    for (int k = 0; k < 3; ++k) {
        if (b.bc[k] != KMC_BC_REFLECT && b.bc[k] != KMC_BC_PERIODIC && b.bc[k] != KMC_BC_ABSORB) return KMC_EINVAL;
        if (b.bc[k] == KMC_BC_ABSORB && b.geometry != KMC_GEOM_BOX) return KMC_EINVAL;
        if (b.ncell[k] < 1) return KMC_EINVAL;
        if (b.bc[k] == KMC_BC_PERIODIC && b.ncell[k] < 3) return KMC_EINVAL;
        if (!std::isfinite(b.lo[k]) || !std::isfinite(b.hi[k]) || !(b.hi[k] > b.lo[k])) return KMC_EINVAL;
        if (!finite_pos(b.inv_h[k])) return KMC_EINVAL;
        // inv_h must be ncell / (hi - lo) up to its rounding: binning uses
        // the caller's value, while the FP32 screen's error bounds take the
        // cell edge (hi - lo) / ncell, so a coarser binning would break them
        if (std::fabs(b.inv_h[k] * (b.hi[k] - b.lo[k]) / (double)b.ncell[k] - 1.0) > 1e-12) return KMC_EINVAL;
        // the 27-cell neighbourhood must contain every point closer than D
        if (b.inv_h[k] * D > 1.0 + 1e-9) return KMC_EINVAL;
        if (b.geometry == KMC_GEOM_SPHERE) {
            if (b.bc[k] != KMC_BC_REFLECT) return KMC_EINVAL;
            if (!finite_pos(b.sphere_r) || b.lo[k] > -b.sphere_r || b.hi[k] < b.sphere_r) return KMC_EINVAL;
        }
    }
    return KMC_OK;
}

int check_cfg(const kmc_config& c)
{
    if (c.precision != KMC_FP64 && c.precision != KMC_FP32_SCREEN) return KMC_EINVAL;
    if (c.kinematics != KMC_KIN_AT_TSTAR && c.kinematics != KMC_KIN_VEL_ONLY) return KMC_EINVAL;
    if (c.block_size != 0 && (c.block_size < 64 || c.block_size > 1024 || c.block_size % 64 != 0)) return KMC_EINVAL;
    if (c.use_graph != 0 && c.use_graph != 1) return KMC_EINVAL;
    if (c.profile != 0 && c.profile != 1) return KMC_EINVAL;
    if (!std::isfinite(c.guard_scale) || (c.guard_scale != 0.0 && c.guard_scale != -1.0 && c.guard_scale < 1.0))
        return KMC_EINVAL;
    if (c.dt_rule != KMC_DT_FIXED && c.dt_rule != KMC_DT_ADAPTIVE) return KMC_EINVAL;
    if (c.search_mode != KMC_SEARCH_HALF && c.search_mode != KMC_SEARCH_FULL) return KMC_EINVAL;
    if (c.dims != 0 && c.dims != 2 && c.dims != 3) return KMC_EINVAL;
    if (c.dt_factor != 0.0 && !finite_pos(c.dt_factor)) return KMC_EINVAL;
    if (c.tile < 0 || c.tile > 2) return KMC_EINVAL;
    if (c.reserved != 0) return KMC_EINVAL;
    if (c.adapt_levels < 0 || c.adapt_levels > 3) return KMC_EINVAL;
    if (c.adapt_levels > 0 &&
        (c.adapt_threshold < 1 || c.search_mode != KMC_SEARCH_FULL || c.dims == 2))
        return KMC_EINVAL;
    if (c.species) {
        const kmc_species& sp = *c.species;
        if (sp.count < 1 || sp.count > KMC_MAX_SPECIES || sp.reserved != 0) return KMC_EINVAL;
        for (uint32_t k = 0; k < sp.count; ++k)
            if (!finite_pos(sp.radius[k]) || !finite_pos(sp.mass[k])) return KMC_EINVAL;
    }
    return KMC_OK;
}

// Squared diameter of a pair of kinds: (radius_s + radius_t)^2 in binary64.
double kinds_D2(const kmc_species& sp, uint32_t s, uint32_t t)
{
    const double d = sp.radius[s] + sp.radius[t];
    return d * d;
}

double kinds_D2max(const kmc_species& sp)
{
    double m = 0.0;
    for (uint32_t s = 0; s < sp.count; ++s)
        for (uint32_t t = 0; t < sp.count; ++t) m = std::max(m, kinds_D2(sp, s, t));
    return m;
}

struct Totals {
    uint64_t N = 0, C = 0;
};

int totals(const kmc_box* boxes, uint32_t nboxes, Totals& t)
{
    for (uint32_t b = 0; b < nboxes; ++b) {
        t.N += boxes[b].n;
        t.C += (uint64_t)boxes[b].ncell[0] * (uint64_t)boxes[b].ncell[1] * (uint64_t)boxes[b].ncell[2] + 1u;
    }
    if (t.N > 0x7FFFFFFFull) return KMC_EOVERFLOW;
    if (t.C > 0xFFFFFFFEull) return KMC_EOVERFLOW;
    return KMC_OK;
}

int validate(const kmc_box* boxes, uint32_t nboxes, const kmc_config* cfg, Totals& t)
{
    if (!boxes || !cfg || nboxes == 0) return KMC_EINVAL;
    for (uint32_t b = 0; b < nboxes; ++b) {
        int rc = check_box(boxes[b]);
        if (rc != KMC_OK) return rc;
    }
    int rc = check_cfg(*cfg);
    if (rc != KMC_OK) return rc;
    if (cfg->adapt_levels > 0)
        for (uint32_t b = 0; b < nboxes; ++b)
            for (int k = 0; k < 3; ++k)
                if (boxes[b].bc[k] == KMC_BC_ABSORB || boxes[b].ncell[k] > (1 << 27)) return KMC_EINVAL;
    if (cfg->dims == 2)
        for (uint32_t b = 0; b < nboxes; ++b)
            if (boxes[b].ncell[2] != 1 || boxes[b].bc[2] != KMC_BC_REFLECT || boxes[b].geometry != KMC_GEOM_BOX)
                return KMC_EINVAL;
    if (cfg->species) {
        // every neighbour closer than the largest pair diameter lies in the 27 cells
        const double Dmax = std::sqrt(kinds_D2max(*cfg->species));
        for (uint32_t b = 0; b < nboxes; ++b)
            for (int k = 0; k < 3; ++k)
                if (boxes[b].inv_h[k] * Dmax > 1.0 + 1e-9) return KMC_EINVAL;
    }
    return totals(boxes, nboxes, t);
}

uint32_t history_len(const kmc_config& c) { return c.history ? c.history : 1024u; }

// Carve the workspace; with base == nullptr only the size is computed.
size_t layout(Plan& p, char* base, uint32_t nboxes, const kmc_config& cfg, const Totals& t)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* ptr = base ? base + off : nullptr;
        off += align_up(bytes);
        return ptr;
    };
    const size_t N = t.N, C = t.C;
    const uint32_t H = history_len(cfg);
    const uint32_t nblk = (uint32_t)((C + kScanTile - 1) / kScanTile);
    const uint32_t cap = cfg.recheck_capacity ? cfg.recheck_capacity : (uint32_t)N;
    p.ctl = (Ctl*)take(sizeof(Ctl));
    p.boxes = (BoxDev*)take(sizeof(BoxDev) * nboxes);
    p.hist_np = (unsigned long long*)take(sizeof(unsigned long long) * H);
    p.hist_dig = (unsigned long long*)take(sizeof(unsigned long long) * H);
    p.acc = (StepAcc*)take(sizeof(StepAcc) * kAccLanes);
    p.A = (double*)take(sizeof(double) * 6 * N);
    p.B = (P64*)take(sizeof(P64) * N);
    const uint32_t blk = cfg.block_size ? (uint32_t)cfg.block_size : 256u;
    const uint32_t nblk_part = (uint32_t)((N + blk - 1) / blk);
    p.vmax_part = (float*)take(sizeof(float) * (nblk_part ? nblk_part : 1));
    p.box_vmax = (unsigned int*)take(sizeof(unsigned int) * nboxes);
    p.v2_part = (unsigned long long*)take(sizeof(unsigned long long) * (nblk_part ? nblk_part : 1));
    p.box_v2 = (unsigned long long*)take(sizeof(unsigned long long) * nboxes);
    p.box_sb = (ScreenBounds*)take(sizeof(ScreenBounds) * kSpanClasses * nboxes);
    p.idA = (uint32_t*)take(4 * N);
    p.idB = (uint32_t*)take(4 * N);
    // the binned cell is stored only for adaptive bins (the uniform grid's
    // sorted copy recomputes it from the position)
    p.cell = cfg.adapt_levels > 0 ? (uint32_t*)take(4 * N) : nullptr;
    p.slot = (uint32_t*)take(4 * N);
    p.partner = (int32_t*)take(4 * N);
    p.sl_cnt = (uint32_t*)take(4 * N);
    p.sl = (SlotEntry*)take(sizeof(SlotEntry) * N * kSlots);
    p.fb_key = (double*)take(8 * N);
    p.fb_j = (int32_t*)take(4 * N);
    p.boxidx = nboxes > 1 ? (uint32_t*)take(4 * N) : nullptr;
    p.count = (uint32_t*)take(4 * C);
    p.start = (uint32_t*)take(4 * (C + 1));
    p.partial = (uint32_t*)take(4 * (size_t)(nblk ? nblk : 1));
    p.recheck = (uint32_t*)take(4 * (size_t)(cap ? cap : 1));
    p.ovf = (uint2*)take(sizeof(uint2) * 2 * (N ? N : 1));
    p.adapt_L = cfg.adapt_levels;
    p.adapt_T = cfg.adapt_threshold;
    if (cfg.adapt_levels > 0) {
        // leaf tables: a split bin at level l holds more than T 8^(l-1)
        // particles, so the 8^l + 1 entries of all split bins number at most
        // 8 N / T + N + 1
        const size_t cap = 8 * N / cfg.adapt_threshold + N + 1;
        p.level = (uint8_t*)take(C ? C : 1);
        p.mixed = (uint8_t*)take(C ? C : 1);
        p.pool_base = (uint32_t*)take(4 * (C ? C : 1));
        p.refined = (uint32_t*)take(4 * (C ? C : 1));
        p.pool = (uint32_t*)take(4 * cap);
        p.leaf_slot = (uint32_t*)take(4 * (N ? N : 1));
        p.pool_cap = (uint32_t)std::min<size_t>(cap, 0xFFFFFFFFu);
    } else {
        p.level = p.mixed = nullptr;
        p.pool_base = p.refined = p.pool = p.leaf_slot = nullptr;
        p.pool_cap = 0;
    }
    p.nspecies = cfg.species ? (int32_t)cfg.species->count : 0;
    if (cfg.species) {
        p.spA = (uint8_t*)take(N ? N : 1);
        p.spB = (uint8_t*)take(N ? N : 1);
        p.sp_D2 = (const double*)take(sizeof(double) * kMaxKinds * kMaxKinds);
        p.sp_mass = (const double*)take(sizeof(double) * kMaxKinds);
        p.box_kD2 = (float*)take(sizeof(float) * kMaxKinds * kMaxKinds * kSpanClasses * nboxes);
    } else {
        p.spA = p.spB = nullptr;
        p.sp_D2 = p.sp_mass = nullptr;
        p.box_kD2 = nullptr;
    }
    p.N = (uint32_t)N;
    p.C = (uint32_t)C;
    p.nboxes = nboxes;
    p.H = H;
    p.nblk_scan = nblk;
    p.recheck_cap = cap;
    p.ovf_cap = (uint32_t)(N ? 2 * N : 1);
    p.seed = cfg.seed;
    p.precision = cfg.precision;
    p.kinematics = cfg.kinematics;
    p.block = cfg.block_size ? cfg.block_size : 256;
    p.nblk_part = nblk_part;
    p.guard = cfg.guard_scale > 0.0 ? (float)cfg.guard_scale : (cfg.guard_scale < 0.0 ? 0.0f : 4.0f);
    p.dt_rule = cfg.dt_rule;
    p.search_mode = cfg.search_mode;
    p.tile = cfg.tile;
    p.dims = cfg.dims == 2 ? 2 : 3;
    p.dt_factor = cfg.dt_factor != 0.0 ? cfg.dt_factor : 1.0;
    return off;
}

void fill_box_dev(BoxDev& d, const kmc_box& b, uint32_t coff, uint32_t poff)
{
    std::memset(&d, 0, sizeof(d));
    for (int k = 0; k < 3; ++k) {
        d.lo[k] = b.lo[k];
        d.hi[k] = b.hi[k];
        d.L[k] = b.hi[k] - b.lo[k];
        d.inv_h[k] = b.inv_h[k];
        d.nc[k] = b.ncell[k];
        d.periodic[k] = b.bc[k] == KMC_BC_PERIODIC ? 1 : 0;
        d.absorb[k] = b.bc[k] == KMC_BC_ABSORB ? 1 : 0;
    }
    // Bound on |r_k| for a neighbour pair (the FP32 screen's error bounds
    // scale with it): two cell edges, plus rounding of the cell index.
    for (int k = 0; k < 3; ++k) {
        const double h = d.L[k] / (double)b.ncell[k];
        d.rmax[k] = 2.0 * h * (1.0 + 1e-9);
    }
    d.D2 = b.D2;
    d.dt = b.dt;
    d.dt_cap = b.dt;
    for (int k = 0; k < 3; ++k) d.h[k] = d.L[k] / (double)b.ncell[k];
    d.dx = d.L[0] / (double)b.ncell[0];
    for (int k = 1; k < 3; ++k) {
        const double e = d.L[k] / (double)b.ncell[k];
        if (e < d.dx) d.dx = e;
    }
    d.time = 0.0;
    d.sphere = b.geometry == KMC_GEOM_SPHERE ? 1 : 0;
    d.R = b.sphere_r;
    d.R2 = b.sphere_r * b.sphere_r;
    d.coff = coff;
    d.poff = poff;
    d.n = b.n;
    d.D2_32 = (float)b.D2;
    d.dt_32 = (float)b.dt;
}

int dev_err(hipError_t e) { return e == hipSuccess ? KMC_OK : KMC_EDEVICE; }

}  // namespace

// Workspace of kmc_init_scratch: one copy per GPU, resident until the process
// ends.  In host code its name is only a handle: the device address comes
// from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[KMC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array.
int scratch_of_current_device(void** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return KMC_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return KMC_EDEVICE;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return KMC_OK;
}

void fold_events(kmc_ctx* c)
{
    for (auto& set : c->ev_pending) {
        for (int k = 0; k < KMC_PHASE_COUNT; ++k) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, set[k], set[k + 1]) == hipSuccess) c->ms[k] += ms;
        }
        float ks = 0.f;
        if (hipEventElapsedTime(&ks, set[KMC_PHASE_COUNT + 1], set[KMC_PHASE_FINISH]) == hipSuccess)
            c->search_kernel_ms += ks;
        c->timed_steps += 1;
        for (auto e : set) c->ev_free.push_back(e);
    }
    c->ev_pending.clear();
}

}  // namespace

extern "C" {

int kmc_abi_version(void) { return KMC_ABI_VERSION; }

const char* kmc_strerror(int status)
{
    switch (status) {
    case KMC_OK: return "ok";
    case KMC_EINVAL: return "invalid argument";
    case KMC_ENOMEM: return "workspace too small or host allocation failed";
    case KMC_EDEVICE: return "HIP runtime error";
    case KMC_EOVERFLOW: return "size exceeds the library's index range";
    case KMC_ESTATE: return "call not valid in the current state";
    default: return "unknown status";
    }
}

int kmc_workspace_bytes(const kmc_box* boxes, uint32_t nboxes, const kmc_config* cfg, size_t* bytes)
{
    if (!bytes) return KMC_EINVAL;
    Totals t;
    int rc = validate(boxes, nboxes, cfg, t);
    if (rc != KMC_OK) return rc;
    Plan p;
    *bytes = layout(p, nullptr, nboxes, *cfg, t);
    return KMC_OK;
}

int kmc_init(const kmc_box* boxes, uint32_t nboxes, const kmc_config* cfg, const double* d_state,
             void* d_workspace, size_t workspace_bytes, void* stream, kmc_ctx** out)
{
    if (!out || !d_workspace) return KMC_EINVAL;
    *out = nullptr;
    Totals t;
    int rc = validate(boxes, nboxes, cfg, t);
    if (rc != KMC_OK) return rc;
    if (t.N > 0 && !d_state) return KMC_EINVAL;
    if ((uintptr_t)d_workspace % kAlign != 0) return KMC_EINVAL;
    Plan probe;
    const size_t need = layout(probe, nullptr, nboxes, *cfg, t);
    if (workspace_bytes < need) return KMC_ENOMEM;

    if (cfg->species && t.N > 0 && !cfg->species->d_kind) return KMC_EINVAL;
    kmc_ctx* c = new (std::nothrow) kmc_ctx();
    if (!c) return KMC_ENOMEM;
    c->cfg = *cfg;
    if (cfg->species) {
        c->species = *cfg->species;
        c->species.d_kind = nullptr;   // read once, below
        c->cfg.species = &c->species;
    }
    c->boxes.assign(boxes, boxes + nboxes);
    layout(c->plan, (char*)d_workspace, nboxes, *cfg, t);
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return KMC_EDEVICE; }

    std::vector<BoxDev> bd(nboxes);
    uint64_t coff = 0, poff = 0;
    for (uint32_t b = 0; b < nboxes; ++b) {
        fill_box_dev(bd[b], boxes[b], (uint32_t)coff, (uint32_t)poff);
        coff += (uint64_t)boxes[b].ncell[0] * boxes[b].ncell[1] * boxes[b].ncell[2] + 1u;   // + absorbed cell
        poff += boxes[b].n;
    }
    // particle kinds: the pair tables, and each box's D2 is the largest pair value
    std::vector<double> d2tab(kMaxKinds * kMaxKinds, 0.0), mtab(kMaxKinds, 0.0);
    if (cfg->species) {
        const kmc_species& sp = *cfg->species;
        for (uint32_t a = 0; a < sp.count; ++a) {
            mtab[a] = sp.mass[a];
            for (uint32_t b2 = 0; b2 < sp.count; ++b2) d2tab[a * kMaxKinds + b2] = kinds_D2(sp, a, b2);
        }
        const double D2max = kinds_D2max(sp);
        for (auto& d : bd) {
            d.D2 = D2max;
            d.D2_32 = (float)D2max;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(c->plan.boxes, bd.data(), sizeof(BoxDev) * nboxes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && cfg->species) {
        e = hipMemcpyAsync((void*)c->plan.sp_D2, d2tab.data(), sizeof(double) * d2tab.size(), hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync((void*)c->plan.sp_mass, mtab.data(), sizeof(double) * mtab.size(), hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) e = launch_init(c->plan, d_state, cfg->species ? cfg->species->d_kind : nullptr, s);
    unsigned long long bad_kinds = 0;
    if (e == hipSuccess) {
        // the step counter starts at step0 (k_init_ctl wrote 0); the kind
        // check counted its failures in the control block's scratch word
        unsigned long long step0 = cfg->step0;
        e = hipMemcpyAsync(&c->plan.ctl->step, &step0, sizeof(step0), hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&bad_kinds, &c->plan.ctl->scratch, sizeof(bad_kinds), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);   // host buffers live on this stack frame
    }
    if (e != hipSuccess) { delete c; return KMC_EDEVICE; }
    if (bad_kinds != 0) { delete c; return KMC_EINVAL; }
    *out = c;
    return KMC_OK;
}

int kmc_init_scratch(const kmc_box* boxes, uint32_t nboxes, const kmc_config* cfg, const double* d_state,
                     void* stream, kmc_ctx** out)
{
    if (!out) return KMC_EINVAL;
    *out = nullptr;
    Totals t;
    int rc = validate(boxes, nboxes, cfg, t);
    if (rc != KMC_OK) return rc;
    Plan probe;
    if (layout(probe, nullptr, nboxes, *cfg, t) > KMC_SCRATCH_BYTES) return KMC_ENOMEM;
    void* ws = nullptr;
    rc = scratch_of_current_device(&ws);
    if (rc != KMC_OK) return rc;
    return kmc_init(boxes, nboxes, cfg, d_state, ws, KMC_SCRATCH_BYTES, stream, out);
}

int kmc_step(kmc_ctx* c, uint32_t nsteps, void* stream)
{
    if (!c) return KMC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (nsteps == 0) return KMC_OK;
    const bool graph = c->cfg.use_graph && !c->cfg.profile;
    if (graph && !c->exec) {
        if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess)
            return KMC_EDEVICE;
        hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t le = launch_step(c->plan, c->cap_stream, nullptr);
            e = hipStreamEndCapture(c->cap_stream, &c->graph);
            if (e == hipSuccess && le != hipSuccess) e = le;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&c->exec, c->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            // drop a partial capture so the next call captures afresh
            if (c->graph) (void)hipGraphDestroy(c->graph);
            c->graph = nullptr;
            c->exec = nullptr;
            return KMC_EDEVICE;
        }
    }
    for (uint32_t k = 0; k < nsteps; ++k) {
        hipError_t e;
        if (graph) {
            e = hipGraphLaunch(c->exec, s);
        } else if (c->cfg.profile) {
            std::vector<hipEvent_t> set;
            set.reserve(KMC_PHASE_COUNT + 2);
            while (set.size() < (size_t)KMC_PHASE_COUNT + 2) {
                hipEvent_t ev = nullptr;
                if (!c->ev_free.empty()) { ev = c->ev_free.back(); c->ev_free.pop_back(); }
                else if (hipEventCreate(&ev) != hipSuccess) {
                    // keep the events taken so far for later calls
                    c->ev_free.insert(c->ev_free.end(), set.begin(), set.end());
                    return KMC_EDEVICE;
                }
                set.push_back(ev);
            }
            e = launch_step(c->plan, s, set.data());
            c->ev_pending.push_back(std::move(set));
        } else {
            e = launch_step(c->plan, s, nullptr);
        }
        if (e != hipSuccess) return KMC_EDEVICE;
    }
    c->stepped = true;
    return KMC_OK;
}

int kmc_read_partners(kmc_ctx* c, int32_t* d_partner_by_id, void* stream)
{
    if (!c || (!d_partner_by_id && c->plan.N > 0)) return KMC_EINVAL;
    if (!c->stepped) return KMC_ESTATE;
    return dev_err(launch_read_partners(c->plan, d_partner_by_id, (hipStream_t)stream));
}

int kmc_read_state(kmc_ctx* c, double* d_state_by_id, void* stream)
{
    if (!c || (!d_state_by_id && c->plan.N > 0)) return KMC_EINVAL;
    return dev_err(launch_read_state(c->plan, d_state_by_id, (hipStream_t)stream));
}

int kmc_read_history(kmc_ctx* c, uint64_t* h_npairs, uint64_t* h_digest, uint32_t capacity,
                     uint32_t* count, void* stream)
{
    if (!c || !count || (capacity > 0 && (!h_npairs || !h_digest))) return KMC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const Plan& p = c->plan;
    Ctl ctl;
    std::vector<unsigned long long> np(p.H), dg(p.H);
    hipError_t e = hipMemcpyAsync(&ctl, p.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(np.data(), p.hist_np, np.size() * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dg.data(), p.hist_dig, dg.size() * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return KMC_EDEVICE;
    uint64_t avail = ctl.steps_done < p.H ? ctl.steps_done : p.H;
    if (avail > capacity) avail = capacity;
    for (uint64_t k = 0; k < avail; ++k) {
        const uint64_t step = ctl.steps_done - avail + k;
        h_npairs[k] = np[step % p.H];
        h_digest[k] = dg[step % p.H];
    }
    *count = (uint32_t)avail;
    return KMC_OK;
}

int kmc_count_pair_tests(kmc_ctx* c, uint64_t* h_pair_tests, void* stream)
{
    if (!c || !h_pair_tests) return KMC_EINVAL;
    if (!c->stepped) return KMC_ESTATE;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* d = &c->plan.ctl->scratch;
    unsigned long long h = 0;
    hipError_t e = hipMemsetAsync(d, 0, sizeof(h), s);
    if (e == hipSuccess) e = launch_count_tests(c->plan, d, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return KMC_EDEVICE;
    *h_pair_tests = h;
    return KMC_OK;
}

int kmc_read_time(kmc_ctx* c, double* h_dt, double* h_time, uint32_t capacity, void* stream)
{
    if (!c) return KMC_EINVAL;
    const uint32_t nb = c->plan.nboxes;
    if ((h_dt || h_time) && capacity < nb) return KMC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    std::vector<BoxDev> bd(nb);
    hipError_t e = hipMemcpyAsync(bd.data(), c->plan.boxes, sizeof(BoxDev) * nb, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return KMC_EDEVICE;
    for (uint32_t b = 0; b < nb; ++b) {
        if (h_dt) h_dt[b] = bd[b].dt;
        if (h_time) h_time[b] = bd[b].time;
    }
    return KMC_OK;
}

int kmc_get_stats(kmc_ctx* c, kmc_stats* out, void* stream)
{
    if (!c || !out) return KMC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    Ctl ctl;
    hipError_t e = hipMemcpyAsync(&ctl, c->plan.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return KMC_EDEVICE;
    fold_events(c);
    std::memset(out, 0, sizeof(*out));
    out->steps = ctl.steps_done;
    out->n_total = c->plan.N;
    out->cells_total = c->plan.C;
    out->rechecks = ctl.rechecks_total;
    out->fallbacks = ctl.fallbacks_total;
    out->candidates = ctl.candidates_total;
    out->absorbed = ctl.absorbed_total;
    for (int k = 0; k < 8; ++k) out->ms[k] = c->ms[k];
    out->search_kernel_ms = c->search_kernel_ms;
    out->timed_steps = c->timed_steps;
    return KMC_OK;
}

int kmc_box_with_kappa(const kmc_box* box, double kappa, kmc_box* out)
{
    if (!box || !out || !std::isfinite(kappa) || !(kappa >= 1.0)) return KMC_EINVAL;
    if (check_box(*box) != KMC_OK) return KMC_EINVAL;
    kmc_box b = *box;
    const double D = std::sqrt(box->D2);
    for (int k = 0; k < 3; ++k) {
        const double L = box->hi[k] - box->lo[k];
        double m = std::floor(L / (kappa * D));
        if (m < 1.0) m = 1.0;
        if (m > 2147483647.0) return KMC_EOVERFLOW;
        if (box->bc[k] == KMC_BC_PERIODIC && m < 3.0) return KMC_EINVAL;
        b.ncell[k] = (int32_t)m;
        b.inv_h[k] = m / L;
    }
    if (check_box(b) != KMC_OK) return KMC_EINVAL;
    *out = b;
    return KMC_OK;
}

int kmc_autotune(const kmc_box* boxes, uint32_t nboxes, const kmc_config* cfg, const double* d_state,
                 void* d_workspace, size_t workspace_bytes, uint32_t flags, uint32_t steps, void* stream,
                 kmc_box* out_boxes, kmc_config* out_cfg, kmc_tuning* out)
{
    if (!out_boxes || !out_cfg || !out || !d_workspace) return KMC_EINVAL;
    Totals t;
    int rc = validate(boxes, nboxes, cfg, t);
    if (rc != KMC_OK) return rc;
    if (t.N > 0 && !d_state) return KMC_EINVAL;
    if (flags == 0) flags = KMC_TUNE_LAUNCH;
    if (flags & ~(uint32_t)(KMC_TUNE_LAUNCH | KMC_TUNE_CELLS | KMC_TUNE_PRECISION | KMC_TUNE_ADAPT))
        return KMC_EINVAL;
    if ((flags & KMC_TUNE_ADAPT) && cfg->adapt_levels == 0) return KMC_EINVAL;
    if (steps == 0) steps = 3;
    if (steps > 1000) return KMC_EINVAL;

    std::vector<double> kappas{0.0};
    if (flags & KMC_TUNE_CELLS) kappas = {1.0, 1.25, 1.5, 2.0};
    std::vector<int32_t> precs{cfg->precision};
    if (flags & KMC_TUNE_PRECISION) precs = {KMC_FP64, KMC_FP32_SCREEN};
    std::vector<uint32_t> thresholds{cfg->adapt_threshold};
    if (flags & KMC_TUNE_ADAPT) thresholds = {4u, 8u, 16u, 32u};
    const bool launch = (flags & KMC_TUNE_LAUNCH) != 0;
    std::memset(out, 0, sizeof(*out));
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return KMC_EDEVICE;
    }
    std::vector<kmc_box> bx(boxes, boxes + nboxes), best_boxes;
    kmc_config best_cfg{};
    double best_ms = INFINITY;
    int status = KMC_OK;
    uint32_t k = 0;
    // time one candidate (NaN when it cannot run: grid or workspace); returns
    // its ms per step
    auto trial = [&](const kmc_config& c, double kappa, bool grid_ok) -> double {
        if (k >= KMC_TUNE_MAX || status != KMC_OK) return NAN;
        out->search_mode[k] = c.search_mode;
        out->block_size[k] = c.block_size;
        out->kappa[k] = kappa;
        out->precision[k] = c.precision;
        out->tile[k] = c.tile;
        out->adapt_threshold[k] = c.adapt_levels > 0 ? c.adapt_threshold : 0u;
        out->ms_per_step[k] = NAN;
        size_t need = 0;
        kmc_ctx* ctx = nullptr;
        double r = NAN;
        if (grid_ok && kmc_workspace_bytes(bx.data(), nboxes, &c, &need) == KMC_OK && need <= workspace_bytes &&
            kmc_init(bx.data(), nboxes, &c, d_state, d_workspace, workspace_bytes, stream, &ctx) == KMC_OK) {
            float ms = 0.f;
            hipError_t e = kmc_step(ctx, 1, stream) == KMC_OK ? hipEventRecord(e0, s) : hipErrorUnknown;
            if (e == hipSuccess) e = kmc_step(ctx, steps, stream) == KMC_OK ? hipEventRecord(e1, s) : hipErrorUnknown;
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            kmc_destroy(ctx);
            if (e != hipSuccess) {
                status = KMC_EDEVICE;
            } else {
                r = (double)ms / steps;
                out->ms_per_step[k] = r;
                if (r < best_ms) {
                    best_ms = r;
                    out->best = k;
                    best_boxes = bx;
                    best_cfg = c;
                }
            }
        }
        ++k;
        return r;
    };
    for (double kappa : kappas) {
        bool ok = true;
        for (uint32_t b = 0; b < nboxes && ok; ++b)
            ok = kappa == 0.0 ? (bx[b] = boxes[b], true) : kmc_box_with_kappa(&boxes[b], kappa, &bx[b]) == KMC_OK;
        for (uint32_t thr : thresholds) {
            kmc_config base = *cfg;
            base.use_graph = 0;
            base.profile = 0;
            base.adapt_threshold = thr;
            if (launch) {
                base.block_size = 256;
                base.tile = 0;
            }
            // stage 1: precision x search organisation (adaptive bins take the
            // full search only)
            kmc_config cur = base;
            double cur_ms = INFINITY;
            std::vector<int32_t> modes{cfg->search_mode};
            if (launch && cfg->adapt_levels == 0) modes = {KMC_SEARCH_HALF, KMC_SEARCH_FULL};
            else if (launch) modes = {KMC_SEARCH_FULL};
            for (int32_t pr : precs)
                for (int32_t mode : modes) {
                    kmc_config c = base;
                    c.precision = pr;
                    c.search_mode = mode;
                    const double r = trial(c, kappa, ok);
                    if (r < cur_ms) { cur_ms = r; cur = c; }
                }
            if (launch && std::isfinite(cur_ms)) {
                // stage 2: the other tile shapes; stage 3: the other block sizes
                const kmc_config t0 = cur;
                for (int32_t tile : {1, 2}) {
                    kmc_config c = t0;
                    c.tile = tile;
                    const double r = trial(c, kappa, ok);
                    if (r < cur_ms) { cur_ms = r; cur = c; }
                }
                const kmc_config b0 = cur;
                for (int32_t blk : {128, 512}) {
                    kmc_config c = b0;
                    c.block_size = blk;
                    const double r = trial(c, kappa, ok);
                    if (r < cur_ms) { cur_ms = r; cur = c; }
                }
            }
            if (status != KMC_OK) break;
        }
        if (status != KMC_OK) break;
    }
    out->ntried = k;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status != KMC_OK) return status;
    if (best_boxes.empty()) return KMC_ENOMEM;
    std::copy(best_boxes.begin(), best_boxes.end(), out_boxes);
    *out_cfg = *cfg;
    out_cfg->search_mode = best_cfg.search_mode;
    out_cfg->block_size = best_cfg.block_size;
    out_cfg->tile = best_cfg.tile;
    out_cfg->precision = best_cfg.precision;
    out_cfg->adapt_threshold = best_cfg.adapt_threshold;
    return KMC_OK;
}

void kmc_destroy(kmc_ctx* c)
{
    if (!c) return;
    if (c->exec) (void)hipGraphExecDestroy(c->exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (auto& set : c->ev_pending)
        for (auto e : set) (void)hipEventDestroy(e);
    for (auto e : c->ev_free) (void)hipEventDestroy(e);
    delete c;
}

}  // extern "C"
