"""Thin Python binding of libkmc.so (the C ABI in include/kmc.h).

Argument marshalling only: every step of the collision step runs in the HIP
kernels of libkmc.so.  PyTorch supplies device memory (state, workspace,
outputs) and the current HIP stream.  If the library has not been built the
binding raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkmc.so")

KMC_OK, KMC_EINVAL, KMC_ENOMEM, KMC_EDEVICE, KMC_EOVERFLOW, KMC_ESTATE = 0, -1, -2, -3, -4, -5
KMC_FP64, KMC_FP32_SCREEN = 0, 1
KMC_GEOM_BOX, KMC_GEOM_SPHERE = 0, 1
KMC_BC_REFLECT, KMC_BC_PERIODIC, KMC_BC_ABSORB = 0, 1, 2
KMC_KIN_AT_TSTAR, KMC_KIN_VEL_ONLY = 0, 1
KMC_DT_FIXED, KMC_DT_ADAPTIVE = 0, 1
KMC_SEARCH_HALF, KMC_SEARCH_FULL = 0, 1
PHASES = ("bin", "scan", "scatter", "search", "finish", "recheck", "resolve")

_lib = None


class KmcBox(C.Structure):
    _fields_ = [
        ("n", C.c_uint32),
        ("geometry", C.c_int32),
        ("bc", C.c_int32 * 3),
        ("ncell", C.c_int32 * 3),
        ("lo", C.c_double * 3),
        ("hi", C.c_double * 3),
        ("inv_h", C.c_double * 3),
        ("sphere_r", C.c_double),
        ("D2", C.c_double),
        ("dt", C.c_double),
    ]


KMC_MAX_SPECIES = 8


class KmcSpecies(C.Structure):
    _fields_ = [
        ("count", C.c_uint32),
        ("reserved", C.c_uint32),
        ("radius", C.c_double * KMC_MAX_SPECIES),
        ("mass", C.c_double * KMC_MAX_SPECIES),
        ("d_kind", C.c_void_p),
    ]


class KmcConfig(C.Structure):
    _fields_ = [
        ("seed", C.c_uint64),
        ("step0", C.c_uint64),
        ("precision", C.c_int32),
        ("kinematics", C.c_int32),
        ("history", C.c_uint32),
        ("recheck_capacity", C.c_uint32),
        ("use_graph", C.c_int32),
        ("block_size", C.c_int32),
        ("profile", C.c_int32),
        ("dt_rule", C.c_int32),
        ("search_mode", C.c_int32),
        ("dims", C.c_int32),
        ("tile", C.c_int32),
        ("reserved", C.c_int32),
        ("guard_scale", C.c_double),
        ("dt_factor", C.c_double),
        ("species", C.POINTER(KmcSpecies)),
        ("adapt_levels", C.c_int32),
        ("adapt_threshold", C.c_uint32),
    ]


class KmcStats(C.Structure):
    _fields_ = [
        ("steps", C.c_uint64),
        ("n_total", C.c_uint64),
        ("cells_total", C.c_uint64),
        ("rechecks", C.c_uint64),
        ("fallbacks", C.c_uint64),
        ("ms", C.c_double * 8),
        ("timed_steps", C.c_uint64),
        ("search_kernel_ms", C.c_double),
        ("candidates", C.c_uint64),
        ("absorbed", C.c_uint64),
    ]


EXPORTS = ("kmc_workspace_bytes", "kmc_init", "kmc_step", "kmc_read_partners", "kmc_read_state",
           "kmc_read_history", "kmc_read_time", "kmc_count_pair_tests", "kmc_get_stats", "kmc_destroy",
           "kmc_strerror", "kmc_abi_version", "kmc_autotune", "kmc_box_with_kappa", "kmc_init_scratch")

KMC_SCRATCH_BYTES = 64 << 20


KMC_TUNE_LAUNCH, KMC_TUNE_CELLS, KMC_TUNE_PRECISION, KMC_TUNE_ADAPT = 1, 2, 4, 8
KMC_TUNE_MAX = 64
# the layout of the structures below; the library reports its own
KMC_ABI_VERSION = 5


class KmcTuning(C.Structure):
    _fields_ = [
        ("ntried", C.c_uint32),
        ("best", C.c_uint32),
        ("ms_per_step", C.c_double * KMC_TUNE_MAX),
        ("search_mode", C.c_int32 * KMC_TUNE_MAX),
        ("block_size", C.c_int32 * KMC_TUNE_MAX),
        ("kappa", C.c_double * KMC_TUNE_MAX),
        ("precision", C.c_int32 * KMC_TUNE_MAX),
        ("tile", C.c_int32 * KMC_TUNE_MAX),
        ("adapt_threshold", C.c_uint32 * KMC_TUNE_MAX),
    ]


class KmcError(RuntimeError):
    pass


def load(path=LIB_PATH):
    """Load libkmc.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise KmcError(f"{path} is missing: build it with __graft_entry__.build() "
                       "(there is no CPU fallback)")
    # torch first: it ships its own HIP runtime, which the library then binds
    # to (same soname).  Loaded the other way round the process would hold two
    # runtimes, and torch's device pointers would be invalid in the library's.
    import torch  # noqa: F401
    L = C.CDLL(path)
    vp, sz = C.c_void_p, C.c_size_t
    bp, cp = C.POINTER(KmcBox), C.POINTER(KmcConfig)
    L.kmc_workspace_bytes.argtypes = [bp, C.c_uint32, cp, C.POINTER(sz)]
    L.kmc_init.argtypes = [bp, C.c_uint32, cp, vp, vp, sz, vp, C.POINTER(vp)]
    L.kmc_init_scratch.argtypes = [bp, C.c_uint32, cp, vp, vp, C.POINTER(vp)]
    L.kmc_step.argtypes = [vp, C.c_uint32, vp]
    L.kmc_read_partners.argtypes = [vp, vp, vp]
    L.kmc_read_state.argtypes = [vp, vp, vp]
    L.kmc_read_history.argtypes = [vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.c_uint32,
                                   C.POINTER(C.c_uint32), vp]
    L.kmc_read_time.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_uint32, vp]
    L.kmc_count_pair_tests.argtypes = [vp, C.POINTER(C.c_uint64), vp]
    L.kmc_get_stats.argtypes = [vp, C.POINTER(KmcStats), vp]
    L.kmc_autotune.argtypes = [bp, C.c_uint32, cp, vp, vp, sz, C.c_uint32, C.c_uint32, vp, bp, cp,
                               C.POINTER(KmcTuning)]
    L.kmc_box_with_kappa.argtypes = [bp, C.c_double, bp]
    L.kmc_destroy.argtypes = [vp]
    L.kmc_destroy.restype = None
    L.kmc_strerror.argtypes = [C.c_int]
    L.kmc_strerror.restype = C.c_char_p
    L.kmc_abi_version.argtypes = []
    for f in ("kmc_workspace_bytes", "kmc_init", "kmc_step", "kmc_read_partners", "kmc_read_state",
              "kmc_read_history", "kmc_read_time", "kmc_count_pair_tests", "kmc_get_stats", "kmc_abi_version",
              "kmc_autotune", "kmc_box_with_kappa", "kmc_init_scratch"):
        getattr(L, f).restype = C.c_int
    if L.kmc_abi_version() != KMC_ABI_VERSION:
        raise KmcError(f"{path}: ABI version {L.kmc_abi_version()}, this binding expects {KMC_ABI_VERSION} "
                       "(rebuild the library)")
    _lib = L
    return L


def _check(rc, what):
    if rc != KMC_OK:
        msg = load().kmc_strerror(rc).decode()
        raise KmcError(f"{what} failed: {msg} ({rc})")


def make_boxes(boxes):
    """ctypes array of kmc_box from objects with the attributes of
    paper_1310_3437_amd.inputs.Box."""
    arr = (KmcBox * len(boxes))()
    for k, b in enumerate(boxes):
        kb = arr[k]
        kb.n = int(b.n)
        kb.geometry = KMC_GEOM_SPHERE if b.sphere else KMC_GEOM_BOX
        inv_h = b.inv_h
        for a in range(3):
            absorb = getattr(b, "absorb", (False, False, False))[a]
            kb.bc[a] = KMC_BC_ABSORB if absorb else (KMC_BC_PERIODIC if b.periodic[a] else KMC_BC_REFLECT)
            kb.ncell[a] = int(b.ncell[a])
            kb.lo[a] = float(b.lo[a])
            kb.hi[a] = float(b.hi[a])
            kb.inv_h[a] = float(inv_h[a])
        kb.sphere_r = float(b.R)
        kb.D2 = float(b.D2)
        kb.dt = float(b.dt)
    return arr


def make_species(radius, mass, d_kind_ptr=0):
    """kmc_species for kinds with the given effective radii and masses; the
    per-particle kinds live at device address d_kind_ptr (uint8, id order)."""
    sp = KmcSpecies()
    if not 1 <= len(radius) <= KMC_MAX_SPECIES or len(mass) != len(radius):
        raise ValueError("1..8 kinds, one radius and one mass each")
    sp.count = len(radius)
    for k in range(len(radius)):
        sp.radius[k] = float(radius[k])
        sp.mass[k] = float(mass[k])
    sp.d_kind = int(d_kind_ptr)
    return sp


def make_config(seed=1, step0=0, precision=KMC_FP64, kinematics=KMC_KIN_AT_TSTAR, history=0,
                recheck_capacity=0, use_graph=False, block_size=0, profile=False, guard_scale=0.0,
                dt_rule=KMC_DT_FIXED, dt_factor=0.0, search_mode=KMC_SEARCH_HALF, dims=3, species=None, tile=0,
                adapt_levels=0, adapt_threshold=0):
    """kmc_config from keyword arguments; species: a KmcSpecies (kept alive
    with the returned structure) or None for one kind of particle."""
    c = KmcConfig()
    if species is not None:
        c.species = C.pointer(species)
        c._species = species
    c.seed = int(seed) & ((1 << 64) - 1)
    c.step0 = int(step0)
    c.precision = int(precision)
    c.kinematics = int(kinematics)
    c.history = int(history)
    c.recheck_capacity = int(recheck_capacity)
    c.use_graph = 1 if use_graph else 0
    c.block_size = int(block_size)
    c.profile = 1 if profile else 0
    c.guard_scale = float(guard_scale)
    c.dt_rule = int(dt_rule)
    c.dt_factor = float(dt_factor)
    c.search_mode = int(search_mode)
    c.dims = int(dims)
    c.tile = int(tile)
    c.adapt_levels = int(adapt_levels)
    c.adapt_threshold = int(adapt_threshold)
    return c


def _box_from_kmc(kb, like):
    """inputs.Box-like copy of `like` with the grid of the kmc_box kb."""
    import dataclasses
    return dataclasses.replace(like, ncell=tuple(int(kb.ncell[k]) for k in range(3)))


def box_with_kappa(box, kappa):
    """The box with the cell grid floor(L / (kappa D)) of KMC_TUNE_CELLS."""
    src = make_boxes([box])
    out = KmcBox()
    _check(load().kmc_box_with_kappa(src, float(kappa), C.byref(out)), "kmc_box_with_kappa")
    nb = _box_from_kmc(out, box)
    if tuple(nb.inv_h) != tuple(out.inv_h):
        raise KmcError("inv_h of the tuned grid differs from ncell / (hi - lo)")
    return nb


def _tune_key(boxes, device_name, flags, steps, config, kinds=None):
    import hashlib
    import json
    desc = dict(device=device_name, flags=int(flags), steps=int(steps),
                kinds=None if kinds is None else [list(map(float, kinds[1])), list(map(float, kinds[2]))],
                config={k: config[k] for k in sorted(config) if k not in ("seed", "step0", "history", "profile",
                                                                          "use_graph", "species")},
                boxes=[dict(n=int(b.n), lo=list(map(float, b.lo)), hi=list(map(float, b.hi)),
                            ncell=list(map(int, b.ncell)), periodic=list(map(bool, b.periodic)),
                            absorb=list(map(bool, getattr(b, "absorb", (False,) * 3))),
                            inv_h=[float(x).hex() for x in b.inv_h],
                            sphere=bool(b.sphere), R=float(b.R), D2=float(b.D2), dt=float(b.dt)) for b in boxes])
    return hashlib.sha256(json.dumps(desc, sort_keys=True).encode()).hexdigest()


def autotune(boxes, state, device="cuda", flags=KMC_TUNE_LAUNCH, steps=3, cache=None, kinds=None, **config):
    """Run kmc_autotune on `state`; returns (boxes, config dict, tuning dict).
    The boxes differ from the input only with KMC_TUNE_CELLS.  kinds as for
    Sim (pass them to Sim again with the returned configuration).  With
    `cache` (a JSON file path) a previous choice for the same device, boxes,
    flags, kinds and configuration is reused without timing, so repeated runs
    make the same choice."""
    import json
    import torch
    boxes = list(boxes)
    key = None
    if cache is not None:
        key = _tune_key(boxes, torch.cuda.get_device_name(torch.device(device)), flags, steps, config, kinds)
        if os.path.exists(cache):
            with open(cache) as fh:
                hit = json.load(fh).get(key)
            if hit is not None:
                kappa = hit["kappa"]
                nb = [box_with_kappa(b, kappa) for b in boxes] if kappa > 0 else boxes
                cfg_hit = dict(config, search_mode=hit["search_mode"], block_size=hit["block_size"],
                               tile=hit["tile"], precision=hit["precision"])
                if hit.get("adapt_threshold"):
                    cfg_hit["adapt_threshold"] = hit["adapt_threshold"]
                return nb, cfg_hit, dict(best=hit["best"], tried=hit["tried"], cached=True)
    spc = {}
    if kinds is not None:
        kind_t = torch.as_tensor(np.asarray(kinds[0]), dtype=torch.uint8).to(device).contiguous()
        spc = dict(species=make_species(kinds[1], kinds[2], kind_t.data_ptr()))
    cfg = make_config(**config, **spc)
    arr = make_boxes(boxes)
    st = torch.as_tensor(state, dtype=torch.float64).to(device).contiguous()
    # the largest candidate: the finest grid (kappa = 1), the smallest blocks
    # and, when the precision is tuned, the FP32 screen's extra sorted copy
    probe = [box_with_kappa(b, 1.0) for b in boxes] if flags & KMC_TUNE_CELLS else boxes
    pcfg = dict(config, block_size=64)
    if flags & KMC_TUNE_PRECISION:
        pcfg["precision"] = KMC_FP32_SCREEN
    if flags & KMC_TUNE_ADAPT:
        pcfg["adapt_threshold"] = 4   # the smallest threshold needs the largest leaf tables
    need = workspace_bytes(probe, make_config(**pcfg, **spc))
    ws = torch.empty(need + 256, dtype=torch.uint8, device=device)
    ptr = (ws.data_ptr() + 255) // 256 * 256
    out_b = (KmcBox * len(boxes))()
    out_c = KmcConfig()
    tun = KmcTuning()
    stream = C.c_void_p(torch.cuda.current_stream(torch.device(device)).cuda_stream)
    _check(load().kmc_autotune(arr, len(boxes), C.byref(cfg), C.c_void_p(st.data_ptr()), C.c_void_p(ptr),
                               C.c_size_t(need), int(flags), int(steps), stream, out_b, C.byref(out_c),
                               C.byref(tun)), "kmc_autotune")
    new_boxes = [_box_from_kmc(out_b[k], boxes[k]) for k in range(len(boxes))]
    new_cfg = dict(config, search_mode=int(out_c.search_mode), block_size=int(out_c.block_size),
                   tile=int(out_c.tile), precision=int(out_c.precision))
    if flags & KMC_TUNE_ADAPT:
        new_cfg["adapt_threshold"] = int(out_c.adapt_threshold)
    tried = [dict(ms_per_step=tun.ms_per_step[k], search_mode=tun.search_mode[k], block_size=tun.block_size[k],
                  kappa=tun.kappa[k], precision=tun.precision[k], tile=tun.tile[k],
                  adapt_threshold=int(tun.adapt_threshold[k])) for k in range(tun.ntried)]
    if cache is not None:
        db = {}
        if os.path.exists(cache):
            with open(cache) as fh:
                db = json.load(fh)
        best = tried[int(tun.best)]
        db[key] = dict(search_mode=best["search_mode"], block_size=best["block_size"], kappa=best["kappa"],
                       tile=best["tile"], precision=best["precision"],
                       adapt_threshold=best["adapt_threshold"] if flags & KMC_TUNE_ADAPT else 0,
                       best=int(tun.best), tried=[{k: (None if isinstance(v, float) and v != v else v)
                                                   for k, v in t.items()} for t in tried])
        tmp = cache + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(db, fh, indent=1)
        os.replace(tmp, cache)
    return new_boxes, new_cfg, dict(best=int(tun.best), tried=tried, cached=False)


def workspace_bytes(boxes, config):
    arr = make_boxes(boxes)
    n = C.c_size_t(0)
    _check(load().kmc_workspace_bytes(arr, len(boxes), C.byref(config), C.byref(n)), "kmc_workspace_bytes")
    return int(n.value)


class Sim:
    """A context of libkmc.so over one or more boxes.

    state: (6, N) float64 array (numpy or torch, any device) in the layout of
    kmc_init: x, y, z, vx, vy, vz rows, boxes concatenated in order.
    """

    def __init__(self, boxes, state, device="cuda", kinds=None, scratch=False, **config):
        """kinds: None (one kind of particle) or (kind, radius, mass): the kind
        of each particle (N integers, id order) and each kind's effective
        radius and mass.  scratch: create the context with kmc_init_scratch
        (the library's static per-device workspace, no workspace tensor)."""
        import torch
        self._torch = torch
        L = load()
        self.boxes = list(boxes)
        self.device = torch.device(device)
        if kinds is not None:
            kind, radius, mass = kinds
            kind = np.asarray(kind)
            if kind.shape != (sum(int(b.n) for b in self.boxes),):
                raise ValueError("kinds: one kind per particle")
            if kind.size and (int(kind.min()) < 0 or int(kind.max()) > 255):
                raise ValueError("kinds: values must fit in a byte (the library checks them against the count)")
            self._kind = torch.as_tensor(kind, dtype=torch.uint8).to(self.device).contiguous()
            config = dict(config, species=make_species(radius, mass, self._kind.data_ptr()))
        self.config = make_config(**config)
        self._boxarr = make_boxes(self.boxes)
        st = torch.as_tensor(state, dtype=torch.float64).to(self.device).contiguous()
        if st.ndim != 2 or st.shape[0] != 6 or st.shape[1] != sum(int(b.n) for b in self.boxes):
            raise ValueError("state must be (6, sum of box n) float64")
        self.n = int(st.shape[1])
        ctx = C.c_void_p(0)
        if scratch:
            self.workspace = None
            _check(L.kmc_init_scratch(self._boxarr, len(self.boxes), C.byref(self.config),
                                      C.c_void_p(st.data_ptr()), self._stream(), C.byref(ctx)), "kmc_init_scratch")
        else:
            nbytes = workspace_bytes(self.boxes, self.config)
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            self._ws_ptr = (base + 255) // 256 * 256
            _check(L.kmc_init(self._boxarr, len(self.boxes), C.byref(self.config), C.c_void_p(st.data_ptr()),
                              C.c_void_p(self._ws_ptr), C.c_size_t(nbytes), self._stream(), C.byref(ctx)),
                   "kmc_init")
        self._ctx = ctx
        torch.cuda.current_stream(self.device).synchronize()
        self._kind = None   # read by kmc_init only

    def _stream(self):
        return C.c_void_p(self._torch.cuda.current_stream(self.device).cuda_stream)

    def step(self, n=1):
        _check(load().kmc_step(self._ctx, int(n), self._stream()), "kmc_step")

    def partners(self):
        """Last step's chosen partner id per particle id (int32 device tensor, -1 = none)."""
        out = self._torch.empty(self.n, dtype=self._torch.int32, device=self.device)
        _check(load().kmc_read_partners(self._ctx, C.c_void_p(out.data_ptr()), self._stream()),
               "kmc_read_partners")
        return out

    def state(self):
        """Current state in id order, (6, N) float64 device tensor."""
        out = self._torch.empty((6, self.n), dtype=self._torch.float64, device=self.device)
        _check(load().kmc_read_state(self._ctx, C.c_void_p(out.data_ptr()), self._stream()), "kmc_read_state")
        return out

    def history(self, capacity=None):
        """(npairs, digest) of the most recent steps, oldest first (uint64 numpy arrays)."""
        cap = int(capacity if capacity is not None else (self.config.history or 1024))
        np_ = np.zeros(cap, dtype=np.uint64)
        dg = np.zeros(cap, dtype=np.uint64)
        cnt = C.c_uint32(0)
        _check(load().kmc_read_history(self._ctx, np_.ctypes.data_as(C.POINTER(C.c_uint64)),
                                       dg.ctypes.data_as(C.POINTER(C.c_uint64)), cap, C.byref(cnt),
                                       self._stream()), "kmc_read_history")
        return np_[:cnt.value], dg[:cnt.value]

    def time(self):
        """(dt of the last step, simulated time) per box, float64 numpy arrays."""
        nb = len(self.boxes)
        dt = np.zeros(nb, dtype=np.float64)
        tm = np.zeros(nb, dtype=np.float64)
        _check(load().kmc_read_time(self._ctx, dt.ctypes.data_as(C.POINTER(C.c_double)),
                                    tm.ctypes.data_as(C.POINTER(C.c_double)), nb, self._stream()),
               "kmc_read_time")
        return dt, tm

    def pair_tests(self):
        t = C.c_uint64(0)
        _check(load().kmc_count_pair_tests(self._ctx, C.byref(t), self._stream()), "kmc_count_pair_tests")
        return int(t.value)

    def stats(self):
        s = KmcStats()
        _check(load().kmc_get_stats(self._ctx, C.byref(s), self._stream()), "kmc_get_stats")
        return dict(steps=s.steps, n_total=s.n_total, cells_total=s.cells_total, rechecks=s.rechecks,
                    fallbacks=s.fallbacks, timed_steps=s.timed_steps, search_kernel_ms=s.search_kernel_ms,
                    candidates=s.candidates, absorbed=s.absorbed,
                    ms={PHASES[k]: s.ms[k] for k in range(len(PHASES))})

    def close(self):
        if getattr(self, "_ctx", None):
            load().kmc_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
