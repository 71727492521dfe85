"""ctypes wrapper of the CPU oracle (oracle/liborc.so).

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the
benchmark's CPU-baseline leg.  The product (paper_1310_3437_amd) never
imports this module.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

from . import build as _build

_LIB = None


class OrcBox(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("sphere", C.c_int32),
        ("periodic", C.c_int32 * 3),
        ("ncell", C.c_int32 * 3),
        ("kinematics", C.c_int32),
        ("dims", C.c_int32),
        ("absorb", C.c_int32 * 3),
        ("lo", C.c_double * 3),
        ("hi", C.c_double * 3),
        ("inv_h", C.c_double * 3),
        ("R", C.c_double),
        ("D2", C.c_double),
        ("dt", C.c_double),
        ("seed", C.c_uint64),
        ("nspecies", C.c_int32),
        ("pad_", C.c_int32),
        ("species", C.POINTER(C.c_uint8)),
        ("radius", C.POINTER(C.c_double)),
        ("mass", C.POINTER(C.c_double)),
        ("adapt_levels", C.c_int32),
        ("adapt_threshold", C.c_int32),
    ]


class OrcPairQ(C.Structure):
    _fields_ = [
        ("r", C.c_double * 3),
        ("g", C.c_double * 3),
        ("b", C.c_double),
        ("g2", C.c_double),
        ("c2", C.c_double),
        ("key", C.c_double),
        ("acc", C.c_int32),
    ]


def lib():
    """Load liborc.so, building it first only if it does not exist."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build(force=True)
        L = C.CDLL(_build.LIB)
        dp = C.POINTER(C.c_double)
        u32p = C.POINTER(C.c_uint32)
        i32p = C.POINTER(C.c_int32)
        u64p = C.POINTER(C.c_uint64)
        bp = C.POINTER(OrcBox)
        L.orc_cell_coords.argtypes = [bp, C.c_double, C.c_double, C.c_double, i32p]
        L.orc_pair.argtypes = [bp, dp, dp, i32p, C.POINTER(OrcPairQ)]
        L.orc_find_partners.argtypes = [bp, dp, u32p, i32p, C.c_int, u64p]
        L.orc_find_partners_bruteforce.argtypes = [bp, dp, u32p, i32p]
        L.orc_philox4x64_10.argtypes = [u64p, u64p, u64p]
        L.orc_philox4x64_10.restype = None
        L.orc_direction.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, dp]
        L.orc_direction.restype = None
        L.orc_direction2.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, dp]
        L.orc_direction2.restype = None
        L.orc_pair_hash.argtypes = [C.c_uint32, C.c_uint32]
        L.orc_pair_hash.restype = C.c_uint64
        L.orc_step.argtypes = [bp, dp, u32p, C.c_uint64, i32p, u64p, u64p, C.c_int, u64p]
        L.orc_step_ex.argtypes = [bp, dp, u32p, C.POINTER(C.c_uint8), C.c_uint64, i32p, u64p, u64p, C.c_int,
                                  u64p]
        L.orc_adaptive_dt_ex.argtypes = [bp, dp, C.POINTER(C.c_uint8), C.c_double, dp]
        L.orc_count_accepted.argtypes = [bp, dp, u32p, C.c_int, u64p, u64p]
        L.orc_adaptive_dt.argtypes = [bp, dp, C.c_double, dp]
        L.orc_step_sampled.argtypes = [bp, dp, u32p, C.c_uint64, C.POINTER(C.c_int64), C.c_int64, i32p,
                                       dp, C.c_int]
        L.orc_max_threads.argtypes = []
        for f in ("orc_cell_coords", "orc_pair", "orc_find_partners", "orc_find_partners_bruteforce",
                  "orc_step", "orc_step_ex", "orc_count_accepted", "orc_step_sampled", "orc_adaptive_dt",
                  "orc_adaptive_dt_ex",
                  "orc_max_threads"):
            getattr(L, f).restype = C.c_int
        _LIB = L
    return _LIB


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def make_box(box, seed=1, kinematics=0, dims=3, kinds=None, adapt=(0, 0)):
    """OrcBox from a paper_1310_3437_amd.inputs.Box (or any object with the
    same attributes).  kinds = (species, radius, mass): per-particle kind
    (uint8, the box's particles) and per-kind effective radius and mass, or
    None for one kind of particle.  adapt = (levels, threshold) of the
    density-adaptive bins ((0, 0): the uniform grid)."""
    ob = OrcBox()
    ob.adapt_levels = int(adapt[0])
    ob.adapt_threshold = int(adapt[1])
    if kinds is not None:
        sp, rad, mass = kinds
        sp = np.ascontiguousarray(sp, dtype=np.uint8)
        rad = np.ascontiguousarray(rad, dtype=np.float64)
        mass = np.ascontiguousarray(mass, dtype=np.float64)
        ob.nspecies = int(rad.shape[0])
        ob.species = _ptr(sp, C.c_uint8)
        ob.radius = _ptr(rad, C.c_double)
        ob.mass = _ptr(mass, C.c_double)
        ob._keep = (sp, rad, mass)   # the arrays live as long as the structure
    ob.n = int(box.n)
    ob.sphere = 1 if box.sphere else 0
    for k in range(3):
        ob.periodic[k] = 1 if box.periodic[k] else 0
        ob.absorb[k] = 1 if getattr(box, "absorb", (False,) * 3)[k] else 0
        ob.ncell[k] = int(box.ncell[k])
        ob.lo[k] = float(box.lo[k])
        ob.hi[k] = float(box.hi[k])
        ob.inv_h[k] = float(box.inv_h[k])
    ob.kinematics = int(kinematics)
    ob.dims = int(dims)
    ob.R = float(box.R)
    ob.D2 = float(box.D2)
    ob.dt = float(box.dt)
    ob.seed = int(seed) & ((1 << 64) - 1)
    return ob


def _soa(state):
    s = np.ascontiguousarray(state, dtype=np.float64)
    assert s.ndim == 2 and s.shape[0] == 6
    return s


def cell_coords(box, x, y, z):
    c = (C.c_int32 * 3)()
    ob = make_box(box)
    rc = lib().orc_cell_coords(C.byref(ob), float(x), float(y), float(z), c)
    assert rc == 0
    return tuple(c)


def pair(box, pi, pj, wrap=(0, 0, 0)):
    """Pair quantities (dict) of searcher state pi[6] and candidate pj[6]."""
    ob = make_box(box)
    a = np.ascontiguousarray(pi, dtype=np.float64)
    b = np.ascontiguousarray(pj, dtype=np.float64)
    w = np.ascontiguousarray(wrap, dtype=np.int32)
    q = OrcPairQ()
    rc = lib().orc_pair(C.byref(ob), _ptr(a, C.c_double), _ptr(b, C.c_double), _ptr(w, C.c_int32), C.byref(q))
    assert rc == 0
    return dict(r=tuple(q.r), g=tuple(q.g), b=q.b, g2=q.g2, c2=q.c2, key=q.key, acc=bool(q.acc))


def find_partners(box, state, ids=None, nthreads=0, brute=False, kinds=None, adapt=(0, 0)):
    """Partner array (indices into the box's particles, -1 for none)."""
    s = _soa(state)
    n = s.shape[1]
    ids = np.arange(n, dtype=np.uint32) if ids is None else np.ascontiguousarray(ids, dtype=np.uint32)
    out = np.empty(n, dtype=np.int32)
    ob = make_box(box, kinds=kinds, adapt=adapt)
    ob.n = n
    if brute:
        rc = lib().orc_find_partners_bruteforce(C.byref(ob), _ptr(s, C.c_double), _ptr(ids, C.c_uint32),
                                                _ptr(out, C.c_int32))
        tests = None
    else:
        t = C.c_uint64(0)
        rc = lib().orc_find_partners(C.byref(ob), _ptr(s, C.c_double), _ptr(ids, C.c_uint32),
                                     _ptr(out, C.c_int32), int(nthreads), C.byref(t))
        tests = int(t.value)
    if rc != 0:
        raise ValueError(f"orc_find_partners failed ({rc})")
    return out, tests


def count_accepted(box, state, ids=None, nthreads=0, kinds=None):
    """Acceptable ordered pairs (and pair tests) of the cell-list search."""
    s = _soa(state)
    n = s.shape[1]
    ids = np.arange(n, dtype=np.uint32) if ids is None else np.ascontiguousarray(ids, dtype=np.uint32)
    ob = make_box(box, kinds=kinds)
    ob.n = n
    acc = C.c_uint64(0)
    tests = C.c_uint64(0)
    rc = lib().orc_count_accepted(C.byref(ob), _ptr(s, C.c_double), _ptr(ids, C.c_uint32), int(nthreads),
                                  C.byref(acc), C.byref(tests))
    if rc != 0:
        raise ValueError(f"orc_count_accepted failed ({rc})")
    return int(acc.value), int(tests.value)


def philox(ctr, key):
    c = np.ascontiguousarray(np.array(ctr, dtype=np.uint64))
    k = np.ascontiguousarray(np.array(key, dtype=np.uint64))
    o = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_ptr(c, C.c_uint64), _ptr(k, C.c_uint64), _ptr(o, C.c_uint64))
    return [int(x) for x in o]


def direction(seed, step, a, dims=3):
    o = np.zeros(3, dtype=np.float64)
    f = lib().orc_direction2 if dims == 2 else lib().orc_direction
    f(int(seed), int(step), int(a), _ptr(o, C.c_double))
    return o


def pair_hash(a, b):
    return int(lib().orc_pair_hash(int(a), int(b)))


def adaptive_dt(box, state, factor=1.0, gone=None):
    """The adaptive time step of one box for the given state (particles with
    gone[i] != 0 excluded)."""
    s = _soa(state)
    ob = make_box(box)
    ob.n = s.shape[1]
    out = C.c_double(0.0)
    g = None if gone is None else _ptr(np.ascontiguousarray(gone, dtype=np.uint8), C.c_uint8)
    rc = lib().orc_adaptive_dt_ex(C.byref(ob), _ptr(s, C.c_double), g, float(factor), C.byref(out))
    if rc != 0:
        raise ValueError(f"orc_adaptive_dt failed ({rc})")
    return float(out.value)


def step_sampled(box, state, ids, step, sel, seed=1, kinematics=0, nthreads=0, dims=3, kinds=None, adapt=(0, 0)):
    """The oracle step of one box evaluated at the particles `sel` only
    (indices into the box); `state` is not modified.  Returns (partner
    indices of the selected particles, their (6, len(sel)) post-step state)."""
    s = _soa(state)
    n = s.shape[1]
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    ob = make_box(box, seed=seed, kinematics=kinematics, dims=dims, kinds=kinds, adapt=adapt)
    ob.n = n
    partner = np.empty(len(sel), dtype=np.int32)
    out = np.empty((len(sel), 6), dtype=np.float64)
    rc = lib().orc_step_sampled(C.byref(ob), _ptr(s, C.c_double), _ptr(ids, C.c_uint32), int(step),
                                _ptr(sel, C.c_int64), len(sel), _ptr(partner, C.c_int32),
                                _ptr(out, C.c_double), int(nthreads))
    if rc != 0:
        raise ValueError(f"orc_step_sampled failed ({rc})")
    return partner, out.T.copy()


def step_box(box, state, ids, step, seed=1, kinematics=0, nthreads=0, dims=3, gone=None, kinds=None, adapt=(0, 0)):
    """One oracle step of one box, in place on `state` ((6, n) float64,
    C-contiguous) and on `gone` (uint8 per particle, 1 = absorbed; required
    with absorbing faces).  kinds as in make_box.  Returns (partner indices,
    npairs, digest, pair_tests)."""
    assert state.dtype == np.float64 and state.flags.c_contiguous and state.shape[0] == 6
    n = state.shape[1]
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    ob = make_box(box, seed=seed, kinematics=kinematics, dims=dims, kinds=kinds, adapt=adapt)
    ob.n = n
    partner = np.empty(n, dtype=np.int32)
    npairs = C.c_uint64(0)
    dig = C.c_uint64(0)
    tests = C.c_uint64(0)
    if gone is not None:
        assert gone.dtype == np.uint8 and gone.flags.c_contiguous and gone.shape == (n,)
    rc = lib().orc_step_ex(C.byref(ob), _ptr(state, C.c_double), _ptr(ids, C.c_uint32),
                           None if gone is None else _ptr(gone, C.c_uint8), int(step),
                           _ptr(partner, C.c_int32), C.byref(npairs), C.byref(dig), int(nthreads),
                           C.byref(tests))
    if rc != 0:
        raise ValueError(f"orc_step failed ({rc})")
    return partner, int(npairs.value), int(dig.value), int(tests.value)


class Run:
    """Oracle state of a whole workload (all boxes), advanced step by step.

    Particle ids are the global indices of the initial state (box b's
    particles are ids offsets[b] .. offsets[b+1]-1), as in the GPU library.
    """

    def __init__(self, workload, step0=0, nthreads=0):
        self.w = workload
        self.off = workload.offsets
        self.state = [np.array(workload.state[:, self.off[b]:self.off[b + 1]], dtype=np.float64, order="C")
                      for b in range(len(workload.boxes))]
        self.ids = [np.arange(self.off[b], self.off[b + 1], dtype=np.uint32)
                    for b in range(len(workload.boxes))]
        self.step_index = int(step0)
        self.nthreads = nthreads
        self.partner_by_id = None
        self.pair_tests = 0
        self.gone = [np.zeros(self.off[b + 1] - self.off[b], dtype=np.uint8) for b in range(len(workload.boxes))]
        self.time = [0.0] * len(workload.boxes)
        self.dt_last = [float(b.dt) for b in workload.boxes]

    def step(self):
        """Advance every box by one step; returns (npairs, digest) summed
        over boxes (digest mod 2^64)."""
        tot_pairs, tot_dig, tests = 0, 0, 0
        pb = np.full(self.off[-1], -1, dtype=np.int64)
        for b, box in enumerate(self.w.boxes):
            if getattr(self.w, "dt_rule", 0) == 1:
                box = dataclasses.replace(box, dt=adaptive_dt(box, self.state[b], self.w.dt_factor, self.gone[b]))
            self.dt_last[b] = float(box.dt)
            self.time[b] += float(box.dt)
            p, npairs, dig, t = step_box(box, self.state[b], self.ids[b], self.step_index,
                                         seed=self.w.seed, kinematics=self.w.kinematics,
                                         dims=getattr(self.w, "dims", 3), gone=self.gone[b],
                                         nthreads=self.nthreads, kinds=self.kinds(b),
                                         adapt=(getattr(self.w, "adapt_levels", 0),
                                                getattr(self.w, "adapt_threshold", 0)))
            ids = self.ids[b]
            has = p >= 0
            pb[ids[has]] = ids[p[has]]
            tot_pairs += npairs
            tot_dig = (tot_dig + dig) & ((1 << 64) - 1)
            tests += t
        self.partner_by_id = pb
        self.pair_tests = tests
        self.step_index += 1
        return tot_pairs, tot_dig

    def kinds(self, b):
        """(species, radius, mass) of box b's particles, or None for one kind."""
        sp = getattr(self.w, "species", None)
        if sp is None:
            return None
        return sp[self.off[b]:self.off[b + 1]], self.w.radius, self.w.mass

    def absorbed(self):
        """Particles absorbed so far (all boxes)."""
        return int(sum(int(g.sum()) for g in self.gone))

    def full_state(self):
        """(6, N) state in id order."""
        return np.concatenate(self.state, axis=1)
