"""GPU checks of the FP32 screen on adversarial inputs.

Isolated pairs (and triples) are placed so that the FP64 decision sits within
2^-18 .. 2^-50 relative of an acceptance boundary: the interaction radius
(d_min = D), the end of the step (t* = dt), the start of the step (t* = 0),
and near-equal keys of two candidates.  Variants add a large common velocity
(cancellation in g = v_j - v_i) and coordinates far from the origin.  The
screen must reproduce the FP64 oracle exactly (it drops a pair only when the
FP64 definition certainly rejects it, and every pair it keeps is decided in
FP64); with its error bounds switched off (guard -1) it must not, which shows
the bounds carry the exactness.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1310_3437_amd import inputs as I

pytestmark = pytest.mark.gpu


def adversarial(seed=0, bulk=0.0, origin=0.0, kinds=("radius", "tend", "tzero", "tie")):
    """Pairs/triples near decision boundaries, one group per cell on a
    3-spaced lattice of a 30^3 periodic grid (groups never share a
    neighbourhood)."""
    rng = np.random.default_rng(seed)
    nc, L = 30, 1.0
    h = L / nc
    D = 0.9 * h
    dt = 0.01
    pts = []
    for a in range(10):
        for b in range(10):
            for c in range(10):
                ctr = origin + (np.array([3 * a + 1, 3 * b + 1, 3 * c + 1]) + 0.5) * h
                kind = kinds[rng.integers(len(kinds))]
                gdir = rng.standard_normal(3)
                gdir /= np.linalg.norm(gdir)
                perp = np.cross(gdir, rng.standard_normal(3))
                perp /= np.linalg.norm(perp)
                gmag = rng.uniform(0.5, 2.0)
                eps = 2.0 ** -rng.integers(18, 51) * (1 if rng.random() < 0.5 else -1)
                if kind == "radius":
                    t0, d = rng.uniform(0.2, 0.8) * dt, D * (1 + eps)
                elif kind == "tend":
                    t0, d = dt * (1 + eps), D * rng.uniform(0.1, 0.9)
                elif kind == "tzero":
                    t0, d = eps * dt, D * rng.uniform(0.1, 0.9)
                else:
                    t0, d = rng.uniform(0.2, 0.8) * dt, D * rng.uniform(0.2, 0.6)
                g = gdir * gmag
                r = -g * t0 + perp * d
                V0 = rng.standard_normal(3) * bulk
                pts.append((ctr - r / 2, V0 - g / 2))
                pts.append((ctr + r / 2, V0 + g / 2))
                if kind == "tie":
                    # a third particle seeing the first at a near-equal key
                    perp2 = np.cross(gdir, perp)
                    r2 = -g * t0 + perp2 * d * (1 + eps)
                    pts.append((ctr - r / 2 + r2, V0 - g / 2 + g))
    n = len(pts)
    s = np.empty((6, n))
    for k, (x, v) in enumerate(pts):
        s[0:3, k] = x
        s[3:6, k] = v
    lo = origin
    s[0:3] = lo + np.mod(s[0:3] - lo, L)
    box = I.Box(n=n, lo=(lo,) * 3, hi=(lo + L,) * 3, ncell=(nc,) * 3, periodic=(True,) * 3, D2=D * D, dt=dt)
    perm = rng.permutation(n)
    return I.Workload("adversarial", [box], s[:, perm].copy(), 1)


def gpu_vs_oracle(kmc, w, precision, steps=1, **cfg):
    sim = kmc.Sim(w.boxes, w.state, seed=w.seed, precision=precision, **cfg)
    ref = O.Run(w)
    mism = 0
    for _ in range(steps):
        sim.step(1)
        ref.step()
        mism += int((sim.partners().cpu().numpy() != ref.partner_by_id).sum())
    stats = sim.stats()
    same_state = bool(np.array_equal(sim.state().cpu().numpy(), ref.full_state()))
    sim.close()
    return mism, same_state, stats


@pytest.mark.parametrize("mode", ["half", "full"])
@pytest.mark.parametrize("variant", [dict(), dict(bulk=20.0), dict(origin=1000.0), dict(bulk=5.0, origin=-300.0)])
def test_screen_exact_on_adversarial_pairs(kmc, variant, mode):
    w = adversarial(seed=11, **variant)
    sm = kmc.KMC_SEARCH_FULL if mode == "full" else kmc.KMC_SEARCH_HALF
    print(f"\n[screen] adversarial {variant} N={w.n} search={mode}", flush=True)
    mism64, st64, s64 = gpu_vs_oracle(kmc, w, kmc.KMC_FP64, steps=2, search_mode=sm)
    assert mism64 == 0 and st64
    mism, same, stats = gpu_vs_oracle(kmc, w, kmc.KMC_FP32_SCREEN, steps=2, search_mode=sm)
    print(f"[screen] mismatches={mism} candidates fp32={stats['candidates']} fp64={s64['candidates']}",
          flush=True)
    assert mism == 0 and same
    # the screen keeps every acceptable pair, and near-boundary rejects too
    assert stats["candidates"] >= s64["candidates"]


def adversarial_sparse_row(seed=0, spacing=200, nx=30000, kinds=("radius", "tend", "tzero")):
    """Near-boundary pairs along one sparse cell row: a pair every `spacing`
    cells of an nx-cell periodic x axis (cell edge 1/30), so that the 64
    consecutive particles of a wave lie thousands of cells apart.  The FP32
    screen's error bounds hold for search groups of at most 64 cells along
    x, which the search enforces by splitting such rows."""
    rng = np.random.default_rng(seed)
    h = 1.0 / 30.0
    D = 0.9 * h
    dt = 0.01
    pts = []
    for a in range(nx // spacing):
        ctr = np.array([(spacing * a + 1.5) * h, 1.5 * h, 1.5 * h])
        kind = kinds[rng.integers(len(kinds))]
        gdir = rng.standard_normal(3)
        gdir /= np.linalg.norm(gdir)
        perp = np.cross(gdir, rng.standard_normal(3))
        perp /= np.linalg.norm(perp)
        gmag = rng.uniform(0.5, 2.0)
        eps = 2.0 ** -rng.integers(18, 51) * (1 if rng.random() < 0.5 else -1)
        if kind == "radius":
            t0, d = rng.uniform(0.2, 0.8) * dt, D * (1 + eps)
        elif kind == "tend":
            t0, d = dt * (1 + eps), D * rng.uniform(0.1, 0.9)
        else:
            t0, d = eps * dt, D * rng.uniform(0.1, 0.9)
        g = gdir * gmag
        r = -g * t0 + perp * d
        pts.append((ctr - r / 2, -g / 2))
        pts.append((ctr + r / 2, g / 2))
    n = len(pts)
    s = np.empty((6, n))
    for k, (x, v) in enumerate(pts):
        s[0:3, k] = x
        s[3:6, k] = v
    L = (nx * h, 3 * h, 3 * h)
    for k in range(3):
        s[k] = np.mod(s[k], L[k])
    box = I.Box(n=n, lo=(0.0, 0.0, 0.0), hi=L, ncell=(nx, 3, 3), periodic=(True,) * 3, D2=D * D, dt=dt)
    perm = rng.permutation(n)
    return I.Workload("adversarial_sparse_row", [box], s[:, perm].copy(), 1)


@pytest.mark.parametrize("mode", ["half", "full"])
@pytest.mark.parametrize("spacing", [6, 30, 200])
def test_screen_exact_on_a_sparse_row(kmc, mode, spacing):
    """A wave's lanes span about 190, 930 or 6200 cells: the screen's
    thresholds for groups of up to 256, 1024 and 4096 cells (the widest
    rows split into groups of 4096)."""
    w = adversarial_sparse_row(seed=13, spacing=spacing, nx=150 * spacing)
    sm = kmc.KMC_SEARCH_FULL if mode == "full" else kmc.KMC_SEARCH_HALF
    print(f"\n[screen] sparse row, a pair every {spacing} cells, N={w.n} search={mode}", flush=True)
    mism64, st64, s64 = gpu_vs_oracle(kmc, w, kmc.KMC_FP64, steps=2, search_mode=sm)
    assert mism64 == 0 and st64
    mism, same, stats = gpu_vs_oracle(kmc, w, kmc.KMC_FP32_SCREEN, steps=2, search_mode=sm)
    print(f"[screen] mismatches={mism} candidates fp32={stats['candidates']} fp64={s64['candidates']}",
          flush=True)
    assert mism == 0 and same
    assert stats["candidates"] >= s64["candidates"]


def adversarial_outside(seed=0, lengths=100):
    """The adversarial pairs of the periodic 30^3 grid, with the pairs of the
    last lattice column moved `lengths` box lengths beyond hi along x: they
    are binned in the last cell (cells clamp), far from it.  A single wrap at
    the end of a step does not bring them back, so they stay outside."""
    w = adversarial(seed=seed, kinds=("radius", "tend", "tzero"))
    s = w.state.copy()
    b = w.boxes[0]
    L = b.hi[0] - b.lo[0]
    h = L / b.ncell[0]
    far = s[0] >= b.lo[0] + 27 * h          # lattice column a = 9 (cells 27..29)
    s[0, far] += lengths * L
    return I.Workload("adversarial_outside", [b], s, 1), int(far.sum())


@pytest.mark.parametrize("mode", ["half", "full"])
def test_screen_exact_with_particles_outside_the_grid(kmc, mode):
    w, nfar = adversarial_outside(seed=16)
    sm = kmc.KMC_SEARCH_FULL if mode == "full" else kmc.KMC_SEARCH_HALF
    print(f"\n[screen] {nfar} particles outside the grid, N={w.n} search={mode}", flush=True)
    mism64, st64, s64 = gpu_vs_oracle(kmc, w, kmc.KMC_FP64, steps=2, search_mode=sm)
    assert mism64 == 0 and st64 and s64["fallbacks"] == 0
    mism, same, stats = gpu_vs_oracle(kmc, w, kmc.KMC_FP32_SCREEN, steps=2, search_mode=sm)
    print(f"[screen] mismatches={mism} fallbacks={stats['fallbacks']}", flush=True)
    assert mism == 0 and same
    # both steps had particles outside: the FP32 path took the FP64 search
    assert stats["fallbacks"] == 2


def scaled(w, pos=1.0, vel=1.0):
    """The workload in other units: positions times `pos`, velocities times
    `vel`, dt times pos / vel.  Powers of two scale the FP64 definition
    exactly, so the partners are those of the unscaled workload."""
    b = w.boxes[0]
    s = w.state.copy()
    s[0:3] *= pos
    s[3:6] *= vel
    box = I.Box(n=b.n, lo=tuple(pos * x for x in b.lo), hi=tuple(pos * x for x in b.hi), ncell=b.ncell,
                periodic=b.periodic, D2=b.D2 * pos * pos, dt=b.dt * pos / vel)
    return I.Workload(w.name + "_scaled", [box], s, w.seed)


@pytest.mark.parametrize("mode", ["half", "full"])
def test_rounding_level_excursions_take_no_fallback(kmc, mode):
    """Particles one ulp beyond lo or hi (as a mirror image can land) stay
    within the bounds' slack: the FP32 path keeps the screen and is exact."""
    w = adversarial(seed=21, kinds=("radius", "tend", "tzero"))
    s = w.state.copy()
    b = w.boxes[0]
    rng = np.random.default_rng(21)
    pick = rng.choice(w.n, 60, replace=False)
    for k, i in enumerate(pick):
        ax = k % 3
        s[ax, i] = np.nextafter(b.hi[ax], np.inf) if k % 2 else np.nextafter(b.lo[ax], -np.inf)
    w2 = I.Workload("adversarial_ulp", [b], s, w.seed)
    sm = kmc.KMC_SEARCH_FULL if mode == "full" else kmc.KMC_SEARCH_HALF
    mism, same, stats = gpu_vs_oracle(kmc, w2, kmc.KMC_FP32_SCREEN, steps=2, search_mode=sm)
    print(f"\n[screen] one ulp outside ({mode}): mismatches={mism} fallbacks={stats['fallbacks']}", flush=True)
    assert mism == 0 and same and stats["fallbacks"] == 0


@pytest.mark.parametrize("mode", ["half", "full"])
@pytest.mark.parametrize("units", [dict(pos=2.0 ** -50), dict(vel=2.0 ** 70)], ids=["tiny_lengths", "huge_speeds"])
def test_screen_exact_outside_its_safe_range(kmc, units, mode):
    """Cell edges below 2^-40 (FP32 thresholds would underflow) or speeds
    above 2^40 (FP32 products would overflow): the FP32 path takes the FP64
    search for every step and stays exact."""
    base = adversarial(seed=19, kinds=("radius", "tend", "tzero"))
    w = scaled(base, **units)
    sm = kmc.KMC_SEARCH_FULL if mode == "full" else kmc.KMC_SEARCH_HALF
    print(f"\n[screen] units {units} N={w.n} search={mode}", flush=True)
    mism, same, stats = gpu_vs_oracle(kmc, w, kmc.KMC_FP32_SCREEN, steps=2, search_mode=sm)
    print(f"[screen] mismatches={mism} fallbacks={stats['fallbacks']}", flush=True)
    assert mism == 0 and same and stats["fallbacks"] == 2
    # the units do not change the oracle's partners
    ra, rb = O.Run(base), O.Run(w)
    ra.step()
    rb.step()
    assert np.array_equal(ra.partner_by_id, rb.partner_by_id)


@pytest.mark.parametrize("mode", ["half", "full"])
def test_negative_control_without_error_bounds(kmc, mode):
    """With the error bounds disabled the FP32 screen decides near-boundary
    pairs from FP32 values alone and must disagree with the oracle."""
    w = adversarial(seed=12, kinds=("radius", "tend", "tzero"))
    sm = kmc.KMC_SEARCH_FULL if mode == "full" else kmc.KMC_SEARCH_HALF
    mism, _, stats = gpu_vs_oracle(kmc, w, kmc.KMC_FP32_SCREEN, guard_scale=-1.0, search_mode=sm)
    print(f"\n[screen] guard off ({mode}): mismatches={mism} rechecks={stats['rechecks']}", flush=True)
    assert mism > 0
    mism_on, _, _ = gpu_vs_oracle(kmc, w, kmc.KMC_FP32_SCREEN, search_mode=sm)
    assert mism_on == 0


def dense_gas(n=20_000, D=0.1, dt=0.05, seed=5):
    """Uniform gas with many acceptable partners per particle (about 70 at
    the defaults, about 7 with D=0.05, dt=0.02)."""
    rng = np.random.default_rng(seed)
    s = np.empty((6, n))
    s[0:3] = rng.random((3, n))
    s[3:6] = rng.standard_normal((3, n))
    box = I.Box(n=n, lo=(0, 0, 0), hi=(1, 1, 1), ncell=(10, 10, 10), periodic=(True,) * 3, D2=D * D, dt=dt)
    return I.Workload("dense", [box], s, 2)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_candidate_overflow_paths(kmc, precision):
    prec = kmc.KMC_FP64 if precision == "fp64" else kmc.KMC_FP32_SCREEN
    # medium density: lanes overflow their registers and particles their
    # candidate slots (full re-search), without a whole-step fallback
    w = dense_gas(D=0.05, dt=0.02)
    mism, same, stats = gpu_vs_oracle(kmc, w, prec, steps=2)
    assert mism == 0 and same
    assert stats["rechecks"] > 0 and stats["fallbacks"] == 0
    # extreme density: exact by re-search or by the whole-step fallback
    w = dense_gas()
    mism, same, stats = gpu_vs_oracle(kmc, w, prec, steps=2)
    assert mism == 0 and same
    assert stats["rechecks"] > w.n // 2 or stats["fallbacks"] > 0
    # a recheck list of one entry forces the fallback every step
    mism, same, stats = gpu_vs_oracle(kmc, w, prec, recheck_capacity=1, use_graph=True, steps=2)
    assert mism == 0 and same
    assert stats["fallbacks"] == 2
    # the full-neighbourhood search needs neither
    mism, same, stats = gpu_vs_oracle(kmc, w, prec, steps=2, search_mode=kmc.KMC_SEARCH_FULL)
    assert mism == 0 and same
    assert stats["rechecks"] == 0 and stats["fallbacks"] == 0


@pytest.mark.parametrize("guard", [1.0, 16.0])
def test_guard_scale_does_not_change_results(kmc, guard):
    w = I.c1_small(steps=3)
    mism, same, _ = gpu_vs_oracle(kmc, w, kmc.KMC_FP32_SCREEN, steps=3, guard_scale=guard)
    assert mism == 0 and same


def test_screen_is_tight_on_a_gas(kmc):
    w = I.c3_sphere(n=400_000, steps=2)
    _, _, s64 = gpu_vs_oracle(kmc, w, kmc.KMC_FP64, steps=2)
    mism, same, stats = gpu_vs_oracle(kmc, w, kmc.KMC_FP32_SCREEN, steps=2)
    assert mism == 0 and same
    extra = stats["candidates"] / max(s64["candidates"], 1) - 1.0
    print(f"\n[screen] c3 N=4e5: screen keeps {100 * extra:.3f}% more pairs than FP64 accepts; "
          f"rechecks {stats['rechecks']}", flush=True)
    assert 0.0 <= extra < 0.01
    assert stats["rechecks"] < 0.001 * 2 * w.n
