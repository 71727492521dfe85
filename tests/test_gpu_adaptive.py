"""GPU parity of the density-adaptive bins (Section 1: an adaptive bin size
against the load imbalance of dense bins; Section 4: smaller bins where the
density is higher) against the oracle's adaptive mode.

Every step the partner array, the collision count and digest and the pair
tests must equal the oracle's, and the FP64 state must be bit-identical, in
both precisions, on gases where split and unsplit cells meet (Gaussian blobs,
clusters across periodic seams, a reflecting sphere, several boxes, particle
kinds).  At N = 1e7 (the blob workload) the step is checked at sampled
particles against the oracle's per-particle evaluation.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1310_3437_amd import inputs as I

pytestmark = pytest.mark.gpu


def _adapt(w, levels, threshold):
    w.adapt_levels, w.adapt_threshold = levels, threshold
    return w


def run_adaptive(kmc, w, steps, precision, **cfg):
    print(f"\n[adapt] {w.name} N={w.n} boxes={len(w.boxes)} L={w.adapt_levels} T={w.adapt_threshold} "
          f"{precision} {cfg}", flush=True)
    prec = kmc.KMC_FP64 if precision == "fp64" else kmc.KMC_FP32_SCREEN
    kinds = None if w.species is None else (w.species, w.radius, w.mass)
    sim = kmc.Sim(w.boxes, w.state, device="cuda:0", seed=w.seed, kinematics=w.kinematics, precision=prec,
                  search_mode=kmc.KMC_SEARCH_FULL, adapt_levels=w.adapt_levels,
                  adapt_threshold=w.adapt_threshold, kinds=kinds, **cfg)
    ref = O.Run(w)
    hist = []
    for s in range(steps):
        sim.step(1)
        hist.append(ref.step())
        p = sim.partners().cpu().numpy()
        bad = np.flatnonzero(p != ref.partner_by_id)
        assert bad.size == 0, f"step {s}: {bad.size} partner mismatches, first ids {bad[:5]}"
        assert sim.pair_tests() == ref.pair_tests, f"step {s}: pair tests differ"
    hn, hd = sim.history()
    assert [(int(a), int(b)) for a, b in zip(hn, hd)][-steps:] == hist
    assert np.array_equal(sim.state().cpu().numpy(), ref.full_state())
    stats = sim.stats()
    sim.close()
    print(f"[adapt] ok pairs {[h[0] for h in hist]} fallbacks {stats['fallbacks']}", flush=True)
    return hist


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("levels,threshold", [(1, 4), (2, 8), (3, 8), (3, 2)])
def test_blobs(kmc, precision, levels, threshold):
    w = _adapt(I.c5_blobs(n=80_000, steps=3), levels, threshold)
    run_adaptive(kmc, w, 3, precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_clusters_across_periodic_seams_and_walls(kmc, precision):
    """Dense clusters placed on the periodic seams and corners (split cells
    whose touching leaves lie across the seam), and the same gas between
    reflecting walls."""
    rng = np.random.default_rng(31)
    for periodic in (True, False):
        box, s = I.uniform_box(30_000, L=1.0, D=0.02, periodic=periodic, ic_seed=32, dt=0.002)
        k = 18_000
        centres = np.array([[0.0, 0.5, 0.5], [0.0, 0.0, 0.0], [0.98, 0.02, 0.5]]).T
        which = rng.integers(0, 3, k)
        pts = centres[:, which] + 0.015 * rng.standard_normal((3, k))
        s[0:3, :k] = np.mod(pts, 1.0) if periodic else np.clip(pts, 0.0, 1.0)
        s[0:3][s[0:3] >= 1.0] = 0.0 if periodic else 1.0
        w = _adapt(I.Workload("clusters", [box], s, 3), 3, 4)
        run_adaptive(kmc, w, 3, precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_sphere_batch_and_graph(kmc, precision):
    """A reflecting sphere with its dense infalling core, a batch of boxes in
    one launch, and graph replay."""
    w = _adapt(I.c3_sphere(n=120_000, steps=3), 2, 3)
    run_adaptive(kmc, w, 3, precision, use_graph=True)
    w = _adapt(I.c4_batch(nboxes=8, n_lo=500, n_hi=6000, steps=3), 2, 2)
    run_adaptive(kmc, w, 3, precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_kinds(kmc, precision):
    w = _adapt(I.c6_mixture(n=40_000, ic_seed=21, steps=2), 2, 2)
    run_adaptive(kmc, w, 2, precision)


def test_unsplit_equals_the_uniform_grid(kmc):
    """A threshold no cell exceeds: the adaptive path gives the plain
    step's results (and every particle goes through the plain search)."""
    w = I.c5_blobs(n=60_000, steps=2)
    hist = run_adaptive(kmc, _adapt(w, 3, 1 << 30), 2, "fp32")
    ref = O.Run(I.c5_blobs(n=60_000, steps=2))
    assert hist == [ref.step(), ref.step()]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_blobs_1e7_sampled(kmc, precision):
    """The blob workload at N = 1e7 with three levels and threshold 8:
    partners and post-step states at sampled particles (random ones,
    colliders, and particles of split cells) equal the oracle's evaluation
    of the same step; collision count and digest match the partner array."""
    import torch
    w = _adapt(I.c5_blobs(steps=1), 3, 8)
    n = w.n
    prec = kmc.KMC_FP64 if precision == "fp64" else kmc.KMC_FP32_SCREEN
    print(f"\n[adapt] c5_blobs N={n} {precision}", flush=True)
    sim = kmc.Sim(w.boxes, w.state, device="cuda:0", seed=w.seed, precision=prec,
                  search_mode=kmc.KMC_SEARCH_FULL, adapt_levels=3, adapt_threshold=8)
    sim.step(1)
    p = sim.partners().cpu().numpy()
    st = sim.state()
    hn, hd = sim.history()
    sim.close()
    idx = np.arange(n)
    has = p >= 0
    mutual = np.zeros(n, dtype=bool)
    mutual[has] = p[p[has]] == idx[has]
    assert int(hn[-1]) == int((mutual & (idx < p)).sum())
    rng = np.random.default_rng(7)
    box = w.boxes[0]
    # particles of dense cells (the split ones)
    cells = np.floor(w.state[0:3] * np.array(box.inv_h)[:, None]).astype(np.int64)
    lin = cells[0] + box.ncell[0] * (cells[1] + box.ncell[1] * cells[2])
    cnt = np.bincount(lin, minlength=box.ncells)
    dense = np.flatnonzero(cnt[lin] > 64)
    sel = np.unique(np.concatenate([rng.choice(n, 1500, replace=False),
                                    rng.choice(dense, 1500, replace=False),
                                    rng.choice(np.flatnonzero(mutual), 500, replace=False)])).astype(np.int64)
    ref_p, ref_s = O.step_sampled(box, w.state, np.arange(n, dtype=np.uint32), 0, sel, seed=w.seed, adapt=(3, 8))
    bad = np.flatnonzero(p[sel] != ref_p)
    assert bad.size == 0, f"{bad.size} of {sel.size} sampled partners differ, first ids {sel[bad[:5]]}"
    got = st[:, torch.as_tensor(sel, device=st.device)].cpu().numpy()
    assert np.array_equal(got, ref_s)
    print(f"[adapt] {sel.size} sampled particles identical ({len(dense)} in cells of > 64)", flush=True)


def test_autotuned_threshold(kmc):
    """KMC_TUNE_ADAPT times the thresholds 4, 8, 16 and 32 and returns one of
    them; the run with the returned configuration equals the oracle's
    adaptive mode at that threshold."""
    w = _adapt(I.c5_blobs(n=80_000, steps=2), 3, 8)
    boxes, cfg, tun = kmc.autotune(w.boxes, w.state, device="cuda:0", steps=1, seed=w.seed,
                                   flags=kmc.KMC_TUNE_LAUNCH | kmc.KMC_TUNE_ADAPT,
                                   search_mode=kmc.KMC_SEARCH_FULL, adapt_levels=3, adapt_threshold=8)
    assert cfg["adapt_threshold"] in (4, 8, 16, 32)
    assert sorted({t["adapt_threshold"] for t in tun["tried"]}) == [4, 8, 16, 32]
    assert all(t["search_mode"] == kmc.KMC_SEARCH_FULL for t in tun["tried"])
    w.adapt_threshold = cfg["adapt_threshold"]
    run_adaptive(kmc, w, 2, "fp64", block_size=cfg["block_size"], tile=cfg["tile"])
