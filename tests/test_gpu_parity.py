"""GPU parity: the HIP path of libkmc.so against the CPU oracle.

Every step the partner array (by id), the collision count and the digest
must equal the oracle's exactly, and the FP64 state must agree to 1e-12
relative (bit-identical is expected: both evaluate the same IEEE-754
binary64 expressions in the same order).  Sizes are chosen so the oracle
finishes in seconds while spanning many blocks with a ragged tail.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1310_3437_amd import inputs as I

pytestmark = pytest.mark.gpu


def state_close(a, b, boxes, offsets):
    """Max relative state difference: |dx| / box extent, |dv| / max |v|."""
    worst = 0.0
    for k, bx in enumerate(boxes):
        s, e = offsets[k], offsets[k + 1]
        if e == s:
            continue
        ext = max(float(bx.hi[a] - bx.lo[a]) for a in range(3))
        dx = np.abs(a_[0:3, s:e] - b[0:3, s:e]).max() / ext if (a_ := a) is not None else 0.0
        vmax = np.abs(b[3:6, s:e]).max()
        dv = np.abs(a[3:6, s:e] - b[3:6, s:e]).max() / max(vmax, 1e-300)
        worst = max(worst, dx, dv)
    return worst


PRECISIONS = ["fp64", "fp32"]


def _prec(kmc, name):
    return kmc.KMC_FP64 if name == "fp64" else kmc.KMC_FP32_SCREEN


def run_parity(kmc, w, steps, check_every=1, precision="fp64", **cfg):
    print(f"\n[parity] {w.name} N={w.n} boxes={len(w.boxes)} steps={steps} {precision} cfg={cfg}", flush=True)
    cfg["precision"] = _prec(kmc, precision)
    if w.dt_rule:
        cfg.update(dt_rule=w.dt_rule, dt_factor=w.dt_factor)
    if w.dims == 2:
        cfg.update(dims=2)
    sim = kmc.Sim(w.boxes, w.state, device="cuda:0", seed=w.seed, kinematics=w.kinematics, **cfg)
    ref = O.Run(w)
    digests = []
    for s in range(steps):
        sim.step(1)
        npairs, dig = ref.step()
        digests.append((npairs, dig))
        if (s + 1) % check_every == 0 or s == steps - 1:
            p = sim.partners().cpu().numpy()
            bad = np.nonzero(p != ref.partner_by_id)[0]
            assert bad.size == 0, f"step {s}: {bad.size} partner mismatches, first ids {bad[:5]}"
    hn, hd = sim.history()
    got = [(int(a), int(b)) for a, b in zip(hn, hd)][-steps:]
    assert got == digests, "per-step (npairs, digest) differ"
    st = sim.state().cpu().numpy()
    ref_st = ref.full_state()
    rel = state_close(st, ref_st, w.boxes, w.offsets)
    assert rel <= 1e-12, f"state differs by {rel:.3e} relative"
    exact = bool(np.array_equal(st, ref_st))
    dt, tm = sim.time()
    assert list(dt) == ref.dt_last and list(tm) == ref.time, "time steps differ"
    stats = sim.stats()
    assert stats["absorbed"] == ref.absorbed(), (stats["absorbed"], ref.absorbed())
    print(f"[parity] ok exact={exact} rechecks={stats['rechecks']} fallbacks={stats['fallbacks']}", flush=True)
    sim.close()
    run_parity.last_stats = stats
    run_parity.last_state = st
    return digests, exact


@pytest.mark.parametrize("precision", PRECISIONS)
def test_c1_small_full(kmc, precision):
    w = I.c1_small()
    d, exact = run_parity(kmc, w, w.steps, precision=precision)
    assert exact
    assert sum(n for n, _ in d) > 1000


@pytest.mark.parametrize("cfg", [dict(use_graph=True), dict(block_size=64),
                                 dict(block_size=1024, use_graph=True),
                                 dict(block_size=512, use_graph=True, precision="fp32")])
def test_c1_launch_shapes(kmc, cfg):
    w = I.c1_small(steps=6)
    _, exact = run_parity(kmc, w, w.steps, **cfg)
    assert exact


@pytest.mark.parametrize("precision", PRECISIONS)
def test_c2_shock_scaled(kmc, precision):
    w = I.c2_shock(n=40_000, steps=15)
    _, exact = run_parity(kmc, w, w.steps, check_every=5, precision=precision)
    assert exact


@pytest.mark.parametrize("precision", PRECISIONS)
def test_c3_sphere_scaled(kmc, precision):
    w = I.c3_sphere(n=150_000, steps=3)
    _, exact = run_parity(kmc, w, w.steps, precision=precision)
    assert exact


@pytest.mark.parametrize("precision", PRECISIONS)
def test_c4_batch_scaled(kmc, precision):
    w = I.c4_batch(nboxes=12, n_lo=100, n_hi=4000, steps=4)
    _, exact = run_parity(kmc, w, w.steps, use_graph=True, precision=precision)
    assert exact


@pytest.mark.parametrize("precision", PRECISIONS)
def test_c5_blobs_scaled(kmc, precision):
    w = I.c5_blobs(n=60_000, steps=3)
    _, exact = run_parity(kmc, w, w.steps, precision=precision)
    assert exact


@pytest.mark.parametrize("precision", PRECISIONS)
def test_long_run_graph_replay(kmc, precision):
    """Sixty steps replayed from one captured graph (checked every ten steps):
    lists, counters and the history ring stay exact over many steps."""
    w = I.c1_small(n=20_000, steps=60)
    d, exact = run_parity(kmc, w, 60, check_every=10, precision=precision, use_graph=True, history=64)
    assert exact and min(n for n, _ in d) > 500


def test_velocity_only_kinematics(kmc):
    w = I.c1_small(steps=3)
    w.kinematics = 1
    _, exact = run_parity(kmc, w, w.steps)
    assert exact


def test_tiny_and_degenerate(kmc):
    # one particle, a head-on pair, three-body chain with a key tie
    b1 = I.Box(n=1, lo=(0, 0, 0), hi=(1, 1, 1), ncell=(3, 3, 3), periodic=(True,) * 3, D2=0.01, dt=0.05)
    s1 = np.array([[0.99], [0.5], [0.01], [0.5], [0.0], [-0.5]])
    run_parity(kmc, I.Workload("one", [b1], s1, 3), 3)
    b2 = I.Box(n=2, lo=(-1, -1, -1), hi=(1, 1, 1), ncell=(64, 64, 64), D2=2.0 ** -10, dt=2.0 ** -6)
    s2 = np.zeros((6, 2))
    s2[0, 0], s2[3, 0], s2[0, 1], s2[3, 1] = -2.0 ** -7, 1.0, 2.0 ** -7, -1.0
    d, exact = run_parity(kmc, I.Workload("head_on", [b2], s2, 1, seed=9), 1)
    assert d[0][0] == 1 and exact
    b3 = I.Box(n=3, lo=(-1, -1, -1), hi=(1, 1, 1), ncell=(64, 64, 64), D2=2.0 ** -10, dt=2.0 ** -6)
    s3 = np.zeros((6, 3))
    s3[0:3, 0] = (-2.0 ** -6, 2.0 ** -7, 0.0)
    s3[3:6, 0] = (1.0, 0.0, 0.0)
    s3[0:3, 2] = (2.0 ** -6, 0.0, 0.0)
    s3[3:6, 2] = (-1.0, 0.0, 0.0)
    d, exact = run_parity(kmc, I.Workload("three", [b3], s3, 1), 1)
    assert d[0][0] == 1 and exact


def test_particles_on_cell_faces(kmc):
    rng = np.random.default_rng(3)
    n = 20_000
    box = I.Box(n=n, lo=(0, 0, 0), hi=(1, 1, 1), ncell=(20, 20, 20), periodic=(True, False, True),
                D2=0.045 ** 2, dt=0.01)
    s = np.empty((6, n))
    s[0:3] = rng.integers(0, 20, (3, n)) / 20.0
    s[0:3] += (rng.random((3, n)) < 0.5) * rng.random((3, n)) * 0.05
    s[0:3] = np.minimum(s[0:3], 1.0)
    s[0][s[0] >= 1.0] = 0.0
    s[2][s[2] >= 1.0] = 0.0
    s[3:6] = rng.standard_normal((3, n))
    _, exact = run_parity(kmc, I.Workload("faces", [box], s, 3), 3)
    assert exact


def test_empty_box_and_empty_boxes_in_batch(kmc):
    b0 = I.Box(n=0, lo=(0, 0, 0), hi=(1, 1, 1), ncell=(4, 4, 4), periodic=(True,) * 3, D2=0.01, dt=0.01)
    w = I.c1_small(n=2000, steps=2)
    batch = I.Workload("mixed", [b0, w.boxes[0], b0], w.state, 2)
    run_parity(kmc, batch, 2)


def test_resume_and_determinism(kmc):
    w = I.c1_small(steps=6)
    a = kmc.Sim(w.boxes, w.state, seed=w.seed)
    a.step(6)
    ha = a.history()
    sa = a.state().cpu().numpy()
    b = kmc.Sim(w.boxes, w.state, seed=w.seed)
    b.step(3)
    mid = b.state().cpu().numpy()
    hb1 = b.history()
    c = kmc.Sim(w.boxes, mid, seed=w.seed, step0=3)
    c.step(3)
    hc = c.history()
    assert np.array_equal(c.state().cpu().numpy(), sa)
    assert list(ha[1]) == list(hb1[1]) + list(hc[1])
    d = kmc.Sim(w.boxes, w.state, seed=w.seed, use_graph=True)
    d.step(6)
    assert np.array_equal(d.state().cpu().numpy(), sa)
    for s in (a, b, c, d):
        s.close()


def test_pair_test_count_matches_oracle(kmc):
    w = I.c3_sphere(n=100_000, steps=1)
    sim = kmc.Sim(w.boxes, w.state, seed=w.seed)
    sim.step(1)
    ref = O.Run(w)
    ref.step()
    assert sim.pair_tests() == ref.pair_tests
    sim.close()


def _adaptive(w, factor, cap_scale):
    import dataclasses
    w.boxes = [dataclasses.replace(b, dt=b.dt * cap_scale) for b in w.boxes]
    w.dt_rule, w.dt_factor = 1, factor
    return w


@pytest.mark.parametrize("precision", PRECISIONS)
def test_adaptive_time_step_c1(kmc, precision):
    """The adaptive step of Section 1 (dt = dx / v_max, capped by the box
    dt), recomputed on the device every step."""
    w = _adaptive(I.c1_small(steps=8), 1.0, 100.0)
    run_parity(kmc, w, 8, precision=precision)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_adaptive_time_step_batch_and_sphere(kmc, precision):
    w = _adaptive(I.c4_batch(nboxes=12, n_lo=100, n_hi=4000, steps=4), 0.5, 10.0)
    run_parity(kmc, w, 4, precision=precision, use_graph=True)
    w = _adaptive(I.c3_sphere(n=150_000, steps=3), 0.3, 10.0)
    run_parity(kmc, w, 3, precision=precision, block_size=128)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_paper_time_step_full_search_many_kept_pairs(kmc, precision):
    """Section 1's own regime (dt = dx / v_max, no cap below it) gives each
    particle many acceptable partners per step; with the full search every
    lane then keeps more pairs than its deferred slots, so both the deferred
    FP64 decisions and the immediate ones run (FP32 screen), in graph
    replay, and the result is still the oracle's."""
    # the Fig. 1 gas (one speed, random directions) at three particles per
    # cell: about 11 acceptable partners per particle and step
    w = I.ppc_sweep_case(n=100_000, ppc=3.0)
    run_parity(kmc, w, 3, precision=precision, search_mode=kmc.KMC_SEARCH_FULL, use_graph=True)
    st = run_parity.last_stats
    # pairs decided in FP64 (FP32 screen) or accepted (FP64), per particle-step
    per = st["candidates"] / (w.n * 3)
    print(f"[parity] decided or accepted pairs per particle-step {per:.2f}", flush=True)
    assert per > 5.0, per   # well above the four deferred slots of a lane


@pytest.mark.parametrize("precision", PRECISIONS)
def test_paper_time_step_half_search_overflow_paths(kmc, precision):
    """The same gas with the half-neighbourhood search: lanes keep more
    pairs than their register slots (the overflow pair list), particles
    collect more candidates than their list slots (the FP64 re-search), or
    the whole step falls back to the FP64 search; every path must still give
    the oracle's result."""
    w = I.ppc_sweep_case(n=100_000, ppc=3.0)
    run_parity(kmc, w, 3, precision=precision, search_mode=kmc.KMC_SEARCH_HALF)
    st = run_parity.last_stats
    assert st["rechecks"] > 0 or st["fallbacks"] > 0, st


@pytest.mark.parametrize("precision", PRECISIONS)
def test_full_neighbourhood_search_mode(kmc, precision):
    """KMC_SEARCH_FULL (running minimum over the whole neighbourhood, no
    candidate lists) gives the oracle's result on every workload shape."""
    cases = [(I.c1_small(steps=4), 4), (I.c2_shock(n=40_000, steps=5), 5), (I.c3_sphere(n=150_000, steps=2), 2),
             (I.c4_batch(nboxes=12, n_lo=100, n_hi=4000, steps=2), 2), (I.c5_blobs(n=60_000, steps=2), 2)]
    for w, steps in cases:
        run_parity(kmc, w, steps, precision=precision, search_mode=kmc.KMC_SEARCH_FULL)
    assert run_parity.last_stats["rechecks"] == 0 and run_parity.last_stats["fallbacks"] == 0


def test_autotune_launch_and_cells(kmc):
    """kmc_autotune times every candidate; its launch choice leaves the
    results unchanged, and a tuned cell grid is a different (valid) grid that
    the oracle reproduces when given the same boxes."""
    w = I.c5_blobs(n=60_000, steps=2)
    boxes, cfg, tun = kmc.autotune(w.boxes, w.state, device="cuda:0", flags=kmc.KMC_TUNE_LAUNCH, steps=2,
                                   seed=w.seed, precision=kmc.KMC_FP32_SCREEN)
    print(f"\n[tune] launch: {cfg['search_mode']}/{cfg['block_size']}/tile {cfg['tile']} "
          f"{[round(t['ms_per_step'], 3) for t in tun['tried']]}", flush=True)
    # organisations x 1 precision, then 2 more tile shapes, then 2 more block sizes
    assert boxes == w.boxes and len(tun["tried"]) == 6
    assert all(np.isfinite(t["ms_per_step"]) for t in tun["tried"])
    assert {t["tile"] for t in tun["tried"]} == {0, 1, 2}
    assert {t["block_size"] for t in tun["tried"]} == {128, 256, 512}
    assert {t["precision"] for t in tun["tried"]} == {kmc.KMC_FP32_SCREEN}
    best = tun["tried"][tun["best"]]
    assert best["ms_per_step"] == min(t["ms_per_step"] for t in tun["tried"])
    run_parity(kmc, w, 2, precision="fp32", search_mode=cfg["search_mode"], block_size=cfg["block_size"],
               tile=cfg["tile"])

    boxes, cfg, tun = kmc.autotune(w.boxes, w.state, device="cuda:0",
                                   flags=kmc.KMC_TUNE_LAUNCH | kmc.KMC_TUNE_CELLS, steps=2,
                                   seed=w.seed, precision=kmc.KMC_FP32_SCREEN)
    best = tun["tried"][tun["best"]]
    print(f"[tune] cells: kappa {best['kappa']} grid {boxes[0].ncell} "
          f"{cfg['search_mode']}/{cfg['block_size']}", flush=True)
    assert len(tun["tried"]) == 24
    assert boxes[0] == kmc.box_with_kappa(w.boxes[0], best["kappa"])
    w.boxes = boxes
    run_parity(kmc, w, 2, precision="fp32", search_mode=cfg["search_mode"], block_size=cfg["block_size"],
               tile=cfg["tile"])


def test_autotune_precision(kmc):
    """KMC_TUNE_PRECISION also times both precisions (the partners and
    states are the same bit for bit); the tuned configuration reproduces the
    oracle."""
    w = I.c3_sphere(n=150_000, steps=2)
    boxes, cfg, tun = kmc.autotune(w.boxes, w.state, device="cuda:0",
                                   flags=kmc.KMC_TUNE_LAUNCH | kmc.KMC_TUNE_PRECISION, steps=2, seed=w.seed)
    tried = tun["tried"]
    print(f"\n[tune] precision: {cfg['precision']} {cfg['search_mode']}/{cfg['block_size']}/tile {cfg['tile']} "
          f"{[(t['precision'], t['search_mode'], round(t['ms_per_step'], 3)) for t in tried]}", flush=True)
    assert len(tried) == 8
    assert {(t["precision"], t["search_mode"]) for t in tried[:4]} == {(0, 0), (0, 1), (1, 0), (1, 1)}
    best = tried[tun["best"]]
    assert best["ms_per_step"] == min(t["ms_per_step"] for t in tried)
    assert cfg["precision"] == best["precision"] and cfg["tile"] == best["tile"]
    run_parity(kmc, w, 2, precision="fp32" if cfg["precision"] == kmc.KMC_FP32_SCREEN else "fp64",
               search_mode=cfg["search_mode"], block_size=cfg["block_size"], tile=cfg["tile"])


@pytest.mark.parametrize("tile", [1, 2])
@pytest.mark.parametrize("mode", ["half", "full"])
@pytest.mark.parametrize("precision", PRECISIONS)
def test_tile_shapes(kmc, precision, mode, tile):
    """The other tile shapes of the search kernel (small LDS chunks; large
    chunks with fewer waves per SIMD) give the oracle's results."""
    sm = kmc.KMC_SEARCH_FULL if mode == "full" else kmc.KMC_SEARCH_HALF
    for w, steps in [(I.c3_sphere(n=150_000, steps=2), 2), (I.c5_blobs(n=60_000, steps=2), 2),
                     (I.c4_batch(nboxes=6, n_lo=100, n_hi=3000, steps=2), 2)]:
        run_parity(kmc, w, steps, precision=precision, search_mode=sm, tile=tile)


def test_autotune_cache_reuses_the_choice(kmc, tmp_path):
    w = I.c1_small(steps=1)
    cache = str(tmp_path / "tune.json")
    b1, c1, t1 = kmc.autotune(w.boxes, w.state, device="cuda:0", steps=1, cache=cache, seed=w.seed)
    b2, c2, t2 = kmc.autotune(w.boxes, w.state, device="cuda:0", steps=1, cache=cache, seed=w.seed)
    assert not t1["cached"] and t2["cached"]
    assert (b1, c1["search_mode"], c1["block_size"]) == (b2, c2["search_mode"], c2["block_size"])


@pytest.mark.parametrize("mode", ["half", "full"])
@pytest.mark.parametrize("precision", PRECISIONS)
def test_planar_mode(kmc, precision, mode):
    """Two-dimensional runs (one cell layer along z, planar scatter)."""
    sm = kmc.KMC_SEARCH_FULL if mode == "full" else kmc.KMC_SEARCH_HALF
    w = I.c1_planar(steps=6)
    run_parity(kmc, w, 6, precision=precision, search_mode=sm)
    st = run_parity.last_state
    assert np.all(st[2] == 0.5) and np.all(st[5] == 0.0)
    w = _adaptive(I.c1_planar(n=50_000, D=0.004, steps=3), 0.5, 10.0)
    run_parity(kmc, w, 3, precision=precision, search_mode=sm, use_graph=True)


@pytest.mark.parametrize("mode", ["half", "full"])
@pytest.mark.parametrize("precision", PRECISIONS)
def test_absorbing_faces(kmc, precision, mode):
    """Absorbing faces (Section 1): particles beyond them leave the gas; they
    no longer search, collide or move, and their last state is kept."""
    import dataclasses
    sm = kmc.KMC_SEARCH_FULL if mode == "full" else kmc.KMC_SEARCH_HALF
    w = I.c2_shock(n=40_000, steps=12)
    w.boxes = [dataclasses.replace(b, absorb=(True, False, False)) for b in w.boxes]
    run_parity(kmc, w, 12, precision=precision, search_mode=sm)
    assert run_parity.last_stats["absorbed"] > 0
    # periodic y and z, absorbing x, adaptive step, graph replay
    w = _adaptive(I.c1_small(steps=6), 1.0, 10.0)
    w.boxes = [dataclasses.replace(b, periodic=(False, True, True), absorb=(True, False, False)) for b in w.boxes]
    run_parity(kmc, w, 6, precision=precision, search_mode=sm, use_graph=True)
    assert run_parity.last_stats["absorbed"] > 0


@pytest.mark.parametrize("use_graph", [False, True])
def test_history_keeps_exactly_its_capacity(kmc, use_graph):
    """With history = H the library keeps the last H steps: after exactly H
    steps all H rows (the oldest included) equal the oracle's, and after
    more steps the last H do."""
    w = I.c1_small(steps=8)
    H = 5
    sim = kmc.Sim(w.boxes, w.state, device="cuda:0", seed=w.seed, history=H, use_graph=use_graph)
    ref = O.Run(w)
    want = []
    for s in range(8):
        sim.step(1)
        want.append(ref.step())
        if s + 1 in (H, 8):
            hn, hd = sim.history()
            got = [(int(a), int(b)) for a, b in zip(hn, hd)]
            assert len(got) == H and got == want[-H:], f"after {s + 1} steps"
            assert all(n > 0 for n, _ in got)
    sim.close()
