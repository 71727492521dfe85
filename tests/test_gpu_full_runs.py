"""GPU parity over whole runs of the benchmark workloads, at their full sizes
and step counts, against the oracle's record of the same runs
(tests/golden/full_<name>.json, written by tests/golden/make_full_runs.py
with the CPU oracle alone).

Every step: the partner array (the partner id of every particle id, -1 for
none) must hash to the oracle's, the ordered pair tests of the 27-cell
search must be the oracle's, and the step's collision count and digest must
be the oracle's.  After the last step the (6, N) FP64 state in id order
must hash to the oracle's (bit-exact; the sampled particles stored beside the
hash give the size of any difference).  Both precisions run; the headline
workload (c3_sphere at N = 1e8) runs in graph-replay mode, as the benchmark
times it.
"""
import hashlib
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1310_3437_amd import inputs as I

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden(name):
    with open(os.path.join(HERE, "golden", f"full_{name}.json")) as f:
        return json.load(f)


def _sha(a):
    h = hashlib.sha256()
    mv = memoryview(np.ascontiguousarray(a)).cast("B")
    for s in range(0, len(mv), 1 << 26):
        h.update(mv[s:s + (1 << 26)])
    return h.hexdigest()


def _workload(g):
    w = I.CONFIGS[g["workload"]](steps=g["steps"], **g["generator_kwargs"])
    fp = g["input"]
    assert w.n == fp["n"] and len(w.boxes) == fp["nboxes"]
    assert [float(b.dt).hex() for b in w.boxes[:4]] == fp["dt"]
    assert [float(b.D2).hex() for b in w.boxes[:4]] == fp["D2"]
    assert _sha(w.state) == fp["state_sha256"], "the input generator no longer gives the recorded input"
    return w


def _check_run(kmc, w, g, precision, **cfg):
    import torch
    name = g["workload"]
    prec = kmc.KMC_FP64 if precision == "fp64" else kmc.KMC_FP32_SCREEN
    print(f"\n[run] {name} N={w.n} steps={g['steps']} {precision} {cfg}", flush=True)
    sim = kmc.Sim(w.boxes, w.state, device="cuda:0", seed=g["seed"], kinematics=g["kinematics"],
                  precision=prec, history=max(64, g["steps"]), **cfg)
    for e in g["per_step"]:
        sim.step(1)
        p = sim.partners().cpu().numpy()
        assert p.dtype == np.int32
        if _sha(p.astype("<i4")) != e["partners_sha256"]:
            raise AssertionError(f"{name} {precision}: partner array differs from the oracle's at step {e['step']}")
        assert sim.pair_tests() == e["pair_tests"], f"{name} {precision}: pair tests differ at step {e['step']}"
    hn, hd = sim.history()
    got = [(int(a), int(b)) for a, b in zip(hn, hd)]
    want = [(e["npairs"], int(e["digest"], 16)) for e in g["per_step"]]
    assert got == want, f"{name} {precision}: per-step collision counts or digests differ"
    st = sim.state()
    ids = torch.as_tensor(np.asarray(g["sample_ids"], dtype=np.int64), device=st.device)
    sample = st[:, ids].cpu().numpy()
    ref = np.array([[float.fromhex(v) for v in row] for row in g["sample_state"]]).T
    if _sha(st.cpu().numpy().astype("<f8")) != g["final_state_sha256"]:
        scale = np.maximum(np.abs(ref).max(axis=1, keepdims=True), 1e-300)
        rel = float((np.abs(sample - ref) / scale).max())
        raise AssertionError(f"{name} {precision}: final state differs from the oracle's "
                             f"(sampled max relative difference {rel:.3e})")
    assert np.array_equal(sample, ref)
    stats = sim.stats()
    sim.close()
    print(f"[run] ok: {sum(n for n, _ in got)} collisions over {len(got)} steps, "
          f"rechecks {stats['rechecks']}, fallbacks {stats['fallbacks']}", flush=True)


@pytest.mark.timeout(600)
def test_c2_shock_1e6_200_steps(kmc):
    g = _golden("c2_shock")
    w = _workload(g)
    _check_run(kmc, w, g, "fp32", use_graph=True)
    _check_run(kmc, w, g, "fp64")


@pytest.mark.timeout(600)
def test_c4_batch_256_boxes_50_steps(kmc):
    g = _golden("c4_batch")
    w = _workload(g)
    _check_run(kmc, w, g, "fp32", use_graph=True)
    _check_run(kmc, w, g, "fp64", search_mode=kmc.KMC_SEARCH_FULL)


@pytest.mark.timeout(900)
def test_c3_sphere_1e8_20_steps_graph_replay(kmc):
    g = _golden("c3_sphere")
    w = _workload(g)
    for precision in ("fp32", "fp64"):
        _check_run(kmc, w, g, precision, use_graph=True)


@pytest.mark.timeout(900)
def test_c5_blobs_1e7_3_steps(kmc):
    """The uneven gas (up to 1.7e3 particles per cell): the full search in
    both precisions (the FP32 screen in graph replay), and the half search,
    whose candidate lists overflow there (its whole-step FP64 search then
    decides the step)."""
    g = _golden("c5_blobs")
    w = _workload(g)
    _check_run(kmc, w, g, "fp32", search_mode=kmc.KMC_SEARCH_FULL, use_graph=True)
    _check_run(kmc, w, g, "fp64", search_mode=kmc.KMC_SEARCH_FULL)
    _check_run(kmc, w, g, "fp32")


def _sampled_every_step(kmc, w, steps, precision, **cfg):
    """Run `steps` steps; before each, read the state back (id order) and
    evaluate the oracle's step at sampled particles of it (random ones, ones
    in cells of more than 64 particles, and this step's colliders): their
    partners and post-step states must equal the GPU's, and the step's
    collision count must follow from the partner array."""
    import torch
    prec = kmc.KMC_FP64 if precision == "fp64" else kmc.KMC_FP32_SCREEN
    print(f"\n[sampled] {w.name} N={w.n} steps={steps} {precision} {cfg}", flush=True)
    sim = kmc.Sim(w.boxes, w.state, device="cuda:0", seed=w.seed, kinematics=w.kinematics, precision=prec,
                  history=max(64, steps), **cfg)
    box = w.boxes[0]
    n = w.n
    ids = np.arange(n, dtype=np.uint32)
    idx = np.arange(n)
    rng = np.random.default_rng(11)
    inv_h = np.array(box.inv_h)[:, None]
    lo = np.array(box.lo)[:, None]
    pre = sim.state().cpu().numpy()
    counts = []
    for s in range(steps):
        sim.step(1)
        p = sim.partners().cpu().numpy()
        has = p >= 0
        mutual = np.zeros(n, dtype=bool)
        mutual[has] = p[p[has]] == idx[has]
        counts.append(int((mutual & (idx < p)).sum()))
        cells = np.clip(np.floor((pre[0:3] - lo) * inv_h).astype(np.int64), 0, np.array(box.ncell)[:, None] - 1)
        lin = cells[0] + box.ncell[0] * (cells[1] + box.ncell[1] * cells[2])
        dense = np.flatnonzero(np.bincount(lin, minlength=box.ncells)[lin] > 64)
        col = np.flatnonzero(mutual)
        sel = np.unique(np.concatenate([rng.choice(n, 500, replace=False),
                                        rng.choice(dense, min(500, dense.size), replace=False),
                                        rng.choice(col, min(500, col.size), replace=False)])).astype(np.int64)
        ref_p, ref_s = O.step_sampled(box, pre, ids, s, sel, seed=w.seed, kinematics=w.kinematics)
        bad = np.flatnonzero(p[sel] != ref_p)
        assert bad.size == 0, f"step {s}: {bad.size} of {sel.size} sampled partners differ, first ids {sel[bad[:5]]}"
        st = sim.state()
        got = st[:, torch.as_tensor(sel, device=st.device)].cpu().numpy()
        assert np.array_equal(got, ref_s), f"step {s}: sampled post-step states differ"
        pre = st.cpu().numpy()
        if s % 10 == 9:
            print(f"[sampled] step {s + 1}: {sel.size} sampled particles identical", flush=True)
    hn, _ = sim.history()
    assert [int(a) for a in hn] == counts
    stats = sim.stats()
    sim.close()
    print(f"[sampled] ok: {sum(counts)} collisions over {steps} steps, fallbacks {stats['fallbacks']}", flush=True)


@pytest.mark.timeout(900)
def test_c5_blobs_1e7_50_steps_sampled(kmc):
    """The uneven gas over its full 50 steps (the whole-run record above
    holds 3: the oracle needs ten minutes per step there), checked every step
    at about 1500 sampled particles, FP32 screen in graph replay and FP64,
    with the full search the autotuner picks for it."""
    w = I.c5_blobs(steps=50)
    _sampled_every_step(kmc, w, 50, "fp32", search_mode=kmc.KMC_SEARCH_FULL, use_graph=True)
    _sampled_every_step(kmc, w, 50, "fp64", search_mode=kmc.KMC_SEARCH_FULL)


@pytest.mark.timeout(900)
def test_c3_sphere_1e8_200_steps_screen_equals_fp64(kmc):
    """Ten times the headline run's length (the infalling core keeps
    densifying, which widens the velocity spread the FP32 screen's bounds
    must cover): the screen's and plain FP64's per-step collision counts and
    digests, and their final FP64 states, are identical."""
    import torch
    w = I.c3_sphere(steps=200)
    out = {}
    for precision in ("fp32", "fp64"):
        prec = kmc.KMC_FP64 if precision == "fp64" else kmc.KMC_FP32_SCREEN
        print(f"\n[long] c3_sphere N={w.n} 200 steps {precision}", flush=True)
        sim = kmc.Sim(w.boxes, w.state, device="cuda:0", seed=w.seed, precision=prec, history=256, use_graph=True)
        for k in range(4):
            sim.step(50)
            torch.cuda.synchronize()
            print(f"[long] {precision}: {50 * (k + 1)} steps", flush=True)
        hn, hd = sim.history()
        st = sim.state().cpu().numpy()
        stats = sim.stats()
        sim.close()
        out[precision] = ([(int(a), int(b)) for a, b in zip(hn, hd)], _sha(st.astype("<f8")), stats)
        print(f"[long] {precision}: {sum(a for a, _ in out[precision][0])} collisions, rechecks "
              f"{stats['rechecks']}, fallbacks {stats['fallbacks']}", flush=True)
    assert len(out["fp32"][0]) == 200
    assert out["fp32"][0] == out["fp64"][0], "per-step counts or digests differ between the precisions"
    assert out["fp32"][1] == out["fp64"][1], "final states differ between the precisions"
