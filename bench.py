"""Benchmark of the DCA collision step on one MI355X.

Workload (the headline configuration): N = 1e8 particles uniform in a ball
of radius 1 with radial infall v = -0.5 x + N(0, 0.1^2), reflecting sphere,
399^3 cells of edge ~D (about three particles per cell), seeded synthetic
input.  The plain FP64 path and the FP32-screen path each pick their launch
configuration with the autotuner on this input (search organisation, tile
shape, block size: the results do not depend on them), then run W untimed
and K timed steps from the same initial state, replayed from a captured
hipGraph as a caller would run them; `value` is the FP32-screen path's particle-steps/s
when that path is built, else the FP64 path's.  Their per-step pair counts
and digests must be identical to each other and, for the headline workload,
to the oracle's record of the same run (tests/golden/full_c3_sphere.json).

A second run of each path from the same initial state records HIP events on
the launch stream around every phase (profile mode, no graph): the per-phase
times and the search kernel's average launch time, from which the roofline
object of the dominant kernel (the partner search) is computed.
`cpu_baseline` times the CPU oracle (test infrastructure) on a bounded sample
of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n N] [--no-cpu]
                    [--workload c3_sphere|c2_shock|c4_batch|c5_blobs|c6_mixture] [--dt-rule adaptive]
                    [--search half|full] [--autotune none|launch|cells] [--adapt L,T|L,auto]
                    [--paths fp64,fp32,tuned] [--block B] [--tile 0|1|2] [--ppc-sweep]

`--paths ... tuned` adds a path whose precision, search organisation, tile
shape and block size the autotuner picks on the workload itself (both
precisions give the same partners); `tuned_over_best_fixed` compares it with
the faster fixed precision.

The other workloads (shock tube, 256-box batch, Gaussian blobs, mixture)
print the same line for their own configuration; the headline is c3_sphere.
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s at N=1e8 (FP32-screen vs plain FP64, identical pair lists)"
# Algorithmic floating-point operations of one ordered pair test (an FMA
# counts 2): r, g: 6 subtractions; b, g2: 2 x (1 mul + 2 fma) = 10;
# c = r x g: 3 x (1 mul + 1 fma) = 9; c2: 1 mul + 2 fma = 5; the thresholds
# dt*g2 and D2*g2: 2; the comparisons g2 > 0, b <= 0, -b <= dt g2,
# c2 < D2 g2 and the argmin: 5 -> 37.  A pair test is one ordered (i, j != i)
# pair of i's 27-cell neighbourhood, counted alike for both paths.
FLOP_PER_PAIR_TEST = 37
# Published vector peaks of MI355X: FP32 157.3 TFLOP/s (packed FP32), FP64
# and unpacked FP32 78.6 TFLOP/s (256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz).
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
# Algorithmic HBM bytes per particle-step of the whole FP64 step on the
# uniform grid (bin 28: slot and count, scan ~5, sorted copy 112, search 52,
# resolve/scatter/stream 110); the cell is recomputed, not stored.
STEP_BYTES_PER_PARTICLE = 307
# Algorithmic HBM bytes per particle of one search launch: read the sorted
# records once (FP64 48 B, FP32 screen 24 B) and write the result (4 B).
SEARCH_BYTES_PER_PARTICLE = {"fp64": 52, "fp32_screen": 28}
GOLDEN = os.path.join(ROOT, "tests", "golden", "full_{}.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("kmc_device.hip", "kmc_internal.h"):
        with open(os.path.join(ROOT, "paper_1310_3437_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(path_name, launches_bytes):
    """HBM traffic measured by rocprofv3 counters for the current kernel
    source, if a committed summary exists for it (else None)."""
    f = os.path.join(ROOT, "profiles", "search_traffic.json")
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        d = json.load(fh)
    if d.get("source_hash") != kernel_source_hash():
        return None
    e = d.get(path_name)
    return None if e is None else e.get("bytes_per_launch")


def _sim(kmc, w, precision, search_mode, block_size, steps, warmup, tile=0, **mode):
    kinds = None if w.species is None else (w.species, w.radius, w.mass)
    return kmc.Sim(w.boxes, w.state, device="cuda:0", seed=w.seed, precision=precision,
                   history=max(64, steps + warmup), dt_rule=w.dt_rule,
                   dt_factor=w.dt_factor if w.dt_rule else 0.0, search_mode=search_mode,
                   block_size=block_size, kinds=kinds, tile=tile, adapt_levels=w.adapt_levels,
                   adapt_threshold=w.adapt_threshold, **mode)


def run_path(kmc, w, precision, steps, warmup, search_mode=0, block_size=0, tile=0):
    """One path timed twice from the same initial state: (1) graph replay,
    the step as a caller runs it (value, ms/step, the per-step history);
    (2) profile mode, HIP events on the launch stream around every phase and
    around the search kernel alone, plus the pair tests of every step."""
    import torch
    name = "fp64" if precision == kmc.KMC_FP64 else "fp32_screen"
    log(f"[bench] {name}: init N={w.n} (graph replay)")
    sim = _sim(kmc, w, precision, search_mode, block_size, steps, warmup, tile, use_graph=True)
    sim.step(warmup)
    torch.cuda.synchronize()
    s0 = sim.stats()
    log(f"[bench] {name}: warmup done, timing {steps} steps")
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    s1 = sim.stats()
    hn, hd = sim.history()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    log(f"[bench] {name}: {1e3 * el / steps:.3f} ms/step (graph); profiling the phases")

    sim = _sim(kmc, w, precision, search_mode, block_size, steps, warmup, tile, profile=True)
    sim.step(warmup)
    torch.cuda.synchronize()
    p0 = sim.stats()
    tests = []
    for _ in range(steps):
        sim.step(1)
        tests.append(sim.pair_tests())   # a separate kernel between steps: outside every phase
    torch.cuda.synchronize()
    p1 = sim.stats()
    ph = sim.history()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    ms_phase = {k: (p1["ms"][k] - p0["ms"][k]) / steps for k in p1["ms"]}
    search_kernel_ms = (p1["search_kernel_ms"] - p0["search_kernel_ms"]) / steps
    out = dict(
        value=w.n * steps / el,
        ms_per_step=1e3 * el / steps,
        timing="hipGraph replay",
        ms_phase=ms_phase,
        ms_per_step_profiled=sum(ms_phase.values()),
        search_kernel_ms=search_kernel_ms,
        rechecks_per_step=(s1["rechecks"] - s0["rechecks"]) / steps,
        fallbacks=s1["fallbacks"] - s0["fallbacks"],
        # pairs recorded per particle-step: FP64 the acceptable pairs, the
        # FP32 screen the pairs it could not reject (decided again in FP64)
        candidates_per_particle_step=(s1["candidates"] - s0["candidates"]) / (steps * w.n),
        history=[(int(a), int(b)) for a, b in zip(hn, hd)],
        profiled_history_equal=[(int(a), int(b)) for a, b in zip(*ph)] == [(int(a), int(b)) for a, b in zip(hn, hd)],
        pair_tests=sum(tests) / len(tests),
    )
    log(f"[bench] {name}: search kernel {search_kernel_ms:.3f} ms, profiled step {out['ms_per_step_profiled']:.3f} ms")
    return out


def golden_check(name, n, results):
    """Compare each path's per-step (pair count, digest) with the oracle's
    record of the same run, where one exists for this workload and size."""
    f = GOLDEN.format(name)
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        g = json.load(fh)
    if g["input"]["n"] != n:
        return None
    want = [(int(e["npairs"]), int(e["digest"], 16)) for e in g["per_step"]]
    out = {"file": os.path.relpath(f, ROOT)}
    for k, r in results.items():
        m = min(len(want), len(r["history"]))
        out[k] = r["history"][:m] == want[:m]
        out["steps_compared"] = m
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def workload(name, n, dt_rule, adapt=None):
    from paper_1310_3437_amd import inputs
    if name == "c3_sphere":
        w = inputs.c3_sphere(n=n)
        b = w.boxes[0]
        desc = (f"c3_sphere: N={n:.0e} uniform ball R=1, v=-0.5x+N(0,0.1^2), reflecting sphere, "
                f"{b.ncell[0]}^3 cells (edge {b.h[0]:.5f} >= D={w.info['D']:.5f}), dt={b.dt:.4e}")
    elif name == "c2_shock":
        w = inputs.c2_shock(n=n)
        b = w.boxes[0]
        desc = (f"c2_shock: N={n:.0e} tube 1x0.1x0.1, reflecting walls, 8/9 of N left (sigma_v 1), "
                f"1/9 right (sigma_v 0.35), {b.ncell[0]}x{b.ncell[1]}x{b.ncell[2]} cells, dt={b.dt:.4e}")
    elif name == "c4_batch":
        w = inputs.c4_batch()
        desc = (f"c4_batch: {len(w.boxes)} periodic boxes, N_b log-uniform in [1e3, 1e5] "
                f"(total {w.n}), ~3 particles per cell, one launch per phase for all boxes")
    elif name == "c5_blobs":
        w = inputs.c5_blobs(n=n)
        b = w.boxes[0]
        desc = (f"c5_blobs: N={n:.0e} in 64 Gaussian blobs, periodic unit cube, D={w.info['D']:.2e}, "
                f"{b.ncell[0]}^3 cells, dt={b.dt:.4e}")
    elif name == "c6_mixture":
        w = inputs.c6_mixture(n=n)
        b = w.boxes[0]
        desc = (f"c6_mixture: N={n:.0e} three kinds (radius 1:2:3, mass 1:4:9, fractions 0.5/0.3/0.2), "
                f"periodic unit cube, Maxwellian at one temperature, {b.ncell[0]}^3 cells "
                f"(edge {b.h[0]:.5f} >= largest pair diameter {2 * max(w.radius):.5f}), dt={b.dt:.4e}")
    else:
        raise SystemExit(f"bench.py: unknown workload {name}")
    if dt_rule == "adaptive":
        import dataclasses
        w.boxes = [dataclasses.replace(b, dt=10.0 * b.dt) for b in w.boxes]
        w.dt_rule = 1
        desc += "; adaptive dt = dx / v_max (cap 10x the fixed dt)"
    if adapt:
        w.adapt_levels, w.adapt_threshold = adapt
        desc += (f"; density-adaptive bins: a cell is split (up to {adapt[0]} halvings) while it holds more "
                 f"than {adapt[1]} x 8^level particles")
    return w, desc


def cpu_workload(name, n_sample):
    from paper_1310_3437_amd import inputs
    if name == "c3_sphere":
        return inputs.c3_sphere(n=n_sample, steps=1), f"the c3_sphere recipe at N={n_sample:.0e} (same density law)"
    if name == "c2_shock":
        return inputs.c2_shock(n=n_sample, steps=1), f"the c2_shock recipe at N={n_sample:.0e}"
    if name == "c4_batch":
        return inputs.c4_batch(nboxes=64, steps=1), "the first 64 boxes of the c4_batch recipe"
    if name == "c6_mixture":
        return inputs.c6_mixture(n=n_sample, steps=1), f"the c6_mixture recipe at N={n_sample:.0e}"
    return inputs.c5_blobs(n=n_sample, steps=1), f"the c5_blobs recipe at N={n_sample:.0e} (same particles per cell)"


def cpu_baseline(name, n_sample, steps):
    from oracle import oracle as O
    w, what = cpu_workload(name, n_sample)
    log(f"[bench] cpu baseline: {steps} oracle steps on {what}")
    r = O.Run(w)
    nt = O.lib().orc_max_threads()
    tests = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        r.step()
        tests += r.pair_tests
    el = time.perf_counter() - t0
    out = dict(value=w.n * steps / el, unit="particle-steps/s", cores=int(nt), kind="oracle",
               sample=f"{steps} oracle steps (search with {nt} OpenMP threads, serial bin/resolve/stream) "
                      f"of {what}, {el:.1f} s; {tests / el:.3e} pair-tests/s",
               pair_tests_per_s=tests / el, seconds=el, cpu=cpu_model(), nproc=os.cpu_count())
    g = GOLDEN.format(name)
    if os.path.exists(g):
        with open(g) as fh:
            ctx = json.load(fh)["oracle_context"]
        # the whole-run record written with the oracle (its own machine)
        out["full_run_record"] = dict(ctx, file=os.path.relpath(g, ROOT))
    return out


def ppc_sweep(kmc, args):
    """Wall time per step and per unit of simulated time against particles
    per cell at N = 1e8 (the study of Section 2, Fig. 1, on one GPU)."""
    import torch
    from paper_1310_3437_amd import inputs
    n = int(args.n) if args.n else 100_000_000
    state = None
    rows = []
    for ppc in (3, 4, 6, 8, 12, 16, 24):
        w = inputs.ppc_sweep_case(n=n, ppc=ppc, state=state)
        state = w.state
        # with dt = dx / v_max every particle has ~10^2 acceptable partners
        # per step (mean free path far below the cell edge): the
        # full-neighbourhood search is the organisation for this regime
        for mode in ("full",):
            sm = kmc.KMC_SEARCH_FULL if mode == "full" else kmc.KMC_SEARCH_HALF
            log(f"[sweep] ppc {w.info['ppc']:.2f} cells {w.boxes[0].ncell[0]}^3 search {mode}")
            sim = kmc.Sim(w.boxes, w.state, device="cuda:0", seed=w.seed, precision=kmc.KMC_FP32_SCREEN,
                          dt_rule=1, dt_factor=1.0, search_mode=sm, history=64)
            sim.step(args.warmup)
            torch.cuda.synchronize()
            dt0, t0_sim = sim.time()
            t0 = time.perf_counter()
            sim.step(args.steps)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            dt1, t1_sim = sim.time()
            tests = sim.pair_tests()
            sim.close()
            del sim
            torch.cuda.empty_cache()
            ms = 1e3 * el / args.steps
            rows.append(dict(ppc=w.info["ppc"], cells=w.boxes[0].ncell[0], search=mode, ms_per_step=ms,
                             dt=float(dt1[0]), wall_s_per_unit_time=el / float(t1_sim[0] - t0_sim[0]),
                             pair_tests_per_step=tests))
            log(f"[sweep]   {ms:.2f} ms/step, dt {dt1[0]:.3e}, {rows[-1]['wall_s_per_unit_time']:.3f} s per unit time")
    print(json.dumps({"sweep": "ppc", "N": n, "precision": "fp32_screen", "steps": args.steps,
                      "workload": "periodic unit cube, one speed (1), random directions, D=(3/N)^(1/3), "
                                  "adaptive dt = dx/v_max", "rows": rows}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3_sphere")
    ap.add_argument("--n", type=float, default=None, help="particles (default: the workload's full size)")
    ap.add_argument("--dt-rule", default="fixed", choices=("fixed", "adaptive"))
    ap.add_argument("--search", default=None, choices=("half", "full"),
                    help="partner-search organisation (the result is the same; default half, or the "
                         "autotuner's choice)")
    ap.add_argument("--autotune", default=None, choices=("none", "launch", "cells"),
                    help="kmc_autotune before timing: launch (search organisation, block size; results "
                         "unchanged) or cells (also the cell edge, which changes the partner criteria); "
                         "default cells for c4_batch, launch for c3_sphere and c5_blobs, none otherwise, "
                         "and none whenever --search is given (it fixes the organisation)")
    ap.add_argument("--adapt", default=None,
                    help="density-adaptive bins L,T (at most L halvings of a cell, split while it holds more than "
                         "T 8^level particles; T = auto: chosen by the autotuner); changes the neighbourhoods, so "
                         "it is a variant of the workload")
    ap.add_argument("--block", type=int, default=0, help="threads per block of the streaming kernels (0: 256)")
    ap.add_argument("--tile", type=int, default=0, help="tile shape of the search kernel (0, 1, 2)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sample", type=float, default=None)
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--paths", default="fp64,fp32")
    ap.add_argument("--ppc-sweep", action="store_true",
                    help="wall time against particles per cell (Fig. 1 study) instead of the benchmark")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 2 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the collision step runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU slab decomposition is designed, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1310_3437_amd import kmc
    kmc.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    if args.ppc_sweep:
        ppc_sweep(kmc, args)
        return
    full = dict(c3_sphere=1e8, c2_shock=1e6, c4_batch=None, c5_blobs=1e7, c6_mixture=1e8)
    sample = dict(c3_sphere=1e7, c2_shock=1e6, c4_batch=None, c5_blobs=3e5, c6_mixture=1e7)
    if args.workload not in full:
        raise SystemExit(f"bench.py: unknown workload {args.workload}")
    n_arg = args.n if args.n is not None else full[args.workload]
    t0 = time.perf_counter()
    search_given = args.search is not None
    adapt, adapt_auto = None, False
    if args.adapt:
        lv, th = args.adapt.split(",")
        adapt_auto = th == "auto"
        adapt = (int(lv), 8 if adapt_auto else int(th))
        args.search = "full"
    w, desc = workload(args.workload, int(n_arg) if n_arg else None, args.dt_rule, adapt)
    n = w.n
    log(f"[bench] generated {args.workload} N={n} in {time.perf_counter() - t0:.1f} s")
    adapt_tuning = None
    if adapt_auto:
        # the autotuner picks the adaptive-bin threshold (a grid choice: it
        # changes the neighbourhoods), then every path runs with it
        kinds = None if w.species is None else (w.species, w.radius, w.mass)
        log("[bench] autotune of the adaptive-bin threshold")
        _, cfg, info = kmc.autotune(w.boxes, w.state, device="cuda:0", steps=3, kinds=kinds,
                                    flags=kmc.KMC_TUNE_LAUNCH | kmc.KMC_TUNE_PRECISION | kmc.KMC_TUNE_ADAPT,
                                    seed=w.seed, dt_rule=w.dt_rule, dt_factor=w.dt_factor if w.dt_rule else 0.0,
                                    search_mode=kmc.KMC_SEARCH_FULL, adapt_levels=w.adapt_levels,
                                    adapt_threshold=w.adapt_threshold)
        w.adapt_threshold = int(cfg["adapt_threshold"])
        best_by_t = {}
        for t in info["tried"]:
            if t["ms_per_step"] == t["ms_per_step"]:
                th = t["adapt_threshold"]
                best_by_t[th] = min(best_by_t.get(th, float("inf")), t["ms_per_step"])
        adapt_tuning = dict(threshold=w.adapt_threshold, best_ms_per_step_by_threshold=best_by_t,
                            candidates=len(info["tried"]))
        desc = desc.replace("than 8 x 8^level", f"than {w.adapt_threshold} x 8^level (threshold autotuned)")

    tune = args.autotune or ("none" if search_given else
                             dict(c3_sphere="launch", c4_batch="cells", c5_blobs="launch").get(args.workload, "none"))
    paths = [p for p in args.paths.split(",") if p in ("fp64", "fp32", "tuned")]
    if os.environ.get("KMC_BENCH_NO_F32") is not None:
        paths = [p for p in paths if p != "fp32"]
    results, tuned = {}, {}
    for name in paths:
        prec = kmc.KMC_FP64 if name == "fp64" else kmc.KMC_FP32_SCREEN
        search = kmc.KMC_SEARCH_FULL if args.search == "full" else kmc.KMC_SEARCH_HALF
        block, tile = args.block, args.tile
        wp = w
        if tune != "none" or name == "tuned":
            # "tuned": the autotuner also chooses the precision (both give the
            # same partners), so the path is never slower than its choice
            flags = kmc.KMC_TUNE_LAUNCH | (kmc.KMC_TUNE_CELLS if tune == "cells" else 0) | \
                (kmc.KMC_TUNE_PRECISION if name == "tuned" else 0)
            kinds = None if w.species is None else (w.species, w.radius, w.mass)
            log(f"[bench] {name}: autotune ({tune})")
            nb, cfg, info = kmc.autotune(w.boxes, w.state, device="cuda:0", flags=flags, steps=3, kinds=kinds,
                                         precision=prec, seed=w.seed, dt_rule=w.dt_rule,
                                         dt_factor=w.dt_factor if w.dt_rule else 0.0, search_mode=search,
                                         adapt_levels=w.adapt_levels, adapt_threshold=w.adapt_threshold)
            import dataclasses
            wp = dataclasses.replace(w, boxes=nb)
            search, block, tile = cfg["search_mode"], cfg["block_size"], cfg["tile"]
            prec = cfg["precision"]
            best = info["tried"][info["best"]]
            tuned[name] = dict(search_mode="full" if search == kmc.KMC_SEARCH_FULL else "half",
                               block_size=block, tile=tile, kappa=best["kappa"],
                               precision="fp32_screen" if prec == kmc.KMC_FP32_SCREEN else "fp64",
                               ms_per_step_tuning=best["ms_per_step"], candidates=len(info["tried"]))
        results[name] = run_path(kmc, wp, prec, args.steps, args.warmup, search, block, tile)
        results[name]["search"] = "full" if search == kmc.KMC_SEARCH_FULL else "half"

    same_grid = len({json.dumps(t.get("kappa")) for t in tuned.values()}) <= 1
    identical = None
    if "fp64" in results and "fp32" in results and same_grid:
        identical = results["fp64"]["history"] == results["fp32"]["history"]
        if "tuned" in results:
            identical = identical and results["tuned"]["history"] == results["fp64"]["history"]
    golden = golden_check(args.workload, n, results) if (args.dt_rule == "fixed" and tune != "cells"
                                                          and not adapt) else None
    if golden is not None and identical is not None:
        identical = identical and all(golden[k] for k in results)
    head_key = "fp32" if "fp32" in results else ("fp64" if "fp64" in results else "tuned")
    head = results[head_key]
    head_name = "fp32_screen" if head_key == "fp32" else "fp64"
    if head_key == "tuned":
        head_name = tuned["tuned"]["precision"]
    search_ms = head["search_kernel_ms"]
    tests = head["pair_tests"]
    achieved = FLOP_PER_PAIR_TEST * tests / (search_ms * 1e-3) / 1e12
    peak = PEAK_FP32_TFLOPS if head_name == "fp32_screen" else PEAK_FP64_TFLOPS
    # the half-neighbourhood search evaluates each unordered pair once
    evals = tests / 2 if head["search"] == "half" else tests
    executed = FLOP_PER_PAIR_TEST * evals / (search_ms * 1e-3) / 1e12
    sbytes = SEARCH_BYTES_PER_PARTICLE[head_name] * n
    headline = (args.workload == "c3_sphere" and n == 100_000_000 and args.dt_rule == "fixed"
                and head["search"] == "half")
    traffic = traffic_for(head_name, None) if headline else None
    metric = METRIC if args.workload == "c3_sphere" and n == 100_000_000 else \
        f"particle-steps/s on {args.workload} (FP32-screen vs plain FP64, identical pair lists)"
    line = {
        "metric": metric,
        "value": head["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head_name == "fp32_screen" else "f64",
        "data": "synthetic",
        "config": {
            "workload": desc,
            "N": n,
            "path": head_name,
            "search": head["search"],
            "timing": "hipGraph replay",
        },
        "roofline": {
            "kernel": ("k_search_full + k_search_adapt<" if adapt else f"k_search_{head['search']}<")
                      + ("PolF32" if head_name == "fp32_screen" else "PolF64")
                      + ("<true>>" if w.species is not None else "<false>>")
                      + (" (FP32 screen)" if head_name == "fp32_screen" else " (FP64)"),
            "bound": "alu",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": traffic,
            "flop_per_pair_test": FLOP_PER_PAIR_TEST,
            "pair_tests_per_launch": tests,
            "avg_launch_ms": search_ms,
            # the same flops per evaluation the kernel executes (each unordered
            # pair once in the half search), against the FP64 / unpacked-FP32
            # rate that code without packed FP32 can reach
            "executed": {"pair_evals_per_launch": evals, "achieved": executed, "peak": PEAK_FP64_TFLOPS,
                         "frac": executed / PEAK_FP64_TFLOPS},
            # algorithmic bytes of the search (read the sorted records once,
            # write the result) per launch time, against HBM peak
            "hbm_algorithmic": {"bytes_per_particle": SEARCH_BYTES_PER_PARTICLE[head_name],
                                "achieved_GBs": sbytes / (search_ms * 1e-3) / 1e9,
                                "frac": sbytes / (search_ms * 1e-3) / 1e9 / PEAK_HBM_GBS},
        },
        "roofline_step": {
            "bound": "hbm",
            "achieved": STEP_BYTES_PER_PARTICLE * n / (head["ms_per_step"] * 1e-3) / 1e9,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": STEP_BYTES_PER_PARTICLE * n / (head["ms_per_step"] * 1e-3) / 1e9 / PEAK_HBM_GBS,
            "bytes_per_particle_step": STEP_BYTES_PER_PARTICLE,
        },
        "pair_tests_per_s": tests * head["value"] / n,
        "identical_pair_lists": identical,
        "oracle_record_match": golden,
        "paths": {k: {kk: vv for kk, vv in v.items() if kk != "history"} for k, v in results.items()},
    }
    if tuned:
        line["autotuned"] = tuned
    if "fp64" in results and "fp32" in results:
        line["fp32_over_fp64"] = results["fp32"]["value"] / results["fp64"]["value"]
    if adapt_tuning is not None:
        line["adapt_autotuned"] = adapt_tuning
    if "tuned" in results:
        fixed = [results[k]["value"] for k in ("fp64", "fp32") if k in results]
        if fixed:
            line["tuned_over_best_fixed"] = results["tuned"]["value"] / max(fixed)
    if args.copy_calibration:
        # an elementwise kernel that reads and writes 2 GiB each
        src = torch.ones(1 << 29, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = 1 << 31
        del src, dst
    if not args.no_cpu:
        cs = args.cpu_sample if args.cpu_sample is not None else sample[args.workload]
        line["cpu_baseline"] = cpu_baseline(args.workload, int(cs) if cs else None, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
