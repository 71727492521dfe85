"""Benchmark of the DCA collision step on one MI355X.

Workload (the headline configuration): N = 1e8 particles uniform in a ball
of radius 1 with radial infall v = -0.5 x + N(0, 0.1^2), reflecting sphere,
399^3 cells of edge ~D (about three particles per cell), seeded synthetic
input.  The plain FP64 path and the FP32-screen path each run W untimed and K
timed steps from the same initial state; their per-step pair counts and
digests must be identical.  `value` is the FP32-screen path's particle-steps/s
when that path is built, else the FP64 path's.

Per-phase times come from HIP events the library records on the launch
stream around every phase (profile mode).  The roofline object describes the
dominant kernel (the partner search).  `cpu_baseline` times the CPU oracle
(test infrastructure) on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n N] [--no-cpu]
                    [--workload c3_sphere|c2_shock|c4_batch|c5_blobs|c6_mixture] [--dt-rule adaptive]

The other workloads (shock tube, 256-box batch, Gaussian blobs) print the same
line for their own configuration; the headline is c3_sphere.
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
# Algorithmic floating-point operations of one pair evaluation (an FMA counts
# 2): r, g: 6 subtractions; b, g2: 2 x (1 mul + 2 fma) = 10; c = r x g:
# 3 x (1 mul + 1 fma) = 9; c2: 1 mul + 2 fma = 5; dt*g2, D2*g2: 2.  The pair
# quantities are symmetric, so one evaluation decides both orders of an
# unordered neighbour pair: the search kernel evaluates pair_tests / 2.
FLOP_PER_PAIR_EVAL = 32
PEAK_VALU_TFLOPS = 78.6     # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz (FP64, or unpacked FP32)
PEAK_HBM_GBS = 8000.0
# Algorithmic HBM bytes per particle-step of the FP64 step (bin 32, scan ~5,
# sorted copy 116, search 52, resolve/scatter/stream 110).
STEP_BYTES_PER_PARTICLE = 315


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


def run_path(kmc, w, precision, steps, warmup, pair_tests, search_mode=0):
    import torch
    name = "fp64" if precision == kmc.KMC_FP64 else "fp32_screen"
    log(f"[bench] {name}: init N={w.n}")
    kinds = None if w.species is None else (w.species, w.radius, w.mass)
    sim = kmc.Sim(w.boxes, w.state, device="cuda:0", seed=w.seed, precision=precision,
                  history=max(64, steps + warmup), profile=True, dt_rule=w.dt_rule,
                  dt_factor=w.dt_factor if w.dt_rule else 0.0, search_mode=search_mode, kinds=kinds)
    sim.step(warmup)
    torch.cuda.synchronize()
    s0 = sim.stats()
    if pair_tests is None:
        pair_tests = sim.pair_tests()
    log(f"[bench] {name}: warmup done, timing {steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    s1 = sim.stats()
    hn, hd = sim.history()
    ms_phase = {k: (s1["ms"][k] - s0["ms"][k]) / steps for k in s1["ms"]}
    search_kernel_ms = (s1["search_kernel_ms"] - s0["search_kernel_ms"]) / steps
    out = dict(
        value=w.n * steps / el,
        ms_per_step=1e3 * el / steps,
        ms_phase=ms_phase,
        search_kernel_ms=search_kernel_ms,
        rechecks_per_step=(s1["rechecks"] - s0["rechecks"]) / steps,
        fallbacks=s1["fallbacks"] - s0["fallbacks"],
        # pairs recorded per particle-step: FP64 the acceptable pairs, the
        # FP32 screen the pairs it could not reject (decided again in FP64)
        candidates_per_particle_step=(s1["candidates"] - s0["candidates"]) / (steps * w.n),
        history=[(int(a), int(b)) for a, b in zip(hn, hd)],
        pair_tests=pair_tests,
    )
    sim.close()
    del sim
    torch.cuda.empty_cache()
    log(f"[bench] {name}: {out['ms_per_step']:.3f} ms/step, search kernel {search_kernel_ms:.3f} ms")
    return out


def workload(name, n, dt_rule):
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


def cpu_baseline(name, n_sample):
    from oracle import oracle as O
    w, what = cpu_workload(name, n_sample)
    log(f"[bench] cpu baseline: oracle step on {what}")
    r = O.Run(w)
    n_sample = w.n
    nt = O.lib().orc_max_threads()
    t0 = time.perf_counter()
    r.step()
    el = time.perf_counter() - t0
    return dict(value=n_sample / el, unit="particle-steps/s", cores=int(nt), kind="oracle",
                sample=f"one oracle step (search with {nt} OpenMP threads, serial bin/resolve/stream) "
                       f"of {what}, {el:.1f} s; {r.pair_tests / el:.3e} pair-tests/s",
                pair_tests_per_s=r.pair_tests / el, seconds=el,
                cpu=platform.processor() or platform.machine())


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
    ap.add_argument("--search", default="half", choices=("half", "full"),
                    help="partner-search organisation (the result is the same)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sample", type=float, default=None)
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
    from paper_1310_3437_amd import inputs, kmc
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
    w, desc = workload(args.workload, int(n_arg) if n_arg else None, args.dt_rule)
    n = w.n
    log(f"[bench] generated {args.workload} N={n} in {time.perf_counter() - t0:.1f} s")

    results = {}
    pair_tests = None
    have_f32 = "fp32" in args.paths and os.environ.get("KMC_BENCH_NO_F32") is None
    for name in args.paths.split(","):
        prec = kmc.KMC_FP64 if name == "fp64" else kmc.KMC_FP32_SCREEN
        if name == "fp32" and not have_f32:
            continue
        r = run_path(kmc, w, prec, args.steps, args.warmup, pair_tests,
                     kmc.KMC_SEARCH_FULL if args.search == "full" else kmc.KMC_SEARCH_HALF)
        pair_tests = r["pair_tests"]
        results[name] = r

    identical = None
    if "fp64" in results and "fp32" in results:
        identical = results["fp64"]["history"] == results["fp32"]["history"]
    head = results.get("fp32") or results["fp64"]
    head_name = "fp32_screen" if "fp32" in results else "fp64"
    search_ms = head["search_kernel_ms"]
    # the half-neighbourhood search evaluates each unordered pair once, the
    # full one each ordered pair
    evals = head["pair_tests"] // 2 if args.search == "half" else head["pair_tests"]
    flops = FLOP_PER_PAIR_EVAL * evals
    achieved = flops / (search_ms * 1e-3) / 1e12
    headline = (args.workload == "c3_sphere" and n == 100_000_000 and args.dt_rule == "fixed"
                and args.search == "half")
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
        },
        "roofline": {
            "kernel": f"k_search_{args.search}<" + ("PolF32" if head_name == "fp32_screen" else "PolF64")
                      + ("<true>>" if w.species is not None else "<false>>")
                      + (" (FP32 screen)" if head_name == "fp32_screen" else " (FP64)"),
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_VALU_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_VALU_TFLOPS,
            "traffic": traffic,
            "flop_per_pair_eval": FLOP_PER_PAIR_EVAL,
            "pair_evals_per_launch": evals,
            "avg_launch_ms": search_ms,
        },
        "roofline_step": {
            "bound": "hbm",
            "achieved": STEP_BYTES_PER_PARTICLE * n / (head["ms_per_step"] * 1e-3) / 1e9,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": STEP_BYTES_PER_PARTICLE * n / (head["ms_per_step"] * 1e-3) / 1e9 / PEAK_HBM_GBS,
            "bytes_per_particle_step": STEP_BYTES_PER_PARTICLE,
        },
        "pair_tests_per_s": head["pair_tests"] * head["value"] / n,
        "identical_pair_lists": identical,
        "paths": {k: {kk: vv for kk, vv in v.items() if kk != "history"} for k, v in results.items()},
    }
    if "fp64" in results and "fp32" in results:
        line["fp32_over_fp64"] = results["fp32"]["value"] / results["fp64"]["value"]
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
        line["cpu_baseline"] = cpu_baseline(args.workload, int(cs) if cs else None)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
