"""Write the oracle's record of whole runs of the benchmark workloads.

For each workload at its full size and step count this runs the CPU oracle
(`oracle/`, FP64, the definition of the step) from the seeded initial state of
`paper_1310_3437_amd.inputs` and stores, in tests/golden/full_<name>.json:

  * a fingerprint of the input (sha256 of the initial (6, N) float64 state in
    id order, N, the boxes' time steps and D2) so that a changed generator is
    detected before any comparison;
  * per step: the collision count, the digest (sum of the pair hashes of the
    colliding pairs mod 2^64), the ordered pair tests of the 27-cell search,
    and the sha256 of the partner array (int32 partner id per particle id,
    -1 for none, little endian) -- the collision-pair list of every step;
  * after the last step: the sha256 of the (6, N) float64 state in id order
    and the exact state (hex floats) of a fixed sample of particles, for
    diagnosis when the hash differs;
  * the oracle's wall time per step, its thread count and the CPU model
    (context only; these depend on the machine that ran the script).

Only the oracle and the input generators are used.  Run from the repository
root:  python tests/golden/make_full_runs.py [names ...] [--threads T]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1310_3437_amd import inputs as I  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

# workload -> (generator keyword arguments, steps); the sizes and step counts
# are those of the five benchmark configurations (c5_blobs: the oracle's
# search costs ~3e10 pair tests per step there, so fewer steps are recorded)
RUNS = {
    "c2_shock": (dict(n=1_000_000), 200),
    "c4_batch": (dict(nboxes=256), 50),
    "c3_sphere": (dict(n=100_000_000), 20),
    "c5_blobs": (dict(n=10_000_000), 3),
}
NSAMPLE = 512


def sha256_of(a):
    h = hashlib.sha256()
    a = np.ascontiguousarray(a)
    mv = memoryview(a).cast("B")
    step = 1 << 26
    for s in range(0, len(mv), step):
        h.update(mv[s:s + step])
    return h.hexdigest()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def input_fingerprint(w):
    return dict(n=int(w.n), nboxes=len(w.boxes), state_sha256=sha256_of(w.state),
                dt=[float(b.dt).hex() for b in w.boxes[:4]], D2=[float(b.D2).hex() for b in w.boxes[:4]],
                ncell=[list(map(int, b.ncell)) for b in w.boxes[:4]])


def record(name, threads):
    kw, steps = RUNS[name]
    t0 = time.time()
    w = I.CONFIGS[name](steps=steps, **kw)
    fp = input_fingerprint(w)
    print(f"[golden] {name}: N={w.n} boxes={len(w.boxes)} steps={steps} generated in {time.time() - t0:.1f} s",
          flush=True)
    run = O.Run(w, nthreads=threads)
    w.state = None   # the run holds its own copy
    per_step = []
    for s in range(steps):
        t1 = time.time()
        npairs, dig = run.step()
        dt_wall = time.time() - t1
        pb = run.partner_by_id.astype(np.int32)
        per_step.append(dict(step=s, npairs=int(npairs), digest=f"{dig:016x}", pair_tests=int(run.pair_tests),
                             partners_sha256=sha256_of(pb.astype("<i4")), seconds=round(dt_wall, 3)))
        print(f"[golden] {name} step {s}: pairs={npairs} tests={run.pair_tests} {dt_wall:.1f} s", flush=True)
    st = run.full_state()
    rng = np.random.default_rng(20261203)
    sample = np.unique(np.concatenate([rng.choice(st.shape[1], min(NSAMPLE, st.shape[1]), replace=False),
                                       [0, st.shape[1] - 1]])).astype(np.int64)
    out = dict(
        _about=("Oracle record of a whole run (tests/golden/make_full_runs.py): per-step collision count, "
                "digest, pair tests and sha256 of the int32 partner-id array; sha256 of the final (6, N) "
                "float64 state in id order and the exact final state of sampled ids."),
        workload=name, generator_kwargs=kw, steps=steps, seed=int(w.seed), kinematics=int(w.kinematics),
        input=fp, per_step=per_step,
        final_state_sha256=sha256_of(st.astype("<f8")),
        sample_ids=[int(i) for i in sample],
        sample_state=[[float(v).hex() for v in st[:, i]] for i in sample],
        oracle_context=dict(threads=int(threads if threads > 0 else O.lib().orc_max_threads()),
                            cpu=cpu_model(), seconds_total=round(sum(p["seconds"] for p in per_step), 1)),
    )
    path = os.path.join(HERE, f"full_{name}.json")
    with open(path + ".tmp", "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    os.replace(path + ".tmp", path)
    print(f"[golden] wrote {path}", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*", default=list(RUNS))
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    for name in a.names:
        record(name, a.threads)


if __name__ == "__main__":
    main()
