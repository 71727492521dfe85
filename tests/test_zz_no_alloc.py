"""kmc_init_scratch (the entry point for callers that cannot allocate device
memory) against kmc_init with a caller-owned workspace: the same partners
every step, the same per-step collision counts and digests and the same
state bit for bit, on two calls in a row (the second with fewer particles,
so the scratch array still holds the first call's data)."""
import ctypes as C

import numpy as np
import pytest

from paper_1310_3437_amd import inputs as I

pytestmark = pytest.mark.gpu


def _run(kmc, w, steps, scratch, **cfg):
    sim = kmc.Sim(w.boxes, w.state, device="cuda:0", seed=w.seed, scratch=scratch, **cfg)
    parts = []
    for _ in range(steps):
        sim.step(1)
        parts.append(sim.partners().cpu().numpy())
    hn, hd = sim.history()
    st = sim.state().cpu().numpy()
    sim.close()
    return parts, [(int(a), int(b)) for a, b in zip(hn, hd)], st


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_scratch_context_equals_workspace_context(kmc, precision):
    prec = kmc.KMC_FP64 if precision == "fp64" else kmc.KMC_FP32_SCREEN
    first = I.c1_small(n=20_000, steps=6)
    second = I.c4_batch(nboxes=3, n_lo=1000, n_hi=3000, steps=6)
    assert second.n < first.n
    for w in (first, second):
        print(f"\n[scratch] {w.name} N={w.n} boxes={len(w.boxes)} {precision}", flush=True)
        ref = _run(kmc, w, w.steps, False, precision=prec)
        got = _run(kmc, w, w.steps, True, precision=prec)
        for s in range(w.steps):
            assert np.array_equal(got[0][s], ref[0][s]), f"{w.name}: partners differ at step {s}"
        assert got[1] == ref[1], f"{w.name}: per-step counts or digests differ"
        assert sum(n for n, _ in ref[1]) > 0
        assert np.array_equal(got[2], ref[2]), f"{w.name}: states differ"


def test_scratch_rejects_boxes_beyond_its_size(kmc):
    big = I.Box(n=1_000_000, lo=(0, 0, 0), hi=(1, 1, 1), ncell=(100, 100, 100), periodic=(True,) * 3,
                D2=1e-4, dt=1e-3)
    assert kmc.workspace_bytes([big], kmc.make_config()) > kmc.KMC_SCRATCH_BYTES
    st = np.zeros((6, big.n))
    with pytest.raises(kmc.KmcError, match="kmc_init_scratch"):
        kmc.Sim([big], st, device="cuda:0", scratch=True)
    ctx = C.c_void_p(0)
    rc = kmc.load().kmc_init_scratch(kmc.make_boxes([big]), 1, C.byref(kmc.make_config()), C.c_void_p(0),
                                     C.c_void_p(0), C.byref(ctx))
    assert rc == kmc.KMC_ENOMEM and not ctx.value
