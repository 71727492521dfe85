"""CPU checks of the C-ABI library: it loads, exports every function that
include/kmc.h declares, and its host-side validation (kmc_workspace_bytes,
which touches no device) rejects invalid boxes and configurations."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1310_3437_amd import inputs as I
from paper_1310_3437_amd import kmc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "kmc.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(kmc_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_function():
    L = kmc.load()
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(kmc.EXPORTS)
    assert L.kmc_abi_version() == kmc.KMC_ABI_VERSION == 5


def test_one_hip_runtime_whatever_the_import_order():
    """kmc.load() before torch: the process must still hold one HIP runtime
    (torch ships its own copy; two would make torch's device pointers
    invalid in the library)."""
    import subprocess
    import sys
    code = ("from paper_1310_3437_amd import kmc; kmc.load(); import torch; "
            "maps = open('/proc/self/maps').read().split(chr(10)); "
            "print(sorted({l.split()[-1] for l in maps if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    libs = eval(out.stdout.strip().splitlines()[-1])
    assert len(libs) == 1, libs


def test_struct_sizes_match_header():
    # kmc_box: 32 bytes of ints, 12 doubles; kmc_config: 80 bytes, the
    # species pointer and the two adaptive-bin words; kmc_species: two u32,
    # 2 x 8 doubles, a pointer
    assert C.sizeof(kmc.KmcBox) == 128
    assert C.sizeof(kmc.KmcConfig) == 96
    assert C.sizeof(kmc.KmcStats) == 136
    assert C.sizeof(kmc.KmcSpecies) == 144
    # kmc_tuning: two u32, then per candidate (64) ms, mode, block, kappa,
    # precision, tile, adaptive threshold
    assert C.sizeof(kmc.KmcTuning) == 8 + 64 * (8 + 4 + 4 + 8 + 4 + 4 + 4)


def test_autotune_rejects_bad_flags_before_touching_the_device():
    """Unknown flags, and the adaptive-threshold flag without adaptive
    bins, are refused by the host-side checks."""
    L = kmc.load()
    boxes = [_good()]
    arr = kmc.make_boxes(boxes)
    out_b = (kmc.KmcBox * 1)()
    out_c = kmc.KmcConfig()
    tun = kmc.KmcTuning()
    fake = C.c_void_p(1 << 20)
    for flags, cfg in ((16, {}), (kmc.KMC_TUNE_ADAPT, {}),
                       (kmc.KMC_TUNE_ADAPT | kmc.KMC_TUNE_LAUNCH, dict(precision=kmc.KMC_FP32_SCREEN))):
        c = kmc.make_config(**cfg)
        rc = L.kmc_autotune(arr, 1, C.byref(c), fake, fake, C.c_size_t(1 << 20), flags, 2, None, out_b,
                            C.byref(out_c), C.byref(tun))
        assert rc == kmc.KMC_EINVAL, (flags, rc)


def _ws(boxes, **cfg):
    arr = kmc.make_boxes(boxes)
    c = kmc.make_config(**cfg)
    n = C.c_size_t(0)
    return kmc.load().kmc_workspace_bytes(arr, len(boxes), C.byref(c), C.byref(n)), n.value


def test_workspace_size_scales_with_particles_and_cells():
    w = I.c1_small()
    rc, n1 = _ws(w.boxes)
    assert rc == 0 and n1 > 4096 * 100
    rc, n2 = _ws(w.boxes, precision=kmc.KMC_FP32_SCREEN)
    assert rc == 0 and n2 >= n1
    big = I.Box(n=10_000_000, lo=(0, 0, 0), hi=(1, 1, 1), ncell=(300, 300, 300),
                periodic=(True,) * 3, D2=1e-6, dt=1e-3)
    rc, n3 = _ws([big])
    assert rc == 0 and n3 >= 10_000_000 * 116 + 27_000_000 * 8


def _good():
    return I.Box(n=100, lo=(0, 0, 0), hi=(1, 1, 1), ncell=(4, 4, 4), periodic=(True,) * 3,
                 D2=0.2 ** 2, dt=0.01)


@pytest.mark.parametrize("mutate", [
    lambda b: setattr(b, "D2", 0.0),
    lambda b: setattr(b, "dt", -1.0),
    lambda b: setattr(b, "dt", float("nan")),
    lambda b: setattr(b, "ncell", (2, 4, 4)),          # periodic axis with < 3 cells
    lambda b: setattr(b, "ncell", (0, 4, 4)),
    lambda b: setattr(b, "hi", (-0.5, 1, 1)),          # negative extent
    lambda b: setattr(b, "D2", 0.3 ** 2),              # cell edge 0.25 < D
    lambda b: (setattr(b, "sphere", True), setattr(b, "R", 0.5)),   # sphere with periodic axes
    lambda b: (setattr(b, "periodic", (False,) * 3), setattr(b, "absorb", (True, False, False)),
               setattr(b, "sphere", True), setattr(b, "R", 0.5)),   # absorbing faces need a box
])
def test_invalid_boxes_rejected(mutate):
    b = _good()
    assert _ws([b])[0] == 0
    mutate(b)
    assert _ws([b])[0] == kmc.KMC_EINVAL


@pytest.mark.parametrize("scale", [0.5, 1.0 - 1e-9, 1.0 + 1e-9, 2.0])
def test_inv_h_must_match_the_grid(scale):
    """inv_h is the caller's, but it must be ncell / (hi - lo) up to
    rounding on every axis: binning with another value would make bins of a
    width the FP32 screen's error bounds do not describe."""
    arr = kmc.make_boxes([_good()])
    c = kmc.make_config(precision=kmc.KMC_FP32_SCREEN)
    n = C.c_size_t(0)
    L = kmc.load()
    assert L.kmc_workspace_bytes(arr, 1, C.byref(c), C.byref(n)) == 0
    for k in range(3):
        arr = kmc.make_boxes([_good()])
        arr[0].inv_h[k] = arr[0].inv_h[k] * scale
        assert L.kmc_workspace_bytes(arr, 1, C.byref(c), C.byref(n)) == kmc.KMC_EINVAL
    # one rounding of ncell / (hi - lo) away is accepted
    arr = kmc.make_boxes([_good()])
    arr[0].inv_h[0] = float(np.nextafter(arr[0].inv_h[0], np.inf))
    assert L.kmc_workspace_bytes(arr, 1, C.byref(c), C.byref(n)) == 0


@pytest.mark.parametrize("cfg", [
    dict(precision=7), dict(kinematics=3), dict(block_size=100), dict(block_size=2048),
    dict(dt_rule=2), dict(dt_rule=1, dt_factor=-1.0), dict(dt_rule=1, dt_factor=float("inf")),
    dict(search_mode=2), dict(search_mode=-1), dict(dims=1), dict(dims=4), dict(tile=3), dict(tile=-1),
    dict(adapt_levels=4, adapt_threshold=8, search_mode=1), dict(adapt_levels=-1),
    dict(adapt_levels=2, adapt_threshold=0, search_mode=1),          # threshold must be >= 1
    dict(adapt_levels=2, adapt_threshold=8, search_mode=0),          # needs the full search
])
def test_invalid_configs_rejected(cfg):
    assert _ws([_good()], **cfg)[0] == kmc.KMC_EINVAL


def test_reserved_config_words_must_be_zero():
    arr = kmc.make_boxes([_good()])
    c = kmc.make_config()
    c.reserved = 1
    n = C.c_size_t(0)
    assert kmc.load().kmc_workspace_bytes(arr, 1, C.byref(c), C.byref(n)) == kmc.KMC_EINVAL


def test_too_many_particles_overflow():
    b = _good()
    b.n = 2 ** 32 - 1
    bb = _good()
    assert _ws([b, bb])[0] == kmc.KMC_EOVERFLOW


def test_null_arguments():
    L = kmc.load()
    c = kmc.make_config()
    n = C.c_size_t(0)
    assert L.kmc_workspace_bytes(None, 1, C.byref(c), C.byref(n)) == kmc.KMC_EINVAL
    assert L.kmc_workspace_bytes(kmc.make_boxes([_good()]), 0, C.byref(c), C.byref(n)) == kmc.KMC_EINVAL
    assert L.kmc_strerror(-1) == b"invalid argument"
    L.kmc_destroy(None)


def test_box_with_kappa_grid():
    """The cell grid of the autotuner's cell-edge candidates (host helper)."""
    b = I.Box(n=10, lo=(0, 0, -1), hi=(1, 2, 1), ncell=(10, 20, 20), periodic=(True, True, False),
              D2=0.09 ** 2, dt=0.01)
    for kappa, want in [(1.0, (11, 22, 22)), (1.25, (8, 17, 17)), (2.0, (5, 11, 11))]:
        nb = kmc.box_with_kappa(b, kappa)
        assert nb.ncell == want
        assert all(nb.h[k] >= kappa * 0.09 for k in range(3))
        assert nb.n == b.n and nb.lo == b.lo and nb.D2 == b.D2
    with pytest.raises(kmc.KmcError):
        kmc.box_with_kappa(b, 0.5)
    small = I.Box(n=10, lo=(0, 0, 0), hi=(0.25, 1, 1), ncell=(3, 3, 3), periodic=(True,) * 3, D2=0.08 ** 2, dt=0.1)
    kmc.box_with_kappa(small, 1.0)              # 3 cells: allowed
    with pytest.raises(kmc.KmcError):
        kmc.box_with_kappa(small, 1.25)         # 2 cells on a periodic axis


def test_planar_mode_needs_one_reflecting_z_layer():
    w = I.c1_planar()
    assert _ws(w.boxes, dims=2)[0] == 0
    b = I.c1_small().boxes[0]                   # 30 cells along z
    assert _ws([b], dims=2)[0] == kmc.KMC_EINVAL
    import dataclasses
    per = dataclasses.replace(w.boxes[0], periodic=(True, True, True), ncell=(50, 50, 3))
    assert _ws([per], dims=2)[0] == kmc.KMC_EINVAL


def test_absorbing_faces_accepted_and_one_extra_cell_per_box():
    b = _good()
    b.periodic = (False, True, True)
    b.absorb = (True, False, False)
    rc, n1 = _ws([b])
    assert rc == 0


def _species(count=2, radius=(0.05, 0.1), mass=(1.0, 2.0), reserved=0):
    sp = kmc.KmcSpecies()
    sp.count = count
    sp.reserved = reserved
    for k in range(len(radius)):
        sp.radius[k] = radius[k]
    for k in range(len(mass)):
        sp.mass[k] = mass[k]
    return sp


def test_species_workspace_and_validation():
    rc, n0 = _ws([_good()])
    rc, n1 = _ws([_good()], species=_species())
    assert rc == 0 and n1 >= n0 + 2 * 100     # two kind arrays of one byte per particle
    for bad in [_species(count=0), _species(count=9), _species(reserved=1),
                _species(radius=(0.05, 0.0)), _species(radius=(0.05, float("nan"))),
                _species(mass=(1.0, -2.0)), _species(mass=(float("inf"), 1.0)),
                _species(radius=(0.05, 0.13))]:          # largest pair 0.26 > cell edge 0.25
        assert _ws([_good()], species=bad)[0] == kmc.KMC_EINVAL
    # the box's own D2 is still validated, the pair table decides the cell check
    assert _ws([_good()], species=_species(radius=(0.05, 0.125)))[0] == 0


def test_scratch_entry_point_rejects_oversized_boxes_before_any_device_work():
    """kmc_init_scratch sizes the boxes against KMC_SCRATCH_BYTES first: too
    large a workspace returns KMC_ENOMEM (no device is touched), invalid
    boxes KMC_EINVAL."""
    L = kmc.load()
    big = I.Box(n=1_000_000, lo=(0, 0, 0), hi=(1, 1, 1), ncell=(100, 100, 100), periodic=(True,) * 3,
                D2=1e-4, dt=1e-3)
    assert _ws([big])[1] > kmc.KMC_SCRATCH_BYTES
    ctx = C.c_void_p(0)
    cfg = kmc.make_config()
    assert L.kmc_init_scratch(kmc.make_boxes([big]), 1, C.byref(cfg), None, None, C.byref(ctx)) == kmc.KMC_ENOMEM
    bad = _good()
    bad.D2 = 0.0
    assert L.kmc_init_scratch(kmc.make_boxes([bad]), 1, C.byref(cfg), None, None, C.byref(ctx)) == kmc.KMC_EINVAL
    assert L.kmc_init_scratch(kmc.make_boxes([_good()]), 1, C.byref(cfg), None, None, None) == kmc.KMC_EINVAL
    assert not ctx.value


def test_adaptive_bins_validation():
    """Adaptive bins need the full search, three dimensions, no absorbing
    faces and at most 2^27 cells per axis."""
    ok = dict(adapt_levels=3, adapt_threshold=8, search_mode=kmc.KMC_SEARCH_FULL)
    assert _ws([_good()], **ok)[0] == 0
    b = _good()
    b.periodic = (False, True, True)
    b.absorb = (True, False, False)
    assert _ws([b], **ok)[0] == kmc.KMC_EINVAL
    w = I.c1_planar()
    assert _ws(w.boxes, dims=2, **ok)[0] == kmc.KMC_EINVAL
    # the leaf tables: 8 N / T + N + 1 entries of 4 bytes, and per cell a
    # level, a flag, a table offset and a list slot
    n0 = _ws([_good()], search_mode=kmc.KMC_SEARCH_FULL)[1]
    n1 = _ws([_good()], **ok)[1]
    assert n1 >= n0 + 4 * (8 * 100 // 8 + 100 + 1) + 4 * 100 + 10 * 64
