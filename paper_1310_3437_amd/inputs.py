"""Seeded synthetic workloads for the DCA collision step.

This module only *generates inputs*: initial positions and velocities and the
scalar parameters (bin grid, interaction diameter, time step) that both the
GPU library and the CPU oracle receive bit-identically.  It contains none of
the collision step's arithmetic.

The paper's own test gases have random positions and random velocity
directions (Section 2, Fig. 1 caption; Section 3, Fig. 3 caption); the
workloads below follow that recipe and the five configurations of the
benchmark plan:

  c1_small   N=4096 periodic unit cube, Maxwellian sigma_v=1, mean free path 0.05
  c2_shock   1-D shock tube 1 x 0.1 x 0.1, reflecting walls, 8:1 density jump
  c3_sphere  uniform ball of radius 1 with radial infall, reflecting sphere
  c4_batch   256 independent periodic boxes of log-uniform size
  c5_blobs   64 Gaussian blobs in a periodic unit cube (uneven occupancy)

Conventions where a configuration leaves a parameter open:
  * bins: the first cell edge >= the interaction diameter D on every axis,
    i.e. ncell_k = floor(L_k / D) (the paper sets the bin width as the
    characteristic length, Section 1);
  * interaction diameter from density where no mean free path is given:
    D = (3 / n)^(1/3), i.e. about three particles per bin, the optimum of the
    paper's bins-per-particle study (Section 2);
  * time step: 0.2 bin widths of mean displacement, dt = 0.2 h / <|v|>.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MEAN_SPEED_PER_SIGMA = math.sqrt(8.0 / math.pi)   # <|v|> of a Maxwellian per sigma_v


@dataclass
class Box:
    """One independent simulation box (bin grid, boundaries, physics scalars)."""
    n: int
    lo: tuple
    hi: tuple
    ncell: tuple
    periodic: tuple = (False, False, False)
    sphere: bool = False
    absorb: tuple = (False, False, False)   # absorbing faces per axis (not periodic)
    R: float = 0.0
    D2: float = 0.0
    dt: float = 0.0

    @property
    def inv_h(self):
        return tuple(float(self.ncell[k]) / (float(self.hi[k]) - float(self.lo[k])) for k in range(3))

    @property
    def h(self):
        return tuple((float(self.hi[k]) - float(self.lo[k])) / float(self.ncell[k]) for k in range(3))

    @property
    def ncells(self):
        return int(self.ncell[0]) * int(self.ncell[1]) * int(self.ncell[2])


@dataclass
class Workload:
    name: str
    boxes: list
    state: np.ndarray            # (6, N) float64: x, y, z, vx, vy, vz; boxes concatenated
    steps: int
    seed: int = 1
    kinematics: int = 0          # 0: scatter at t*, 1: velocity-only
    dt_rule: int = 0             # 0: fixed dt per box, 1: adaptive (box dt is the cap)
    dt_factor: float = 1.0       # adaptive rule: factor C in dt = C dx / v_max
    dims: int = 3                # 2: planar mode (one cell along z, z and vz fixed)
    species: np.ndarray = None   # (N,) uint8 kind of each particle (id order), None: one kind
    radius: tuple = ()           # per kind: effective radius (a pair interacts below the sum)
    mass: tuple = ()             # per kind: mass
    adapt_levels: int = 0        # density-adaptive bins: at most this many halvings of a bin (0: uniform)
    adapt_threshold: int = 0     # ... a bin is split while it holds more than threshold * 8^level particles
    info: dict = field(default_factory=dict)

    @property
    def n(self):
        return int(self.state.shape[1])

    @property
    def offsets(self):
        off = [0]
        for b in self.boxes:
            off.append(off[-1] + int(b.n))
        return off


def _ncell_for(L, D):
    return max(1, int(math.floor(L / D)))


def _mean_speed(v):
    """Sample mean of |v| over a (3, n) velocity array, computed in chunks."""
    n = v.shape[1]
    tot = 0.0
    step = 1 << 22
    for s in range(0, n, step):
        c = v[:, s:s + step]
        tot += float(np.sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]).sum())
    return tot / max(n, 1)


def uniform_box(n, L=1.0, D=None, sigma_v=1.0, periodic=True, ic_seed=1, ncell=None,
                dt=None, same_speed=False):
    """n particles uniform in [0, L)^3 with Maxwellian (or fixed-speed,
    random-direction) velocities; periodic or reflecting walls."""
    rng = np.random.default_rng(ic_seed)
    s = np.empty((6, n), dtype=np.float64)
    s[0:3] = rng.random((3, n)) * L
    if same_speed:
        d = rng.standard_normal((3, n))
        d /= np.sqrt((d * d).sum(axis=0))
        s[3:6] = d * sigma_v
        mean_speed = sigma_v
    else:
        s[3:6] = rng.standard_normal((3, n)) * sigma_v
        mean_speed = MEAN_SPEED_PER_SIGMA * sigma_v
    if D is None:
        D = (3.0 / (n / L ** 3)) ** (1.0 / 3.0)
    nc = ncell if ncell is not None else _ncell_for(L, D)
    h = L / nc
    if dt is None:
        dt = 0.2 * h / mean_speed
    box = Box(n=n, lo=(0.0, 0.0, 0.0), hi=(L, L, L), ncell=(nc, nc, nc),
              periodic=(periodic,) * 3, D2=D * D, dt=dt)
    return box, s


def c1_small(n=4096, mfp=0.05, ic_seed=1, steps=10, seed=1):
    """Periodic unit cube, Maxwellian sigma_v = 1, sigma from the mean free
    path lambda = 1 / (sqrt(2) n sigma); cell edge = first h >= D."""
    dens = n / 1.0
    sigma = 1.0 / (math.sqrt(2.0) * dens * mfp)
    D = math.sqrt(sigma / math.pi)
    nc = _ncell_for(1.0, D)
    h = 1.0 / nc
    dt = 0.2 * h / MEAN_SPEED_PER_SIGMA
    box, s = uniform_box(n, 1.0, D=D, sigma_v=1.0, periodic=True, ic_seed=ic_seed, ncell=nc, dt=dt)
    return Workload("c1_small", [box], s, steps, seed,
                    info=dict(sigma=sigma, D=D, h=h, mfp=mfp))


def c2_shock(n=1_000_000, mfp_left=0.002, ic_seed=2, steps=200, seed=1):
    """Shock tube 1 x 0.1 x 0.1 with reflecting walls: the left half holds 8/9
    of the particles (Maxwellian sigma_v = 1), the right half 1/9 (sigma_v =
    0.35); sigma from the left mean free path."""
    Lx, Ly, Lz = 1.0, 0.1, 0.1
    rng = np.random.default_rng(ic_seed)
    nl = int(round(n * 8.0 / 9.0))
    nr = n - nl
    s = np.empty((6, n), dtype=np.float64)
    s[0, :nl] = rng.random(nl) * (0.5 * Lx)
    s[0, nl:] = 0.5 * Lx + rng.random(nr) * (0.5 * Lx)
    s[1] = rng.random(n) * Ly
    s[2] = rng.random(n) * Lz
    s[3:6, :nl] = rng.standard_normal((3, nl)) * 1.0
    s[3:6, nl:] = rng.standard_normal((3, nr)) * 0.35
    dens_l = nl / (0.5 * Lx * Ly * Lz)
    sigma = 1.0 / (math.sqrt(2.0) * dens_l * mfp_left)
    D = math.sqrt(sigma / math.pi)
    nc = (_ncell_for(Lx, D), _ncell_for(Ly, D), _ncell_for(Lz, D))
    h = min(Lx / nc[0], Ly / nc[1], Lz / nc[2])
    mean_speed = MEAN_SPEED_PER_SIGMA * (nl * 1.0 + nr * 0.35) / n
    dt = 0.2 * h / mean_speed
    box = Box(n=n, lo=(0.0, 0.0, 0.0), hi=(Lx, Ly, Lz), ncell=nc,
              periodic=(False, False, False), D2=D * D, dt=dt)
    return Workload("c2_shock", [box], s, steps, seed,
                    info=dict(sigma=sigma, D=D, h=h, n_left=nl, n_right=nr))


def c3_sphere(n=100_000_000, R=1.0, infall=0.5, sigma_v=0.1, ic_seed=3, steps=20, seed=1):
    """Uniform ball of radius R with v = -infall * x + N(0, sigma_v^2),
    reflecting sphere; D = (3/n)^(1/3) (about three particles per bin)."""
    rng = np.random.default_rng(ic_seed)
    s = np.empty((6, n), dtype=np.float64)
    got = 0
    chunk = 1 << 23
    while got < n:
        p = rng.random((3, chunk)) * (2.0 * R) - R
        keep = (p * p).sum(axis=0) < R * R
        p = p[:, keep]
        take = min(p.shape[1], n - got)
        s[0:3, got:got + take] = p[:, :take]
        got += take
    for s0 in range(0, n, chunk):
        e = min(n, s0 + chunk)
        s[3:6, s0:e] = -infall * s[0:3, s0:e] + rng.standard_normal((3, e - s0)) * sigma_v
    dens = n / (4.0 / 3.0 * math.pi * R ** 3)
    D = (3.0 / dens) ** (1.0 / 3.0)
    nc = _ncell_for(2.0 * R, D)
    h = 2.0 * R / nc
    mean_speed = _mean_speed(s[3:6])
    dt = 0.2 * h / mean_speed
    box = Box(n=n, lo=(-R, -R, -R), hi=(R, R, R), ncell=(nc, nc, nc),
              periodic=(False, False, False), sphere=True, R=R, D2=D * D, dt=dt)
    return Workload("c3_sphere", [box], s, steps, seed,
                    info=dict(sigma=math.pi * D * D, D=D, h=h, mean_speed=mean_speed))


def c4_batch(nboxes=256, n_lo=1e3, n_hi=1e5, ensemble_seed=4, kappa=1.0, steps=50, seed=1):
    """Independent periodic boxes: N_b log-uniform in [n_lo, n_hi], density
    n_b ~ U[0.5, 4], sigma_v,b ~ U[0.5, 2]; box b draws its particles with
    seed 4000 + b.  Cell edge h_b = L_b / floor(L_b / (kappa D_b))."""
    rng = np.random.default_rng(ensemble_seed)
    ns = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), nboxes))).astype(np.int64)
    dens = rng.uniform(0.5, 4.0, nboxes)
    sv = rng.uniform(0.5, 2.0, nboxes)
    boxes, parts = [], []
    for b in range(nboxes):
        n = int(ns[b])
        L = (n / dens[b]) ** (1.0 / 3.0)
        D = (3.0 / dens[b]) ** (1.0 / 3.0)
        nc = max(3, int(math.floor(L / (kappa * D))))
        h = L / nc
        dt = 0.2 * h / (MEAN_SPEED_PER_SIGMA * sv[b])
        box, s = uniform_box(n, L, D=D, sigma_v=float(sv[b]), periodic=True,
                             ic_seed=4000 + b, ncell=nc, dt=dt)
        boxes.append(box)
        parts.append(s)
    state = np.concatenate(parts, axis=1)
    return Workload("c4_batch", boxes, state, steps, seed,
                    info=dict(kappa=kappa, nboxes=nboxes))


def c5_blobs(n=10_000_000, nblobs=64, D=None, ic_seed=5, steps=50, seed=1):
    """64 isotropic Gaussian blobs (centres uniform, widths log-uniform in
    [0.005, 0.05]) in a periodic unit cube; bulk blob velocity N(0, 0.5^2)
    plus thermal N(0, 0.1^2).  D = 3e-3 at N = 1e7, scaled as N^(-1/3) for
    other N (same particles per cell)."""
    if D is None:
        D = 3.0e-3 * (1e7 / n) ** (1.0 / 3.0)
    rng = np.random.default_rng(ic_seed)
    centres = rng.random((nblobs, 3))
    widths = np.exp(rng.uniform(math.log(0.005), math.log(0.05), nblobs))
    vbulk = rng.standard_normal((nblobs, 3)) * 0.5
    which = rng.integers(0, nblobs, n)
    s = np.empty((6, n), dtype=np.float64)
    chunk = 1 << 22
    for s0 in range(0, n, chunk):
        e = min(n, s0 + chunk)
        w = which[s0:e]
        s[0:3, s0:e] = np.mod(centres[w].T + widths[w] * rng.standard_normal((3, e - s0)), 1.0)
        s[3:6, s0:e] = vbulk[w].T + rng.standard_normal((3, e - s0)) * 0.1
    # np.mod can return exactly 1.0 for tiny negative inputs; fold onto [0, 1)
    s[0:3][s[0:3] >= 1.0] = 0.0
    nc = _ncell_for(1.0, D)
    h = 1.0 / nc
    mean_speed = _mean_speed(s[3:6])
    dt = 0.2 * h / mean_speed
    box = Box(n=n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), ncell=(nc, nc, nc),
              periodic=(True, True, True), D2=D * D, dt=dt)
    return Workload("c5_blobs", [box], s, steps, seed,
                    info=dict(D=D, h=h, nblobs=nblobs, mean_speed=mean_speed))


def c1_planar(n=4096, D=0.02, ic_seed=11, steps=10, seed=1):
    """Planar variant of c1_small: n particles uniform in the periodic unit
    square (z = 0.5 in a single reflecting cell layer of [0, 1]), 2-D
    Maxwellian velocities sigma_v = 1 (vz = 0), cells of edge >= D, dt =
    0.2 h / <|v|> with <|v|> = sqrt(pi / 2) for the 2-D Maxwellian."""
    rng = np.random.default_rng(ic_seed)
    s = np.zeros((6, n), dtype=np.float64)
    s[0:2] = rng.random((2, n))
    s[2] = 0.5
    s[3:5] = rng.standard_normal((2, n))
    nc = _ncell_for(1.0, D)
    h = 1.0 / nc
    dt = 0.2 * h / math.sqrt(math.pi / 2.0)
    box = Box(n=n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), ncell=(nc, nc, 1),
              periodic=(True, True, False), D2=D * D, dt=dt)
    return Workload("c1_planar", [box], s, steps, seed=seed, dims=2, info=dict(D=D))


def ppc_sweep_case(n=100_000_000, ppc=3.0, speed=1.0, ic_seed=6, seed=1, state=None):
    """The timing study of Section 2 (Fig. 1): n particles of one speed with
    random directions, uniform in a periodic unit cube, a fixed interaction
    diameter D = (3/n)^(1/3) (three particles per cell at the finest grid) and
    a grid of floor((n/ppc)^(1/3)) cells per side, so that the mean number of
    particles per cell is about ppc (>= 3).  The time step follows the
    paper's adaptive rule dt = dx / v_max (the box dt is only its cap).
    `state` reuses positions and velocities of a previous call."""
    D = (3.0 / n) ** (1.0 / 3.0)
    nc = int(math.floor((n / ppc) ** (1.0 / 3.0)))
    nc = min(nc, int(math.floor(1.0 / D)))
    if state is None:
        box, s = uniform_box(n, L=1.0, D=D, sigma_v=speed, periodic=True, ic_seed=ic_seed, ncell=nc,
                             dt=1.0, same_speed=True)
    else:
        s = state
        box = Box(n=n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), ncell=(nc, nc, nc), periodic=(True,) * 3,
                  D2=D * D, dt=1.0)
    w = Workload(f"ppc_sweep_{ppc:g}", [box], s, 1, seed=seed, dt_rule=1, dt_factor=1.0,
                 info=dict(D=D, ppc=n / nc ** 3))
    return w


def c6_mixture(n=10_000_000, radius=(0.5, 1.0, 1.5), mass=(1.0, 4.0, 9.0), frac=(0.5, 0.3, 0.2), periodic=True,
               ic_seed=7, steps=10, seed=1):
    """Three kinds of particle in a unit cube (Section 1: every particle
    carries its own mass and effective radius).  Kind k has effective radius
    r0 * radius[k] and mass mass[k], and makes up the fraction frac[k] of the
    particles (each particle's kind drawn independently); positions uniform;
    Maxwellian velocities at one temperature (sigma_v = 1 / sqrt(mass[k])).
    r0 makes the largest pair diameter 2 r0 max(radius) equal to (3/n)^(1/3)
    (about three particles per cell on the finest admissible grid), the cell
    edge is the first >= that diameter, and dt = 0.2 h / <|v|> of the
    lightest kind.  The box D2 is the largest pair value."""
    rng = np.random.default_rng(ic_seed)
    kind = rng.choice(len(radius), size=n, p=np.asarray(frac, dtype=np.float64) / sum(frac)).astype(np.uint8)
    s = np.empty((6, n), dtype=np.float64)
    s[0:3] = rng.random((3, n))
    sig = 1.0 / np.sqrt(np.asarray(mass, dtype=np.float64))
    s[3:6] = rng.standard_normal((3, n)) * sig[kind]
    Dmax = (3.0 / n) ** (1.0 / 3.0)
    r0 = Dmax / (2.0 * max(radius))
    rad = tuple(r0 * r for r in radius)
    Dm = 2.0 * max(rad)
    nc = _ncell_for(1.0, Dm)
    h = 1.0 / nc
    dt = 0.2 * h / (MEAN_SPEED_PER_SIGMA * float(sig.max()))
    box = Box(n=n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), ncell=(nc, nc, nc), periodic=(periodic,) * 3,
              D2=Dm * Dm, dt=dt)
    return Workload("c6_mixture", [box], s, steps, seed=seed, species=kind, radius=rad,
                    mass=tuple(float(m) for m in mass), info=dict(radius=rad, frac=frac, h=h))


CONFIGS = {
    "c1_small": c1_small,
    "c2_shock": c2_shock,
    "c3_sphere": c3_sphere,
    "c4_batch": c4_batch,
    "c5_blobs": c5_blobs,
    "c6_mixture": c6_mixture,
}
