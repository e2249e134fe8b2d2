"""Seeded synthetic workloads (initial states and parameters).

This module only builds inputs: positions, velocities, types, static bonds
and the parameter sets of the three single-system workloads.  It contains
none of the method's arithmetic (no forces, no integration, no bonding
sweep) and is the one piece of code that both the HIP library's callers and
the FP64 oracle's tests consume.

The paper runs on no public dataset; every input here is synthetic, drawn
with ``numpy.random.default_rng(seed)``:

* ``small``      512 particles (256 A + 256 B, valence 1), density 0.1,
                 uniform placement with overlap rejection (r >= sigma_ij),
                 harmonic A-B bond k=100, r0=1, capture radius 1.3,
                 eps = 5 kT, P0_on = 1;
* ``telechelic`` 1000 chains of 10 beads (FENE k=30, R0=1.5; ends A with
                 valence 1, middles M with valence 0) + 500 crosslinkers B
                 (valence 4), density 0.3, eps = 6 kT;
* ``gel``        N particles (default 200000) at density 0.3: 20% A
                 (sigma 1, valence 6), 50% B (sigma 0.5, valence 2), 30% C
                 (sigma 0.5, valence 1); A-B eps = 8 kT with P0_on = 1 and
                 A-C eps = 4 kT with P0_on = 0.25; bond rest length
                 sigma_AB = 0.75, capture radius 1.3 r0.

All use Langevin kT = 1, gamma = 1, dt = 0.005, sweeps every 10 steps.
"""

import math
from dataclasses import dataclass, field

import numpy as np

HARMONIC = 0
FENE = 1


@dataclass
class Workload:
    name: str
    n: int
    L: float
    types: list            # per type: (valence, sigma, eps, mass)
    pos: np.ndarray        # (n, 3) float32 in [-L/2, L/2)
    vel: np.ndarray        # (n, 3) float32
    type_id: np.ndarray    # (n,) uint32
    bond_types: list       # (kind, k, r0 or R0)
    static_pairs: np.ndarray   # (m, 2) uint32 tags
    static_types: np.ndarray   # (m,) uint32
    reactions: list        # dicts: type_a, type_b, bond_type, r_min, r_max, k_on, k_off, epsilon, p_on0, self_avoid
    dt: float = 0.005
    kT: float = 1.0
    gamma: float = 1.0
    period: int = 10
    steps: int = 1000
    seed: int = 1
    extra: dict = field(default_factory=dict)


def box_length(n, density):
    return (n / density) ** (1.0 / 3.0)


class _Grid:
    """Spatial hash used only to reject overlapping placements."""

    def __init__(self, L, cell):
        self.L = L
        self.nc = max(1, int(math.floor(L / cell)))
        self.cells = {}
        self.pts = []

    def _cell(self, p):
        c = np.floor((p + 0.5 * self.L) / self.L * self.nc).astype(np.int64) % self.nc
        return int(c[0]), int(c[1]), int(c[2])

    def near(self, p):
        cx, cy, cz = self._cell(p)
        nc = self.nc
        rng = range(-1, 2) if nc >= 3 else range(0, nc)
        seen = set()
        for dx in rng:
            for dy in rng:
                for dz in rng:
                    key = ((cx + dx) % nc, (cy + dy) % nc, (cz + dz) % nc)
                    if key in seen:
                        continue
                    seen.add(key)
                    yield from self.cells.get(key, ())

    def dist(self, p, q):
        d = q - p
        d -= self.L * np.round(d / self.L)
        return math.sqrt(float(d @ d))

    def add(self, p, payload):
        self.cells.setdefault(self._cell(p), []).append(len(self.pts))
        self.pts.append((p, payload))


def _wrap32(x, L):
    x = np.asarray(x, dtype=np.float64)
    x = x - L * np.floor(x / L + 0.5)
    x32 = x.astype(np.float32)
    half = np.float32(0.5 * L)
    x32[x32 >= half] -= np.float32(L)
    x32[x32 < -half] += np.float32(L)
    x32[x32 >= half] = -half
    return x32


def _velocities(n, masses, kT, rng):
    v = rng.standard_normal((n, 3)) * np.sqrt(kT / masses)[:, None]
    p = (masses[:, None] * v).sum(axis=0) / masses.sum()
    v -= p
    return v.astype(np.float32)


def _place_uniform(grid, types_to_place, sigma, rng, L, max_tries=100000):
    """Uniform positions, rejecting r < sigma_ij to anything already placed."""
    out = []
    for t in types_to_place:
        for _ in range(max_tries):
            p = rng.uniform(-0.5 * L, 0.5 * L, 3)
            ok = True
            for idx in grid.near(p):
                q, tq = grid.pts[idx]
                if grid.dist(p, q) < 0.5 * (sigma[t] + sigma[tq]):
                    ok = False
                    break
            if ok:
                grid.add(p, t)
                out.append(p)
                break
        else:
            raise RuntimeError("placement failed: density too high")
    return out


def small(seed=1, n=512, density=0.1, eps_bond=5.0):
    """512 A/B particles with valence 1 (the small plain-method workload)."""
    rng = np.random.default_rng(seed)
    L = box_length(n, density)
    types = [(1, 1.0, 1.0, 1.0), (1, 1.0, 1.0, 1.0)]
    sigma = np.array([t[1] for t in types])
    tid = np.array([0] * (n // 2) + [1] * (n - n // 2), dtype=np.uint32)
    grid = _Grid(L, 1.0)
    order = rng.permutation(n)
    pos = np.zeros((n, 3))
    placed = _place_uniform(grid, tid[order], sigma, rng, L)
    pos[order] = np.array(placed)
    masses = np.ones(n)
    return Workload(
        name="small", n=n, L=L, types=types, pos=_wrap32(pos, L),
        vel=_velocities(n, masses, 1.0, rng), type_id=tid,
        bond_types=[(HARMONIC, 100.0, 1.0)],
        static_pairs=np.zeros((0, 2), dtype=np.uint32),
        static_types=np.zeros(0, dtype=np.uint32),
        reactions=[dict(type_a=0, type_b=1, bond_type=0, r_min=0.0, r_max=1.3,
                        k_on=math.nan, k_off=math.nan, epsilon=eps_bond, p_on0=1.0,
                        self_avoid=0)],
        steps=1000, seed=seed)


def telechelic(seed=1, n_chains=1000, chain_len=10, n_cross=500, density=0.3,
               eps_bond=6.0):
    """Telechelic chains with valence-4 crosslinkers."""
    rng = np.random.default_rng(seed)
    n = n_chains * chain_len + n_cross
    L = box_length(n, density)
    # type 0 = A chain end (valence 1), 1 = M chain middle, 2 = B crosslinker (valence 4)
    types = [(1, 1.0, 1.0, 1.0), (0, 1.0, 1.0, 1.0), (4, 1.0, 1.0, 1.0)]
    grid = _Grid(L, 1.0)
    pos = []
    tid = []
    pairs = []
    step_len, min_sep = 0.97, 0.9
    for c in range(n_chains):
        while True:           # grow one chain by a self-avoiding random walk
            beads = []
            start = rng.uniform(-0.5 * L, 0.5 * L, 3)
            if any(grid.dist(start, grid.pts[i][0]) < 1.0 for i in grid.near(start)):
                continue
            beads.append(start)
            for b in range(1, chain_len):
                for _ in range(200):
                    d = rng.standard_normal(3)
                    p = beads[-1] + step_len * d / np.linalg.norm(d)
                    p = p - L * np.floor(p / L + 0.5)
                    ok = all(grid.dist(p, grid.pts[i][0]) >= min_sep for i in grid.near(p))
                    ok = ok and all(grid.dist(p, q) >= min_sep for q in beads[:-1])
                    if ok:
                        beads.append(p)
                        break
                else:
                    break
            if len(beads) == chain_len:
                break
        base = len(pos)
        for b, p in enumerate(beads):
            grid.add(p, 0)
            pos.append(p)
            tid.append(0 if b in (0, chain_len - 1) else 1)
            if b > 0:
                pairs.append((base + b - 1, base + b))
    sigma = np.array([1.0, 1.0, 1.0])
    placed = _place_uniform(grid, [2] * n_cross, sigma, rng, L)
    pos.extend(placed)
    tid.extend([2] * n_cross)
    pos = np.array(pos)
    masses = np.ones(n)
    return Workload(
        name="telechelic", n=n, L=L, types=types, pos=_wrap32(pos, L),
        vel=_velocities(n, masses, 1.0, rng), type_id=np.array(tid, dtype=np.uint32),
        bond_types=[(FENE, 30.0, 1.5), (HARMONIC, 100.0, 1.0)],
        static_pairs=np.array(pairs, dtype=np.uint32).reshape(-1, 2),
        static_types=np.zeros(len(pairs), dtype=np.uint32),
        reactions=[dict(type_a=0, type_b=2, bond_type=1, r_min=0.0, r_max=1.3,
                        k_on=math.nan, k_off=math.nan, epsilon=eps_bond, p_on0=1.0,
                        self_avoid=0)],
        steps=100000, seed=seed)


def gel(seed=1, n=200000, density=0.3, eps_ab=8.0, eps_ac=4.0):
    """Multi-partner gel: A (valence 6) with B (valence 2) and C (valence 1)."""
    rng = np.random.default_rng(seed)
    L = box_length(n, density)
    n_a = n // 5
    n_b = n // 2
    n_c = n - n_a - n_b
    types = [(6, 1.0, 1.0, 1.0), (2, 0.5, 1.0, 1.0), (1, 0.5, 1.0, 1.0)]
    sigma = np.array([t[1] for t in types])
    tid = np.array([0] * n_a + [1] * n_b + [2] * n_c, dtype=np.uint32)
    grid = _Grid(L, 1.0)
    order = rng.permutation(n)
    pos = np.zeros((n, 3))
    pos[order] = np.array(_place_uniform(grid, tid[order], sigma, rng, L))
    r0 = 0.5 * (1.0 + 0.5)
    masses = np.ones(n)
    return Workload(
        name="gel", n=n, L=L, types=types, pos=_wrap32(pos, L),
        vel=_velocities(n, masses, 1.0, rng), type_id=tid,
        bond_types=[(HARMONIC, 100.0, r0), (HARMONIC, 100.0, r0)],
        static_pairs=np.zeros((0, 2), dtype=np.uint32),
        static_types=np.zeros(0, dtype=np.uint32),
        reactions=[
            dict(type_a=0, type_b=1, bond_type=0, r_min=0.0, r_max=1.3 * r0,
                 k_on=math.nan, k_off=math.nan, epsilon=eps_ab, p_on0=1.0, self_avoid=0),
            dict(type_a=0, type_b=2, bond_type=1, r_min=0.0, r_max=1.3 * r0,
                 k_on=math.nan, k_off=math.nan, epsilon=eps_ac, p_on0=0.25, self_avoid=0),
        ],
        steps=10000, seed=seed)


WORKLOADS = {"small": small, "telechelic": telechelic, "gel": gel}
