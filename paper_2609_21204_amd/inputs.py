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
                 sigma_AB = 0.75, capture radius 1.3 r0;
* ``replica_set`` parameter-sweep replicas (N log-uniform in [256, 8192],
                 eps ~ U[2, 10], density ~ U[0.05, 0.4], B valence 1/2/4,
                 monomers or telechelic chains), built by ``replica``.

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
    bond_types: list       # (kind, k, r0 or R0), or (tether kind, k_b, l_min, l_c1, l_c0, l_max)
    static_pairs: np.ndarray   # (m, 2) uint32 tags
    static_types: np.ndarray   # (m,) uint32
    reactions: list        # dicts: type_a, type_b, bond_type, r_min, r_max, k_on, k_off, epsilon, p_on0, self_avoid,
                           # optionally melt = (lambda, T_melt, k_on_melt, k_off_melt) or slip = a
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
    """Multi-partner gel: A (valence 6) with B (valence 2) and C (valence 1),
    uniform positions with overlap rejection."""
    return _gel(seed, n, density, eps_ab, eps_ac)


def _gel(seed, n, density, eps_ab, eps_ac, pos=None, tid=None, rng=None):
    if rng is None:
        rng = np.random.default_rng(seed)
    L = box_length(n, density)
    n_a = n // 5
    n_b = n // 2
    n_c = n - n_a - n_b
    types = [(6, 1.0, 1.0, 1.0), (2, 0.5, 1.0, 1.0), (1, 0.5, 1.0, 1.0)]
    sigma = np.array([t[1] for t in types])
    if pos is None:
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


def gel_lattice(seed=1, n=200000, density=0.3, eps_ab=8.0, eps_ac=4.0):
    """The gel chemistry of `gel` placed without rejection sampling, for
    systems of millions of particles: n of the m^3 sites of a cubic lattice
    of spacing a = L / m (m^3 >= n, a >= 1.2 at density <= 0.5) are taken at
    random, types are dealt out at random, and each position is jittered by
    up to (a - 1.05) / 2 per axis, so that no two particles come closer than
    1.05 (above every WCA sigma_ij <= 1) and nothing overlaps."""
    rng = np.random.default_rng(seed)
    L = box_length(n, density)
    m = int(math.floor(L / 1.2))
    while m ** 3 < n:
        m -= 1
    a = L / m
    if a < 1.15:
        raise ValueError("density too high for the lattice placement")
    site = rng.choice(m ** 3, n, replace=False)
    ijk = np.stack([site % m, (site // m) % m, site // (m * m)], axis=1).astype(np.float64)
    jit = 0.5 * (a - 1.05)
    pos = (ijk + 0.5) * a - 0.5 * L + rng.uniform(-jit, jit, (n, 3))
    n_a = n // 5
    n_b = n // 2
    tid = np.repeat(np.arange(3, dtype=np.uint32), [n_a, n_b, n - n_a - n_b])[rng.permutation(n)]
    w = _gel(seed, n, density, eps_ab, eps_ac, pos=pos, tid=tid, rng=rng)
    w.name = "gel-lattice"
    return w


def _snake_lattice(L, spacing_min):
    """Sites of a simple cubic lattice filling the periodic box, listed along
    a boustrophedon path (x fastest, direction reversed every row and every
    plane), so that consecutive sites are lattice neighbours.  Spacing
    a = L / floor(L / spacing_min) >= spacing_min."""
    m = int(math.floor(L / spacing_min))
    a = L / m
    k = np.arange(m)
    sites = []
    for z in range(m):
        ys = k if z % 2 == 0 else k[::-1]
        for r, y in enumerate(ys):
            xs = k if (z * m + r) % 2 == 0 else k[::-1]
            sites.append(np.stack([xs, np.full(m, y), np.full(m, z)], axis=1))
    sites = np.concatenate(sites).astype(np.float64)
    return (sites + 0.5) * a - 0.5 * L, a


def replica(seed, n, eps, density, cap_b, kind, kT=1.0):
    """One replica of the parameter sweep: A sites of valence 1 binding B
    sites of valence cap_b (harmonic k = 100, r0 = 1, capture radius 1.3,
    P0_on = 1, bond free energy eps in units of kT), with as many B valences
    as A sites, thermostatted at kT (velocities drawn at kT).

    kind "mono": n A/B monomers.  kind "chains": telechelic chains of 10
    beads (FENE k = 30, R0 = 1.5; ends A, middles M of valence 0) plus B
    crosslinkers.  Particles sit on distinct sites of a lattice of spacing
    >= 0.97 (chains on consecutive sites of a boustrophedon path, so every
    FENE bond starts at the lattice spacing < R0 and no two beads overlap)."""
    rng = np.random.default_rng(seed)
    L = box_length(n, density)
    sites, a = _snake_lattice(L, 0.97)
    nsites = len(sites)
    if kind == "mono":
        n_a = int(round(n * cap_b / (cap_b + 1.0)))
        n_b = n - n_a
        types = [(1, 1.0, 1.0, 1.0), (cap_b, 1.0, 1.0, 1.0)]
        pick = rng.choice(nsites, n, replace=False)
        tid = np.array([0] * n_a + [1] * n_b, dtype=np.uint32)[rng.permutation(n)]
        pos = sites[pick]
        pairs = np.zeros((0, 2), dtype=np.uint32)
        bond_types = [(HARMONIC, 100.0, 1.0)]
        rx_bond, ta, tb = 0, 0, 1
    elif kind == "chains":
        chain_len = 10
        # 2 ends per chain = cap_b valences per crosslinker
        n_chains = max(1, int(round(n * cap_b / (chain_len * cap_b + 2.0))))
        n_b = max(1, int(round(2.0 * n_chains / cap_b)))
        n = n_chains * chain_len + n_b
        L = box_length(n, density)
        sites, a = _snake_lattice(L, 0.97)
        nsites = len(sites)
        nseg = nsites // chain_len
        if nseg < n_chains or nsites - n_chains * chain_len < n_b:
            raise RuntimeError("replica too dense for the lattice")
        segs = rng.choice(nseg, n_chains, replace=False)
        chain_sites = (segs[:, None] * chain_len + np.arange(chain_len)[None, :]).reshape(-1)
        free = np.ones(nsites, dtype=bool)
        free[chain_sites] = False
        b_sites = rng.choice(np.flatnonzero(free), n_b, replace=False)
        pos = np.concatenate([sites[chain_sites], sites[b_sites]])
        tid = np.concatenate([np.tile(np.array([0] + [1] * (chain_len - 2) + [0], dtype=np.uint32), n_chains),
                              np.full(n_b, 2, dtype=np.uint32)])
        types = [(1, 1.0, 1.0, 1.0), (0, 1.0, 1.0, 1.0), (cap_b, 1.0, 1.0, 1.0)]
        base = (np.arange(n_chains) * chain_len)[:, None]
        pairs = np.stack([(base + np.arange(chain_len - 1)).reshape(-1),
                          (base + np.arange(1, chain_len)).reshape(-1)], axis=1).astype(np.uint32)
        bond_types = [(FENE, 30.0, 1.5), (HARMONIC, 100.0, 1.0)]
        rx_bond, ta, tb = 1, 0, 2
    else:
        raise ValueError(kind)
    masses = np.ones(n)
    return Workload(
        name=f"replica_{kind}", n=n, L=L, types=types, pos=_wrap32(pos, L),
        vel=_velocities(n, masses, kT, rng), type_id=tid,
        bond_types=bond_types, static_pairs=pairs,
        static_types=np.zeros(len(pairs), dtype=np.uint32),
        reactions=[dict(type_a=ta, type_b=tb, bond_type=rx_bond, r_min=0.0, r_max=1.3,
                        k_on=math.nan, k_off=math.nan, epsilon=float(eps), p_on0=1.0, self_avoid=0)],
        kT=float(kT), steps=20000, seed=seed,
        extra=dict(eps=float(eps), density=float(density), cap_b=int(cap_b), kind=kind, kT=float(kT)))


def replica_set(seed=1, count=1024, n_min=256, n_max=8192):
    """Parameter-sweep replicas: N log-uniform in [n_min, n_max], eps ~ U[2, 10],
    density ~ U[0.05, 0.4], B valence in {1, 2, 4}, kind mono or chains with
    probability 1/2 each; replica k is seeded with seed * 100003 + k."""
    rng = np.random.default_rng(seed)
    n = np.exp(rng.uniform(math.log(n_min), math.log(n_max), count)).astype(int)
    eps = rng.uniform(2.0, 10.0, count)
    rho = rng.uniform(0.05, 0.4, count)
    cap = rng.choice([1, 2, 4], count)
    kind = np.where(rng.random(count) < 0.5, "mono", "chains")
    return [replica(seed * 100003 + k, int(n[k]), eps[k], rho[k], int(cap[k]), str(kind[k]))
            for k in range(count)]


WORKLOADS = {"small": small, "telechelic": telechelic, "gel": gel, "gel-lattice": gel_lattice}
