"""Shared test helpers: build the oracle (or the library) from a workload."""

import math

import numpy as np

from oracle import OracleSystem, Reaction


def oracle_from_workload(w, kinetic_T=False):
    o = OracleSystem(w.n, len(w.types), w.L, w.seed)
    for t, (val, sig, eps, m) in enumerate(w.types):
        o.set_type(t, val, sig, eps, m)
    for bt in w.bond_types:
        if bt[0] == 2:                                  # tether: (kind, k_b, l_min, l_c1, l_c0, l_max)
            o.add_tether_bond_type(*bt[1:])
        else:
            o.add_bond_type(*bt)
    o.set_particles(w.pos, w.vel, w.type_id)
    if len(w.static_pairs):
        o.add_static_bonds(w.static_pairs, w.static_types)
    for a, r in enumerate(w.reactions):
        r = dict(r)
        melt, slip = r.pop("melt", None), r.pop("slip", None)
        o.add_reaction(Reaction(**r))
        if melt is not None:
            o.set_melting(a, *melt)
        if slip is not None:
            o.set_slip(a, slip)
    o.set_integrator(w.dt, w.kT, w.gamma, w.period, kinetic_T)
    o.commit()
    return o


def min_image_brute(xi, xj, L):
    """Shortest periodic separation by trying all 27 images (test-only)."""
    best = None
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            for c in (-1, 0, 1):
                d = (xj[0] + a * L - xi[0], xj[1] + b * L - xi[1], xj[2] + c * L - xi[2])
                r = math.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])
                if best is None or r < best:
                    best = r
    return best


def random_frozen_system(rng, n=40, L=4.0, n_types=3, valence=(2, 4, 1),
                         sigma=(0.0, 0.0, 0.0), reactions=(), seed=5,
                         static_pairs=(), bond_k=100.0, r0=1.0, dt=0.005, period=10):
    """Small random system without pair forces (sigma 0) for sweep tests."""
    o = OracleSystem(n, n_types, L, seed)
    for t in range(n_types):
        o.set_type(t, valence[t], sigma[t], 1.0, 1.0)
    pos = rng.uniform(-L / 2, L / 2, (n, 3)).astype(np.float32)
    types = rng.integers(0, n_types, n)
    o.set_particles(pos, np.zeros((n, 3)), types)
    fene = o.add_bond_type(1, 30.0, 1.5 * L)
    for k, rx in enumerate(reactions):
        o.add_bond_type(0, bond_k, r0)
    if len(static_pairs):
        o.add_static_bonds(static_pairs, [fene] * len(static_pairs))
    for k, rx in enumerate(reactions):
        a, b, eps, p_on, sa, rmin, rmax = rx
        o.add_reaction(Reaction(a, b, 1 + k, rmin, rmax, epsilon=eps, p_on0=p_on,
                                self_avoid=sa))
    o.set_integrator(dt, 1.0, 1.0, period)
    o.commit()
    return o
