"""Pins of the oracle's network analyses (CPU only): bond correlation, bond
multiplicity per molecule pair and cluster sizes on small bond networks
built by hand, whose answers are counted out below from their definitions."""

import numpy as np

from oracle import OracleSystem, Reaction


def _network():
    """12 particles in 5 molecules (static chains 0-1-2, 3-4, 5-6-7, 8 and
    9-10-11) and a hand-set dynamic bond table."""
    o = OracleSystem(12, 1, 20.0, 1)
    o.set_type(0, 4, 0.0, 0.0, 1.0)
    rng = np.random.default_rng(0)
    o.set_particles(rng.uniform(-9, 9, (12, 3)), np.zeros((12, 3)), [0] * 12)
    fene = o.add_bond_type(1, 1.0, 50.0)
    o.add_bond_type(0, 1.0, 1.0)
    o.add_bond_type(0, 1.0, 1.0)
    o.add_static_bonds([(0, 1), (1, 2), (3, 4), (5, 6), (6, 7), (9, 10), (10, 11)], [fene] * 7)
    o.add_reaction(Reaction(0, 0, 1, 0.0, 1.0, epsilon=1.0, p_on0=0.5, self_avoid=0))
    o.add_reaction(Reaction(0, 0, 2, 0.0, 1.0, epsilon=1.0, p_on0=0.5, self_avoid=0))
    o.commit()
    # molecules: M0 = {0,1,2}, M1 = {3,4}, M2 = {5,6,7}, M3 = {8}, M4 = {9,10,11}
    # M0-M1 joined twice, M0-M2 once, M1-M2 three times, one loop inside M0,
    # M4 and M3 unbonded
    o.dyn = {(0, 3): 0, (2, 4): 0, (1, 5): 1, (3, 6): 0, (4, 7): 1, (4, 5): 0, (0, 2): 0}
    return o


def test_multiplicity_counts_bonds_per_molecule_pair():
    o = _network()
    hist, pairs, intra = o.bond_multiplicity(4)
    assert hist.tolist() == [1, 1, 1, 0] and pairs == 3 and intra == 1
    hist, pairs, intra = o.bond_multiplicity(2)          # m >= 2 folded into the last bin
    assert hist.tolist() == [1, 2]


def test_cluster_sizes():
    o = _network()
    # {0..7} joined by static and dynamic bonds (8 particles), {8}, {9,10,11}
    hist, n = o.cluster_sizes(10)
    assert n == 3 and hist[0] == 1 and hist[2] == 1 and hist[7] == 1 and hist.sum() == 3
    hist, n = o.cluster_sizes(3)
    assert hist.tolist() == [1, 0, 2]
    o.dyn = {}
    hist, n = o.cluster_sizes(4)
    assert n == 5 and hist.tolist() == [1, 1, 3, 0]


def test_bond_correlation():
    o = _network()
    o.bond_reference()
    assert o.bond_correlation() == (7, 7)
    del o.dyn[(0, 3)]                   # broken
    o.dyn[(1, 5)] = 0                   # same pair, other reaction: not the same bond
    o.dyn[(8, 9)] = 0                   # new bond: not in the reference
    assert o.bond_correlation() == (7, 5)
    o.dyn[(0, 3)] = 0                   # formed again: present
    assert o.bond_correlation() == (7, 6)
