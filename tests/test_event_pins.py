"""Pins of the oracle's per-sweep event lists (bonds formed and broken by the
last sweep), CPU only.

A hand-counted case from the sweep's rules (Sec. 2.3): with P_on = P_off = 1
every free pair at r0 forms and every bond present at the start of the sweep
breaks, while a bond formed in the sweep is not tested for breaking in the
same sweep.  Then the bookkeeping identity on a random system, pinned by the
bond table the algorithm produces and by its counters, not by the lists
themselves: after = before - broken + formed, formed disjoint from before,
broken contained in before, list lengths equal to the counter increments.
"""

import math

import numpy as np

from oracle import OracleSystem, Reaction
from oracle.dybond import BOND_HARMONIC
from helpers import oracle_from_workload
from paper_2609_21204_amd import inputs

# two A-B pairs at r0 = 1, far apart (L = 10, r_max = 1.3)
POS = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [-4.0, -4.0, -4.0], [-3.0, -4.0, -4.0]])


def _two_pairs():
    o = OracleSystem(4, 2, 10.0, 3)
    o.set_type(0, 1, 1.0, 1.0, 1.0)
    o.set_type(1, 1, 1.0, 1.0, 1.0)
    bt = o.add_bond_type(BOND_HARMONIC, 100.0, 1.0)
    o.set_particles(POS, np.zeros((4, 3)), [0, 1, 0, 1])
    # epsilon 0 and P0_on 1: P0_off = P0_on e^0 = 1
    o.add_reaction(Reaction(type_a=0, type_b=1, bond_type=bt, r_min=0.0, r_max=1.3, k_on=math.nan,
                            k_off=math.nan, epsilon=0.0, p_on0=1.0, self_avoid=0))
    o.set_integrator(0.005, 1.0, 1.0, 10)
    o.commit()
    return o, bt


def test_certain_forming_and_breaking_alternate():
    o, bt = _two_pairs()
    assert o.sweep_events("formed")[1] is None          # no sweep yet
    o.set_state(0, POS, np.zeros((4, 3)), [(0, 1)], [bt])
    o.sweep_frozen(10)
    f, s = o.sweep_events("formed")
    b, _ = o.sweep_events("broken")
    assert s == 10
    assert f.tolist() == [[2, 3, bt]] and b.tolist() == [[0, 1, bt]]
    assert o.bonds().tolist() == [[2, 3, bt]]           # the new bond survived its own sweep
    o.sweep_frozen(20)
    f, s = o.sweep_events("formed")
    b, _ = o.sweep_events("broken")
    assert s == 20 and f.tolist() == [[0, 1, bt]] and b.tolist() == [[2, 3, bt]]
    o.set_state(0, POS, np.zeros((4, 3)))
    assert o.sweep_events("broken")[1] is None and len(o.sweep_events("broken")[0]) == 0


def _rows(a):
    return {tuple(r) for r in np.asarray(a).tolist()}


def test_events_account_for_the_change_of_the_bond_table():
    w = inputs.small(seed=5, eps_bond=2.0)              # P0_off = e^-2: both forming and breaking
    o = oracle_from_workload(w)
    o.step(30)
    seen_f = seen_b = 0
    for key in (1000, 1010, 1020, 1030, 1040):
        before = _rows(o.bonds())
        c0 = o.counters.copy()
        o.sweep_frozen(key)
        after = _rows(o.bonds())
        f, s = o.sweep_events("formed")
        b, _ = o.sweep_events("broken")
        f, b = _rows(f), _rows(b)
        assert s == key
        assert not (f & before) and b <= before
        assert after == (before - b) | f
        dc = o.counters - c0
        assert len(f) == dc[:, 1].sum() and len(b) == dc[:, 2].sum()
        seen_f += len(f)
        seen_b += len(b)
    assert seen_f > 0 and seen_b > 0


def test_events_across_two_reactions_on_one_pair():
    """Two reactions on the same A-B pair, each with its own bond type
    (reading of two reactions on one type pair), valence 1, P_on = P_off = 1,
    the pair bonded by reaction 0 at the start of the sweep.  Reactions run
    in the sweep's random order: reaction 0 first breaks the bond, and then
    reaction 1 forms it again with its own bond type; reaction 1 first finds
    both sites full, and reaction 0 then only breaks.  Counted by hand for
    each order."""
    from oracle.philox import reaction_order
    pos = POS[:2]
    seen = set()
    for key in range(10, 400, 10):
        o = OracleSystem(2, 2, 10.0, 5)
        o.set_type(0, 1, 1.0, 1.0, 1.0)
        o.set_type(1, 1, 1.0, 1.0, 1.0)
        b0 = o.add_bond_type(BOND_HARMONIC, 100.0, 1.0)
        b1 = o.add_bond_type(BOND_HARMONIC, 100.0, 1.0)
        o.set_particles(pos, np.zeros((2, 3)), [0, 1])
        for bt in (b0, b1):
            o.add_reaction(Reaction(type_a=0, type_b=1, bond_type=bt, r_min=0.0, r_max=1.3, k_on=math.nan,
                                    k_off=math.nan, epsilon=0.0, p_on0=1.0, self_avoid=0))
        o.set_integrator(0.005, 1.0, 1.0, 10)
        o.commit()
        o.set_state(0, pos, np.zeros((2, 3)), [(0, 1)], [b0])
        order = tuple(reaction_order(5, key, 2))
        o.sweep_frozen(key)
        f, _ = o.sweep_events("formed")
        b, _ = o.sweep_events("broken")
        assert b.tolist() == [[0, 1, b0]]
        if order == (0, 1):
            assert f.tolist() == [[0, 1, b1]] and o.bonds().tolist() == [[0, 1, b1]]
        else:
            assert f.tolist() == [] and o.bonds().tolist() == []
        seen.add(order)
    assert seen == {(0, 1), (1, 0)}
