"""Per-sweep event lists (bonds formed and broken by the last sweep) on the
GPU, through the C ABI: equal to the oracle's after frozen sweeps from
identical states, consistent with the GPU's own bond tables and counters
after MD steps (graph-replayed and launched one by one), and the read-out's
error paths."""

import ctypes

import numpy as np
import pytest

from helpers import oracle_from_workload
from paper_2609_21204_amd import dybond as db
from paper_2609_21204_amd import inputs
from test_gpu_parity import assert_same_bonds, counters, log, sync_oracle

pytestmark = pytest.mark.gpu


def _rows(a):
    return {tuple(r) for r in np.asarray(a, dtype=np.int64).tolist()}


def _check_identity(before, after, s, c0, label):
    """after = before - broken + formed; formed new, broken old; list
    lengths equal to the counter increments of the one sweep."""
    f, _ = s.sweep_events(db.DB_EVENT_FORMED)
    b, _ = s.sweep_events(db.DB_EVENT_BROKEN)
    f, b = _rows(f), _rows(b)
    assert not (f & before) and b <= before, label
    assert after == (before - b) | f, label
    dc = counters(s) - c0
    assert len(f) == dc[:, 1].sum() and len(b) == dc[:, 2].sum(), f"{label}: {len(f)}, {len(b)} vs {dc.tolist()}"
    return len(f), len(b)


@pytest.mark.parametrize("name,warm", [("small", 60), ("telechelic", 100)])
def test_events_of_frozen_sweeps_match_oracle(name, warm):
    w = inputs.WORKLOADS[name](seed=8)
    w.reactions = [dict(w.reactions[0], epsilon=2.0)]         # P0_off = P0_on e^-2: bonds also break
    log(f"case events/{name}")
    with db.System.from_workload(w) as s:
        assert s.sweep_events(db.DB_EVENT_FORMED)[1] == db.NO_SWEEP
        s.step(warm)
        o = oracle_from_workload(w)
        sync_oracle(s, o)
        assert s.sweep_events(db.DB_EVENT_BROKEN)[1] == warm       # the last sweep of the steps
        nf = nb = 0
        for key in (3000, 3010, 3020, 2 ** 33 + 11):
            before, c0 = _rows(s.bonds()), counters(s)
            s.sweep_frozen(key)
            o.sweep_frozen(key)
            assert_same_bonds(s, o, f"{name} key {key}")      # bonds and both event lists
            f, b = _check_identity(before, _rows(s.bonds()), s, c0, f"{name} key {key}")
            nf, nb = nf + f, nb + b
        log(f"{name}: {nf} formed, {nb} broken over 4 frozen sweeps")
        assert nf > 0 and nb > 0


def test_events_after_md_steps_graph_replayed_and_single():
    """The sweep at the end of a graph-replayed span records the same events
    as the same sweep launched step by step; each is the sweep's change of
    the bond table."""
    w = inputs.small(seed=9, eps_bond=2.0)
    log("case events after MD steps")
    with db.System.from_workload(w) as g, db.System.from_workload(w) as p:
        g.step(240)                                   # two captured 120-step spans
        for _ in range(23):
            p.step(10)                                # launched one by one (shorter than a span)
        before, c0 = _rows(p.bonds()), counters(p)
        p.step(10)                                    # its last sweep at step 240
        _check_identity(before, _rows(p.bonds()), p, c0, "sweep at 240")
        for kind in (db.DB_EVENT_FORMED, db.DB_EVENT_BROKEN):
            eg, sg = g.sweep_events(kind)
            ep, sp = p.sweep_events(kind)
            assert sg == sp == 240 and np.array_equal(eg, ep), f"event list {kind}"
        assert np.array_equal(g.bonds(), p.bonds())
        p.step(5)                                     # no sweep: the lists stay those of step 240
        assert p.sweep_events(db.DB_EVENT_FORMED)[1] == 240


def test_event_readout_errors_and_reset():
    w = inputs.small(seed=10, eps_bond=2.0)
    log("case event read-out errors")
    with db.System.from_workload(w) as s:
        s.step(50)
        lib = db.load()
        cnt, step = ctypes.c_uint64(), ctypes.c_uint64()
        m = len(s.sweep_events(db.DB_EVENT_FORMED)[0])
        assert m > 1
        buf = np.zeros(2 * m, np.uint32)
        bt = np.zeros(m, np.uint32)
        st = lib.db_read_sweep_events(s.h, db.DB_EVENT_FORMED, buf.ctypes.data, bt.ctypes.data, m - 1,
                                      ctypes.byref(cnt), ctypes.byref(step))
        assert st == db.DB_ETRUNC and cnt.value == m and step.value == 50
        assert lib.db_read_sweep_events(s.h, 2, None, None, 0, ctypes.byref(cnt), None) == db.DB_EINVAL
        assert lib.db_read_sweep_events(s.h, db.DB_EVENT_FORMED, None, None, 0, None, None) == db.DB_EINVAL
        # a replaced state has had no sweep
        pos, vel, b = s.positions(), s.velocities(), s.bonds()
        s.set_state(50, pos, vel, b[:, :2], b[:, 2])
        for kind in (db.DB_EVENT_FORMED, db.DB_EVENT_BROKEN):
            e, sk = s.sweep_events(kind)
            assert len(e) == 0 and sk == db.NO_SWEEP


def test_tiny_system_certain_forming_and_breaking():
    """Four particles, two A-B pairs at r0 far apart, P0_on = P0_off = 1
    (epsilon 0): each sweep breaks every bond present at its start and forms
    every free pair, and never tests a bond it formed itself; counted by hand
    from the sweep's rules, the same as the oracle's pin."""
    pos = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [-4.0, -4.0, -4.0], [-3.0, -4.0, -4.0]], np.float32)
    log("case events, four particles")
    with db.System(4, 2, 10.0, 3) as s:
        db.db_set_type(s.h, 0, 1, 1.0, 1.0, 1.0)
        db.db_set_type(s.h, 1, 1, 1.0, 1.0, 1.0)
        db.db_add_bond_type(s.h, db.DB_BOND_HARMONIC, 100.0, 1.0)
        db.db_set_particles(s.h, pos, np.zeros((4, 3)), [0, 1, 0, 1])
        db.db_add_reaction(s.h, db.make_reaction(0, 1, 0, 0.0, 1.3, epsilon=0.0, p_on0=1.0, self_avoid=0))
        db.db_commit(s.h)
        s.set_state(0, pos, np.zeros((4, 3)), [[0, 1]], [0])
        expect = [([[2, 3, 0]], [[0, 1, 0]]), ([[0, 1, 0]], [[2, 3, 0]])]
        for k, key in enumerate((10, 20, 30, 40)):
            s.sweep_frozen(key)
            f, sf = s.sweep_events(db.DB_EVENT_FORMED)
            b, _ = s.sweep_events(db.DB_EVENT_BROKEN)
            ef, eb = expect[k % 2]
            assert sf == key and f.tolist() == ef and b.tolist() == eb, (key, f.tolist(), b.tolist())
            assert s.bonds().tolist() == ef
        ob = s.observables()
        assert ob["forms"].tolist() == [4] and ob["breaks"].tolist() == [4] and ob["attempts"].tolist() == [4]


def test_events_across_two_reactions_on_one_pair_match_oracle():
    """Two reactions on one A-B pair with their own bond types, P_on =
    P_off = 1, the pair bonded by reaction 0 when each sweep starts: in one
    reaction order the bond breaks and forms again with reaction 1's type,
    in the other it only breaks.  Bonds and both event lists equal the
    oracle's for sweeps of both orders."""
    import math
    from oracle import OracleSystem, Reaction
    from oracle.dybond import BOND_HARMONIC
    from oracle.philox import reaction_order
    pos = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0]], np.float32)
    log("case events, two reactions on one pair")
    o = OracleSystem(2, 2, 10.0, 5)
    with db.System(2, 2, 10.0, 5) as s:
        for t in range(2):
            db.db_set_type(s.h, t, 1, 1.0, 1.0, 1.0)
            o.set_type(t, 1, 1.0, 1.0, 1.0)
        for _ in range(2):
            db.db_add_bond_type(s.h, db.DB_BOND_HARMONIC, 100.0, 1.0)
            o.add_bond_type(BOND_HARMONIC, 100.0, 1.0)
        db.db_set_particles(s.h, pos, np.zeros((2, 3)), [0, 1])
        o.set_particles(pos, np.zeros((2, 3)), [0, 1])
        for bt in range(2):
            db.db_add_reaction(s.h, db.make_reaction(0, 1, bt, 0.0, 1.3, epsilon=0.0, p_on0=1.0, self_avoid=0))
            o.add_reaction(Reaction(0, 1, bt, 0.0, 1.3, k_on=math.nan, k_off=math.nan, epsilon=0.0, p_on0=1.0,
                                    self_avoid=0))
        db.db_commit(s.h)
        o.set_integrator(0.005, 1.0, 1.0, 10)
        o.commit()
        seen = set()
        for key in range(10, 200, 10):
            s.set_state(0, pos, np.zeros((2, 3)), [[0, 1]], [0])
            o.set_state(0, pos, np.zeros((2, 3)), [(0, 1)], [0])
            s.sweep_frozen(key)
            o.sweep_frozen(key)
            assert_same_bonds(s, o, f"two reactions, key {key}")
            seen.add(tuple(reaction_order(5, key, 2)))
        assert seen == {(0, 1), (1, 0)}
