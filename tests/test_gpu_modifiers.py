"""Rate modifiers (melting, slip bonds) and FENE / tether bonds as the bonds
of a reaction, on the GPU through the C ABI, against the FP64 oracle: bond
sets and counters bit for bit after frozen sweeps from identical states,
forces within the force tolerance, and the batched path equal to db_step."""

import math

import numpy as np
import pytest

from helpers import oracle_from_workload
from paper_2609_21204_amd import dybond as db
from paper_2609_21204_amd import inputs
from test_gpu_parity import _assert_same_state, assert_forces, assert_same_bonds, counters, log, sync_oracle

pytestmark = pytest.mark.gpu

NDT = 10 * 0.005


def _small(seed, bond=None, **rx_extra):
    """The small A-B workload (eps 5, P0_on 1) with changes to its reaction."""
    w = inputs.small(seed=seed)
    rx = dict(w.reactions[0])
    if bond is not None:
        w.bond_types = [bond]
    rx.update(rx_extra)
    w.reactions = [rx]
    return w


def _melt_half_bound():
    """k_on^melt = 0, k_off^melt = k_on - k_off: half bound at T_melt = 1."""
    k_on = 1.0 / NDT
    k_off = k_on * math.exp(-5.0)
    return (5.0, 1.0, 0.0, k_on - k_off)


def _frozen_parity(s, o, keys, label):
    sync_oracle(s, o)
    c0 = counters(s)
    for key in keys:
        s.sweep_frozen(key)
        o.sweep_frozen(key)
        assert_same_bonds(s, o, f"{label} key {key}")
    assert np.array_equal(counters(s) - c0, o.counters), f"{label}: counters"
    log(f"{label}: {len(o.dyn)} bonds, counters {o.counters.tolist()}")
    return o.counters


def test_slip_bonds_match_oracle():
    w = _small(4, slip=1.5)
    log("case slip")
    with db.System.from_workload(w) as s:
        s.step(60)
        o = oracle_from_workload(w)
        c = _frozen_parity(s, o, (1000, 1010, 1020, 1030, 2 ** 33 + 7), "slip")
        assert c[0, 2] > 0                        # bonds did break


def test_melting_at_a_set_point_and_after_a_temperature_change():
    w = _small(5, melt=_melt_half_bound())
    log("case melting, set point")
    with db.System.from_workload(w) as s:
        s.step(50)
        o = oracle_from_workload(w)
        c = _frozen_parity(s, o, (500, 510, 520, 530), "melting kT=1 (T_melt)")
        assert c[0, 1] > 0 and c[0, 2] > 0
        for kT in (0.8, 1.3):
            db.db_set_temperature(s.h, kT)
            o.set_temperature(kT)
            s.step(20)
            o2 = oracle_from_workload(w)
            o2.set_temperature(kT)
            _frozen_parity(s, o2, (600, 610, 620), f"melting kT={kT}")
        # far above T_melt nothing forms any more
        db.db_set_temperature(s.h, 3.0)
        o3 = oracle_from_workload(w)
        o3.set_temperature(3.0)
        c = _frozen_parity(s, o3, (700, 710), "melting kT=3")
        assert c[0, 1] == 0


def test_melting_with_the_kinetic_temperature():
    w = _small(9, melt=_melt_half_bound())
    log("case melting, kinetic kT")
    with db.System.from_workload(w, kt_source=db.DB_KT_KINETIC) as s:
        s.step(40)
        o = oracle_from_workload(w, kinetic_T=True)
        _frozen_parity(s, o, (400, 410, 420), "melting kinetic")


def test_fene_bonds_of_a_reaction():
    """The telechelic system with its A-B reaction on a soft FENE bond type
    (k 3, R0 1.5: U_b(1) = 2 kT, so that the acceptance e^{-U_b/kT} lets
    bonds form; window to 1.3): MD with dynamic FENE bonds, then sweeps and
    forces."""
    w = inputs.telechelic(seed=4)
    w.bond_types = list(w.bond_types) + [(db.DB_BOND_FENE, 3.0, 1.5)]
    w.reactions = [dict(w.reactions[0], bond_type=len(w.bond_types) - 1)]
    log(f"case FENE reaction n={w.n}")
    with db.System.from_workload(w) as s:
        s.step(100)
        o = oracle_from_workload(w)
        _frozen_parity(s, o, (2000, 2010, 2020), "FENE reaction")
        assert len(o.dyn) > 0
        assert_forces(s, o, "FENE reaction")


def test_tether_bonds_with_slip():
    """A tether bond type (k_b 1, l_min 0.5, l_c1 0.9, l_c0 1.1, l_max 1.5) as
    the reaction's bond, window [0.6, 1.3], and the slip modifier on it."""
    w = _small(6, bond=(db.DB_BOND_TETHER, 1.0, 0.5, 0.9, 1.1, 1.5), r_min=0.6, r_max=1.3, slip=2.0)
    log("case tether + slip")
    with db.System.from_workload(w) as s:
        s.step(30)
        o = oracle_from_workload(w)
        c = _frozen_parity(s, o, (300, 310, 320, 330), "tether + slip")
        assert c[0, 1] > 0
        assert_forces(s, o, "tether bonds")


@pytest.mark.parametrize("plan", [None, [(2 ** 32 - 1, 64)]], ids=["default", "one-wave"])
def test_batched_runs_with_modifiers_match_plain_runs(plan):
    """The full kernel variant in the default plan (positions of each system
    held in LDS) and with one wave per system (too little LDS per workgroup
    for that: positions read from memory) equals db_step."""
    ws = [_small(4, slip=1.5), _small(5, melt=_melt_half_bound()),
          _small(6, bond=(db.DB_BOND_TETHER, 1.0, 0.5, 0.9, 1.1, 1.5), r_min=0.6, r_max=1.3)]
    kts = [db.DB_KT_SETPOINT, db.DB_KT_KINETIC, db.DB_KT_SETPOINT]
    log(f"case batch with modifiers, plan {plan}")
    plain = [db.System.from_workload(w, kt_source=k) for w, k in zip(ws, kts)]
    batch = [db.System.from_workload(w, kt_source=k) for w, k in zip(ws, kts)]
    try:
        for p in plain:
            p.step(120)
        if plan is None:
            db.db_step_batch([b.h for b in batch], 120)
        else:
            db.db_step_batch_plan([b.h for b in batch], 120, plan)
        for k, (p, b) in enumerate(zip(plain, batch)):
            _assert_same_state(p, b, f"system {k}")
            assert counters(p)[0, 1] > 0
    finally:
        for x in plain + batch:
            x.close()


def test_batch_mixing_lean_and_full_systems():
    """One batch with systems that need the full kernel variant and systems
    that do not: both groups run as branches of one graph, all equal to
    db_step."""
    ws = [inputs.small(seed=11), _small(12, slip=1.0), inputs.replica_set(seed=13, count=2)[1],
          _small(14, melt=_melt_half_bound())]
    log("case batch, lean and full variants: sizes " + " ".join(str(w.n) for w in ws))
    plain = [db.System.from_workload(w) for w in ws]
    batch = [db.System.from_workload(w) for w in ws]
    try:
        for p in plain:
            p.step(90)
        db.db_step_batch_plan([b.h for b in batch], 90, [(600, 256), (2 ** 32 - 1, 1024)])
        for k, (p, b) in enumerate(zip(plain, batch)):
            _assert_same_state(p, b, f"system {k}")
    finally:
        for x in plain + batch:
            x.close()


@pytest.mark.parametrize("shape", [(4, 0), (4, 4)])
def test_step_shapes_with_modifiers_and_the_kinetic_temperature(shape):
    """Four threads per particle (each particle's four threads integrate it
    together, one coordinate per thread) against the automatic shape of
    these small systems: the full kernel variant with melting under the
    kinetic temperature (the step that ends in a sweep sums m v^2) and with
    tether + slip bonds, and the lean variant under the kinetic temperature;
    trajectories bit for bit."""
    cases = [(_small(5, melt=_melt_half_bound()), db.DB_KT_KINETIC),
             (_small(6, bond=(db.DB_BOND_TETHER, 1.0, 0.5, 0.9, 1.1, 1.5), r_min=0.6, r_max=1.3, slip=2.0),
              db.DB_KT_SETPOINT),
             (inputs.small(seed=7), db.DB_KT_KINETIC)]
    for k, (w, kt) in enumerate(cases):
        log(f"case step shape {shape} with modifiers, system {k}")
        ref = db.System.from_workload(w, kt_source=kt)
        alt = db.System.from_workload(w, kt_source=kt)
        try:
            db.db_set_step_shape(alt.h, *shape)
            assert db.db_get_step_shape(ref.h)[0] != 4
            ref.step(150)
            alt.step(150)
            _assert_same_state(ref, alt, f"system {k}, shape {shape}")
            assert counters(ref)[0, 1] > 0
        finally:
            ref.close()
            alt.close()
