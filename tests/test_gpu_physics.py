"""Full MD with bonding sweeps on the GPU against a closed form: the mobile
isolated A-B dimer in a periodic box.  With acceptance P0_on e^{-U_b/kT}
(Eq. pon) and breaking P0_off = P0_on e^{-eps}, detailed balance gives the
stationary bonded probability P_b = K Z_b / (Z_u + K Z_b) with K = e^{eps},
Z_b = 4 pi int_{r_min}^{r_max} r^2 e^{-(U_WCA + U_b)/kT} dr (WCA also acts
on the bonded pair) and Z_u = L^3 - 4 pi int r^2 (1 - e^{-U_WCA/kT}) dr.
At L = 5, kT = 1, harmonic k = 100, r0 = 1, eps = 5, window [0, 1.5]:
P_b = 0.66873539 (quadrature below).  1024 independent dimers run as one
batch; the bonded fraction is averaged over 40 snapshots 2000 steps
apart."""

import math

import numpy as np
import pytest
from scipy.integrate import quad

from paper_2609_21204_amd import dybond as db
from test_gpu_parity import _assert_same_state, log

L, EPS, K_BOND, R0, R_MAX = 5.0, 5.0, 100.0, 1.0, 1.5


def _wca(r):
    rc = 2 ** (1 / 6)
    if r >= rc:
        return 0.0
    x = (1.0 / r) ** 6
    return 4.0 * (x * x - x) + 1.0


def closed_form_pb():
    rc = 2 ** (1 / 6)
    z_u = L ** 3 - 4 * math.pi * quad(lambda r: r * r * (1 - math.exp(-_wca(r))), 1e-9, rc, limit=200,
                                      points=[0.9, 1.0])[0]
    z_b = 4 * math.pi * quad(lambda r: r * r * math.exp(-_wca(r) - 0.5 * K_BOND * (r - R0) ** 2), 1e-9, R_MAX,
                             limit=200, points=[0.9, 1.0, rc])[0]
    k = math.exp(EPS)
    return k * z_b / (z_u + k * z_b)


def _dimer(seed):
    s = db.System(2, 2, L, seed)
    for t in range(2):
        db.db_set_type(s.h, t, 1, 1.0, 1.0, 1.0)
    db.db_add_bond_type(s.h, db.DB_BOND_HARMONIC, K_BOND, R0)
    db.db_set_particles(s.h, [[-1.0, 0.0, 0.0], [1.0, 0.0, 0.0]], np.zeros((2, 3)), [0, 1])
    db.db_add_reaction(s.h, db.make_reaction(0, 1, 0, 0.0, R_MAX, epsilon=EPS, p_on0=1.0, self_avoid=0))
    db.db_set_integrator(s.h, 0.005, 1.0, 1.0, 10)
    db.db_commit(s.h)
    return s


def _n_bonds(s):
    cnt = db._U64()
    st = db.load().db_read_bonds(s.h, None, None, 0, db.ctypes.byref(cnt))
    assert st in (db.DB_OK, db.DB_ETRUNC)
    return cnt.value


def test_closed_form_value():
    assert closed_form_pb() == pytest.approx(0.66873539, abs=1e-8)


@pytest.mark.gpu
def test_dimers_batched_equal_plain_runs():
    log("case dimers, batch vs plain")
    plain = [_dimer(100 + k) for k in range(4)]
    batch = [_dimer(100 + k) for k in range(4)]
    try:
        for p in plain:
            p.step(600)
        db.db_step_batch([b.h for b in batch], 600)
        for k, (p, b) in enumerate(zip(plain, batch)):
            _assert_same_state(p, b, f"dimer {k}")
    finally:
        for x in plain + batch:
            x.close()


@pytest.mark.gpu
def test_mobile_dimer_bonded_fraction_matches_closed_form():
    n_rep, n_snap, gap = 1024, 40, 2000
    log(f"case mobile dimer: {n_rep} replicas, {n_snap} snapshots every {gap} steps")
    systems = [_dimer(1 + k) for k in range(n_rep)]
    try:
        hs = [s.h for s in systems]
        db.db_step_batch(hs, 20000)                      # 100 tau of burn-in
        bonded = np.zeros((n_snap, n_rep))
        for q in range(n_snap):
            db.db_step_batch(hs, gap)
            bonded[q] = [_n_bonds(s) for s in systems]
        assert bonded.max() <= 1
        pb = bonded.mean()
        sd = math.sqrt(pb * (1 - pb) / bonded.size)
        ref = closed_form_pb()
        forms = sum(int(s.observables()["forms"][0]) for s in systems)
        log(f"P_b = {pb:.4f} +- {sd:.4f} (closed form {ref:.4f}); {forms} bonds formed in all")
        assert forms > 20 * n_rep                        # many transitions per replica
        assert abs(pb - ref) < 0.01
    finally:
        for s in systems:
            s.close()
