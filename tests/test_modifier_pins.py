"""Pins of the oracle's rate modifiers and dynamic bond evaluators (CPU only).

Melting (Eqs. gT, kT), slip bonds (Eq. slip), FENE and tether bonds as the
bonds of a reaction.  Each pin comes from outside the oracle's own code:
values of the potentials worked out by hand at chosen points, central
finite differences, the limits and symmetries of the switch, the paper's
statement that k_off^melt = k_on^init - k_off^init leaves half of the pairs
bound at T_melt, Bell's force form of the slip exponent, and stationary
fractions of the two-state chain of many independent frozen dimers.
"""

import math

import numpy as np
import pytest

from oracle import OracleSystem, Reaction
from oracle.dybond import (BOND_FENE, BOND_HARMONIC, OracleError, melt_switch, melted_probabilities,
                           slip_probability)

TETHER = dict(k_b=2.0, l_min=0.5, l_c1=0.8, l_c0=1.2, l_max=1.6)


def _tether_system():
    o = OracleSystem(2, 1, 10.0, 1)
    o.set_type(0, 0, 0.0, 0.0, 1.0)
    o.set_particles(np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0]]), np.zeros((2, 3)), [0, 0])
    bt = o.add_tether_bond_type(**TETHER)
    o.add_static_bonds([(0, 1)], [bt])
    o.commit()
    return o, bt


def test_tether_energy_at_hand_computed_points():
    o, bt = _tether_system()
    # r = 1.4: 2 e^{1/(1.2-1.4)} / (1.6-1.4) = 10 e^-5 ; r = 0.6: 2 e^{1/(0.6-0.8)} / (0.6-0.5) = 20 e^-5
    assert o.bond_energy_force(bt, 1.4)[0] == pytest.approx(10.0 * math.exp(-5.0), rel=1e-14)
    assert o.bond_energy_force(bt, 0.6)[0] == pytest.approx(20.0 * math.exp(-5.0), rel=1e-14)
    for r in (0.8, 0.9, 1.0, 1.2):             # flat between l_c1 and l_c0
        assert o.bond_energy_force(bt, r) == (0.0, 0.0)
    # smooth at both ends of the flat region, divergent at l_min and l_max
    assert o.bond_energy_force(bt, 1.2 + 1e-3)[0] < 1e-300
    assert o.bond_energy_force(bt, 0.8 - 1e-3)[0] < 1e-300
    assert o.bond_energy_force(bt, 1.6 - 1e-4)[0] > 100.0 and o.bond_energy_force(bt, 0.5 + 1e-4)[0] > 100.0
    assert o.bond_in_domain(bt, 1.59) and not o.bond_in_domain(bt, 1.6) and not o.bond_in_domain(bt, 0.5)


def test_tether_force_is_minus_the_gradient():
    o, bt = _tether_system()
    h = 1e-6
    for r in (0.55, 0.62, 0.75, 0.79, 1.21, 1.3, 1.45, 1.58):
        fd = (o.bond_energy_force(bt, r + h)[0] - o.bond_energy_force(bt, r - h)[0]) / (2 * h)
        assert o.bond_energy_force(bt, r)[1] == pytest.approx(fd, rel=1e-6, abs=1e-9)
    # the static bond's force on the pair: -dU/dr along the bond, equal and opposite
    o.x[1] = [1.4, 0.0, 0.0]
    F, PE = o.forces(o.x)
    dU = o.bond_energy_force(bt, 1.4)[1]
    assert F[0] == pytest.approx([dU, 0.0, 0.0]) and F[1] == pytest.approx([-dU, 0.0, 0.0])
    assert PE == pytest.approx(10.0 * math.exp(-5.0))
    o.x[1] = [1.7, 0.0, 0.0]
    with pytest.raises(OracleError) as e:
        o.forces(o.x)                          # beyond l_max
    assert e.value.code == "EBOND"


def test_melting_switch():
    lam, Tm = 7.0, 1.3
    assert melt_switch(lam, Tm, Tm) == 0.5
    for x in (0.01, 0.1, 0.4):
        assert melt_switch(lam, Tm, Tm + x) + melt_switch(lam, Tm, Tm - x) == pytest.approx(1.0, abs=1e-15)
    assert melt_switch(lam, Tm, Tm + 10.0) == pytest.approx(1.0, abs=1e-15)
    assert melt_switch(lam, Tm, Tm - 10.0) == pytest.approx(0.0, abs=1e-15)
    assert melt_switch(0.0, Tm, 5.0) == 0.5                     # no sharpness: halfway everywhere
    on, off = melted_probabilities(0.4, 0.1, 0.0, 0.3, lam, Tm, Tm)
    assert on == pytest.approx(0.2) and off == pytest.approx(0.2)


def test_slip_probability_limits_and_bell_form():
    assert slip_probability(0.01, 0.0, 3.0, 1.0) == 0.01          # a = 0: no load dependence
    assert slip_probability(0.01, 2.0, 0.0, 1.0) == 0.01          # unstretched bond
    assert slip_probability(0.01, 2.0, 1.0, 1.0) == pytest.approx(0.01 * math.exp(2.0))
    assert slip_probability(0.5, 3.0, 4.0, 1.0) == 1.0            # capped
    assert slip_probability(0.01, 2.0, 0.0, 0.0) == 0.01          # T -> 0, both ends defined
    assert slip_probability(0.01, 2.0, 0.3, 0.0) == 1.0
    # harmonic bond: a sqrt(U/kT) = f x*/kT with tension f = k |r - r0| and
    # Bell distance x* = a sqrt(kT / 2k)
    k, r0, r, a, kT = 100.0, 1.0, 1.07, 1.5, 0.8
    U = 0.5 * k * (r - r0) ** 2
    f, xs = k * abs(r - r0), a * math.sqrt(kT / (2.0 * k))
    assert a * math.sqrt(U / kT) == pytest.approx(f * xs / kT, rel=1e-14)


def _dimers(n_pairs, r, rx_kw, kind=BOND_HARMONIC, bond=(100.0, 1.0), tether=None, kT=1.0, seed=5,
            melt=None, slip=None):
    """n_pairs A-B pairs at separation r along x, on a grid of spacing 4."""
    side = int(math.ceil(n_pairs ** (1.0 / 3.0)))
    L = 4.0 * side
    pts, types = [], []
    for k in range(n_pairs):
        c = np.array([k % side, (k // side) % side, k // (side * side)], dtype=np.float64) * 4.0 - 0.5 * L + 0.3
        pts += [c, c + [r, 0.0, 0.0]]
        types += [0, 1]
    o = OracleSystem(2 * n_pairs, 2, L, seed)
    o.set_type(0, 1, 0.0, 0.0, 1.0)
    o.set_type(1, 1, 0.0, 0.0, 1.0)
    o.set_particles(np.array(pts), np.zeros((2 * n_pairs, 3)), types)
    bt = o.add_tether_bond_type(**tether) if tether else o.add_bond_type(kind, *bond)
    o.add_reaction(Reaction(0, 1, bt, rx_kw.pop("r_min", 0.0), rx_kw.pop("r_max", 1.3), self_avoid=0, **rx_kw))
    o.set_integrator(0.005, kT, 1.0, 10)
    if melt:
        o.set_melting(0, *melt)
    if slip is not None:
        o.set_slip(0, slip)
    o.commit()
    return o


def _stationary(o, n_sw, n_pairs, burn=200):
    bound = []
    for s in range(1, n_sw + 1):
        o.sweep(s)
        if s > burn:
            bound.append(len(o.dyn) / n_pairs)
    return float(np.mean(bound)), (n_sw - burn) * n_pairs


def _check_two_state(pb, samples, p, q):
    tau = (2 - p - q) / (p + q)
    assert abs(pb - p / (p + q)) < 4.5 * math.sqrt(p * q / (p + q) ** 2 * tau / samples), (pb, p / (p + q))


def test_melting_leaves_half_bound_at_T_melt():
    """k_on^melt = 0 and k_off^melt = k_on^init - k_off^init: half of the
    pairs bound at T_melt (the uniqueness statement of Sec. 2.4)."""
    ndt = 10 * 0.005
    k_on, eps = 4.0, 1.0
    k_off = k_on * math.exp(-eps)
    lam, Tm = 6.0, 1.1
    melt = (lam, Tm, 0.0, k_on - k_off)
    o = _dimers(64, 1.0, dict(k_on=k_on, epsilon=eps), kT=Tm, melt=melt)
    pb, n = _stationary(o, 1500, 64)
    _check_two_state(pb, n, 0.5 * k_on * ndt, 0.5 * (k_off + k_on - k_off) * ndt)
    assert abs(pb - 0.5) < 0.03
    # well above the melting point binding stops; well below it is the initial chemistry
    hot = _dimers(64, 1.0, dict(k_on=k_on, epsilon=eps), kT=Tm + 3.0, melt=melt)
    assert _stationary(hot, 400, 64)[0] < 0.01
    cold = _dimers(64, 1.0, dict(k_on=k_on, epsilon=eps), kT=Tm - 3.0, melt=melt)
    pb, n = _stationary(cold, 1500, 64)
    _check_two_state(pb, n, k_on * ndt, k_off * ndt)


def test_slip_bond_dimers_reach_the_two_state_fraction():
    r, a, p_on0, eps = 1.08, 1.2, 0.5, 0.5
    U = 0.5 * 100.0 * (r - 1.0) ** 2
    o = _dimers(64, r, dict(p_on0=p_on0, epsilon=eps), slip=a)
    pb, n = _stationary(o, 1500, 64)
    p = p_on0 * math.exp(-U)
    q = p_on0 * math.exp(-eps) * math.exp(a * math.sqrt(U))
    _check_two_state(pb, n, p, q)
    # the same chemistry without the modifier binds more
    plain = _dimers(64, r, dict(p_on0=p_on0, epsilon=eps))
    pb0, _ = _stationary(plain, 1500, 64)
    assert pb0 > pb + 0.05


def test_fene_as_the_bond_of_a_reaction():
    """FENE at r = R0 / sqrt(2): U = k R0^2 ln(2) / 2; acceptance e^{-U/kT}."""
    k, R0 = 1.0, 1.5
    r = R0 / math.sqrt(2.0)
    o = _dimers(64, r, dict(p_on0=0.6, epsilon=0.2, r_max=1.4), kind=BOND_FENE, bond=(k, R0))
    assert o.bond_energy_force(0, r)[0] == pytest.approx(0.5 * k * R0 * R0 * math.log(2.0), rel=1e-14)
    pb, n = _stationary(o, 1500, 64)
    _check_two_state(pb, n, 0.6 * math.exp(-0.5 * k * R0 * R0 * math.log(2.0)), 0.6 * math.exp(-0.2))
    # a FENE window reaching R0 is rejected
    with pytest.raises(OracleError) as e:
        _dimers(4, r, dict(p_on0=0.6, epsilon=0.2, r_max=1.5), kind=BOND_FENE, bond=(k, R0))
    assert e.value.code == "EINVAL"


def test_tether_as_the_bond_of_a_reaction():
    """Inside the flat region U = 0: the pair binds with P0_on itself."""
    o = _dimers(64, 1.0, dict(p_on0=0.3, epsilon=0.4, r_min=0.6, r_max=1.5), tether=TETHER)
    pb, n = _stationary(o, 1500, 64)
    _check_two_state(pb, n, 0.3, 0.3 * math.exp(-0.4))
    with pytest.raises(OracleError):
        _dimers(4, 1.0, dict(p_on0=0.3, epsilon=0.4, r_min=0.4, r_max=1.5), tether=TETHER)


def test_proposal_target_length_follows_the_bond():
    """FENE proposals take the nearest partner (its minimum is at r = 0);
    tether ones the partner nearest the middle of the flat region."""
    def one_a_two_b(make_bond, rmin, rmax):
        o = OracleSystem(3, 2, 10.0, 2)
        o.set_type(0, 1, 0.0, 0.0, 1.0)
        o.set_type(1, 1, 0.0, 0.0, 1.0)
        o.set_particles(np.array([[0.0, 0.0, 0.0], [0.7, 0.0, 0.0], [0.0, 1.05, 0.0]]), np.zeros((3, 3)),
                        [0, 1, 1])
        bt = make_bond(o)
        o.add_reaction(Reaction(0, 1, bt, rmin, rmax, p_on0=1.0, epsilon=5.0, self_avoid=0))
        o.commit()
        return o.propose(0, o.occ.copy())
    fene = one_a_two_b(lambda o: o.add_bond_type(BOND_FENE, 1.0, 1.5), 0.0, 1.4)
    assert fene[0] == 1
    teth = one_a_two_b(lambda o: o.add_tether_bond_type(**TETHER), 0.6, 1.5)
    assert teth[0] == 2                     # |1.05 - 1.0| < |0.7 - 1.0|


def test_melted_probabilities_are_checked():
    with pytest.raises(OracleError) as e:
        _dimers(2, 1.0, dict(k_on=4.0, epsilon=1.0), melt=(5.0, 1.0, 30.0, 0.0))   # 30 n dt > 1
    assert e.value.code == "ERANGE"


def test_decision_math_against_the_exact_functions():
    """The oracle's exp, log1p and tanh of the bond decisions (Cody-Waite
    exp, atanh-series log1p, tanh from exp) against the correctly rounded
    library functions: within 1, 3 ulp and 3e-16, and exact where the
    mathematics is (exp 0 = 1, log1p 0 = 0, tanh 0 = 0, tanh odd, exp of a
    sum as the product within rounding, e^(ln 2) = 2 within an ulp)."""
    from oracle.detmath import exp_det, log1p_det, tanh_det
    rng = np.random.default_rng(5)
    for x in rng.uniform(-40.0, 40.0, 20000).tolist() + rng.uniform(-1e-3, 1e-3, 2000).tolist():
        assert abs(exp_det(x) - math.exp(x)) <= math.ulp(math.exp(x))
    for z in rng.uniform(-0.999, 5.0, 20000).tolist() + rng.uniform(-1e-7, 1e-7, 2000).tolist():
        ref = math.log1p(z)
        assert abs(log1p_det(z) - ref) <= 3 * math.ulp(ref)
    for x in rng.uniform(-25.0, 25.0, 20000).tolist():
        assert abs(tanh_det(x) - math.tanh(x)) <= 3e-16
        assert tanh_det(-x) == -tanh_det(x)
    assert exp_det(0.0) == 1.0 and log1p_det(0.0) == 0.0 and tanh_det(0.0) == 0.0
    assert abs(exp_det(math.log(2.0)) - 2.0) <= math.ulp(2.0)
    assert exp_det(-800.0) == 0.0 and tanh_det(30.0) == 1.0
    for a, b in (np.round(rng.uniform(-5.0, 5.0, (200, 2)) * 2.0 ** 30) / 2.0 ** 30).tolist():   # a + b exact
        assert abs(exp_det(a + b) - exp_det(a) * exp_det(b)) <= 4 * math.ulp(exp_det(a + b))
