"""Plain FP64 CPU oracle of one Langevin MD step with dynamic bonding.

TEST INFRASTRUCTURE ONLY: the product path never imports this module.

What it computes (paper sections in parentheses):

* forces: WCA on every pair closer than 2**(1/6) sigma_ij, harmonic, FENE
  and tether bonds (the bond evaluators the paper's method accepts, Sec. 2.2);
* BAOAB Langevin integration (the paper uses the integrator of its MD
  engine; BAOAB, Leimkuhler & Matthews 2013, is the reading here);
* every ``sweep_period`` steps, one bonding sweep (Sec. 2.3): for each
  reaction, in an order redrawn every sweep, proposal -> matching ->
  acceptance with P_on(r) = P0_on exp(-U_b(r)/kT) (Eq. pon) -> breaking of
  the bonds of that reaction present at the start of the sweep with
  P0_off (Eq. pon); rates from k n dt (Eq. probs) and K = e^eps
  (Eq. epsilon); optional rate modifiers per reaction (Sec. 2.4): melting,
  rates interpolated between their initial and melted values by
  g(T) = [tanh(lambda (T - T_melt)) + 1] / 2 (Eqs. gT, kT), or slip bonds,
  P_off(r) = P0_off exp(a sqrt(U_b(r)/kT)) (Eq. slip);
* the bonds each sweep formed and broke (its event lists), in the order the
  sweep makes them and read out sorted;
* observables: bond counts, bonded fraction, largest cluster, energies;
* network analyses of the kind the paper's examples measure on assembled
  gels (Sec. 4): the bond correlation function (the fraction of the bonds of
  a reference time still present), the number of molecule pairs joined by
  m dynamic bonds (bond multiplicity), and the cluster-size distribution.

Particle index == tag throughout.  All arithmetic is FP64 numpy; library
primitives used as steps: scipy's periodic k-d tree to enumerate candidate
pairs (its distances are re-evaluated exactly below), numpy sorts, and
scipy's connected components.

Readings of points the paper leaves open are listed next to the code that
implements them; the central ones are:

* valence: a site holds at most ``valence`` dynamic bonds (the paper has
  valence 1, Sec. 2.1); a site is visible to a sweep iff its occupancy is
  below its valence; a site takes part in at most one trial per reaction per
  sweep; a pair that is already bonded (any bond) is never proposed;
* matching: proposals are claimed greedily in ascending priority
  key = (w0 << 32) | tag, with w0 the first word of the MATCH stream of the
  proposer (the paper's CPU path processes candidate sites in a fresh
  pseudo-random order each sweep, Sec. 2.5);
* ties in |r - r0| go to the smaller partner tag;
* distances: positions converted to FP64, d = x_j - x_i,
  d -= rint(d / L) * L (as d * (1/L)), r = sqrt((dx*dx + dy*dy) + dz*dz),
  window r_min <= r <= r_max inclusive;
* kT = 0: the Boltzmann factor is 1 for U_b <= 0 and 0 otherwise; the slip
  factor is 1 for U_b = 0 and infinite (P_off = 1) for U_b > 0 (a > 0);
* the target length r0 of a proposal is the minimum of the reaction's bond
  potential: r0 (harmonic), 0 (FENE), the middle of the flat region
  (l_c1 + l_c0)/2 (tether);
* the temperature of the modifiers is the sweep's kT (set point, or the
  kinetic temperature in that mode), with k_B = 1.
"""

import math
from dataclasses import dataclass

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components
from scipy.spatial import cKDTree

from .detmath import exp_det, log1p_det, tanh_det
from .philox import (KIND_INIT, KIND_MATCH, KIND_OFF, KIND_ON, KIND_THERMO,
                     box_muller3, philox4x32_10, reaction_order, step_words,
                     stream_key, u53)

BOND_HARMONIC = 0
BOND_FENE = 1
BOND_TETHER = 2

WCA_RC = 2.0 ** (1.0 / 6.0)


class OracleError(Exception):
    """Invalid configuration or state; ``code`` names the library status."""

    def __init__(self, code, msg):
        super().__init__(f"{code}: {msg}")
        self.code = code


@dataclass
class Reaction:
    """One reaction channel alpha (Sec. 2.1; registered per type pair, Sec. 2.6).

    Any two of (k_on, k_off, epsilon, p_on0) fix the others, except that
    k_on and p_on0 carry the same information (Eq. probs); NaN = not given.
    ``self_avoid`` has no default (Sec. 2.4): None is rejected at commit.
    """
    type_a: int
    type_b: int
    bond_type: int
    r_min: float
    r_max: float
    k_on: float = math.nan
    k_off: float = math.nan
    epsilon: float = math.nan
    p_on0: float = math.nan
    self_avoid: object = None


def resolve_rates(k_on, k_off, epsilon, p_on0, dt, period):
    """Close the rate parameters of one reaction (Eqs. epsilon and probs).

    Returns (k_on, k_off, epsilon, P0_on, P0_off).  Order of evaluation:
    k_on from p_on0 / (n dt) if only p_on0 is given; then the missing one of
    (k_on, k_off, epsilon) from K = k_on / k_off = e^epsilon; finally
    P0 = k n dt (P0_on is p_on0 itself when given).  Over-specified inputs
    must agree to 1e-9 relative.  P0 > 1 is rejected (Eq. probs holds only
    while both probabilities stay below one).
    """
    nan = math.isnan
    ndt = float(period) * dt
    if not nan(p_on0):
        if not nan(k_on):
            if abs(p_on0 - k_on * ndt) > 1e-9 * max(1.0, abs(p_on0)):
                raise OracleError("EINVAL", "k_on and p_on0 disagree")
        else:
            k_on = p_on0 / ndt
    known = (not nan(k_on)) + (not nan(k_off)) + (not nan(epsilon))
    if known < 2:
        raise OracleError("EINVAL", "rates under-determined")
    if not nan(k_on) and not nan(k_off):
        if not nan(epsilon):
            if k_off <= 0.0 or k_on <= 0.0 or \
                    abs(epsilon - math.log(k_on / k_off)) > 1e-9 * max(1.0, abs(epsilon)):
                raise OracleError("EINVAL", "k_on, k_off and epsilon disagree")
        elif k_on > 0.0 and k_off > 0.0:
            epsilon = math.log(k_on / k_off)
    elif not nan(k_on):
        k_off = k_on * math.exp(-epsilon)
    else:
        k_on = k_off * math.exp(epsilon)
    p_on = p_on0 if not nan(p_on0) else k_on * ndt
    p_off = k_off * ndt
    for v in (k_on, k_off, p_on, p_off):
        if not math.isfinite(v) or v < 0.0:
            raise OracleError("ERANGE", "negative or non-finite rate")
    if p_on > 1.0 or p_off > 1.0:
        raise OracleError("ERANGE", "P0 = k n dt exceeds 1")
    return k_on, k_off, epsilon, p_on, p_off


def melt_switch(lam, T_melt, T):
    """g(T) = [tanh(lambda (T - T_melt)) + 1] / 2 (Eq. gT)."""
    return 0.5 * (tanh_det(lam * (T - T_melt)) + 1.0)


def melted_probabilities(p_on_init, p_off_init, p_on_melt, p_off_melt, lam, T_melt, T):
    """Per-sweep probabilities at temperature T with the melting modifier:
    each rate is k_init (1 - g) + k_melt g (Eq. kT), and P0 = k n dt
    (Eq. probs) is linear in k, so the same mix applies to the P0."""
    g = melt_switch(lam, T_melt, T)
    return p_on_init * (1.0 - g) + p_on_melt * g, p_off_init * (1.0 - g) + p_off_melt * g


def slip_probability(p_off0, a, U, kT):
    """P_off(r) = P0_off exp(a sqrt(U_b(r) / kT)) (Eq. slip), capped at 1;
    for kT = 0 the factor is 1 when U_b = 0 and unbounded otherwise."""
    if kT > 0.0:
        return min(1.0, p_off0 * exp_det(a * math.sqrt(U / kT)))
    if U > 0.0 and a > 0.0:
        return 1.0
    return p_off0


class OracleSystem:
    """A periodic cubic box of N particles with static and dynamic bonds."""

    def __init__(self, n, n_types, box_L, seed):
        self.n = int(n)
        self.n_types = int(n_types)
        self.L = float(box_L)
        self.invL = 1.0 / self.L
        self.seed = int(seed) & 0xFFFFFFFF
        self.valence = np.zeros(n_types, dtype=np.int64)
        self.sigma = np.ones(n_types)
        self.eps = np.ones(n_types)
        self.mass = np.ones(n_types)
        self.bond_kinds = []      # (kind, k, r0 or R0[, l_min, l_c1, l_c0, l_max])
        self.reactions = []
        self.modifiers = {}       # reaction -> ("melt", lam, T_melt, k_on_melt, k_off_melt) | ("slip", a)
        self.static = []          # (i, j, bond_type)
        self.x = None
        self.v = None
        self.types = None
        self.dt, self.kT, self.gamma, self.period = 0.005, 1.0, 1.0, 10
        self.kinetic_T = False
        self.step_count = 0
        self.committed = False
        self.events = None        # set to a list to record (s, a, kind, i, j)
        self.last_sweep = None    # step key and the bonds formed / broken by the last sweep

    # ---------------------------------------------------------------- setup
    def set_type(self, t, valence, sigma, eps, mass):
        self.valence[t] = valence
        self.sigma[t] = sigma
        self.eps[t] = eps
        self.mass[t] = mass

    def add_bond_type(self, kind, k, r0):
        self.bond_kinds.append((int(kind), float(k), float(r0)))
        return len(self.bond_kinds) - 1

    def add_tether_bond_type(self, k_b, l_min, l_c1, l_c0, l_max):
        """Tether bond: U = U_rep + U_att with
        U_att(r) = k_b exp(1/(l_c0 - r)) / (l_max - r) for r > l_c0,
        U_rep(r) = k_b exp(1/(r - l_c1)) / (r - l_min) for r < l_c1,
        zero between l_c1 and l_c0; defined on l_min < r < l_max."""
        self.bond_kinds.append((BOND_TETHER, float(k_b), 0.5 * (l_c1 + l_c0),
                                float(l_min), float(l_c1), float(l_c0), float(l_max)))
        return len(self.bond_kinds) - 1

    def set_melting(self, a, lam, T_melt, k_on_melt, k_off_melt):
        self.modifiers[a] = ("melt", float(lam), float(T_melt), float(k_on_melt), float(k_off_melt))

    def set_slip(self, a, coeff):
        self.modifiers[a] = ("slip", float(coeff))

    def set_temperature(self, kT):
        self.kT = float(kT)

    def set_particles(self, pos, vel, types):
        """Initial state; ``vel=None`` asks for Maxwell-Boltzmann velocities,
        drawn at commit (see ``maxwell_boltzmann_velocities``)."""
        self.x = np.array(pos, dtype=np.float64).reshape(self.n, 3)
        self.v = None if vel is None else np.array(vel, dtype=np.float64).reshape(self.n, 3)
        self.types = np.array(types, dtype=np.int64).reshape(self.n)
        self.img = np.zeros((self.n, 3), dtype=np.int64)

    def maxwell_boltzmann_velocities(self):
        """Velocities of the set-point temperature with zero total momentum.

        Each Cartesian component of particle t is sqrt(kT / m) g, with three
        standard normals g from one block of the INIT stream (counter
        (0, 0, t, 0), Box-Muller as for the thermal noise); then the
        mass-weighted mean velocity sum_t m_t v_t / sum_t m_t is subtracted,
        so the total momentum is zero.  The velocities follow the
        equilibrium distribution of the thermostat the paper's MD runs under
        (Sec. 2.2 uses the kinetic temperature of these velocities).
        """
        k0, k1 = stream_key(self.seed, KIND_INIT)
        w = philox4x32_10(0, 0, np.arange(self.n, dtype=np.uint64), 0, k0, k1)
        g = np.stack(box_muller3(*w), axis=1)
        m = self.mass[self.types][:, None]
        v = np.sqrt(self.kT / m) * g
        return v - np.sum(m * v, axis=0) / np.sum(m)

    def add_static_bonds(self, pairs, bond_types):
        pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
        bond_types = np.asarray(bond_types, dtype=np.int64).reshape(-1)
        for (i, j), b in zip(pairs, bond_types):
            self.static.append((int(i), int(j), int(b)))

    def add_reaction(self, rx):
        self.reactions.append(rx)
        return len(self.reactions) - 1

    def set_integrator(self, dt, kT, gamma, sweep_period, kinetic_T=False):
        self.dt, self.kT, self.gamma = float(dt), float(kT), float(gamma)
        self.period = int(sweep_period)
        self.kinetic_T = bool(kinetic_T)

    def commit(self):
        """Validate, close the rate parameters and derive molecule ids."""
        if self.x is None:
            raise OracleError("ESTATE", "particles not set")
        if self.v is None:
            self.v = self.maxwell_boltzmann_velocities()
        self.rates = []
        seen_bt = set()
        for rx in self.reactions:
            if rx.self_avoid not in (0, 1, False, True):
                raise OracleError("EINVAL", "self_avoid must be stated")
            if not (0 <= rx.type_a < self.n_types and 0 <= rx.type_b < self.n_types):
                raise OracleError("EINVAL", "reaction type out of range")
            if not (0 <= rx.bond_type < len(self.bond_kinds)):
                raise OracleError("EINVAL", "bond type out of range")
            bk = self.bond_kinds[rx.bond_type]
            if bk[0] == BOND_FENE and not rx.r_max < bk[2]:
                raise OracleError("EINVAL", "FENE reaction window must end below R0")
            if bk[0] == BOND_TETHER and not (bk[3] < rx.r_min and rx.r_max < bk[6]):
                raise OracleError("EINVAL", "tether reaction window must lie inside (l_min, l_max)")
            if rx.bond_type in seen_bt:
                raise OracleError("EINVAL", "each reaction owns its bond type")
            seen_bt.add(rx.bond_type)
            if not (0.0 <= rx.r_min < rx.r_max):
                raise OracleError("EINVAL", "bad window")
            self.rates.append(resolve_rates(rx.k_on, rx.k_off, rx.epsilon, rx.p_on0,
                                            self.dt, self.period))
        self.melt_p = {}
        for a, mod in self.modifiers.items():
            if not 0 <= a < len(self.reactions):
                raise OracleError("EINVAL", "modifier of an unknown reaction")
            if mod[0] == "melt":
                _, lam, T_melt, k_on_m, k_off_m = mod
                ndt = float(self.period) * self.dt
                pm_on, pm_off = k_on_m * ndt, k_off_m * ndt
                if not (lam >= 0.0 and math.isfinite(T_melt) and 0.0 <= pm_on <= 1.0 and 0.0 <= pm_off <= 1.0):
                    raise OracleError("ERANGE", "melted rates out of range")
                self.melt_p[a] = (pm_on, pm_off, lam, T_melt)
            elif not mod[1] >= 0.0:
                raise OracleError("EINVAL", "slip coefficient must be >= 0")
        # sigma_ij / eps_ij tables (arithmetic / geometric means)
        self.sig_ij = 0.5 * (self.sigma[:, None] + self.sigma[None, :])
        self.eps_ij = np.sqrt(self.eps[:, None] * self.eps[None, :])
        active = (self.sig_ij > 0) & (self.eps_ij > 0)
        self.rc_max = float(np.max(np.where(active, WCA_RC * self.sig_ij, 0.0)))
        # molecule ids: components of the static bond graph (Sec. 2.4)
        self.mol = self._components(self.static_pairs_array())
        # dynamic bonds: pair (lo, hi) -> reaction index
        self.dyn = {}
        self.occ = np.zeros(self.n, dtype=np.int64)
        self.counters = np.zeros((len(self.reactions), 3), dtype=np.int64)  # attempts, forms, breaks
        self.static_set = {(min(i, j), max(i, j)) for i, j, _ in self.static}
        self.committed = True
        self._check_fene(self.x)
        self.F, self.PE = self.forces(self.x)

    # ------------------------------------------------------------ geometry
    def delta(self, xi, xj):
        """Minimum-image displacement x_j - x_i in FP64 (reading A4)."""
        d = xj - xi
        k = np.rint(d * self.invL)
        return d - k * self.L

    @staticmethod
    def norm(d):
        r2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
        return np.sqrt(r2)

    def pairs_within(self, x, cutoff):
        """All pairs i < j with exact distance r <= cutoff.

        Candidates come from a periodic k-d tree queried slightly beyond the
        cutoff; the distance is then recomputed with ``delta``/``norm``.
        Returns (i, j, d, r) with d = minimum-image x_j - x_i.
        """
        y = np.mod(x + 0.5 * self.L, self.L)
        y[y >= self.L] = 0.0
        tree = cKDTree(y, boxsize=self.L)
        p = tree.query_pairs(cutoff * (1.0 + 1e-9) + 1e-9, output_type="ndarray")
        if len(p) == 0:
            e = np.zeros(0, dtype=np.int64)
            return e, e, np.zeros((0, 3)), np.zeros(0)
        i, j = p[:, 0].astype(np.int64), p[:, 1].astype(np.int64)
        sw = i > j
        i[sw], j[sw] = j[sw], i[sw].copy()
        d = self.delta(x[i], x[j])
        r = self.norm(d)
        keep = r <= cutoff
        return i[keep], j[keep], d[keep], r[keep]

    # -------------------------------------------------------------- forces
    def bond_energy_force(self, bt, r):
        """U(r) and dU/dr of bond type ``bt`` (harmonic, FENE or tether)."""
        kind, k, r0 = self.bond_kinds[bt][:3]
        if kind == BOND_HARMONIC:
            d = r - r0
            return (0.5 * k) * (d * d), k * d
        if kind == BOND_FENE:
            x2 = (r * r) / (r0 * r0)
            return -0.5 * k * r0 * r0 * log1p_det(-x2), k * r / (1.0 - x2)
        l_min, l_c1, l_c0, l_max = self.bond_kinds[bt][3:]
        U, dU = 0.0, 0.0
        if r > l_c0:                       # attraction beyond l_c0
            e = exp_det(1.0 / (l_c0 - r))
            U += k * e / (l_max - r)
            dU += k * e * (1.0 / ((l_c0 - r) ** 2 * (l_max - r)) + 1.0 / (l_max - r) ** 2)
        if r < l_c1:                       # repulsion below l_c1
            e = exp_det(1.0 / (r - l_c1))
            U += k * e / (r - l_min)
            dU -= k * e * (1.0 / ((r - l_c1) ** 2 * (r - l_min)) + 1.0 / (r - l_min) ** 2)
        return U, dU

    def bond_in_domain(self, bt, r):
        """FENE needs r < R0, tether l_min < r < l_max."""
        kind = self.bond_kinds[bt][0]
        if kind == BOND_FENE:
            return r < self.bond_kinds[bt][2]
        if kind == BOND_TETHER:
            return self.bond_kinds[bt][3] < r < self.bond_kinds[bt][6]
        return True

    def _check_fene(self, x):
        for i, j, b in self.static:
            r = self.norm(self.delta(x[i], x[j]))
            if not self.bond_in_domain(b, r):
                raise OracleError("EBOND", f"bond {i}-{j} outside its range r={r}")

    def forces(self, x):
        """Total force on every particle and total potential energy (FP64)."""
        F = np.zeros((self.n, 3))
        PE = 0.0
        if self.rc_max > 0:
            i, j, d, r = self.pairs_within(x, self.rc_max)
            ti, tj = self.types[i], self.types[j]
            sig, eps = self.sig_ij[ti, tj], self.eps_ij[ti, tj]
            m = (r < WCA_RC * sig) & (sig > 0) & (eps > 0)
            i, j, d, r, sig, eps = i[m], j[m], d[m], r[m], sig[m], eps[m]
            sr6 = (sig / r) ** 6
            PE += float(np.sum(4.0 * eps * (sr6 * sr6 - sr6) + eps))
            dudr = 4.0 * eps * (-12.0 * sr6 * sr6 + 6.0 * sr6) / r
            fi = (dudr / r)[:, None] * d          # force on i; d points i -> j
            np.add.at(F, i, fi)
            np.add.at(F, j, -fi)
        for i, j, bt in self.all_bonds():
            d = self.delta(x[i], x[j])
            r = float(self.norm(d))
            if not self.bond_in_domain(bt, r):
                raise OracleError("EBOND", f"bond {i}-{j} outside its range")
            U, dudr = self.bond_energy_force(bt, r)
            PE += float(U)
            fi = (dudr / r) * d
            F[i] += fi
            F[j] -= fi
        return F, PE

    def force_contribution_norms(self, x, counts=False):
        """Per particle, the sum over its interactions (WCA pairs inside the
        cutoff, static and dynamic bonds) of |F_ij|: the scale of the force
        tolerances, which a net force that cancels to near zero would not
        give.  With ``counts`` also the number of those interactions."""
        S = np.zeros(self.n)
        C = np.zeros(self.n, dtype=np.int64)
        if self.rc_max > 0:
            i, j, d, r = self.pairs_within(x, self.rc_max)
            ti, tj = self.types[i], self.types[j]
            sig, eps = self.sig_ij[ti, tj], self.eps_ij[ti, tj]
            m = (r < WCA_RC * sig) & (sig > 0) & (eps > 0)
            i, j, r, sig, eps = i[m], j[m], r[m], sig[m], eps[m]
            sr6 = (sig / r) ** 6
            f = np.abs(4.0 * eps * (-12.0 * sr6 * sr6 + 6.0 * sr6) / r)
            np.add.at(S, i, f)
            np.add.at(S, j, f)
            np.add.at(C, i, 1)
            np.add.at(C, j, 1)
        for i, j, bt in self.all_bonds():
            r = float(self.norm(self.delta(x[i], x[j])))
            _, dudr = self.bond_energy_force(bt, r)
            S[i] += abs(dudr)
            S[j] += abs(dudr)
            C[i] += 1
            C[j] += 1
        return (S, C) if counts else S

    def all_bonds(self):
        """Static bonds followed by dynamic bonds, as (i, j, bond_type)."""
        out = list(self.static)
        for (i, j), a in sorted(self.dyn.items()):
            out.append((i, j, self.reactions[a].bond_type))
        return out

    def static_pairs_array(self):
        if not self.static:
            return np.zeros((0, 2), dtype=np.int64)
        return np.array([(i, j) for i, j, _ in self.static], dtype=np.int64)

    def _components(self, pairs):
        if len(pairs) == 0:
            return np.arange(self.n)
        g = coo_matrix((np.ones(len(pairs)), (pairs[:, 0], pairs[:, 1])),
                       shape=(self.n, self.n))
        _, lab = connected_components(g, directed=False)
        return lab

    # ----------------------------------------------------------- integrate
    def thermo_noise(self, s):
        """Three standard normals per particle from the THERMO stream at step s."""
        k0, k1 = stream_key(self.seed, KIND_THERMO)
        s_lo, s_hi = step_words(s)
        tags = np.arange(self.n, dtype=np.uint64)
        w = philox4x32_10(s_lo, s_hi, tags, 0, k0, k1)
        g0, g1, g2 = box_muller3(*w)
        return np.stack([g0, g1, g2], axis=1)

    def step(self, nsteps=1):
        """BAOAB steps; a sweep follows the position update of step s when
        s % period == 0, before the forces at the new positions."""
        m = self.mass[self.types][:, None]
        h = 0.5 * self.dt
        c1 = math.exp(-self.gamma * self.dt)
        c2 = math.sqrt(1.0 - c1 * c1)
        sd = np.sqrt(self.kT / m)
        for _ in range(int(nsteps)):
            s = self.step_count + 1
            self.v = self.v + h * self.F / m          # B
            self.x = self.x + h * self.v              # A
            self.v = c1 * self.v + c2 * sd * self.thermo_noise(s)   # O
            self.x = self.x + h * self.v              # A
            shift = np.floor((self.x + 0.5 * self.L) * self.invL)
            self.x = self.x - shift * self.L
            self.img += shift.astype(np.int64)
            if s % self.period == 0:
                self.sweep(s)
            self.F, self.PE = self.forces(self.x)
            self.v = self.v + h * self.F / m          # B
            self.step_count = s

    # -------------------------------------------------------------- sweep
    def current_kT(self):
        """Temperature of the acceptance factor (Eq. pon): the thermostat's
        set point, or in kinetic mode the instantaneous kinetic temperature
        of Sec. 2.2, sum_i m_i |v_i|^2 / (3 N) with k_B = 1 and 3N degrees of
        freedom (the velocities as they stand when the sweep runs)."""
        if not self.kinetic_T:
            return self.kT
        m = self.mass[self.types]
        return float(np.sum(m[:, None] * self.v * self.v)) / (3.0 * self.n)

    def bonded(self, i, j):
        p = (min(i, j), max(i, j))
        return p in self.dyn or p in self.static_set

    def sweep(self, s):
        """One bonding sweep with step key s (Sec. 2.3)."""
        kT = self.current_kT()
        start = dict(self.dyn)          # table at the start of the sweep
        self.last_sweep = {"step": s, "formed": [], "broken": []}
        for a in reaction_order(self.seed, s, len(self.reactions)):
            self._react(a, s, start, kT)

    def propose(self, a, occ0):
        """Proposal phase of reaction a: proposer -> partner (dict).

        Every site of the reaction's types whose occupancy (as it stood before
        this reaction) is below its valence scans its neighbours and keeps the
        free partner of the complementary type in [r_min, r_max] minimising
        |r - r0|, smaller tag on ties; never itself, never an already bonded
        partner, never one of its own molecule when self_avoid is set.
        """
        rx = self.reactions[a]
        kind = self.bond_kinds[rx.bond_type][0]
        r0 = 0.0 if kind == BOND_FENE else self.bond_kinds[rx.bond_type][2]
        i, j, _, r = self.pairs_within(self.x, rx.r_max)
        src = np.concatenate([i, j])
        dst = np.concatenate([j, i])
        rr = np.concatenate([r, r])
        ts, td = self.types[src], self.types[dst]
        ok = ((ts == rx.type_a) & (td == rx.type_b)) | ((ts == rx.type_b) & (td == rx.type_a))
        ok &= (occ0[src] < self.valence[ts]) & (occ0[dst] < self.valence[td])
        ok &= (rr >= rx.r_min) & (rr <= rx.r_max)
        if rx.self_avoid:
            ok &= self.mol[src] != self.mol[dst]
        src, dst, rr = src[ok], dst[ok], rr[ok]
        if len(src) and (self.dyn or self.static_set):
            lo, hi = np.minimum(src, dst), np.maximum(src, dst)
            keys = lo * self.n + hi
            bonded = np.array([p[0] * self.n + p[1] for p in
                               list(self.dyn.keys()) + list(self.static_set)], dtype=np.int64)
            keep = ~np.isin(keys, bonded)
            src, dst, rr = src[keep], dst[keep], rr[keep]
        score = np.abs(rr - r0)
        order = np.lexsort((dst, score, src))       # by src, then score, then tag
        src, dst = src[order], dst[order]
        first = np.ones(len(src), dtype=bool)
        first[1:] = src[1:] != src[:-1]
        return dict(zip(src[first].tolist(), dst[first].tolist()))

    def match_keys(self, a, s, proposers):
        k0, k1 = stream_key(self.seed, KIND_MATCH, a)
        s_lo, s_hi = step_words(s)
        tags = np.asarray(proposers, dtype=np.uint64)
        w0 = philox4x32_10(s_lo, s_hi, tags, 0, k0, k1)[0]
        return (w0 << np.uint64(32)) | tags

    def match(self, a, s, props):
        """Greedy matching in ascending priority key: a proposal is claimed
        when neither of its two sites has been claimed by an earlier one."""
        proposers = sorted(props)
        keys = self.match_keys(a, s, proposers)
        claimed = set()
        pairs = []
        for idx in np.argsort(keys, kind="stable"):
            i = proposers[idx]
            j = props[i]
            if i in claimed or j in claimed:
                continue
            claimed.add(i)
            claimed.add(j)
            pairs.append((i, j))
        return pairs

    def acceptance_probability(self, p_on0, U, kT):
        """P_on = P0_on exp(-U_b/kT) (Eq. pon), capped at 1; kT = 0 reading."""
        if kT > 0.0:
            return min(1.0, p_on0 * exp_det(-U / kT))
        return p_on0 if U <= 0.0 else 0.0

    def pair_u53(self, kind, a, s, i, j):
        k0, k1 = stream_key(self.seed, kind, a)
        s_lo, s_hi = step_words(s)
        w = philox4x32_10(s_lo, s_hi, min(i, j), max(i, j), k0, k1)
        return float(u53(w[0], w[1]))

    def _react(self, a, s, start, kT):
        rx = self.reactions[a]
        _, _, _, p_on, p_off = self.rates[a]
        if a in self.melt_p:
            pm_on, pm_off, lam, T_melt = self.melt_p[a]
            p_on, p_off = melted_probabilities(p_on, p_off, pm_on, pm_off, lam, T_melt, kT)
        slip = self.modifiers[a][1] if self.modifiers.get(a, ("",))[0] == "slip" else None
        occ0 = self.occ.copy()
        props = self.propose(a, occ0)
        pairs = self.match(a, s, props)
        for i, j in pairs:                                  # acceptance
            self.counters[a, 0] += 1
            r = float(self.norm(self.delta(self.x[i], self.x[j])))
            U, _ = self.bond_energy_force(rx.bond_type, r)
            P = self.acceptance_probability(p_on, float(U), kT)
            if self.pair_u53(KIND_ON, a, s, i, j) < P:
                self.dyn[(min(i, j), max(i, j))] = a
                self.occ[i] += 1
                self.occ[j] += 1
                self.counters[a, 1] += 1
                self.last_sweep["formed"].append((min(i, j), max(i, j), rx.bond_type))
                if self.events is not None:
                    self.events.append((s, a, "form", min(i, j), max(i, j), r))
        for (i, j), b in sorted(start.items()):             # breaking
            if b != a:
                continue
            q = p_off
            if slip is not None:
                r = float(self.norm(self.delta(self.x[i], self.x[j])))
                U, _ = self.bond_energy_force(rx.bond_type, r)
                q = slip_probability(p_off, slip, float(U), kT)
            if self.pair_u53(KIND_OFF, a, s, i, j) < q:
                del self.dyn[(i, j)]
                self.occ[i] -= 1
                self.occ[j] -= 1
                self.counters[a, 2] += 1
                self.last_sweep["broken"].append((i, j, rx.bond_type))
                if self.events is not None:
                    self.events.append((s, a, "break", i, j, None))

    def sweep_frozen(self, step_key):
        """One sweep at the current positions without moving particles."""
        self.sweep(int(step_key))
        self.F, self.PE = self.forces(self.x)

    # ---------------------------------------------------------- state I/O
    def set_state(self, step, pos, vel, dyn_pairs=(), dyn_bond_types=()):
        self.step_count = int(step)
        self.x = np.array(pos, dtype=np.float64).reshape(self.n, 3)
        self.v = np.array(vel, dtype=np.float64).reshape(self.n, 3)
        bt2rx = {rx.bond_type: a for a, rx in enumerate(self.reactions)}
        self.dyn = {}
        self.occ = np.zeros(self.n, dtype=np.int64)
        for (i, j), b in zip(np.asarray(dyn_pairs, dtype=np.int64).reshape(-1, 2),
                             np.asarray(dyn_bond_types, dtype=np.int64).reshape(-1)):
            i, j = int(min(i, j)), int(max(i, j))
            self.dyn[(i, j)] = bt2rx[int(b)]
            self.occ[i] += 1
            self.occ[j] += 1
        if np.any(self.occ > self.valence[self.types]):
            raise OracleError("EINVAL", "state exceeds a valence")
        self.last_sweep = None
        self.F, self.PE = self.forces(self.x)

    def bonds(self):
        """Dynamic bonds as an (m, 3) array (tag_lo, tag_hi, bond_type), sorted."""
        rows = [(i, j, self.reactions[a].bond_type) for (i, j), a in self.dyn.items()]
        rows.sort()
        return np.array(rows, dtype=np.int64).reshape(-1, 3)

    def sweep_events(self, which):
        """Bonds formed (which = "formed") or broken ("broken") by the last
        sweep as a sorted (m, 3) array (tag_lo, tag_hi, bond_type), and that
        sweep's step key (None when no sweep has run since the state was set).
        A reaction forms bonds, then breaks its own bonds present at the start
        of the sweep (Sec. 2.3)."""
        if self.last_sweep is None:
            return np.zeros((0, 3), dtype=np.int64), None
        rows = sorted(self.last_sweep[which])
        return np.array(rows, dtype=np.int64).reshape(-1, 3), self.last_sweep["step"]

    # ------------------------------------------------------------ analyses
    def bond_reference(self):
        """Remember the current dynamic bonds (pair -> reaction)."""
        self.ref_bonds = dict(self.dyn)

    def bond_correlation(self):
        """(reference bonds, those present now between the same two sites
        with the same reaction); a bond that broke and formed again counts
        as present."""
        ref = self.ref_bonds
        return len(ref), sum(1 for pair, a in ref.items() if self.dyn.get(pair) == a)

    def bond_multiplicity(self, length):
        """Histogram of the number of dynamic bonds joining each pair of
        distinct molecules: hist[m - 1] for m < length, hist[length - 1] for
        m >= length; also the number of bonded molecule pairs and of bonds
        within one molecule."""
        per_pair = {}
        intra = 0
        for (i, j) in self.dyn:
            a, b = int(self.mol[i]), int(self.mol[j])
            if a == b:
                intra += 1
                continue
            key = (min(a, b), max(a, b))
            per_pair[key] = per_pair.get(key, 0) + 1
        hist = np.zeros(length, dtype=np.int64)
        for m in per_pair.values():
            hist[min(m, length) - 1] += 1
        return hist, len(per_pair), intra

    def cluster_sizes(self, length):
        """Histogram of cluster sizes (components of static + dynamic bonds):
        hist[k - 1] clusters of k particles for k < length, hist[length - 1]
        clusters of length or more; also the number of clusters."""
        pairs = [(i, j) for i, j, _ in self.static] + list(self.dyn.keys())
        lab = self._components(np.array(pairs, dtype=np.int64).reshape(-1, 2))
        sizes = np.bincount(lab)
        sizes = sizes[sizes > 0]
        hist = np.zeros(length, dtype=np.int64)
        for k in sizes:
            hist[min(int(k), length) - 1] += 1
        return hist, len(sizes)

    def observables(self):
        m = self.mass[self.types]
        KE = 0.5 * float(np.sum(m[:, None] * self.v * self.v))
        out = {"KE": KE, "T_kin": 2.0 * KE / (3.0 * self.n), "PE": self.PE}
        R = len(self.reactions)
        nb = np.zeros(R, dtype=np.int64)
        for a in self.dyn.values():
            nb[a] += 1
        frac = np.zeros(R)
        for a, rx in enumerate(self.reactions):
            cap_a = float(np.sum(self.valence[self.types][self.types == rx.type_a]))
            cap_b = float(np.sum(self.valence[self.types][self.types == rx.type_b]))
            denom = cap_a / 2.0 if rx.type_a == rx.type_b else min(cap_a, cap_b)
            frac[a] = nb[a] / denom if denom > 0 else 0.0
        out["n_bonds"] = nb
        out["bonded_fraction"] = frac
        out["attempts"] = self.counters[:, 0].copy()
        out["forms"] = self.counters[:, 1].copy()
        out["breaks"] = self.counters[:, 2].copy()
        pairs = [(i, j) for i, j, _ in self.static] + list(self.dyn.keys())
        lab = self._components(np.array(pairs, dtype=np.int64).reshape(-1, 2))
        out["largest_cluster_fraction"] = float(np.max(np.bincount(lab))) / self.n
        return out
