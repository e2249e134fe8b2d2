/*
 * dybond.h -- C ABI of the MI355X dynamic-bonding Langevin MD library.
 *
 * One time step (db_step) of a periodic, cubic, coarse-grained particle system:
 *   - Langevin integration (BAOAB) of positions and velocities;
 *   - a neighbour list with a skin, rebuilt from a cell list on the steps
 *     after which some particle has moved by more than half the skin;
 *   - WCA pair forces on all pairs plus harmonic / FENE / tether bond forces;
 *   - every `sweep_period` steps, a bonding sweep that forms and breaks
 *     dynamic bonds between partner species under per-site valence caps,
 *     consistent with the equilibrium constant K = k_on / k_off = e^eps of
 *     each reaction (paper Sec. 2.1, Eq. epsilon; sweep Sec. 2.3; acceptance
 *     Eq. pon; per-sweep probabilities Eq. probs).
 *
 * Conventions for every entry point
 *   - Host arrays passed in are borrowed for the duration of the call and
 *     copied; the library keeps no pointer to them.
 *   - Per-particle arrays are in TAG order: tag = index into the arrays given
 *     to db_set_particles.  The library may keep particles in a different
 *     order internally; no result depends on that order.
 *   - Outputs go to caller-allocated host buffers.  A buffer that is too small
 *     yields DB_ETRUNC with the required size in the count argument.
 *   - No exception and no abort crosses the ABI.  Every call returns a
 *     db_status; db_last_error() gives a message for the last failure.
 *   - A HIP runtime error makes the handle unusable (sticky DB_EDEVICE).
 *   - Results are a pure function of (initial state, parameters, seed, step).
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - Set-up calls (db_create ... db_validate) touch no GPU.  The device is
 *     first used by db_commit.
 *
 * Limits: n < 2^24 particles, at most 8 particle types, 8 bond types,
 * 8 reactions, valence <= 8 per type, <= 8 static bonds per particle.
 */
#ifndef DYBOND_H
#define DYBOND_H

#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define DB_API __attribute__((visibility("default")))
#else
#define DB_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct db_system db_system;   /* opaque; created by db_create, freed by db_destroy */

typedef enum {
    DB_OK = 0,
    DB_EINVAL = 1,     /* invalid argument or configuration */
    DB_ENOMEM = 2,     /* host or device allocation failed */
    DB_EDEVICE = 3,    /* HIP runtime error (sticky) or no usable device */
    DB_ESTATE = 4,     /* call not valid in the current state (e.g. before commit) */
    DB_ERANGE = 5,     /* a per-sweep probability k n dt exceeds 1 (Eq. probs) */
    DB_EBOND = 6,      /* a FENE bond reached r >= R0, or a force left the representable range */
    DB_ETRUNC = 7,     /* output buffer too small; required size returned */
    DB_EOVERFLOW = 8   /* more particles in one cell than the cell capacity */
} db_status;

/* Bond potentials (Sec. 2.2: the bond of a reaction supplies both the force
 * and the energy U_b of Eq. pon). */
typedef enum {
    DB_BOND_HARMONIC = 0,      /* U = k/2 (r - r0)^2 */
    DB_BOND_FENE = 1,          /* U = -k R0^2/2 ln(1 - r^2/R0^2), r0 argument = R0 */
    DB_BOND_TETHER = 2         /* registered with db_add_tether_bond_type */
} db_bond_kind;

/* Temperature T of the acceptance factor exp(-U_b / kT) of Eq. pon. */
typedef enum {
    DB_KT_SETPOINT = 0,        /* the thermostat set point kT */
    DB_KT_KINETIC = 1          /* the instantaneous kinetic temperature
                                  sum(m v^2) / (3N) at the sweep (Sec. 2.2) */
} db_kt_source;

#define DB_MAX_REACTIONS 8

/* One reaction channel alpha (Sec. 2.1, registered per type pair as in Sec. 2.6).
 * Sites of type_a bond to sites of type_b (type_a == type_b allowed) with the
 * harmonic bond type `bond_type`, whose r0 is the rest length used by the
 * proposal rule; each reaction must own a distinct bond type (bonds break by
 * their own bond type, App. A).  Candidate pairs lie in [r_min, r_max].
 * Rates: give any two of k_on, k_off, epsilon, p_on0 (NaN = not given;
 * k_on and p_on0 carry the same information since P0_on = k_on n dt).
 * self_avoid: 1 = sites of one molecule (static-bond component) never bond to
 * each other, 0 = they may; any other value is DB_EINVAL (no default, Sec. 2.4). */
typedef struct {
    uint32_t type_a, type_b, bond_type;
    double r_min, r_max;
    double k_on, k_off, epsilon, p_on0;
    int32_t self_avoid;
} db_reaction_desc;

typedef struct {
    uint64_t step;
    uint32_t n_reactions;
    uint32_t pad;
    uint64_t n_bonds[DB_MAX_REACTIONS];     /* dynamic bonds currently formed by each reaction */
    uint64_t attempts[DB_MAX_REACTIONS];    /* cumulative acceptance trials (claimed pairs) */
    uint64_t forms[DB_MAX_REACTIONS];       /* cumulative bonds formed */
    uint64_t breaks[DB_MAX_REACTIONS];      /* cumulative bonds broken */
    double bonded_fraction[DB_MAX_REACTIONS]; /* n_bonds / min(valence sum of type_a, of type_b);
                                                 homotypic: n_bonds / (valence sum / 2) */
    double largest_cluster_fraction;        /* largest component of static + dynamic bonds / N */
    double pe;                              /* potential energy (pairs + bonds) */
    double ke;                              /* kinetic energy, sum m v^2 / 2 */
    double t_kin;                           /* 2 KE / (3N) */
} db_observables;

/* Create an empty system of n particles and n_types types in a cube of side
 * box_L (positions in [-L/2, L/2)).  `seed` keys every random stream (Sec. 2.5).
 * `device` is the HIP device index used from db_commit on.  *out receives the
 * handle (caller frees with db_destroy).  No GPU work. */
DB_API db_status db_create(uint32_t n, uint32_t n_types, double box_L, uint32_t seed, int device,
                    db_system** out);

/* Free the handle and all its host and device memory.  NULL is ignored. */
DB_API void db_destroy(db_system* sys);

/* Per-type parameters (Sec. 2.1: reactive sites are particles of a type;
 * the paper's sites hold one dynamic bond, the valence generalises that to
 * a cap of `valence` dynamic bonds per site): valence (0 = not reactive,
 * at most 8), WCA sigma and epsilon (sigma_ij is the arithmetic mean,
 * eps_ij the geometric mean; sigma 0 switches WCA off for the type), and
 * mass (> 0).  Defaults: valence 0, sigma 1, eps 1, mass 1.  Host only.
 * Errors: DB_EINVAL (type out of range, bad value), DB_ESTATE (after
 * db_commit). */
DB_API db_status db_set_type(db_system* sys, uint32_t type, uint32_t valence, double wca_sigma,
                      double wca_eps, double mass);

/* Initial state of the particles (Sec. 2.1: the system whose sites react),
 * in tag order: pos3[3n] in [-L/2, L/2) (x, y, z per particle), vel3[3n]
 * and type[n] < n_types; the arrays are copied.  vel3 == NULL asks for
 * Maxwell-Boltzmann velocities at the set-point kT with zero total
 * momentum, drawn by db_validate / db_commit from the INIT random stream
 * (component c of tag t is sqrt(kT / m) g_c, g three Box-Muller normals of
 * the Philox block (0, 0, t, 0); then the mass-weighted mean velocity is
 * subtracted), so they follow the integrator's parameters whatever the
 * order of the set-up calls.  Host only.  Errors: DB_EINVAL (pos3 or type
 * NULL, a position outside the box, a type out of range), DB_ESTATE (after
 * db_commit: use db_set_state). */
DB_API db_status db_set_particles(db_system* sys, const float* pos3, const float* vel3,
                           const uint32_t* type);

/* Register a bond type (Sec. 2.2: the bond potential a reaction forms is
 * also the U_b(r) of its acceptance, Eq. pon, and its minimum is the target
 * length r0 of the proposal rule, Sec. 2.3): kind DB_BOND_HARMONIC or
 * DB_BOND_FENE, stiffness k >= 0, rest length r0 >= 0 (harmonic) or FENE
 * maximum extension R0 > 0; *id (may be NULL) receives its index.  Host
 * only.  Errors: DB_EINVAL (bad kind or value, more than 8 bond types),
 * DB_ESTATE (after db_commit). */
DB_API db_status db_add_bond_type(db_system* sys, db_bond_kind kind, double k, double r0, uint32_t* id);

/* Register a tether bond type (Sec. 2.2 names it among the bond potentials
 * a reaction may use): U(r) = U_att + U_rep with
 *   U_att = k_b exp(1/(l_c0 - r)) / (l_max - r)   for r > l_c0,
 *   U_rep = k_b exp(1/(r - l_c1)) / (r - l_min)   for r < l_c1,
 * zero for l_c1 <= r <= l_c0; defined on l_min < r < l_max (a bond outside
 * stops the run with DB_EBOND, as an overstretched FENE bond).  Requires
 * k_b >= 0 and 0 <= l_min < l_c1 < l_c0 < l_max.  Usable for static bonds
 * and as the bond of a reaction.  Errors: DB_EINVAL, DB_ESTATE. */
DB_API db_status db_add_tether_bond_type(db_system* sys, double k_b, double l_min, double l_c1, double l_c0,
                                         double l_max, uint32_t* id);

/* Add m static (never-breaking) bonds: tag_pairs[2m] and bond_types[m]
 * (copied).  Static bonds define the molecules used by self_avoid
 * (Sec. 2.4).  Host only; checked by db_validate (tags, bond types, at most
 * 8 static bonds per particle).  Errors: DB_EINVAL (NULL arrays with m > 0),
 * DB_ESTATE (after db_commit). */
DB_API db_status db_add_static_bonds(db_system* sys, const uint32_t* tag_pairs,
                              const uint32_t* bond_types, uint64_t m);

/* Register a reaction channel (Sec. 2.1, keyed by its type pair as in
 * Sec. 2.6; the descriptor is copied); *id (may be NULL) receives its
 * index.  The processing order of the reactions is redrawn at random every
 * sweep (Sec. 2.3).  Rates are closed by db_validate (Eq. epsilon, Eq.
 * probs).  Host only.  Errors: DB_EINVAL (NULL descriptor, more than 8
 * reactions), DB_ESTATE (after db_commit); the descriptor's values are
 * checked by db_validate. */
DB_API db_status db_add_reaction(db_system* sys, const db_reaction_desc* desc, uint32_t* id);

/* Rate modifiers of a reaction (Sec. 2.4; at most one per reaction, the two
 * are mutually exclusive; before db_commit).
 *
 * Melting (Eqs. gT, kT): with g(T) = [tanh(lambda (T - T_melt)) + 1] / 2,
 * each rate becomes k(T) = k_init (1 - g) + k_melt g, where k_init are the
 * reaction's own closed rates and k_on_melt, k_off_melt the melted ones;
 * the per-sweep probabilities are k(T) n dt (Eq. probs).  T is the sweep's
 * temperature: the set point (db_set_temperature changes it), or the
 * kinetic temperature in DB_KT_KINETIC mode.  Errors: DB_EINVAL (lambda < 0,
 * non-finite values, negative rates, unknown reaction, slip already set),
 * DB_ERANGE at validation when k_melt n dt exceeds 1.
 *
 * Slip bond (Eq. slip): bonds of the reaction break with
 * P_off(r) = min(1, P0_off exp(a sqrt(U_b(r) / kT))), r the bond's length at
 * the sweep and U_b the energy of the reaction's bond type; at kT = 0 the
 * factor is 1 for U_b = 0 and P_off = 1 otherwise (a > 0).  Errors:
 * DB_EINVAL (a < 0 or non-finite, unknown reaction, melting already set). */
DB_API db_status db_set_reaction_melting(db_system* sys, uint32_t reaction, double lambda, double T_melt,
                                         double k_on_melt, double k_off_melt);
DB_API db_status db_set_reaction_slip(db_system* sys, uint32_t reaction, double a);

/* Integrator and sweep trigger (Sec. 2.3: a sweep runs every n MD steps,
 * between the position update and the force; Eq. probs: P0 = k n dt):
 * time step dt > 0, Langevin thermostat kT >= 0, friction gamma >= 0,
 * sweep period n >= 1, temperature of the acceptance factor (Eq. pon,
 * Sec. 2.2).  Defaults 0.005, 1, 1, 10, DB_KT_SETPOINT.  Host only.
 * Errors: DB_EINVAL (value out of range), DB_ESTATE (after db_commit). */
DB_API db_status db_set_integrator(db_system* sys, double dt, double kT, double gamma,
                            uint32_t sweep_period, db_kt_source kt_source);

/* Change the set-point temperature kT (>= 0), before or after db_commit:
 * the thermostat's noise, the acceptance factor and the melting modifier
 * use the new value from the next step on (for temperature ramps such as
 * melting curves).  Errors: DB_EINVAL, DB_EDEVICE. */
DB_API db_status db_set_temperature(db_system* sys, double kT);

/* Particle slots per cell of the neighbour cell list.  0 (default) = chosen
 * at commit from the density and the fullest cell of the initial state (at
 * least 16); any other value in [1, 1024] is used as given.  A cell that
 * fills up during a run makes db_step return DB_EOVERFLOW. */
DB_API db_status db_set_cell_capacity(db_system* sys, uint32_t slots);

/* Neighbour list used by the force and the bonding sweep: radius
 * r_search + skin (r_search = max(WCA cutoff, r_max of every reaction)),
 * rebuilt on the device whenever some particle has moved by more than
 * skin / 2 since the last build, with at most max_neighbors entries per
 * particle.  skin < 0 selects the default 0.3; max_neighbors == 0 selects
 * max(64, 2.5 x the mean neighbour count at the system's density + 32);
 * the skin shrinks automatically when the box holds fewer than 3 cells of
 * side r_search + skin.  A particle with more neighbours makes db_step return
 * DB_EOVERFLOW. */
DB_API db_status db_set_neighbor_list(db_system* sys, double skin, uint32_t max_neighbors);

/* Schedule of the matching phase of every sweep (Sec. 2.3: greedy matching
 * of the proposals in ascending priority key).  grid_rounds (1..8, default 1)
 * local-minimum rounds run over the whole particle grid; the surviving
 * proposals are then matched by one workgroup, in LDS when there are at most
 * lds_limit of them (0..256, default 256), else in global memory.  Every
 * schedule yields the same matching; this only moves work between launches.
 * Before db_commit only (DB_ESTATE after); DB_EINVAL out of range. */
DB_API db_status db_set_matching(db_system* sys, uint32_t grid_rounds, uint32_t lds_limit);

/* Launch shape of the step kernel and the proposal kernel of the sweep:
 * threads that share one particle (1, 2, 4, 8, 16 or 32, both kernels; 0 =
 * automatic: 8 in both below 32 768 particles, 4 in the step kernel and 2
 * in the proposal kernel up to 1.5 M particles, 1 and 2 from there on) and, with 4
 * threads per particle, how many neighbour-list entries each thread loads
 * before its first gather (1, 2 or 4; 0 = automatic: 1; the next three
 * entries per thread of a longer list are loaded with the first gathers,
 * where the list has them, and any beyond in further rounds).  Any shape
 * gives the same result bit for
 * bit (forces are summed exactly); it changes only the speed.  May be
 * called before or after db_commit.  Errors: DB_EINVAL, DB_EDEVICE. */
DB_API db_status db_set_step_shape(db_system* sys, uint32_t threads_per_particle, uint32_t list_batch);
/* The shape in use (after commit; list_batch as resolved) or requested
 * (before; 0 = automatic). */
DB_API db_status db_get_step_shape(const db_system* sys, uint32_t* threads_per_particle, uint32_t* list_batch);

/* Validate the configuration and close the rate parameters of every reaction
 * (Eq. epsilon, Eq. probs) without touching a GPU.  Errors: DB_EINVAL (bad
 * or missing parameter, under-determined or inconsistent rates, box smaller
 * than 3 cells of side max(WCA cutoff, r_max)), DB_ERANGE (P0 > 1). */
DB_API db_status db_validate(db_system* sys);

/* Resolved parameters of reaction `id` after a successful db_validate:
 * resolved->k_on/k_off/epsilon filled in, *p_on0 and *p_off0 receive the
 * per-sweep probabilities P0 = k n dt.  Host only. */
DB_API db_status db_get_reaction(const db_system* sys, uint32_t id, db_reaction_desc* resolved,
                          double* p_on0, double* p_off0);

/* db_validate (rate closure, Eq. epsilon and Eq. probs, with P0 <= 1
 * required; molecules as the components of the static bonds, Sec. 2.4),
 * then allocate device memory on the handle's device, upload the state,
 * build the neighbour list and compute the initial forces.  Device memory
 * is owned by the handle until db_destroy.  Errors as db_validate, plus
 * DB_EDEVICE (no device, HIP error), DB_ENOMEM, DB_EBOND (a bond already
 * outside its range), DB_EOVERFLOW (cell or neighbour capacity),
 * DB_ESTATE (already committed). */
DB_API db_status db_commit(db_system* sys);

/* Advance n_steps Langevin MD time steps (BAOAB) with the bonding sweep of
 * Sec. 2.3 at every step s with s % sweep_period == 0, after the position
 * update and before the forces at the new positions; each sweep forms bonds
 * with P_on = P0_on exp(-U_b(r)/kT) and breaks the bonds present at its
 * start with P0_off (Eq. pon, Eq. probs).  Synchronous: returns when the
 * GPU work is done.  A system of at most 768 particles advanced by 200 or
 * more steps in one call, with the automatic launch shape, can run as a
 * batch of one (db_step_batch: one workgroup takes every step) instead of
 * the grid kernels, with the same result bit for bit: the first such call
 * times 100 steps on each and later calls keep the faster.  Errors: DB_ESTATE (not committed, invalid state),
 * DB_EDEVICE, DB_ENOMEM; DB_EBOND / DB_EOVERFLOW leave the state invalid
 * (DB_ESTATE) until db_set_state. */
DB_API db_status db_step(db_system* sys, uint64_t n_steps);

/* Launch plan of a batch (db_step_batch): the systems fall into size
 * classes, class k holding those with n <= n_max[k] that no earlier class
 * holds (the last class also takes every larger system), and every system
 * of class k runs in one workgroup of threads[k] threads.  n_max ascending;
 * threads a multiple of 64 in [64, 1024].  The plan changes only the speed:
 * results are bitwise the same under any plan. */
#define DB_BATCH_MAX_CLASSES 8
typedef struct {
    uint32_t n_classes;                        /* 1..DB_BATCH_MAX_CLASSES */
    uint32_t n_max[DB_BATCH_MAX_CLASSES];
    uint32_t threads[DB_BATCH_MAX_CLASSES];
} db_batch_plan;

/* Advance `count` committed systems on one device by n_steps each (batched
 * replicas of a parameter sweep) under the plan stored for the device
 * (db_set_batch_plan, db_batch_autotune; by default one class of
 * 1024-thread workgroups).  One workgroup per system runs all of its steps,
 * with workgroup barriers between the phases of a step and the system's own
 * device state and buffers.  All launches of a call form one HIP graph: each
 * occupied size class is a branch of its own (the classes run concurrently),
 * a chain of launches of at most 2000 steps each (a bound on how long one
 * kernel runs) that hand each system's step and buffer indices on in device
 * memory.  The result is bitwise identical to db_step(systems[k], n_steps)
 * on every system (same forces, integrator, random streams and greedy
 * matching); positions may be numbered differently inside the library,
 * which db_read_* never show.  Synchronous.  Errors: DB_EINVAL (null or
 * empty list, a system listed twice, systems on different devices),
 * DB_ESTATE (a system not committed or invalid), DB_EDEVICE; per-system
 * errors as db_step (the first in list order is returned, each system's own
 * message is in its db_last_error). */
DB_API db_status db_step_batch(db_system* const* systems, uint32_t count, uint64_t n_steps);

/* db_step_batch under an explicit plan (not stored).  Errors as
 * db_step_batch, and DB_EINVAL for a malformed plan (message in the first
 * system's db_last_error). */
DB_API db_status db_step_batch_plan(db_system* const* systems, uint32_t count, uint64_t n_steps,
                                    const db_batch_plan* plan);

/* Store the plan db_step_batch uses on HIP device `device` (NULL restores
 * the default); read it back with db_get_batch_plan.  Thread-safe.  Errors:
 * DB_EINVAL (malformed plan), DB_EDEVICE (no such device). */
DB_API db_status db_set_batch_plan(int device, const db_batch_plan* plan);
DB_API db_status db_get_batch_plan(int device, db_batch_plan* plan);

/* Autotuner of the batch launch.  Size classes are the octaves of n (n <=
 * 512, <= 1024, <= 2048, <= 4096, larger).  Starting from 1024 threads in
 * every class, each occupied class in turn, smallest first, tries 256 and
 * 512 threads, and keeps a size when the whole batch then runs at least 2 %
 * faster (device time of trial_steps steps, after one untimed trial) than
 * the plan in hand timed both just before and just after the candidate (the
 * systems evolve between trials, and with them the cost of a step).
 * Adjacent classes with the same size are merged in every plan tried and in
 * the result (each class is a concurrent branch of the batch's graph, which
 * costs time when it gains nothing), so a batch that gains from no change
 * gets the one-class default back.  Every
 * trial advances all systems by trial_steps (1..2000): since results do not
 * depend on the plan, the trials are ordinary steps of the run, and
 * *steps_done (may be NULL) receives their number.  The chosen plan is
 * stored for the device and copied to *best (may be NULL); trial_ms (may be
 * NULL) receives the time of each timed trial in order, at most trial_len
 * values.  Errors as db_step_batch. */
DB_API db_status db_batch_autotune(db_system* const* systems, uint32_t count, uint32_t trial_steps,
                                   db_batch_plan* best, uint64_t* steps_done, double* trial_ms,
                                   uint32_t trial_len);

/* One bonding sweep of Sec. 2.3 (proposal, greedy matching, acceptance by
 * Eq. pon, breaking of the bonds present at its start; reactions in the
 * random order of that step) at the current positions, with the random
 * streams keyed as for a sweep at step `step_key`; particles do not move,
 * velocities are unchanged, the step counter is unchanged.  Synchronous.
 * Errors: DB_ESTATE, DB_EDEVICE, DB_EBOND (a reaction's bond out of range
 * in the forces evaluated after the sweep). */
DB_API db_status db_sweep_frozen(db_system* sys, uint64_t step_key);

/* Replace the dynamic state: step counter, pos3[3n], vel3[3n] (tag order) and
 * the m dynamic bonds dyn_tag_pairs[2m] with their bond types (each must be
 * the bond type of a reaction whose type pair matches the two sites; valences
 * must hold).  Static bonds and parameters are unchanged. */
DB_API db_status db_set_state(db_system* sys, uint64_t step, const float* pos3, const float* vel3,
                       const uint32_t* dyn_tag_pairs, const uint32_t* dyn_bond_types,
                       uint64_t m);

/* Checkpoint and exact resume.  Every random number of the method is a pure
 * function of the seed, the step, the stream and the particle tags (Sec. 2.5:
 * counter-based Philox keyed by step and tags), so the generator has no
 * state of its own; the dynamic state is the step counter, positions, the
 * velocity the integrator carries between steps (BAOAB: the velocity after
 * the second half drift, before the next step's closing half kick), periodic
 * image counters, the dynamic bonds and the cumulative attempt / form /
 * break counters.  A system restored from a checkpoint continues bit for
 * bit as the saved one would have (positions, velocities, bonds, counters
 * and sweep events), also under db_step_batch.  db_set_state cannot promise
 * that: it takes full-step velocities, from which the carried velocity is
 * recomputed in FP32 (v - h F / m), which can differ from the saved one in
 * its last bit.
 *
 * db_save_checkpoint writes the state of a committed system into buf (the
 * caller's host memory, `cap` bytes) and sets *size to the checkpoint's size
 * (48 + 24 reactions + 36 n + 12 m bytes for m dynamic bonds); with cap <
 * *size nothing is written and DB_ETRUNC is returned (buf may then be NULL,
 * which makes cap = 0 a size query).  The bytes are self-contained: a header
 * (magic, format version, n, reactions, step, m, a fingerprint of the
 * set-up, a hash of the payload), then the counters, positions, carried
 * velocities and images in tag order, and the bond table; little-endian.
 * Errors: DB_EINVAL (size NULL, buf NULL with cap >= *size), DB_ESTATE,
 * DB_ETRUNC, DB_EDEVICE.
 *
 * db_load_checkpoint replaces the dynamic state of a committed system that
 * was set up with the same calls (n, box, seed, types, particle types,
 * static bonds, bond types, reactions, rate modifiers, integrator settings;
 * launch shapes, neighbour-list and matching settings may differ), as
 * db_set_state does: lists are rebuilt, no sweep has run on the new state
 * (db_read_sweep_events reports none), the bond reference of
 * db_bond_correlation is kept.  Also allowed on a system left invalid by an
 * error.  Errors: DB_EINVAL (buf NULL, wrong magic or version, a different
 * n, reaction count or set-up, a size that does not match the header, a
 * damaged payload, an invalid state as for db_set_state), DB_ESTATE (not
 * committed), DB_EOVERFLOW / DB_EBOND (as db_set_state), DB_EDEVICE. */
DB_API db_status db_save_checkpoint(db_system* sys, void* buf, uint64_t cap, uint64_t* size);
DB_API db_status db_load_checkpoint(db_system* sys, const void* buf, uint64_t size);

/* Positions pos3[3n] in [-L/2, L/2) (tag order, caller's buffer);
 * image3[3n] (may be NULL) receives the periodic image counters.  Before
 * db_commit: the positions given to db_set_particles (images 0), no GPU
 * touched.  Errors: DB_EINVAL (pos3 NULL), DB_ESTATE, DB_EDEVICE. */
DB_API db_status db_read_positions(db_system* sys, float* pos3, int32_t* image3);

/* Full-step velocities vel3[3n] (tag order, caller's buffer).  Before
 * db_commit: the velocities given to db_set_particles, or those db_validate
 * drew when it was given NULL (DB_ESTATE before that), no GPU touched.
 * Errors: DB_EINVAL (vel3 NULL), DB_ESTATE, DB_EDEVICE. */
DB_API db_status db_read_velocities(db_system* sys, float* vel3);

/* Forces force3[3n] (tag order, caller's buffer) at the current positions
 * and bonds: WCA on all pairs plus the static and dynamic bond forces.
 * Errors: DB_EINVAL (force3 NULL), DB_ESTATE, DB_EDEVICE, DB_EBOND. */
DB_API db_status db_read_forces(db_system* sys, float* force3);

/* The dynamic bond table after the last sweep (Sec. 2.5: the table each
 * sweep edits, read back by tag), sorted by (tag_lo, tag_hi, bond_type):
 * tag_pairs[2*cap] (tag_lo < tag_hi) and bond_types[cap], caller's
 * buffers.  *count receives the number of bonds (also on DB_ETRUNC).
 * Synchronous.  Errors: DB_EINVAL (count NULL, NULL arrays with bonds to
 * write), DB_ESTATE, DB_EDEVICE, DB_ETRUNC (cap too small). */
DB_API db_status db_read_bonds(db_system* sys, uint32_t* tag_pairs, uint32_t* bond_types,
                        uint64_t cap, uint64_t* count);

/* db_read_bonds for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * The same result and conventions as db_read_bonds, but the device staging
 * of the sorted table goes through one fixed array the library holds on
 * each device until the process ends (12 MiB: DB_NOALLOC_BONDS_MAX bonds),
 * so the call makes no device allocation and frees nothing.  Every call on
 * a device shares that device's array: calls that overlap on one device (on
 * several handles or threads at once) race and must not be made.  Errors:
 * as db_read_bonds, plus DB_ENOMEM when the system holds more than
 * DB_NOALLOC_BONDS_MAX bonds (*count receives their number; read them with
 * db_read_bonds). */
#define DB_NOALLOC_BONDS_MAX (1u << 20)
DB_API db_status db_read_bonds_noalloc(db_system* sys, uint32_t* tag_pairs, uint32_t* bond_types,
                                       uint64_t cap, uint64_t* count);

/* Bonds formed and broken by the most recent bonding sweep (Sec. 2.3: the
 * formation pass of each reaction, then the breaking of the bonds of that
 * reaction present when the sweep began), recorded on the device while the
 * sweep runs, by db_step, db_step_batch* and db_sweep_frozen alike.
 * which: DB_EVENT_FORMED or DB_EVENT_BROKEN.  tag_pairs[2*cap] (tag_lo <
 * tag_hi) and bond_types[cap] receive the events sorted by (tag_lo, tag_hi,
 * bond_type), the bond type being that of the reaction; *count receives
 * their number (also on DB_ETRUNC); *sweep_step (may be NULL) the step key of
 * that sweep, or UINT64_MAX when no sweep has run since db_commit or
 * db_set_state (then *count is 0).  A bond formed by one reaction and broken
 * by a later reaction of the same sweep cannot occur (a reaction breaks only
 * its own bonds).  Over one sweep, the dynamic bonds after it are those
 * before it minus the broken ones plus the formed ones.  Synchronous; buffers
 * are the caller's.  Errors: DB_EINVAL (count NULL, bad `which`, NULL arrays
 * when *count > 0), DB_ESTATE, DB_ETRUNC. */
enum { DB_EVENT_FORMED = 0, DB_EVENT_BROKEN = 1 };
DB_API db_status db_read_sweep_events(db_system* sys, int which, uint32_t* tag_pairs, uint32_t* bond_types,
                                      uint64_t cap, uint64_t* count, uint64_t* sweep_step);

/* Observables of the current state, computed on the device (the bond
 * statistics of Sec. 2.2 and the network measures of Sec. 4): bonds and
 * cumulative attempt / form / break counters per reaction, bonded fraction,
 * largest-cluster fraction over static + dynamic bonds, potential and
 * kinetic energy, kinetic temperature.  *out is the caller's.
 * Synchronous.  Errors: DB_EINVAL (out NULL), DB_ESTATE, DB_EDEVICE. */
DB_API db_status db_read_observables(db_system* sys, db_observables* out);

/* Network analyses of the bond network, computed on the device from the
 * current state (the quantities the paper's examples measure on assembled
 * gels, Sec. 4); synchronous; results are integer counts, the same whatever
 * the internal numbering.  Call them between db_step calls to follow a run.
 *
 * db_bond_reference remembers the current dynamic bonds (by tag);
 * db_bond_correlation then gives the number of those reference bonds and
 * how many are present now between the same two sites with the same bond
 * type (a bond that broke and formed again counts as present); the bond
 * correlation function is n_intact / n_reference.  Errors: DB_ESTATE (no
 * reference yet, or the system's state), DB_EINVAL (NULL outputs).
 *
 * db_bond_multiplicity: pairs of distinct molecules (components of the
 * static bonds) joined by m dynamic bonds, hist[m - 1] for m < len and
 * hist[len - 1] for m >= len (1 <= len <= 256); *n_pairs = bonded molecule
 * pairs, *n_intra = dynamic bonds inside one molecule (loops).
 *
 * db_cluster_sizes: clusters (components of static + dynamic bonds) of k
 * particles in hist[k - 1] for k < len, of len or more in hist[len - 1]
 * (1 <= len <= 256); *n_clusters = all clusters, single particles included.
 * Errors: DB_EINVAL (len out of range, NULL outputs), as db_read_observables. */
DB_API db_status db_bond_reference(db_system* sys);
DB_API db_status db_bond_correlation(db_system* sys, uint64_t* n_reference, uint64_t* n_intact);
DB_API db_status db_bond_multiplicity(db_system* sys, uint64_t* hist, uint32_t len, uint64_t* n_pairs,
                                      uint64_t* n_intra);
DB_API db_status db_cluster_sizes(db_system* sys, uint64_t* hist, uint32_t len, uint64_t* n_clusters);

/* Device-side read-outs, for callers that keep the data on the GPU (for
 * example in PyTorch tensors): the same values as db_read_positions,
 * db_read_velocities and db_read_forces, written as 3 n floats in tag order
 * to dev_out3, device memory of the system's device that the caller owns.
 * The work is enqueued on hip_stream (a hipStream_t; NULL = the system's own
 * stream) after everything already enqueued for the system, and the
 * system's later work waits for it; the call itself does not wait, so
 * dev_out3 is ready once hip_stream reaches this point.  Errors found by
 * this work (as the force evaluation's DB_EBOND) are reported by the next
 * call that checks.  Errors: DB_EINVAL (dev_out3 NULL), DB_ESTATE,
 * DB_EDEVICE. */
DB_API db_status db_read_positions_device(db_system* sys, float* dev_pos3, void* hip_stream);
DB_API db_status db_read_velocities_device(db_system* sys, float* dev_vel3, void* hip_stream);
DB_API db_status db_read_forces_device(db_system* sys, float* dev_force3, void* hip_stream);

/* Number of neighbour-list builds the system's steps have made since
 * db_commit (its initial build included; a build runs after every step that
 * moved some particle by more than half the skin, and after every spatial
 * renumbering; batched steps are not counted): the rebuild rate that the
 * list's cost is spread over.  Synchronous.  Errors: DB_EINVAL (builds
 * NULL), DB_ESTATE, DB_EDEVICE. */
DB_API db_status db_read_list_builds(db_system* sys, uint64_t* builds);

/* Current step counter (host mirror). */
DB_API uint64_t db_get_step(const db_system* sys);

/* Message of the last failed call on this handle ("" if none); NULL handle
 * gives the message of the last failed db_create.  Owned by the library. */
DB_API const char* db_last_error(const db_system* sys);

/* Launch the library's kernels on `hip_stream` (a hipStream_t created by the
 * caller at default priority; NULL = the library's own stream). */
DB_API db_status db_set_stream(db_system* sys, void* hip_stream);

/* Enable (1) or disable (0) HIP-event timing of every kernel launch; the
 * timing is taken on the stream the kernels are launched on and disables
 * graph replay while on. */
DB_API db_status db_kernel_timing(db_system* sys, int enable);

/* Number of timed launches and their total duration in ms of the kernel
 * named `kernel` (e.g. "k_step") since timing was enabled. */
DB_API db_status db_read_kernel_time(db_system* sys, const char* kernel, uint64_t* launches,
                              double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* DYBOND_H */
