/* Host-only use of the C ABI from plain C99 (no GPU is touched before
 * db_commit): a two-type system of 8 particles with one harmonic A-B
 * reaction given by epsilon and p_on0; validation resolves the rates
 * (Eq. epsilon, Eq. probs) and the program prints them, then checks that an
 * invalid self_avoid value and a probability above 1 are rejected.
 * Exit status 0 on success; the resolved values go to stdout for the test
 * that builds and runs this file to compare. */
#include <math.h>
#include <stdio.h>

#include "dybond.h"

static int check(db_status st, db_status want, const char* what, const db_system* s) {
    if (st != want) {
        fprintf(stderr, "%s: status %d, expected %d (%s)\n", what, (int)st, (int)want, db_last_error(s));
        return 1;
    }
    return 0;
}

int main(void) {
    db_system* s = NULL;
    const float pos[8 * 3] = {-4, -4, -4, -2, -4, -4, 0, -4, -4, 2, -4, -4,
                              -4, 2, 2, -2, 2, 2, 0, 2, 2, 2, 2, 2};
    const uint32_t type[8] = {0, 1, 0, 1, 0, 1, 0, 1};
    uint32_t bt = 99, rx = 99;
    int bad = 0;
    bad |= check(db_create(8, 2, 10.0, 7u, 0, &s), DB_OK, "db_create", s);
    if (bad) return 1;
    bad |= check(db_set_type(s, 0, 1, 1.0, 1.0, 1.0), DB_OK, "db_set_type 0", s);
    bad |= check(db_set_type(s, 1, 1, 1.0, 1.0, 1.0), DB_OK, "db_set_type 1", s);
    bad |= check(db_set_particles(s, pos, NULL, type), DB_OK, "db_set_particles", s);
    bad |= check(db_add_bond_type(s, DB_BOND_HARMONIC, 100.0, 1.0, &bt), DB_OK, "db_add_bond_type", s);
    db_reaction_desc d;
    d.type_a = 0;
    d.type_b = 1;
    d.bond_type = bt;
    d.r_min = 0.0;
    d.r_max = 1.3;
    d.k_on = NAN;
    d.k_off = NAN;
    d.epsilon = 5.0;
    d.p_on0 = 1.0;
    d.self_avoid = 0;
    bad |= check(db_add_reaction(s, &d, &rx), DB_OK, "db_add_reaction", s);
    bad |= check(db_set_integrator(s, 0.005, 1.0, 1.0, 10, DB_KT_SETPOINT), DB_OK, "db_set_integrator", s);
    bad |= check(db_validate(s), DB_OK, "db_validate", s);
    db_reaction_desc r;
    double p_on0 = 0.0, p_off0 = 0.0;
    bad |= check(db_get_reaction(s, rx, &r, &p_on0, &p_off0), DB_OK, "db_get_reaction", s);
    printf("%u %u %.17g %.17g %.17g %.17g %.17g\n", bt, rx, r.k_on, r.k_off, r.epsilon, p_on0, p_off0);
    db_destroy(s);

    /* self_avoid must be stated as 0 or 1 (checked by db_validate), and a
     * per-sweep probability above 1 is an error, not clamped */
    for (int c = 0; c < 2; ++c) {
        s = NULL;
        bad |= check(db_create(8, 2, 10.0, 7u, 0, &s), DB_OK, "db_create", s);
        if (!s) return 1;
        bad |= check(db_set_type(s, 0, 1, 1.0, 1.0, 1.0), DB_OK, "db_set_type 0", s);
        bad |= check(db_set_type(s, 1, 1, 1.0, 1.0, 1.0), DB_OK, "db_set_type 1", s);
        bad |= check(db_set_particles(s, pos, NULL, type), DB_OK, "db_set_particles", s);
        bad |= check(db_add_bond_type(s, DB_BOND_HARMONIC, 100.0, 1.0, &bt), DB_OK, "db_add_bond_type", s);
        d.bond_type = bt;
        if (c == 0) {
            d.self_avoid = 2;
        } else {
            d.self_avoid = 1;
            d.epsilon = NAN;
            d.p_on0 = NAN;
            d.k_on = 400.0;       /* P0_on = k n dt = 400 * 10 * 0.005 = 20 > 1 */
            d.k_off = 1.0;
        }
        bad |= check(db_add_reaction(s, &d, &rx), DB_OK, "db_add_reaction", s);
        bad |= check(db_set_integrator(s, 0.005, 1.0, 1.0, 10, DB_KT_SETPOINT), DB_OK, "db_set_integrator", s);
        bad |= check(db_validate(s), c == 0 ? DB_EINVAL : DB_ERANGE, c == 0 ? "self_avoid 2" : "P0 > 1", s);
        db_destroy(s);
    }
    return bad;
}
