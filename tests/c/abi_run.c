/* A whole run through the C ABI from plain C99, with no Python and no
 * PyTorch in the process: the system described in the text file argv[1] is
 * set up, committed to device 0, advanced argv[3] steps with db_step (in
 * calls of at most argv[4] steps), and its bonds, positions and velocities
 * are written in binary to argv[2] for the test that compares them with a
 * run of the same system driven from Python.
 *
 * Input (whitespace separated; floats in C99 hex notation where exactness
 * matters, "nan" for rates not given):
 *   n ntypes L seed
 *   ntypes x { valence sigma eps mass }
 *   nbt, nbt x { kind k r0 }                      (harmonic or FENE)
 *   nstatic, nstatic x { tag_i tag_j bond_type }
 *   nrx, nrx x { type_a type_b bond_type r_min r_max k_on k_off epsilon p_on0 self_avoid }
 *   dt kT gamma period
 *   n x { x y z vx vy vz type }
 * Output: uint64 step, uint64 nbonds, nbonds x {uint32 tag_lo, tag_hi, type},
 * then n x 3 float positions and n x 3 float velocities (tag order). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "dybond.h"

#define CHECK(call)                                                                         \
    do {                                                                                    \
        db_status st_ = (call);                                                             \
        if (st_ != DB_OK) {                                                                 \
            fprintf(stderr, "%s failed: status %d (%s)\n", #call, (int)st_, db_last_error(s)); \
            return 1;                                                                       \
        }                                                                                   \
    } while (0)

static int rd(FILE* f, const char* fmt, void* p) { return fscanf(f, fmt, p) == 1 ? 0 : 1; }

int main(int argc, char** argv) {
    if (argc != 5) {
        fprintf(stderr, "usage: abi_run input output steps chunk\n");
        return 2;
    }
    FILE* f = fopen(argv[1], "r");
    if (!f) return 2;
    unsigned n, ntypes, seed;
    double L;
    if (fscanf(f, "%u %u %lf %u", &n, &ntypes, &L, &seed) != 4) return 2;
    db_system* s = NULL;
    CHECK(db_create(n, ntypes, L, seed, 0, &s));
    for (unsigned t = 0; t < ntypes; ++t) {
        unsigned val;
        double sig, eps, m;
        if (fscanf(f, "%u %lf %lf %lf", &val, &sig, &eps, &m) != 4) return 2;
        CHECK(db_set_type(s, t, val, sig, eps, m));
    }
    unsigned nbt;
    if (rd(f, "%u", &nbt)) return 2;
    for (unsigned b = 0; b < nbt; ++b) {
        int kind;
        double k, r0;
        uint32_t id;
        if (fscanf(f, "%d %lf %lf", &kind, &k, &r0) != 3) return 2;
        CHECK(db_add_bond_type(s, (db_bond_kind)kind, k, r0, &id));
    }
    unsigned nstat;
    if (rd(f, "%u", &nstat)) return 2;
    uint32_t* pairs = malloc(sizeof(uint32_t) * 2 * (nstat + 1));
    uint32_t* stype = malloc(sizeof(uint32_t) * (nstat + 1));
    for (unsigned k = 0; k < nstat; ++k)
        if (fscanf(f, "%u %u %u", &pairs[2 * k], &pairs[2 * k + 1], &stype[k]) != 3) return 2;
    if (nstat) CHECK(db_add_static_bonds(s, pairs, stype, nstat));
    unsigned nrx;
    if (rd(f, "%u", &nrx)) return 2;
    for (unsigned a = 0; a < nrx; ++a) {
        db_reaction_desc d;
        uint32_t id;
        if (fscanf(f, "%u %u %u %lf %lf %lf %lf %lf %lf %d", &d.type_a, &d.type_b, &d.bond_type, &d.r_min,
                   &d.r_max, &d.k_on, &d.k_off, &d.epsilon, &d.p_on0, &d.self_avoid) != 10)
            return 2;
        CHECK(db_add_reaction(s, &d, &id));
    }
    double dt, kT, gamma;
    unsigned period;
    if (fscanf(f, "%lf %lf %lf %u", &dt, &kT, &gamma, &period) != 4) return 2;
    float* pos = malloc(sizeof(float) * 3 * n);
    float* vel = malloc(sizeof(float) * 3 * n);
    uint32_t* type = malloc(sizeof(uint32_t) * n);
    for (unsigned i = 0; i < n; ++i) {
        double x[6];
        if (fscanf(f, "%lf %lf %lf %lf %lf %lf %u", &x[0], &x[1], &x[2], &x[3], &x[4], &x[5], &type[i]) != 7)
            return 2;
        for (int c = 0; c < 3; ++c) {
            pos[3 * i + c] = (float)x[c];
            vel[3 * i + c] = (float)x[3 + c];
        }
    }
    fclose(f);
    CHECK(db_set_particles(s, pos, vel, type));
    CHECK(db_set_integrator(s, dt, kT, gamma, period, DB_KT_SETPOINT));
    CHECK(db_commit(s));
    const uint64_t steps = strtoull(argv[3], NULL, 10), chunk = strtoull(argv[4], NULL, 10);
    for (uint64_t done = 0; done < steps;) {
        const uint64_t k = steps - done < chunk ? steps - done : chunk;
        CHECK(db_step(s, k));
        done += k;
    }
    uint64_t nb = 0;
    db_status st = db_read_bonds(s, NULL, NULL, 0, &nb);
    if (st != DB_OK && st != DB_ETRUNC) CHECK(st);
    uint32_t* bp = malloc(sizeof(uint32_t) * 2 * (nb + 1));
    uint32_t* bty = malloc(sizeof(uint32_t) * (nb + 1));
    CHECK(db_read_bonds(s, bp, bty, nb, &nb));
    CHECK(db_read_positions(s, pos, NULL));
    CHECK(db_read_velocities(s, vel));
    FILE* o = fopen(argv[2], "wb");
    if (!o) return 2;
    const uint64_t step = db_get_step(s);
    fwrite(&step, 8, 1, o);
    fwrite(&nb, 8, 1, o);
    for (uint64_t k = 0; k < nb; ++k) {
        const uint32_t r[3] = {bp[2 * k], bp[2 * k + 1], bty[k]};
        fwrite(r, 4, 3, o);
    }
    fwrite(pos, 4, 3 * (size_t)n, o);
    fwrite(vel, 4, 3 * (size_t)n, o);
    fclose(o);
    db_destroy(s);
    free(pairs);
    free(stype);
    free(pos);
    free(vel);
    free(type);
    free(bp);
    free(bty);
    return 0;
}
