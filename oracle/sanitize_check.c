/*
 * sanitize_check.c -- TEST INFRASTRUCTURE: exercises every entry point of the
 * FP64 oracle (lbm_oracle.c, compiled into this one translation unit) on
 * small cavities, so that a build with -fsanitize=address,undefined reports
 * any out-of-bounds access, use after free, leak or undefined arithmetic in
 * the oracle's host code.  Exit status 0 when every call succeeded and the
 * few consistency checks below hold.  Run by tests/test_sanitizers.py.
 */
#include "lbm_oracle.c"

#include <stdio.h>

static int fails = 0;
#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++fails;                                                         \
        }                                                                    \
    } while (0)

static double total_mass(oracle *o)
{
    const size_t cells = (size_t)o->n * o->n * o->n;
    double *rho = malloc(sizeof(double) * cells);
    oracle_macro(o, rho, NULL, NULL, NULL, NULL);
    double m = 0.0;
    for (size_t c = 0; c < cells; ++c)
        m += rho[c];
    free(rho);
    return m;
}

int main(void)
{
    double d[6], m[361], mi[361], nn[49], ni[49], w19[19], w7[7], out[19], v[3] = {0.01, -0.02, 0.03};
    int e19[57], e7[21];
    oracle_derive(16, 1e3, 0.71, 0.1, d);
    CHECK(d[4] > 0.0 && d[4] < 2.0);
    oracle_matrices(m, mi, nn, ni);
    oracle_matrices(NULL, mi, NULL, ni);
    oracle_velocities(e19, w19, e7, w7);
    oracle_meq(1.01, 0.01, 0.02, -0.03, out);
    oracle_feq(1.01, v, out);
    oracle_geq(0.3, v, out);
    oracle_force(1.01, v, 1e-4, out);
    oracle_guo_force(1.01, v, 1e-4, out);
    CHECK(oracle_create(1, 1, 1e3, 0.71, 0.1, 0.5, -0.5, 0.0, 1.0, NULL, NULL, NULL, 0, NULL) == NULL);
    CHECK(oracle_create(6, 4, 1e3, 0.71, 0.1, 0.5, -0.5, 0.0, 1.0, NULL, NULL, NULL, 0, NULL) == NULL);
    CHECK(oracle_create(6, 1, 1e3, 0.71, 0.1, 0.5, -0.5, 0.0, 1.0, NULL, NULL, NULL, 3, NULL) == NULL);

    const double s19[19] = {1.0, 1.19, 1.4, 1.0, 1.2, 1.0, 1.2, 1.0, 1.2, 1.7,
                            1.4, 1.7, 1.4, 1.7, 1.7, 1.7, 1.98, 1.98, 1.98};
    const double tau7[7] = {1.0, 0.7, 0.7, 0.7, 0.9, 1.1, 1.2};
    const double aniso[6] = {1.0, 1.5, 0.8, 0.2, -0.1, 0.05};
    for (int wt = 0; wt <= 3; ++wt) {
        for (int fm = 0; fm <= 2; ++fm) {
            const int n = 5 + wt;
            const size_t cells = (size_t)n * n * n;
            double *th0 = malloc(sizeof(double) * cells);
            for (size_t c = 0; c < cells; ++c)
                th0[c] = 1e-3 * (double)((c * 7919) % 13) / 13.0;
            oracle *o = oracle_create(n, wt, 1e5, 0.71, 0.1, 0.5, -0.5, 0.0, 1.0,
                                      fm == 1 ? s19 : NULL, fm == 1 ? tau7 : NULL,
                                      fm == 2 ? aniso : NULL, fm, th0);
            CHECK(o != NULL);
            if (!o) {
                free(th0);
                continue;
            }
            const double m0 = total_mass(o);
            oracle_step(o, 25);
            CHECK(oracle_time(o) == 25);
            CHECK(fabs(total_mass(o) - m0) < 1e-11 * m0);
            double *f = malloc(sizeof(double) * 19 * cells), *g = malloc(sizeof(double) * 7 * cells);
            double *r = malloc(sizeof(double) * 5 * cells), *map = malloc(sizeof(double) * n * n);
            oracle_macro(o, r, r + cells, r + 2 * cells, r + 3 * cells, r + 4 * cells);
            for (int st = 0; st <= 2; ++st) {
                double nu[3];
                oracle_nusselt(o, st, nu, map);
                oracle_nusselt(o, st, nu, NULL);
            }
            oracle_get_state(o, f, g);
            double fo[19], go[7];
            const int corners[4][3] = {{0, 0, 0}, {n - 1, n - 1, n - 1}, {0, n - 1, 1}, {n / 2, 0, n - 1}};
            for (int k = 0; k < 4; ++k)
                oracle_step_node(o, f, g, corners[k][0], corners[k][1], corners[k][2], fo, go);
            oracle_collide_node(o, f, g, fo, go);
            oracle_set_state(o, f, g, 3);
            oracle *p = oracle_create_params(n, wt, 1e5, 0.71, 0.1, 0.5, -0.5, 0.0, 1.0, NULL, NULL,
                                             NULL, fm);
            CHECK(p != NULL);
            if (p) {
                double nu[3], dd[6];
                oracle_nusselt_state(p, g, 0, nu, map);
                oracle_derived_of(p, dd);
                oracle_step_node(p, f, g, 1, 1, 1, fo, go);
                oracle_destroy(p);
            }
            free(f); free(g); free(r); free(map); free(th0);
            oracle_destroy(o);
        }
    }
    oracle_destroy(NULL);
    CHECK(oracle_threads() >= 1);
    if (fails)
        fprintf(stderr, "%d checks failed\n", fails);
    else
        printf("sanitize_check: all oracle entry points ran clean\n");
    return fails ? 1 : 0;
}
