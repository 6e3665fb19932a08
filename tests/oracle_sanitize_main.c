/*
 * Driver that builds the FP64 oracle together with AddressSanitizer and
 * UndefinedBehaviorSanitizer (host code only, gcc) and runs every public
 * entry point on small problems of each dimension, flux family, prolongation
 * mode and time-step rule.  Any out-of-bounds access, leak, signed overflow or
 * other undefined behaviour aborts with a non-zero exit status; the test in
 * test_oracle_sanitized.py compiles and runs it.
 */
#include "../oracle/oracle.c"

#include <stdio.h>

static int check_finite(const double *a, int64_t n, const char *what)
{
    for (int64_t i = 0; i < n; i++)
        if (!isfinite(a[i])) {
            fprintf(stderr, "%s: non-finite value at %lld\n", what, (long long)i);
            return 1;
        }
    return 0;
}

static int run(const orc_problem *p, const orc_config *c, double T, const char *name)
{
    int64_t total = orc_total_nodes(p, c);
    int nfin = c->nr << c->nl;
    int64_t ftot = 1;
    for (int k = 0; k < p->d; k++) ftot *= nfin;
    double *st = malloc(sizeof(double) * total);
    double *U = malloc(sizeof(double) * ftot);
    double *ex = malloc(sizeof(double) * ftot);
    orc_restrict(p, c, st);
    orc_stats stats;
    int rc = orc_evolve(p, c, T, st, NULL, &stats);
    if (rc != 0) {
        fprintf(stderr, "%s: evolve returned %d\n", name, rc);
        return 1;
    }
    orc_prolong_combine(p, c, st, U);
    orc_exact_fine(p, c, stats.t, ex);
    double l1, linf;
    orc_norms(U, ex, ftot, &l1, &linf);
    /* a few points through the point-wise combination, corners included */
    int J[3 * ORC_MAXD] = {0};
    for (int k = 0; k < p->d; k++) {
        J[k] = 0;
        J[ORC_MAXD + k] = nfin - 1;
        J[2 * ORC_MAXD + k] = (nfin / 2 + k) % nfin;
    }
    double pts[3];
    orc_prolong_combine_points(p, c, st, 3, J, pts);
    /* one grid's spatial operator */
    int lev[ORC_MAXD] = {0, 0, 0, 0};
    lev[0] = c->nl;
    orc_grid g;
    orc_grid_make(p, c->nr, lev, &g);
    double *u = malloc(sizeof(double) * g.size), *L = malloc(sizeof(double) * g.size);
    orc_restrict_grid(p, &g, u);
    orc_rhs(p, c, lev, u, L);
    int bad = check_finite(st, total, name) | check_finite(U, ftot, name) | check_finite(pts, 3, name) |
              check_finite(L, g.size, name);
    printf("%-28s d=%d steps=%lld L1=%.3e Linf=%.3e\n", name, p->d, (long long)stats.steps, l1, linf);
    free(st);
    free(U);
    free(ex);
    free(u);
    free(L);
    return bad;
}

int main(void)
{
    int fails = 0;
    for (int d = 1; d <= 4; d++) {
        orc_problem p;
        memset(&p, 0, sizeof p);
        p.d = d;
        p.flux = ORC_FLUX_ADVECTION;
        p.ic = ORC_IC_SINE;
        for (int k = 0; k < d; k++) {
            p.lo[k] = 0.0;
            p.hi[k] = 2.0;
            p.fp[k] = (k % 2) ? -1.0 : 1.0;
        }
        p.ip[0] = 0.1;
        p.ip[1] = 1.0;
        p.ip[2] = M_PI;
        orc_config c = {4, d == 4 ? 1 : 2, ORC_DT_CFL, ORC_PROLONG_WENO5, 0, 1, 0.5, 1e-3, 1e-3};
        fails |= run(&p, &c, 0.05, "advection weno5");
        c.prolong = ORC_PROLONG_LAGRANGE5;
        c.linear = 1;
        c.dt_mode = ORC_DT_POW53;
        fails |= run(&p, &c, 0.02, "advection linear lagrange5");
        p.flux = ORC_FLUX_BURGERS;
        c.prolong = ORC_PROLONG_WENO5;
        c.linear = 0;
        c.dt_mode = ORC_DT_CFL;
        fails |= run(&p, &c, 0.03, "burgers");
        if (d % 2 == 0) {
            orc_problem v;
            memset(&v, 0, sizeof v);
            v.d = d;
            v.flux = ORC_FLUX_VLASOV;
            v.ic = ORC_IC_MAXWELL_COS;
            for (int k = 0; k < d / 2; k++) {
                v.lo[k] = 0.0;
                v.hi[k] = 4.0 * M_PI;
                v.lo[d / 2 + k] = -6.0;
                v.hi[d / 2 + k] = 6.0;
            }
            v.fp[0] = 0.3;
            v.fp[1] = 0.5;
            v.ip[0] = 0.05;
            v.ip[1] = 0.5;
            orc_config cv = {4, d == 4 ? 1 : 3, ORC_DT_CFL, ORC_PROLONG_WENO5, 0, 1, 0.4, 1e-3, 1e-3};
            fails |= run(&v, &cv, 0.2, "vlasov");
        }
    }
    /* the grid set alone for every dimension and level the library accepts in tests */
    for (int d = 1; d <= 4; d++)
        for (int nl = 0; nl <= 7; nl++) {
            int G = orc_num_grids(d, nl);
            int *lv = malloc(sizeof(int) * ORC_MAXD * G), *cf = malloc(sizeof(int) * G);
            int s = 0;
            orc_grid_set(d, nl, lv, cf);
            for (int g = 0; g < G; g++) s += cf[g];
            if (s != 1) fails = 1;
            free(lv);
            free(cf);
        }
    printf(fails ? "SANITIZED RUN FAILED\n" : "SANITIZED RUN OK\n");
    return fails;
}
