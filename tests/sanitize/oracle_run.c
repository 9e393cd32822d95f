/* Memory and undefined-behaviour check of the FP64 oracle: every entry point
 * on small lattices (one of them non-cubic, one with L5 = 1), built with
 * -fsanitize=address,undefined by tests/test_sanitizers.py.  Values are
 * arbitrary; only the solve uses unit links so that it converges. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int X, Y, Z, T, L5;
    int antiperiodic_t;
    double M5, b5, c5, mq;
} oracle_params;
typedef struct {
    int iters, restarts;
    double true_resid, schur_resid;
} oracle_solve_info;

void oracle_gamma(int, double *);
void oracle_dslash4(const oracle_params *, const double *, const double *, double *, int);
void oracle_dw4(const oracle_params *, const double *, const double *, double *, int);
void oracle_C(const oracle_params *, const double *, double *, int);
void oracle_B(const oracle_params *, const double *, double *, int);
void oracle_K5(const oracle_params *, const double *, double *, int);
void oracle_K5inv(const oracle_params *, const double *, double *, int);
void oracle_Binv(const oracle_params *, const double *, double *, int);
void oracle_hop(const oracle_params *, const double *, const double *, double *, int, int);
void oracle_D5(const oracle_params *, const double *, const double *, double *, int);
void oracle_schur(const oracle_params *, const double *, const double *, double *, int);
void oracle_schur_sym(const oracle_params *, const double *, const double *, double *, int);
void oracle_schur_rp(const oracle_params *, const double *, const double *, double *, int);
void oracle_prep_source(const oracle_params *, const double *, const double *, double *);
void oracle_reconstruct(const oracle_params *, const double *, const double *, double *);
double oracle_true_residual(const oracle_params *, const double *, const double *, const double *);
int oracle_solve(const oracle_params *, const double *, const double *, double *, double, int, oracle_solve_info *);
double oracle_cgls_step(const oracle_params *, const double *, double *, double *, double *, double *, double *,
                        double *);
void oracle_D5_sites(const oracle_params *, const double *, const double *, const long *, int, double *);
void oracle_schur_sites(const oracle_params *, const double *, const double *, const long *, int, int, double *);

static double *rnd(long n, unsigned *seed)
{
    double *a = malloc(sizeof(double) * n);
    for (long i = 0; i < n; ++i) {
        *seed = *seed * 1103515245u + 12345u;
        a[i] = (double)((*seed >> 8) & 0xffff) / 65536.0 - 0.5;
    }
    return a;
}

static int run(int X, int Y, int Z, int T, int L5)
{
    oracle_params p = {X, Y, Z, T, L5, 1, 1.3, 1.5, 0.5, 0.05};
    const long V = (long)X * Y * Z * T, n4 = 24 * V, n5 = n4 * L5, nu = V * 4 * 18;
    unsigned seed = 7u + (unsigned)(X + 3 * L5);
    double *U = rnd(nu, &seed), *a = rnd(n5, &seed), *b = rnd(n5, &seed), *c = rnd(n5, &seed);
    double g[32];
    for (int mu = 0; mu < 4; ++mu) oracle_gamma(mu, g);
    for (int dag = 0; dag < 2; ++dag) {
        oracle_dslash4(&p, U, a, b, dag);
        oracle_dw4(&p, U, a, b, dag);
        oracle_C(&p, a, b, dag);
        oracle_B(&p, a, b, dag);
        oracle_K5(&p, a, b, dag);
        oracle_K5inv(&p, a, b, dag);
        oracle_Binv(&p, a, b, dag);
        oracle_hop(&p, U, a, b, dag, 0);
        oracle_hop(&p, U, a, b, dag, 1);
        oracle_D5(&p, U, a, b, dag);
        oracle_schur(&p, U, a, b, dag);
        oracle_schur_sym(&p, U, a, b, dag);
        oracle_schur_rp(&p, U, a, b, dag);
    }
    oracle_prep_source(&p, U, a, b);
    oracle_reconstruct(&p, U, a, b);
    (void)oracle_true_residual(&p, U, a, b);
    long sites[3] = {0, V - 1, V / 2};
    double *out = malloc(sizeof(double) * 3 * 24 * L5);
    oracle_D5_sites(&p, U, a, sites, 3, out);
    oracle_schur_sites(&p, U, a, sites, 3, 0, out);
    oracle_schur_sites(&p, U, a, sites, 3, 1, out);
    double gam = 1.0, *r = rnd(n5, &seed), *pv = rnd(n5, &seed), *s = rnd(n5, &seed);
    (void)oracle_cgls_step(&p, U, c, r, pv, s, b, &gam);
    /* unit links: the solve converges */
    memset(U, 0, sizeof(double) * nu);
    for (long l = 0; l < V * 4; ++l)
        for (int k = 0; k < 3; ++k) U[l * 18 + 2 * (4 * k)] = 1.0;
    oracle_solve_info info;
    const int st = oracle_solve(&p, U, a, c, 1e-10, 5000, &info);
    free(U); free(a); free(b); free(c); free(out); free(r); free(pv); free(s);
    if (st != 0 || !(info.true_resid <= 1e-10)) {
        printf("solve failed on %dx%dx%dx%d L5=%d: status %d resid %g\n", X, Y, Z, T, L5, st, info.true_resid);
        return 1;
    }
    return 0;
}

int main(void)
{
    int bad = run(2, 2, 2, 4, 4) + run(2, 4, 2, 6, 3) + run(2, 2, 2, 2, 1);
    printf(bad ? "oracle sanitizer run: FAILED\n" : "oracle sanitizer run: ok\n");
    return bad;
}
