/*
 * mdwf_oracle.c -- plain, slow FP64 CPU reference for the Moebius
 * domain-wall operator and its even-odd CG solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU baseline leg of
 * the benchmark do.  It shares no code, header or table with the HIP path.
 *
 * Every routine works on full-lattice fields and loops over all sites; parity
 * restrictions are applied as masks (sites of the other parity are skipped or
 * zeroed), never by checkerboard indexing.  Fields are arrays of C99
 * `double complex`:
 *
 *   gauge   U[site][mu][a][b]            mu = 0..3 -> x, y, z, t
 *   4D      psi[site][spin][colour]
 *   5D      psi[s][site][spin][colour]   s = 0..L5-1 slowest
 *   site    = x + X*(y + Y*(z + Z*t)),   parity = (x+y+z+t) mod 2
 *
 * Definitions (paper, Sec. II and the cited Moebius construction):
 *   Wilson operator with Wilson parameter r = 1 and domain-wall height M5:
 *     D_W psi(x) = (4 - M5) psi(x) - 1/2 Dslash psi(x)
 *     Dslash psi(x) = sum_mu (1 - g_mu) U_mu(x) psi(x+mu)
 *                          + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu)
 *   with hops across the t boundary multiplied by -1 when the time direction
 *   is antiperiodic.  Euclidean chiral basis, g5 = diag(1,1,-1,-1);
 *   P+ = spins {0,1}, P- = spins {2,3}.
 *
 *   Fifth dimension: (C psi)_s = P- psi_{s+1} + P+ psi_{s-1}, where inside C
 *   the out-of-range slices are psi_{L5} = -m_q psi_0 and
 *   psi_{-1} = -m_q psi_{L5-1} (the quark mass couples the two walls).
 *
 *   Moebius 5D operator: D5 = D_W (b5 + c5 C) + (1 - C).
 *   Its 4D-site-local part is K5 = (4 - M5)(b5 + c5 C) + 1 - C and its hopping
 *   part is -1/2 Dslash B with B = b5 + c5 C.  With these, the combinations
 *   D_+ = b5 D_W + 1 and D_- = c5 D_W - 1 give the paper's Moebius kernel
 *   (b5 + c5) D_W / (2 + (b5 - c5) D_W) = (D_+ + D_-)(D_+ - D_-)^-1 (Sec. II).
 *
 *   Even-odd (asymmetric) preconditioning on 4D parity, solving for the even
 *   sites (the paper's Sec. VII names the asymmetric and symmetric forms):
 *     S   = K5 - 1/4 D_eo B K5^-1 D_oe B
 *     b'_e = b_e + 1/2 D_eo B K5^-1 b_o
 *     x_o = K5^-1 (b_o + 1/2 D_oe B x_e)
 *
 *   K5^-1 is computed here by dense Gaussian elimination of the L5 x L5 matrix
 *   of K5 on each chirality (no closed form is used).
 */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

typedef struct {
    int X, Y, Z, T, L5;
    int antiperiodic_t;
    double M5, b5, c5, mq;
} oracle_params;

typedef struct {
    int iters;
    int restarts;
    double true_resid;   /* ||b - D5 x|| / ||b|| on the reconstructed x */
    double schur_resid;  /* last tracked ||r|| / ||b|| */
} oracle_solve_info;

/* ------------------------------------------------------------------ gamma */

/* Euclidean chiral basis: g_k = [[0, -i s_k], [i s_k, 0]], g_4 = [[0,1],[1,0]]
 * for k = 1, 2, 3 (x, y, z) and 4 (t). */
static cplx G[4][4][4];
static int gamma_ready = 0;

static void init_gamma(void)
{
    if (gamma_ready) return;
    cplx s[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    memset(G, 0, sizeof(G));
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                G[k][i][2 + j] = -I * s[k][i][j];
                G[k][2 + i][j] = I * s[k][i][j];
            }
    for (int i = 0; i < 2; ++i) {
        G[3][i][2 + i] = 1;
        G[3][2 + i][i] = 1;
    }
    gamma_ready = 1;
}

void oracle_gamma(int mu, double *out /* 4x4 complex, re/im interleaved */)
{
    init_gamma();
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            out[2 * (4 * i + j)] = creal(G[mu][i][j]);
            out[2 * (4 * i + j) + 1] = cimag(G[mu][i][j]);
        }
}

/* ------------------------------------------------------------- geometry */

static long volume(const oracle_params *p) { return (long)p->X * p->Y * p->Z * p->T; }

static void coords(const oracle_params *p, long site, int c[4])
{
    c[0] = (int)(site % p->X); site /= p->X;
    c[1] = (int)(site % p->Y); site /= p->Y;
    c[2] = (int)(site % p->Z); site /= p->Z;
    c[3] = (int)site;
}

static long site_of(const oracle_params *p, const int c[4])
{
    return c[0] + (long)p->X * (c[1] + (long)p->Y * (c[2] + (long)p->Z * c[3]));
}

static int parity_of(const oracle_params *p, long site)
{
    int c[4];
    coords(p, site, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

/* Neighbour of `site` one step in direction mu (dir = +1 or -1); *bc gets the
 * boundary phase of that hop (-1 across the antiperiodic t boundary). */
static long neighbour(const oracle_params *p, long site, int mu, int dir, double *bc)
{
    int c[4], L[4] = {p->X, p->Y, p->Z, p->T};
    coords(p, site, c);
    int v = c[mu] + dir;
    *bc = 1.0;
    if (v >= L[mu]) { v -= L[mu]; if (mu == 3 && p->antiperiodic_t) *bc = -1.0; }
    if (v < 0) { v += L[mu]; if (mu == 3 && p->antiperiodic_t) *bc = -1.0; }
    c[mu] = v;
    return site_of(p, c);
}

/* ------------------------------------------------------------ 4D Wilson */

/* acc = (Dslash in)(x) for one site x of a 4D field:
 *   sum_mu (1 - sg g_mu) U_mu(x) in(x+mu) + (1 + sg g_mu) U_mu(x-mu)^+ in(x-mu)
 * with sg = +1 for Dslash and sg = -1 for its adjoint. */
static void hop_site(const oracle_params *p, const cplx *U, const cplx *in, long x, int dag,
                     cplx acc[4][3])
{
    init_gamma();
    const double sg = dag ? -1.0 : 1.0;
    memset(acc, 0, 12 * sizeof(cplx));
    for (int mu = 0; mu < 4; ++mu) {
        for (int dir = +1; dir >= -1; dir -= 2) {
            double bc;
            long y = neighbour(p, x, mu, dir, &bc);
            const cplx *psi = in + 12 * y;
            /* colour: forward uses U_mu(x), backward U_mu(x-mu)^+ */
            cplx tmp[4][3];
            for (int sp = 0; sp < 4; ++sp)
                for (int a = 0; a < 3; ++a) {
                    cplx v = 0;
                    for (int b = 0; b < 3; ++b) {
                        cplx u = (dir > 0) ? U[(x * 4 + mu) * 9 + a * 3 + b]
                                           : conj(U[(y * 4 + mu) * 9 + b * 3 + a]);
                        v += u * psi[sp * 3 + b];
                    }
                    tmp[sp][a] = v;
                }
            /* spin: (1 - dir*sg g_mu) */
            const double gs = -dir * sg;
            for (int sp = 0; sp < 4; ++sp)
                for (int a = 0; a < 3; ++a) {
                    cplx v = tmp[sp][a];
                    for (int sq = 0; sq < 4; ++sq) v += gs * G[mu][sp][sq] * tmp[sq][a];
                    acc[sp][a] += bc * v;
                }
        }
    }
}

/* Dslash (or its adjoint) on a 4D field.  Only sites whose parity equals
 * `out_parity` are written (all sites when out_parity < 0); the others are
 * set to zero. */
static void dslash4(const oracle_params *p, const cplx *U, const cplx *in, cplx *out,
                    int dag, int out_parity)
{
    const long V = volume(p);
    init_gamma();   /* before any thread reads the table */
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x) {
        cplx acc[4][3];
        memset(acc, 0, sizeof(acc));
        if (out_parity < 0 || parity_of(p, x) == out_parity) hop_site(p, U, in, x, dag, acc);
        memcpy(out + 12 * x, acc, sizeof(acc));
    }
}

/* D_W (or D_W^+) on a 4D field, all sites. */
static void dw4(const oracle_params *p, const cplx *U, const cplx *in, cplx *out, int dag)
{
    const long n = 12 * volume(p);
    dslash4(p, U, in, out, dag, -1);
    for (long i = 0; i < n; ++i) out[i] = (4.0 - p->M5) * in[i] - 0.5 * out[i];
}

/* ------------------------------------------------------ fifth dimension */

/* C (dag = 0) or C^+ (dag = 1) on a 5D field. */
static void apply_C(const oracle_params *p, const cplx *in, cplx *out, int dag)
{
    const long V = volume(p), L5 = p->L5;
#pragma omp parallel for collapse(2) schedule(static)
    for (long s = 0; s < L5; ++s)
        for (long x = 0; x < V; ++x)
            for (int sp = 0; sp < 4; ++sp) {
                /* C: P- reads s+1, P+ reads s-1; C^+ swaps the two */
                int upper = sp < 2;
                long from = (upper != dag) ? s - 1 : s + 1;
                double f = 1.0;
                if (from < 0) { from += L5; f = -p->mq; }
                if (from >= L5) { from -= L5; f = -p->mq; }
                for (int a = 0; a < 3; ++a)
                    out[(s * V + x) * 12 + sp * 3 + a] = f * in[(from * V + x) * 12 + sp * 3 + a];
            }
}

/* B = b5 + c5 C  (or B^+ = b5 + c5 C^+). */
static void apply_B(const oracle_params *p, const cplx *in, cplx *out, int dag)
{
    const long n = 12 * volume(p) * p->L5;
    apply_C(p, in, out, dag);
    for (long i = 0; i < n; ++i) out[i] = p->b5 * in[i] + p->c5 * out[i];
}

/* K5 = (4 - M5) B + 1 - C  (or its adjoint). */
static void apply_K5(const oracle_params *p, const cplx *in, cplx *out, int dag)
{
    const long n = 12 * volume(p) * p->L5;
    cplx *c = malloc(n * sizeof(cplx));
    apply_C(p, in, c, dag);
    for (long i = 0; i < n; ++i)
        out[i] = (4.0 - p->M5) * (p->b5 * in[i] + p->c5 * c[i]) + in[i] - c[i];
    free(c);
}

/* Dense L5 x L5 matrix of K5 (or K5^+) restricted to one chirality, built by
 * applying the definition to unit vectors along s. */
static void k5_matrix(const oracle_params *p, int upper, int dag, double *K)
{
    const int L5 = p->L5;
    for (int j = 0; j < L5; ++j)
        for (int i = 0; i < L5; ++i) {
            /* (C e_j)_i : C on P+ maps slice i-1 -> i, on P- slice i+1 -> i */
            double cij = 0.0;
            int from_up = (upper != dag) ? i - 1 : i + 1;
            double f = 1.0;
            if (from_up < 0) { from_up += L5; f = -p->mq; }
            if (from_up >= L5) { from_up -= L5; f = -p->mq; }
            if (from_up == j) cij = f;
            double id = (i == j) ? 1.0 : 0.0;
            K[i * L5 + j] = (4.0 - p->M5) * (p->b5 * id + p->c5 * cij) + id - cij;
        }
}

/* Solve A y = r in place (y overwrites r) by Gaussian elimination with partial
 * pivoting; A is n x n real, destroyed. */
static void gauss_solve(int n, double *A, cplx *r)
{
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int i = k + 1; i < n; ++i)
            if (fabs(A[i * n + k]) > fabs(A[piv * n + k])) piv = i;
        if (piv != k) {
            for (int j = 0; j < n; ++j) {
                double t = A[k * n + j]; A[k * n + j] = A[piv * n + j]; A[piv * n + j] = t;
            }
            cplx t = r[k]; r[k] = r[piv]; r[piv] = t;
        }
        for (int i = k + 1; i < n; ++i) {
            double f = A[i * n + k] / A[k * n + k];
            for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
            r[i] -= f * r[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        cplx v = r[k];
        for (int j = k + 1; j < n; ++j) v -= A[k * n + j] * r[j];
        r[k] = v / A[k * n + k];
    }
}

/* Solve the L5 x L5 system M y = v on every 4D site, spin and colour, with
 * M = Mc[0] on the upper (P+) spins and Mc[1] on the lower (P-) spins. */
static void solve_fifth(const oracle_params *p, double *const Mc[2], const cplx *in, cplx *out)
{
    const long V = volume(p);
    const int L5 = p->L5;
    if (L5 > 32) {   /* the per-site scratch below holds L5 <= 32 */
        fprintf(stderr, "oracle: L5 = %d exceeds 32\n", L5);
        abort();
    }
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x) {
        double A[32 * 32];
        cplx col[32];
        for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a) {
                for (int s = 0; s < L5; ++s) col[s] = in[((long)s * V + x) * 12 + sp * 3 + a];
                memcpy(A, Mc[sp < 2 ? 0 : 1], sizeof(double) * L5 * L5);
                gauss_solve(L5, A, col);
                for (int s = 0; s < L5; ++s) out[((long)s * V + x) * 12 + sp * 3 + a] = col[s];
            }
    }
}

/* K5^-1 (or (K5^+)^-1): for every 4D site, spin and colour, solve the L5 x L5
 * system of that chirality. */
static void apply_K5inv(const oracle_params *p, const cplx *in, cplx *out, int dag)
{
    const int L5 = p->L5;
    double *K[2];
    for (int u = 0; u < 2; ++u) {
        K[u] = malloc(sizeof(double) * L5 * L5);
        k5_matrix(p, u == 0, dag, K[u]);
    }
    solve_fifth(p, K, in, out);
    free(K[0]); free(K[1]);
}

/* Dense L5 x L5 matrix of B = b5 + c5 C (or B^+) on one chirality, from the
 * definition of C applied to unit vectors along s. */
static void b_matrix(const oracle_params *p, int upper, int dag, double *Bm)
{
    const int L5 = p->L5;
    for (int j = 0; j < L5; ++j)
        for (int i = 0; i < L5; ++i) {
            double cij = 0.0;
            int from = (upper != dag) ? i - 1 : i + 1;
            double f = 1.0;
            if (from < 0) { from += L5; f = -p->mq; }
            if (from >= L5) { from -= L5; f = -p->mq; }
            if (from == j) cij = f;
            Bm[i * L5 + j] = p->b5 * (i == j ? 1.0 : 0.0) + p->c5 * cij;
        }
}

/* B^-1 (or (B^+)^-1), by Gaussian elimination per 4D site, spin and colour. */
static void apply_Binv(const oracle_params *p, const cplx *in, cplx *out, int dag)
{
    const int L5 = p->L5;
    double *Bm[2];
    for (int u = 0; u < 2; ++u) {
        Bm[u] = malloc(sizeof(double) * L5 * L5);
        b_matrix(p, u == 0, dag, Bm[u]);
    }
    solve_fifth(p, Bm, in, out);
    free(Bm[0]); free(Bm[1]);
}

/* Dslash (or Dslash^+) on every slice, input masked to parity 1-out_parity,
 * output on parity out_parity (zero elsewhere). */
static void hop5(const oracle_params *p, const cplx *U, const cplx *in, cplx *out,
                 int dag, int out_parity)
{
    const long V = volume(p), n4 = 12 * V;
    cplx *tmp = malloc(n4 * sizeof(cplx));
    for (int s = 0; s < p->L5; ++s) {
        const cplx *src = in + s * n4;
#pragma omp parallel for schedule(static)
        for (long x = 0; x < V; ++x) {
            int keep = parity_of(p, x) != out_parity;
            for (int k = 0; k < 12; ++k) tmp[12 * x + k] = keep ? src[12 * x + k] : 0;
        }
        dslash4(p, U, tmp, out + s * n4, dag, out_parity);
    }
    free(tmp);
}

static void mask_parity(const oracle_params *p, cplx *f, int keep_parity)
{
    const long V = volume(p);
    for (int s = 0; s < p->L5; ++s)
        for (long x = 0; x < V; ++x)
            if (parity_of(p, x) != keep_parity)
                memset(f + ((long)s * V + x) * 12, 0, 12 * sizeof(cplx));
}

/* ---------------------------------------------------------- public API */

static long n5(const oracle_params *p) { return 12 * volume(p) * p->L5; }

void oracle_dslash4(const oracle_params *p, const double *U, const double *in,
                    double *out, int dag)
{
    dslash4(p, (const cplx *)U, (const cplx *)in, (cplx *)out, dag, -1);
}

void oracle_dw4(const oracle_params *p, const double *U, const double *in, double *out, int dag)
{
    dw4(p, (const cplx *)U, (const cplx *)in, (cplx *)out, dag);
}

void oracle_C(const oracle_params *p, const double *in, double *out, int dag)
{
    apply_C(p, (const cplx *)in, (cplx *)out, dag);
}

void oracle_B(const oracle_params *p, const double *in, double *out, int dag)
{
    apply_B(p, (const cplx *)in, (cplx *)out, dag);
}

void oracle_K5(const oracle_params *p, const double *in, double *out, int dag)
{
    apply_K5(p, (const cplx *)in, (cplx *)out, dag);
}

void oracle_K5inv(const oracle_params *p, const double *in, double *out, int dag)
{
    apply_K5inv(p, (const cplx *)in, (cplx *)out, dag);
}

/* Bare hop between parities on every slice: out_{out_parity} = Dslash in. */
void oracle_Binv(const oracle_params *p, const double *in, double *out, int dag)
{
    apply_Binv(p, (const cplx *)in, (cplx *)out, dag);
}

void oracle_hop(const oracle_params *p, const double *U, const double *in, double *out,
                int dag, int out_parity)
{
    hop5(p, (const cplx *)U, (const cplx *)in, (cplx *)out, dag, out_parity);
}

/* D5 = D_W B + 1 - C, applied slice by slice (dag: D5^+ = B^+ D_W^+ + 1 - C^+). */
void oracle_D5(const oracle_params *p, const double *Ud, const double *ind, double *outd, int dag)
{
    const cplx *U = (const cplx *)Ud, *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    const long n = n5(p), n4 = 12 * volume(p);
    cplx *t = malloc(n * sizeof(cplx)), *c = malloc(n * sizeof(cplx));
    if (!dag) {
        apply_B(p, in, t, 0);
        for (int s = 0; s < p->L5; ++s) dw4(p, U, t + s * n4, out + s * n4, 0);
    } else {
        for (int s = 0; s < p->L5; ++s) dw4(p, U, in + s * n4, t + s * n4, 1);
        apply_B(p, t, out, 1);
    }
    apply_C(p, in, c, dag);
    for (long i = 0; i < n; ++i) out[i] += in[i] - c[i];
    free(t); free(c);
}

/* Schur complement on the even sites, S = K5 - 1/4 D_eo B K5^-1 D_oe B, or its
 * adjoint S^+ = K5^+ - 1/4 B^+ D_oe^+ K5^-+ B^+ D_eo^+.  The odd half of `in`
 * is ignored; the odd half of `out` is zero. */
void oracle_schur(const oracle_params *p, const double *Ud, const double *ind, double *outd, int dag)
{
    const cplx *U = (const cplx *)Ud;
    cplx *out = (cplx *)outd;
    const long n = n5(p);
    cplx *x = malloc(n * sizeof(cplx)), *t1 = malloc(n * sizeof(cplx)), *t2 = malloc(n * sizeof(cplx));
    memcpy(x, ind, n * sizeof(cplx));
    mask_parity(p, x, 0);
    if (!dag) {
        apply_B(p, x, t1, 0);
        hop5(p, U, t1, t2, 0, 1);       /* D_oe B x          (odd)  */
        apply_K5inv(p, t2, t1, 0);      /* K5^-1 ...                */
        apply_B(p, t1, t2, 0);          /* B K5^-1 ...              */
        hop5(p, U, t2, t1, 0, 0);       /* D_eo B K5^-1 D_oe B x    */
        apply_K5(p, x, out, 0);
    } else {
        hop5(p, U, x, t1, 1, 1);        /* D_eo^+ x          (odd)  */
        apply_B(p, t1, t2, 1);          /* B^+ ...                  */
        apply_K5inv(p, t2, t1, 1);      /* K5^-+ B^+ ...            */
        hop5(p, U, t1, t2, 1, 0);       /* D_oe^+ ...        (even) */
        apply_B(p, t2, t1, 1);          /* B^+ D_oe^+ ...           */
        apply_K5(p, x, out, 1);
    }
    for (long i = 0; i < n; ++i) out[i] -= 0.25 * t1[i];
    mask_parity(p, out, 0);
    free(x); free(t1); free(t2);
}

/* Symmetric form of the even-odd operator (Sec. VII names it beside the
 * asymmetric one): Shat = K5^-1 S = 1 - 1/4 K5^-1 D_eo B K5^-1 D_oe B on the
 * even sites, or its adjoint Shat^+ = S^+ K5^-+.  Solving Shat x_e = K5^-1 b'_e
 * gives the same x_e as S x_e = b'_e. */
void oracle_schur_sym(const oracle_params *p, const double *Ud, const double *ind, double *outd, int dag)
{
    cplx *out = (cplx *)outd;
    const long n = n5(p);
    cplx *t = malloc(n * sizeof(cplx));
    if (!dag) {
        oracle_schur(p, Ud, ind, (double *)t, 0);
        apply_K5inv(p, t, out, 0);
    } else {
        memcpy(t, ind, n * sizeof(cplx));
        mask_parity(p, t, 0);
        apply_K5inv(p, t, out, 1);
        memcpy(t, out, n * sizeof(cplx));
        oracle_schur(p, Ud, (const double *)t, outd, 1);
    }
    mask_parity(p, out, 0);
    free(t);
}

/* The Schur operator preconditioned on the right by B^-1: S B^-1 on the even
 * sites, or its adjoint B^-+ S^+.  If S B^-1 y = b'_e then x_e = B^-1 y solves
 * S x_e = b'_e, with the same residual b'_e - S x_e. */
void oracle_schur_rp(const oracle_params *p, const double *Ud, const double *ind, double *outd, int dag)
{
    cplx *out = (cplx *)outd;
    const long n = n5(p);
    cplx *t = malloc(n * sizeof(cplx));
    if (!dag) {
        memcpy(t, ind, n * sizeof(cplx));
        mask_parity(p, t, 0);
        apply_Binv(p, t, out, 0);
        memcpy(t, out, n * sizeof(cplx));
        oracle_schur(p, Ud, (const double *)t, outd, 0);
    } else {
        oracle_schur(p, Ud, ind, (double *)t, 1);
        apply_Binv(p, t, out, 1);
    }
    mask_parity(p, out, 0);
    free(t);
}

/* b'_e = b_e + 1/2 D_eo B K5^-1 b_o (odd half of the output zero). */
void oracle_prep_source(const oracle_params *p, const double *Ud, const double *bd, double *outd)
{
    const cplx *U = (const cplx *)Ud;
    cplx *out = (cplx *)outd;
    const long n = n5(p);
    cplx *bo = malloc(n * sizeof(cplx)), *t1 = malloc(n * sizeof(cplx)), *t2 = malloc(n * sizeof(cplx));
    memcpy(bo, bd, n * sizeof(cplx));
    mask_parity(p, bo, 1);
    apply_K5inv(p, bo, t1, 0);
    apply_B(p, t1, t2, 0);
    hop5(p, U, t2, t1, 0, 0);
    memcpy(out, bd, n * sizeof(cplx));
    mask_parity(p, out, 0);
    for (long i = 0; i < n; ++i) out[i] += 0.5 * t1[i];
    mask_parity(p, out, 0);
    free(bo); free(t1); free(t2);
}

/* x_o = K5^-1 (b_o + 1/2 D_oe B x_e); x holds x_e on entry (its odd half is
 * ignored) and the full solution on exit. */
void oracle_reconstruct(const oracle_params *p, const double *Ud, const double *bd, double *xd)
{
    const cplx *U = (const cplx *)Ud, *b = (const cplx *)bd;
    cplx *x = (cplx *)xd;
    const long n = n5(p);
    cplx *t1 = malloc(n * sizeof(cplx)), *t2 = malloc(n * sizeof(cplx));
    mask_parity(p, x, 0);
    apply_B(p, x, t1, 0);
    hop5(p, U, t1, t2, 0, 1);
    for (long i = 0; i < n; ++i) t2[i] = 0.5 * t2[i];
    memcpy(t1, b, n * sizeof(cplx));
    mask_parity(p, t1, 1);
    for (long i = 0; i < n; ++i) t1[i] += t2[i];
    apply_K5inv(p, t1, t2, 0);
    mask_parity(p, t2, 1);
    for (long i = 0; i < n; ++i) x[i] += t2[i];
    free(t1); free(t2);
}

static double norm2(const cplx *a, long n)
{
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return s;
}

/* ||b - D5 x|| / ||b|| */
double oracle_true_residual(const oracle_params *p, const double *U, const double *bd, const double *xd)
{
    const long n = n5(p);
    cplx *r = malloc(n * sizeof(cplx));
    const cplx *b = (const cplx *)bd;
    oracle_D5(p, U, xd, (double *)r, 0);
    for (long i = 0; i < n; ++i) r[i] = b[i] - r[i];
    double res = sqrt(norm2(r, n) / norm2(b, n));
    free(r);
    return res;
}

/* Solve D5 x = b: source preparation, CG on the normal equations of the Schur
 * system in its least-squares (CGLS) form, odd-site reconstruction.  The
 * recursion tracks r = b' - S x_e and s = S^+ r; it stops when ||r|| falls
 * below tol/2 * ||b|| and then checks the true residual of the full system,
 * restarting from the true r if that check fails.  Returns 0 on success,
 * 1 if max_iter was reached. */
int oracle_solve(const oracle_params *p, const double *Ud, const double *bd, double *xd,
                 double tol, int max_iter, oracle_solve_info *info)
{
    const long n = n5(p);
    const cplx *b = (const cplx *)bd;
    cplx *x = (cplx *)xd;
    cplx *bp = malloc(n * sizeof(cplx)), *r = malloc(n * sizeof(cplx)),
         *s = malloc(n * sizeof(cplx)), *pv = malloc(n * sizeof(cplx)),
         *q = malloc(n * sizeof(cplx)), *xe = malloc(n * sizeof(cplx));
    const double bnorm = sqrt(norm2(b, n));
    int it = 0, restarts = 0, status = 1;
    double rnorm = 0.0, true_res = INFINITY;

    oracle_prep_source(p, Ud, bd, (double *)bp);
    memset(xe, 0, n * sizeof(cplx));
    memcpy(r, bp, n * sizeof(cplx));

    while (it < max_iter) {
        /* (re)start: s = S^+ r, p = s */
        oracle_schur(p, Ud, (const double *)r, (double *)s, 1);
        memcpy(pv, s, n * sizeof(cplx));
        double gam = norm2(s, n);
        rnorm = sqrt(norm2(r, n));
        while (it < max_iter && rnorm > 0.5 * tol * bnorm) {
            oracle_schur(p, Ud, (const double *)pv, (double *)q, 0);
            double alpha = gam / norm2(q, n);
            for (long i = 0; i < n; ++i) { xe[i] += alpha * pv[i]; r[i] -= alpha * q[i]; }
            oracle_schur(p, Ud, (const double *)r, (double *)s, 1);
            double gnew = norm2(s, n);
            double beta = gnew / gam;
            gam = gnew;
            for (long i = 0; i < n; ++i) pv[i] = s[i] + beta * pv[i];
            rnorm = sqrt(norm2(r, n));
            ++it;
        }
        memcpy(x, xe, n * sizeof(cplx));
        oracle_reconstruct(p, Ud, bd, xd);
        true_res = oracle_true_residual(p, Ud, bd, xd);
        if (true_res <= tol) { status = 0; break; }
        /* restart from the true Schur residual */
        oracle_schur(p, Ud, (const double *)xe, (double *)q, 0);
        for (long i = 0; i < n; ++i) r[i] = bp[i] - q[i];
        ++restarts;
        if (restarts > 50) break;
    }
    if (info) {
        info->iters = it;
        info->restarts = restarts;
        info->true_resid = true_res;
        info->schur_resid = rnorm / bnorm;
    }
    free(bp); free(r); free(s); free(pv); free(q); free(xe);
    return status;
}

/* ------------------------------------------------------ sampled sites */

/* (D5 in)(x, s) for the 4D sites listed in `sites` and every slice s;
 * out[n][L5][12].  Evaluated site by site from the definition
 * D5 = D_W B + 1 - C (the full-lattice B and C passes are O(volume)). */
void oracle_D5_sites(const oracle_params *p, const double *Ud, const double *ind,
                     const long *sites, int nsites, double *outd)
{
    const cplx *U = (const cplx *)Ud, *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    const long V = volume(p), n = n5(p);
    const int L5 = p->L5;
    cplx *b = malloc(n * sizeof(cplx)), *c = malloc(n * sizeof(cplx));
    apply_B(p, in, b, 0);
    apply_C(p, in, c, 0);
    for (int k = 0; k < nsites; ++k) {
        const long x = sites[k];
        for (int s = 0; s < L5; ++s) {
            cplx acc[4][3];
            hop_site(p, U, b + (long)s * V * 12, x, 0, acc);
            const long o = ((long)s * V + x) * 12;
            for (int i = 0; i < 12; ++i)
                out[((long)k * L5 + s) * 12 + i] =
                    (4.0 - p->M5) * b[o + i] - 0.5 * (&acc[0][0])[i] + in[o + i] - c[o + i];
        }
    }
    free(b); free(c);
}

/* (S in)(x, s) or (S^+ in)(x, s) for even 4D sites `sites` and every slice;
 * out[n][L5][12].  The odd-site intermediate is evaluated only on the eight
 * neighbours of each sampled site:
 *   S   = K5   - 1/4 D_eo (B K5^-1) D_oe B
 *   S^+ = K5^+ - 1/4 B^+ D_oe^+ K5^-+ B^+ D_eo^+ */
void oracle_schur_sites(const oracle_params *p, const double *Ud, const double *ind,
                        const long *sites, int nsites, int dag, double *outd)
{
    const cplx *U = (const cplx *)Ud;
    cplx *out = (cplx *)outd;
    const long V = volume(p), n = n5(p), n4 = 12 * V;
    const int L5 = p->L5;
    cplx *x = malloc(n * sizeof(cplx)), *src = malloc(n * sizeof(cplx)),
         *kx = malloc(n * sizeof(cplx)), *nb = calloc(n, sizeof(cplx));
    memcpy(x, ind, n * sizeof(cplx));
    mask_parity(p, x, 0);
    apply_K5(p, x, kx, dag);
    if (!dag) apply_B(p, x, src, 0);       /* B x, input of D_oe      */
    else memcpy(src, x, n * sizeof(cplx)); /* x,  input of D_eo^+     */
    double *K[2], *A = malloc(sizeof(double) * L5 * L5);
    cplx *col = malloc(sizeof(cplx) * L5), *v = malloc(sizeof(cplx) * L5 * 12),
         *w = malloc(sizeof(cplx) * L5 * 12);
    for (int u = 0; u < 2; ++u) {
        K[u] = malloc(sizeof(double) * L5 * L5);
        k5_matrix(p, u, dag, K[u]);
    }
    for (int k = 0; k < nsites; ++k) {
        const long xs = sites[k];
        long ys[8];
        int m = 0;
        for (int mu = 0; mu < 4; ++mu)
            for (int dir = +1; dir >= -1; dir -= 2) {
                double bc;
                ys[m++] = neighbour(p, xs, mu, dir, &bc);
            }
        /* odd neighbours: v = (B K5^-1)(D_oe B x) or K5^-+ B^+ (D_eo^+ x) */
        for (int m2 = 0; m2 < 8; ++m2) {
            const long y = ys[m2];
            for (int s = 0; s < L5; ++s) {
                cplx acc[4][3];
                hop_site(p, U, src + (long)s * n4, y, dag, acc);
                memcpy(v + s * 12, acc, sizeof(acc));
            }
            if (dag) {   /* B^+ on the slices of y */
                for (int s = 0; s < L5; ++s)
                    for (int sp = 0; sp < 4; ++sp) {
                        long from = (sp < 2) ? s + 1 : s - 1;
                        double f = 1.0;
                        if (from < 0) { from += L5; f = -p->mq; }
                        if (from >= L5) { from -= L5; f = -p->mq; }
                        for (int a = 0; a < 3; ++a)
                            w[s * 12 + sp * 3 + a] = p->b5 * v[s * 12 + sp * 3 + a] + p->c5 * f * v[from * 12 + sp * 3 + a];
                    }
                memcpy(v, w, sizeof(cplx) * L5 * 12);
            }
            for (int sp = 0; sp < 4; ++sp)   /* K5^-1 or K5^-+ */
                for (int a = 0; a < 3; ++a) {
                    for (int s = 0; s < L5; ++s) col[s] = v[s * 12 + sp * 3 + a];
                    memcpy(A, K[sp < 2], sizeof(double) * L5 * L5);
                    gauss_solve(L5, A, col);
                    for (int s = 0; s < L5; ++s) v[s * 12 + sp * 3 + a] = col[s];
                }
            if (!dag) {  /* B on the slices of y */
                for (int s = 0; s < L5; ++s)
                    for (int sp = 0; sp < 4; ++sp) {
                        long from = (sp < 2) ? s - 1 : s + 1;
                        double f = 1.0;
                        if (from < 0) { from += L5; f = -p->mq; }
                        if (from >= L5) { from -= L5; f = -p->mq; }
                        for (int a = 0; a < 3; ++a)
                            w[s * 12 + sp * 3 + a] = p->b5 * v[s * 12 + sp * 3 + a] + p->c5 * f * v[from * 12 + sp * 3 + a];
                    }
                memcpy(v, w, sizeof(cplx) * L5 * 12);
            }
            for (int s = 0; s < L5; ++s) memcpy(nb + (long)s * n4 + 12 * y, v + s * 12, 12 * sizeof(cplx));
        }
        /* back to x: D_eo (or D_oe^+) of the neighbour values */
        for (int s = 0; s < L5; ++s) {
            cplx acc[4][3];
            hop_site(p, U, nb + (long)s * n4, xs, dag, acc);
            memcpy(w + s * 12, acc, sizeof(acc));
        }
        if (dag) {   /* B^+ on the slices of x */
            for (int s = 0; s < L5; ++s)
                for (int sp = 0; sp < 4; ++sp) {
                    long from = (sp < 2) ? s + 1 : s - 1;
                    double f = 1.0;
                    if (from < 0) { from += L5; f = -p->mq; }
                    if (from >= L5) { from -= L5; f = -p->mq; }
                    for (int a = 0; a < 3; ++a)
                        v[s * 12 + sp * 3 + a] = p->b5 * w[s * 12 + sp * 3 + a] + p->c5 * f * w[from * 12 + sp * 3 + a];
                }
            memcpy(w, v, sizeof(cplx) * L5 * 12);
        }
        for (int s = 0; s < L5; ++s)
            for (int i = 0; i < 12; ++i)
                out[((long)k * L5 + s) * 12 + i] = kx[((long)s * V + xs) * 12 + i] - 0.25 * w[s * 12 + i];
        for (int m2 = 0; m2 < 8; ++m2)   /* clear the scratch entries */
            for (int s = 0; s < L5; ++s) memset(nb + (long)s * n4 + 12 * ys[m2], 0, 12 * sizeof(cplx));
    }
    free(K[0]); free(K[1]); free(A); free(col); free(v); free(w);
    free(x); free(src); free(kx); free(nb);
}

/* (S B^-1 in)(x, s) or (B^-+ S^+ in)(x, s) for even 4D sites `sites` and every
 * slice; out[n][L5][12].  B^-1 is 4D-site-local, so the forward operator is
 * oracle_schur_sites of B^-1 in (a full-lattice site-local pass), and the
 * adjoint solves B^+ y = (S^+ in)(x, .) on the slices of each sampled site. */
void oracle_schur_rp_sites(const oracle_params *p, const double *Ud, const double *ind,
                           const long *sites, int nsites, int dag, double *outd)
{
    const long n = n5(p);
    const int L5 = p->L5;
    cplx *out = (cplx *)outd;
    if (!dag) {
        cplx *x = malloc(n * sizeof(cplx)), *y = malloc(n * sizeof(cplx));
        memcpy(x, ind, n * sizeof(cplx));
        mask_parity(p, x, 0);
        apply_Binv(p, x, y, 0);
        oracle_schur_sites(p, Ud, (const double *)y, sites, nsites, 0, outd);
        free(x); free(y);
        return;
    }
    oracle_schur_sites(p, Ud, ind, sites, nsites, 1, outd);
    double *Bm[2], *A = malloc(sizeof(double) * L5 * L5);
    cplx *col = malloc(sizeof(cplx) * L5);
    for (int u = 0; u < 2; ++u) {
        Bm[u] = malloc(sizeof(double) * L5 * L5);
        b_matrix(p, u == 0, 1, Bm[u]);
    }
    for (int k = 0; k < nsites; ++k)
        for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a) {
                for (int s = 0; s < L5; ++s) col[s] = out[((long)k * L5 + s) * 12 + sp * 3 + a];
                memcpy(A, Bm[sp < 2 ? 0 : 1], sizeof(double) * L5 * L5);
                gauss_solve(L5, A, col);
                for (int s = 0; s < L5; ++s) out[((long)k * L5 + s) * 12 + sp * 3 + a] = col[s];
            }
    free(Bm[0]); free(Bm[1]); free(A); free(col);
}

/* One CGLS iteration of the asymmetric Schur system (S, S^+ and the vector
 * updates of the recursion in oracle_solve) on given full-size vectors: the
 * unit of work of the oracle's solve, timed on lattices where a whole solve
 * would take too long.  Returns ||r||^2 after the step. */
double oracle_cgls_step(const oracle_params *p, const double *Ud, double *xd, double *rd,
                        double *pd, double *sd, double *qd, double *gam)
{
    const long n = n5(p);
    cplx *x = (cplx *)xd, *r = (cplx *)rd, *pv = (cplx *)pd, *s = (cplx *)sd, *q = (cplx *)qd;
    oracle_schur(p, Ud, pd, qd, 0);
    double alpha = *gam / norm2(q, n);
    for (long i = 0; i < n; ++i) { x[i] += alpha * pv[i]; r[i] -= alpha * q[i]; }
    oracle_schur(p, Ud, rd, sd, 1);
    double gnew = norm2(s, n), beta = gnew / *gam;
    *gam = gnew;
    for (long i = 0; i < n; ++i) pv[i] = s[i] + beta * pv[i];
    return norm2(r, n);
}

/* Threads of the OpenMP timing build (the plain build runs on one thread and
 * returns 1).  Results do not depend on it: only site loops without
 * reductions run in parallel. */
int oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
