/*
 * FP64 reference ("oracle") for the O(a)-improved Wilson (clover) quark
 * operator of Boku, Ishikawa, Kuramashi and Meadows, arXiv:1709.08785.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or helper with the GPU library; the two never include or
 * link each other.
 *
 * Everything here is the plain definition, written with whole 4x4 spin
 * matrices and whole 3x3 colour matrices (no spin projection, no SU(3)
 * reconstruction, no even-odd split, no blocking):
 *
 *   D(n,m) = F(n) delta(n,m) - kappa H(n,m)                      (Sec. II-A, eq. 3)
 *   H psi(n) = sum_mu (1 - g_mu) U_mu(n) psi(n+mu)
 *            + (1 + g_mu) U_mu(n-mu)^dagger psi(n-mu)             (Sec. II-A, eq. 4)
 *
 * with periodic boundaries in all four directions (Sec. II-A).  The paper
 * states only that the gamma matrices are Hermitian with g_t diagonal; this
 * file uses the Dirac representation
 *   g_k = [[0, -i s_k], [i s_k, 0]] (k = x, y, z),  g_t = diag(1, 1, -1, -1).
 * The paper calls F a 12x12 Hermitian matrix built from the links without
 * giving a formula; this file uses the Sheikholeslami-Wohlert clover term in
 * the kappa normalisation:
 *   Q_{mu nu}(n) = sum of the four counter-clockwise plaquettes at n,
 *   Fhat_{mu nu} = (Q_{mu nu} - Q_{mu nu}^dagger) / 8,
 *   F(n) = 1 - kappa c_SW sum_{mu<nu} (g_mu g_nu) (x) Fhat_{mu nu}(n).
 *
 * Layouts (complex128 = two doubles, C order), extents L = {Lx, Ly, Lz, Lt}:
 *   links  U[mu][t][z][y][x][i][j], spinors psi[t][z][y][x][alpha][a],
 *   site matrices F[t][z][y][x][12][12] with row/column index 3*alpha + a.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ------------------------------------------------------------------ */
/* geometry                                                            */
/* ------------------------------------------------------------------ */

static long volume(const int *L) { return (long)L[0] * L[1] * L[2] * L[3]; }

static void coords(const int *L, long n, int c[4])
{
    c[0] = (int)(n % L[0]); n /= L[0];
    c[1] = (int)(n % L[1]); n /= L[1];
    c[2] = (int)(n % L[2]); n /= L[2];
    c[3] = (int)n;
}

static long site(const int *L, const int c[4])
{
    return c[0] + (long)L[0] * (c[1] + (long)L[1] * (c[2] + (long)L[2] * c[3]));
}

/* site index of n + s * mu-hat, periodic */
static long shifted(const int *L, const int c[4], int mu, int s)
{
    int d[4] = {c[0], c[1], c[2], c[3]};
    d[mu] = ((d[mu] + s) % L[mu] + L[mu]) % L[mu];
    return site(L, d);
}

/* site index of n + s1 * mu-hat + s2 * nu-hat, periodic */
static long shifted2(const int *L, const int c[4], int mu, int s1, int nu, int s2)
{
    int d[4] = {c[0], c[1], c[2], c[3]};
    d[mu] = ((d[mu] + s1) % L[mu] + L[mu]) % L[mu];
    d[nu] = ((d[nu] + s2) % L[nu] + L[nu]) % L[nu];
    return site(L, d);
}

/* ------------------------------------------------------------------ */
/* gamma matrices, Dirac representation                                */
/* ------------------------------------------------------------------ */

static void pauli(int k, cplx s[2][2])
{
    memset(s, 0, sizeof(cplx) * 4);
    if (k == 0) { s[0][1] = 1; s[1][0] = 1; }
    if (k == 1) { s[0][1] = -I; s[1][0] = I; }
    if (k == 2) { s[0][0] = 1; s[1][1] = -1; }
}

/* g_mu for mu = 0..3 (x, y, z, t); mu = 4 gives g5 = g_x g_y g_z g_t */
static void gamma_mat(int mu, cplx g[4][4])
{
    memset(g, 0, sizeof(cplx) * 16);
    if (mu < 3) {
        cplx s[2][2];
        pauli(mu, s);
        for (int i = 0; i < 2; i++)
            for (int j = 0; j < 2; j++) {
                g[i][2 + j] = -I * s[i][j];
                g[2 + i][j] = I * s[i][j];
            }
    } else if (mu == 3) {
        g[0][0] = 1; g[1][1] = 1; g[2][2] = -1; g[3][3] = -1;
    } else {
        cplx a[4][4], b[4][4], t[4][4];
        gamma_mat(0, a);
        gamma_mat(1, b);
        for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++) {
                t[i][j] = 0;
                for (int k = 0; k < 4; k++) t[i][j] += a[i][k] * b[k][j];
            }
        for (int m = 2; m < 4; m++) {
            gamma_mat(m, b);
            for (int i = 0; i < 4; i++)
                for (int j = 0; j < 4; j++) {
                    a[i][j] = 0;
                    for (int k = 0; k < 4; k++) a[i][j] += t[i][k] * b[k][j];
                }
            memcpy(t, a, sizeof(t));
        }
        memcpy(g, t, sizeof(t));
    }
}

void or_gamma(int mu, cplx *out)
{
    cplx g[4][4];
    gamma_mat(mu, g);
    memcpy(out, g, sizeof(g));
}

/* ------------------------------------------------------------------ */
/* 3x3 colour matrices                                                 */
/* ------------------------------------------------------------------ */

static void m3_mul(const cplx *a, const cplx *b, cplx *c)
{
    cplx t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            t[3 * i + j] = 0;
            for (int k = 0; k < 3; k++) t[3 * i + j] += a[3 * i + k] * b[3 * k + j];
        }
    memcpy(c, t, sizeof(t));
}

static void m3_dag(const cplx *a, cplx *c)
{
    cplx t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) t[3 * i + j] = conj(a[3 * j + i]);
    memcpy(c, t, sizeof(t));
}

static const cplx *link(const cplx *U, long V, int mu, long n) { return U + ((long)mu * V + n) * 9; }

/* ------------------------------------------------------------------ */
/* hopping term H (eq. 4)                                              */
/* ------------------------------------------------------------------ */

static void hop_site(const int *L, const cplx *U, const cplx *in, long n, cplx *acc)
{
    long V = volume(L);
    int c[4];
    coords(L, n, c);
    for (int k = 0; k < 12; k++) acc[k] = 0;
    for (int mu = 0; mu < 4; mu++) {
        cplx g[4][4];
        gamma_mat(mu, g);
        for (int dir = 0; dir < 2; dir++) {
            long m = shifted(L, c, mu, dir == 0 ? +1 : -1);
            const cplx *psi = in + m * 12;
            cplx u[9], ucp[12];
            if (dir == 0) {
                memcpy(u, link(U, V, mu, n), sizeof(u));              /* U_mu(n)            */
            } else {
                m3_dag(link(U, V, mu, m), u);                        /* U_mu(n - mu)^dag   */
            }
            /* colour multiplication of every spin component */
            for (int al = 0; al < 4; al++)
                for (int i = 0; i < 3; i++) {
                    cplx s = 0;
                    for (int j = 0; j < 3; j++) s += u[3 * i + j] * psi[3 * al + j];
                    ucp[3 * al + i] = s;
                }
            /* spin matrix (1 - g_mu) forward, (1 + g_mu) backward */
            double sg = (dir == 0) ? -1.0 : 1.0;
            for (int al = 0; al < 4; al++)
                for (int be = 0; be < 4; be++) {
                    cplx p = ((al == be) ? 1.0 : 0.0) + sg * g[al][be];
                    if (p == 0) continue;
                    for (int i = 0; i < 3; i++) acc[3 * al + i] += p * ucp[3 * be + i];
                }
        }
    }
}

void or_hop(const int *L, const cplx *U, const cplx *in, cplx *out)
{
    long V = volume(L);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < V; n++) hop_site(L, U, in, n, out + n * 12);
}

/* ------------------------------------------------------------------ */
/* clover term F                                                       */
/* ------------------------------------------------------------------ */

/* Q_{mu nu}(n): the four counter-clockwise plaquettes in the (mu, nu) plane at n */
static void clover_leaves(const int *L, const cplx *U, long n, int mu, int nu, cplx *Q)
{
    long V = volume(L);
    int c[4];
    coords(L, n, c);
    long n_pm = shifted(L, c, mu, +1), n_pn = shifted(L, c, nu, +1);
    long n_mm = shifted(L, c, mu, -1), n_mn = shifted(L, c, nu, -1);
    long n_pn_mm = shifted2(L, c, nu, +1, mu, -1);
    long n_mm_mn = shifted2(L, c, mu, -1, nu, -1);
    long n_pm_mn = shifted2(L, c, mu, +1, nu, -1);
    cplx a[9], b[9], t[9];
    for (int k = 0; k < 9; k++) Q[k] = 0;

    /* U_mu(n) U_nu(n+mu) U_mu(n+nu)^dag U_nu(n)^dag */
    m3_mul(link(U, V, mu, n), link(U, V, nu, n_pm), t);
    m3_dag(link(U, V, mu, n_pn), a); m3_mul(t, a, t);
    m3_dag(link(U, V, nu, n), a);    m3_mul(t, a, t);
    for (int k = 0; k < 9; k++) Q[k] += t[k];

    /* U_nu(n) U_mu(n+nu-mu)^dag U_nu(n-mu)^dag U_mu(n-mu) */
    m3_dag(link(U, V, mu, n_pn_mm), a); m3_mul(link(U, V, nu, n), a, t);
    m3_dag(link(U, V, nu, n_mm), a);    m3_mul(t, a, t);
    m3_mul(t, link(U, V, mu, n_mm), t);
    for (int k = 0; k < 9; k++) Q[k] += t[k];

    /* U_mu(n-mu)^dag U_nu(n-mu-nu)^dag U_mu(n-mu-nu) U_nu(n-nu) */
    m3_dag(link(U, V, mu, n_mm), a);
    m3_dag(link(U, V, nu, n_mm_mn), b); m3_mul(a, b, t);
    m3_mul(t, link(U, V, mu, n_mm_mn), t);
    m3_mul(t, link(U, V, nu, n_mn), t);
    for (int k = 0; k < 9; k++) Q[k] += t[k];

    /* U_nu(n-nu)^dag U_mu(n-nu) U_nu(n+mu-nu) U_mu(n)^dag */
    m3_dag(link(U, V, nu, n_mn), a); m3_mul(a, link(U, V, mu, n_mn), t);
    m3_mul(t, link(U, V, nu, n_pm_mn), t);
    m3_dag(link(U, V, mu, n), a);    m3_mul(t, a, t);
    for (int k = 0; k < 9; k++) Q[k] += t[k];
}

/* 12x12 F(n), row/column index 3*alpha + a */
static void clover_site(const int *L, const cplx *U, double kappa, double csw, long n, cplx *F)
{
    for (int k = 0; k < 144; k++) F[k] = 0;
    for (int k = 0; k < 12; k++) F[13 * k] = 1;
    for (int mu = 0; mu < 4; mu++)
        for (int nu = mu + 1; nu < 4; nu++) {
            cplx Q[9], Qd[9], Fh[9], gm[4][4], gn[4][4], gg[4][4];
            clover_leaves(L, U, n, mu, nu, Q);
            m3_dag(Q, Qd);
            for (int k = 0; k < 9; k++) Fh[k] = (Q[k] - Qd[k]) / 8.0;
            gamma_mat(mu, gm);
            gamma_mat(nu, gn);
            for (int i = 0; i < 4; i++)
                for (int j = 0; j < 4; j++) {
                    gg[i][j] = 0;
                    for (int k = 0; k < 4; k++) gg[i][j] += gm[i][k] * gn[k][j];
                }
            for (int al = 0; al < 4; al++)
                for (int be = 0; be < 4; be++) {
                    if (gg[al][be] == 0) continue;
                    for (int a = 0; a < 3; a++)
                        for (int b = 0; b < 3; b++)
                            F[(3 * al + a) * 12 + 3 * be + b] -= kappa * csw * gg[al][be] * Fh[3 * a + b];
                }
        }
}

void or_clover_field(const int *L, const cplx *U, double kappa, double csw, cplx *F)
{
    long V = volume(L);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < V; n++) clover_site(L, U, kappa, csw, n, F + n * 144);
}

/* Q_{mu nu}(n) for every site (3x3 per site), exposed for checks of the leaves */
void or_clover_leaves(const int *L, const cplx *U, int mu, int nu, cplx *Q)
{
    long V = volume(L);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < V; n++) clover_leaves(L, U, n, mu, nu, Q + n * 9);
}

/* out(n) = M(n) in(n) for a field of 12x12 site matrices */
void or_site_apply(const int *L, const cplx *M, const cplx *in, cplx *out)
{
    long V = volume(L);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < V; n++) {
        const cplx *m = M + n * 144;
        cplx t[12];
        for (int i = 0; i < 12; i++) {
            cplx s = 0;
            for (int j = 0; j < 12; j++) s += m[12 * i + j] * in[n * 12 + j];
            t[i] = s;
        }
        memcpy(out + n * 12, t, sizeof(t));
    }
}

/* inverse of one 12x12 matrix by Gauss-Jordan elimination with partial
   pivoting; returns 0 when the matrix is singular, 1 otherwise */
static int invert12(const cplx *M, cplx *Minv)
{
    cplx a[12][24];
    for (int i = 0; i < 12; i++)
        for (int j = 0; j < 12; j++) {
            a[i][j] = M[12 * i + j];
            a[i][12 + j] = (i == j) ? 1.0 : 0.0;
        }
    for (int col = 0; col < 12; col++) {
        int piv = col;
        for (int r = col + 1; r < 12; r++)
            if (cabs(a[r][col]) > cabs(a[piv][col])) piv = r;
        if (cabs(a[piv][col]) == 0.0) return 0;
        if (piv != col)
            for (int j = 0; j < 24; j++) { cplx t = a[col][j]; a[col][j] = a[piv][j]; a[piv][j] = t; }
        cplx d = 1.0 / a[col][col];
        for (int j = 0; j < 24; j++) a[col][j] *= d;
        for (int r = 0; r < 12; r++) {
            if (r == col) continue;
            cplx f = a[r][col];
            if (f == 0) continue;
            for (int j = 0; j < 24; j++) a[r][j] -= f * a[col][j];
        }
    }
    for (int i = 0; i < 12; i++)
        for (int j = 0; j < 12; j++) Minv[12 * i + j] = a[i][12 + j];
    return 1;
}

/* inverse of every 12x12 site matrix.  Returns the number of singular sites
   (0 on success). */
long or_site_invert(const int *L, const cplx *M, cplx *Minv)
{
    long V = volume(L), bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (long n = 0; n < V; n++)
        if (!invert12(M + n * 144, Minv + n * 144)) bad++;
    return bad;
}

/* ------------------------------------------------------------------ */
/* the Wilson-clover operator D = F - kappa H (eq. 3)                  */
/* ------------------------------------------------------------------ */

void or_apply_D(const int *L, const cplx *U, const cplx *F, double kappa, const cplx *in, cplx *out)
{
    long V = volume(L);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < V; n++) {
        cplx h[12], t[12];
        hop_site(L, U, in, n, h);
        const cplx *m = F + n * 144;
        for (int i = 0; i < 12; i++) {
            cplx s = 0;
            for (int j = 0; j < 12; j++) s += m[12 * i + j] * in[n * 12 + j];
            t[i] = s - kappa * h[i];
        }
        memcpy(out + n * 12, t, sizeof(t));
    }
}

/* (D in)(n) at a list of sites only, building F(n) from the links on the fly.
   For checks of full-size lattices where a whole F field would not fit. */
void or_apply_D_sites(const int *L, const cplx *U, double kappa, double csw, const cplx *in,
                      const long *sites, long nsites, cplx *out)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (long s = 0; s < nsites; s++) {
        long n = sites[s];
        cplx h[12], F[144];
        hop_site(L, U, in, n, h);
        clover_site(L, U, kappa, csw, n, F);
        for (int i = 0; i < 12; i++) {
            cplx a = 0;
            for (int j = 0; j < 12; j++) a += F[12 * i + j] * in[n * 12 + j];
            out[s * 12 + i] = a - kappa * h[i];
        }
    }
}

/* F(n) in(n), or F(n)^-1 in(n) when inverse is set, at a list of sites, with
   F(n) built from the links on the fly (Sec. II-A).  Returns the number of
   singular clover matrices. */
long or_clover_sites(const int *L, const cplx *U, double kappa, double csw, const cplx *in,
                     const long *sites, long nsites, int inverse, cplx *out)
{
    long bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : bad)
    for (long s = 0; s < nsites; s++) {
        long n = sites[s];
        cplx F[144], Fi[144];
        const cplx *M = F;
        clover_site(L, U, kappa, csw, n, F);
        if (inverse) {
            if (!invert12(F, Fi)) { bad++; continue; }
            M = Fi;
        }
        for (int i = 0; i < 12; i++) {
            cplx a = 0;
            for (int j = 0; j < 12; j++) a += M[12 * i + j] * in[n * 12 + j];
            out[s * 12 + i] = a;
        }
    }
    return bad;
}

/* MULT at a list of sites (Sec. II-B, eq. 9): out(n) = F(n)^-1 (H in)(n), with
   F(n) built and inverted on the fly.  H at n reads only the neighbours, all
   of the other parity.  Returns the number of singular clover matrices. */
long or_htilde_sites(const int *L, const cplx *U, double kappa, double csw, const cplx *in,
                     const long *sites, long nsites, cplx *out)
{
    long bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : bad)
    for (long s = 0; s < nsites; s++) {
        long n = sites[s];
        cplx h[12], F[144], Fi[144];
        hop_site(L, U, in, n, h);
        clover_site(L, U, kappa, csw, n, F);
        if (!invert12(F, Fi)) { bad++; continue; }
        for (int i = 0; i < 12; i++) {
            cplx a = 0;
            for (int j = 0; j < 12; j++) a += Fi[12 * i + j] * h[j];
            out[s * 12 + i] = a;
        }
    }
    return bad;
}

/* (D-hat_ee xe)(n) = xe(n) - kappa^2 [F_ee^-1 H_eo F_oo^-1 H_oe xe](n) (Sec. II-B,
   eq. 8, read with H_oe as the inner factor) at a list of even sites only, for
   checks of lattices where whole clover fields would not fit.  xe is a
   full-lattice field; only its even sites are read.  The clover blocks of the
   listed sites and of their odd neighbours are built and inverted on the fly.
   Returns the number of singular clover matrices met (0 on success). */
long or_dhat_ee_sites(const int *L, const cplx *U, double kappa, double csw, const cplx *xe,
                      const long *sites, long nsites, cplx *out)
{
    long V = volume(L), bad = 0;
    /* odd neighbours of the listed sites, each once */
    char *mark = calloc((size_t)V, 1);
    long *odd = malloc(sizeof(long) * 8 * (nsites > 0 ? nsites : 1));
    long nodd = 0;
    for (long s = 0; s < nsites; s++) {
        int c[4];
        coords(L, sites[s], c);
        for (int mu = 0; mu < 4; mu++)
            for (int sg = -1; sg <= 1; sg += 2) {
                long m = shifted(L, c, mu, sg);
                if (!mark[m]) { mark[m] = 1; odd[nodd++] = m; }
            }
    }
    /* y(m) = F_oo^-1(m) (H_oe xe)(m) at those odd sites, zero elsewhere; H_oe
       at an odd site reads only its even neighbours */
    cplx *y = calloc((size_t)V * 12, sizeof(cplx));
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : bad)
    for (long k = 0; k < nodd; k++) {
        long m = odd[k];
        cplx h[12], F[144], Fi[144];
        hop_site(L, U, xe, m, h);
        clover_site(L, U, kappa, csw, m, F);
        if (!invert12(F, Fi)) { bad++; continue; }
        for (int i = 0; i < 12; i++) {
            cplx a = 0;
            for (int j = 0; j < 12; j++) a += Fi[12 * i + j] * h[j];
            y[m * 12 + i] = a;
        }
    }
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : bad)
    for (long s = 0; s < nsites; s++) {
        long n = sites[s];
        cplx h[12], F[144], Fi[144];
        hop_site(L, U, y, n, h);
        clover_site(L, U, kappa, csw, n, F);
        if (!invert12(F, Fi)) { bad++; continue; }
        for (int i = 0; i < 12; i++) {
            cplx a = 0;
            for (int j = 0; j < 12; j++) a += Fi[12 * i + j] * h[j];
            out[s * 12 + i] = xe[n * 12 + i] - kappa * kappa * a;
        }
    }
    free(y);
    free(odd);
    free(mark);
    return bad;
}

/* ||b - D x||^2 and ||b||^2 over the whole lattice, F built on the fly.
   Accumulated per site, then summed in site order. */
void or_residual(const int *L, const cplx *U, double kappa, double csw, const cplx *b, const cplx *x,
                 double *res2, double *b2)
{
    long V = volume(L);
    double *part = (double *)malloc(sizeof(double) * 2 * V);
#pragma omp parallel for schedule(dynamic, 256)
    for (long n = 0; n < V; n++) {
        cplx h[12], F[144];
        hop_site(L, U, x, n, h);
        clover_site(L, U, kappa, csw, n, F);
        double r = 0, bb = 0;
        for (int i = 0; i < 12; i++) {
            cplx a = 0;
            for (int j = 0; j < 12; j++) a += F[12 * i + j] * x[n * 12 + j];
            cplx d = b[n * 12 + i] - (a - kappa * h[i]);
            r += creal(d) * creal(d) + cimag(d) * cimag(d);
            bb += creal(b[n * 12 + i]) * creal(b[n * 12 + i]) + cimag(b[n * 12 + i]) * cimag(b[n * 12 + i]);
        }
        part[2 * n] = r;
        part[2 * n + 1] = bb;
    }
    double r = 0, bb = 0;
    for (long n = 0; n < V; n++) { r += part[2 * n]; bb += part[2 * n + 1]; }
    free(part);
    *res2 = r;
    *b2 = bb;
}

/* ------------------------------------------------------------------ */
/* plain BiCGStab (van der Vorst) on the full operator                 */
/* ------------------------------------------------------------------ */

static cplx vdot(long N, const cplx *a, const cplx *b)
{
    double re = 0, im = 0;
#pragma omp parallel for reduction(+ : re, im) schedule(static)
    for (long i = 0; i < N; i++) {
        cplx p = conj(a[i]) * b[i];
        re += creal(p);
        im += cimag(p);
    }
    return re + I * im;
}

static double vnorm2(long N, const cplx *a) { return creal(vdot(N, a, a)); }

/* Solve D x = b.  x holds the initial guess on entry.  Iterates until the
   recursive residual falls below tol, then recomputes the true residual and
   restarts from it when that is still above tol.  Returns 0 on success,
   1 when maxit is reached, 2 on breakdown.  iters and relres report the
   iteration count and the final true relative residual. */
int or_bicgstab(const int *L, const cplx *U, const cplx *F, double kappa, const cplx *b, cplx *x,
                double tol, int maxit, int *iters, double *relres)
{
    long V = volume(L), N = V * 12;
    cplx *r = malloc(sizeof(cplx) * N), *rt = malloc(sizeof(cplx) * N), *p = malloc(sizeof(cplx) * N);
    cplx *v = malloc(sizeof(cplx) * N), *s = malloc(sizeof(cplx) * N), *t = malloc(sizeof(cplx) * N);
    double bn = sqrt(vnorm2(N, b));
    int it = 0, status = 1;
    if (bn == 0) {
        memset(x, 0, sizeof(cplx) * N);
        *iters = 0;
        *relres = 0;
        free(r); free(rt); free(p); free(v); free(s); free(t);
        return 0;
    }
    for (int restart = 0; restart < 20 && it < maxit; restart++) {
        or_apply_D(L, U, F, kappa, x, t);
        for (long i = 0; i < N; i++) { r[i] = b[i] - t[i]; rt[i] = r[i]; p[i] = 0; v[i] = 0; }
        if (sqrt(vnorm2(N, r)) / bn < tol) { status = 0; break; }
        cplx rho = 1, alpha = 1, omega = 1;
        int broke = 0;
        while (it < maxit) {
            it++;
            cplx rho1 = vdot(N, rt, r);
            if (cabs(rho1) == 0) { broke = 1; break; }
            cplx beta = (rho1 / rho) * (alpha / omega);
            for (long i = 0; i < N; i++) p[i] = r[i] + beta * (p[i] - omega * v[i]);
            or_apply_D(L, U, F, kappa, p, v);
            cplx den = vdot(N, rt, v);
            if (cabs(den) == 0) { broke = 1; break; }
            alpha = rho1 / den;
            for (long i = 0; i < N; i++) s[i] = r[i] - alpha * v[i];
            if (sqrt(vnorm2(N, s)) / bn < tol) {
                for (long i = 0; i < N; i++) x[i] += alpha * p[i];
                break;
            }
            or_apply_D(L, U, F, kappa, s, t);
            double tt = vnorm2(N, t);
            if (tt == 0) { broke = 1; break; }
            omega = vdot(N, t, s) / tt;
            for (long i = 0; i < N; i++) { x[i] += alpha * p[i] + omega * s[i]; r[i] = s[i] - omega * t[i]; }
            rho = rho1;
            if (sqrt(vnorm2(N, r)) / bn < tol) break;
        }
        or_apply_D(L, U, F, kappa, x, t);
        for (long i = 0; i < N; i++) r[i] = b[i] - t[i];
        double rr = sqrt(vnorm2(N, r)) / bn;
        *relres = rr;
        if (rr < tol) { status = 0; break; }
        if (broke && it >= maxit) { status = 2; break; }
    }
    if (status != 0) {
        or_apply_D(L, U, F, kappa, x, t);
        for (long i = 0; i < N; i++) r[i] = b[i] - t[i];
        *relres = sqrt(vnorm2(N, r)) / bn;
    } else {
        or_apply_D(L, U, F, kappa, x, t);
        for (long i = 0; i < N; i++) r[i] = b[i] - t[i];
        *relres = sqrt(vnorm2(N, r)) / bn;
    }
    *iters = it;
    free(r); free(rt); free(p); free(v); free(s); free(t);
    return status;
}

/* ------------------------------------------------------------------ */
/* link gradient                                                        */
/* ------------------------------------------------------------------ */

/* Gradient, in the convention dg = Re sum_links sum_ab conj(G_ab) dU_ab, of
     g(U) = -Re <lam, D[U] x>          (lam and x held fixed).
   At lam = D^-dagger eta and x = D^-1 b this is the gradient of
   L = Re <eta, D^-1 b> with respect to the links, because
   dL = -Re <lam, (dD) x> with dD = dF - kappa dH (eq. 3).
   Hopping part (eq. 4), for link U_mu(m):
     G += kappa sum_alpha [ lam(m)_alpha conj(((1 - g_mu) x(m+mu))_alpha)^T
                          + ((1 + g_mu) x(m))_alpha conj(lam(m+mu)_alpha)^T ]   (outer products in colour)
   Clover part: dF = -kappa c_SW sum_{mu<nu} g_mu g_nu (x) dFhat_{mu nu}, dFhat = (dQ - dQ^dag)/8,
   so dg = (kappa c_SW / 8) Re tr(N^T dQ) per site and plane with
     M_ab = sum_{alpha beta} conj(lam_{alpha a}) (g_mu g_nu)_{alpha beta} x_{beta b},  N = M - M^dag.
   A leaf W = f1 f2 f3 f4 whose factor k is a link (or its dagger) contributes, with
   A = f1..f_{k-1} and B = f_{k+1}..f4:  G += (kappa c_SW / 8) (B N^T A)^dagger for an
   undaggered factor and (kappa c_SW / 8) B N^T A for a daggered one.
   G has the canonical link layout. */

/* the four counter-clockwise leaves of Q_{mu nu}(n): per factor (0 = mu-link,
   1 = nu-link), its root offset along (mu, nu), and whether it is daggered */
static const int kLeaf[4][4][4] = {
    {{0, 0, 0, 0}, {1, 1, 0, 0}, {0, 0, 1, 1}, {1, 0, 0, 1}},
    {{1, 0, 0, 0}, {0, -1, 1, 1}, {1, -1, 0, 1}, {0, -1, 0, 0}},
    {{0, -1, 0, 1}, {1, -1, -1, 1}, {0, -1, -1, 0}, {1, 0, -1, 0}},
    {{1, 0, -1, 1}, {0, 0, -1, 0}, {1, 1, -1, 0}, {0, 0, 0, 1}},
};

void or_link_grad(const int *L, const cplx *U, const cplx *lam, const cplx *x, double kappa, double csw,
                  int include_clover, cplx *G)
{
    long V = volume(L);
    memset(G, 0, sizeof(cplx) * 36 * V);
#pragma omp parallel for schedule(static)
    for (long m = 0; m < V; m++) {
        int c[4];
        coords(L, m, c);
        for (int mu = 0; mu < 4; mu++) {
            cplx g[4][4];
            gamma_mat(mu, g);
            long mp = shifted(L, c, mu, +1);
            cplx y[12], z[12];   /* y = (1 - g) x(m+mu), z = (1 + g) x(m) */
            for (int al = 0; al < 4; al++)
                for (int a = 0; a < 3; a++) {
                    cplx sy = 0, sz = 0;
                    for (int be = 0; be < 4; be++) {
                        cplx d = (al == be) ? 1.0 : 0.0;
                        sy += (d - g[al][be]) * x[mp * 12 + 3 * be + a];
                        sz += (d + g[al][be]) * x[m * 12 + 3 * be + a];
                    }
                    y[3 * al + a] = sy;
                    z[3 * al + a] = sz;
                }
            cplx *Gl = G + ((long)mu * V + m) * 9;
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) {
                    cplx s = 0;
                    for (int al = 0; al < 4; al++)
                        s += lam[m * 12 + 3 * al + a] * conj(y[3 * al + b]) + z[3 * al + a] * conj(lam[mp * 12 + 3 * al + b]);
                    Gl[3 * a + b] += kappa * s;
                }
        }
    }
    if (!include_clover || csw == 0.0) return;
    const double fac = kappa * csw / 8.0;
    for (long n = 0; n < V; n++) {
        int c[4];
        coords(L, n, c);
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++) {
                cplx gm[4][4], gn[4][4], gg[4][4], M[9], N[9], NT[9];
                gamma_mat(mu, gm);
                gamma_mat(nu, gn);
                for (int i = 0; i < 4; i++)
                    for (int j = 0; j < 4; j++) {
                        gg[i][j] = 0;
                        for (int k = 0; k < 4; k++) gg[i][j] += gm[i][k] * gn[k][j];
                    }
                for (int a = 0; a < 3; a++)
                    for (int b = 0; b < 3; b++) {
                        cplx s = 0;
                        for (int al = 0; al < 4; al++)
                            for (int be = 0; be < 4; be++)
                                s += conj(lam[n * 12 + 3 * al + a]) * gg[al][be] * x[n * 12 + 3 * be + b];
                        M[3 * a + b] = s;
                    }
                for (int a = 0; a < 3; a++)
                    for (int b = 0; b < 3; b++) N[3 * a + b] = M[3 * a + b] - conj(M[3 * b + a]);
                for (int a = 0; a < 3; a++)
                    for (int b = 0; b < 3; b++) NT[3 * a + b] = N[3 * b + a];
                for (int lf = 0; lf < 4; lf++) {
                    cplx f[4][9];
                    long site_of[4];
                    int dir_of[4];
                    for (int k = 0; k < 4; k++) {
                        const int *e = kLeaf[lf][k];
                        int dir = e[0] == 0 ? mu : nu;
                        long sn = shifted2(L, c, mu, e[1], nu, e[2]);
                        site_of[k] = sn;
                        dir_of[k] = dir;
                        if (e[3]) m3_dag(link(U, V, dir, sn), f[k]);
                        else memcpy(f[k], link(U, V, dir, sn), sizeof(cplx) * 9);
                    }
                    for (int k = 0; k < 4; k++) {
                        cplx A[9], B[9], P[9];
                        for (int q = 0; q < 9; q++) { A[q] = (q % 4 == 0) ? 1.0 : 0.0; B[q] = A[q]; }
                        for (int j = 0; j < k; j++) m3_mul(A, f[j], A);
                        for (int j = k + 1; j < 4; j++) m3_mul(B, f[j], B);
                        m3_mul(B, NT, P);
                        m3_mul(P, A, P);
                        cplx *Gl = G + ((long)dir_of[k] * V + site_of[k]) * 9;
                        if (kLeaf[lf][k][3]) {
                            for (int q = 0; q < 9; q++) Gl[q] += fac * P[q];
                        } else {
                            for (int a = 0; a < 3; a++)
                                for (int b = 0; b < 3; b++) Gl[3 * a + b] += fac * conj(P[3 * b + a]);
                        }
                    }
                }
            }
    }
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
