/*
 * FP64 CPU oracle for the twisted-mass disconnected-loop hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source, header, table or constant
 * with the HIP library.
 *
 * Style: plain, slow, obviously correct.  Every operator is applied from its
 * definition: explicit 4x4 spin matrices (no spin projection), explicit 3x3
 * colour matrices, full-lattice vectors with parity masks for the even-odd
 * Schur complement, numerically inverted twist matrices, and the adjoint of
 * the hopping term built block by block.  Canonical layouts only:
 *   site   s = x + Lx*(y + Ly*(z + Lz*t)),  coordinates ordered (x,y,z,t)
 *   spinor psi[s][spin 4][colour 3]   (complex double, interleaved)
 *   links  U[mu][s][row 3][col 3],  U_mu(x) on the link x -> x+mu
 * The fermion boundary phase (t_bc = -1 antiperiodic, +1 periodic) sits on
 * hops that cross the t boundary and is never stored in U.
 *
 * Conventions (readings of the paper; each is listed with its reason in the
 * design notes):
 *   eps = 2*kappa*mu (kappa normalisation of the twisted-mass operator, as in
 *         the Hopping Parameter Expansion section, where B = (1 + i 2 kappa mu
 *         gamma5)^-1 and H = 2 kappa * (hopping term)).
 *   R   = 1 + i eps gamma5           (local twist; B = R^-1)
 *   H psi(x) = -kappa sum_mu [ (1-gamma_mu) U_mu(x) psi(x+mu)
 *                             +(1+gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
 *   M(mu) = R + H ;  the d flavour uses eps -> -eps (section "one-end trick").
 *   Even-odd Schur system (appendix A.1, eq. A.2, "asymmetric"):
 *     Ahat = R_ee - H_eo R_oo^-1 H_oe,  bhat_e = b_e - H_eo R_oo^-1 b_o,
 *     psi_o = R_oo^-1 (b_o - H_oe psi_e).
 *   Symmetric form (eq. A.3): 1 - R_ee^-1 H_eo R_oo^-1 H_oe, rhs R_ee^-1 bhat_e.
 *   Gamma basis: chiral, gamma_k = [[0,-i s_k],[i s_k,0]], gamma_4 = [[0,1],[1,0]],
 *   gamma5 = gamma1 gamma2 gamma3 gamma4;  Gamma_n = g1^n0 g2^n1 g3^n2 g4^n3.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

typedef double complex cplx;

/* ------------------------------------------------------------------ */
/* geometry                                                            */
/* ------------------------------------------------------------------ */

static long vol(const int L[4]) { return (long)L[0] * L[1] * L[2] * L[3]; }

static void coords(const int L[4], long s, int c[4])
{
    c[0] = (int)(s % L[0]); s /= L[0];
    c[1] = (int)(s % L[1]); s /= L[1];
    c[2] = (int)(s % L[2]); s /= L[2];
    c[3] = (int)s;
}

static long lex(const int L[4], const int c[4])
{
    return c[0] + (long)L[0] * (c[1] + (long)L[1] * (c[2] + (long)L[2] * c[3]));
}

static int parity(const int L[4], long s)
{
    int c[4];
    coords(L, s, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

/* neighbour of s one step along mu in direction dir (+1/-1); *phase gets the
 * fermion boundary factor of that hop */
static long step(const int L[4], int t_bc, long s, int mu, int dir, double *phase)
{
    int c[4];
    coords(L, s, c);
    c[mu] += dir;
    *phase = 1.0;
    if (c[mu] >= L[mu]) { c[mu] -= L[mu]; if (mu == 3) *phase = t_bc; }
    if (c[mu] < 0)      { c[mu] += L[mu]; if (mu == 3) *phase = t_bc; }
    return lex(L, c);
}

void or_site_parity(const int L[4], int *par_out)
{
    long V = vol(L);
    for (long s = 0; s < V; s++) par_out[s] = parity(L, s);
}

void or_neighbours(const int L[4], long *nb_out)
{
    /* nb_out[s][2*mu + (0: +mu, 1: -mu)] */
    long V = vol(L);
    for (long s = 0; s < V; s++)
        for (int mu = 0; mu < 4; mu++) {
            double ph;
            nb_out[8 * s + 2 * mu + 0] = step(L, 1, s, mu, +1, &ph);
            nb_out[8 * s + 2 * mu + 1] = step(L, 1, s, mu, -1, &ph);
        }
}

/* ------------------------------------------------------------------ */
/* gamma matrices                                                      */
/* ------------------------------------------------------------------ */

static void matmul4(const cplx A[4][4], const cplx B[4][4], cplx C[4][4])
{
    cplx T[4][4];
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            cplx acc = 0;
            for (int k = 0; k < 4; k++) acc += A[i][k] * B[k][j];
            T[i][j] = acc;
        }
    memcpy(C, T, sizeof(T));
}

static void gamma_mu(int mu, cplx G[4][4])
{
    /* Pauli matrices sigma_1..3 */
    const cplx sig[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    memset(G, 0, sizeof(cplx) * 16);
    if (mu == 3) {
        for (int i = 0; i < 2; i++) { G[i][i + 2] = 1; G[i + 2][i] = 1; }
        return;
    }
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) {
            G[i][j + 2] = -I * sig[mu][i][j];
            G[i + 2][j] = I * sig[mu][i][j];
        }
}

static void identity4(cplx G[4][4])
{
    memset(G, 0, sizeof(cplx) * 16);
    for (int i = 0; i < 4; i++) G[i][i] = 1;
}

void or_gamma(int n, double *out /* [4][4] complex */)
{
    cplx G[4][4], g[4][4];
    identity4(G);
    for (int mu = 0; mu < 4; mu++)
        if ((n >> mu) & 1) {
            gamma_mu(mu, g);
            matmul4(G, g, G);
        }
    memcpy(out, G, sizeof(G));
}

static void gamma5(cplx G[4][4]) { or_gamma(15, (double *)G); }

/* ------------------------------------------------------------------ */
/* local spin matrices                                                  */
/* ------------------------------------------------------------------ */

/* general 4x4 complex inverse, Gauss-Jordan with partial pivoting */
static void inv4(const cplx A[4][4], cplx Ai[4][4])
{
    cplx a[4][8];
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 8; j++) a[i][j] = (j < 4) ? A[i][j] : (cplx)(j - 4 == i);
    for (int c = 0; c < 4; c++) {
        int piv = c;
        for (int r = c + 1; r < 4; r++)
            if (cabs(a[r][c]) > cabs(a[piv][c])) piv = r;
        if (piv != c)
            for (int j = 0; j < 8; j++) { cplx t = a[c][j]; a[c][j] = a[piv][j]; a[piv][j] = t; }
        cplx d = a[c][c];
        for (int j = 0; j < 8; j++) a[c][j] /= d;
        for (int r = 0; r < 4; r++)
            if (r != c) {
                cplx f = a[r][c];
                for (int j = 0; j < 8; j++) a[r][j] -= f * a[c][j];
            }
    }
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) Ai[i][j] = a[i][j + 4];
}

static void adj4(const cplx A[4][4], cplx Ad[4][4])
{
    cplx T[4][4];
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) T[i][j] = conj(A[j][i]);
    memcpy(Ad, T, sizeof(T));
}

/* which = 0: R, 1: R^dag, 2: R^-1, 3: (R^-1)^dag, with R = 1 + i eps gamma5 */
static void twist_matrix(double eps, int which, cplx T[4][4])
{
    cplx g5[4][4], R[4][4];
    gamma5(g5);
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) R[i][j] = (i == j) + I * eps * g5[i][j];
    if (which == 0) { memcpy(T, R, sizeof(R)); return; }
    if (which == 1) { adj4(R, T); return; }
    cplx Ri[4][4];
    inv4(R, Ri);
    if (which == 2) { memcpy(T, Ri, sizeof(Ri)); return; }
    adj4(Ri, T);
}

/* out[s] = (S (x) 1_colour) in[s] for every site */
static void apply_spin_local(long V, const cplx S[4][4], const cplx *in, cplx *out)
{
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        const cplx *p = in + 12 * s;
        cplx r[12];
        for (int a = 0; a < 4; a++)
            for (int c = 0; c < 3; c++) {
                cplx acc = 0;
                for (int b = 0; b < 4; b++) acc += S[a][b] * p[3 * b + c];
                r[3 * a + c] = acc;
            }
        memcpy(out + 12 * s, r, sizeof(r));
    }
}

void or_twist(const int L[4], double eps, int which, const double *in, double *out)
{
    cplx T[4][4];
    twist_matrix(eps, which, T);
    apply_spin_local(vol(L), T, (const cplx *)in, (cplx *)out);
}

/* ------------------------------------------------------------------ */
/* hopping term                                                         */
/* ------------------------------------------------------------------ */

/* acc += phase * (P (x) W) psi, with W = U or U^dag */
static void add_block(cplx acc[12], double coef, const cplx P[4][4], const cplx *U,
                      int dagger_U, const cplx *psi)
{
    cplx W[3][3];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) W[i][j] = dagger_U ? conj(U[3 * j + i]) : U[3 * i + j];
    cplx Wpsi[4][3];
    for (int b = 0; b < 4; b++)
        for (int i = 0; i < 3; i++) {
            cplx t = 0;
            for (int j = 0; j < 3; j++) t += W[i][j] * psi[3 * b + j];
            Wpsi[b][i] = t;
        }
    for (int a = 0; a < 4; a++)
        for (int i = 0; i < 3; i++) {
            cplx t = 0;
            for (int b = 0; b < 4; b++) t += P[a][b] * Wpsi[b][i];
            acc[3 * a + i] += coef * t;
        }
}

/*
 * adj = 0:  out = H psi
 *   (H psi)(x) = -kappa sum_mu [(1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^dag psi(x-mu)]
 * adj = 1:  out = H^dag psi, the block-wise conjugate transpose of the same
 *   matrix: the block H[y][x] for y = x-mu is -kappa (1-g_mu) U_mu(x-mu), its
 *   adjoint -kappa (1-g_mu) U_mu(x-mu)^dag multiplies psi(x-mu); the block
 *   H[y][x] for y = x+mu is -kappa (1+g_mu) U_mu(x)^dag, its adjoint
 *   -kappa (1+g_mu) U_mu(x) multiplies psi(x+mu).
 */
void or_hop(const int L[4], double kappa, int t_bc, const double *Ud, const double *ind,
            double *outd, int adj)
{
    const cplx *U = (const cplx *)Ud;
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    long V = vol(L);
    cplx Pm[4][4][4], Pp[4][4][4]; /* 1 - g_mu, 1 + g_mu */
    for (int mu = 0; mu < 4; mu++) {
        cplx g[4][4];
        gamma_mu(mu, g);
        for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++) {
                Pm[mu][i][j] = (i == j) - g[i][j];
                Pp[mu][i][j] = (i == j) + g[i][j];
            }
    }
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        cplx acc[12] = {0};
        for (int mu = 0; mu < 4; mu++) {
            double phf, phb;
            long sf = step(L, t_bc, s, mu, +1, &phf);
            long sb = step(L, t_bc, s, mu, -1, &phb);
            const cplx *Uf = U + 9 * ((long)mu * V + s);   /* U_mu(x)    */
            const cplx *Ub = U + 9 * ((long)mu * V + sb);  /* U_mu(x-mu) */
            if (!adj) {
                add_block(acc, -kappa * phf, (const cplx(*)[4])Pm[mu], Uf, 0, in + 12 * sf);
                add_block(acc, -kappa * phb, (const cplx(*)[4])Pp[mu], Ub, 1, in + 12 * sb);
            } else {
                add_block(acc, -kappa * phf, (const cplx(*)[4])Pp[mu], Uf, 0, in + 12 * sf);
                add_block(acc, -kappa * phb, (const cplx(*)[4])Pm[mu], Ub, 1, in + 12 * sb);
            }
        }
        memcpy(out + 12 * s, acc, sizeof(acc));
    }
}

/* out = M psi (adj=0) or M^dag psi (adj=1), M = R + H */
void or_apply_M(const int L[4], double kappa, double eps, int t_bc, const double *U,
                const double *in, double *out, int adj)
{
    long V = vol(L);
    cplx *tmp = malloc(sizeof(cplx) * 12 * V);
    or_hop(L, kappa, t_bc, U, in, (double *)tmp, adj);
    or_twist(L, eps, adj ? 1 : 0, in, out);
    cplx *o = (cplx *)out;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < 12 * V; i++) o[i] += tmp[i];
    free(tmp);
}

/* zero every site whose parity is not p */
static void keep_parity(const int L[4], int p, cplx *v)
{
    long V = vol(L);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++)
        if (parity(L, s) != p) memset(v + 12 * s, 0, sizeof(cplx) * 12);
}

/*
 * Schur complement on the even sites, applied to the even part of a full
 * vector; odd sites of the output are zero.
 *   form 0 (A.2): Ahat = R_ee - H_eo R_oo^-1 H_oe
 *   form 1 (A.3): Ahat = 1 - R_ee^-1 H_eo R_oo^-1 H_oe
 * adj = 1 applies the adjoint, built from H^dag and the adjoint twists, with the
 * factors in reverse order.
 */
void or_schur(const int L[4], double kappa, double eps, int t_bc, const double *U,
              const double *in, double *out, int adj, int form)
{
    long V = vol(L);
    size_t n = sizeof(cplx) * 12 * V;
    cplx *xe = malloc(n), *y = malloc(n), *z = malloc(n);
    cplx *o = (cplx *)out;
    memcpy(xe, in, n);
    keep_parity(L, 0, xe);
    if (form == 0) {
        /* R_ee x - H_eo R_oo^-1 H_oe x; adjoint: R^dag x - H^dag_eo (R^-1)^dag H^dag_oe x */
        or_hop(L, kappa, t_bc, U, (double *)xe, (double *)y, adj);
        keep_parity(L, 1, y);
        or_twist(L, eps, adj ? 3 : 2, (double *)y, (double *)z);
        or_hop(L, kappa, t_bc, U, (double *)z, (double *)y, adj);
        keep_parity(L, 0, y);
        or_twist(L, eps, adj ? 1 : 0, (double *)xe, (double *)z);
        for (long i = 0; i < 12 * V; i++) o[i] = z[i] - y[i];
    } else if (!adj) {
        /* x - R_ee^-1 H_eo R_oo^-1 H_oe x */
        or_hop(L, kappa, t_bc, U, (double *)xe, (double *)y, 0);
        keep_parity(L, 1, y);
        or_twist(L, eps, 2, (double *)y, (double *)z);
        or_hop(L, kappa, t_bc, U, (double *)z, (double *)y, 0);
        keep_parity(L, 0, y);
        or_twist(L, eps, 2, (double *)y, (double *)z);
        for (long i = 0; i < 12 * V; i++) o[i] = xe[i] - z[i];
    } else {
        /* x - H^dag_eo (R_oo^-1)^dag H^dag_oe (R_ee^-1)^dag x */
        or_twist(L, eps, 3, (double *)xe, (double *)y);
        or_hop(L, kappa, t_bc, U, (double *)y, (double *)z, 1);
        keep_parity(L, 1, z);
        or_twist(L, eps, 3, (double *)z, (double *)y);
        or_hop(L, kappa, t_bc, U, (double *)y, (double *)z, 1);
        keep_parity(L, 0, z);
        for (long i = 0; i < 12 * V; i++) o[i] = xe[i] - z[i];
    }
    keep_parity(L, 0, o);
    free(xe); free(y); free(z);
}

/* bhat_e = b_e - H_eo R_oo^-1 b_o  (form 0); times R_ee^-1 for form 1.
 * Output: even sites hold bhat_e, odd sites zero. */
void or_source_prep(const int L[4], double kappa, double eps, int t_bc, const double *U,
                    const double *b, double *bhat, int form)
{
    long V = vol(L);
    size_t n = sizeof(cplx) * 12 * V;
    cplx *bo = malloc(n), *y = malloc(n), *z = malloc(n);
    memcpy(bo, b, n);
    keep_parity(L, 1, bo);
    or_twist(L, eps, 2, (double *)bo, (double *)y);
    or_hop(L, kappa, t_bc, U, (double *)y, (double *)z, 0);
    keep_parity(L, 0, z);
    cplx *o = (cplx *)bhat;
    const cplx *bb = (const cplx *)b;
    for (long i = 0; i < 12 * V; i++) o[i] = bb[i] - z[i];
    keep_parity(L, 0, o);
    if (form == 1) {
        or_twist(L, eps, 2, bhat, (double *)y);
        memcpy(bhat, y, n);
    }
    free(bo); free(y); free(z);
}

/* full = (psi_e, psi_o) with psi_o = R_oo^-1 (b_o - H_oe psi_e) */
void or_reconstruct(const int L[4], double kappa, double eps, int t_bc, const double *U,
                    const double *b, const double *xe_in, double *full)
{
    long V = vol(L);
    size_t n = sizeof(cplx) * 12 * V;
    cplx *xe = malloc(n), *y = malloc(n), *z = malloc(n);
    memcpy(xe, xe_in, n);
    keep_parity(L, 0, xe);
    or_hop(L, kappa, t_bc, U, (double *)xe, (double *)y, 0);
    const cplx *bb = (const cplx *)b;
    for (long i = 0; i < 12 * V; i++) y[i] = bb[i] - y[i];
    keep_parity(L, 1, y);
    or_twist(L, eps, 2, (double *)y, (double *)z);
    keep_parity(L, 1, z);
    cplx *o = (cplx *)full;
    for (long i = 0; i < 12 * V; i++) o[i] = xe[i] + z[i];
    free(xe); free(y); free(z);
}

/* ------------------------------------------------------------------ */
/* vector helpers                                                       */
/* ------------------------------------------------------------------ */

static double norm2(long n, const cplx *v)
{
    double s = 0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (long i = 0; i < n; i++) s += creal(v[i]) * creal(v[i]) + cimag(v[i]) * cimag(v[i]);
    return s;
}

/* ------------------------------------------------------------------ */
/* solver: CG on the normal equations of the Schur system               */
/* ------------------------------------------------------------------ */

/*
 * Solve M x = b.  Textbook CGNR on Ahat^dag Ahat x_e = Ahat^dag bhat_e from
 * x_e = 0, carrying the Schur residual rho = bhat_e - Ahat x_e alongside the
 * normal residual; stop when |rho| <= tol * |b| (for form 0, |rho| equals the
 * full-system residual |b - M x| once x_o is reconstructed).  maxiter bounds
 * the iterations; iters_out gets the count.  Returns the true relative
 * residual |b - M x| / |b| of the reconstructed full solution.
 */
double or_cgnr(const int L[4], double kappa, double eps, int t_bc, const double *U,
               const double *b, double *x_full, double tol, int maxiter, int form,
               int *iters_out)
{
    long V = vol(L);
    long n12 = 12 * V;
    size_t n = sizeof(cplx) * n12;
    cplx *bh = malloc(n), *x = calloc(n12, sizeof(cplx)), *rho = malloc(n), *r = malloc(n);
    cplx *p = malloc(n), *q = malloc(n), *s = malloc(n);
    or_source_prep(L, kappa, eps, t_bc, U, b, (double *)bh, form);
    double bnorm = sqrt(norm2(n12, (const cplx *)b));
    double target = tol * bnorm;
    memcpy(rho, bh, n);
    or_schur(L, kappa, eps, t_bc, U, (double *)rho, (double *)r, 1, form);
    memcpy(p, r, n);
    double rr = norm2(n12, r);
    int it = 0;
    while (sqrt(norm2(n12, rho)) > target && it < maxiter && rr > 0) {
        or_schur(L, kappa, eps, t_bc, U, (double *)p, (double *)q, 0, form);
        double qq = norm2(n12, q);
        double alpha = rr / qq;
        for (long i = 0; i < n12; i++) { x[i] += alpha * p[i]; rho[i] -= alpha * q[i]; }
        or_schur(L, kappa, eps, t_bc, U, (double *)q, (double *)s, 1, form);
        for (long i = 0; i < n12; i++) r[i] -= alpha * s[i];
        double rr_new = norm2(n12, r);
        double beta = rr_new / rr;
        for (long i = 0; i < n12; i++) p[i] = r[i] + beta * p[i];
        rr = rr_new;
        it++;
    }
    if (iters_out) *iters_out = it;
    or_reconstruct(L, kappa, eps, t_bc, U, b, (double *)x, x_full);
    /* true residual of the full system */
    or_apply_M(L, kappa, eps, t_bc, U, x_full, (double *)s, 0);
    const cplx *bb = (const cplx *)b;
    for (long i = 0; i < n12; i++) s[i] = bb[i] - s[i];
    double res = sqrt(norm2(n12, s)) / bnorm;
    free(bh); free(x); free(rho); free(r); free(p); free(q); free(s);
    return res;
}

/* a fixed number of CG iterations on the Schur normal equations, for timing;
 * returns the Schur residual norm reached */
double or_cgnr_iterations(const int L[4], double kappa, double eps, int t_bc, const double *U,
                          const double *b, int niter)
{
    long V = vol(L);
    long n12 = 12 * V;
    size_t n = sizeof(cplx) * n12;
    cplx *x = calloc(n12, sizeof(cplx)), *rho = malloc(n), *r = malloc(n);
    cplx *p = malloc(n), *q = malloc(n), *s = malloc(n);
    or_source_prep(L, kappa, eps, t_bc, U, b, (double *)rho, 0);
    or_schur(L, kappa, eps, t_bc, U, (double *)rho, (double *)r, 1, 0);
    memcpy(p, r, n);
    double rr = norm2(n12, r);
    for (int it = 0; it < niter; it++) {
        or_schur(L, kappa, eps, t_bc, U, (double *)p, (double *)q, 0, 0);
        double alpha = rr / norm2(n12, q);
        for (long i = 0; i < n12; i++) { x[i] += alpha * p[i]; rho[i] -= alpha * q[i]; }
        or_schur(L, kappa, eps, t_bc, U, (double *)q, (double *)s, 1, 0);
        for (long i = 0; i < n12; i++) r[i] -= alpha * s[i];
        double rr_new = norm2(n12, r);
        double beta = rr_new / rr;
        for (long i = 0; i < n12; i++) p[i] = r[i] + beta * p[i];
        rr = rr_new;
    }
    double res = sqrt(norm2(n12, rho));
    free(x); free(rho); free(r); free(p); free(q); free(s);
    return res;
}

/* ------------------------------------------------------------------ */
/* Z4 noise                                                             */
/* ------------------------------------------------------------------ */

/*
 * SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): state advances by the
 * golden-ratio increment 0x9e3779b97f4a7c15 and each output is the
 * variant-13 finaliser of the state.  Output number c (c = 0, 1, ...) of the
 * stream seeded with `seed` is therefore mix(seed + (c+1)*increment).
 */
uint64_t or_splitmix64(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + (c + 1) * 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/*
 * Z4 noise vector number r (section II.A: entries drawn from {1, i, -1, -i}).
 * Entry (site s, spin a, colour c) is i^k with k the top two bits of stream
 * output number ((r*V + s)*4 + a)*3 + c.
 */
void or_noise_z4(const int L[4], uint64_t seed, long r, double *out)
{
    long V = vol(L);
    cplx *o = (cplx *)out;
    const cplx pw[4] = {1, I, -1, -I};
    for (long s = 0; s < V; s++)
        for (int a = 0; a < 4; a++)
            for (int c = 0; c < 3; c++) {
                uint64_t idx = (uint64_t)(((r * V + s) * 4 + a) * 3 + c);
                int k = (int)(or_splitmix64(seed, idx) >> 62);
                o[12 * s + 3 * a + c] = pw[k];
            }
}

/* ------------------------------------------------------------------ */
/* contractions                                                         */
/* ------------------------------------------------------------------ */

/*
 * Standard estimator at every time slice (section II.C, eq. loopSt):
 *   out[n][t] += sum_{x in t} eta(x)^dag Gamma_n s(x),  n = 0..15.
 * Accumulates into out (complex [16][Lt]).
 */
void or_contract_std(const int L[4], const double *etad, const double *sd, double *outd)
{
    const cplx *eta = (const cplx *)etad, *s = (const cplx *)sd;
    cplx *out = (cplx *)outd;
    long V = vol(L);
    for (int n = 0; n < 16; n++) {
        cplx G[4][4];
        or_gamma(n, (double *)G);
        for (long x = 0; x < V; x++) {
            int c[4];
            coords(L, x, c);
            cplx acc = 0;
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++)
                    for (int col = 0; col < 3; col++)
                        acc += conj(eta[12 * x + 3 * a + col]) * G[a][b] * s[12 * x + 3 * b + col];
            out[n * L[3] + c[3]] += acc;
        }
    }
}

/*
 * One-end estimator (section II.C, eq. loopVv, left-hand side with X = Gamma_n):
 *   out[n][t] += 2 i eps sum_{x in t} s(x)^dag gamma5 Gamma_n s(x).
 */
void or_contract_oneend(const int L[4], double eps, const double *sd, double *outd)
{
    const cplx *s = (const cplx *)sd;
    cplx *out = (cplx *)outd;
    long V = vol(L);
    cplx g5[4][4];
    gamma5(g5);
    for (int n = 0; n < 16; n++) {
        cplx G[4][4], X[4][4];
        or_gamma(n, (double *)G);
        matmul4(g5, G, X);
        for (long x = 0; x < V; x++) {
            int c[4];
            coords(L, x, c);
            cplx acc = 0;
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++)
                    for (int col = 0; col < 3; col++)
                        acc += conj(s[12 * x + 3 * a + col]) * X[a][b] * s[12 * x + 3 * b + col];
            out[n * L[3] + c[3]] += 2.0 * I * eps * acc;
        }
    }
}

/* ------------------------------------------------------------------ */
/* hopping parameter expansion                                          */
/* ------------------------------------------------------------------ */

/* out = (B H)^k psi with B = R^-1 (section II.E, eq. HPE) */
void or_bh_power(const int L[4], double kappa, double eps, int t_bc, const double *U,
                 const double *in, double *out, int k)
{
    long V = vol(L);
    size_t n = sizeof(cplx) * 12 * V;
    cplx *a = malloc(n), *h = malloc(n);
    memcpy(a, in, n);
    for (int i = 0; i < k; i++) {
        or_hop(L, kappa, t_bc, U, (double *)a, (double *)h, 0);
        or_twist(L, eps, 2, (double *)h, (double *)a);
    }
    memcpy(out, a, n);
    free(a); free(h);
}

/*
 * Exactly computed part of the expansion for ultra-local insertions:
 *   out[n][t] = sum_{x in t} tr[ (Gamma_n (x) 1_c) (B + B H B H B)_{xx} ]
 * The odd powers B H B and (B H)^3 B have no diagonal on a bipartite
 * lattice.  The diagonal of B H B H B is the sum over every pair of hops
 * x -> y -> x of B H[x][y] B H[y][x] B; each hop block is
 * (spin projector) (x) (colour link) times -kappa and the boundary phase,
 * so the trace factorises into a spin trace times a colour trace.
 */
void or_hpe_exact(const int L[4], double kappa, double eps, int t_bc, const double *Ud,
                  double *outd)
{
    const cplx *U = (const cplx *)Ud;
    cplx *out = (cplx *)outd;
    long V = vol(L);
    cplx B[4][4];
    twist_matrix(eps, 2, B);
    cplx Pm[4][4][4], Pp[4][4][4];
    for (int mu = 0; mu < 4; mu++) {
        cplx g[4][4];
        gamma_mu(mu, g);
        for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++) {
                Pm[mu][i][j] = (i == j) - g[i][j];
                Pp[mu][i][j] = (i == j) + g[i][j];
            }
    }
    cplx G[16][4][4];
    for (int n = 0; n < 16; n++) or_gamma(n, (double *)G[n]);
    memset(out, 0, sizeof(cplx) * 16 * L[3]);
    for (long x = 0; x < V; x++) {
        int c[4];
        coords(L, x, c);
        /* spin part of the diagonal, colour traced: D = 3 B + sum over paths */
        cplx D[4][4];
        for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++) D[i][j] = 3.0 * B[i][j];
        for (int mu = 0; mu < 4; mu++)
            for (int d1 = 0; d1 < 2; d1++) {
                double ph1;
                int dir1 = d1 ? -1 : +1;
                long y = step(L, t_bc, x, mu, dir1, &ph1);
                /* block H[x][y]: forward hop uses (1-g) U_mu(x); backward (1+g) U_mu(y)^dag */
                const cplx(*P1)[4] = d1 ? (const cplx(*)[4])Pp[mu] : (const cplx(*)[4])Pm[mu];
                cplx C1[3][3];
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++)
                        C1[i][j] = d1 ? conj(U[9 * ((long)mu * V + y) + 3 * j + i])
                                      : U[9 * ((long)mu * V + x) + 3 * i + j];
                for (int nu = 0; nu < 4; nu++)
                    for (int d2 = 0; d2 < 2; d2++) {
                        double ph2;
                        int dir2 = d2 ? -1 : +1;
                        long z = step(L, t_bc, y, nu, dir2, &ph2);
                        if (z != x) continue;
                        const cplx(*P2)[4] = d2 ? (const cplx(*)[4])Pp[nu] : (const cplx(*)[4])Pm[nu];
                        cplx C2[3][3];
                        for (int i = 0; i < 3; i++)
                            for (int j = 0; j < 3; j++)
                                C2[i][j] = d2 ? conj(U[9 * ((long)nu * V + x) + 3 * j + i])
                                              : U[9 * ((long)nu * V + y) + 3 * i + j];
                        cplx trc = 0;
                        for (int i = 0; i < 3; i++)
                            for (int k = 0; k < 3; k++) trc += C1[i][k] * C2[k][i];
                        cplx S[4][4];
                        matmul4(B, P1, S);
                        matmul4(S, B, S);
                        matmul4(S, P2, S);
                        matmul4(S, B, S);
                        cplx f = kappa * kappa * ph1 * ph2 * trc;
                        for (int i = 0; i < 4; i++)
                            for (int j = 0; j < 4; j++) D[i][j] += f * S[i][j];
                    }
            }
        for (int n = 0; n < 16; n++) {
            cplx tr = 0;
            for (int i = 0; i < 4; i++)
                for (int j = 0; j < 4; j++) tr += G[n][i][j] * D[j][i];
            out[n * L[3] + c[3]] += tr;
        }
    }
}

/* ------------------------------------------------------------------ */
/* sampled evaluation for large lattices                               */
/* ------------------------------------------------------------------ */

/* one row block of H applied to psi at site s: (H psi)(s) (adj = 0) */
static void hop_at(const int L[4], double kappa, int t_bc, const cplx *U, const cplx *psi, long s,
                   cplx out[12], const cplx Pm[4][4][4], const cplx Pp[4][4][4], long V)
{
    cplx acc[12] = {0};
    for (int mu = 0; mu < 4; mu++) {
        double phf, phb;
        long sf = step(L, t_bc, s, mu, +1, &phf);
        long sb = step(L, t_bc, s, mu, -1, &phb);
        add_block(acc, -kappa * phf, (const cplx(*)[4])Pm[mu], U + 9 * ((long)mu * V + s), 0, psi + 12 * sf);
        add_block(acc, -kappa * phb, (const cplx(*)[4])Pp[mu], U + 9 * ((long)mu * V + sb), 1, psi + 12 * sb);
    }
    memcpy(out, acc, sizeof(acc));
}

/*
 * (Ahat x)(s) = R x(s) - sum_y H[s][y] R^-1 (H x)(y) at the even sites listed
 * in `sites` (form A.2), evaluated row by row from the definition, for
 * lattices too large for the full-vector routines; x is a full vector whose
 * odd sites are ignored.  out: [nsites][12].
 */
void or_schur_at(const int L[4], double kappa, double eps, int t_bc, const double *Ud,
                 const double *xd, const long *sites, long nsites, double *outd)
{
    const cplx *U = (const cplx *)Ud, *x = (const cplx *)xd;
    cplx *out = (cplx *)outd;
    long V = vol(L);
    cplx Pm[4][4][4], Pp[4][4][4], R[4][4], Ri[4][4];
    for (int mu = 0; mu < 4; mu++) {
        cplx g[4][4];
        gamma_mu(mu, g);
        for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++) {
                Pm[mu][i][j] = (i == j) - g[i][j];
                Pp[mu][i][j] = (i == j) + g[i][j];
            }
    }
    twist_matrix(eps, 0, R);
    twist_matrix(eps, 2, Ri);
#pragma omp parallel for schedule(dynamic)
    for (long n = 0; n < nsites; n++) {
        long s = sites[n];
        /* x restricted to even sites, read through a masked copy of the
         * neighbourhood: the odd values needed are (R^-1 H x_e)(y) for the 8
         * odd neighbours y of s */
        cplx acc[12] = {0};
        for (int mu = 0; mu < 4; mu++)
            for (int d = 0; d < 2; d++) {
                double ph;
                long y = step(L, t_bc, s, mu, d ? -1 : +1, &ph);
                /* (H x_e)(y): every neighbour of the odd site y is even */
                cplx hy[12], ry[12];
                hop_at(L, kappa, t_bc, U, x, y, hy, (const cplx(*)[4][4])Pm, (const cplx(*)[4][4])Pp, V);
                for (int a = 0; a < 4; a++)
                    for (int c = 0; c < 3; c++) {
                        cplx t = 0;
                        for (int b = 0; b < 4; b++) t += Ri[a][b] * hy[3 * b + c];
                        ry[3 * a + c] = t;
                    }
                /* block H[s][y] applied to ry */
                const cplx *Ublk = d ? U + 9 * ((long)mu * V + y) : U + 9 * ((long)mu * V + s);
                add_block(acc, -kappa * ph, d ? (const cplx(*)[4])Pp[mu] : (const cplx(*)[4])Pm[mu], Ublk, d,
                          ry);
            }
        for (int a = 0; a < 4; a++)
            for (int c = 0; c < 3; c++) {
                cplx t = 0;
                for (int b = 0; b < 4; b++) t += R[a][b] * x[12 * s + 3 * b + c];
                out[12 * n + 3 * a + c] = t - acc[3 * a + c];
            }
    }
}

/* ------------------------------------------------------------------ */
/* gauge-covariant parallel-transport network                          */
/* ------------------------------------------------------------------ */

/*
 * Path k: 0 identity; 1..4 one hop in +mu (mu = k-1): (T phi)(x) =
 * U_mu(x) phi(x+mu); 5..8 one hop in -mu (mu = k-5): (T phi)(x) =
 * U_mu(x-mu)^dag phi(x-mu); the fermion boundary phase rides on hops across
 * the time boundary.  adj = 1 applies the adjoint (block-wise conjugate
 * transpose of the same matrix).
 */
void or_transport(const int L[4], int t_bc, const double *Ud, int k, const double *ind, double *outd,
                  int adj)
{
    const cplx *U = (const cplx *)Ud, *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    long V = vol(L);
    if (k == 0) {
        memcpy(out, in, sizeof(cplx) * 12 * V);
        return;
    }
    const int mu = (k - 1) & 3;
    const int fwd = k <= 4;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; x++) {
        double ph;
        /* matrix element T[x][y] = W for y = x + d; its adjoint has element
         * T^dag[y][x] = W^dag, i.e. (T^dag f)(x) = W(x - d -> x)^dag f(x - d) */
        int dir = fwd ? +1 : -1;
        if (adj) dir = -dir;
        long y = step(L, t_bc, x, mu, dir, &ph);
        const cplx *W;
        int dagger;
        if (!adj) {
            W = fwd ? U + 9 * ((long)mu * V + x) : U + 9 * ((long)mu * V + y);
            dagger = !fwd;
        } else {
            /* row y of T holds W_T(y) acting on f(x); adjoint takes its dagger */
            W = fwd ? U + 9 * ((long)mu * V + y) : U + 9 * ((long)mu * V + x);
            dagger = fwd;
        }
        for (int a = 0; a < 4; a++)
            for (int i = 0; i < 3; i++) {
                cplx t = 0;
                for (int j = 0; j < 3; j++)
                    t += (dagger ? conj(W[3 * j + i]) : W[3 * i + j]) * in[12 * y + 3 * a + j];
                out[12 * x + 3 * a + i] = ph * t;
            }
    }
}

/* out(x) += S in(x) for a 4x4 spin matrix S (complex [4][4]) */
static void spin_mac(long V, const cplx *S, const cplx *in, cplx *out)
{
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; x++)
        for (int a = 0; a < 4; a++)
            for (int c = 0; c < 3; c++) {
                cplx t = 0;
                for (int b = 0; b < 4; b++) t += S[4 * a + b] * in[12 * x + 3 * b + c];
                out[12 * x + 3 * a + c] += t;
            }
}

/*
 * Two linear parallel-transport layers, 1 -> nc -> 1 channels:
 *   phi_c = sum_k W1[k][c] T_k in,     out = sum_{k,c} W2[k][c] T_k phi_c,
 * W1, W2: complex [9][nc][4][4] spin matrices.  Evaluated layer by layer.
 */
void or_ptc_forward(const int L[4], int t_bc, const double *U, int nc, const double *W1d,
                    const double *W2d, const double *ind, double *outd)
{
    const cplx *W1 = (const cplx *)W1d, *W2 = (const cplx *)W2d;
    long V = vol(L);
    size_t n = sizeof(cplx) * 12 * V;
    cplx *T = malloc(n), *phi = malloc(n * nc), *out = (cplx *)outd;
    memset(phi, 0, n * nc);
    for (int k = 0; k < 9; k++) {
        or_transport(L, t_bc, U, k, ind, (double *)T, 0);
        for (int c = 0; c < nc; c++) spin_mac(V, W1 + 16 * (k * nc + c), T, phi + 12 * V * c);
    }
    memset(out, 0, n);
    for (int k = 0; k < 9; k++)
        for (int c = 0; c < nc; c++) {
            or_transport(L, t_bc, U, k, (double *)(phi + 12 * V * c), (double *)T, 0);
            spin_mac(V, W2 + 16 * (k * nc + c), T, out);
        }
    free(T);
    free(phi);
}

/* Path k at site x: neighbour y, link W (row-major) to apply (daggered for
 * backward hops) and boundary phase; k = 0 is the identity (y = x). */
static long path_link(const int L[4], int t_bc, const cplx *U, int k, long x, cplx W[9], double *ph)
{
    long V = vol(L);
    if (k == 0) {
        for (int e = 0; e < 9; e++) W[e] = (e % 4 == 0) ? 1.0 : 0.0;
        *ph = 1.0;
        return x;
    }
    const int mu = (k - 1) & 3, fwd = k <= 4;
    long y = step(L, t_bc, x, mu, fwd ? +1 : -1, ph);
    const cplx *Um = fwd ? U + 9 * ((long)mu * V + x) : U + 9 * ((long)mu * V + y);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) W[3 * i + j] = fwd ? Um[3 * i + j] : conj(Um[3 * j + i]);
    return y;
}

/* out += S (W f) * ph for one site: colour link W, then spin matrix S */
static void site_acc(const cplx *S, const cplx W[9], double ph, const cplx f[12], cplx out[12])
{
    cplx t[12];
    for (int a = 0; a < 4; a++)
        for (int i = 0; i < 3; i++) {
            cplx v = 0;
            for (int j = 0; j < 3; j++) v += W[3 * i + j] * f[3 * a + j];
            t[3 * a + i] = ph * v;
        }
    for (int a = 0; a < 4; a++)
        for (int c = 0; c < 3; c++) {
            cplx v = 0;
            for (int b = 0; b < 4; b++) v += S[4 * a + b] * t[3 * b + c];
            out[3 * a + c] += v;
        }
}

/*
 * The same two layers as or_ptc_forward, evaluated only at the given sites
 * straight from the definition (for lattices where whole-lattice hidden
 * fields are too large): N(psi)(x) = sum_{k,c} W2[k][c] (T_k phi_c)(x) with
 * phi_c(y) = sum_k' W1[k'][c] (T_k' psi)(y) formed at the nine sites y the
 * paths of x reach.  out: [nsites][12].
 */
void or_ptc_at(const int L[4], int t_bc, const double *Ud, int nc, const double *W1d, const double *W2d,
               const double *ind, const long *sites, long nsites, double *outd)
{
    const cplx *U = (const cplx *)Ud, *W1 = (const cplx *)W1d, *W2 = (const cplx *)W2d;
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
#pragma omp parallel for schedule(dynamic)
    for (long n = 0; n < nsites; n++) {
        const long x = sites[n];
        cplx acc[12] = {0};
        for (int k = 0; k < 9; k++) {
            cplx W[9];
            double ph;
            const long y = path_link(L, t_bc, U, k, x, W, &ph);
            for (int c = 0; c < nc; c++) {
                cplx phi[12] = {0};
                for (int kp = 0; kp < 9; kp++) {
                    cplx W1l[9];
                    double ph1;
                    const long z = path_link(L, t_bc, U, kp, y, W1l, &ph1);
                    site_acc(W1 + 16 * (kp * nc + c), W1l, ph1, in + 12 * z, phi);
                }
                site_acc(W2 + 16 * (k * nc + c), W, ph, phi, acc);
            }
        }
        for (int e = 0; e < 12; e++) out[12 * n + e] = acc[e];
    }
}

/*
 * Gradient of a loss l(out), out = N(in), with respect to the real and
 * imaginary parts of every weight, accumulated into G1, G2 as complex numbers
 * dl/dRe(w) + i dl/dIm(w), given delta = 2 dl/d(conj out) (for l = |out - e|^2 / |e|^2
 * that is 2 (out - e) / |e|^2), by reverse-mode differentiation of the forward
 * pass above:
 *   G2[k][c] = sum_x delta(x) (T_k phi_c)(x)^dag      (spin outer product,
 *                                                      colour traced)
 *   g_c      = sum_k T_k^dag (W2[k][c]^dag delta)
 *   G1[k][c] = sum_x g_c(x) (T_k in)(x)^dag.
 */
static void ptc_grad_from_delta(const int L[4], int t_bc, const double *U, int nc, const cplx *W1,
                                const cplx *W2, const double *ind, const cplx *delta, cplx *G1, cplx *G2)
{
    long V = vol(L);
    size_t n = sizeof(cplx) * 12 * V;
    cplx *T = malloc(n), *phi = malloc(n * nc), *g = malloc(n), *tmp = malloc(n), *Tin = malloc(n * 9);
    /* hidden layer again (kept for the gradients) */
    memset(phi, 0, n * nc);
    for (int k = 0; k < 9; k++) {
        or_transport(L, t_bc, U, k, ind, (double *)(Tin + 12 * V * k), 0);
        for (int c = 0; c < nc; c++) spin_mac(V, W1 + 16 * (k * nc + c), Tin + 12 * V * k, phi + 12 * V * c);
    }
    for (int c = 0; c < nc; c++) {
        memset(g, 0, n);
        for (int k = 0; k < 9; k++) {
            or_transport(L, t_bc, U, k, (double *)(phi + 12 * V * c), (double *)T, 0);
            cplx *G = G2 + 16 * (k * nc + c);
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++) {
                    cplx acc = 0;
                    for (long x = 0; x < V; x++)
                        for (int col = 0; col < 3; col++)
                            acc += delta[12 * x + 3 * a + col] * conj(T[12 * x + 3 * b + col]);
                    G[4 * a + b] += acc;
                }
            /* W2^dag delta, then transported back */
            cplx Wd[16];
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++) Wd[4 * a + b] = conj(W2[16 * (k * nc + c) + 4 * b + a]);
            memset(tmp, 0, n);
            spin_mac(V, Wd, delta, tmp);
            or_transport(L, t_bc, U, k, (double *)tmp, (double *)T, 1);
            for (long i = 0; i < 12 * V; i++) g[i] += T[i];
        }
        for (int k = 0; k < 9; k++) {
            cplx *G = G1 + 16 * (k * nc + c);
            const cplx *ti = Tin + 12 * V * k;
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++) {
                    cplx acc = 0;
                    for (long x = 0; x < V; x++)
                        for (int col = 0; col < 3; col++) acc += g[12 * x + 3 * a + col] * conj(ti[12 * x + 3 * b + col]);
                    G[4 * a + b] += acc;
                }
        }
    }
    free(T); free(phi); free(g); free(tmp); free(Tin);
}

/*
 * Error loss of one pair, l = |N(in) - e|^2 / |e|^2, and its gradient
 * (accumulated into G1, G2); delta = 2 (out - e) / |e|^2.  Returns l.
 */
double or_ptc_loss_grad(const int L[4], int t_bc, const double *U, int nc, const double *W1d,
                        const double *W2d, const double *ind, const double *ed, double *G1d,
                        double *G2d)
{
    const cplx *e = (const cplx *)ed;
    long V = vol(L);
    size_t n = sizeof(cplx) * 12 * V;
    cplx *out = malloc(n), *delta = malloc(n);
    or_ptc_forward(L, t_bc, U, nc, W1d, W2d, ind, (double *)out);
    double en = 0, l = 0;
    for (long i = 0; i < 12 * V; i++) en += creal(e[i] * conj(e[i]));
    for (long i = 0; i < 12 * V; i++) {
        cplx d = out[i] - e[i];
        l += creal(d * conj(d));
        delta[i] = 2.0 * d / en;
    }
    l /= en;
    ptc_grad_from_delta(L, t_bc, U, nc, (const cplx *)W1d, (const cplx *)W2d, ind, delta, (cplx *)G1d,
                        (cplx *)G2d);
    free(out); free(delta);
    return l;
}

/*
 * Residual loss of one residual r = in: with w = M N(r) - r,
 * l = |w|^2 / |r|^2 (how far M N is from the identity on r, the quantity a
 * right preconditioner N of M is judged by), and its gradient: l depends on
 * out = N(r) through w, so delta = 2 dl/d(conj out) = 2 M^dag w / |r|^2.
 * Returns l.
 */
double or_ptc_res_loss_grad(const int L[4], double kappa, double eps, int t_bc, const double *U, int nc,
                            const double *W1d, const double *W2d, const double *ind, double *G1d, double *G2d)
{
    const cplx *r = (const cplx *)ind;
    long V = vol(L);
    size_t n = sizeof(cplx) * 12 * V;
    cplx *out = malloc(n), *w = malloc(n), *delta = malloc(n);
    or_ptc_forward(L, t_bc, U, nc, W1d, W2d, ind, (double *)out);
    or_apply_M(L, kappa, eps, t_bc, U, (const double *)out, (double *)w, 0);
    double rn = 0, l = 0;
    for (long i = 0; i < 12 * V; i++) {
        rn += creal(r[i] * conj(r[i]));
        w[i] -= r[i];
        l += creal(w[i] * conj(w[i]));
    }
    or_apply_M(L, kappa, eps, t_bc, U, (const double *)w, (double *)delta, 1);
    for (long i = 0; i < 12 * V; i++) delta[i] *= 2.0 / rn;
    ptc_grad_from_delta(L, t_bc, U, nc, (const cplx *)W1d, (const cplx *)W2d, ind, delta, (cplx *)G1d,
                        (cplx *)G2d);
    free(out); free(w); free(delta);
    return l / rn;
}

/* OpenMP threads of the oracle's parallel loops (timing only; results do not
 * depend on it beyond reduction order) */
void or_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int or_get_threads(void) { return omp_get_max_threads(); }
