/*
 * FP64 reference oracle for fused lattice field expressions and APE link
 * smearing.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  The HIP library never calls
 * it, and the two share no source, header, table or helper.
 *
 * It is deliberately plain: C99, double precision, explicit real/imaginary
 * arithmetic written out term by term, one loop over lattice sites (OpenMP
 * only splits that loop), no blocking or reordering beyond the definitions.
 * Reductions store one value per site and sum the array serially with
 * Neumaier compensation, so the result does not depend on the thread count.
 *
 * Host canonical layout (shared with the input generators):
 *   extents L = {Lx, Ly, Lz, Lt}; site = x + Lx*(y + Ly*(z + Lz*t));
 *   links    double[V][4][3][3][2]  (site, direction mu, row a, column b, re/im)
 *   fermions double[V][4][3][2]     (site, spin, colour, re/im)
 * All directions are periodic.
 *
 * What is computed, and where it is defined:
 *   - shift(X, FORWARD, mu)(x) = X(x + mu) and the hop U_mu(x) X(x + mu):
 *     the paper's Jacobi-smearing listing (expressions E_1/E_2) and the
 *     hopping term of the smearing operator K in section 7.
 *   - chi = sum_mu U_mu(x) psi(x+mu) + a phi(x): the forward hop summed over
 *     mu plus the axpy of expression E_3 (section 7); a*phi is added once.
 *   - the backward hop U_mu(x-mu)^dagger X(x-mu), the other term of K, with a
 *     mask of directions for either hop.
 *   - Jacobi smearing: the truncated power series of K^{-1} = (1 - kappa H)^{-1}
 *     applied to a source (section 7), H the hop in both directions summed over
 *     the smeared directions.
 *   - The APE step (staple sum, combination with weight alpha, row
 *     Gram-Schmidt reunitarisation) and the plaquette are not in the paper;
 *     they follow the workload definition of one APE step on a periodic
 *     lattice with all directions smeared from the unsmeared links.
 *
 * Parity pins for every function live in tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double re, im; } cplx;
typedef struct { cplx e[3][3]; } mat3;

/* ------------------------------------------------------------------ */
/* complex scalar arithmetic                                           */
/* ------------------------------------------------------------------ */
static cplx c_make(double re, double im) { cplx z; z.re = re; z.im = im; return z; }
static cplx c_add(cplx a, cplx b) { return c_make(a.re + b.re, a.im + b.im); }
static cplx c_sub(cplx a, cplx b) { return c_make(a.re - b.re, a.im - b.im); }
static cplx c_mul(cplx a, cplx b) { return c_make(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }
static cplx c_conj(cplx a) { return c_make(a.re, -a.im); }
static cplx c_scale(double s, cplx a) { return c_make(s * a.re, s * a.im); }
static double c_abs2(cplx a) { return a.re * a.re + a.im * a.im; }

/* ------------------------------------------------------------------ */
/* 3x3 complex matrices                                                */
/* ------------------------------------------------------------------ */
static mat3 m_zero(void) { mat3 m; memset(&m, 0, sizeof m); return m; }

/* C = A B */
static mat3 m_mul(const mat3 *A, const mat3 *B)
{
    mat3 C;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = c_make(0.0, 0.0);
            for (int k = 0; k < 3; ++k) s = c_add(s, c_mul(A->e[i][k], B->e[k][j]));
            C.e[i][j] = s;
        }
    return C;
}

/* C = A^dagger */
static mat3 m_dag(const mat3 *A)
{
    mat3 C;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C.e[i][j] = c_conj(A->e[j][i]);
    return C;
}

static mat3 m_add(const mat3 *A, const mat3 *B)
{
    mat3 C;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C.e[i][j] = c_add(A->e[i][j], B->e[i][j]);
    return C;
}

static double m_retrace(const mat3 *A) { return A->e[0][0].re + A->e[1][1].re + A->e[2][2].re; }

/* ------------------------------------------------------------------ */
/* lattice indexing (periodic)                                         */
/* ------------------------------------------------------------------ */
typedef struct { int L[4]; long V; } lat;

static lat lat_make(const int *L)
{
    lat g;
    for (int d = 0; d < 4; ++d) g.L[d] = L[d];
    g.V = (long)L[0] * L[1] * L[2] * L[3];
    return g;
}

static void site_coords(const lat *g, long s, int c[4])
{
    for (int d = 0; d < 4; ++d) { c[d] = (int)(s % g->L[d]); s /= g->L[d]; }
}

static long coords_site(const lat *g, const int c[4])
{
    return c[0] + (long)g->L[0] * (c[1] + (long)g->L[1] * (c[2] + (long)g->L[2] * c[3]));
}

/* site reached from s by `step` (+1 or -1) in direction mu, wrapping around */
static long hop(const lat *g, long s, int mu, int step)
{
    int c[4];
    site_coords(g, s, c);
    c[mu] = ((c[mu] + step) % g->L[mu] + g->L[mu]) % g->L[mu];
    return coords_site(g, c);
}

static mat3 load_link(const double *U, long s, int mu)
{
    mat3 m;
    const double *p = U + ((s * 4 + mu) * 9) * 2;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) m.e[a][b] = c_make(p[(a * 3 + b) * 2], p[(a * 3 + b) * 2 + 1]);
    return m;
}

static void store_link(double *U, long s, int mu, const mat3 *m)
{
    double *p = U + ((s * 4 + mu) * 9) * 2;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            p[(a * 3 + b) * 2] = m->e[a][b].re;
            p[(a * 3 + b) * 2 + 1] = m->e[a][b].im;
        }
}

static cplx load_fermion(const double *f, long s, int spin, int col)
{
    const double *p = f + ((s * 4 + spin) * 3 + col) * 2;
    return c_make(p[0], p[1]);
}

static void store_fermion(double *f, long s, int spin, int col, cplx v)
{
    double *p = f + ((s * 4 + spin) * 3 + col) * 2;
    p[0] = v.re;
    p[1] = v.im;
}

/* Neumaier-compensated serial sum. */
double oracle_neumaier_sum(long n, const double *x)
{
    double s = 0.0, comp = 0.0;
    for (long i = 0; i < n; ++i) {
        double t = s + x[i];
        if (fabs(s) >= fabs(x[i])) comp += (s - t) + x[i];
        else comp += (x[i] - t) + s;
        s = t;
    }
    return s + comp;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* shift expression                                                    */
/* ------------------------------------------------------------------ */

/* chi at one site: sum_{mu in mask} h_mu(x) + a*phi(x) (phi may be NULL), with the
 * hop h_mu(x) = U_mu(x) psi(x+mu) for sign > 0 (shift(psi, FORWARD, mu) times the
 * link) and h_mu(x) = U_mu(x-mu)^dagger psi(x-mu) for sign < 0 (the backward term
 * of the smearing operator K, section 7).  U acts on colour and is the identity
 * in spin. */
static void shift_site(const lat *g, const double *U, const double *psi, const double *phi, double a,
                       unsigned mask, int sign, long s, cplx acc[4][3])
{
    for (int sp = 0; sp < 4; ++sp)
        for (int c = 0; c < 3; ++c) acc[sp][c] = c_make(0.0, 0.0);
    for (int mu = 0; mu < 4; ++mu) {
        if (!((mask >> mu) & 1u)) continue;
        if (sign > 0) {
            mat3 u = load_link(U, s, mu);
            long fwd = hop(g, s, mu, +1);
            for (int sp = 0; sp < 4; ++sp)
                for (int ca = 0; ca < 3; ++ca)
                    for (int cb = 0; cb < 3; ++cb)
                        acc[sp][ca] = c_add(acc[sp][ca], c_mul(u.e[ca][cb], load_fermion(psi, fwd, sp, cb)));
        } else {
            long back = hop(g, s, mu, -1);
            mat3 lb = load_link(U, back, mu);
            /* (U^dagger)_{ab} = conj(U_{ba}) */
            for (int sp = 0; sp < 4; ++sp)
                for (int ca = 0; ca < 3; ++ca)
                    for (int cb = 0; cb < 3; ++cb)
                        acc[sp][ca] = c_add(acc[sp][ca], c_mul(c_conj(lb.e[cb][ca]), load_fermion(psi, back, sp, cb)));
        }
    }
    if (phi)
        for (int sp = 0; sp < 4; ++sp)
            for (int c = 0; c < 3; ++c) acc[sp][c] = c_add(acc[sp][c], c_scale(a, load_fermion(phi, s, sp, c)));
}

/* chi(x) = sum_{mu in mask} h_mu(x) + a*phi(x) for every site, h_mu the forward
 * (sign > 0) or backward (sign < 0) hop of shift_site.  If norm2 is not NULL it
 * receives sum over sites, spins and colours of |chi|^2. */
void oracle_shift_expr(const int *L, const double *U, const double *psi, const double *phi, double a,
                       unsigned mask, int sign, double *chi, double *norm2)
{
    lat g = lat_make(L);
    double *site_norm = norm2 ? (double *)malloc(sizeof(double) * (size_t)g.V) : NULL;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < g.V; ++s) {
        cplx acc[4][3];
        shift_site(&g, U, psi, phi, a, mask, sign, s, acc);
        double n2 = 0.0;
        for (int sp = 0; sp < 4; ++sp)
            for (int c = 0; c < 3; ++c) {
                store_fermion(chi, s, sp, c, acc[sp][c]);
                n2 += c_abs2(acc[sp][c]);
            }
        if (site_norm) site_norm[s] = n2;
    }
    if (norm2) {
        *norm2 = oracle_neumaier_sum(g.V, site_norm);
        free(site_norm);
    }
}

/* chi(x) = sum_{mu=0..3} U_mu(x) psi(x+mu) + a*phi(x): all four forward hops. */
void oracle_shift_mul_axpy(const int *L, const double *U, const double *psi, const double *phi,
                           double a, double *chi, double *norm2)
{
    oracle_shift_expr(L, U, psi, phi, a, 0xFu, +1, chi, norm2);
}

/* n_iter repetitions of: chi_k = shift_mul_axpy(U, psi_{k-1}, phi, a);
 *                        psi_k = psi_{k-1} - c * chi_k.
 * psi is updated in place; norms (may be NULL) receives |chi_k|^2. */
void oracle_shift_chain(const int *L, const double *U, double *psi, const double *phi, double a,
                        double c, int n_iter, double *norms)
{
    lat g = lat_make(L);
    size_t nf = (size_t)g.V * 4 * 3 * 2;
    double *chi = (double *)malloc(sizeof(double) * nf);
    for (int k = 0; k < n_iter; ++k) {
        oracle_shift_mul_axpy(L, U, psi, phi, a, chi, norms ? &norms[k] : NULL);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < (long)nf; ++i) psi[i] = psi[i] - c * chi[i];
    }
    free(chi);
}

/* Shift expression evaluated only at the listed sites (for sampled checks of
 * large lattices), written as double[n][4][3][2]. */
void oracle_shift_sites(const int *L, const double *U, const double *psi, const double *phi, double a, long n,
                        const long *sites, double *chi)
{
    lat g = lat_make(L);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        cplx acc[4][3];
        shift_site(&g, U, psi, phi, a, 0xFu, +1, sites[i], acc);
        for (int sp = 0; sp < 4; ++sp)
            for (int c = 0; c < 3; ++c) store_fermion(chi, i, sp, c, acc[sp][c]);
    }
}

/* ------------------------------------------------------------------ */
/* Jacobi smearing (the paper's application, section 7)                */
/* ------------------------------------------------------------------ */

/* Hopping term of the smearing operator K, over the directions in mask:
 * (H psi)(x) = sum_{mu in mask} [ U_mu(x) psi(x+mu) + U_mu(x-mu)^dagger psi(x-mu) ]. */
void oracle_hop(const int *L, const double *U, const double *psi, unsigned mask, double *out)
{
    lat g = lat_make(L);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < g.V; ++s) {
        cplx acc[4][3];
        for (int sp = 0; sp < 4; ++sp)
            for (int c = 0; c < 3; ++c) acc[sp][c] = c_make(0.0, 0.0);
        for (int mu = 0; mu < 4; ++mu) {
            if (!((mask >> mu) & 1u)) continue;
            mat3 uf = load_link(U, s, mu);
            long fwd = hop(&g, s, mu, +1);
            long bwd = hop(&g, s, mu, -1);
            mat3 ub = load_link(U, bwd, mu);
            for (int sp = 0; sp < 4; ++sp)
                for (int ca = 0; ca < 3; ++ca)
                    for (int cb = 0; cb < 3; ++cb) {
                        acc[sp][ca] = c_add(acc[sp][ca], c_mul(uf.e[ca][cb], load_fermion(psi, fwd, sp, cb)));
                        /* (U^dagger)_{ab} = conj(U_{ba}) */
                        acc[sp][ca] = c_add(acc[sp][ca], c_mul(c_conj(ub.e[cb][ca]), load_fermion(psi, bwd, sp, cb)));
                    }
        }
        for (int sp = 0; sp < 4; ++sp)
            for (int c = 0; c < 3; ++c) store_fermion(out, s, sp, c, acc[sp][c]);
    }
}

/* Jacobi smearing (section 7).  The smearing operator is K = 1 - kappa H, H
 * the hopping term above, and the smeared source is the truncated power
 * series of K^{-1} applied to the source s0, divided by a normalisation:
 *   chi_N = (1/norm) sum_{n=0}^{N} (kappa H)^n s0.
 * The terms are built one from the other, t_0 = s0 and t_{n+1} = kappa H t_n,
 * and added in the order n = 0..N.  chi holds s0 on entry and chi_N on exit. */
void oracle_jacobi_smear(const int *L, const double *U, double *chi, double kappa, int n_iter, double norm,
                         unsigned mask)
{
    lat g = lat_make(L);
    size_t nf = (size_t)g.V * 4 * 3 * 2;
    double *term = (double *)malloc(sizeof(double) * nf);
    double *sum = (double *)malloc(sizeof(double) * nf);
    double *h = (double *)malloc(sizeof(double) * nf);
    memcpy(term, chi, sizeof(double) * nf);
    memcpy(sum, chi, sizeof(double) * nf);
    for (int n = 1; n <= n_iter; ++n) {
        oracle_hop(L, U, term, mask, h);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < (long)nf; ++i) {
            term[i] = kappa * h[i];
            sum[i] += term[i];
        }
    }
#pragma omp parallel for schedule(static)
    for (long i = 0; i < (long)nf; ++i) chi[i] = sum[i] / norm;
    free(term);
    free(sum);
    free(h);
}

/* ------------------------------------------------------------------ */
/* APE smearing                                                        */
/* ------------------------------------------------------------------ */

/* upper staple of U_mu(x) in the (mu, nu) plane: U_nu(x) U_mu(x+nu) U_nu(x+mu)^dagger */
static mat3 staple_upper(const lat *g, const double *U, long s, int mu, int nu)
{
    mat3 a = load_link(U, s, nu);
    mat3 b = load_link(U, hop(g, s, nu, +1), mu);
    mat3 c = load_link(U, hop(g, s, mu, +1), nu);
    mat3 cd = m_dag(&c);
    mat3 ab = m_mul(&a, &b);
    return m_mul(&ab, &cd);
}

/* lower staple: U_nu(x-nu)^dagger U_mu(x-nu) U_nu(x-nu+mu) */
static mat3 staple_lower(const lat *g, const double *U, long s, int mu, int nu)
{
    long sm = hop(g, s, nu, -1);
    mat3 a = load_link(U, sm, nu);
    mat3 b = load_link(U, sm, mu);
    mat3 c = load_link(U, hop(g, sm, mu, +1), nu);
    mat3 ad = m_dag(&a);
    mat3 ab = m_mul(&ad, &b);
    return m_mul(&ab, &c);
}

/* Sup(x,mu) = sum_{nu != mu} upper staples, Slo(x,mu) = sum_{nu != mu} lower
 * staples, nu taken in increasing order.  Either output may be NULL. */
void oracle_staple_sums(const int *L, const double *U, double *Sup, double *Slo)
{
    lat g = lat_make(L);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < g.V; ++s)
        for (int mu = 0; mu < 4; ++mu) {
            mat3 up = m_zero(), lo = m_zero();
            for (int nu = 0; nu < 4; ++nu) {
                if (nu == mu) continue;
                mat3 su = staple_upper(&g, U, s, mu, nu);
                mat3 sl = staple_lower(&g, U, s, mu, nu);
                up = m_add(&up, &su);
                lo = m_add(&lo, &sl);
            }
            if (Sup) store_link(Sup, s, mu, &up);
            if (Slo) store_link(Slo, s, mu, &lo);
        }
}

static int reunitarise(const mat3 *W, mat3 *V);
static int polar_project(const mat3 *W, mat3 *V);

/* W_mu(x) = (1-alpha) U_mu(x) + alpha * (mean of the staples of U_mu(x) in
 * the planes (mu, nu), nu in mask, nu != mu): with all four directions that
 * is alpha/6 times the sum of six staples, with the three spatial ones
 * alpha/4 times the sum of four.  The staples are accumulated for
 * nu = 0..3 in increasing order, upper before lower. */
static mat3 ape_w_link(const lat *g, const double *U, long s, int mu, double alpha, unsigned mask)
{
    mat3 S = m_zero();
    int n = 0;
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu || !((mask >> nu) & 1u)) continue;
        mat3 su = staple_upper(g, U, s, mu, nu);
        S = m_add(&S, &su);
        mat3 sl = staple_lower(g, U, s, mu, nu);
        S = m_add(&S, &sl);
        n += 2;
    }
    const double wt = n > 0 ? alpha / n : 0.0;
    mat3 u = load_link(U, s, mu);
    mat3 W;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            W.e[i][j] = c_add(c_scale(1.0 - alpha, u.e[i][j]), c_scale(wt, S.e[i][j]));
    return W;
}

/* One smeared link: directions outside the mask keep U_mu(x) unchanged,
 * the others are Proj[W_mu(x)].  Returns 1 for a degenerate W. */
static int ape_link(const lat *g, const double *U, long s, int mu, double alpha, unsigned mask, int proj,
                    mat3 *V)
{
    if (!((mask >> mu) & 1u)) {
        *V = load_link(U, s, mu);
        return 0;
    }
    mat3 w = ape_w_link(g, U, s, mu, alpha, mask);
    return proj ? polar_project(&w, V) : reunitarise(&w, V);
}

/* Reunitarise by rows: u = r1/|r1|; v = r2 - (sum_j conj(u_j) r2_j) u, v /= |v|;
 * w = conj(u x v).  Returns 0, or 1 if a row norm was zero (the output is then NaN). */
static int reunitarise(const mat3 *W, mat3 *V)
{
    cplx u[3], v[3];
    double n0 = 0.0;
    for (int j = 0; j < 3; ++j) n0 += c_abs2(W->e[0][j]);
    n0 = sqrt(n0);
    int bad = (n0 == 0.0);
    for (int j = 0; j < 3; ++j) u[j] = c_scale(1.0 / n0, W->e[0][j]);

    cplx d = c_make(0.0, 0.0);
    for (int j = 0; j < 3; ++j) d = c_add(d, c_mul(c_conj(u[j]), W->e[1][j]));
    for (int j = 0; j < 3; ++j) v[j] = c_sub(W->e[1][j], c_mul(d, u[j]));
    double n1 = 0.0;
    for (int j = 0; j < 3; ++j) n1 += c_abs2(v[j]);
    n1 = sqrt(n1);
    bad |= (n1 == 0.0);
    for (int j = 0; j < 3; ++j) v[j] = c_scale(1.0 / n1, v[j]);

    for (int j = 0; j < 3; ++j) {
        V->e[0][j] = u[j];
        V->e[1][j] = v[j];
    }
    V->e[2][0] = c_conj(c_sub(c_mul(u[1], v[2]), c_mul(u[2], v[1])));
    V->e[2][1] = c_conj(c_sub(c_mul(u[2], v[0]), c_mul(u[0], v[2])));
    V->e[2][2] = c_conj(c_sub(c_mul(u[0], v[1]), c_mul(u[1], v[0])));
    if (bad) {
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) V->e[i][j] = c_make(NAN, NAN);
    }
    return bad;
}

/* Eigen-decomposition of a real symmetric n x n matrix (n <= 6) by cyclic
 * Jacobi rotations, A = Q diag(lam) Q^T; A is overwritten.  Each rotation
 * zeroes one off-diagonal pair; an element below rounding relative to its
 * two diagonal entries is set to zero instead, and the sweeps stop when a
 * whole sweep finds nothing left to rotate. */
static void sym_jacobi(int n, double A[6][6], double lam[6], double Q[6][6])
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Q[i][j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        int rotated = 0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                if (fabs(A[p][q]) <= 1e-18 * sqrt(fabs(A[p][p] * A[q][q]))) {
                    A[p][q] = A[q][p] = 0.0;
                    continue;
                }
                rotated = 1;
                /* rotation angle that zeroes A[p][q]: tan(2 phi) = 2 A_pq / (A_qq - A_pp) */
                double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
                /* A <- J^T A J with J = [[c, s], [-s, c]] on rows/columns p, q:
                 * the rotated pair is zero and the diagonal moves by t A_pq */
                const double apq = A[p][q];
                A[p][p] -= t * apq;
                A[q][q] += t * apq;
                A[p][q] = A[q][p] = 0.0;
                for (int k = 0; k < n; ++k) {
                    if (k == p || k == q) continue;
                    double akp = A[k][p], akq = A[k][q];
                    A[k][p] = A[p][k] = c * akp - sn * akq;
                    A[k][q] = A[q][k] = sn * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) { /* accumulate Q <- Q J */
                    double qkp = Q[k][p], qkq = Q[k][q];
                    Q[k][p] = c * qkp - sn * qkq;
                    Q[k][q] = sn * qkp + c * qkq;
                }
            }
        if (!rotated) break;
    }
    for (int i = 0; i < n; ++i) lam[i] = A[i][i];
}

/* Bi-covariant projection: V = W (W^dag W)^(-1/2) exp(-i arg(det)/3), the
 * unitary factor of the polar decomposition of W with the phase of its
 * determinant removed on the principal branch.  The inverse square root of
 * the Hermitian H = W^dag W is taken through the real symmetric 6x6 matrix
 * [[Re H, -Im H], [Im H, Re H]], which represents H faithfully (a function of
 * it represents the same function of H).  Returns 1 (output NaN) if H is not
 * positive definite. */
static int polar_project(const mat3 *W, mat3 *V)
{
    mat3 Wd = m_dag(W);
    mat3 H = m_mul(&Wd, W);
    double M[6][6], lam[6], Q[6][6];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            M[i][j] = H.e[i][j].re;
            M[i][j + 3] = -H.e[i][j].im;
            M[i + 3][j] = H.e[i][j].im;
            M[i + 3][j + 3] = H.e[i][j].re;
        }
    sym_jacobi(6, M, lam, Q);
    int bad = 0;
    double f[6];
    for (int k = 0; k < 6; ++k) {
        bad |= !(lam[k] > 0.0);
        f[k] = 1.0 / sqrt(lam[k]);
    }
    mat3 R; /* H^(-1/2): top-left block is its real part, bottom-left its imaginary part */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double re = 0.0, im = 0.0;
            for (int k = 0; k < 6; ++k) {
                re += f[k] * Q[i][k] * Q[j][k];
                im += f[k] * Q[i + 3][k] * Q[j][k];
            }
            R.e[i][j] = c_make(re, im);
        }
    mat3 P = m_mul(W, &R);
    cplx d = c_sub(c_add(c_mul(P.e[0][0], c_sub(c_mul(P.e[1][1], P.e[2][2]), c_mul(P.e[1][2], P.e[2][1]))),
                         c_mul(P.e[0][2], c_sub(c_mul(P.e[1][0], P.e[2][1]), c_mul(P.e[1][1], P.e[2][0])))),
                   c_mul(P.e[0][1], c_sub(c_mul(P.e[1][0], P.e[2][2]), c_mul(P.e[1][2], P.e[2][0]))));
    double ph = -atan2(d.im, d.re) / 3.0;
    cplx z = c_make(cos(ph), sin(ph));
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) V->e[i][j] = bad ? c_make(NAN, NAN) : c_mul(P.e[i][j], z);
    return bad;
}

/* Unprojected APE combination W for every link (every direction, with the
 * staples of the directions in mask). */
void oracle_ape_w(const int *L, const double *U, double alpha, unsigned mask, double *W)
{
    lat g = lat_make(L);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < g.V; ++s)
        for (int mu = 0; mu < 4; ++mu) {
            mat3 w = ape_w_link(&g, U, s, mu, alpha, mask);
            store_link(W, s, mu, &w);
        }
}

/* Row Gram-Schmidt projection of n_links matrices (layout [n][3][3][2]).
 * Returns the number of degenerate inputs. */
long oracle_reunitarise(long n_links, const double *W, double *V)
{
    long bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (long i = 0; i < n_links; ++i) {
        mat3 w, v;
        const double *p = W + (size_t)i * 18;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) w.e[a][b] = c_make(p[(a * 3 + b) * 2], p[(a * 3 + b) * 2 + 1]);
        bad += reunitarise(&w, &v);
        double *q = V + (size_t)i * 18;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                q[(a * 3 + b) * 2] = v.e[a][b].re;
                q[(a * 3 + b) * 2 + 1] = v.e[a][b].im;
            }
    }
    return bad;
}

/* Bi-covariant (polar) projection of n_links matrices (layout [n][3][3][2]).
 * Returns the number of degenerate inputs. */
long oracle_polar_project(long n_links, const double *W, double *V)
{
    long bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (long i = 0; i < n_links; ++i) {
        mat3 w, v;
        const double *p = W + (size_t)i * 18;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) w.e[a][b] = c_make(p[(a * 3 + b) * 2], p[(a * 3 + b) * 2 + 1]);
        bad += polar_project(&w, &v);
        double *q = V + (size_t)i * 18;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                q[(a * 3 + b) * 2] = v.e[a][b].re;
                q[(a * 3 + b) * 2 + 1] = v.e[a][b].im;
            }
    }
    return bad;
}

/* One APE step: V_mu(x) = Proj[W_mu(x)] for the links of the directions in
 * mask, all from the unsmeared U; the other links are copied.
 * Returns the number of degenerate links. */
long oracle_ape_step(const int *L, const double *U, double alpha, unsigned mask, int proj, double *Vout)
{
    lat g = lat_make(L);
    long bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (long s = 0; s < g.V; ++s)
        for (int mu = 0; mu < 4; ++mu) {
            mat3 v;
            bad += ape_link(&g, U, s, mu, alpha, mask, proj, &v);
            store_link(Vout, s, mu, &v);
        }
    return bad;
}

/* n_steps APE steps; Vout receives the last step, U is not modified. */
long oracle_ape_smear(const int *L, const double *U, double alpha, unsigned mask, int proj, int n_steps,
                      double *Vout)
{
    lat g = lat_make(L);
    size_t nl = (size_t)g.V * 4 * 18;
    double *cur = (double *)malloc(sizeof(double) * nl);
    long bad = 0;
    memcpy(cur, U, sizeof(double) * nl);
    for (int k = 0; k < n_steps; ++k) {
        bad += oracle_ape_step(L, cur, alpha, mask, proj, Vout);
        memcpy(cur, Vout, sizeof(double) * nl);
    }
    if (n_steps == 0) memcpy(Vout, U, sizeof(double) * nl);
    free(cur);
    return bad;
}

/* One APE step evaluated only for the listed links (site[i], mu[i]). */
long oracle_ape_links(const int *L, const double *U, double alpha, unsigned mask, int proj, long n,
                      const long *site, const int *mu, double *Vout)
{
    lat g = lat_make(L);
    long bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (long i = 0; i < n; ++i) {
        mat3 v;
        bad += ape_link(&g, U, site[i], mu[i], alpha, mask, proj, &v);
        double *q = Vout + (size_t)i * 18;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                q[(a * 3 + b) * 2] = v.e[a][b].re;
                q[(a * 3 + b) * 2 + 1] = v.e[a][b].im;
            }
    }
    return bad;
}

/* ------------------------------------------------------------------ */
/* plaquette                                                           */
/* ------------------------------------------------------------------ */

/* Re Tr [U_mu(x) U_nu(x+mu) U_mu(x+nu)^dagger U_nu(x)^dagger] */
static double plaq_site(const lat *g, const double *U, long s, int mu, int nu)
{
    mat3 a = load_link(U, s, mu);
    mat3 b = load_link(U, hop(g, s, mu, +1), nu);
    mat3 c = load_link(U, hop(g, s, nu, +1), mu);
    mat3 d = load_link(U, s, nu);
    mat3 cd = m_dag(&c), dd = m_dag(&d);
    mat3 ab = m_mul(&a, &b);
    mat3 abc = m_mul(&ab, &cd);
    mat3 p = m_mul(&abc, &dd);
    return m_retrace(&p);
}

/* out[0] = (1/(18 V)) sum_x sum_{mu<nu} Re Tr P_{mu nu}(x)   (all six planes)
 * out[1] = (1/(9 V))  sum over the three spatial planes (mu < nu < 3)
 * out[2] = (1/(9 V))  sum over the three temporal planes (nu = 3)
 * Unit links give 1 in all three. */
void oracle_plaquette(const int *L, const double *U, double *out)
{
    lat g = lat_make(L);
    double *sp = (double *)malloc(sizeof(double) * (size_t)g.V);
    double *tp = (double *)malloc(sizeof(double) * (size_t)g.V);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < g.V; ++s) {
        double a = 0.0, b = 0.0;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                double p = plaq_site(&g, U, s, mu, nu);
                if (nu == 3) b += p;
                else a += p;
            }
        sp[s] = a;
        tp[s] = b;
    }
    double ssum = oracle_neumaier_sum(g.V, sp);
    double tsum = oracle_neumaier_sum(g.V, tp);
    out[0] = (ssum + tsum) / (18.0 * (double)g.V);
    out[1] = ssum / (9.0 * (double)g.V);
    out[2] = tsum / (9.0 * (double)g.V);
    free(sp);
    free(tp);
}
