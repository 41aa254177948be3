/* Drives every entry point of the C oracle on small ragged lattices, with one
 * and with four OpenMP threads, so that a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer can report any out-of-bounds access, leak or
 * undefined operation in it.  Inputs are fixed pseudo-random numbers (not
 * SU(3) matrices: the memory paths are the same).  Prints "ok" when every
 * output is finite and no projection met a degenerate input. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

double oracle_neumaier_sum(long n, const double *x);
void oracle_set_num_threads(int n);
void oracle_shift_mul_axpy(const int *L, const double *U, const double *psi, const double *phi, double a,
                           double *chi, double *norm2);
void oracle_shift_chain(const int *L, const double *U, double *psi, const double *phi, double a, double c,
                        int n_iter, double *norms);
void oracle_shift_sites(const int *L, const double *U, const double *psi, const double *phi, double a, long n,
                        const long *sites, double *chi);
void oracle_hop(const int *L, const double *U, const double *psi, unsigned mask, double *out);
void oracle_jacobi_smear(const int *L, const double *U, double *chi, double kappa, int n_iter, double norm,
                         unsigned mask);
void oracle_staple_sums(const int *L, const double *U, double *Sup, double *Slo);
void oracle_ape_w(const int *L, const double *U, double alpha, unsigned mask, double *W);
long oracle_reunitarise(long n_links, const double *W, double *V);
long oracle_polar_project(long n_links, const double *W, double *V);
long oracle_ape_smear(const int *L, const double *U, double alpha, unsigned mask, int proj, int n_steps,
                      double *Vout);
long oracle_ape_links(const int *L, const double *U, double alpha, unsigned mask, int proj, long n,
                      const long *site, const int *mu, double *Vout);
void oracle_plaquette(const int *L, const double *U, double *out);

static uint64_t state = 88172645463325252ull;

static double uniform(void) /* xorshift64, in [-0.5, 0.5) */
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) / 9007199254740992.0 - 0.5;
}

static double *fresh(size_t n)
{
    double *p = malloc(n * sizeof *p);
    for (size_t i = 0; i < n; ++i) p[i] = uniform();
    return p;
}

static int finite_all(const double *p, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(p[i])) return 0;
    return 1;
}

int main(void)
{
    const int lattices[3][4] = {{3, 5, 4, 7}, {2, 2, 2, 2}, {4, 3, 2, 5}};
    int fails = 0;
    for (int threads = 1; threads <= 4; threads += 3) {
        oracle_set_num_threads(threads);
        for (int t = 0; t < 3; ++t) {
            const int *L = lattices[t];
            const long V = (long)L[0] * L[1] * L[2] * L[3];
            const size_t nl = (size_t)V * 72, nf = (size_t)V * 24;
            double *U = fresh(nl), *psi = fresh(nf), *phi = fresh(nf), *chi = fresh(nf);
            double *W = fresh(nl), *S = fresh(nl), *Vo = fresh(nl);
            double n2, norms[3], plaq[3];
            const long sites[3] = {0, V / 2, V - 1};
            const int mus[3] = {0, 2, 3};
            long bad = 0;
            oracle_shift_mul_axpy(L, U, psi, phi, 0.3, chi, &n2);
            oracle_shift_chain(L, U, psi, phi, 0.3, 0.1, 3, norms);
            oracle_shift_sites(L, U, psi, phi, 0.3, 3, sites, chi);
            oracle_hop(L, U, psi, 0xF, chi);
            oracle_jacobi_smear(L, U, psi, 0.2, 3, 1.5, 0x7);
            oracle_staple_sums(L, U, W, S);
            oracle_ape_w(L, U, 0.5, 0xF, W);
            bad += oracle_reunitarise(V * 4, W, Vo);
            bad += oracle_polar_project(V * 4, W, Vo);
            bad += oracle_ape_smear(L, U, 0.5, 0x7, 0, 2, Vo);
            bad += oracle_ape_smear(L, U, 0.5, 0xF, 1, 1, Vo);
            bad += oracle_ape_links(L, U, 0.5, 0xF, 0, 3, sites, mus, Vo);
            oracle_plaquette(L, U, plaq);
            const double sum = oracle_neumaier_sum((long)nf, psi);
            if (bad || !finite_all(chi, nf) || !finite_all(psi, nf) || !finite_all(Vo, nl) || !finite_all(norms, 3) ||
                !finite_all(plaq, 3) || !isfinite(n2) || !isfinite(sum)) {
                printf("FAIL threads %d lattice %dx%dx%dx%d (degenerate %ld)\n", threads, L[0], L[1], L[2], L[3], bad);
                fails++;
            }
            free(U), free(psi), free(phi), free(chi), free(W), free(S), free(Vo);
        }
    }
    if (!fails) printf("ok\n");
    return fails != 0;
}
