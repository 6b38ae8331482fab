/* Drives the C oracle's routines on small seeded inputs for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_oracle_sanitize.py).
 * Besides any memory or UB error the sanitizers report, it checks
 * invariants the mathematics fixes: the Jacobi eigenpairs reconstruct A with
 * orthonormal vectors, 2 sum f = N_e and Tr D = N_e at the bisected mu, the
 * canonical response conserves charge, and the pair forces sum to zero
 * (translation invariance).  Exit status 0 when every check holds. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_jacobi(int N, double *A, double *evals, double *Vt, double tol, int max_sweeps);
double orc_fermi_mu(int N, const double *ev, double beta, double ne, double *f);
int orc_density(int N, const double *Vt, const double *f, double *D);
double orc_response_diag(int N, const double *Vt, const double *ev, double beta, double mu,
                         const double *h, double *dd);
int orc_h0(int nat, int no, const double *pos, const double *onsite, const double *jitter,
           const double *B, double decay, double rc, double w, double *H0);
int orc_gamma(int nat, const double *pos, const double *U, double soft, double *G);
double orc_erep(int nat, const double *pos, double A, double decay, double rc, double w,
                double *F);
int orc_forces(int nat, int no, const double *pos, const double *B, double decay, double rc,
               double w, double soft, const double *D, const double *q, const double *n,
               double *F);

static unsigned long long state = 0x9e3779b97f4a7c15ULL;
static double uniform(void) {            /* splitmix64, in [-1, 1) */
    unsigned long long z = (state += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    z ^= z >> 31;
    return (double)(z >> 11) / 9007199254740992.0 * 2.0 - 1.0;
}
static int fails = 0;
static void check(int ok, const char *what, double val) {
    printf("%-48s %s (%.3e)\n", what, ok ? "ok" : "FAILED", val);
    if (!ok) ++fails;
}

int main(void) {
    /* 1. Jacobi on a seeded symmetric 12 x 12 matrix */
    const int N = 12;
    double *A = malloc(sizeof(double) * N * N), *A0 = malloc(sizeof(double) * N * N);
    double *ev = malloc(sizeof(double) * N), *Vt = malloc(sizeof(double) * N * N);
    for (int i = 0; i < N; ++i)
        for (int j = 0; j <= i; ++j) A[i * N + j] = A[j * N + i] = uniform();
    memcpy(A0, A, sizeof(double) * N * N);
    int sweeps = orc_jacobi(N, A, ev, Vt, 1e-14, 50);
    check(sweeps >= 0, "jacobi converged", (double)sweeps);
    double rec = 0.0, orth = 0.0;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            double a = 0.0, o = 0.0;
            for (int k = 0; k < N; ++k) {
                a += ev[k] * Vt[k * N + i] * Vt[k * N + j];
                o += Vt[i * N + k] * Vt[j * N + k];
            }
            rec = fmax(rec, fabs(a - A0[i * N + j]));
            orth = fmax(orth, fabs(o - (i == j)));
        }
    check(rec < 1e-12, "jacobi: sum lambda v v^T = A", rec);
    check(orth < 1e-12, "jacobi: orthonormal eigenvectors", orth);

    /* 2-4. occupations, density, canonical response at beta = 10 */
    const double beta = 10.0, ne = 10.0;
    double *f = malloc(sizeof(double) * N), *D = malloc(sizeof(double) * N * N);
    double *h = malloc(sizeof(double) * N), *dd = malloc(sizeof(double) * N);
    double mu = orc_fermi_mu(N, ev, beta, ne, f);
    double cnt = 0.0;
    for (int i = 0; i < N; ++i) cnt += 2.0 * f[i];
    check(fabs(cnt - ne) < 1e-9, "2 sum f = N_e at the bisected mu", fabs(cnt - ne));
    orc_density(N, Vt, f, D);
    double tr = 0.0, asym = 0.0;
    for (int i = 0; i < N; ++i) {
        tr += D[i * N + i];
        for (int j = 0; j < N; ++j) asym = fmax(asym, fabs(D[i * N + j] - D[j * N + i]));
    }
    check(fabs(tr - ne) < 1e-9, "Tr D = N_e", fabs(tr - ne));
    check(asym < 1e-13, "D symmetric", asym);
    for (int i = 0; i < N; ++i) h[i] = uniform();
    orc_response_diag(N, Vt, ev, beta, mu, h, dd);
    double sdd = 0.0, amax = 0.0;
    for (int i = 0; i < N; ++i) { sdd += dd[i]; amax = fmax(amax, fabs(dd[i])); }
    check(fabs(sdd) < 1e-12 * (1.0 + amax) && amax > 0.0, "canonical response: sum dD_ii = 0",
          fabs(sdd));

    /* 5. model tables and forces: 8 atoms x 2 orbitals */
    const int nat = 8, no = 2, M = nat * no;
    double pos[3 * 8], onsite[2] = {-1.0, -0.4}, jit[16], B[4] = {-1.0, 0.3, 0.3, -0.6};
    double U[8], q[8], n[8], G[64], Fb[24], Fr[24];
    for (int I = 0; I < nat; ++I) {
        pos[3 * I] = 2.2 * (I % 2) + 0.1 * uniform();
        pos[3 * I + 1] = 2.2 * ((I / 2) % 2) + 0.1 * uniform();
        pos[3 * I + 2] = 2.2 * (I / 4) + 0.1 * uniform();
        U[I] = 1.0 + 0.2 * uniform();
        n[I] = 0.05 * uniform();
        q[I] = 0.05 * uniform();
    }
    for (int i = 0; i < M; ++i) jit[i] = 0.05 * uniform();
    double *H0 = malloc(sizeof(double) * M * M), *Dm = malloc(sizeof(double) * M * M);
    orc_h0(nat, no, pos, onsite, jit, B, 1.2, 5.0, 0.5, H0);
    double hs = 0.0;
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) hs = fmax(hs, fabs(H0[i * M + j] - H0[j * M + i]));
    check(hs == 0.0, "H0 symmetric", hs);
    orc_gamma(nat, pos, U, 1.0, G);
    for (int i = 0; i < M; ++i)          /* any symmetric D */
        for (int j = 0; j <= i; ++j) Dm[i * M + j] = Dm[j * M + i] = 0.3 * uniform();
    orc_forces(nat, no, pos, B, 1.2, 5.0, 0.5, 1.0, Dm, q, n, Fb);
    memset(Fr, 0, sizeof Fr);
    double er = orc_erep(nat, pos, 5.8, 0.6, 5.0, 0.5, Fr);
    double net[3] = {0, 0, 0}, fmag = 0.0;
    for (int I = 0; I < nat; ++I)
        for (int c = 0; c < 3; ++c) {
            net[c] += Fb[3 * I + c] + Fr[3 * I + c];
            fmag = fmax(fmag, fabs(Fb[3 * I + c]));
        }
    double nm = fmax(fabs(net[0]), fmax(fabs(net[1]), fabs(net[2])));
    check(isfinite(er) && fmag > 0.0, "forces and repulsion finite, nonzero", fmag);
    check(nm < 1e-12 * (1.0 + fmag), "pair forces sum to zero", nm);

    free(A); free(A0); free(ev); free(Vt); free(f); free(D); free(h); free(dd);
    free(H0); free(Dm);
    printf("%d failed\n", fails);
    return fails ? 1 : 0;
}
