/*
 * CPU oracle for finite-temperature XL-BOMD (Niklasson, "Next generation
 * extended Lagrangian first principles molecular dynamics").
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, FP64 C written for clarity, not
 * speed.  It is used by tests/, by the smoke check and by the benchmark's
 * CPU baseline; the HIP library never links or calls it and shares no code
 * with it.
 *
 * Contents (each function cites the passage it follows):
 *   - the synthetic SCC tight-binding model: H0, Coulomb matrix, repulsion
 *     (Section VI, SCC-DFTB description, specialised to an orthogonal basis);
 *   - a cyclic Jacobi eigensolver (stands in for the one diagonalization per
 *     step the paper performs, Section III.B);
 *   - Fermi-Dirac occupations with the chemical potential found by
 *     bisection, and the Fermi-Dirac entropy (Section IV.B, Eqs. 36-38);
 *   - the density matrix D = 2 Q f Q^T and Mulliken charges;
 *   - the canonical (fixed electron number) first-order response of the
 *     charges to a potential perturbation, in closed form through divided
 *     differences of the occupations (Section V.B);
 *   - Hellmann-Feynman forces at fixed n (the fixed-n derivative in Eq. 40).
 *
 * Every function returns 0 on success, a negative value on bad input.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Model                                                               */
/* ------------------------------------------------------------------ */

/* Smooth cutoff s(r): 1 below rc - w, 0 above rc, quintic C2 ramp between.
 * w == 0 gives a hard cutoff (s = 1 for r < rc).  Reading: the workloads
 * state hopping "for r < rc"; a hard cutoff makes the potential surface
 * discontinuous, so a ramp of width w ends it smoothly. */
void orc_taper(double r, double rc, double w, double *s, double *ds)
{
    if (r >= rc) { *s = 0.0; *ds = 0.0; return; }
    if (w <= 0.0 || r <= rc - w) { *s = 1.0; *ds = 0.0; return; }
    double t = (r - (rc - w)) / w;
    double t2 = t * t, t3 = t2 * t;
    *s = 1.0 - 10.0 * t3 + 15.0 * t3 * t - 6.0 * t3 * t2;
    *ds = (-30.0 * t2 + 60.0 * t3 - 30.0 * t3 * t) / w;
}

static double dist3(const double *a, const double *b, double d[3])
{
    d[0] = a[0] - b[0]; d[1] = a[1] - b[1]; d[2] = a[2] - b[2];
    return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

/* Charge-independent Hamiltonian H0 (N x N, N = nat*no, row-major).
 * Orbital index of orbital a on atom I is I*no + a.
 *   H0[Ia,Ia] = onsite[a] + jitter[Ia];  H0[Ia,Ib] = 0 for a != b;
 *   H0[Ia,Jb] = B[a,b] * exp(-r_IJ / decay) * s(r_IJ)   for I != J. */
int orc_h0(int nat, int no, const double *pos, const double *onsite,
           const double *jitter, const double *B, double decay, double rc,
           double w, double *H0)
{
    if (nat <= 0 || no <= 0) return -1;
    int N = nat * no;
    memset(H0, 0, sizeof(double) * (size_t)N * N);
    for (int I = 0; I < nat; ++I)
        for (int a = 0; a < no; ++a)
            H0[(size_t)(I * no + a) * N + I * no + a] =
                onsite[a] + (jitter ? jitter[I * no + a] : 0.0);
    for (int I = 0; I < nat; ++I)
        for (int J = 0; J < nat; ++J) {
            if (I == J) continue;
            double d[3];
            double r = dist3(pos + 3 * I, pos + 3 * J, d);
            if (r >= rc) continue;
            double s, ds;
            orc_taper(r, rc, w, &s, &ds);
            double h = exp(-r / decay) * s;
            for (int a = 0; a < no; ++a)
                for (int b = 0; b < no; ++b)
                    H0[(size_t)(I * no + a) * N + J * no + b] = B[a * no + b] * h;
        }
    return 0;
}

/* Coulomb matrix over atoms: Gamma[I,I] = U_I; Gamma[I,J] = 1/sqrt(r^2+a^2).
 * Open boundaries, plain pair sum. */
int orc_gamma(int nat, const double *pos, const double *U, double soft,
              double *G)
{
    if (nat <= 0) return -1;
    for (int I = 0; I < nat; ++I)
        for (int J = 0; J < nat; ++J) {
            if (I == J) { G[(size_t)I * nat + J] = U[I]; continue; }
            double d[3];
            double r = dist3(pos + 3 * I, pos + 3 * J, d);
            G[(size_t)I * nat + J] = 1.0 / sqrt(r * r + soft * soft);
        }
    return 0;
}

/* Pair repulsion E_rep = sum_{I<J} A exp(-r/decay) s(r); adds -dE/dR to F. */
double orc_erep(int nat, const double *pos, double A, double decay,
                double rc, double w, double *F)
{
    double e = 0.0;
    if (A == 0.0) return 0.0;
    for (int I = 0; I < nat; ++I)
        for (int J = I + 1; J < nat; ++J) {
            double d[3];
            double r = dist3(pos + 3 * I, pos + 3 * J, d);
            if (r >= rc) continue;
            double s, ds;
            orc_taper(r, rc, w, &s, &ds);
            double ex = A * exp(-r / decay);
            e += ex * s;
            double dedr = ex * (ds - s / decay);
            if (F)
                for (int c = 0; c < 3; ++c) {
                    double g = dedr * d[c] / r;   /* dE/dR_I */
                    F[3 * I + c] -= g;
                    F[3 * J + c] += g;
                }
        }
    return e;
}

/* Hellmann-Feynman forces at fixed n and fixed D (the fixed-n derivative in Eq. 40):
 *   band:    -2 sum_{J!=I} sum_ab B_ab d/dR_I[h(r)s(r)] D[Ia,Jb]
 *   Coulomb: -1/2 sum_{J!=I} [(2q_I-n_I) n_J + (2q_J-n_J) n_I] dGamma_IJ/dR_I
 * Repulsion is added separately by orc_erep.  F is overwritten. */
int orc_forces(int nat, int no, const double *pos, const double *B,
               double decay, double rc, double w, double soft,
               const double *D, const double *q, const double *n, double *F)
{
    if (nat <= 0 || no <= 0) return -1;
    int N = nat * no;
    memset(F, 0, sizeof(double) * 3 * (size_t)nat);
    for (int I = 0; I < nat; ++I)
        for (int J = 0; J < nat; ++J) {
            if (I == J) continue;
            double d[3];
            double r = dist3(pos + 3 * I, pos + 3 * J, d);
            double g = 0.0;   /* scalar radial derivative dE/dr */
            if (r < rc) {
                double s, ds;
                orc_taper(r, rc, w, &s, &ds);
                double ex = exp(-r / decay);
                double dh = ex * (ds - s / decay);
                double bd = 0.0;
                for (int a = 0; a < no; ++a)
                    for (int b = 0; b < no; ++b)
                        bd += B[a * no + b] * D[(size_t)(I * no + a) * N + J * no + b];
                g += 2.0 * dh * bd;
            }
            double inv = 1.0 / sqrt(r * r + soft * soft);
            double dgam = -r * inv * inv * inv;    /* d gamma / dr */
            g += 0.5 * ((2.0 * q[I] - n[I]) * n[J] + (2.0 * q[J] - n[J]) * n[I]) * dgam;
            for (int c = 0; c < 3; ++c) F[3 * I + c] -= g * d[c] / r;
        }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Cyclic Jacobi eigensolver                                           */
/* ------------------------------------------------------------------ */

/* Diagonalise the symmetric matrix A (N x N, row-major, destroyed) by cyclic
 * Jacobi rotations until the off-diagonal Frobenius norm is below
 * tol * ||A||_F.  On return evals[i] holds eigenvalue i and ROW i of Vt
 * (Vt[i*N+k]) the matching normalised eigenvector.  Returns the number of
 * sweeps, or -1 if max_sweeps was reached.
 *
 * Each rotation in the (p,q) plane is chosen to zero A[p,q]; rows p and q
 * are combined and, A being symmetric, the columns are their mirror. */
int orc_jacobi(int N, double *A, double *evals, double *Vt, double tol,
               int max_sweeps)
{
    if (N <= 0) return -1;
    double fro = 0.0;
    for (size_t i = 0; i < (size_t)N * N; ++i) fro += A[i] * A[i];
    fro = sqrt(fro);
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) Vt[(size_t)i * N + j] = (i == j);
    if (fro == 0.0) { for (int i = 0; i < N; ++i) evals[i] = 0.0; return 0; }
    for (int sweep = 0; sweep <= max_sweeps; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < N; ++p)
            for (int q = p + 1; q < N; ++q) off += 2.0 * A[(size_t)p * N + q] * A[(size_t)p * N + q];
        if (sqrt(off) <= tol * fro) {
            for (int i = 0; i < N; ++i) evals[i] = A[(size_t)i * N + i];
            return sweep;
        }
        if (sweep == max_sweeps) break;
        for (int p = 0; p < N - 1; ++p)
            for (int q = p + 1; q < N; ++q) {
                double *rp = A + (size_t)p * N, *rq = A + (size_t)q * N;
                double apq = rp[q];
                if (apq == 0.0) continue;
                double app = rp[p], aqq = rq[q];
                /* tan of the rotation angle: root of t^2 + 2 theta t - 1 = 0
                 * of smaller magnitude, theta = (aqq - app) / (2 apq) */
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) /
                           (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < N; ++k) {
                    if (k == p || k == q) continue;
                    double apk = rp[k], aqk = rq[k];
                    double np_ = c * apk - s * aqk, nq_ = s * apk + c * aqk;
                    rp[k] = np_; rq[k] = nq_;
                    A[(size_t)k * N + p] = np_;
                    A[(size_t)k * N + q] = nq_;
                }
                rp[p] = app - t * apq;
                rq[q] = aqq + t * apq;
                rp[q] = 0.0;
                rq[p] = 0.0;
                double *vp = Vt + (size_t)p * N, *vq = Vt + (size_t)q * N;
                for (int k = 0; k < N; ++k) {
                    double a = vp[k], b = vq[k];
                    vp[k] = c * a - s * b;
                    vq[k] = s * a + c * b;
                }
            }
    }
    for (int i = 0; i < N; ++i) evals[i] = A[(size_t)i * N + i];
    return -1;
}

/* ------------------------------------------------------------------ */
/* Fermi-Dirac occupations, chemical potential, entropy (Eqs. 36-38)  */
/* ------------------------------------------------------------------ */

/* f(x) = 1/(exp(x)+1), evaluated without overflow. */
double orc_fermi(double x)
{
    if (x > 0) { double e = exp(-x); return e / (1.0 + e); }
    return 1.0 / (1.0 + exp(x));
}

/* Electron count 2 * sum_i f(beta (eps_i - mu)) (two electrons per orbital). */
static double count_electrons(int N, const double *ev, double beta, double mu)
{
    double s = 0.0;
    for (int i = 0; i < N; ++i) s += orc_fermi(beta * (ev[i] - mu));
    return 2.0 * s;
}

/* Chemical potential with 2 sum f_i = ne, by bisection on the strictly
 * increasing count (unique for beta < inf).  Writes f_i, returns mu. */
double orc_fermi_mu(int N, const double *ev, double beta, double ne,
                    double *f)
{
    double lo = ev[0], hi = ev[0];
    for (int i = 1; i < N; ++i) { if (ev[i] < lo) lo = ev[i]; if (ev[i] > hi) hi = ev[i]; }
    lo -= 50.0 / beta + 1.0;
    hi += 50.0 / beta + 1.0;
    for (int it = 0; it < 400; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        if (count_electrons(N, ev, beta, mid) < ne) lo = mid; else hi = mid;
    }
    double mu = 0.5 * (lo + hi);
    for (int i = 0; i < N; ++i) f[i] = orc_fermi(beta * (ev[i] - mu));
    return mu;
}

/* Per-orbital Fermi-Dirac entropy -f ln f - (1-f) ln(1-f), with 0 ln 0 = 0,
 * written through x = beta (eps - mu) as ln(1 + e^-|x|) + |x| / (1 + e^|x|). */
double orc_entropy_x(double x)
{
    double a = fabs(x);
    return log1p(exp(-a)) + a / (1.0 + exp(a));
}

/* Total entropy of the spin-paired system: S = 2 sum_i s(x_i) (Eq. 38, with
 * the factor two of D = 2 f). */
double orc_entropy(int N, const double *ev, double beta, double mu)
{
    double s = 0.0;
    for (int i = 0; i < N; ++i) s += orc_entropy_x(beta * (ev[i] - mu));
    return 2.0 * s;
}

/* D = 2 sum_k f_k v_k v_k^T, eigenvectors v_k are the rows of Vt. */
int orc_density(int N, const double *Vt, const double *f, double *D)
{
    if (N <= 0) return -1;
    #pragma omp parallel for schedule(dynamic, 8)
    for (int i = 0; i < N; ++i) {
        double *Di = D + (size_t)i * N;
        for (int j = 0; j < N; ++j) Di[j] = 0.0;
        for (int k = 0; k < N; ++k) {
            const double *vk = Vt + (size_t)k * N;
            double a = 2.0 * f[k] * vk[i];
            if (a == 0.0) continue;
            for (int j = 0; j < N; ++j) Di[j] += a * vk[j];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Canonical first-order response (Section V.B)                        */
/* ------------------------------------------------------------------ */

static double lncosh(double y)
{
    double a = fabs(y);
    return a + log1p(exp(-2.0 * a)) - M_LN2;
}

static double ln_sinhc(double d)   /* ln(sinh(d)/d) */
{
    double a = fabs(d);
    if (a < 1e-4) return log1p(a * a / 6.0);
    return a + log1p(-exp(-2.0 * a)) - M_LN2 - log(a);
}

/* Divided difference (f(x_a) - f(x_b)) / (eps_a - eps_b) of the occupation,
 * with x = beta (eps - mu); the limit a == b is the derivative
 * -beta f (1 - f).  Uses f_a - f_b = -sinh(d) / (2 cosh(x_a/2) cosh(x_b/2)),
 * d = (x_a - x_b)/2, which has no cancellation for close eigenvalues. */
double orc_fermi_divdiff(double xa, double xb, double beta)
{
    double d = 0.5 * (xa - xb);
    double l = log(0.25 * beta) + ln_sinhc(d) - lncosh(0.5 * xa) - lncosh(0.5 * xb);
    return -exp(l);
}

/* Diagonal of the canonical density-matrix response D' to the perturbation
 * H1 = diag(h) (h per orbital), at fixed electron number:
 *   D' = V [ Delta o (V^T H1 V - mu' I) ] V^T,   Delta_ij = 2 (f_i - f_j)/(e_i - e_j),
 *   mu' = sum_i Delta_ii (V^T H1 V)_ii / sum_i Delta_ii,
 * with the eigenvectors v_i as the rows of Vt.
 * Writes dd[p] = D'[p,p] and returns mu'. */
/* F[i*N + j] = orc_fermi_divdiff(x[i], x[j], beta) for all pairs */
void orc_fermi_divdiff_matrix(int N, const double *x, double beta, double *F)
{
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j)
            F[(size_t)i * N + j] = orc_fermi_divdiff(x[i], x[j], beta);
}

double orc_response_diag(int N, const double *Vt, const double *ev,
                         double beta, double mu, const double *h, double *dd)
{
    double *M = (double *)malloc(sizeof(double) * (size_t)N * N);
    double *T = (double *)calloc((size_t)N * N, sizeof(double));
    double *x = (double *)malloc(sizeof(double) * (size_t)N);
    for (int i = 0; i < N; ++i) x[i] = beta * (ev[i] - mu);
    /* H1' = V^T diag(h) V, element (i,j) = sum_k v_i[k] h[k] v_j[k] */
    #pragma omp parallel for schedule(dynamic, 8)
    for (int i = 0; i < N; ++i) {
        const double *vi = Vt + (size_t)i * N;
        for (int j = i; j < N; ++j) {
            const double *vj = Vt + (size_t)j * N;
            double s = 0.0;
            for (int k = 0; k < N; ++k) s += vi[k] * h[k] * vj[k];
            M[(size_t)i * N + j] = s;
            M[(size_t)j * N + i] = s;
        }
    }
    double num = 0.0, den = 0.0;
    for (int i = 0; i < N; ++i) {
        double dii = 2.0 * orc_fermi_divdiff(x[i], x[i], beta);
        num += dii * M[(size_t)i * N + i];
        den += dii;
    }
    double mup = (den != 0.0) ? num / den : 0.0;
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            double dij = 2.0 * orc_fermi_divdiff(x[i], x[j], beta);
            M[(size_t)i * N + j] = dij * (M[(size_t)i * N + j] - (i == j ? mup : 0.0));
        }
    /* T = M Vt, then D'[p,p] = sum_i Vt[i,p] T[i,p] */
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < N; ++i) {
        double *Ti = T + (size_t)i * N;
        for (int j = 0; j < N; ++j) {
            double a = M[(size_t)i * N + j];
            const double *vj = Vt + (size_t)j * N;
            for (int p = 0; p < N; ++p) Ti[p] += a * vj[p];
        }
    }
    for (int p = 0; p < N; ++p) dd[p] = 0.0;
    for (int i = 0; i < N; ++i)
        for (int p = 0; p < N; ++p) dd[p] += Vt[(size_t)i * N + p] * T[(size_t)i * N + p];
    free(M); free(T); free(x);
    return mup;
}
