// Device-side decisions of a planned XL-BOMD step.
//
// A planned step enqueues a fixed sequence of launches: the level count of
// the expansion and the Newton-Schulz schedule of every level come from a
// plan made on the host from an earlier spectral interval widened by a
// margin, and every decision that depends on the step's own numbers is
// taken here, on the device, so that the step needs no host
// synchronisation and can be captured into a HIP graph and replayed:
//   - the spectral interval (Gershgorin tightened by the Lanczos
//     coefficients) and the predicted chemical potential, checked against
//     the plan;
//   - whether the expansion is rerun at the corrected chemical potential
//     (a second expansion into separate buffers whose product launches
//     skip themselves when it is not needed, adopted only when it ran);
//   - the second-order correction of D at the final chemical potential;
//   - the rank of the sequential Krylov kernel (residual floor, breakdown
//     of a direction);
//   - divergence.
// A step whose numbers leave the plan (interval beyond the plan's,
// chemical potential not converged after one rerun, non-finite values)
// raises a flag; the host then restores the state saved at the start of
// the step and repeats it with host decisions.
#pragma once
#include "common.hpp"

namespace xl {

// doubles of the planned step's device block
enum PsIdx : int {
    PS_MU0 = 0,    // chemical potential of the first expansion
    PS_MU1 = 1,    // of the second (rerun) expansion
    PS_MU = 2,     // final mu = expansion mu + dmu
    PS_MUP = 3,    // mu(t - dt)
    PS_MUPP = 4,   // mu(t - 2 dt)
    PS_ELO = 5, PS_EHI = 6, PS_XMAX = 7,
    PS_MLO = 8, PS_MHI = 9,   // bracket of mu: N(mlo) < N_e < N(mhi)
    PS_DMU = 10,   // correction applied to D
    PS_RMS = 11, PS_SUMQ = 12,
    PS_NRM = 16,   // 2 norms per Krylov direction (raw, orthogonalised)
    PS_ST2 = 48,   // N0, N', dmu, N'' of the second expansion
    PS_COUNT = 64
};
// ints of the planned step's device block
enum PiIdx : int {
    PI_FLAGS = 0,   // bit set: the step left the plan (FLAG_*)
    PI_SKIP2 = 1,   // 1: no rerun (the second expansion's products skip)
    PI_RANK = 2,    // rank of the kernel built in the step
    PI_MUKNOWN = 3, // entries of the mu history (0..2)
    PI_RERUN = 4,   // 1 if the expansion was rerun
    PI_COUNT = 16
};
constexpr int FLAG_INTERVAL = 1;   // spectrum beyond the plan's interval
constexpr int FLAG_SPARSE = 2;     // sparse seed planned but no longer valid
constexpr int FLAG_MU = 4;         // mu not within the threshold after one rerun
constexpr int FLAG_DIVERGED = 8;   // non-finite value or residual above 1e3

// Smallest and largest eigenvalue of the symmetric tridiagonal matrix
// (diagonal a[0..m), off-diagonal b[0..m-1)) by Sturm-count bisection.
__device__ inline void tridiag_extremes_dev(const double *a, const double *b, int m, double &lo,
                                            double &hi) {
    double gl = 1e300, gh = -1e300;
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < m ? fabs(b[i]) : 0.0);
        gl = fmin(gl, a[i] - r);
        gh = fmax(gh, a[i] + r);
    }
    for (int side = 0; side < 2; ++side) {
        const int k = side == 0 ? 0 : m - 1;   // k-th smallest eigenvalue
        double l = gl, h = gh;
        for (int it = 0; it < 200 && h - l > 1e-13 * (fabs(l) + fabs(h) + 1e-300); ++it) {
            const double x = 0.5 * (l + h);
            int below = 0;
            double q = 1.0;
            for (int i = 0; i < m; ++i) {
                q = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / q : 0.0);
                if (q == 0.0) q = -1e-300;
                if (q < 0.0) ++below;
            }
            if (below > k) h = x; else l = x;
        }
        if (side == 0) lo = 0.5 * (l + h); else hi = 0.5 * (l + h);
    }
}

// The step's spectral interval, the predicted chemical potential and the
// check against the plan (one thread).  gersh = {min lo, max hi, largest
// neighbour count}; ab = Lanczos alpha[0..m) then beta[0..m).
__global__ void plan_interval_kernel(const double *gersh, const double *ab, int m, int nat,
                                     double beta, double xmax_plan, int sparse_plan,
                                     int nb_max_limit, double *ps, int *pi) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double elo = gersh[0], ehi = gersh[1];
    const int nbm = (int)gersh[2];
    const double *a = ab, *b = ab + m;
    bool ok = true;
    for (int j = 0; j < m; ++j)
        if (!isfinite(a[j]) || !isfinite(b[j]) || !(b[j] > 1e-12 * (fabs(ehi) + fabs(elo))))
            ok = false;
    if (ok) {
        double tlo, thi;
        tridiag_extremes_dev(a, b, m, tlo, thi);
        const double bm = b[m - 1];
        elo = fmax(elo, tlo - bm);
        ehi = fmin(ehi, thi + bm);
    }
    int flags = 0;
    if (!isfinite(elo) || !isfinite(ehi)) flags |= FLAG_DIVERGED;
    const int known = pi[PI_MUKNOWN];
    double mu0 = known >= 2 ? 2.0 * ps[PS_MUP] - ps[PS_MUPP] : ps[PS_MUP];
    const double mlo = elo - 40.0 / beta, mhi = ehi + 40.0 / beta;
    mu0 = fmin(fmax(mu0, mlo), mhi);
    const double xmax = beta * fmax(fabs(elo - mu0), fabs(ehi - mu0)) * 1.02 + 1e-12;
    if (!(xmax <= xmax_plan)) flags |= FLAG_INTERVAL;
    if (sparse_plan && !(nbm > 0 && nbm <= nb_max_limit && 4 * nbm <= nat)) flags |= FLAG_SPARSE;
    ps[PS_MU0] = mu0;
    ps[PS_ELO] = elo;
    ps[PS_EHI] = ehi;
    ps[PS_XMAX] = xmax;
    ps[PS_MLO] = mlo;
    ps[PS_MHI] = mhi;
    pi[PI_FLAGS] = flags;
}

// After the first expansion (st1 = {N0, N', dmu, N''} at mu0): accept, or
// choose the chemical potential of one rerun (the model step inside the
// bracket, else its midpoint).  One thread.
__global__ void plan_mu_kernel(const double *st1, double beta, double ne, double tau,
                               double *ps, int *pi) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double N0 = st1[0], dmu = st1[2], mu0 = ps[PS_MU0];
    double mlo = ps[PS_MLO], mhi = ps[PS_MHI];
    if (!isfinite(N0)) pi[PI_FLAGS] |= FLAG_DIVERGED;
    if (N0 < ne) mlo = fmax(mlo, mu0); else mhi = fmin(mhi, mu0);
    if (isfinite(dmu) && beta * fabs(dmu) <= tau) {
        pi[PI_SKIP2] = 1;
        pi[PI_RERUN] = 0;
        ps[PS_MU1] = mu0;
    } else {
        double next = mu0 + (isfinite(dmu) ? dmu : 0.0);
        if (!(next > mlo && next < mhi) || !isfinite(dmu)) next = 0.5 * (mlo + mhi);
        pi[PI_SKIP2] = 0;
        pi[PI_RERUN] = 1;
        ps[PS_MU1] = next;
    }
    ps[PS_MLO] = mlo;
    ps[PS_MHI] = mhi;
}

// After the (possibly skipped) second expansion: the correction dmu of D
// and the final chemical potential.  One thread.
__global__ void plan_mu2_kernel(const double *st1, const double *st2, double beta, double tau,
                                double *ps, int *pi) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double dmu, mu_e;
    if (pi[PI_RERUN]) {
        dmu = st2[2];
        mu_e = ps[PS_MU1];
        if (!(isfinite(dmu) && beta * fabs(dmu) <= tau)) pi[PI_FLAGS] |= FLAG_MU;
        if (!isfinite(st2[0])) pi[PI_FLAGS] |= FLAG_DIVERGED;
    } else {
        dmu = st1[2];
        mu_e = ps[PS_MU0];
    }
    if (!isfinite(dmu)) dmu = 0.0;
    ps[PS_DMU] = dmu;
    ps[PS_MU] = mu_e + dmu;
}

// The copies of a table of (source, destination, 8-byte words) triples,
// one per blockIdx.y, unless *skip is set; grid.x blocks stride the words.
__global__ __launch_bounds__(256) void pred_copy_table_kernel(const int *skip, const long *tab) {
    if (*skip) return;
    const long *e = tab + 3 * (long)blockIdx.y;
    const unsigned long long *src = reinterpret_cast<const unsigned long long *>(e[0]);
    unsigned long long *dst = reinterpret_cast<unsigned long long *>(e[1]);
    const long n8 = e[2];
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n8;
         i += (long)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// D(mu_e + d) = (1 + bd/2) I + (-2 + bd^2/2) Z + (-2 bd) Z^2 + (-2 bd^2) Z Z^2,
// bd = beta d, d = ps[PS_DMU] (second order in d); P = Z Z^2.  The
// padding rows and columns of D are zero.
template <typename T>
__global__ __launch_bounds__(256) void density_combine_kernel(int n, int ld, const T *Z,
                                                              const T *Z2, const T *P,
                                                              const double *ps, double beta,
                                                              T *D) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)ld * ld) return;
    const int i = (int)(t / ld), j = (int)(t % ld);
    double v = 0.0;
    if (i < n && j < n) {
        const double bd = beta * ps[PS_DMU];
        v = (-2.0 + 0.5 * bd * bd) * (double)Z[t] - 2.0 * bd * (double)Z2[t] -
            2.0 * bd * bd * (double)P[t];
        if (i == j) v += 1.0 + 0.5 * bd;
    }
    D[t] = (T)v;
}

// Rank of the sequential Krylov kernel built in the step from the norms
// {raw, orthogonalised} of its directions: 0 if the first direction is zero
// or its residual's RMS is at or below the floor, else the number of
// directions before the first whose orthogonalised norm is at or below
// 1e-10 of its raw norm.  One thread.
__global__ void plan_rank_kernel(const double *nrm, int m, double gamma, int nat, double floor_rms,
                                 int *pi) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int rank = 0;
    if (m > 0 && nrm[1] > 0.0 && nrm[0] / (gamma * sqrt((double)nat)) > floor_rms) {
        rank = 1;
        while (rank < m && nrm[2 * rank + 1] > 1e-10 * nrm[2 * rank]) ++rank;
    }
    pi[PI_RANK] = rank;
}

// n(t+dt) by Eq. 23 into row 0 of a history kept in order (row k holds
// n(t - k dt)), the older rows shifted down by one; one thread per atom.
__global__ __launch_bounds__(256) void verlet_shift_kernel(int nat, int kmax, double kappa,
                                                           double alpha, const double *cvec,
                                                           const double *kr, double *hist) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nat) return;
    double val = 2.0 * hist[i] - hist[(long)nat + i] - kappa * kr[i];
    double d = 0.0;
    for (int k = 0; k <= kmax; ++k) d += cvec[k] * hist[(long)k * nat + i];
    val += alpha * d;
    for (int k = kmax; k >= 1; --k) hist[(long)k * nat + i] = hist[(long)(k - 1) * nat + i];
    hist[i] = val;
}

// Residual RMS, divergence check and the chemical-potential history after
// the charges (chg = {sum r^2, sum q}).  One thread.
__global__ void plan_finish_kernel(const double *chg, int nat, double *ps, int *pi) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double rms = sqrt(chg[0] / nat);
    ps[PS_RMS] = rms;
    ps[PS_SUMQ] = chg[1];
    if (!isfinite(rms) || rms > 1e3) pi[PI_FLAGS] |= FLAG_DIVERGED;
    ps[PS_MUPP] = ps[PS_MUP];
    ps[PS_MUP] = ps[PS_MU];
    pi[PI_MUKNOWN] = min(pi[PI_MUKNOWN] + 1, 2);
}

}  // namespace xl
