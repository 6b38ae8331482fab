// Non-orthogonal basis (the SCC-DFTB setting of Section VI: non-orthogonal
// atomic orbitals, Mulliken charges, Pulay forces), on the synthetic model:
//   S[Ia,Ib] = delta_ab,  S[Ia,Jb] = Bs_ab exp(-r/decay_s) s(r)  (I != J),
//   H[n] = H0 + (S V + V S)/2,  V = diag(Gamma n) on each atom's orbitals,
// solved through the Loewdin factor X = S^-1/2: the expansion runs on
// H' = X H X, D = X D' X, q_I = sum_a (D S)[Ia,Ia] - Z_I, and the forces
// gain -Tr[M dS/dR] with M = (V D + D V)/2 - E, E the energy-weighted
// density matrix X (D' H') X.  Dense FP64 kernels around the FP64 products.
#pragma once
#include "model.hpp"

namespace xl {

// S and H = H0 + (S V + V S)/2 over the padded array: the padding of S is
// the identity (its inverse square root stays a decoupled identity block),
// the padding of H zero.  Grid (ld / 256, ld), one thread per entry.
__global__ __launch_bounds__(256) void overlap_hamiltonian_kernel(ModelDev m, const double *v,
                                                                  double *S, double *H) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= m.ld) return;
    double sv = (i == j) ? 1.0 : 0.0, hv = 0.0;
    if (i < m.n && j < m.n) {
        const int I = i / m.no, a = i % m.no, J = j / m.no, b = j % m.no;
        if (I == J) {
            if (a == b) hv = m.onsite[a] + (m.jit ? m.jit[i] : 0.0) + v[I];
        } else {
            double dx, dy, dz;
            const double r = pair_dist(m.pos, I, J, dx, dy, dz);
            if (r < m.rc) {
                double s, ds;
                taper(r, m.rc, m.width, s, ds);
                sv = m.sblk[a * m.no + b] * exp(-r / m.sdecay) * s;
                hv = m.hop[a * m.no + b] * exp(-r / m.decay) * s + 0.5 * sv * (v[I] + v[J]);
            }
        }
    }
    const long o = (long)i * m.ld + j;
    S[o] = sv;
    H[o] = hv;
}

// Gershgorin interval of each row of a dense symmetric matrix (real block):
// [A_ii - R_i, A_ii + R_i], R_i = sum_{j != i} |A_ij|.  One wave per row.
__global__ __launch_bounds__(256) void dense_gershgorin_kernel(int n, int ld, const double *A,
                                                               double *lo, double *hi) {
    const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (i >= n) return;
    const double *row = A + (long)i * ld;
    double s = 0.0;
    for (int j = lane; j < n; j += 64)
        if (j != i) s += fabs(row[j]);
    s = wave_sum(s);
    if (lane == 0) {
        lo[i] = row[i] - s;
        hi[i] = row[i] + s;
    }
}

// Y = sc (A - mu I) over the real block, zero in the padding.
__global__ __launch_bounds__(256) void seed_dense_kernel(int n, int ld, const double *A,
                                                         double mu, double sc, double *Y) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= ld) return;
    const long o = (long)i * ld + j;
    double val = 0.0;
    if (i < n && j < n) val = sc * (A[o] - (i == j ? mu : 0.0));
    Y[o] = val;
}

// out[i] = sum_j (T_ij - delta_ij)^2 over all ld columns of row i < ld.
// One wave per row.
__global__ __launch_bounds__(256) void row_dev_identity_kernel(int ld, const double *T,
                                                               double *out) {
    const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (i >= ld) return;
    const double *row = T + (long)i * ld;
    double s = 0.0;
    for (int j = lane; j < ld; j += 64) {
        const double e = row[j] - (i == j ? 1.0 : 0.0);
        s += e * e;
    }
    s = wave_sum(s);
    if (lane == 0) out[i] = s;
}

// out[0] = max_i x[i] (one block).
__global__ __launch_bounds__(1024) void max_kernel(int n, const double *x, double *out) {
    __shared__ double sh[1024];
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) a = fmax(a, x[i]);
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// Mulliken populations per orbital: pop[i] = (D S)_ii = sum_j D_ij S_ij
// (S symmetric).  One wave per row of the real block.
__global__ __launch_bounds__(256) void mulliken_rows_kernel(int n, int ld, const double *D,
                                                            const double *S, double *pop) {
    const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (i >= n) return;
    const double *a = D + (long)i * ld, *b = S + (long)i * ld;
    double s = 0.0;
    for (int j = lane; j < n; j += 64) s += a[j] * b[j];
    s = wave_sum(s);
    if (lane == 0) pop[i] = s;
}

// q_I = sum_a pop[Ia] - zc;  r = q - n;  out[0] = sum r^2, out[1] = sum q.
__global__ __launch_bounds__(1024) void charges_pop_kernel(int nat, int no, const double *pop,
                                                           double zc, const double *nvec,
                                                           double *q, double *r, double *out) {
    __shared__ double sh[16];
    double s2 = 0.0, sq = 0.0;
    for (int I = threadIdx.x; I < nat; I += blockDim.x) {
        double p = 0.0;
        for (int a = 0; a < no; ++a) p += pop[I * no + a];
        const double qi = p - zc;
        q[I] = qi;
        const double ri = qi - nvec[I];
        r[I] = ri;
        s2 += ri * ri;
        sq += qi;
    }
    s2 = block_sum(s2, sh);
    sq = block_sum(sq, sh);
    if (threadIdx.x == 0) {
        out[0] = s2;
        out[1] = sq;
    }
}

// out[i] = sum over the nchunk row chunks of part[c * n + i] (the partial
// column sums of coldot_kernel).
__global__ __launch_bounds__(256) void chunk_sum_kernel(int n, int nchunk, const double *part,
                                                        double *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += part[(long)c * n + i];
    out[i] = s;
}

// Overlap part of the forces, added to F:
//   F_I -= 2 sum_{J != I} sum_ab M[Ia,Jb] dS[Ia,Jb]/dr (R_I - R_J)/r,
//   M = D (v_I + v_J)/2 - E
// (both blocks (Ia,Jb) and (Jb,Ia) of the symmetric M and S).  One wave
// per atom.
__global__ __launch_bounds__(256) void overlap_forces_kernel(ModelDev m, const double *D,
                                                             const double *E, const double *v,
                                                             double *F) {
    const int I = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (I >= m.nat) return;
    const int no = m.no;
    double fx = 0, fy = 0, fz = 0;
    for (int J = lane; J < m.nat; J += 64) {
        if (J == I) continue;
        double dx, dy, dz;
        const double r = pair_dist(m.pos, I, J, dx, dy, dz);
        if (r >= m.rc) continue;
        double s, ds;
        taper(r, m.rc, m.width, s, ds);
        const double dsr = exp(-r / m.sdecay) * (ds - s / m.sdecay);
        const double vh = 0.5 * (v[I] + v[J]);
        double acc = 0.0;
        for (int a = 0; a < no; ++a) {
            const long row = (long)(I * no + a) * m.ld + J * no;
            for (int b = 0; b < no; ++b)
                acc += m.sblk[a * no + b] * (D[row + b] * vh - E[row + b]);
        }
        const double g = 2.0 * dsr * acc;
        fx -= g * dx / r;
        fy -= g * dy / r;
        fz -= g * dz / r;
    }
    fx = wave_sum(fx);
    fy = wave_sum(fy);
    fz = wave_sum(fz);
    if (lane == 0) {
        F[3 * I] += fx;
        F[3 * I + 1] += fy;
        F[3 * I + 2] += fz;
    }
}

// A = I over the padded array.
__global__ __launch_bounds__(256) void identity_kernel(long ld, double *A) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ld * ld) return;
    A[t] = (t / ld == t % ld) ? 1.0 : 0.0;
}

}  // namespace xl
