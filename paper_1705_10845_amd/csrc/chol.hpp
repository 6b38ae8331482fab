// FP64 log-determinant of a symmetric positive definite matrix by a blocked
// right-looking Cholesky factorisation.  Used only for the electronic
// entropy, where every matrix factorised (I + T0, I + 4 Z_k^2) has its
// spectrum in [1/2, 2], so no pivoting is needed.
//
// Outer panels of NB = 128 columns.  Inside a panel, inner panels of CB = 32
// columns: one kernel factors the 32 x 32 diagonal block in LDS and solves
// every row below it; a small kernel applies the inner panel to the rest of
// the outer panel's columns.  The rank-128 update of the trailing matrix,
// which holds nearly all the flops, runs on the FP64 MFMA product kernel
// (C = C - P^T P with P the transposed panel, symmetric output).
#pragma once
#include "common.hpp"
#include "gemm.hpp"

namespace xl {

constexpr int CB = 32;    // inner panel width
constexpr int NB = 128;   // outer panel width

// Factor the CB x CB diagonal block at (q, q) in LDS (lower), then solve
// the rows below it: L_iq = A_iq L_qq^-T, one thread per row.  Every block
// factors the diagonal block itself; block 0 writes it back and adds
// 2 sum ln L_ii to *acc.  One wavefront per block (CHOL_PT threads), so the
// 3 CB barriers of the factorisation are single-wave barriers.
constexpr int CHOL_PT = 64;
__global__ __launch_bounds__(CHOL_PT) void chol_panel_kernel(int n, int ld, int q, double *A,
                                                             double *acc) {
    __shared__ double L[CB][CB + 1];
    for (int t = threadIdx.x; t < CB * CB; t += blockDim.x)
        L[t / CB][t % CB] = A[(long)(q + t / CB) * ld + q + t % CB];
    __syncthreads();
    for (int k = 0; k < CB; ++k) {
        const double d = sqrt(L[k][k]);
        __syncthreads();                       // every thread has read L_kk
        if (threadIdx.x == 0) L[k][k] = d;
        if (threadIdx.x > k && threadIdx.x < CB) L[threadIdx.x][k] /= d;
        __syncthreads();
        for (int t = threadIdx.x; t < CB * CB; t += blockDim.x) {
            const int i = t / CB, j = t % CB;
            if (j > k && j <= i) L[i][j] -= L[i][k] * L[j][k];
        }
        __syncthreads();
    }
    if (blockIdx.x == 0) {
        for (int t = threadIdx.x; t < CB * CB; t += blockDim.x) {
            const int i = t / CB, j = t % CB;
            A[(long)(q + i) * ld + q + j] = (j <= i) ? L[i][j] : 0.0;
        }
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int k = 0; k < CB; ++k) s += log(L[k][k]);
            acc[0] += 2.0 * s;
        }
    }
    const int i = q + CB + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x[CB];
    double *row = A + (long)i * ld + q;
    for (int k = 0; k < CB; ++k) {
        double s = row[k];
        for (int t = 0; t < k; ++t) s -= x[t] * L[k][t];
        x[k] = s / L[k][k];
    }
    for (int k = 0; k < CB; ++k) row[k] = x[k];
}

// Apply the inner panel (columns q .. q + CB) to the columns
// [q + CB, jend) of the outer panel: A_ij -= sum_k L_ik L_jk for i >= j,
// 64 x 64 tiles, 256 threads (4 x 4 per thread).
__global__ __launch_bounds__(256) void chol_update_kernel(int n, int ld, int q, int jend,
                                                          double *A) {
    const int tj = blockIdx.x, ti = blockIdx.y;
    const int base = q + CB;
    const int i0 = base + ti * 64, j0 = base + tj * 64;
    if (j0 >= i0 + 64) return;               // strictly upper tile
    __shared__ double Li[64][CB + 1], Lj[64][CB + 1];
    for (int t = threadIdx.x; t < 64 * CB; t += 256) {
        const int r = t / CB, k = t % CB;
        Li[r][k] = (i0 + r < n) ? A[(long)(i0 + r) * ld + q + k] : 0.0;
        Lj[r][k] = (j0 + r < jend) ? A[(long)(j0 + r) * ld + q + k] : 0.0;
    }
    __syncthreads();
    const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;
    double s[4][4] = {};
    for (int k = 0; k < CB; ++k)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) s[a][b] += Li[tr + 16 * a][k] * Lj[tc + 16 * b][k];
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            const int i = i0 + tr + 16 * a, j = j0 + tc + 16 * b;
            if (i < n && j < jend && j <= i) A[(long)i * ld + j] -= s[a][b];
        }
}

// P[k][i] = A[(r0 + i) ld + c0 + k] for k < NB, i < m (P has leading
// dimension m): the panel rows below the outer diagonal block, transposed
// so the product kernel reads them as k-rows.
__global__ __launch_bounds__(256) void chol_transpose_kernel(int m, int ld, int r0, int c0,
                                                             const double *A, double *P) {
    __shared__ double t[32][33];
    const int i0 = blockIdx.x * 32, k0 = blockIdx.y * 32;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;   // 32 x 8
    for (int r = ty; r < 32; r += 8)
        t[r][tx] = (i0 + r < m) ? A[(long)(r0 + i0 + r) * ld + c0 + k0 + tx] : 0.0;
    __syncthreads();
    for (int r = ty; r < 32; r += 8)
        if (i0 + tx < m) P[(long)(k0 + r) * m + i0 + tx] = t[tx][r];
}

// ln det of the n x n matrix A (destroyed; only its lower triangle is
// read), n % NB == 0; P is an NB x n workspace, ws (ws_elems doubles) the
// split-k workspace of the product kernel.  The result is written to *out
// (device).
inline void chol_logdet(int n, int ld, double *A, double *P, double *ws, long ws_elems,
                        double *out, hipStream_t st) {
    if (n % NB) throw InvalidArg("chol_logdet: n must be a multiple of 128");
    XL_HIP(hipMemsetAsync(out, 0, sizeof(double), st));
    for (int p = 0; p < n; p += NB) {
        const int pe = p + NB;
        for (int q = p; q < pe; q += CB) {
            const int rest = n - q - CB;
            hipLaunchKernelGGL(chol_panel_kernel, dim3(std::max(1, ceil_div(rest, CHOL_PT))),
                               dim3(CHOL_PT), 0, st, n, ld, q, A, out);
            XL_LAUNCH_CHECK();
            if (q + CB < pe) {
                hipLaunchKernelGGL(chol_update_kernel,
                                   dim3(ceil_div(pe - q - CB, 64), ceil_div(rest, 64)), dim3(256),
                                   0, st, n, ld, q, pe, A);
                XL_LAUNCH_CHECK();
            }
        }
        const int m = n - pe;
        if (m <= 0) break;
        hipLaunchKernelGGL(chol_transpose_kernel, dim3(ceil_div(m, 32), NB / 32), dim3(256), 0,
                           st, m, ld, pe, p, A, P);
        XL_LAUNCH_CHECK();
        GemmArgs<double> g;                    // A22 <- A22 - L21 L21^T
        g.n = m; g.ld = ld; g.k = NB; g.lda = m;
        g.A0 = P; g.B0 = P;
        g.C = A + (long)pe * ld + pe; g.X = g.C;
        g.alpha = -1.0; g.beta = 1.0;
        g.ws = ws; g.ws_elems = ws_elems;
        gemm(g, true, st);
    }
}

}  // namespace xl
