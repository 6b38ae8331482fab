// FP64 log-determinant of a symmetric positive definite matrix by a blocked
// right-looking Cholesky factorisation.  Used only for the electronic
// entropy, where every matrix factorised (I + T0, I + 4 Z_k^2) has its
// spectrum in [1/2, 2], so no pivoting is needed.
#pragma once
#include "common.hpp"

namespace xl {

constexpr int CB = 32;   // panel width

// Factor the CB x CB diagonal block at (p, p) in place (lower), add
// 2 sum ln L_ii to *acc.  One block of CB*CB threads.
__global__ __launch_bounds__(1024) void chol_diag_kernel(int ld, int p,
                                                         double *A, double *acc) {
    __shared__ double L[CB][CB + 1];
    const int tx = threadIdx.x % CB, ty = threadIdx.x / CB;
    L[ty][tx] = A[(long)(p + ty) * ld + p + tx];
    __syncthreads();
    for (int k = 0; k < CB; ++k) {
        if (ty == 0 && tx == 0) L[k][k] = sqrt(L[k][k]);
        __syncthreads();
        if (ty == 0 && tx > k) L[tx][k] /= L[k][k];
        __syncthreads();
        if (ty > k && tx > k && tx <= ty) L[ty][tx] -= L[ty][k] * L[tx][k];
        __syncthreads();
    }
    A[(long)(p + ty) * ld + p + tx] = (tx <= ty) ? L[ty][tx] : 0.0;
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < CB; ++k) s += log(L[k][k]);
        acc[0] += 2.0 * s;
    }
}

// Rows below the diagonal block: L_ip = A_ip L_pp^-T (forward substitution
// per row).  One thread per row, L_pp in LDS.
__global__ __launch_bounds__(256) void chol_panel_kernel(int n, int ld, int p,
                                                         double *A) {
    __shared__ double L[CB][CB + 1];
    for (int t = threadIdx.x; t < CB * CB; t += blockDim.x)
        L[t / CB][t % CB] = A[(long)(p + t / CB) * ld + p + t % CB];
    __syncthreads();
    const int i = p + CB + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x[CB];
    double *row = A + (long)i * ld + p;
    for (int k = 0; k < CB; ++k) {
        double s = row[k];
        for (int t = 0; t < k; ++t) s -= x[t] * L[k][t];
        x[k] = s / L[k][k];
    }
    for (int k = 0; k < CB; ++k) row[k] = x[k];
}

// Trailing update A_ij -= sum_k L_ik L_jk over the panel columns, lower
// triangle only, 64 x 64 output tiles, 256 threads (4 x 4 per thread).
__global__ __launch_bounds__(256) void chol_update_kernel(int n, int ld, int p,
                                                          double *A) {
    const int tj = blockIdx.x, ti = blockIdx.y;
    if (tj > ti) return;
    const int base = p + CB;
    const int i0 = base + ti * 64, j0 = base + tj * 64;
    __shared__ double Li[64][CB + 1], Lj[64][CB + 1];
    for (int t = threadIdx.x; t < 64 * CB; t += 256) {
        const int r = t / CB, k = t % CB;
        Li[r][k] = (i0 + r < n) ? A[(long)(i0 + r) * ld + p + k] : 0.0;
        Lj[r][k] = (j0 + r < n) ? A[(long)(j0 + r) * ld + p + k] : 0.0;
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
            if (i < n && j < n && j <= i) A[(long)i * ld + j] -= s[a][b];
        }
}

// ln det of the leading n x n block of A (destroyed); n % CB == 0 is padded
// by the caller with identity rows if needed.  Result written to *out
// (device) as the accumulation starting from 0.
inline void chol_logdet(int n, int ld, double *A, double *out, hipStream_t st) {
    if (n % CB) throw InvalidArg("chol_logdet: n must be a multiple of 32");
    XL_HIP(hipMemsetAsync(out, 0, sizeof(double), st));
    for (int p = 0; p < n; p += CB) {
        hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(CB * CB), 0, st, ld, p, A, out);
        XL_LAUNCH_CHECK();
        const int rest = n - p - CB;
        if (rest <= 0) break;
        hipLaunchKernelGGL(chol_panel_kernel, dim3(ceil_div(rest, 256)), dim3(256), 0, st,
                           n, ld, p, A);
        XL_LAUNCH_CHECK();
        const int nt = ceil_div(rest, 64);
        hipLaunchKernelGGL(chol_update_kernel, dim3(nt, nt), dim3(256), 0, st, n, ld, p, A);
        XL_LAUNCH_CHECK();
    }
}

}  // namespace xl
