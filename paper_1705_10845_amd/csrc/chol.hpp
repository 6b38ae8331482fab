// FP64 log-determinants of a batch of symmetric positive definite matrices by
// a blocked right-looking Cholesky factorisation (the batch index is the
// last grid dimension of every launch).  Used only for the electronic
// entropy, where every matrix factorised (I + T0, I + 4 Z_k^2) has its
// spectrum in [1/2, 2], so no pivoting is needed; the L + 1 factorisations
// of one evaluation are independent and run as one batch, which divides the
// number of latency-bound panel launches by L + 1.
//
// Outer panels of NB = 128 columns.  Inside a panel, inner panels of CB = 32
// columns, one kernel launch each: it applies the panel's earlier inner
// panels (left-looking), factors the 32 x 32 diagonal block in registers and
// solves every row below it.  The rank-128 update of the trailing matrix,
// which holds nearly all the flops, runs on the FP64 MFMA product kernel
// (C = C - P^T P with P the transposed panel, symmetric output).
#pragma once
#include "common.hpp"
#include "gemm.hpp"

namespace xl {

constexpr int CB = 32;    // inner panel width
constexpr int NB = 128;   // outer panel width

// lane value of a double held by lane `src` (a constant), broadcast
__device__ __forceinline__ double lane_bcast(double v, int src) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// Inner panel q (columns q .. q + CB) of the outer panel that starts at p,
// left-looking over the outer panel's earlier inner panels (columns
// p .. q, already final): one wavefront per block.
//  1. the diagonal block A_qq - L_q,[p,q) L_q,[p,q)^T, row i in the
//     registers of lane i, is factored in registers (pivot and column
//     entries broadcast from their lanes);
//  2. every row i below is updated the same way and solved against the
//     factor: L_iq = (A_iq - L_i,[p,q) L_q,[p,q)^T) L_qq^-T.
// Every block factors the diagonal block itself from the original entries,
// so none of them may be overwritten during the launch: the factored block
// stays in LDS only (no later step reads it: inner panels further right
// read only rows below it, the trailing update only rows below the outer
// panel).  Block 0 adds 2 sum ln L_ii to *acc.
constexpr int CHOL_PT = 64;
__global__ __launch_bounds__(CHOL_PT) void chol_panel_kernel(int n, int ld, int p, int q,
                                                             double *A, long sA, double *acc) {
    __shared__ double Lp[CB][NB - CB + 1];   // L[q + j][p + k], k < q - p
    A += blockIdx.y * sA;                    // matrix of the batch
    acc += blockIdx.y;
    __shared__ double Ld[CB][CB + 1];        // factored diagonal block
    const int w = q - p, lane = threadIdx.x;
    // w is a multiple of CB: eight independent loads in flight per thread
#pragma unroll 8
    for (int t = lane; t < CB * w; t += CHOL_PT)
        Lp[t / w][t % w] = A[(long)(q + t / w) * ld + p + t % w];
    __syncthreads();
    double row[CB];
    const int ri = lane < CB ? lane : CB - 1;   // lanes >= CB shadow the last row
#pragma unroll
    for (int j = 0; j < CB; ++j) row[j] = A[(long)(q + ri) * ld + q + j];
    for (int k = 0; k < w; ++k) {
        const double lik = Lp[ri][k];
#pragma unroll
        for (int j = 0; j < CB; ++j) row[j] -= lik * Lp[j][k];
    }
#pragma unroll
    for (int k = 0; k < CB; ++k) {
        const double d = sqrt(lane_bcast(row[k], k));
        row[k] = (lane == k) ? d : row[k] / d;         // L_ik for i > k
#pragma unroll
        for (int j = k + 1; j < CB; ++j) {
            const double ljk = lane_bcast(row[k], j);
            if (lane > k) row[j] -= row[k] * ljk;
        }
    }
    if (lane < CB) {
#pragma unroll
        for (int j = 0; j < CB; ++j) Ld[lane][j] = (j <= lane) ? row[j] : 0.0;
    }
    __syncthreads();
    if (blockIdx.x == 0 && lane == 0) {
        double s = 0.0;
        for (int k = 0; k < CB; ++k) s += log(Ld[k][k]);
        acc[0] += 2.0 * s;
    }
    const int i = q + CB + blockIdx.x * CHOL_PT + lane;
    if (i >= n) return;
    double x[CB];
    double *rowp = A + (long)i * ld;
#pragma unroll
    for (int j = 0; j < CB; ++j) x[j] = rowp[q + j];
#pragma unroll 8
    for (int k = 0; k < w; ++k) {
        const double lik = rowp[p + k];
#pragma unroll
        for (int j = 0; j < CB; ++j) x[j] -= lik * Lp[j][k];
    }
#pragma unroll
    for (int k = 0; k < CB; ++k) {
        double s = x[k];
#pragma unroll
        for (int t = 0; t < k; ++t) s -= x[t] * Ld[k][t];
        x[k] = s / Ld[k][k];
    }
#pragma unroll
    for (int j = 0; j < CB; ++j) rowp[q + j] = x[j];
}

// P[k][i] = A[(r0 + i) ld + c0 + k] for k < NB, i < m (P has leading
// dimension m): the panel rows below the outer diagonal block, transposed
// so the product kernel reads them as k-rows.
__global__ __launch_bounds__(256) void chol_transpose_kernel(int m, int ld, int r0, int c0,
                                                             const double *A, long sA, double *P,
                                                             long sP) {
    __shared__ double t[32][33];
    A += blockIdx.z * sA;
    P += blockIdx.z * sP;
    const int i0 = blockIdx.x * 32, k0 = blockIdx.y * 32;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;   // 32 x 8
    for (int r = ty; r < 32; r += 8)
        t[r][tx] = (i0 + r < m) ? A[(long)(r0 + i0 + r) * ld + c0 + k0 + tx] : 0.0;
    __syncthreads();
    for (int r = ty; r < 32; r += 8)
        if (i0 + tx < m) P[(long)(k0 + r) * m + i0 + tx] = t[tx][r];
}

__global__ void chol_zero_kernel(int nb, double *out) {
    if ((int)threadIdx.x < nb) out[threadIdx.x] = 0.0;
}

// ln det of each of the nb n x n matrices A + b sA (destroyed; only the
// lower triangles are read), n % NB == 0, into out[b] (device).  P is an
// NB x n workspace per matrix (stride sP >= NB n), ws (ws_elems doubles)
// the split-k workspace of the product kernel.
inline void chol_logdet(int n, int ld, int nb, double *A, long sA, double *P, long sP, double *ws,
                        long ws_elems, double *out, hipStream_t st) {
    if (n % NB) throw InvalidArg("chol_logdet: n must be a multiple of 128");
    if (nb < 1 || nb > 1024 || sP < (long)NB * n) throw InvalidArg("chol_logdet: bad batch");
    // the accumulators are cleared by a kernel, not a memset node, so the
    // sequence stays valid inside a captured graph
    hipLaunchKernelGGL(chol_zero_kernel, dim3(1), dim3(1024), 0, st, nb, out);
    XL_LAUNCH_CHECK();
    for (int p = 0; p < n; p += NB) {
        const int pe = p + NB;
        for (int q = p; q < pe; q += CB) {
            const int rest = n - q - CB;
            hipLaunchKernelGGL(chol_panel_kernel, dim3(std::max(1, ceil_div(rest, CHOL_PT)), nb),
                               dim3(CHOL_PT), 0, st, n, ld, p, q, A, sA, out);
            XL_LAUNCH_CHECK();
        }
        const int m = n - pe;
        if (m <= 0) break;
        hipLaunchKernelGGL(chol_transpose_kernel, dim3(ceil_div(m, 32), NB / 32, nb), dim3(256),
                           0, st, m, ld, pe, p, A, sA, P, sP);
        XL_LAUNCH_CHECK();
        GemmArgs<double> g;                    // A22 <- A22 - L21 L21^T
        g.n = m; g.ld = ld; g.k = NB; g.lda = m;
        g.A0 = P; g.B0 = P;
        g.C = A + (long)pe * ld + pe; g.X = g.C;
        g.alpha = -1.0; g.beta = 1.0;
        g.batch = nb; g.sA0 = sP; g.sB0 = sP; g.sC = sA; g.sX = sA;
        g.ws = ws; g.ws_elems = ws_elems;
        gemm(g, true, st);
    }
}

}  // namespace xl
