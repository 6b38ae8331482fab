// Dense MFMA products for the Fermi-operator expansion and its response.
//
// Every product in the expansion has a symmetric left operand (a function of
// H, or the symmetrised response A'), so the kernel reads the left operand as
// rows of A^T = A: both operands are loaded as contiguous k-rows, which keeps
// every global load a coalesced 16-byte vector.  When the product itself is a
// function of H (Z^2, A Y, Y (2I - A Y), Y Z, ...) the output is symmetric:
// only the upper block triangle is computed and each tile is mirrored.
//
// Tile: 128 x 128 per 256-thread workgroup (4 waves in 2 x 2, 64 x 64 per
// wave as 4 x 4 blocks of the 16x16x4 MFMA), double-buffered LDS, k-tile of
// 16 (FP32) or 8 (FP64) elements = 64 bytes per row.
#pragma once
#include "common.hpp"

namespace xl {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4v __attribute__((ext_vector_type(4)));
typedef double f64x2v __attribute__((ext_vector_type(2)));

template <typename T> struct MF;
template <> struct MF<float> {
    using acc_t = f32x4;
    using vec_t = f32x4v;
    static constexpr int BK = 16;
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // row within the 16x16 block of accumulator element r of lane group g
    // (g = lane / 16; the column is lane % 16)
    static __device__ __forceinline__ int out_row(int g, int r) { return 4 * g + r; }
};
template <> struct MF<double> {
    using acc_t = f64x4;
    using vec_t = f64x2v;
    static constexpr int BK = 8;
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // the FP64 instruction interleaves: element r of lane group g is row 4r + g
    static __device__ __forceinline__ int out_row(int g, int r) { return 4 * r + g; }
};

// C = alpha * sum_s A_s^T B_s + beta * X + beta2 * X2 + gamma * I ; optionally
// C2 = p0 * I + p1 * C.  A_s must be symmetric (A_s^T = A_s) for the result
// to be the product A_s B_s.  kscale (optional) multiplies row k of B_0 by
// kscale[k].  All matrices n x n with leading dimension ld; n % 128 == 0.
// Batch index = blockIdx.z; strides in elements (0 = shared operand).
template <typename T> struct GemmArgs {
    int n = 0, ld = 0, batch = 1;
    const T *A0 = nullptr, *B0 = nullptr, *A1 = nullptr, *B1 = nullptr;
    const T *X = nullptr, *X2 = nullptr;
    const double *kscale = nullptr;
    T *C = nullptr, *C2 = nullptr;
    T alpha = 1, beta = 0, beta2 = 0, gamma = 0, p0 = 0, p1 = 0;
    long sA0 = 0, sB0 = 0, sA1 = 0, sB1 = 0, sX = 0, sX2 = 0, sC = 0, sC2 = 0, sK = 0;
};

constexpr int GT = 128;   // output tile edge

template <typename T, bool SYM>
__global__ __launch_bounds__(256) void gemm_tn_kernel(GemmArgs<T> p) {
    using M = MF<T>;
    using acc_t = typename M::acc_t;
    using vec_t = typename M::vec_t;
    constexpr int BK = M::BK;
    constexpr int VEC = 16 / sizeof(T);
    constexpr int VPR = GT / VEC;              // vectors per tile row
    constexpr int PAD = 4;
    __shared__ __attribute__((aligned(16))) T As[2][BK][GT + PAD];
    __shared__ __attribute__((aligned(16))) T Bs[2][BK][GT + PAD];

    const int ti = blockIdx.y, tj = blockIdx.x;
    if (SYM && ti > tj) return;
    const long bz = blockIdx.z;
    const T *A0 = p.A0 + bz * p.sA0, *B0 = p.B0 + bz * p.sB0;
    const T *A1 = p.A1 ? p.A1 + bz * p.sA1 : nullptr;
    const T *B1 = p.B1 ? p.B1 + bz * p.sB1 : nullptr;
    const double *ks = p.kscale ? p.kscale + bz * p.sK : nullptr;
    const int ld = p.ld;
    const int i0 = ti * GT, j0 = tj * GT;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wr = wid >> 1, wc = wid & 1;

    acc_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

    const int nk1 = p.n / BK;
    const int nkt = A1 ? 2 * nk1 : nk1;

    // two 16-byte vectors of A and two of B per thread per k-tile
    vec_t ra[2], rb[2];
    int lrow[2], lcol[2];
#pragma unroll
    for (int v = 0; v < 2; ++v) {
        const int vi = tid + 256 * v;
        lrow[v] = vi / VPR;
        lcol[v] = (vi % VPR) * VEC;
    }
    auto gload = [&](int kt) {
        const bool second = kt >= nk1;
        const T *Ap = second ? A1 : A0;
        const T *Bp = second ? B1 : B0;
        const int kb = (second ? kt - nk1 : kt) * BK;
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const long k = kb + lrow[v];
            ra[v] = *reinterpret_cast<const vec_t *>(Ap + k * ld + i0 + lcol[v]);
            rb[v] = *reinterpret_cast<const vec_t *>(Bp + k * ld + j0 + lcol[v]);
            if (ks && !second) {
                const T s = (T)ks[k];
#pragma unroll
                for (int e = 0; e < VEC; ++e) rb[v][e] *= s;
            }
        }
    };
    // (GT + PAD) * sizeof(T) is a multiple of 16 bytes: one 16-byte LDS
    // store per vector
    auto sstore = [&](int buf) {
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            *reinterpret_cast<vec_t *>(&As[buf][lrow[v]][lcol[v]]) = ra[v];
            *reinterpret_cast<vec_t *>(&Bs[buf][lrow[v]][lcol[v]]) = rb[v];
        }
    };

    gload(0);
    sstore(0);
    __syncthreads();
    const int fr = lane >> 4, fc = lane & 15;
    for (int kt = 0; kt < nkt; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nkt) gload(kt + 1);
#pragma unroll
        for (int s = 0; s < BK / 4; ++s) {
            T a[4], b[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a[q] = As[buf][4 * s + fr][wr * 64 + q * 16 + fc];
                b[q] = Bs[buf][4 * s + fr][wc * 64 + q * 16 + fc];
            }
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) acc[x][y] = M::mma(a[x], b[y], acc[x][y]);
        }
        if (kt + 1 < nkt) sstore(buf ^ 1);
        __syncthreads();
    }

    // epilogue: lane (fr, fc) of block (x, y) holds rows M::out_row(fr, r),
    // column fc
    T *C = p.C + bz * p.sC;
    T *C2 = p.C2 ? p.C2 + bz * p.sC2 : nullptr;
    const T *X = p.X ? p.X + bz * p.sX : nullptr;
    const T *X2 = p.X2 ? p.X2 + bz * p.sX2 : nullptr;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = i0 + wr * 64 + x * 16 + M::out_row(fr, r);
                const int col = j0 + wc * 64 + y * 16 + fc;
                const long o = (long)row * ld + col;
                T val = p.alpha * acc[x][y][r];
                if (X) val += p.beta * X[o];
                if (X2) val += p.beta2 * X2[o];
                if (row == col) val += p.gamma;
                T val2 = 0;
                if (C2) val2 = p.p1 * val + (row == col ? p.p0 : (T)0);
                if (!SYM) {
                    C[o] = val;
                    if (C2) C2[o] = val2;
                } else if (ti < tj || row <= col) {
                    const long ot = (long)col * ld + row;
                    C[o] = val;
                    C[ot] = val;
                    if (C2) {
                        C2[o] = val2;
                        C2[ot] = val2;
                    }
                }
            }
}

template <typename T>
void gemm(const GemmArgs<T> &a, bool sym, hipStream_t st) {
    if (a.n % GT != 0 || a.ld % 4 != 0)
        throw InvalidArg("gemm: n must be a multiple of 128");
    dim3 grid(a.n / GT, a.n / GT, a.batch);
    if (sym)
        hipLaunchKernelGGL((gemm_tn_kernel<T, true>), grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((gemm_tn_kernel<T, false>), grid, dim3(256), 0, st, a);
    XL_LAUNCH_CHECK();
}

}  // namespace xl
