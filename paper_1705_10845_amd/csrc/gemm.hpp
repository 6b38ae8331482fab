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
// 32 (FP32) or 16 (FP64) elements = 128 bytes per row.  The grid is 1-D over
// the tiles actually computed (the upper block triangle for symmetric
// outputs); consecutive tiles of a block row go to the same XCD so they
// share the A panel in that XCD's L2.
#pragma once
#include "common.hpp"

#include <cmath>

namespace xl {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4v __attribute__((ext_vector_type(4)));
typedef double f64x2v __attribute__((ext_vector_type(2)));

template <typename T> struct MF;
template <> struct MF<float> {
    using acc_t = f32x4;
    using vec_t = f32x4v;
    static constexpr int BK = 32;
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
    static constexpr int BK = 16;
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
    T *ws = nullptr;        // split-k partial tiles (nullptr: no split)
    long ws_elems = 0;
};

constexpr int GT = 128;   // output tile edge

constexpr int NXCD = 8;   // XCDs per MI355X; workgroups go round-robin to them

// tile (ti, tj) of linear tile index u: row-major over the upper block
// triangle (SYM) or the full grid
template <bool SYM>
__device__ __forceinline__ void tile_of(int u, int nt, int &ti, int &tj) {
    if (!SYM) {
        ti = u / nt;
        tj = u % nt;
        return;
    }
    int row = 0, start = 0;
    while (start + (nt - row) <= u) {
        start += nt - row;
        ++row;
    }
    ti = row;
    tj = row + (u - start);
}

// Write one 128 x 128 output tile from the accumulators of thread
// (wr, wc, fr, fc): C = alpha acc + beta X + beta2 X2 + gamma I (+ C2), with
// the symmetric mirror when SYM.
template <typename T, bool SYM>
__device__ __forceinline__ void epilogue(const GemmArgs<T> &p, long bz, int ti, int tj, int wr,
                                         int wc, int fr, int fc,
                                         const typename MF<T>::acc_t (&acc)[4][4]) {
    using M = MF<T>;
    const int ld = p.ld;
    const int i0 = ti * GT, j0 = tj * GT;
    // lane (fr, fc) of block (x, y) holds rows M::out_row(fr, r), column fc
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


template <typename T, bool SYM>
__global__ __launch_bounds__(256) void gemm_tn_kernel(GemmArgs<T> p, int ntiles, int per_xcd,
                                                      int nsplit) {
    using M = MF<T>;
    using acc_t = typename M::acc_t;
    using vec_t = typename M::vec_t;
    constexpr int BK = M::BK;
    constexpr int VEC = 16 / sizeof(T);
    constexpr int VPR = GT / VEC;              // vectors per tile row
    constexpr int NV = BK * GT / VEC / 256;    // 16-byte vectors per thread
    constexpr int PAD = 4;
    __shared__ __attribute__((aligned(16))) T As[2][BK][GT + PAD];
    __shared__ __attribute__((aligned(16))) T Bs[2][BK][GT + PAD];

    // XCD-aware remap: block b runs on XCD b % NXCD; give each XCD a
    // contiguous run of tiles
    // unit = (tile, k-split); the splits of one tile are consecutive units
    const int b = blockIdx.x;
    const int unit = (b % NXCD) * per_xcd + b / NXCD;
    if (unit >= ntiles * nsplit) return;
    const int u = unit / nsplit, split = unit % nsplit;
    const int nt = p.n / GT;
    int ti, tj;
    tile_of<SYM>(u, nt, ti, tj);
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
    const int nktot = A1 ? 2 * nk1 : nk1;
    const int kt0 = (int)((long)nktot * split / nsplit);
    const int kt1 = (int)((long)nktot * (split + 1) / nsplit);

    // NV 16-byte vectors of A and NV of B per thread per k-tile
    vec_t ra[NV], rb[NV];
    int lrow[NV], lcol[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
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
        for (int v = 0; v < NV; ++v) {
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
        for (int v = 0; v < NV; ++v) {
            *reinterpret_cast<vec_t *>(&As[buf][lrow[v]][lcol[v]]) = ra[v];
            *reinterpret_cast<vec_t *>(&Bs[buf][lrow[v]][lcol[v]]) = rb[v];
        }
    };

    gload(kt0);
    sstore(0);
    __syncthreads();
    const int fr = lane >> 4, fc = lane & 15;
    for (int kt = kt0; kt < kt1; ++kt) {
        const int buf = (kt - kt0) & 1;
        if (kt + 1 < kt1) gload(kt + 1);
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
        if (kt + 1 < kt1) sstore(buf ^ 1);
        __syncthreads();
    }

    if (nsplit > 1) {
        // partial tile: each thread stores its 64 accumulators contiguously
        T *w = p.ws + ((long)bz * ntiles * nsplit + unit) * (GT * GT) + (long)tid * 64;
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y)
#pragma unroll
                for (int r = 0; r < 4; ++r) w[(x * 4 + y) * 4 + r] = acc[x][y][r];
        return;
    }

    epilogue<T, SYM>(p, bz, ti, tj, wr, wc, fr, fc, acc);
}

// Sum the k-split partial tiles of each tile and apply the epilogue.  Same
// thread layout as the product kernel, so every thread reads back exactly
// the accumulators its counterpart wrote (contiguous 64 per thread).
template <typename T, bool SYM>
__global__ __launch_bounds__(256) void gemm_fixup_kernel(GemmArgs<T> p, int ntiles, int nsplit) {
    using acc_t = typename MF<T>::acc_t;
    const int u = blockIdx.x;
    const long bz = blockIdx.z;
    const int nt = p.n / GT;
    int ti, tj;
    tile_of<SYM>(u, nt, ti, tj);
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wr = wid >> 1, wc = wid & 1, fr = lane >> 4, fc = lane & 15;
    acc_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
    for (int s = 0; s < nsplit; ++s) {
        const T *w = p.ws + ((long)bz * ntiles * nsplit + (long)u * nsplit + s) * (GT * GT) +
                     (long)tid * 64;
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[x][y][r] += w[(x * 4 + y) * 4 + r];
    }
    epilogue<T, SYM>(p, bz, ti, tj, wr, wc, fr, fc, acc);
}

inline int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
    }
    return cus;
}

// Number of k-splits for a launch: the smallest split count whose last
// round of workgroups is nearly full (the product kernels run one (FP64) or
// two (FP32) workgroups per CU).
template <typename T> int choose_split(int ntiles, int nkt, long batch) {
    const long slots = (long)device_cus() * (sizeof(T) == 8 ? 1 : 2);
    double best = -1.0;
    int bs = 1;
    for (int s : {1, 2, 3, 4, 6, 8}) {
        if (s > 1 && nkt / s < 8) break;
        const double units = (double)ntiles * s * batch;
        const double rounds = std::ceil(units / slots);
        double eff = units / (rounds * slots);
        eff *= 1.0 - 0.01 * (s - 1);          // partial-tile traffic
        if (eff > best + 1e-9) { best = eff; bs = s; }
    }
    return bs;
}

template <typename T> long split_ws_elems(int n, bool sym, int dual, long batch) {
    const int nt = n / GT;
    const int ntiles = sym ? nt * (nt + 1) / 2 : nt * nt;
    const int nkt = (n / MF<T>::BK) * (dual ? 2 : 1);
    return (long)ntiles * choose_split<T>(ntiles, nkt, batch) * batch * GT * GT;
}

template <typename T>
void gemm(const GemmArgs<T> &a, bool sym, hipStream_t st) {
    if (a.n % GT != 0 || a.ld % 4 != 0)
        throw InvalidArg("gemm: n must be a multiple of 128");
    const int nt = a.n / GT;
    const int ntiles = sym ? nt * (nt + 1) / 2 : nt * nt;
    const int nkt = (a.n / MF<T>::BK) * (a.A1 ? 2 : 1);
    int nsplit = a.ws ? choose_split<T>(ntiles, nkt, a.batch) : 1;
    if (nsplit > 1 && (long)ntiles * nsplit * a.batch * GT * GT > a.ws_elems) nsplit = 1;
    const int units = ntiles * nsplit;
    const int per = (units + NXCD - 1) / NXCD;
    dim3 grid(per * NXCD, 1, a.batch);
    if (sym)
        hipLaunchKernelGGL((gemm_tn_kernel<T, true>), grid, dim3(256), 0, st, a, ntiles, per, nsplit);
    else
        hipLaunchKernelGGL((gemm_tn_kernel<T, false>), grid, dim3(256), 0, st, a, ntiles, per, nsplit);
    XL_LAUNCH_CHECK();
    if (nsplit > 1) {
        dim3 g2(ntiles, 1, a.batch);
        if (sym)
            hipLaunchKernelGGL((gemm_fixup_kernel<T, true>), g2, dim3(256), 0, st, a, ntiles, nsplit);
        else
            hipLaunchKernelGGL((gemm_fixup_kernel<T, false>), g2, dim3(256), 0, st, a, ntiles, nsplit);
        XL_LAUNCH_CHECK();
    }
}

}  // namespace xl
