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
#include <type_traits>

namespace xl {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4v __attribute__((ext_vector_type(4)));
typedef double f64x2v __attribute__((ext_vector_type(2)));

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// hi and lo bf16 pairs of two FP32 values (element 0 in the low half)
__device__ __forceinline__ void split_pair(float x0, float x1, unsigned &hi, unsigned &lo) {
    const f32x2 x = {x0, x1};
    hi = __builtin_bit_cast(unsigned, __builtin_convertvector(x, bf16x2));
    const f32x2 h = {__builtin_bit_cast(float, hi << 16),
                     __builtin_bit_cast(float, hi & 0xffff0000u)};
    lo = __builtin_bit_cast(unsigned, __builtin_convertvector(x - h, bf16x2));
}


__device__ __forceinline__ uint16_t bf16_bits(float x) {
    const bf16x2 h = __builtin_convertvector(f32x2{x, 0.f}, bf16x2);
    return (uint16_t)(__builtin_bit_cast(unsigned, h) & 0xffffu);
}
__device__ __forceinline__ float bf16_val(uint16_t b) {
    return __builtin_bit_cast(float, (unsigned)b << 16);
}
// write x as the (hi, lo) pair of a split matrix (planes pl elements apart)
__device__ __forceinline__ void put_split(uint16_t *C, long pl, long o, float x) {
    const uint16_t h = bf16_bits(x);
    C[o] = h;
    C[o + pl] = bf16_bits(x - bf16_val(h));
}
__device__ __forceinline__ float get_split(const uint16_t *X, long pl, long o) {
    return bf16_val(X[o]) + bf16_val(X[o + pl]);
}

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
// to be the product A_s B_s.  kscale (optional) multiplies row k of B_0 (and
// of B_1 with kscale_both) by kscale[k].  Output n x n with leading dimension ld (also for X, X2, C2);
// the operands are k x n with leading dimension lda (k = 0: k = n; lda = 0:
// lda = ld).  n % 128 == 0, k % 32 == 0.
// Batch index = blockIdx.z; strides in elements (0 = shared operand).
template <typename T> struct GemmArgs {
    int n = 0, ld = 0, batch = 1;
    int k = 0, lda = 0;     // contraction length and operand stride (0: n, ld)
    const T *A0 = nullptr, *B0 = nullptr, *A1 = nullptr, *B1 = nullptr;
    const T *X = nullptr, *X2 = nullptr;
    const double *kscale = nullptr;
    bool kscale_both = false;   // also scale row k of B_1 (else B_0 only)
    T *C = nullptr, *C2 = nullptr;   // C may be null when a copy below is set
    float *Cf = nullptr;    // optional FP32 copy of C (FP64 products only)
    uint16_t *Cs = nullptr; // optional split bf16 copy of C (planes Cs_pl apart)
    uint16_t *Cs2 = nullptr;// optional split bf16 copy of C2 (planes Cs_pl apart)
    long Cs_pl = 0;
    T alpha = 1, beta = 0, beta2 = 0, gamma = 0, p0 = 0, p1 = 0;
    long sA0 = 0, sB0 = 0, sA1 = 0, sB1 = 0, sX = 0, sX2 = 0, sC = 0, sC2 = 0, sK = 0;
    T *ws = nullptr;        // split-k partial tiles (nullptr: no split)
    long ws_elems = 0;
    bool split3 = false;    // FP32 only: bf16x3 products (gemm_bf3_kernel)
    const int *skip = nullptr;  // device flag: the launch does nothing while it is set
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

// Write the 16 x 16 block at (r0, c0) of a 128 x 128 output tile from the
// accumulator of lane (fr, fc): C = alpha acc + beta X + beta2 X2 + gamma I
// (+ C2, + FP32 / split copies), with the symmetric mirror when SYM.
template <typename T, bool SYM>
__device__ __forceinline__ void epilogue_block(const GemmArgs<T> &p, long bz, int ti, int tj,
                                               int r0, int c0, int fr, int fc,
                                               const typename MF<T>::acc_t &acc) {
    using M = MF<T>;
    const int ld = p.ld;
    const int i0 = ti * GT, j0 = tj * GT;
    // lane (fr, fc) of block (x, y) holds rows M::out_row(fr, r), column fc
    T *C = p.C ? p.C + bz * p.sC : nullptr;
    T *C2 = p.C2 ? p.C2 + bz * p.sC2 : nullptr;
    const T *X = p.X ? p.X + bz * p.sX : nullptr;
    const T *X2 = p.X2 ? p.X2 + bz * p.sX2 : nullptr;
    float *Cf = p.Cf ? p.Cf + bz * p.sC : nullptr;
    uint16_t *Cs = p.Cs;    // unbatched (expansion products)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = i0 + r0 + M::out_row(fr, r);
        const int col = j0 + c0 + fc;
        const long o = (long)row * ld + col;
        T val = p.alpha * acc[r];
        if (X) val += p.beta * X[o];
        if (X2) val += p.beta2 * X2[o];
        if (row == col) val += p.gamma;
        T val2 = 0;
        if (C2 || p.Cs2) val2 = p.p1 * val + (row == col ? p.p0 : (T)0);
        if (!SYM) {
            if (C) C[o] = val;
            if (C2) C2[o] = val2;
            if (Cf) Cf[o] = (float)val;
            if (Cs) put_split(Cs, p.Cs_pl, o, (float)val);
            if (p.Cs2) put_split(p.Cs2, p.Cs_pl, o, (float)val2);
        } else if (ti < tj || row <= col) {
            const long ot = (long)col * ld + row;
            if (C) {
                C[o] = val;
                C[ot] = val;
            }
            if (C2) {
                C2[o] = val2;
                C2[ot] = val2;
            }
            if (p.Cs2) {
                put_split(p.Cs2, p.Cs_pl, o, (float)val2);
                put_split(p.Cs2, p.Cs_pl, ot, (float)val2);
            }
            if (Cf) {
                Cf[o] = (float)val;
                Cf[ot] = (float)val;
            }
            if (Cs) {
                put_split(Cs, p.Cs_pl, o, (float)val);
                put_split(Cs, p.Cs_pl, ot, (float)val);
            }
        }
    }
}

// Write the 64 x (16 YB) output block of wave (wr, wc) of a tile.
template <typename T, bool SYM, int YB>
__device__ __forceinline__ void epilogue(const GemmArgs<T> &p, long bz, int ti, int tj, int wr,
                                         int wc, int fr, int fc,
                                         const typename MF<T>::acc_t (&acc)[4][YB]) {
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < YB; ++y)
            epilogue_block<T, SYM>(p, bz, ti, tj, wr * 64 + x * 16, wc * 16 * YB + y * 16, fr, fc,
                                   acc[x][y]);
}


// NW waves per workgroup in 2 rows x NW/2 columns; each wave owns a
// 64 x (256 / NW) block as 4 x YB 16x16 accumulator blocks (YB = 16 / NW).
template <typename T, bool SYM, int NW = 4>
__global__ __launch_bounds__(64 * NW, 2) void gemm_tn_kernel(GemmArgs<T> p, int ntiles, int nfull,
                                                          int nsplit, int per_xcd) {
    if (p.skip && *p.skip) return;   // skipped launch (device flag)
    // per_xcd: tail units per XCD
    using M = MF<T>;
    using acc_t = typename M::acc_t;
    using vec_t = typename M::vec_t;
    constexpr int NTH = 64 * NW, WCN = NW / 2, YB = 16 / NW;
    constexpr int BK = M::BK;
    constexpr int VEC = 16 / sizeof(T);
    constexpr int VPR = GT / VEC;              // vectors per tile row
    constexpr int NV = BK * GT / VEC / NTH;    // 16-byte vectors per thread
    constexpr int PAD = 4;
    __shared__ __attribute__((aligned(16))) T As[2][BK][GT + PAD];
    __shared__ __attribute__((aligned(16))) T Bs[2][BK][GT + PAD];

    // XCD-aware remap: block b runs on XCD b % NXCD; give each XCD a
    // contiguous run of tiles
    // units: tiles [0, nfull) whole, then each remaining tile as nsplit
    // k-range units (filling the last round of workgroups).  Blocks are
    // dispatched in order, whole tiles first; within each region every XCD
    // (block b runs on XCD b % NXCD) gets a contiguous run of units.
    const int b = blockIdx.x;
    const int ntail = ntiles - nfull;
    const int nfull_pad = ((nfull + NXCD - 1) / NXCD) * NXCD;
    int unit;
    if (b < nfull_pad) {
        unit = (b % NXCD) * (nfull_pad / NXCD) + b / NXCD;
        if (unit >= nfull) return;
    } else {
        const int bb = b - nfull_pad;
        unit = nfull + (bb % NXCD) * per_xcd + bb / NXCD;
        if (unit >= nfull + ntail * nsplit) return;
    }
    const bool part = unit >= nfull;
    const int w = unit - nfull;                         // tail unit index
    const int u = part ? nfull + w / nsplit : unit;
    const int split = part ? w % nsplit : 0;
    const int ns = part ? nsplit : 1;
    const int nt = p.n / GT;
    int ti, tj;
    tile_of<SYM>(u, nt, ti, tj);
    const long bz = blockIdx.z;
    const T *A0 = p.A0 + bz * p.sA0, *B0 = p.B0 + bz * p.sB0;
    const T *A1 = p.A1 ? p.A1 + bz * p.sA1 : nullptr;
    const T *B1 = p.B1 ? p.B1 + bz * p.sB1 : nullptr;
    const double *ks = p.kscale ? p.kscale + bz * p.sK : nullptr;
    const int lda = p.lda ? p.lda : p.ld;
    const int i0 = ti * GT, j0 = tj * GT;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wr = wid / WCN, wc = wid % WCN;

    acc_t acc[4][YB];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < YB; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

    const int nk1 = (p.k ? p.k : p.n) / BK;
    const int nktot = A1 ? 2 * nk1 : nk1;
    const int kt0 = (int)((long)nktot * split / ns);
    const int kt1 = (int)((long)nktot * (split + 1) / ns);

    // NV 16-byte vectors of A and NV of B per thread per k-tile
    vec_t ra[NV], rb[NV];
    int lrow[NV], lcol[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int vi = tid + NTH * v;
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
            ra[v] = *reinterpret_cast<const vec_t *>(Ap + k * lda + i0 + lcol[v]);
            rb[v] = *reinterpret_cast<const vec_t *>(Bp + k * lda + j0 + lcol[v]);
            if (ks && (!second || p.kscale_both)) {
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
    // branch-free k step (one scheduling region): at the last k-tile the
    // global load repeats it and the LDS store fills the idle buffer
    for (int kt = kt0; kt < kt1; ++kt) {
        const int buf = (kt - kt0) & 1;
        gload(min(kt + 1, kt1 - 1));
#pragma unroll
        for (int s = 0; s < BK / 4; ++s) {
            T a[4], b[YB];
#pragma unroll
            for (int q = 0; q < 4; ++q) a[q] = As[buf][4 * s + fr][wr * 64 + q * 16 + fc];
#pragma unroll
            for (int q = 0; q < YB; ++q) b[q] = Bs[buf][4 * s + fr][wc * 16 * YB + q * 16 + fc];
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < YB; ++y) acc[x][y] = M::mma(a[x], b[y], acc[x][y]);
        }
        sstore(buf ^ 1);
        if constexpr (sizeof(T) == 8) {
            // FP64: each sub-step's LDS reads ahead of its MFMAs, the global
            // loads after the first, the LDS stores last
#pragma unroll
            for (int s = 0; s < BK / 4; ++s) {
                __builtin_amdgcn_sched_group_barrier(0x100, 4 + YB, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 4 * YB, 0);
                if (s == 0) __builtin_amdgcn_sched_group_barrier(0x020, 2 * NV, 0);
            }
            __builtin_amdgcn_sched_group_barrier(0x200, 2 * NV, 0);
            __builtin_amdgcn_sched_barrier(0);
        }
        __syncthreads();
    }

    if (part) {
        // partial tile: accumulator block g = YB x + y of thread tid as one
        // 4-vector at [(g * NTH + tid) * 4] (vector stores, contiguous
        // across the workgroup)
        acc_t *wp = reinterpret_cast<acc_t *>(p.ws + ((long)bz * ntail * nsplit + w) * (GT * GT)) + tid;
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < YB; ++y) wp[(x * YB + y) * NTH] = acc[x][y];
        return;
    }

    epilogue<T, SYM, YB>(p, bz, ti, tj, wr, wc, fr, fc, acc);
}

// ---------------------------------------------------------------------------
// Split-precision FP32 product on the bf16 matrix cores.  Each FP32 operand
// x is written as hi + lo with hi = bf16(x) and lo = bf16(x - hi) (the
// residual is exact in FP32), and the product is hi*hi + hi*lo + lo*hi with
// FP32 accumulation; the dropped lo*lo term and the rounding of lo leave a
// relative error of about 2^-16 per operand, against 2^-8 for plain bf16.
// Three 16x16x32 bf16 MFMAs replace eight 16x16x4 FP32 MFMAs per 16x16x32
// block: at the bf16 rate this is 16/3 of the FP32 matrix-core rate.
//
// Operands stay FP32 in HBM (same arguments, schedule, epilogue and split-k
// partials as the FP32 kernel).  Each thread loads a 4 (k) x 4 (i) block of
// each operand tile with four 16-byte row loads, splits it, and stores it
// transposed into LDS as [i][k] rows of hi and of lo parts, so a lane's MFMA
// fragment (8 consecutive k of one row) is one 16-byte LDS read.  Row pitch
// 40 bf16 (80 bytes): the 16-byte fragment reads of 16 consecutive rows and
// the 8-byte stores of a 16-lane group fall in distinct banks.
// ---------------------------------------------------------------------------
constexpr int B3K = 32;          // k per tile = k of one bf16 MFMA
constexpr int B3P = 20;          // LDS row pitch in 32-bit words (40 bf16)

template <bool SYM>
__global__ __launch_bounds__(256, 2) void gemm_bf3_kernel(GemmArgs<float> p, int ntiles, int nfull,
                                                       int nsplit, int per_xcd) {
    if (p.skip && *p.skip) return;   // skipped launch (device flag)
    using acc_t = f32x4;
    // [buffer][hi, lo][row i][k pairs]
    __shared__ __attribute__((aligned(16))) unsigned As[2][2][GT][B3P];
    __shared__ __attribute__((aligned(16))) unsigned Bs[2][2][GT][B3P];

    // unit -> tile, as in gemm_tn_kernel
    const int b = blockIdx.x;
    const int ntail = ntiles - nfull;
    const int nfull_pad = ((nfull + NXCD - 1) / NXCD) * NXCD;
    int unit;
    if (b < nfull_pad) {
        unit = (b % NXCD) * (nfull_pad / NXCD) + b / NXCD;
        if (unit >= nfull) return;
    } else {
        const int bb = b - nfull_pad;
        unit = nfull + (bb % NXCD) * per_xcd + bb / NXCD;
        if (unit >= nfull + ntail * nsplit) return;
    }
    const bool part = unit >= nfull;
    const int w = unit - nfull;
    const int u = part ? nfull + w / nsplit : unit;
    const int split = part ? w % nsplit : 0;
    const int ns = part ? nsplit : 1;
    const int nt = p.n / GT;
    int ti, tj;
    tile_of<SYM>(u, nt, ti, tj);
    const long bz = blockIdx.z;
    const float *A0 = p.A0 + bz * p.sA0, *B0 = p.B0 + bz * p.sB0;
    const float *A1 = p.A1 ? p.A1 + bz * p.sA1 : nullptr;
    const float *B1 = p.B1 ? p.B1 + bz * p.sB1 : nullptr;
    const double *ks = p.kscale ? p.kscale + bz * p.sK : nullptr;
    const int lda = p.lda ? p.lda : p.ld;
    const int i0 = ti * GT, j0 = tj * GT;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wr = wid >> 1, wc = wid & 1;

    acc_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = acc_t{0, 0, 0, 0};

    const int nk1 = (p.k ? p.k : p.n) / B3K;
    const int nktot = A1 ? 2 * nk1 : nk1;
    const int kt0 = (int)((long)nktot * split / ns);
    const int kt1 = (int)((long)nktot * (split + 1) / ns);

    // loader: k rows 4 kq .. 4 kq + 3, tile columns 4 xv .. 4 xv + 3
    // (loads run one k-tile ahead)
    const int kq = tid & 7, xv = tid >> 3;
    f32x4 ra[4], rb[4];
    auto gload = [&](int kt) {
        const bool second = kt >= nk1;
        const float *Ap = second ? A1 : A0;
        const float *Bp = second ? B1 : B0;
        const int kb = (second ? kt - nk1 : kt) * B3K + 4 * kq;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const long k = kb + v;
            ra[v] = *reinterpret_cast<const f32x4 *>(Ap + k * lda + i0 + 4 * xv);
            rb[v] = *reinterpret_cast<const f32x4 *>(Bp + k * lda + j0 + 4 * xv);
            if (ks && (!second || p.kscale_both)) rb[v] *= (float)ks[k];
        }
    };
    // column e of the 4 x 4 block: k-consecutive, split, one 8-byte store
    // per part
    auto sstore = [&](int buf) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            unsigned h0, h1, l0, l1;
            split_pair(ra[0][e], ra[1][e], h0, l0);
            split_pair(ra[2][e], ra[3][e], h1, l1);
            *reinterpret_cast<u32x2 *>(&As[buf][0][4 * xv + e][2 * kq]) = u32x2{h0, h1};
            *reinterpret_cast<u32x2 *>(&As[buf][1][4 * xv + e][2 * kq]) = u32x2{l0, l1};
            split_pair(rb[0][e], rb[1][e], h0, l0);
            split_pair(rb[2][e], rb[3][e], h1, l1);
            *reinterpret_cast<u32x2 *>(&Bs[buf][0][4 * xv + e][2 * kq]) = u32x2{h0, h1};
            *reinterpret_cast<u32x2 *>(&Bs[buf][1][4 * xv + e][2 * kq]) = u32x2{l0, l1};
        }
    };

    gload(kt0);
    sstore(0);
    __syncthreads();
    const int fr = lane >> 4, fc = lane & 15;
    for (int kt = kt0; kt < kt1; ++kt) {
        const int buf = (kt - kt0) & 1;
        if (kt + 1 < kt1) gload(kt + 1);
        // fragment of lane (fr, fc): row fc of the 16-row block, k 8 fr .. 8 fr + 7
        bf16x8 ah[4], al[4], bh[4], bl[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int ra_ = wr * 64 + q * 16 + fc, rb_ = wc * 64 + q * 16 + fc;
            ah[q] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4 *>(&As[buf][0][ra_][4 * fr]));
            al[q] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4 *>(&As[buf][1][ra_][4 * fr]));
            bh[q] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4 *>(&Bs[buf][0][rb_][4 * fr]));
            bl[q] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4 *>(&Bs[buf][1][rb_][4 * fr]));
        }
        // small terms first
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) {
                acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[x], bh[y], acc[x][y], 0, 0, 0);
                acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[x], bl[y], acc[x][y], 0, 0, 0);
                acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[x], bh[y], acc[x][y], 0, 0, 0);
            }
        if (kt + 1 < kt1) sstore(buf ^ 1);
        __syncthreads();
    }

    if (part) {
        acc_t *wp = reinterpret_cast<acc_t *>(p.ws + ((long)bz * ntail * nsplit + w) * (GT * GT)) + tid;
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) wp[(x * 4 + y) * 256] = acc[x][y];
        return;
    }
    // the 16x16 bf16 MFMA leaves its accumulators in the FP32 16x16x4 layout
    epilogue<float, SYM, 4>(p, bz, ti, tj, wr, wc, fr, fc, acc);
}

// Sum the k-split partial tiles of each tile and apply the epilogue.  One
// workgroup per (tile, accumulator block g = 4x + y): every thread reads
// back, from each partial, the one accumulator vector its counterpart in
// the product kernel wrote for block g (4 KB contiguous per workgroup and
// partial), so the reduction runs on 16 workgroups per tile.
// 256 threads per workgroup whatever NW: for NW = 8 each (tile, block)
// pair is covered by two workgroups, one per half of the product's threads.
template <typename T, bool SYM, int NW = 4>
__global__ __launch_bounds__(256) void gemm_fixup_kernel(GemmArgs<T> p, int ntiles,
                                                         int nfull, int nsplit) {
    if (p.skip && *p.skip) return;   // skipped launch (device flag)
    using acc_t = typename MF<T>::acc_t;
    constexpr int NTH = 64 * NW, WCN = NW / 2, YB = 16 / NW, NH = NTH / 256;
    const int ntail = ntiles - nfull;
    const int u = nfull + blockIdx.x;
    const int g = blockIdx.y / NH, x = g / YB, y = g % YB;
    const long bz = blockIdx.z;
    const int nt = p.n / GT;
    int ti, tj;
    tile_of<SYM>(u, nt, ti, tj);
    const int tid = (blockIdx.y % NH) * 256 + threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wr = wid / WCN, wc = wid % WCN, fr = lane >> 4, fc = lane & 15;
    acc_t acc = acc_t{0, 0, 0, 0};
    const acc_t *wp = reinterpret_cast<const acc_t *>(
                          p.ws + ((long)bz * ntail * nsplit + (long)blockIdx.x * nsplit) *
                                     (GT * GT)) + g * NTH + tid;
    for (int s = 0; s < nsplit; ++s) acc += wp[(long)s * (GT * GT / 4)];
    epilogue_block<T, SYM>(p, bz, ti, tj, wr * 64 + x * 16, wc * 16 * YB + y * 16, fr, fc, acc);
}

// CU count of the current device, read once (thread-safe initialisation:
// systems stepped by several host threads share it)
inline int device_cus() {
    static const int cus = [] {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            n <= 0)
            return 256;
        return n;
    }();
    return cus;
}

// Work schedule of one launch (per_cu workgroups per CU: two for the
// 128 x 128 kernels, one for the 256 x 128 split kernel).
// More tiles than workgroup slots: whole tiles fill complete rounds and only
// the tiles of the last, partial round are split along k over the
// otherwise idle slots.  Fewer tiles than slots: every tile is split into
// the same number of k-ranges, the smallest count whose round is nearly
// full.  Split partial tiles are summed by a fix-up kernel.  Batched
// launches have tiles enough: no split.
struct Sched {
    int nfull, nsplit;
};
template <typename T> Sched schedule(int ntiles, int nkt, long batch, int per_cu = 2) {
    const long slots = (long)device_cus() * per_cu;
    if (batch > 1) return {ntiles, 1};
    if (ntiles > slots) {
        const long rounds = ntiles / slots;
        const int tail = (int)(ntiles - rounds * slots);
        if (tail == 0) return {ntiles, 1};
        const int s = (int)std::min<long>(slots / tail, nkt / 8);
        if (s < 2) return {ntiles, 1};
        return {(int)(rounds * slots), s};
    }
    double best = -1.0;
    int bs = 1;
    for (int s : {1, 2, 3, 4, 6, 8}) {
        if (s > 1 && nkt / s < 8) break;
        const double units = (double)ntiles * s;
        const double rounds = std::ceil(units / slots);
        const double eff = units / (rounds * slots) * (1.0 - 0.01 * (s - 1));
        if (eff > best + 1e-9) { best = eff; bs = s; }
    }
    return {bs > 1 ? 0 : ntiles, bs};
}

template <typename T> long split_ws_elems(int n, bool sym, int dual, long batch) {
    const int nt = n / GT;
    const int ntiles = sym ? nt * (nt + 1) / 2 : nt * nt;
    const int nkt = (n / MF<T>::BK) * (dual ? 2 : 1);
    const Sched s = schedule<T>(ntiles, nkt, batch);
    return std::max(1L, (long)(ntiles - s.nfull) * s.nsplit * batch * GT * GT);
}

// waves per workgroup of the FP64 / FP32 product kernel: 8 (four per SIMD)
// measured faster than 4 for both precisions at N = 4096
template <typename T> constexpr int TN_WAVES = 8;

template <typename T>
void gemm(const GemmArgs<T> &a, bool sym, hipStream_t st) {
    const int K = a.k ? a.k : a.n;
    if (a.n % GT != 0 || a.ld % 4 != 0 || K % 32 != 0 || (a.lda ? a.lda : a.ld) % 4 != 0)
        throw InvalidArg("gemm: n must be a multiple of 128 and k of 32");
    if (a.split3 && !std::is_same<T, float>::value)
        throw InvalidArg("gemm: split bf16x3 products take FP32 operands");
    const int nt = a.n / GT;
    const int ntiles = sym ? nt * (nt + 1) / 2 : nt * nt;
    const int nkt = (K / MF<T>::BK) * (a.A1 ? 2 : 1);
    Sched s = a.ws ? schedule<T>(ntiles, nkt, a.batch) : Sched{ntiles, 1};
    if (s.nsplit > 1 && (long)(ntiles - s.nfull) * s.nsplit * a.batch * GT * GT > a.ws_elems)
        s = Sched{ntiles, 1};
    const int nfull_pad = ((s.nfull + NXCD - 1) / NXCD) * NXCD;
    const int tail_units = (ntiles - s.nfull) * s.nsplit;
    const int per = (tail_units + NXCD - 1) / NXCD;     // tail units per XCD
    dim3 grid(nfull_pad + per * NXCD, 1, a.batch);
    if constexpr (std::is_same<T, float>::value) {
        if (a.split3) {
            if (sym)
                hipLaunchKernelGGL((gemm_bf3_kernel<true>), grid, dim3(256), 0, st, a, ntiles,
                                   s.nfull, s.nsplit, per);
            else
                hipLaunchKernelGGL((gemm_bf3_kernel<false>), grid, dim3(256), 0, st, a, ntiles,
                                   s.nfull, s.nsplit, per);
        }
    }
    constexpr int NW = TN_WAVES<T>;
    if (!a.split3) {
        if (sym)
            hipLaunchKernelGGL((gemm_tn_kernel<T, true, NW>), grid, dim3(64 * NW), 0, st, a,
                               ntiles, s.nfull, s.nsplit, per);
        else
            hipLaunchKernelGGL((gemm_tn_kernel<T, false, NW>), grid, dim3(64 * NW), 0, st, a,
                               ntiles, s.nfull, s.nsplit, per);
    }
    XL_LAUNCH_CHECK();
    if (s.nfull < ntiles) {
        // the split kernel keeps the 4-wave accumulator layout
        const bool w8 = !a.split3 && NW == 8;
        // (accumulator blocks per thread) x (256-thread groups of the product)
        dim3 g2(ntiles - s.nfull, 16, a.batch);
        if (w8) {
            if (sym)
                hipLaunchKernelGGL((gemm_fixup_kernel<T, true, 8>), g2, dim3(256), 0, st, a,
                                   ntiles, s.nfull, s.nsplit);
            else
                hipLaunchKernelGGL((gemm_fixup_kernel<T, false, 8>), g2, dim3(256), 0, st, a,
                                   ntiles, s.nfull, s.nsplit);
        } else if (sym) {
            hipLaunchKernelGGL((gemm_fixup_kernel<T, true, 4>), g2, dim3(256), 0, st, a, ntiles,
                               s.nfull, s.nsplit);
        } else {
            hipLaunchKernelGGL((gemm_fixup_kernel<T, false, 4>), g2, dim3(256), 0, st, a,
                               ntiles, s.nfull, s.nsplit);
        }
        XL_LAUNCH_CHECK();
    }
}

}  // namespace xl
