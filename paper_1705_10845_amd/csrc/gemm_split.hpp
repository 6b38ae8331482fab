// Split bf16x3 products on pre-split operands.
//
// Storage: an n x n "split matrix" is two bf16 planes, hi and lo, each row
// major with leading dimension ld; plane lo starts `pl` elements after plane
// hi (so a split matrix occupies the bytes of one FP32 matrix).  x = hi + lo
// with hi = bf16(x), lo = bf16(x - hi) of the FP32 value.
//
// Product: C[i][j] = alpha sum_s sum_k A_s[i][k] B_s[j][k] + beta X[i][j]
// (+ beta2 X2[i][j]) + gamma delta_ij, i.e. both operands are read as rows
// with k contiguous ("NT").  Every operand of the response recursion is
// symmetric, or is stored transposed by the product that makes it, so this
// is the matrix product the recursion needs.  C and X are split matrices
// too; X may instead be an FP64 matrix (Xd), X2 is FP64, and the result may
// go (also) to an FP64 matrix Cd.  The epilogue sum and its coefficients
// are FP64.
//
// With `hi_only` the product is a plain bf16 one: only the hi planes of A
// and B are loaded and multiplied (hi.hi, relative error ~2^-8 per
// operand); the result is still written as a split matrix (its FP32 value).
//
// Against gemm_bf3_kernel (FP32 operands split while staging) the k-tiles
// here are copied into LDS as 16-byte chunks with no conversion work, the
// workgroup has 8 waves (four per SIMD at two workgroups per CU), and
// the chunk order within each 64-byte LDS row is permuted by a function of
// the row (`swz`) so that neither the chunk stores (4 lanes per row) nor the
// 16-byte fragment reads (16 consecutive rows, one chunk) conflict in banks.
#pragma once
#include "gemm.hpp"

namespace xl {

struct SplitArgs {
    int n = 0, ld = 0, batch = 1;
    long pl = 0;                                  // plane offset (elements)
    const uint16_t *A0 = nullptr, *B0 = nullptr, *A1 = nullptr, *B1 = nullptr;
    const uint16_t *X = nullptr;
    const double *Xd = nullptr, *Xd2 = nullptr;   // FP64 X (instead of X), second term
    uint16_t *C = nullptr;
    double *Cd = nullptr;                         // FP64 result (C may be null)
    double alpha = 1.0, beta = 0.0, beta2 = 0.0, gamma = 0.0;
    long sA0 = 0, sB0 = 0, sA1 = 0, sB1 = 0, sX = 0, sC = 0;   // batch strides (elements)
    float *ws = nullptr;                          // split-k partial tiles (FP32)
    long ws_elems = 0;
    const int *skip = nullptr;                    // device flag: skip the launch while set
    bool hi_only = false;                         // plain bf16 product (hi planes only)
};

// chunk permutation of LDS row r (values 0..3, rows in pairs): with it the
// 16-byte fragment reads (16 consecutive rows, one chunk each) and the chunk
// stores (4 lanes per row) of these kernels count no LDS bank conflicts
// (SQ_LDS_BANK_CONFLICT = 0 at N = 4096; the permutations that also spread
// every 4 rows of equal residue mod 4, or none at all, count ~36% of the
// LDS-active cycles as conflicts)
__device__ __forceinline__ int swz(int r) { return (r >> 1) & 3; }

// Write the 16 x 16 accumulator block whose first row / column are
// (i0 + r0, j0 + c0), from lane (fr, fc).  With SYM only elements on or
// above the diagonal are written, each with its mirror (the tiles of a
// symmetric product cover every such element exactly once).
template <bool SYM>
__device__ __forceinline__ void epilogue_split_at(const SplitArgs &p, long bz, int i0, int j0,
                                                  int r0, int c0, int fr, int fc,
                                                  const f32x4 &acc) {
    const int ld = p.ld;
    uint16_t *C = p.C ? p.C + bz * p.sC : nullptr;
    double *Cd = p.Cd ? p.Cd + bz * p.sC : nullptr;
    const uint16_t *X = p.X ? p.X + bz * p.sX : nullptr;
    const double *Xd = p.Xd ? p.Xd + bz * p.sX : nullptr;
    const double *Xd2 = p.Xd2 ? p.Xd2 + bz * p.sX : nullptr;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = i0 + r0 + 4 * fr + r;
        const int col = j0 + c0 + fc;
        const long o = (long)row * ld + col;
        if (SYM && row > col) continue;
        double val = p.alpha * (double)acc[r];
        if (X) val += p.beta * (double)get_split(X, p.pl, o);
        if (Xd) val += p.beta * Xd[o];
        if (Xd2) val += p.beta2 * Xd2[o];
        if (row == col) val += p.gamma;
        const long ot = (long)col * ld + row;
        if (C) {
            put_split(C, p.pl, o, (float)val);
            if (SYM && row != col) put_split(C, p.pl, ot, (float)val);
        }
        if (Cd) {
            Cd[o] = val;
            if (SYM && row != col) Cd[ot] = val;
        }
    }
}
template <bool SYM>
__device__ __forceinline__ void epilogue_split_block(const SplitArgs &p, long bz, int ti,
                                                     int tj, int r0, int c0, int fr, int fc,
                                                     const f32x4 &acc) {
    epilogue_split_at<SYM>(p, bz, ti * GT, tj * GT, r0, c0, fr, fc, acc);
}

// 512 threads = 8 waves in 2 (rows) x 4 (columns), 64 x 32 per wave
// (4 x 2 accumulator blocks): two workgroups per CU put four waves on every
// SIMD, which the bf16 matrix-core instruction needs to issue at full rate
// (two waves per SIMD reach less than half of it).
constexpr int BS_T = 512;

template <bool SYM, bool HI>
__global__ __launch_bounds__(BS_T, 2) void gemm_bs_kernel(SplitArgs p, int ntiles, int nfull,
                                                       int nsplit, int per_xcd) {
    if (p.skip && *p.skip) return;   // skipped launch (device flag)
    using acc_t = f32x4;
    // [buffer][hi, lo][row][16-byte chunk]: 32 k per row
    __shared__ __attribute__((aligned(16))) u32x4 As[2][2][GT][4];
    __shared__ __attribute__((aligned(16))) u32x4 Bs[2][2][GT][4];

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
    const uint16_t *A0 = p.A0 + bz * p.sA0, *B0 = p.B0 + bz * p.sB0;
    const uint16_t *A1 = p.A1 ? p.A1 + bz * p.sA1 : nullptr;
    const uint16_t *B1 = p.B1 ? p.B1 + bz * p.sB1 : nullptr;
    const int ld = p.ld;
    const long pl = p.pl;
    const int i0 = ti * GT, j0 = tj * GT;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wr = wid >> 2, wc = wid & 3;

    acc_t acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[a][c] = acc_t{0, 0, 0, 0};

    const int nk1 = p.n / B3K;
    const int nktot = A1 ? 2 * nk1 : nk1;
    const int kt0 = (int)((long)nktot * split / ns);
    const int kt1 = (int)((long)nktot * (split + 1) / ns);

    // chunk v of thread tid: plane (idx >> 9), row ((idx >> 2) & 127),
    // chunk (idx & 3) of the 128 x 32 k-tile, idx = tid + 512 v (HI: the
    // hi plane only, v = 0)
    constexpr int NV = HI ? 1 : 2;
    u32x4 ra[NV], rb[NV];
    auto gload = [&](int kt) {
        const bool second = kt >= nk1;
        const uint16_t *Ap = second ? A1 : A0;
        const uint16_t *Bp = second ? B1 : B0;
        const int kb = (second ? kt - nk1 : kt) * B3K;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int idx = tid + BS_T * v;
            const int pln = idx >> 9, row = (idx >> 2) & 127, ch = idx & 3;
            const long off = pln * pl + kb + 8 * ch;
            ra[v] = *reinterpret_cast<const u32x4 *>(Ap + off + (long)(i0 + row) * ld);
            rb[v] = *reinterpret_cast<const u32x4 *>(Bp + off + (long)(j0 + row) * ld);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int idx = tid + BS_T * v;
            const int pln = idx >> 9, row = (idx >> 2) & 127, ch = idx & 3;
            As[buf][pln][row][ch ^ swz(row)] = ra[v];
            Bs[buf][pln][row][ch ^ swz(row)] = rb[v];
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
        bf16x8 ah[4], al[4], bh[2], bl[2];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = wr * 64 + q * 16 + fc, c = fr ^ swz(r);
            ah[q] = __builtin_bit_cast(bf16x8, As[buf][0][r][c]);
            if (!HI) al[q] = __builtin_bit_cast(bf16x8, As[buf][1][r][c]);
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int r = wc * 32 + q * 16 + fc, c = fr ^ swz(r);
            bh[q] = __builtin_bit_cast(bf16x8, Bs[buf][0][r][c]);
            if (!HI) bl[q] = __builtin_bit_cast(bf16x8, Bs[buf][1][r][c]);
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                if (!HI) {
                    acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[x], bh[y], acc[x][y], 0, 0, 0);
                    acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[x], bl[y], acc[x][y], 0, 0, 0);
                }
                acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[x], bh[y], acc[x][y], 0, 0, 0);
            }
        if (kt + 1 < kt1) sstore(buf ^ 1);
        __syncthreads();
    }

    if (part) {
        // block g = 2x + y of thread tid at [(g * 512 + tid) * 4]
        acc_t *wp = reinterpret_cast<acc_t *>(p.ws + ((long)bz * ntail * nsplit + w) * (GT * GT)) + tid;
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) wp[(x * 2 + y) * BS_T] = acc[x][y];
        return;
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
            epilogue_split_block<SYM>(p, bz, ti, tj, wr * 64 + x * 16, wc * 32 + y * 16, fr, fc,
                                      acc[x][y]);
}

// One workgroup per (tail tile, block g): thread tid sums the vectors its
// counterpart wrote for block g in every partial.
template <bool SYM>
__global__ __launch_bounds__(BS_T) void gemm_bs_fixup_kernel(SplitArgs p, int ntiles, int nfull,
                                                             int nsplit) {
    if (p.skip && *p.skip) return;   // skipped launch (device flag)
    const int ntail = ntiles - nfull;
    const int u = nfull + blockIdx.x;
    const int g = blockIdx.y, x = g >> 1, y = g & 1;
    const long bz = blockIdx.z;
    const int nt = p.n / GT;
    int ti, tj;
    tile_of<SYM>(u, nt, ti, tj);
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wr = wid >> 2, wc = wid & 3, fr = lane >> 4, fc = lane & 15;
    f32x4 acc = f32x4{0, 0, 0, 0};
    const f32x4 *wp = reinterpret_cast<const f32x4 *>(
                          p.ws + ((long)bz * ntail * nsplit + (long)blockIdx.x * nsplit) *
                                     (GT * GT)) + g * BS_T + tid;
    for (int s = 0; s < nsplit; ++s) acc += wp[(long)s * (GT * GT / 4)];
    epilogue_split_block<SYM>(p, bz, ti, tj, wr * 64 + x * 16, wc * 32 + y * 16, fr, fc, acc);
}

// ---------------------------------------------------------------------------
// Wide variant: 256 x 128 workgroup tile, one workgroup of 8 waves per CU
// (two per SIMD), used when n % 256 == 0.  Waves in 4 rows x 2 columns of
// 64 x 64 (4 x 4 accumulator blocks, 48 MFMAs per 32-wide k-tile).  The
// operand tiles go from global memory straight into LDS
// (global_load_lds_dwordx4: lane l of a wave writes the 16 bytes it fetched
// at M0 + 16 l, so each load instruction of a wave fills one contiguous 1 KB
// run of LDS): no staging registers and no LDS store instructions.  The
// swizzle of a row's four 16-byte chunks is applied on the fetch side (LDS
// slot s of row r receives chunk s ^ swz(r)).  Three k-tile buffers of
// 48 KB: during step t the waves run the MFMAs of k-tile t from registers,
// read the fragments of t + 1 from LDS into a second register set and issue
// the loads of t + 3 into the buffer t vacated; a step ends when this wave's
// loads of t + 2 have landed (each wave waits for its own, then the barrier
// makes all of them visible), so a load has two steps to arrive.  The
// barrier is a bare s_barrier with explicit waits: the workgroup fence of
// __syncthreads would also wait for the loads of t + 3.  Tiles of a
// symmetric product: in 256-row block bi, the 128-column blocks bj >= 2 bi.
// ---------------------------------------------------------------------------
constexpr int BW_NTH = 512;
constexpr int BW_M = 256;
// smallest n for the 256 x 128 kernel: below it the few tiles of a product
// leave its three-deep k pipeline latency-bound, and the 128 x 128 kernel
// is faster (a 64-atom x 4-orbital step: 3.64 -> 2.87 ms; N = 512: -6%)
constexpr int BW_MIN_N = 1024;
constexpr int BW_TILE = BW_M * GT;     // elements of one tile

inline int wide_tiles(int n, bool sym) {
    const int nbi = n / BW_M, nbj = n / GT;
    if (!sym) return nbi * nbj;
    int t = 0;
    for (int bi = 0; bi < nbi; ++bi) t += nbj - 2 * bi;
    return t;
}
// Tile order: groups of BW_GM 256-row blocks, column by column inside a
// group, so that the workgroups an XCD runs at once (a contiguous range of
// units) share few row and column panels in its L2.
constexpr int BW_GM = 4;
template <bool SYM>
__device__ __forceinline__ void tilew_of(int u, int nbj, int &bi, int &bj) {
    const int nbi = nbj / 2;
    int bi0 = 0, start = 0, gm = 0;
    for (;;) {
        gm = min(BW_GM, nbi - bi0);
        int cnt = gm * nbj;
        if (SYM) cnt -= gm * (2 * bi0 + gm - 1);     // rows keep bj >= 2 bi
        if (u < start + cnt) break;
        start += cnt;
        bi0 += BW_GM;
    }
    int v = u - start;
    if (!SYM) {
        bi = bi0 + v % gm;
        bj = v / gm;
        return;
    }
    for (int c = 2 * bi0;; ++c) {
        const int h = min(gm, c / 2 - bi0 + 1);
        if (v < h) {
            bi = bi0 + v;
            bj = c;
            return;
        }
        v -= h;
    }
}

struct BwFrag {
    bf16x8 ah[4], al[4], bh[4], bl[4];
};

// Epilogue of a whole 256 x 128 tile of a symmetric product with a split
// output.  Every element on or above the diagonal is written from the
// accumulator layout as in epilogue_split_at, and its FP32 value replaces
// the accumulator.  The mirror images, which written the same way would be
// 2-byte stores 2 ld bytes apart, then go through LDS one 128-row band at a
// time (stg: 128 x 128 floats in the tile's k-tile buffers, free after the
// k loop; element (r, c) at r * 128 + (c ^ (r & 31)) to spread the banks)
// and are written as rows of the transposed band, four consecutive elements
// per lane, one 8-byte store per plane.  The mirror gets the same FP32
// value, so the output is the same bit for bit.  Called by every thread of
// the workgroup (it has barriers).
__device__ __forceinline__ void bw_sym_epilogue(const SplitArgs &p, long bz, int i0, int j0,
                                                int wr, int wc, int fr, int fc, int tid,
                                                f32x4 (&acc)[4][4], float *stg) {
    const int ld = p.ld;
    uint16_t *C = p.C + bz * p.sC;
    const uint16_t *X = p.X ? p.X + bz * p.sX : nullptr;
    const double *Xd = p.Xd ? p.Xd + bz * p.sX : nullptr;
    const double *Xd2 = p.Xd2 ? p.Xd2 + bz * p.sX : nullptr;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = i0 + wr * 64 + x * 16 + 4 * fr + r;
                const int col = j0 + wc * 64 + y * 16 + fc;
                float v = 0.f;
                if (row <= col) {
                    const long o = (long)row * ld + col;
                    double val = p.alpha * (double)acc[x][y][r];
                    if (X) val += p.beta * (double)get_split(X, p.pl, o);
                    if (Xd) val += p.beta * Xd[o];
                    if (Xd2) val += p.beta2 * Xd2[o];
                    if (row == col) val += p.gamma;
                    v = (float)val;
                    put_split(C, p.pl, o, v);
                }
                acc[x][y][r] = v;
            }
    const int wrf = __builtin_amdgcn_readfirstlane(wr);
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
        if ((wrf >> 1) == h) {             // the band's two wave rows stage it
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int rl = (wr & 1) * 64 + x * 16 + 4 * fr + r;
                        const int cl = wc * 64 + y * 16 + fc;
                        stg[rl * 128 + (cl ^ (rl & 31))] = acc[x][y][r];
                    }
        }
        __syncthreads();
        // output rows j0 + c, columns i0 + 128 h + r4 .. + 3; element k is
        // the mirror of (i0 + 128 h + r4 + k, j0 + c), written when that
        // lies strictly above the diagonal
#pragma unroll
        for (int it = 0; it < 8; ++it) {
            const int e = it * 512 + tid;
            const int c = e >> 5, r4 = (e & 31) * 4;
            const int orow = j0 + c, ocol = i0 + 128 * h + r4;
            float v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int rl = r4 + k;
                v[k] = stg[rl * 128 + (c ^ (rl & 31))];
            }
            const long o = (long)orow * ld + ocol;
            if (ocol + 3 < orow) {
                unsigned h0, l0, h1, l1;
                split_pair(v[0], v[1], h0, l0);
                split_pair(v[2], v[3], h1, l1);
                *reinterpret_cast<u32x2 *>(C + o) = u32x2{h0, h1};
                *reinterpret_cast<u32x2 *>(C + o + p.pl) = u32x2{l0, l1};
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (ocol + k < orow) put_split(C, p.pl, o + k, v[k]);
            }
        }
        __syncthreads();
    }
}

struct BwTile {
    u32x4 a[2][BW_M][4];   // A planes (hi, lo): 256 rows x 32 k
    u32x4 b[2][GT][4];     // B planes: 128 rows x 32 k
};
constexpr int BW_NBUF = 3;

// s_waitcnt vmcnt(VM) lgkmcnt(0) (expcnt not waited on)
template <int VM> __device__ __forceinline__ void wait_vm_lgkm0() {
    static_assert(VM >= 0 && VM < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((VM & 15) | ((VM >> 4) << 14) | (7 << 4));
}
// barrier without a memory fence; the empty asm statements keep the
// compiler from moving LDS accesses across it
__device__ __forceinline__ void bare_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

template <bool SYM, bool HI>
__global__ __launch_bounds__(BW_NTH, 1) void gemm_bw_kernel(SplitArgs p, int ntiles, int nfull,
                                                          int nsplit, int per_xcd) {
    if (p.skip && *p.skip) return;   // skipped launch (device flag)
    using acc_t = f32x4;
    constexpr int NTH = BW_NTH;
    constexpr int NPL = HI ? 1 : 2;                    // planes loaded (HI: hi only)
    constexpr int NA = NPL * 1024 / NTH, NB = NPL * 512 / NTH;   // loads per thread per k-tile
    constexpr int ND = NA + NB;
    __shared__ __attribute__((aligned(1024))) BwTile Lt[BW_NBUF];

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
    int bi, bj;
    tilew_of<SYM>(u, p.n / GT, bi, bj);
    const long bz = blockIdx.z;
    const uint16_t *A0 = p.A0 + bz * p.sA0, *B0 = p.B0 + bz * p.sB0;
    const uint16_t *A1 = p.A1 ? p.A1 + bz * p.sA1 : nullptr;
    const uint16_t *B1 = p.B1 ? p.B1 + bz * p.sB1 : nullptr;
    const int ld = p.ld;
    const long pl = p.pl;
    const int i0 = bi * BW_M, j0 = bj * GT;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wid >> 1, wc = wid & 1;
    const int fr = lane >> 4, fc = lane & 15;

    acc_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = acc_t{0, 0, 0, 0};

    const int nk1 = p.n / B3K;
    const int nktot = A1 ? 2 * nk1 : nk1;
    const int kt0 = (int)((long)nktot * split / ns);
    const int kt1 = (int)((long)nktot * (split + 1) / ns);

    // k-tile kt into buffer buf: load v of wave wid fills the 1 KB run
    // (8 v + wid) of the A planes (v < NA) or of the B planes
    auto dload = [&](int kt, int buf) {
        const bool second = kt >= nk1;
        const uint16_t *Ap = second ? A1 : A0;
        const uint16_t *Bp = second ? B1 : B0;
        const int kb = (second ? kt - nk1 : kt) * B3K;
        char *la = reinterpret_cast<char *>(&Lt[buf].a[0][0][0]);
        char *lb = reinterpret_cast<char *>(&Lt[buf].b[0][0][0]);
#pragma unroll
        for (int v = 0; v < NA; ++v) {
            const int idx = tid + NTH * v;
            const int pln = idx >> 10, row = (idx >> 2) & (BW_M - 1);
            const int ch = (idx & 3) ^ swz(row);
            __builtin_amdgcn_global_load_lds(
                (const void __attribute__((address_space(1))) *)(Ap + pln * pl + kb + 8 * ch +
                                                                (long)(i0 + row) * ld),
                (void __attribute__((address_space(3))) *)(la + (8 * v + wid) * 1024), 16, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < NB; ++v) {
            const int idx = tid + NTH * v;
            const int pln = idx >> 9, row = (idx >> 2) & (GT - 1);
            const int ch = (idx & 3) ^ swz(row);
            __builtin_amdgcn_global_load_lds(
                (const void __attribute__((address_space(1))) *)(Bp + pln * pl + kb + 8 * ch +
                                                                (long)(j0 + row) * ld),
                (void __attribute__((address_space(3))) *)(lb + (8 * v + wid) * 1024), 16, 0, 0);
        }
    };
    auto fread = [&](int buf, BwFrag &f) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = wr * 64 + q * 16 + fc, c = fr ^ swz(r);
            f.ah[q] = __builtin_bit_cast(bf16x8, Lt[buf].a[0][r][c]);
            if (!HI) f.al[q] = __builtin_bit_cast(bf16x8, Lt[buf].a[1][r][c]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = wc * 64 + q * 16 + fc, c = fr ^ swz(r);
            f.bh[q] = __builtin_bit_cast(bf16x8, Lt[buf].b[0][r][c]);
            if (!HI) f.bl[q] = __builtin_bit_cast(bf16x8, Lt[buf].b[1][r][c]);
        }
    };
    auto mfma = [&](const bf16x8 (&a)[4], const bf16x8 (&bb)[4]) {
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y)
                acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[x], bb[y], acc[x][y], 0, 0, 0);
    };
    // One step, branch-free: near the end of the range
    // the loads repeat the last k-tile into the vacated buffer and the
    // fragment read takes stale data that is never used.
    constexpr int NMF = HI ? 16 : 48, NRD = HI ? 8 : 16, MPR = HI ? 1 : 2;
    auto step = [&](int kt, const BwFrag &cur, BwFrag &nxt) {
        const int r = kt - kt0;
        fread((r + 1) % BW_NBUF, nxt);
        if (!HI) {
            mfma(cur.al, cur.bh);
            mfma(cur.ah, cur.bl);
        }
        dload(min(kt + 3, kt1 - 1), r % BW_NBUF);   // every wave read t's fragments before the last barrier
        mfma(cur.ah, cur.bh);
#pragma unroll
        for (int i = 0; i < NRD; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // LDS read
            __builtin_amdgcn_sched_group_barrier(0x008, MPR, 0); // MFMA
        }
#pragma unroll
        for (int i = 0; i < ND; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);   // direct load
            __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);   // MFMA
        }
        __builtin_amdgcn_sched_group_barrier(0x008, NMF - NRD * MPR - 2 * ND, 0);
        __builtin_amdgcn_sched_barrier(0);
        wait_vm_lgkm0<ND>();        // this wave's loads of t + 2 landed, t + 1 read
        bare_barrier();
    };

    BwFrag f0, f1;
    dload(kt0, 0);
    dload(min(kt0 + 1, kt1 - 1), 1);
    dload(min(kt0 + 2, kt1 - 1), 2);
    wait_vm_lgkm0<2 * ND>();        // k-tile kt0
    bare_barrier();
    fread(0, f0);
    wait_vm_lgkm0<ND>();            // k-tile kt0 + 1; f0 read
    bare_barrier();
    for (int kt = kt0; kt < kt1; kt += 2) {
        step(kt, f0, f1);
        if (kt + 1 < kt1) step(kt + 1, f1, f0);
    }
    wait_vm_lgkm0<0>();             // no load may land in the staging area below
    bare_barrier();

    if (part) {
        acc_t *wp = reinterpret_cast<acc_t *>(p.ws + ((long)bz * ntail * nsplit + w) * BW_TILE) + tid;
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) wp[(x * 4 + y) * NTH] = acc[x][y];
        return;
    }
    if constexpr (SYM) {
        if (p.C && !p.Cd) {
            bw_sym_epilogue(p, bz, i0, j0, wr, wc, fr, fc, tid, acc,
                            reinterpret_cast<float *>(&Lt[0].a[0][0][0]));
            return;
        }
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
            epilogue_split_at<SYM>(p, bz, i0, j0, wr * 64 + x * 16, wc * 64 + y * 16, fr, fc,
                                   acc[x][y]);
}

// One 256-thread workgroup per (tail tile, block g, half of the product's
// threads): sums the vectors its counterparts wrote in every partial.
// grid.y = 16 blocks x 2 halves.
template <bool SYM>
__global__ __launch_bounds__(256) void gemm_bw_fixup_kernel(SplitArgs p, int ntiles, int nfull,
                                                            int nsplit) {
    if (p.skip && *p.skip) return;   // skipped launch (device flag)
    constexpr int NTH = BW_NTH;
    const int ntail = ntiles - nfull;
    const int u = nfull + blockIdx.x;
    const int g = blockIdx.y >> 1, x = g >> 2, y = g & 3;
    const long bz = blockIdx.z;
    int bi, bj;
    tilew_of<SYM>(u, p.n / GT, bi, bj);
    const int tid = (blockIdx.y & 1) * 256 + threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wr = wid >> 1, wc = wid & 1, fr = lane >> 4, fc = lane & 15;
    f32x4 acc = f32x4{0, 0, 0, 0};
    const f32x4 *wp = reinterpret_cast<const f32x4 *>(
                          p.ws + ((long)bz * ntail * nsplit + (long)blockIdx.x * nsplit) *
                                     BW_TILE) + g * NTH + tid;
    for (int s = 0; s < nsplit; ++s) acc += wp[(long)s * (BW_TILE / 4)];
    epilogue_split_at<SYM>(p, bz, bi * BW_M, bj * GT, wr * 64 + x * 16, wc * 64 + y * 16, fr, fc,
                           acc);
}

inline long split_bs_ws_elems(int n, bool sym, int dual, long batch) {
    long e = split_ws_elems<float>(n, sym, dual, batch);
    if (n % BW_M == 0 && n >= BW_MIN_N) {
        const int nt = wide_tiles(n, sym);
        const Sched s = schedule<float>(nt, (n / B3K) * (dual ? 2 : 1), batch, 1);
        e = std::max(e, (long)(nt - s.nfull) * s.nsplit * batch * BW_TILE);
    }
    return e;
}

inline void gemm_split(const SplitArgs &a, bool sym, hipStream_t st) {
    if (a.n % GT != 0 || a.ld % 8 != 0 || a.pl % 8 != 0)
        throw InvalidArg("gemm_split: n must be a multiple of 128");
    if (!a.C && !a.Cd) throw InvalidArg("gemm_split: no output");
    if (a.n % BW_M == 0 && a.n >= BW_MIN_N) {   // 256 x 128 tiles, one workgroup per CU
        const int ntiles = wide_tiles(a.n, sym);
        const int nkt = (a.n / B3K) * (a.A1 ? 2 : 1);
        Sched s = a.ws ? schedule<float>(ntiles, nkt, a.batch, 1) : Sched{ntiles, 1};
        if (s.nsplit > 1 && (long)(ntiles - s.nfull) * s.nsplit * a.batch * BW_TILE > a.ws_elems)
            s = Sched{ntiles, 1};
        const int nfull_pad = ((s.nfull + NXCD - 1) / NXCD) * NXCD;
        const int tail_units = (ntiles - s.nfull) * s.nsplit;
        const int per = (tail_units + NXCD - 1) / NXCD;
        dim3 grid(nfull_pad + per * NXCD, 1, a.batch);
        auto kern = sym ? (a.hi_only ? gemm_bw_kernel<true, true> : gemm_bw_kernel<true, false>)
                        : (a.hi_only ? gemm_bw_kernel<false, true> : gemm_bw_kernel<false, false>);
        hipLaunchKernelGGL(kern, grid, dim3(BW_NTH), 0, st, a, ntiles, s.nfull, s.nsplit, per);
        XL_LAUNCH_CHECK();
        if (s.nfull < ntiles) {
            dim3 g2(ntiles - s.nfull, 32, a.batch);   // 16 blocks x 2 halves
            if (sym)
                hipLaunchKernelGGL((gemm_bw_fixup_kernel<true>), g2, dim3(256), 0, st, a,
                                   ntiles, s.nfull, s.nsplit);
            else
                hipLaunchKernelGGL((gemm_bw_fixup_kernel<false>), g2, dim3(256), 0, st, a,
                                   ntiles, s.nfull, s.nsplit);
            XL_LAUNCH_CHECK();
        }
        return;
    }
    const int nt = a.n / GT;
    const int ntiles = sym ? nt * (nt + 1) / 2 : nt * nt;
    const int nkt = (a.n / B3K) * (a.A1 ? 2 : 1);
    Sched s = a.ws ? schedule<float>(ntiles, nkt, a.batch) : Sched{ntiles, 1};
    if (s.nsplit > 1 && (long)(ntiles - s.nfull) * s.nsplit * a.batch * GT * GT > a.ws_elems)
        s = Sched{ntiles, 1};
    const int nfull_pad = ((s.nfull + NXCD - 1) / NXCD) * NXCD;
    const int tail_units = (ntiles - s.nfull) * s.nsplit;
    const int per = (tail_units + NXCD - 1) / NXCD;
    dim3 grid(nfull_pad + per * NXCD, 1, a.batch);
    auto kern = sym ? (a.hi_only ? gemm_bs_kernel<true, true> : gemm_bs_kernel<true, false>)
                    : (a.hi_only ? gemm_bs_kernel<false, true> : gemm_bs_kernel<false, false>);
    hipLaunchKernelGGL(kern, grid, dim3(BS_T), 0, st, a, ntiles, s.nfull, s.nsplit, per);
    XL_LAUNCH_CHECK();
    if (s.nfull < ntiles) {
        dim3 g2(ntiles - s.nfull, 8, a.batch);
        if (sym)
            hipLaunchKernelGGL((gemm_bs_fixup_kernel<true>), g2, dim3(BS_T), 0, st, a, ntiles,
                               s.nfull, s.nsplit);
        else
            hipLaunchKernelGGL((gemm_bs_fixup_kernel<false>), g2, dim3(BS_T), 0, st, a, ntiles,
                               s.nfull, s.nsplit);
        XL_LAUNCH_CHECK();
    }
}

}  // namespace xl
