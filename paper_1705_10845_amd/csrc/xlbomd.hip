// Host orchestration and C ABI of the XL-BOMD library (gfx950).
//
// Per step (Eqs. 22-23): half kick + drift of the nuclei, the dissipative
// Verlet update of n, the one-shot electronic solve of the linearised
// functional at the new (R, n), Hellmann-Feynman forces at fixed n, the
// low-rank kernel K_m and K_m r for the next n update, the second half kick.
//
// Electronic solve without diagonalisation.  With X = beta (H - mu I), the
// occupation f(x) = 1/(1+e^x) = (1 - tanh(x/2))/2.  tanh doubles its
// argument under t -> 2t / (1 + t^2), so starting from t0 ~ tanh(x/2^(L+1))
// and applying the map L times gives tanh(x/2); D = 2f(H) = I - t_L.  In
// matrix form with Z = t/2 every level is
//     A_k = I + 4 Z_k^2,   Y_k = A_k^-1,   Z_{k+1} = 2 Y_k Z_k,
// D = I - 2 Z_L.  A_k has its spectrum in [1, 1 + t_k,max^2] within [1, 2],
// so Y_k follows from a fixed Chebyshev-optimal linear guess plus a few
// Newton-Schulz steps Y <- Y (2I - A Y), the number of steps chosen per level
// from the known spectral bound.  The seed t0 = y - y^3/3 + 2 y^5/15,
// y = X/2^(L+1), is tanh(y) to O(y^7), which lets L be well under half of
// what t0 = y needs for the same truncation error.  All products are dense
// symmetric GEMMs on MFMA (FP64 or FP32).  On the split path (MIXED_BF16X3)
// the inverse of each level runs as split bf16x3 products and Z_{k+1} is
// then corrected with the FP64 residual 2 Z_k - A_k Z_{k+1}: only A_k, the
// residual, the seed, Z_L^2 and D stay FP64 products.  The chemical
// potential follows in FP64 from the root of the quadratic model of Tr D
// in mu (rerun of the expansion if beta |dmu| is above a threshold), and D
// is corrected to second order with dD/dmu = (beta/2)(I - 4 Z_L^2) and
// d2D/dmu2 = beta^2 (Z_L - 4 Z_L^3).
//
// Response (Section V.B).  Differentiating the same recursion along a
// perturbation H1 = diag(Gamma v) gives, with Z'_0 from the seed,
//     A'_k = 4 (Z_k Z'_k + Z'_k Z_k),
//     Z'_{k+1} = Y_k (2 Z'_k - A'_k Z_{k+1}),
// and D' = -2 Z'_L, made canonical (fixed electron number) by mu'.
#include "../../include/xlbomd.h"
#include "common.hpp"
#include "gemm.hpp"
#include "gemm_split.hpp"
#include "model.hpp"
#include "chol.hpp"
#include "planned.hpp"
#include "overlap.hpp"

#include <algorithm>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <atomic>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

using namespace xl;

namespace {

thread_local std::string g_err;

bool debug() {
    static const bool on = std::getenv("XLBOMD_DEBUG") != nullptr;
    return on;
}

// A named ROCTX range over a phase of the host orchestration (visible with
// rocprofv3 --marker-trace; a no-op call when no tool is attached).  The
// range covers the host's enqueueing and its synchronisations, not device
// time that runs on after the phase returns.
struct Phase {
    explicit Phase(const char *name) { roctxRangePush(name); }
    ~Phase() { roctxRangePop(); }
    Phase(const Phase &) = delete;
    Phase &operator=(const Phase &) = delete;
};

// Table I: kappa, alpha and c_0..c_K of the dissipative term of Eq. 23.
struct DampRow {
    double kappa, alpha;
    int nc;
    double c[8];
};
const DampRow kDamp[3] = {
    {1.82, 0.018, 6, {-6, 14, -8, -3, 4, -1}},
    {1.84, 0.0055, 7, {-14, 36, -27, -2, 12, -6, 1}},
    {1.86, 0.0016, 8, {-36, 99, -88, 11, 32, -25, 8, -1}},
};

template <typename T> T *dalloc(size_t n) {
    void *p = nullptr;
    if (n == 0) n = 1;
    if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        throw NoMem("device allocation of " + std::to_string(n * sizeof(T)) + " bytes failed");
    }
    return (T *)p;
}

// Device buffers of one system, returned at destruction to the allocator
// that gave them (the caller's xlbomd_allocator, else hipFree).
struct DevFree {
    std::vector<void *> ptrs;
    xlbomd_allocator al{};
    ~DevFree() {
        for (void *p : ptrs) {
            if (al.free) al.free(p, al.ctx);
            else (void)hipFree(p);
        }
    }
};

// Fermi function written without overflow
double fermi(double x) {
    if (x > 0) {
        const double e = std::exp(-x);
        return e / (1.0 + e);
    }
    return 1.0 / (1.0 + std::exp(x));
}

// The scalar map the matrix expansion applies to each eigenvalue.
double foe_scalar(double x, int L) {
    const double y = std::ldexp(x, -(L + 1));
    const double y2 = y * y;
    double t = y * (1.0 - y2 / 3.0 + 2.0 * y2 * y2 / 15.0);   // tanh(y) to O(y^7)
    for (int k = 0; k < L; ++k) t = 2.0 * t / (1.0 + t * t);
    return 0.5 * (1.0 - t);
}

// Extreme eigenvalues of the symmetric tridiagonal matrix with diagonal
// a[0..m) and off-diagonal b[0..m-1), by Sturm-count bisection.
void tridiag_extremes(const double *a, const double *b, int m, double &lo, double &hi) {
    double gl = 1e300, gh = -1e300;
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
        gl = std::min(gl, a[i] - r);
        gh = std::max(gh, a[i] + r);
    }
    auto below = [&](double x) {    // number of eigenvalues < x
        int c = 0;
        double q = 1.0;
        for (int i = 0; i < m; ++i) {
            q = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / q : 0.0);
            if (q == 0.0) q = -1e-300;
            if (q < 0.0) ++c;
        }
        return c;
    };
    auto kth = [&](int k) {         // k-th smallest eigenvalue (0-based)
        double l = gl, h = gh;
        for (int it = 0; it < 200 && h - l > 1e-13 * (std::fabs(l) + std::fabs(h) + 1e-300); ++it) {
            const double x = 0.5 * (l + h);
            if (below(x) > k) h = x; else l = x;
        }
        return 0.5 * (l + h);
    };
    lo = kth(0);
    hi = kth(m - 1);
}

// Largest deviation of the L-level expansion from the Fermi function on
// [-xmax, xmax] (a uniform grid plus a dense one near the Fermi level).
double level_error(double xmax, int L) {
    double err = 0.0;
    const int G = 2000;
    for (int g = 0; g <= G; ++g) {
        const double x = -xmax + 2.0 * xmax * g / G;
        err = std::max(err, std::fabs(foe_scalar(x, L) - fermi(x)));
    }
    for (int g = 0; g <= 400; ++g) {
        const double x = -12.0 + 24.0 * g / 400.0;
        if (std::fabs(x) <= xmax) err = std::max(err, std::fabs(foe_scalar(x, L) - fermi(x)));
    }
    return err;
}

// Largest xmax (at most 2^(L+1), i.e. |y| <= 1) for which L levels stay
// within tol.  The deviation over [-xmax, xmax] does not decrease with xmax,
// so the reach is found once per (L, tol) by bisection and kept.
double level_reach(int L, double tol) {
    static std::mutex mu;
    static std::map<std::pair<int, double>, double> known;
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_pair(L, tol);
    const auto it = known.find(key);
    if (it != known.end()) return it->second;
    double lo = 0.0, hi = std::ldexp(1.0, L + 1);
    if (level_error(hi, L) > tol) {
        for (int i = 0; i < 60 && hi - lo > 1e-12 * hi; ++i) {
            const double m = 0.5 * (lo + hi);
            if (level_error(m, L) <= tol) lo = m; else hi = m;
        }
        hi = lo;
    }
    known.emplace(key, hi);
    return hi;
}

// Smallest L whose expansion keeps |y| <= 1 (where the quintic seed is
// increasing and below 1) and stays within `tol` of the Fermi function on
// [-xmax, xmax].
int choose_levels(double xmax, double tol) {
    for (int L = 1; L <= 40; ++L)
        if (xmax <= level_reach(L, tol)) return L;
    return 40;
}

}  // namespace

// ---------------------------------------------------------------------------
// Precision-independent state of one system
// ---------------------------------------------------------------------------
struct SysBase {
    virtual ~SysBase() = default;
    xlbomd_desc d{};
    // RMS residual tolerance of the SCF loop in progress (0: none); the split
    // path's expansion refines twice per level below 1e-8 (once otherwise)
    double scf_need = 0.0;
    struct ScfNeed {
        double &ref;
        ScfNeed(double &r, double v) : ref(r) { ref = v; }
        ~ScfNeed() { ref = 0.0; }
    };
    int nat = 0, no = 0, N = 0, Np = 0;
    double beta = 0.0, zc = 0.0;
    hipStream_t st = nullptr;
    bool own_stream = false;
    DevFree mem;
    // n elements of device memory owned by the system: from the caller's
    // allocator when the descriptor gives one, else hipMalloc
    // a captured step's launches are valid while no buffer has been
    // allocated or given back since the capture
    long alloc_epoch = 0;
    bool capturing = false;      // a planned step is being captured into a graph
    template <typename T> T *dev(size_t n) {
        if (capturing) throw StateError("device allocation during graph capture");
        ++alloc_epoch;
        if (!mem.al.alloc) {
            T *p = dalloc<T>(n);
            mem.ptrs.push_back(p);
            return p;
        }
        const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
        void *p = mem.al.alloc(bytes, mem.al.ctx);
        if (!p) throw NoMem("allocator returned no memory for " + std::to_string(bytes) + " bytes");
        if (reinterpret_cast<uintptr_t>(p) % 256)
            throw InvalidArg("allocator memory must be 256-byte aligned");
        mem.ptrs.push_back(p);
        return (T *)p;
    }
    // gives a buffer from dev() back before destruction (a grown buffer
    // replaces it), once the stream has drained so that no queued work
    // still uses it; the caller drops its pointer
    void release(void *p) {
        if (!p) return;
        if (capturing) throw StateError("buffer release during graph capture");
        ++alloc_epoch;
        sync();
        const auto it = std::find(mem.ptrs.begin(), mem.ptrs.end(), p);
        if (it == mem.ptrs.end()) return;
        mem.ptrs.erase(it);
        if (mem.al.free) mem.al.free(p, mem.al.ctx);
        else (void)hipFree(p);
    }
    ModelDev md{};

    // device arrays (FP64)
    double *pos = nullptr, *vel = nullptr, *mass = nullptr, *force = nullptr;
    double *onsite = nullptr, *jit = nullptr, *hop = nullptr, *U = nullptr;
    double *hist = nullptr, *kr = nullptr, *q = nullptr, *r = nullptr;
    double *ncur = nullptr, *vpot = nullptr, *glo = nullptr, *ghi = nullptr;
    double *g = nullptr, *epart = nullptr, *scal = nullptr, *cvec = nullptr;
    double *V = nullptr, *W = nullptr, *Vprev = nullptr, *vtmp = nullptr;
    double *qp = nullptr, *hb = nullptr, *ub = nullptr, *part = nullptr, *vin = nullptr;
    double *hscal = nullptr;   // pinned host scalars
    // non-orthogonal basis (overlap block given): the overlap block, and
    // every atom's neighbour count set to -1 (dense rows) for the Lanczos
    // matvecs on the dense H' = X H X
    bool ov = false;
    double *sblk = nullptr;
    int *nbc_dense = nullptr;
    int head = 0;              // ring index of n(t) in hist
    int mcap = 0, rank_built = 0, rank_prev = 0, step_no = 0;
    // columns of V, W from the last rebuild, and on-the-fly directions
    // appended after them since (rank_built = rank_rb + otf_count)
    int rank_rb = 0, otf_count = 0;
    int bcap = 0;              // response batch capacity
    double *fscr = nullptr;    // forces of an energy evaluation (the MD forces stay)
    double *rdiag = nullptr;   // residual handed to a diagnostic kernel build
    // a kernel for the dynamics whose build stopped at rank 0 (a zero or
    // floor-level residual, e.g. right after a converged SCF) is rebuilt at
    // the next step, whatever the refresh period
    bool kernel_pending = false;
    // the electronic state (D, q, r) belongs to a diagnostic solve
    // (xlbomd_solve, xlbomd_scf) or to nothing yet (a restored checkpoint),
    // not to the MD state n(t), R(t)
    bool el_stale = false;

    // The trajectory's kernel lives in V, W, Vprev (the previous build's
    // images W, block mode), gj (with rank_built, rank_prev, full_built).  Diagnostic calls (xlbomd_kernel_apply,
    // xlbomd_scf) build theirs in a second set swapped in for the call, so
    // the MD kernel applied between rebuilds is never replaced by theirs.
    struct KernSet {
        double *V = nullptr, *W = nullptr, *Vprev = nullptr, *gj = nullptr;
        int rank_built = 0, rank_prev = 0, rank_rb = 0, otf_count = 0;
        bool full_built = false;
    } kdiag;
    void swap_kernel_set();
    struct DiagKernel {
        SysBase &s;
        explicit DiagKernel(SysBase &s_) : s(s_) {
            if (!s.kdiag.V) {
                s.kdiag.V = s.dev<double>((size_t)s.mcap * s.nat);
                s.kdiag.W = s.dev<double>((size_t)s.mcap * s.nat);
                s.kdiag.Vprev = s.dev<double>((size_t)s.mcap * s.nat);
            }
            s.swap_kernel_set();
        }
        ~DiagKernel() { s.swap_kernel_set(); }
        DiagKernel(const DiagKernel &) = delete;
        DiagKernel &operator=(const DiagKernel &) = delete;
    };

    // electronic state of the last solve
    double mu = 0.0, mu_prev = 0.0, mu_prev2 = 0.0;
    int mu_known = 0;          // number of valid entries in mu history
    int L = 0, ns_total = 0, reruns = 0, scf_iters = 0;
    double dmu = 0.0, trd = 0.0, rms = 0.0, sumq = 0.0, sc = 0.0;
    double elo = 0.0, ehi = 0.0, t0max = 0.0;
    bool have_energy = false;
    xlbomd_report last{};

    // Optional live timing of the dense products with HIP events recorded on
    // the library stream around each launch.
    // duration of a step on the stream (reported when a report is asked)
    hipEvent_t step_ev[2] = {nullptr, nullptr};
    void step_timer(bool start) {
        if (!step_ev[0]) {
            XL_HIP(hipEventCreate(&step_ev[0]));
            XL_HIP(hipEventCreate(&step_ev[1]));
        }
        XL_HIP(hipEventRecord(step_ev[start ? 0 : 1], st));
    }
    double step_ms() {
        XL_HIP(hipEventSynchronize(step_ev[1]));
        float ms = 0.f;
        XL_HIP(hipEventElapsedTime(&ms, step_ev[0], step_ev[1]));
        return ms;
    }
    struct Prof {
        bool on = false;
        std::vector<hipEvent_t> ev;
        std::vector<double> flops;
        std::vector<int> cls;      // 0 FP64, 1 FP32, 2 split bf16x3
        size_t used = 0;
    } prof;

    void prof_begin() {
        if (!prof.on || capturing) return;
        if (prof.used + 2 > prof.ev.size()) {
            for (int i = 0; i < 256; ++i) {
                hipEvent_t e;
                XL_HIP(hipEventCreate(&e));
                prof.ev.push_back(e);
            }
        }
        XL_HIP(hipEventRecord(prof.ev[prof.used], st));
    }
    void prof_end(double flops, int cls) {
        if (!prof.on || capturing) return;
        XL_HIP(hipEventRecord(prof.ev[prof.used + 1], st));
        prof.flops.push_back(flops);
        prof.cls.push_back(cls);
        prof.used += 2;
    }
    // algorithmic flops of one product on the real n x n block: each output
    // entry needs 2 n_k flops; a symmetric output has n (n+1)/2 entries
    double gemm_flops(bool sym, int npairs) const {
        const double n = N, ent = sym ? 0.5 * n * (n + 1.0) : n * n;
        return ent * 2.0 * n * npairs;
    }

    void sync() { XL_HIP(hipStreamSynchronize(st)); }

    // launches of foe_core skip themselves while *cur_skip is set (the
    // second expansion of a planned step); seed_sparse: the last expansion
    // used the sparse-dense seed products
    const int *cur_skip = nullptr;
    bool seed_sparse = false;

    // truncation target of the expansion against the Fermi function, and
    // the threshold on beta |dmu| above which the expansion is rerun at the
    // corrected chemical potential (descriptor values, else by precision)
    double trunc_tol() const {
        return d.foe_tol > 0.0 ? d.foe_tol : (d.precision == XLBOMD_FP64 ? 2e-10 : 1e-9);
    }
    double mu_tol() const {
        return d.mu_tol > 0.0 ? d.mu_tol : (d.precision == XLBOMD_FP64 ? 1e-6 : 1e-3);
    }
    // level count for the half-width xmax of the spectrum of beta (H - mu):
    // the smallest meeting the truncation target, or the descriptor's
    // request raised where the seed would leave |x / 2^(L+1)| <= 1
    int levels_for(double xmax) const {
        if (d.foe_levels > 0) {
            int Lmin = 1;
            while (Lmin < 40 && std::ldexp(xmax, -(Lmin + 1)) > 1.0) ++Lmin;
            return std::max(d.foe_levels, Lmin);
        }
        return choose_levels(xmax, trunc_tol());
    }

    void upload_model(const xlbomd_desc *ds) {
        d = *ds;
        if (d.allocator) mem.al = *d.allocator;   // kept by value
        d.allocator = nullptr;
        nat = d.n_atoms;
        no = d.n_orb;
        N = nat * no;
        Np = ((N + GT - 1) / GT) * GT;
        beta = 1.0 / d.te;
        zc = d.n_electrons / nat;
        if (d.stream) {
            st = (hipStream_t)d.stream;
        } else {
            XL_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            own_stream = true;
        }
        auto A = [&](auto *&p, size_t n) {
            using E = std::remove_pointer_t<std::remove_reference_t<decltype(p)>>;
            p = dev<E>(n);
        };
        A(pos, 3 * nat); A(vel, 3 * nat); A(mass, nat); A(force, 3 * nat);
        A(onsite, no); A(jit, N); A(hop, no * no); A(U, nat);
        const int K = d.kmax + 1;
        A(hist, (size_t)K * nat); A(kr, nat); A(q, nat); A(r, nat); A(ncur, nat);
        A(vpot, nat); A(glo, N); A(ghi, N); A(g, N); A(epart, 4 * nat);
        A(scal, 64); A(cvec, 8);
        A(lz_v, N); A(lz_vp, N); A(lz_w, N); A(lz_v0, N); A(lz_ab, 2 * LZ_M);
        A(nbl, (size_t)nat * NB_MAX); A(nbc, nat);
        sp_g = spmm_group(no);
        sp_ng = ceil_div(nat, sp_g);
        sp_gs = sp_g * NB_MAX;
        if ((long)ceil_div(nat, 32) * 4 > 48 * 1024)
            throw InvalidArg("more atoms than the neighbour-list union kernel supports (393216)");
        A(gnb, (size_t)sp_ng * sp_gs); A(gmask, (size_t)sp_ng * sp_gs); A(gcnt, sp_ng);
        mcap = std::max(1, std::min(d.kernel_rank + d.kernel_otf, 16));
        A(V, (size_t)mcap * nat); A(W, (size_t)mcap * nat); A(Vprev, (size_t)mcap * nat);
        A(vtmp, nat); A(vin, (size_t)mcap * nat); A(qp, (size_t)mcap * nat); A(hb, (size_t)mcap * nat);
        A(fscr, 3 * nat); A(rdiag, nat);
        ov = d.overlap_block != nullptr;
        if (ov) {
            A(sblk, no * no);
            nbc_dense = dev<int>(nat);
            XL_HIP(hipMemsetAsync(nbc_dense, 0xff, nat * sizeof(int), st));   // all -1
        }
        A(ub, (size_t)mcap * Np);
        A(part, (size_t)mcap * ((Np + 63) / 64) * N + 3 * (size_t)N);
        void *hp = nullptr;
        XL_HIP(hipHostMalloc(&hp, 64 * sizeof(double), hipHostMallocDefault));
        hscal = (double *)hp;

        auto up = [&](double *dst, const double *src, size_t n) {
            XL_HIP(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyHostToDevice, st));
        };
        up(pos, d.pos, 3 * nat);
        if (d.vel) up(vel, d.vel, 3 * nat);
        else XL_HIP(hipMemsetAsync(vel, 0, 3 * nat * sizeof(double), st));
        up(mass, d.mass, nat);
        up(onsite, d.onsite, no);
        if (d.onsite_jitter) up(jit, d.onsite_jitter, N);
        else XL_HIP(hipMemsetAsync(jit, 0, N * sizeof(double), st));
        up(hop, d.hop_block, no * no);
        up(U, d.hubbard_u, nat);
        if (ov) up(sblk, d.overlap_block, no * no);
        XL_HIP(hipMemsetAsync(ub, 0, (size_t)mcap * Np * sizeof(double), st));
        {   // fixed pseudo-random Lanczos start vector (xorshift64), unit norm
            std::vector<double> v0(N);
            unsigned long long x = 0x9e3779b97f4a7c15ull;
            double nn = 0.0;
            for (int i = 0; i < N; ++i) {
                x ^= x << 13; x ^= x >> 7; x ^= x << 17;
                v0[i] = (double)(x >> 11) * (1.0 / 9007199254740992.0) - 0.5;
                nn += v0[i] * v0[i];
            }
            for (auto &e : v0) e /= std::sqrt(nn);
            up(lz_v0, v0.data(), N);
            sync();
        }
        const DampRow &row = kDamp[d.kmax - 5];
        up(cvec, row.c, row.nc);
        sync();   // host arrays may be released after the call

        md.nat = nat; md.no = no; md.n = N; md.ld = Np;
        md.pos = pos; md.onsite = onsite; md.jit = jit; md.hop = hop; md.U = U;
        md.decay = d.hop_decay; md.rc = d.hop_cutoff; md.width = d.taper_width;
        md.soft = d.gamma_soft; md.rep_a = d.rep_a; md.rep_decay = d.rep_decay;
        md.sblk = sblk; md.sdecay = d.overlap_decay;
        d.overlap_block = nullptr;   // host array: not kept
    }

    double *hist_row(int k) {
        const int K = d.kmax + 1;
        return hist + (size_t)(((head + k) % K + K) % K) * nat;
    }

    // ---- precision-dependent parts ----
    virtual void alloc_matrices(int Lcap) = 0;
    virtual void lanczos() = 0;             // LZ_M steps on H into lz_ab (device)
    virtual void foe(double mu0) = 0;       // expansion at mu0 -> Z, Y, g, dmu
    virtual void finish_density() = 0;      // D_c and charges
    virtual void responses(int nb, const double *v, double *qout, double *wout) = 0;
    virtual void forces_parts(double *F) = 0;   // forces into F (3 n_atoms), energy parts
    virtual double entropy_ts() = 0;        // Te * S at the corrected state
    virtual int levels_cap() const = 0;
    virtual void solve_planned() = 0;       // planned solve at n(t) = history row 0
    virtual void kernel_planned() = 0;      // sequential kernel, rank on the device
    // non-orthogonal basis: S, X = S^-1/2 (when the positions changed), H
    // and H' = X H X at the potentials vpot; the interval of H' into
    // glo/ghi and its ends into scal[8..9]
    virtual void overlap_prepare() { throw InvalidArg("overlap needs XLBOMD_FP64"); }

    // ---- electronic solve at charges n (device, nat) ----
    void gershgorin() {
        hipLaunchKernelGGL(gershgorin_kernel, dim3(ceil_div(nat, 4)), dim3(256), 0, st, md,
                           vpot, glo, ghi);
        XL_LAUNCH_CHECK();
        hipLaunchKernelGGL(minmax_kernel, dim3(1), dim3(1024), 0, st, N, glo, ghi, scal + 8);
        XL_LAUNCH_CHECK();
    }

    // Spectral interval of H: Gershgorin, tightened by LZ_M Lanczos steps
    // (neighbour-block matvecs) from a fixed random vector.  Each side becomes the extreme Ritz value
    // widened by the last Lanczos coefficient beta_m (the norm of the
    // residual vector; the extreme Ritz values converge from inside), and is
    // kept only when tighter than Gershgorin.  On a breakdown or a
    // non-finite coefficient Gershgorin stays.  (Gershgorin overestimates the
    // half-width about twofold on dense 3-D lattices; the level count of the
    // expansion follows it.)
    static constexpr int LZ_M = 12;
    // neighbour lists of the current positions (sparse seed products): the
    // seed's powers of Y are sparse-dense products when every atom has at
    // most NB_MAX neighbours and at most a quarter of all atoms
    int *nbl = nullptr, *nbc = nullptr;
    int nb_max = 0;
    // unions of the neighbour lists of groups of sp_g consecutive atoms
    // (sp_ng groups, sp_gs entries each) for the sparse-dense seed products
    int *gnb = nullptr, *gcnt = nullptr;
    unsigned *gmask = nullptr;
    int sp_g = 1, sp_ng = 0, sp_gs = 0;
    void neighbour_lists() {
        hipLaunchKernelGGL(neighbours_kernel, dim3(nat), dim3(64), 0, st, md, nbl, nbc);
        hipLaunchKernelGGL(group_union_kernel, dim3(sp_ng), dim3(256),
                           ceil_div(nat, 32) * sizeof(unsigned), st, nat, sp_g,
                           (const int *)nbl, (const int *)nbc, gnb, gmask, gcnt, sp_gs);
        hipLaunchKernelGGL(max_count_kernel, dim3(1), dim3(1024), 0, st, nat, (const int *)nbc,
                           scal + 10);
        XL_LAUNCH_CHECK();
    }
    bool sparse_seed() const {
        return !ov && nb_max > 0 && nb_max <= NB_MAX && 4 * nb_max <= nat;
    }
    double *lz_v = nullptr, *lz_vp = nullptr, *lz_w = nullptr, *lz_v0 = nullptr, *lz_ab = nullptr;
    void spectral_tighten() {
        const double *a = hscal + 16, *b = hscal + 16 + LZ_M;
        for (int j = 0; j < LZ_M; ++j)
            if (!std::isfinite(a[j]) || !std::isfinite(b[j]) || !(b[j] > 1e-12 * (std::fabs(ehi) + std::fabs(elo))))
                return;
        double tlo, thi;
        tridiag_extremes(a, b, LZ_M, tlo, thi);
        const double bm = b[LZ_M - 1];
        elo = std::max(elo, tlo - bm);
        ehi = std::min(ehi, thi + bm);
    }

    double initial_mu() {
        // Fermi level of the diagonal of H alone (host bisection on N values)
        std::vector<double> v(nat), jh(N), on(no);
        XL_HIP(hipMemcpyAsync(v.data(), vpot, nat * sizeof(double), hipMemcpyDeviceToHost, st));
        XL_HIP(hipMemcpyAsync(jh.data(), jit, N * sizeof(double), hipMemcpyDeviceToHost, st));
        XL_HIP(hipMemcpyAsync(on.data(), onsite, no * sizeof(double), hipMemcpyDeviceToHost, st));
        sync();
        std::vector<double> e(N);
        for (int i = 0; i < N; ++i) e[i] = on[i % no] + jh[i] + v[i / no];
        double lo = elo - 1.0, hi = ehi + 1.0;
        for (int it = 0; it < 200; ++it) {
            const double m = 0.5 * (lo + hi);
            double s = 0.0;
            for (double x : e) s += 2.0 * fermi(beta * (x - m));
            if (s < d.n_electrons) lo = m; else hi = m;
        }
        return 0.5 * (lo + hi);
    }

    // One-shot electronic solve at n (device pointer, nat).  mu0 < -1e300
    // requests a fresh guess.
    void solve(const double *n_dev, double mu_guess, bool have_guess) {
        Phase ph("xlbomd:solve");
        if (n_dev != ncur)
            XL_HIP(hipMemcpyAsync(ncur, n_dev, nat * sizeof(double), hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL(gamma_matvec_kernel, dim3(ceil_div((long)nat * 64, 256)), dim3(256),
                           0, st, md, 1, ncur, vpot);
        XL_LAUNCH_CHECK();
        if (ov) overlap_prepare();
        else gershgorin();
        neighbour_lists();
        lanczos();
        XL_HIP(hipMemcpyAsync(hscal, scal + 8, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
        XL_HIP(hipMemcpyAsync(hscal + 16, lz_ab, 2 * LZ_M * sizeof(double),
                              hipMemcpyDeviceToHost, st));
        sync();
        elo = hscal[0];
        ehi = hscal[1];
        nb_max = (int)hscal[2];
        spectral_tighten();
        if (!std::isfinite(elo) || !std::isfinite(ehi)) throw Diverged("non-finite spectral bounds");
        double mu0 = have_guess ? mu_guess : initial_mu();
        const double tau = mu_tol();
        reruns = 0;
        ns_total = 0;
        // N(mu) = Tr D is strictly increasing: keep a bracket [mlo, mhi]
        // with N(mlo) < N_e < N(mhi) and take the model step only inside it
        double mlo = elo - 40.0 / beta, mhi = ehi + 40.0 / beta;
        mu0 = std::min(std::max(mu0, mlo), mhi);
        for (int it = 0;; ++it) {
            foe(mu0);
            XL_HIP(hipMemcpyAsync(hscal, scal, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
            sync();
            trd = hscal[0];
            dmu = hscal[2];   // root of the quadratic model of the count
            if (debug())
                std::fprintf(stderr, "[xlbomd] solve it %d mu0 %.10f elo %.6f ehi %.6f L %d "
                             "N0 %.10f dN %.6e dmu %.3e d2N %.6e\n", it, mu0, elo, ehi, L,
                             hscal[0], hscal[1], hscal[2], hscal[3]);
            if (!std::isfinite(trd)) throw Diverged("non-finite electron count");
            if (trd < d.n_electrons) mlo = std::max(mlo, mu0); else mhi = std::min(mhi, mu0);
            if (std::isfinite(dmu) && beta * std::fabs(dmu) <= tau) break;
            if (it >= 60) throw NoConv("chemical potential did not converge");
            double next = mu0 + (std::isfinite(dmu) ? dmu : 0.0);
            if (!(next > mlo && next < mhi) || !std::isfinite(dmu)) next = 0.5 * (mlo + mhi);
            mu0 = next;
            ++reruns;
        }
        mu = mu0 + dmu;
        finish_density();
        XL_HIP(hipMemcpyAsync(hscal, scal + 16, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        sync();
        rms = std::sqrt(hscal[0] / nat);
        sumq = hscal[1];
        if (!std::isfinite(rms)) throw Diverged("non-finite residual");
    }

    double predict_mu() const {
        if (mu_known >= 2) return 2.0 * mu_prev - mu_prev2;
        return mu_prev;
    }
    void push_mu() {
        mu_prev2 = mu_prev;
        mu_prev = mu;
        mu_known = std::min(mu_known + 1, 2);
    }

    // ---- low-rank kernel (Eqs. 48-51) at the last solve, applied to r ----
    // floor: a kernel for the dynamics (applied to later residuals) is K0
    // when the residual's RMS is at or below 1e-8 (its direction is rounding
    // noise); the SCF applies each kernel to its own residual (no floor).
    // `res` is the residual the directions start from (default: r of the
    // last solve).  A build for the dynamics (floor) that ends at rank 0
    // although m > 0 leaves kernel_pending set: the next step rebuilds.
    int build_kernel(int m, int mode, bool use_prev, bool floor = true,
                     const double *res = nullptr) {
        Phase ph("xlbomd:kernel");
        if (!res) res = r;
        m = std::min(m, mcap);
        if (d.kernel_rank <= 0) m = 0;
        const double gam = d.k0_gamma;
        int rank = 0;
        if (m > 0) {
            // v_1 = K0 r / |K0 r|, K0 = -gamma I
            hipLaunchKernelGGL(orth_kernel, dim3(1), dim3(1024), 0, st, nat, 0, V, res, -gam, V,
                               scal + 24);
            XL_LAUNCH_CHECK();
            XL_HIP(hipMemcpyAsync(hscal + 24, scal + 24, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
            sync();
            const double rms_r = hscal[24] / (gam * std::sqrt((double)nat));
            if (hscal[24 + 1] > 0.0 && (!floor || rms_r > 1e-8)) rank = 1;
        }
        if (rank > 0 && mode == 1) {
            // block mode: v_1 plus the previous build's images
            // w_j = (J - I) v_j (kept in Vprev), orthogonalised in order,
            // all responses in one batch; successive builds form a
            // subspace iteration with J - I towards its stiffest modes
            if (use_prev)
                for (int j = 1; j < m && j - 1 < rank_prev; ++j) {
                    hipLaunchKernelGGL(orth_kernel, dim3(1), dim3(1024), 0, st, nat, j, V,
                                       Vprev + (size_t)(j - 1) * nat, 1.0, V + (size_t)j * nat,
                                       scal + 24);
                    XL_LAUNCH_CHECK();
                    XL_HIP(hipMemcpyAsync(hscal + 24, scal + 24, 2 * sizeof(double),
                                          hipMemcpyDeviceToHost, st));
                    sync();
                    if (!(hscal[25] > 1e-10 * hscal[24])) break;
                    rank = j + 1;
                }
            responses(rank, V, qp, W);
        } else if (rank > 0) {
            // sequential Krylov: v_{j+1} = orth(w_j)
            for (int j = 0; j < m; ++j) {
                responses(1, V + (size_t)j * nat, qp, W + (size_t)j * nat);
                rank = j + 1;
                if (j + 1 == m) break;
                hipLaunchKernelGGL(orth_kernel, dim3(1), dim3(1024), 0, st, nat, j + 1, V,
                                   W + (size_t)j * nat, 1.0, V + (size_t)(j + 1) * nat,
                                   scal + 24);
                XL_LAUNCH_CHECK();
                XL_HIP(hipMemcpyAsync(hscal + 24, scal + 24, 2 * sizeof(double),
                                      hipMemcpyDeviceToHost, st));
                sync();
                if (!(hscal[25] > 1e-10 * hscal[24])) break;
            }
        }
        rank_built = rank;
        rank_rb = rank;
        otf_count = 0;
        full_built = false;
        if (rank > 0) {
            XL_HIP(hipMemcpyAsync(Vprev, W, (size_t)rank * nat * sizeof(double),
                                  hipMemcpyDeviceToDevice, st));
            rank_prev = rank;
        } else {
            rank_prev = 0;      // a rank-0 build leaves no directions to reuse
        }
        if (floor) kernel_pending = (m > 0 && rank == 0);
        return rank;
    }

    // On-the-fly rank-1 update between rebuilds (Section V.E): the previous
    // step's kernel is the estimate K0(t), improved by one rank-1 update
    // along v = K0(t) r / |K0(t) r| orthogonalised against the kept
    // directions, with its response at the current state.  The updates
    // accumulate after the rebuild's directions in a window of kernel_otf
    // columns; when it is full the oldest leaves first.
    void otf_update() {
        const int win = std::min(d.kernel_otf, mcap - rank_rb);
        if (win <= 0) return;
        apply_kernel(r, vtmp);                          // K0(t) r(t)
        if (otf_count >= win) {
            const size_t b = nat * sizeof(double);
            for (int j = rank_rb; j + 1 < rank_built; ++j) {
                XL_HIP(hipMemcpyAsync(V + (size_t)j * nat, V + (size_t)(j + 1) * nat, b,
                                      hipMemcpyDeviceToDevice, st));
                XL_HIP(hipMemcpyAsync(W + (size_t)j * nat, W + (size_t)(j + 1) * nat, b,
                                      hipMemcpyDeviceToDevice, st));
            }
            --otf_count;
            rank_built = rank_rb + otf_count;
        }
        const int j = rank_built;
        hipLaunchKernelGGL(orth_kernel, dim3(1), dim3(1024), 0, st, nat, j, V, vtmp, 1.0,
                           V + (size_t)j * nat, scal + 24);
        XL_LAUNCH_CHECK();
        XL_HIP(hipMemcpyAsync(hscal + 24, scal + 24, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        sync();
        if (!(hscal[24] > 0.0 && hscal[25] > 1e-10 * hscal[24])) return;
        responses(1, V + (size_t)j * nat, qp, W + (size_t)j * nat);
        ++otf_count;
        rank_built = rank_rb + otf_count;
    }

    // K_m r with the low-rank kernel last built (at most mcap directions)
    void apply_kernel(const double *rin, double *out) {
        if (rank_built < 0 || rank_built > mcap)
            throw StateError("no low-rank kernel of rank " + std::to_string(rank_built) +
                             " can be applied (capacity " + std::to_string(mcap) + ")");
        hipLaunchKernelGGL(kernel_apply_kernel, dim3(1), dim3(1024), 0, st, nat, rank_built, V, W,
                           rin, d.k0_gamma, out, scal + 32, (const int *)nullptr);
        XL_LAUNCH_CHECK();
    }

    // re-solve at the MD state n(t), R(t) when the electronic state belongs
    // to a diagnostic solve or a restored checkpoint (forces unchanged)
    void refresh_electronic() {
        if (!el_stale) return;
        solve(hist_row(0), mu_prev, mu_known > 0);
        el_stale = false;
    }

    // ---- energy report at the current state ----
    void energy(xlbomd_report *rep) {
        Phase ph("xlbomd:energy");
        forces_parts(fscr);
        hipLaunchKernelGGL(sum_rows_kernel, dim3(1), dim3(1024), 0, st, nat, 3, epart, scal + 40);
        XL_LAUNCH_CHECK();
        hipLaunchKernelGGL(kinetic_kernel, dim3(1), dim3(1024), 0, st, nat, vel, mass, scal + 44);
        XL_LAUNCH_CHECK();
        const double ts = entropy_ts();
        XL_HIP(hipMemcpyAsync(hscal + 40, scal + 40, 5 * sizeof(double), hipMemcpyDeviceToHost, st));
        sync();
        rep->e_band = hscal[40];
        rep->e_coul = hscal[41];
        rep->e_rep = hscal[42];
        rep->te_s = ts;
        rep->omega = rep->e_band + rep->e_coul + rep->e_rep - ts;
        rep->e_kin = hscal[44];
        rep->e_total = rep->omega + rep->e_kin;
        rep->has_energy = 1;
    }

    void fill_report(xlbomd_report *rep) {
        rep->k0_gamma = d.k0_gamma;
        rep->rms_res = rms;
        rep->mu = mu;
        rep->d_nelec = sumq;   // sum of net charges = Tr D - N_e
        rep->step = step_no;
        rep->foe_levels = L;
        rep->ns_iters = ns_total;
        rep->mu_reruns = reruns;
        rep->scf_iters = scf_iters;
        rep->kernel_rank = rank_built;
    }

    // ---- one XL-BOMD step (Eqs. 22-23) ----
    // ---- full kernel K = (J - I)^-1 (krylov_mode 2, Eq. 43) ----
    // J from N_at canonical responses to unit charge vectors, in batches of
    // mcap directions; [J^T - I | I] reduced by Gauss-Jordan with partial
    // pivoting in FP64; K r is then a dense product until the next rebuild.
    double *gj = nullptr, *gjf = nullptr, *dirs = nullptr, *qdir = nullptr;
    int *gjflag = nullptr;
    bool full_built = false;
    void build_full_kernel() {
        if (!gj) gj = dev<double>((size_t)2 * nat * nat);   // per kernel set
        if (!gjf) {                                           // shared work space
            gjf = dev<double>(nat);
            dirs = dev<double>((size_t)mcap * nat);
            qdir = dev<double>((size_t)mcap * nat);
            gjflag = dev<int>(1);
        }
        for (int i0 = 0; i0 < nat; i0 += mcap) {
            const int nb = std::min(mcap, nat - i0);
            hipLaunchKernelGGL(unit_dirs_kernel, dim3(ceil_div((long)nb * nat, 256)), dim3(256), 0,
                               st, nat, i0, nb, dirs);
            XL_LAUNCH_CHECK();
            responses(nb, dirs, qdir, nullptr);
            hipLaunchKernelGGL(gj_rows_kernel, dim3(ceil_div((long)nb * 2 * nat, 256)), dim3(256),
                               0, st, nat, i0, nb, qdir, gj);
            XL_LAUNCH_CHECK();
        }
        XL_HIP(hipMemsetAsync(gjflag, 0, sizeof(int), st));
        for (int k = 0; k < nat; ++k) {
            hipLaunchKernelGGL(gj_pivot_kernel, dim3(1), dim3(1024), 0, st, nat, k, gj, gjf, gjflag);
            XL_LAUNCH_CHECK();
            hipLaunchKernelGGL(gj_update_kernel, dim3(ceil_div(2L * nat, 256), nat), dim3(256), 0,
                               st, nat, k, gj, gjf);
            XL_LAUNCH_CHECK();
        }
        int flag = 0;
        XL_HIP(hipMemcpyAsync(&flag, gjflag, sizeof(int), hipMemcpyDeviceToHost, st));
        sync();
        if (flag) throw Diverged("full kernel: J - I is singular");
        full_built = true;
        rank_built = nat;
    }
    void apply_full(const double *rin, double *out) {
        hipLaunchKernelGGL(full_apply_kernel, dim3(ceil_div(nat, 256)), dim3(256), 0, st, nat, gj,
                           rin, out);
        XL_LAUNCH_CHECK();
    }
    bool full_mode() const { return d.krylov_mode == 2; }

    void md_step(bool want_energy, xlbomd_report *rep) {
        Phase ph("xlbomd:step");
        leave_planned();
        const double dt = d.dt;
        const int nthr3 = ceil_div(3 * nat, 256);
        hipLaunchKernelGGL(kick_drift_kernel, dim3(nthr3), dim3(256), 0, st, nat, 0.5 * dt, dt,
                           force, mass, vel, pos);
        XL_LAUNCH_CHECK();
        const DampRow &row = kDamp[d.kmax - 5];
        const int K = d.kmax + 1;
        const int dst = ((head - 1) % K + K) % K;   // oldest slot becomes n(t+dt)
        hipLaunchKernelGGL(verlet_n_kernel, dim3(ceil_div(nat, 256)), dim3(256), 0, st, nat,
                           d.kmax, head, dst, row.kappa, row.alpha, cvec, kr, hist);
        XL_LAUNCH_CHECK();
        head = dst;
        solve(hist_row(0), predict_mu(), mu_known > 0);
        el_stale = false;
        // a runaway residual stops the step before its forces move the
        // nuclei: positions and velocities stay at the half step, where the
        // previous forces took them
        if (rms > 1e3) throw Diverged("residual above 1e3");
        push_mu();
        forces_parts(force);
        ++step_no;
        if (full_mode()) {
            if (step_no % std::max(1, d.kernel_every) == 0 || !full_built) build_full_kernel();
            apply_full(r, kr);
        } else {
            if (step_no % std::max(1, d.kernel_every) == 0 || kernel_pending)
                build_kernel(d.kernel_rank, d.krylov_mode, true);
            else if (d.kernel_otf > 0)
                otf_update();
            apply_kernel(r, kr);
        }
        hipLaunchKernelGGL(kick_drift_kernel, dim3(nthr3), dim3(256), 0, st, nat, 0.5 * dt, 0.0,
                           force, mass, vel, (double *)nullptr);
        XL_LAUNCH_CHECK();
        have_energy = want_energy;
        if (want_energy) energy(&last);
        if (rep) {
            if (want_energy) *rep = last;
            else std::memset(rep, 0, sizeof(*rep));
            fill_report(rep);
            rep->has_energy = want_energy ? 1 : 0;
        }
    }

    // ---- planned steps: device-side decisions, optional HIP graph replay ----
    // step_mode 0: host decisions (solve, spectral interval, mu reruns and
    // Krylov breakdowns read back to the host).  1: planned steps, every
    // decision on the device (planned.hpp), one synchronisation at the end
    // of a step to read its status.  2: as 1, each step replayed from a HIP
    // graph captured once per plan.  Planned steps need a kernel rebuilt
    // every step from sequential Krylov directions without on-the-fly
    // updates (krylov_mode 0, kernel_every 1, kernel_otf 0).
    struct Plan {
        int L = 0;            // levels of the expansion
        double xmax = 0.0;    // half-width of beta (H - mu) the expansion is sized for
        bool sparse = false;  // sparse-dense seed products
    };
    int step_mode = 0;
    double plan_margin = 0.25;     // headroom of a plan's interval
    Plan plan{};
    bool have_plan = false;
    bool planned_ready = false;    // ordered n history and device mu history in place
    double *psd = nullptr, *hps = nullptr;      // device block, pinned status copy
    int *psi = nullptr, *hpi = nullptr;
    double *snap = nullptr, *histtmp = nullptr;
    hipGraphExec_t gexec = nullptr;
    long graph_epoch = -1, warm_epoch = -1;
    long n_planned = 0, n_replays = 0, n_captures = 0, n_fallbacks = 0;
    // a planned step begun by xlbomd_step_begin and not yet ended
    bool in_flight = false, in_flight_energy = false;
    hipEvent_t done_ev = nullptr;

    bool planned_capable() const {
        return d.krylov_mode == 0 && d.kernel_every == 1 && d.kernel_otf == 0 && !ov;
    }
    void drop_graph() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        gexec = nullptr;
        graph_epoch = -1;
    }
    size_t snap_len() const { return (size_t)(13 + d.kmax + 2 * mcap) * nat; }
    // the plan: the interval of the last solve around the predicted mu,
    // widened by plan_margin (25% unless set)
    void make_plan() {
        const double mp = mu_known > 0 ? predict_mu() : mu;
        const double x = beta * std::max(std::fabs(elo - mp), std::fabs(ehi - mp)) * 1.02 + 1e-12;
        plan.xmax = (1.0 + plan_margin) * x;
        plan.L = levels_for(plan.xmax);
        plan.sparse = sparse_seed();
        have_plan = true;
        drop_graph();
        warm_epoch = -1;          // the new plan's first step runs directly (it may allocate)
    }
    // n history in order (row k = n(t - k dt)), mu history on the device
    void prepare_planned() {
        if (!psd) {
            psd = dev<double>(PS_COUNT);
            psi = dev<int>(PI_COUNT);
            snap = dev<double>(snap_len());
            histtmp = dev<double>((size_t)(d.kmax + 1) * nat);
            void *hp = nullptr;
            XL_HIP(hipHostMalloc(&hp, PS_COUNT * sizeof(double) + PI_COUNT * sizeof(int),
                                 hipHostMallocDefault));
            hps = (double *)hp;
            hpi = (int *)(hps + PS_COUNT);
        }
        const int K = d.kmax + 1;
        if (head != 0) {
            const size_t b = nat * sizeof(double);
            for (int k = 0; k < K; ++k)
                XL_HIP(hipMemcpyAsync(histtmp + (size_t)k * nat, hist_row(k), b,
                                      hipMemcpyDeviceToDevice, st));
            XL_HIP(hipMemcpyAsync(hist, histtmp, K * b, hipMemcpyDeviceToDevice, st));
            head = 0;
        }
        std::fill(hps, hps + PS_COUNT, 0.0);
        std::fill(hpi, hpi + PI_COUNT, 0);
        hps[PS_MUP] = mu_prev;
        hps[PS_MUPP] = mu_prev2;
        hpi[PI_MUKNOWN] = mu_known;
        XL_HIP(hipMemcpyAsync(psd, hps, PS_COUNT * sizeof(double), hipMemcpyHostToDevice, st));
        XL_HIP(hipMemcpyAsync(psi, hpi, PI_COUNT * sizeof(int), hipMemcpyHostToDevice, st));
        sync();
        if (!have_plan) make_plan();
        planned_ready = true;
    }
    // one planned step, enqueued (no host synchronisation)
    void md_step_planned() {
        Phase ph("xlbomd:planned_step");
        const double dt = d.dt;
        const int nthr3 = ceil_div(3 * nat, 256);
        const int K = d.kmax + 1;
        {   // the state at the start of the step
            const size_t b = nat * sizeof(double);
            double *p = snap;
            auto put = [&](const double *src, size_t n) {
                XL_HIP(hipMemcpyAsync(p, src, n * b, hipMemcpyDeviceToDevice, st));
                p += n * nat;
            };
            put(pos, 3); put(vel, 3); put(force, 3); put(hist, K); put(kr, 1);
            put(V, mcap); put(W, mcap);
        }
        hipLaunchKernelGGL(kick_drift_kernel, dim3(nthr3), dim3(256), 0, st, nat, 0.5 * dt, dt,
                           force, mass, vel, pos);
        XL_LAUNCH_CHECK();
        const DampRow &row = kDamp[d.kmax - 5];
        hipLaunchKernelGGL(verlet_shift_kernel, dim3(ceil_div(nat, 256)), dim3(256), 0, st, nat,
                           d.kmax, row.kappa, row.alpha, (const double *)cvec, (const double *)kr,
                           hist);
        XL_LAUNCH_CHECK();
        solve_planned();
        forces_parts(force);
        kernel_planned();
        hipLaunchKernelGGL(kick_drift_kernel, dim3(nthr3), dim3(256), 0, st, nat, 0.5 * dt, 0.0,
                           force, mass, vel, (double *)nullptr);
        XL_LAUNCH_CHECK();
        XL_HIP(hipMemcpyAsync(hps, psd, PS_COUNT * sizeof(double), hipMemcpyDeviceToHost, st));
        XL_HIP(hipMemcpyAsync(hpi, psi, PI_COUNT * sizeof(int), hipMemcpyDeviceToHost, st));
    }
    // enqueue one planned step: replay the captured graph, or capture it
    // (when the previous planned step allocated nothing since), or run it
    // directly (which may allocate buffers on its first run)
    void planned_launch() {
        if (!planned_ready) prepare_planned();
        ++n_planned;
        if (step_mode == 2) {
            if (gexec && graph_epoch == alloc_epoch) {
                XL_HIP(hipGraphLaunch(gexec, st));
                ++n_replays;
                return;
            }
            if (warm_epoch == alloc_epoch) {
                drop_graph();
                hipGraph_t gr = nullptr;
                XL_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                capturing = true;
                try {
                    md_step_planned();
                } catch (...) {
                    capturing = false;
                    (void)hipStreamEndCapture(st, &gr);
                    if (gr) (void)hipGraphDestroy(gr);
                    throw;
                }
                capturing = false;
                XL_HIP(hipStreamEndCapture(st, &gr));
                const hipError_t e = hipGraphInstantiate(&gexec, gr, nullptr, nullptr, 0);
                (void)hipGraphDestroy(gr);
                if (e != hipSuccess) {
                    gexec = nullptr;
                    throw HipError(std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
                }
                graph_epoch = alloc_epoch;
                ++n_captures;
                XL_HIP(hipGraphLaunch(gexec, st));
                ++n_replays;
                return;
            }
        }
        md_step_planned();
        warm_epoch = alloc_epoch;
    }
    // wait for the planned step, commit it or, if it left its plan, restore
    // the state it started from and take the step with host decisions
    void planned_complete(bool want_energy, xlbomd_report *rep) {
        sync();
        // a runaway (or non-finite) residual is retaken the same way: the
        // host-decision step reports it before its forces move the nuclei
        if (hpi[PI_FLAGS] != 0 || !(hps[PS_RMS] <= 1e3)) {
            if (debug())
                std::fprintf(stderr, "[xlbomd] planned step %d left its plan (flags %d): "
                             "host decisions\n", step_no + 1, hpi[PI_FLAGS]);
            const size_t b = nat * sizeof(double);
            const int K = d.kmax + 1;
            const double *p = snap;
            auto get = [&](double *dst, size_t n) {
                XL_HIP(hipMemcpyAsync(dst, p, n * b, hipMemcpyDeviceToDevice, st));
                p += n * nat;
            };
            get(pos, 3); get(vel, 3); get(force, 3); get(hist, K); get(kr, 1);
            get(V, mcap); get(W, mcap);
            sync();
            ++n_fallbacks;
            planned_ready = false;
            have_plan = false;          // planned again from this step's interval
            drop_graph();
            md_step(want_energy, rep);
            return;
        }
        ++step_no;
        mu = hps[PS_MU];
        mu_prev2 = mu_prev;
        mu_prev = mu;
        mu_known = std::min(mu_known + 1, 2);
        dmu = hps[PS_DMU];
        rms = hps[PS_RMS];
        sumq = hps[PS_SUMQ];
        elo = hps[PS_ELO];
        ehi = hps[PS_EHI];
        reruns = hpi[PI_RERUN];
        rank_built = rank_rb = hpi[PI_RANK];
        otf_count = 0;
        rank_prev = rank_built;
        full_built = false;
        kernel_pending = false;
        el_stale = false;
        have_energy = want_energy;
        if (want_energy) energy(&last);
        if (rep) {
            if (want_energy) *rep = last;
            else std::memset(rep, 0, sizeof(*rep));
            fill_report(rep);
            rep->has_energy = want_energy ? 1 : 0;
        }
    }
    // any step or call with host decisions: the ordered history and the
    // device mu history are set up again before the next planned step
    void leave_planned() { planned_ready = false; }

    // K0 = -gamma I with gamma from the stiffest charge-response mode (the
    // descriptor's k0_gamma == 0): power iteration v <- -J v / |J v| from
    // v = r/|r| gives |lambda_max(J)| ~ |J v|, and gamma = 1.5 / (1 +
    // |lambda|) rounded down to two significant digits, in [1e-4, 1], keeps
    // every eigenvalue of K0 (J - I) below 1.5, inside the stability range
    // kappa e < 4 of the electronic Verlet step.  At the solve of the
    // current n.
    double auto_gamma(int iters = 20) {
        // v = r / |r| (scale 1); r = 0 falls back to e_0
        hipLaunchKernelGGL(orth_kernel, dim3(1), dim3(1024), 0, st, nat, 0, V, r, 1.0, vin,
                           scal + 24);
        XL_LAUNCH_CHECK();
        XL_HIP(hipMemcpyAsync(hscal + 24, scal + 24, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        sync();
        if (!(hscal[25] > 0.0)) {
            std::vector<double> e0(nat, 0.0);
            e0[0] = 1.0;
            XL_HIP(hipMemcpyAsync(vin, e0.data(), nat * sizeof(double), hipMemcpyHostToDevice, st));
            sync();
        }
        double lam = 0.0;
        for (int it = 0; it < iters; ++it) {
            responses(1, vin, qp, nullptr);            // qp = J v
            hipLaunchKernelGGL(orth_kernel, dim3(1), dim3(1024), 0, st, nat, 0, V, qp, -1.0, vin,
                               scal + 24);
            XL_LAUNCH_CHECK();
            XL_HIP(hipMemcpyAsync(hscal + 24, scal + 24, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
            sync();
            lam = hscal[24];
        }
        // 1.5 / (1 + |lambda|) rounded down to two significant digits (a
        // relative grid keeps the choice insensitive to rounding in lambda)
        const double g0 = 1.5 / (1.0 + lam);
        double g = 1.0;
        if (g0 < 1.0) {
            const double sc = std::pow(10.0, 1.0 - std::floor(std::log10(g0)));
            g = std::floor(g0 * sc) / sc;
        }
        if (debug()) std::fprintf(stderr, "[xlbomd] auto gamma: |lambda| %.4f gamma %.2f\n", lam, g);
        return std::min(1.0, std::max(1e-4, g));
    }

    // ---- initial state (Eqs. 20, 52) ----
    void init() {
        Phase ph("xlbomd:init");
        XL_HIP(hipMemsetAsync(ncur, 0, nat * sizeof(double), st));
        if (d.k0_gamma <= 0.0) {
            solve(ncur, 0.0, false);
            d.k0_gamma = auto_gamma();
        }
        const double tol = d.scf_tol > 0 ? d.scf_tol : 1e-10;
        const int maxit = d.scf_max_iter > 0 ? d.scf_max_iter : 200;
        bool have = false;
        ScfNeed need(scf_need, tol);
        for (scf_iters = 0;; ++scf_iters) {
            solve(ncur, mu, have);
            have = true;
            if (debug())
                std::fprintf(stderr, "[xlbomd] scf it %d rms %.3e mu %.8f reruns %d rank %d\n",
                             scf_iters, rms, mu, reruns, rank_built);
            if (rms <= tol) break;
            if (scf_iters >= maxit) throw NoConv("initial SCF did not reach the tolerance");
            // n <- n - K_j (q[n] - n), fresh rank-m kernel each iteration
            rank_prev = 0;
            build_kernel(d.kernel_rank, 0, false, false);
            apply_kernel(r, vtmp);
            hipLaunchKernelGGL(axpy_kernel, dim3(ceil_div(nat, 256)), dim3(256), 0, st, nat, -1.0,
                               vtmp, ncur);
            XL_LAUNCH_CHECK();
        }
        const int K = d.kmax + 1;
        for (int k = 0; k < K; ++k)
            XL_HIP(hipMemcpyAsync(hist + (size_t)k * nat, ncur, nat * sizeof(double),
                                  hipMemcpyDeviceToDevice, st));
        head = 0;
        mu_known = 0;
        push_mu();
        el_stale = false;
        forces_parts(force);
        rank_prev = 0;
        if (full_mode()) {
            build_full_kernel();
            apply_full(r, kr);
        } else {
            build_kernel(d.kernel_rank, d.krylov_mode, false);
            apply_kernel(r, kr);
        }
        step_no = 0;
        sync();
    }

    // Kernel SCF (Eq. 52) at the current positions from n0 (device copy in
    // ncur): n <- n - K_m (q[n] - n) with a fresh rank-m kernel (sequential
    // directions) per iteration; rank 0 is K0 alone (linear mixing).  The
    // MD history and K r are left as they are.  Returns true if RMS(r) <= tol.
    bool scf_run(int rank, double gamma, double tol, int max_iter, double *rms_hist,
                 int *n_eval) {
        Phase ph("xlbomd:scf");
        const double g_saved = d.k0_gamma;
        if (gamma > 0.0) d.k0_gamma = gamma;
        bool have = false, ok = false;
        int it = 0;
        ScfNeed need(scf_need, tol);
        *n_eval = 0;
        try {
            for (;; ++it) {
                // an iterate the electronic solve cannot handle (no chemical
                // potential, non-finite bounds) or a residual above 1e3 (as in
                // the MD step; charges are bounded by the orbital count) means
                // the iteration diverged; the evaluations so far stay reported
                try {
                    solve(ncur, mu, have);
                } catch (const NoConv &e) {
                    throw Diverged(std::string("scf diverged: ") + e.what());
                }
                have = true;
                if (rms_hist) rms_hist[it] = rms;
                *n_eval = it + 1;
                if (!(rms <= 1e3)) throw Diverged("scf diverged: residual above 1e3");
                if (rms <= tol) { ok = true; break; }
                if (it >= max_iter) break;
                rank_prev = 0;
                build_kernel(rank, 0, false, false);
                apply_kernel(r, vtmp);
                hipLaunchKernelGGL(axpy_kernel, dim3(ceil_div(nat, 256)), dim3(256), 0, st, nat,
                                   -1.0, vtmp, ncur);
                XL_LAUNCH_CHECK();
            }
        } catch (...) {
            d.k0_gamma = g_saved;
            throw;
        }
        d.k0_gamma = g_saved;
        sync();
        return ok;
    }
};

// ---- checkpoint: everything the next step reads ----
namespace {
struct CkHead {
    uint64_t magic;
    int32_t version, nat, no, kmax, mcap, krylov_mode, precision, full;
    int32_t step_no, rank_built, rank_prev, mu_known, kernel_pending;
    int32_t rank_rb, otf_count;
    double mu, mu_prev, mu_prev2, k0_gamma;
};
static_assert(sizeof(CkHead) % 8 == 0, "checkpoint header keeps the doubles aligned");
constexpr uint64_t kCkMagic = 0x584c424f4d44434bull;   // "XLBOMDCK"

size_t ck_doubles(const SysBase &s) {
    const size_t nat = s.nat, K = s.d.kmax + 1, m = s.mcap;
    return 9 * nat + K * nat + nat + 3 * m * nat + (s.full_mode() ? 2 * nat * nat : 0);
}
size_t state_bytes(const SysBase &s) { return sizeof(CkHead) + 8 * ck_doubles(s); }

void save_state(SysBase &s, char *buf) {
    CkHead h{};
    h.magic = kCkMagic;
    h.version = 1;
    h.nat = s.nat; h.no = s.no; h.kmax = s.d.kmax; h.mcap = s.mcap;
    h.krylov_mode = s.d.krylov_mode; h.precision = s.d.precision;
    h.full = s.full_built ? 1 : 0;
    h.step_no = s.step_no; h.rank_built = s.rank_built; h.rank_prev = s.rank_prev;
    h.mu_known = s.mu_known; h.kernel_pending = s.kernel_pending ? 1 : 0;
    h.rank_rb = s.rank_rb; h.otf_count = s.otf_count;
    h.mu = s.mu; h.mu_prev = s.mu_prev; h.mu_prev2 = s.mu_prev2; h.k0_gamma = s.d.k0_gamma;
    std::memcpy(buf, &h, sizeof(h));
    double *p = reinterpret_cast<double *>(buf + sizeof(h));
    const size_t nat = s.nat, m = s.mcap;
    auto get = [&](const double *src, size_t n) {
        if (src) XL_HIP(hipMemcpyAsync(p, src, n * sizeof(double), hipMemcpyDeviceToHost, s.st));
        else std::memset(p, 0, n * sizeof(double));
        p += n;
    };
    get(s.pos, 3 * nat);
    get(s.vel, 3 * nat);
    get(s.force, 3 * nat);
    for (int k = 0; k <= s.d.kmax; ++k) get(s.hist_row(k), nat);
    get(s.kr, nat);
    get(s.V, m * nat);
    get(s.W, m * nat);
    get(s.Vprev, m * nat);
    if (s.full_mode()) get(s.full_built ? s.gj : nullptr, 2 * nat * nat);
    s.sync();
}

void load_state(SysBase &s, const char *buf, size_t bytes) {
    if (bytes != state_bytes(s)) throw InvalidArg("checkpoint size does not match this handle");
    CkHead h;
    std::memcpy(&h, buf, sizeof(h));
    if (h.magic != kCkMagic || h.version != 1) throw InvalidArg("not an xlbomd checkpoint");
    if (h.nat != s.nat || h.no != s.no || h.kmax != s.d.kmax || h.mcap != s.mcap ||
        h.krylov_mode != s.d.krylov_mode || h.precision != s.d.precision)
        throw InvalidArg("checkpoint written by a handle with another descriptor");
    if (h.rank_built < 0 || h.rank_built > (h.full ? s.nat : s.mcap) || h.rank_prev < 0 ||
        h.rank_prev > s.mcap || h.mu_known < 0 || h.mu_known > 2 || !(h.k0_gamma > 0.0) ||
        h.rank_rb < 0 || h.otf_count < 0 || (!h.full && h.rank_rb + h.otf_count != h.rank_built))
        throw InvalidArg("checkpoint fields out of range");
    const double *p = reinterpret_cast<const double *>(buf + sizeof(h));
    const size_t nat = s.nat, m = s.mcap;
    auto put = [&](double *dst, size_t n) {
        XL_HIP(hipMemcpyAsync(dst, p, n * sizeof(double), hipMemcpyHostToDevice, s.st));
        p += n;
    };
    put(s.pos, 3 * nat);
    put(s.vel, 3 * nat);
    put(s.force, 3 * nat);
    for (int k = 0; k <= s.d.kmax; ++k) put(s.hist + (size_t)k * nat, nat);
    s.head = 0;
    put(s.kr, nat);
    put(s.V, m * nat);
    put(s.W, m * nat);
    put(s.Vprev, m * nat);
    if (s.full_mode()) {
        if (h.full) {
            if (!s.gj) s.gj = s.dev<double>(2 * nat * nat);
            put(s.gj, 2 * nat * nat);
        } else {
            p += 2 * nat * nat;
        }
    }
    s.sync();
    s.full_built = h.full != 0;
    s.step_no = h.step_no;
    s.rank_built = h.rank_built;
    s.rank_prev = h.rank_prev;
    s.mu_known = h.mu_known;
    s.kernel_pending = h.kernel_pending != 0;
    s.rank_rb = h.rank_rb;
    s.otf_count = h.otf_count;
    s.mu = h.mu;
    s.mu_prev = h.mu_prev;
    s.mu_prev2 = h.mu_prev2;
    s.d.k0_gamma = h.k0_gamma;
    s.have_energy = false;
    s.el_stale = true;    // D, q, r are solved again before anything reads them
    s.leave_planned();
}
}  // namespace

void SysBase::swap_kernel_set() {
    std::swap(V, kdiag.V);
    std::swap(W, kdiag.W);
    std::swap(Vprev, kdiag.Vprev);
    std::swap(gj, kdiag.gj);
    std::swap(rank_built, kdiag.rank_built);
    std::swap(rank_prev, kdiag.rank_prev);
    std::swap(rank_rb, kdiag.rank_rb);
    std::swap(otf_count, kdiag.otf_count);
    std::swap(full_built, kdiag.full_built);
}

// ---------------------------------------------------------------------------
// Precision-dependent dense algebra.  TF: expansion (density matrix, charges,
// forces, energy); TR: the kernel's responses.  MIXED runs TF = double,
// TR = float: the physics at FP64, the preconditioner at FP32.
// ---------------------------------------------------------------------------
template <typename TF, typename TR> struct Sys : SysBase {
    static constexpr bool SAME = std::is_same<TF, TR>::value;
    bool resp_split = false;       // response products as split bf16x3 (TR = float)
    // the kernel's response products as plain bf16 products (hi planes of
    // the split operands only; XLBOMD_MIXED_BF16)
    bool resp_bf16 = false;
    bool hi_now = false;           // set while responses_split runs
    std::vector<TF *> Z, Yk;       // Z_0..Z_L, Y_0..Y_{L-1}
    std::vector<TF *> Ak;          // A_k = I + 4 Z_k^2, k < L (kept for the entropy)
    TF *Ys = nullptr, *Y2 = nullptr, *Y3 = nullptr, *E = nullptr, *Wk = nullptr;
    TF *Dc = nullptr, *ZL2 = nullptr;
    std::vector<TR *> Zr, Yr;      // response copies (alias when SAME)
    TR *Ysr = nullptr, *Y2r = nullptr, *Y3r = nullptr, *Y4r = nullptr;
    TR *Zp = nullptr, *Ap = nullptr, *Tb = nullptr;   // response batch buffers
    double *m3 = nullptr;
    // non-orthogonal basis (FP64 only): S, X = S^-1/2, Sh = S^1/2, H, H',
    // D' (mu-corrected, orthogonalised basis), two work matrices, the
    // Mulliken form of dD/dmu per orbital
    double *Sm = nullptr, *Xm = nullptr, *Shm = nullptr, *Hm = nullptr, *Hpm = nullptr;
    double *Dpm = nullptr, *Tm = nullptr, *Wm = nullptr, *gov = nullptr;
    std::vector<double> ov_pos;    // positions X was computed at
    long gov_for = -1;             // expansion gov belongs to
    int ov_ns = 0;                 // Newton-Schulz steps of the last X
    double *e64[16] = {};                             // FP64 energy workspace
    int Lcap = 0, Lr = -1;                            // Lr: levels converted

    size_t mat() const { return (size_t)Np * Np; }
    template <typename U> U *amat() {
        return this->template dev<U>(mat());
    }
    int levels_cap() const override { return Lcap; }

    void ov_alloc() {
        if (Sm) return;
        Sm = amat<double>(); Xm = amat<double>(); Shm = amat<double>(); Hm = amat<double>();
        Hpm = amat<double>(); Dpm = amat<double>(); Tm = amat<double>(); Wm = amat<double>();
        gov = this->template dev<double>(Np);
    }
    GemmArgs<double> b64() const {
        GemmArgs<double> a;
        a.n = Np;
        a.ld = Np;
        return a;
    }
    // X = S^-1/2 and Sh = S^1/2 by the coupled Newton-Schulz iteration
    // Y_0 = S/c, Z_0 = I, T = (3I - Z Y)/2, Y <- Y T, Z <- T Z (Y -> (S/c)^1/2,
    // Z -> (S/c)^-1/2; every iterate is a polynomial in S, so every product
    // is symmetric), with c the Gershgorin bound of S, until |T - I| is
    // below 1e-12 in every row (then one last step).
    void inverse_sqrt() {
        hipLaunchKernelGGL(dense_gershgorin_kernel, dim3(ceil_div((long)N * 64, 256)), dim3(256),
                           0, st, N, Np, (const double *)Sm, glo, ghi);
        hipLaunchKernelGGL(minmax_kernel, dim3(1), dim3(1024), 0, st, N, glo, ghi, scal + 8);
        XL_LAUNCH_CHECK();
        XL_HIP(hipMemcpyAsync(hscal, scal + 8, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        sync();
        const double c = std::max(hscal[1], 1.0);
        convert(Sm, Shm, 1.0 / c);                    // Y_0 (in Shm)
        hipLaunchKernelGGL(identity_kernel, dim3(ceil_div((long)mat(), 256)), dim3(256), 0, st,
                           (long)Np, Xm);             // Z_0 (in Xm)
        XL_LAUNCH_CHECK();
        for (int it = 0;; ++it) {
            auto t = b64();                           // T = 3/2 I - Z Y / 2
            t.A0 = Xm; t.B0 = Shm; t.alpha = -0.5; t.gamma = 1.5; t.C = Tm;
            run_gemm(t, true);
            hipLaunchKernelGGL(row_dev_identity_kernel, dim3(ceil_div((long)Np * 64, 256)),
                               dim3(256), 0, st, Np, (const double *)Tm, part);
            hipLaunchKernelGGL(max_kernel, dim3(1), dim3(1024), 0, st, Np, (const double *)part,
                               scal + 12);
            XL_LAUNCH_CHECK();
            auto y = b64();                           // Y <- Y T
            y.A0 = Shm; y.B0 = Tm; y.C = Wm;
            run_gemm(y, true);
            auto z = b64();                           // Z <- T Z
            z.A0 = Tm; z.B0 = Xm; z.C = Dpm;
            run_gemm(z, true);
            std::swap(Shm, Wm);
            std::swap(Xm, Dpm);
            XL_HIP(hipMemcpyAsync(hscal + 12, scal + 12, sizeof(double), hipMemcpyDeviceToHost, st));
            sync();
            const double err = std::sqrt(hscal[12]);
            if (!std::isfinite(err)) throw Diverged("non-finite overlap inverse square root");
            if (err < 1e-12) { ov_ns = it + 1; break; }
            if (it >= 60)
                throw NoConv("overlap inverse square root did not converge (S not positive definite?)");
        }
        convert(Xm, Xm, 1.0 / std::sqrt(c));          // X = Z / sqrt(c)
        convert(Shm, Shm, std::sqrt(c));              // Sh = sqrt(c) Y
    }
    void overlap_prepare() override {
        if constexpr (!(SAME && std::is_same<TF, double>::value)) {
            throw InvalidArg("the non-orthogonal basis needs XLBOMD_FP64");
        } else {
            ov_alloc();
            hipLaunchKernelGGL(overlap_hamiltonian_kernel, dim3(ceil_div(Np, 256), Np), dim3(256), 0,
                               st, md, (const double *)vpot, Sm, Hm);
            XL_LAUNCH_CHECK();
            std::vector<double> p(3 * (size_t)nat);
            XL_HIP(hipMemcpyAsync(p.data(), pos, p.size() * sizeof(double), hipMemcpyDeviceToHost, st));
            sync();
            if (p != ov_pos) {
                inverse_sqrt();
                ov_pos = p;
            }
            auto a = b64();                           // H X
            a.A0 = Hm; a.B0 = Xm; a.C = Tm;
            run_gemm(a, false);
            a = b64();                                // H' = X (H X)
            a.A0 = Xm; a.B0 = Tm; a.C = Hpm;
            run_gemm(a, true);
            hipLaunchKernelGGL(dense_gershgorin_kernel, dim3(ceil_div((long)N * 64, 256)),
                               dim3(256), 0, st, N, Np, (const double *)Hpm, glo, ghi);
            hipLaunchKernelGGL(minmax_kernel, dim3(1), dim3(1024), 0, st, N, glo, ghi, scal + 8);
            XL_LAUNCH_CHECK();
        }
    }

    void lanczos() override {
        if (!Ys) alloc_matrices(std::max(Lcap, 1));
        if (ov) {
            // H' (dense) in the seed buffer; dense-row matvecs
            hipLaunchKernelGGL(seed_dense_kernel, dim3(ceil_div(Np, 256), Np), dim3(256), 0, st, N,
                               Np, (const double *)Hpm, 0.0, 1.0, (double *)Ys);
            XL_LAUNCH_CHECK();
            XL_HIP(hipMemcpyAsync(lz_v, lz_v0, N * sizeof(double), hipMemcpyDeviceToDevice, st));
            for (int j = 0; j < LZ_M; ++j) {
                hipLaunchKernelGGL((sp_matvec_kernel<TF>), dim3(nat), dim3(64), 0, st, N, no, Np,
                                   (const int *)nbl, (const int *)nbc_dense, (const TF *)Ys,
                                   (const double *)lz_v, lz_w);
                hipLaunchKernelGGL(lanczos_step_kernel, dim3(1), dim3(1024), 0, st, N, j, LZ_M,
                                   lz_v, lz_vp, lz_w, lz_ab);
            }
            XL_LAUNCH_CHECK();
            return;
        }
        // H itself (scale 1, no shift) in the seed buffer; the expansion
        // rebuilds its seed there
        hipLaunchKernelGGL((build_seed_kernel<TF>), dim3(ceil_div(Np, 256), Np), dim3(256), 0, st,
                           md, vpot, 0.0, 1.0, Ys, (const double *)nullptr);
        XL_LAUNCH_CHECK();
        XL_HIP(hipMemcpyAsync(lz_v, lz_v0, N * sizeof(double), hipMemcpyDeviceToDevice, st));
        for (int j = 0; j < LZ_M; ++j) {
            hipLaunchKernelGGL((sp_matvec_kernel<TF>), dim3(nat), dim3(64), 0, st, N, no, Np,
                               (const int *)nbl, (const int *)nbc, (const TF *)Ys,
                               (const double *)lz_v, lz_w);
            hipLaunchKernelGGL(lanczos_step_kernel, dim3(1), dim3(1024), 0, st, N, j, LZ_M, lz_v,
                               lz_vp, lz_w, lz_ab);
        }
        XL_LAUNCH_CHECK();
    }

    void alloc_matrices(int cap) override {
        if (cap <= Lcap) return;
        while ((int)Z.size() < cap + 1) Z.push_back(amat<TF>());
        while ((int)Yk.size() < cap) Yk.push_back(amat<TF>());
        while ((int)Ak.size() < cap) Ak.push_back(amat<TF>());
        if (!Ys) {
            Ys = amat<TF>(); Y2 = amat<TF>(); Y3 = amat<TF>(); E = amat<TF>();
            Wk = amat<TF>(); Dc = amat<TF>(); ZL2 = amat<TF>();
            m3 = this->template dev<double>(Np);
        }
        Lcap = cap;
    }
    void alloc_resp(int nb) {
        if (nb <= bcap) return;
        // the smaller batch buffers go back before the larger ones are taken
        this->release(Zp); this->release(Ap); this->release(Tb); this->release(Xb);
        for (auto &q : Sd) { this->release(q); q = nullptr; }
        Zp = Ap = Tb = Xb = nullptr;
        bcap = 0;
        TR *zp = this->template dev<TR>(mat() * nb), *ap = this->template dev<TR>(mat() * nb),
           *tb = this->template dev<TR>(mat() * nb);
        Zp = zp; Ap = ap; Tb = tb;
        if (resp_split) {
            Xb = this->template dev<TR>(mat() * nb);
            for (auto &q : Sd) q = this->template dev<TR>(mat() * nb);
        }
        if (ov) Xb = this->template dev<TR>(mat() * nb);
        bcap = nb;
    }
    TR *Xb = nullptr;                 // fourth response buffer (split path)
    TR *Sd[3] = {};                   // rows of Y D, Y^2 D, Y^3 D (split path)
    double *Pb = nullptr;             // Y D Y^3 per direction (sparse seed)
    int pb_cap = 0;
    // split bf16 view of a TR matrix buffer (planes mat() elements apart)
    uint16_t *s16(TR *p) const { return reinterpret_cast<uint16_t *>(p); }
    // response operand copy written by an expansion product: split planes
    // for the split path, FP32 otherwise
    template <typename G> void copy_out(G &g, TR *dst) {
        if constexpr (FUSE_COPY) {
            if (resp_split) {
                g.Cs = s16(dst);
                g.Cs_pl = (long)mat();
            } else {
                g.Cf = dst;
            }
        }
    }

    // split-k workspace per precision (allocated on first use)
    void *ws_d = nullptr, *ws_f = nullptr;
    long ws_dn = 0, ws_fn = 0;
    template <typename U> void attach_ws(GemmArgs<U> &a) {
        void *&w = sizeof(U) == 8 ? ws_d : ws_f;
        long &wn = sizeof(U) == 8 ? ws_dn : ws_fn;
        if (!w) {
            wn = std::max(split_ws_elems<U>(Np, true, 1, 1), split_ws_elems<U>(Np, false, 1, 1));
            if (sizeof(U) == 4)     // the split products' 256 x 128 tiles
                wn = std::max({wn, split_bs_ws_elems(Np, true, 1, 1),
                               split_bs_ws_elems(Np, false, 1, 1)});
            w = this->template dev<U>(wn);
        }
        a.ws = (U *)w;
        a.ws_elems = wn;
    }

    template <typename U> void run_gemm(GemmArgs<U> a, bool sym) {
        attach_ws(a);
        if (cur_skip) a.skip = cur_skip;
        prof_begin();
        gemm(a, sym, st);
        prof_end(gemm_flops(sym, a.A1 ? 2 : 1) * a.batch, sizeof(U) == 8 ? 0 : (a.split3 ? 2 : 1));
    }
    template <typename U> GemmArgs<U> base() const {
        GemmArgs<U> a;
        a.n = Np;
        a.ld = Np;
        return a;
    }
    template <typename S, typename D> void convert(const S *src, D *dst, double scale) {
        hipLaunchKernelGGL((convert_kernel<S, D>), dim3(ceil_div((long)mat(), 256)), dim3(256), 0,
                           st, (long)mat(), src, scale, dst);
        XL_LAUNCH_CHECK();
    }

    // FP32 copies of the response operands, written by the expansion's own
    // product epilogues when the two precisions differ (no separate pass)
    static constexpr bool FUSE_COPY = !SAME && std::is_same<TF, double>::value &&
                                      std::is_same<TR, float>::value;
    void alloc_resp_copies() {
        while ((int)Zr.size() < L + 1) Zr.push_back(amat<TR>());
        while ((int)Yr.size() < L) Yr.push_back(amat<TR>());
        if (!Ysr) { Ysr = amat<TR>(); Y2r = amat<TR>(); Y3r = amat<TR>(); }
        if (resp_split && !Sy[0])
            for (auto &q : Sy) q = amat<TR>();
    }
    TR *Sy[3] = {};                   // split Y, Y^2, Y^3 (split path)

    void foe(double mu0) override {
        const double xmax = beta * std::max(std::fabs(elo - mu0), std::fabs(ehi - mu0)) * 1.02 + 1e-12;
        foe_core(levels_for(xmax), xmax, mu0, nullptr, nullptr, sparse_seed(), scal, g);
    }

    // One expansion of L levels sized for the half-width xmax of the
    // spectrum of beta (H - mu0) (the seed bound and the Newton-Schulz
    // schedule of every level follow from L and xmax).  mu0 is read from
    // the device when mu_dev is given; while *skip is set the product
    // launches do nothing; `sparse` selects the sparse-dense seed products.
    // The chemical-potential moments {N0, N', dmu, N''} go to st_out, the
    // diagonal of dD/dmu to g_out.
    void foe_core(int Lq, double xmax, double mu0, const double *mu_dev, const int *skip,
                  bool sparse, double *st_out, double *g_out) {
        Phase ph("xlbomd:expansion");
        L = Lq;
        cur_skip = skip;
        seed_sparse = sparse;
        alloc_matrices(L);
        Lr = -1;
        ++expansion_id;
        if constexpr (FUSE_COPY) alloc_resp_copies();
        sc = std::ldexp(beta, -(L + 1));
        // Y = sc (H - mu0 I)  (H' = X H X in a non-orthogonal basis)
        if (ov) {
            if (mu_dev) throw InvalidArg("planned steps need an orthogonal basis");
            hipLaunchKernelGGL(seed_dense_kernel, dim3(ceil_div(Np, 256), Np), dim3(256), 0, st, N,
                               Np, (const double *)Hpm, mu0, sc, (double *)Ys);
        } else {
            hipLaunchKernelGGL((build_seed_kernel<TF>), dim3(ceil_div(Np, 256), Np), dim3(256), 0,
                               st, md, vpot, mu0, sc, Ys, mu_dev);
        }
        XL_LAUNCH_CHECK();
        const double ymax = std::ldexp(xmax, -(L + 1)), ym2 = ymax * ymax;
        t0max = ymax * (1.0 - ym2 / 3.0 + 2.0 * ym2 * ym2 / 15.0);
        if (sparse) {
            // Y2 = Y Y, Y3 = Y Y2, Y4 = Y Y3 (kept for the seed response),
            // Z0 = Y/2 - Y3/6 + Y Y4 / 15, each a sparse-dense product
            SpmmArgs<TF> a{};
            a.Y = Ys; a.B = Ys; a.C = Y2;
            if constexpr (FUSE_COPY) {
                a.Cf = Y2r;
                if (resp_split) { a.Cs = s16(Sy[1]); a.pl = (long)mat(); }
            }
            spmm(a);
            a = SpmmArgs<TF>{};
            a.Y = Ys; a.B = Y2; a.C = Y3;
            if constexpr (FUSE_COPY) {
                a.Cf = Y3r;
                if (resp_split) { a.Cs = s16(Sy[2]); a.pl = (long)mat(); }
            }
            spmm(a);
            if (!Y4r) Y4r = amat<TR>();
            TF *Y4t;
            if constexpr (SAME) Y4t = (TF *)Y4r;
            else {
                if (!Y4f) Y4f = amat<TF>();
                Y4t = Y4f;
            }
            a = SpmmArgs<TF>{};
            a.Y = Ys; a.B = Y3; a.C = Y4t;
            if constexpr (FUSE_COPY) {
                if (resp_split) { a.Cs = s16(Y4r); a.pl = (long)mat(); }
                else a.Cf = (float *)Y4r;
            }
            spmm(a);
            Y4_for = expansion_id;
            a = SpmmArgs<TF>{};
            a.Y = Ys; a.B = Y4t; a.alpha = 1.0 / 15.0;
            a.X = Y3; a.beta = -1.0 / 6.0; a.X2 = Ys; a.beta2 = 0.5;
            a.C = Z[0];
            if constexpr (FUSE_COPY) {
                if (resp_split) { a.Cs = s16(Zr[0]); a.pl = (long)mat(); }
                else a.Cf = (float *)Zr[0];
            }
            spmm(a);
        } else {   // Y2 = Y Y ; Y3 = Y Y2 ; Z0 = Y/2 - Y3/6 + Y3 Y2 / 15 (= tanh(Y)/2 to O(Y^7))
            auto a = base<TF>();
            a.A0 = Ys; a.B0 = Ys; a.C = Y2;
            if constexpr (FUSE_COPY) {
                a.Cf = Y2r;
                if (resp_split) { a.Cs = s16(Sy[1]); a.Cs_pl = (long)mat(); }
            }
            run_gemm(a, true);
            a = base<TF>();
            a.A0 = Ys; a.B0 = Y2; a.C = Y3;
            if constexpr (FUSE_COPY) {
                a.Cf = Y3r;
                if (resp_split) { a.Cs = s16(Sy[2]); a.Cs_pl = (long)mat(); }
            }
            run_gemm(a, true);
            a = base<TF>();
            a.A0 = Y3; a.B0 = Y2; a.alpha = (TF)(1.0 / 15.0);
            a.X = Y3; a.beta = (TF)(-1.0 / 6.0); a.X2 = Ys; a.beta2 = (TF)0.5;
            a.C = Z[0];
            copy_out(a, Zr[0]);
            run_gemm(a, true);
        }
        // Newton-Schulz target per level: far below the truncation bound; on
        // the split path the split products' own accuracy (the level is then
        // brought to FP64 accuracy by a residual refinement of Z_{k+1})
        const bool refine = FUSE_COPY && resp_split;
        const double nstol = refine ? 3e-5 : (sizeof(TF) == 8) ? 1e-12 : 1e-8;
        double t = t0max;
        for (int k = 0; k < L; ++k) {
            // spectrum of A_k within [1, 1 + b]; Chebyshev-optimal first
            // guesses of degree 1 (residual b^2/(2c^2 - b^2), free in the
            // epilogue of Z^2) or degree 2 (residual 1/|T3(u0)|, one GEMM)
            const double b = t * t, c = 2.0 + b;
            const double den = 2.0 * c * c - b * b;
            auto steps = [&](double e) {
                int ns = 0;
                while (e > nstol && ns < 10) { e = e * e; ++ns; }
                return ns;
            };
            const int ns1 = steps(b * b / den);
            const double al = 2.0 / b, be = -c / b;
            const double D3 = 4.0 * be * be * be - 3.0 * be;
            const int ns2 = b > 0.0 ? steps(1.0 / std::fabs(D3)) : ns1;
            const bool quad = (1 + 2 * ns2) < 2 * ns1;
            const int ns = quad ? ns2 : ns1;
            ns_total += ns;
            if (refine) {
                const double lin[2] = {8.0 * c / den, -8.0 / den};
                const double qd[3] = {-4.0 * al * al * al / D3, -12.0 * al * al * be / D3,
                                      -(12.0 * al * be * be - 3.0 * al) / D3};
                level_split(k, quad, ns, lin, qd,
                            (scf_need > 0.0 && scf_need < 1e-8) ? 2 : 1);
                t = 2.0 * t / (1.0 + t * t);
                continue;
            }
            auto a = base<TF>();
            TF *Am = Ak[k];
            a.A0 = Z[k]; a.B0 = Z[k]; a.alpha = (TF)4.0; a.gamma = (TF)1.0; a.C = Am;
            if (!quad) {
                a.C2 = Yk[k]; a.p0 = (TF)(8.0 * c / den); a.p1 = (TF)(-8.0 / den);
            }
            run_gemm(a, true);
            if (quad) {
                // Y = p0 I + p1 A + p2 A^2,  p(a) = (1 - T3(u(a))/T3(u0)) / a
                auto q = base<TF>();
                q.A0 = Am; q.B0 = Am; q.C = Yk[k];
                q.alpha = (TF)(-4.0 * al * al * al / D3);
                q.X = Am; q.beta = (TF)(-12.0 * al * al * be / D3);
                q.gamma = (TF)(-(12.0 * al * be * be - 3.0 * al) / D3);
                if (ns == 0) copy_out(q, Yr[k]);
                run_gemm(q, true);
            }
            for (int j = 0; j < ns; ++j) {
                auto e1 = base<TF>();   // E = 2I - A Y
                e1.A0 = Am; e1.B0 = Yk[k]; e1.alpha = (TF)-1.0; e1.gamma = (TF)2.0; e1.C = E;
                run_gemm(e1, true);
                auto e2 = base<TF>();   // Y <- Y E
                e2.A0 = Yk[k]; e2.B0 = E; e2.C = Wk;
                if (j + 1 == ns) copy_out(e2, Yr[k]);
                run_gemm(e2, true);
                std::swap(Yk[k], Wk);
            }
            if constexpr (FUSE_COPY) {
                if (ns == 0 && !quad) {
                    if (resp_split) {
                        hipLaunchKernelGGL(convert_split_kernel, dim3(ceil_div((long)mat(), 256)),
                                           dim3(256), 0, st, (long)mat(), (const double *)Yk[k],
                                           1.0, s16(Yr[k]), (long)mat());
                        XL_LAUNCH_CHECK();
                    } else {
                        convert(Yk[k], Yr[k], 1.0);
                    }
                }
            }
            auto z = base<TF>();        // Z_{k+1} = 2 Y_k Z_k
            z.A0 = Yk[k]; z.B0 = Z[k]; z.alpha = (TF)2.0; z.C = Z[k + 1];
            copy_out(z, Zr[k + 1]);
            run_gemm(z, true);
            t = 2.0 * t / (1.0 + t * t);
        }
        {   // Z_L^2 for the electron-count derivatives and the mu correction
            auto a = base<TF>();
            a.A0 = Z[L]; a.B0 = Z[L]; a.C = ZL2;
            if constexpr (FUSE_COPY) {
                if (resp_split) {
                    if (!ZL2s) ZL2s = amat<TR>();
                    a.Cs = s16(ZL2s); a.Cs_pl = (long)mat();
                }
            }
            run_gemm(a, true);
        }
        hipLaunchKernelGGL((zz2_rows_kernel<TF>), dim3(ceil_div((long)N * 64, 256)), dim3(256), 0,
                           st, N, Np, Z[L], ZL2, m3);
        XL_LAUNCH_CHECK();
        hipLaunchKernelGGL((mu_step_kernel<TF>), dim3(1), dim3(1024), 0, st, N, Np, Z[L], ZL2, m3,
                           beta, d.n_electrons, g_out, st_out);
        XL_LAUNCH_CHECK();
        if constexpr (FUSE_COPY) {
            convert(Ys, Ysr, 1.0);
            if (resp_split) {
                hipLaunchKernelGGL(convert_split_kernel, dim3(ceil_div((long)mat(), 256)),
                                   dim3(256), 0, st, (long)mat(), (const double *)Ys, 1.0,
                                   s16(Sy[0]), (long)mat());
                XL_LAUNCH_CHECK();
            }
            Lr = L;                     // response operands are current
        }
        cur_skip = nullptr;
    }

    // One level on the split path.  A_k = I + 4 Z_k^2 in FP64 (kept for the
    // entropy) with a split copy; Y_k ~ A_k^-1 from the Chebyshev guess and
    // ns Newton-Schulz steps, all split bf16x3 products (error ~1e-5); then
    // Z~ = 2 Y_k Z_k (FP64 result), the FP64 residual R = 2 Z_k - A_k Z~ and
    // Z_{k+1} = Z~ + Y_k R, whose error is that of Z~ times that of Y_k.  R
    // is a full product: Z~ commutes with A_k only to the split products'
    // accuracy, so R is not symmetric.  It is formed transposed,
    // R^T = 2 Z_k - Z~ A_k, which is the row layout the split product reads.
    TR *Asp = nullptr, *Esp = nullptr, *Ysp = nullptr, *Rsp = nullptr;
    SplitArgs sbase() const {
        SplitArgs a;
        a.n = Np;
        a.ld = Np;
        a.pl = (long)mat();
        return a;
    }
    void level_split(int k, bool quad, int ns, const double *lin, const double *qd, int nref) {
        if constexpr (FUSE_COPY) {
            if (!Asp) { Asp = amat<TR>(); Esp = amat<TR>(); Ysp = amat<TR>(); Rsp = amat<TR>(); }
            TF *Am = Ak[k];
            auto a = base<TF>();            // A_k, its split copy, the linear guess
            a.A0 = Z[k]; a.B0 = Z[k]; a.alpha = 4.0; a.gamma = 1.0; a.C = Am;
            a.Cs = s16(Asp); a.Cs_pl = (long)mat();
            if (!quad) { a.Cs2 = s16(Yr[k]); a.p0 = lin[0]; a.p1 = lin[1]; }
            run_gemm(a, true);
            if (quad) {                     // Y = p0 I + p1 A + p2 A^2
                SplitArgs q = sbase();
                q.A0 = s16(Asp); q.B0 = s16(Asp); q.X = s16(Asp); q.C = s16(Yr[k]);
                q.alpha = (float)qd[0]; q.beta = (float)qd[1]; q.gamma = (float)qd[2];
                run_split<TR>(q, true);
            }
            for (int j = 0; j < ns; ++j) {
                SplitArgs e = sbase();      // E = 2I - A Y
                e.A0 = s16(Asp); e.B0 = s16(Yr[k]); e.alpha = -1.f; e.gamma = 2.f;
                e.C = s16(Esp);
                run_split<TR>(e, true);
                SplitArgs y = sbase();      // Y <- Y E
                y.A0 = s16(Yr[k]); y.B0 = s16(Esp); y.C = s16(Ysp);
                run_split<TR>(y, true);
                std::swap(Yr[k], Ysp);
            }
            SplitArgs z = sbase();          // Z~ = 2 Y Z_k, FP64 result
            z.A0 = s16(Yr[k]); z.B0 = s16(Zr[k]); z.alpha = 2.f; z.Cd = Wk;
            run_split<TR>(z, true);
            for (int i = 0; i < nref; ++i) {
                const bool last = i + 1 == nref;
                auto r = base<TF>();        // R^T = 2 Z_k - Z~ A_k, split copy only
                r.A0 = Wk; r.B0 = Am; r.alpha = -1.0; r.X = Z[k]; r.beta = 2.0;
                r.Cs = s16(Rsp); r.Cs_pl = (long)mat();
                run_gemm(r, false);
                SplitArgs u = sbase();      // Z~ <- Z~ + Y R; the last one is
                u.A0 = s16(Yr[k]);          // Z_{k+1} (FP64 and split)
                u.B0 = s16(Rsp); u.Xd = Wk; u.beta = 1.f;
                // in place is safe: each upper element is read and written by
                // one thread, which also writes its mirror (never read)
                u.Cd = last ? Z[k + 1] : Wk;
                if (last) u.C = s16(Zr[k + 1]);
                run_split<TR>(u, true);
            }
        }
    }

    TR *ZL2s = nullptr;               // split copy of Z_L^2 (split path)
    TF *Y4f = nullptr;                // FP64 Y^4 of the sparse seed (when TF != TR)
    void spmm(SpmmArgs<TF> a, int nb = 1) {
        a.nat = nat; a.ld = Np;
        a.gnb = gnb; a.gcnt = gcnt; a.gmask = gmask; a.gstride = sp_gs;
        if (cur_skip) a.skip = cur_skip;
        if (nb > 1 && Np > N) throw InvalidArg("spmm: batched products need an unpadded matrix");
        const dim3 g(ceil_div(Np, 256), sp_ng, nb);
        switch (no) {
#define XL_SPMM(K) case K: hipLaunchKernelGGL((spmm_seed_kernel<TF, K>), g, dim3(256), 0, st, a); break;
            XL_SPMM(1) XL_SPMM(2) XL_SPMM(3) XL_SPMM(4) XL_SPMM(5) XL_SPMM(6) XL_SPMM(7) XL_SPMM(8)
#undef XL_SPMM
            default: throw InvalidArg("spmm: orbitals per atom must be 1..8");
        }
        XL_LAUNCH_CHECK();
        if (Np > N) {
            hipLaunchKernelGGL((zero_rows_kernel<TF>), dim3(ceil_div((long)(Np - N) * Np, 256)),
                               dim3(256), 0, st, N, Np, a.C, a.Cf, a.Cs, a.pl);
            XL_LAUNCH_CHECK();
        }
    }

    void finish_density() override {
        // D(mu0 + d) = I - 2Z + d (beta/2)(I - 4Z^2) + d^2/2 beta^2 (Z - 4Z^3)
        const double bd = beta * dmu;
        if constexpr (FUSE_COPY) {
            if (resp_split) {
                // only the Z Z^2 term is a product, with a coefficient of
                // 2 (beta d)^2 <= 2e-6 (the mu threshold bounds beta |d|):
                // split products change D by ~1e-11 at most; the other terms
                // are FP64 in the epilogue
                SplitArgs a = sbase();
                a.A0 = s16(Zr[L]); a.B0 = s16(ZL2s); a.alpha = -2.0 * bd * bd;
                a.Xd = Z[L]; a.beta = -2.0 + 0.5 * bd * bd;
                a.Xd2 = ZL2; a.beta2 = -2.0 * bd;
                a.gamma = 1.0 + 0.5 * bd; a.Cd = Dc;
                run_split<TR>(a, true);
                hipLaunchKernelGGL((charges_kernel<TF>), dim3(1), dim3(1024), 0, st, nat, no, Np,
                                   Dc, zc, ncur, q, r, scal + 16);
                XL_LAUNCH_CHECK();
                return;
            }
        }
        auto a = base<TF>();
        a.A0 = Z[L]; a.B0 = ZL2; a.alpha = (TF)(-2.0 * bd * bd);
        a.X = Z[L]; a.beta = (TF)(-2.0 + 0.5 * bd * bd);
        a.X2 = ZL2; a.beta2 = (TF)(-2.0 * bd);
        a.gamma = (TF)(1.0 + 0.5 * bd); a.C = Dc;
        if constexpr (SAME && std::is_same<TF, double>::value) {
            if (ov) {
                // D' in the orthogonalised basis, D = X D' X, Mulliken q
                a.C = Dpm;
                run_gemm(a, true);
                auto b = b64();
                b.A0 = Dpm; b.B0 = Xm; b.C = Tm;
                run_gemm(b, false);
                b = b64();
                b.A0 = Xm; b.B0 = Tm; b.C = Dc;
                run_gemm(b, true);
                hipLaunchKernelGGL(mulliken_rows_kernel, dim3(ceil_div((long)N * 64, 256)),
                                   dim3(256), 0, st, N, Np, (const double *)Dc,
                                   (const double *)Sm, rdpop());
                hipLaunchKernelGGL(charges_pop_kernel, dim3(1), dim3(1024), 0, st, nat, no,
                                   (const double *)rdpop(), zc, (const double *)ncur, q, r,
                                   scal + 16);
                XL_LAUNCH_CHECK();
                return;
            }
        }
        run_gemm(a, true);
        hipLaunchKernelGGL((charges_kernel<TF>), dim3(1), dim3(1024), 0, st, nat, no, Np, Dc, zc,
                           ncur, q, r, scal + 16);
        XL_LAUNCH_CHECK();
    }
    // Mulliken populations per orbital (the first Np entries of gov's
    // neighbour: a buffer of its own)
    double *pop = nullptr;
    double *rdpop() {
        if (!pop) pop = this->template dev<double>(Np);
        return pop;
    }

    // ---- planned step: the solve and the kernel without host decisions ----
    // The buffers one expansion writes.  A planned step runs a second
    // expansion (the rerun at the corrected chemical potential) into a set
    // of its own, swapped in for its enqueue, and copies it over the first
    // only when it ran.
    struct ExpSet {
        std::vector<TF *> Z, Yk, Ak;
        TF *Ys = nullptr, *Y2 = nullptr, *Y3 = nullptr, *E = nullptr, *Wk = nullptr;
        TF *ZL2 = nullptr, *Y4f = nullptr;
        double *m3 = nullptr, *g = nullptr;
        std::vector<TR *> Zr, Yr;
        TR *Ysr = nullptr, *Y2r = nullptr, *Y3r = nullptr, *Y4r = nullptr, *ZL2s = nullptr;
        TR *Sy[3] = {};
        TR *Asp = nullptr, *Esp = nullptr, *Ysp = nullptr, *Rsp = nullptr;
        int Lcap = 0;
    } alt;
    void swap_set() {
        std::swap(Z, alt.Z); std::swap(Yk, alt.Yk); std::swap(Ak, alt.Ak);
        std::swap(Ys, alt.Ys); std::swap(Y2, alt.Y2); std::swap(Y3, alt.Y3);
        std::swap(E, alt.E); std::swap(Wk, alt.Wk); std::swap(ZL2, alt.ZL2);
        std::swap(Y4f, alt.Y4f); std::swap(m3, alt.m3); std::swap(g, alt.g);
        std::swap(Zr, alt.Zr); std::swap(Yr, alt.Yr);
        std::swap(Ysr, alt.Ysr); std::swap(Y2r, alt.Y2r); std::swap(Y3r, alt.Y3r);
        std::swap(Y4r, alt.Y4r); std::swap(ZL2s, alt.ZL2s);
        for (int q = 0; q < 3; ++q) std::swap(Sy[q], alt.Sy[q]);
        std::swap(Asp, alt.Asp); std::swap(Esp, alt.Esp); std::swap(Ysp, alt.Ysp);
        std::swap(Rsp, alt.Rsp); std::swap(Lcap, alt.Lcap);
    }
    // the second expansion's results replace the first's where it ran: one
    // launch over a table of (source, destination, words), copied to the
    // device by the step itself from pinned host memory (the buffers' roles
    // alternate between steps with the Newton-Schulz ping-pong, so each
    // enqueue, and each captured graph, carries its own table; a direct step
    // synchronises before the next rewrites it)
    long *cp_tab = nullptr, *cp_host = nullptr;
    int cp_cap = 0;
    void adopt() {
        std::vector<long> t;
        auto cp = [&](const void *src, void *dst, size_t bytes) {
            if (!src || !dst || src == dst) return;
            t.push_back(reinterpret_cast<long>(src));
            t.push_back(reinterpret_cast<long>(dst));
            t.push_back((long)(bytes / 8));
        };
        const size_t mf = mat() * sizeof(TF), mr = mat() * sizeof(TR);
        for (int k = 0; k <= L; ++k) cp(alt.Z[k], Z[k], mf);
        for (int k = 0; k < L; ++k) {
            cp(alt.Yk[k], Yk[k], mf);
            cp(alt.Ak[k], Ak[k], mf);
        }
        cp(alt.Ys, Ys, mf); cp(alt.Y2, Y2, mf); cp(alt.Y3, Y3, mf); cp(alt.ZL2, ZL2, mf);
        if (seed_sparse) cp(alt.Y4r, Y4r, mr);
        if constexpr (FUSE_COPY) {
            for (int k = 0; k <= L; ++k) cp(alt.Zr[k], Zr[k], mr);
            for (int k = 0; k < L; ++k) cp(alt.Yr[k], Yr[k], mr);
            cp(alt.Ysr, Ysr, mr); cp(alt.Y2r, Y2r, mr); cp(alt.Y3r, Y3r, mr);
            for (int q = 0; q < 3; ++q) cp(alt.Sy[q], Sy[q], mr);
            cp(alt.ZL2s, ZL2s, mr);
        }
        cp(alt.g, g, (size_t)N * sizeof(double));
        const int n = (int)(t.size() / 3);
        if (n > cp_cap) {
            if (capturing) throw StateError("copy table grew during graph capture");
            this->release(cp_tab);
            cp_tab = nullptr;
            if (cp_host) {
                sync();
                XL_HIP(hipHostFree(cp_host));
                cp_host = nullptr;
            }
            cp_cap = 0;
            cp_tab = this->template dev<long>(3 * (size_t)n);
            void *hp = nullptr;
            XL_HIP(hipHostMalloc(&hp, 3 * (size_t)n * sizeof(long), hipHostMallocDefault));
            cp_host = (long *)hp;
            cp_cap = n;
        }
        std::memcpy(cp_host, t.data(), t.size() * sizeof(long));
        XL_HIP(hipMemcpyAsync(cp_tab, cp_host, t.size() * sizeof(long), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(pred_copy_table_kernel, dim3(256, n), dim3(256), 0, st,
                           (const int *)(psi + PI_SKIP2), (const long *)cp_tab);
        XL_LAUNCH_CHECK();
    }
    ~Sys() override {
        if (cp_host) (void)hipHostFree(cp_host);
    }
    // D at the final chemical potential: P = Z_L Z_L^2, then the
    // second-order correction with dmu from the device
    TF *Pd = nullptr;
    void finish_density_planned() {
        if (!Pd) Pd = amat<TF>();
        bool done = false;
        if constexpr (FUSE_COPY) {
            if (resp_split) {
                SplitArgs a = sbase();
                a.A0 = s16(Zr[L]); a.B0 = s16(ZL2s); a.Cd = Pd;
                run_split<TR>(a, true);
                done = true;
            }
        }
        if (!done) {
            auto a = base<TF>();
            a.A0 = Z[L]; a.B0 = ZL2; a.C = Pd;
            run_gemm(a, true);
        }
        hipLaunchKernelGGL((density_combine_kernel<TF>), dim3(ceil_div((long)mat(), 256)),
                           dim3(256), 0, st, N, Np, (const TF *)Z[L], (const TF *)ZL2,
                           (const TF *)Pd, (const double *)psd, beta, Dc);
        XL_LAUNCH_CHECK();
        hipLaunchKernelGGL((charges_kernel<TF>), dim3(1), dim3(1024), 0, st, nat, no, Np, Dc, zc,
                           ncur, q, r, scal + 16);
        XL_LAUNCH_CHECK();
    }
    void solve_planned() override {
        XL_HIP(hipMemcpyAsync(ncur, hist, nat * sizeof(double), hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL(gamma_matvec_kernel, dim3(ceil_div((long)nat * 64, 256)), dim3(256),
                           0, st, md, 1, ncur, vpot);
        XL_LAUNCH_CHECK();
        gershgorin();
        neighbour_lists();
        lanczos();
        hipLaunchKernelGGL(plan_interval_kernel, dim3(1), dim3(64), 0, st, (const double *)(scal + 8),
                           (const double *)lz_ab, LZ_M, nat, beta, plan.xmax, plan.sparse ? 1 : 0,
                           NB_MAX, psd, psi);
        XL_LAUNCH_CHECK();
        ns_total = 0;
        foe_core(plan.L, plan.xmax, 0.0, psd + PS_MU0, nullptr, plan.sparse, scal, g);
        hipLaunchKernelGGL(plan_mu_kernel, dim3(1), dim3(64), 0, st, (const double *)scal, beta,
                           d.n_electrons, mu_tol(), psd, psi);
        XL_LAUNCH_CHECK();
        const int ns_first = ns_total;
        swap_set();
        if (!g) g = this->template dev<double>(Np);
        try {
            foe_core(plan.L, plan.xmax, 0.0, psd + PS_MU1, psi + PI_SKIP2, plan.sparse,
                     psd + PS_ST2, g);
        } catch (...) {
            swap_set();
            throw;
        }
        swap_set();
        ns_total = ns_first;
        hipLaunchKernelGGL(plan_mu2_kernel, dim3(1), dim3(64), 0, st, (const double *)scal,
                           (const double *)(psd + PS_ST2), beta, mu_tol(), psd, psi);
        XL_LAUNCH_CHECK();
        adopt();
        finish_density_planned();
        hipLaunchKernelGGL(plan_finish_kernel, dim3(1), dim3(64), 0, st,
                           (const double *)(scal + 16), nat, psd, psi);
        XL_LAUNCH_CHECK();
    }
    // the sequential Krylov kernel with its rank decided on the device
    void kernel_planned() override {
        const int m = d.kernel_rank <= 0 ? 0 : std::min(d.kernel_rank, mcap);
        const double gam = d.k0_gamma;
        if (m > 0) {
            hipLaunchKernelGGL(orth_kernel, dim3(1), dim3(1024), 0, st, nat, 0, V, r, -gam, V,
                               psd + PS_NRM);
            XL_LAUNCH_CHECK();
            for (int j = 0; j < m; ++j) {
                responses(1, V + (size_t)j * nat, qp, W + (size_t)j * nat);
                if (j + 1 == m) break;
                hipLaunchKernelGGL(orth_kernel, dim3(1), dim3(1024), 0, st, nat, j + 1, V,
                                   W + (size_t)j * nat, 1.0, V + (size_t)(j + 1) * nat,
                                   psd + PS_NRM + 2 * (j + 1));
                XL_LAUNCH_CHECK();
            }
        }
        hipLaunchKernelGGL(plan_rank_kernel, dim3(1), dim3(64), 0, st,
                           (const double *)(psd + PS_NRM), m, gam, nat, 1e-8, psi);
        XL_LAUNCH_CHECK();
        hipLaunchKernelGGL(kernel_apply_kernel, dim3(1), dim3(1024), 0, st, nat, m, V, W, r, gam,
                           kr, scal + 32, (const int *)(psi + PI_RANK));
        XL_LAUNCH_CHECK();
    }

    void forces_parts(double *F) override {
        Phase ph("xlbomd:forces");
        hipLaunchKernelGGL((forces_kernel<TF>), dim3(ceil_div((long)nat * 64, 256)), dim3(256), 0,
                           st, md, Dc, q, ncur, vpot, F, epart);
        XL_LAUNCH_CHECK();
        if constexpr (SAME && std::is_same<TF, double>::value) {
            if (ov) {
                // energy-weighted density matrix E = X (D' H') X, D' H'
                // symmetrised (they commute up to the truncation error),
                // then the overlap part of the forces
                auto a = b64();
                a.A0 = Dpm; a.B0 = Hpm; a.A1 = Hpm; a.B1 = Dpm; a.alpha = 0.5; a.C = Tm;
                run_gemm(a, true);
                a = b64();
                a.A0 = Tm; a.B0 = Xm; a.C = Hm;
                run_gemm(a, false);
                a = b64();
                a.A0 = Xm; a.B0 = Hm; a.C = Wm;
                run_gemm(a, true);
                hipLaunchKernelGGL(overlap_forces_kernel, dim3(ceil_div((long)nat * 64, 256)),
                                   dim3(256), 0, st, md, (const double *)Dc, (const double *)Wm,
                                   (const double *)vpot, F);
                XL_LAUNCH_CHECK();
            }
        }
    }

    // response operands in TR (converted once per expansion when TF != TR)
    void response_operands() {
        if (Lr != L) {
            if constexpr (SAME) {
                Zr.assign(Z.begin(), Z.end());
                Yr.assign(Yk.begin(), Yk.end());
                Ysr = (TR *)Ys;
                Y2r = (TR *)Y2;
                Y3r = (TR *)Y3;
            } else {
                alloc_resp_copies();
                for (int k = 0; k <= L; ++k) convert(Z[k], Zr[k], 1.0);
                for (int k = 0; k < L; ++k) convert(Yk[k], Yr[k], 1.0);
                convert(Ys, Ysr, 1.0);
                convert(Y2, Y2r, 1.0);
                convert(Y3, Y3r, 1.0);
            }
            Lr = L;
        }
        if (!ov && Y4_for != expansion_id) {   // Y^4 for the seed response, in TR (split when
            if (!Y4r) Y4r = amat<TR>(); // the responses are)
            if (resp_split) {
                SplitArgs a = sbase();
                a.A0 = s16(Sy[1]); a.B0 = s16(Sy[1]); a.C = s16(Y4r);
                run_split<TR>(a, true);
            } else {
                auto a = base<TR>();
                a.A0 = Y2r; a.B0 = Y2r; a.C = Y4r;
                run_gemm(a, true);
            }
            Y4_for = expansion_id;
        }
    }
    long expansion_id = 0, Y4_for = -1;    // expansion counter, Y^4 made for

    template <typename U> void run_split(SplitArgs a, bool sym) {
        GemmArgs<float> w;
        attach_ws(w);
        a.ws = w.ws;
        a.ws_elems = w.ws_elems;
        if (cur_skip) a.skip = cur_skip;
        a.hi_only = hi_now;
        prof_begin();
        gemm_split(a, sym, st);
        prof_end(gemm_flops(sym, a.A1 ? 2 : 1) * a.batch, a.hi_only ? 3 : 2);
    }

    // Responses with the recursion's operands in split bf16 storage: the
    // seed's row-scaled products on FP32 operands, then per level
    // A' = 4 (Z Z' + Z' Z), T^T = 2 Z' - Z_{k+1} A' (T stored transposed),
    // Z'_{k+1} = Y_k T, all on pre-split operands; last level diag(Y T).
    void responses_split(int nb, const double *v, double *qout, double *wout) {
        struct Hi {
            bool &f;
            Hi(bool &f_, bool on) : f(f_) { f = on; }
            ~Hi() { f = false; }
        } hi(hi_now, resp_bf16);
        const long sm = (long)mat();
        hipLaunchKernelGGL(gamma_matvec_kernel, dim3(ceil_div((long)nat * nb * 64, 256)),
                           dim3(256), 0, st, md, nb, v, hb);
        XL_LAUNCH_CHECK();
        hipLaunchKernelGGL(expand_orbital_kernel, dim3(ceil_div((long)N * nb, 256)), dim3(256), 0,
                           st, nat, no, nb, sc, hb, (long)Np, ub);
        XL_LAUNCH_CHECK();
        const long s2 = 2 * sm;            // batch stride of split buffers
        if (seed_sparse && Np == N) {
            // G = (Y D) Y and P = (Y D) Y^3 as sparse-dense products (the
            // column scale applied to the rows of B), H13 = Y D Y^3 + Y^3 D Y
            // = P + P^T, and H2 = Y2 D Y2 on pre-split operands
            const dim3 cg(ceil_div(Np / 8, 256), Np, nb);
            hipLaunchKernelGGL(colscale_split_kernel, cg, dim3(256), 0, st, Np,
                               (const float *)Y2r, ub, (long)Np, s16(Sd[1]), sm, s2);
            XL_LAUNCH_CHECK();
            if (!Pb || pb_cap < nb) {
                this->release(Pb);
                Pb = nullptr;
                pb_cap = 0;
                Pb = this->template dev<double>(mat() * nb);
                pb_cap = nb;
            }
            SpmmArgs<TF> a{};
            a.Y = Ys; a.B = Ys; a.u = ub; a.su = Np; a.Cs = s16(Tb); a.pl = sm; a.sCs = s2;
            spmm(a, nb);
            a = SpmmArgs<TF>{};
            a.Y = Ys; a.B = Y3; a.u = ub; a.su = Np; a.C = (TF *)Pb; a.sC = sm;
            spmm(a, nb);
            hipLaunchKernelGGL(sym_split_kernel, dim3(Np / 32, Np / 32, nb), dim3(256), 0, st, Np,
                               (const double *)Pb, sm, s16(Xb), sm, s2);
            XL_LAUNCH_CHECK();
            SplitArgs h = sbase();
            h.batch = nb; h.A0 = s16(Sy[1]); h.B0 = s16(Sd[1]); h.sB0 = s2;
            h.C = s16(Ap); h.sC = s2;
            run_split<TR>(h, true);
            hipLaunchKernelGGL(seed_resp_split_kernel, dim3(ceil_div(Np, 256), Np, nb), dim3(256),
                               0, st, N, Np, (const uint16_t *)s16(Tb), (const uint16_t *)s16(Ap),
                               (const uint16_t *)s16(Xb), (const float *)Y2r,
                               (const uint16_t *)s16(Y4r), ub, (long)Np, sm, s16(Zp), sm);
            XL_LAUNCH_CHECK();
        } else {   // rows of Y D, Y^2 D, Y^3 D (D = diag(u), split), then on pre-split
            // operands G = Y D Y, H2 = Y2 D Y2, H13 = Y D Y3 + Y3 D Y, then Z'_0
            const dim3 cg(ceil_div(Np / 8, 256), Np, nb);
            hipLaunchKernelGGL(colscale_split_kernel, cg, dim3(256), 0, st, Np,
                               (const float *)Ysr, ub, (long)Np, s16(Sd[0]), sm, s2);
            hipLaunchKernelGGL(colscale_split_kernel, cg, dim3(256), 0, st, Np,
                               (const float *)Y2r, ub, (long)Np, s16(Sd[1]), sm, s2);
            hipLaunchKernelGGL(colscale_split_kernel, cg, dim3(256), 0, st, Np,
                               (const float *)Y3r, ub, (long)Np, s16(Sd[2]), sm, s2);
            XL_LAUNCH_CHECK();
            SplitArgs a = sbase();
            a.batch = nb; a.A0 = s16(Sy[0]); a.B0 = s16(Sd[0]); a.sB0 = s2;
            a.C = s16(Tb); a.sC = s2;
            run_split<TR>(a, true);
            a.A0 = s16(Sy[1]); a.B0 = s16(Sd[1]); a.C = s16(Ap);
            run_split<TR>(a, true);
            a.A0 = s16(Sy[0]); a.B0 = s16(Sd[2]); a.A1 = s16(Sy[2]); a.B1 = s16(Sd[0]); a.sB1 = s2;
            a.C = s16(Xb);
            run_split<TR>(a, true);
            hipLaunchKernelGGL(seed_resp_split_kernel, dim3(ceil_div(Np, 256), Np, nb), dim3(256),
                               0, st, N, Np, (const uint16_t *)s16(Tb), (const uint16_t *)s16(Ap),
                               (const uint16_t *)s16(Xb), (const float *)Y2r,
                               (const uint16_t *)s16(Y4r), ub, (long)Np, sm, s16(Zp), sm);
            XL_LAUNCH_CHECK();
        }
        for (int k = 0; k < L; ++k) {
            SplitArgs a;                    // A' = 4 (Z Z' + Z' Z)
            a.n = Np; a.ld = Np; a.pl = sm; a.batch = nb;
            a.A0 = s16(Zr[k]); a.B0 = s16(Zp); a.sB0 = s2; a.A1 = s16(Zp); a.sA1 = s2;
            a.B1 = s16(Zr[k]); a.alpha = 4.f; a.C = s16(Ap); a.sC = s2;
            run_split<float>(a, true);
            SplitArgs b;                    // T^T = 2 Z' - Z_{k+1} A'
            b.n = Np; b.ld = Np; b.pl = sm; b.batch = nb;
            b.A0 = s16(Zr[k + 1]); b.B0 = s16(Ap); b.sB0 = s2; b.alpha = -1.f;
            b.X = s16(Zp); b.sX = s2; b.beta = 2.f; b.C = s16(Tb); b.sC = s2;
            run_split<float>(b, false);
            if (k + 1 < L) {
                SplitArgs c;                // Z'_{k+1} = Y_k T
                c.n = Np; c.ld = Np; c.pl = sm; c.batch = nb;
                c.A0 = s16(Yr[k]); c.B0 = s16(Tb); c.sB0 = s2; c.C = s16(Zp); c.sC = s2;
                run_split<float>(c, true);
            }
        }
        hipLaunchKernelGGL(coldot_split_kernel, dim3(N, nb), dim3(256), 0, st, N, Np,
                           (const uint16_t *)s16(Yr[L - 1]), (const uint16_t *)s16(Tb), sm, s2,
                           part, (long)N);
        XL_LAUNCH_CHECK();
        hipLaunchKernelGGL(resp_charges_kernel, dim3(nb), dim3(1024), 0, st, nat, no, 1, part,
                           (long)N, g, v, qout, wout);
        XL_LAUNCH_CHECK();
    }

    void responses(int nb, const double *v, double *qout, double *wout) override {
        if (nb <= 0) return;
        alloc_resp(nb);
        response_operands();
        if constexpr (FUSE_COPY) {
            if (resp_split) {
                responses_split(nb, v, qout, wout);
                return;
            }
        }
        const long sm = (long)mat();
        // h = Gamma v, u = sc * h per orbital
        hipLaunchKernelGGL(gamma_matvec_kernel, dim3(ceil_div((long)nat * nb * 64, 256)),
                           dim3(256), 0, st, md, nb, v, hb);
        XL_LAUNCH_CHECK();
        hipLaunchKernelGGL(expand_orbital_kernel, dim3(ceil_div((long)N * nb, 256)), dim3(256), 0,
                           st, nat, no, nb, sc, hb, (long)Np, ub);
        XL_LAUNCH_CHECK();
        if constexpr (SAME && std::is_same<TF, double>::value) {
            if (ov) {
                responses_ov(nb, v, qout, wout);
                return;
            }
        }
        {   // G = Y D Y, H2 = Y2 D Y2, H13 = Y D Y3 + Y3 D Y, then Z'_0
            auto a = base<TR>();
            a.batch = nb; a.A0 = Ysr; a.B0 = Ysr; a.kscale = ub; a.sK = Np;
            a.split3 = resp_split;
            a.C = Tb; a.sC = sm;
            run_gemm(a, true);
            a.A0 = Y2r; a.B0 = Y2r; a.C = Ap;
            run_gemm(a, true);
            a.A0 = Ysr; a.B0 = Y3r; a.A1 = Y3r; a.B1 = Ysr; a.kscale_both = true; a.C = Zp;
            run_gemm(a, true);
            hipLaunchKernelGGL((seed_resp_kernel<TR>), dim3(ceil_div(Np, 256), Np, nb), dim3(256),
                               0, st, N, Np, Tb, Ap, Zp, Y2r, Y4r, ub, (long)Np, sm, Zp);
            XL_LAUNCH_CHECK();
        }
        for (int k = 0; k < L; ++k) {
            auto a = base<TR>();           // A' = 4 (Z Z' + Z' Z)
            a.batch = nb;
            a.A0 = Zr[k]; a.B0 = Zp; a.sB0 = sm; a.A1 = Zp; a.sA1 = sm; a.B1 = Zr[k];
            a.alpha = (TR)4.0; a.C = Ap; a.sC = sm; a.split3 = resp_split;
            run_gemm(a, true);
            auto b = base<TR>();           // T = 2 Z' - A' Z_{k+1}
            b.batch = nb;
            b.A0 = Ap; b.sA0 = sm; b.B0 = Zr[k + 1]; b.alpha = (TR)-1.0;
            b.X = Zp; b.sX = sm; b.beta = (TR)2.0; b.C = Tb; b.sC = sm; b.split3 = resp_split;
            run_gemm(b, false);
            if (k + 1 < L) {
                auto c = base<TR>();       // Z'_{k+1} = Y_k T
                c.batch = nb;
                c.A0 = Yr[k]; c.B0 = Tb; c.sB0 = sm; c.C = Zp; c.sC = sm; c.split3 = resp_split;
                run_gemm(c, true);
            }
        }
        const int nchunk = (N + 63) / 64;
        const long sP = (long)nchunk * N;
        hipLaunchKernelGGL((coldot_kernel<TR>), dim3(ceil_div(N, 256), nchunk, nb), dim3(256), 0,
                           st, N, Np, Yr[L - 1], Tb, sm, part, sP);
        XL_LAUNCH_CHECK();
        hipLaunchKernelGGL(resp_charges_kernel, dim3(nb), dim3(1024), 0, st, nat, no, nchunk, part,
                           sP, g, v, qout, wout);
        XL_LAUNCH_CHECK();
    }

    // Responses in a non-orthogonal basis (FP64).  The perturbation of H'
    // is dense: Y1 = sc X H1 X = (Sh U X + X U Sh)/2 with U = sc diag(Gamma v)
    // per orbital (X S = Sh); the seed Z_0 = Y/2 - Y^3/6 + Y^5/15 is
    // differentiated along the products that formed it,
    //   (Y^2)' = Y1 Y + Y Y1,  (Y^3)' = Y1 Y^2 + Y (Y^2)',
    //   Z'_0 = Y1/2 - (Y^3)'/6 + ((Y^3)' Y^2 + Y^3 (Y^2)')/15,
    // then the levels as in the orthogonal basis, Z'_L in full, and the
    // Mulliken charges of D1 = -2 X Z'_L X: sum over each atom's orbitals of
    // diag(X Z'_L Sh); the canonical shift uses the same form of dD'/dmu.
    void responses_ov(int nb, const double *v, double *qout, double *wout) {
        const long sm = (long)mat();
        if (gov_for != expansion_id) {        // dD'/dmu = (beta/2)(I - 4 Z_L^2)
            auto a = b64();
            a.A0 = (const double *)ZL2; a.B0 = Shm; a.alpha = -2.0 * beta;
            a.X = Shm; a.beta = 0.5 * beta; a.C = Tm;
            run_gemm(a, false);
            const int nchunk = (N + 63) / 64;
            hipLaunchKernelGGL((coldot_kernel<double>), dim3(ceil_div(N, 256), nchunk, 1), dim3(256),
                               0, st, N, Np, (const double *)Xm, (const double *)Tm, 0L, part, 0L);
            hipLaunchKernelGGL(chunk_sum_kernel, dim3(ceil_div(N, 256)), dim3(256), 0, st, N, nchunk,
                               (const double *)part, gov);
            XL_LAUNCH_CHECK();
            gov_for = expansion_id;
        }
        double *Y1 = (double *)Tb, *Y2d = (double *)Ap, *Y3d = (double *)Zp;
        const double *Yd = (const double *)Ys, *Y2m = (const double *)Y2, *Y3m = (const double *)Y3;
        auto a = b64();                                  // Y1
        a.batch = nb; a.A0 = Shm; a.B0 = Xm; a.A1 = Xm; a.B1 = Shm;
        a.kscale = ub; a.sK = Np; a.kscale_both = true; a.alpha = 0.5; a.C = Y1; a.sC = sm;
        run_gemm(a, true);
        a = b64();                                       // (Y^2)'
        a.batch = nb; a.A0 = Y1; a.sA0 = sm; a.B0 = Yd; a.A1 = Yd; a.B1 = Y1; a.sB1 = sm;
        a.C = Y2d; a.sC = sm;
        run_gemm(a, true);
        a = b64();                                       // (Y^3)'
        a.batch = nb; a.A0 = Y1; a.sA0 = sm; a.B0 = Y2m; a.A1 = Yd; a.B1 = Y2d; a.sB1 = sm;
        a.C = Y3d; a.sC = sm;
        run_gemm(a, true);
        a = b64();                                       // Z'_0
        a.batch = nb; a.A0 = Y3d; a.sA0 = sm; a.B0 = Y2m; a.A1 = Y3m; a.B1 = Y2d; a.sB1 = sm;
        a.alpha = 1.0 / 15.0; a.X = Y3d; a.sX = sm; a.beta = -1.0 / 6.0;
        a.X2 = Y1; a.sX2 = sm; a.beta2 = 0.5; a.C = (double *)Xb; a.sC = sm;
        run_gemm(a, true);
        std::swap(Zp, Xb);
        for (int k = 0; k < L; ++k) {
            auto p = base<TR>();           // A' = 4 (Z Z' + Z' Z)
            p.batch = nb;
            p.A0 = Zr[k]; p.B0 = Zp; p.sB0 = sm; p.A1 = Zp; p.sA1 = sm; p.B1 = Zr[k];
            p.alpha = (TR)4.0; p.C = Ap; p.sC = sm;
            run_gemm(p, true);
            auto b = base<TR>();           // T = 2 Z' - A' Z_{k+1}
            b.batch = nb;
            b.A0 = Ap; b.sA0 = sm; b.B0 = Zr[k + 1]; b.alpha = (TR)-1.0;
            b.X = Zp; b.sX = sm; b.beta = (TR)2.0; b.C = Tb; b.sC = sm;
            run_gemm(b, false);
            auto c = base<TR>();           // Z'_{k+1} = Y_k T
            c.batch = nb;
            c.A0 = Yr[k]; c.B0 = Tb; c.sB0 = sm; c.C = Zp; c.sC = sm;
            run_gemm(c, true);
        }
        a = b64();                                       // Z'_L Sh
        a.batch = nb; a.A0 = (const double *)Zp; a.sA0 = sm; a.B0 = Shm; a.C = (double *)Ap;
        a.sC = sm;
        run_gemm(a, false);
        const int nchunk = (N + 63) / 64;
        const long sP = (long)nchunk * N;
        hipLaunchKernelGGL((coldot_kernel<double>), dim3(ceil_div(N, 256), nchunk, nb), dim3(256), 0,
                           st, N, Np, (const double *)Xm, (const double *)Ap, sm, part, sP);
        XL_LAUNCH_CHECK();
        hipLaunchKernelGGL(resp_charges_kernel, dim3(nb), dim3(1024), 0, st, nat, no, nchunk, part,
                           sP, (const double *)gov, v, qout, wout);
        XL_LAUNCH_CHECK();
    }

    // ---- entropy without eigenvalues ----
    // With F = 1/2 I - Z_L the occupations and X_eff = 2^(L+1) atanh(2 Z_0)
    // the argument the expansion actually applies (f_L = 1/(1 + e^X_eff)):
    //   S/2 = -ln det(1/2 I + Z_L) + <F, X_eff>
    //   ln det(1/2 I + Z_L) = 2^L ln det(1/2 I + Z_0)
    //                       + sum_k 2^(L-1-k) (N ln 2 - ln det A_k)
    // (from 1/2 + z_{k+1} = 2 (1/2 + z_k)^2 / (1 + 4 z_k^2)), and the mu
    // correction adds dmu <X_eff, (1/2)(I - 4 Z_L^2)>.
    double *w64(int i) {
        if (!e64[i]) {
            e64[i] = this->template dev<double>(mat());
        }
        return e64[i];
    }
    const double *as64(const TF *src, int slot, double scale) {
        if constexpr (std::is_same<TF, double>::value) {
            if (scale == 1.0) return src;
        }
        double *dst = w64(slot);
        convert(src, dst, scale);
        return dst;
    }

    // ln det of the first nb matrices of the batch buffer (destroyed), to
    // hscal[48 ..)
    double *cholP = nullptr, *cholA = nullptr, *cholOut = nullptr;
    int chol_cap = 0;
    double *chol_batch(int nb) {       // nb padded Np x Np FP64 matrices
        if (nb > chol_cap) {
            this->release(cholA);
            this->release(cholP);
            cholA = cholP = nullptr;
            chol_cap = 0;
            cholA = this->template dev<double>(mat() * nb);
            cholP = this->template dev<double>((size_t)NB * Np * nb);
            if (!cholOut) {
                cholOut = this->template dev<double>(16);
            }
            chol_cap = nb;
        }
        return cholA;
    }
    void logdets(int nb) {
        GemmArgs<double> w;
        attach_ws(w);
        chol_logdet(Np, Np, nb, cholA, (long)mat(), cholP, (long)NB * Np, w.ws, w.ws_elems,
                    cholOut, st);
        XL_HIP(hipMemcpyAsync(hscal + 48, cholOut, nb * sizeof(double), hipMemcpyDeviceToHost, st));
        sync();
    }

    double entropy_ts() override {
        GemmArgs<double> a;
        a.n = Np; a.ld = Np;
        attach_ws(a);                    // split-k for the N x N products
        const double *T0 = as64(Z[0], 0, 2.0);          // T0 = 2 Z_0
        // log-determinants of I + T0 (index 0) and A_0 .. A_{L-1} (index
        // k + 1), factorised in batches of at most 16 matrices (the
        // factorisation overwrites its copies)
        const int nmat = L + 1, cap = std::min(nmat, 16);
        double *C = chol_batch(cap);
        std::vector<double> lds(nmat);
        for (int i0 = 0; i0 < nmat; i0 += cap) {
            const int nb = std::min(cap, nmat - i0);
            for (int j = 0; j < nb; ++j) {
                const int i = i0 + j;
                double *Cj = C + (size_t)j * mat();
                if (i == 0) {
                    // I + T0 over the padded array: the padding is an
                    // identity block (ln det 1 = 0), so the factorisation
                    // runs on whole 128-blocks
                    hipLaunchKernelGGL(add_diag_copy_kernel, dim3(ceil_div((long)mat(), 256)),
                                       dim3(256), 0, st, Np, Np, T0, 1.0, Cj);
                    XL_LAUNCH_CHECK();
                    continue;
                }
                const int k = i - 1;
                if constexpr (std::is_same<TF, double>::value) {
                    // the expansion's own A_k
                    XL_HIP(hipMemcpyAsync(Cj, Ak[k], mat() * sizeof(double),
                                          hipMemcpyDeviceToDevice, st));
                } else {
                    // FP32 expansion: A_k again in FP64 from Z_k
                    const double *Zk = as64(Z[k], 2, 1.0);
                    GemmArgs<double> b = a;
                    b.A0 = Zk; b.B0 = Zk; b.alpha = 4.0; b.gamma = 1.0; b.C = Cj;
                    gemm(b, true, st);
                }
            }
            logdets(nb);
            for (int j = 0; j < nb; ++j) lds[i0 + j] = hscal[48 + j];
        }
        const double ln2 = std::log(2.0);
        double lnF = std::ldexp(-N * ln2 + lds[0], L);   // ln det(I + T0) first
        for (int k = 0; k < L; ++k) lnF += std::ldexp(N * ln2 - lds[1 + k], L - 1 - k);
        // X_eff = 2^(L+1) atanh(T0) = T0 q(W), W = T0^2, q(w) = sum_j c_j w^j
        // with c_j = 2^(L+1) / (2j + 1), truncated where the next term is
        // below 1e-14 in the trace; q by Paterson-Stockmeyer: baby steps
        // W^0..W^s, then Horner in W^s over blocks of s coefficients
        const double *ZL = as64(Z[L], 2, 1.0);
        const double *Z2 = nullptr;
        double *W = w64(4);
        if constexpr (std::is_same<TF, double>::value) {
            // the expansion's own FP64 Z_L^2, and W = T0^2 = 4 Z_0^2 = A_0 - I
            // (A_0 over the padded array has a unit diagonal in the padding)
            Z2 = ZL2;
            if (L > 0) {
                hipLaunchKernelGGL(add_diag_copy_kernel, dim3(ceil_div((long)mat(), 256)),
                                   dim3(256), 0, st, Np, Np, (const double *)Ak[0], -1.0, W);
                XL_LAUNCH_CHECK();
            }
        }
        if (!Z2) {
            double *z2 = w64(3);
            GemmArgs<double> b = a;
            b.A0 = ZL; b.B0 = ZL; b.C = z2;
            gemm(b, true, st);
            Z2 = z2;
        }
        if (!(std::is_same<TF, double>::value && L > 0)) {
            GemmArgs<double> b = a;
            b.A0 = T0; b.B0 = T0; b.C = W;
            gemm(b, true, st);
        }
        const double scale = std::ldexp(1.0, L + 1);
        int J = 0;
        while (J < 63 && std::pow(t0max, 2 * J + 3) * scale / (2 * J + 3) * N >= 1e-14) ++J;
        const int nc = J + 1;                                  // coefficients c_0..c_J
        const int sps = std::max(1, (int)std::ceil(std::sqrt((double)nc)));
        const int nblk = (nc + sps - 1) / sps;
        std::vector<const double *> Wp(sps + 1, nullptr);      // Wp[l] = W^l (Wp[0] = I)
        Wp[1] = W;
        for (int l = 2; l <= sps; ++l) {
            double *dst = w64(4 + l - 1);
            GemmArgs<double> b = a;
            b.A0 = Wp[l - 1]; b.B0 = W; b.C = dst;
            gemm(b, true, st);
            Wp[l] = dst;
        }
        double *R = w64(4 + sps), *Rn = w64(5 + sps), *Bt = w64(6 + sps);
        auto block = [&](int i, double *out) {   // sum_l c_{i s + l} W^l
            LinComb lc{};
            for (int l = 0; l < sps && i * sps + l < nc; ++l) {
                const double c = scale / (2 * (i * sps + l) + 1);
                if (l == 0) { lc.wI = c; continue; }
                lc.x[lc.m] = Wp[l];
                lc.w[lc.m] = c;
                ++lc.m;
            }
            hipLaunchKernelGGL(lincomb_kernel, dim3(ceil_div((long)mat(), 256)), dim3(256), 0, st,
                               (long)Np, lc, out);
            XL_LAUNCH_CHECK();
        };
        block(nblk - 1, R);
        for (int i = nblk - 2; i >= 0; --i) {
            block(i, Bt);
            GemmArgs<double> b = a;                   // R <- R W^s + B_i
            b.A0 = R; b.B0 = Wp[sps]; b.X = Bt; b.beta = 1.0; b.C = Rn;
            gemm(b, true, st);
            std::swap(R, Rn);
        }
        {
            GemmArgs<double> b = a;                   // X_eff = T0 q(W)
            b.A0 = T0; b.B0 = R; b.C = Rn;
            gemm(b, true, st);
        }
        hipLaunchKernelGGL(frob3_kernel, dim3(N), dim3(256), 0, st, N, Np, Rn, ZL, Z2, part);
        XL_LAUNCH_CHECK();
        hipLaunchKernelGGL(sum_rows_kernel, dim3(1), dim3(1024), 0, st, N, 3, part, scal + 52);
        XL_LAUNCH_CHECK();
        XL_HIP(hipMemcpyAsync(hscal + 52, scal + 52, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
        sync();
        const double trX = hscal[52], zx = hscal[53], z2x = hscal[54];
        const double s1 = 0.5 * trX - zx;             // <1/2 I - Z_L, X_eff>
        const double s2 = trX - 4.0 * z2x;            // <X_eff, I - 4 Z_L^2>
        const double S0 = 2.0 * (-lnF + s1);
        if (debug()) {
            std::fprintf(stderr, "[xlbomd] entropy L %d t0max %.6f J %d lnF %.10f trX %.10f "
                         "zx %.10f z2x %.10f S0 %.10f dmu %.3e lds:", L, t0max, J, lnF, trX, zx,
                         z2x, S0, dmu);
            for (double v : lds) std::fprintf(stderr, " %.10f", v);
            std::fprintf(stderr, "\n");
        }
        return S0 / beta + dmu * 0.5 * s2;
    }
};

// ---------------------------------------------------------------------------
// Fixed scratch of the allocation-free split product: its split-k partial
// tiles (FP32).  32 MiB per device, held until the process ends; every
// multiple of 128 up to 46336 fits except some between 2176 and 3712.
// ---------------------------------------------------------------------------
constexpr long kScratchFloats = 8L << 20;
static __device__ __align__(256) float scratch[kScratchFloats];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch` per device

// The device address of `scratch` on the current device, looked up once per
// device with that device current (in host code the array's name is not a
// device address)
float *scratch_on_device() {
    int dev = 0;
    XL_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw InvalidArg("device index above 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        XL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw HipError("hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_ptr[dev] = static_cast<float *>(p);
    }
    return g_scratch_ptr[dev];
}
}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
struct xlbomd_system {
    std::unique_ptr<SysBase> s;
};

namespace {

int fail(int code, const std::string &m) {
    g_err = m;
    return code;
}

template <typename F> int guarded(F &&f) {
    try {
        g_err.clear();
        f();
        return XLBOMD_OK;
    } catch (const InvalidArg &e) {
        return fail(XLBOMD_E_INVALID, e.what());
    } catch (const NoMem &e) {
        return fail(XLBOMD_E_NOMEM, e.what());
    } catch (const NoConv &e) {
        return fail(XLBOMD_E_NOCONV, e.what());
    } catch (const Diverged &e) {
        return fail(XLBOMD_E_DIVERGED, e.what());
    } catch (const HipError &e) {
        return fail(XLBOMD_E_HIP, e.what());
    } catch (const std::exception &e) {
        return fail(XLBOMD_E_STATE, e.what());
    } catch (...) {
        return fail(XLBOMD_E_STATE, "unknown error");
    }
}

void validate(const xlbomd_desc *d) {
    if (!d) throw InvalidArg("null descriptor");
    if (d->n_atoms <= 0 || d->n_orb <= 0 || d->n_orb > 8)
        throw InvalidArg("n_atoms must be > 0 and n_orb in 1..8");
    // a padded N x N matrix stays below 2^31 elements (46336 = 362 * 128)
    if ((long)d->n_atoms * d->n_orb > 46336)
        throw InvalidArg("n_atoms * n_orb must be at most 46336");
    if (d->allocator && (!d->allocator->alloc || !d->allocator->free))
        throw InvalidArg("allocator needs both alloc and free");
    if (!d->pos || !d->mass || !d->onsite || !d->hop_block || !d->hubbard_u)
        throw InvalidArg("pos, mass, onsite, hop_block and hubbard_u are required");
    const double n2 = 2.0 * d->n_atoms * d->n_orb;
    if (!(d->n_electrons > 0.0 && d->n_electrons < n2))
        throw InvalidArg("n_electrons must lie in (0, 2 n_atoms n_orb)");
    if (!(d->te > 0.0) || !(d->dt > 0.0)) throw InvalidArg("te and dt must be > 0");
    if (d->kmax < 5 || d->kmax > 7) throw InvalidArg("kmax must be 5, 6 or 7");
    if (d->kernel_rank < 0 || d->kernel_rank > d->n_atoms || d->kernel_rank > 16)
        throw InvalidArg("kernel_rank must be in 0..min(n_atoms, 16)");
    if (d->kernel_every < 1) throw InvalidArg("kernel_every must be >= 1");
    if (d->kernel_otf < 0 || d->kernel_rank + d->kernel_otf > 16)
        throw InvalidArg("kernel_otf must be in 0..16 - kernel_rank");
    if (d->foe_levels < 0 || d->foe_levels > 40) throw InvalidArg("foe_levels must be in 0..40");
    if (d->krylov_mode < 0 || d->krylov_mode > 2) throw InvalidArg("krylov_mode is 0, 1 or 2");
    if (!(d->k0_gamma >= 0.0 && d->k0_gamma <= 1.0))
        throw InvalidArg("k0_gamma must be in (0, 1], or 0 for the automatic rule");
    if (d->foe_tol != 0.0 && !(d->foe_tol >= 1e-14 && d->foe_tol <= 1e-3))
        throw InvalidArg("foe_tol must be 0 or in [1e-14, 1e-3]");
    if (d->mu_tol != 0.0 && !(d->mu_tol >= 1e-12 && d->mu_tol <= 1e-1))
        throw InvalidArg("mu_tol must be 0 or in [1e-12, 1e-1]");
    if (d->precision < XLBOMD_FP64 || d->precision > XLBOMD_MIXED_BF16)
        throw InvalidArg("precision must be XLBOMD_FP64, XLBOMD_FP32, XLBOMD_MIXED, "
                         "XLBOMD_MIXED_BF16X3 or XLBOMD_MIXED_BF16");
    if (!(d->hop_decay > 0.0) || !(d->hop_cutoff > 0.0) || d->taper_width < 0.0 ||
        !(d->gamma_soft > 0.0) || (d->rep_a != 0.0 && !(d->rep_decay > 0.0)))
        throw InvalidArg("model lengths must be positive");
    for (int i = 0; i < d->n_atoms; ++i)
        if (!(d->mass[i] > 0.0)) throw InvalidArg("masses must be positive");
    if (d->overlap_block) {
        if (d->precision != XLBOMD_FP64)
            throw InvalidArg("a non-orthogonal basis needs XLBOMD_FP64");
        if (!(d->overlap_decay > 0.0)) throw InvalidArg("overlap_decay must be > 0");
        for (int a = 0; a < d->n_orb; ++a)
            for (int b = 0; b < d->n_orb; ++b)
                if (!std::isfinite(d->overlap_block[a * d->n_orb + b]) ||
                    d->overlap_block[a * d->n_orb + b] != d->overlap_block[b * d->n_orb + a])
                    throw InvalidArg("overlap_block must be finite and symmetric");
    }
}

}  // namespace

extern "C" {

int xlbomd_init_system(const xlbomd_desc *desc, xlbomd_system **out) {
    if (!out) return fail(XLBOMD_E_INVALID, "null output handle");
    *out = nullptr;
    std::unique_ptr<xlbomd_system> h(new xlbomd_system);
    const int rc = guarded([&] {
        validate(desc);
        if (desc->precision == XLBOMD_FP64) h->s.reset(new Sys<double, double>());
        else if (desc->precision == XLBOMD_FP32) h->s.reset(new Sys<float, float>());
        else {
            auto *m = new Sys<double, float>();
            m->resp_split = desc->precision == XLBOMD_MIXED_BF16X3 ||
                            desc->precision == XLBOMD_MIXED_BF16;
            m->resp_bf16 = desc->precision == XLBOMD_MIXED_BF16;
            h->s.reset(m);
        }
        h->s->upload_model(desc);
        h->s->init();
    });
    if (rc == XLBOMD_OK) *out = h.release();
    return rc;
}

int xlbomd_step(xlbomd_system *h, int32_t n_steps, xlbomd_report *last) {
    if (!h || !h->s) return fail(XLBOMD_E_INVALID, "null handle");
    if (n_steps < 0) return fail(XLBOMD_E_INVALID, "n_steps < 0");
    return guarded([&] {
        SysBase &s = *h->s;
        if (s.in_flight) throw StateError("a step begun on this handle has not ended");
        for (int i = 0; i < n_steps; ++i) {
            const int ev = s.d.energy_every;
            const bool is_last = (i + 1 == n_steps);
            const bool want = ev > 0 && ((s.step_no + 1) % ev == 0);
            const bool timed = is_last && last;
            if (timed) s.step_timer(true);
            if (s.step_mode != 0) {
                s.planned_launch();
                s.planned_complete(want, is_last ? last : nullptr);
            } else {
                s.md_step(want, is_last ? last : nullptr);
            }
            if (timed) {
                s.step_timer(false);
                last->ms_step = s.step_ms();
            }
        }
        s.sync();
    });
}

int xlbomd_step_batch(xlbomd_system *const *hs, int32_t count, int32_t n_steps,
                      xlbomd_report *reports, int32_t *status) {
    if (!hs || count < 0 || n_steps < 0) return fail(XLBOMD_E_INVALID, "bad batch arguments");
    for (int i = 0; i < count; ++i)
        if (!hs[i] || !hs[i]->s) return fail(XLBOMD_E_INVALID, "null handle in batch");
    for (int i = 0; i < count; ++i)
        if (hs[i]->s->in_flight) return fail(XLBOMD_E_STATE, "a step begun on a handle has not ended");
    for (int i = 0; i < count; ++i)
        for (int j = i + 1; j < count; ++j)
            if (hs[i] == hs[j]) return fail(XLBOMD_E_INVALID, "handle repeated in batch");
    std::vector<int> rc(count, XLBOMD_OK);
    std::vector<std::string> msg(count);
    bool all_planned = count > 0;
    for (int i = 0; i < count; ++i) all_planned = all_planned && hs[i]->s->step_mode != 0;
    if (all_planned) {
        // planned steps from one host thread: every system's step (a graph
        // replay in step mode 2) is enqueued on its own stream before any is
        // waited for, so the device runs them concurrently
        auto one = [&](int i, auto &&f) {
            if (rc[i] != XLBOMD_OK) return;
            rc[i] = guarded(f);
            if (rc[i] != XLBOMD_OK) msg[i] = xlbomd_last_error();
        };
        for (int t = 0; t < n_steps; ++t) {
            std::vector<char> want(count, 0);
            for (int i = 0; i < count; ++i)
                one(i, [&] {
                    SysBase &s = *hs[i]->s;
                    const int ev = s.d.energy_every;
                    want[i] = ev > 0 && ((s.step_no + 1) % ev == 0);
                    s.planned_launch();
                });
            for (int i = 0; i < count; ++i)
                one(i, [&] {
                    SysBase &s = *hs[i]->s;
                    s.planned_complete(want[i] != 0,
                                       (t + 1 == n_steps && reports) ? &reports[i] : nullptr);
                });
        }
    } else {
    auto run = [&](int i) {
        rc[i] = xlbomd_step(hs[i], n_steps, reports ? &reports[i] : nullptr);
        if (rc[i] != XLBOMD_OK) msg[i] = xlbomd_last_error();
    };
    if (count == 1) {
        run(0);
    } else {
        std::vector<std::thread> th;
        th.reserve(count);
        for (int i = 0; i < count; ++i) th.emplace_back(run, i);
        for (auto &x : th) x.join();
    }
    }
    int first = XLBOMD_OK;
    for (int i = 0; i < count; ++i) {
        if (status) status[i] = rc[i];
        if (rc[i] != XLBOMD_OK && first == XLBOMD_OK) {
            first = rc[i];
            g_err = "system " + std::to_string(i) + ": " + msg[i];
        }
    }
    return first;
}

int xlbomd_set_step_mode(xlbomd_system *h, int32_t mode) {
    if (!h || !h->s) return fail(XLBOMD_E_INVALID, "null handle");
    return guarded([&] {
        SysBase &s = *h->s;
        if (mode < 0 || mode > 2) throw InvalidArg("step mode must be 0, 1 or 2");
        if (mode != 0 && !s.planned_capable())
            throw InvalidArg("planned steps need krylov_mode 0, kernel_every 1, kernel_otf 0 "
                             "and an orthogonal basis");
        if (mode != s.step_mode) s.drop_graph();
        s.step_mode = mode;
    });
}

int xlbomd_step_begin(xlbomd_system *h) {
    if (!h || !h->s) return fail(XLBOMD_E_INVALID, "null handle");
    return guarded([&] {
        SysBase &s = *h->s;
        if (s.step_mode == 0) throw StateError("xlbomd_step_begin takes planned steps (step mode 1 or 2)");
        if (s.in_flight) throw StateError("a step begun on this handle has not ended");
        if (!s.done_ev) XL_HIP(hipEventCreateWithFlags(&s.done_ev, hipEventDisableTiming));
        const int ev = s.d.energy_every;
        s.in_flight_energy = ev > 0 && ((s.step_no + 1) % ev == 0);
        s.planned_launch();
        XL_HIP(hipEventRecord(s.done_ev, s.st));
        s.in_flight = true;
    });
}

int xlbomd_step_end(xlbomd_system *h, int32_t wait, int32_t *done, xlbomd_report *rep) {
    if (!h || !h->s || !done) return fail(XLBOMD_E_INVALID, "null argument");
    *done = 0;
    return guarded([&] {
        SysBase &s = *h->s;
        if (!s.in_flight) throw StateError("no step begun on this handle");
        if (!wait) {
            const hipError_t e = hipEventQuery(s.done_ev);
            if (e == hipErrorNotReady) return;
            if (e != hipSuccess) XL_HIP(e);
        }
        s.in_flight = false;
        s.planned_complete(s.in_flight_energy, rep);
        *done = 1;
    });
}

int xlbomd_set_plan_margin(xlbomd_system *h, double margin) {
    if (!h || !h->s) return fail(XLBOMD_E_INVALID, "null handle");
    if (!(margin >= -0.9 && margin <= 10.0))
        return fail(XLBOMD_E_INVALID, "plan margin must be in [-0.9, 10]");
    return guarded([&] {
        SysBase &s = *h->s;
        s.plan_margin = margin;
        s.have_plan = false;
        s.drop_graph();
    });
}

int xlbomd_step_stats(xlbomd_system *h, int64_t *out) {
    if (!h || !h->s || !out) return fail(XLBOMD_E_INVALID, "null argument");
    return guarded([&] {
        SysBase &s = *h->s;
        out[0] = s.n_planned;
        out[1] = s.n_replays;
        out[2] = s.n_captures;
        out[3] = s.n_fallbacks;
    });
}

int xlbomd_kernel_update(xlbomd_system *h, int32_t rank) {
    if (!h || !h->s) return fail(XLBOMD_E_INVALID, "null handle");
    return guarded([&] {
        SysBase &s = *h->s;
        const int m = rank > 0 ? rank : s.d.kernel_rank;
        if (m > s.mcap) throw InvalidArg("rank above the descriptor's kernel_rank");
        s.refresh_electronic();
        if (s.full_mode()) {
            s.build_full_kernel();
            s.apply_full(s.r, s.kr);
        } else {
            s.build_kernel(m, s.d.krylov_mode, true);
            s.apply_kernel(s.r, s.kr);
        }
        s.sync();
    });
}

int xlbomd_forces(xlbomd_system *h, double *forces, xlbomd_report *energy) {
    if (!h || !h->s) return fail(XLBOMD_E_INVALID, "null handle");
    return guarded([&] {
        SysBase &s = *h->s;
        if (energy) {
            s.refresh_electronic();
            s.energy(energy);
            s.fill_report(energy);
        }
        if (forces)
            XL_HIP(hipMemcpyAsync(forces, s.force, 3 * s.nat * sizeof(double),
                                  hipMemcpyDeviceToHost, s.st));
        s.sync();
    });
}

int xlbomd_get_charges(xlbomd_system *h, double *n_out, double *q_out) {
    if (!h || !h->s) return fail(XLBOMD_E_INVALID, "null handle");
    return guarded([&] {
        SysBase &s = *h->s;
        if (q_out) s.refresh_electronic();
        if (n_out)
            XL_HIP(hipMemcpyAsync(n_out, s.hist_row(0), s.nat * sizeof(double),
                                  hipMemcpyDeviceToHost, s.st));
        if (q_out)
            XL_HIP(hipMemcpyAsync(q_out, s.q, s.nat * sizeof(double), hipMemcpyDeviceToHost, s.st));
        s.sync();
    });
}

int xlbomd_set_state(xlbomd_system *h, const double *pos, const double *vel,
                     const double *n_hist, const double *kr) {
    if (!h || !h->s) return fail(XLBOMD_E_INVALID, "null handle");
    return guarded([&] {
        SysBase &s = *h->s;
        const size_t b3 = 3 * s.nat * sizeof(double), b1 = s.nat * sizeof(double);
        if (pos) XL_HIP(hipMemcpyAsync(s.pos, pos, b3, hipMemcpyHostToDevice, s.st));
        if (vel) XL_HIP(hipMemcpyAsync(s.vel, vel, b3, hipMemcpyHostToDevice, s.st));
        if (n_hist) {
            const int K = s.d.kmax + 1;
            for (int k = 0; k < K; ++k)
                XL_HIP(hipMemcpyAsync(s.hist + (size_t)k * s.nat, n_hist + (size_t)k * s.nat, b1,
                                      hipMemcpyHostToDevice, s.st));
            s.head = 0;
        }
        s.sync();
        s.leave_planned();
        s.mu_known = 0;
        s.solve(s.hist_row(0), 0.0, false);
        s.el_stale = false;
        s.push_mu();
        s.forces_parts(s.force);
        // the trajectory's kernel at the new state (its K r unless kr is
        // given); block mode restarts its direction history
        s.rank_prev = 0;
        if (s.full_mode()) {
            s.build_full_kernel();
            s.apply_full(s.r, s.kr);
        } else {
            s.build_kernel(s.d.kernel_rank, s.d.krylov_mode, false);
            s.apply_kernel(s.r, s.kr);
        }
        if (kr) XL_HIP(hipMemcpyAsync(s.kr, kr, b1, hipMemcpyHostToDevice, s.st));
        s.sync();
    });
}

int xlbomd_get_state(xlbomd_system *h, double *pos, double *vel, double *n_hist,
                     double *kr) {
    if (!h || !h->s) return fail(XLBOMD_E_INVALID, "null handle");
    return guarded([&] {
        SysBase &s = *h->s;
        const size_t b3 = 3 * s.nat * sizeof(double), b1 = s.nat * sizeof(double);
        if (pos) XL_HIP(hipMemcpyAsync(pos, s.pos, b3, hipMemcpyDeviceToHost, s.st));
        if (vel) XL_HIP(hipMemcpyAsync(vel, s.vel, b3, hipMemcpyDeviceToHost, s.st));
        if (n_hist)
            for (int k = 0; k <= s.d.kmax; ++k)
                XL_HIP(hipMemcpyAsync(n_hist + (size_t)k * s.nat, s.hist_row(k), b1,
                                      hipMemcpyDeviceToHost, s.st));
        if (kr) XL_HIP(hipMemcpyAsync(kr, s.kr, b1, hipMemcpyDeviceToHost, s.st));
        s.sync();
    });
}

int xlbomd_state_size(xlbomd_system *h, size_t *bytes) {
    if (!h || !h->s || !bytes) return fail(XLBOMD_E_INVALID, "null argument");
    return guarded([&] { *bytes = state_bytes(*h->s); });
}

int xlbomd_save_state(xlbomd_system *h, void *buf, size_t bytes) {
    if (!h || !h->s || !buf) return fail(XLBOMD_E_INVALID, "null argument");
    return guarded([&] {
        if (bytes < state_bytes(*h->s)) throw InvalidArg("checkpoint buffer too small");
        save_state(*h->s, static_cast<char *>(buf));
    });
}

int xlbomd_load_state(xlbomd_system *h, const void *buf, size_t bytes) {
    if (!h || !h->s || !buf) return fail(XLBOMD_E_INVALID, "null argument");
    return guarded([&] { load_state(*h->s, static_cast<const char *>(buf), bytes); });
}

int xlbomd_solve(xlbomd_system *h, const double *n, double *q_out, xlbomd_report *rep) {
    if (!h || !h->s || !n) return fail(XLBOMD_E_INVALID, "null argument");
    return guarded([&] {
        SysBase &s = *h->s;
        XL_HIP(hipMemcpyAsync(s.vtmp, n, s.nat * sizeof(double), hipMemcpyHostToDevice, s.st));
        s.el_stale = true;
        s.solve(s.vtmp, s.mu, s.mu_known > 0);
        if (q_out)
            XL_HIP(hipMemcpyAsync(q_out, s.q, s.nat * sizeof(double), hipMemcpyDeviceToHost, s.st));
        if (rep) {
            std::memset(rep, 0, sizeof(*rep));
            s.fill_report(rep);
        }
        s.sync();
    });
}

int xlbomd_response(xlbomd_system *h, int32_t count, const double *v, double *dq_out) {
    if (!h || !h->s || !v || !dq_out) return fail(XLBOMD_E_INVALID, "null argument");
    return guarded([&] {
        SysBase &s = *h->s;
        if (count < 1 || count > s.mcap) throw InvalidArg("count must be in 1..kernel capacity");
        XL_HIP(hipMemcpyAsync(s.vin, v, (size_t)count * s.nat * sizeof(double),
                              hipMemcpyHostToDevice, s.st));
        s.responses(count, s.vin, s.qp, nullptr);
        XL_HIP(hipMemcpyAsync(dq_out, s.qp, (size_t)count * s.nat * sizeof(double),
                              hipMemcpyDeviceToHost, s.st));
        s.sync();
    });
}

int xlbomd_kernel_apply(xlbomd_system *h, int32_t rank, const double *rr, double *kr_out) {
    if (!h || !h->s || !rr || !kr_out) return fail(XLBOMD_E_INVALID, "null argument");
    return guarded([&] {
        SysBase &s = *h->s;
        if (rank < -1 || rank > s.mcap) throw InvalidArg("rank above capacity");
        XL_HIP(hipMemcpyAsync(s.rdiag, rr, s.nat * sizeof(double), hipMemcpyHostToDevice, s.st));
        SysBase::DiagKernel scope(s);        // the trajectory's kernel stays
        s.rank_prev = 0;
        if (rank == -1) {
            s.build_full_kernel();
            s.apply_full(s.rdiag, s.vtmp);
        } else {
            s.build_kernel(rank, 0, false, false, s.rdiag);
            s.apply_kernel(s.rdiag, s.vtmp);
        }
        XL_HIP(hipMemcpyAsync(kr_out, s.vtmp, s.nat * sizeof(double), hipMemcpyDeviceToHost, s.st));
        s.sync();
    });
}

int xlbomd_scf(xlbomd_system *h, const double *n0, int32_t rank, double gamma, double tol,
               int32_t max_iter, double *n_out, double *rms_hist, int32_t *n_eval) {
    if (!h || !h->s || !n_eval) return fail(XLBOMD_E_INVALID, "null argument");
    if (max_iter < 0 || !(tol > 0.0) || !(gamma >= 0.0 && gamma <= 1.0))
        return fail(XLBOMD_E_INVALID, "scf: max_iter >= 0, tol > 0, gamma in [0, 1]");
    bool ok = false;
    const int rc = guarded([&] {
        SysBase &s = *h->s;
        if (rank < 0 || rank > s.mcap) throw InvalidArg("scf: rank above the kernel capacity");
        if (n0)
            XL_HIP(hipMemcpyAsync(s.ncur, n0, s.nat * sizeof(double), hipMemcpyHostToDevice, s.st));
        else
            XL_HIP(hipMemsetAsync(s.ncur, 0, s.nat * sizeof(double), s.st));
        *n_eval = 0;
        s.el_stale = true;
        SysBase::DiagKernel scope(s);        // the trajectory's kernel stays
        ok = s.scf_run(rank, gamma, tol, max_iter, rms_hist, n_eval);
        if (n_out)
            XL_HIP(hipMemcpyAsync(n_out, s.ncur, s.nat * sizeof(double), hipMemcpyDeviceToHost, s.st));
        s.sync();
    });
    if (rc == XLBOMD_OK && !ok) return fail(XLBOMD_E_NOCONV, "scf: tolerance not reached");
    return rc;
}

int xlbomd_profile(xlbomd_system *h, int32_t enable, double *out) {
    if (!h || !h->s) return fail(XLBOMD_E_INVALID, "null handle");
    return guarded([&] {
        SysBase &s = *h->s;
        s.sync();
        if (enable) {
            s.prof.on = true;
            s.prof.used = 0;
            s.prof.flops.clear();
            s.prof.cls.clear();
            return;
        }
        double acc[4][5] = {{0, 0, 0, 1e300, 0}, {0, 0, 0, 1e300, 0}, {0, 0, 0, 1e300, 0},
                            {0, 0, 0, 1e300, 0}};
        const size_t n = s.prof.used / 2;
        for (size_t i = 0; i < n; ++i) {
            float e = 0.0f;
            XL_HIP(hipEventElapsedTime(&e, s.prof.ev[2 * i], s.prof.ev[2 * i + 1]));
            double *a = acc[s.prof.cls[i]];
            a[0] += e;
            a[1] += s.prof.flops[i];
            a[2] += 1.0;
            a[3] = std::min(a[3], (double)e);
            a[4] = std::max(a[4], (double)e);
        }
        s.prof.on = false;
        if (out)
            for (int p = 0; p < 4; ++p) {
                if (acc[p][2] == 0.0) acc[p][3] = 0.0;
                for (int k = 0; k < 5; ++k) out[5 * p + k] = acc[p][k];
            }
    });
}

int xlbomd_selftest_gemm(int32_t n, int32_t precision, int32_t sym, const double *A,
                         const double *B, double *C) {
    if (n <= 0 || n % 128 || !A || !B || !C) return fail(XLBOMD_E_INVALID, "bad self-test args");
    if (precision != XLBOMD_FP64 && precision != XLBOMD_FP32 && precision != XLBOMD_MIXED_BF16X3)
        return fail(XLBOMD_E_INVALID, "self-test precision: FP64, FP32 or MIXED_BF16X3");
    return guarded([&] {
        const size_t nn = (size_t)n * n;
        double *dA = dalloc<double>(nn), *dB = dalloc<double>(nn), *dC = dalloc<double>(nn);
        DevFree fr;
        fr.ptrs = {dA, dB, dC};
        XL_HIP(hipMemcpy(dA, A, nn * 8, hipMemcpyHostToDevice));
        XL_HIP(hipMemcpy(dB, B, nn * 8, hipMemcpyHostToDevice));
        auto go = [&](auto tag) {
            using T = decltype(tag);
            T *a = dalloc<T>(nn), *b = dalloc<T>(nn), *c = dalloc<T>(nn);
            fr.ptrs.push_back(a); fr.ptrs.push_back(b); fr.ptrs.push_back(c);
            const int g = ceil_div((long)nn, 256);
            hipLaunchKernelGGL((convert_kernel<double, T>), dim3(g), dim3(256), 0, 0, (long)nn, dA, 1.0, a);
            hipLaunchKernelGGL((convert_kernel<double, T>), dim3(g), dim3(256), 0, 0, (long)nn, dB, 1.0, b);
            GemmArgs<T> ga;
            ga.n = n; ga.ld = n; ga.A0 = a; ga.B0 = b; ga.C = c;
            ga.split3 = precision == XLBOMD_MIXED_BF16X3;
            ga.ws_elems = split_ws_elems<T>(n, sym != 0, 0, 1);
            ga.ws = dalloc<T>(ga.ws_elems);
            fr.ptrs.push_back(ga.ws);
            gemm(ga, sym != 0, 0);
            hipLaunchKernelGGL((convert_kernel<T, double>), dim3(g), dim3(256), 0, 0, (long)nn, c, 1.0, dC);
        };
        if (precision == XLBOMD_FP64) go(double{}); else go(float{});
        XL_HIP(hipDeviceSynchronize());
        XL_HIP(hipMemcpy(C, dC, nn * 8, hipMemcpyDeviceToHost));
    });
}

int xlbomd_selftest_gemm_time(int32_t n, int32_t precision, int32_t sym, int32_t dual,
                              int32_t reps, double *ms_per_launch) {
    if (n <= 0 || n % 128 || reps <= 0 || !ms_per_launch)
        return fail(XLBOMD_E_INVALID, "bad self-test args");
    if (precision != XLBOMD_FP64 && precision != XLBOMD_FP32 && precision != XLBOMD_MIXED_BF16X3)
        return fail(XLBOMD_E_INVALID, "self-test precision: FP64, FP32 or MIXED_BF16X3");
    return guarded([&] {
        const size_t nn = (size_t)n * n;
        DevFree fr;
        auto go = [&](auto tag) {
            using T = decltype(tag);
            T *a = dalloc<T>(nn), *b = dalloc<T>(nn), *c = dalloc<T>(nn);
            fr.ptrs = {a, b, c};
            const unsigned nblk = (unsigned)((nn + 255) / 256);
            hipLaunchKernelGGL((fill_hash_kernel<T>), dim3(nblk), dim3(256), 0, nullptr,
                               (long)nn, 0x1705u, a);
            XL_LAUNCH_CHECK();
            hipLaunchKernelGGL((fill_hash_kernel<T>), dim3(nblk), dim3(256), 0, nullptr,
                               (long)nn, 0x10845u, b);
            XL_LAUNCH_CHECK();
            GemmArgs<T> ga;
            ga.n = n; ga.ld = n; ga.A0 = a; ga.B0 = b; ga.C = c;
            if (dual) { ga.A1 = b; ga.B1 = a; }
            ga.split3 = precision == XLBOMD_MIXED_BF16X3;
            ga.ws_elems = split_ws_elems<T>(n, sym != 0, dual, 1);
            ga.ws = dalloc<T>(ga.ws_elems);
            fr.ptrs.push_back(ga.ws);
            gemm(ga, sym != 0, 0);
            hipEvent_t e0, e1;
            XL_HIP(hipEventCreate(&e0));
            XL_HIP(hipEventCreate(&e1));
            XL_HIP(hipEventRecord(e0, 0));
            for (int r = 0; r < reps; ++r) gemm(ga, sym != 0, 0);
            XL_HIP(hipEventRecord(e1, 0));
            XL_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            XL_HIP(hipEventElapsedTime(&ms, e0, e1));
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            *ms_per_launch = ms / reps;
        };
        if (precision == XLBOMD_FP64) go(double{}); else go(float{});
    });
}

int xlbomd_selftest_gemm_presplit(int32_t n, int32_t sym, int32_t reps, const double *A,
                                  const double *B, double *C, double *ms_per_launch) {
    if (n <= 0 || n % 128 || reps < 0 || !A || !B || !C || (reps > 0 && !ms_per_launch))
        return fail(XLBOMD_E_INVALID, "bad self-test args");
    return guarded([&] {
        const size_t nn = (size_t)n * n;
        double *dA = dalloc<double>(nn), *dB = dalloc<double>(nn), *dC = dalloc<double>(nn);
        uint16_t *a = dalloc<uint16_t>(2 * nn), *b = dalloc<uint16_t>(2 * nn),
                 *c = dalloc<uint16_t>(2 * nn);
        SplitArgs ga;
        ga.n = n; ga.ld = n; ga.pl = (long)nn; ga.A0 = a; ga.B0 = b; ga.C = c;
        ga.hi_only = (sym & 2) != 0;
        sym &= 1;
        ga.ws_elems = split_bs_ws_elems(n, sym != 0, 0, 1);
        float *ws = dalloc<float>(ga.ws_elems);
        ga.ws = ws;
        DevFree fr;
        fr.ptrs = {dA, dB, dC, a, b, c, ws};
        XL_HIP(hipMemcpy(dA, A, nn * 8, hipMemcpyHostToDevice));
        XL_HIP(hipMemcpy(dB, B, nn * 8, hipMemcpyHostToDevice));
        const int g = ceil_div((long)nn, 256);
        hipLaunchKernelGGL(convert_split_kernel, dim3(g), dim3(256), 0, 0, (long)nn, dA, 1.0, a, (long)nn);
        hipLaunchKernelGGL(convert_split_kernel, dim3(g), dim3(256), 0, 0, (long)nn, dB, 1.0, b, (long)nn);
        gemm_split(ga, sym != 0, 0);
        hipLaunchKernelGGL(from_split_kernel, dim3(g), dim3(256), 0, 0, (long)nn, c, (long)nn, dC);
        XL_HIP(hipDeviceSynchronize());
        XL_HIP(hipMemcpy(C, dC, nn * 8, hipMemcpyDeviceToHost));
        if (reps > 0) {
            hipEvent_t e0, e1;
            XL_HIP(hipEventCreate(&e0));
            XL_HIP(hipEventCreate(&e1));
            XL_HIP(hipEventRecord(e0, 0));
            for (int r = 0; r < reps; ++r) gemm_split(ga, sym != 0, 0);
            XL_HIP(hipEventRecord(e1, 0));
            XL_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            XL_HIP(hipEventElapsedTime(&ms, e0, e1));
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            *ms_per_launch = ms / reps;
        }
    });
}

int xlbomd_selftest_logdet(int32_t n, int32_t nb, double shift, const double *A,
                           double *out) {
    if (n <= 0 || n % 128 || nb < 1 || nb > 1024 || !A || !out)
        return fail(XLBOMD_E_INVALID, "bad self-test args");
    if (!std::isfinite(shift)) return fail(XLBOMD_E_INVALID, "self-test shift must be finite");
    return guarded([&] {
        const size_t nn = (size_t)n * n;
        double *dA = dalloc<double>(nn), *batch = dalloc<double>(nn * nb);
        double *P = dalloc<double>((size_t)NB * n * nb), *dout = dalloc<double>(nb);
        DevFree fr;
        fr.ptrs = {dA, batch, P, dout};
        XL_HIP(hipMemcpy(dA, A, nn * 8, hipMemcpyHostToDevice));
        for (int b = 0; b < nb; ++b) {
            hipLaunchKernelGGL(add_diag_copy_kernel, dim3(ceil_div((long)nn, 256)), dim3(256), 0,
                               0, n, n, (const double *)dA, b * shift, batch + (size_t)b * nn);
            XL_LAUNCH_CHECK();
        }
        chol_logdet(n, n, nb, batch, (long)nn, P, (long)NB * n, nullptr, 0, dout, 0);
        XL_HIP(hipDeviceSynchronize());
        XL_HIP(hipMemcpy(out, dout, nb * sizeof(double), hipMemcpyDeviceToHost));
    });
}

int xlbomd_gemm_presplit_noalloc(int32_t n, int32_t sym, const void *A, const void *B,
                                 void *C, void *stream) {
    if (n <= 0 || n % 128 || n > 46336 || !A || !B || !C)
        return fail(XLBOMD_E_INVALID, "n must be a positive multiple of 128 up to 46336 and "
                                      "A, B, C device pointers");
    return guarded([&] {
        const long need = split_bs_ws_elems(n, sym != 0, 0, 1);
        if (need > kScratchFloats)
            throw InvalidArg("n = " + std::to_string(n) + (sym ? " (symmetric)" : "") +
                             ": the split-k partial tiles need " + std::to_string(4 * need) +
                             " bytes, above the " + std::to_string(4 * kScratchFloats) +
                             "-byte scratch array");
        SplitArgs ga;
        ga.n = n; ga.ld = n; ga.pl = (long)n * n;
        ga.A0 = static_cast<const uint16_t *>(A);
        ga.B0 = static_cast<const uint16_t *>(B);
        ga.C = static_cast<uint16_t *>(C);
        ga.ws = scratch_on_device();
        ga.ws_elems = kScratchFloats;
        gemm_split(ga, sym != 0, static_cast<hipStream_t>(stream));
    });
}

void xlbomd_destroy(xlbomd_system *h) {
    if (!h) return;
    if (h->s) {
        (void)hipStreamSynchronize(h->s->st);
        if (h->s->hscal) (void)hipHostFree(h->s->hscal);
        if (h->s->hps) (void)hipHostFree(h->s->hps);
        h->s->drop_graph();
        if (h->s->done_ev) (void)hipEventDestroy(h->s->done_ev);
        for (hipEvent_t e : h->s->prof.ev) (void)hipEventDestroy(e);
        for (hipEvent_t e : h->s->step_ev)
            if (e) (void)hipEventDestroy(e);
        if (h->s->own_stream) (void)hipStreamDestroy(h->s->st);
    }
    delete h;
}

const char *xlbomd_last_error(void) { return g_err.c_str(); }

const char *xlbomd_version(void) { return "xlbomd-gfx950 0.1"; }

}  // extern "C"
