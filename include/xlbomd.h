/*
 * xlbomd.h - C ABI of the MI355X (gfx950) finite-temperature XL-BOMD library.
 *
 * Method: A. M. N. Niklasson, "Next generation extended Lagrangian first
 * principles molecular dynamics".  One library handle holds one system:
 * nuclear positions R, velocities, the extended electronic variable n (net
 * Mulliken charges per atom) with its Verlet history, and a low-rank kernel
 * K ~ (J - I)^-1.  A step is the integration scheme of Eqs. 22-23:
 *   - half kick and drift of the nuclei (velocity Verlet);
 *   - n(t+dt) = 2n(t) - n(t-dt) - kappa K r(t) + alpha sum_k c_k n(t-k dt)
 *     with the Table I coefficients (K_max = 5, 6 or 7);
 *   - H[n] = H0(R) + diag(Gamma n) (Section IV.A, SCC tight binding), the
 *     Fermi-Dirac density matrix D = 2 f(H) at fixed electron number
 *     (Section IV.B, Eq. 36), net charges q and the residual r = q - n;
 *   - Hellmann-Feynman forces at fixed n (the fixed-n derivative in Eq. 40);
 *   - the rank-m kernel from Sherman-Morrison updates of K0 = -gamma I
 *     (Eqs. 48-51) along Krylov directions whose responses dq/dv come from
 *     density-matrix perturbation theory (Section V.B);
 *   - the second half kick.
 *
 * Conventions:
 *   - All pointers in this header are HOST pointers.  Arrays passed in are
 *     caller-owned and copied during the call; device memory is owned by the
 *     library until xlbomd_destroy.
 *   - Every call returns an xlbomd_status.  No call aborts, no C++ exception
 *     crosses the ABI.  On failure xlbomd_last_error() (thread-local) gives a
 *     message.  A handle is not re-entrant: calls on one handle must not
 *     overlap.  Different handles may be used from different threads.
 *   - Layouts: positions/velocities/forces are n_atoms x 3 row-major doubles;
 *     per-atom vectors have n_atoms doubles; the orbital index of orbital a on
 *     atom I is I*n_orb + a.
 *   - Units are model units with k_B = 1 (te is an energy).
 *   - Everything crossing the ABI is FP64; the working precision of the dense
 *     matrix algebra is chosen by xlbomd_desc.precision.
 */
#ifndef XLBOMD_H
#define XLBOMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct xlbomd_system xlbomd_system;   /* opaque, library-owned */

typedef enum {
    XLBOMD_OK = 0,
    XLBOMD_E_INVALID = -1,   /* bad argument or descriptor                */
    XLBOMD_E_NOMEM = -2,     /* device allocation failed                  */
    XLBOMD_E_NOCONV = -3,    /* SCF or chemical-potential solve failed    */
    XLBOMD_E_DIVERGED = -4,  /* NaN/Inf or runaway residual detected      */
    XLBOMD_E_HIP = -5,       /* HIP runtime error                         */
    XLBOMD_E_STATE = -6      /* call not valid in the handle's state      */
} xlbomd_status;

typedef enum {
    XLBOMD_FP64 = 0,         /* every dense product in FP64 (FP64 MFMA)   */
    XLBOMD_FP32 = 1,         /* dense products in FP32 MFMA; mu, kernel
                                solve, Verlet and energy sums in FP64     */
    XLBOMD_MIXED = 2,        /* density-matrix expansion in FP64 MFMA (it
                                fixes charges, forces, energy); the
                                kernel's response products in FP32 MFMA   */
    XLBOMD_MIXED_BF16X3 = 3, /* split-precision bf16x3 products: each FP32
                                operand is split into bf16 hi + lo parts
                                and hi*hi + hi*lo + lo*hi is accumulated
                                in FP32 on the bf16 matrix cores (relative
                                error ~2^-16 per operand).  All response
                                products are split; in the expansion the
                                seed, A_k = I + 4 Z_k^2, Z_L^2 and D are
                                FP64, the inverse of A_k is split and
                                Z_{k+1} is refined against an FP64
                                residual of A_k Z_{k+1} = 2 Z_k (once per
                                level in a step: charges within ~1e-9 of
                                the FP64 path; twice inside an SCF whose
                                tolerance is below 1e-8)                   */
    XLBOMD_MIXED_BF16 = 4    /* the expansion of XLBOMD_MIXED_BF16X3 (the
                                same charges, forces and energy at a given
                                n) with plain bf16 response products: the
                                hi parts only, one bf16 matrix-core product
                                each (relative error ~2^-8 per operand).
                                The kernel is a preconditioner, so this
                                changes the path of n, not the accuracy of
                                the quantities computed from it          */
} xlbomd_precision;

/* Optional source of the device memory a system holds (PyTorch's caching
 * allocator, a pool, a fixed arena).  alloc returns `bytes` of device memory
 * on the current device, 256-byte aligned, or NULL (the call then fails
 * with XLBOMD_E_NOMEM); free returns a pointer alloc gave.  The library
 * calls alloc during xlbomd_init_system and, for buffers first needed
 * later (responses of a larger batch, the energy workspace), inside other
 * calls on the same handle, on the calling thread.  Every pointer goes back
 * through free in xlbomd_destroy, after the handle's stream has drained.
 * The struct is copied at init; ctx must stay valid until xlbomd_destroy. */
typedef struct {
    void *(*alloc)(size_t bytes, void *ctx);
    void (*free)(void *ptr, void *ctx);
    void *ctx;
} xlbomd_allocator;

/* System descriptor.  Model (SCC tight binding, orthogonal unless an
 * overlap block is given):
 *   H0[Ia,Ia] = onsite[a] + onsite_jitter[Ia]
 *   H0[Ia,Jb] = hop_block[a*n_orb+b] exp(-r/hop_decay) s(r), I != J, r < hop_cutoff
 *   s(r): 1 below hop_cutoff - taper_width, quintic C2 ramp to 0 at hop_cutoff
 *   Gamma[I,I] = hubbard_u[I], Gamma[I,J] = 1/sqrt(r^2 + gamma_soft^2)
 *   E_rep = sum_{I<J} rep_a exp(-r/rep_decay) s(r)
 *   H[n] = H0 + diag(Gamma n) on each atom's orbitals
 *   q_I = sum_a D[Ia,Ia] - n_electrons/n_atoms
 * In a non-orthogonal basis (overlap_block, Section VI's SCC-DFTB setting):
 *   S[Ia,Ib] = delta_ab, S[Ia,Jb] = overlap_block[a*n_orb+b] exp(-r/overlap_decay) s(r)
 *   H[n] = H0 + (S V + V S)/2, V = diag(Gamma n) on each atom's orbitals
 *   D = 2 f at the generalised eigenproblem H C = S C E (through X = S^-1/2)
 *   q_I = sum_a (D S)[Ia,Ia] - n_electrons/n_atoms (Mulliken)
 *   forces include -Tr[(V D + D V)/2 dS/dR] and the Pulay term Tr[E dS/dR]
 *   with the energy-weighted density matrix E */
typedef struct {
    int32_t n_atoms, n_orb;       /* n_orb in 1..8; N = n_atoms*n_orb at most
                                     46336, so that a padded N x N matrix has
                                     fewer than 2^31 elements               */
    const double *pos;            /* n_atoms*3                              */
    const double *vel;            /* n_atoms*3, NULL = zero                 */
    const double *mass;           /* n_atoms                                */
    const double *onsite;         /* n_orb                                  */
    const double *onsite_jitter;  /* n_atoms*n_orb, NULL = zero             */
    const double *hop_block;      /* n_orb*n_orb, symmetric                 */
    double hop_decay, hop_cutoff, taper_width;
    const double *hubbard_u;      /* n_atoms                                */
    double gamma_soft, rep_a, rep_decay;
    double n_electrons;           /* in (0, 2*n_atoms*n_orb)                */
    double te;                    /* electronic temperature, > 0            */
    double dt;                    /* time step, > 0                         */
    int32_t kmax;                 /* 5, 6 or 7: Table I row                 */
    int32_t kernel_rank;          /* m in 0..min(n_atoms, 16) (0 = K0 only) */
    int32_t kernel_every;         /* rebuild the kernel every k steps (>=1) */
    int32_t krylov_mode;          /* 0 sequential Krylov (v_{j+1} from this
                                     build's w_j = (J - I) v_j), 1 block (v_1
                                     and the previous build's w_j, all m
                                     responses in one batch), 2 full
                                     kernel (J - I)^-1 from n_atoms responses
                                     in batches of min(kernel_rank, 16),
                                     rebuilt every kernel_every steps; the
                                     initial SCF still uses rank kernel_rank */
    double k0_gamma;              /* K0 = -k0_gamma I, in (0, 1]; 0 = choose
                                     at init from the stiffest response mode:
                                     20 power iterations v <- -Jv/|Jv| from
                                     r/|r| give |lambda|, and gamma =
                                     1.5/(1+|lambda|) rounded down to two
                                     significant digits, in [1e-4, 1]       */
    int32_t precision;            /* xlbomd_precision                       */
    double scf_tol;               /* RMS residual of the initial SCF        */
    int32_t scf_max_iter;
    int32_t energy_every;         /* energy evaluation period (0 = never
                                     inside xlbomd_step)                    */
    void *stream;                 /* hipStream_t to run on; NULL = library's
                                     own stream.  Every call synchronises
                                     with this stream before it returns
                                     (the chemical potential, the level
                                     count and the kernel's rank are
                                     decided on the host from device
                                     values), so calls cannot be captured
                                     into a HIP graph                       */
    const xlbomd_allocator *allocator; /* device memory source; NULL =
                                     hipMalloc / hipFree                    */
    int32_t foe_levels;           /* 0: the smallest level count meeting the
                                     truncation target foe_tol on the
                                     spectral interval; 1..40: that count,
                                     raised where the seed would leave
                                     |x / 2^(L+1)| <= 1                     */
    double foe_tol;               /* truncation target of the expansion, the
                                     largest deviation of the L-level map
                                     from the Fermi function on the
                                     interval: 0 = 2e-10 (FP64) / 1e-9
                                     (other precisions); else in
                                     [1e-14, 1e-3]                          */
    double mu_tol;                /* the expansion is rerun at the corrected
                                     chemical potential while beta |dmu| is
                                     above this: 0 = 1e-6 (FP64) / 1e-3
                                     (other precisions); else in
                                     [1e-12, 1e-1]                          */
    int32_t kernel_otf;           /* on-the-fly rank-1 updates between
                                     rebuilds (Section V.E), 0 = none: at
                                     every step that does not rebuild, the
                                     previous step's kernel K0 gets one
                                     rank-1 update along K0 r / |K0 r|
                                     (orthogonalised against the kept
                                     directions, response at the current
                                     state); up to kernel_otf such directions
                                     are kept after the rebuild's, the oldest
                                     leaving first.  kernel_rank + kernel_otf
                                     <= 16                                  */
    const double *overlap_block;  /* n_orb*n_orb, symmetric: the overlap
                                     block of a non-orthogonal basis (model
                                     above), or NULL for an orthogonal one.
                                     Needs XLBOMD_FP64 and host decisions
                                     (step mode 0); positions where S is not
                                     positive definite fail with
                                     XLBOMD_E_NOCONV                        */
    double overlap_decay;         /* overlap decay length, > 0 with a block */
} xlbomd_desc;

typedef struct {
    double omega;      /* shadow free energy Omega[n](R)                    */
    double e_band, e_coul, e_rep, te_s;  /* its parts: Tr[H0 D], Coulomb,
                                            repulsion, Te * S               */
    double e_kin;      /* nuclear kinetic energy                            */
    double e_total;    /* e_kin + omega: the constant of motion             */
    double rms_res;    /* RMS of r = q[n] - n                               */
    double mu;         /* chemical potential                                */
    double d_nelec;    /* Tr D - n_electrons after the mu correction        */
    int32_t step;      /* steps taken since init                            */
    int32_t foe_levels, ns_iters, mu_reruns, scf_iters, kernel_rank;
    int32_t has_energy;/* 1 if the energy fields are valid                  */
    double k0_gamma;   /* the K0 constant in use                            */
    double ms_step;    /* device time of the reported step in milliseconds
                          (HIP events on the handle's stream; xlbomd_step
                          only, 0 elsewhere)                                 */
} xlbomd_report;

/* Create a system: copies the descriptor's arrays to the device, solves the
 * ground state by the kernel SCF of Eq. 52 from n = 0 to RMS(r) <= scf_tol,
 * sets the initial conditions of Eq. 20 (history filled with n(t0)),
 * computes F(t0) and the kernel at t0.  On success *out owns the handle. */
int xlbomd_init_system(const xlbomd_desc *desc, xlbomd_system **out);

/* Advance n_steps XL-BOMD steps (Eqs. 22-23).  The free energy is
 * evaluated on steps whose index is a multiple of desc.energy_every.  If
 * last != NULL the report of the final step is written (its energy fields
 * are valid when has_energy is 1; xlbomd_forces evaluates them on demand).
 * Returns XLBOMD_E_DIVERGED if a non-finite value or a residual above 1e3
 * appears.  A runaway residual is caught right after the step's solve,
 * before its forces are computed: positions and velocities are left at the
 * half step (moved by the previous forces only).  To go on, restore a
 * checkpoint taken with xlbomd_get_state via xlbomd_set_state, or converge
 * the electrons at the current positions (xlbomd_scf) and set the charge
 * history to the result with xlbomd_set_state. */
int xlbomd_step(xlbomd_system *h, int32_t n_steps, xlbomd_report *last);

/* Advance n_steps steps of `count` independent systems concurrently.  When
 * every handle takes planned steps (xlbomd_set_step_mode 1 or 2) one host
 * thread enqueues each system's step on its own stream (a graph replay in
 * mode 2) before waiting for any, so the device runs them together;
 * otherwise each handle is stepped by its own host thread.  Handles must
 * be distinct and must not share a stream (shared streams serialise).
 * reports (count entries) and status (count entries) are optional.
 * Returns the first failing status, with the system index in
 * xlbomd_last_error(); the other systems still advance. */
int xlbomd_step_batch(xlbomd_system *const *hs, int32_t count, int32_t n_steps,
                      xlbomd_report *reports, int32_t *status);

/* How xlbomd_step and xlbomd_step_batch take a step.
 *   0 (default): host decisions.  The level count of the expansion and its
 *     Newton-Schulz schedule follow the step's spectral interval, the
 *     expansion is rerun until the chemical potential is within the
 *     threshold, and the Krylov directions stop at a breakdown; each of
 *     these reads device values back to the host.
 *   1: planned steps.  A plan (level count and schedule for the last
 *     interval widened by a margin, xlbomd_set_plan_margin) is made on the
 *     host; every decision of a
 *     step is then taken on the device: the interval and the predicted
 *     chemical potential are checked against the plan, one rerun of the
 *     expansion at the corrected chemical potential runs only when needed
 *     (its launches skip themselves otherwise), D gets the second-order
 *     correction, and the kernel's rank comes from the direction norms.
 *     One synchronisation per step reads the step's status.  A step that
 *     leaves its plan (interval beyond it, chemical potential not within the
 *     threshold after one rerun, a non-finite value) is taken again with
 *     host decisions from the state saved at its start, and the next step
 *     is planned anew.
 *   2: as 1, with each step replayed from a HIP graph captured once per
 *     plan (the first step of a plan runs directly, the second is captured).
 * Modes 1 and 2 need krylov_mode 0, kernel_every 1 and kernel_otf 0
 * (XLBOMD_E_INVALID otherwise).  Steps that evaluate the energy do so after
 * the planned step, with host synchronisation. */
int xlbomd_set_step_mode(xlbomd_system *h, int32_t mode);

/* One planned step in two halves, for a caller that steps many systems
 * from one thread and starts each system's next step as soon as its last
 * one is done.  xlbomd_step_begin enqueues the step (step mode 1 or 2, else
 * XLBOMD_E_STATE) and returns at once.  xlbomd_step_end finishes it: with
 * wait == 0 it returns with *done = 0 while the device is still busy with
 * the step, else (or once the step is done) it commits the step as
 * xlbomd_step would (taking it again with host decisions if it left its
 * plan, evaluating the energy on a step of the energy cadence), writes the
 * report if rep != NULL and sets *done = 1.  Between the two calls no
 * other call may use the handle; xlbomd_step and xlbomd_step_batch return
 * XLBOMD_E_STATE on a handle with a step begun and not ended. */
int xlbomd_step_begin(xlbomd_system *h);
int xlbomd_step_end(xlbomd_system *h, int32_t wait, int32_t *done, xlbomd_report *rep);

/* Headroom of a plan: the level count and schedule are sized for the last
 * spectral interval widened by (1 + margin) around the predicted chemical
 * potential (0.25 by default; more headroom means more levels and fewer
 * new plans).  In [-0.9, 10]; a negative margin makes every planned step
 * leave its plan, so each is taken again with host decisions (a check of
 * that path).  The next planned step makes a new plan. */
int xlbomd_set_plan_margin(xlbomd_system *h, double margin);

/* Counters of planned steps since init: out[0] planned steps taken, out[1]
 * of them replayed from a graph, out[2] graphs captured, out[3] planned
 * steps that left their plan and were taken again with host decisions. */
int xlbomd_step_stats(xlbomd_system *h, int64_t *out);

/* Rebuild the low-rank kernel at the current state with rank `rank`
 * (<= 0 keeps the descriptor's rank) and refresh K r (Eqs. 50-51). */
int xlbomd_kernel_update(xlbomd_system *h, int32_t rank);

/* Copy the current forces (n_atoms*3) and, if energy != NULL, evaluate and
 * return the energy terms at the current state. */
int xlbomd_forces(xlbomd_system *h, double *forces, xlbomd_report *energy);

/* Current n(t) and q[n(t)] (n_atoms each; either may be NULL). */
int xlbomd_get_charges(xlbomd_system *h, double *n_out, double *q_out);

/* Overwrite the dynamical state: positions and velocities (n_atoms*3), the
 * n history (kmax+1 rows of n_atoms: n(t), n(t-dt), ...) and the stored
 * K r(t) used for the next n update (n_atoms).  Any of them may be NULL to
 * keep the current value.  The electronic solve, the forces and the
 * trajectory's kernel are recomputed at the new state (kr, if given, is
 * kept as passed); the chemical-potential history restarts from that
 * solve and the step count is kept.  This is a frozen-state entry point
 * (parity checks, perturbations); an exact checkpoint of everything the
 * next step reads is xlbomd_save_state / xlbomd_load_state. */
int xlbomd_set_state(xlbomd_system *h, const double *pos, const double *vel,
                     const double *n_hist, const double *kr);

/* Read the dynamical state (same layouts as xlbomd_set_state). */
int xlbomd_get_state(xlbomd_system *h, double *pos, double *vel,
                     double *n_hist, double *kr);

/* Checkpoint / resume.  A checkpoint holds everything the next step reads:
 * positions, velocities and forces, the n history of Eq. 23, K r(t), the
 * trajectory's kernel (directions V, W = J V - V, the previous build's
 * W for block mode, the full kernel of krylov_mode 2), the chemical-potential
 * history that predicts the next solve's mu, the step count and the K0
 * constant.  Stepping a handle after xlbomd_load_state repeats, bit for
 * bit, what the saved handle did after xlbomd_save_state.
 *   xlbomd_state_size: *bytes = the checkpoint size of this handle.
 *   xlbomd_save_state: writes the checkpoint into buf (caller-owned host
 *     memory of at least xlbomd_state_size bytes; `bytes` is its size).
 *   xlbomd_load_state: restores a checkpoint written by a handle with the
 *     same descriptor (atoms, orbitals, kmax, kernel capacity, Krylov mode,
 *     precision); XLBOMD_E_INVALID otherwise or if `bytes` does not match.
 *     Charges, forces and energies asked for before the next step are
 *     evaluated at the restored state. */
int xlbomd_state_size(xlbomd_system *h, size_t *bytes);
int xlbomd_save_state(xlbomd_system *h, void *buf, size_t bytes);
int xlbomd_load_state(xlbomd_system *h, const void *buf, size_t bytes);

/* Electronic solve at the current positions for the charge vector n
 * (n_atoms): writes q[n] (n_atoms) and, if rep != NULL, mu, RMS(q-n) and
 * the FOE statistics.  Does not change the dynamical state; a later
 * xlbomd_forces energy, xlbomd_get_charges or xlbomd_kernel_update first
 * solves again at the MD state. */
int xlbomd_solve(xlbomd_system *h, const double *n, double *q_out,
                 xlbomd_report *rep);

/* Canonical first-order response dq/dlambda of q[n + lambda v] at the last
 * xlbomd_solve (Section V.B), for `count` directions v (count rows of
 * n_atoms), written to dq_out (count rows of n_atoms). */
int xlbomd_response(xlbomd_system *h, int32_t count, const double *v,
                    double *dq_out);

/* Apply the rank-m kernel built at the last xlbomd_solve to r (n_atoms):
 * kr_out = K_m r (Eq. 50 in closed Woodbury form), the first direction
 * along K0 r and the next ones sequential Krylov directions; rank = -1
 * applies the full kernel (J - I)^-1 of Eq. 43 (krylov_mode 2
 * construction).  The kernel is built in storage of its own: the
 * trajectory's kernel, applied between rebuilds, is not changed. */
int xlbomd_kernel_apply(xlbomd_system *h, int32_t rank, const double *r,
                        double *kr_out);

/* Ground state by the kernel SCF of Eq. 52 (Section V.F, Section VI), at
 * the handle's current nuclear positions and independent of its MD state:
 * starting from n0 (n_atoms host array; NULL = zeros) iterate
 *   n <- n - K_m (q[n] - n)
 * with a fresh rank-m kernel per iteration, built from sequential Krylov
 * directions and canonical responses (rank 0: K0 = -gamma I alone, i.e.
 * linear mixing), until RMS(q[n] - n) <= tol or max_iter kernel updates.
 * rank <= min(kernel_rank, 16) of the descriptor; gamma in (0, 1] replaces
 * the handle's K0 constant for this call (0 keeps it).
 * Outputs (each nullable except n_eval): n_out (n_atoms) the last n;
 * rms_hist (max_iter + 1 entries) the RMS residual of every evaluated n;
 * *n_eval the number of evaluations.  XLBOMD_E_NOCONV if tol was not
 * reached within max_iter kernel updates (the outputs are still written).
 * XLBOMD_E_DIVERGED if an iterate could not be evaluated (no chemical
 * potential, non-finite spectral bounds) or its RMS residual is above 1e3;
 * *n_eval and rms_hist then cover the evaluations before it, n_out is not
 * written.  The MD history, K r and the trajectory's kernel are not
 * touched (the SCF's kernels are built in storage of their own). */
int xlbomd_scf(xlbomd_system *h, const double *n0, int32_t rank, double gamma, double tol,
               int32_t max_iter, double *n_out, double *rms_hist, int32_t *n_eval);

/* Live timing of the dense MFMA products.  enable != 0 starts recording a
 * HIP event pair on the handle's stream around every product launched by
 * later calls; enable == 0 stops and, if out != NULL, writes 20 doubles:
 * out[0..4] for FP64 products, out[5..9] for FP32 products, out[10..14]
 * for split bf16x3 products and out[15..19] for plain bf16 products, each
 *   {total kernel milliseconds, total algorithmic flops (2 n_k flops per
 *    output entry on the real n x n block; symmetric outputs count n(n+1)/2
 *    entries), number of launches, shortest launch ms, longest launch ms}. */
int xlbomd_profile(xlbomd_system *h, int32_t enable, double *out);

/* Kernel-level test hook: C = A B with the library's dense product kernel
 * (A must be symmetric; it is read as A^T).  n x n row-major host arrays,
 * n a positive multiple of 128; precision XLBOMD_FP64, XLBOMD_FP32 (the
 * inputs are rounded to it) or XLBOMD_MIXED_BF16X3 (inputs rounded to FP32,
 * split bf16x3 product); sym != 0 computes only the upper block
 * triangle and mirrors it (valid when A B is symmetric).  Synchronous. */
int xlbomd_selftest_gemm(int32_t n, int32_t precision, int32_t sym, const double *A,
                         const double *B, double *C);

/* Benchmark hook for the same kernel: average milliseconds per launch over
 * `reps` back-to-back launches on n x n device operands filled with
 * pseudo-random values in [-1, 1) (dual != 0: two products concatenated
 * along k, as in the response). */
int xlbomd_selftest_gemm_time(int32_t n, int32_t precision, int32_t sym, int32_t dual,
                              int32_t reps, double *ms_per_launch);

/* Kernel-level test hook for the split product on pre-split operands (the
 * MIXED_BF16X3 response recursion): A and B (n x n row-major host arrays,
 * n a positive multiple of 128) are rounded to FP32 and stored as bf16
 * hi/lo planes; C = A B^T, i.e. C[i][j] = sum_k A[i][k] B[j][k], with the
 * result itself stored split and returned as hi + lo.  Bit 0 of sym
 * computes the upper block triangle and mirrors it (valid when A B^T is
 * symmetric); bit 1 multiplies the hi planes only (the plain bf16 product
 * of XLBOMD_MIXED_BF16).  With
 * reps > 0 the product is then launched reps more times and *ms_per_launch
 * receives the average time.  Synchronous. */
int xlbomd_selftest_gemm_presplit(int32_t n, int32_t sym, int32_t reps, const double *A,
                                  const double *B, double *C, double *ms_per_launch);

/* Kernel-level test hook for the batched FP64 log-determinant behind the
 * electronic entropy of the free energy (the Fermi-Dirac entropy term of
 * the Mermin functional, evaluated as log-determinants of the expansion's
 * level matrices): slot b < nb of the batch holds A + b shift I, and
 * out[b] receives its ln det.  A is an n x n row-major symmetric positive
 * definite host array (only its lower triangle is read), n a positive
 * multiple of 128, nb >= 1; every slot must stay positive definite
 * (a non-positive pivot gives NaN).  The slots are factorised as one
 * batch, as in the entropy evaluation.  Synchronous. */
int xlbomd_selftest_logdet(int32_t n, int32_t nb, double shift, const double *A,
                           double *out);

/* The split product of xlbomd_selftest_gemm_presplit on device operands,
 * allocating nothing: for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  A, B and C are device pointers to n x n row-major matrices
 * stored as two bf16 planes, hi then lo n*n elements later (the value is
 * hi + lo); C = A B^T, i.e. C[i][j] = sum_k A[i][k] B[j][k] (sym != 0: the
 * upper block triangle is computed and mirrored, valid when A B^T is
 * symmetric); C must not overlap A or B.  n is a positive multiple of 128
 * up to 46336 whose split-k partial tiles fit the library's fixed scratch
 * array of 32 MiB per device: every such n except some between 2176 and
 * 3712, which return XLBOMD_E_INVALID naming the bytes needed.  The call is
 * enqueued on `stream` (a hipStream_t; NULL = the null stream) and returns
 * without waiting.  Every call on a device shares that device's scratch
 * array, which keeps the last call's partial tiles: calls that overlap on
 * one device (other streams, other threads) race. */
int xlbomd_gemm_presplit_noalloc(int32_t n, int32_t sym, const void *A, const void *B,
                                 void *C, void *stream);

void xlbomd_destroy(xlbomd_system *h);

/* Message of the last failed call on this thread ("" if none). */
const char *xlbomd_last_error(void);

/* Library version string. */
const char *xlbomd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* XLBOMD_H */
