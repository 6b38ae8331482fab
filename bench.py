"""Benchmark: XL-BOMD steps/s on one MI355X for the N = 4096 workload.

Workload: 1024 atoms x 4 orbitals (s + 3p) on a jittered 8x8x16 cubic
lattice, Te = 0.05, rank-4 sequential-Krylov kernel rebuilt every step,
Table I K_max = 5 integrator.  `value` is the mixed path: the density-matrix
expansion in FP64 MFMA (it fixes charges, forces and energy, which then meet
the FP64 tolerances) and the kernel's response products as split bf16x3
products on the bf16 matrix cores (FP32 accumulation); the chemical
potential, Krylov solve, Verlet and energy sums are FP64.  The same path
with FP32 response products, the FP64-plain path (at the mixed path's
accuracy targets, which `mixed_over_fp64` compares against, and at its own
tighter ones) and the all-FP32 path are timed the same way beside it, then
the serving stream (independent systems of 16-512 atoms arriving as a
Poisson process, p50/p99 step latency) and the oracle's CPU baseline.

Prints one JSON line.  The oracle (test infrastructure) is used only for the
CPU baseline leg.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# dense MFMA TFLOP/s, MI355X; a split bf16x3 product is three bf16 products,
# so its algorithmic peak is a third of the bf16 rate
PEAK = {"f32": 157.3, "f64": 78.6, "bf3": 2500.0 / 3, "bf16": 2500.0}
KERNEL = {"f64": "gemm_tn_kernel<double>", "f32": "gemm_tn_kernel<float>",
          "bf3": "split bf16x3 products: gemm_bw_kernel (256 x 128 tiles, pre-split "
                 "operands) with its split-k fix-up",
          "bf16": "plain bf16 products: gemm_bw_kernel on the hi planes only"}


def _sync():
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.synchronize()
    except ImportError:
        pass


def _stream():
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except ImportError:
        pass
    return None


ENERGY_EVERY = 10   # free-energy report cadence (every 10th step, in the timed region)

# HBM bytes per launch of each product class in this workload's timed
# region (product kernel + its split-k fix-up, averaged over the launches),
# from `rocprofv3 --pmc FETCH_SIZE` and `--pmc WRITE_SIZE` runs of this
# script scaled by the same counters' readings for a 1 GiB device copy
# (profiles/gemm_hbm_traffic_n4096.md).  Valid only for the product-kernel
# source they were measured with.
GEMM_SRC = [os.path.join(ROOT, "paper_1705_10845_amd", "csrc", f)
            for f in ("gemm.hpp", "gemm_split.hpp")]
TRAFFIC = {"sha256": "65676722a64c06bf94bba9af8e9ba6be2ff18ba3432808deebfa9bc7c4a1c7f5",
           "f64": 3.333e9, "bf3": 7.166e8}


def gemm_src_hash():
    h = hashlib.sha256()
    for p in GEMM_SRC:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic(key):
    return TRAFFIC.get(key) if gemm_src_hash() == TRAFFIC["sha256"] else None


def time_path(system, precision, steps, warmup, label, **kw):
    from paper_1705_10845_amd import XLBOMD
    t0 = time.perf_counter()
    g = XLBOMD(system, precision=precision, stream=_stream(),
               scf_tol=2e-5 if precision == 1 else 1e-9, energy_every=ENERGY_EVERY, **kw)
    t_init = time.perf_counter() - t0
    print(f"[bench] {label}: init (SCF) {t_init:.1f}s", file=sys.stderr, flush=True)
    if warmup:
        g.step(warmup, report=False)
    _sync()
    g.profile_start()
    t0 = time.perf_counter()
    rep = g.step(steps, report=True)
    _sync()
    dt = time.perf_counter() - t0
    prof = g.profile_stop()
    print(f"[bench] {label}: {steps} steps in {dt:.3f}s, rms res {rep['rms_res']:.2e}, "
          f"L={rep['foe_levels']}, reruns={rep['mu_reruns']}", file=sys.stderr, flush=True)
    g.close()
    return dict(steps_per_s=steps / dt, ms_per_step=1e3 * dt / steps, prof=prof,
                report=rep, init_s=t_init)


def _oracle_step_seconds(n_atoms, threads):
    """Wall time of one oracle XL-BOMD step (Jacobi diagonalisation,
    closed-form responses of the rank-4 kernel, forces, Verlet) on an
    n_atoms sub-lattice of the N = 4096 workload's model, with `threads`
    OpenMP threads for the oracle's parallel loops."""
    import ctypes
    import numpy as np
    from synth import lattice_system
    from oracle import reference as R
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(threads))
    except OSError:
        pass
    s = lattice_system(n_atoms, "c2", seed=17050002)
    m = R.Model(s)
    st = R.State(pos=s.pos.copy(), vel=s.vel.copy(), force=np.zeros((m.nat, 3)),
                 n_hist=np.zeros((s.kmax + 1, m.nat)), kr=np.zeros(m.nat),
                 K=None, V=None, el=None)
    t0 = time.perf_counter()
    R.md_step(m, st, gamma=0.01, want_energy=False)
    return time.perf_counter() - t0


def cpu_baseline():
    """The oracle timed on a ladder of sizes and extrapolated to N = 4096.

    One oracle step at N = 256 and N = 512 (64 and 128 atoms of the same
    model) on one thread fixes the cost exponent p; the N = 4096 step time
    is the N = 512 time times 8^p.  The dominant cost, the cyclic Jacobi
    sweeps, is single-threaded; the N = 512 step is also timed with every
    host core given to the oracle's OpenMP loops (responses, density)."""
    import math
    t256 = _oracle_step_seconds(64, 1)
    t512 = _oracle_step_seconds(128, 1)
    cores = os.cpu_count() or 1
    t512_all = _oracle_step_seconds(128, cores)
    p = math.log(t512 / t256) / math.log(2.0)
    t4096 = t512 * 8.0 ** p
    return {"value": 1.0 / t4096, "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": f"one oracle step (Jacobi, rank-4 kernel, forces) at N=256 and N=512 "
                      f"on one thread: {t256:.2f}s and {t512:.2f}s, cost ~N^{p:.2f}, "
                      f"extrapolated to {t4096:.0f}s per step at N=4096; the N=512 step "
                      f"with {cores} threads for the OpenMP loops took {t512_all:.2f}s "
                      f"(the Jacobi sweeps are serial)",
            "ladder_s": {"N256_1thread": t256, "N512_1thread": t512,
                         f"N512_{cores}threads": t512_all},
            "exponent": p, "extrapolated_s_per_step_N4096": t4096}


def serving(n_requests=64, slots=8, budget_gib=96, step_mode=0):
    """The serving workload: Poisson stream (200/s) of independent systems,
    16-512 atoms x 4 orbitals, Te U[0.02, 0.1], rank 2-6, 100 steps each,
    admitted by HBM footprint; the headline (MIXED_BF16X3) precision.
    Eight systems run at once: they already keep the GPU busy, and each
    further one stretches every running system's step (host-decision mode
    on this stream: 4 slots 400 steps/s at p99 26.5 ms, 8 slots 435 at
    53.4 ms, 16 slots 421 at 120 ms, 32 slots 400 at 191 ms).
    step_mode 2: planned steps replayed from each system's graph, all
    systems driven from one host thread; 0: host decisions, one worker
    thread per running system."""
    from synth import serving_stream
    from paper_1705_10845_amd.serve import Server
    from paper_1705_10845_amd import MIXED_BF16X3
    stream = serving_stream(n_requests)
    srv = Server(hbm_budget=budget_gib << 30, max_slots=slots, precision=MIXED_BF16X3,
                 steps=100, verbose=False, step_mode=step_mode)
    stats, summ = srv.run(stream)
    if summ["errors"]:
        print("[bench] serving errors:", [s.error for s in stats if s.error][:3], file=sys.stderr)
    summ["slots"] = slots
    summ["workload"] = (f"first {n_requests} requests of the stream: 16-512 atoms x 4 "
                        "orbitals (log-uniform), "
                        "Poisson 200/s, Te U[0.02,0.1], rank U{2..6}, 100 steps each, "
                        "MIXED_BF16X3")
    print(f"[bench] serving (step mode {step_mode}): {summ['total_steps']} steps in "
          f"{summ['wall_s']:.1f}s, p50 {summ['p50_step_ms']:.2f} ms, p99 "
          f"{summ['p99_step_ms']:.2f} ms", file=sys.stderr, flush=True)
    return summ


def time_graph(system, precision, steps, warmup):
    """Steps/s of the same workload with planned steps replayed from a HIP
    graph (no per-product timing in this mode)."""
    from paper_1705_10845_amd import XLBOMD
    g = XLBOMD(system, precision=precision, stream=_stream(), scf_tol=1e-9,
               energy_every=ENERGY_EVERY)
    g.set_step_mode(2)
    if warmup:
        g.step(max(warmup, 2), report=False)
    _sync()
    t0 = time.perf_counter()
    rep = g.step(steps, report=True)
    _sync()
    dt = time.perf_counter() - t0
    st = g.step_stats()
    g.close()
    print(f"[bench] mixed, planned graph steps: {steps} steps in {dt:.3f}s, {st}",
          file=sys.stderr, flush=True)
    return {"value": steps / dt, "ms_per_step": 1e3 * dt / steps, "steps": steps,
            "foe_levels": rep["foe_levels"], "stats": st}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-mixed-fp32", action="store_true",
                    help="skip the mixed path with FP32 response products")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving leg (p50/p99 step latency)")
    ap.add_argument("--serving-requests", type=int, default=64)
    ap.add_argument("--no-bf16", action="store_true",
                    help="skip the plain-bf16 response tier (XLBOMD_MIXED_BF16)")
    ap.add_argument("--no-nonorth", action="store_true",
                    help="skip the FP64 leg of the workload in a non-orthogonal basis")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the planned-graph leg of the headline workload")
    ap.add_argument("--serving-only", action="store_true")
    ap.add_argument("--only", choices=["mixed_bf16", "nonorth"],
                    help="time one other leg alone (for kernel traces of it)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: every system is stepped on one "
              "device (independent systems shard by system, without "
              "communication); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    from synth import make_system, with_overlap
    from paper_1705_10845_amd import FP32, FP64, MIXED, MIXED_BF16, MIXED_BF16X3
    s = make_system("c2")
    if args.serving_only:
        t0 = time.perf_counter()
        summ = serving(args.serving_requests)
        summ["wall_total_s"] = time.perf_counter() - t0
        print(json.dumps({"serving": summ}), flush=True)
        return

    if args.only:
        sysm, prec = ((s, MIXED_BF16) if args.only == "mixed_bf16"
                      else (with_overlap(s), FP64))
        r = time_path(sysm, prec, args.steps, args.warmup, args.only)
        print(json.dumps({args.only: {"value": r["steps_per_s"], "ms_per_step": r["ms_per_step"],
                                      "steps": args.steps, "warmup": args.warmup,
                                      "foe_levels": r["report"]["foe_levels"]}}), flush=True)
        return

    mixed = time_path(s, MIXED_BF16X3, args.steps, args.warmup, "mixed (bf16x3 responses)")
    mixed32 = None if args.no_mixed_fp32 else time_path(s, MIXED, args.steps, 1,
                                                        "mixed (FP32 responses)")
    # the same expansion with plain bf16 response products (the BF16 tier)
    mixed16 = None if args.no_bf16 else time_path(s, MIXED_BF16, args.steps, 1,
                                                  "mixed (plain bf16 responses)")
    # FP64 at the mixed path's accuracy targets (truncation 1e-9, mu rerun
    # threshold 1e-3), and at its own tighter defaults (2e-10, 1e-6)
    fp64 = None if args.no_fp64 else time_path(s, FP64, args.fp64_steps, 1,
                                                "fp64 (mixed targets)", foe_tol=1e-9,
                                                mu_tol=1e-3)
    fp64t = None if args.no_fp64 else time_path(s, FP64, args.fp64_steps, 1,
                                                 "fp64 (FP64 targets)")
    fp32 = None if args.no_fp32 else time_path(s, FP32, args.steps, 1, "fp32")
    # the same workload in a non-orthogonal basis (overlap, Loewdin solve,
    # Mulliken charges from D S, Pulay forces): FP64 at its own targets
    nonorth = None if args.no_nonorth else time_path(with_overlap(s), FP64, args.fp64_steps, 1,
                                                     "fp64, non-orthogonal basis")

    def roof(prof, steps):
        # the dominant product class of the step (the most kernel time)
        key = max(PEAK, key=lambda k: prof[k]["ms"])
        p = prof[key]
        ach = p["flops"] / (p["ms"] * 1e-3) / 1e12 if p["ms"] > 0 else 0.0
        return {"bound": "mfma", "achieved": ach, "peak": PEAK[key], "unit": "TFLOP/s",
                "frac": ach / PEAK[key], "traffic": traffic(key), "kernel": KERNEL[key],
                "launches": p["launches"], "avg_launch_ms": p["ms"] / max(1, p["launches"]),
                "gemm_ms_per_step": p["ms"] / steps,
                "other_classes_ms_per_step": {k: prof[k]["ms"] / steps for k in PEAK
                                              if k != key and prof[k]["ms"] > 0}}

    def summary(r, steps):
        out = {"value": r["steps_per_s"], "ms_per_step": r["ms_per_step"], "steps": steps,
               "foe_levels": r["report"]["foe_levels"], "mu_reruns_last": r["report"]["mu_reruns"]}
        for k in PEAK:
            p = r["prof"][k]
            if p["ms"] > 0:
                out[f"mfma_{k}_tflops"] = p["flops"] / (p["ms"] * 1e-3) / 1e12
                out[f"gemm_{k}_ms_per_step"] = p["ms"] / steps
        return out

    out = {
        "metric": "MD steps/s at N=4096 (mixed vs FP64 plain), % MFMA peak, p99 step latency",
        "value": mixed["steps_per_s"],
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+bf16x3",
        "data": "synthetic",
        "config": {"workload": "c2: 1024 atoms x 4 orbitals (N=4096) jittered cubic "
                               "lattice, Te=0.05, rank-4 sequential Krylov kernel every "
                               "step, K0 from the stability rule, K_max=5, free energy "
                               "every 10th step; mixed "
                               "path: density-matrix expansion with an FP64 "
                               "sparse-dense seed, FP64 MFMA A_k, residuals, Z_L^2 "
                               "and D, level inverses in split bf16x3 refined against "
                               "FP64 residuals; split bf16x3 MFMA kernel responses "
                               "(FP32 accumulation); FP64 mu/Krylov/Verlet/energy sums",
                   "n_orbitals": 4096, "kernel_rank": 4, "energy_every": ENERGY_EVERY,
                   "foe_levels": mixed["report"]["foe_levels"]},
        "roofline": roof(mixed["prof"], args.steps),
        "mixed": summary(mixed, args.steps),
    }
    if mixed32 is not None:
        out["mixed_fp32_responses"] = summary(mixed32, args.steps)
    if mixed16 is not None:
        out["mixed_bf16_responses"] = summary(mixed16, args.steps)
        out["mixed_bf16_responses"]["precision"] = (
            "XLBOMD_MIXED_BF16: the headline's expansion (same charges, forces and energy "
            "at a given n), plain bf16 response products (the BF16 tier)")
    if fp64 is not None:
        # equal accuracy: both paths at truncation 1e-9 and mu threshold 1e-3
        out["fp64_plain"] = summary(fp64, args.fp64_steps)
        out["fp64_plain"]["targets"] = "foe_tol 1e-9, mu_tol 1e-3 (the mixed path's)"
        out["mixed_over_fp64"] = mixed["steps_per_s"] / fp64["steps_per_s"]
        out["fp64_plain_own_targets"] = summary(fp64t, args.fp64_steps)
        out["fp64_plain_own_targets"]["targets"] = "foe_tol 2e-10, mu_tol 1e-6"
        out["mixed_over_fp64_own_targets"] = mixed["steps_per_s"] / fp64t["steps_per_s"]
    if fp32 is not None:
        out["fp32"] = summary(fp32, args.steps)
    if nonorth is not None:
        out["fp64_nonorthogonal"] = summary(nonorth, args.fp64_steps)
        out["fp64_nonorthogonal"]["workload"] = (
            "the same system with overlap block -0.3 B / max|B| (hopping block B) and the "
            "hopping's decay length; FP64, Newton-Schulz S^-1/2 per step, dense X H X seed")
    if not args.no_graph:
        out["mixed_planned_graph"] = time_graph(s, MIXED_BF16X3, args.steps, args.warmup)
    if not args.no_serving:
        # host decisions (a worker thread per running system) serve this
        # stream faster than planned steps replayed from graphs, whose
        # every step also launches the (mostly skipped) rerun expansion
        out["serving"] = serving(args.serving_requests, step_mode=0)
        out["serving_planned_graphs"] = serving(args.serving_requests, step_mode=2)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
