"""Micro-benchmark of the dense product kernels (and a plain device copy).

    python -m paper_1705_10845_amd.kernel_bench [--n 4096] [--prec 0,1,3]
                                                [--reps 10] [--copy-gib 1]

Times the library's product kernels at n x n through the C ABI hooks
`xlbomd_selftest_gemm_time` / `xlbomd_selftest_gemm_presplit` for each
precision (0 FP64, 1 FP32, 3 split bf16x3 on FP32 operands, 4 split bf16x3
on pre-split operands, 5 plain bf16 on the hi planes of pre-split operands)
in three launch shapes (symmetric output, full output, two products
concatenated along k) and prints algorithmic TFLOP/s against the dense MFMA
peak.  With --copy-gib > 0 it first runs one device-to-device copy of that
size: under `rocprofv3 --pmc FETCH_SIZE` / `WRITE_SIZE` this copy is the
calibration of the counters (known bytes read and written).
"""
import argparse
import sys

PEAK = {0: 78.6, 1: 157.3, 3: 2500.0 / 3, 4: 2500.0 / 3, 5: 2500.0}
NAME = {0: "f64", 1: "f32", 3: "bf16x3", 4: "bf16x3 pre-split", 5: "bf16 pre-split"}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--prec", default="0,1,3")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--copy-gib", type=float, default=0.0)
    args = ap.parse_args(argv)
    if args.copy_gib > 0:
        import torch    # before the library: the copy runs on torch's runtime
    from . import binding as B
    B.lib()
    if args.copy_gib > 0:
        x = torch.ones(int(args.copy_gib * (1 << 30)) // 8, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        y = x.clone()
        torch.cuda.synchronize()
        del x, y
        print(f"copy: {args.copy_gib} GiB read, {args.copy_gib} GiB written", flush=True)
    n = args.n
    for prec in (int(p) for p in args.prec.split(",")):
        for sym, dual in ((True, False), (False, False), (True, True)):
            if prec in (4, 5):  # operands of the response recursion, pre-split
                if dual:
                    continue
                import numpy as np
                rng = np.random.default_rng(1)
                A = rng.standard_normal((n, n))
                A = A + A.T
                _, ms = B.selftest_gemm_presplit(A, A, sym=sym, reps=args.reps,
                                                 hi_only=prec == 5)
            else:
                ms = B.selftest_gemm_time(n, prec, sym, dual, reps=args.reps)
            ent = n * (n + 1) / 2 if sym else n * n
            tf = ent * 2 * n * (2 if dual else 1) / (ms * 1e-3) / 1e12
            print(f"n={n} {NAME[prec]} sym={sym} dual={dual}: {ms:.3f} ms/launch "
                  f"{tf:.1f} TFLOP/s ({100 * tf / PEAK[prec]:.0f}% of {PEAK[prec]:.1f})",
                  flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
