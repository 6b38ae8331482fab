"""Run an XL-BOMD trajectory and log it, one JSON object per line.

Each line is the report of one chunk of steps (the last step of the
chunk): step index, free energy Omega and its parts (band, Coulomb,
repulsion, T_e S), kinetic and total energy, RMS residual |q[n] - n|,
chemical potential, electron-count error, expansion levels, Newton-Schulz
iterations, chemical-potential reruns, kernel rank, the library's own time
for the step and the host wall time per step of the chunk.  Energy fields
are null for steps on which no energy was evaluated (the handle's
`energy_every` cadence).  `recover` restarts the electrons after a step
that reported a divergence.

    python -m paper_1705_10845_amd.trajectory --system c2 --steps 100 \\
        --every 10 --energy-every 10 --log c2.jsonl
"""
import argparse
import json
import sys
import time

import numpy as np

_ENERGY = ("omega", "e_band", "e_coul", "e_rep", "te_s", "e_kin", "e_total")
_ALWAYS = ("step", "rms_res", "mu", "d_nelec", "foe_levels", "ns_iters", "mu_reruns",
           "kernel_rank", "ms_step")


def record(rep, wall_ms_per_step):
    """The logged fields of one step report (a dict from XLBOMD.step)."""
    out = {k: rep[k] for k in _ALWAYS}
    has = bool(rep["has_energy"])
    out.update({k: (rep[k] if has else None) for k in _ENERGY})
    out["wall_ms_per_step"] = wall_ms_per_step
    return out


# status codes of the C ABI that a recovery answers
_DIVERGED, _NOCONV = -4, -3


def recover(md, tol=1e-8, max_iter=200, rank=1):
    """After a step reported a divergence: re-converge the electrons at the
    current positions by the kernel SCF from n = 0, and refill the charge
    history with the result (the initial boundary condition of the
    extended Lagrangian).  Returns the converged n; raises if the SCF does
    not converge."""
    n, hist, ok = md.scf(rank=rank, tol=tol, max_iter=max_iter)
    if not ok:
        raise RuntimeError(f"recovery SCF did not converge (RMS {hist[-1]:.2e} after "
                           f"{len(hist)} evaluations)")
    n = np.asarray(n, dtype=np.float64)
    md.set_state(n_hist=np.tile(n, (md.kmax + 1, 1)))
    return n


def run(md, steps, every=1, log=None, recover_on_divergence=False):
    """Take `steps` MD steps of the handle `md`, `every` at a time, and
    write each chunk's report as one JSON line to `log` (a path, a
    writable text file, or None).  With recover_on_divergence, a chunk that
    reports a divergence (or a failed chemical-potential solve) is followed
    by `recover` and a line {"event": "recovered", ...}, and the run goes
    on; the steps of that chunk are not repeated.  Returns the list of
    records."""
    from .binding import XlbomdError
    if steps < 0 or every < 1:
        raise ValueError("steps must be >= 0 and every >= 1")
    own = isinstance(log, str)
    fh = open(log, "w") if own else log
    recs = []

    def emit(r):
        recs.append(r)
        if fh is not None:
            fh.write(json.dumps(r) + "\n")
            fh.flush()

    try:
        done = 0
        while done < steps:
            k = min(every, steps - done)
            t0 = time.perf_counter()
            try:
                rep = md.step(k)
            except XlbomdError as e:
                if not recover_on_divergence or e.code not in (_DIVERGED, _NOCONV):
                    raise
                done += k
                n = recover(md)
                emit({"event": "recovered", "after_steps": done, "error": str(e),
                      "n_rms": float(np.sqrt(np.mean(n * n)))})
                continue
            wall = (time.perf_counter() - t0) * 1e3 / k
            done += k
            emit(record(rep, wall))
    finally:
        if own:
            fh.close()
    return recs


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--system", default="c2", help="synthetic workload c1, c2, c3 or c5")
    ap.add_argument("--precision", default="MIXED_BF16X3")
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--every", type=int, default=10, help="steps per logged line")
    ap.add_argument("--energy-every", type=int, default=10)
    ap.add_argument("--log", default=None, help="JSONL file (default: stdout)")
    args = ap.parse_args(argv)
    from synth import make_system
    from . import binding
    s = make_system(args.system)
    md = binding.XLBOMD(s, precision=getattr(binding, args.precision),
                        energy_every=args.energy_every)
    try:
        run(md, args.steps, args.every, args.log if args.log else sys.stdout)
    finally:
        md.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
