"""Writes <name>_n<N>_sample.txt: the oracle's charges on a seeded sample of
atoms of a workload at a fixed, seeded charge vector n, and its chemical
potential.  Workloads: c3 (small gap, 2048 atoms x 4 orbitals, N = 8192,
T_e = 0.02) and c5 (4096 randomly packed atoms x 4 orbitals, N = 16384).

Calls only the oracle (the Fermi-Dirac density of Section IV.B, Eq. 36,
at fixed electron number, and the net Mulliken charges of Section VI);
numpy's eigh stands in for the oracle's Jacobi sweeps at this size.

    python tests/golden/make_sample.py c3    (about two minutes of CPU)
    python tests/golden/make_sample.py c5    (about ten minutes, ~15 GB)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from synth import make_system          # noqa: E402
from oracle import reference as R      # noqa: E402

N_SEED, SAMPLE_SEED, N_SAMPLE = 11, 12, 128


def charge_vector(n_atoms):
    n = 0.02 * np.random.default_rng(N_SEED).standard_normal(n_atoms)
    return n - n.mean()


def sample_atoms(n_atoms):
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(n_atoms, N_SAMPLE, replace=False))


def _eigh_rows(H):
    w, V = np.linalg.eigh(H)
    return w, np.ascontiguousarray(V.T)


def sample_path(name, n_orbitals):
    return os.path.join(HERE, f"{name}_n{n_orbitals}_sample.txt")


def main(name):
    s = make_system(name)
    n = charge_vector(s.n_atoms)
    ref = R.electronic(R.Model(s), s.pos, n, eig=_eigh_rows)
    atoms = sample_atoms(s.n_atoms)
    path = sample_path(name, s.n)
    with open(path, "w") as f:
        f.write(f"# oracle charges of the {name} workload ({s.n_atoms} atoms x {s.n_orb} "
                f"orbitals, Te = {s.te})\n")
        f.write(f"# at n = 0.02 N(0,1) (PCG64 seed {N_SEED}, mean removed); "
                f"atoms sampled with seed {SAMPLE_SEED}\n")
        f.write("# D = 2 f(H[n]) at fixed electron number (Section IV.B, Eq. 36), net\n")
        f.write("# Mulliken charges (Section VI); written by make_sample.py from the\n")
        f.write("# oracle only\n")
        f.write(f"mu {ref.mu:.17e}\n")
        for a in atoms:
            f.write(f"{a} {ref.q[a]:.17e}\n")
    print("wrote", path)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "c3")
