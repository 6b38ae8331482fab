"""Writes the stored oracle values of the large workloads, at a fixed, seeded
charge vector n (PCG64 seed 11, mean removed):

  <name>_n<N>_sample.txt  (c3, c5): the chemical potential, the free
      energy and its parts, and for a seeded sample of 128 atoms the net
      charge, the canonical response dq/dlambda along the unit direction v1
      (Section V.B) and the force at fixed n (Eq. 40).
  c2_n4096_full.txt  (c2, 1024 atoms x 4 orbitals): mu, the free energy and
      its parts, and per atom the net charge q, the canonical responses
      dq/dlambda of q[n + lambda v] to two fixed unit directions v1, v2
      (Section V.B), K_4 r from the literal Sherman-Morrison sequence of
      rank-1 updates (Eqs. 48-51; K0 = -0.01 I, sequential directions from
      K0 r), and the forces at fixed n (Eq. 40).
  c2ov_n4096_full.txt  the same for the c2 system in a non-orthogonal
      basis (synth.with_overlap: overlap block -0.3 B / max|B|, the
      hopping's decay length; Section VI's SCC-DFTB setting): Loewdin
      solve, Mulliken charges from D S, Pulay forces.

Every value comes from the oracle (oracle/reference.py and its C loops: the
Fermi-Dirac density at fixed electron number of Section IV.B, Eq. 36, the
net Mulliken charges of Section VI, the closed-form canonical response by
divided differences, the explicit kernel sequence, the Hellmann-Feynman
forces and the eigenvalue entropy), with one substitution: numpy's eigh
stands in for the oracle's Jacobi sweeps, which are too slow at these sizes.
Nothing here calls the HIP library.

    python tests/golden/make_sample.py c2    (about five minutes of CPU)
    python tests/golden/make_sample.py c2ov  (about eight minutes)
    python tests/golden/make_sample.py c3    (about five minutes)
    python tests/golden/make_sample.py c5    (about half an hour, ~25 GB)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from synth import make_system, with_overlap   # noqa: E402
from oracle import reference as R      # noqa: E402

N_SEED, SAMPLE_SEED, N_SAMPLE = 11, 12, 128
DIR_SEEDS = (21, 22)
KERNEL_RANK = 4
KERNEL_GAMMA = 0.01          # K0 = -0.01 I for the stored K_4 r

SUBSTITUTION = ("# numpy's eigh stands in for the oracle's Jacobi sweeps at this size;\n"
                "# everything else is the oracle's (make_sample.py)\n")


def charge_vector(n_atoms):
    n = 0.02 * np.random.default_rng(N_SEED).standard_normal(n_atoms)
    return n - n.mean()


def unit_direction(n_atoms, seed):
    v = np.random.default_rng(seed).standard_normal(n_atoms)
    return v / np.linalg.norm(v)


def sample_atoms(n_atoms):
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(n_atoms, N_SAMPLE, replace=False))


def _eigh_rows(H):
    w, V = np.linalg.eigh(H)
    return w, np.ascontiguousarray(V.T)


def sample_path(name, n_orbitals):
    return os.path.join(HERE, f"{name}_n{n_orbitals}_sample.txt")


def full_path(name, n_orbitals):
    return os.path.join(HERE, f"{name}_n{n_orbitals}_full.txt")


def write_sample(name):
    s = make_system(name)
    m = R.Model(s)
    n = charge_vector(s.n_atoms)
    ref = R.electronic(m, s.pos, n, eig=_eigh_rows)
    print("solved", flush=True)
    en = R.free_energy(m, s.pos, ref)
    F = R.forces(m, s.pos, ref)
    dq = R.response(m, ref, unit_direction(s.n_atoms, DIR_SEEDS[0]))
    print("response", flush=True)
    atoms = sample_atoms(s.n_atoms)
    path = sample_path(name, s.n)
    with open(path, "w") as f:
        f.write(f"# oracle values of the {name} workload ({s.n_atoms} atoms x {s.n_orb} "
                f"orbitals, Te = {s.te})\n")
        f.write(f"# at n = 0.02 N(0,1) (PCG64 seed {N_SEED}, mean removed); "
                f"atoms sampled with seed {SAMPLE_SEED}\n")
        f.write("# D = 2 f(H[n]) at fixed electron number (Section IV.B, Eq. 36); mu;\n")
        f.write("# Omega = Tr[H0 D] + (2q - n)^T Gamma n / 2 + E_rep - Te S and its parts\n")
        f.write("# (Eqs. 35, 37, 38); per sampled atom: net Mulliken charge q (Section VI),\n")
        f.write(f"# the canonical response dq/dlambda along the unit direction v1 (N(0,1)\n")
        f.write(f"# with PCG64 seed {DIR_SEEDS[0]}, normalised; Section V.B), forces Fx Fy Fz\n")
        f.write(SUBSTITUTION)
        f.write(f"mu {ref.mu:.17e}\n")
        for k in ("omega", "e_band", "e_coul", "e_rep", "te_s"):
            f.write(f"{k} {en[k]:.17e}\n")
        f.write("# atom q dq_v1 Fx Fy Fz\n")
        for a in atoms:
            vals = [ref.q[a], dq[a], F[a, 0], F[a, 1], F[a, 2]]
            f.write(f"{a} " + " ".join(f"{v:.17e}" for v in vals) + "\n")
    print("wrote", path)


def read_sample(name, n_orbitals):
    """(scalars dict, sampled atom indices, per-atom array (n, 5)) of a
    sample file."""
    scal, atoms, rows = {}, [], []
    for line in open(sample_path(name, n_orbitals)):
        if line.startswith("#"):
            continue
        parts = line.split()
        if len(parts) == 2:
            scal[parts[0]] = float(parts[1])
        else:
            atoms.append(int(parts[0]))
            rows.append([float(x) for x in parts[1:]])
    return scal, np.array(atoms), np.array(rows)


def full_system(name):
    return with_overlap(make_system("c2")) if name == "c2ov" else make_system(name)


def write_full(name):
    s = full_system(name)
    m = R.Model(s)
    n = charge_vector(s.n_atoms)
    el = R.electronic(m, s.pos, n, eig=_eigh_rows)
    print("solved", flush=True)
    en = R.free_energy(m, s.pos, el)
    F = R.forces(m, s.pos, el)
    dq = [R.response(m, el, unit_direction(s.n_atoms, sd)) for sd in DIR_SEEDS]
    print("responses", flush=True)
    kres = R.kernel_sm(m, el, KERNEL_GAMMA, KERNEL_RANK, mode=0)
    assert kres.rank == KERNEL_RANK
    kr = kres.K @ el.r
    path = full_path(name, s.n)
    with open(path, "w") as f:
        f.write(f"# oracle values of the {name} workload ({s.n_atoms} atoms x {s.n_orb} "
                f"orbitals, Te = {s.te}) at n = 0.02 N(0,1)\n")
        f.write(f"# (PCG64 seed {N_SEED}, mean removed), positions as generated\n")
        f.write("# mu; Omega = Tr[H0 D] + (2q - n)^T Gamma n / 2 + E_rep - Te S and its\n")
        f.write("# parts (Eqs. 35, 37, 38); per atom: net charge q (Section VI),\n")
        f.write(f"# canonical responses dq/dlambda along unit directions v1, v2 (N(0,1)\n")
        f.write(f"# with PCG64 seeds {DIR_SEEDS[0]}, {DIR_SEEDS[1]}, normalised; Section V.B),\n")
        f.write(f"# K_{KERNEL_RANK} r with r = q - n from the Sherman-Morrison sequence of\n")
        f.write(f"# Eqs. 48-51 (K0 = -{KERNEL_GAMMA} I, sequential directions), forces Fx Fy Fz\n")
        if s.overlap_block is not None:
            f.write("# non-orthogonal basis (overlap block -0.3 B / max|B|, the hopping's decay\n")
            f.write("# length): Loewdin solve, Mulliken charges from D S, Pulay forces\n")
        f.write(SUBSTITUTION)
        f.write(f"mu {el.mu:.17e}\n")
        for k in ("omega", "e_band", "e_coul", "e_rep", "te_s"):
            f.write(f"{k} {en[k]:.17e}\n")
        f.write("# atom q dq_v1 dq_v2 K4r Fx Fy Fz\n")
        for a in range(s.n_atoms):
            vals = [el.q[a], dq[0][a], dq[1][a], kr[a], F[a, 0], F[a, 1], F[a, 2]]
            f.write(f"{a} " + " ".join(f"{v:.17e}" for v in vals) + "\n")
    print("wrote", path)


def read_full(name, n_orbitals):
    """(scalars dict, per-atom array of shape (n_atoms, 7)) of a full file."""
    scal, rows = {}, []
    for line in open(full_path(name, n_orbitals)):
        if line.startswith("#"):
            continue
        parts = line.split()
        if len(parts) == 2:
            scal[parts[0]] = float(parts[1])
        else:
            rows.append([float(x) for x in parts[1:]])
    return scal, np.array(rows)


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "c3"
    if which in ("c2", "c2ov"):
        write_full(which)
    else:
        write_sample(which)
