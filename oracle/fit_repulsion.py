"""Choose the pair-repulsion prefactor A of a synthetic model (oracle tool).

The workloads specify hopping and Coulomb terms but no repulsive pair term;
without one the band energy is purely attractive and a cluster collapses.
SCC-DFTB carries a repulsive pair potential (Section VI), so the model adds
E_rep = sum_{I<J} A exp(-r/decay) s(r) with A fixed once per model: the value
for which the unjittered lattice has zero virial sum_I F_I . (R_I - R_c) at
the self-consistent ground state.  The virial is linear in A, so two
evaluations fix it.

Usage: python -m oracle.fit_repulsion c1
"""
import sys

import numpy as np

from synth import CONFIGS, make_system
from . import reference as R


def virial(model, pos, el):
    F = R.forces(model, pos, el)
    c = pos.mean(axis=0)
    return float(np.sum(F * (pos - c)))


def fit(name, dims=None):
    cfg = CONFIGS[name]
    s = make_system(name)
    # unjittered lattice of the same model (optionally a smaller box)
    nx, ny, nz = dims or cfg["dims"]
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz),
                             indexing="ij"), -1).reshape(-1, 3) * cfg["spacing"]
    nat = g.shape[0]
    s = s.replace(pos=g.astype(float), n_atoms=nat,
                  onsite_jitter=np.zeros(nat * s.n_orb),
                  hubbard_u=s.hubbard_u[:nat], mass=s.mass[:nat],
                  vel=np.zeros((nat, 3)), n_electrons=float(nat * s.n_orb))
    w = []
    for a in (0.0, 1.0):
        m = R.Model(s.replace(rep_a=a))
        el, _ = R.scf(m, s.pos, s.k0_gamma, s.rank, tol=1e-10, max_iter=500)
        w.append(virial(m, s.pos, el))
    a = -w[0] / (w[1] - w[0])
    return a


if __name__ == "__main__":
    for name in sys.argv[1:]:
        print(name, fit(name))
