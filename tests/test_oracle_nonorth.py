"""Pins of the oracle's non-orthogonal basis (the SCC-DFTB setting of
Section VI: non-orthogonal atomic orbitals, Mulliken charges from D S, Pulay
forces) against facts other than the oracle itself: the generalised
eigenproblem from a library routine, a two-atom closed form worked by hand
(eigenvalues, chemical potential, Mulliken populations, free energy and the
force along the bond, Pulay term included), finite differences of the free
energy and of the charges, the orthogonal closed form as the S = I special
case, idempotency in the S metric at low temperature, and energy
conservation of the dynamics."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from synth import make_system, lattice_system, with_overlap
from oracle import reference as R


def _charges0(m):
    n = 0.05 * np.random.default_rng(1).standard_normal(m.nat)
    return n - n.mean()


def test_generalised_eigenproblem_matches_library():
    s = with_overlap(lattice_system(20, "c2", seed=3))
    m = R.Model(s)
    n = _charges0(m)
    el = R.electronic(m, s.pos, n)
    w, C = sla.eigh(el.H, el.S)            # LAPACK's generalised solver
    assert np.abs(np.sort(el.evals) - w).max() < 1e-12
    Co = el.eigvecs()
    assert np.abs(Co.T @ el.S @ Co - np.eye(m.N)).max() < 1e-12
    assert np.abs(el.H @ Co - el.S @ Co * el.evals[None, :]).max() < 1e-11
    # electron count in the S metric
    assert abs(np.trace(el.D @ el.S) - s.n_electrons) < 1e-10


def _ov_dimer(te=0.2, sov=0.3, rep=0.0):
    """Two atoms, one orbital each, equal onsite energies, two electrons."""
    r = 1.7
    pos = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
    s = make_system("c1").replace(
        n_atoms=2, pos=pos, vel=np.zeros((2, 3)), mass=np.ones(2),
        onsite=np.array([-0.2]), onsite_jitter=np.zeros(2),
        hop_block=np.array([[-1.0]]), hop_decay=1.0, hop_cutoff=4.0,
        taper_width=0.5, hubbard_u=np.array([1.0, 1.0]), n_electrons=2.0,
        te=te, rep_a=rep, overlap_block=np.array([[sov]]), overlap_decay=0.8)
    return s, R.Model(s), pos, r


def test_dimer_closed_form_nonorthogonal():
    """H = [[e, t], [t, e]], S = [[1, s], [s, 1]] (n = 0: H = H0), with
    t = -exp(-r), s = 0.3 exp(-r/0.8) below the taper: eigenvalues
    (e + t)/(1 + s) and (e - t)/(1 - s), eigenvectors [1, +-1]/sqrt(2(1 +- s)),
    mu halfway between them (one level per spin below, one above, two
    electrons), Mulliken populations f+ + f- = 1 on each atom (q = 0, while
    the diagonal of D alone is f+/(1+s) + f-/(1-s) != 1), band energy
    2 (f+ e+ + f- e-), and the force along the bond
    -2 (f+ de+/dr + f- de-/dr) with de/dr from the quotient rule: the
    Pulay term is the s'(r) part."""
    te = 0.2
    s, m, pos, r = _ov_dimer(te)
    e, t, so = -0.2, -math.exp(-r), 0.3 * math.exp(-r / 0.8)
    ep, em = (e + t) / (1 + so), (e - t) / (1 - so)
    mu = 0.5 * (ep + em)
    fp = 1.0 / (1.0 + math.exp((ep - mu) / te))
    fm = 1.0 / (1.0 + math.exp((em - mu) / te))
    el = R.electronic(m, pos, np.zeros(2))
    assert np.allclose(np.sort(el.evals), [ep, em], atol=1e-14, rtol=0)
    assert abs(el.mu - mu) < 1e-12
    Dcf = fp / (1 + so) * np.ones((2, 2)) + fm / (1 - so) * np.array([[1, -1], [-1, 1]])
    assert np.abs(el.D - Dcf).max() < 1e-13
    assert abs(el.D[0, 0] - 1.0) > 1e-3          # the diagonal alone is not the population
    assert np.abs(el.q).max() < 1e-13
    fe = R.free_energy(m, pos, el)
    assert abs(fe["e_band"] - 2 * (fp * ep + fm * em)) < 1e-13
    ent = -2 * sum(f * math.log(f) + (1 - f) * math.log(1 - f) for f in (fp, fm))
    assert abs(fe["te_s"] - te * ent) < 1e-13
    dt, ds = -t, -so / 0.8                        # d/dr of t = -e^{-r}, s
    dep = (dt * (1 + so) - (e + t) * ds) / (1 + so) ** 2
    dem = (-dt * (1 - so) + (e - t) * ds) / (1 - so) ** 2
    f_bond = -2.0 * (fp * dep + fm * dem)        # -dOmega/dr (n = 0: no Coulomb)
    F = R.forces(m, pos, el)
    assert abs(F[0, 0] + f_bond) < 1e-13 and abs(F[1, 0] - f_bond) < 1e-13
    assert np.abs(F[:, 1:]).max() < 1e-15


def test_forces_are_minus_gradient_nonorthogonal():
    s = with_overlap(lattice_system(8, "c2", seed=4), 0.4)
    m = R.Model(s)
    n = _charges0(m)
    F = R.forces(m, s.pos, R.electronic(m, s.pos, n))
    h = 1e-5
    for I in range(m.nat):
        for c in range(3):
            p = s.pos.copy()
            p[I, c] += h
            a = R.free_energy(m, p, R.electronic(m, p, n))["omega"]
            p[I, c] -= 2 * h
            b = R.free_energy(m, p, R.electronic(m, p, n))["omega"]
            assert abs(-(a - b) / (2 * h) - F[I, c]) < 2e-8, (I, c)


def test_response_matches_finite_difference_nonorthogonal():
    s = with_overlap(lattice_system(16, "c2", seed=5))
    m = R.Model(s)
    el = R.electronic(m, s.pos, _charges0(m))
    for seed in (2, 3):
        v = np.random.default_rng(seed).standard_normal(m.nat)
        v /= np.linalg.norm(v)
        a = R.response(m, el, v)
        b = R.response_fd(m, s.pos, el, v)
        assert np.abs(a - b).max() < 1e-7 * np.abs(a).max()
        assert abs(a.sum()) < 1e-12                 # canonical: Tr[D1 S] = 0


def test_unit_overlap_reduces_to_orthogonal_closed_forms():
    """A decay length so short that every overlap between atoms underflows
    to zero takes the non-orthogonal code path with S = I exactly; charges,
    density, energy, forces and responses equal the orthogonal path's
    (diagonal-perturbation closed form)."""
    s0 = lattice_system(12, "c2", seed=6)
    s1 = s0.replace(overlap_block=np.ones((4, 4)), overlap_decay=1e-3)
    m0, m1 = R.Model(s0), R.Model(s1)
    assert m1.nonorth and np.array_equal(m1.overlap(s0.pos), np.eye(m1.N))
    n = _charges0(m0)
    e0, e1 = R.electronic(m0, s0.pos, n), R.electronic(m1, s0.pos, n)
    assert e1.S is not None and e0.S is None
    assert np.abs(e0.D - e1.D).max() < 1e-12 and np.abs(e0.q - e1.q).max() < 1e-12
    f0, f1 = R.free_energy(m0, s0.pos, e0), R.free_energy(m1, s0.pos, e1)
    assert abs(f0["omega"] - f1["omega"]) < 1e-11
    assert np.abs(R.forces(m0, s0.pos, e0) - R.forces(m1, s0.pos, e1)).max() < 1e-11
    v = np.random.default_rng(4).standard_normal(m0.nat)
    assert np.abs(R.response(m0, e0, v) - R.response(m1, e1, v)).max() < 1e-11


def test_low_temperature_idempotent_in_the_overlap_metric():
    # 24 electrons in 48 orbitals: the s-like band filled, a gap of ~0.27
    s = with_overlap(lattice_system(12, "c2", seed=7)).replace(te=0.005, n_electrons=24.0)
    m = R.Model(s)
    el = R.electronic(m, s.pos, np.zeros(m.nat))
    k = int(s.n_electrons) // 2                  # doubly occupied levels
    gap = np.sort(el.evals)[k] - np.sort(el.evals)[k - 1]
    assert gap > 20 * s.te                       # a gapped filling
    P = 0.5 * el.D
    assert np.abs(P @ el.S @ P - P).max() < 1e-10
    assert abs(np.trace(el.D @ el.S) - s.n_electrons) < 1e-10


def test_no_energy_drift_nonorthogonal():
    s = with_overlap(make_system("c1"))
    m = R.Model(s)
    st, E = R.run(m, 150)
    et = np.array([e["e_total"] for e in E])
    ek = np.array([e["e_kin"] for e in E])
    slope = np.polyfit(np.arange(len(et)), et, 1)[0]
    assert ek.max() - ek.min() > 50 * et.std()  # energy is exchanged ...
    assert abs(slope) * len(et) < 2.0 * et.std() + 1e-6   # ... and conserved
