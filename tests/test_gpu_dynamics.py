"""GPU dynamics against the oracle: kernel modes, refresh cadence, the mixed
path's one-step parity, and long-run energy conservation."""
import os

import numpy as np
import pytest

from synth import make_system, lattice_system
from oracle import reference as R

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1705_10845_amd as P
    P.lib()
    return P


def _traj(P, s, steps, precision, check_every=1):
    m = R.Model(s)
    st = R.init_state(m, scf_tol=1e-11)
    g = P.XLBOMD(s, precision=precision, scf_tol=1e-11)
    worst = dict(dq=0.0, dF=0.0, dn=0.0)
    for i in range(steps):
        st = R.md_step(m, st, want_energy=False)
        g.step(1, report=False)
        if (i + 1) % check_every == 0:
            F, _ = g.forces(energy=False)
            n, q = g.charges()
            worst["dq"] = max(worst["dq"], np.abs(q - st.el.q).max())
            worst["dF"] = max(worst["dF"], np.abs(F - st.force).max())
            worst["dn"] = max(worst["dn"], np.abs(n - st.el.n).max())
    g.close()
    return worst


def test_block_krylov_mode_trajectory(P):
    """krylov_mode 1: v1 plus the previous build's directions, one batched
    response launch (small-gap model, rank 3)."""
    s = lattice_system(40, "c3", seed=12, rank=3, krylov_mode=1, k0_gamma=0.1)
    w = _traj(P, s, 30, P.FP64)
    print("block mode 30 steps:", {k: f"{v:.2e}" for k, v in w.items()})
    # small-gap model: the charge Jacobian reaches |J| ~ 90, so the charges
    # carry the rounding-level growth of n amplified by |J|
    assert w["dn"] < 1e-8 and w["dF"] < 1e-5
    assert w["dq"] < 1e-8 + 100.0 * w["dn"]


def test_kernel_refresh_every_k_trajectory(P):
    """kernel rebuilt every 4th step, applied to each step's residual."""
    s = lattice_system(40, "c2", seed=13, rank=2, kernel_every=4)
    w = _traj(P, s, 24, P.FP64)
    print("refresh every 4, 24 steps:", {k: f"{v:.2e}" for k, v in w.items()})
    assert w["dq"] < 1e-8 and w["dF"] < 1e-5 and w["dn"] < 1e-8


def test_mixed_one_step(P):
    s = lattice_system(40, "c2", seed=3)
    m = R.Model(s)
    st = R.init_state(m, scf_tol=1e-11)
    for _ in range(3):
        st = R.md_step(m, st)
    ref = R.md_step(m, st)
    g = P.XLBOMD(s, precision=P.MIXED, scf_tol=1e-9)
    g.set_state(pos=st.pos, vel=st.vel, n_hist=st.n_hist, kr=st.kr)
    g.step(1, report=False)
    state = g.get_state()
    n, q = g.charges()
    F, e = g.forces()
    dq = np.abs(q - ref.el.q).max()
    dF = np.abs(F - ref.force).max()
    dO = abs(e["omega"] - ref.energy["omega"]) / abs(ref.energy["omega"])
    dkr = np.abs(state["kr"] - ref.kr).max() / np.abs(ref.kr).max()
    print(f"MIXED one step: dq {dq:.2e} dF {dF:.2e} rel dOmega {dO:.2e} rel dKr {dkr:.2e}")
    assert dq < 1e-8 and dF < 1e-5 and dO < 1e-8 and dkr < 1e-3
    g.close()


def test_energy_conservation_10k_steps_c1(P):
    """10^4 steps of the 64-atom cluster (FP64): no systematic drift of the
    shadow-Hamiltonian total energy, fluctuation of the oracle's size."""
    s = make_system("c1")
    g = P.XLBOMD(s, precision=P.FP64, scf_tol=1e-11, energy_every=10)
    E, res = [], []
    for blk in range(1000):
        rep = g.step(10)
        assert rep["has_energy"] == 1
        E.append(rep["e_total"])
        res.append(rep["rms_res"])
    g.close()
    E = np.array(E)
    t = np.arange(E.size)
    slope = np.polyfit(t, E, 1)[0]
    drift = abs(slope) * E.size
    print(f"10^4 steps: total energy mean {E.mean():.6f} std {E.std():.2e} "
          f"linear drift over run {drift:.2e}, mean RMS residual {np.mean(res):.2e}")
    # the cluster evaporates within a few hundred steps (largest neighbour
    # count 30 -> 2-9), so the run is one chaotic realisation: two
    # realisations that differ only in rounding give a fitted drift of 1.8
    # and 2.1 std and a first-to-last-quarter shift of 1.2 and 1.4 std
    q = E.size // 4
    assert drift < 3.0 * E.std() + 1e-6
    assert abs(E[-q:].mean() - E[:q].mean()) < 2.0 * E.std() + 1e-6
    assert E.std() < 5e-3


def test_auto_gamma_matches_oracle(P):
    s = lattice_system(40, "c4", seed=17, rank=3)
    assert s.k0_gamma == 0.0
    m = R.Model(s)
    st = R.init_state(m, scf_tol=1e-10)
    g = P.XLBOMD(s, precision=P.FP64, scf_tol=1e-10)
    rep = g.step(2)
    st = R.md_step(m, R.md_step(m, st, want_energy=False), want_energy=False)
    n, q = g.charges()
    print("auto gamma", rep["k0_gamma"], "oracle", m.gamma_used, "dq", np.abs(q - st.el.q).max())
    assert rep["k0_gamma"] == m.gamma_used
    assert np.abs(q - st.el.q).max() < 1e-8
    g.close()


def test_mixed_split_one_step(P):
    """MIXED_BF16X3: FP64 expansion, split bf16x3 response products.  One
    step from the oracle's state: n, charges, forces and energy at FP64
    tolerances (the step applies the kernel of the state it starts from);
    the new K r, built from split responses, to 1e-3 relative."""
    s = lattice_system(40, "c2", seed=3)
    m = R.Model(s)
    st = R.init_state(m, scf_tol=1e-11)
    for _ in range(3):
        st = R.md_step(m, st)
    ref = R.md_step(m, st)
    g = P.XLBOMD(s, precision=P.MIXED_BF16X3, scf_tol=1e-9)
    g.set_state(pos=st.pos, vel=st.vel, n_hist=st.n_hist, kr=st.kr)
    g.step(1, report=False)
    state = g.get_state()
    n, q = g.charges()
    F, e = g.forces()
    dq = np.abs(q - ref.el.q).max()
    dn = np.abs(state["n_hist"][0] - ref.n_hist[0]).max()
    dF = np.abs(F - ref.force).max()
    dO = abs(e["omega"] - ref.energy["omega"]) / abs(ref.energy["omega"])
    dkr = np.abs(state["kr"] - ref.kr).max() / np.abs(ref.kr).max()
    print(f"MIXED_BF16X3 one step: dn {dn:.2e} dq {dq:.2e} dF {dF:.2e} "
          f"rel dOmega {dO:.2e} rel dKr {dkr:.2e}")
    assert dq < 1e-8 and dn < 1e-10 and dF < 1e-5 and dO < 1e-8 and dkr < 1e-3


@pytest.mark.parametrize("kmax", [6, 7])
def test_table_I_rows_trajectory(P, kmax):
    """Table I rows K_max = 6 and 7 (kappa, alpha, c_k) against the oracle."""
    s = make_system("c1", kmax=kmax)
    w = _traj(P, s, 40, P.FP64)
    print(f"K_max {kmax}, 40 steps:", {k: f"{v:.2e}" for k, v in w.items()})
    assert w["dq"] < 1e-8 and w["dF"] < 1e-5 and w["dn"] < 1e-8


def test_full_kernel_apply_matches_oracle(P):
    """krylov_mode 2: K = (J - I)^-1 from all N_at responses, dense FP64
    Gauss-Jordan, against the oracle's dense inverse."""
    s = lattice_system(40, "c2", seed=9)
    m = R.Model(s)
    g = P.XLBOMD(s.replace(rank=8), precision=P.FP64, scf_tol=1e-9)
    n = 0.05 * np.random.default_rng(4).standard_normal(s.n_atoms)
    n -= n.mean()
    g.solve(n)
    el = R.electronic(m, s.pos, n)
    kr = g.kernel_apply(-1, el.r)
    ref = R.kernel_full(m, el) @ el.r
    err = np.abs(kr - ref).max() / np.abs(ref).max()
    print(f"full kernel K r rel err {err:.2e}")
    g.close()
    assert err < 1e-8


def test_full_kernel_trajectory(P):
    """Full kernel rebuilt every 5 steps in the dynamics (c1, 30 steps)."""
    s = make_system("c1", krylov_mode=2, kernel_every=5, rank=16)
    w = _traj(P, s, 30, P.FP64)
    print("full kernel 30 steps:", {k: f"{v:.2e}" for k, v in w.items()})
    assert w["dq"] < 1e-8 and w["dF"] < 1e-5 and w["dn"] < 1e-8


def test_checkpoint_resume(P):
    """get_state / set_state: a run resumed from a checkpoint in a fresh
    handle continues the original trajectory (to the solver tolerances)."""
    s = lattice_system(40, "c2", seed=21)
    g = P.XLBOMD(s, precision=P.MIXED_BF16X3, scf_tol=1e-10)
    g.step(4, report=False)
    ck = g.get_state()
    g.step(4, report=False)
    n_a, q_a = g.charges()
    F_a, _ = g.forces(energy=False)
    g.close()
    h = P.XLBOMD(s, precision=P.MIXED_BF16X3, scf_tol=1e-10)
    h.set_state(pos=ck["pos"], vel=ck["vel"], n_hist=ck["n_hist"], kr=ck["kr"])
    h.step(4, report=False)
    n_b, q_b = h.charges()
    F_b, _ = h.forces(energy=False)
    h.close()
    dn, dq, dF = np.abs(n_a - n_b).max(), np.abs(q_a - q_b).max(), np.abs(F_a - F_b).max()
    print(f"resume after 4 + 4 steps: dn {dn:.1e} dq {dq:.1e} dF {dF:.1e}")
    # n differs by the mu-solve tolerance (the resumed run has no mu history
    # to predict from); the charges carry it amplified by |J|
    assert dn < 1e-8 and dq < 1e-8 + 100.0 * dn and dF < 1e-6


def test_divergence_is_reported(P):
    """K0 = -I on the stiff s+3p model puts modes of K0 (J - I) near -70, far
    outside the electronic integrator's stability range: the run blows up
    and the library reports it as an error (diverged or no convergence)."""
    s = lattice_system(40, "c2", seed=1, k0_gamma=1.0, rank=1)
    with pytest.raises(P.XlbomdError) as e:
        g = P.XLBOMD(s, precision=P.FP64, scf_tol=1e-10, scf_max_iter=60)
        try:
            g.step(200, report=False)
        finally:
            g.close()
    print("error code", e.value.code, str(e.value))
    assert e.value.code in (-3, -4)


def _eigh_rows(H):
    w, V = np.linalg.eigh(H)
    return w, np.ascontiguousarray(V.T)


_C2_REF = {}


def _c2_oracle(s, n):
    """The oracle's solve of the N = 4096 workload at n (eigh for Jacobi),
    shared by the tests at this size."""
    key = n.tobytes()
    if key not in _C2_REF:
        _C2_REF[key] = R.electronic(R.Model(s), s.pos, n, eig=_eigh_rows)
    return _C2_REF[key]


def test_split_expansion_matches_fp64_at_n4096(P):
    """The 4096-orbital workload the bench times, at a fixed n.

    Against the oracle's solve (Jacobi replaced by numpy's eigh at this
    size; its Fermi bisection, density and Mulliken charges unchanged): a
    diagonal element of D = 2 f(H) is a convex combination of 2 f over the
    spectrum, so it is off by at most twice the expansion's truncation
    bound (2e-10 FP64, 1e-9 the other modes) and an atom's 4 orbitals by 8
    times it, i.e. 1.6e-9 (FP64) and 8e-9 (MIXED_BF16X3) before rounding and
    the chemical potential's tolerance.

    MIXED shares the 1e-9 target (8e-9 per atom).  FP32 does not meet the
    1e-6 bound at this size (test_fp32_expansion_at_n4096).

    Between the two GPU paths: MIXED_BF16X3 runs the inverse of every level
    in split bf16x3 and refines Z_{k+1} once against an FP64 residual; its
    charges agree with the FP64 path's to the truncation bounds plus the
    refinement's accuracy (error of Y times error of Z~, ~1e-10)."""
    s = make_system("c2")
    n = 0.02 * np.random.default_rng(6).standard_normal(s.n_atoms)
    n -= n.mean()
    ref = _c2_oracle(s, n)
    out = {}
    for prec in (P.FP64, P.MIXED_BF16X3, P.MIXED):
        g = P.XLBOMD(s, precision=prec, scf_tol=1e-9)
        q, rep = g.solve(n)
        out[prec] = q
        g.close()
        err = np.abs(q - ref.q).max()
        print(f"N=4096 precision {prec}: charges vs oracle {err:.2e}, "
              f"mu {rep['mu']:.12f} vs {ref.mu:.12f}")
    assert np.abs(out[P.FP64] - ref.q).max() < 2e-9
    assert np.abs(out[P.MIXED_BF16X3] - ref.q).max() < 1e-8
    # MIXED: FP64 expansion with the 1e-9 target
    assert np.abs(out[P.MIXED] - ref.q).max() < 1e-8
    dq = np.abs(out[P.FP64] - out[P.MIXED_BF16X3]).max()
    print(f"N=4096 charges, split path vs FP64 path: {dq:.2e}")
    assert dq < 1e-8


@pytest.mark.xfail(reason="XLBOMD_FP32 has no higher-precision refinement: besides "
                   "the rounding of beta (H - mu) (~eps32 beta |H| on the near-mu "
                   "levels), every FP32 product over k = 4096 carries ~eps32 sqrt(k) "
                   "relative error, and the recursion doubles errors near mu at each "
                   "of its 5 levels: ~1e-5 against the 1e-6 bound", strict=False)
def test_fp32_expansion_at_n4096(P):
    s = make_system("c2")
    n = 0.02 * np.random.default_rng(6).standard_normal(s.n_atoms)
    n -= n.mean()
    ref = _c2_oracle(s, n)
    g = P.XLBOMD(s, precision=P.FP32, scf_tol=2e-5)
    q, rep = g.solve(n)
    g.close()
    err = np.abs(q - ref.q).max()
    print(f"N=4096 FP32: charges vs oracle {err:.2e}")
    assert err < 1e-6



def _golden(name, n_orbitals):
    """The oracle's stored sample for a workload and its recipe."""
    import importlib.util
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    spec = importlib.util.spec_from_file_location("make_sample",
                                                  os.path.join(here, "make_sample.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    scal, atoms, rows = gen.read_sample(name, n_orbitals)
    return gen, scal, atoms, rows


def _large_sample_check(P, name, n_orbitals, scf_tol):
    """Charges and chemical potential of the solve at the stored n, then the
    forces, free energy and one canonical response of the MD state at that
    n, against the oracle's stored sample.  Bounds as at N = 4096: charges
    1e-8 (8x the 1e-9 truncation target, rounded up), mu 1e-9, forces 1e-5,
    relative free energy 1e-8, the response 1e-3 relative (split products)."""
    gen, scal, atoms, rows = _golden(name, n_orbitals)
    s = make_system(name)
    n = gen.charge_vector(s.n_atoms)
    g = P.XLBOMD(s, precision=P.MIXED_BF16X3, scf_tol=scf_tol)
    q, rep = g.solve(n)
    g.set_state(n_hist=np.tile(n, (s.kmax + 1, 1)))
    F, e = g.forces()
    v = gen.unit_direction(s.n_atoms, gen.DIR_SEEDS[0])
    dq = g.response(v[None, :])[0]
    g.close()
    err = dict(q=np.abs(q[atoms] - rows[:, 0]).max(), mu=abs(rep["mu"] - scal["mu"]),
               F=np.abs(F[atoms] - rows[:, 2:5]).max(),
               omega=abs(e["omega"] - scal["omega"]) / abs(scal["omega"]),
               resp=np.abs(dq[atoms] - rows[:, 1]).max() / np.abs(rows[:, 1]).max())
    print(f"N={n_orbitals} MIXED_BF16X3, {rep['foe_levels']} levels vs stored oracle sample:",
          {k: f"{x:.2e}" for k, x in err.items()})
    bounds = dict(q=1e-8, mu=1e-9, F=1e-5, omega=1e-8, resp=1e-3)
    for k, b in bounds.items():
        assert err[k] < b, (k, err[k], b)


def test_small_gap_workload_at_n8192(P):
    """The small-gap workload (2048 atoms x 4 orbitals, N = 8192, T_e = 0.02,
    7 levels) at a fixed n in the headline precision, against the oracle's
    values on a seeded sample of 128 atoms (charges, forces, one response),
    its chemical potential and free energy, all stored by a script that runs
    the oracle alone."""
    _large_sample_check(P, "c3", 8192, 1e-5)


def test_random_packing_workload_at_n16384(P):
    """The largest workload (4096 randomly packed atoms x 4 orbitals,
    N = 16384, irregular neighbour counts) at a fixed n in the headline
    precision, against the oracle's stored sample of 128 atoms, its
    chemical potential and free energy.  A loose initial SCF keeps the test
    short: the solve at n does not depend on it."""
    _large_sample_check(P, "c5", 16384, 1e-3)


def test_energy_conservation_split_path_c1(P):
    """2000 steps of the 64-atom cluster on the split path (level inverses
    in bf16x3 refined against FP64 residuals, split responses) against the
    same run in FP64: the shadow total energy fluctuates by the same amount
    and shows no systematic drift, i.e. the refinement's rounding noise
    (~1e-10 in the charges) does not break the conservation."""
    s = make_system("c1")
    out = {}
    for prec in (P.FP64, P.MIXED_BF16X3):
        g = P.XLBOMD(s, precision=prec, scf_tol=1e-10, energy_every=10)
        E = np.array([g.step(10)["e_total"] for _ in range(200)])
        g.close()
        slope = np.polyfit(np.arange(E.size), E, 1)[0]
        out[prec] = (E, abs(slope) * E.size, E.std())
        print(f"precision {prec}: total energy std {E.std():.2e}, linear drift {out[prec][1]:.2e}")
    E64, d64, s64 = out[P.FP64]
    E3, d3, s3 = out[P.MIXED_BF16X3]
    assert d3 < 2.0 * s3 + 1e-6
    assert s3 < 1.5 * s64 + 1e-6
    # same initial ground state: the conserved level is the same
    assert abs(E3.mean() - E64.mean()) < s64 + 1e-6


def _dt_rung(P, dt, t_end=8.0, nat=24):
    """Mean distance of the GPU trajectory's n to the ground state at the same
    geometry, and of its shadow free energy to the Born-Oppenheimer one,
    sampled every 2 time units (ground states from the oracle's SCF at the
    GPU's positions)."""
    # the exact kernel (J - I)^-1, rebuilt every step (the full-rank
    # Sherman-Morrison sequence equals it)
    s = lattice_system(nat, "c1", seed=21, dt=dt, k0_gamma=0.1, rank=16,
                       krylov_mode=2, kernel_every=1)
    s = s.replace(mass=np.full(nat, 10.0))
    m = R.Model(s)
    g = P.XLBOMD(s, precision=P.FP64, scf_tol=1e-12)
    every = int(round(2.0 / dt))
    res, dom = [], []
    for _ in range(int(round(t_end / dt)) // every):
        g.step(every, report=False)
        pos = g.get_state()["pos"]
        n, _ = g.charges()
        _, e = g.forces()
        el_bo, _ = R.scf(m, pos, 0.1, nat, tol=1e-12, n0=n)
        res.append(np.sqrt(np.mean((n - el_bo.n) ** 2)))
        dom.append(abs(e["omega"] - R.free_energy(m, pos, el_bo)["omega"]))
    g.close()
    return np.mean(res), np.mean(dom)


def test_dt_ladder_scaling(P):
    """Section VI.C on the GPU path: halving dt divides the distance of n to
    the ground state by ~4 (dt^2) and the shadow free energy's distance to
    the Born-Oppenheimer free energy by ~16 (dt^4)."""
    rungs = {dt: _dt_rung(P, dt) for dt in (0.4, 0.2, 0.1)}
    for dt, (r, e) in rungs.items():
        print(f"dt {dt}: rms(n - n_BO) {r:.3e}, |Omega - Omega_BO| {e:.3e}")
    (r1, e1), (r2, e2) = rungs[0.4], rungs[0.2]
    print(f"ratios 0.4/0.2: {r1 / r2:.2f} {e1 / e2:.2f}; 0.2/0.1: "
          f"{r2 / rungs[0.1][0]:.2f} {e2 / rungs[0.1][1]:.2f}")
    assert 3.0 < r1 / r2 < 5.5
    assert 10.0 < e1 / e2 < 25.0
    # closer to the asymptotic 4 and 16 one rung further down
    (r3, e3) = rungs[0.1]
    assert 3.5 < r2 / r3 < 4.5
    assert 13.0 < e2 / e3 < 19.0


def test_report_step_time(P):
    """The report of xlbomd_step carries the device time of its last step,
    and the forces call, which runs no step, reports none."""
    s = make_system("c1")
    g = P.XLBOMD(s, precision=P.FP64, scf_tol=1e-10)
    rep = g.step(3)
    _, e = g.forces()
    g.close()
    print(f"ms_step {rep['ms_step']:.3f}")
    assert 0.0 < rep["ms_step"] < 1e4
    assert e["ms_step"] == 0.0
