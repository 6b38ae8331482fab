"""GPU parity of the non-orthogonal basis (Section VI's SCC-DFTB setting:
overlap S, Mulliken charges from D S, Pulay forces), FP64 path through the
C ABI, against the CPU oracle: solves, responses and K r at fixed n, forces
and free energy of a moving state, one step from a frozen state, a
30-step trajectory, the S = I special case against the GPU's own orthogonal
path, and energy conservation over 400 steps.

Tolerances are the FP64 path's: charges 1e-8, forces 1e-5, relative free
energy 1e-8; responses and K r 1e-6 relative."""
import numpy as np
import pytest

from synth import make_system, lattice_system, with_overlap
from oracle import reference as R

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import paper_1705_10845_amd as P
    P.lib()
    return P


def _rand_n(nat, seed, scale=0.05):
    n = scale * np.random.default_rng(seed).standard_normal(nat)
    return n - n.mean()


CASES = {
    "c1": lambda: with_overlap(make_system("c1")),                         # N = 64
    "lat40": lambda: with_overlap(lattice_system(40, "c2", seed=3)),       # N = 160: ragged tail
    "lat96": lambda: with_overlap(lattice_system(96, "c2", seed=4), 0.4),  # N = 384: 3 tiles
}


@pytest.mark.parametrize("name", list(CASES))
def test_solve_response_kernel_nonorth(gpu, name):
    s = CASES[name]()
    m = R.Model(s)
    g = gpu.XLBOMD(s.replace(rank=3), precision=gpu.FP64, scf_tol=1e-9)
    n = _rand_n(s.n_atoms, 7)
    q, rep = g.solve(n)
    el = R.electronic(m, s.pos, n)
    dq = np.abs(q - el.q).max()
    dmu = abs(rep["mu"] - el.mu)
    V = np.random.default_rng(5).standard_normal((2, s.n_atoms))
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    dres = g.response(V)
    ref = np.stack([R.response(m, el, v) for v in V])
    er = np.abs(dres - ref).max() / np.abs(ref).max()
    kr = g.kernel_apply(3, el.r)
    kref = R.kernel_sm(m, el, rep["k0_gamma"], 3).K @ el.r      # the handle's K0
    ek = np.abs(kr - kref).max() / np.abs(kref).max()
    print(f"{name}: max|dq| {dq:.2e} dmu {dmu:.1e} response rel {er:.2e} K3 r rel {ek:.2e} "
          f"L={rep['foe_levels']}")
    assert dq < 1e-8 and dmu < 1e-7
    assert er < 1e-6 and np.abs(dres.sum(axis=1)).max() < 1e-9
    assert ek < 1e-6
    g.close()


@pytest.mark.parametrize("name", ["c1", "lat40"])
def test_forces_energy_and_one_step_nonorth(gpu, name):
    s = CASES[name]()
    m = R.Model(s)
    st = R.init_state(m, scf_tol=1e-11)
    for _ in range(2):
        st = R.md_step(m, st)
    ref = R.md_step(m, st)
    g = gpu.XLBOMD(s, precision=gpu.FP64, scf_tol=1e-9)
    g.set_state(pos=st.pos, vel=st.vel, n_hist=st.n_hist, kr=st.kr)
    F, e = g.forces()
    n, q = g.charges()
    dq = np.abs(q - st.el.q).max()
    dF = np.abs(F - st.force).max()
    dO = abs(e["omega"] - st.energy["omega"]) / abs(st.energy["omega"])
    g.step(1)
    state = g.get_state()
    n1, q1 = g.charges()
    F1, e1 = g.forces()
    dn1 = np.abs(state["n_hist"][0] - ref.n_hist[0]).max()
    dq1 = np.abs(q1 - ref.el.q).max()
    dF1 = np.abs(F1 - ref.force).max()
    dO1 = abs(e1["omega"] - ref.energy["omega"]) / abs(ref.energy["omega"])
    print(f"{name}: frozen dq {dq:.2e} dF {dF:.2e} rel dOmega {dO:.2e}; one step dn {dn1:.2e} "
          f"dq {dq1:.2e} dF {dF1:.2e} rel dOmega {dO1:.2e}")
    assert dq < 1e-8 and dF < 1e-5 and dO < 1e-8
    assert dn1 < 1e-10 and dq1 < 1e-8 and dF1 < 1e-5 and dO1 < 1e-8
    g.close()


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_trajectory_nonorth(gpu, mode):
    """30 steps of the 64-atom cluster in a non-orthogonal basis, with each
    kernel mode (sequential, block, full), against the oracle's steps."""
    s = CASES["c1"]().replace(rank=2, krylov_mode=mode, kernel_every=1 if mode == 0 else 3)
    m = R.Model(s)
    st = R.init_state(m, scf_tol=1e-11)
    g = gpu.XLBOMD(s, precision=gpu.FP64, scf_tol=1e-11)
    worst = dict(dn=0.0, dq=0.0, dF=0.0)
    for i in range(30):
        st = R.md_step(m, st, want_energy=False)
        g.step(1, report=False)
        if (i + 1) % 10 == 0:
            n, q = g.charges()
            F, _ = g.forces(energy=False)
            worst["dn"] = max(worst["dn"], np.abs(n - st.el.n).max())
            worst["dq"] = max(worst["dq"], np.abs(q - st.el.q).max())
            worst["dF"] = max(worst["dF"], np.abs(F - st.force).max())
    F, e = g.forces()
    eo = R.energy_report(m, st)
    dO = abs(e["omega"] - eo["omega"]) / abs(eo["omega"])
    g.close()
    print(f"mode {mode}: 30 steps vs oracle", {k: f"{v:.1e}" for k, v in worst.items()},
          f"rel dOmega {dO:.1e}")
    assert worst["dn"] < 1e-8 and worst["dq"] < 1e-8 and worst["dF"] < 1e-5 and dO < 1e-8


def test_unit_overlap_equals_orthogonal_path(gpu):
    """Overlaps between atoms that underflow to zero: the non-orthogonal
    path (S = I, X = I after the Newton-Schulz iteration) gives the
    orthogonal path's charges, forces, energy, responses and steps."""
    s0 = lattice_system(40, "c2", seed=6)
    s1 = s0.replace(overlap_block=np.ones((4, 4)), overlap_decay=1e-3)
    out = []
    for s in (s0, s1):
        g = gpu.XLBOMD(s, precision=gpu.FP64, scf_tol=1e-10)
        g.step(3, report=False)
        n, q = g.charges()
        F, e = g.forces()
        V = np.random.default_rng(2).standard_normal((1, s.n_atoms))
        out.append(dict(q=q, F=F, om=e["omega"], resp=g.response(V)[0], n=n))
        g.close()
    d = {k: float(np.max(np.abs(np.asarray(out[0][k]) - np.asarray(out[1][k])))) for k in out[0]}
    print("S = I vs orthogonal path:", {k: f"{v:.1e}" for k, v in d.items()})
    assert d["q"] < 1e-10 and d["n"] < 1e-10 and d["F"] < 1e-9
    assert d["om"] < 1e-9 * abs(out[0]["om"])
    assert d["resp"] < 1e-9 * np.abs(out[0]["resp"]).max()


def test_energy_conservation_nonorth(gpu):
    """400 steps of the 64-atom cluster with overlap: kinetic energy is
    exchanged and the total shows no systematic drift."""
    s = CASES["c1"]()
    g = gpu.XLBOMD(s, precision=gpu.FP64, scf_tol=1e-10, energy_every=1)
    et, ek = [], []
    for _ in range(400):
        r = g.step(1)
        et.append(r["e_total"])
        ek.append(r["e_kin"])
    g.close()
    et, ek = np.array(et), np.array(ek)
    slope = np.polyfit(np.arange(len(et)), et, 1)[0]
    print(f"400 steps: E_kin range {ek.max() - ek.min():.3e}, E_tot std {et.std():.2e}, "
          f"drift over the run {slope * len(et):.2e}")
    assert ek.max() - ek.min() > 50 * et.std()
    assert abs(slope) * len(et) < 2.0 * et.std() + 1e-8


def test_nonorth_refuses_planned_steps_and_other_precisions(gpu):
    """Planned steps and the reduced precisions are not built for a
    non-orthogonal basis: both are refused with XLBOMD_E_INVALID."""
    s = CASES["c1"]()
    g = gpu.XLBOMD(s, precision=gpu.FP64, scf_tol=1e-9)
    with pytest.raises(gpu.XlbomdError) as e:
        g.set_step_mode(2)
    assert e.value.code == -1 and "orthogonal" in str(e.value)
    g.step(2, report=False)              # still stepping with host decisions
    g.close()
    with pytest.raises(gpu.XlbomdError) as e:
        gpu.XLBOMD(s, precision=gpu.MIXED_BF16X3)
    assert e.value.code == -1


def test_nonorth_checkpoint_resumes_bit_for_bit(gpu):
    """save_state after 3 steps, 4 more steps; a fresh handle that loads the
    checkpoint (and recomputes S^-1/2 at the restored positions) takes the
    same 4 steps to the same state, bit for bit."""
    s = CASES["lat40"]().replace(rank=2, kernel_every=2)
    g = gpu.XLBOMD(s, precision=gpu.FP64, scf_tol=1e-10, energy_every=2)
    g.step(3, report=False)
    blob = g.save_state()
    ra = g.step(4)
    sa = g.get_state()
    qa = g.charges()[1]
    g.close()
    h = gpu.XLBOMD(s, precision=gpu.FP64, scf_tol=1e-10, energy_every=2)
    h.step(1, report=False)
    h.load_state(blob)
    rb = h.step(4)
    sb = h.get_state()
    qb = h.charges()[1]
    h.close()
    d = max(float(np.abs(np.asarray(sa[k]) - np.asarray(sb[k])).max()) for k in sa)
    print(f"resumed vs original: max state diff {d:.1e}, charges {np.abs(qa - qb).max():.1e}")
    assert d == 0.0 and np.array_equal(qa, qb)
    assert ra["e_total"] == rb["e_total"]


def test_nonorth_dimer_closed_form_on_the_gpu(gpu):
    """The two-atom closed form of the oracle's pins, through the GPU path:
    eigenvalues (e +- t)/(1 +- s), mu halfway, Mulliken charges 0, band
    energy and the force along the bond with its Pulay part."""
    import math
    r, te = 1.7, 0.2
    pos = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
    s = make_system("c1").replace(
        n_atoms=2, pos=pos, vel=np.zeros((2, 3)), mass=np.ones(2),
        onsite=np.array([-0.2]), onsite_jitter=np.zeros(2),
        hop_block=np.array([[-1.0]]), hop_decay=1.0, hop_cutoff=4.0,
        taper_width=0.5, hubbard_u=np.array([1.0, 1.0]), n_electrons=2.0,
        te=te, rep_a=0.0, rank=1, overlap_block=np.array([[0.3]]), overlap_decay=0.8)
    e, t, so = -0.2, -math.exp(-r), 0.3 * math.exp(-r / 0.8)
    ep, em = (e + t) / (1 + so), (e - t) / (1 - so)
    mu = 0.5 * (ep + em)
    fp = 1.0 / (1.0 + math.exp((ep - mu) / te))
    fm = 1.0 / (1.0 + math.exp((em - mu) / te))
    dt, ds = -t, -so / 0.8
    dep = (dt * (1 + so) - (e + t) * ds) / (1 + so) ** 2
    dem = (-dt * (1 - so) + (e - t) * ds) / (1 - so) ** 2
    f_bond = -2.0 * (fp * dep + fm * dem)
    g = gpu.XLBOMD(s, precision=gpu.FP64, scf_tol=1e-12)
    g.set_state(n_hist=np.zeros((s.kmax + 1, 2)))
    F, en = g.forces()
    n, q = g.charges()
    g.close()
    print(f"dimer: q {q}, mu {en['mu']:.12f} ({mu:.12f}), F_x {F[:, 0]} ({-f_bond:.12f}), "
          f"e_band {en['e_band']:.12f} ({2 * (fp * ep + fm * em):.12f})")
    assert np.abs(q).max() < 1e-10
    assert abs(en["mu"] - mu) < 1e-9
    assert abs(en["e_band"] - 2 * (fp * ep + fm * em)) < 1e-10
    assert abs(F[0, 0] + f_bond) < 1e-10 and abs(F[1, 0] - f_bond) < 1e-10
