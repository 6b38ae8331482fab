"""Pins of the CPU oracle against facts fixed by the paper and the mathematics.

Each test checks the oracle against something other than itself: a closed
form worked by hand, a library routine (numpy eigh) for a step the oracle
implements from scratch, a finite difference, an identity the paper states,
or a scaling law the paper reports.  A plausible slip anywhere in the oracle
(a dropped term, a wrong sign, a transposed operand) fails one of them.
"""
import math

import numpy as np
import pytest

from synth import make_system, lattice_system
from oracle import reference as R


def _dimer(delta=0.3, t_hop=-0.7, te=0.2, n=(0.0, 0.0), u=1.0):
    """Two atoms, one orbital each, two electrons."""
    s = make_system("c1")
    r = 1.5
    pos = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
    # hopping B exp(-r/lambda) s(r) with s = 1 at r = 1.5 < rc - w
    B = t_hop / math.exp(-r / 1.0)
    s = s.replace(n_atoms=2, pos=pos, vel=np.zeros((2, 3)), mass=np.ones(2),
                  onsite=np.array([0.0]),
                  onsite_jitter=np.array([delta, -delta]),
                  hop_block=np.array([[B]]), hop_decay=1.0, hop_cutoff=4.0,
                  taper_width=0.5, hubbard_u=np.array([u, u]),
                  n_electrons=2.0, te=te, rep_a=0.0)
    return R.Model(s), pos, np.array(n, dtype=float)


def _dimer_closed_form(delta, t, beta):
    """Eigen-closed form of the 2x2 problem H = [[e+d, t], [t, e-d]], N_e = 2.

    mu sits at the mean onsite energy by particle-hole symmetry; with
    w = sqrt(d^2 + t^2) and T = tanh(beta w / 2):
      D11 = 1 - (d/w) T,  D12 = -(t/w) T,  q1 = -(d/w) T,
      S = 4 s(beta w), s the per-orbital Fermi entropy,
      Tr[H D] = 2 e - 2 w T.
    """
    w = math.hypot(delta, t)
    T = math.tanh(0.5 * beta * w)
    x = beta * w
    s = math.log1p(math.exp(-x)) + x / (1.0 + math.exp(x))
    return dict(D11=1 - delta / w * T, D12=-t / w * T, q1=-delta / w * T,
                S=4 * s, eband=-2 * w * T, w=w, T=T)


# ---------------------------------------------------------------------------
# Jacobi eigensolver
# ---------------------------------------------------------------------------
def test_jacobi_2x2_closed_form():
    a, b, c = 0.3, -0.8, -0.5
    ev, Vt = R.jacobi(np.array([[a, b], [b, c]]))
    m, w = 0.5 * (a + c), math.hypot(0.5 * (a - c), b)
    assert np.allclose(sorted(ev), [m - w, m + w], atol=1e-15, rtol=0)


@pytest.mark.parametrize("n", [1, 7, 40, 96])
def test_jacobi_vs_library(n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n))
    A = 0.5 * (A + A.T)
    ev, Vt = R.jacobi(A)
    # residual, orthogonality, and the spectrum against LAPACK (tests only)
    assert np.abs(Vt.T @ np.diag(ev) @ Vt - A).max() < 1e-12
    assert np.abs(Vt @ Vt.T - np.eye(n)).max() < 1e-12
    assert np.allclose(np.sort(ev), np.linalg.eigvalsh(A), atol=1e-12)


def test_jacobi_degenerate():
    # a matrix with a triply degenerate eigenvalue
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    lam = np.array([-1.0, 0.2, 0.2, 0.2, 0.7, 1.5])
    A = Q @ np.diag(lam) @ Q.T
    ev, Vt = R.jacobi(A)
    assert np.allclose(np.sort(ev), lam, atol=1e-13)
    assert np.abs(Vt.T @ np.diag(ev) @ Vt - A).max() < 1e-13


# ---------------------------------------------------------------------------
# Fermi-Dirac occupations, mu, density matrix, entropy (Eqs. 36-38)
# ---------------------------------------------------------------------------
def test_dimer_closed_form():
    d, t, te = 0.3, -0.7, 0.2
    m, pos, n = _dimer(d, t, te)
    el = R.electronic(m, pos, n)
    cf = _dimer_closed_form(d, t, 1.0 / te)
    assert abs(el.mu - 0.0) < 1e-12
    assert abs(el.D[0, 0] - cf["D11"]) < 1e-13
    assert abs(el.D[0, 1] - cf["D12"]) < 1e-13
    assert abs(el.q[0] - cf["q1"]) < 1e-13 and abs(el.q.sum()) < 1e-13
    assert abs(R.entropy(m, el) - cf["S"]) < 1e-13
    assert abs(np.sum(el.H0 * el.D) - cf["eband"]) < 1e-13



def _fermi_entropy(f):
    """Per-orbital entropy -[f ln f + (1-f) ln(1-f)] of an occupation f."""
    return -(f * math.log(f) + (1.0 - f) * math.log(1.0 - f))


@pytest.mark.parametrize("ne", [0.3, 1.0, 1.7])
def test_single_orbital_atom_closed_form(ne):
    """One atom with one orbital: H is the scalar h = onsite + jitter, D is
    the electron count itself, 2 f(beta (h - mu)) = ne gives
    mu = h - T ln(2/ne - 1), the net charge and the force vanish, the band
    energy is h ne and S = 2 s(ne/2) (2 ln 2 at half filling)."""
    s = lattice_system(1, "c1", seed=8, rank=1).replace(n_electrons=ne)
    m = R.Model(s)
    el = R.electronic(m, s.pos, np.zeros(1))
    h = float(s.onsite[0] + s.onsite_jitter[0])
    T = s.te
    assert abs(el.mu - (h - T * math.log(2.0 / ne - 1.0))) < 1e-12
    assert abs(el.D[0, 0] - ne) < 1e-13 and abs(el.q[0]) < 1e-13
    assert abs(np.sum(el.H0 * el.D) - h * ne) < 1e-13
    assert abs(R.entropy(m, el) - 2.0 * _fermi_entropy(ne / 2.0)) < 1e-12
    st = R.init_state(m, scf_tol=1e-11)
    assert np.abs(st.force).max() == 0.0
    if ne == 1.0:
        assert abs(st.energy["te_s"] - 2.0 * T * math.log(2.0)) < 1e-13


def test_four_orbital_atom_against_root_finder():
    """One atom with four orbitals and no hopping inside the atom: H is
    diagonal, so D = diag(2 f(beta (e_a - mu))) with mu the root of the
    electron count, found here by scipy's brentq on the scalar equation."""
    from scipy.optimize import brentq
    s = lattice_system(1, "c2", seed=8, rank=1)
    m = R.Model(s)
    el = R.electronic(m, s.pos, np.zeros(1))
    e = s.onsite + s.onsite_jitter
    beta = 1.0 / s.te
    occ = lambda mu: 2.0 / (1.0 + np.exp(beta * (e - mu)))
    mu = brentq(lambda x: occ(x).sum() - s.n_electrons, e.min() - 5, e.max() + 5, xtol=1e-15)
    f = occ(mu) / 2.0
    assert abs(el.mu - mu) < 1e-11
    assert np.abs(el.D - np.diag(2.0 * f)).max() < 1e-12
    assert abs(R.entropy(m, el) - 2.0 * sum(_fermi_entropy(x) for x in f)) < 1e-11


def test_trace_equals_electron_count():
    s = lattice_system(40, "c2", seed=11)
    m = R.Model(s)
    el = R.electronic(m, s.pos, np.zeros(m.nat))
    assert abs(np.trace(el.D) - s.n_electrons) < 1e-10
    assert abs(el.q.sum()) < 1e-10
    # D is symmetric with occupations in [0, 2]
    ev = np.linalg.eigvalsh(el.D)
    assert ev.min() > -1e-12 and ev.max() < 2 + 1e-12


def test_low_temperature_idempotent_and_aufbau():
    # gapped dimer chain at Te -> 0: D/2 becomes a projector on the lowest
    # N_e/2 eigenvectors (aufbau)
    s = lattice_system(8, "c2", seed=2)
    s = s.replace(te=1e-4, onsite_jitter=np.zeros(32))
    m = R.Model(s)
    el = R.electronic(m, s.pos, np.zeros(m.nat))
    evs = np.sort(el.evals)
    nocc = int(s.n_electrons // 2)
    gap = evs[nocc] - evs[nocc - 1]
    assert gap > 40 * s.te
    P = 0.5 * el.D
    bound = 4 * math.exp(-0.5 * gap / s.te) + 1e-12
    assert np.abs(P @ P - P).max() < bound
    w, U = np.linalg.eigh(el.H)
    Pa = U[:, :nocc] @ U[:, :nocc].T
    assert np.abs(P - Pa).max() < bound


def test_entropy_matches_occupation_formula():
    s = lattice_system(30, "c2", seed=4)
    m = R.Model(s)
    el = R.electronic(m, s.pos, 0.01 * np.arange(30))
    f = np.clip(el.f, 1e-300, 1 - 1e-16)
    direct = -2 * np.sum(f * np.log(f) + (1 - f) * np.log1p(-f))
    assert abs(R.entropy(m, el) - direct) < 1e-10


# ---------------------------------------------------------------------------
# Response (Section V.B)
# ---------------------------------------------------------------------------
def test_dimer_response_closed_form():
    d, t, te, u = 0.3, -0.7, 0.2, 1.3
    m, pos, n = _dimer(d, t, te, u=u)
    el = R.electronic(m, pos, n)
    G = m.gamma(pos)
    v = np.array([0.8, -0.25])
    h = G @ v
    dd = 0.5 * (h[0] - h[1])          # change of the onsite half-splitting
    cf = _dimer_closed_form(d, t, 1.0 / te)
    w, T, beta = cf["w"], cf["T"], 1.0 / te
    Tp = 0.5 * beta * (1 - T * T)
    dq1 = -(T / w + d * d * (Tp * w - T) / w ** 3) * dd
    q = R.response(m, el, v)
    assert abs(q[0] - dq1) < 1e-12 and abs(q[1] + dq1) < 1e-12


def test_response_matches_finite_difference():
    s = lattice_system(24, "c2", seed=8)
    m = R.Model(s)
    rng = np.random.default_rng(0)
    n = 0.05 * rng.standard_normal(m.nat)
    n -= n.mean()
    el = R.electronic(m, s.pos, n)
    for _ in range(3):
        v = rng.standard_normal(m.nat)
        v /= np.linalg.norm(v)
        a = R.response(m, el, v)
        b = R.response_fd(m, s.pos, el, v, h=1e-4)
        assert np.abs(a - b).max() < 1e-7 * max(1.0, np.abs(a).max())
        assert abs(a.sum()) < 1e-11          # canonical: charge conserved


def test_response_reciprocity():
    # J = chi Gamma with chi symmetric  =>  Gamma J symmetric
    s = lattice_system(20, "c2", seed=9)
    m = R.Model(s)
    el = R.electronic(m, s.pos, np.zeros(m.nat))
    J = R.jacobian(m, el)
    GJ = el.G @ J
    assert np.abs(GJ - GJ.T).max() < 1e-11


# ---------------------------------------------------------------------------
# Kernel (Eqs. 48-51)
# ---------------------------------------------------------------------------
def _small_case(nat=16, seed=5):
    s = lattice_system(nat, "c2", seed=seed)
    m = R.Model(s)
    rng = np.random.default_rng(seed)
    n = 0.03 * rng.standard_normal(nat)
    return m, s, R.electronic(m, s.pos, n)


def test_full_rank_kernel_is_inverse_jacobian():
    m, s, el = _small_case()
    k = R.kernel_sm(m, el, 0.4, m.nat)
    J = R.jacobian(m, el)
    assert k.rank == m.nat
    assert np.abs(k.K - np.linalg.inv(J - np.eye(m.nat))).max() < 1e-10


def test_kernel_full_matches_full_rank_sequence():
    # the dense inverse of krylov_mode 2 against the Sherman-Morrison
    # sequence of Eq. 50 run over all N_at directions (a different route)
    m, s, el = _small_case()
    Kf = R.kernel_full(m, el)
    Ksm = R.kernel_sm(m, el, 0.25, m.nat).K
    J = R.jacobian(m, el)
    assert np.abs(Kf - Ksm).max() < 1e-9 * np.abs(Kf).max()
    assert np.abs(Kf @ (J - np.eye(m.nat)) - np.eye(m.nat)).max() < 1e-10


def test_kernel_woodbury_and_reproduction():
    # K_m from the Sherman-Morrison sequence equals the closed Woodbury form
    # a^-1 (I - W M V^T) + V M V^T, M = (V^T W)^-1, a = -1/gamma, and it maps
    # each w_j = J v_j - v_j back onto v_j.
    m, s, el = _small_case()
    gamma = 0.3
    k = R.kernel_sm(m, el, gamma, 4)
    V = k.V
    J = R.jacobian(m, el)
    W = (J - np.eye(m.nat)) @ V
    M = np.linalg.inv(V.T @ W)
    a = -1.0 / gamma
    Kw = (np.eye(m.nat) - W @ M @ V.T) / a + V @ M @ V.T
    assert np.abs(k.K - Kw).max() < 1e-12
    assert np.abs(k.K @ W - V).max() < 1e-12
    assert np.abs(V.T @ V - np.eye(4)).max() < 1e-13


def test_kernel_depends_on_span_only():
    # directions orth(w_j) span the same Krylov space as orth(K_j r): same K r
    m, s, el = _small_case(seed=6)
    gamma, rank = 0.3, 3
    k = R.kernel_sm(m, el, gamma, rank)
    J = R.jacobian(m, el)
    r = el.r
    V = np.zeros((m.nat, 0))
    v = r / np.linalg.norm(r)
    for j in range(rank):
        V = np.column_stack([V, v])
        w = (J - np.eye(m.nat)) @ v
        y = w - V @ (V.T @ w)
        y -= V @ (V.T @ y)
        v = y / np.linalg.norm(y)
    W = (J - np.eye(m.nat)) @ V
    M = np.linalg.inv(V.T @ W)
    Kr = -gamma * (r - W @ (M @ (V.T @ r))) + V @ (M @ (V.T @ r))
    assert np.abs(k.K @ r - Kr).max() < 1e-11


def test_kernel_rank0_is_scaled_delta():
    m, s, el = _small_case()
    k = R.kernel_sm(m, el, 0.25, 0)
    assert np.allclose(k.K, -0.25 * np.eye(m.nat))


# ---------------------------------------------------------------------------
# Integrator (Eqs. 22-23, Table I)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kmax", [5, 6, 7])
def test_table_I_dissipation_is_consistent(kmax):
    kappa, alpha, c = R.TABLE_I[kmax]
    assert len(c) == kmax + 1
    assert sum(c) == 0                      # a constant n is not damped
    # linear test: dt^2 nddot = -kappa (n - n*) with an exact kernel.
    # n_{+} = (2 - kappa) n - n_{-} + alpha sum_k c_k n_{-k}
    p = np.zeros(kmax + 2)
    p[0] = 1.0
    p[1] = -(2.0 - kappa) - alpha * c[0]
    p[2] = 1.0 - alpha * c[1]
    for k in range(2, kmax + 1):
        p[k + 1] = -alpha * c[k]
    roots = np.roots(p)
    assert np.abs(roots).max() < 0.98       # damped
    # without dissipation Verlet is marginally stable for kappa < 2
    p0 = [1.0, -(2.0 - kappa), 1.0]
    assert abs(np.abs(np.roots(p0)).max() - 1.0) < 1e-12


def test_forces_are_minus_gradient_of_free_energy():
    s = make_system("c1")
    m = R.Model(s)
    rng = np.random.default_rng(1)
    n = 0.05 * rng.standard_normal(m.nat)
    el = R.electronic(m, s.pos, n)
    F = R.forces(m, s.pos, el)
    h = 1e-4
    for I in (0, 21, 63):
        for c in range(3):
            p = s.pos.copy()
            p[I, c] += h
            ep = R.free_energy(m, p, R.electronic(m, p, n))["omega"]
            p[I, c] -= 2 * h
            em = R.free_energy(m, p, R.electronic(m, p, n))["omega"]
            assert abs(-(ep - em) / (2 * h) - F[I, c]) < 1e-8
    assert np.abs(F.sum(axis=0)).max() < 1e-12   # translation invariance


def test_forces_orbital_block_model():
    # same check on the s+3p model (non-trivial hopping block)
    s = lattice_system(12, "c2", seed=3)
    m = R.Model(s)
    n = 0.02 * np.random.default_rng(2).standard_normal(m.nat)
    el = R.electronic(m, s.pos, n)
    F = R.forces(m, s.pos, el)
    h = 1e-4
    for I in (0, 7):
        for c in range(3):
            p = s.pos.copy()
            p[I, c] += h
            ep = R.free_energy(m, p, R.electronic(m, p, n))["omega"]
            p[I, c] -= 2 * h
            em = R.free_energy(m, p, R.electronic(m, p, n))["omega"]
            assert abs(-(ep - em) / (2 * h) - F[I, c]) < 1e-8


def test_scf_reaches_ground_state():
    s = make_system("c1")
    m = R.Model(s)
    el, hist = R.scf(m, s.pos, s.k0_gamma, s.rank, tol=1e-10)
    assert hist[-1] <= 1e-10
    # with the exact kernel the kernel SCF is Newton: quadratic convergence
    el2, hist2 = R.scf(m, s.pos, s.k0_gamma, m.nat, tol=1e-12)
    assert len(hist2) <= 6
    assert np.abs(el2.n - el.n).max() < 1e-9


# ---------------------------------------------------------------------------
# Dynamics: the paper's scaling claims (Section VI.C)
# ---------------------------------------------------------------------------
def _run(dt, t_end, nat=24):
    s = lattice_system(nat, "c1", seed=21, dt=dt, k0_gamma=0.1, rank=nat)
    s = s.replace(mass=np.full(nat, 10.0))
    m = R.Model(s)
    st = R.init_state(m, scf_tol=1e-12)
    steps = int(round(t_end / dt))
    res, dom = [], []
    for i in range(steps):
        st = R.md_step(m, st)
        if (i + 1) % int(round(2.0 / dt)) == 0:
            # distance to the converged ground state at this geometry
            el_bo, _ = R.scf(m, st.pos, 0.1, nat, tol=1e-12, n0=st.el.n)
            res.append(np.sqrt(np.mean((st.el.n - el_bo.n) ** 2)))
            om_bo = R.free_energy(m, st.pos, el_bo)["omega"]
            dom.append(abs(st.energy["omega"] - om_bo))
    return np.mean(res), np.mean(dom)


def test_dt_scaling_of_density_and_shadow_energy():
    # n - rho_min ~ dt^2 and Omega[n] - Omega_BO ~ dt^4 (Section VI.C)
    r1, e1 = _run(0.4, 8.0)
    r2, e2 = _run(0.2, 8.0)
    assert 3.0 < r1 / r2 < 5.5
    assert 10.0 < e1 / e2 < 25.0


def test_no_systematic_energy_drift():
    s = make_system("c1")
    m = R.Model(s)
    st, E = R.run(m, 400)
    et = np.array([e["e_total"] for e in E])
    t = np.arange(len(et))
    slope = np.polyfit(t, et, 1)[0]
    assert abs(slope) * len(et) < 2.0 * et.std() + 1e-6
    assert et.std() < 1e-2


def test_kernel_of_a_zero_residual_is_K0():
    # the direction of a numerically zero residual is noise: rank-0 kernel
    m, s, el = _small_case()
    el.q = el.n + 1e-12 * np.random.default_rng(0).standard_normal(m.nat)
    k = R.kernel_sm(m, el, 0.2, 3)
    assert k.rank == 0
    assert np.allclose(k.K, -0.2 * np.eye(m.nat))


def test_auto_gamma_bounds_the_stiffest_mode():
    # the power-iteration estimate approaches the largest |eigenvalue| of J
    # from below, and the chosen gamma keeps gamma (1 - lambda_J) near or
    # below 1.5 for every mode (exact spectrum from a library eigensolver)
    s = lattice_system(24, "c4", seed=31)
    m = R.Model(s)
    el = R.electronic(m, s.pos, np.zeros(m.nat))
    g, lam = R.auto_gamma(m, el)
    J = R.jacobian(m, el)
    lam_exact = np.abs(np.linalg.eigvals(J)).max()
    assert 0.94 * lam_exact <= lam <= lam_exact * (1 + 1e-12)
    assert g * (1.0 + lam_exact) <= 1.6
    # two significant digits, rounded down: within 10% below 1.5 / (1 + lam)
    assert g >= 0.9 * 1.5 / (1.0 + lam) * (1.0 - 1e-12)
    assert float(f"{g:.2g}") == g


def test_kernel_after_converged_init_is_built_at_the_first_step():
    # reading of Section V.E (kernel reused between rebuilds): right after a
    # converged SCF the residual is rounding noise, the build for the
    # dynamics stops at rank 0 (K0 alone), and the first MD step builds
    # again whatever the refresh period; later steps reuse that kernel
    s = make_system("c1", kernel_every=50, rank=2)
    m = R.Model(s)
    st = R.init_state(m, scf_tol=1e-11)
    assert st.pending and st.V.shape[1] == 0
    assert np.allclose(st.K, -s.k0_gamma * np.eye(m.nat))
    st1 = R.md_step(m, st, want_energy=False)
    assert not st1.pending and st1.V.shape[1] == 2
    assert not np.allclose(st1.K, -s.k0_gamma * np.eye(m.nat))
    st2 = R.md_step(m, st1, want_energy=False)
    assert st2.K is st1.K and not st2.pending


def test_kernel_from_images_and_on_the_fly_updates():
    # the Sherman-Morrison sequence over stored images reproduces a build's
    # kernel, and the kernel after on-the-fly updates (Section V.E) maps
    # every kept image back to its direction: K w_j = v_j, i.e. it is the
    # inverse of J_m - I on the kept directions
    s = lattice_system(20, "c2", seed=5, rank=2, kernel_every=50, kernel_otf=2,
                       k0_gamma=0.05)
    m = R.Model(s)
    st = R.init_state(m, scf_tol=1e-11)
    st = R.md_step(m, st, want_energy=False)          # rebuild (pending)
    kres_K = R.kernel_from_images(0.05, st.V, st.W)
    assert np.abs(kres_K - st.K).max() < 1e-12 * np.abs(st.K).max()
    assert st.n_rb == 2 and st.V.shape[1] == 2
    ranks = []
    for _ in range(4):
        st = R.md_step(m, st, want_energy=False)
        ranks.append(st.V.shape[1])
        assert np.abs(st.V.T @ st.V - np.eye(st.V.shape[1])).max() < 1e-12
        assert np.abs(st.K @ st.W - st.V).max() < 1e-10
    assert ranks == [3, 4, 4, 4]                      # window of 2, oldest leaves
