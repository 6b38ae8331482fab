"""CPU oracle for finite-temperature XL-BOMD, FP64.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the HIP library (which shares no code
with it).  Heavy loops (model, Jacobi, occupations, response, forces) are in
xlbomd_oracle.c; this module strings them together in the order the paper
states the method.

Paper map (A. M. N. Niklasson, "Next generation extended Lagrangian first
principles molecular dynamics"):
  electronic solve    Section IV.A-B: H[n] = H0 + diag(Gamma n), Fermi-Dirac
                      occupations with mu from sum f = N_occ (Eq. 36),
                      D = 2 f(H), net Mulliken charges q (Section VI).
  free energy         Eqs. 35, 37, 38 specialised to SCC tight binding:
                      Omega = Tr[H0 D] + 1/2 (2q - n)^T Gamma n + E_rep - Te S.
  forces              Eq. 40, the partial derivative at fixed n.
  response            Section V.B: canonical first-order response of q to a
                      potential perturbation along v (directional derivative
                      of q[n + lambda v]).
  kernel              Eqs. 48-51: K0 = (J0 - I)^-1, J0 = c I, followed by the
                      Sherman-Morrison sequence of rank-1 updates over
                      orthonormal directions, the first along K0 r.
  integration         Eq. 22 (velocity Verlet for the nuclei; the position
                      update is read with the velocity, not the
                      acceleration) and Eq. 23 with the K_max = 5, 6, 7
                      rows of Table I.
  initial state       Eq. 20 with the ground state from the kernel SCF of
                      Eq. 52.
  non-orthogonal      Section VI (the SCC-DFTB model: non-orthogonal atomic
  basis               orbitals, Mulliken charges, Pulay forces), on the
                      synthetic model: overlap S, H[n] = H0 + (S V + V S)/2
                      with V the orbital potentials, the generalised
                      eigenproblem through the Loewdin factor X = S^-1/2
                      (H' = X H X), D = X D' X, q_I = sum_a (D S)[Ia,Ia] -
                      Z_I, and the energy-weighted density matrix in the
                      forces.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import build as _build

_c = ctypes
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        L.orc_h0.argtypes = [_c.c_int, _c.c_int, _dp, _dp, _dp, _dp,
                             _c.c_double, _c.c_double, _c.c_double, _dp]
        L.orc_gamma.argtypes = [_c.c_int, _dp, _dp, _c.c_double, _dp]
        L.orc_erep.argtypes = [_c.c_int, _dp, _c.c_double, _c.c_double,
                               _c.c_double, _c.c_double, _dp]
        L.orc_erep.restype = _c.c_double
        L.orc_forces.argtypes = [_c.c_int, _c.c_int, _dp, _dp, _c.c_double,
                                 _c.c_double, _c.c_double, _c.c_double,
                                 _dp, _dp, _dp, _dp]
        L.orc_jacobi.argtypes = [_c.c_int, _dp, _dp, _dp, _c.c_double,
                                 _c.c_int]
        L.orc_fermi_mu.argtypes = [_c.c_int, _dp, _c.c_double, _c.c_double,
                                   _dp]
        L.orc_fermi_mu.restype = _c.c_double
        L.orc_entropy.argtypes = [_c.c_int, _dp, _c.c_double, _c.c_double]
        L.orc_entropy.restype = _c.c_double
        L.orc_entropy_x.argtypes = [_c.c_double]
        L.orc_entropy_x.restype = _c.c_double
        L.orc_fermi.argtypes = [_c.c_double]
        L.orc_fermi.restype = _c.c_double
        L.orc_fermi_divdiff.argtypes = [_c.c_double, _c.c_double, _c.c_double]
        L.orc_fermi_divdiff.restype = _c.c_double
        L.orc_fermi_divdiff_matrix.argtypes = [_c.c_int, _dp, _c.c_double, _dp]
        L.orc_density.argtypes = [_c.c_int, _dp, _dp, _dp]
        L.orc_response_diag.argtypes = [_c.c_int, _dp, _dp, _c.c_double,
                                        _c.c_double, _dp, _dp]
        L.orc_response_diag.restype = _c.c_double
        L.orc_taper.argtypes = [_c.c_double, _c.c_double, _c.c_double,
                                _c.POINTER(_c.c_double),
                                _c.POINTER(_c.c_double)]
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# Table I: dissipation coefficients of Eq. 23 (kappa, alpha, c_0..c_K).
# ---------------------------------------------------------------------------
TABLE_I = {
    5: (1.82, 0.018, (-6, 14, -8, -3, 4, -1)),
    6: (1.84, 0.0055, (-14, 36, -27, -2, 12, -6, 1)),
    7: (1.86, 0.0016, (-36, 99, -88, 11, 32, -25, 8, -1)),
}


# ---------------------------------------------------------------------------
# Model
# ---------------------------------------------------------------------------
class Model:
    """SCC tight-binding model built from raw synthetic parameters."""

    def __init__(self, s):
        self.s = s
        self.nat = int(s.n_atoms)
        self.no = int(s.n_orb)
        self.N = self.nat * self.no
        self.beta = 1.0 / s.te
        self.zcore = np.full(self.nat, s.n_electrons / self.nat)
        self.mass = _f64(s.mass)

    def h0(self, pos):
        s = self.s
        H = np.zeros((self.N, self.N))
        rc = lib().orc_h0(self.nat, self.no, _f64(pos), _f64(s.onsite),
                          _f64(s.onsite_jitter), _f64(s.hop_block),
                          s.hop_decay, s.hop_cutoff, s.taper_width, H)
        assert rc == 0
        return H

    def gamma(self, pos):
        G = np.zeros((self.nat, self.nat))
        assert lib().orc_gamma(self.nat, _f64(pos), _f64(self.s.hubbard_u),
                               self.s.gamma_soft, G) == 0
        return G

    def erep(self, pos, want_force=False):
        F = np.zeros(3 * self.nat)
        e = lib().orc_erep(self.nat, _f64(pos), self.s.rep_a,
                           self.s.rep_decay, self.s.hop_cutoff,
                           self.s.taper_width, F)
        return (e, F.reshape(self.nat, 3)) if want_force else e

    def orbital_potential(self, G, n):
        """diag of the charge-dependent Hamiltonian part, per orbital."""
        return np.repeat(G @ n, self.no)

    @property
    def nonorth(self):
        b = getattr(self.s, "overlap_block", None)
        return b is not None and bool(np.any(np.asarray(b) != 0.0))

    def overlap(self, pos):
        """Overlap matrix S: the identity on each atom's own block and
        S[Ia,Jb] = Bs_ab exp(-r/decay_s) s(r) between atoms (the hopping's
        form with unit onsite entries, its own block and decay, the same
        cutoff and ramp)."""
        s = self.s
        S = np.zeros((self.N, self.N))
        rc = lib().orc_h0(self.nat, self.no, _f64(pos), np.ones(self.no),
                          np.zeros(self.N), _f64(s.overlap_block),
                          s.overlap_decay, s.hop_cutoff, s.taper_width, S)
        assert rc == 0
        return S

    def loewdin(self, pos, eig=None):
        """(S, X = S^-1/2) from the eigen-decomposition of S (Jacobi, or
        `eig` with the same return convention)."""
        S = self.overlap(pos)
        ev, Vt = (eig or jacobi)(S)
        if ev.min() <= 0.0:
            raise ValueError("overlap matrix is not positive definite")
        X = Vt.T @ np.diag(1.0 / np.sqrt(ev)) @ Vt
        return S, X


# ---------------------------------------------------------------------------
# Electronic solve (Section IV.A-B)
# ---------------------------------------------------------------------------
@dataclass
class Electronic:
    H0: np.ndarray
    G: np.ndarray
    H: np.ndarray
    evals: np.ndarray
    Vt: np.ndarray          # eigenvectors as rows
    mu: float
    f: np.ndarray
    D: np.ndarray
    q: np.ndarray
    n: np.ndarray
    S: Optional[np.ndarray] = None   # overlap (non-orthogonal basis)
    X: Optional[np.ndarray] = None   # S^-1/2; eigenvectors of X H X in Vt

    @property
    def r(self):
        return self.q - self.n

    def eigvecs(self):
        """Generalised eigenvectors C (columns): H C = S C diag(evals),
        C^T S C = I (orthonormal eigenvectors in the orthogonal basis)."""
        return self.Vt.T if self.X is None else self.X @ self.Vt.T


def jacobi(A, tol=1e-14, max_sweeps=60):
    """Eigen-decomposition of a symmetric matrix by cyclic Jacobi."""
    N = A.shape[0]
    W = _f64(A).copy()
    ev = np.zeros(N)
    Vt = np.zeros((N, N))
    sweeps = lib().orc_jacobi(N, W, ev, Vt, tol, max_sweeps)
    if sweeps < 0:
        raise RuntimeError("Jacobi did not converge")
    return ev, Vt


def fermi_mu(evals, beta, ne):
    f = np.zeros(len(evals))
    mu = lib().orc_fermi_mu(len(evals), _f64(evals), beta, ne, f)
    return mu, f


def density(Vt, f):
    N = Vt.shape[0]
    D = np.zeros((N, N))
    lib().orc_density(N, _f64(Vt), _f64(f), D)
    return D


def charges(model, D, S=None):
    """Net Mulliken charges q_I = sum_a (D S)[Ia,Ia] - Z_I (S = I: the
    diagonal sums of the orthogonal basis)."""
    pop = np.diag(D) if S is None else np.einsum("ij,ji->i", D, S)
    return pop.reshape(model.nat, model.no).sum(axis=1) - model.zcore


def hamiltonian(model, H0, G, n, S=None):
    """H[n] = H0 + (S V + V S)/2, V = diag of the orbital potentials
    (Gamma n on each atom's orbitals); S = I gives H0 + V."""
    v = model.orbital_potential(G, n)
    if S is None:
        return H0 + np.diag(v)
    return H0 + 0.5 * (S * v[None, :] + v[:, None] * S)


def electronic(model, pos, n, H0=None, G=None, eig=None, ov=None):
    """One-shot solve of the linearised functional at fixed n.

    `eig` (default: `jacobi`) returns (eigenvalues, eigenvectors as rows);
    a library eigensolver may stand in for Jacobi on matrices too large for
    it, the rest of the solve being unchanged.  In a non-orthogonal basis
    `ov` = (S, X) from `Model.loewdin` (computed here when not given); the
    eigenproblem is that of H' = X H X, and D = X D' X."""
    if H0 is None:
        H0 = model.h0(pos)
    if G is None:
        G = model.gamma(pos)
    S = X = None
    if model.nonorth:
        S, X = ov if ov is not None else model.loewdin(pos, eig)
    H = hamiltonian(model, H0, G, n, S)
    ev, Vt = (eig or jacobi)(H if X is None else X @ H @ X)
    mu, f = fermi_mu(ev, model.beta, model.s.n_electrons)
    D = density(Vt, f)
    if X is not None:
        D = X @ D @ X
    q = charges(model, D, S)
    return Electronic(H0=H0, G=G, H=H, evals=ev, Vt=Vt, mu=mu, f=f, D=D, q=q,
                      n=np.array(n, dtype=np.float64), S=S, X=X)


# ---------------------------------------------------------------------------
# Free energy and forces (Eqs. 35, 37, 38, 40)
# ---------------------------------------------------------------------------
def entropy(model, el):
    return lib().orc_entropy(model.N, _f64(el.evals), model.beta, el.mu)


def free_energy(model, pos, el) -> Dict[str, float]:
    """Shadow free energy Omega[n](R) and its parts."""
    e_band = float(np.sum(el.H0 * el.D))
    e_coul = 0.5 * float((2.0 * el.q - el.n) @ (el.G @ el.n))
    e_rep = model.erep(pos)
    ts = model.s.te * entropy(model, el)
    return dict(omega=e_band + e_coul + e_rep - ts, e_band=e_band,
                e_coul=e_coul, e_rep=e_rep, te_s=ts)


def forces(model, pos, el):
    """-dOmega/dR at fixed n (Hellmann-Feynman; D is variational)."""
    s = model.s
    F = np.zeros(3 * model.nat)
    assert lib().orc_forces(model.nat, model.no, _f64(pos),
                            _f64(s.hop_block), s.hop_decay, s.hop_cutoff,
                            s.taper_width, s.gamma_soft, _f64(el.D),
                            _f64(el.q), _f64(el.n), F) == 0
    _, Fr = model.erep(pos, want_force=True)
    F = F.reshape(model.nat, 3) + Fr
    if el.S is not None:
        # S(R) enters twice: through H = H0 + (S V + V S)/2, which gives
        # sum_ab dS_ab D_ab (V_a + V_b)/2, and through the normalisation of
        # the generalised eigenvectors, which gives -Tr[E dS] with the
        # energy-weighted density matrix E = 2 sum_i f_i e_i c_i c_i^T (the
        # basis-set dependent Pulay term).  Both are -Tr[M dS/dR] for
        # M = (V D + D V)/2 - E, the hopping-force contraction with the
        # overlap's block and decay in place of the hopping's (and no
        # Coulomb term).
        v = model.orbital_potential(el.G, el.n)
        C = el.eigvecs()
        E = (C * (2.0 * el.f * el.evals)[None, :]) @ C.T
        M = 0.5 * (v[:, None] * el.D + el.D * v[None, :]) - E
        Fs = np.zeros(3 * model.nat)
        zero = np.zeros(model.nat)
        assert lib().orc_forces(model.nat, model.no, _f64(pos),
                                _f64(s.overlap_block), s.overlap_decay,
                                s.hop_cutoff, s.taper_width, s.gamma_soft,
                                _f64(M), zero, zero, Fs) == 0
        F = F + Fs.reshape(model.nat, 3)
    return F


# ---------------------------------------------------------------------------
# Response and kernel (Section V)
# ---------------------------------------------------------------------------
def response(model, el, v):
    """Directional derivative of q[n + lambda v] at lambda = 0 (canonical).

    The perturbation of n by v shifts the orbital potentials by Gamma v; the
    density-matrix response follows in closed form from the eigenpairs.
    """
    h = model.orbital_potential(el.G, v)
    if el.S is not None:
        return _response_nonorth(model, el, h)
    dd = np.zeros(model.N)
    lib().orc_response_diag(model.N, _f64(el.Vt), _f64(el.evals), model.beta,
                            el.mu, _f64(h), dd)
    return dd.reshape(model.nat, model.no).sum(axis=1)


def _response_nonorth(model, el, h):
    """Canonical response in a non-orthogonal basis: the perturbation of H
    is H1 = (S diag(h) + diag(h) S)/2; in the generalised eigenbasis C
    (C^T S C = I) its matrix is P = C^T H1 C and the response of the
    occupation matrix is the divided difference of 2 f times P - mu' I,
    with mu' chosen so that the electron count Tr[D1 S] = Tr[P1] stays
    fixed (the closed form of the orthogonal case); q1 = Mulliken charges
    of D1 = C P1 C^T."""
    S = el.S
    C = el.eigvecs()
    P = C.T @ (0.5 * (S * h[None, :] + h[:, None] * S)) @ C
    x = model.beta * (el.evals - el.mu)
    Fd = np.empty((model.N, model.N))
    lib().orc_fermi_divdiff_matrix(model.N, _f64(x), model.beta, Fd)
    fd = np.diag(Fd)
    mup = float(fd @ np.diag(P)) / float(fd.sum())
    P1 = 2.0 * Fd * (P - mup * np.eye(model.N))
    D1 = C @ P1 @ C.T
    return charges(model, D1, S) + model.zcore


def response_fd(model, pos, el, v, h=1e-4):
    """Central finite difference of q along v (independent check)."""
    qp = electronic(model, pos, el.n + h * v, el.H0, el.G).q
    qm = electronic(model, pos, el.n - h * v, el.H0, el.G).q
    return (qp - qm) / (2.0 * h)


def jacobian(model, el):
    """Full charge Jacobian J = dq/dn, one response per atom."""
    J = np.zeros((model.nat, model.nat))
    for j in range(model.nat):
        e = np.zeros(model.nat)
        e[j] = 1.0
        J[:, j] = response(model, el, e)
    return J


def kernel_full(model, el):
    """The exact kernel K = (J - I)^{-1} of Eq. 43 (krylov_mode 2: all
    N_at responses, dense inverse)."""
    J = jacobian(model, el)
    return np.linalg.inv(J - np.eye(model.nat))


R_FLOOR = 1e-8     # RMS residual below which the kernel is K0


@dataclass
class KernelResult:
    K: np.ndarray          # explicit N_at x N_at kernel K_m
    V: np.ndarray          # directions actually used (N_at x m')
    rank: int
    W: Optional[np.ndarray] = None   # their images (J - I) v_j (N_at x m')


def _orth(x, V):
    """Gram-Schmidt of x against the columns of V (twice), normalised."""
    y = x.copy()
    for _ in range(2):
        for j in range(V.shape[1]):
            y -= (V[:, j] @ y) * V[:, j]
    nrm = np.linalg.norm(y)
    return y, nrm


def kernel_from_images(gamma, V, W):
    """The Sherman-Morrison sequence of Eq. 50 from K0 = -gamma I over given
    orthonormal directions V (columns, in order) whose images
    w_j = (J - I) v_j are given in W: a kernel whose images were evaluated
    at different times (the directions an earlier build left plus those
    added since)."""
    nat = V.shape[0]
    J = (1.0 - 1.0 / gamma) * np.eye(nat)
    K = -gamma * np.eye(nat)
    for j in range(V.shape[1]):
        v = V[:, j]
        u = W[:, j] + v - J @ v
        J = J + np.outer(u, v)
        Ku = K @ u
        K = K - np.outer(Ku, v @ K) / (1.0 + v @ Ku)
    return K


def kernel_sm(model, el, gamma, m, mode=0, v_prev=None, resp=None,
              floor=R_FLOOR):
    """Rank-m kernel by the Sherman-Morrison sequence (Eq. 50).

    K0 = -gamma I, i.e. J0 = (1 - 1/gamma) I (Eqs. 48-49).  Directions:
      mode 0: v_1 = K0 r / |K0 r| (Eq. 51), then each v_j is K_{j-1} r
              orthogonalised against v_1..v_{j-1} (Section V.F);
      mode 1: v_1 as above, then the previous build's images
              w_j = (J - I) v_j, passed as v_prev[:, 0..m-2], orthogonalised
              in that order: the directions do not depend on this build's
              responses (all m can be evaluated together), and successive
              builds are a subspace iteration with J - I, which turns the
              directions towards its stiffest modes.
    A direction whose orthogonalised norm falls below 1e-10 of its raw norm
    ends the sequence (the space is exhausted).  For a kernel that the
    dynamics will apply to later residuals, a residual with RMS at or below
    `floor` gives the rank-0 kernel K0: its direction is rounding noise
    (e.g. right after a converged SCF).  The SCF, which applies each kernel
    to the residual that built it, passes floor = 0.  `resp` overrides the
    response function (defaults to the closed-form canonical response).
    """
    nat = model.nat
    resp = resp or (lambda v: response(model, el, v))
    c = 1.0 - 1.0 / gamma
    J = c * np.eye(nat)
    K = -gamma * np.eye(nat)
    r = el.r
    Vs = np.zeros((nat, 0))
    Ws = np.zeros((nat, 0))
    for i in range(m):
        if mode == 1 and i > 0:
            if v_prev is None or i - 1 >= v_prev.shape[1]:
                break
            cand = v_prev[:, i - 1]
        else:
            cand = K @ r
        raw = np.linalg.norm(cand)
        if raw == 0.0:
            break
        if i == 0 and raw / (gamma * np.sqrt(nat)) <= floor:
            break
        v, nrm = _orth(cand, Vs)
        if nrm <= 1e-10 * raw:
            break
        v = v / nrm
        jv = resp(v)
        u = jv - J @ v
        J = J + np.outer(u, v)
        Ku = K @ u
        vK = v @ K
        K = K - np.outer(Ku, vK) / (1.0 + v @ Ku)
        Vs = np.column_stack([Vs, v])
        Ws = np.column_stack([Ws, jv - v])
    return KernelResult(K=K, V=Vs, rank=Vs.shape[1], W=Ws)


# ---------------------------------------------------------------------------
# Integration (Eqs. 20, 22, 23, 52)
# ---------------------------------------------------------------------------
@dataclass
class State:
    pos: np.ndarray
    vel: np.ndarray
    force: np.ndarray
    n_hist: np.ndarray            # (kmax+1, nat): n(t), n(t-dt), ...
    kr: np.ndarray                # K_m r(t), used for n(t+dt)
    K: Optional[np.ndarray]       # explicit kernel of the last build
    V: Optional[np.ndarray]       # its directions
    el: Electronic
    W: Optional[np.ndarray] = None  # their images (J - I) v_j
    n_rb: int = 0                   # columns of V from the last rebuild
    W_rb: Optional[np.ndarray] = None  # the last rebuild's images (block mode)
    step: int = 0
    energy: Dict[str, float] = field(default_factory=dict)
    # the last low-rank build for the dynamics stopped at rank 0 although a
    # positive rank was asked for (a zero or floor-level residual, e.g. just
    # after the converged SCF): the next step builds again, whatever the
    # refresh period (reading of Section V.E's on-the-fly reuse)
    pending: bool = False


AUTO_GAMMA_ITERS = 20


def auto_gamma(model, el, iters=AUTO_GAMMA_ITERS):
    """K0 = -gamma I with gamma from the stiffest charge-response mode.

    Power iteration v <- -J v / |J v| from v = r/|r| (e_0 if r = 0) gives
    |lambda_max(J)| ~ |J v|; gamma = 1.5 / (1 + |lambda|) rounded down to
    two significant digits, clipped to [1e-4, 1], keeps every eigenvalue e
    of K0 (J - I) below 1.5, so the kernel SCF contracts and the electronic
    Verlet step (stable for kappa e < 4, Section II.F) stays stable on modes
    the low-rank update does not capture.  The relative grid makes the
    choice insensitive to rounding in lambda.
    """
    r = el.r
    v = r.copy() if np.linalg.norm(r) > 0 else np.eye(model.nat)[0]
    v = v / np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = response(model, el, v)
        lam = np.linalg.norm(w)
        v = -w / lam
    g0 = 1.5 / (1.0 + lam)
    g = 1.0
    if g0 < 1.0:
        sc = 10.0 ** (1.0 - math.floor(math.log10(g0)))
        g = math.floor(g0 * sc) / sc
    return float(min(1.0, max(1e-4, g))), float(lam)


def scf(model, pos, gamma, m, tol=1e-10, max_iter=200, n0=None,
        mode=0):
    """Ground state by the kernel SCF of Eq. 52, from n = 0."""
    H0 = model.h0(pos)
    G = model.gamma(pos)
    n = np.zeros(model.nat) if n0 is None else np.array(n0, dtype=float)
    hist = []
    for it in range(max_iter):
        el = electronic(model, pos, n, H0, G)
        rms = float(np.sqrt(np.mean(el.r ** 2)))
        hist.append(rms)
        if rms <= tol:
            return el, hist
        kr = kernel_sm(model, el, gamma, m, mode=0, floor=0.0)
        n = n - kr.K @ el.r
    raise RuntimeError(f"SCF did not converge: {hist[-5:]}")


def init_state(model, pos=None, vel=None, scf_tol=1e-10, gamma=None,
               rank=None):
    s = model.s
    pos = _f64(s.pos if pos is None else pos).copy()
    vel = _f64(s.vel if vel is None else vel).copy()
    gamma = s.k0_gamma if gamma is None else gamma
    rank = s.rank if rank is None else rank
    if gamma <= 0.0:      # automatic stability rule at n = 0
        gamma, _ = auto_gamma(model, electronic(model, pos, np.zeros(model.nat)))
        model.gamma_used = gamma
    el, _ = scf(model, pos, gamma, rank, tol=scf_tol)
    hist = np.tile(el.n, (s.kmax + 1, 1))            # Eq. 20: ndot(t0) = 0
    pending = False
    if s.krylov_mode == 2:
        K, V, W = kernel_full(model, el), None, None
    else:
        kres = kernel_sm(model, el, gamma, rank, mode=s.krylov_mode)
        K, V, W = kres.K, kres.V, kres.W
        pending = rank > 0 and kres.rank == 0
    st = State(pos=pos, vel=vel, force=forces(model, pos, el), n_hist=hist,
               kr=K @ el.r, K=K, V=V, W=W, el=el, pending=pending,
               n_rb=0 if V is None else V.shape[1], W_rb=W)
    st.energy = energy_report(model, st)
    return st


def energy_report(model, st):
    fe = free_energy(model, st.pos, st.el)
    ke = 0.5 * float(np.sum(model.mass[:, None] * st.vel ** 2))
    fe.update(e_kin=ke, e_total=fe["omega"] + ke,
              rms_res=float(np.sqrt(np.mean(st.el.r ** 2))), mu=st.el.mu)
    return fe


def md_step(model, st, gamma=None, rank=None, want_energy=True):
    """One XL-BOMD step, t -> t + dt (Eqs. 22, 23)."""
    s = model.s
    if gamma is None:
        gamma = s.k0_gamma if s.k0_gamma > 0 else model.gamma_used
    rank = s.rank if rank is None else rank
    kappa, alpha, ck = TABLE_I[s.kmax]
    dt = s.dt
    m = model.mass[:, None]
    vel = st.vel + 0.5 * dt * st.force / m
    pos = st.pos + dt * vel
    h = st.n_hist
    n_new = 2.0 * h[0] - h[1] - kappa * st.kr
    for k, c in enumerate(ck):
        n_new = n_new + alpha * c * h[k]
    hist = np.vstack([n_new[None, :], h[:-1]])
    el = electronic(model, pos, n_new)
    F = forces(model, pos, el)
    step = st.step + 1
    pending = False
    n_rb, W_rb = st.n_rb, st.W_rb
    if (step % s.kernel_every == 0 or st.K is None) and s.krylov_mode == 2:
        K, V, W = kernel_full(model, el), None, None
    elif step % s.kernel_every == 0 or st.K is None or st.pending:
        kres = kernel_sm(model, el, gamma, rank, mode=s.krylov_mode,
                         v_prev=st.W_rb)
        K, V, W = kres.K, kres.V, kres.W
        n_rb, W_rb = kres.rank, kres.W
        pending = rank > 0 and kres.rank == 0
    elif getattr(s, "kernel_otf", 0) > 0:
        # Section V.E: the previous step's kernel is the estimate K0(t) that
        # one rank-1 update along v = K0(t) r / |K0(t) r| improves; the
        # updates accumulate between rebuilds in a window of kernel_otf
        # directions (the oldest leaves when it is full)
        V, W, n_rb, W_rb = st.V, st.W, st.n_rb, st.W_rb
        if V.shape[1] - n_rb >= s.kernel_otf:
            V = np.delete(V, n_rb, axis=1)
            W = np.delete(W, n_rb, axis=1)
        cand = st.K @ el.r
        raw = np.linalg.norm(cand)
        v, nrm = _orth(cand, V)
        if raw > 0.0 and nrm > 1e-10 * raw:
            v = v / nrm
            V = np.column_stack([V, v])
            W = np.column_stack([W, response(model, el, v) - v])
        K = kernel_from_images(gamma, V, W)
    else:
        K, V, W, n_rb, W_rb = st.K, st.V, st.W, st.n_rb, st.W_rb
    kr = K @ el.r
    vel = vel + 0.5 * dt * F / m
    nst = State(pos=pos, vel=vel, force=F, n_hist=hist, kr=kr, K=K, V=V,
                W=W, el=el, step=step, pending=pending, n_rb=n_rb, W_rb=W_rb)
    if want_energy:
        nst.energy = energy_report(model, nst)
    return nst


def run(model, steps, st=None, callback=None, **kw):
    st = st if st is not None else init_state(model)
    out = [st.energy]
    for _ in range(steps):
        st = md_step(model, st, **kw)
        out.append(st.energy)
        if callback:
            callback(st)
    return st, out
