"""Synthetic self-consistent-charge tight-binding systems.

The paper's own test systems (a solvated hydroquinone radical, liquid water,
liquid nitromethane; Section VI) and their SCC-DFTB parameter tables are not
available, so five synthetic workloads stand in for them. Every array is drawn
from numpy's PCG64 with a fixed seed (17050000 + config index), so the oracle
and the GPU library see bit-identical inputs.

Only raw parameters come out of here: positions, masses, per-orbital onsite
energies and their jitter, the hopping block, Hubbard U values and scalar
constants. The model built from them (Hamiltonian, Coulomb matrix, repulsion,
forces) lives separately in the oracle and in the HIP library.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

SEED_BASE = 17050000


@dataclasses.dataclass
class System:
    """Raw parameters of one synthetic system (all float64 / int)."""
    name: str
    n_atoms: int
    n_orb: int
    pos: np.ndarray            # (n_atoms, 3)
    vel: np.ndarray            # (n_atoms, 3)
    mass: np.ndarray           # (n_atoms,)
    onsite: np.ndarray         # (n_orb,) per-orbital onsite energy
    onsite_jitter: np.ndarray  # (n_atoms * n_orb,) additive onsite jitter
    hop_block: np.ndarray      # (n_orb, n_orb) symmetric hopping block B
    hop_decay: float           # lambda in exp(-r / lambda)
    hop_cutoff: float          # r_c
    taper_width: float         # width of the smooth cutoff ramp (0 = hard)
    hubbard_u: np.ndarray      # (n_atoms,)
    gamma_soft: float          # Coulomb softening a in 1/sqrt(r^2 + a^2)
    rep_a: float               # pair repulsion prefactor (0 disables)
    rep_decay: float           # pair repulsion decay length
    n_electrons: float
    te: float                  # electronic temperature, energy units
    dt: float
    kmax: int                  # dissipation order (row of Table I)
    rank: int                  # kernel rank m
    kernel_every: int          # kernel rebuild period in steps
    krylov_mode: int           # 0 sequential Krylov, 1 block directions
    k0_gamma: float            # K0 = -gamma * I
    steps: int
    kernel_otf: int = 0        # on-the-fly rank-1 directions kept between rebuilds
    # non-orthogonal basis: overlap block Bs (n_orb, n_orb) and its decay
    # length, S[Ia,Jb] = Bs_ab exp(-r / overlap_decay) s(r); None = orthogonal
    overlap_block: Optional[np.ndarray] = None
    overlap_decay: float = 0.0

    @property
    def n(self) -> int:
        return self.n_atoms * self.n_orb

    def replace(self, **kw) -> "System":
        return dataclasses.replace(self, **kw)


# ---------------------------------------------------------------------------
# Geometry helpers (pure layout; no model arithmetic)
# ---------------------------------------------------------------------------

def _cubic_sites(dims, spacing):
    nx, ny, nz = dims
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz),
                             indexing="ij"), axis=-1).reshape(-1, 3)
    return g.astype(np.float64) * spacing


def _near_cubic_dims(n_sites):
    """Smallest near-cubic box of lattice sites holding n_sites."""
    s = max(1, int(round(n_sites ** (1.0 / 3.0))))
    dims = [s, s, s]
    i = 0
    while dims[0] * dims[1] * dims[2] < n_sites:
        dims[i % 3] += 1
        i += 1
    return tuple(dims)


def _random_packing(rng, n_atoms, side, rmin):
    """Random sequential addition in a cube, rejecting pairs closer than rmin."""
    cell = rmin
    nc = max(1, int(side // cell))
    grid: Dict[tuple, List[int]] = {}
    pts = np.zeros((n_atoms, 3))
    k = 0
    tries = 0
    while k < n_atoms:
        tries += 1
        if tries > 1000 * n_atoms:
            raise RuntimeError("random packing failed")
        p = rng.uniform(0.0, side, size=3)
        c = tuple(np.minimum((p // cell).astype(int), nc - 1))
        ok = True
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for j in grid.get((c[0] + dx, c[1] + dy, c[2] + dz), ()):
                        d = pts[j] - p
                        if d @ d < rmin * rmin:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            pts[k] = p
            grid.setdefault(c, []).append(k)
            k += 1
    return pts


def _sym_block(rng, n_orb):
    g = rng.uniform(-1.0, 1.0, size=(n_orb, n_orb))
    return 0.5 * (g + g.T)


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

# Shared constants of the s + 3p model (workloads 2, 3, 4, 5).
_SP_ONSITE = np.array([-1.0, -0.4, -0.4, -0.4])
_SP_ONSITE_SMALL_GAP = _SP_ONSITE / 6.0   # onsite spread 0.1

CONFIGS = {
    # 64-atom s-orbital cluster, plain FP64.
    "c1": dict(index=1, dims=(4, 4, 4), spacing=2.0, jitter=0.1, n_orb=1,
               onsite=np.array([0.0]), onsite_jitter=0.5, hop_block="c1",
               hop_decay=1.0, hop_cutoff=4.0, taper_width=0.5,
               u_range=(1.0, 1.0), gamma_soft=1.0, rep_a=1.6, rep_decay=0.5,
               te=0.1, dt=0.5, kmax=5, rank=1, kernel_every=1,
               krylov_mode=0, k0_gamma=0.1, steps=200),
    # 1024 atoms x (s + 3p), N = 4096.
    "c2": dict(index=2, dims=(8, 8, 16), spacing=2.5, jitter=0.15, n_orb=4,
               onsite=_SP_ONSITE, onsite_jitter=0.0, hop_block="rand",
               hop_decay=1.2, hop_cutoff=5.0, taper_width=0.5,
               u_range=(0.8, 1.2), gamma_soft=1.0, rep_a=5.8, rep_decay=0.6,
               te=0.05, dt=0.5, kmax=5, rank=4, kernel_every=1,
               krylov_mode=0, k0_gamma=0.0, steps=1000),
    # Small-gap metallic case, N = 8192.
    "c3": dict(index=3, dims=(8, 16, 16), spacing=2.5, jitter=0.15, n_orb=4,
               onsite=_SP_ONSITE_SMALL_GAP, onsite_jitter=0.0,
               hop_block="rand", hop_decay=1.2, hop_cutoff=5.0,
               taper_width=0.5, u_range=(0.8, 1.2), gamma_soft=1.0,
               rep_a=5.8, rep_decay=0.6, te=0.02, dt=0.5, kmax=5, rank=8,
               kernel_every=1, krylov_mode=0, k0_gamma=0.0, steps=500),
    # Serving stream element template (sizes drawn per request).
    "c4": dict(index=4, dims=None, spacing=2.5, jitter=0.15, n_orb=4,
               onsite=_SP_ONSITE, onsite_jitter=0.0, hop_block="rand",
               hop_decay=1.2, hop_cutoff=5.0, taper_width=0.5,
               u_range=(0.8, 1.2), gamma_soft=1.0, rep_a=5.8, rep_decay=0.6,
               te=0.05, dt=0.5, kmax=5, rank=4, kernel_every=1,
               krylov_mode=0, k0_gamma=0.0, steps=100),
    # 4096 randomly packed atoms, N = 16384.
    "c5": dict(index=5, dims=None, spacing=None, jitter=0.0, n_orb=4,
               onsite=_SP_ONSITE, onsite_jitter=0.0, hop_block="rand",
               hop_decay=1.2, hop_cutoff=5.0, taper_width=0.5,
               u_range=(0.8, 1.2), gamma_soft=1.0, rep_a=5.8, rep_decay=0.6,
               te=0.05, dt=0.5, kmax=5, rank=6, kernel_every=50,
               krylov_mode=0, k0_gamma=0.0, steps=2000, kernel_otf=10,
               n_atoms=4096, density=0.06, rmin=1.2),
}


def _finish(name, cfg, rng, pos, n_atoms, overrides):
    n_orb = cfg["n_orb"]
    if cfg["hop_block"] == "c1":
        hop = np.array([[-1.0]])
    else:
        hop = _sym_block(rng, n_orb)
    lo, hi = cfg["u_range"]
    u = (np.full(n_atoms, lo) if lo == hi
         else rng.uniform(lo, hi, size=n_atoms))
    oj = cfg["onsite_jitter"]
    jit = (rng.uniform(-oj, oj, size=n_atoms * n_orb) if oj > 0
           else np.zeros(n_atoms * n_orb))
    sysd = dict(
        name=name, n_atoms=n_atoms, n_orb=n_orb,
        pos=np.ascontiguousarray(pos, dtype=np.float64),
        vel=np.zeros((n_atoms, 3)),
        mass=np.full(n_atoms, float(cfg.get("mass", 40.0))),
        onsite=np.asarray(cfg["onsite"], dtype=np.float64).copy(),
        onsite_jitter=jit, hop_block=hop,
        hop_decay=float(cfg["hop_decay"]), hop_cutoff=float(cfg["hop_cutoff"]),
        taper_width=float(cfg["taper_width"]), hubbard_u=u,
        gamma_soft=float(cfg["gamma_soft"]), rep_a=float(cfg["rep_a"]),
        rep_decay=float(cfg["rep_decay"]),
        n_electrons=float(n_atoms * n_orb), te=float(cfg["te"]),
        dt=float(cfg["dt"]), kmax=int(cfg["kmax"]), rank=int(cfg["rank"]),
        kernel_every=int(cfg["kernel_every"]),
        krylov_mode=int(cfg["krylov_mode"]), k0_gamma=float(cfg["k0_gamma"]),
        steps=int(cfg["steps"]), kernel_otf=int(cfg.get("kernel_otf", 0)))
    sysd.update(overrides)
    return System(**sysd)


def make_system(name: str, seed: Optional[int] = None, **overrides) -> System:
    """Build workload `name` ("c1" .. "c5") from its fixed seed."""
    cfg = CONFIGS[name]
    rng = np.random.Generator(np.random.PCG64(
        SEED_BASE + cfg["index"] if seed is None else seed))
    if name == "c5":
        n_atoms = cfg["n_atoms"]
        side = (n_atoms / cfg["density"]) ** (1.0 / 3.0)
        pos = _random_packing(rng, n_atoms, side, cfg["rmin"])
    elif name == "c4":
        raise ValueError("c4 is a stream: use serving_stream()")
    else:
        sites = _cubic_sites(cfg["dims"], cfg["spacing"])
        pos = sites + rng.uniform(-cfg["jitter"], cfg["jitter"],
                                  size=sites.shape)
        n_atoms = sites.shape[0]
    return _finish(name, cfg, rng, pos, n_atoms, overrides)


def lattice_system(n_atoms: int, template: str = "c2", seed: int = 1,
                   **overrides) -> System:
    """First n_atoms sites of a near-cubic lattice with `template`'s model.

    Used for small parity cases and for the serving stream's requests.
    """
    cfg = dict(CONFIGS[template])
    rng = np.random.Generator(np.random.PCG64(seed))
    spacing = cfg["spacing"] if cfg["spacing"] else 2.5
    jitter = cfg["jitter"] if cfg["jitter"] else 0.15
    dims = _near_cubic_dims(n_atoms)
    sites = _cubic_sites(dims, spacing)[:n_atoms]
    pos = sites + rng.uniform(-jitter, jitter, size=sites.shape)
    return _finish(f"{template}-lat{n_atoms}", cfg, rng, pos, n_atoms,
                   overrides)


def packed_system(n_atoms: int, template: str = "c5", seed: int = 1,
                  **overrides) -> System:
    """n_atoms randomly packed atoms at `template`'s density and minimum
    distance, with its model: the large workload's geometry (irregular
    neighbour counts, atoms in no spatial order) at any size."""
    cfg = dict(CONFIGS[template])
    rng = np.random.Generator(np.random.PCG64(seed))
    side = (n_atoms / cfg["density"]) ** (1.0 / 3.0)
    pos = _random_packing(rng, n_atoms, side, cfg["rmin"])
    return _finish(f"{template}-packed{n_atoms}", cfg, rng, pos, n_atoms, overrides)


def with_overlap(s: System, scale: float = 0.3) -> System:
    """The same system in a non-orthogonal basis: overlap block
    -scale * B / max|B| for the hopping block B (bonding hoppings are
    negative where overlaps are positive, as in extended-Hueckel-type
    parametrisations) with the hopping's decay length."""
    hb = np.asarray(s.hop_block, dtype=np.float64)
    return s.replace(name=s.name + "-ov", overlap_block=-scale * hb / np.abs(hb).max(),
                     overlap_decay=float(s.hop_decay))


def serving_stream(n_requests: int = 256, rate_hz: float = 200.0,
                   seed: Optional[int] = None):
    """Poisson arrival stream of independent systems (the serving workload).

    Returns a list of (arrival_time_s, System). Sizes are log-uniform in
    16..512 atoms, Te uniform in [0.02, 0.1], kernel rank uniform in 2..6.
    """
    cfg = CONFIGS["c4"]
    rng = np.random.Generator(np.random.PCG64(
        SEED_BASE + cfg["index"] if seed is None else seed))
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate_hz)
        n_at = int(round(math.exp(rng.uniform(math.log(16), math.log(512)))))
        te = float(rng.uniform(0.02, 0.1))
        rank = int(rng.integers(2, 7))
        sub_seed = int(rng.integers(0, 2**31 - 1))
        s = lattice_system(n_at, "c4", seed=sub_seed, te=te, rank=rank)
        s.name = f"req{i:03d}-n{n_at}"
        out.append((t, s))
    return out
