"""Descriptor checks of xlbomd_init_system, on the CPU: every rule rejects
its case with XLBOMD_E_INVALID and a message naming the field.  The check
runs before the library makes any device call, so no GPU is needed; every
case below is invalid, so none of them reaches the device."""
import ctypes
import os

import numpy as np
import pytest

from paper_1705_10845_amd import binding as B
from synth import make_system

pytestmark = pytest.mark.skipif(not os.path.exists(B.LIB_PATH), reason="library not built")


def _c1():
    return make_system("c1")          # 64 atoms x 1 orbital, 64 electrons


def _small(**kw):
    s = _c1()
    return s.replace(n_atoms=4, n_electrons=4.0, **kw)


CASES = [
    ("empty", dict(n_atoms=0), "n_atoms"),
    ("negative atoms", dict(n_atoms=-3), "n_atoms"),
    ("above the size limit", dict(n_atoms=46337), "n_atoms * n_orb"),
    ("size limit by orbitals", dict(n_atoms=5793, n_orb=8), "n_atoms * n_orb"),
    ("no orbitals", dict(n_orb=0), "n_orb"),
    ("nine orbitals", dict(n_orb=9), "n_orb"),
    ("no electrons", dict(n_electrons=0.0), "n_electrons"),
    ("full shell", dict(n_electrons=128.0), "n_electrons"),
    ("nan electrons", dict(n_electrons=float("nan")), "n_electrons"),
    ("zero temperature", dict(te=0.0), "te"),
    ("negative dt", dict(dt=-0.1), "dt"),
    ("kmax 4", dict(kmax=4), "kmax"),
    ("kmax 8", dict(kmax=8), "kmax"),
    ("rank 17", dict(rank=17), "kernel_rank"),
    ("negative rank", dict(rank=-1), "kernel_rank"),
    ("refresh 0", dict(kernel_every=0), "kernel_every"),
    ("krylov mode 3", dict(krylov_mode=3), "krylov_mode"),
    ("gamma above 1", dict(k0_gamma=1.5), "k0_gamma"),
    ("negative gamma", dict(k0_gamma=-0.1), "k0_gamma"),
    ("zero hop decay", dict(hop_decay=0.0), "model lengths"),
    ("zero cutoff", dict(hop_cutoff=0.0), "model lengths"),
    ("negative taper", dict(taper_width=-0.5), "model lengths"),
    ("zero softening", dict(gamma_soft=0.0), "model lengths"),
    ("repulsion without decay", dict(rep_a=1.0, rep_decay=0.0), "model lengths"),
]


def _rejected(system, **kw):
    with pytest.raises(B.XlbomdError) as e:
        B.XLBOMD(system, **kw)
    return e.value


@pytest.mark.parametrize("name,change,field", CASES, ids=[c[0] for c in CASES])
def test_descriptor_rule(name, change, field):
    e = _rejected(_c1().replace(**change))
    assert e.code == -1
    assert field in str(e)


def test_rank_above_atom_count():
    e = _rejected(_small(rank=5))
    assert e.code == -1 and "kernel_rank" in str(e)


def test_masses_must_be_positive():
    s = _c1()
    m = s.mass.copy()
    m[17] = 0.0
    e = _rejected(s.replace(mass=m))
    assert e.code == -1 and "masses" in str(e)


def test_level_request_and_precision_ranges():
    e = _rejected(_c1(), foe_levels=41)
    assert e.code == -1 and "foe_levels" in str(e)
    e = _rejected(_c1(), foe_levels=-1)
    assert e.code == -1 and "foe_levels" in str(e)
    e = _rejected(_c1(), precision=5)
    assert e.code == -1 and "precision" in str(e)


def test_allocator_needs_free():
    class Half:
        struct = B.Allocator(B._ALLOC_FN(lambda n, c: None), B._FREE_FN(), None)
    e = _rejected(_c1(), allocator=Half())
    assert e.code == -1 and "allocator" in str(e)


def test_missing_arrays_and_handles():
    """Null arrays, a null descriptor and a null output handle are rejected
    through the raw ABI, and the error text is kept for xlbomd_last_error."""
    L = B.lib()
    h = ctypes.c_void_p()
    assert L.xlbomd_init_system(None, ctypes.byref(h)) == -1
    assert b"descriptor" in L.xlbomd_last_error()
    s = _c1()
    d = B.Desc()
    d.n_atoms, d.n_orb, d.n_electrons = s.n_atoms, s.n_orb, s.n_electrons
    assert L.xlbomd_init_system(ctypes.byref(d), ctypes.byref(h)) == -1
    assert b"required" in L.xlbomd_last_error()
    assert L.xlbomd_init_system(ctypes.byref(d), None) == -1
    assert h.value is None
    # a null handle is refused by every per-handle call
    assert L.xlbomd_step(None, 1, None) == -1
    assert L.xlbomd_kernel_update(None, 0) == -1
    F = np.zeros(3)
    assert L.xlbomd_forces(None, F.ctypes.data_as(B._dp), None) == -1


def test_overlap_rules():
    s = _c1()
    ok_block = np.array([[0.3]])
    e = _rejected(s.replace(overlap_block=ok_block, overlap_decay=1.0), precision=B.MIXED_BF16X3)
    assert e.code == -1 and "XLBOMD_FP64" in str(e)
    e = _rejected(s.replace(overlap_block=ok_block, overlap_decay=0.0))
    assert e.code == -1 and "overlap_decay" in str(e)
    s4 = _c1().replace(n_orb=2, n_electrons=64.0, onsite=np.zeros(2), hop_block=-np.eye(2))
    e = _rejected(s4.replace(overlap_block=np.array([[0.1, 0.2], [0.0, 0.1]]),
                             overlap_decay=1.0))
    assert e.code == -1 and "symmetric" in str(e)
