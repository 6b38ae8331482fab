"""ctypes binding of libxlbomd.so: argument marshalling only.

Every step of the method runs in the HIP library; this module converts
numpy arrays to host pointers and maps status codes to exceptions.  It
raises if the library is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libxlbomd.so")

FP64, FP32, MIXED, MIXED_BF16X3, MIXED_BF16 = 0, 1, 2, 3, 4
_dp = ctypes.POINTER(ctypes.c_double)


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    """xlbomd_allocator: the device-memory source of a system."""
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", ctypes.c_void_p)]


class TorchAllocator:
    """Device memory for a system from PyTorch's caching allocator.

    Every buffer the library asks for is a uint8 tensor on `device` (sizes
    rounded up to 256 bytes; the caching allocator's blocks are 512-byte
    aligned), held here until the library gives it back at xlbomd_destroy.
    """

    def __init__(self, device=None):
        import torch
        self._torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.live = {}

        def _alloc(nbytes, ctx):
            try:
                t = self._torch.empty(((int(nbytes) + 255) // 256) * 256,
                                      dtype=self._torch.uint8, device=self.device)
            except Exception:
                return None
            self.live[t.data_ptr()] = t
            return t.data_ptr()

        def _free(ptr, ctx):
            self.live.pop(ptr, None)

        self._fns = (_ALLOC_FN(_alloc), _FREE_FN(_free))
        self.struct = Allocator(self._fns[0], self._fns[1], None)

    @property
    def bytes_held(self):
        return sum(t.numel() for t in self.live.values())


class Desc(ctypes.Structure):
    _fields_ = [
        ("n_atoms", ctypes.c_int32), ("n_orb", ctypes.c_int32),
        ("pos", _dp), ("vel", _dp), ("mass", _dp), ("onsite", _dp),
        ("onsite_jitter", _dp), ("hop_block", _dp),
        ("hop_decay", ctypes.c_double), ("hop_cutoff", ctypes.c_double),
        ("taper_width", ctypes.c_double), ("hubbard_u", _dp),
        ("gamma_soft", ctypes.c_double), ("rep_a", ctypes.c_double),
        ("rep_decay", ctypes.c_double), ("n_electrons", ctypes.c_double),
        ("te", ctypes.c_double), ("dt", ctypes.c_double),
        ("kmax", ctypes.c_int32), ("kernel_rank", ctypes.c_int32),
        ("kernel_every", ctypes.c_int32), ("krylov_mode", ctypes.c_int32),
        ("k0_gamma", ctypes.c_double), ("precision", ctypes.c_int32),
        ("scf_tol", ctypes.c_double), ("scf_max_iter", ctypes.c_int32),
        ("energy_every", ctypes.c_int32), ("stream", ctypes.c_void_p),
        ("allocator", ctypes.POINTER(Allocator)), ("foe_levels", ctypes.c_int32),
        ("foe_tol", ctypes.c_double), ("mu_tol", ctypes.c_double),
        ("kernel_otf", ctypes.c_int32),
        ("overlap_block", _dp), ("overlap_decay", ctypes.c_double),
    ]


class Report(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in (
        "omega", "e_band", "e_coul", "e_rep", "te_s", "e_kin", "e_total",
        "rms_res", "mu", "d_nelec")] + [(k, ctypes.c_int32) for k in (
            "step", "foe_levels", "ns_iters", "mu_reruns", "scf_iters",
            "kernel_rank", "has_energy")] + [("k0_gamma", ctypes.c_double),
                                             ("ms_step", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class XlbomdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"xlbomd error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} missing: run "
                              "python -m paper_1705_10845_amd.build")
        # PyTorch carries a HIP runtime of its own.  Initialised first, it is
        # the one the library binds to, so torch streams and torch memory
        # (TorchAllocator) are valid in library calls; loaded the other way
        # round, torch would find no GPU.
        try:
            import torch
            if torch.cuda.is_available():
                torch.cuda.init()
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.xlbomd_init_system.argtypes = [ctypes.POINTER(Desc),
                                         ctypes.POINTER(vp)]
        L.xlbomd_step.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(Report)]
        L.xlbomd_kernel_update.argtypes = [vp, ctypes.c_int32]
        L.xlbomd_set_step_mode.argtypes = [vp, ctypes.c_int32]
        L.xlbomd_step_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
        L.xlbomd_set_plan_margin.argtypes = [vp, ctypes.c_double]
        L.xlbomd_step_begin.argtypes = [vp]
        L.xlbomd_step_end.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(Report)]
        L.xlbomd_step_batch.argtypes = [ctypes.POINTER(vp), ctypes.c_int32,
                                        ctypes.c_int32, ctypes.POINTER(Report),
                                        ctypes.POINTER(ctypes.c_int32)]
        L.xlbomd_forces.argtypes = [vp, _dp, ctypes.POINTER(Report)]
        L.xlbomd_get_charges.argtypes = [vp, _dp, _dp]
        L.xlbomd_set_state.argtypes = [vp, _dp, _dp, _dp, _dp]
        L.xlbomd_get_state.argtypes = [vp, _dp, _dp, _dp, _dp]
        L.xlbomd_state_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.xlbomd_save_state.argtypes = [vp, ctypes.c_void_p, ctypes.c_size_t]
        L.xlbomd_load_state.argtypes = [vp, ctypes.c_void_p, ctypes.c_size_t]
        L.xlbomd_solve.argtypes = [vp, _dp, _dp, ctypes.POINTER(Report)]
        L.xlbomd_response.argtypes = [vp, ctypes.c_int32, _dp, _dp]
        L.xlbomd_kernel_apply.argtypes = [vp, ctypes.c_int32, _dp, _dp]
        L.xlbomd_scf.argtypes = [vp, _dp, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_int32, _dp, _dp, ctypes.POINTER(ctypes.c_int32)]
        L.xlbomd_profile.argtypes = [vp, ctypes.c_int32, _dp]
        L.xlbomd_selftest_gemm.argtypes = [ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_int32, _dp, _dp, _dp]
        L.xlbomd_selftest_gemm_time.argtypes = [ctypes.c_int32] * 5 + [_dp]
        L.xlbomd_selftest_gemm_presplit.argtypes = [ctypes.c_int32] * 3 + [_dp, _dp, _dp, _dp]
        L.xlbomd_selftest_logdet.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                             _dp, _dp]
        L.xlbomd_gemm_presplit_noalloc.argtypes = [ctypes.c_int32, ctypes.c_int32, vp, vp,
                                                   vp, vp]
        L.xlbomd_destroy.argtypes = [vp]
        L.xlbomd_destroy.restype = None
        L.xlbomd_last_error.restype = ctypes.c_char_p
        L.xlbomd_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


EXPORTED = ("xlbomd_init_system", "xlbomd_step", "xlbomd_step_batch",
            "xlbomd_set_step_mode", "xlbomd_set_plan_margin", "xlbomd_step_stats",
            "xlbomd_step_begin", "xlbomd_step_end",
            "xlbomd_kernel_update",
            "xlbomd_forces", "xlbomd_get_charges", "xlbomd_set_state",
            "xlbomd_get_state", "xlbomd_state_size", "xlbomd_save_state",
            "xlbomd_load_state", "xlbomd_solve", "xlbomd_response",
            "xlbomd_kernel_apply", "xlbomd_scf", "xlbomd_profile", "xlbomd_selftest_gemm",
            "xlbomd_selftest_gemm_time", "xlbomd_selftest_gemm_presplit",
            "xlbomd_selftest_logdet", "xlbomd_gemm_presplit_noalloc",
            "xlbomd_destroy", "xlbomd_last_error",
            "xlbomd_version")


def _check(rc):
    if rc != 0:
        raise XlbomdError(rc, lib().xlbomd_last_error().decode())


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def _c(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def selftest_gemm(A, B, precision=FP64, sym=False):
    """C = A B through the library's MFMA product kernel (test hook)."""
    A, B = _c(A), _c(B)
    n = A.shape[0]
    C = np.zeros((n, n))
    _check(lib().xlbomd_selftest_gemm(n, precision, 1 if sym else 0,
                                      _ptr(A), _ptr(B), _ptr(C)))
    return C


def selftest_gemm_time(n, precision=FP64, sym=False, dual=False, reps=10):
    """Milliseconds per launch of the product kernel (benchmark hook)."""
    out = np.zeros(1)
    _check(lib().xlbomd_selftest_gemm_time(n, precision, int(sym), int(dual),
                                           reps, _ptr(out)))
    return float(out[0])


def selftest_gemm_presplit(A, B, sym=False, reps=0, hi_only=False):
    """C = A B^T with the split product on pre-split operands (test hook;
    hi_only: the plain bf16 product of the hi planes).  Returns C, or
    (C, ms per launch) when reps > 0."""
    A = _c(A); B = _c(B)
    n = A.shape[0]
    C = np.zeros((n, n))
    ms = np.zeros(1)
    flags = (1 if sym else 0) | (2 if hi_only else 0)
    _check(lib().xlbomd_selftest_gemm_presplit(n, flags, reps, _ptr(A), _ptr(B),
                                               _ptr(C), _ptr(ms)))
    return (C, float(ms[0])) if reps > 0 else C


def selftest_logdet(A, nb=1, shift=0.0):
    """ln det(A + b shift I) for b < nb, factorised as one batch by the
    library's blocked FP64 Cholesky (test hook)."""
    A = _c(A)
    out = np.zeros(nb)
    _check(lib().xlbomd_selftest_logdet(A.shape[0], int(nb), float(shift), _ptr(A), _ptr(out)))
    return out


def gemm_presplit_noalloc(n, sym, A_ptr, B_ptr, C_ptr, stream=None):
    """C = A B^T on pre-split device operands (device addresses of two bf16
    planes each), enqueued on `stream` without allocating."""
    _check(lib().xlbomd_gemm_presplit_noalloc(int(n), 1 if sym else 0, A_ptr, B_ptr, C_ptr,
                                              stream))


def step_batch(systems, n_steps=1):
    """Step several XLBOMD handles concurrently (native threads, one stream
    each).  Returns (reports, statuses)."""
    k = len(systems)
    arr = (ctypes.c_void_p * k)(*[s._h.value for s in systems])
    reps = (Report * k)()
    st = (ctypes.c_int32 * k)()
    rc = lib().xlbomd_step_batch(arr, k, n_steps, reps, st)
    return [r.as_dict() for r in reps], list(st), rc


class XLBOMD:
    """One system living on the GPU (a library handle)."""

    def __init__(self, system, precision=FP64, scf_tol=None, scf_max_iter=300,
                 energy_every=0, stream=None, allocator=None, foe_levels=0,
                 foe_tol=0.0, mu_tol=0.0, **override):
        """allocator: None (hipMalloc), "torch" (a TorchAllocator on the
        current device) or an object with a ctypes `struct` (Allocator);
        it is kept alive with the handle.  foe_levels: 0 chooses the level
        count from the truncation target, 1..40 requests one.  foe_tol and
        mu_tol override the truncation target and the chemical-potential
        rerun threshold (0 = the precision's defaults)."""
        s = system.replace(**override) if override else system
        self.nat, self.no = int(s.n_atoms), int(s.n_orb)
        self.kmax = int(s.kmax)
        keep = dict(pos=_c(s.pos), vel=_c(s.vel), mass=_c(s.mass),
                    onsite=_c(s.onsite), jit=_c(s.onsite_jitter),
                    hop=_c(s.hop_block), u=_c(s.hubbard_u))
        d = Desc()
        d.n_atoms, d.n_orb = self.nat, self.no
        d.pos, d.vel, d.mass = _ptr(keep["pos"]), _ptr(keep["vel"]), _ptr(keep["mass"])
        d.onsite, d.onsite_jitter = _ptr(keep["onsite"]), _ptr(keep["jit"])
        d.hop_block, d.hubbard_u = _ptr(keep["hop"]), _ptr(keep["u"])
        d.hop_decay, d.hop_cutoff = s.hop_decay, s.hop_cutoff
        d.taper_width, d.gamma_soft = s.taper_width, s.gamma_soft
        d.rep_a, d.rep_decay = s.rep_a, s.rep_decay
        d.n_electrons, d.te, d.dt = s.n_electrons, s.te, s.dt
        d.kmax, d.kernel_rank = s.kmax, s.rank
        d.kernel_every, d.krylov_mode = s.kernel_every, s.krylov_mode
        d.k0_gamma, d.precision = s.k0_gamma, precision
        d.scf_tol = scf_tol if scf_tol is not None else (
            1e-6 if precision == FP32 else 1e-10)
        d.scf_max_iter, d.energy_every = scf_max_iter, energy_every
        d.stream = stream
        d.foe_levels = foe_levels
        d.foe_tol, d.mu_tol = float(foe_tol), float(mu_tol)
        d.kernel_otf = int(getattr(s, "kernel_otf", 0))
        ob = getattr(s, "overlap_block", None)
        if ob is not None:                  # non-orthogonal basis
            keep["ov"] = _c(ob)
            d.overlap_block = _ptr(keep["ov"])
            d.overlap_decay = float(s.overlap_decay)
        if allocator == "torch":
            allocator = TorchAllocator()
        self.allocator = allocator
        if allocator is not None:
            d.allocator = ctypes.pointer(allocator.struct)
        self._h = ctypes.c_void_p()
        _check(lib().xlbomd_init_system(ctypes.byref(d), ctypes.byref(self._h)))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().xlbomd_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1, report=True):
        rep = Report()
        _check(lib().xlbomd_step(self._h, n, ctypes.byref(rep) if report else None))
        return rep.as_dict() if report else None

    def set_step_mode(self, mode):
        """0: host decisions; 1: planned steps (decisions on the device);
        2: planned steps replayed from a captured HIP graph."""
        _check(lib().xlbomd_set_step_mode(self._h, int(mode)))

    def step_begin(self):
        """Enqueue one planned step and return at once."""
        _check(lib().xlbomd_step_begin(self._h))

    def step_end(self, wait=True, report=False):
        """Finish the begun step: False while the device is still busy
        (wait=False), else True (with the report dict when asked)."""
        done = ctypes.c_int32(0)
        rep = Report()
        _check(lib().xlbomd_step_end(self._h, 1 if wait else 0, ctypes.byref(done),
                                     ctypes.byref(rep) if report else None))
        if not done.value:
            return False
        return rep.as_dict() if report else True

    def set_plan_margin(self, margin):
        """Headroom of a plan's interval (0.25 by default; below 0 every
        planned step leaves its plan)."""
        _check(lib().xlbomd_set_plan_margin(self._h, float(margin)))

    def step_stats(self):
        out = (ctypes.c_int64 * 4)()
        _check(lib().xlbomd_step_stats(self._h, out))
        return dict(planned=out[0], replays=out[1], captures=out[2], fallbacks=out[3])

    def kernel_update(self, rank=0):
        _check(lib().xlbomd_kernel_update(self._h, rank))

    def forces(self, energy=True):
        F = np.zeros((self.nat, 3))
        rep = Report()
        _check(lib().xlbomd_forces(self._h, _ptr(F),
                                   ctypes.byref(rep) if energy else None))
        return F, (rep.as_dict() if energy else None)

    def charges(self):
        n, q = np.zeros(self.nat), np.zeros(self.nat)
        _check(lib().xlbomd_get_charges(self._h, _ptr(n), _ptr(q)))
        return n, q

    def set_state(self, pos=None, vel=None, n_hist=None, kr=None):
        a = [_c(pos, (self.nat, 3)), _c(vel, (self.nat, 3)),
             _c(n_hist, (self.kmax + 1, self.nat)), _c(kr, (self.nat,))]
        _check(lib().xlbomd_set_state(self._h, *[_ptr(x) for x in a]))

    def get_state(self):
        pos, vel = np.zeros((self.nat, 3)), np.zeros((self.nat, 3))
        hist, kr = np.zeros((self.kmax + 1, self.nat)), np.zeros(self.nat)
        _check(lib().xlbomd_get_state(self._h, _ptr(pos), _ptr(vel),
                                      _ptr(hist), _ptr(kr)))
        return dict(pos=pos, vel=vel, n_hist=hist, kr=kr)

    def save_state(self) -> bytes:
        """Checkpoint of everything the next step reads (opaque bytes)."""
        size = ctypes.c_size_t(0)
        _check(lib().xlbomd_state_size(self._h, ctypes.byref(size)))
        buf = ctypes.create_string_buffer(size.value)
        _check(lib().xlbomd_save_state(self._h, buf, size.value))
        return buf.raw

    def load_state(self, blob: bytes):
        """Restore a checkpoint from save_state of a handle with the same
        descriptor; the next steps repeat the saved run bit for bit."""
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        _check(lib().xlbomd_load_state(self._h, buf, len(blob)))

    def solve(self, n):
        n = _c(n, (self.nat,))
        q = np.zeros(self.nat)
        rep = Report()
        _check(lib().xlbomd_solve(self._h, _ptr(n), _ptr(q), ctypes.byref(rep)))
        return q, rep.as_dict()

    def response(self, V):
        V = _c(np.atleast_2d(V))
        out = np.zeros_like(V)
        _check(lib().xlbomd_response(self._h, V.shape[0], _ptr(V), _ptr(out)))
        return out

    def profile_start(self):
        _check(lib().xlbomd_profile(self._h, 1, None))

    def profile_stop(self):
        """GEMM timing since profile_start: {'f64': {...}, 'f32': {...},
        'bf3': {...}, 'bf16': {...}} (split bf16x3 products in 'bf3', plain
        bf16 products in 'bf16')."""
        out = np.zeros(20)
        _check(lib().xlbomd_profile(self._h, 0, _ptr(out)))
        res = {}
        for key, o in (("f64", out[:5]), ("f32", out[5:10]), ("bf3", out[10:15]),
                       ("bf16", out[15:])):
            res[key] = dict(ms=o[0], flops=o[1], launches=int(o[2]),
                            min_ms=o[3], max_ms=o[4])
        return res

    def scf(self, n0=None, rank=1, gamma=0.0, tol=1e-10, max_iter=100):
        """Kernel SCF (Eq. 52) at the current positions.  Returns
        (n, rms history, converged); a diverged iteration raises XlbomdError
        (code -4) carrying the history so far as `rms_hist`."""
        n0 = None if n0 is None else _c(n0, (self.nat,))
        n = np.zeros(self.nat)
        hist = np.zeros(max_iter + 1)
        ne = ctypes.c_int32(0)
        rc = lib().xlbomd_scf(self._h, _ptr(n0), rank, gamma, tol, max_iter, _ptr(n),
                              _ptr(hist), ctypes.byref(ne))
        done = hist[:ne.value].copy()
        if rc not in (0, -3):
            try:
                _check(rc)
            except XlbomdError as e:
                e.rms_hist = done     # the evaluations before the failure
                raise
        return n, done, rc == 0

    def kernel_apply(self, rank, r):
        r = _c(r, (self.nat,))
        out = np.zeros(self.nat)
        _check(lib().xlbomd_kernel_apply(self._h, rank, _ptr(r), _ptr(out)))
        return out
