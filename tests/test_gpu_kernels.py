"""Kernel-level GPU parity: the MFMA product kernels against numpy (FP64
reference), through the C ABI test hook."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FP64, FP32, SPLIT = 0, 1, 3        # xlbomd_precision values of the hook


@pytest.fixture(scope="module")
def B():
    from paper_1705_10845_amd import binding
    binding.lib()
    return binding


def _bf16_rne(x32):
    """bf16 value (as FP32) of FP32 x, round to nearest even."""
    b = x32.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def split_bf16x3(x):
    """hi, lo bf16 parts of the FP32 rounding of x (lo = bf16(x - hi))."""
    x32 = x.astype(np.float32)
    hi = _bf16_rne(x32)
    lo = _bf16_rne(x32 - hi)
    return hi.astype(np.float64), lo.astype(np.float64)


@pytest.mark.parametrize("n", [128, 256, 384, 1024])
@pytest.mark.parametrize("prec", [FP64, FP32, SPLIT])
@pytest.mark.parametrize("sym", [False, True])
def test_gemm(B, n, prec, sym):
    rng = np.random.default_rng(n + 7 * prec)
    A = rng.standard_normal((n, n)); A = 0.5 * (A + A.T)
    if sym:        # A B symmetric when B is a polynomial in A
        Bm = A @ A + 0.3 * A
    else:
        Bm = rng.standard_normal((n, n))
    scale = np.abs(A).max() * np.abs(Bm).max()
    if prec == FP32:
        A32, B32 = A.astype(np.float32).astype(np.float64), Bm.astype(np.float32).astype(np.float64)
        ref = A32 @ B32
        tol = 2e-5 * np.sqrt(n) * scale
    elif prec == SPLIT:
        ah, al = split_bf16x3(A)
        bh, bl = split_bf16x3(Bm)
        # the split product exactly: hi*hi + hi*lo + lo*hi (lo*lo dropped);
        # what remains is FP32 accumulation
        ref = ah @ bh + ah @ bl + al @ bh
        tol = 2e-6 * np.sqrt(n) * scale
    else:
        ref = A @ Bm
        tol = 1e-13 * n * scale
    C = B.selftest_gemm(A, Bm, precision=prec, sym=sym)
    err = np.abs(C - ref).max()
    print(f"n={n} prec={prec} sym={sym}: max err {err:.2e} (tol {tol:.1e})")
    assert err < tol
    if prec == SPLIT:
        # against the exact product: each operand carries ~2^-16 relative
        # error after the split, and the dropped lo*lo term is ~2^-16 of a
        # product
        exact = np.abs(C - A @ Bm).max()
        print(f"   split vs exact FP64 product: {exact:.2e}")
        assert exact < 3e-5 * np.sqrt(n) * scale
    if sym:
        assert np.array_equal(C, C.T)


def test_split_gemm_dual_kscale_batch(B):
    """The split kernel through the argument set the response uses: two
    products along k, a row scale of B_0, a batch of two and the X epilogue
    term, at a ragged size (N = 160, padded to 256)."""
    import paper_1705_10845_amd as P
    from synth import lattice_system
    s = lattice_system(40, "c2", seed=5)
    from oracle import reference as R
    m = R.Model(s)
    n = 0.05 * np.random.default_rng(8).standard_normal(s.n_atoms)
    n -= n.mean()
    el = R.electronic(m, s.pos, n)
    V = np.random.default_rng(9).standard_normal((2, s.n_atoms))
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    ref = np.stack([R.response(m, el, v) for v in V])
    out = {}
    for prec in (P.MIXED, P.MIXED_BF16X3):
        g = P.XLBOMD(s, precision=prec, scf_tol=1e-9)
        g.solve(n)
        out[prec] = g.response(V)
        g.close()
    e32 = np.abs(out[P.MIXED] - ref).max() / np.abs(ref).max()
    e3 = np.abs(out[P.MIXED_BF16X3] - ref).max() / np.abs(ref).max()
    print(f"response rel err: FP32 products {e32:.2e}, split bf16x3 products {e3:.2e}")
    assert e3 < 1e-3
    assert np.abs(out[P.MIXED_BF16X3].sum(axis=1)).max() < 1e-9


@pytest.mark.parametrize("n", [128, 256, 384, 512, 1024, 2048])
@pytest.mark.parametrize("sym", [False, True])
def test_gemm_presplit(B, n, sym):
    """Split product on pre-split operands: C = A B^T from the bf16 hi/lo
    planes of the FP32 roundings of A and B, stored split itself."""
    rng = np.random.default_rng(3 * n + int(sym))
    A = rng.standard_normal((n, n)); A = 0.5 * (A + A.T)
    Bm = A @ A + 0.3 * A if sym else rng.standard_normal((n, n))
    ah, al = split_bf16x3(A)
    bh, bl = split_bf16x3(Bm)
    ref = ah @ bh.T + ah @ bl.T + al @ bh.T
    scale = np.abs(A).max() * np.abs(Bm).max()
    C = B.selftest_gemm_presplit(A, Bm, sym=sym)
    # FP32 accumulation, then the output's own hi + lo rounding (2^-17 relative)
    tol = 2e-6 * np.sqrt(n) * scale + 2.0 ** -15 * np.abs(ref).max()
    err = np.abs(C - ref).max()
    exact = np.abs(C - A @ Bm.T).max()
    print(f"presplit n={n} sym={sym}: vs emulation {err:.2e} (tol {tol:.1e}), vs exact {exact:.2e}")
    assert err < tol
    assert exact < 3e-5 * np.sqrt(n) * scale
    if sym:
        assert np.array_equal(C, C.T)


@pytest.mark.parametrize("n", [128, 384, 1024, 2048])
@pytest.mark.parametrize("sym", [False, True])
def test_gemm_presplit_bf16(B, n, sym):
    """Plain bf16 product (XLBOMD_MIXED_BF16's responses): C = A_hi B_hi^T
    from the hi planes only, against the same product emulated on the CPU
    (hi planes from the same rounding), and within bf16 accuracy of A B^T."""
    rng = np.random.default_rng(5 * n + int(sym))
    A = rng.standard_normal((n, n)); A = 0.5 * (A + A.T)
    Bm = A @ A + 0.3 * A if sym else rng.standard_normal((n, n))
    ah, _ = split_bf16x3(A)
    bh, _ = split_bf16x3(Bm)
    ref = ah @ bh.T
    if sym:
        # A_hi B_hi^T is symmetric only to bf16 accuracy: the kernel computes
        # the upper block triangle and mirrors it
        ref = np.triu(ref) + np.triu(ref, 1).T
    scale = np.abs(A).max() * np.abs(Bm).max()
    C = B.selftest_gemm_presplit(A, Bm, sym=sym, hi_only=True)
    tol = 2e-6 * np.sqrt(n) * scale + 2.0 ** -15 * np.abs(ref).max()
    err = np.abs(C - ref).max()
    exact = np.abs(C - A @ Bm.T).max()
    print(f"bf16 n={n} sym={sym}: vs emulation {err:.2e} (tol {tol:.1e}), vs exact {exact:.2e}")
    assert err < tol
    assert exact < 2e-2 * np.sqrt(n) * scale
    if sym:
        assert np.array_equal(C, C.T)


@pytest.mark.parametrize("n,nb", [(128, 1), (384, 3), (2048, 40)])
def test_batched_logdet(B, n, nb):
    """ln det(A + b s I), b < nb, from the batched blocked Cholesky of the
    entropy evaluation against numpy's eigenvalues.  The 2048 x 2048 batch
    of 40 has more panel blocks per launch than the GPU holds at once, so
    blocks of a matrix run after that matrix's first block has finished:
    each block must factor the diagonal block from entries no other block
    of the launch has overwritten."""
    rng = np.random.default_rng(n + nb)
    M = rng.standard_normal((n, n)) / np.sqrt(n)
    A = np.eye(n) + 0.2 * (M + M.T)              # spectrum in about [0.4, 1.6]
    w = np.linalg.eigvalsh(A)
    shift = 0.01
    ref = np.array([np.log(w + b * shift).sum() for b in range(nb)])
    ld = B.selftest_logdet(A, nb=nb, shift=shift)
    err = np.abs(ld - ref).max()
    print(f"logdet n={n} nb={nb}: max err {err:.2e} (|ld| up to {np.abs(ref).max():.1f})")
    assert w.min() > 0.05
    assert err < 1e-10 * n
