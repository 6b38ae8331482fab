"""Kernel-level GPU parity: the MFMA product kernel against numpy (FP64
reference), through the C ABI test hook."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_1705_10845_amd import binding
    binding.lib()
    return binding


@pytest.mark.parametrize("n", [128, 256, 384, 1024])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("sym", [False, True])
def test_gemm(B, n, prec, sym):
    rng = np.random.default_rng(n + 7 * prec)
    A = rng.standard_normal((n, n)); A = 0.5 * (A + A.T)
    if sym:        # A B symmetric when B is a polynomial in A
        Bm = A @ A + 0.3 * A
    else:
        Bm = rng.standard_normal((n, n))
    if prec == 1:
        A32, B32 = A.astype(np.float32).astype(np.float64), Bm.astype(np.float32).astype(np.float64)
        ref = A32 @ B32
        tol = 2e-5 * np.sqrt(n) * np.abs(A32).max() * np.abs(B32).max()
    else:
        ref = A @ Bm
        tol = 1e-13 * n * np.abs(A).max() * np.abs(Bm).max()
    C = B.selftest_gemm(A, Bm, precision=prec, sym=sym)
    err = np.abs(C - ref).max()
    print(f"n={n} prec={prec} sym={sym}: max err {err:.2e} (tol {tol:.1e})")
    assert err < tol
    if sym:
        assert np.array_equal(C, C.T)
