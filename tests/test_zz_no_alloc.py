"""The allocation-free split product (xlbomd_gemm_presplit_noalloc) against
the allocating entry point it varies (xlbomd_selftest_gemm_presplit), on two
calls in a row, the second with a smaller input, through the C ABI.

The operands are split on the device the way the library splits them
(FP32, then bf16 hi by round-to-nearest-even and lo = bf16 of the
remainder); both entry points then run the same kernels on the same tile
schedule, so the results agree bit for bit, which the test asserts, with the
product's own accuracy bound (~2^-16 relative per operand) as the stated
tolerance for the comparison to numpy."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1705_10845_amd as P
    P.lib()
    return P


def _split_planes(torch, x):
    """(hi, lo) bf16 planes of an FP64 host array, as one int16 device tensor."""
    x32 = torch.from_numpy(x).to("cuda").float()
    hi = x32.to(torch.bfloat16)
    lo = (x32 - hi.float()).to(torch.bfloat16)
    return torch.cat([hi.reshape(-1).view(torch.int16), lo.reshape(-1).view(torch.int16)])


def _value(torch, planes, n):
    hi = planes[: n * n].view(torch.bfloat16).double()
    lo = planes[n * n:].view(torch.bfloat16).double()
    return (hi + lo).reshape(n, n).cpu().numpy()


def test_noalloc_split_product_matches_the_allocating_one(P):
    import torch
    from paper_1705_10845_amd import binding as B
    rng = np.random.default_rng(17)
    stream = torch.cuda.current_stream()
    for n, sym in ((1024, False), (1024, True), (384, False), (256, True)):
        A = rng.uniform(-1.0, 1.0, (n, n))
        Bm = A if sym else rng.uniform(-1.0, 1.0, (n, n))    # A A^T is symmetric
        ref = B.selftest_gemm_presplit(A, Bm, sym=sym)
        a, b = _split_planes(torch, A), _split_planes(torch, Bm)
        c = torch.full((2 * n * n,), 0x7fc0, dtype=torch.int16, device="cuda")   # NaN bits
        torch.cuda.synchronize()
        B.gemm_presplit_noalloc(n, sym, a.data_ptr(), b.data_ptr(), c.data_ptr(),
                                ctypes.c_void_p(stream.cuda_stream))
        torch.cuda.synchronize()
        got = _value(torch, c, n)
        exact = A @ Bm.T
        diff = np.abs(got - ref).max()
        err = np.abs(got - exact).max() / np.abs(exact).max()
        print(f"n={n} sym={sym}: vs allocating entry point {diff:.1e}, vs FP64 {err:.1e}")
        assert diff == 0.0
        assert err < 1e-4


def test_noalloc_rejects_sizes_beyond_the_scratch(P):
    import torch
    from paper_1705_10845_amd import binding as B
    n = 2688       # its split-k tail needs more than the 32 MiB array
    bufs = [torch.zeros(2 * n * n, dtype=torch.int16, device="cuda") for _ in range(3)]
    with pytest.raises(B.XlbomdError) as e:
        B.gemm_presplit_noalloc(n, False, *[t.data_ptr() for t in bufs])
    assert e.value.code == -1 and "scratch" in str(e.value)
    with pytest.raises(B.XlbomdError):
        B.gemm_presplit_noalloc(100, False, *[t.data_ptr() for t in bufs])
    torch.cuda.synchronize()
