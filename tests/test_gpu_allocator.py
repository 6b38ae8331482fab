"""Device memory from a caller-supplied allocator (xlbomd_allocator), here
PyTorch's caching allocator, against the library's own hipMalloc."""
import numpy as np
import pytest

from synth import make_system

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1705_10845_amd as P
    P.lib()
    return P


def test_torch_allocator_matches_hipmalloc(P):
    """Ten steps of the 64-atom cluster with memory from torch: the same
    trajectory as with hipMalloc, the buffers held as torch tensors while the
    handle lives (including the energy workspace allocated on demand), and
    every one given back at close."""
    import torch
    s = make_system("c1")
    runs = {}
    for alloc in (None, "torch"):
        g = P.XLBOMD(s, precision=P.FP64, scf_tol=1e-10, energy_every=5, allocator=alloc)
        rep = g.step(10)
        n, q = g.charges()
        F, e = g.forces()
        a = g.allocator
        held = a.bytes_held if a is not None else 0
        torch_mem = torch.cuda.memory_allocated()
        g.close()
        runs[alloc] = dict(n=n, q=q, F=F, E=rep["e_total"], held=held, a=a, tm=torch_mem)
    r0, r1 = runs[None], runs["torch"]
    print(f"torch allocator held {r1['held'] / 1e6:.1f} MB in {len(r1['a'].live)} live tensors "
          f"after close; dq {np.abs(r0['q'] - r1['q']).max():.1e}")
    assert r1["held"] > 0 and r1["tm"] >= r1["held"]
    assert len(r1["a"].live) == 0
    assert np.abs(r0["n"] - r1["n"]).max() < 1e-12
    assert np.abs(r0["q"] - r1["q"]).max() < 1e-12
    assert np.abs(r0["F"] - r1["F"]).max() < 1e-10
    assert abs(r0["E"] - r1["E"]) < 1e-10 * abs(r0["E"])


class _Alloc:
    def __init__(self, P, alloc, free):
        self.struct = P.Allocator(alloc, free, None)


def test_allocator_errors(P):
    """An allocator without free is rejected; one that returns no memory
    fails the init with XLBOMD_E_NOMEM."""
    B = P.binding
    s = make_system("c1")
    no_free = _Alloc(P, B._ALLOC_FN(lambda n, c: None), B._FREE_FN())
    with pytest.raises(P.XlbomdError) as e:
        P.XLBOMD(s, precision=P.FP64, allocator=no_free)
    assert e.value.code == -1
    empty = _Alloc(P, B._ALLOC_FN(lambda n, c: None), B._FREE_FN(lambda p, c: None))
    with pytest.raises(P.XlbomdError) as e:
        P.XLBOMD(s, precision=P.FP64, allocator=empty)
    assert e.value.code == -2


def test_torch_allocator_under_batch_stepping(P):
    """Three systems share one TorchAllocator and step together through
    xlbomd_step_batch, evaluating the free energy every other step.  The
    energy workspace, allocated on demand at the first evaluation, comes
    through the Python callback from the library's worker threads.
    The charges equal those of the same systems stepped alone on hipMalloc
    memory, and every buffer is given back when the handles close."""
    import threading
    from synth import lattice_system
    from paper_1705_10845_amd.binding import step_batch

    def systems():
        return [lattice_system(n, "c4", seed=100 + n, rank=r)
                for n, r in ((16, 2), (40, 3), (70, 4))]

    alone = []
    for s in systems():
        g = P.XLBOMD(s, precision=P.MIXED, energy_every=2)
        g.step(5, report=False)
        alone.append(g.charges()[1])
        g.close()

    a = P.TorchAllocator()
    inner = a._fns[0]
    callers = []

    def alloc(n, ctx):
        callers.append(threading.get_ident())
        return inner(n, ctx)

    fn = P.binding._ALLOC_FN(alloc)
    a._fns = (fn, a._fns[1], inner)
    a.struct = P.Allocator(fn, a._fns[1], None)

    gs = [P.XLBOMD(s, precision=P.MIXED, energy_every=2, allocator=a) for s in systems()]
    n_init = len(callers)
    reps, st, rc = step_batch(gs, 5)
    assert rc == 0 and st == [0, 0, 0]
    workers = {t for t in callers[n_init:] if t != threading.get_ident()}
    print(f"{n_init} allocations at init, {len(callers) - n_init} inside the batch "
          f"from {len(workers)} worker threads; {a.bytes_held / 1e6:.1f} MB held")
    assert workers
    for g, q in zip(gs, alone):
        assert np.abs(g.charges()[1] - q).max() <= 1e-12
        g.close()
    assert len(a.live) == 0


def test_grown_buffers_are_returned(P):
    """Block-mode kernels grow the response batch from one direction at
    init to three in the steps.  The smaller batch buffers go back to the
    allocator when the larger ones are taken, not at close.  The trajectory
    equals the one on hipMalloc memory."""
    from synth import lattice_system

    def system():
        return lattice_system(40, "c3", seed=12, rank=3, krylov_mode=1, k0_gamma=0.1)

    g = P.XLBOMD(system(), precision=P.MIXED_BF16X3)
    g.step(5, report=False)
    q0 = g.charges()[1]
    g.close()

    a = P.TorchAllocator()
    inner_free = a._fns[1]
    freed = []

    def free(ptr, ctx):
        freed.append(ptr)
        return inner_free(ptr, ctx)

    fn = P.binding._FREE_FN(free)
    a._fns = (a._fns[0], fn, inner_free)
    a.struct = P.Allocator(a._fns[0], fn, None)
    g = P.XLBOMD(system(), precision=P.MIXED_BF16X3, allocator=a)
    g.step(5, report=False)
    early = len(freed)
    q1 = g.charges()[1]
    g.close()
    print(f"{early} buffers returned before close, {len(freed) - early} at close")
    assert early > 0
    assert len(a.live) == 0
    assert np.abs(q1 - q0).max() <= 1e-12
