"""GPU tests of the concurrent paths: native batch stepping and the
continuous-batching server.  Each result must be the same alone and in the
mix (the kernels are deterministic: fixed reduction orders, no atomics)."""
import numpy as np
import pytest

from synth import lattice_system, serving_stream

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1705_10845_amd as P
    P.lib()
    return P


def _systems():
    return [lattice_system(n, "c4", seed=100 + n, rank=r)
            for n, r in ((16, 2), (40, 3), (70, 4))]


def test_batch_equals_alone(P):
    from paper_1705_10845_amd.binding import step_batch
    alone = []
    for s in _systems():
        g = P.XLBOMD(s, precision=P.MIXED)
        g.step(5, report=False)
        alone.append(g.charges()[1])
        g.close()
    gs = [P.XLBOMD(s, precision=P.MIXED) for s in _systems()]
    reps, st, rc = step_batch(gs, 5)
    assert rc == 0 and st == [0, 0, 0]
    for g, q in zip(gs, alone):
        d = np.abs(g.charges()[1] - q).max()
        print("alone vs batch max|dq|", d)
        assert d <= 1e-12
        g.close()


@pytest.mark.parametrize("mode", [2, 0])
def test_server_alone_equals_mix(P, mode):
    """Step mode 2 (planned steps replayed from each system's graph, all
    driven from one host thread) and step mode 0 (host decisions, a worker
    thread per running system): every request's final charges are the same
    served in the mix as served alone, bit for bit."""
    from paper_1705_10845_amd.serve import Server
    stream = serving_stream(6, rate_hz=200.0, seed=7)
    stream = [(t, s.replace(n_atoms=s.n_atoms)) for t, s in stream
              if s.n_atoms <= 160][:4]
    srv = Server(hbm_budget=8 << 30, max_slots=4, steps=8, step_mode=mode)
    mixed_stats, summ = srv.run(stream)
    assert summ["errors"] == 0, [s.error for s in mixed_stats]
    print(summ)
    for (t, s), st in zip(sorted(stream, key=lambda x: x[0]), mixed_stats):
        solo = Server(hbm_budget=8 << 30, max_slots=1, steps=8, step_mode=mode)
        one, _ = solo.run([(0.0, s)])
        d = np.abs(one[0].final["q"] - st.final["q"]).max()
        assert d == 0.0, (s.name, d)
    assert summ["peak_hbm_bytes"] <= summ["hbm_budget"]
    assert all(len(st.step_latency) == 8 for st in mixed_stats)


def test_step_begin_end(P):
    """xlbomd_step_begin / _end: the two halves of a planned step equal
    xlbomd_step; calls out of order are refused."""
    s = lattice_system(30, "c4", seed=5, rank=2)
    out = []
    for split in (False, True):
        g = P.XLBOMD(s, precision=P.MIXED_BF16X3, scf_tol=1e-10)
        g.set_step_mode(2)
        if split:
            with pytest.raises(P.XlbomdError):
                g.step_end()
            for _ in range(5):
                g.step_begin()
                with pytest.raises(P.XlbomdError):
                    g.step(1)
                while not g.step_end(wait=False):
                    pass
        else:
            g.step(5, report=False)
        out.append(g.charges()[1])
        g.close()
    assert np.abs(out[0] - out[1]).max() == 0.0
    g = P.XLBOMD(s, precision=P.MIXED_BF16X3, scf_tol=1e-10)
    with pytest.raises(P.XlbomdError):
        g.step_begin()                      # step mode 0: host decisions
    g.close()
