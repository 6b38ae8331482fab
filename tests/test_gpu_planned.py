"""Planned steps (every decision of a step on the device) and their HIP
graph replay, through the C ABI: replayed steps equal the same planned steps
enqueued directly, bit for bit; planned trajectories follow the oracle's;
a step that leaves its plan is taken again with host decisions; and systems
stepped together from one host thread (graph replays on their own streams)
end as they do alone."""
import numpy as np
import pytest

from synth import make_system, lattice_system
from oracle import reference as R

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1705_10845_amd as P
    P.lib()
    return P


def _snap(g):
    st = g.get_state()
    n, q = g.charges()
    F, _ = g.forces(energy=False)
    return dict(pos=st["pos"], vel=st["vel"], hist=st["n_hist"], kr=st["kr"], q=q, F=F)


CASES = [("c1", "FP64"), ("lat40", "MIXED_BF16X3"), ("lat160", "MIXED_BF16X3")]


def _system(name):
    if name == "c1":
        return make_system("c1")
    n = int(name[3:])
    return lattice_system(n, "c2", seed=7)


@pytest.mark.parametrize("name,prec", CASES)
def test_graph_replay_equals_planned_steps(P, name, prec):
    """12 steps: planned steps enqueued directly (mode 1) against the same
    steps replayed from a captured graph (mode 2; the first step of the plan
    runs directly, the second is captured, the rest replay)."""
    s = _system(name)
    out, stats = [], []
    for mode in (1, 2):
        g = P.XLBOMD(s, precision=getattr(P, prec), scf_tol=1e-10)
        g.set_step_mode(mode)
        rep = g.step(12)
        out.append(_snap(g))
        stats.append((g.step_stats(), rep))
        g.close()
    d = {k: float(np.abs(out[0][k] - out[1][k]).max()) for k in out[0]}
    print(f"{name} {prec}: graph vs direct planned steps", {k: f"{v:.1e}" for k, v in d.items()},
          "stats", stats[1][0], "L", stats[1][1]["foe_levels"])
    assert max(d.values()) == 0.0
    assert stats[0][0]["planned"] == 12 and stats[0][0]["replays"] == 0
    assert stats[1][0]["fallbacks"] == 0 and stats[1][0]["captures"] == 1
    assert stats[1][0]["replays"] == 11


@pytest.mark.parametrize("mode", [1, 2])
def test_planned_trajectory_follows_the_oracle(P, mode):
    """30 steps of the 64-atom cluster in FP64 against the oracle's steps."""
    s = make_system("c1")
    m = R.Model(s)
    st = R.init_state(m, scf_tol=1e-11)
    g = P.XLBOMD(s, precision=P.FP64, scf_tol=1e-11)
    g.set_step_mode(mode)
    worst = dict(dn=0.0, dq=0.0, dF=0.0)
    for i in range(30):
        st = R.md_step(m, st, want_energy=False)
        g.step(1, report=False)
        if (i + 1) % 5 == 0:
            n, q = g.charges()
            F, _ = g.forces(energy=False)
            worst["dn"] = max(worst["dn"], np.abs(n - st.el.n).max())
            worst["dq"] = max(worst["dq"], np.abs(q - st.el.q).max())
            worst["dF"] = max(worst["dF"], np.abs(F - st.force).max())
    F, e = g.forces()
    eo = R.energy_report(m, st)
    dO = abs(e["omega"] - eo["omega"]) / abs(eo["omega"])
    stats = g.step_stats()
    g.close()
    print(f"mode {mode}: 30 planned steps vs oracle", {k: f"{v:.1e}" for k, v in worst.items()},
          f"rel dOmega {dO:.1e}", stats)
    assert worst["dn"] < 1e-8 and worst["dq"] < 1e-8 and worst["dF"] < 1e-5 and dO < 1e-8
    assert stats["planned"] >= 30


def test_energy_steps_between_planned_steps(P):
    """Energy every 3rd step: the energy is evaluated after the planned step
    (host synchronisation) and matches the same run with host decisions."""
    s = lattice_system(40, "c2", seed=9)
    res = []
    for mode in (0, 2):
        g = P.XLBOMD(s, precision=P.FP64, scf_tol=1e-10, energy_every=3)
        g.set_step_mode(mode)
        reps = [g.step(3) for _ in range(4)]
        res.append([r["e_total"] for r in reps])
        if mode == 2:
            stats = g.step_stats()
        g.close()
    d = np.abs(np.array(res[0]) - np.array(res[1])).max()
    print("energies, host decisions vs planned graph steps:", res, f"max diff {d:.1e}", stats)
    assert d < 1e-8 * abs(res[0][0])
    assert stats["fallbacks"] == 0 and stats["replays"] >= 8


@pytest.mark.parametrize("prec", ["FP64", "MIXED_BF16X3"])
def test_step_that_leaves_its_plan_is_taken_with_host_decisions(P, prec):
    """A plan sized for half of the last interval (margin -0.5) makes every
    planned step leave it (the interval check on the device); each step is
    restored from the state saved at its start and taken again with host
    decisions, so the run equals the one with host decisions throughout,
    bit for bit, and then the default margin plans again."""
    s = lattice_system(40, "c2", seed=11)
    out = []
    for mode in (0, 2):
        g = P.XLBOMD(s, precision=getattr(P, prec), scf_tol=1e-10)
        g.set_step_mode(mode)
        if mode:
            g.set_plan_margin(-0.5)
        g.step(6, report=False)
        out.append(_snap(g))
        stats = g.step_stats()
        if mode:
            g.set_plan_margin(0.25)
            g.step(4, report=False)
            after = g.step_stats()
        g.close()
    d = {k: float(np.abs(out[0][k] - out[1][k]).max()) for k in out[0]}
    print(f"{prec} forced departures from the plan:", stats, "then", after,
          {k: f"{v:.1e}" for k, v in d.items()})
    assert stats["fallbacks"] == 6 and stats["planned"] == 6
    assert max(d.values()) == 0.0
    assert after["fallbacks"] == 6 and after["replays"] >= 2


def test_batch_of_graphs_alone_equals_in_the_mix(P):
    """Systems of 24, 40 and 96 atoms, each in step mode 2: stepped together
    by xlbomd_step_batch (one host thread, one stream each) and each alone,
    the same steps give the same states, bit for bit."""
    import ctypes
    import torch
    systems = [lattice_system(n, "c4", seed=30 + n, te=0.05, rank=3) for n in (24, 40, 96)]
    alone = []
    for s in systems:
        g = P.XLBOMD(s, precision=P.MIXED_BF16X3, scf_tol=1e-10)
        g.set_step_mode(2)
        g.step(8, report=False)
        alone.append(_snap(g))
        g.close()
    streams = [torch.cuda.Stream() for _ in systems]
    hs = [P.XLBOMD(s, precision=P.MIXED_BF16X3, scf_tol=1e-10, stream=st.cuda_stream)
          for s, st in zip(systems, streams)]
    for h in hs:
        h.set_step_mode(2)
    from paper_1705_10845_amd import binding as B
    for _ in range(8):
        reps, status, rc = B.step_batch(hs, 1)
        assert rc == 0 and status == [0, 0, 0]
    mixed = [_snap(h) for h in hs]
    stats = [h.step_stats() for h in hs]
    for h in hs:
        h.close()
    for a, b in zip(alone, mixed):
        d = max(float(np.abs(a[k] - b[k]).max()) for k in a)
        assert d == 0.0
    print("batch of graphs:", stats)
    assert all(st["replays"] >= 6 for st in stats)
