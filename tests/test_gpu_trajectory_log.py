"""The trajectory log through the library: the c1 cluster (N = 64, FP64)
for 6 steps logged every 2, energy every 2, against the same handle's
direct reports."""
import json

import numpy as np
import pytest

from synth import make_system

pytestmark = pytest.mark.gpu


def test_trajectory_log_on_the_gpu(tmp_path):
    import paper_1705_10845_amd as P
    from paper_1705_10845_amd import trajectory
    s = make_system("c1")
    path = str(tmp_path / "c1.jsonl")
    g = P.XLBOMD(s, precision=P.FP64, scf_tol=1e-10, energy_every=2)
    recs = trajectory.run(g, steps=6, every=2, log=path)
    n_log = g.charges()[0]
    g.close()
    lines = [json.loads(x) for x in open(path)]
    print(lines[-1])
    assert lines == recs
    assert [r["step"] for r in lines] == [2, 4, 6]
    assert all(r["e_total"] is not None and np.isfinite(r["e_total"]) for r in lines)
    assert all(np.isfinite(r["rms_res"]) and r["rms_res"] >= 0.0 for r in lines)
    # the same trajectory stepped directly
    h = P.XLBOMD(s, precision=P.FP64, scf_tol=1e-10, energy_every=2)
    for _ in range(3):
        rep = h.step(2)
    n_direct = h.charges()[0]
    h.close()
    assert rep["e_total"] == lines[-1]["e_total"]
    assert np.array_equal(n_log, n_direct)


@pytest.mark.parametrize("mode", [0, 2])
def test_recovery_after_forced_divergence(mode):
    """Failure detection and recovery, forced from the host: the older rows
    of the charge history are set to values of order 1e3 (set_state; the
    current row, which set_state solves at and takes the forces from, is
    left as it was).  The next step's Verlet update of n then drives the
    residual past the library's divergence bound (RMS > 1e3), which it
    reports before that step's forces move the nuclei.  `recover`
    re-converges the electrons at the current positions and refills the
    history.  The trajectory then goes on next to an undisturbed one (the
    recovered step lacks its second half-kick).  In step mode 2 (planned
    steps replayed from graphs) the runaway step leaves its plan and is
    retaken with host decisions, which report it the same way.  Every
    kernel runs in bounds and every loop is bounded; only the values are
    extreme."""
    import paper_1705_10845_amd as P
    from paper_1705_10845_amd import trajectory
    from synth import lattice_system
    s = lattice_system(40, "c2", seed=3)
    ref = P.XLBOMD(s, precision=P.FP64, scf_tol=1e-10, energy_every=1)
    ref_recs = trajectory.run(ref, steps=9)
    pos_ref = ref.get_state()["pos"]
    ref.close()
    g = P.XLBOMD(s, precision=P.FP64, scf_tol=1e-10, energy_every=1)
    g.set_step_mode(mode)
    g.step(3)
    st = g.get_state()
    bad = st["n_hist"].copy()
    bad[1:] += 2e3 * np.random.default_rng(4).standard_normal(bad[1:].shape)
    g.set_state(n_hist=bad)
    recs = trajectory.run(g, steps=6, every=1, recover_on_divergence=True)
    pos = g.get_state()["pos"]
    g.close()
    for r in recs:
        print({k: r.get(k) for k in ("event", "step", "rms_res", "e_total", "n_rms")})
    assert recs[0].get("event") == "recovered" and recs[0]["n_rms"] > 0.0
    rest = recs[1:]
    assert len(rest) == 5 and all("event" not in r for r in rest)
    assert max(r["rms_res"] for r in rest) < 1e-2
    dpos = np.abs(pos - pos_ref).max()
    de = abs(rest[-1]["e_total"] - ref_recs[-1]["e_total"])
    print(f"after recovery: max|dR| {dpos:.2e} against the undisturbed run, "
          f"|dE_tot| {de:.2e}")
    assert dpos < 5e-2 and de < 5e-2
