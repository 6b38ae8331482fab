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
