"""Host logic of the trajectory log (paper_1705_10845_amd.trajectory) on a
stand-in handle: one JSON line per chunk, the last chunk shortened to the
step count, energy fields null on steps without an energy evaluation."""
import io
import json

import pytest

from paper_1705_10845_amd import trajectory


class _FakeHandle:
    """Steps a counter; an energy report every `energy_every` steps."""

    def __init__(self, energy_every):
        self.n = 0
        self.every = energy_every

    def step(self, k):
        self.n += k
        has = self.every > 0 and self.n % self.every == 0
        rep = dict(step=self.n, rms_res=1e-3, mu=-0.5, d_nelec=0.0, foe_levels=5,
                   ns_iters=12, mu_reruns=0, kernel_rank=4, ms_step=1.0, has_energy=int(has))
        rep.update({k: float(self.n) for k in ("omega", "e_band", "e_coul", "e_rep", "te_s",
                                               "e_kin", "e_total")})
        return rep


def test_lines_per_chunk_and_null_energy():
    buf = io.StringIO()
    recs = trajectory.run(_FakeHandle(energy_every=4), steps=10, every=3, log=buf)
    lines = [json.loads(x) for x in buf.getvalue().splitlines()]
    assert lines == recs
    assert [r["step"] for r in lines] == [3, 6, 9, 10]
    # energy only where the cadence put one (none of 3, 6, 9, 10 is a multiple of 4)
    assert all(r["omega"] is None and r["e_total"] is None for r in lines)
    recs = trajectory.run(_FakeHandle(energy_every=2), steps=4, every=2)
    assert [r["e_total"] for r in recs] == [2.0, 4.0]
    assert all(r["wall_ms_per_step"] >= 0.0 for r in recs)


def test_rejects_bad_arguments():
    with pytest.raises(ValueError):
        trajectory.run(_FakeHandle(1), steps=5, every=0)
    with pytest.raises(ValueError):
        trajectory.run(_FakeHandle(1), steps=-1)
