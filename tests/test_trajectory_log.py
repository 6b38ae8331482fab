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


class _FailingHandle(_FakeHandle):
    """Reports a divergence on the chunk that reaches step `fail_at`; the
    recovery's SCF and history refill are recorded."""

    kmax = 5

    def __init__(self, fail_at):
        super().__init__(energy_every=1)
        self.fail_at = fail_at
        self.calls = []

    def step(self, k):
        if self.n < self.fail_at <= self.n + k:
            from paper_1705_10845_amd.binding import XlbomdError
            self.n += k
            self.fail_at = -1
            raise XlbomdError(-4, "residual above 1e3")
        return super().step(k)

    def scf(self, rank=1, tol=1e-8, max_iter=200):
        self.calls.append("scf")
        return [0.1, -0.1], [1.0, 1e-9], True

    def set_state(self, n_hist=None):
        self.calls.append(("n_hist", len(n_hist)))


def test_recovery_after_a_reported_divergence():
    h = _FailingHandle(fail_at=5)
    recs = trajectory.run(h, steps=8, every=2, recover_on_divergence=True)
    assert [r.get("event") for r in recs] == [None, None, "recovered", None]
    assert recs[2]["after_steps"] == 6 and "residual" in recs[2]["error"]
    assert h.calls == ["scf", ("n_hist", 6)]
    from paper_1705_10845_amd.binding import XlbomdError
    with pytest.raises(XlbomdError):
        trajectory.run(_FailingHandle(fail_at=1), steps=2, every=1)
