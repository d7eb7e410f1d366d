"""Host logic of the continuous-batching server, on the CPU: the batch is
replaced by a stand-in that advances each member's state by a known amount,
so admission order, the memory budget, the slot limit, chunking to the exact
step count, the step rule of new requests and early retirement of a bad
member can be checked without a GPU."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2202_11890_amd import inputs, mprk

torch = pytest.importorskip("torch")

from paper_2202_11890_amd import serving  # noqa: E402

BAD = 1000.0      # a member whose density passes this reports a bad state


class FakeBatch:
    """Stands in for mprk.Batch: each step adds dt to the lower state and
    subtracts it from the upper one."""

    made = []

    def __init__(self, members, stream=None, exec_mode=None, tile=None):
        self.members = [list(m) for m in members]
        self.closed = False
        FakeBatch.made.append(self)

    @staticmethod
    def rule(cfg):
        return 2.0 ** -4 * (1 + cfg.nx % 3)

    def stable_dts(self, cr=0.5, dn=0.25):
        return [self.rule(m[0]) for m in self.members]

    def set_dt(self, i, dt):
        self.members[i][3] = dt

    def run_status(self, k):
        assert not self.closed and k >= 1
        stats, bad_any = [], False
        for cfg, ql, qu, dt in self.members:
            for _ in range(k):
                ql += dt
                qu -= dt
            bad = int(float(ql[0, 0, 0]) > BAD)
            bad_any = bad_any or bool(bad)
            stats.append({"status": bad})
        return (mprk.ENONFINITE if bad_any else mprk.OK), stats

    def close(self):
        self.closed = True


def make_requests():
    out = []
    for i, (nx, steps, dt) in enumerate([(16, 7, None), (20, 12, 0.125), (24, 3, None), (16, 25, None),
                                         (28, 9, 0.25), (20, 1, None)]):
        w = inputs.small().with_(nx=nx, nz_lower=8, nz_upper=8, seed=500 + i)
        ql, qu = inputs.initial_state(w)
        if i == 3:
            ql = ql + (BAD - 1.0)          # crosses BAD after a few steps
        out.append(serving.Request(i, mprk.config_of_workload(w), ql, qu, steps, 0.0, dt))
    return out


@pytest.fixture
def fake(monkeypatch):
    FakeBatch.made = []
    monkeypatch.setattr(serving.mprk, "Batch", FakeBatch)
    return FakeBatch


def test_schedule_budget_slots_and_exact_steps(fake):
    reqs = make_requests()
    init = {r.rid: (r.q_lower.copy(), r.q_upper.copy()) for r in reqs}
    fp = max(serving.footprint(r.cfg) for r in reqs)
    budget = 3 * fp
    srv = serving.Server("cpu", budget, max_slots=2, chunk=4)
    res = {r.rid: r for r in srv.run(reqs)}
    assert sorted(res) == [r.rid for r in reqs]
    assert max(n for _, n, _ in srv.log) <= 2
    assert max(u for _, _, u in srv.log) <= budget
    assert all(b.closed for b in fake.made)
    order = sorted(res.values(), key=lambda x: x.admitted)
    assert [x.rid for x in order] == sorted(res)            # admitted in arrival (id) order
    for r in reqs:
        got = res[r.rid]
        want_dt = r.dt if r.dt is not None else FakeBatch.rule(r.cfg)
        assert got.dt == want_dt
        if r.rid == 3:
            continue
        assert got.status == 0 and got.steps == r.steps
        l0, u0 = init[r.rid]
        for _ in range(r.steps):          # the stand-in's arithmetic, step by step
            l0 = l0 + want_dt
            u0 = u0 - want_dt
        assert np.array_equal(got.q_lower, l0) and np.array_equal(got.q_upper, u0)


def test_bad_member_leaves_early_and_others_finish(fake):
    reqs = make_requests()
    srv = serving.Server("cpu", 1 << 40, max_slots=8, chunk=2)
    res = {r.rid: r for r in srv.run(reqs)}
    bad = res[3]
    assert bad.status == 1 and bad.steps < reqs[3].steps
    assert all(res[i].status == 0 and res[i].steps == reqs[i].steps for i in res if i != 3)


def test_chunks_end_exactly_at_each_step_count(fake):
    reqs = [r for r in make_requests() if r.rid != 3]
    srv = serving.Server("cpu", 1 << 40, max_slots=8, chunk=5)
    res = srv.run(reqs)
    assert sorted(x.steps for x in res) == sorted(r.steps for r in reqs)
    # steps 7, 12, 3, 9, 1 in chunks of at most 5, each chunk ending where the
    # next request finishes: chunks of 1, 2, 4, 2, 3 steps, one request leaving
    # after each; one batch for the first admission and one after each of the
    # first four departures
    assert len(srv.log) == 5 and [n for _, n, _ in srv.log] == [4, 3, 2, 1, 0]
    assert srv.rebuilds == 5 == len(fake.made)


def test_admission_charges_the_whole_batch_workspace(fake):
    """A batch's workspace grows with its largest m*s times its member count,
    so a mix of members with different m needs more than the sum of their
    one-member footprints; admission charges the workspace of the batch it
    would create.  With a budget of exactly the summed footprints of a mix,
    the whole mix is not admitted at once, and after every chunk the states
    plus the batch workspace stay within the budget."""
    reqs = []
    for i, m in enumerate([2, 8, 2, 8, 2, 8]):
        w = inputs.small().with_(nx=256, nz_lower=64, nz_upper=64, m=m, seed=700 + i)
        ql, qu = inputs.initial_state(w)
        reqs.append(serving.Request(i, mprk.config_of_workload(w), ql, qu, 3, 0.0, 0.01))
    summed = sum(serving.footprint(r.cfg) for r in reqs)
    whole = sum(serving.state_bytes(r.cfg) for r in reqs) + serving.batch_bytes([r.cfg for r in reqs])
    assert whole > summed                       # the overshoot a per-member charge would allow
    srv = serving.Server("cpu", summed, max_slots=16, chunk=3)
    res = srv.run(reqs)
    assert len(res) == len(reqs)
    assert max(n for _, n, _ in srv.log) < len(reqs)
    assert max(u for _, _, u in srv.log) <= summed
