"""Serving with continuous batching: every request's result is bit-identical
whether it runs alone or in the mix, admission respects the memory budget
and the slot count, and requests share the device (more than one in the
batch at a time)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2202_11890_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2202_11890_amd import mprk, serving  # noqa: E402
from tests.test_parity_gpu import problem_of, state_err  # noqa: E402

DEV = torch.device("cuda:0")


def requests(flux_bits=64):
    rng = np.random.default_rng(5)
    out = []
    for i in range(9):
        nx = int(rng.integers(24, 97))
        nz = max(8, nx // 2)
        w = inputs.small().with_(nx=nx, nz_lower=nz, nz_upper=nz, m=int(rng.choice([2, 4])),
                                 seed=300 + i)
        ql, qu = inputs.initial_state(w)
        arrival = 0.0 if i < 6 else 0.02 * (i - 5)
        out.append(serving.Request(i, mprk.config_of_workload(w, flux_bits=flux_bits), ql, qu,
                                   int(rng.integers(5, 30)), arrival))
    return out


@pytest.mark.parametrize("flux_bits", [64, 32])
def test_served_results_equal_alone(flux_bits):
    reqs = requests(flux_bits)
    budget = 3 * max(serving.footprint(r.cfg) for r in reqs)
    srv = serving.Server(DEV, budget, max_slots=4, chunk=7)
    held = []
    real_rebuild = srv._rebuild

    def rebuild():
        # Device bytes really held right after each rebuild: the admitted
        # requests' states plus the new batch's workspace tensor.
        real_rebuild()
        states = sum(a.ql.numel() * 8 + a.qu.numel() * 8 for a in srv.active)
        states += sum(o[0].ql.numel() * 8 + o[0].qu.numel() * 8 for o in srv.outgoing)
        ws = srv.batch.workspace.numel() if srv.batch is not None else 0
        assert ws == srv.ws_bytes
        held.append(states + ws)

    srv._rebuild = rebuild
    res = {r.rid: r for r in srv.run(reqs)}
    assert held and max(held) <= budget
    assert sorted(res) == [r.rid for r in reqs]
    assert max(n for _, n, _ in srv.log) >= 2          # requests shared the device
    assert max(u for _, _, u in srv.log) <= budget
    assert srv.rebuilds > 2
    for r in reqs:
        alone = serving.Server(DEV, budget, max_slots=1, chunk=1000).run([r])[0]
        got = res[r.rid]
        assert got.status == 0 and got.steps == r.steps and got.dt == alone.dt
        assert np.array_equal(got.q_lower, alone.q_lower) and np.array_equal(got.q_upper, alone.q_upper)


def test_served_request_matches_oracle():
    r = requests()[2]
    res = serving.Server(DEV, 1 << 30, chunk=4).run([r])[0]
    w = r.cfg
    pb = oracle.Problem(w.nx, w.nz_lower, w.nz_upper, w.dx, w.dz_lower, w.dz_upper,
                        n_buffer=w.n_buffer, mu_lower=w.mu_lower, mu_upper=w.mu_upper)
    assert res.dt == pytest.approx(oracle.dt_rule(pb, r.q_lower, r.q_upper, w.m), rel=1e-13)
    ol, ou = r.q_lower.copy(), r.q_upper.copy()
    oracle.mprk_run(pb, w.base_rk, w.m, res.dt, r.steps, ol, ou)
    assert np.all(state_err(res.q_lower, ol) <= 1e-12) and np.all(state_err(res.q_upper, ou) <= 1e-12)
