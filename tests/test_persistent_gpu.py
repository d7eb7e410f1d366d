"""Persistent (dataflow) execution: bit-identical to one launch per stage, and
parity with the FP64 oracle; the bounded wait reports MPRK_ETIMEOUT instead
of hanging when its limit is forced to zero from the host."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2202_11890_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2202_11890_amd import mprk  # noqa: E402
from tests.test_parity_gpu import problem_of, state_err  # noqa: E402

DEV = torch.device("cuda:0")


def run(w, ql, qu, dt, n, mode, check_every=0):
    tl = torch.from_numpy(np.ascontiguousarray(ql)).to(DEV)
    tu = torch.from_numpy(np.ascontiguousarray(qu)).to(DEV)
    sol = mprk.Solver(mprk.config_of_workload(w), tl, tu, exec_mode=mode)
    st = sol.run(dt, n, check_every)
    torch.cuda.synchronize()
    out = tl.cpu().numpy(), tu.cpu().numpy()
    sol.close()
    return out, st


CASES = [
    ("small", inputs.small(), 20),
    ("sr", inputs.small().with_(m=1), 10),
    ("rk3-m4", inputs.small().with_(base=3, m=4, n_buffer=5), 8),
    ("ragged", inputs.small().with_(nx=50, nz_lower=21, nz_upper=37, m=3, n_buffer=19), 6),
    ("fast-upper-unaligned", inputs.small().with_(nx=45, nz_lower=41, nz_upper=18,
                                                  fast_is_lower=False, t_lower=1.0, t_upper=16.0,
                                                  n_buffer=11), 6),
    ("tiny", inputs.small().with_(nx=5, nz_lower=3, nz_upper=4, n_buffer=1, m=8), 6),
    ("gravity", inputs.small().with_(nx=36, nz_lower=18, nz_upper=22, gravity=-0.05, base=3,
                                     m=2, n_buffer=6), 6),
]


@pytest.mark.parametrize("name,w,n", CASES, ids=[c[0] for c in CASES])
def test_persistent_equals_launch_bitwise(name, w, n):
    print("persistent vs launch", name, flush=True)
    ql, qu = inputs.initial_state(w)
    dt = oracle.dt_rule(problem_of(w), ql, qu, w.m)
    (al, au), sa = run(w, ql, qu, dt, n, mprk.EXEC_LAUNCH)
    (bl, bu), sb = run(w, ql, qu, dt, n, mprk.EXEC_PERSISTENT, check_every=3)
    assert sb["status"] == 0 and sb["steps_done"] == n
    assert np.array_equal(al, bl) and np.array_equal(au, bu)


def test_persistent_large_equals_launch_bitwise():
    w = inputs.large()
    print("persistent vs launch large", flush=True)
    ql, qu = inputs.initial_state(w)
    dt = oracle.dt_rule(problem_of(w), ql, qu, w.m)
    (al, au), _ = run(w, ql, qu, dt, 3, mprk.EXEC_LAUNCH)
    (bl, bu), _ = run(w, ql, qu, dt, 3, mprk.EXEC_PERSISTENT)
    assert np.array_equal(al, bl) and np.array_equal(au, bu)


def test_persistent_matches_oracle():
    w = inputs.small()
    ql, qu = inputs.initial_state(w)
    dt = oracle.dt_rule(problem_of(w), ql, qu, w.m)
    (gl, gu), st = run(w, ql, qu, dt, 100, mprk.EXEC_PERSISTENT, check_every=25)
    ol, ou = ql.copy(), qu.copy()
    oracle.mprk_run(problem_of(w), w.base, w.m, dt, 100, ol, ou)
    assert np.all(state_err(gl, ol) <= 1e-12) and np.all(state_err(gu, ou) <= 1e-12)


def test_persistent_timeout_is_reported_and_recoverable():
    """A zero limit on the launch's run time makes the first wait that is not
    already met abort the run: every workgroup exits and the call returns
    MPRK_ETIMEOUT; a later run with the normal limit is correct again."""
    w = inputs.large()
    ql, qu = inputs.initial_state(w)
    dt = oracle.dt_rule(problem_of(w), ql, qu, w.m)
    tl = torch.from_numpy(ql).to(DEV)
    tu = torch.from_numpy(qu).to(DEV)
    sol = mprk.Solver(mprk.config_of_workload(w), tl, tu, exec_mode=mprk.EXEC_PERSISTENT)
    sol.set_wait_limit(0.0)
    with pytest.raises(mprk.MprkError) as e:
        sol.run(dt, 2)
    assert e.value.code == mprk.ETIMEOUT
    sol.set_wait_limit(10.0)
    tl.copy_(torch.from_numpy(ql))
    tu.copy_(torch.from_numpy(qu))
    sol.run(dt, 2)
    torch.cuda.synchronize()
    got = tl.cpu().numpy(), tu.cpu().numpy()
    sol.close()
    (al, au), _ = run(w, ql, qu, dt, 2, mprk.EXEC_LAUNCH)
    assert np.array_equal(got[0], al) and np.array_equal(got[1], au)
