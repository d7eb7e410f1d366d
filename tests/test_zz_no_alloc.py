"""The allocation-free diagnostics entry point (mprk_diagnostics_static),
called through the C ABI, against the existing mprk_diagnostics of a context
on the same states: two calls in a row, the second with a smaller input (the
file-scope device scratch keeps the first call's contents), then a 3D state
and a bad state.  Both run the same reduction kernels, so the stats must be
bit-identical."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2202_11890_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2202_11890_amd import mprk  # noqa: E402

DEV = torch.device("cuda:0")
FIELDS = ("totals_lower", "totals_upper", "lambda_lower", "lambda_upper", "courant_lower",
          "courant_upper", "visc_lower", "visc_upper", "status")


def say(*a):
    print(*a, flush=True)


def both(cfg, ql, qu, make_solver):
    """(rc, stats) of the static entry point and of a context's diagnostics."""
    tl = torch.from_numpy(np.ascontiguousarray(ql)).to(DEV)
    tu = torch.from_numpy(np.ascontiguousarray(qu)).to(DEV)
    stream = torch.cuda.current_stream(DEV)
    torch.cuda.synchronize()
    rc_s, st_s = mprk.mprk_diagnostics_static(cfg, tl.data_ptr(), tu.data_ptr(), stream.cuda_stream)
    sol = make_solver(tl, tu)
    rc_c, st_c = mprk.mprk_diagnostics(sol.ctx)
    sol.close()
    return (rc_s, st_s.as_dict()), (rc_c, st_c.as_dict())


def same(a, b):
    for f in FIELDS:
        assert a[f] == b[f], (f, a[f], b[f])
    assert a["steps_done"] == 0


def test_static_diagnostics_equal_context_diagnostics_two_calls():
    w1 = inputs.large()
    w2 = inputs.small().with_(nx=40, nz_lower=20, nz_upper=18)
    cases = [("1024x512 random", w1, inputs.random_state(w1, 21, amp=0.2)),
             ("40x20/18 gaussian", w2, inputs.initial_state(w2))]
    for name, w, (ql, qu) in cases:
        say("static diagnostics:", name)
        cfg = mprk.config_of_workload(w)
        (rc_s, st_s), (rc_c, st_c) = both(cfg, ql, qu, lambda a, b: mprk.Solver(cfg, a, b))
        assert rc_s == mprk.OK and rc_c == mprk.OK
        same(st_s, st_c)
        assert st_s["totals_lower"][0] > 0 and st_s["lambda_upper"] > 0


def test_static_diagnostics_3d_and_bad_state():
    w = inputs.small3d().with_(nx=20, ny=12, nz_lower=9, nz_upper=7)
    ql, qu = inputs.random_state3(w, 4, amp=0.1)
    cfg = mprk.config3_of_workload(w)
    say("static diagnostics: 3D", w.nx, w.ny, w.nz_lower, w.nz_upper)
    (rc_s, st_s), (rc_c, st_c) = both(cfg, ql, qu, lambda a, b: mprk.Solver(cfg, a, b))
    assert rc_s == mprk.OK and rc_c == mprk.OK
    same(st_s, st_c)
    w2 = inputs.small().with_(nx=16, nz_lower=8, nz_upper=8)
    ql, qu = inputs.initial_state(w2)
    qu[0, 3, 5] = np.nan
    cfg2 = mprk.config_of_workload(w2)
    say("static diagnostics: bad state")
    (rc_s, st_s), (rc_c, st_c) = both(cfg2, ql, qu, lambda a, b: mprk.Solver(cfg2, a, b))
    assert rc_s == mprk.ENONFINITE and rc_c == mprk.ENONFINITE
    assert st_s["status"] == 1 and st_c["status"] == 1


def test_static_diagnostics_rejects_bad_arguments():
    w = inputs.small()
    ql, qu = inputs.initial_state(w)
    tl = torch.from_numpy(ql).to(DEV)
    tu = torch.from_numpy(qu).to(DEV)
    bad = mprk.config_of_workload(w)
    bad.m = 0
    rc, _ = mprk.mprk_diagnostics_static(bad, tl.data_ptr(), tu.data_ptr(), None)
    assert rc == mprk.EINVAL
    rc, _ = mprk.mprk_diagnostics_static(mprk.config_of_workload(w), None, tu.data_ptr(), None)
    assert rc == mprk.EINVAL
