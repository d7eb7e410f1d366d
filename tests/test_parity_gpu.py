"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle on
the same seeded inputs.

Tolerances (derived from the arithmetic):
  * states after N steps: per component, max |q_gpu - q_oracle| divided by
    the component's magnitude (max |rho|, max |rho E|; for both momentum
    components the larger momentum magnitude, floored at 1e-3 max(rho) a_max)
    must not exceed 1e-12;
  * a single RHS evaluation: |R_gpu - R_oracle| <= 1e-13 * S_v, with S_v the
    magnitude of the face fluxes divided by the cell size (the RHS is a
    difference of two fluxes of that size, so its rounding error scales with
    it, not with R itself).
"""
from __future__ import annotations

import os

import numpy as np
import pytest

import oracle
from paper_2202_11890_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2202_11890_amd import mprk  # noqa: E402

DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)


def problem_of(w):
    return oracle.Problem(w.nx, w.nz_lower, w.nz_upper, w.dx, w.dz_lower, w.dz_upper,
                          fast_is_lower=w.fast_is_lower, n_buffer=w.n_buffer, gamma=w.gamma,
                          prandtl=w.prandtl, mu_lower=w.mu_lower, mu_upper=w.mu_upper,
                          gravity=w.gravity)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def state_err(got, ref, gamma=1.4):
    """Per-component relative error of a domain state."""
    rho = ref[0]
    p = (gamma - 1) * (ref[3] - 0.5 * (ref[1] ** 2 + ref[2] ** 2) / rho)
    a = np.sqrt(gamma * p / rho).max()
    mom = max(np.abs(ref[1]).max(), np.abs(ref[2]).max(), 1e-3 * rho.max() * a)
    scale = np.array([np.abs(ref[0]).max(), mom, mom, np.abs(ref[3]).max()])
    return np.abs(got - ref).max(axis=(1, 2)) / scale


def rhs_scale(q, dmin, gamma=1.4):
    rho, mx, mz, en = q
    u, w = mx / rho, mz / rho
    p = (gamma - 1) * (en - 0.5 * rho * (u * u + w * w))
    a = np.sqrt(gamma * p / rho)
    s = np.abs(u) + np.abs(w) + a
    f = [np.abs(mx) + np.abs(mz) + s * rho,
         np.abs(mx * u) + np.abs(mx * w) + p + s * np.abs(mx),
         np.abs(mz * u) + np.abs(mz * w) + p + s * np.abs(mz),
         (np.abs(en) + p) * (np.abs(u) + np.abs(w)) + s * np.abs(en)]
    return np.array([x.max() for x in f]) / dmin


def run_gpu(w, ql, qu, dt, n, **over):
    tl, tu = dev(ql), dev(qu)
    sol = mprk.Solver(mprk.config_of_workload(w, **over), tl, tu)
    st = sol.run(dt, n)
    torch.cuda.synchronize()
    out = tl.cpu().numpy(), tu.cpu().numpy()
    sol.close()
    return out, st


def run_oracle(w, ql, qu, dt, n):
    a, b = ql.copy(), qu.copy()
    oracle.mprk_run(problem_of(w), w.base, w.m, dt, n, a, b)
    return a, b


# ---------------------------------------------------------------------------
CASES_RHS = [
    ("small", inputs.small()),
    ("ragged", inputs.small().with_(nx=50, nz_lower=21, nz_upper=13, lz_lower=3.0, lz_upper=2.0)),
    ("fast-upper", inputs.small().with_(nx=45, nz_lower=19, nz_upper=34, fast_is_lower=False,
                                        t_lower=1.0, t_upper=16.0)),
    ("gravity", inputs.small().with_(nx=36, nz_lower=18, nz_upper=22, gravity=-0.05,
                                     mu_lower=3e-3, mu_upper=4e-4)),
    ("tiny", inputs.small().with_(nx=5, nz_lower=3, nz_upper=4, n_buffer=1)),
    # viscous fluxes of the order of the inviscid ones (fine anisotropic grid,
    # large and unequal viscosities): the viscous coefficients per direction
    # and domain at full weight
    ("viscous", inputs.small().with_(nx=30, nz_lower=16, nz_upper=14, lx=1.0, lz_lower=0.8, lz_upper=0.5,
                                     mu_lower=0.05, mu_upper=0.02)),
]


@pytest.mark.parametrize("name,w", CASES_RHS, ids=[c[0] for c in CASES_RHS])
@pytest.mark.parametrize("kind", ["gauss", "random"])
def test_rhs_matches_oracle(name, w, kind):
    say("rhs", name, kind, w.nx, w.nz_lower, w.nz_upper)
    if kind == "gauss":
        ql, qu = inputs.initial_state(w)
    else:
        ql, qu = inputs.random_state(w, 3, amp=0.1)
    rl, ru = oracle.rhs(problem_of(w), ql, qu)
    tl, tu = dev(ql), dev(qu)
    gl, gu = torch.full_like(tl, np.nan), torch.full_like(tu, np.nan)
    sol = mprk.Solver(mprk.config_of_workload(w), tl, tu)
    sol.rhs(tl, tu, gl, gu, mprk.REGION_ALL)
    torch.cuda.synchronize()
    for g, r, q, dz in ((gl, rl, ql, w.dz_lower), (gu, ru, qu, w.dz_upper)):
        g = g.cpu().numpy()
        err = np.abs(g - r).max(axis=(1, 2)) / rhs_scale(q, min(w.dx, dz))
        assert np.all(err <= 1e-13), err
    sol.close()


@pytest.mark.parametrize("fast_lower", [True, False])
def test_rhs_region_masks_write_only_their_rows(fast_lower):
    w = inputs.small().with_(nx=40, nz_lower=17, nz_upper=15, n_buffer=3, fast_is_lower=fast_lower)
    ql, qu = inputs.random_state(w, 5)
    rl, ru = oracle.rhs(problem_of(w), ql, qu)
    tl, tu = dev(ql), dev(qu)
    sol = mprk.Solver(mprk.config_of_workload(w), tl, tu)
    nzs = w.nz_upper if fast_lower else w.nz_lower
    b_rows = set(range(w.n_buffer)) if fast_lower else set(range(nzs - w.n_buffer, nzs))
    for mask in range(1, 8):
        gl, gu = torch.full_like(tl, 7.0), torch.full_like(tu, 7.0)
        sol.rhs(tl, tu, gl, gu, mask)
        torch.cuda.synchronize()
        G = {True: gl.cpu().numpy(), False: gu.cpu().numpy()}
        Rr = {True: rl, False: ru}
        for lower in (True, False):
            is_fast = lower == fast_lower
            nz = w.nz_lower if lower else w.nz_upper
            for k in range(nz):
                if is_fast:
                    want = bool(mask & mprk.REGION_F)
                else:
                    want = bool(mask & (mprk.REGION_B if k in b_rows else mprk.REGION_S))
                row = G[lower][:, k]
                if want:
                    assert np.allclose(row, Rr[lower][:, k], rtol=0, atol=1e-11), (mask, lower, k)
                else:
                    assert np.all(row == 7.0), (mask, lower, k)
    sol.close()


def test_rhs_large_full_size():
    w = inputs.large()
    say("rhs large", w.nx, w.nz_lower)
    ql, qu = inputs.initial_state(w)
    rl, ru = oracle.rhs(problem_of(w), ql, qu)
    tl, tu = dev(ql), dev(qu)
    gl, gu = torch.empty_like(tl), torch.empty_like(tu)
    sol = mprk.Solver(mprk.config_of_workload(w), tl, tu)
    sol.rhs(tl, tu, gl, gu)
    torch.cuda.synchronize()
    for g, r, q, dz in ((gl, rl, ql, w.dz_lower), (gu, ru, qu, w.dz_upper)):
        err = np.abs(g.cpu().numpy() - r).max(axis=(1, 2)) / rhs_scale(q, min(w.dx, dz))
        assert np.all(err <= 1e-13), err
    sol.close()


# ---------------------------------------------------------------------------
CASES_RUN = [
    ("small-100", inputs.small(), 100),
    ("small-sr", inputs.small().with_(m=1), 40),
    ("rk3-m4", inputs.small().with_(base=3, m=4, n_buffer=5), 30),
    ("rk3-m4-nb4", inputs.small().with_(base=3, m=4, n_buffer=4), 30),
    ("ragged-m3", inputs.small().with_(nx=50, nz_lower=21, nz_upper=37, m=3, n_buffer=19), 25),
    ("fast-upper", inputs.small().with_(nx=45, nz_lower=33, nz_upper=18, fast_is_lower=False,
                                        t_lower=1.0, t_upper=16.0, n_buffer=3), 30),
    ("gravity-rk3", inputs.small().with_(nx=36, nz_lower=18, nz_upper=22, gravity=-0.05,
                                         base=3, m=2, n_buffer=6), 30),
    ("tiny-nb1", inputs.small().with_(nx=5, nz_lower=3, nz_upper=4, n_buffer=1, m=8), 20),
    ("viscous-rk3", inputs.small().with_(nx=30, nz_lower=16, nz_upper=14, lx=1.0, lz_lower=0.8, lz_upper=0.5,
                                         mu_lower=0.05, mu_upper=0.02, base=3, m=2, n_buffer=5), 30),
    ("rk3-m8", inputs.small().with_(nx=41, nz_lower=23, nz_upper=19, base=3, m=8, n_buffer=5), 12),
]


@pytest.mark.parametrize("name,w,n", CASES_RUN, ids=[c[0] for c in CASES_RUN])
def test_run_matches_oracle(name, w, n):
    say("run", name, w.nx, w.nz_lower, w.nz_upper, "base", w.base, "m", w.m, "nb", w.n_buffer)
    ql, qu = inputs.initial_state(w)
    dt = oracle.dt_rule(problem_of(w), ql, qu, w.m)
    (gl, gu), st = run_gpu(w, ql, qu, dt, n)
    ol, ou = run_oracle(w, ql, qu, dt, n)
    assert st["status"] == 0 and st["steps_done"] == n
    el, eu = state_err(gl, ol), state_err(gu, ou)
    say("  err lower", el, "upper", eu)
    assert np.all(el <= 1e-12) and np.all(eu <= 1e-12)


def test_large_two_hundred_steps_matches_oracle():
    """The 1024 x 512 workload in the benchmark's launch configuration, 200
    slow steps (a fifth of the benchmark run; the oracle takes about a minute
    on 16 host threads, in chunks of 50 steps, restarts being bitwise),
    compared after 50 and after 200 steps."""
    w = inputs.large()
    say("run large 200 steps")
    ql, qu = inputs.initial_state(w)
    pb = problem_of(w)
    dt = oracle.dt_rule(pb, ql, qu, w.m)
    tl, tu = dev(ql), dev(qu)
    sol = mprk.Solver(mprk.config_of_workload(w), tl, tu)
    ol, ou = ql.copy(), qu.copy()
    done = 0
    for upto in (50, 200):
        st = sol.run(dt, upto - done, check_every=10)
        torch.cuda.synchronize()
        assert st["status"] == 0 and st["steps_done"] == upto
        gl, gu = tl.cpu().numpy(), tu.cpu().numpy()
        while done < upto:
            oracle.mprk_run(pb, w.base, w.m, dt, 50, ol, ou)
            done += 50
            say("  oracle", done, "steps")
        el, eu = state_err(gl, ol), state_err(gu, ou)
        say("  after", upto, "steps: err lower", el, "upper", eu)
        assert np.all(el <= 1e-12) and np.all(eu <= 1e-12)
    sol.close()


@pytest.mark.skipif(not os.environ.get("MPRK_LONG_PARITY"),
                    reason="about five minutes of oracle time; set MPRK_LONG_PARITY=1 to run")
def test_large_thousand_steps_matches_oracle():
    """The whole 1024 x 512 benchmark run (1000 slow steps) against the oracle,
    which runs in chunks of 50 steps (restarts are bitwise) and reports its
    progress."""
    w = inputs.large()
    ql, qu = inputs.initial_state(w)
    dt = oracle.dt_rule(problem_of(w), ql, qu, w.m)
    (gl, gu), st = run_gpu(w, ql, qu, dt, w.steps)
    assert st["status"] == 0 and st["steps_done"] == w.steps
    ol, ou = ql.copy(), qu.copy()
    pb = problem_of(w)
    for done in range(0, w.steps, 50):
        oracle.mprk_run(pb, w.base, w.m, dt, min(50, w.steps - done), ol, ou)
        say("  oracle", done + 50, "steps")
    el, eu = state_err(gl, ol), state_err(gu, ou)
    say("  err lower", el, "upper", eu)
    assert np.all(el <= 1e-12) and np.all(eu <= 1e-12)


def test_deterministic_bitwise():
    w = inputs.small().with_(base=3, m=4, n_buffer=5)
    ql, qu = inputs.initial_state(w)
    dt = oracle.dt_rule(problem_of(w), ql, qu, w.m)
    a, _ = run_gpu(w, ql, qu, dt, 20)
    b, _ = run_gpu(w, ql, qu, dt, 20)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_conservation_on_gpu():
    w = inputs.small()
    ql, qu = inputs.initial_state(w)
    dt = oracle.dt_rule(problem_of(w), ql, qu, w.m)
    tl, tu = dev(ql), dev(qu)
    sol = mprk.Solver(mprk.config_of_workload(w), tl, tu)
    s0 = sol.diagnostics()
    s1 = sol.run(dt, 100)
    m0 = np.array(s0["totals_lower"]) + np.array(s0["totals_upper"])
    m1 = np.array(s1["totals_lower"]) + np.array(s1["totals_upper"])
    assert abs(s1["totals_lower"][0] - s0["totals_lower"][0]) <= 1e-13 * s0["totals_lower"][0]
    assert abs(s1["totals_upper"][0] - s0["totals_upper"][0]) <= 1e-13 * s0["totals_upper"][0]
    assert abs(m1[1] - m0[1]) <= 1e-13 * m0[0]
    assert abs(m1[3] - m0[3]) <= 1e-13 * m0[3]
    sol.close()


def test_free_stream_bitwise_on_gpu():
    w = inputs.small().with_(nx=24, nz_lower=11, nz_upper=9, lz_lower=2.0, base=3, m=4,
                             n_buffer=5)
    ql, qu = inputs.uniform_state(w, 1.0, 0.3, 0.0, 1 / 1.4)
    (gl, gu), _ = run_gpu(w, ql, qu, 0.01, 5)
    assert np.array_equal(gl, ql) and np.array_equal(gu, qu)


def test_diagnostics_match_oracle():
    w = inputs.small().with_(nx=72, nz_lower=40, nz_upper=24)
    ql, qu = inputs.random_state(w, 9, amp=0.2)
    pb = problem_of(w)
    tl, tu = dev(ql), dev(qu)
    sol = mprk.Solver(mprk.config_of_workload(w), tl, tu)
    st = sol.diagnostics()
    tot = oracle.totals(pb, ql, qu)
    assert np.allclose(st["totals_lower"][:4], tot[0], rtol=1e-14, atol=1e-15)
    assert np.allclose(st["totals_upper"][:4], tot[1], rtol=1e-14, atol=1e-15)
    assert st["totals_lower"][4] == 0.0 and st["totals_upper"][4] == 0.0
    lam, cour, vis, bad = oracle.wave_measures(pb, ql, qu)
    assert st["lambda_lower"] == pytest.approx(lam[0], rel=1e-14)
    assert st["lambda_upper"] == pytest.approx(lam[1], rel=1e-14)
    assert st["courant_lower"] == pytest.approx(cour[0], rel=1e-14)
    assert st["visc_upper"] == pytest.approx(vis[1], rel=1e-14)
    assert sol.stable_dt() == pytest.approx(oracle.dt_rule(pb, ql, qu, w.m), rel=1e-14)
    sol.close()


def test_nonfinite_state_is_reported():
    w = inputs.small().with_(nx=16, nz_lower=8, nz_upper=8)
    ql, qu = inputs.initial_state(w)
    qu[0, 3, 5] = np.nan
    tl, tu = dev(ql), dev(qu)
    sol = mprk.Solver(mprk.config_of_workload(w), tl, tu)
    with pytest.raises(mprk.MprkError) as e:
        sol.run(0.01, 3, check_every=1)
    assert e.value.code == mprk.ENONFINITE
    sol.close()
