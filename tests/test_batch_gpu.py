"""Batches, execution modes and tile shapes on the GPU.

A member's arithmetic does not depend on the rest of the batch, on the
execution mode (one launch per stage, a graph per slow step, persistent
dataflow) or on the tile shape: every face is evaluated by the same
operations from the same inputs.  So these tests demand bit-identical
states, and tie the batch to the FP64 oracle through one member.
"""
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
from tests.test_parity_gpu import dev, problem_of, say, state_err  # noqa: E402

# Uneven members: sizes, rate ratios (including single rate), base methods,
# which domain is fast, buffer widths.
MEMBERS = [
    inputs.small().with_(nx=40, nz_lower=20, nz_upper=18, m=2, seed=11),
    inputs.small().with_(nx=37, nz_lower=33, nz_upper=21, base=3, m=4, n_buffer=5, seed=12),
    inputs.small().with_(nx=64, nz_lower=16, nz_upper=24, m=8, fast_is_lower=False,
                         t_lower=1.0, t_upper=16.0, n_buffer=3, seed=13),
    inputs.small().with_(nx=20, nz_lower=9, nz_upper=11, m=1, n_buffer=2, seed=14),
    inputs.small().with_(nx=50, nz_lower=21, nz_upper=37, m=3, n_buffer=19, mu_lower=3e-3,
                         mu_upper=5e-4, seed=15),
]


def states(ws):
    out = []
    for w in ws:
        ql, qu = inputs.initial_state(w)
        dt = oracle.dt_rule(problem_of(w), ql, qu, w.m)
        out.append((w, ql, qu, dt))
    return out


def run_batch(sts, nsteps, flux_bits=64, exec_mode=mprk.EXEC_LAUNCH, tile=None, segments=(None,)):
    tens = [(dev(ql), dev(qu)) for _, ql, qu, _ in sts]
    mem = [(mprk.config_of_workload(w, flux_bits=flux_bits), tl, tu, dt)
           for (w, _, _, dt), (tl, tu) in zip(sts, tens)]
    b = mprk.Batch(mem, exec_mode=exec_mode, tile=tile)
    for seg in segments:
        b.run(nsteps if seg is None else seg, check_every=0)
    torch.cuda.synchronize()
    out = [(tl.cpu().numpy(), tu.cpu().numpy()) for tl, tu in tens]
    b.close()
    return out


def run_single(w, ql, qu, dt, nsteps, flux_bits=64, exec_mode=mprk.EXEC_LAUNCH, tile=None):
    tl, tu = dev(ql), dev(qu)
    sol = mprk.Solver(mprk.config_of_workload(w, flux_bits=flux_bits), tl, tu, exec_mode=exec_mode,
                      tile=tile)
    sol.run(dt, nsteps)
    torch.cuda.synchronize()
    out = tl.cpu().numpy(), tu.cpu().numpy()
    sol.close()
    return out


def same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("flux_bits", [64, 32])
def test_batch_member_equals_single_context_bitwise(flux_bits):
    sts = states(MEMBERS)
    got = run_batch(sts, 6, flux_bits)
    for (w, ql, qu, dt), g in zip(sts, got):
        say("member", w.nx, w.nz_lower, w.nz_upper, "m", w.m, "base", w.base)
        ref = run_single(w, ql, qu, dt, 6, flux_bits)
        assert same(g, ref)


def test_batch_member_matches_oracle():
    sts = states(MEMBERS)
    got = run_batch(sts, 10)
    for (w, ql, qu, dt), (gl, gu) in zip(sts, got):
        ol, ou = ql.copy(), qu.copy()
        oracle.mprk_run(problem_of(w), w.base, w.m, dt, 10, ol, ou)
        el, eu = state_err(gl, ol), state_err(gu, ou)
        say("member m", w.m, "err", el.max(), eu.max())
        assert np.all(el <= 1e-12) and np.all(eu <= 1e-12)


@pytest.mark.parametrize("mode", [mprk.EXEC_GRAPH, mprk.EXEC_PERSISTENT])
def test_batch_modes_bitwise(mode):
    sts = states(MEMBERS)
    ref = run_batch(sts, 7)
    # several run segments: graph replays / persistent launches with the
    # host's reductions and synchronisation in between
    got = run_batch(sts, 7, exec_mode=mode, segments=(2, 1, 4))
    assert all(same(a, b) for a, b in zip(ref, got))


@pytest.mark.parametrize("flux_bits", [64, 32])
@pytest.mark.parametrize("tile", [mprk.TILE_16X32, mprk.TILE_64X8, mprk.TILE_32X8])
def test_tile_shapes_bitwise(tile, flux_bits):
    """Every tile shape gives the default shape's bits, with either flux
    precision (a face on a tile edge is computed by the same operations
    whichever tile and call site computes it)."""
    sts = states(MEMBERS)
    ref = run_batch(sts, 5, flux_bits)
    got = run_batch(sts, 5, flux_bits, tile=tile)
    assert all(same(a, b) for a, b in zip(ref, got))
    w, ql, qu, dt = sts[1]
    assert same(run_single(w, ql, qu, dt, 5, flux_bits, tile=tile), run_single(w, ql, qu, dt, 5, flux_bits))


@pytest.mark.parametrize("tile", [mprk.TILE_16X32, mprk.TILE_32X8])
def test_tile_shapes_persistent_bitwise(tile):
    w, ql, qu, dt = states(MEMBERS[:2])[1]
    ref = run_single(w, ql, qu, dt, 4)
    got = run_single(w, ql, qu, dt, 4, exec_mode=mprk.EXEC_PERSISTENT, tile=tile)
    assert same(ref, got)


def test_single_context_graph_mode():
    w, ql, qu, dt = states(MEMBERS[1:2])[0]
    tl, tu = dev(ql), dev(qu)
    sol = mprk.Solver(mprk.config_of_workload(w), tl, tu, exec_mode=mprk.EXEC_GRAPH)
    sol.run(dt, 3)
    d1 = sol.diagnostics()              # eager work between replays
    sol.run(0.5 * dt, 2)                # another dt: the graph is rebuilt
    sol.set_tile(mprk.TILE_64X8)
    sol.run(dt, 2)                      # another shape: rebuilt again
    torch.cuda.synchronize()
    got = tl.cpu().numpy(), tu.cpu().numpy()
    sol.close()
    tl, tu = dev(ql), dev(qu)
    ref = mprk.Solver(mprk.config_of_workload(w), tl, tu)
    ref.run(dt, 3)
    ref.run(0.5 * dt, 2)
    ref.run(dt, 2)
    torch.cuda.synchronize()
    assert same(got, (tl.cpu().numpy(), tu.cpu().numpy()))
    assert d1["steps_done"] == 3
    ref.close()


def test_tuner_times_every_shape_and_leaves_states_alone():
    sts = states(MEMBERS)
    tens = [(dev(ql), dev(qu)) for _, ql, qu, _ in sts]
    mem = [(mprk.config_of_workload(w), tl, tu, dt) for (w, _, _, dt), (tl, tu) in zip(sts, tens)]
    b = mprk.Batch(mem)
    ms, best = b.tune(2)
    say("tuner ms per step", ms, "best", mprk.TILE_NAMES[best])
    assert len(ms) == mprk.TILE_SHAPES and all(x > 0 for x in ms)
    assert ms[best] == min(ms)
    for (_, ql, qu, _), (tl, tu) in zip(sts, tens):
        assert np.array_equal(tl.cpu().numpy(), ql) and np.array_equal(tu.cpu().numpy(), qu)
    b.run(4)
    torch.cuda.synchronize()
    got = [(tl.cpu().numpy(), tu.cpu().numpy()) for tl, tu in tens]
    b.close()
    ref = run_batch(sts, 4)
    assert all(same(a, c) for a, c in zip(ref, got))


def test_batch_stable_dt_and_set_dt():
    sts = states(MEMBERS)
    tens = [(dev(ql), dev(qu)) for _, ql, qu, _ in sts]
    mem = [(mprk.config_of_workload(w), tl, tu, 1.0) for (w, _, _, _), (tl, tu) in zip(sts, tens)]
    b = mprk.Batch(mem)
    dts = b.stable_dts()
    for (w, ql, qu, dt), d in zip(sts, dts):
        assert d == pytest.approx(dt, rel=1e-13)
    for i, d in enumerate(dts):
        b.set_dt(i, d)
    b.run(3)
    torch.cuda.synchronize()
    got = [(tl.cpu().numpy(), tu.cpu().numpy()) for tl, tu in tens]
    b.close()
    ref = run_batch([(w, ql, qu, d) for (w, ql, qu, _), d in zip(sts, dts)], 3)
    assert all(same(a, c) for a, c in zip(ref, got))


def test_batch_reports_a_bad_member():
    sts = states(MEMBERS[:3])
    w, ql, qu, dt = sts[1]
    qu = qu.copy()
    qu[0, 2, 3] = np.nan
    sts[1] = (w, ql, qu, dt)
    tens = [(dev(a), dev(b)) for _, a, b, _ in sts]
    mem = [(mprk.config_of_workload(w), tl, tu, dt) for (w, _, _, dt), (tl, tu) in zip(sts, tens)]
    b = mprk.Batch(mem)
    with pytest.raises(mprk.MprkError) as e:
        b.run(2, check_every=1)
    assert e.value.code == mprk.ENONFINITE
    st = b.diagnostics(check=False)
    assert [s["status"] for s in st] == [0, 1, 0]
    b.close()


def test_adaptive_steps_follow_each_members_state():
    """Adaptive steps: the run equals running chunk by chunk and resetting
    every member's step from its own diagnostics in between."""
    sts = states(MEMBERS)
    tens = [(dev(ql), dev(qu)) for _, ql, qu, _ in sts]
    mem = [(mprk.config_of_workload(w), tl, tu, dt) for (w, _, _, dt), (tl, tu) in zip(sts, tens)]
    b = mprk.Batch(mem, exec_mode=mprk.EXEC_GRAPH)
    b.set_adaptive(0.5, 0.25)
    b.run(9, check_every=3)
    dts = b.dts()
    torch.cuda.synchronize()
    got = [(tl.cpu().numpy(), tu.cpu().numpy()) for tl, tu in tens]
    b.close()
    tens = [(dev(ql), dev(qu)) for _, ql, qu, _ in sts]
    mem = [(mprk.config_of_workload(w), tl, tu, dt) for (w, _, _, dt), (tl, tu) in zip(sts, tens)]
    r = mprk.Batch(mem)
    for _ in range(3):
        r.run(3)
        for i, d in enumerate(r.stable_dts(0.5, 0.25)):
            r.set_dt(i, d)
    assert r.dts() == dts
    torch.cuda.synchronize()
    ref = [(tl.cpu().numpy(), tu.cpu().numpy()) for tl, tu in tens]
    r.close()
    assert all(same(a, c) for a, c in zip(ref, got))
    assert any(d != s[3] for d, s in zip(dts, sts))
