"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/mprk.h, and its host-only entry points (validation,
workspace size, status strings, step rule, argument errors) behave as
documented."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

from paper_2202_11890_amd import inputs, mprk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "mprk.h")).read()
    return sorted(set(re.findall(r"\b(mprk_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = mprk.load()
    names = _declared()
    assert set(names) == set(mprk.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def _cfg(**kw):
    w = inputs.small()
    return mprk.config_of_workload(w, **kw)


@pytest.mark.parametrize("over,code", [
    ({}, mprk.OK),
    ({"abi_version": 99}, mprk.EINVAL),
    ({"dim": 3}, mprk.EINVAL),
    ({"dim": 3, "ny": 8, "dy": 0.1}, mprk.OK),
    ({"dim": 3, "ny": 8, "dy": 0.0}, mprk.EINVAL),
    ({"dim": 3, "ny": 3, "dy": 0.1}, mprk.EINVAL),
    ({"dim": 1}, mprk.EINVAL),
    ({"ny": 2}, mprk.EINVAL),
    ({"nx": 3}, mprk.EINVAL),
    ({"nz_lower": 2}, mprk.EINVAL),
    ({"dx": 0.0}, mprk.EINVAL),
    ({"dz_upper": float("nan")}, mprk.EINVAL),
    ({"fast_is_lower": 2}, mprk.EINVAL),
    ({"base_rk": 4}, mprk.EINVAL),
    ({"m": 0}, mprk.EINVAL),
    ({"n_buffer": 0}, mprk.EINVAL),
    ({"n_buffer": 31}, mprk.EINVAL),
    ({"n_buffer": 30}, mprk.OK),
    ({"gamma": 1.0}, mprk.EINVAL),
    ({"prandtl": 0.0}, mprk.EINVAL),
    ({"mu_lower": 0.0}, mprk.EINVAL),
    ({"gravity": float("inf")}, mprk.EINVAL),
    ({"flux_bits": 32}, mprk.OK),
    ({"flux_bits": 16}, mprk.EINVAL),
    ({"n_buffer": 2, "strict_buffer": 1}, mprk.EBUFFER),
    ({"n_buffer": 3, "strict_buffer": 1}, mprk.OK),
    ({"n_buffer": 4, "base_rk": 3, "strict_buffer": 1}, mprk.EBUFFER),
    ({"n_buffer": 1, "m": 1, "strict_buffer": 1}, mprk.OK),
    # empty and negative sizes
    ({"nx": 0}, mprk.EINVAL),
    ({"nx": -64}, mprk.EINVAL),
    ({"nz_upper": 0}, mprk.EINVAL),
    ({"dim": 3, "ny": 0, "dy": 0.1}, mprk.EINVAL),
    # rate ratio 1..64
    ({"m": 64}, mprk.OK),
    ({"m": 65}, mprk.EINVAL),
    # at most 2^28 cells per domain (no overflow in the product)
    ({"nx": 1 << 18, "nz_lower": 1024, "nz_upper": 1024}, mprk.OK),
    ({"nx": (1 << 18) + 1, "nz_lower": 1024, "nz_upper": 1024}, mprk.EINVAL),
    ({"nx": (1 << 31) - 1}, mprk.EINVAL),
    ({"dim": 3, "nx": 1024, "ny": 1024, "dy": 0.1, "nz_lower": 256, "nz_upper": 256}, mprk.OK),
    ({"dim": 3, "nx": 1024, "ny": 1024, "dy": 0.1, "nz_lower": 256, "nz_upper": 257}, mprk.EINVAL),
    ({"dim": 3, "nx": 1 << 16, "ny": 1 << 16, "dy": 0.1}, mprk.EINVAL),
])
def test_validate(over, code):
    cfg = _cfg()
    for k, v in over.items():
        setattr(cfg, k, v)
    rc, msg = mprk.mprk_validate(cfg)
    assert rc == code, msg


def test_short_buffer_is_a_warning_without_strict_mode():
    rc, msg = mprk.mprk_validate(_cfg(n_buffer=2))
    assert rc == mprk.OK and "warning" in msg


def test_workspace_bytes():
    def expect(cfg):
        a = lambda n: (n + 255) // 256 * 256
        s = cfg.base_rk
        n_lo = 4 * cfg.nz_lower * cfg.nx * 8
        n_up = 4 * cfg.nz_upper * cfg.nx * 8
        tot = (s - 1) * (a(n_lo) + a(n_up))
        if cfg.m > 1:
            tot += s * a(4 * 2 * cfg.nx * 8) + a(4 * cfg.n_buffer * cfg.nx * 8)
        tot += a(2 * 256 * 14 * 8) + a(2 * 14 * 8)
        return tot

    def tables(cfg):
        # persistent-execution tables: m*s stage records, one 16-B record and
        # one counter per fixed tile of the shape with the most tiles, a
        # member record, the abort flag
        ntiles = max(-(-cfg.nx // tx) * (-(-cfg.nz_lower // tz) - (-cfg.nz_upper // tz))
                     for tx, tz in ((32, 16), (16, 32), (64, 8), (32, 8)))
        return cfg.m * cfg.base_rk * 2048 + ntiles * 20 + 4096

    for kw in ({}, {"m": 1}, {"base_rk": 3, "n_buffer": 5}, {"fast_is_lower": 0}):
        cfg = _cfg(**kw)
        extra = mprk.mprk_workspace_bytes(cfg) - expect(cfg)
        assert 0 < extra <= tables(cfg)
    big = mprk.config_of_workload(inputs.large())
    extra = mprk.mprk_workspace_bytes(big) - expect(big)
    assert 0 < extra <= tables(big)
    assert mprk.mprk_workspace_bytes(_cfg(m=0)) == 0


def test_create_rejects_bad_arguments_before_touching_the_device():
    cfg = _cfg()
    need = mprk.mprk_workspace_bytes(cfg)
    fake = 1 << 20   # never dereferenced: every case fails validation first
    assert mprk.mprk_create(cfg, None, fake, fake, need, None)[0] == mprk.EINVAL
    assert mprk.mprk_create(cfg, fake, fake, None, need, None)[0] == mprk.EWORKSPACE
    assert mprk.mprk_create(cfg, fake, fake, fake, need - 8, None)[0] == mprk.EWORKSPACE
    assert mprk.mprk_create(cfg, fake, fake, fake + 8, need, None)[0] == mprk.EWORKSPACE
    bad = _cfg(m=0)
    assert mprk.mprk_create(bad, fake, fake, fake, need, None)[0] == mprk.EINVAL
    lib = mprk.load()
    assert lib.mprk_step(None, ctypes.c_double(0.1)) == mprk.EINVAL
    assert lib.mprk_rhs(None, None, None, None, None, 7) == mprk.EINVAL
    assert lib.mprk_destroy(None) == mprk.EINVAL


def test_strerror_covers_every_code():
    seen = set()
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        s = mprk.strerror(code)
        assert s and s != "unknown status"
        seen.add(s)
    assert len(seen) == 8
    assert mprk.strerror(-99) == "unknown status"


def test_stable_dt_rule_matches_the_oracle_rule():
    import oracle

    w = inputs.large().with_(nx=128, nz_lower=64, nz_upper=64)
    ql, qu = inputs.initial_state(w)
    pb = oracle.Problem(w.nx, w.nz_lower, w.nz_upper, w.dx, w.dz_lower, w.dz_upper,
                        n_buffer=w.n_buffer)
    lam, cour, vis, bad = oracle.wave_measures(pb, ql, qu)
    st = mprk.mprk_stats()
    st.lambda_lower, st.lambda_upper = lam
    st.courant_lower, st.courant_upper = cour
    st.visc_lower, st.visc_upper = vis
    for m in (1, 2, 4, 8):
        cfg = mprk.config_of_workload(w, m=m)
        rc, dt = mprk.mprk_stable_dt(cfg, st, 0.5, 0.25)
        assert rc == mprk.OK
        assert dt == pytest.approx(oracle.dt_rule(pb, ql, qu, m), rel=1e-15)
    st.status = 1
    assert mprk.mprk_stable_dt(mprk.config_of_workload(w), st, 0.5, 0.25)[0] == mprk.ENONFINITE


def _member(w=None, ql=1 << 20, qu=(1 << 20) + (1 << 24), dt=0.01, **kw):
    w = w or inputs.small()
    return mprk.mprk_member(mprk.config_of_workload(w, **kw), ql, qu, dt)


def test_batch_validation_rules():
    a = _member()
    b = _member(ql=3 << 24, qu=4 << 24, m=4, base_rk=3, n_buffer=5)
    assert mprk.mprk_batch_validate([a, b])[0] == mprk.OK
    assert mprk.mprk_batch_validate([])[0] == mprk.EINVAL
    assert mprk.mprk_batch_validate([a, _member(ql=3 << 24, qu=4 << 24, flux_bits=32)])[0] == mprk.EINVAL
    assert mprk.mprk_batch_validate([a, _member(ql=3 << 24, qu=4 << 24, dt=0.0)])[0] == mprk.EINVAL
    rc, msg = mprk.mprk_batch_validate([a, _member(ql=3 << 24, qu=4 << 24, m=0)])
    assert rc == mprk.EINVAL and "member 1" in msg


def test_batch_workspace_covers_every_member():
    ws = [inputs.small(), inputs.small().with_(nx=37, nz_lower=33, nz_upper=21, base=3, m=4,
                                               n_buffer=5)]
    mem = [_member(w, ql=(2 * i + 1) << 24, qu=(2 * i + 2) << 24, base_rk=w.base, m=w.m,
                   n_buffer=w.n_buffer) for i, w in enumerate(ws)]
    total = mprk.mprk_batch_workspace_bytes(mem)
    single = sum(mprk.mprk_workspace_bytes(m.cfg) for m in mem)
    # member scratch is the single-context workspace minus its persistent tables
    assert total > 0.5 * single
    assert mprk.mprk_batch_workspace_bytes(mem[:1]) < total


def test_batch_create_rejects_overlap_and_small_workspace():
    a = _member()
    b = _member(ql=(1 << 20) + 4096, qu=5 << 24)        # overlaps a's lower state
    need = mprk.mprk_batch_workspace_bytes([a, b])
    fake = 1 << 30
    assert mprk.mprk_batch_create([a, b], fake, need, None)[0] == mprk.EINVAL
    c = _member(ql=5 << 24, qu=6 << 24)
    need = mprk.mprk_batch_workspace_bytes([a, c])
    assert mprk.mprk_batch_create([a, c], fake, need - 256, None)[0] == mprk.EWORKSPACE
    assert mprk.mprk_batch_create([a, c], fake + 8, need, None)[0] == mprk.EWORKSPACE
    lib = mprk.load()
    assert lib.mprk_batch_run(None, 1, 0, None) == mprk.EINVAL
    assert lib.mprk_batch_set_tile(None, 0) == mprk.EINVAL
    assert lib.mprk_batch_destroy(None) == mprk.EINVAL


def test_tile_shape_and_exec_arguments_checked():
    lib = mprk.load()
    assert lib.mprk_set_tile(None, 0) == mprk.EINVAL
    assert lib.mprk_set_exec(None, mprk.EXEC_GRAPH) == mprk.EINVAL


def test_batch_adaptive_arguments_checked():
    lib = mprk.load()
    assert lib.mprk_batch_set_adaptive(None, 0.5, 0.25) == mprk.EINVAL
    assert lib.mprk_batch_get_dt(None, 0, None) == mprk.EINVAL


def test_serving_footprint_and_budget_check():
    pytest.importorskip("torch")
    from paper_2202_11890_amd import serving

    w = inputs.small()
    cfg = mprk.config_of_workload(w)
    state = 8 * 4 * w.nx * (w.nz_lower + w.nz_upper)
    fp = serving.footprint(cfg)
    assert fp > state
    ql, qu = inputs.initial_state(w)
    srv = serving.Server("cpu", fp - 1)
    with pytest.raises(ValueError):
        srv.run([serving.Request(0, cfg, ql, qu, 5)])


def test_workspace_bytes_3d():
    w = inputs.small3d()
    cfg = mprk.config3_of_workload(w)
    a = lambda n: (n + 255) // 256 * 256
    plane = w.nx * w.ny * 8
    core = (w.base - 1) * (a(5 * w.nz_lower * plane) + a(5 * w.nz_upper * plane))
    core += w.base * a(5 * 2 * plane) + a(5 * w.n_buffer * plane)
    core += a(2 * 256 * 14 * 8) + a(2 * 14 * 8)
    got = mprk.mprk_workspace_bytes(cfg)
    assert core < got <= core + w.m * w.base * 2048 + 64 * 1024
    # batches hold 2D problems only
    m = mprk.mprk_member(cfg, 1 << 20, 1 << 28, 0.01)
    assert mprk.mprk_batch_validate([m])[0] == mprk.EUNSUPPORTED


def test_bench_refuses_more_than_one_gpu():
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_counter_profiles_are_reported_only_for_the_kernels_they_measured():
    """The HBM-traffic summaries under profiles/ carry the hash of the kernel
    sources they were taken with (code without comments, per-source compiler
    flags); the benchmark reports their traffic only while that hash matches
    the current sources, and null once a kernel has changed."""
    import json

    import bench

    for kernel, workload in (("stage_kernel", "large"), ("march_kernel3", "large3d")):
        path = os.path.join(ROOT, "profiles", "%s_%s_hbm_traffic.json" % (kernel, workload))
        d = json.load(open(path))
        assert d["hbm_bytes_per_launch"] > 0 and len(d["kernel_source_hash"]) >= 16
        got = bench.traffic_from_profiles(workload, kernel)
        if d["kernel_source_hash"] == bench.kernel_source_hash(kernel):
            assert got == d["hbm_bytes_per_launch"]
        else:
            assert got is None


def test_time_at_error_interpolates_in_log_log():
    """The benchmark's equal-error helper: time along a power law is
    recovered exactly between runs, a target coarser than the coarsest run
    costs that run's time, a finer one is extrapolated along the two finest."""
    import bench

    k = np.array([1.0, 2.0, 4.0, 8.0])
    errors = 3e-4 / k ** 2          # second order: error ~ dt^2, time ~ 1/dt
    times = 0.5 * k
    t, how = bench.time_at_error(errors, times, 3e-4 / 3.0 ** 2)
    assert how == "interpolated" and t == pytest.approx(1.5, rel=1e-12)
    t, how = bench.time_at_error(errors, times, 1e-3)
    assert how == "capped" and t == 0.5
    t, how = bench.time_at_error(errors, times, 3e-4 / 16.0 ** 2)
    assert how == "extrapolated" and t == pytest.approx(8.0, rel=1e-12)
