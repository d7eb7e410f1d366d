"""Benchmark: MPRK vs single-rate RK on two coupled 2D Navier-Stokes domains.

One *step* is one slow step of the whole hot path (every stage launch of the
MPRK schedule, with the device reductions every --check-every steps) on the
1024x512-per-domain workload (SSP-RK3 base, m = 4, 4 buffer rows, FP64),
inputs resident in HBM before timing starts.

The JSON line reports MPRK cell-stage updates per second (cell-stage counts of
Section 4: s N_S + m s (N_B + N_F) per slow step), per-step p50/p99 latency,
the single-rate RK3 at the fast step dt/m on the same GPU, the errors of both
against a fine single-rate reference (equal-accuracy comparison), the stage
kernel's roofline position, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
FP64_VECTOR_PEAK_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed slow steps (default: workload's 1000)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["large", "small"], default="large")
    ap.add_argument("--check-every", type=int, default=10)
    ap.add_argument("--exec", choices=["persistent", "launch"], default="launch",
                    help="persistent: one cooperative launch per check segment; launch: one per stage")
    ap.add_argument("--tile", choices=["32x16", "16x32", "64x8", "32x8"], default=None,
                    help="2D tile shape of the headline, FP32-flux and single-rate runs (default: the "
                         "library's, 32x16)")
    ap.add_argument("--latency-steps", type=int, default=200)
    ap.add_argument("--profile-steps", type=int, default=50)
    ap.add_argument("--no-sr", action="store_true", help="skip the single-rate comparison")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-flux run")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched-ensemble run")
    ap.add_argument("--ensemble-members", type=int, default=64)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving run")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D run")
    ap.add_argument("--steps-3d", type=int, default=None, help="default: the workload's 200")
    ap.add_argument("--flux-3d", type=int, choices=[32, 64], default=32,
                    help="face-flux precision of the 3D run (the workload's is 32)")
    ap.add_argument("--serving-requests", type=int, default=120)
    ap.add_argument("--serving-load", type=float, default=0.7,
                    help="Poisson arrival rate as a fraction of the measured saturated capacity")
    ap.add_argument("--ensemble-steps", type=int, default=None, help="default: the members' 500")
    ap.add_argument("--ensemble-mode", choices=["graph", "launch", "persistent"], default=None,
                    help="time only this execution mode of the ensemble (no tuner, single-rate or "
                         "equal-error runs; for profiling)")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the equal-error comparison")
    ap.add_argument("--eq-steps", type=int, default=100,
                    help="horizon of the equal-error comparison, in slow steps of the stable dt")
    ap.add_argument("--no-buffer6", action="store_true",
                    help="skip the run with 6 buffer rows (the exactly conservative width for SSP-RK3)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run plain device copies of this many MiB (counter calibration)")
    return ap.parse_args()


def l2(dx, dzs, diffs):
    """Per-component L2 norm weighted by cell size (Section 5 error norm)."""
    out = np.zeros(4)
    for d, dz in zip(diffs, dzs):
        out += (d.astype(np.float64) ** 2).sum(axis=(1, 2)) * dx * dz
    return np.sqrt(out)


def time_at_error(errors, times, target):
    """Time a method needs to reach L2 error `target`, from its runs at several
    step sizes: piecewise-linear interpolation of log(time) against log(error)
    over the runs sorted by error.  A target above the largest error (a
    coarser step than the method's coarsest run, which sits at its stability
    limit) costs the coarsest run's time ("capped"); a target below the
    smallest error is extrapolated with the slope of the two finest runs
    ("extrapolated").  Returns (time, how)."""
    e = np.asarray(errors, dtype=np.float64)
    t = np.asarray(times, dtype=np.float64)
    order = np.argsort(e)
    e, t = np.log(e[order]), np.log(t[order])
    x = np.log(target)
    if x >= e[-1]:
        return float(np.exp(t[-1])), "capped"
    if x < e[0]:
        slope = (t[1] - t[0]) / (e[1] - e[0])
        return float(np.exp(t[0] + slope * (x - e[0]))), "extrapolated"
    return float(np.exp(np.interp(x, e, t))), "interpolated"


KERNEL_SOURCES = {"stage_kernel": ("mprk_kernels.hip", "mprk_internal.h", "mprk_device.h"),
                  "stage_kernel3": ("mprk_kernels3d.hip", "mprk_internal.h", "mprk_device.h"),
                  "march_kernel3": ("mprk_kernels3d.hip", "mprk_internal.h", "mprk_device.h")}


def code_text(path: str) -> bytes:
    """A source file without its comments and blank lines (the sources hold
    no string literal containing a comment marker)."""
    text = re.sub(r"/\*.*?\*/", "", open(path).read(), flags=re.S)
    lines = (re.sub(r"//.*", "", ln).rstrip() for ln in text.splitlines())
    return "\n".join(ln for ln in lines if ln).encode()


def kernel_source_hash(kernel: str = "stage_kernel"):
    """Hash of a kernel's code (comments aside) and of its per-source compiler
    flags."""
    from __graft_entry__ import EXTRA_FLAGS

    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        h.update(code_text(os.path.join(ROOT, "paper_2202_11890_amd", "csrc", f)))
        h.update(" ".join(EXTRA_FLAGS.get(f, [])).encode())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload: str, kernel: str = "stage_kernel"):
    """HBM bytes per stage launch from a committed counter summary, if its
    kernel-source hash matches the current sources (else None)."""
    path = os.path.join(ROOT, "profiles", "%s_%s_hbm_traffic.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except ValueError:
        return None
    if d.get("kernel_source_hash") != kernel_source_hash(kernel):
        return None
    return d.get("hbm_bytes_per_launch")


def drift(s0, s1, ie=3):
    """Change of the conserved totals between two stats: mass of each domain
    relative to its own mass, total x-momentum relative to the total mass,
    total energy relative to itself (Section 5.1's conservation check)."""
    a0 = np.array([s0["totals_lower"], s0["totals_upper"]])
    a1 = np.array([s1["totals_lower"], s1["totals_upper"]])
    return {
        "mass_lower": float(abs(a1[0, 0] - a0[0, 0]) / a0[0, 0]),
        "mass_upper": float(abs(a1[1, 0] - a0[1, 0]) / a0[1, 0]),
        "x_momentum": float(abs(a1[:, 1].sum() - a0[:, 1].sum()) / a0[:, 0].sum()),
        "energy": float(abs(a1[:, ie].sum() - a0[:, ie].sum()) / a0[:, ie].sum()),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2202_11890_amd import costmodel, inputs, mprk

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = inputs.large() if args.workload == "large" else inputs.small()
    K = args.steps if args.steps is not None else w.steps
    W = args.warmup
    s, m = w.base, w.m
    nzf = w.nz_lower if w.fast_is_lower else w.nz_upper
    nzs = w.nz_upper if w.fast_is_lower else w.nz_lower
    nF, nB, nS = costmodel.partition_counts(w.nx, nzf, nzs, w.n_buffer)
    cs_step = costmodel.mprk_cell_stages(nF, nB, nS, m, s)
    sr_cs_step = costmodel.sr_cell_stages(nF + nB + nS, m, s)
    bytes_step = costmodel.algorithmic_bytes_per_step(nF, nB, nS, m, s)

    ql0, qu0 = inputs.initial_state(w)
    tl0 = torch.from_numpy(ql0).to(dev)
    tu0 = torch.from_numpy(qu0).to(dev)
    tl, tu = tl0.clone(), tu0.clone()
    cfg = mprk.config_of_workload(w)
    exec_mode = mprk.EXEC_PERSISTENT if args.exec == "persistent" else mprk.EXEC_LAUNCH
    tile = mprk.TILE_NAMES.index(args.tile) if args.tile else None
    sol = mprk.Solver(cfg, tl, tu, exec_mode=exec_mode, tile=tile)
    dt = sol.stable_dt(w.cfl, w.dnum)

    # ---- warm-up, then restore the initial state
    sol.run(dt, max(W, 1), check_every=0)
    tl.copy_(tl0)
    tu.copy_(tu0)
    torch.cuda.synchronize()

    tot0 = sol.diagnostics()            # conserved totals at t = 0 (outside the timed region)

    # ---- timed region: K slow steps (wall clock and events on the stream)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(sol.stream)
    st = sol.run(dt, K, check_every=args.check_every)
    ev1.record(sol.stream)
    torch.cuda.synchronize()
    t_mprk = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_step = 1e3 * t_mprk / K
    value = cs_step * K / t_mprk
    mprk_final = (tl.cpu().numpy(), tu.cpu().numpy())
    print("# mprk: %d steps in %.3f s (%.1f us/step), status %d" %
          (K, t_mprk, 1e6 * t_mprk / K, st["status"]), file=sys.stderr, flush=True)
    conservation = {"n_buffer_%d" % w.n_buffer: drift(tot0, st)}

    # ---- per-step latency (events on the solver's stream)
    lat = []
    stream = sol.stream
    for _ in range(args.latency_steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sol.step(dt)
        e1.record(stream)
        lat.append((e0, e1))
    torch.cuda.synchronize()
    lat_ms = np.array([a.elapsed_time(b) for a, b in lat])

    # ---- dominant kernel time per launch.  Launches run back to back on the
    # stream, so the event time of the timed region divided by the number of
    # launches of the dominant kernel is its average duration (the reductions
    # every check_every steps are included, about 1%).  In launch mode that
    # kernel is the stage kernel (m*s launches per step; events bracketing
    # every launch are also reported); in persistent mode it is the
    # persistent kernel (one launch per check segment of check_every steps).
    launches_per_step = m * s
    if args.exec == "launch":
        sol.profile(True)
        for _ in range(args.profile_steps):
            sol.step(dt)
        k_ms, k_n = sol.profile_take()
        sol.profile(False)
        kernel_name = "stage_kernel"
        n_launch = K * launches_per_step
        bytes_per_launch = bytes_step / launches_per_step
        bracketed = round(k_ms * 1e3 / k_n, 3)
    else:
        kernel_name = "persistent_kernel"
        seg = args.check_every if args.check_every > 0 else K
        n_launch = -(-K // seg)
        bytes_per_launch = bytes_step * K / n_launch
        bracketed = None
    avg_launch_s = gpu_ms * 1e-3 / n_launch
    achieved = bytes_per_launch / avg_launch_s / 1e9
    # the counter summary covers the default launch configuration only
    traffic = traffic_from_profiles(args.workload) if (args.exec == "launch" and args.tile in (None, "32x16")) else None
    roofline = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,                 # counter HBM bytes per launch
        "traffic_gbs": None if traffic is None else round(traffic / avg_launch_s / 1e9, 1),
        "kernel": kernel_name,
        "avg_launch_us": round(avg_launch_s * 1e6, 3),
        "avg_launch_us_bracketed": bracketed,
        "algorithmic_bytes_per_launch": int(bytes_per_launch),
        "stage_time_us": round(gpu_ms * 1e3 / (K * launches_per_step), 3),
    }
    print("# %s: %.2f us/launch, %.0f GB/s algorithmic" %
          (kernel_name, avg_launch_s * 1e6, achieved), file=sys.stderr, flush=True)

    out = {
        "metric": "cell-stage updates/s, MPRK vs single-rate RK at equal error; p50/p99 latency",
        "value": value,
        "unit": "cell-stage updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "nx": w.nx, "nz_lower": w.nz_lower, "nz_upper": w.nz_upper,
            "base": "SSP-RK3" if s == 3 else "RK2", "m": m, "n_buffer": w.n_buffer,
            "dt": dt, "cfl": w.cfl, "diffusion_number": w.dnum,
            "check_every": args.check_every,
            "exec": args.exec,
            "tile": args.tile or "32x16",
            "cell_stages_per_step": cs_step,
            "parallelism": "single GPU",
        },
        "latency_ms_per_step": {"p50": float(np.percentile(lat_ms, 50)),
                                "p99": float(np.percentile(lat_ms, 99)),
                                "n": int(lat_ms.size)},
        "sr_equivalent_rate": sr_cs_step * K / t_mprk,
        "model_speedup": costmodel.speedup_from_counts(nF, nB, nS, m, s),
        "roofline": roofline,
    }
    sol.close()

    # ---- the same run with FP32 face fluxes (state and sums in FP64)
    if not args.no_fp32:
        tl.copy_(tl0)
        tu.copy_(tu0)
        f32 = mprk.Solver(mprk.config_of_workload(w, flux_bits=32), tl, tu, exec_mode=exec_mode, tile=tile)
        f32.run(dt, max(W, 1), check_every=0)
        tl.copy_(tl0)
        tu.copy_(tu0)
        torch.cuda.synchronize()
        e32a = torch.cuda.Event(enable_timing=True)
        e32b = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e32a.record(f32.stream)
        fst = f32.run(dt, K, check_every=args.check_every)
        e32b.record(f32.stream)
        torch.cuda.synchronize()
        t_32 = time.perf_counter() - t0
        gpu32_ms = e32a.elapsed_time(e32b)
        f32.close()
        del e32a, e32b
        dif = []
        for g, r in zip((tl.cpu().numpy(), tu.cpu().numpy()), mprk_final):
            scale = np.abs(r).max(axis=(1, 2))
            scale[1:3] = max(scale[1], scale[2])
            dif.append((np.abs(g - r).max(axis=(1, 2)) / scale).tolist())
        # Same algorithmic bytes per stage launch as FP64 (the state, stage
        # values and sums are FP64 either way); launch mode only.
        launch32_s = gpu32_ms * 1e-3 / (K * launches_per_step)
        ach32 = bytes_step / launches_per_step / launch32_s / 1e9
        # counter bytes of the FP32 instantiation (default tile) from its own summary
        t32 = traffic_from_profiles("fp32flux_" + args.workload) if args.tile in (None, "32x16") else None
        out["fp32_flux"] = {
            "value": cs_step * K / t_32, "ms_per_step": 1e3 * t_32 / K, "status": fst["status"],
            "speedup_vs_f64": t_mprk / t_32, "tile": args.tile or "32x16",
            "max_rel_diff_vs_f64": {"lower": dif[0], "upper": dif[1]},
            "roofline": None if args.exec != "launch" else {
                "bound": "hbm", "kernel": "stage_kernel (FP32 fluxes)", "achieved": round(ach32, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach32 / HBM_PEAK_GBS, 4),
                "traffic": t32, "traffic_gbs": None if t32 is None else round(t32 / launch32_s / 1e9, 1),
                "avg_launch_us": round(launch32_s * 1e6, 3)},
        }
        print("# fp32 flux: %.1f us/step, speedup %.3f" % (1e6 * t_32 / K, t_mprk / t_32),
              file=sys.stderr, flush=True)

    # ---- single-rate RK at the fast step on the same GPU
    if not args.no_sr:
        tl.copy_(tl0)
        tu.copy_(tu0)
        sr = mprk.Solver(mprk.config_of_workload(w, m=1), tl, tu, exec_mode=exec_mode, tile=tile)
        sr.run(dt / m, 2, check_every=0)
        tl.copy_(tl0)
        tu.copy_(tu0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sst = sr.run(dt / m, K * m, check_every=args.check_every * m)
        torch.cuda.synchronize()
        t_sr = time.perf_counter() - t0
        sr.close()
        out["single_rate"] = {
            "method": "SSP-RK3" if s == 3 else "RK2", "dt": dt / m, "steps": K * m,
            "value": sr_cs_step * K / t_sr, "seconds": t_sr, "status": sst["status"],
            "time_to_solution_speedup": t_sr / t_mprk,
        }
        print("# single rate: %.3f s, speedup %.3f" % (t_sr, t_sr / t_mprk), file=sys.stderr,
              flush=True)

    # ---- the same run with 6 buffer rows (>= 2s - 1: exactly conservative)
    if not args.no_buffer6:
        tl.copy_(tl0)
        tu.copy_(tu0)
        nb6 = mprk.Solver(mprk.config_of_workload(w, n_buffer=6), tl, tu, exec_mode=exec_mode, tile=tile)
        nb6.run(dt, max(W, 1), check_every=0)
        tl.copy_(tl0)
        tu.copy_(tu0)
        t6 = nb6.diagnostics()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st6 = nb6.run(dt, K, check_every=args.check_every)
        torch.cuda.synchronize()
        t_6 = time.perf_counter() - t0
        nb6.close()
        nF6, nB6, nS6 = costmodel.partition_counts(w.nx, nzf, nzs, 6)
        cs6 = costmodel.mprk_cell_stages(nF6, nB6, nS6, m, s)
        d6 = drift(t6, st6)
        d6.update({"value": cs6 * K / t_6, "ms_per_step": 1e3 * t_6 / K, "status": st6["status"]})
        conservation["n_buffer_6"] = d6
        print("# 6 buffer rows: %.1f us/step, mass drift %.1e / %.1e, energy drift %.1e" % (
            1e6 * t_6 / K, d6["mass_lower"], d6["mass_upper"], d6["energy"]), file=sys.stderr, flush=True)
    out["conservation"] = conservation

    # ---- MPRK against single-rate RK at equal error (RK3 and RK2 bases)
    if not args.no_accuracy:
        out["equal_error"] = equal_error_leg(args, torch, dev, w, tile, exec_mode)

    # ---- CPU oracle on a bounded sample (test infrastructure, host cores)
    if not args.no_cpu:
        import oracle

        pb = oracle.Problem(w.nx, w.nz_lower, w.nz_upper, w.dx, w.dz_lower, w.dz_upper,
                            fast_is_lower=w.fast_is_lower, n_buffer=w.n_buffer, gamma=w.gamma,
                            prandtl=w.prandtl, mu_lower=w.mu_lower, mu_upper=w.mu_upper,
                            gravity=w.gravity)
        a, b = ql0.copy(), qu0.copy()
        n = 0
        t0 = time.perf_counter()
        while True:
            oracle.mprk_step(pb, s, m, dt, a, b)
            n += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds or n >= K:
                break
        out["cpu_baseline"] = {
            "value": cs_step * n / el, "unit": "cell-stage updates/s",
            "cores": oracle.threads(), "kind": "oracle",
            "sample": "%d slow steps of the same workload from its initial state (%.1f s)" % (n, el),
        }
        print("# cpu oracle: %d steps in %.1f s on %d threads" % (n, el, oracle.threads()),
              file=sys.stderr, flush=True)
        # the same oracle on one thread, on a shorter sample
        nthr = oracle.threads()
        oracle.set_threads(1)
        a, b = ql0.copy(), qu0.copy()
        n1 = 0
        t0 = time.perf_counter()
        while True:
            oracle.mprk_step(pb, s, m, dt, a, b)
            n1 += 1
            el1 = time.perf_counter() - t0
            if el1 >= args.cpu_seconds / 2 or n1 >= K:
                break
        oracle.set_threads(nthr)
        out["cpu_baseline"]["single_thread"] = {
            "value": cs_step * n1 / el1, "cores": 1,
            "sample": "%d slow steps from the initial state (%.1f s)" % (n1, el1),
        }
        print("# cpu oracle, one thread: %d steps in %.1f s" % (n1, el1), file=sys.stderr, flush=True)

    # The paper's own figures (CPU wall clocks, converted to cell-stage
    # updates/s with the same counting): context, not a like-for-like target.
    out["paper_context"] = {
        "note": "CPU wall-clock figures of the paper converted to cell-stage updates/s "
                "(s*N_S + m*s*(N_B + N_F) per MPRK step); different problems and code, precision not stated",
        "rows": [
            {"workload": "2D thermal convection, MPRK2 m=2 (Table 5)", "mprk": 2.36e6, "single_rate": 2.47e6,
             "hardware": "not stated"},
            {"workload": "2D thermal convection, MPRK2 m=4 (Table 7)", "mprk": 2.23e6, "single_rate": 1.88e6,
             "hardware": "not stated"},
            {"workload": "weak scaling, wind-driven flow, 32768 cores (Table 8)", "mprk": 1.46e9,
             "single_rate": 3.66e9, "hardware": "Theta: Cray XC40, Xeon Phi 7230 (64 cores per node)"},
            {"workload": "weak scaling, thermal bubble, 32768 cores (Table 9)", "mprk": 2.31e9,
             "single_rate": 4.13e9, "hardware": "Theta: Cray XC40, Xeon Phi 7230 (64 cores per node)"},
        ],
        "unit": "cell-stage updates/s",
    }

    if not args.no_ensemble:
        out["ensemble"] = ensemble_leg(args, torch, dev)
    if not args.no_serving:
        out["serving"] = serving_leg(args, torch, dev)
    if not args.no_3d:
        out["3d"] = leg_3d(args, torch, dev)

    print(json.dumps(out), flush=True)

    # Release every HIP object the run created (events, device tensors, the
    # caching allocator's blocks) while the runtime is fully up, rather than
    # in interpreter finalisation (where a profiler's own exit handlers may
    # already be tearing the runtime down).
    del lat, ev0, ev1
    del tl, tu, tl0, tu0
    import gc

    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def equal_error_leg(args, torch, dev, w, tile, exec_mode):
    """MPRK against single-rate RK on the same GPU at equal error (the paper's
    practice: errors beside wall clocks, Tables 5 and 7).  For the SSP-RK3 base
    (MPRK3, the headline) and the RK2 base of Table 1 (MPRK2): from the same
    initial state to t_end = H dt (dt the stable slow step), MPRK runs at dt,
    dt/2, dt/4, dt/8 and single-rate runs at dt/m, dt/(2m), dt/(4m) (dt/m is
    the single-rate stability limit: nothing coarser is stable), each timed on
    the GPU with the same check cadence in simulated time, and their L2 errors
    (Section 5 norm) against single-rate RK at dt/(16 m).  The time each
    method needs for a target error comes from log-log interpolation over its
    runs; the ratio single-rate time / MPRK time at each single-rate run's
    error is the equal-error speedup (below 1: MPRK is slower at that
    accuracy).  MPRK is at most second order (Remark 2).  The same study runs
    on a variant whose error comes from the fast domain."""
    from paper_2202_11890_amd import inputs, mprk

    H = args.eq_steps
    R = 16
    res = {"protocol": "t_end = %d slow steps of the stable dt; MPRK at dt/k, k = 1, 2, 4, 8; "
                       "single rate at dt/(m k), k = 1, 2, 4; reference single rate at dt/(%d m); "
                       "time at a target error by log-log interpolation; matched on the density "
                       "L2 error" % (H, R)}
    # On the workload itself the error is set by the slow rows next to the
    # lid, which heat up by conduction from the 16 times hotter fast domain
    # and which MPRK integrates with the m-times larger step.  A variant (not
    # one of the benchmark workloads) shows the multirate case: equal
    # temperatures, the fast domain fast because its cells are 4 times
    # thinner (as in the 3D workload), and the pulse in the fast domain
    # (seed 43: centre 0.68 below the lid), so the slow domain carries little
    # of the error.
    variant = w.with_(t_lower=1.0, t_upper=1.0, lz_lower=1.25, seed=43)
    cases = [("SSP-RK3", w.with_(base=3)), ("RK2", w.with_(base=2)),
             ("variant SSP-RK3: equal temperatures, fast domain by its cells, pulse in it",
              variant.with_(base=3)),
             ("variant RK2: equal temperatures, fast domain by its cells, pulse in it",
              variant.with_(base=2))]
    for name, wb in cases:
        m = wb.m
        ql0, qu0 = inputs.initial_state(wb)
        tl0 = torch.from_numpy(ql0).to(dev)
        tu0 = torch.from_numpy(qu0).to(dev)
        tl, tu = tl0.clone(), tu0.clone()
        sol = mprk.Solver(mprk.config_of_workload(wb), tl, tu, exec_mode=exec_mode, tile=tile)
        dt = sol.stable_dt(wb.cfl, wb.dnum)
        sol.close()

        def run(m_run, step, n, check):
            tl.copy_(tl0)
            tu.copy_(tu0)
            sv = mprk.Solver(mprk.config_of_workload(wb, m=m_run), tl, tu, exec_mode=exec_mode,
                             tile=tile)
            sv.run(step, 1, check_every=0)
            tl.copy_(tl0)
            tu.copy_(tu0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = sv.run(step, n, check_every=check)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            sv.close()
            return el, st["status"], (tl.cpu().numpy(), tu.cpu().numpy())

        ce = args.check_every if args.check_every > 0 else H
        _, st_ref, ref = run(1, dt / (m * R), H * m * R, ce * m * R)
        dzs = (wb.dz_lower, wb.dz_upper)

        def err(q):
            return [float(x) for x in l2(wb.dx, dzs, [q[0] - ref[0], q[1] - ref[1]])]

        mp, sr = [], []
        for k in (1, 2, 4, 8):
            t, stt, q = run(m, dt / k, H * k, ce * k)
            mp.append({"dt_div": k, "seconds": t, "status": stt, "l2": err(q)})
        for k in (1, 2, 4):
            t, stt, q = run(1, dt / (m * k), H * m * k, ce * m * k)
            sr.append({"dt_div": m * k, "seconds": t, "status": stt, "l2": err(q)})
        me = [r["l2"][0] for r in mp]
        mt = [r["seconds"] for r in mp]
        se = [r["l2"][0] for r in sr]
        stt_ = [r["seconds"] for r in sr]
        matched = []
        for r in sr:
            tm, how = time_at_error(me, mt, r["l2"][0])
            matched.append({"target": "single rate at dt/%d" % r["dt_div"], "l2_rho": r["l2"][0],
                            "seconds_single_rate": r["seconds"], "seconds_mprk": tm, "mprk": how,
                            "speedup": r["seconds"] / tm})
        ts, how = time_at_error(se, stt_, mp[0]["l2"][0])
        matched.append({"target": "MPRK at dt", "l2_rho": mp[0]["l2"][0], "seconds_single_rate": ts,
                        "single_rate": how, "seconds_mprk": mp[0]["seconds"],
                        "speedup": ts / mp[0]["seconds"]})
        res[name] = {"seed": wb.seed, "pulse_centre": list(inputs.centre(wb)), "dt": dt, "m": m,
                     "t_end": H * dt, "reference_status": st_ref,
                     "mprk": mp, "single_rate": sr, "matched": matched,
                     "equal_error_speedup": matched[0]["speedup"],
                     "error_ratio_at_fixed_step": mp[0]["l2"][0] / sr[0]["l2"][0]}
        print("# equal error, %s: MPRK error at dt %.2e vs single rate at dt/m %.2e; speedup at the "
              "single-rate error %.3f (%s), at the MPRK error %.3f (%s)" % (
                  name, mp[0]["l2"][0], sr[0]["l2"][0], matched[0]["speedup"], matched[0]["mprk"],
                  matched[-1]["speedup"], matched[-1]["single_rate"]), file=sys.stderr, flush=True)
    return res


def cs_of(ws):
    """MPRK cell-stage updates of one slow step of every member."""
    from paper_2202_11890_amd import costmodel

    cs = 0
    for w in ws:
        nF, nB, nS = costmodel.partition_counts(w.nx, w.nz_lower, w.nz_upper, w.n_buffer)
        cs += costmodel.mprk_cell_stages(nF, nB, nS, w.m, w.base)
    return cs


def ensemble_leg(args, torch, dev):
    """Batched uneven ensemble (FP32 face fluxes, FP64 state).  Tile shape from
    the autotuner; every member advanced together with adaptive steps (each
    member's step reset from its own state every CH slow steps); the same
    members then run single-rate with each member's step divided by its m,
    chunk by chunk, so both reach the same times."""
    from paper_2202_11890_amd import costmodel, inputs, mprk

    CH = 20
    ws = inputs.ensemble(args.ensemble_members)
    K = args.ensemble_steps if args.ensemble_steps is not None else ws[0].steps
    K = max(CH, K // CH * CH)
    init = [inputs.initial_state(w) for w in ws]
    tens = [(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)) for a, b in init]
    keep = [(a.clone(), b.clone()) for a, b in tens]
    cr, dn = ws[0].cfl, ws[0].dnum

    def restore():
        for (a, b), (c, d) in zip(tens, keep):
            a.copy_(c)
            b.copy_(d)
        torch.cuda.synchronize()

    batch = mprk.Batch([(mprk.config_of_workload(w, flux_bits=32), a, b, 1.0)
                        for w, (a, b) in zip(ws, tens)])
    dts0 = batch.stable_dts(cr, dn)

    def reset_dts(bt, scale=None):
        for i, d in enumerate(dts0):
            bt.set_dt(i, d if scale is None else d / scale[i])

    reset_dts(batch)
    if args.ensemble_mode is not None:
        mode = {"graph": mprk.EXEC_GRAPH, "launch": mprk.EXEC_LAUNCH,
                "persistent": mprk.EXEC_PERSISTENT}[args.ensemble_mode]
        # a fixed tile (within 0.1% of the tuner's pick on this ensemble), so
        # that one-mode runs profiled separately share their tile shape
        batch.set_tile(mprk.TILE_32X8)
        batch.set_exec(mode)
        batch.set_adaptive(cr, dn)
        t0 = time.perf_counter()
        rc, st = batch.run_status(K, check_every=CH)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        batch.close()
        print("# ensemble, %s mode only: %d steps in %.3f s" % (args.ensemble_mode, K, el),
              file=sys.stderr, flush=True)
        return {"mode": args.ensemble_mode, "steps": K, "seconds": el, "status": rc,
                "value": cs_of(ws) * K / el, "unit": "cell-stage updates/s"}
    tuner_ms, best = batch.tune(3)
    print("# ensemble tuner (ms per slow step): %s -> %s" % (
        ", ".join("%s %.3f" % (mprk.TILE_NAMES[k], v) for k, v in enumerate(tuner_ms)),
        mprk.TILE_NAMES[best]), file=sys.stderr, flush=True)
    cs = 0
    cells = 0
    for w in ws:
        nF, nB, nS = costmodel.partition_counts(w.nx, w.nz_lower, w.nz_upper, w.n_buffer)
        cs += costmodel.mprk_cell_stages(nF, nB, nS, w.m, w.base)
        cells += w.nx * (w.nz_lower + w.nz_upper)

    def timed(bt, mode, nsteps, hist=None, chunk=CH):
        bt.set_exec(mode)
        bt.set_adaptive(0.0, dn)
        bt.run(1, check_every=0)
        restore()
        reset_dts(bt)
        bt.set_adaptive(cr, dn)
        bad = 0
        t0 = time.perf_counter()
        for _ in range(nsteps // chunk):
            if hist is not None:
                hist.append(bt.dts())
            st = bt.run(chunk, check_every=chunk)
            bad += sum(x["status"] for x in st)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, bad

    hist = []
    t_graph, bad = timed(batch, mprk.EXEC_GRAPH, K, hist)
    final = [(a.cpu().numpy(), b.cpu().numpy()) for a, b in tens]
    t_launch, _ = timed(batch, mprk.EXEC_LAUNCH, K)
    t_pers, _ = timed(batch, mprk.EXEC_PERSISTENT, K)
    batch.close()
    rate = cs * K / t_graph
    print("# ensemble: %d members, %d steps in %.3f s (graph), %.3e cell-stage/s" % (
        len(ws), K, t_graph, rate), file=sys.stderr, flush=True)

    # single rate at each member's fast step (its MPRK step / m, replayed
    # chunk by chunk), one batch per value of m
    t_sr = 0.0
    cs_sr = 0
    sr_final = [None] * len(ws)
    for mval in sorted(set(w.m for w in ws)):
        idx = [i for i, w in enumerate(ws) if w.m == mval]
        restore()
        sb = mprk.Batch([(mprk.config_of_workload(ws[i], flux_bits=32, m=1), tens[i][0], tens[i][1],
                          dts0[i] / mval) for i in idx], exec_mode=mprk.EXEC_GRAPH, tile=best)
        sb.run(1, check_every=0)
        restore()
        t0 = time.perf_counter()
        for h in hist:
            for j, i in enumerate(idx):
                sb.set_dt(j, h[i] / mval)
            sb.run(CH * mval, check_every=CH * mval)
        torch.cuda.synchronize()
        t_sr += time.perf_counter() - t0
        sb.close()
        for i in idx:
            sr_final[i] = (tens[i][0].cpu().numpy(), tens[i][1].cpu().numpy())
            w = ws[i]
            cs_sr += costmodel.sr_cell_stages(w.nx * (w.nz_lower + w.nz_upper), mval, w.base)
    diff = 0.0
    for (a, b), (c, d) in zip(final, sr_final):
        for x, y in ((a, c), (b, d)):
            scale = np.abs(y).max(axis=(1, 2))
            scale[1:3] = max(scale[1], scale[2])
            diff = max(diff, float((np.abs(x - y).max(axis=(1, 2)) / scale).max()))
    restore()
    print("# ensemble single rate: %.3f s, time-to-solution speedup %.3f" % (t_sr, t_sr / t_graph),
          file=sys.stderr, flush=True)
    eq = None if args.no_accuracy else ensemble_equal_error(args, torch, ws, tens, restore, dts0, best)
    return {
        "workload": "%d uneven two-domain members (nx 128..512, nz 64..256, m in {2,4,8}), MPRK2, "
                    "FP32 flux / FP64 state, adaptive steps every %d" % (len(ws), CH),
        "cells": cells, "steps": K, "cell_stages_per_step": cs,
        "value": max(rate, cs * K / t_launch), "unit": "cell-stage updates/s",
        "best_mode": "graph" if rate >= cs * K / t_launch else "launch",
        "seconds_graph": t_graph, "seconds_launch": t_launch, "status_bad": bad,
        "tile": mprk.TILE_NAMES[best],
        "tuner_ms_per_step": {mprk.TILE_NAMES[k]: v for k, v in enumerate(tuner_ms)},
        "modes": {"graph": rate, "launch": cs * K / t_launch,
                  "persistent": cs * K / t_pers, "steps_persistent": K},
        "single_rate": {"seconds": t_sr, "value": cs_sr * K / t_sr,
                        "time_to_solution_speedup": t_sr / t_graph,
                        "max_rel_diff_mprk_vs_single_rate": diff},
        "equal_error": eq,
    }


def ensemble_equal_error(args, torch, ws, tens, restore, dts0, tile):
    """Equal-error comparison per ensemble member, with fixed steps (each
    member's initial stable step dt_i) over H slow steps: MPRK at dt_i/k
    (k = 1, 2, 4), single rate at dt_i/m_i, and a single-rate reference at
    dt_i/(16 m_i), all with FP64 fluxes (the time-discretization error of the
    smallest-amplitude members is below the FP32 flux rounding).  Member i
    matches single rate's error at MPRK refinement k_i (log-log interpolation
    of its errors in k); the batch's MPRK time at equal error is the k = 1
    batch time with each member's work scaled by its k_i, against the measured
    single-rate batch time."""
    from paper_2202_11890_amd import costmodel, mprk

    H, R = 40, 16

    def batch_run(m_of, step_of, nsteps, idx):
        restore()
        b = mprk.Batch([(mprk.config_of_workload(ws[i], m=m_of(i)), tens[i][0], tens[i][1], step_of(i))
                        for i in idx], exec_mode=mprk.EXEC_LAUNCH, tile=tile)
        b.run(1, check_every=0)
        restore()
        t0 = time.perf_counter()
        st = b.run(nsteps, check_every=nsteps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        b.close()
        return el, sum(x["status"] for x in st), {i: (tens[i][0].cpu().numpy(), tens[i][1].cpu().numpy())
                                                  for i in idx}

    allm = list(range(len(ws)))
    groups = {}
    for i, w in enumerate(ws):
        groups.setdefault(w.m, []).append(i)
    ref, sr1, t_sr, bad = {}, {}, 0.0, 0
    for mval, idx in sorted(groups.items()):
        _, b_, q = batch_run(lambda i: 1, lambda i: dts0[i] / (mval * R), H * mval * R, idx)
        ref.update(q)
        bad += b_
        t, b_, q = batch_run(lambda i: 1, lambda i: dts0[i] / mval, H * mval, idx)
        sr1.update(q)
        t_sr += t
        bad += b_

    def err(i, q):
        w = ws[i]
        return float(l2(w.dx, (w.dz_lower, w.dz_upper), [q[0] - ref[i][0], q[1] - ref[i][1]])[0])

    ks = (1, 2, 4)
    mp_err = {i: [] for i in allm}
    mp_t = []
    for k in ks:
        t, b_, q = batch_run(lambda i: ws[i].m, lambda i: dts0[i] / k, H * k, allm)
        mp_t.append(t)
        bad += b_
        for i in allm:
            mp_err[i].append(err(i, q[i]))
    restore()
    cs, kstar, hows, ratio = [], [], [], []
    for i, w in enumerate(ws):
        nF, nB, nS = costmodel.partition_counts(w.nx, w.nz_lower, w.nz_upper, w.n_buffer)
        cs.append(costmodel.mprk_cell_stages(nF, nB, nS, w.m, w.base))
        e_sr = err(i, sr1[i])
        k_i, how = time_at_error(mp_err[i], ks, e_sr)
        kstar.append(k_i)
        hows.append(how)
        ratio.append(mp_err[i][0] / e_sr)
    cs = np.array(cs, dtype=np.float64)
    kstar = np.array(kstar)
    t_mprk_eq = mp_t[0] * float((cs * kstar).sum() / cs.sum())
    out = {
        "protocol": "fixed steps, %d slow steps of each member's stable dt; MPRK at dt/k, k = 1, 2, 4; "
                    "single rate at dt/m; reference single rate at dt/(%d m); FP64 fluxes; matched per "
                    "member on the density L2 error" % (H, R),
        "seconds_mprk": dict(zip(("k1", "k2", "k4"), mp_t)),
        "seconds_single_rate": t_sr,
        "seconds_mprk_at_equal_error": t_mprk_eq,
        "equal_error_speedup": t_sr / t_mprk_eq,
        "fixed_step_speedup": t_sr / mp_t[0],
        "member_refinement_for_equal_error": {"median": float(np.median(kstar)), "min": float(kstar.min()),
                                              "max": float(kstar.max())},
        "member_error_ratio_mprk_over_sr": {"median": float(np.median(ratio)), "min": float(min(ratio)),
                                            "max": float(max(ratio))},
        "members_extrapolated": int(sum(h == "extrapolated" for h in hows)),
        "members_capped": int(sum(h == "capped" for h in hows)),
        "status_bad": bad,
    }
    print("# equal error per member (%d members): single rate %.3f s, MPRK at equal error %.3f s (speedup %.3f); "
          "median refinement %.2f, median error ratio %.1f" % (
              len(ws), t_sr, t_mprk_eq, t_sr / t_mprk_eq, np.median(kstar), np.median(ratio)),
          file=sys.stderr, flush=True)
    return out


def leg_3d(args, torch, dev):
    """The 3D workload (two stacked 256x256x128 domains, dz_fast = dz_slow/4,
    MPRK3 m = 4, FP32 flux / FP64 state): rate, per-launch kernel time from
    HIP events around every stage launch, algorithmic HBM bandwidth."""
    from paper_2202_11890_amd import costmodel, inputs, mprk

    w = inputs.large3d()
    K = args.steps_3d if args.steps_3d is not None else w.steps
    ql, qu = inputs.initial_state3(w)
    tl0, tu0 = torch.from_numpy(ql).to(dev), torch.from_numpy(qu).to(dev)
    tl, tu = tl0.clone(), tu0.clone()
    sol = mprk.Solver(mprk.config3_of_workload(w, flux_bits=args.flux_3d), tl, tu)
    dt = sol.stable_dt(w.cfl, w.dnum)
    sol.run(dt, 2)
    tl.copy_(tl0)
    tu.copy_(tu0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = sol.run(dt, K, check_every=args.check_every)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    sol.profile(True)
    for _ in range(5):
        sol.step(dt)
    k_ms, k_n = sol.profile_take()
    sol.profile(False)
    sol.close()
    plane = w.nx * w.ny
    nF, nB, nS = w.nz_lower * plane, w.n_buffer * plane, (w.nz_upper - w.n_buffer) * plane
    cs = costmodel.mprk_cell_stages(nF, nB, nS, w.m, w.base)
    # 5 FP64 components: read Q_j, read U except at stage 1, write Q_j+1
    bytes_step = 40.0 * (3.0 - 1.0 / w.base) * cs
    per_launch = bytes_step / (w.m * w.base)
    avg = k_ms * 1e-3 / k_n
    gbs = per_launch / avg / 1e9
    # FP32 fluxes run the z-marching kernel, FP64 fluxes the brick kernel; the
    # counter summary covers the FP32-flux kernel only
    kname = "march_kernel3" if args.flux_3d == 32 else "stage_kernel3"
    traffic = traffic_from_profiles("large3d", kname) if args.flux_3d == 32 else None
    print("# 3d: %d steps, %.3f ms/step, %.3e cell-stage/s, stage kernel %.1f us, %.0f GB/s" % (
        K, 1e3 * t / K, cs * K / t, avg * 1e6, gbs), file=sys.stderr, flush=True)
    return {
        "workload": w.name + ", FP%d flux / FP64 state, dz_fast = dz_slow/4" % args.flux_3d,
        "value": cs * K / t, "unit": "cell-stage updates/s", "steps": K, "ms_per_step": 1e3 * t / K,
        "dt": dt, "status": st["status"], "cell_stages_per_step": cs,
        "stage_kernel": {"kernel": kname, "avg_launch_us_bracketed": avg * 1e6,
                         "algorithmic_bytes_per_launch": int(per_launch),
                         "achieved_gbs": gbs, "frac_of_8tbs": gbs / HBM_PEAK_GBS,
                         "traffic": traffic,
                         "traffic_gbs": None if traffic is None else round(traffic / avg / 1e9, 1)},
    }


def serving_leg(args, torch, dev):
    """Continuous-batching server: saturated capacity (every request waiting at
    t = 0), then Poisson arrivals at a fraction of that capacity; p50/p99
    request latency and aggregate cell-stage updates/s."""
    from paper_2202_11890_amd import costmodel, inputs, mprk, serving

    n = args.serving_requests
    budget = 32 << 30

    def make(rate, seed):
        reqs, cs = [], {}
        for i, (t, w) in enumerate(inputs.serving_requests(n, rate, seed)):
            ql, qu = inputs.initial_state(w)
            reqs.append(serving.Request(i, mprk.config_of_workload(w), ql, qu, w.steps,
                                        t if rate > 0 else 0.0))
            nF, nB, nS = costmodel.partition_counts(w.nx, w.nz_lower, w.nz_upper, w.n_buffer)
            cs[i] = costmodel.mprk_cell_stages(nF, nB, nS, w.m, w.base) * w.steps
        return reqs, cs

    reqs, cs = make(1.0, 11)
    for r in reqs:
        r.arrival = 0.0
    srv = serving.Server(dev, budget, max_slots=64, chunk=10)
    t0 = time.perf_counter()
    res = srv.run(reqs)
    sat = serving.summarize(res, cs, time.perf_counter() - t0)
    sat["host_seconds"] = dict(srv.seconds)
    sat["batch_rebuilds"] = srv.rebuilds
    capacity = sat["requests"] / sat["makespan_s"]
    rate = args.serving_load * capacity
    reqs, cs = make(rate, 12)
    srv = serving.Server(dev, budget, max_slots=64, chunk=10)
    t0 = time.perf_counter()
    res = srv.run(reqs)
    load = serving.summarize(res, cs, time.perf_counter() - t0)
    load["arrival_rate_per_s"] = rate
    load["mean_active"] = float(np.mean([a for _, a, _ in srv.log])) if srv.log else 0.0
    load["batch_rebuilds"] = srv.rebuilds
    load["host_seconds"] = dict(srv.seconds)
    print("# serving: capacity %.1f req/s (%.3e cell-stage/s); at %.1f req/s p50 %.3f s p99 %.3f s" % (
        capacity, sat["cell_stage_updates_per_s"], rate, load["latency_s"]["p50"],
        load["latency_s"]["p99"]), file=sys.stderr, flush=True)
    print("# serving saturated: %d rebuilds, seconds %s" % (
        sat["batch_rebuilds"], {k: round(v, 3) for k, v in sat["host_seconds"].items()}),
        file=sys.stderr, flush=True)
    eq = None
    if not args.no_accuracy:
        # Equal error per request, on the first 16 requests of the saturated
        # set (the same study as the ensemble's).
        sample = [w for _, w in inputs.serving_requests(16, 1.0, 11)]
        tens = [(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev))
                for a, b in (inputs.initial_state(w) for w in sample)]
        keep = [(a.clone(), b.clone()) for a, b in tens]

        def restore():
            for (a, b), (c, d) in zip(tens, keep):
                a.copy_(c)
                b.copy_(d)
            torch.cuda.synchronize()

        probe = mprk.Batch([(mprk.config_of_workload(w), a, b, 1.0) for w, (a, b) in zip(sample, tens)])
        dts0 = probe.stable_dts(0.5, 0.25)
        probe.close()
        eq = ensemble_equal_error(args, torch, sample, tens, restore, dts0, None)
    return {
        "workload": "%d requests, nx log-uniform 64..1024 (nz = nx/2), 50..500 slow steps, m in {2,4}, "
                    "MPRK2, FP64; budget %d GiB, 64 slots, 10-step chunks" % (n, budget >> 30),
        "saturated": sat, "capacity_requests_per_s": capacity, "poisson": load,
        "equal_error": eq,
    }


if __name__ == "__main__":
    main()
