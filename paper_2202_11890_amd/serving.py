"""Serving loop with continuous batching over the batch C ABI.

Requests (a two-domain problem, its initial state and a number of slow
steps) arrive over time.  The server keeps every admitted request's state
resident in device memory and advances all of them together as one batch
(``mprk_batch_*``), a chunk of slow steps at a time.  Between chunks,
finished requests leave (their state is copied to pinned host memory on a
copy stream while the next chunk runs, and their memory is released when the
copy completes) and requests that have arrived are admitted while the device
memory budget (the states held, plus the workspace of the batch that the
admission would make, ``mprk_batch_workspace_bytes``) and the slot count
allow, so new work joins work already on the device.

A request's arithmetic is that of a batch member: it does not depend on what
else is in the batch or on how its steps are split into chunks (each member
keeps the fixed slow step computed from its own initial state), so every
result is bit-identical to the same request run alone.

All computation runs in the HIP library; this module schedules.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, List, Optional

import numpy as np

from . import mprk


@dataclasses.dataclass
class Request:
    rid: int
    cfg: "mprk.mprk_config"
    q_lower: np.ndarray            # initial state, float64 [4, nz_lower, nx]
    q_upper: np.ndarray
    steps: int                     # slow steps to run
    arrival: float = 0.0           # seconds after the server starts
    dt: Optional[float] = None     # slow step (None: the stable-step rule of its initial state)
    cell_stages_per_step: int = 0  # for the throughput figure (optional)


@dataclasses.dataclass
class Result:
    rid: int
    q_lower: np.ndarray
    q_upper: np.ndarray
    dt: float
    steps: int
    arrival: float
    admitted: float
    finished: float
    status: int

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def state_bytes(cfg) -> int:
    """Device bytes of a request's two state arrays."""
    return 8 * 4 * cfg.nx * (cfg.nz_lower + cfg.nz_upper)


def batch_bytes(cfgs) -> int:
    """Device bytes of the workspace of a batch of these configurations, as
    mprk.Batch allocates it (mprk_batch_workspace_bytes plus alignment
    slack).  A batch's workspace is not the sum of its members' one-member
    workspaces (its launch tables grow with the largest m*s times the number
    of members), so admission asks for the whole prospective batch."""
    if not cfgs:
        return 0
    probes = []
    base = 1 << 20
    for cfg in cfgs:
        n = state_bytes(cfg)
        probes.append(mprk.mprk_member(cfg, base, base + n // 2, 1.0))
        base += n
    return mprk.mprk_batch_workspace_bytes(probes) + 256


def footprint(cfg) -> int:
    """Device bytes of a request alone: its states and a one-member batch."""
    return state_bytes(cfg) + batch_bytes([cfg])


class _Active:
    __slots__ = ("req", "ql", "qu", "dt", "done", "admitted", "bytes")

    def __init__(self, req, ql, qu, dt, admitted, nbytes):
        self.req, self.ql, self.qu, self.dt = req, ql, qu, dt
        self.done = 0
        self.admitted = admitted
        self.bytes = nbytes


class Server:
    """Continuous-batching server.

    budget_bytes : device memory the admitted requests may hold.
    max_slots    : most requests in the batch at once.
    chunk        : slow steps between scheduling points.
    cr, dn       : step rule for requests without dt (mprk_stable_dt).
    """

    def __init__(self, device, budget_bytes: int, max_slots: int = 64, chunk: int = 10,
                 exec_mode: int = mprk.EXEC_LAUNCH, tile: Optional[int] = None, cr: float = 0.5,
                 dn: float = 0.25, clock: Callable[[], float] = time.perf_counter):
        import torch

        self.torch = torch
        self.device = device
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.chunk = int(chunk)
        self.exec_mode = exec_mode
        self.tile = tile
        self.cr, self.dn = cr, dn
        self.clock = clock
        self.batch = None
        self.dirty = False
        self.active: List[_Active] = []
        self.used = 0                # state bytes of admitted and outgoing requests
        self.ws_bytes = 0            # workspace bytes of the current batch
        self.rebuilds = 0
        self.log = []                # (time, active count, device bytes held: states and
                                     # the batch workspace) after each chunk
        # host seconds spent admitting (copies in), rebuilding the batch (with
        # the step rule of new requests), running chunks and retiring (copies out)
        self.seconds = {"admit": 0.0, "rebuild": 0.0, "run": 0.0, "retire": 0.0}
        # finished requests whose states are on their way to pinned host
        # memory (a copy stream overlaps the copies with the next chunk)
        self.outgoing = []
        self.copy_stream = None      # created at the first retirement

    # -- helpers -----------------------------------------------------------
    def _rebuild(self):
        if self.batch is not None:
            self.batch.close()
            self.batch = None
        self.ws_bytes = 0
        if self.active:
            self.batch = mprk.Batch([(a.req.cfg, a.ql, a.qu, a.dt if a.dt is not None else 1.0)
                                     for a in self.active], exec_mode=self.exec_mode, tile=self.tile)
            self.ws_bytes = batch_bytes([a.req.cfg for a in self.active])
            self.rebuilds += 1
            # Step rule for requests admitted without one, from their initial
            # state: one batched reduction for all of them (each member's
            # reduction is its own, so the step is the one it would get alone).
            if any(a.dt is None for a in self.active):
                dts = self.batch.stable_dts(self.cr, self.dn)
                for i, a in enumerate(self.active):
                    if a.dt is None:
                        a.dt = dts[i]
                        self.batch.set_dt(i, a.dt)
        self.dirty = False

    def _copy_out(self, a, first):
        """Start copying a finished request's state to host memory: (lower,
        upper, completion event, or None when the copy is already done)."""
        torch = self.torch
        if torch.device(self.device).type != "cuda":
            return a.ql.clone(), a.qu.clone(), None
        if first:
            if self.copy_stream is None:
                self.copy_stream = torch.cuda.Stream(self.device)
            self.copy_stream.wait_stream(torch.cuda.current_stream(self.device))
        hl = torch.empty(tuple(a.ql.shape), dtype=a.ql.dtype, pin_memory=True)
        hu = torch.empty(tuple(a.qu.shape), dtype=a.qu.dtype, pin_memory=True)
        with torch.cuda.stream(self.copy_stream):
            hl.copy_(a.ql, non_blocking=True)
            hu.copy_(a.qu, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.copy_stream)
        return hl, hu, ev

    def _drain(self, results, t0, block=False):
        """Turn finished copies into results (all of them when block)."""
        keep = []
        for a, hl, hu, ev, status in self.outgoing:
            if block and ev is not None:
                ev.synchronize()
            if block or ev is None or ev.query():
                results.append(Result(a.req.rid, hl.numpy(), hu.numpy(), a.dt, a.done, a.req.arrival,
                                      a.admitted, self.clock() - t0, status))
                self.used -= a.bytes
            else:
                keep.append((a, hl, hu, ev, status))
        self.outgoing = keep

    # -- main loop ---------------------------------------------------------
    def run(self, requests: List[Request]) -> List[Result]:
        torch = self.torch
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in pending:
            if footprint(r.cfg) > self.budget:
                raise ValueError("request %d needs more memory than the whole budget" % r.rid)
        results: List[Result] = []
        t0 = self.clock()
        while pending or self.active or self.outgoing:
            self._drain(results, t0)
            now = self.clock() - t0
            # admit, in arrival order, while memory and slots allow
            ta = self.clock()
            while pending and pending[0].arrival <= now and len(self.active) < self.max_slots:
                r = pending[0]
                need = state_bytes(r.cfg)
                # The new states are allocated while the current batch (and
                # its workspace) still exists; the rebuild then frees that
                # workspace before allocating the new batch's.
                ws = batch_bytes([a.req.cfg for a in self.active] + [r.cfg])
                if self.used + need + max(ws, self.ws_bytes) > self.budget:
                    break
                pending.pop(0)
                ql = torch.from_numpy(np.ascontiguousarray(r.q_lower)).to(self.device)
                qu = torch.from_numpy(np.ascontiguousarray(r.q_upper)).to(self.device)
                # dt None: set at the next rebuild, from this initial state
                self.active.append(_Active(r, ql, qu, r.dt, self.clock() - t0, need))
                self.used += need
                self.dirty = True
            self.seconds["admit"] += self.clock() - ta
            if not self.active:
                if self.outgoing:
                    self._drain(results, t0, block=True)
                    continue
                if not pending:
                    break
                # idle until the next arrival
                wait = pending[0].arrival - (self.clock() - t0)
                if wait > 0:
                    time.sleep(wait)
                continue
            if self.dirty or self.batch is None:
                tb = self.clock()
                self._rebuild()
                self.seconds["rebuild"] += self.clock() - tb
            # advance everyone by a chunk, or less so that the first request
            # to finish ends exactly at its step count
            k = min(self.chunk, min(a.req.steps - a.done for a in self.active))
            tr = self.clock()
            rc, stats = self.batch.run_status(k)
            self.seconds["run"] += self.clock() - tr
            if rc not in (mprk.OK, mprk.ENONFINITE):
                raise mprk.MprkError(rc, "mprk_batch_run")
            for a in self.active:
                a.done += k
            # retire finished requests, and requests whose state went bad:
            # their states are copied to pinned host memory on the copy
            # stream, after this chunk, while the next chunk computes; their
            # device memory counts against the budget until the copy is done
            tr = self.clock()
            keep = []
            first = True
            for a, st in zip(self.active, stats):
                if a.done >= a.req.steps or st["status"]:
                    hl, hu, ev = self._copy_out(a, first)
                    first = False
                    self.outgoing.append((a, hl, hu, ev, st["status"]))
                else:
                    keep.append(a)
            if len(keep) != len(self.active):
                self.active = keep
                self.dirty = True
            self.seconds["retire"] += self.clock() - tr
            self.log.append((self.clock() - t0, len(self.active), self.used + self.ws_bytes))
        if self.batch is not None:
            self.batch.close()
            self.batch = None
        return results


def summarize(results: List[Result], cell_stages: dict, makespan: float) -> dict:
    """p50 / p99 latency and aggregate cell-stage updates/s of a served run."""
    lat = np.array([r.latency for r in results])
    total = sum(cell_stages[r.rid] for r in results)
    return {
        "requests": len(results),
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "mean": float(lat.mean())},
        "makespan_s": makespan,
        "cell_stage_updates_per_s": total / makespan if makespan > 0 else 0.0,
        "bad": int(sum(r.status for r in results)),
    }
