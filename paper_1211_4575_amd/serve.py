"""Serving: many small particle-in-cell runs (a parameter scan) sharing one GPU by continuous
batching.

Requests arrive over time.  A request is admitted, in arrival order, as soon as a batch slot
is free and the device memory it needs (its mesh and particle arrays plus the library's
scratch, ``pp_workspace_size``) fits the budget.  Its particles are generated in device
memory and the run joins a ``pp_batch``; each batch step advances every member run by one
step of the method with one launch per phase (gather/push/deposit, line solve, sort, field
step), so runs that arrived at different times share the device.  A run leaves the batch
after its last step; its memory goes back to the budget once the device has passed that
step.  Completion times come from GPU events: latency = (device done with the request's last
step) - (arrival).

The scheduler talks to a small backend interface (:class:`DeviceBackend` on the GPU); the
same scheduler logic runs against a simulated device in the CPU tests.
"""
from __future__ import annotations

import math
import threading
import time
from collections import deque
from dataclasses import dataclass, field


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    done: float
    steps: int
    updates: int
    status: str = "ok"
    flags: int = 0
    info: dict = field(default_factory=dict)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def percentile(values, q):
    """q-th percentile (0..100) by linear interpolation between order statistics."""
    v = sorted(values)
    if not v:
        return math.nan
    x = (len(v) - 1) * q / 100.0
    lo = int(math.floor(x))
    hi = min(lo + 1, len(v) - 1)
    return v[lo] + (v[hi] - v[lo]) * (x - lo)


def summarize(results, t_first=None):
    """p50/p99 latency, aggregate updates/s over [first arrival, last completion]."""
    ok = [r for r in results if r.status == "ok"]
    if not ok:
        return dict(completed=0)
    t0 = min(r.arrival for r in results) if t_first is None else t_first
    t1 = max(r.done for r in ok)
    upd = sum(r.updates for r in ok)
    return dict(completed=len(ok), failed=sum(r.status == "failed" for r in results),
                cancelled=sum(r.status == "cancelled" for r in results),
                rejected=sum(r.status == "rejected" for r in results), p50_s=percentile([r.latency for r in ok], 50),
                p99_s=percentile([r.latency for r in ok], 99), makespan_s=t1 - t0,
                updates=upd, updates_per_s=upd / (t1 - t0) if t1 > t0 else math.nan)


class Scheduler:
    """Admission by memory footprint and slot count, continuous batching, completion by event.

    ``max_inflight`` bounds how many batch steps the host enqueues ahead of the device, so
    that a new arrival joins within about that many steps."""

    def __init__(self, backend, mem_budget: int, max_slots: int, max_inflight: int = 2, on_complete=None):
        self.be = backend
        self.on_complete = on_complete  # called with each Result as it completes
        self.mem_budget = int(mem_budget)
        self.max_slots = int(max_slots)
        self.max_inflight = max(1, int(max_inflight))
        self.peak_members = 0
        self.peak_bytes = 0
        self.batch_steps = 0
        self._cancel = set()
        self._cancel_lock = threading.Lock()

    def cancel(self, rid: int):
        """Cancel request ``rid`` (callable from any thread or from on_complete): a pending
        request is dropped, a running one leaves the batch before the next step and is reported
        "cancelled" once the device has finished its last step; the others are unaffected."""
        with self._cancel_lock:
            self._cancel.add(rid)

    def run(self, requests, cancel_after=None):
        """Serve ``requests``; ``cancel_after`` maps rid -> number of steps after which that
        request is cancelled (a budget per request)."""
        be = self.be
        cancel_after = dict(cancel_after or {})
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        active = {}  # rid -> [handle, request, steps left, admitted, bytes]
        inflight = deque()  # (token, entries that finished with that step)
        used = 0
        results = []

        def complete(entries, t_done):
            nonlocal used
            for h, req, left, t_adm, need in entries:
                flags, info = be.retire(h)
                used -= need
                status = "cancelled" if left > 0 else ("ok" if flags == 0 else "failed")
                results.append(Result(req.rid, req.arrival, t_adm, t_done, req.steps - left,
                                      req.updates * (req.steps - left) // max(req.steps, 1), status, flags, info))
                if self.on_complete is not None:
                    self.on_complete(results[-1], len(active))

        def take_cancellations():
            with self._cancel_lock:
                todo, self._cancel = self._cancel, set()
            for rid in todo:
                for i, req in enumerate(pending):
                    if req.rid == rid:
                        del pending[i]
                        results.append(Result(req.rid, req.arrival, math.nan, math.nan, 0, 0, "cancelled"))
                        break
                if rid in active:  # leaves now; reported when the device is past its last step
                    e = active.pop(rid)
                    be.leave(e[0])
                    if inflight:
                        inflight[-1][1].append(e)
                    else:
                        complete([e], be.now())

        be.start()
        while pending or active or inflight:
            take_cancellations()
            now = be.now()
            while pending and pending[0].arrival <= now and len(active) < self.max_slots:
                req = pending[0]
                need = be.footprint(req)
                if need > self.mem_budget:
                    pending.popleft()
                    results.append(Result(req.rid, req.arrival, math.nan, math.nan, req.steps, req.updates,
                                          "rejected", 0, dict(bytes=need)))
                    continue
                if used + need > self.mem_budget:
                    break
                pending.popleft()
                h = be.admit(req)
                used += need
                active[req.rid] = [h, req, req.steps, be.now(), need]
            self.peak_members = max(self.peak_members, len(active))
            self.peak_bytes = max(self.peak_bytes, used)
            if active:
                tok = be.step()
                self.batch_steps += 1
                finished = []
                for rid in list(active):
                    e = active[rid]
                    e[2] -= 1
                    if e[2] == 0:
                        be.leave(e[0])
                        finished.append(e)
                        del active[rid]
                    elif rid in cancel_after and e[1].steps - e[2] >= cancel_after[rid]:
                        self.cancel(rid)
                inflight.append((tok, finished))
                while len(inflight) > self.max_inflight:
                    tok0, fin = inflight.popleft()
                    complete(fin, be.wait(tok0))
                while inflight:
                    t = be.done(inflight[0][0])
                    if t is None:
                        break
                    complete(inflight.popleft()[1], t)
            elif inflight:
                tok0, fin = inflight.popleft()
                complete(fin, be.wait(tok0))
            elif pending:
                be.sleep_until(pending[0].arrival)
        be.finish()
        return sorted(results, key=lambda r: r.rid)


def fifo_one_at_a_time(requests, service_s):
    """Completion times of the requests served one at a time in arrival order, each taking
    ``service_s[rid]`` seconds: start = max(arrival, previous done)."""
    out = []
    t = -math.inf
    for r in sorted(requests, key=lambda r: (r.arrival, r.rid)):
        start = max(r.arrival, t)
        t = start + service_s[r.rid]
        out.append(Result(r.rid, r.arrival, start, t, r.steps, r.updates))
    return sorted(out, key=lambda r: r.rid)


# ---------------------------------------------------------------------------------------------
# GPU backend
# ---------------------------------------------------------------------------------------------
class DeviceBackend:
    """Runs requests through libpp on the current device: split-precision FP32 runs in one
    pp_batch on the current stream, particles generated on the device."""

    SPLIT_BYTES_PER_PARTICLE = 2 * (4 + 3 * 4 + 3 * 4)  # cell, offsets, u; current + sort buffer

    def __init__(self, max_slots: int, relax_tol: float = 1e-8, relax_max_iter: int = 100):
        import torch

        from . import inputs_device as ind
        from . import pp

        self.torch, self.pp, self.ind = torch, pp, ind
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self.stream = torch.cuda.current_stream(self.dev)
        self.relax_tol, self.relax_max_iter = relax_tol, relax_max_iter
        self.batch = pp.pp_batch_create(int(max_slots), self.stream.cuda_stream)
        self.t0 = None
        self.start_ev = None

    # -- requests -> runs --
    def params(self, req, precision=None):
        pp = self.pp
        d = req.dx
        return pp.make_params(req.n, d=(d, d, d), dt=req.cfl * d, shape_order=3, field_order=6, alpha=0.55,
                              precision=pp.PP_PREC_FP32_SPLIT if precision is None else precision,
                              relax_tol=self.relax_tol, relax_max_iter=self.relax_max_iter, rho_background=1.0)

    def footprint(self, req) -> int:
        nc = req.n[0] * req.n[1] * req.n[2]
        mesh = 3 * 3 * nc * 8
        parts = 2 * req.n_per_beam * self.SPLIT_BYTES_PER_PARTICLE
        return mesh + parts + self.pp.pp_workspace_size(self.params(req), req.n_per_beam, 2)

    def make_run(self, req, split=True):
        """A pp.Run of the request (two beams on a quiet lattice), generated on the device."""
        torch, pp = self.torch, self.pp
        npart = req.n_per_beam
        rt = torch.float32 if split else torch.float64
        cells = [torch.empty(npart, dtype=torch.int32, device=self.dev) for _ in range(2)] if split else None
        offs = [torch.empty((3, npart), dtype=rt, device=self.dev) for _ in range(2)]
        us = [torch.empty((3, npart), dtype=rt, device=self.dev) for _ in range(2)]
        self.ind.two_stream_lattice(req.seed, req.wl_id, req.n, req.per_dim, req.v_beam, req.uth,
                                    self.ind.split_mode(split, 3), cells,
                                    [[o[d] for d in range(3)] for o in offs], [[u[d] for d in range(3)] for u in us],
                                    self.stream.cuda_stream)
        species = []
        for s in range(2):
            sp = dict(q=-1.0, m=1.0, w=0.5 / req.ppc, u=us[s])
            if split:
                sp.update(cell=cells[s], off=offs[s])
            else:
                sp.update(pos=offs[s])
            species.append(sp)
        P = self.params(req, None if split else pp.PP_PREC_FP64)
        return pp.Run(P, species, device=self.dev, with_id=False)

    # -- scheduler interface --
    def start(self):
        self.torch.cuda.synchronize(self.dev)
        self.start_ev = self.torch.cuda.Event(enable_timing=True)
        self.start_ev.record(self.stream)
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def admit(self, req):
        run = self.make_run(req, split=True)
        self.pp.pp_batch_add(self.batch, run.handle)
        return run

    def step(self):
        try:
            self.pp.pp_batch_step(self.batch)
        except self.pp.PPError as e:
            # a member's relaxation capped by its relax_max_iter: the step was still taken
            if e.status != self.pp.PP_E_NOCONV:
                raise
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record(self.stream)
        return ev

    def leave(self, run):
        self.pp.pp_batch_remove(self.batch, run.handle)

    def _t(self, ev) -> float:
        return self.start_ev.elapsed_time(ev) / 1e3

    def done(self, ev):
        return self._t(ev) if ev.query() else None

    def wait(self, ev) -> float:
        ev.synchronize()
        return self._t(ev)

    def retire(self, run):
        pp = self.pp
        d = run.diagnostics(pp.PP_DIAG_MOMENTS | pp.PP_DIAG_FIELDS)
        info = dict(kinetic=d.kinetic[0] + d.kinetic[1], field_E=d.field_E, field_Ex=d.field_Ex, field_B=d.field_B,
                    step=d.step)
        run.close()
        return int(d.flags), info

    def sleep_until(self, t):
        dt = t - self.now()
        if dt > 0:
            time.sleep(dt)

    def finish(self):
        self.torch.cuda.synchronize(self.dev)

    def close(self):
        if self.batch is not None:
            self.pp.pp_batch_destroy(self.batch)
            self.batch = None

    # -- one-at-a-time references --
    def step_seconds(self, req, split, steps=3, warmup=1):
        """Measured seconds per step of the request stepped alone (FP64 plain form if not
        split), and the seconds to set it up."""
        torch = self.torch
        torch.cuda.synchronize(self.dev)
        t0 = time.perf_counter()
        run = self.make_run(req, split=split)
        torch.cuda.synchronize(self.dev)
        t_setup = time.perf_counter() - t0
        for _ in range(warmup):
            run.step()
        torch.cuda.synchronize(self.dev)
        t0 = time.perf_counter()
        for _ in range(steps):
            run.step()
        torch.cuda.synchronize(self.dev)
        per = (time.perf_counter() - t0) / steps
        run.close()
        return per, t_setup


def one_at_a_time_reference(backend, requests, split, steps=3):
    """Service time of every request when run alone, from the measured per-step time of each
    distinct (grid, lattice) class times its step count, plus its set-up time; then the
    one-at-a-time FIFO queue over the same arrivals."""
    classes = {}
    for r in requests:
        key = (r.n, r.per_dim)
        if key not in classes:
            classes[key] = backend.step_seconds(r, split=split, steps=steps)
    service = {r.rid: classes[(r.n, r.per_dim)][1] + classes[(r.n, r.per_dim)][0] * r.steps for r in requests}
    res = fifo_one_at_a_time(requests, service)
    per_class = {f"{k[0][0]}x{k[0][1]}x{k[0][2]}/ppc{k[1][0] * k[1][1] * k[1][2]}": round(v[0] * 1e3, 3)
                 for k, v in classes.items()}
    return res, per_class
