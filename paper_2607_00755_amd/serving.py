"""Continuous-batching request loop for parameter-scan solves.

Each request is one solve of the expanding-universe equation (adaptive Heun in
u = ln a with radiation-era Hubble drift, projected collision operator) for
its own coupling lambda, initial bimodal distribution and end time, on the
grid of its size N.  The loop

* admits requests as they arrive, as long as their N-group has a free slot
  and the device-memory budget holds the group's kernel tensors plus the slot
  state (admission by footprint; a group's tensors are built when its first
  request is admitted and freed when it drains);
* keeps every solve's state resident on the device in a stepper slot;
* advances all running slots of an N-group together, so that each iteration
  is one batched evaluation per group, each group on its own stream;
* retires finished solves, records arrival-to-result latency, and frees the
  slot for the next arrival;
* cancels requests on demand (`Server.cancel`): a waiting request is dropped,
  a running one has its slot released on its group's stream (ordered after
  the work already enqueued there), and the other solves of the group go on
  unchanged.

Request status: 1 reached its end time, 2 stopped at the step cap before it
(reported as truncated, not as completed), -1 non-finite state, -2 step-size
underflow, -4 refused (does not fit the memory budget), -5 cancelled.

All numerical work runs in libkxg; this module only schedules.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import inputs, kxg


@dataclass
class Request:
    rid: int
    solve: inputs.Solve
    arrival: float                 # seconds after the start of the run
    admitted: float = -1.0
    finished: float = -1.0
    steps: int = 0
    rejected: int = 0
    status: int = 0
    result: Optional[np.ndarray] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def u_end_of(t_end_hubble: float) -> float:
    """Radiation era: a/a_i = sqrt(2 H_i t), so u_end = ln(a/a_i) at t_end."""
    return 0.5 * math.log(2.0 * t_end_hubble)


@dataclass
class Group:
    n: int
    kernel: kxg.Kernel
    stepper: kxg.Stepper
    stream: object
    b_cap: int
    free: List[int] = field(default_factory=list)
    slots: Dict[int, Request] = field(default_factory=dict)
    p: Optional[np.ndarray] = None
    bytes: int = 0
    iters: int = 0
    batch_sum: int = 0
    event: object = None          # completion event of the last enqueued chunk
    busy: bool = False


class Server:
    """Continuous-batching loop over libkxg steppers, one group per grid size."""

    def __init__(self, prec: int = kxg.F32, b_cap: int = 128, budget_bytes: int = 8 << 30,
                 iters_per_tick: int = 64, pmin: float = inputs.SERVING_PMIN,
                 pmax: float = inputs.SERVING_PMAX, rtol: float = 1e-6,
                 keep_results: bool = False, max_steps: int = 200000):
        import torch
        self.torch = torch
        self.prec = prec
        self.b_cap = b_cap
        self.budget = int(budget_bytes)
        self.iters_per_tick = iters_per_tick
        self.pmin, self.pmax = pmin, pmax
        self.rtol = rtol
        self.keep_results = keep_results
        self.max_steps = max_steps
        self.groups: Dict[int, Group] = {}
        self.used_bytes = 0
        self.refused = 0
        self._cancel: set = set()
        self._held: Dict[int, int] = {}

    # ---------------------------------------------------------------- memory
    def slot_bytes(self, n: int) -> int:
        # stepper state (x, operator input, k1, x*) + loss-rate row + slot
        # records; used for the estimate before a group is built (the
        # stepper's evaluation workspace is charged once it exists)
        return 5 * n * 8 + 2 * 96 + 8

    def group_bytes(self, n: int) -> int:
        g = self.groups.get(n)
        if g is not None:
            return g.bytes
        return 0

    def _open_group(self, n: int) -> Optional[Group]:
        p = inputs.log_grid(n, self.pmin, self.pmax)
        # estimate before building, of the peak during the build: the dense
        # FP64 tensor (released at the end of a lean build unless FP64 is
        # served), the packed operand (at most the full packing) and the
        # slot state; after the build the handle's real holding is charged
        nb = (n + 15) // 16
        packed = ((n + 31) // 32) * nb * (nb + 1) // 2 * 16 * 512 * 4
        est = 8 * n ** 3 + packed + self.b_cap * self.slot_bytes(n)
        est = max(est, self._held.get(n, 0))     # what this group held when last built
        if self.used_bytes + est > self.budget:
            return None
        torch = self.torch
        stream = torch.cuda.Stream()
        ker = kxg.Kernel(p, precs=(self.prec,), b_cap=self.b_cap, stream=stream, lean=True)
        st = kxg.Stepper(ker, kind=kxg.HEUN, prec=self.prec, b_cap=self.b_cap,
                         expansion=kxg.EXP_RADIATION, rtol=self.rtol)
        real = ker.bytes(-1) + st.bytes()
        self._held[n] = real
        if self.used_bytes + real > self.budget:
            # the estimate did not include the evaluation workspaces: the
            # group does not fit after all
            del st, ker
            return None
        g = Group(n, ker, st, stream, self.b_cap, free=list(range(self.b_cap)), p=p, bytes=real,
                  event=torch.cuda.Event())
        self.groups[n] = g
        self.used_bytes += real
        return g

    def _close_group(self, n: int) -> None:
        g = self.groups.pop(n)
        g.stream.synchronize()
        self.used_bytes -= g.bytes
        del g

    # ---------------------------------------------------------------- loop
    def _admit(self, req: Request, now: float) -> bool:
        n = req.solve.n
        g = self.groups.get(n)
        if g is None:
            g = self._open_group(n)
            if g is None:
                return False
        if not g.free:
            return False
        slot = min(g.free)
        g.free.remove(slot)
        torch = self.torch
        with torch.cuda.stream(g.stream):
            f0 = torch.tensor(req.solve.f0(g.p), device="cuda")
            g.stepper.set(slot, f0, lam=req.solve.lam, t_end=u_end_of(req.solve.t_end),
                          dt=1e-3, h_i=0.0, max_steps=self.max_steps, stream=g.stream)
        g.slots[slot] = req
        req.admitted = now
        return True

    def _retire(self, g: Group, now: float, done: List[Request]) -> None:
        states = g.stepper.query(stream=g.stream)
        for slot, req in list(g.slots.items()):
            s = states[slot]
            if s["status"] == 0:
                continue
            req.finished = now
            req.steps, req.rejected, req.status = s["steps"], s["rejected"], s["status"]
            if self.keep_results:
                with self.torch.cuda.stream(g.stream):
                    out = self.torch.empty(g.n, dtype=self.torch.float64, device="cuda")
                    g.stepper.get(slot, out=out, stream=g.stream)
                    req.result = out.cpu().numpy()
            g.stepper.release(slot, stream=g.stream)
            del g.slots[slot]
            g.free.append(slot)
            done.append(req)

    def cancel(self, rid: int) -> None:
        """Cancel request `rid` (its index in the list given to run): it is
        taken out at the next turn of the loop, wherever it is by then."""
        self._cancel.add(int(rid))

    def _apply_cancellations(self, waiting: List[Request], now: float,
                             done: List[Request]) -> List[Request]:
        if not self._cancel:
            return waiting
        keep = []
        for req in waiting:
            if req.rid in self._cancel:
                self._cancel.discard(req.rid)
                req.status, req.finished = -5, now
                done.append(req)
            else:
                keep.append(req)
        for g in self.groups.values():
            for slot, req in list(g.slots.items()):
                if req.rid not in self._cancel:
                    continue
                self._cancel.discard(req.rid)
                # enqueued on the group's stream, after the chunk in flight
                g.stepper.release(slot, stream=g.stream)
                del g.slots[slot]
                g.free.append(slot)
                req.status, req.finished = -5, now
                done.append(req)
        return keep

    def run(self, requests: List[inputs.Solve], realtime: bool = True,
            on_tick=None) -> List[Request]:
        """Serve the requests (arrival times in seconds from the start)."""
        torch = self.torch
        pending = [Request(i, s, s.arrival) for i, s in enumerate(requests)]
        pending.sort(key=lambda r: r.arrival)
        waiting: List[Request] = []
        done: List[Request] = []
        t0 = time.perf_counter()
        nxt = 0
        while len(done) < len(pending):
            now = time.perf_counter() - t0
            while nxt < len(pending) and (pending[nxt].arrival <= now or not realtime):
                waiting.append(pending[nxt])
                nxt += 1
            waiting = self._apply_cancellations(waiting, now, done)
            # admission (FIFO, later requests may pass a blocked one of another N)
            still = []
            for req in waiting:
                if not self._admit(req, now):
                    still.append(req)
            waiting = still
            active = [g for g in self.groups.values() if g.slots]
            if not active:
                if waiting and not any(g.slots for g in self.groups.values()):
                    # nothing running and nothing fits: free idle groups, else refuse
                    idle = [n for n, g in self.groups.items() if not g.slots]
                    if idle:
                        for n in idle:
                            self._close_group(n)
                        continue
                    req = waiting.pop(0)
                    req.status, req.finished = -4, now
                    self.refused += 1
                    done.append(req)
                    continue
                if nxt < len(pending) and realtime:
                    time.sleep(max(0.0, min(pending[nxt].arrival - now, 0.002)))
                continue
            # Each group runs on its own stream and is re-fed as soon as its own
            # previous chunk of iterations has completed (non-blocking poll), so
            # fast groups never wait for slow ones.
            progressed = False
            for g in active:
                if g.busy:
                    if not g.event.query():
                        continue
                    g.busy = False
                    self._retire(g, time.perf_counter() - t0, done)
                    progressed = True
                if g.slots:
                    g.stepper.advance(self.iters_per_tick, stream=g.stream)
                    g.iters += self.iters_per_tick
                    g.batch_sum += self.iters_per_tick * len(g.slots)
                    g.event.record(g.stream)
                    g.busy = True
                    progressed = True
            if not progressed:
                time.sleep(5e-5)
            # release the tensors of groups that drained and are not needed
            for n in [n for n, g in self.groups.items() if not g.slots and not g.busy]:
                if not any(r.solve.n == n for r in waiting) and self.used_bytes > self.budget // 2:
                    self._close_group(n)
            if on_tick:
                on_tick(len(done), len(pending))
        if self.groups:
            torch.cuda.synchronize()
        return done

    def stats(self, done: List[Request], warm: int = 0) -> dict:
        """Latency and throughput over the requests from `warm` on.  Only
        solves that reached their end time (status 1) count as completed;
        step-capped ones (2) are truncated, cancelled (-5) and refused (-4)
        ones are counted apart, everything else is failed."""
        mine = [r for r in done if r.rid >= warm]
        ok = [r for r in mine if r.status == 1]
        lat = np.array([r.latency for r in ok]) if ok else np.array([np.nan])
        span = (max(r.finished for r in ok) - min(r.arrival for r in ok)) if ok else float("nan")
        # queue build-up: median latency of the last quarter of the arrivals
        # over that of the first quarter (about 1 while the loop keeps up)
        by_arr = sorted(ok, key=lambda r: r.arrival)
        qn = len(by_arr) // 4
        growth = (float(np.median([r.latency for r in by_arr[-qn:]])) /
                  float(np.median([r.latency for r in by_arr[:qn]]))) if qn >= 4 else float("nan")
        # keeping up: the completion rate while requests still arrive (from
        # one median latency after the first arrival to the last arrival)
        # over the arrival rate; about 1 below capacity, capacity / offered
        # rate above it, where the backlog grows until the last arrival
        keep_up = float("nan")
        arr = sorted(r.arrival for r in mine)
        if len(arr) >= 8 and ok:
            t0, ta = arr[0], arr[-1]
            w0 = t0 + float(np.median(lat))
            if ta - w0 > 0 and ta > t0:
                out_rate = sum(1 for r in ok if w0 <= r.finished <= ta) / (ta - w0)
                keep_up = out_rate / ((len(arr) - 1) / (ta - t0))
        return {
            "completed": len(ok),
            "truncated": sum(1 for r in mine if r.status == 2),
            "failed": sum(1 for r in mine if r.status not in (1, 2, -4, -5)),
            "refused": sum(1 for r in mine if r.status == -4),
            "cancelled": sum(1 for r in mine if r.status == -5),
            "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)),
            "solves_per_s": len(ok) / span if span and span > 0 else float("nan"),
            "queue_growth": growth,
            "keep_up": keep_up,
            "mean_steps": float(np.mean([r.steps for r in ok])) if ok else float("nan"),
            "max_steps": int(max(r.steps for r in ok)) if ok else 0,
            "mean_batch": {n: g.batch_sum / max(g.iters, 1) for n, g in self.groups.items()},
            "per_n": {str(n): {"completed": len(rs),
                               "p50_s": float(np.percentile([r.latency for r in rs], 50)),
                               "p99_s": float(np.percentile([r.latency for r in rs], 99)),
                               "mean_steps": float(np.mean([r.steps for r in rs])),
                               "max_steps": int(max(r.steps for r in rs))}
                      for n in sorted({r.solve.n for r in ok})
                      for rs in [[r for r in ok if r.solve.n == n]]},
        }
