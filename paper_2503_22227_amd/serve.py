"""Continuous-batching server for encrypted private-table queries.

The paper's query stage (section IV) runs one query after another on the GPU,
with keys and tables kept resident.  This server admits queries continuously:

* arrivals go to a FIFO admission queue;
* a query is admitted when a stream slot is free and its HBM footprint (peak
  live ciphertexts of its op list plus its slot's key-switching workspace)
  fits in what the budget has left; keys and tables are resident and counted
  apart;
* every scheduler tick enqueues the next ops of every admitted query on that
  query's own stream (at most ``depth`` chunks in flight per query), so the
  kernels of different queries overlap on the device; a query that finishes
  releases its slot and budget at once and the next one is admitted;
* latency = arrival to result on the host.

The device work sits behind an executor interface (``start``, ``issue``,
``poll``, ``finish``), and time behind ``clock``/``sleep``, so the scheduler is
tested on the CPU with a fake executor and a synthetic clock.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional


@dataclass
class Request:
    rid: int
    arrival: float                      # seconds after the run starts
    ops: list
    inputs: dict                        # register name -> operand
    outputs: tuple                      # registers to return
    footprint: int                      # bytes while admitted
    admitted: Optional[float] = None
    finished: Optional[float] = None
    result: Optional[dict] = None
    error: Optional[str] = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.finished is None else self.finished - self.arrival


@dataclass
class ServerStats:
    completed: int = 0
    failed: int = 0
    peak_bytes: int = 0
    peak_inflight: int = 0
    makespan: float = 0.0
    latencies: List[float] = field(default_factory=list)

    def percentile(self, p: float) -> float:
        xs = sorted(self.latencies)
        if not xs:
            return float("nan")
        k = min(len(xs) - 1, max(0, int(round(p / 100.0 * (len(xs) - 1)))))
        return xs[k]


class Server:
    def __init__(self, executor, budget_bytes: int, slots: int = 4, ops_per_chunk: int = 16, depth: int = 2,
                 clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.chunk = int(ops_per_chunk)
        self.depth = int(depth)
        self.clock = clock
        self.sleep = sleep

    def run(self, requests: List[Request]) -> ServerStats:
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        queue: deque = deque()
        free_slots = list(range(self.slots))
        inflight: Dict[int, dict] = {}
        used = 0
        st = ServerStats()
        t0 = self.clock()
        while pending or queue or inflight:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            # admission, FIFO: the head waits until it fits
            while queue and free_slots:
                head = queue[0]
                if head.footprint > self.budget:
                    queue.popleft()
                    head.error = "footprint %d exceeds the budget %d" % (head.footprint, self.budget)
                    head.finished = now
                    st.failed += 1
                    continue
                if used + head.footprint > self.budget:
                    break
                queue.popleft()
                slot = free_slots.pop(0)
                try:
                    handle = self.ex.start(head, slot)
                except Exception as e:  # noqa: BLE001 - one failed request must not stop the others
                    head.error = "start: %s" % e
                    head.finished = self.clock() - t0
                    st.failed += 1
                    free_slots.append(slot)
                    continue
                head.admitted = now
                used += head.footprint
                inflight[head.rid] = {"req": head, "slot": slot, "handle": handle, "next": 0, "chunks": 0}
                st.peak_bytes = max(st.peak_bytes, used)
                st.peak_inflight = max(st.peak_inflight, len(inflight))
            progressed = False
            for rid in list(inflight):
                f = inflight[rid]
                req = f["req"]
                try:
                    done_chunks = self.ex.poll(f["handle"])
                    outstanding = f["chunks"] - done_chunks
                    if f["next"] < len(req.ops) and outstanding < self.depth:
                        end = min(len(req.ops), f["next"] + self.chunk)
                        self.ex.issue(f["handle"], f["next"], end)
                        f["next"] = end
                        f["chunks"] += 1
                        progressed = True
                    elif f["next"] >= len(req.ops) and outstanding == 0:
                        req.result = self.ex.finish(f["handle"])
                        req.finished = self.clock() - t0
                        st.completed += 1
                        st.latencies.append(req.latency)
                        used -= req.footprint
                        free_slots.append(f["slot"])
                        del inflight[rid]
                        progressed = True
                except Exception as e:  # noqa: BLE001
                    req.error = "run: %s" % e
                    req.finished = self.clock() - t0
                    st.failed += 1
                    used -= req.footprint
                    free_slots.append(f["slot"])
                    del inflight[rid]
                    progressed = True
            if not progressed:
                nxt = pending[0].arrival - (self.clock() - t0) if (pending and not queue and not inflight) else 0.0
                self.sleep(max(nxt, 0.0) if nxt > 0 else 20e-6)
        st.makespan = self.clock() - t0
        return st


class GpuQueryExecutor:
    """Executor of op lists on the GPU: one torch stream per slot, registers freed
    after their last use, one event per issued chunk."""

    def __init__(self, op_executor, slots: int):
        import torch
        self.torch = torch
        self.opx = op_executor
        self.streams = [torch.cuda.Stream() for _ in range(slots)]

    def start(self, req: Request, slot: int):
        from .pdq import last_uses
        return {"req": req, "slot": slot, "regs": dict(req.inputs), "events": [],
                "last": last_uses(req.ops, req.outputs)}

    def issue(self, h, begin: int, end: int) -> None:
        torch = self.torch
        s = self.streams[h["slot"]]
        req = h["req"]
        with torch.cuda.stream(s):
            for i in range(begin, end):
                op = req.ops[i]
                self.opx.step(op, h["regs"], slot=h["slot"])
                for r in op[2:]:
                    if isinstance(r, str) and h["last"].get(r, -1) <= i and r not in req.outputs:
                        h["regs"].pop(r, None)
            ev = torch.cuda.Event()
            ev.record(s)
        h["events"].append(ev)

    def poll(self, h) -> int:
        n = 0
        for ev in h["events"]:
            if not ev.query():
                break
            n += 1
        return n

    def finish(self, h) -> dict:
        s = self.streams[h["slot"]]
        s.synchronize()
        return {r: h["regs"][r].cpu() for r in h["req"].outputs}
