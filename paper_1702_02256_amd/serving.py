"""Serving loop for SPIIR banks: continuous batching over several detector streams.

Strain blocks of uneven length arrive per detector stream.  Every stream is
bound to one template bank whose filter state stays resident on the device
across blocks.  The scheduler

* admits banks by HBM footprint (a bank waits until its footprint fits the
  budget left by the banks already admitted);
* keeps, per stream, a FIFO of arrived blocks;
* whenever fewer than ``max_inflight`` batches are on the device, forms the
  next batch from everything that has arrived: the pending blocks of each
  stream are merged into one contiguous request (up to the bank's max block),
  one request per bank, at most ``max_batch`` requests, and submits it as one
  ``spiir_process_batch`` launch sequence on the next of ``n_streams`` device
  streams, so batches overlap on the device;
* records, per block, the time from arrival to the completion of the batch
  that carried it.

Merging never changes results: the library's output does not depend on how a
stream is cut into blocks (bit for bit), nor on which other banks share a
batch.  The ``plain`` policy (one block per launch, no merging, no batching,
one in flight) is the comparison point.

The backend is pluggable: ``HipBackend`` drives libspiir.so; tests drive the
same scheduler with a CPU backend on a virtual clock.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Block:
    stream: int
    seq: int
    start: int          # first sample of the block in its stream
    n: int
    arrival: float      # seconds on the scheduler clock
    done: float = -1.0  # completion time on the scheduler clock

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class Request:
    stream: int
    start: int
    n: int
    blocks: list


@dataclass
class Stats:
    blocks: list = field(default_factory=list)
    batches: int = 0
    requests: int = 0
    filter_samples: int = 0
    wall: float = 0.0
    admitted_at: dict = field(default_factory=dict)

    def latencies(self) -> np.ndarray:
        return np.array([b.latency for b in self.blocks if b.done >= 0])

    def summary(self) -> dict:
        lat = self.latencies() * 1e3
        out = {
            "blocks": len(lat),
            "batches": self.batches,
            "requests": self.requests,
            "filter_samples_per_s": self.filter_samples / self.wall if self.wall > 0 else 0.0,
            "wall_s": self.wall,
        }
        if len(lat):
            out.update({"p50_ms": float(np.percentile(lat, 50)),
                        "p99_ms": float(np.percentile(lat, 99)),
                        "max_ms": float(lat.max()), "mean_ms": float(lat.mean())})
        return out


class Scheduler:
    """Continuous-batching scheduler (see the module docstring)."""

    def __init__(self, backend, tables_per_stream, max_block: int, hbm_budget: int | None = None,
                 policy: str = "batched", max_batch: int = 16, max_inflight: int = 2):
        if policy not in ("batched", "plain"):
            raise ValueError(policy)
        self.be = backend
        self.tables = list(tables_per_stream)
        self.max_block = int(max_block)
        self.policy = policy
        self.max_batch = 1 if policy == "plain" else int(max_batch)
        self.max_inflight = 1 if policy == "plain" else int(max_inflight)
        self.budget = hbm_budget
        self.used = 0
        self.handles = [None] * len(self.tables)
        self.waiting_admission = deque(range(len(self.tables)))
        self.pending = [deque() for _ in self.tables]
        self.inflight = deque()   # (ticket, [Request])
        self.stats = Stats()

    # ---------------------------------------------------------- admission
    def _admit(self, now: float):
        while self.waiting_admission:
            s = self.waiting_admission[0]
            need = self.be.footprint(self.tables[s], self.max_block)
            if self.budget is not None and self.used + need > self.budget:
                break
            self.handles[s] = self.be.create(self.tables[s], self.max_block)
            self.used += need
            self.stats.admitted_at[s] = now
            self.waiting_admission.popleft()

    def release(self, stream: int):
        """Destroy a stream's bank and return its footprint to the budget."""
        h = self.handles[stream]
        if h is not None:
            self.used -= self.be.footprint(self.tables[stream], self.max_block)
            self.be.destroy(h)
            self.handles[stream] = None

    # ---------------------------------------------------------- batching
    def _form_batch(self):
        reqs = []
        order = sorted((s for s in range(len(self.tables)) if self.pending[s]
                        and self.handles[s] is not None),
                       key=lambda s: self.pending[s][0].arrival)
        for s in order:
            if len(reqs) >= self.max_batch:
                break
            q = self.pending[s]
            first = q.popleft()
            blocks, n = [first], first.n
            if self.policy == "batched":
                while q and q[0].start == first.start + n and n + q[0].n <= self.max_block:
                    b = q.popleft()
                    blocks.append(b)
                    n += b.n
            reqs.append(Request(s, first.start, n, blocks))
            if self.policy == "plain":
                break
        return reqs

    def _retire_ready(self, t0: float):
        """Stamp and drop the leading in-flight batches that have completed."""
        while self.inflight:
            ticket, reqs = self.inflight[0]
            if not self.be.done(ticket):
                return
            t = self.be.clock() - t0
            for r in reqs:
                for b in r.blocks:
                    b.done = t
            self.inflight.popleft()

    def _release_finished(self, future_streams):
        """Free the banks of streams with nothing left to process."""
        busy = {r.stream for _, reqs in self.inflight for r in reqs}
        for s in range(len(self.tables)):
            if (self.handles[s] is not None and not self.pending[s] and s not in busy
                    and s not in future_streams):
                self.release(s)

    def run(self, arrivals, release_finished: bool = False) -> Stats:
        """arrivals: Blocks (any order); returns per-block latencies and totals."""
        arrivals = deque(sorted(arrivals, key=lambda b: b.arrival))
        self.stats.blocks = list(arrivals)
        # banks that fit are admitted before the clock starts: creating a bank
        # (planning, upload) is not part of any block's latency
        self._admit(0.0)
        t0 = self.be.clock()
        self.be.start(t0)
        while True:
            now = self.be.clock() - t0
            self._admit(now)
            while arrivals and arrivals[0].arrival <= now:
                b = arrivals.popleft()
                self.pending[b.stream].append(b)
            self._retire_ready(t0)
            if release_finished:
                self._release_finished({b.stream for b in arrivals})
                self._admit(self.be.clock() - t0)
            pend = any(self.pending[s] and self.handles[s] is not None
                       for s in range(len(self.tables)))
            if pend and len(self.inflight) < self.max_inflight:
                reqs = self._form_batch()
                ticket = self.be.submit([(self.handles[r.stream], r.stream, r.start, r.n)
                                         for r in reqs])
                self.inflight.append((ticket, reqs))
                self.stats.batches += 1
                self.stats.requests += len(reqs)
                self.stats.filter_samples += sum(
                    self.be.filter_samples(self.tables[r.stream], r.n) for r in reqs)
                continue
            waiting = any(self.pending[s] for s in range(len(self.tables)))
            if not arrivals and not waiting and not self.inflight:
                break
            next_t = t0 + arrivals[0].arrival if arrivals else None
            if self.inflight:
                self.be.wait(self.inflight[0][0], next_t)
            elif next_t is not None:
                self.be.wait(None, next_t)
            else:
                raise RuntimeError("a bank does not fit the HBM budget and nothing will free it")
        self.stats.wall = self.be.clock() - t0
        return self.stats


def make_arrivals(lengths_times) -> list:
    """[(lengths, times)] per stream -> Block list."""
    out = []
    for s, (lens, times) in enumerate(lengths_times):
        pos = 0
        for i, (n, t) in enumerate(zip(lens, times)):
            out.append(Block(s, i, pos, int(n), float(t)))
            pos += int(n)
    return out


class HipBackend:
    """Drives libspiir.so: device-resident inputs per stream, per-bank output
    buffers, ``n_streams`` device streams used round robin, completion events."""

    def __init__(self, streams_x, n_streams: int = 2, keep_outputs: bool = False, **bank_kw):
        import torch

        from . import spiir as S
        self.torch, self.S = torch, S
        self.x = [torch.from_numpy(np.asarray(x, np.float32)).cuda() for x in streams_x]
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.next_stream = 0
        self.bank_kw = bank_kw
        self.keep = keep_outputs
        self.outputs = {}      # stream -> list of (start, tensor)
        self.zbuf = {}

    def clock(self) -> float:
        return time.perf_counter()

    def start(self, t0: float):
        self.torch.cuda.synchronize()

    def wait(self, ticket, until):
        """Return when `ticket` completes or the clock reaches `until` (either may be None)."""
        while True:
            if ticket is not None and ticket.query():
                return
            if until is not None and time.perf_counter() >= until:
                return

    def footprint(self, tables, max_block) -> int:
        return self.S.spiir_footprint(tables, max_block, **self.bank_kw)

    def filter_samples(self, tables, n) -> int:
        return tables.filter_samples_per_block(n)

    def create(self, tables, max_block):
        bank = self.S.Bank(tables, max_block, **self.bank_kw)
        if not self.keep:
            for st in self.streams:   # output buffers exist before any block arrives
                self.zbuf[(id(bank), st.cuda_stream)] = self.torch.empty(
                    (bank.n_templates, bank.max_block), dtype=self.torch.complex64, device="cuda")
        return bank

    def destroy(self, bank):
        for st in self.streams:
            self.zbuf.pop((id(bank), st.cuda_stream), None)
        bank.destroy()

    def submit(self, items):
        torch = self.torch
        st = self.streams[self.next_stream]
        self.next_stream = (self.next_stream + 1) % len(self.streams)
        reqs = []
        for bank, s, start, n in items:
            if self.keep:
                z = torch.empty((bank.n_templates, n), dtype=torch.complex64, device="cuda")
                self.outputs.setdefault(s, []).append((start, z))
            else:
                key = (id(bank), st.cuda_stream)
                z = self.zbuf.get(key)
                if z is None:
                    z = torch.empty((bank.n_templates, bank.max_block), dtype=torch.complex64,
                                    device="cuda")
                    self.zbuf[key] = z
            reqs.append((bank, self.x[s][start:start + n], z))
        self.S.spiir_process_batch(reqs, stream=st)
        ev = torch.cuda.Event()
        ev.record(st)
        return ev

    def done(self, ev) -> bool:
        return ev.query()
