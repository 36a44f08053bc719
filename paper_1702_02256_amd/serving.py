"""Serving loop for SPIIR banks: continuous batching over several detector streams.

Strain blocks of uneven length arrive per detector stream.  Every bank is
bound to one stream and keeps its filter state resident on the device across
blocks; a stream may feed several banks (a large template set is split into
banks, and the same bank is run on every detector, as in the paper's search,
§5).  The scheduler

* admits banks by HBM footprint (a bank waits until its footprint fits the
  budget left by the banks already admitted; it then starts from its
  stream's first block);
* keeps, per stream, the blocks that have arrived, and per bank the next
  block it has to filter;
* whenever fewer than ``max_inflight`` batches are on the device, forms the
  next batch: the banks with work pending, oldest pending block first, each
  bank's pending blocks merged into one contiguous request (up to the bank's
  max block), at most ``max_batch`` requests, submitted as one
  ``spiir_process_batch`` launch sequence on the next of the backend's device
  streams, so batches overlap on the device;
* stamps a block done when every bank of its stream has filtered it, and
  records the time from its arrival to then.

Merging never changes results: the library's output does not depend on how a
stream is cut into blocks (bit for bit), nor on which other banks share a
batch.  The ``plain`` policy (one block of one bank per launch, one launch in
flight) is the comparison point.

The backend is pluggable: ``HipBackend`` drives libspiir.so; tests drive the
same scheduler with a CPU backend on a virtual clock.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

# Launch shape for banks served by the batched policy: a batched launch covers
# every bank of the batch at once, so its banks take the shape of a bank that
# fills the device (4 filters per lane, 8 waves per group) even when each bank
# alone would get the library's smaller default (4-wave groups for banks of
# under about 4 rounds of workgroups).  Pass it in ``bank_kw`` of HipBackend;
# the plain policy keeps the per-bank default.
BATCHED_BANK_SHAPE = {"filters_per_lane": 4, "waves_per_group": 8}


@dataclass
class Block:
    stream: int
    seq: int
    start: int          # first sample of the block in its stream
    n: int
    arrival: float      # seconds on the scheduler clock
    done: float = -1.0  # completion time on the scheduler clock
    remaining: int = 0  # banks of the stream that have not filtered it yet

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class Request:
    unit: int
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
    last_arrival: float = 0.0
    aborted: bool = False     # stopped because the backlog exceeded the bound
    admitted_at: dict = field(default_factory=dict)

    def latencies(self) -> np.ndarray:
        return np.array([b.latency for b in self.blocks if b.done >= 0])

    def summary(self) -> dict:
        lat = self.latencies() * 1e3
        out = {
            "blocks": len(lat),
            "blocks_arrived": len(self.blocks),
            "batches": self.batches,
            "requests": self.requests,
            "filter_samples_per_s": self.filter_samples / self.wall if self.wall > 0 else 0.0,
            "wall_s": self.wall,
            "drain_s": self.wall - self.last_arrival,
            "aborted": self.aborted,
        }
        if len(lat):
            out.update({"p50_ms": float(np.percentile(lat, 50)),
                        "p99_ms": float(np.percentile(lat, 99)),
                        "max_ms": float(lat.max()), "mean_ms": float(lat.mean())})
        return out


class Scheduler:
    """Continuous-batching scheduler (see the module docstring).

    ``tables_per_stream``: one bank per stream (bank s on stream s); or
    ``units``: a list of (stream, tables), several banks per stream allowed.
    ``abort_backlog_s``: stop once the oldest block not yet filtered by every
    bank of its stream is older than this (the device is not keeping up); the
    work in flight is drained first.  ``merge_max``: the longest request that
    merging consecutive blocks may form (default ``max_block``).
    """

    def __init__(self, backend, tables_per_stream=None, max_block: int = 4096,
                 hbm_budget: int | None = None, policy: str = "batched", max_batch: int = 16,
                 max_inflight: int = 2, units=None, abort_backlog_s: float | None = None,
                 merge_max: int | None = None):
        if policy not in ("batched", "plain"):
            raise ValueError(policy)
        if units is None:
            units = list(enumerate(tables_per_stream))
        self.be = backend
        self.units = [(int(s), t) for s, t in units]
        self.n_streams = 1 + max(s for s, _ in self.units)
        self.stream_units = [[u for u, (s, _) in enumerate(self.units) if s == st]
                             for st in range(self.n_streams)]
        self.max_block = int(max_block)
        self.merge_max = min(int(merge_max), self.max_block) if merge_max else self.max_block
        self.policy = policy
        self.max_batch = 1 if policy == "plain" else int(max_batch)
        self.max_inflight = 1 if policy == "plain" else int(max_inflight)
        self.budget = hbm_budget
        self.abort_backlog_s = abort_backlog_s
        self.used = 0
        self.handles = [None] * len(self.units)
        self.released = [False] * len(self.units)
        self.waiting_admission = deque(range(len(self.units)))
        self.arrived = [[] for _ in range(self.n_streams)]  # blocks of each stream, in order
        self.cursor = [0] * len(self.units)                 # next block of its stream per bank
        self.unfinished = [deque() for _ in range(self.n_streams)]  # blocks not yet done
        self.inflight = deque()   # (ticket, [Request])
        self.stats = Stats()

    # ---------------------------------------------------------- admission
    def _footprint(self, u: int) -> int:
        return self.be.footprint(self.units[u][1], self.max_block)

    def _admit(self, now: float):
        while self.waiting_admission:
            u = self.waiting_admission[0]
            need = self._footprint(u)
            if self.budget is not None and self.used + need > self.budget:
                break
            self.handles[u] = self.be.create(self.units[u][1], self.max_block)
            self.used += need
            self.stats.admitted_at[u] = now
            self.waiting_admission.popleft()

    def release(self, u: int):
        """Destroy bank u and return its footprint to the budget."""
        h = self.handles[u]
        if h is not None:
            self.used -= self._footprint(u)
            self.be.destroy(h)
            self.handles[u] = None
            self.released[u] = True

    def release_all(self):
        for u in range(len(self.units)):
            self.release(u)

    # ---------------------------------------------------------- batching
    def _pending(self, u: int) -> bool:
        return self.handles[u] is not None and self.cursor[u] < len(self.arrived[self.units[u][0]])

    def _form_batch(self):
        reqs = []
        cand = [u for u in range(len(self.units)) if self._pending(u)]
        cand.sort(key=lambda u: self.arrived[self.units[u][0]][self.cursor[u]].arrival)
        for u in cand[: self.max_batch]:
            s = self.units[u][0]
            blocks = self.arrived[s]
            first = blocks[self.cursor[u]]
            take, n = [first], first.n
            i = self.cursor[u] + 1
            if self.policy == "batched":
                while i < len(blocks) and n + blocks[i].n <= self.merge_max:
                    take.append(blocks[i])
                    n += blocks[i].n
                    i += 1
            self.cursor[u] = i
            reqs.append(Request(u, s, first.start, n, take))
        return reqs

    def _retire_ready(self, t0: float, block_until_done: bool = False):
        """Stamp and drop the leading in-flight batches that have completed,
        then drop the finished blocks at the head of each stream's backlog."""
        while self.inflight:
            ticket, reqs = self.inflight[0]
            if not self.be.done(ticket):
                if not block_until_done:
                    break
                self.be.wait(ticket, None)
                continue
            t = self.be.clock() - t0
            for r in reqs:
                for b in r.blocks:
                    b.remaining -= 1
                    if b.remaining == 0:
                        b.done = t
            self.inflight.popleft()
        for s in range(self.n_streams):
            q = self.unfinished[s]
            while q and q[0].done >= 0:
                q.popleft()

    def _release_finished(self, future_streams):
        """Free the banks whose stream has nothing left for them."""
        busy = {r.unit for _, reqs in self.inflight for r in reqs}
        for u, (s, _) in enumerate(self.units):
            if (self.handles[u] is not None and not self._pending(u) and u not in busy
                    and s not in future_streams):
                self.release(u)

    def _backlog(self, now: float) -> float:
        oldest = [q[0].arrival for q in self.unfinished if q]
        return now - min(oldest) if oldest else 0.0

    def run(self, arrivals, release_finished: bool = False) -> Stats:
        """arrivals: Blocks (any order); returns per-block latencies and totals."""
        arrivals = deque(sorted(arrivals, key=lambda b: b.arrival))
        self.stats.blocks = list(arrivals)
        self.stats.last_arrival = max((b.arrival for b in arrivals), default=0.0)
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
                b.remaining = len(self.stream_units[b.stream])
                self.arrived[b.stream].append(b)
                self.unfinished[b.stream].append(b)
            self._retire_ready(t0)
            if self.abort_backlog_s is not None and self._backlog(now) > self.abort_backlog_s:
                self.stats.aborted = True
                self._retire_ready(t0, block_until_done=True)
                break
            if release_finished:
                self._release_finished({b.stream for b in arrivals})
                self._admit(self.be.clock() - t0)
            pend = any(self._pending(u) for u in range(len(self.units)))
            if pend and len(self.inflight) < self.max_inflight:
                reqs = self._form_batch()
                ticket = self.be.submit([(self.handles[r.unit], r.stream, r.start, r.n) for r in reqs])
                self.inflight.append((ticket, reqs))
                self.stats.batches += 1
                self.stats.requests += len(reqs)
                self.stats.filter_samples += sum(
                    self.be.filter_samples(self.units[r.unit][1], r.n) for r in reqs)
                continue
            waiting = any(self.unfinished[s] for s in range(self.n_streams))
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
    """Drives libspiir.so: device-resident inputs per stream, ``n_streams``
    device streams used round robin, completion events.

    Outputs: with ``keep_outputs`` every request gets a fresh z buffer (tests
    read them back); otherwise z goes to a pool of buffers, one per (device
    stream, request slot of a batch), each reused in its stream's order, so
    output memory does not grow with the number of banks.  ``peaks``: write no
    z at all and keep only the trigger reduction (spiir_process_batch_peaks)
    in pooled peak buffers.  Banks created with a caller workspace
    (``workspace=WORKSPACE_CALLER`` in ``bank_kw``) take pooled workspaces the
    same way.  ``pool_templates`` and ``pool_workspace`` size the pools (the
    largest bank's templates and workspace); ``pool_bytes`` reports what they
    hold, for the caller's HBM budget.

    A bank for tables that a live bank already uses is made with spiir_clone
    (no planning, no host tables).  ``bank_pool`` may hold ready banks per
    tables object (``{id(tables): [Bank, ...]}``): ``create`` takes one of
    those (reset to zero state) before making a new one, and with
    ``return_to_pool`` ``destroy`` gives banks back to it instead of freeing
    them, so successive runs reuse the same device memory.
    """

    def __init__(self, streams_x, n_streams: int = 2, keep_outputs: bool = False,
                 peaks: bool = False, threshold: float = 0.0, pool_templates: int = 0,
                 pool_workspace: int = 0, max_batch: int = 16, max_block: int = 8192,
                 bank_pool=None, return_to_pool: bool = False, **bank_kw):
        import torch

        from . import spiir as S
        self.torch, self.S = torch, S
        self.x = [torch.from_numpy(np.asarray(x, np.float32)).cuda() for x in streams_x]
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.next_stream = 0
        self.bank_kw = bank_kw
        self.keep = keep_outputs
        self.peaks = peaks
        self.threshold = float(threshold)
        self.outputs = {}      # stream -> list of (start, tensor)
        self.pool = bank_pool if bank_pool is not None else {}
        self.return_to_pool = return_to_pool
        self.live = {}         # id(tables) -> live banks (clone sources)
        self._fp = {}
        self.max_batch = int(max_batch)
        self.max_block = int(max_block)
        self.zpool = self.pkpool = self.wspool = None
        nb = 0
        if not keep_outputs and pool_templates > 0:
            if peaks:
                self.pkpool = [[S.peaks_empty(pool_templates) for _ in range(self.max_batch)]
                               for _ in self.streams]
                nb += len(self.streams) * self.max_batch * pool_templates * 16
            else:
                self.zpool = [[torch.empty((pool_templates, self.max_block), dtype=torch.complex64,
                                           device="cuda") for _ in range(self.max_batch)]
                              for _ in self.streams]
                nb += len(self.streams) * self.max_batch * pool_templates * self.max_block * 8
        if pool_workspace > 0:
            self.wspool = [[S.workspace_empty(pool_workspace) for _ in range(self.max_batch)]
                           for _ in self.streams]
            nb += len(self.streams) * self.max_batch * pool_workspace
        self.pool_bytes = nb

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
        key = (id(tables), int(max_block))
        if key not in self._fp:
            self._fp[key] = self.S.spiir_footprint(tables, max_block, **self.bank_kw)
        return self._fp[key]

    def filter_samples(self, tables, n) -> int:
        return tables.filter_samples_per_block(n)

    def create(self, tables, max_block):
        ready = self.pool.get(id(tables))
        if ready:
            bank = ready.pop()
            bank.reset()
        else:
            live = self.live.get(id(tables))
            bank = live[0].clone() if live else self.S.Bank(tables, max_block, **self.bank_kw)
        bank._tables_id = id(tables)
        self.live.setdefault(id(tables), []).append(bank)
        return bank

    def destroy(self, bank):
        lst = self.live.get(bank._tables_id, [])
        if bank in lst:
            lst.remove(bank)
        if self.return_to_pool:
            self.torch.cuda.synchronize()
            self.pool.setdefault(bank._tables_id, []).append(bank)
        else:
            bank.destroy()

    def submit(self, items):
        torch = self.torch
        si = self.next_stream
        st = self.streams[si]
        self.next_stream = (self.next_stream + 1) % len(self.streams)
        reqs, pks = [], []
        for slot, (bank, s, start, n) in enumerate(items):
            x = self.x[s][start:start + n]
            ws = self.wspool[si][slot] if (self.wspool is not None and bank.plan["workspace"]) else None
            if self.keep:
                z = torch.empty((bank.n_templates, n), dtype=torch.complex64, device="cuda")
                self.outputs.setdefault(s, []).append((start, z))
            elif self.peaks:
                z = None
            elif self.zpool is not None:
                z = self.zpool[si][slot][: bank.n_templates, :n]
            else:
                raise RuntimeError("no output pool: give pool_templates or keep_outputs")
            reqs.append((bank, x, z, ws) if ws is not None else (bank, x, z))
            if self.peaks:
                pks.append(self.pkpool[si][slot][: bank.n_templates])
        if self.peaks:
            self.S.spiir_process_batch_peaks(reqs, pks, self.threshold, stream=st)
        else:
            self.S.spiir_process_batch(reqs, stream=st)
        ev = torch.cuda.Event()
        ev.record(st)
        return ev

    def done(self, ev) -> bool:
        return ev.query()
