"""The serving scheduler on the CPU: an oracle-backed device model on a
virtual clock checks admission by footprint, per-stream ordering, merging of
consecutive blocks, batching across streams and that every stream's output
equals the whole stream filtered at once."""
import numpy as np
import pytest

import oracle
from paper_1702_02256_amd import serving as SV
from paper_1702_02256_amd import workloads as W


class VirtualOracleBackend:
    """A serial device on a virtual clock; each batch costs a fixed launch
    overhead plus a cost per filter-sample; results come from the oracle."""

    def __init__(self, streams_x, s_per_fs=2e-12, launch_s=50e-6, fail_on=None):
        self.t = 0.0
        self.x = streams_x
        self.s_per_fs = s_per_fs
        self.launch_s = launch_s
        self.busy_until = 0.0
        self.outputs = {}
        self.created, self.destroyed = [], []
        self.batches = []
        self.by_bank = {}

    def clock(self):
        return self.t

    def start(self, t0):
        pass

    def wait(self, ticket, until):
        cands = [c for c in ((ticket or {}).get("done_at"), until) if c is not None]
        self.t = max(self.t, min(cands))

    def footprint(self, tables, max_block):
        return 44 * tables.total_filters + 8 * tables.n_templates * max_block

    def filter_samples(self, tables, n):
        return tables.filter_samples_per_block(n)

    def create(self, tables, max_block):
        b = oracle.OracleBank(tables)
        b.tables = tables
        self.created.append(id(b))
        return b

    def destroy(self, b):
        self.destroyed.append(id(b))
        b.close()

    def submit(self, items):
        cost = self.launch_s
        rec = []
        for bank, s, start, n in items:
            assert bank.samples_done == start, "per-stream order violated"
            z = bank.process(self.x[s][start:start + n])
            self.outputs.setdefault(s, []).append((start, z))
            self.by_bank.setdefault(id(bank), (bank, s, []))[2].append((start, z))
            cost += self.s_per_fs * bank.tables.filter_samples_per_block(n)
            rec.append((s, start, n))
        self.batches.append(rec)
        begin = max(self.t, self.busy_until)
        self.busy_until = begin + cost
        return {"done_at": self.busy_until}

    def done(self, ticket):
        return self.t >= ticket["done_at"]


def _setup(n_streams=3, dur_s=6.0, rate=256, speed=1.0, seed=5):
    banks = []
    for s in range(n_streams):
        nf = np.random.default_rng([seed, s]).integers(2, 12, size=(3 + s, 3)).astype(np.int32)
        banks.append(W.random_bank(100 + s, nf, rate, W.multirate_dmax(rate, 3)))
    arr = W.serving_arrivals(seed, n_streams, dur_s, rate_hz=rate, speed=speed)
    total = [int(lens.sum()) for lens, _ in arr]
    xs = [W.noise_stream(200 + s, total[s]) for s in range(n_streams)]
    return banks, arr, xs


def _concat(outputs, s):
    parts = sorted(outputs[s], key=lambda p: p[0])
    pos = 0
    for start, z in parts:
        assert start == pos
        pos += z.shape[1]
    return np.concatenate([z for _, z in parts], axis=1)


@pytest.mark.parametrize("policy", ["batched", "plain"])
def test_outputs_equal_whole_stream(policy):
    banks, arr, xs = _setup()
    be = VirtualOracleBackend(xs)
    sch = SV.Scheduler(be, banks, max_block=512, policy=policy)
    st = sch.run(SV.make_arrivals(arr))
    for s in range(3):
        got = _concat(be.outputs, s)
        ref = oracle.run_stream(banks[s], xs[s])
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert all(b.done >= b.arrival for b in st.blocks)
    assert st.summary()["blocks"] == sum(len(l) for l, _ in arr)


def test_batching_merges_and_spans_streams_under_load():
    banks, arr, xs = _setup(speed=50.0)   # blocks arrive 50x faster than real time
    be = VirtualOracleBackend(xs, s_per_fs=1e-7, launch_s=4e-3)
    sch = SV.Scheduler(be, banks, max_block=1024, policy="batched")
    st = sch.run(SV.make_arrivals(arr))
    nblocks = sum(len(l) for l, _ in arr)
    assert st.requests < nblocks                       # consecutive blocks were merged
    assert any(len(b) > 1 for b in be.batches)         # a batch carried several streams
    for rec in be.batches:
        assert len({s for s, _, _ in rec}) == len(rec)  # a bank at most once per batch
    # plain policy on the same load: one block per launch, larger latencies
    be2 = VirtualOracleBackend(xs, s_per_fs=1e-7, launch_s=4e-3)
    st2 = SV.Scheduler(be2, banks, max_block=1024, policy="plain").run(SV.make_arrivals(arr))
    assert st2.requests == nblocks and st.batches < st2.batches
    # with a fixed cost per launch, fewer larger launches keep the queue short
    assert np.percentile(st.latencies(), 99) < np.percentile(st2.latencies(), 99)


def test_admission_waits_for_footprint():
    banks, arr, xs = _setup(n_streams=3, dur_s=3.0)
    # streams end at different times; the budget fits two banks at once
    arr = [(l[: 3 + 4 * s], t[: 3 + 4 * s]) for s, (l, t) in enumerate(arr)]
    xs = [x[: int(l.sum())] for x, (l, _) in zip(xs, arr)]
    be = VirtualOracleBackend(xs)
    fp = [be.footprint(b, 512) for b in banks]
    budget = fp[0] + fp[2] + 1
    assert fp[1] + fp[2] > budget - fp[0]
    sch = SV.Scheduler(be, banks, max_block=512, hbm_budget=budget)
    st = sch.run(SV.make_arrivals(arr), release_finished=True)
    assert st.admitted_at[0] == 0.0
    late = [s for s in range(3) if st.admitted_at[s] > 0.0]
    assert late, "one bank must wait for the budget"
    for s in range(3):
        ref = oracle.run_stream(banks[s], xs[s])
        got = _concat(be.outputs, s)
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert sch.used <= budget


def test_unadmittable_bank_raises():
    banks, arr, xs = _setup(n_streams=1, dur_s=1.0)
    be = VirtualOracleBackend(xs)
    sch = SV.Scheduler(be, banks, max_block=512, hbm_budget=10)
    with pytest.raises(RuntimeError):
        sch.run(SV.make_arrivals(arr))


def test_several_banks_per_stream():
    """Banks share a stream (one of them twice: two banks of the same tables);
    each filters the whole stream, and a block is done only when all have."""
    banks, arr, xs = _setup(n_streams=2, speed=20.0)
    units = [(0, banks[0]), (0, banks[1]), (1, banks[1]), (0, banks[0])]
    be = VirtualOracleBackend(xs, s_per_fs=1e-8, launch_s=1e-3)
    sch = SV.Scheduler(be, units=units, max_block=512, max_batch=3)
    st = sch.run(SV.make_arrivals(arr))
    assert len(be.by_bank) == 4
    for bank, s, parts in be.by_bank.values():
        parts = sorted(parts, key=lambda p: p[0])
        got = np.concatenate([z for _, z in parts], axis=1)
        ref = oracle.run_stream(bank.tables, xs[s])
        assert got.shape == ref.shape
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    for rec in be.batches:
        assert len(rec) <= 3
    blocks = st.blocks
    assert all(b.done >= b.arrival and b.remaining == 0 for b in blocks)
    assert st.summary()["blocks"] == len(blocks)


def test_backlog_bound_stops_an_overloaded_run():
    banks, arr, xs = _setup(n_streams=2, dur_s=6.0)
    be = VirtualOracleBackend(xs, s_per_fs=1e-4, launch_s=1e-3)   # far slower than real time
    sch = SV.Scheduler(be, banks[:2], max_block=512, abort_backlog_s=1.0)
    st = sch.run(SV.make_arrivals(arr))
    summ = st.summary()
    assert st.aborted and summ["aborted"]
    assert not sch.inflight
    assert summ["blocks"] < summ["blocks_arrived"]
    # the run stopped about when the oldest unfinished block became 1 s old
    assert st.wall < 6.0


class _CostBackend(VirtualOracleBackend):
    """Timing only: a serial device at a fixed filter-sample rate (no filtering)."""

    def create(self, tables, max_block):
        return object()

    def destroy(self, b):
        pass

    def submit(self, items):
        cost = self.launch_s + sum(self.s_per_fs * tb for tb in (self._fs(n) for _, _, _, n in items))
        begin = max(self.t, self.busy_until)
        self.busy_until = begin + cost
        return {"done_at": self.busy_until}

    def _fs(self, n):
        return 1e6 * n


def test_backlog_counts_only_unfinished_blocks_with_two_batches_in_flight():
    """With a second batch always on the device, finished blocks must still
    leave the backlog: a run with spare throughput is not stopped."""
    banks, arr, xs = _setup(n_streams=3, dur_s=8.0, speed=1.0)
    units = [(s, banks[s]) for _ in range(60) for s in range(3)]
    # 60 banks per stream; the device runs at about 1.15x the arrival rate,
    # so a batch is nearly always on it
    be = _CostBackend(xs, s_per_fs=1.0 / (1.15 * 60 * 3 * 1e6 * 256), launch_s=1e-5)
    sch = SV.Scheduler(be, units=units, max_block=1024, policy="batched", max_batch=8,
                       abort_backlog_s=2.0)
    st = sch.run(SV.make_arrivals(arr))
    summ = st.summary()
    assert not st.aborted, summ
    assert summ["blocks"] == summ["blocks_arrived"]


def test_batched_bank_shape_is_the_full_device_default():
    # the shape the batched policy gives every bank is the one the library
    # picks by itself for a bank that fills the device; a small bank alone
    # gets 4-wave groups unless it is given that shape
    from paper_1702_02256_amd import spiir as S
    want = (SV.BATCHED_BANK_SHAPE["filters_per_lane"], 64 * SV.BATCHED_BANK_SHAPE["waves_per_group"])
    for prec in ("fp32", "fp32_compensated"):
        p = S.spiir_plan(W.config3(n_blocks=1).bank, 4096, precision=prec)
        assert (p["filters_per_lane"], p["lanes_per_group"]) == want, prec
    small = W.config3(n_templates=1024, n_blocks=1).bank
    assert S.spiir_plan(small, 4096)["lanes_per_group"] == 256
    p = S.spiir_plan(small, 4096, **SV.BATCHED_BANK_SHAPE)
    assert (p["filters_per_lane"], p["lanes_per_group"]) == want
