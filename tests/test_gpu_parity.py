"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Metric (per template): max_k |z_gpu - z_ref| / max_k |z_ref| over the whole
stream; the bar is 1e-5 for complex FP32 against the FP64 oracle.  Inputs are
the seeded workloads; the oracle gets the FP64 stream, the GPU its FP32
rounding.  Bitwise checks cover what must not depend on how the stream is cut
or batched.
"""
import numpy as np
import pytest

import oracle
from paper_1702_02256_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _torch():
    import torch
    return torch


def _say(msg):
    print(msg, flush=True)


def run_gpu(tables, x, blocks, max_block=None, **kw):
    """Stream x through a fresh bank in the given block lengths -> complex128 [T, n]."""
    torch = _torch()
    from paper_1702_02256_amd import spiir as S
    T = tables.n_templates
    n = int(sum(blocks))
    assert n <= len(x)
    bank = S.Bank(tables, max_block or max(blocks), **kw)
    xt = torch.from_numpy(np.asarray(x[:n], np.float32)).cuda()
    z = torch.zeros((T, n), dtype=torch.complex64, device="cuda")
    pos = 0
    for b in blocks:
        bank.process_block(xt[pos:pos + b], z[:, pos:pos + b])
        pos += b
    torch.cuda.synchronize()
    rc, flags = bank.status()
    assert rc == 0, rc
    out = z.cpu().numpy().astype(np.complex128)
    bank.destroy()
    return out


def rel_err(zg, zr):
    num = np.max(np.abs(zg - zr), axis=1)
    den = np.maximum(np.max(np.abs(zr), axis=1), 1e-300)
    return num / den


def check(zg, zr, tol=TOL, label=""):
    e = rel_err(zg, zr)
    _say(f"{label}: max rel err {e.max():.3e} (median {np.median(e):.3e}, worst template {int(e.argmax())})")
    assert np.all(np.isfinite(zg))
    assert e.max() <= tol, (label, e.max())
    return e


# ---------------------------------------------------------------- the configs


def test_config1_full():
    wl = W.config1()
    x = wl.stream()
    _say("cfg1: 1 template x 128 filters, 4096 samples")
    zg = run_gpu(wl.bank, x, [4096])
    zr = oracle.run_stream(wl.bank, x)
    check(zg, zr, label="cfg1")


def test_config2_subset_all_blocks():
    T = 16
    wl = W.config2(n_templates=T, n_blocks=16)
    x = wl.stream()
    _say("cfg2 subset: 16 x 512 filters, 16 blocks of 2048 at 2048 Hz")
    zg = run_gpu(wl.bank, x, [2048] * 16)
    zr = oracle.run_stream(wl.bank, x)
    check(zg, zr, label="cfg2-16")


def test_config3_subset():
    tsel = [0, 1, 777, 4095]
    wl = W.config3(templates=tsel, n_blocks=4)
    x = wl.stream()
    _say("cfg3 subset: 4 templates x 7 bands, 4 blocks of 4096")
    zg = run_gpu(wl.bank, x, [4096] * 4)
    zr = oracle.run_stream(wl.bank, x)
    check(zg, zr, label="cfg3-sub")


def test_long_stream_error_is_stationary():
    """64 s of the multi-rate bank in 1 s blocks (the stream length of the multi-rate
    workload): the FP32 state carried across blocks does not drift away from the
    FP64 oracle; the error of the last 8 s is of the size of the first 8 s."""
    tsel = [3, 1500, 4000]
    wl = W.config3(templates=tsel, n_blocks=64)
    x = wl.stream()
    _say("cfg3 long stream: 3 templates x 7 bands, 64 blocks of 4096 (64 s)")
    zg = run_gpu(wl.bank, x, [4096] * 64, precision="fp32_compensated")
    zr = oracle.run_stream(wl.bank, x)
    check(zg, zr, label="cfg3-64s")
    win = 8 * 4096
    first = rel_err(zg[:, :win], zr[:, :win])
    last = rel_err(zg[:, -win:], zr[:, -win:])
    _say(f"first 8 s {first.max():.3e}, last 8 s {last.max():.3e}")
    assert np.all(last <= np.maximum(3.0 * first, 2e-6)), (first, last)


def test_config4_subset_uneven():
    tsel = list(range(24))
    wl = W.config4(templates=tsel, n_blocks=2)
    x = wl.stream()
    _say("cfg4 subset: 24 uneven templates, 2 blocks of 4096")
    zg = run_gpu(wl.bank, x, [4096, 4096])
    zr = oracle.run_stream(wl.bank, x)
    check(zg, zr, label="cfg4-sub")


def test_config2_full_size_sampled():
    """All 1024 templates for 16 s, in the benchmark's launch shape; the oracle
    recomputes a random sample of templates (templates are independent)."""
    torch = _torch()
    from paper_1702_02256_amd import spiir as S
    wl = W.config2()
    x = wl.stream()
    _say("cfg2 full: 1024 x 512, 16 blocks, sampled check")
    bank = S.Bank(wl.bank, 2048)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    z = torch.zeros((1024, 2048 * 16), dtype=torch.complex64, device="cuda")
    for i in range(16):
        bank.process_block(xt[i * 2048:(i + 1) * 2048], z[:, i * 2048:(i + 1) * 2048])
    torch.cuda.synchronize()
    sel = np.sort(np.random.default_rng(99).choice(1024, 12, replace=False))
    zg = z[torch.as_tensor(sel, device="cuda")].cpu().numpy().astype(np.complex128)
    zr = oracle.run_stream(wl.bank.subset(sel), x)
    check(zg, zr, label="cfg2-full-sampled")
    bank.destroy()


def test_config3_full_size_sampled():
    torch = _torch()
    from paper_1702_02256_amd import spiir as S
    nb = 16
    wl = W.config3(n_blocks=nb)
    x = wl.stream()
    _say("cfg3 full: 4096 templates x 7 bands, 16 blocks of 4096, compensated, sampled check")
    bank = S.Bank(wl.bank, 4096, precision="fp32_compensated")  # the benchmark's form
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    sel = np.sort(np.random.default_rng(98).choice(4096, 6, replace=False))
    selt = torch.as_tensor(sel, device="cuda")
    z = torch.zeros((4096, 4096), dtype=torch.complex64, device="cuda")
    parts = []
    for i in range(nb):
        bank.process_block(xt[i * 4096:(i + 1) * 4096], z)
        parts.append(z[selt].cpu().numpy().astype(np.complex128))
    zg = np.concatenate(parts, axis=1)
    zr = oracle.run_stream(wl.bank.subset(sel), x)
    check(zg, zr, label="cfg3-full-sampled")
    bank.destroy()


def test_config4_full_size_sampled():
    """All 8192 uneven templates in 2048-sample blocks (the tuned block length)."""
    torch = _torch()
    from paper_1702_02256_amd import spiir as S
    wl = W.config4(n_blocks=2)
    x = wl.stream()[: 4 * 2048]
    _say("cfg4 full: 8192 uneven templates, 4 blocks of 2048, sampled check")
    bank = S.Bank(wl.bank, 2048)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    sel = np.sort(np.random.default_rng(97).choice(8192, 8, replace=False))
    selt = torch.as_tensor(sel, device="cuda")
    z = torch.zeros((8192, 2048), dtype=torch.complex64, device="cuda")
    parts = []
    for i in range(4):
        bank.process_block(xt[i * 2048:(i + 1) * 2048], z)
        parts.append(z[selt].cpu().numpy().astype(np.complex128))
    zg = np.concatenate(parts, axis=1)
    zr = oracle.run_stream(wl.bank.subset(sel), x)
    check(zg, zr, label="cfg4-full-sampled")
    bank.destroy()


def test_serving_bank_full_size_sampled():
    """One serving bank (5462 multi-rate templates) as the serving benchmark
    runs it: compensated, 8192-sample max block, uneven blocks."""
    torch = _torch()
    from paper_1702_02256_amd import spiir as S
    tb = W.serving_banks()[0]
    blocks = [4096, 512, 8192, 1536]
    x = W.noise_stream(2000, sum(blocks))
    _say(f"cfg5 bank full: {tb.n_templates} templates, blocks {blocks}, sampled check")
    bank = S.Bank(tb, 8192, precision="fp32_compensated")
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    sel = np.sort(np.random.default_rng(96).choice(tb.n_templates, 6, replace=False))
    selt = torch.as_tensor(sel, device="cuda")
    parts, pos = [], 0
    for n in blocks:
        z = torch.zeros((tb.n_templates, n), dtype=torch.complex64, device="cuda")
        bank.process_block(xt[pos:pos + n], z)
        parts.append(z[selt].cpu().numpy().astype(np.complex128))
        pos += n
    zg = np.concatenate(parts, axis=1)
    zr = oracle.run_stream(tb.subset(sel), x)
    check(zg, zr, label="cfg5-bank-full-sampled")
    bank.destroy()


# ---------------------------------------------------------------- streaming and edges


def _mr_bank(seed=3, T=5, H=4, lo=1, hi=90, rate=1024):
    nf = np.random.default_rng(seed).integers(lo, hi, size=(T, H)).astype(np.int32)
    return W.random_bank(seed, nf, rate, W.multirate_dmax(rate, H))


def test_block_split_is_bitwise_invariant():
    tb = _mr_bank()
    x = W.noise_stream(5, 4096)
    a = run_gpu(tb, x, [4096], max_block=4096)
    b = run_gpu(tb, x, [1024, 8, 504, 2048, 512], max_block=4096)
    assert np.array_equal(a, b)


def test_output_rows_at_any_alignment():
    """z rows whose start is not 16-byte aligned (odd row stride) take the 8-byte
    store path of the up-add; the values are the same bits."""
    torch = _torch()
    from paper_1702_02256_amd import spiir as S
    tb = _mr_bank(seed=71, T=5, H=3)
    x = W.noise_stream(72, 2048)
    ref = run_gpu(tb, x, [1024, 1024], max_block=1024)
    bank = S.Bank(tb, 1024)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    zbuf = torch.zeros((tb.n_templates, 2 * 1024 + 1), dtype=torch.complex64, device="cuda")
    assert zbuf.stride(0) % 2 == 1
    for b in range(2):
        bank.process_block(xt[b * 1024:(b + 1) * 1024], zbuf[:, b * 1024:(b + 1) * 1024])
    torch.cuda.synchronize()
    got = zbuf[:, :2048].cpu().numpy().astype(np.complex128)
    bank.destroy()
    assert np.array_equal(got, ref)


def test_ragged_blocks_and_tails():
    tb = _mr_bank(seed=4, T=3, H=3)
    x = W.noise_stream(6, 3000)
    blocks = [4, 12, 100, 1000, 4, 1880]
    zg = run_gpu(tb, x, blocks, max_block=2048)
    zr = oracle.run_stream(tb, x[:3000])
    check(zg, zr, label="ragged")


def test_long_blocks_split_inside_the_library():
    """Blocks longer than one internal launch (4096) and delays beyond the block."""
    tb = _mr_bank(seed=8, T=2, H=2, rate=4096)
    x = W.noise_stream(7, 3 * 8192)
    zg = run_gpu(tb, x, [8192, 8192, 8192], max_block=8192)
    zr = oracle.run_stream(tb, x)
    check(zg, zr, label="long-blocks")


def test_edge_shapes():
    # one filter; an empty band; a huge segment spanning several workgroups
    nf = np.array([[1, 0, 2], [0, 0, 3], [2500, 0, 1], [7, 0, 0]], np.int32)
    tb = W.random_bank(11, nf, 512, W.multirate_dmax(512, 3))
    x = W.noise_stream(12, 2048)
    zg = run_gpu(tb, x, [512] * 4)
    zr = oracle.run_stream(tb, x)
    check(zg, zr, label="edges")
    assert np.any(zg[3] != 0) and np.any(zg[1] != 0)


@pytest.mark.parametrize("n_down,n_up", [(17, 15), (48, 24), (32, 2), (20, 33)])
def test_other_resampler_lengths(n_down, n_up):
    """Interpolators other than the common 32 taps take the generic up-add path."""
    nf = np.random.default_rng(15).integers(1, 70, size=(4, 4)).astype(np.int32)
    tb = W.random_bank(15, nf, 1024, W.multirate_dmax(1024, 4), n_taps_down=n_down, n_taps_up=n_up)
    x = W.noise_stream(16, 3 * 1024)
    zg = run_gpu(tb, x, [1024, 512, 8, 1528], max_block=2048)
    zr = oracle.run_stream(tb, x)
    check(zg, zr, label=f"taps {n_down}/{n_up}")


@pytest.mark.parametrize("taps", [32, 1024])
def test_most_bands_and_longest_resamplers(taps):
    """SPIIR_MAX_BANDS bands (the lowest one gets a single sample of a 2048-sample
    block, fewer than the resampler histories hold); with SPIIR_MAX_TAPS taps the
    up-add needs more than 64 KB of LDS."""
    H = 12
    nf = np.random.default_rng(17).integers(1, 20, size=(3, H)).astype(np.int32)
    tb = W.random_bank(17, nf, 4096, W.multirate_dmax(4096, H), n_taps_down=taps, n_taps_up=taps)
    x = W.noise_stream(18, 16384)
    zg = run_gpu(tb, x, [2048, 4096, 8192, 2048], max_block=8192)
    zr = oracle.run_stream(tb, x)
    check(zg, zr, label=f"H=12 taps={taps}")


def test_largest_batch():
    """SPIIR_MAX_BATCH banks of different band counts in one batch, each result
    the bank's own; one more request is refused before anything is enqueued."""
    torch = _torch()
    from paper_1702_02256_amd import spiir as S
    nb = S.MAX_BATCH
    tabs = [_mr_bank(seed=100 + i, T=1 + i % 3, H=1 + i % 4, hi=40) for i in range(nb + 1)]
    xs = [W.noise_stream(200 + i, 1024) for i in range(nb + 1)]
    alone = [run_gpu(tabs[i], xs[i], [1024]) for i in range(nb)]
    banks = [S.Bank(t, 1024) for t in tabs]
    xt = [torch.from_numpy(x.astype(np.float32)).cuda() for x in xs]
    zt = [torch.zeros((t.n_templates, 1024), dtype=torch.complex64, device="cuda") for t in tabs]
    with pytest.raises(S.SpiirError) as ei:
        S.spiir_process_batch([(banks[i], xt[i], zt[i]) for i in range(nb + 1)])
    assert ei.value.code == S.SPIIR_EINVAL
    assert all(b.samples_done == 0 for b in banks)
    S.spiir_process_batch([(banks[i], xt[i], zt[i]) for i in range(nb)])
    torch.cuda.synchronize()
    for i in range(nb):
        assert np.array_equal(zt[i].cpu().numpy().astype(np.complex128), alone[i]), i
    for b in banks:
        b.destroy()


def test_bank_without_filters():
    """A bank whose templates have no filters at all runs (no filter workgroups)
    and outputs exact zeros; also split in time."""
    tb = W.random_bank(81, np.zeros((3, 3), np.int32), 1024, W.multirate_dmax(1024, 3))
    x = W.noise_stream(82, 2048)
    for kw in ({}, {"time_chunks": 4}):
        zg = run_gpu(tb, x, [1024, 1024], max_block=1024, **kw)
        assert np.array_equal(zg, np.zeros_like(zg))


def test_large_delays_use_subblocks():
    nf = np.array([[64], [64]], np.int32)
    tb = W.random_bank(13, nf, 4096, [12000])
    x = W.noise_stream(14, 4 * 4096)
    zg = run_gpu(tb, x, [4096] * 4)
    zr = oracle.run_stream(tb, x)
    check(zg, zr, label="large-delays")


def test_largest_delay_with_the_default_shape():
    nf = np.array([[64], [64]], np.int32)
    tb = W.random_bank(21, nf, 4096, [16383])
    tb.delay = tb.delay.copy()
    tb.delay[:4] = 16383
    x = W.noise_stream(22, 6 * 4096)
    zr = oracle.run_stream(tb, x)
    # the library's shape (one window copy) and the smaller groups two copies need
    for wc in (0, 2):
        zg = run_gpu(tb, x, [4096] * 6, window_copies=wc)
        check(zg, zr, label=f"max-delay, window copies {wc or 'default'}")


@pytest.mark.parametrize("F,Wv", [(1, 1), (2, 2), (4, 4), (8, 4), (8, 8), (4, 8), (1, 8), (6, 8), (6, 2), (6, 5)])
def test_lane_packing_variants(F, Wv):
    tb = _mr_bank(seed=15, T=6, H=3, lo=1, hi=300)
    x = W.noise_stream(16, 2048)
    zg = run_gpu(tb, x, [1024, 1024], filters_per_lane=F, waves_per_group=Wv)
    zr = oracle.run_stream(tb, x)
    check(zg, zr, label=f"F{F}W{Wv}")


def _random_case(i):
    """A seeded random bank, block sequence and launch shape (band count, rates,
    filter counts with empty segments, delays up to one second, resampler
    lengths, lanes, waves, carry chunk, time split, window layout, precision);
    draws that the planner refuses (an explicit shape whose window does not fit
    the LDS) are drawn again."""
    from paper_1702_02256_amd import spiir as S
    rng = np.random.default_rng([777, i])
    while True:
        H = int(rng.integers(1, 6))
        rate = int(rng.choice([512, 1024, 2048]))
        T = int(rng.integers(1, 7))
        nf = rng.integers(0, 120, size=(T, H)) * (rng.random((T, H)) > 0.2)
        dmax = [int(rng.integers(0, max(rate >> h, 2))) for h in range(H)]
        tb = W.random_bank(int(rng.integers(1 << 30)), nf.astype(np.int32), rate, dmax,
                           n_taps_down=int(rng.integers(1, 65)), n_taps_up=int(rng.integers(1, 65)))
        unit = 1 << (H - 1)
        max_block = unit * int(rng.integers(1, 8192 // unit + 1))
        blocks = [unit * int(rng.integers(1, max_block // unit + 1)) for _ in range(int(rng.integers(2, 5)))]
        kw = dict(filters_per_lane=int(rng.choice([1, 2, 4, 6, 8])), waves_per_group=int(rng.choice([1, 2, 3, 4, 5, 8])),
                  carry_chunk=int(rng.choice([16, 32, 64, 128])), time_chunks=int(rng.choice([0, 0, 2, 4, 8])),
                  window_copies=int(rng.choice([0, 1, 2])),
                  precision=str(rng.choice(["fp32", "fp32_compensated"])))
        try:
            S.spiir_plan(tb, max_block, **kw)
        except S.SpiirError:
            continue
        return tb, max_block, blocks, kw


@pytest.mark.parametrize("i", range(48))
def test_random_configurations_match_the_oracle(i):
    tb, max_block, blocks, kw = _random_case(i)
    x = W.noise_stream(900 + i, sum(blocks))
    zg = run_gpu(tb, x, blocks, max_block=max_block, **kw)
    zr = oracle.run_stream(tb, x)
    check(zg, zr, label=f"random {i}: T={tb.n_templates} H={tb.n_filters.shape[1]} blocks={blocks} {kw}")


@pytest.mark.parametrize("C", [16, 64, 256])
def test_carry_chunk_variants(C):
    wl = W.config1()
    x = wl.stream()
    zg = run_gpu(wl.bank, x, [4096], carry_chunk=C)
    zr = oracle.run_stream(wl.bank, x)
    check(zg, zr, label=f"C{C}")


@pytest.mark.parametrize("precision", ["fp32", "fp32_compensated"])
def test_one_and_two_window_copies(precision):
    """The single-copy input window (two 32-bit reads per sample pair) reads the same
    samples as the two-copy one; the two layouts place the filters by different
    LDS bank classes, so they sum in different orders: each meets the bar
    against the oracle, and they agree with each other to within FP32 summation
    rounding.  Checked on a multi-rate bank and a single-rate bank with long
    delays."""
    tb_mr = _mr_bank(seed=61, T=5, H=4, rate=2048)
    tb_sr = W.random_bank(62, np.array([[300], [41], [180]], np.int32), 2048, [4095])
    x = W.noise_stream(63, 4 * 2048)
    for tb in (tb_mr, tb_sr):
        zr = oracle.run_stream(tb, x)
        z1 = run_gpu(tb, x, [2048, 1000, 1048, 4096], max_block=4096, precision=precision,
                     window_copies=1)
        z2 = run_gpu(tb, x, [2048, 1000, 1048, 4096], max_block=4096, precision=precision,
                     window_copies=2)
        check(z1, zr, label=f"one window copy ({precision})")
        check(z2, zr, label=f"two window copies ({precision})")
        d = np.max(np.abs(z1 - z2), axis=1) / np.max(np.abs(zr), axis=1)
        _say(f"one against two window copies ({precision}): max rel difference {d.max():.3e}")
        # the filters' recurrences are the same arithmetic in both layouts; only
        # the order of the FP32 sum over a few hundred partials differs
        assert d.max() < 2e-6, d.max()


def test_compensated_mode():
    T = 8
    wl = W.config2(n_templates=T, n_blocks=4)
    x = wl.stream()
    zr = oracle.run_stream(wl.bank, x[:8192])
    zp = run_gpu(wl.bank, x, [2048] * 4, precision="fp32")
    zc = run_gpu(wl.bank, x, [2048] * 4, precision="fp32_compensated")
    check(zp, zr, label="plain")
    check(zc, zr, label="compensated")


def test_zero_padding_invariance():
    nf = np.array([[20], [33]], np.int32)
    tb = W.random_bank(17, nf, 1024, [200])
    pad = 11
    off = tb.offsets()
    a1, b0, d = [], [], []
    for t in range(2):
        s, m = off[t, 0], nf[t, 0]
        a1 += [tb.a1[s:s + m], np.zeros(pad)]
        b0 += [tb.b0[s:s + m], np.zeros(pad)]
        d += [tb.delay[s:s + m], np.arange(pad, dtype=np.int32)]
    tp = W.BankTables(1024, nf + pad, np.concatenate(a1), np.concatenate(b0), np.concatenate(d))
    x = W.noise_stream(18, 2048)
    za = run_gpu(tb, x, [2048])
    zb = run_gpu(tp, x, [2048])
    check(zb, za, tol=1e-6, label="zero-pad")


# ---------------------------------------------------------------- ABI behaviour on the device


def test_batch_equals_alone_bitwise():
    torch = _torch()
    from paper_1702_02256_amd import spiir as S
    tabs = [_mr_bank(seed=20 + i, T=4 + i, H=3) for i in range(3)]
    xs = [W.noise_stream(30 + i, 2048) for i in range(3)]
    lens = [1024, 512, 2048]
    alone = [run_gpu(tabs[i], xs[i], [lens[i]], max_block=2048) for i in range(3)]
    banks = [S.Bank(t, 2048) for t in tabs]
    xt = [torch.from_numpy(xs[i][:lens[i]].astype(np.float32)).cuda() for i in range(3)]
    zt = [torch.zeros((tabs[i].n_templates, lens[i]), dtype=torch.complex64, device="cuda")
          for i in range(3)]
    S.spiir_process_batch([(banks[i], xt[i], zt[i]) for i in range(3)])
    torch.cuda.synchronize()
    for i in range(3):
        assert np.array_equal(zt[i].cpu().numpy().astype(np.complex128), alone[i]), i
        banks[i].destroy()


def test_mixed_batch_equals_alone_bitwise():
    """One batch over a single-rate bank, a multi-rate bank with the common 32-tap
    resamplers, one with 15-tap resamplers (the generic up-add path) and a bank
    split in time, all compensated (default shape); each result is the bank's own."""
    torch = _torch()
    from paper_1702_02256_amd import spiir as S
    rng = np.random.default_rng(44)
    tabs = [
        W.random_bank(41, rng.integers(5, 90, size=(3, 1)).astype(np.int32), 2048, [900]),
        W.random_bank(42, rng.integers(5, 90, size=(4, 4)).astype(np.int32), 2048,
                      W.multirate_dmax(2048, 4)),
        W.random_bank(43, rng.integers(5, 90, size=(2, 3)).astype(np.int32), 2048,
                      W.multirate_dmax(2048, 3), n_taps_down=15, n_taps_up=15),
        W.random_bank(45, rng.integers(5, 90, size=(2, 1)).astype(np.int32), 2048, [700]),
    ]
    kws = [{}, {}, {}, {"time_chunks": 8}]
    xs = [W.noise_stream(50 + i, 4096) for i in range(4)]
    lens = [1024, 2048, 512, 2048]
    kw0 = dict(precision="fp32_compensated")
    alone = [run_gpu(tabs[i], xs[i], [lens[i], lens[i]], max_block=2048, **kw0, **kws[i])
             for i in range(4)]
    banks = [S.Bank(tabs[i], 2048, **kw0, **kws[i]) for i in range(4)]
    for blk in range(2):
        xt = [torch.from_numpy(xs[i][blk * lens[i]:(blk + 1) * lens[i]].astype(np.float32)).cuda()
              for i in range(4)]
        zt = [torch.zeros((tabs[i].n_templates, lens[i]), dtype=torch.complex64, device="cuda")
              for i in range(4)]
        S.spiir_process_batch([(banks[i], xt[i], zt[i]) for i in range(4)])
        torch.cuda.synchronize()
        for i in range(4):
            got = zt[i].cpu().numpy().astype(np.complex128)
            assert np.array_equal(got, alone[i][:, blk * lens[i]:(blk + 1) * lens[i]]), (blk, i)
    for i in range(4):
        zr = oracle.run_stream(tabs[i], xs[i][:2 * lens[i]])
        check(alone[i], zr, label=f"mixed-batch bank {i}")
        banks[i].destroy()


def test_batch_of_different_launch_shapes_equals_alone_bitwise():
    """Banks of different lanes per filter, group sizes, precisions and time
    splits in one batch (one filter launch per shape), eager and replayed from
    a recording; each result is the bank's own, bit for bit."""
    torch = _torch()
    from paper_1702_02256_amd import spiir as S
    shapes = [dict(filters_per_lane=6, waves_per_group=4, precision="fp32_compensated"), {},
              dict(filters_per_lane=8, waves_per_group=2, time_chunks=4),
              dict(filters_per_lane=1, waves_per_group=1, precision="fp32_compensated"),
              dict(filters_per_lane=4, waves_per_group=8)]
    tabs = [_mr_bank(seed=70 + i, T=2 + i, H=1 + i % 3) for i in range(len(shapes))]
    xs = [W.noise_stream(80 + i, 2048) for i in range(len(shapes))]
    alone = [run_gpu(tabs[i], xs[i], [1024, 1024], max_block=1024, **shapes[i]) for i in range(len(shapes))]
    for graph in (False, True):
        banks = [S.Bank(t, 1024, **kw) for t, kw in zip(tabs, shapes)]
        assert len({(b.plan["filters_per_lane"], b.plan["lanes_per_group"]) for b in banks}) >= 4
        xt = [torch.from_numpy(x.astype(np.float32)).cuda() for x in xs]
        xb = [torch.empty(1024, device="cuda") for _ in xs]
        zt = [torch.zeros((t.n_templates, 1024), dtype=torch.complex64, device="cuda") for t in tabs]
        g = S.Graph([(banks[i], xb[i], zt[i]) for i in range(len(banks))]) if graph else None
        for blk in range(2):
            for i in range(len(banks)):
                xb[i].copy_(xt[i][blk * 1024:(blk + 1) * 1024])
            if g:
                g.launch()
            else:
                S.spiir_process_batch([(banks[i], xb[i], zt[i]) for i in range(len(banks))])
            torch.cuda.synchronize()
            for i in range(len(banks)):
                got = zt[i].cpu().numpy().astype(np.complex128)
                assert np.array_equal(got, alone[i][:, blk * 1024:(blk + 1) * 1024]), (graph, blk, i)
        if g:
            g.destroy()
        for b in banks:
            b.destroy()


def test_created_bank_reports_the_planned_shape():
    """spiir_bank_plan of a created bank equals spiir_plan of its descriptor."""
    from paper_1702_02256_amd import spiir as S
    tb = _mr_bank(seed=91, T=6, H=4, rate=2048)
    for kw in ({}, {"precision": "fp32_compensated"}, {"window_copies": 1, "filters_per_lane": 2},
               {"time_chunks": 4}):
        bank = S.Bank(tb, 2048, **kw)
        assert bank.plan == S.spiir_plan(tb, 2048, **kw), kw
        bank.destroy()


def test_save_load_roundtrip_bitwise():
    torch = _torch()
    from paper_1702_02256_amd import spiir as S
    tb = _mr_bank(seed=40, T=3, H=3)
    x = W.noise_stream(41, 4096)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    bank = S.Bank(tb, 2048)
    z = torch.zeros((3, 2048), dtype=torch.complex64, device="cuda")
    bank.process_block(xt[:2048], z)
    blob = bank.save_state()
    z1 = torch.zeros_like(z)
    bank.process_block(xt[2048:], z1)
    bank.load_state(blob)
    assert bank.samples_done == 2048
    z2 = torch.zeros_like(z)
    bank.process_block(xt[2048:], z2)
    torch.cuda.synchronize()
    assert torch.equal(z1, z2)
    bank.reset()
    assert bank.samples_done == 0
    z3 = torch.zeros_like(z)
    bank.process_block(xt[:2048], z3)
    torch.cuda.synchronize()
    assert torch.equal(z3, z)
    bank.destroy()


def test_state_blob_is_tied_to_the_filter_layout():
    """A blob resumes a bank made from the same tables, and is refused by a bank
    of equal sizes whose delays place the filters differently, or when its
    header is damaged."""
    import dataclasses
    import struct
    torch = _torch()
    from paper_1702_02256_amd import spiir as S
    tb = _mr_bank(seed=42, T=3, H=3)
    xt = torch.from_numpy(W.noise_stream(43, 4096).astype(np.float32)).cuda()
    bank = S.Bank(tb, 2048)
    z = torch.zeros((3, 2048), dtype=torch.complex64, device="cuda")
    bank.process_block(xt[:2048], z)
    blob = bank.save_state()
    fresh = S.Bank(tb, 2048)
    fresh.load_state(blob)
    assert fresh.samples_done == 2048
    z1, z2 = torch.zeros_like(z), torch.zeros_like(z)
    bank.process_block(xt[2048:], z1)
    fresh.process_block(xt[2048:], z2)
    torch.cuda.synchronize()
    assert torch.equal(z1, z2)
    # the same delays reversed inside each (template, band) segment: equal sizes,
    # another placement of the filters over lanes and slots
    segs = np.cumsum(np.concatenate([[0], tb.n_filters.ravel()]))
    d2 = np.concatenate([tb.delay[a:b][::-1] for a, b in zip(segs[:-1], segs[1:])]).astype(np.int32)
    other = S.Bank(dataclasses.replace(tb, delay=d2), 2048)
    assert other.state_size() == len(blob)
    with pytest.raises(S.SpiirError) as ei:
        other.load_state(blob)
    assert ei.value.code == S.SPIIR_EINVAL
    bad = bytearray(blob)
    bad[0] ^= 1  # magic
    with pytest.raises(S.SpiirError):
        fresh.load_state(bytes(bad))
    bad = bytearray(blob)
    struct.pack_into("<q", bad, 48, 2049)  # sample count: not a multiple of 2^(H-1)
    with pytest.raises(S.SpiirError):
        fresh.load_state(bytes(bad))
    with pytest.raises(S.SpiirError):  # a truncated blob
        fresh.load_state(blob[:-4])
    assert other.samples_done == 0 and fresh.samples_done == 4096
    for b in (bank, fresh, other):
        b.destroy()


def test_invalid_block_leaves_state_unchanged():
    torch = _torch()
    from paper_1702_02256_amd import spiir as S
    tb = _mr_bank(seed=50, T=2, H=3)
    x = W.noise_stream(51, 1024)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    bank = S.Bank(tb, 1024)
    z = torch.zeros((2, 1024), dtype=torch.complex64, device="cuda")
    assert bank.process_raw(xt.data_ptr(), 6, z.data_ptr(), 1024) == S.SPIIR_EINVAL
    assert bank.process_raw(xt.data_ptr(), 2048, z.data_ptr(), 4096) == S.SPIIR_EINVAL
    assert bank.process_raw(xt.data_ptr(), 512, z.data_ptr(), 100) == S.SPIIR_EINVAL
    assert bank.samples_done == 0
    bank.process_block(xt, z)
    torch.cuda.synchronize()
    ref = run_gpu(tb, x, [1024])
    assert np.array_equal(z.cpu().numpy().astype(np.complex128), ref)
    bank.destroy()


def test_nonfinite_input_is_flagged_and_reset_clears():
    torch = _torch()
    from paper_1702_02256_amd import spiir as S
    tb = _mr_bank(seed=60, T=3, H=1)
    x = W.noise_stream(61, 1024).astype(np.float32)
    x[100] = np.nan
    bank = S.Bank(tb, 1024)
    z = torch.zeros((3, 1024), dtype=torch.complex64, device="cuda")
    bank.process_block(torch.from_numpy(x).cuda(), z)
    rc, flags = bank.status()
    assert rc == S.SPIIR_ENONFINITE and flags.all()
    bank.reset()
    rc, flags = bank.status()
    assert rc == 0 and not flags.any()
    bank.destroy()
