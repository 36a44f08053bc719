"""Trigger reduction (spiir_process_peaks / spiir_process_batch_peaks).

The reduction decides an index and a count from floating point, so the check
takes those decisions from the GPU's own FP32 output with the same FP32
arithmetic (|z|^2 = re*re + im*im, each step rounded): peak2, index and
n_above must match exactly.  Against the FP64 oracle the peak value is held
to the parity bar, and the index wherever the oracle's peak is separated
from every other sample by more than the tolerance allows.
"""
import numpy as np
import pytest

import oracle
from paper_1702_02256_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _say(msg):
    print(msg, flush=True)


def _ref_peaks(z, thr):
    """Reduction of an FP32 complex [T, n] array in FP32, as the library defines it."""
    re = np.ascontiguousarray(z.real, dtype=np.float32)
    im = np.ascontiguousarray(z.imag, dtype=np.float32)
    m = (re * re).astype(np.float32) + (im * im).astype(np.float32)
    t2 = np.float32(thr) * np.float32(thr)
    return m.max(axis=1), m.argmax(axis=1).astype(np.int32), (m >= t2).sum(axis=1).astype(np.int32)


def _check_exact(got, z, thr, label):
    p2, idx, cnt = _ref_peaks(z, thr)
    assert np.array_equal(got["peak2"].view(np.uint32), p2.view(np.uint32)), label
    assert np.array_equal(got["index"], idx), label
    assert np.array_equal(got["n_above"], cnt), label


def _run(tables, x, blocks, thr, write_z=True, max_block=None, **kw):
    import torch
    from paper_1702_02256_amd import spiir as S
    T = tables.n_templates
    bank = S.Bank(tables, max_block or max(blocks), **kw)
    plain = S.Bank(tables, max_block or max(blocks), **kw)
    xt = torch.from_numpy(np.asarray(x, np.float32)).cuda()
    pk = S.peaks_empty(T)
    out = []
    pos = 0
    for n in blocks:
        z = torch.empty((T, n), dtype=torch.complex64, device="cuda")
        zp = torch.empty((T, n), dtype=torch.complex64, device="cuda")
        bank.process_peaks(xt[pos:pos + n], z if write_z else None, pk, thr)
        plain.process_block(xt[pos:pos + n], zp)
        torch.cuda.synchronize()
        got = S.peaks_unpack(pk)
        zpn = zp.cpu().numpy()
        if write_z:
            assert np.array_equal(z.cpu().numpy().view(np.uint64), zpn.view(np.uint64))
        out.append((got, zpn))
        pos += n
    bank.destroy()
    plain.destroy()
    return out


def test_peaks_multirate_exact_and_vs_oracle():
    wl = W.config3(n_templates=48, n_blocks=3, block=4096)
    x = wl.stream()
    thr = 3e-3
    _say("peaks: 48 templates x 7 bands, blocks 4096, 2048, 2048 + 4096")
    blocks = [4096, 2048, 2048, 4096]
    res = _run(wl.bank, x[:sum(blocks)], blocks, thr)
    zr = oracle.run_stream(wl.bank, x[:sum(blocks)])
    pos = 0
    for i, ((got, zg), n) in enumerate(zip(res, blocks)):
        _check_exact(got, zg, thr, f"block {i}")
        a = np.abs(zr[:, pos:pos + n])
        top = a.max(axis=1)
        scale = np.abs(zr).max(axis=1)
        assert np.all(np.abs(np.sqrt(got["peak2"].astype(np.float64)) - top) <= TOL * scale)
        # where the oracle's peak stands clear of every other sample, the index is the oracle's
        second = np.sort(a, axis=1)[:, -2]
        clear = top - second > 4 * TOL * scale
        assert np.array_equal(got["index"][clear], a.argmax(axis=1)[clear])
        assert clear.sum() > 0
        # elsewhere the GPU's pick is within the tolerance of the oracle's peak
        picked = a[np.arange(a.shape[0]), got["index"]]
        assert np.all(top - picked <= 4 * TOL * scale)
        pos += n
    _say(f"peaks vs oracle ok over {len(blocks)} blocks")


def test_peaks_without_z_and_long_blocks():
    import torch
    from paper_1702_02256_amd import spiir as S
    wl = W.config3(seed=91, n_templates=20, n_blocks=4, block=4096)
    x = wl.stream()[: 2 * 8192]
    thr = 2e-3
    _say("peaks without z: 20 templates, blocks of 8192 (two launch chunks each)")
    with_z = _run(wl.bank, x, [8192, 8192], thr, write_z=True)
    no_z = _run(wl.bank, x, [8192, 8192], thr, write_z=False)
    for (ga, za), (gb, _) in zip(with_z, no_z):
        _check_exact(ga, za, thr, "with z")
        for k in ("peak2", "index", "n_above"):
            assert np.array_equal(ga[k].view(np.uint32), gb[k].view(np.uint32)), k
    # the peak of at least one template falls in the second launch chunk
    assert any((g["index"] >= 4096).any() for g, _ in with_z)


def test_peaks_with_a_time_split():
    """The reduction runs once per block after the chunked filter passes."""
    nf = np.array([[90], [7], [130]], np.int32)
    tb = W.random_bank(17, nf, 4096, [1500])
    x = W.noise_stream(18, 3 * 4096)
    thr = 1e-3
    blocks = [4096, 1000, 3096, 4096]
    _say("peaks with time_chunks=8: 3 templates, blocks 4096, 1000, 3096, 4096")
    res = _run(tb, x, blocks, thr, time_chunks=8, filters_per_lane=1, waves_per_group=2)
    zr = oracle.run_stream(tb, x)
    pos = 0
    for i, ((got, zg), n) in enumerate(zip(res, blocks)):
        _check_exact(got, zg, thr, f"split block {i}")
        top = np.abs(zr[:, pos:pos + n]).max(axis=1)
        scale = np.abs(zr).max(axis=1)
        assert np.all(np.abs(np.sqrt(got["peak2"].astype(np.float64)) - top) <= TOL * scale)
        pos += n


def test_peaks_single_rate_batch_and_ties():
    import torch
    from paper_1702_02256_amd import spiir as S
    wl = W.config2(n_templates=12, n_blocks=2)
    x = wl.stream()
    n = 2048
    a, b = S.Bank(wl.bank, n), S.Bank(wl.bank, n)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    zero = torch.zeros(n, dtype=torch.float32, device="cuda")
    za = torch.empty((12, n), dtype=torch.complex64, device="cuda")
    pa, pb = S.peaks_empty(12), S.peaks_empty(12)
    # a zero block from zero state: every |z|^2 is 0, so the first index wins the tie
    # and every sample is at or above a zero threshold
    S.spiir_process_batch_peaks([(a, zero, za), (b, zero, None)], [pa, pb], 0.0)
    torch.cuda.synchronize()
    for p in (pa, pb):
        g = S.peaks_unpack(p)
        assert np.all(g["peak2"] == 0) and np.all(g["index"] == 0) and np.all(g["n_above"] == n)
    # then real data through the same banks, batched
    S.spiir_process_batch_peaks([(a, xt[:n], za), (b, xt[:n], None)], [pa, pb], 1e-3)
    torch.cuda.synchronize()
    ga, gb = S.peaks_unpack(pa), S.peaks_unpack(pb)
    _check_exact(ga, za.cpu().numpy(), 1e-3, "single-rate batch")
    for k in ("peak2", "index", "n_above"):
        assert np.array_equal(ga[k].view(np.uint32), gb[k].view(np.uint32)), k
    a.destroy()
    b.destroy()


def test_peaks_argument_errors():
    import torch
    from paper_1702_02256_amd import spiir as S
    wl = W.config2(n_templates=4, n_blocks=1)
    bank = S.Bank(wl.bank, 2048)
    x = torch.zeros(2048, dtype=torch.float32, device="cuda")
    pk = S.peaks_empty(4)
    lib = S.load_library()
    for thr in (-1.0, float("nan"), float("inf")):
        assert lib.spiir_process_peaks(bank._h, x.data_ptr(), 2048, None, 0, pk.data_ptr(), thr,
                                       None) == S.SPIIR_EINVAL
    # no z and no peaks
    assert lib.spiir_process_peaks(bank._h, x.data_ptr(), 2048, None, 0, None, 0.0, None) == S.SPIIR_EINVAL
    assert bank.samples_done == 0
    bank.destroy()
