"""The matrix-core engine (SPIIR_ENGINE_MFMA, single-rate banks) through the
C ABI, against the FP64 oracle at 1e-5 of each template's max |z| (the
tolerance for complex FP32 against FP64), and bit for bit where the output
must not depend on how the stream is cut or batched."""
import numpy as np
import pytest

import oracle
from paper_1702_02256_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _say(msg):
    print(msg, flush=True)


def _run(tables, x, blocks, max_block=None, **kw):
    import torch

    from paper_1702_02256_amd import spiir as S
    T = tables.n_templates
    n = int(sum(blocks))
    bank = S.Bank(tables, max_block or max(blocks), engine=S.ENGINE_MFMA, **kw)
    assert bank.plan["engine"] == S.ENGINE_MFMA
    xt = torch.from_numpy(np.asarray(x[:n], np.float32)).cuda()
    z = torch.zeros((T, n), dtype=torch.complex64, device="cuda")
    pos = 0
    for b in blocks:
        bank.process_block(xt[pos:pos + b], z[:, pos:pos + b])
        pos += b
    torch.cuda.synchronize()
    rc, _ = bank.status()
    assert rc == 0, rc
    out = z.cpu().numpy()
    bank.destroy()
    return out


def _check(zg, zr, label):
    e = np.max(np.abs(zg.astype(np.complex128) - zr), axis=1) / np.max(np.abs(zr), axis=1)
    _say(f"{label}: max rel err {e.max():.3e} (median {np.median(e):.3e})")
    assert np.all(np.isfinite(zg))
    assert e.max() <= TOL, (label, e.max())
    return e


def test_single_rate_subset_16_blocks():
    """Eight templates of the single-rate workload (512 filters, delays up to
    4095, 2048 Hz), 16 blocks of 2048 samples with the state carried."""
    wl = W.config2(templates=list(range(8)), n_blocks=16)
    x = wl.stream()
    _say("mfma: 8 x 512 filters, 16 blocks of 2048")
    zg = _run(wl.bank, x, [2048] * 16)
    zr = oracle.run_stream(wl.bank, x)
    e = _check(zg, zr, "mfma-cfg2-8")
    # the error does not grow along the stream
    win = 2 * 2048
    first = np.max(np.abs(zg[:, :win] - zr[:, :win]), axis=1) / np.max(np.abs(zr), axis=1)
    last = np.max(np.abs(zg[:, -win:] - zr[:, -win:]), axis=1) / np.max(np.abs(zr), axis=1)
    assert np.all(last <= np.maximum(3 * first, 2e-6)), (first, last)


def test_uneven_filter_counts_and_long_delays():
    """1, 100, 256, 257 and 700 filters (one to three workgroups per template,
    partly filled), delays up to 8191, blocks of 128 to 4096 samples."""
    nf = np.array([[1], [100], [256], [257], [700]], np.int32)
    tb = W.random_bank(4242, nf, 4096, [8191])
    blocks = [4096, 128, 384, 2048, 1536]
    x = W.noise_stream(4243, sum(blocks))
    _say(f"mfma: filters {nf.ravel().tolist()}, delays <= 8191, blocks {blocks}")
    zg = _run(tb, x, blocks, max_block=4096)
    zr = oracle.run_stream(tb, x)
    _check(zg, zr, "mfma-uneven")


def test_block_split_is_bitwise_invariant():
    wl = W.config2(templates=[3, 700], n_blocks=2)
    x = wl.stream()
    a = _run(wl.bank, x, [2048, 2048])
    b = _run(wl.bank, x, [128, 1920, 1024, 640, 384], max_block=2048)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_matrix_core_bank_in_a_batch_with_a_vector_bank():
    """A matrix-core bank and a vector-engine bank in one batch: each result is
    its own bank's alone, bit for bit (the batch launches one filter kernel per
    engine)."""
    import torch

    from paper_1702_02256_amd import spiir as S
    wl = W.config2(templates=[0, 1, 2], n_blocks=2)
    x = wl.stream()
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    mb = S.Bank(wl.bank, 2048, engine=S.ENGINE_MFMA)
    vb = S.Bank(wl.bank, 2048)
    zm = torch.zeros((3, 4096), dtype=torch.complex64, device="cuda")
    zv = torch.zeros((3, 4096), dtype=torch.complex64, device="cuda")
    for i in range(2):
        sl = slice(2048 * i, 2048 * (i + 1))
        S.spiir_process_batch([(mb, xt[sl], zm[:, sl]), (vb, xt[sl], zv[:, sl])])
    torch.cuda.synchronize()
    alone_m = _run(wl.bank, x, [2048, 2048])
    assert np.array_equal(zm.cpu().numpy().view(np.uint32), alone_m.view(np.uint32))
    zr = oracle.run_stream(wl.bank, x)
    _check(zv.cpu().numpy(), zr, "vector bank in the mixed batch")
    _check(zm.cpu().numpy(), zr, "matrix-core bank in the mixed batch")


def test_block_lengths_must_be_multiples_of_128():
    import torch

    from paper_1702_02256_amd import spiir as S
    wl = W.config2(templates=[0], n_blocks=1)
    bank = S.Bank(wl.bank, 2048, engine=S.ENGINE_MFMA)
    xt = torch.zeros(2048, dtype=torch.float32, device="cuda")
    z = torch.zeros((1, 2048), dtype=torch.complex64, device="cuda")
    with pytest.raises(S.SpiirError) as ei:
        bank.process_block(xt[:1000], z)
    assert ei.value.code == S.SPIIR_EINVAL
    assert bank.samples_done == 0
    bank.destroy()
