"""Recorded batches (spiir_graph_*) through the C ABI.

A graph records one batch over fixed buffers; every replay must equal the
eager call at the same point of the stream bit for bit (the bank's absolute
sample index lives on the device and is advanced by the recorded kernels).
Replays are checked one by one, with eager work and synchronisations between
them, and against the FP64 oracle at the parity bar.
"""
import numpy as np
import pytest

import oracle
from paper_1702_02256_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _say(msg):
    print(msg, flush=True)


def _rel_err(zg, zr):
    num = np.max(np.abs(zg - zr), axis=1)
    den = np.maximum(np.max(np.abs(zr), axis=1), 1e-300)
    return num / den


def test_graph_replays_equal_eager_and_oracle():
    import torch
    from paper_1702_02256_amd import spiir as S
    n, nb = 1024, 6
    wl = W.config3(n_templates=40, n_blocks=2, block=4096)
    x = wl.stream()[: n * nb]
    _say(f"graph: 40 templates x 7 bands, {nb} replays of {n}")
    eager = S.Bank(wl.bank, n)
    rec = S.Bank(wl.bank, n)
    xs = torch.from_numpy(x.astype(np.float32)).cuda()
    xbuf = torch.empty(n, dtype=torch.float32, device="cuda")
    zbuf = torch.empty((40, n), dtype=torch.complex64, device="cuda")
    ze = torch.empty((40, n), dtype=torch.complex64, device="cuda")
    g = S.Graph([(rec, xbuf, zbuf)])
    assert rec.samples_done == 0
    outs = []
    for i in range(nb):
        xbuf.copy_(xs[i * n:(i + 1) * n])
        if i == 3:
            # an eager call on the recorded bank between replays
            rec.process_block(xbuf, zbuf)
        else:
            g.launch()
        eager.process_block(xs[i * n:(i + 1) * n], ze)
        torch.cuda.synchronize()
        a, b = zbuf.cpu().numpy(), ze.cpu().numpy()
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), f"block {i} differs"
        outs.append(a.astype(np.complex128))
    assert rec.samples_done == n * nb
    g.destroy()
    zr = oracle.run_stream(wl.bank, x)
    e = _rel_err(np.concatenate(outs, axis=1), zr)
    _say(f"graph vs oracle: max rel err {e.max():.3e}")
    assert e.max() <= TOL
    eager.destroy()
    rec.destroy()


def test_graph_batch_of_banks_and_long_blocks():
    import torch
    from paper_1702_02256_amd import spiir as S
    # two banks with different shapes in one recorded batch; one block longer
    # than a launch chunk so the recording holds several chunk launches
    wa = W.config3(seed=77, n_templates=24, n_blocks=6, block=4096)
    wb = W.config4(seed=78, n_templates=30, n_blocks=3, block=4096)
    na, nbk = 8192, 4096
    xa = wa.stream()[: 3 * na]
    xb = wb.stream()[: 3 * nbk]
    assert len(xa) == 3 * na and len(xb) == 3 * nbk
    _say("graph batch: cfg3-shaped 24 templates (blocks 8192) + cfg4-shaped 30 (blocks 4096)")
    ea, eb = S.Bank(wa.bank, na), S.Bank(wb.bank, nbk)
    ra, rb = S.Bank(wa.bank, na), S.Bank(wb.bank, nbk)
    xa_t = torch.from_numpy(xa.astype(np.float32)).cuda()
    xb_t = torch.from_numpy(xb.astype(np.float32)).cuda()
    bufa, bufb = torch.empty(na, device="cuda"), torch.empty(nbk, device="cuda")
    za = torch.empty((24, na), dtype=torch.complex64, device="cuda")
    zb = torch.empty((30, nbk), dtype=torch.complex64, device="cuda")
    zea = torch.empty_like(za)
    zeb = torch.empty_like(zb)
    g = S.Graph([(ra, bufa, za), (rb, bufb, zb)])
    s = torch.cuda.Stream()
    for i in range(3):
        with torch.cuda.stream(s):
            bufa.copy_(xa_t[i * na:(i + 1) * na])
            bufb.copy_(xb_t[i * nbk:(i + 1) * nbk])
            g.launch(s)
        S.spiir_process_batch([(ea, xa_t[i * na:(i + 1) * na], zea),
                               (eb, xb_t[i * nbk:(i + 1) * nbk], zeb)])
        torch.cuda.synchronize()
        for got, ref, tag in ((za, zea, "a"), (zb, zeb, "b")):
            assert np.array_equal(got.cpu().numpy().view(np.uint64),
                                  ref.cpu().numpy().view(np.uint64)), f"replay {i} bank {tag}"
    assert ra.samples_done == 3 * na and rb.samples_done == 3 * nbk
    g.destroy()
    for b in (ea, eb, ra, rb):
        b.destroy()


def test_graph_after_state_load_and_reset():
    import torch
    from paper_1702_02256_amd import spiir as S
    n = 2048
    wl = W.config2(n_templates=8, n_blocks=4)
    x = wl.stream()[: 4 * n]
    xs = torch.from_numpy(x.astype(np.float32)).cuda()
    ref = S.Bank(wl.bank, n)
    zr = torch.empty((8, 4 * n), dtype=torch.complex64, device="cuda")
    for i in range(4):
        ref.process_block(xs[i * n:(i + 1) * n], zr[:, i * n:(i + 1) * n])
    rec = S.Bank(wl.bank, n)
    xbuf = torch.empty(n, device="cuda")
    z = torch.empty((8, n), dtype=torch.complex64, device="cuda")
    g = S.Graph([(rec, xbuf, z)])
    for i in range(2):
        xbuf.copy_(xs[i * n:(i + 1) * n])
        g.launch()
    blob = rec.save_state()
    rec.reset()
    assert rec.samples_done == 0
    xbuf.copy_(xs[:n])
    g.launch()
    torch.cuda.synchronize()
    assert np.array_equal(z.cpu().numpy().view(np.uint64), zr[:, :n].cpu().numpy().view(np.uint64))
    rec.load_state(blob)
    for i in range(2, 4):
        xbuf.copy_(xs[i * n:(i + 1) * n])
        g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(z.cpu().numpy().view(np.uint64),
                              zr[:, i * n:(i + 1) * n].cpu().numpy().view(np.uint64)), i
    g.destroy()
    ref.destroy()
    rec.destroy()
