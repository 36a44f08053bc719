"""Parallel-in-time split (time_chunks > 1) through the C ABI.

A split bank runs an end-state pass, a chain pass and the filter pass per
block; its results differ from the sequential form by rounding only, so it is
held to the same bar against the FP64 oracle.  What must not depend on
batching, recording or checkpointing is checked bit for bit.
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


def _run(tables, x, blocks, max_block, **kw):
    import torch
    from paper_1702_02256_amd import spiir as S
    T = tables.n_templates
    bank = S.Bank(tables, max_block, **kw)
    xt = torch.from_numpy(np.asarray(x, np.float32)).cuda()
    z = torch.zeros((T, int(sum(blocks))), dtype=torch.complex64, device="cuda")
    pos = 0
    for n in blocks:
        bank.process_block(xt[pos:pos + n], z[:, pos:pos + n])
        pos += n
    torch.cuda.synchronize()
    rc, _ = bank.status()
    assert rc == 0
    bank.destroy()
    return z.cpu().numpy()


@pytest.mark.parametrize("P,F", [(4, 4), (32, 1), (64, 4)])
def test_single_rate_split_vs_oracle(P, F):
    wl = W.config1()
    blocks = [1000, 3096, 4096, 512, 2000]
    x = W.noise_stream(4242, sum(blocks))
    _say(f"time split P={P} F={F}: 1 x 128 filters, blocks {blocks}")
    zg = _run(wl.bank, x, blocks, 4096, time_chunks=P, filters_per_lane=F, waves_per_group=1)
    zr = oracle.run_stream(wl.bank, x)
    e = _rel_err(zg.astype(np.complex128), zr)
    _say(f"  max rel err {e.max():.3e}")
    assert e.max() <= TOL


def test_automatic_split_equals_the_chosen_split():
    """time_chunks = SPIIR_TIME_CHUNKS_AUTO plans a split for a small multi-rate
    bank; the bank runs exactly as one created with that split given."""
    from paper_1702_02256_amd import spiir as S
    wl = W.config3(n_templates=12, n_blocks=1)
    blocks = [4096, 1024, 3072]
    x = W.noise_stream(4343, sum(blocks))
    plan = S.spiir_plan(wl.bank, 4096, time_chunks=S.TIME_CHUNKS_AUTO)
    P = plan["time_chunks"]
    _say(f"automatic split: P={P}, {plan['n_groups']} groups")
    assert P > 1
    za = _run(wl.bank, x, blocks, 4096, time_chunks=S.TIME_CHUNKS_AUTO)
    zp = _run(wl.bank, x, blocks, 4096, time_chunks=P)
    assert np.array_equal(za.view(np.uint64), zp.view(np.uint64))
    e = _rel_err(za.astype(np.complex128), oracle.run_stream(wl.bank, x))
    _say(f"  max rel err {e.max():.3e}")
    assert e.max() <= TOL


def test_multirate_split_vs_oracle_and_long_blocks():
    wl = W.config3(n_templates=6, n_blocks=1)
    blocks = [4096, 8192, 1024, 2048 + 64]
    x = W.noise_stream(77, sum(blocks))
    _say(f"time split P=8: 6 templates x 7 bands, blocks {blocks}")
    zg = _run(wl.bank, x, blocks, 8192, time_chunks=8)
    zr = oracle.run_stream(wl.bank, x)
    e = _rel_err(zg.astype(np.complex128), zr)
    _say(f"  max rel err {e.max():.3e}")
    assert e.max() <= TOL


def test_split_bank_in_batch_graph_and_checkpoint_bitwise():
    import torch
    from paper_1702_02256_amd import spiir as S
    wa = W.config1()
    wb = W.config3(n_templates=4, n_blocks=1)
    n = 2048
    xa = torch.from_numpy(W.noise_stream(5, 4 * n).astype(np.float32)).cuda()
    xb = torch.from_numpy(W.noise_stream(6, 4 * n).astype(np.float32)).cuda()
    _say("time split: batch with a plain bank, graph replay, save/load; bitwise")
    # reference: each bank alone, eager
    alone_a = S.Bank(wa.bank, n, time_chunks=16)
    alone_b = S.Bank(wb.bank, n)
    za = torch.empty((1, 4 * n), dtype=torch.complex64, device="cuda")
    zb = torch.empty((4, 4 * n), dtype=torch.complex64, device="cuda")
    for i in range(4):
        alone_a.process_block(xa[i * n:(i + 1) * n], za[:, i * n:(i + 1) * n])
        alone_b.process_block(xb[i * n:(i + 1) * n], zb[:, i * n:(i + 1) * n])
    torch.cuda.synchronize()
    ref_a, ref_b = za.cpu().numpy(), zb.cpu().numpy()
    # batched with a plain bank, then recorded and replayed, with a checkpoint in between
    ba = S.Bank(wa.bank, n, time_chunks=16)
    bb = S.Bank(wb.bank, n)
    ya = torch.empty((1, n), dtype=torch.complex64, device="cuda")
    yb = torch.empty((4, n), dtype=torch.complex64, device="cuda")
    S.spiir_process_batch([(ba, xa[:n], ya), (bb, xb[:n], yb)])
    torch.cuda.synchronize()
    assert np.array_equal(ya.cpu().numpy().view(np.uint64), ref_a[:, :n].view(np.uint64))
    assert np.array_equal(yb.cpu().numpy().view(np.uint64), ref_b[:, :n].view(np.uint64))
    blob = ba.save_state()
    bufa = torch.empty(n, device="cuda")
    bufb = torch.empty(n, device="cuda")
    g = S.Graph([(ba, bufa, ya), (bb, bufb, yb)])
    for i in range(1, 4):
        bufa.copy_(xa[i * n:(i + 1) * n])
        bufb.copy_(xb[i * n:(i + 1) * n])
        g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(ya.cpu().numpy().view(np.uint64), ref_a[:, i * n:(i + 1) * n].view(np.uint64)), i
        assert np.array_equal(yb.cpu().numpy().view(np.uint64), ref_b[:, i * n:(i + 1) * n].view(np.uint64)), i
    g.destroy()
    # restore the checkpoint taken after block 0 and replay block 1 eagerly
    ba.load_state(blob)
    ba.process_block(xa[n:2 * n], ya)
    torch.cuda.synchronize()
    assert np.array_equal(ya.cpu().numpy().view(np.uint64), ref_a[:, n:2 * n].view(np.uint64))
    for b in (alone_a, alone_b, ba, bb):
        b.destroy()
