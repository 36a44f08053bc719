"""Caller-owned workspaces and cloned banks, through the C ABI.

A bank created with SPIIR_WORKSPACE_CALLER owns no workspace; each request
brings one.  Where the workspace lives must not change a single bit of the
output or of the carried state, and a clone must behave as a bank created
afresh from the same descriptor.  Parity against the FP64 oracle at 1e-5 of
each template's max |z| (complex FP32 against FP64).
"""
import numpy as np
import pytest

import oracle
from paper_1702_02256_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _say(msg):
    print(msg, flush=True)


def _bank_tables(T=5, H=4, seed=77):
    nf = np.random.default_rng(seed).integers(10, 160, size=(T, H)).astype(np.int32)
    if T > 1 and H > 2:
        nf[1, 2] = 0  # an empty segment
    return W.random_bank(seed, nf, 4096, W.multirate_dmax(4096, H))


def _run(bank, xt, blocks, ws=None, peaks=False):
    import torch
    T = bank.n_templates
    n = int(sum(blocks))
    z = torch.zeros((T, n), dtype=torch.complex64, device="cuda")
    pos = 0
    for b in blocks:
        bank.process_block(xt[pos:pos + b], z[:, pos:pos + b], ws=ws)
        pos += b
    torch.cuda.synchronize()
    rc, _ = bank.status()
    assert rc == 0, rc
    return z.cpu().numpy()


def test_caller_workspace_equals_own_bitwise():
    import torch

    from paper_1702_02256_amd import spiir as S
    tb = _bank_tables()
    x = W.noise_stream(91, 4 * 4096)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    blocks = [4096, 8192, 1024, 512, 2048]  # 8192: two inner chunks of one call
    _say("workspace: own vs caller, 5 templates x 4 bands, blocks " + str(blocks))
    own = S.Bank(tb, 8192)
    cal = S.Bank(tb, 8192, workspace=S.WORKSPACE_CALLER)
    assert own.plan["workspace"] == S.WORKSPACE_OWN and cal.plan["workspace"] == S.WORKSPACE_CALLER
    assert own.workspace_bytes == cal.workspace_bytes > 0
    assert own.plan["footprint"] - cal.plan["footprint"] >= cal.workspace_bytes - 255
    ws = S.workspace_empty(cal.workspace_bytes)
    ws.fill_(0x7f)  # stale contents must not matter
    z0 = _run(own, xt, blocks)
    z1 = _run(cal, xt, blocks, ws=ws)
    assert np.array_equal(z0.view(np.uint32), z1.view(np.uint32))
    assert own.save_state()[128:] == cal.save_state()[128:]
    # the bank's own workspace can also be replaced per request
    own.reset()
    z2 = _run(own, xt, blocks, ws=ws)
    assert np.array_equal(z0.view(np.uint32), z2.view(np.uint32))
    zr = oracle.run_stream(tb, x[:int(sum(blocks))])
    e = np.max(np.abs(z1 - zr), axis=1) / np.max(np.abs(zr), axis=1)
    _say(f"caller workspace: max rel err {e.max():.3e}")
    assert e.max() <= TOL
    own.destroy()
    cal.destroy()


def test_caller_workspace_required_and_aligned():
    import torch

    from paper_1702_02256_amd import spiir as S
    tb = _bank_tables(T=2, H=2)
    cal = S.Bank(tb, 4096, workspace=S.WORKSPACE_CALLER)
    xt = torch.zeros(4096, dtype=torch.float32, device="cuda")
    z = torch.zeros((2, 4096), dtype=torch.complex64, device="cuda")
    with pytest.raises(S.SpiirError) as ei:
        cal.process_block(xt, z)
    assert ei.value.code == S.SPIIR_EINVAL
    ws = S.workspace_empty(cal.workspace_bytes + 256)
    with pytest.raises(S.SpiirError) as ei:
        cal.process_block(xt, z, ws=ws.data_ptr() + 4)
    assert ei.value.code == S.SPIIR_EINVAL
    assert cal.samples_done == 0
    cal.process_block(xt, z, ws=ws.data_ptr() + 256)
    torch.cuda.synchronize()
    assert cal.samples_done == 4096
    cal.destroy()


def test_batch_with_caller_workspaces_equals_alone():
    """Two caller-workspace banks in one batch, each with its own workspace, and
    the same workspaces reused by the next batch in stream order."""
    import torch

    from paper_1702_02256_amd import spiir as S
    ta, tb = _bank_tables(T=3, seed=5), _bank_tables(T=4, seed=6)
    x = W.noise_stream(92, 3 * 4096)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    ba = S.Bank(ta, 4096, workspace=S.WORKSPACE_CALLER)
    bb = S.Bank(tb, 4096, workspace=S.WORKSPACE_CALLER)
    wa, wb = S.workspace_empty(ba.workspace_bytes), S.workspace_empty(bb.workspace_bytes)
    za = torch.zeros((3, 3 * 4096), dtype=torch.complex64, device="cuda")
    zb = torch.zeros((4, 3 * 4096), dtype=torch.complex64, device="cuda")
    for i in range(3):
        sl = slice(i * 4096, (i + 1) * 4096)
        S.spiir_process_batch([(ba, xt[sl], za[:, sl], wa), (bb, xt[sl], zb[:, sl], wb)])
    torch.cuda.synchronize()
    alone_a = _run(S.Bank(ta, 4096), xt, [4096] * 3)
    alone_b = _run(S.Bank(tb, 4096), xt, [4096] * 3)
    assert np.array_equal(za.cpu().numpy().view(np.uint32), alone_a.view(np.uint32))
    assert np.array_equal(zb.cpu().numpy().view(np.uint32), alone_b.view(np.uint32))


def test_clone_is_a_fresh_bank():
    import torch

    from paper_1702_02256_amd import spiir as S
    tb = _bank_tables(T=6, H=5, seed=13)
    x = W.noise_stream(93, 4 * 4096)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    _say("clone: 6 templates x 5 bands, cloned after 2 blocks of its source")
    src = S.Bank(tb, 4096, precision="fp32_compensated")
    _run(src, xt, [4096, 4096])
    cl = src.clone()
    assert cl.plan == src.plan
    fresh = S.Bank(tb, 4096, precision="fp32_compensated")
    zc = _run(cl, xt, [4096, 2048, 2048, 4096])
    zf = _run(fresh, xt, [4096, 2048, 2048, 4096])
    assert np.array_equal(zc.view(np.uint32), zf.view(np.uint32))
    # the source is unchanged by the clone: it continues where it was
    ref = S.Bank(tb, 4096, precision="fp32_compensated")
    _run(ref, xt, [4096, 4096])
    assert src.save_state() == ref.save_state()
    zr = oracle.run_stream(tb, x[:zc.shape[1]])
    e = np.max(np.abs(zc - zr), axis=1) / np.max(np.abs(zr), axis=1)
    _say(f"clone: max rel err {e.max():.3e}")
    assert e.max() <= TOL
    # a state blob of the source loads into the clone (same layout)
    cl.load_state(src.save_state())
    assert cl.samples_done == src.samples_done
    for b in (src, cl, fresh, ref):
        b.destroy()


def test_clone_of_a_caller_workspace_bank_and_of_a_time_split_bank():
    import torch

    from paper_1702_02256_amd import spiir as S
    tb = _bank_tables(T=2, H=3, seed=21)
    x = W.noise_stream(94, 2 * 4096)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    for kw in ({"workspace": S.WORKSPACE_CALLER}, {"time_chunks": 8}):
        src = S.Bank(tb, 4096, **kw)
        cl = src.clone()
        ws = S.workspace_empty(cl.workspace_bytes) if kw.get("workspace") else None
        zc = _run(cl, xt, [4096, 4096], ws=ws)
        zs = _run(src, xt, [4096, 4096], ws=ws)
        assert np.array_equal(zc.view(np.uint32), zs.view(np.uint32)), kw
        src.destroy()
        cl.destroy()
