"""The autotuner picks a valid launch shape and block length on the device,
and the tuned bank stays within the parity bar."""
import numpy as np
import pytest

import oracle
from paper_1702_02256_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_tune_packing_and_block(tmp_path, monkeypatch):
    import torch
    from paper_1702_02256_amd import autotune as A
    from paper_1702_02256_amd import spiir as S
    monkeypatch.setenv(A.CACHE_ENV, str(tmp_path / "tune.json"))
    tb = W.config4(n_templates=64, templates=list(range(64)), n_blocks=1).bank
    t = A.tune_packing(tb, 1024, steps=2)
    assert not t["cached"] and len(t["candidates"]) >= 3
    tried = {(c["filters_per_lane"], c["waves_per_group"], c["time_chunks"]) for c in t["candidates"]}
    assert (t["filters_per_lane"], t["waves_per_group"], t["time_chunks"]) in tried
    # a bank this small also gets the time-split candidates, among them the
    # split the planner picks for each default shape
    assert any(c[2] > 1 for c in tried)
    for F, Wv in A.DEFAULT_CANDIDATES:
        P = S.spiir_plan(tb, 1024, filters_per_lane=F, waves_per_group=Wv,
                         time_chunks=S.TIME_CHUNKS_AUTO)["time_chunks"]
        assert P == 1 or (F, Wv, P) in tried, (F, Wv, P)
    assert A.tune_packing(tb, 1024)["cached"]
    b = A.tune_block(tb, blocks=(256, 1024, 4096), steps=2)
    assert b["block"] in (256, 1024, 4096)
    # the tuned bank still meets the bar against the oracle
    x = W.noise_stream(91, 2048)
    bank = S.Bank(tb, 1024, **A.tuned_bank_kwargs(tb, 1024))
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    z = torch.zeros((64, 2048), dtype=torch.complex64, device="cuda")
    bank.process_block(xt[:1024], z[:, :1024])
    bank.process_block(xt[1024:], z[:, 1024:])
    torch.cuda.synchronize()
    zr = oracle.run_stream(tb, x)
    zg = z.cpu().numpy().astype(np.complex128)
    err = np.max(np.abs(zg - zr), axis=1) / np.max(np.abs(zr), axis=1)
    assert err.max() <= 1e-5
    bank.destroy()
