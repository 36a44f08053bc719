"""A bank from the host planner (single rate -> multi rate) on the GPU, against
the FP64 oracle run on the same planned tables."""
import numpy as np
import pytest

import oracle
from paper_1702_02256_amd import planner as PL
from paper_1702_02256_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_planned_bank_parity():
    import torch
    from paper_1702_02256_amd import spiir as S
    rng = np.random.default_rng(17)
    R, T, M = 4096, 12, 150
    f = rng.uniform(5, 900, T * M) * rng.choice([-1, 1], T * M)
    r = rng.uniform(0.99, 0.9999, T * M)
    tb = W.BankTables(base_rate=R, n_filters=np.full((T, 1), M, np.int32),
                      a1=r * np.exp(2j * np.pi * f / R),
                      b0=(rng.standard_normal(T * M) + 1j * rng.standard_normal(T * M)) * 1e-3,
                      delay=rng.integers(0, 2048, T * M).astype(np.int32))
    pl = PL.plan_multirate(tb, 6, pad_pow2=True)
    print(f"planned bank: filters per band {pl.n_filters.sum(axis=0).tolist()}", flush=True)
    x = W.noise_stream(3, 3 * R)
    bank = S.Bank(pl, R)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    z = torch.empty((T, 3 * R), dtype=torch.complex64, device="cuda")
    for i in range(3):
        bank.process_block(xt[i * R:(i + 1) * R], z[:, i * R:(i + 1) * R])
    torch.cuda.synchronize()
    bank.destroy()
    zr = oracle.run_stream(pl, x)
    zg = z.cpu().numpy().astype(np.complex128)
    e = np.max(np.abs(zg - zr), axis=1) / np.max(np.abs(zr), axis=1)
    print(f"planned bank: max rel err {e.max():.3e}", flush=True)
    assert e.max() <= 1e-5
