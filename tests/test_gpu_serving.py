"""Serving on the GPU: every stream's output from the continuous-batching
scheduler (blocks merged, banks batched, batches overlapping on two device
streams) equals, bit for bit, the same stream processed alone block by block,
and matches the FP64 oracle within 1e-5."""
import numpy as np
import pytest

import oracle
from paper_1702_02256_amd import serving as SV
from paper_1702_02256_amd import workloads as W

pytestmark = pytest.mark.gpu


def _banks(n_streams=3, T=48, seed=9):
    return [W.config3(seed=seed * 10 + s, n_templates=T, n_blocks=1).bank for s in range(n_streams)]


def _alone(tables, x, block=4096):
    import torch
    from paper_1702_02256_amd import spiir as S
    bank = S.Bank(tables, block)
    xt = torch.from_numpy(np.asarray(x, np.float32)).cuda()
    z = torch.empty((tables.n_templates, len(x)), dtype=torch.complex64, device="cuda")
    for i in range(0, len(x), block):
        n = min(block, len(x) - i)
        bank.process_block(xt[i:i + n], z[:, i:i + n])
    torch.cuda.synchronize()
    out = z.cpu().numpy()
    bank.destroy()
    return out


def _collect(be, s):
    import torch
    torch.cuda.synchronize()
    parts = sorted(be.outputs[s], key=lambda p: p[0])
    return np.concatenate([z.cpu().numpy() for _, z in parts], axis=1)


@pytest.mark.parametrize("policy,speed", [("batched", 40.0), ("plain", 40.0), ("batched", 1000.0)])
def test_serving_equals_alone(policy, speed):
    banks = _banks()
    arr = W.serving_arrivals(77, 3, 4.0, rate_hz=4096, speed=speed)
    xs = [W.noise_stream(300 + s, int(l.sum())) for s, (l, _) in enumerate(arr)]
    print(f"serving {policy} x{speed}: blocks {[len(l) for l, _ in arr]}", flush=True)
    be = SV.HipBackend(xs, n_streams=2, keep_outputs=True)
    sch = SV.Scheduler(be, banks, max_block=8192, policy=policy)
    st = sch.run(SV.make_arrivals(arr))
    summ = st.summary()
    print(summ, flush=True)
    assert summ["blocks"] == sum(len(l) for l, _ in arr)
    if policy == "batched" and speed >= 1000:
        assert st.requests < summ["blocks"]
    for s in range(3):
        got = _collect(be, s)
        assert np.array_equal(got, _alone(banks[s], xs[s])), s
    for s in range(3):  # sampled templates of every stream against the oracle
        sel = [0, 17 + s, 47]
        zr = oracle.run_stream(banks[s].subset(sel), xs[s])
        got = _collect(be, s)[sel].astype(np.complex128)
        err = np.max(np.abs(got - zr), axis=1) / np.max(np.abs(zr), axis=1)
        assert err.max() <= 1e-5, (s, err)


def test_admission_by_footprint_on_the_device():
    """The HBM budget holds two of the three banks: the third waits until a
    stream ends and its bank is released, then starts from its stream's first
    block; every stream's output still equals the stream alone and the oracle."""
    from paper_1702_02256_amd import spiir as S
    banks = _banks(T=32, seed=12)
    arr = W.serving_arrivals(78, 3, 3.0, rate_hz=4096, speed=20.0)
    arr = [(l[: 2 + 3 * s], t[: 2 + 3 * s]) for s, (l, t) in enumerate(arr)]  # streams end one after another
    xs = [W.noise_stream(400 + s, int(l.sum())) for s, (l, _) in enumerate(arr)]
    fp = [S.spiir_footprint(b, 8192) for b in banks]
    budget = fp[0] + fp[1] + 1
    assert fp[2] > budget - fp[0] - fp[1]
    be = SV.HipBackend(xs, n_streams=2, keep_outputs=True)
    sch = SV.Scheduler(be, banks, max_block=8192, hbm_budget=budget)
    st = sch.run(SV.make_arrivals(arr), release_finished=True)
    print(st.summary(), st.admitted_at, flush=True)
    assert st.admitted_at[0] == 0.0 and st.admitted_at[1] == 0.0
    assert st.admitted_at[2] > 0.0, "the third bank must wait for the budget"
    assert sch.used <= budget
    for s in range(3):
        got = _collect(be, s)
        assert np.array_equal(got, _alone(banks[s], xs[s])), s
        zr = oracle.run_stream(banks[s].subset([1, 30]), xs[s])
        err = np.max(np.abs(got[[1, 30]].astype(np.complex128) - zr), axis=1) / np.max(np.abs(zr), axis=1)
        assert err.max() <= 1e-5, (s, err)
