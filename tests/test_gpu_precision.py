"""The compensated sum over filters where the sum's rounding is what limits
the result.

On the multi-rate workloads the FP32 recurrence sets the error (about 2e-6 of
max |z| either way), so compensating the sum changes nothing measurable.  Here
the recurrence is one rounded product per filter (a1 = 0, no memory), each
lane holds one filter (no in-lane sum), the 256 filters of each workgroup are
coherent (b0 of one sign, zero delay; the signs follow the planner's placement
of a single delay class), so the partial sums inside a piece grow
to hundreds of times a single output, and the two workgroups' pieces cancel
to about 1%.  The plain sum's roundings are then relative to the large
partial sums; the compensated sum (cross-lane levels accumulated in FP64)
leaves only the products' and the run and piece totals' roundings, and must be
measurably closer to the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_1702_02256_amd import workloads as W

pytestmark = pytest.mark.gpu


def _err(tb, x, precision):
    import torch

    from paper_1702_02256_amd import spiir as S
    bank = S.Bank(tb, len(x), precision=precision, filters_per_lane=1, waves_per_group=4)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    z = torch.zeros((tb.n_templates, len(x)), dtype=torch.complex64, device="cuda")
    bank.process_block(xt, z)
    torch.cuda.synchronize()
    bank.destroy()
    zg = z.cpu().numpy().astype(np.complex128)
    # the oracle gets the same FP32 input, so only the arithmetic differs
    zr = oracle.run_stream(tb, x.astype(np.float32).astype(np.float64))
    return float(np.max(np.abs(zg - zr)) / np.max(np.abs(zr)))


def test_compensated_sum_beats_plain_where_the_sum_dominates():
    rng = np.random.default_rng(808)
    pos = rng.uniform(0.5, 1.5, 256) + 1j * rng.uniform(0.5, 1.5, 256)
    neg = -pos * (1.0 + 0.02 * rng.uniform(0.0, 1.0, 256))
    # With one delay class the planner deals filter j to half-wave row j mod 16
    # of the template's 512 lanes (rows 0-7 are the first workgroup, 8-15 the
    # second), so the filters with j mod 16 < 8 form the first workgroup's piece
    # and the others the second's.
    first = (np.arange(512) % 16) < 8
    b0 = np.empty(512, np.complex128)
    b0[first] = pos
    b0[~first] = neg
    M = len(b0)
    tb = W.BankTables(4096, np.array([[M]], np.int32), np.zeros(M, np.complex128), b0,
                      np.zeros(M, np.int32))
    x = W.noise_stream(809, 4096)
    e_plain = _err(tb, x, "fp32")
    e_comp = _err(tb, x, "fp32_compensated")
    print(f"cancelling 512-filter bank: plain {e_plain:.3e}, compensated {e_comp:.3e}", flush=True)
    assert e_comp < 0.5 * e_plain, (e_plain, e_comp)
