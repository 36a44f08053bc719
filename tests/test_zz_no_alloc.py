"""spiir_process_block_noalloc against spiir_process_block, through the C ABI.

The no-allocation entry point runs the same launch sequence with the
workspace in the library's static device array.  Two calls in a row, the
second with a smaller block, must give the existing entry point's output and
carried state bit for bit (the integer bar: the two share every kernel, so
any difference is a bug, not rounding); the output is also held to the FP64
oracle at 1e-5 of each template's max |z|.
"""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_1702_02256_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _say(msg):
    print(msg, flush=True)


def _tables(T, H, seed, lo=10, hi=200):
    nf = np.random.default_rng(seed).integers(lo, hi, size=(T, H)).astype(np.int32)
    return W.random_bank(seed, nf, 4096, W.multirate_dmax(4096, H))


@pytest.mark.parametrize("workspace", [0, 1])
def test_noalloc_equals_process_block_two_calls(workspace):
    import torch

    from paper_1702_02256_amd import spiir as S
    tb = _tables(6, 5, 301)
    blocks = [4096, 1024]  # the second call is smaller
    n = sum(blocks)
    x = W.noise_stream(302, n)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    _say(f"noalloc: 6 templates x 5 bands, blocks {blocks}, bank workspace mode {workspace}")
    ref = S.Bank(tb, 4096, workspace=S.WORKSPACE_OWN)
    nob = S.Bank(tb, 4096, workspace=workspace)
    assert nob.workspace_bytes <= S.NOALLOC_MAX_WORKSPACE
    z0 = torch.zeros((6, n), dtype=torch.complex64, device="cuda")
    z1 = torch.full((6, n), float("nan"), dtype=torch.complex64, device="cuda")
    pos = 0
    for b in blocks:
        ref.process_block(xt[pos:pos + b], z0[:, pos:pos + b])
        nob.process_block_noalloc(xt[pos:pos + b], z1[:, pos:pos + b])
        pos += b
    torch.cuda.synchronize()
    a, c = z0.cpu().numpy(), z1.cpu().numpy()
    assert np.array_equal(a.view(np.uint32), c.view(np.uint32))
    assert ref.save_state()[128:] == nob.save_state()[128:]
    assert nob.samples_done == n
    rc, _ = nob.status()
    assert rc == 0
    zr = oracle.run_stream(tb, x)
    e = np.max(np.abs(c - zr), axis=1) / np.max(np.abs(zr), axis=1)
    _say(f"noalloc: max rel err {e.max():.3e}")
    assert e.max() <= TOL
    ref.destroy()
    nob.destroy()


def test_noalloc_rejects_a_workspace_beyond_the_static_array():
    import torch

    from paper_1702_02256_amd import spiir as S
    # 300 templates of the multi-rate shape need about 22 MB of workspace per
    # 4096-sample chunk; 600 need more than the 32 MiB array
    tb = W.config3(n_templates=600, n_blocks=1).bank
    big = S.Bank(tb, 4096, workspace=S.WORKSPACE_CALLER)
    assert big.workspace_bytes > S.NOALLOC_MAX_WORKSPACE
    _say(f"noalloc: 600-template bank, workspace {big.workspace_bytes} B > {S.NOALLOC_MAX_WORKSPACE}")
    xt = torch.zeros(4096, dtype=torch.float32, device="cuda")
    z = torch.zeros((600, 4096), dtype=torch.complex64, device="cuda")
    lib = S.load_library()
    rc = lib.spiir_process_block_noalloc(big._h, xt.data_ptr(), 4096, z.data_ptr(), 4096,
                                         C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == S.SPIIR_ENOMEM
    assert big.samples_done == 0
    # invalid arguments are refused before the size check, as by spiir_process_block
    rc = lib.spiir_process_block_noalloc(big._h, xt.data_ptr(), 4095, z.data_ptr(), 4096, None)
    assert rc == S.SPIIR_EINVAL
    big.destroy()
