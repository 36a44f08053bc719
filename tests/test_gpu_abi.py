"""The C ABI's error paths and its use without Python, on the GPU.

* a C program (tests/c/spiir_c_abi.c) that never loads Python or torch creates
  a multi-rate bank, filters two blocks from hipMalloc buffers and destroys it;
  its z is compared with the FP64 oracle at 1e-5 of each template's max |z|;
* the same bank twice in one batch: SPIIR_EORDER, nothing enqueued;
* device memory running out: spiir_clone and spiir_create return
  SPIIR_ENOMEM with *out NULL, and work again once memory is freed;
* a launch sequence that fails (forced from the host through the library's
  SPIIR_TEST_FAIL_ENQUEUE hook, no device fault): the bank is poisoned and
  every later call on it returns SPIIR_EDEVICE, destroy still frees it;
* one HIP runtime in a process that uses torch and the library together.
"""
import ctypes as C
import os
import subprocess
import sys
import tempfile

import numpy as np
import pytest

import oracle
from paper_1702_02256_amd import workloads as W

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
C_BIN = os.path.join(ROOT, "tests", "c", "spiir_c_abi")


def _say(msg):
    print(msg, flush=True)


def _write_input(path, tb, x, max_block, n_blocks, block, precision):
    with open(path, "wb") as f:
        np.array([tb.n_templates, tb.n_bands, tb.base_rate, len(tb.h_down), len(tb.h_up), max_block,
                  n_blocks, block, precision], np.int32).tofile(f)
        np.ascontiguousarray(tb.n_filters.reshape(-1), np.int32).tofile(f)
        np.ascontiguousarray(tb.a1, np.complex128).view(np.float64).tofile(f)
        np.ascontiguousarray(tb.b0, np.complex128).view(np.float64).tofile(f)
        np.ascontiguousarray(tb.delay, np.int32).tofile(f)
        np.ascontiguousarray(tb.h_down, np.float64).tofile(f)
        np.ascontiguousarray(tb.h_up, np.float64).tofile(f)
        np.ascontiguousarray(x[:n_blocks * block], np.float32).tofile(f)


def test_c_program_without_python():
    assert os.path.exists(C_BIN), "build() compiles tests/c/spiir_c_abi"
    nf = np.random.default_rng(55).integers(20, 150, size=(5, 4)).astype(np.int32)
    tb = W.random_bank(55, nf, 4096, W.multirate_dmax(4096, 4))
    n_blocks, block = 3, 2048
    x = W.noise_stream(56, n_blocks * block)
    with tempfile.TemporaryDirectory() as d:
        inp, out = os.path.join(d, "in.bin"), os.path.join(d, "out.bin")
        _write_input(inp, tb, x, 4096, n_blocks, block, 1)
        env = {k: v for k, v in os.environ.items() if not k.startswith("PYTHON")}
        _say("C program: 5 templates x 4 bands, 3 blocks of 2048, compensated sum")
        r = subprocess.run([C_BIN, inp, out], capture_output=True, text=True, timeout=120, env=env)
        _say(r.stdout + r.stderr)
        assert r.returncode == 0, r.stderr
        runtimes = {l.split("runtime: ", 1)[1].strip() for l in r.stdout.splitlines() if l.startswith("runtime: ")}
        assert len({os.path.realpath(p) for p in runtimes}) == 1, runtimes
        assert not any("torch" in p for p in runtimes), runtimes
        z = np.fromfile(out, np.complex64).reshape(tb.n_templates, n_blocks * block)
    zr = oracle.run_stream(tb, x)
    e = np.max(np.abs(z - zr), axis=1) / np.max(np.abs(zr), axis=1)
    _say(f"C program: max rel err {e.max():.3e}")
    assert e.max() <= 1e-5


def test_same_bank_twice_in_a_batch_is_eorder():
    import torch

    from paper_1702_02256_amd import spiir as S
    tb = W.random_bank(7, np.full((2, 2), 30, np.int32), 4096, W.multirate_dmax(4096, 2))
    b = S.Bank(tb, 4096)
    other = S.Bank(tb, 4096)
    xt = torch.randn(4096, device="cuda")
    z = torch.full((2, 4096), 7.0, dtype=torch.complex64, device="cuda")
    z2 = torch.zeros((2, 4096), dtype=torch.complex64, device="cuda")
    with pytest.raises(S.SpiirError) as ei:
        S.spiir_process_batch([(b, xt[:2048], z[:, :2048]), (other, xt, z2), (b, xt[2048:], z[:, 2048:])])
    assert ei.value.code == S.SPIIR_EORDER
    torch.cuda.synchronize()
    assert b.samples_done == 0 and other.samples_done == 0
    assert torch.all(z == 7.0) and torch.all(z2 == 0)   # nothing was enqueued


def test_enomem_when_device_memory_runs_out():
    import torch

    from paper_1702_02256_amd import spiir as S
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    # one filter per template, a million templates: about 33 GB, most of it
    # the workspace; clones of it fill the device until one no longer fits
    T = 1_000_000
    nf = np.ones((T, 1), np.int32)
    tb = W.BankTables(4096, nf, np.full(T, 0.5 + 0.1j), np.full(T, 1e-3 + 0j), np.zeros(T, np.int32))
    free0, total = torch.cuda.mem_get_info()
    big = S.Bank(tb, 4096)
    fp = big.plan["footprint"]
    free1, _ = torch.cuda.mem_get_info()
    _say(f"bank footprint {fp / 1e9:.2f} GB, device memory taken {(free0 - free1) / 1e9:.2f} GB, "
         f"free {free1 / 1e9:.1f} of {total / 1e9:.1f} GB")
    assert 0.95 * fp <= free0 - free1 <= 1.05 * fp + (64 << 20)
    lib = S.load_library()
    clones, rc = [], S.SPIIR_OK
    try:
        for _ in range(int(total // fp) + 2):
            h = C.c_void_p(12345)
            rc = lib.spiir_clone(big._h, None, C.byref(h))
            if rc != S.SPIIR_OK:
                assert h.value is None
                break
            clones.append(h.value)
        _say(f"{len(clones)} clones fit; the next returned {S.spiir_strerror(rc)}")
        assert rc == S.SPIIR_ENOMEM
        h = C.c_void_p(12345)
        hold = S._DescHolder(tb, 4096)
        assert lib.spiir_create(C.byref(hold.desc), None, C.byref(h)) == S.SPIIR_ENOMEM
        assert h.value is None
    finally:
        for h in clones:
            lib.spiir_destroy(h)
    # memory is back: a clone fits again and works
    cl = big.clone()
    xt = torch.zeros(4096, device="cuda")
    z = torch.zeros((T, 8), dtype=torch.complex64, device="cuda")
    cl.process_block(xt[:8], z)
    torch.cuda.synchronize()
    assert cl.status()[0] == 0
    cl.destroy()
    big.destroy()


_POISON = r"""
import torch, numpy as np
from paper_1702_02256_amd import spiir as S, workloads as W
tb = W.random_bank(9, np.full((2, 3), 20, np.int32), 4096, W.multirate_dmax(4096, 3))
b = S.Bank(tb, 4096)
xt = torch.zeros(4096, device="cuda")
z = torch.zeros((2, 4096), dtype=torch.complex64, device="cuda")
codes = []
for call in (lambda: b.process_block(xt, z), lambda: b.process_block(xt, z), b.reset, b.save_state):
    try:
        call()
        codes.append(0)
    except S.SpiirError as e:
        codes.append(e.code)
codes.append(b.status()[0])
codes.append(b.samples_done)
b.destroy()
print("codes", codes)
"""


def test_failed_launch_poisons_the_bank():
    env = dict(os.environ, SPIIR_TEST_FAIL_ENQUEUE="1")
    r = subprocess.run([sys.executable, "-c", _POISON], capture_output=True, text=True, timeout=300,
                       env=env, cwd=ROOT)
    _say(r.stdout + r.stderr[-2000:])
    assert r.returncode == 0
    codes = [l for l in r.stdout.splitlines() if l.startswith("codes")][0]
    # the first call fails and poisons the bank, every later one reports it
    assert codes == "codes [-3, -3, -3, -3, -3, 0]", codes


def test_one_hip_runtime_with_torch():
    import torch

    from paper_1702_02256_amd import spiir as S
    torch.zeros(1, device="cuda")
    S.load_library()
    paths = S.hip_runtime_paths()
    _say(f"HIP runtime: {paths}")
    assert len(paths) == 1
