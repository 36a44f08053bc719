"""The Python binding in a fresh process: the library loaded and a bank
created before anything else touches the GPU leave torch's own HIP runtime
working, and the bank's (torch ships its own runtime next to the one the
library links; the binding starts torch's first)."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = """
import numpy as np
from paper_1702_02256_amd import spiir, workloads
tb = workloads.config3(n_templates=2, n_blocks=1).bank
spiir.spiir_plan(tb, 1024)            # loads the library (host-only call)
bank = spiir.Bank(tb, 1024)           # the first device call of the process
import torch
x = torch.from_numpy(workloads.noise_stream(1, 1024).astype(np.float32)).cuda()
z = torch.zeros((2, 1024), dtype=torch.complex64, device="cuda")
bank.process_block(x, z)
torch.cuda.synchronize()
assert bank.status()[0] == 0 and bool(torch.isfinite(torch.view_as_real(z)).all())
bank.destroy()
print("binding ok", flush=True)
"""


def test_bank_before_torch_touches_the_gpu():
    print("fresh process: bank created before torch uses the GPU", flush=True)
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, capture_output=True, text=True, timeout=110)
    assert r.returncode == 0 and "binding ok" in r.stdout, r.stdout[-2000:] + r.stderr[-2000:]
