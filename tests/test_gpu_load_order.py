"""The library and torch share one HIP runtime whatever is used first: a
fresh process that creates a context before touching torch's device API
still gets torch's GPU (torch ships a HIP runtime under the same soname as
ROCm's, and the binding imports torch before it loads the library)."""

import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = """
import paper_1411_2484_amd as ph
ctx = ph.Context(0, max_instances=16)
ids = ctx.seed_instances(32, 7, 1, (9, 17), 0, 0)
import torch
r = torch.full((4096,), -1.0, dtype=torch.float64, device="cuda:0")
ctx.generate(ph.make_requests(ids, [4096], [0]), None, None, r)
torch.cuda.synchronize()
assert bool(((r > 0) & (r < 1)).all())
ctx.close()
print("load order ok")
"""


def test_context_before_torch_device_use():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    out = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, capture_output=True, text=True, timeout=240)
    assert out.returncode == 0 and "load order ok" in out.stdout, out.stdout + out.stderr
