"""The binding works when the library is loaded before torch touches the GPU.

torch and libahpp.so both link libamdhip64.so.7 and a process keeps the copy
loaded first; the binding loads torch's before the library, so a program that
calls load_library() first still gets torch tensors its kernels can use.  The
check runs in a fresh interpreter, where nothing has imported torch yet.
"""

import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, sys.argv[1])
from paper_2512_11606_amd import ahpp, synth
ahpp.load_library()
g = synth.make_graph("tiny")
dg = ahpp.load_graph(g)
res = ahpp.ahpp_query(dg, 3, 1e-6, k=4)
import torch
pi = res.pi.cpu()
assert pi.shape == (g.n_u,) and float(pi[3]) >= 0.15 - 1e-6, float(pi[3])
assert int(res.topk_n.cpu()[0]) == 4
print("child ok", flush=True)
"""


def test_library_loaded_before_torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[gpu-case] load order child", flush=True)
    out = subprocess.run([sys.executable, "-c", CHILD, ROOT], capture_output=True, text=True, timeout=240)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "child ok" in out.stdout
