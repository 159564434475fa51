"""The library works when it is opened before the caller has touched torch.

torch bundles a HIP runtime under the same sonames as ROCm's; a library opened
first would bind to the other copy and find no device.  load_library
initialises torch before it opens the library, so a fresh process that calls
it first and then runs a scan must succeed (GPU, one child process)."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys
sys.path.insert(0, sys.argv[1]); sys.path.insert(0, sys.argv[1] + "/tests")
import paper_2311_11466_amd as pk
pk.load_library()                      # first: nothing has imported torch yet
import numpy as np
import torch
from ptysynth import make_scan
scan = make_scan("tiny_n32")
dev = torch.device("cuda", 0)
g = pk.Scan(torch.as_tensor(scan.pos).to(dev), torch.as_tensor(scan.intensity.astype(np.float32)).to(dev),
            torch.as_tensor(scan.obj0.astype(np.complex64)).to(dev),
            torch.as_tensor(scan.probe0.astype(np.complex64)).to(dev), blind=True)
g.set_algorithm_named("DC")
g.iterate(2)
m = g.metrics()
g.close()
assert np.isfinite(m["fourier_err"]), m
print("load order ok", m["iteration"], flush=True)
"""


def test_library_opened_before_torch():
    print("case: library opened before torch, child process", flush=True)
    r = subprocess.run([sys.executable, "-c", SCRIPT, ROOT], capture_output=True, text=True, timeout=180)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0 and "load order ok 1" in r.stdout
