"""More N = 256 patterns than one launch of a pass can hold (GPU, ~170 GB).

The three passes of the N = 256 divide put the pattern in the grid's second
dimension, which the device limits to 65536; a scan with more patterns runs
each pass as several launches.  After one iteration each pattern's y is
P_D of its own first exit wave P_0 S_j O_0, so the y of patterns on both
sides of the launch boundary must equal, bit for bit, what a small scan of
just those patterns computes.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N = 256
J = 65535 + 9            # two launches per pass: 65535 patterns, then 9
OBJ = 1024


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.timeout(600)
def test_more_patterns_than_one_launch():
    import torch
    import paper_2311_11466_amd as pk
    dev = torch.device("cuda", 0)
    if torch.cuda.get_device_properties(0).total_memory < 200 * 2**30:
        pytest.skip("needs about 170 GB of device memory")
    say(f"case: N = {N}, J = {J} patterns (two launches per pass)")
    rng = np.random.default_rng(12)
    pos = torch.as_tensor(rng.integers(0, OBJ - N + 1, size=(J, 2)).astype(np.int32), device=dev)
    obj = torch.as_tensor((rng.uniform(0.5, 1, (OBJ, OBJ)) * np.exp(1j * rng.uniform(-1, 1, (OBJ, OBJ))))
                          .astype(np.complex64), device=dev)
    probe = torch.as_tensor((rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))).astype(np.complex64),
                            device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(5)
    intensity = torch.rand((J, N, N), device=dev, generator=gen) * 100.0
    big = pk.Scan(pos, intensity, obj, probe, full_metrics=False)
    big.set_algorithm_named("RAAR", 0.75)
    big.iterate(1)
    y_big = big.get_state()[1]
    big.close()
    del big
    sel = [0, 65533, 65534, 65535, 65536, J - 1]       # both launches, both sides of the boundary
    y_sel = y_big[sel].clone()
    del y_big
    torch.cuda.empty_cache()
    idx = torch.as_tensor(sel, device=dev)
    small = pk.Scan(pos[idx].contiguous(), intensity[idx].contiguous(), obj, probe, full_metrics=False)
    small.set_algorithm_named("RAAR", 0.75)
    small.iterate(1)
    y_small = small.get_state()[1]
    small.close()
    for k, j in enumerate(sel):
        assert torch.equal(y_sel[k].view(torch.int64), y_small[k].view(torch.int64)), j
    assert bool(torch.isfinite(y_sel.view(torch.float32)).all())
