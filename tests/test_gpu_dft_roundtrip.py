"""The divide's 2-D DFTs on their own (GPU, every pattern size).

With (a, b, c) = (1, 0, 0) the iteration is x_{k+1} = P_C^0 P_D^0 x_k = x_k,
formed through the divide: the forward DFT, the spectrum scaled by 1/N^2 (the
relaxed modulus step with c = 0), and the inverse DFT.  One iteration thus
returns x after a float32 DFT round trip, which must reproduce x to the
rounding of the transforms: about 2 log2(N) stages of float32 butterflies, a
relative L2 error of a few 1e-7 (gate 1e-6).  A wrong twiddle, index or sign
in either transform moves the result by order one.  The N = 256 case runs the
three-pass form, the others the fused kernel.
"""
import sys

import numpy as np
import pytest

from gpu_helpers import gpu_scan, rel_l2, to_dev
from ptysynth import make_scan
from ptysynth.scans import small_config

pytestmark = pytest.mark.gpu

GATE = 1e-6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


SCANS = {
    32: lambda: make_scan("tiny_n32"),
    64: lambda: make_scan(small_config("p64", 64, 5, 24, jitter=2, photons=1e6, seed=31)),
    128: lambda: make_scan(small_config("p128", 128, 4, 40, jitter=2, photons=1e6, seed=41)),
    256: lambda: make_scan(small_config("p256", 256, 3, 80, jitter=3, photons=1e5, seed=51)),
}


@pytest.mark.parametrize("n", [32, 64, 128, 256])
def test_dft_round_trip(n):
    scan = SCANS[n]()
    say("case: DFT round trip, N =", n)
    rng = np.random.default_rng(900 + n)
    x = (rng.standard_normal((scan.n_pos, n, n)) + 1j * rng.standard_normal((scan.n_pos, n, n))).astype(np.complex64)
    x[0, 0, :] = 0                                            # a zero row, and one spike, in the first pattern
    x[0, n // 2, n // 3] = 1e3
    g = gpu_scan(scan)
    g.set_state(to_dev(x), None, to_dev(scan.obj0.astype(np.complex64)), to_dev(scan.probe0.astype(np.complex64)))
    g.set_algorithm(1.0, 0.0, 0.0)
    g.iterate(1)
    x1 = g.get_state()[0].cpu().numpy()
    g.close()
    err = rel_l2(x1, x)
    worst = max(rel_l2(x1[j], x[j]) for j in range(scan.n_pos))
    say(f"  relative L2 error {err:.3e}, worst pattern {worst:.3e}")
    assert err <= GATE and worst <= GATE, (err, worst)
