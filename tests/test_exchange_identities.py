"""The DFT identities behind the divide kernel's split exchanges (N = 128).

Half of the work-group keeps its stage-B spectrum and its stage-C sequence
with the two halves swapped, so that both halves of every exchange pass use
the same registers.  That rests on three facts about an M-point DFT (M even)
and the modulus projection, checked here on the CPU:

* negating the odd-indexed inputs swaps the two halves of the output;
* swapping the two halves of the input multiplies the output by (-1)^k;
* the relaxed modulus projection commutes with a change of sign, except where
  the spectrum is zero and the phase is set to zero, where the sign has to be
  applied to the value set.

Each sign change is exact in floating point, and the radix-2 butterflies are
symmetric under a change of sign, so the identities also hold bit for bit for
a decimation-in-frequency transform written the way the kernel's is.
"""
import numpy as np
import pytest


def dif_fft(x):
    """Radix-2 decimation in frequency, float32 arithmetic, natural-order output."""
    x = np.array(x, dtype=np.complex64)
    m = len(x)
    half = m // 2
    while half >= 1:
        span = 2 * half
        for b in range(0, m, span):
            for i in range(half):
                a, c = x[b + i], x[b + i + half]
                w = np.complex64(np.exp(-2j * np.pi * i / span))
                x[b + i] = a + c
                x[b + i + half] = (a - c) * w
        half //= 2
    bits = m.bit_length() - 1
    rev = [int(format(k, f"0{bits}b")[::-1], 2) for k in range(m)]
    return x[rev]


def modulus(X, A, c=2.0):
    """Relaxed modulus projection of one spectrum value (phase 0 where X = 0)."""
    mag = np.abs(X)
    return np.where(mag > 0, X * (c * A / np.where(mag > 0, mag, 1) + 1 - c), c * A + 0j)


@pytest.mark.parametrize("m", [8, 32])
def test_odd_negation_swaps_output_halves(m):
    rng = np.random.default_rng(m)
    x = (rng.standard_normal(m) + 1j * rng.standard_normal(m)).astype(np.complex64)
    sign = np.where(np.arange(m) % 2 == 1, -1, 1).astype(np.float32)
    X = dif_fft(x)
    Xm = dif_fft(x * sign)
    assert np.array_equal(Xm, np.roll(X, m // 2))           # bit for bit
    assert np.allclose(np.fft.fft(x * sign), np.roll(np.fft.fft(x), m // 2))


@pytest.mark.parametrize("m", [8, 32])
def test_half_swapped_input_signs_the_output(m):
    rng = np.random.default_rng(100 + m)
    x = (rng.standard_normal(m) + 1j * rng.standard_normal(m)).astype(np.complex64)
    sign = np.where(np.arange(m) % 2 == 1, -1, 1).astype(np.float32)
    X = dif_fft(x)
    Xs = dif_fft(np.roll(x, m // 2))
    assert np.array_equal(np.abs(Xs), np.abs(X))
    assert np.array_equal(Xs, X * sign)                      # bit for bit
    # and the inverse direction: a half-swapped spectrum gives (-1)^n times the sequence
    assert np.allclose(np.fft.ifft(np.roll(np.fft.fft(x), m // 2)), x * sign, atol=1e-6)


def test_modulus_projection_commutes_with_sign_except_at_zero():
    rng = np.random.default_rng(7)
    X = (rng.standard_normal(64) + 1j * rng.standard_normal(64))
    X[::9] = 0                                              # exact zeros take phase 0
    A = rng.uniform(0.5, 2.0, 64)
    direct = modulus(X, A)
    via_sign = -modulus(-X, A)
    nz = X != 0
    assert np.array_equal(direct[nz], via_sign[nz])
    # at zero the value set must carry the sign: -P(-0) != P(0) ...
    assert not np.allclose(direct[~nz], via_sign[~nz])
    # ... so a holder of -X multiplies the phase-0 value by -1, and negating its
    # result gives P(X) everywhere
    held = modulus(-X, A)
    held = np.where(nz, held, -1 * held)
    assert np.array_equal(-held, direct)
