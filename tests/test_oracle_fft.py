"""Pins of the oracle's FFT (Sec. 2.1: all fields are transformed along x1).

The oracle's radix-2 transform is checked against numpy's FFT, an independent
library routine, for every power-of-two length up to 4096 and for the
real-row forward/inverse pair the field solver uses.
"""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 64, 256, 1024, 4096])
def test_complex_fft_matches_numpy(n):
    gen = np.random.default_rng(n)
    x = gen.standard_normal(n) + 1j * gen.standard_normal(n)
    tol = 1e-14 * max(1, n) * max(1, np.log2(max(n, 2)))
    assert np.abs(oracle.fft(x, -1) - np.fft.fft(x)).max() <= tol * np.abs(x).max() * 4
    # sign +1 is the unnormalised inverse
    assert np.abs(oracle.fft(x, +1) - n * np.fft.ifft(x)).max() <= tol * np.abs(x).max() * 4


def test_fft_rejects_non_power_of_two():
    with pytest.raises(ValueError):
        oracle.fft(np.ones(12))


@pytest.mark.parametrize("n1", [2, 8, 64, 2048])
def test_real_rows_match_numpy(n1):
    gen = np.random.default_rng(n1 + 7)
    f = gen.standard_normal((5, n1))
    F = oracle.rfft_rows(f)
    assert F.shape == (5, n1 // 2 + 1)
    assert np.abs(F - np.fft.rfft(f, axis=-1)).max() <= 1e-12 * n1
    back = oracle.irfft_rows(F, n1)
    assert np.abs(back - f).max() <= 1e-13 * n1
    # the inverse is numpy's irfft, which also drops the imaginary parts of
    # the kappa = 0 and kappa = n1/2 bins
    G = F + 1j * gen.standard_normal(F.shape)
    assert np.abs(oracle.irfft_rows(G, n1) - np.fft.irfft(G, n=n1, axis=-1)).max() <= 1e-13 * n1
