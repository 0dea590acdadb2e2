"""Pins of the library FFT the oracle uses: naive direct-sum DFTs, Parseval, round trips."""

import numpy as np
import pytest

from oracle import dft
from paper_1305_1505_amd import workloads


@pytest.mark.parametrize("n", [4, 6, 8])
def test_forward_matches_direct_sum(n):
    x = workloads.random_real_field(n, 7 + n)
    ref = dft.dft3_forward(x)
    half = np.fft.rfftn(x, axes=(0, 1, 2))
    assert np.max(np.abs(half - ref[:, :, : n // 2 + 1])) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("n", [4, 6, 8])
def test_inverse_half_matches_direct_sum(n):
    spec = workloads.random_half_spectrum(n, 11 + n)
    re, im = dft.dft3_inverse_half(spec, n)
    lib = np.fft.irfftn(spec, s=(n, n, n), axes=(0, 1, 2))
    assert np.max(np.abs(lib - re)) < 1e-13 * np.max(np.abs(re))
    assert np.max(np.abs(im)) < 1e-13 * np.max(np.abs(re))


def test_direct_sum_sign_convention():
    # a single cosine mode: the forward DFT of cos(2 pi q/N) along x has N^3/2 at f = +-1
    n = 6
    q = np.arange(n)
    x = np.cos(2 * np.pi * q / n)[:, None, None] * np.ones((n, n, n))
    ref = dft.dft3_forward(x)
    assert abs(ref[1, 0, 0] - n ** 3 / 2) < 1e-9 and abs(ref[n - 1, 0, 0] - n ** 3 / 2) < 1e-9
    y = np.sin(2 * np.pi * q / n)[:, None, None] * np.ones((n, n, n))
    ref = dft.dft3_forward(y)   # sin: -i N^3/2 at f = +1
    assert abs(ref[1, 0, 0] - (-0.5j * n ** 3)) < 1e-9


@pytest.mark.parametrize("n", [12, 16, 24])
def test_parseval_and_round_trip(n):
    x = workloads.random_real_field(n, 3 * n)
    full = np.fft.fftn(x)
    assert abs(np.sum(np.abs(full) ** 2) / n ** 3 - np.sum(x * x)) < 1e-11 * np.sum(x * x)
    back = np.fft.irfftn(np.fft.rfftn(x, axes=(0, 1, 2)), s=(n, n, n), axes=(0, 1, 2))
    assert np.max(np.abs(back - x)) < 1e-13 * np.max(np.abs(x))
