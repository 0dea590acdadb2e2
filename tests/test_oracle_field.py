"""Pins of the oracle's Gaussian linear field and its sigma_8 normalisation."""

import numpy as np
import pytest
from scipy import integrate

from oracle import field, spectrum
from paper_1305_1505_amd import workloads as W


def test_sigma8_normalisation_independent_quadrature():
    a = spectrum.amplitude_for_sigma8(W.SIGMA8, W.GAMMA, W.NS)
    # a dense composite Simpson rule in ln k (a different integrator than the oracle's quad)
    lnk = np.linspace(np.log(1e-7), np.log(1e3), 1_000_001)
    k = np.exp(lnk)
    y = k ** 3 * a * spectrum.unnormalised_power(k, W.GAMMA, W.NS) * spectrum.tophat_window(8 * k) ** 2
    s2 = integrate.simpson(y, x=lnk) / (2 * np.pi ** 2)
    assert abs(s2 - W.SIGMA8 ** 2) < 1e-11


def test_bbks_limits_and_tophat_series():
    assert abs(spectrum.bbks_transfer(1e-12, 0.21) - 1.0) < 1e-10
    # large-q behaviour: T ~ ln(2.34 q)/(2.34 q) / (6.71 q)
    q = 1e4
    t = spectrum.bbks_transfer(q * 0.21, 0.21)
    assert abs(t / (np.log(2.34 * q) / (2.34 * q) / (6.71 * q)) - 1) < 1e-3
    x = np.array([1e-4, 5e-4, 2e-3, 0.1, 1.0, 10.0])
    ref = 3 * (np.sin(x) - x * np.cos(x)) / x ** 3
    assert np.max(np.abs(spectrum.tophat_window(x) - ref)) < 1e-7


@pytest.mark.parametrize("n", [8, 16])
def test_hermitian_and_zero_modes(n):
    dk = field.linear_field(5, n, 40.0)
    h = n // 2
    assert dk[0, 0, 0] == 0
    assert np.all(dk[h] == 0) and np.all(dk[:, h] == 0) and np.all(dk[:, :, h] == 0)
    # exact conjugate symmetry on the l = 0 plane
    for i in range(n):
        for j in range(n):
            assert dk[(n - i) % n, (n - j) % n, 0] == np.conj(dk[i, j, 0])
    # a Hermitian-consistent half spectrum gives a real full inverse
    full = np.zeros((n, n, n), dtype=complex)
    full[:, :, : h + 1] = dk
    for l in range(h + 1, n):
        full[:, :, l] = np.conj(dk[(-np.arange(n)) % n][:, (-np.arange(n)) % n, n - l])
    x = np.fft.ifftn(full)
    assert np.max(np.abs(x.imag)) < 1e-15 * max(1.0, np.max(np.abs(x.real))) * n ** 1.5


def test_seed_determinism_and_distinct_seeds():
    a = field.linear_field(123, 16, 50.0)
    b = field.linear_field(123, 16, 50.0)
    c = field.linear_field(124, 16, 50.0)
    assert np.array_equal(a, b)
    assert not np.allclose(a, c)


def test_counter_layout_of_one_mode():
    # mode (i, j, l) = (2, 3, 1) of a 16^3 grid draws counter (2*16+3)*9+1
    n, seed, box = 16, 99, 30.0
    dk = field.linear_field(seed, n, box)
    from oracle import philox
    u1, u2 = philox.mode_uniforms(np.array([(2 * n + 3) * (n // 2 + 1) + 1], dtype=np.uint64), seed)
    g = np.sqrt(-2 * np.log(u1)) * np.exp(2j * np.pi * u2)
    a = spectrum.amplitude_for_sigma8(0.8, 0.21, 1.0)
    k = 2 * np.pi / box * np.sqrt(2 ** 2 + 3 ** 2 + 1)
    amp = np.sqrt(spectrum.power(k, a, 0.21, 1.0) * n ** 6 / (2 * box ** 3))
    assert abs(dk[2, 3, 1] - amp * g[0]) < 1e-13 * abs(amp)


def test_measured_power_within_sampling_error():
    n, box = 64, 200.0
    dk = field.linear_field(2024, n, box)
    a = spectrum.amplitude_for_sigma8(0.8, 0.21, 1.0)
    f = field.int_freqs(n)
    fz = np.arange(n // 2 + 1)
    fmag = np.sqrt(f[:, None, None] ** 2 + f[None, :, None] ** 2 + fz[None, None, :] ** 2)
    kmag = 2 * np.pi / box * fmag
    ratio = np.abs(dk) ** 2 / (spectrum.power(kmag, a, 0.21, 1.0) * n ** 6 / box ** 3 + 1e-300)
    # drawn modes (l > 0, no Nyquist, nonzero k): |dk|^2/<|dk|^2> is exponential with mean 1
    sel = (fz[None, None, :] > 0) & (fz[None, None, :] < n // 2) & (fmag > 0)
    sel = sel & (np.abs(f)[:, None, None] != n // 2) & (np.abs(f)[None, :, None] != n // 2)
    r = ratio[np.broadcast_to(sel, ratio.shape)]
    assert abs(r.mean() - 1) < 5 / np.sqrt(r.size)
    # per shell chi-square-like check: shell means within 5 sigma
    shells = np.floor(fmag).astype(int)[np.broadcast_to(sel, ratio.shape)]
    for s in range(2, 30, 3):
        m = r[shells == s]
        assert abs(m.mean() - 1) < 5 / np.sqrt(m.size)


def test_variance_matches_sum_of_power():
    n, box = 32, 64.0
    a = spectrum.amplitude_for_sigma8(0.8, 0.21, 1.0)
    dk = field.linear_field(7, n, box)
    x = np.fft.irfftn(dk, s=(n, n, n), axes=(0, 1, 2))
    f = field.int_freqs(n)
    fz = np.arange(n // 2 + 1)
    kmag = 2 * np.pi / box * np.sqrt(f[:, None, None] ** 2 + f[None, :, None] ** 2 + fz[None, None, :] ** 2)
    w = np.where(fz == 0, 1.0, 2.0)[None, None, :] * np.ones_like(kmag)
    keep = (np.abs(f)[:, None, None] != n // 2) & (np.abs(f)[None, :, None] != n // 2) & (fz[None, None, :] != n // 2)
    expected = np.sum(np.where(keep, w * spectrum.power(kmag, a, 0.21, 1.0), 0.0)) / box ** 3
    # the realised variance scatters around the expectation by O(1/sqrt(modes))
    assert abs(x.var() / expected - 1) < 0.05
