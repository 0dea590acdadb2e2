"""Pins of the oracle's deformation tensor: closed forms, trace = delta, direct-sum DFT."""

import numpy as np
import pytest

from oracle import dft, field, hessian
from paper_1305_1505_amd import workloads as W


def _cos_field_spectrum(n, m, axis, amp, phase=0.0):
    q = np.arange(n)
    shape = [1, 1, 1]
    shape[axis] = n
    x = amp * np.cos(2 * np.pi * m * q / n + phase).reshape(shape) * np.ones((n, n, n))
    return x, np.fft.rfftn(x, axes=(0, 1, 2))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_plane_wave_closed_form(axis):
    n, m, amp, ph, r = 16, 3, 0.7, 0.4, 1.3
    x, spec = _cos_field_spectrum(n, m, axis, amp, ph)
    t6 = hessian.deformation_tensor(spec, r)
    wk = np.exp(-0.5 * (2 * np.pi * m * r / n) ** 2)
    comp = {(0, 0): 0, (1, 1): 3, (2, 2): 5}[(axis, axis)]
    for c in range(6):
        want = wk * x if c == comp else np.zeros_like(x)
        assert np.max(np.abs(t6[c] - want)) < 1e-13


def test_oblique_plane_wave_outer_product():
    # delta = A cos(k.q) with k = 2 pi (1, 2, 3)/N: T_ij = W k^_i k^_j delta
    n, amp, r = 16, 0.5, 0.9
    kv = np.array([1, 2, 3])
    q = np.indices((n, n, n))
    x = amp * np.cos(2 * np.pi * np.tensordot(kv, q, axes=1) / n)
    t6 = hessian.deformation_tensor(np.fft.rfftn(x, axes=(0, 1, 2)), r)
    wk = np.exp(-0.5 * (2 * np.pi * r / n) ** 2 * np.sum(kv ** 2))
    for c, (a, b) in enumerate(hessian.COMPONENTS):
        assert np.max(np.abs(t6[c] - wk * kv[a] * kv[b] / np.sum(kv ** 2) * x)) < 1e-13


def test_triple_cosine_diagonal_and_sphere_point():
    n, m, amp = 12, 2, 0.3
    q = np.arange(n)
    c = np.cos(2 * np.pi * m * q / n)
    x = amp * (c[:, None, None] + c[None, :, None] + c[None, None, :])
    t6 = hessian.deformation_tensor(np.fft.rfftn(x, axes=(0, 1, 2)), None)
    assert np.max(np.abs(t6[0] - amp * c[:, None, None])) < 1e-13
    assert np.max(np.abs(t6[3] - amp * c[None, :, None])) < 1e-13
    assert np.max(np.abs(t6[5] - amp * c[None, None, :])) < 1e-13
    for k in (1, 2, 4):
        assert np.max(np.abs(t6[k])) < 1e-13
    # at q = 0 the tensor is isotropic: each diagonal element = delta/3
    assert abs(t6[0][0, 0, 0] - x[0, 0, 0] / 3) < 1e-13


@pytest.mark.parametrize("r", [None, 0.8, 3.0])
def test_trace_equals_smoothed_density(r):
    n = 24
    dk = field.linear_field(17, n, 60.0)
    t6 = hessian.deformation_tensor(dk, r)
    d = hessian.smoothed_density(dk, r)
    assert np.max(np.abs(t6[0] + t6[3] + t6[5] - d)) < 1e-12 * np.max(np.abs(d))


def test_direct_sum_hessian_tiny_grid():
    # T_ij by the direct real inverse DFT of W k_i k_j / k^2 dk, built from physical k (not f)
    n, box, r = 6, 9.0, 0.7
    spec = W.random_half_spectrum(n, 5)
    t6 = hessian.deformation_tensor(spec, r)
    kf = 2 * np.pi / box
    f = field.int_freqs(n)
    fz = np.arange(n // 2 + 1)
    K = [kf * f[:, None, None] * np.ones((n, n, n // 2 + 1)),
         kf * f[None, :, None] * np.ones((n, n, n // 2 + 1)),
         kf * fz[None, None, :] * np.ones((n, n, n // 2 + 1))]
    k2 = K[0] ** 2 + K[1] ** 2 + K[2] ** 2
    rphys = r * box / n
    nyq = (np.abs(K[0]) == kf * n / 2) | (np.abs(K[1]) == kf * n / 2) | (K[2] == kf * n / 2)
    for c, (a, b) in enumerate(hessian.COMPONENTS):
        mult = np.where((k2 > 0) & ~nyq, K[a] * K[b] / np.where(k2 > 0, k2, 1) * np.exp(-k2 * rphys ** 2 / 2), 0)
        re, im = dft.dft3_inverse_half(mult * spec, n)
        assert np.max(np.abs(t6[c] - re)) < 1e-12 * max(1.0, np.max(np.abs(re)))


def test_smoothing_reduces_variance_monotonically():
    dk = field.linear_field(3, 32, 80.0)
    v = [np.var(hessian.smoothed_density(dk, r)) for r in (0.75, 1.5, 3.0, 6.0)]
    assert all(a > b for a, b in zip(v, v[1:]))
