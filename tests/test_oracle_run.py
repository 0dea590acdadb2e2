"""Pins of the oracle's trajectory maximum and closing displacement fields."""

import numpy as np

from oracle import collapse, field, hessian, run
from paper_1305_1505_amd import workloads as W


def _plane(n, m, amp, axis=0):
    q = np.arange(n)
    shape = [1, 1, 1]
    shape[axis] = n
    x = amp * np.cos(2 * np.pi * m * q / n).reshape(shape) * np.ones((n, n, n))
    return x, np.fft.rfftn(x, axes=(0, 1, 2))


def test_plane_wave_fmax_closed_form():
    # delta = A cos(k x): lambda_1 = max(A W cos, 0), mu2 = mu3 = 0, s = 0 -> F = max(A W cos, 0);
    # W decreases with R, so the maximum sits at the smallest radius where cos > 0.
    n, m, amp = 16, 2, 0.8
    radii = np.array([3.0, 2.0, 1.0, 0.5])
    x, spec = _plane(n, m, amp)
    fmax, ridx = run.collapse_times(spec, radii)
    wmin = np.exp(-0.5 * (2 * np.pi * m * radii[-1] / n) ** 2)
    want = np.maximum(wmin * x, 0)
    assert np.max(np.abs(fmax - want)) < 1e-12
    pos = x > 1e-12
    assert np.all(ridx[pos] == 3)
    # where cos < 0 the tensor is (negative, 0, 0) up to FFT rounding ~1e-17; the E3 cubic's
    # roots then scale like a square or cube root of that rounding, so F is tiny, not exactly 0
    assert np.all(fmax[x < -1e-12] < 1e-6)


def test_range_split_equals_single_run_and_ties_keep_larger_radius():
    n = 16
    dk = field.linear_field(31, n, 40.0)
    radii = W.radii_cells(6, 4.0, 0.75)
    f_all, r_all = run.collapse_times(dk, radii)
    f_a, r_a = run.collapse_times(dk, radii, 0, 2)
    f_b, r_b = run.collapse_times(dk, radii, 2, 6, f_a, r_a)
    assert np.array_equal(f_all, f_b) and np.array_equal(r_all, r_b)
    # a repeated radius never moves R_max to the repeat (strictly larger F is required)
    rep = np.array([radii[0], radii[0]])
    _, rr = run.collapse_times(dk, rep)
    assert np.all((rr == 0) | (rr == run.NEVER))
    # F_max equals the per-radius maximum and R_max is its first argmax
    per = np.stack([run.per_radius_F(dk, r) for r in radii])
    assert np.array_equal(f_all, np.maximum(per.max(0), 0))
    hit = per.max(0) > 0
    assert np.array_equal(r_all[hit], np.argmax(per, 0)[hit].astype(np.uint8))


def test_za_plane_wave_closed_form():
    # delta = A cos(k x): psi1_x = -A sin(k x)/k (so that -d psi1_x/dx = delta), Mpc/h
    n, m, amp, box = 16, 3, 0.4, 50.0
    x, spec = _plane(n, m, amp, axis=1)
    psi = run.za_displacement(spec, box)
    k = 2 * np.pi * m / box
    q = np.arange(n) * box / n
    want = -amp * np.sin(k * q)[None, :, None] / k * np.ones((n, n, n))
    assert np.max(np.abs(psi[1] - want)) < 1e-13 * amp / k
    assert np.max(np.abs(psi[0])) < 1e-14 and np.max(np.abs(psi[2])) < 1e-14


def test_za_divergence_by_finite_differences():
    # smooth field: centred 4th-order differences of psi1 reproduce -delta
    n, box = 48, 96.0
    dk = field.linear_field(77, n, box) * hessian.gaussian_window(n, 4.0)
    psi = run.za_displacement(dk, box)
    h = box / n
    div = sum((-np.roll(p, -2, a) + 8 * np.roll(p, -1, a) - 8 * np.roll(p, 1, a) + np.roll(p, 2, a)) / (12 * h)
              for a, p in enumerate(psi))
    delta = hessian.smoothed_density(field.linear_field(77, n, box), 4.0)
    assert np.sqrt(np.mean((div + delta) ** 2)) < 2e-3 * np.sqrt(np.mean(delta ** 2))


def test_lpt2_plane_wave_vanishes():
    n, box = 16, 40.0
    _, spec = _plane(n, 2, 0.9, axis=2)
    psi2 = run.lpt2_displacement(spec, box)
    assert np.max(np.abs(psi2)) < 1e-15


def test_lpt2_two_orthogonal_waves_closed_form():
    # delta = A cos(k1 x) + B cos(k2 y): mu2 = A B cos(k1 x) cos(k2 y),
    # psi2 = -(3/7) A B/(k1^2+k2^2) (k1 sin(k1 x) cos(k2 y), k2 cos(k1 x) sin(k2 y), 0)
    n, box, a, b, m1, m2 = 16, 32.0, 0.5, 0.3, 1, 3
    q = np.arange(n) * box / n
    k1, k2 = 2 * np.pi * m1 / box, 2 * np.pi * m2 / box
    x = a * np.cos(k1 * q)[:, None, None] + b * np.cos(k2 * q)[None, :, None] + 0 * q[None, None, :]
    spec = np.fft.rfftn(x, axes=(0, 1, 2))
    psi2 = run.lpt2_displacement(spec, box)
    pref = -(3 / 7) * a * b / (k1 ** 2 + k2 ** 2)
    wx = pref * k1 * np.sin(k1 * q)[:, None, None] * np.cos(k2 * q)[None, :, None] * np.ones((n, n, n))
    wy = pref * k2 * np.cos(k1 * q)[:, None, None] * np.sin(k2 * q)[None, :, None] * np.ones((n, n, n))
    assert np.max(np.abs(psi2[0] - wx)) < 1e-13
    assert np.max(np.abs(psi2[1] - wy)) < 1e-13
    assert np.max(np.abs(psi2[2])) < 1e-15


def test_lpt2_divergence_is_minus_three_sevenths_mu2():
    n, box = 32, 64.0
    dk = field.linear_field(5, n, box) * hessian.gaussian_window(n, 3.0)
    mu2 = run.second_order_source(dk)
    psi2 = run.lpt2_displacement(dk, box)
    kf = 2 * np.pi / box
    f = hessian.freq_grids(n)
    div = np.fft.irfftn(sum(1j * kf * f[a] * np.fft.rfftn(psi2[a], axes=(0, 1, 2)) for a in range(3)),
                        s=(n, n, n), axes=(0, 1, 2))
    mu2k = np.fft.rfftn(mu2, axes=(0, 1, 2)) * hessian.nyquist_mask(n)
    mu2k[0, 0, 0] = 0
    ref = -(3 / 7) * np.fft.irfftn(mu2k, s=(n, n, n), axes=(0, 1, 2))
    assert np.max(np.abs(div - ref)) < 1e-12 * np.max(np.abs(ref))
