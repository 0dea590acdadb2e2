"""Pins of the v_max oracle (velocity at the trajectory maximum: the ZA displacement smoothed on
R_max, recorded when F_max is updated)."""

import numpy as np

from oracle import field, hessian, points, run


def test_plane_wave_closed_form():
    """One mode A e^{2 pi i f.q/N} (+ conjugate): T = W f f^T/f^2 d(q) with d(q) = 2 Re(A e^{i th}) / N^3,
    a plane, so F = W d where d > 0 (largest at the smallest radius, W decreasing in R) and
    v_max = W(R_last) (L/2pi) (f/f^2) (-2 Im(A e^{i th})) / N^3 there.  Where d < 0 the exact F is
    0, but lambda_1 = 0 only up to the rounding of the rotated components, whose cube root F is:
    checked for smallness."""
    n, box = 16, 40.0
    fx, fy, fz = 1, -2, 3
    amp = 0.8 + 0.3j
    dk = np.zeros((n, n, n // 2 + 1), dtype=np.complex128)
    dk[fx % n, fy % n, fz] = amp
    radii = [3.0, 1.5, 0.5]
    F, R, V = run.collapse_times_with_velocity(dk, radii, box)
    f = np.array([fx, fy, fz], dtype=np.float64)
    q = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), -1).astype(np.float64)
    ph = amp * np.exp(2j * np.pi * (q @ f) / n)
    d = 2.0 * np.real(ph) / n ** 3
    w_last = np.exp(-0.5 * (2 * np.pi * radii[-1] / n) ** 2 * (f @ f))
    pos = d > 1e-12 * np.max(d)
    assert np.all(R[pos] == len(radii) - 1)
    assert np.all(F[~pos] <= 1e-4 * np.max(F))
    assert np.allclose(F[pos], w_last * d[pos], rtol=1e-10)
    v_ref = w_last * (box / (2 * np.pi)) * (f / (f @ f))[:, None] * (-2.0 * np.imag(ph[pos]) / n ** 3)[None, :]
    assert np.max(np.abs(V[:, pos] - v_ref)) <= 1e-12 * np.max(np.abs(v_ref))


def test_velocity_is_smoothed_za_at_rmax_and_f_unchanged():
    n, box = 24, 60.0
    dk = field.linear_field(31, n, box)
    radii = [6.0, 3.0, 1.5, 0.75]
    F, R, V = run.collapse_times_with_velocity(dk, radii, box)
    F0, R0 = run.collapse_times(dk, radii)
    assert np.array_equal(F, F0) and np.array_equal(R, R0)
    for r in range(len(radii)):
        m = R == r
        z = run.za_displacement(dk * hessian.gaussian_window(n, radii[r]), box)
        assert np.max(np.abs((V - z)[:, m]), initial=0.0) <= 1e-13 * np.max(np.abs(z))
    assert np.all(V[:, R == 255] == 0.0)


def test_velocity_at_points_matches_full_grid():
    n, box = 24, 60.0
    dk = field.linear_field(31, n, box)
    radii = [6.0, 3.0, 1.5, 0.75]
    F, R, V = run.collapse_times_with_velocity(dk, radii, box)
    pts = [(0, 0, 0), (3, 17, 5), (23, 1, 12), (11, 11, 11), (5, 5, 20)]
    fm, ri, vm, _ = points.collapse_times_with_velocity_at_points(dk, pts, radii, box)
    assert list(ri) == [R[p] for p in pts]
    ref = np.array([[V[a][p] for a in range(3)] for p in pts])
    assert np.max(np.abs(vm - ref)) <= 1e-13 * np.max(np.abs(V))
