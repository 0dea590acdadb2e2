"""Pins of oracle.points (direct inverse-DFT sums at single grid points) against the full-grid
oracle, which they must reproduce to rounding, and against closed forms."""

import numpy as np
import pytest

from oracle import field, hessian, points, run

PTS = [(0, 0, 0), (3, 17, 5), (23, 1, 12), (11, 11, 11), (12, 12, 0)]


@pytest.mark.parametrize("n", [12, 24])
def test_tensor_at_points_matches_full_grid(n):
    dk = field.linear_field(7 + n, n, 50.0)
    pts = [(p[0] % n, p[1] % n, p[2] % n) for p in PTS]
    radii = [5.0, 2.0, 0.75, None]
    t = points.tensor_at_points(dk, pts, radii)
    for r, radius in enumerate(radii):
        full = hessian.deformation_tensor(dk, radius)
        ref = np.array([[full[c][p] for c in range(6)] for p in pts])
        assert np.max(np.abs(t[:, r, :] - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_tensor_at_points_plane_wave():
    """A single mode (and its partner) gives T_ab = W f_a f_b / f^2 * 2 |A| cos(2 pi f.q/N + arg A) / N^3."""
    n = 16
    dk = np.zeros((n, n, n // 2 + 1), dtype=np.complex128)
    fx, fy, fz = 2, -3, 4
    amp = 0.7 - 0.2j
    dk[fx % n, fy % n, fz] = amp
    pts = [(1, 2, 3), (5, 0, 9), (15, 15, 15)]
    radius = 1.3
    t = points.tensor_at_points(dk, pts, [radius])
    f = np.array([fx, fy, fz], dtype=np.float64)
    f2 = f @ f
    w = np.exp(-0.5 * (2 * np.pi * radius / n) ** 2 * f2)
    for p, q in enumerate(pts):
        wave = 2.0 * np.real(amp * np.exp(2j * np.pi * (f @ np.array(q)) / n)) / n ** 3
        for c, (a, b) in enumerate(hessian.COMPONENTS):
            assert abs(t[p, 0, c] - w * f[a] * f[b] / f2 * wave) <= 1e-15


def test_collapse_and_za_at_points_match_full_grid():
    n, box = 24, 60.0
    dk = field.linear_field(31, n, box)
    radii = [6.0, 3.0, 1.5, 0.75]
    fmax, ridx, _ = points.collapse_times_at_points(dk, PTS, radii)
    F, R = run.collapse_times(dk, radii)
    assert np.max(np.abs(fmax - np.array([F[p] for p in PTS]))) <= 1e-12 * np.max(np.abs(F))
    assert list(ridx) == [R[p] for p in PTS]
    z = points.za_at_points(dk, PTS, box)
    Z = run.za_displacement(dk, box)
    ref = np.array([[Z[a][p] for a in range(3)] for p in PTS])
    assert np.max(np.abs(z - ref)) <= 1e-13 * np.max(np.abs(Z))


def test_planted_mistake_in_weights_is_caught():
    """Weight 1 instead of 2 on the interior half-spectrum planes must break the agreement."""
    n = 12
    dk = field.linear_field(3, n, 30.0)
    t = points.tensor_at_points(dk, [(1, 2, 3)], [None])
    full = hessian.deformation_tensor(dk, None)
    ref = np.array([full[c][(1, 2, 3)] for c in range(6)])
    orig = points._half_weights
    try:
        points._half_weights = lambda n_: np.ones(n_ // 2 + 1)
        bad = points.tensor_at_points(dk, [(1, 2, 3)], [None])
    finally:
        points._half_weights = orig
    assert np.max(np.abs(t[0, 0] - ref)) <= 1e-13 * np.max(np.abs(ref))
    assert np.max(np.abs(bad[0, 0] - ref)) > 1e-3 * np.max(np.abs(ref))

