"""F_max / R_max over the radii and the closing displacement fields (oracle; test infrastructure only).

Section "Collapse times": for each grid point the code records the highest F along the
trajectory, F_max, and the smoothing scale R_max where it was reached.  Readings: radii are
visited from the largest to the smallest; F_max starts at 0 and the radius index at 255 ("never
collapsed"); an update needs a strictly larger F, so ties keep the larger radius.

Velocity at the trajectory maximum (section "Collapse times", last paragraph): with F_max the
code records v_max, computed from the first derivative of the peculiar potential smoothed on
R_max each time F_max is updated.  Reading: v_max is the Zel'dovich displacement of the field
smoothed on that radius, psi1_R(k) = i k W(kR) dk / k^2 in Mpc/h at D = 1 (the peculiar velocity
is a H f D times it, a factor per output time outside this path); 0 where F_max was never set.

Displacements (sections on fragmentation and on the code, and the 2LPT extension in the
conclusions): the Zel'dovich displacement psi1 = -grad(phi) at D = 1, i.e. psi1(k) = i k dk / k^2,
so that -div(psi1) = delta; and the second-order displacement of standard EdS 2LPT,
psi2(k) = (3/7) i k mu2~(k) / k^2 with mu2~ = rfftn(mu2) and mu2 = sum_{i<j}(T_ii T_jj - T_ij^2)
of the UNSMOOTHED deformation tensor (reading: growth D2 = -(3/7) D^2, no smoothing, no
dealiasing, k = 0 and Nyquist modes of mu2~ zeroed).  Both in Mpc/h, L being the box side.
"""

import numpy as np

from . import collapse, hessian

NEVER = 255


def collapse_times(dk, radii_cells, r_begin=0, r_end=None, fmax=None, ridx=None):
    """Run radii [r_begin, r_end) and update (fmax, ridx); fresh state (0, 255) when not given."""
    n = dk.shape[0]
    if r_end is None:
        r_end = len(radii_cells)
    if fmax is None:
        fmax = np.zeros((n, n, n), dtype=np.float64)
    if ridx is None:
        ridx = np.full((n, n, n), NEVER, dtype=np.uint8)
    for r in range(r_begin, r_end):
        t6 = hessian.deformation_tensor(dk, radii_cells[r])
        f = collapse.inverse_collapse_time(t6)
        up = f > fmax
        fmax = np.where(up, f, fmax)
        ridx = np.where(up, np.uint8(r), ridx)
    return fmax, ridx


def collapse_times_with_velocity(dk, radii_cells, box):
    """(F_max, R_max index, v_max (3, N, N, N) in Mpc/h): v_max is the smoothed ZA displacement
    at the radius of the last update of F_max, 0 where there was none."""
    n = dk.shape[0]
    fmax = np.zeros((n, n, n), dtype=np.float64)
    ridx = np.full((n, n, n), NEVER, dtype=np.uint8)
    vmax = np.zeros((3, n, n, n), dtype=np.float64)
    for r, radius in enumerate(radii_cells):
        f = collapse.inverse_collapse_time(hessian.deformation_tensor(dk, radius))
        up = f > fmax
        fmax = np.where(up, f, fmax)
        ridx = np.where(up, np.uint8(r), ridx)
        v = _gradient_fields(dk * hessian.gaussian_window(n, radius), box)
        vmax = np.where(up[None], v, vmax)
    return fmax, ridx, vmax


def per_radius_F(dk, radius_cells):
    """F(q; R) at one radius (no running maximum)."""
    return collapse.inverse_collapse_time(hessian.deformation_tensor(dk, radius_cells))


def _gradient_fields(spec, box):
    """irfftn(i k_a spec / k^2) for a = x, y, z (Mpc/h), spec on the half spectrum."""
    n = spec.shape[0]
    fx, fy, fz = hessian.freq_grids(n)
    f2 = fx ** 2 + fy ** 2 + fz ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = np.where(f2 > 0, 1.0 / np.where(f2 > 0, f2, 1.0), 0.0)
    g = spec * inv * hessian.nyquist_mask(n) * (box / (2.0 * np.pi))   # i k / k^2 = i (L/2pi) f/f^2
    return np.stack([np.fft.irfftn(1j * fa * g, s=(n, n, n), axes=(0, 1, 2)) for fa in (fx, fy, fz)])


def za_displacement(dk, box):
    """psi1 at D = 1, shape (3, N, N, N), Mpc/h."""
    return _gradient_fields(dk, box)


def second_order_source(dk):
    """mu2(x) of the unsmoothed deformation tensor (the 2LPT source)."""
    xx, xy, xz, yy, yz, zz = hessian.deformation_tensor(dk, None)
    return xx * yy + xx * zz + yy * zz - xy * xy - xz * xz - yz * yz


def lpt2_displacement(dk, box):
    """psi2 at D = 1 (EdS, D2 = -(3/7) D^2), shape (3, N, N, N), Mpc/h."""
    n = dk.shape[0]
    mu2k = np.fft.rfftn(second_order_source(dk), axes=(0, 1, 2))
    mu2k = mu2k * hessian.nyquist_mask(n)
    mu2k[0, 0, 0] = 0.0
    return (3.0 / 7.0) * _gradient_fields(mu2k, box)


def displacements(dk, box):
    """(psi1, psi2), each (3, N, N, N) float64 in Mpc/h at D = 1."""
    return za_displacement(dk, box), lpt2_displacement(dk, box)
