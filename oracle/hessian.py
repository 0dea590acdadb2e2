"""Deformation tensor per smoothing radius (oracle side; test infrastructure only).

Section "Collapse times": for each smoothing radius the field is smoothed with a Gaussian filter
and a series of FFTs gives the deformation tensor, the Hessian of the peculiar potential, whose
trace is the (smoothed) linear density contrast.

With lap(phi) = delta_l, the Fourier multiplier of T_ij = d_i d_j phi is k_i k_j / k^2, so

    T_ij(x) = irfftn( W(kR) * k_i k_j / k^2 * dk ),      W(kR) = exp(-k^2 R^2 / 2),

with the k = 0 term zero.  Readings (the paper states neither): the Gaussian window is
exp(-k^2 R^2/2); radii are given in grid cells (R_phys = R * L / N); and the multiplier is zero
on every mode with a Nyquist index (a derivative has no real-valued representation there).
Because k_i k_j / k^2 and k R are dimensionless, T does not depend on the box size L.

Component order everywhere: (xx, xy, xz, yy, yz, zz).
"""

import numpy as np

from .field import int_freqs

COMPONENTS = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))


def freq_grids(n):
    """Integer frequency grids (fx, fy, fz) broadcastable over the half spectrum (N, N, N/2+1)."""
    f = int_freqs(n)
    fz = np.arange(n // 2 + 1, dtype=np.float64)
    return f[:, None, None], f[None, :, None], fz[None, None, :]


def nyquist_mask(n):
    """1 on ordinary modes, 0 on any mode with a Nyquist index."""
    fx, fy, fz = freq_grids(n)
    h = n // 2
    return ((np.abs(fx) != h) & (np.abs(fy) != h) & (fz != h)).astype(np.float64)


def gaussian_window(n, radius_cells):
    """W(kR) = exp(-k^2 R^2/2) with k R = 2 pi |f| R / N (R in cells)."""
    fx, fy, fz = freq_grids(n)
    f2 = fx ** 2 + fy ** 2 + fz ** 2
    return np.exp(-0.5 * (2.0 * np.pi * radius_cells / n) ** 2 * f2)


def smoothed_potential_spectrum(dk, radius_cells=None):
    """g = M * W * dk / f^2 on the half spectrum (zero at k = 0), f the integer wavevector.

    T_ij = irfftn(f_i f_j g).  radius_cells=None means no smoothing (W = 1).
    """
    n = dk.shape[0]
    fx, fy, fz = freq_grids(n)
    f2 = fx ** 2 + fy ** 2 + fz ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = np.where(f2 > 0, 1.0 / np.where(f2 > 0, f2, 1.0), 0.0)
    g = dk * inv * nyquist_mask(n)
    if radius_cells is not None:
        g = g * gaussian_window(n, radius_cells)
    return g


def deformation_tensor(dk, radius_cells=None, components=COMPONENTS):
    """The components (a, b) of T_ij(x), each a real (N, N, N) array; by default all six
    (xx, xy, xz, yy, yz, zz).  A subset gives the same arrays, for grids where six do not fit."""
    n = dk.shape[0]
    g = smoothed_potential_spectrum(dk, radius_cells)
    f = freq_grids(n)
    out = []
    for a, b in components:
        out.append(np.fft.irfftn(f[a] * f[b] * g, s=(n, n, n), axes=(0, 1, 2)))
    return out


def smoothed_density(dk, radius_cells=None):
    """irfftn(M * W * dk): the smoothed linear density (the trace of T), for pins."""
    n = dk.shape[0]
    g = dk * nyquist_mask(n)
    g[0, 0, 0] = 0.0
    if radius_cells is not None:
        g = g * gaussian_window(n, radius_cells)
    return np.fft.irfftn(g, s=(n, n, n), axes=(0, 1, 2))
