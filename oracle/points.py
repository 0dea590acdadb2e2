"""Deformation tensor, collapse times and ZA displacement at single grid points, by direct
summation of the inverse DFT (oracle side; test infrastructure only).

For grids too large for the full-grid oracle of ``hessian`` and ``run`` in the time a test may
take, these evaluate the same definitions at chosen grid points q = (i, j, l):

    T_ab(q) = (1/N^3) sum_{f} W(f; R) f_a f_b / f^2 M(f) dk(f) exp(2 pi i f.q / N),

the sum running over the full spectrum (section "Collapse times": Gaussian smoothing, the
Hessian of the potential), with dk on the half spectrum extended by Hermitian symmetry: a mode
with 0 < l < N/2 stands for itself and its conjugate partner (twice the real part of its term),
a mode with l = 0 appears together with its partner in the half spectrum (the real part of its
term; the imaginary parts cancel pairwise).  M zeroes k = 0 and every Nyquist mode, exactly as
in ``hessian``.  The Gaussian window depends on f only through |f|^2, so the terms are grouped
by the integer m = |f|^2 first and every radius then costs one sum over m -- an exact
regrouping of the same sum.

Collapse times at a point apply ``collapse.inverse_collapse_time`` to the tensor at each radius
and keep the running maximum exactly as ``run.collapse_times`` does (radii largest first, strict
'>' for an update, 0 and index 255 before any).
"""

import numpy as np

from . import collapse, hessian
from .field import int_freqs
from .run import NEVER


def _phase_rows(n, points):
    """exp(2 pi i f q / N) per axis for each point: three arrays (P, N), (P, N), (P, N/2+1)."""
    f = int_freqs(n)
    fz = np.arange(n // 2 + 1, dtype=np.float64)
    q = np.asarray(points, dtype=np.float64)
    ex = np.exp(2j * np.pi * np.outer(q[:, 0], f) / n)
    ey = np.exp(2j * np.pi * np.outer(q[:, 1], f) / n)
    ez = np.exp(2j * np.pi * np.outer(q[:, 2], fz) / n)
    return ex, ey, ez


def _half_weights(n):
    """Weight of each l on the half spectrum: 1 for l = 0 and l = N/2, 2 otherwise."""
    w = np.full(n // 2 + 1, 2.0)
    w[0] = 1.0
    w[n // 2] = 1.0
    return w


def grouped_tensor_sums(dk, points):
    """S[p, c, m] = sum over modes with |f|^2 = m of w_l Re(f_a f_b / f^2 M dk e^{2 pi i f.q_p/N})
    for the six components c = (a, b) of ``hessian.COMPONENTS``; shape (P, 6, 3 (N/2)^2 + 1)."""
    n = dk.shape[0]
    npts = len(points)
    f = int_freqs(n)
    fy = f[:, None]
    fz = np.arange(n // 2 + 1, dtype=np.float64)[None, :]
    mmax = 3 * (n // 2) ** 2
    ex, ey, ez = _phase_rows(n, points)
    wl = _half_weights(n)[None, :]
    sums = np.zeros((npts, 6, mmax + 1))
    eyz = [ey[p][:, None] * ez[p][None, :] for p in range(npts)]         # phase over (j, l)
    half = n // 2
    for i in range(n):
        fx = f[i]
        f2 = fx * fx + fy * fy + fz * fz                                    # (N, N/2+1)
        mask = (abs(fx) != half) & (np.abs(fy) != half) & (fz != half) & (f2 > 0)
        inv = np.where(mask, 1.0 / np.where(f2 > 0, f2, 1.0), 0.0)
        g = dk[i] * inv * wl                                                # (N, N/2+1)
        m = f2.astype(np.int64).ravel()
        fvec = (np.full_like(f2, fx), np.broadcast_to(fy, f2.shape), np.broadcast_to(fz, f2.shape))
        fab = [(fvec[a] * fvec[b]).ravel() for a, b in hessian.COMPONENTS]
        for p in range(npts):
            term = np.real(g * (ex[p, i] * eyz[p])).ravel()
            for c in range(6):
                sums[p, c] += np.bincount(m, weights=fab[c] * term, minlength=mmax + 1)
    return sums


def grouped_gradient_sums(dk, points):
    """G[p, a, m] = sum over modes with |f|^2 = m of w_l Re(i f_a / f^2 M dk e^{2 pi i f.q_p/N});
    shape (P, 3, 3 (N/2)^2 + 1)."""
    n = dk.shape[0]
    npts = len(points)
    f = int_freqs(n)
    fy = f[:, None]
    fz = np.arange(n // 2 + 1, dtype=np.float64)[None, :]
    mmax = 3 * (n // 2) ** 2
    ex, ey, ez = _phase_rows(n, points)
    wl = _half_weights(n)[None, :]
    sums = np.zeros((npts, 3, mmax + 1))
    eyz = [ey[p][:, None] * ez[p][None, :] for p in range(npts)]
    half = n // 2
    for i in range(n):
        fx = f[i]
        f2 = fx * fx + fy * fy + fz * fz
        mask = (abs(fx) != half) & (np.abs(fy) != half) & (fz != half) & (f2 > 0)
        inv = np.where(mask, 1.0 / np.where(f2 > 0, f2, 1.0), 0.0)
        g = 1j * dk[i] * inv * wl
        m = f2.astype(np.int64).ravel()
        fvec = (np.full_like(f2, fx).ravel(), np.broadcast_to(fy, f2.shape).ravel(),
                np.broadcast_to(fz, f2.shape).ravel())
        for p in range(npts):
            term = (g * (ex[p, i] * eyz[p])).ravel()
            for a in range(3):
                sums[p, a] += np.bincount(m, weights=np.real(fvec[a] * term), minlength=mmax + 1)
    return sums


def tensor_at_points(dk, points, radii_cells):
    """T_ab at each point for each radius (None: no smoothing); shape (P, n_radii, 6)."""
    n = dk.shape[0]
    sums = grouped_tensor_sums(dk, points)
    m = np.arange(sums.shape[2], dtype=np.float64)
    out = np.empty((len(points), len(radii_cells), 6))
    for r, radius in enumerate(radii_cells):
        w = np.ones_like(m) if radius is None else np.exp(-0.5 * (2.0 * np.pi * radius / n) ** 2 * m)
        out[:, r, :] = np.einsum("pcm,m->pc", sums, w) / float(n) ** 3
    return out


def collapse_times_at_points(dk, points, radii_cells):
    """(F_max, R_max index) at each point, and the per-radius F (P, n_radii)."""
    t = tensor_at_points(dk, points, radii_cells)
    npts, nr = t.shape[:2]
    f = collapse.inverse_collapse_time([t[:, :, c].ravel() for c in range(6)]).reshape(npts, nr)
    fmax = np.zeros(npts)
    ridx = np.full(npts, NEVER, dtype=np.uint8)
    for r in range(nr):
        up = f[:, r] > fmax
        fmax = np.where(up, f[:, r], fmax)
        ridx = np.where(up, np.uint8(r), ridx)
    return fmax, ridx, f


def collapse_times_with_velocity_at_points(dk, points, radii_cells, box):
    """As collapse_times_at_points, plus v_max (P, 3) in Mpc/h: the ZA displacement smoothed on
    the radius of the last update of F_max (0 where none), as ``run.collapse_times_with_velocity``."""
    n = dk.shape[0]
    fmax, ridx, f = collapse_times_at_points(dk, points, radii_cells)
    g = grouped_gradient_sums(dk, points)
    m = np.arange(g.shape[2], dtype=np.float64)
    vmax = np.zeros((len(points), 3))
    for p in range(len(points)):
        if ridx[p] != NEVER:
            w = np.exp(-0.5 * (2.0 * np.pi * radii_cells[ridx[p]] / n) ** 2 * m)
            vmax[p] = (g[p] @ w) * (box / (2.0 * np.pi)) / float(n) ** 3
    return fmax, ridx, vmax, f


def za_at_points(dk, points, box):
    """psi1_a(q) = (1/N^3) sum_f i (L/2pi) f_a / f^2 M dk e^{2 pi i f.q/N}; shape (P, 3), Mpc/h."""
    n = dk.shape[0]
    f = int_freqs(n)
    fy = f[:, None]
    fz = np.arange(n // 2 + 1, dtype=np.float64)[None, :]
    ex, ey, ez = _phase_rows(n, points)
    wl = _half_weights(n)[None, :]
    out = np.zeros((len(points), 3))
    eyz = [ey[p][:, None] * ez[p][None, :] for p in range(len(points))]
    half = n // 2
    for i in range(n):
        fx = f[i]
        f2 = fx * fx + fy * fy + fz * fz
        mask = (abs(fx) != half) & (np.abs(fy) != half) & (fz != half) & (f2 > 0)
        inv = np.where(mask, 1.0 / np.where(f2 > 0, f2, 1.0), 0.0)
        g = 1j * dk[i] * inv * wl * (box / (2.0 * np.pi))
        fvec = (fx, fy, fz)
        for p in range(len(points)):
            term = g * (ex[p, i] * eyz[p])
            for a in range(3):
                out[p, a] += np.sum(np.real(fvec[a] * term))
    return out / float(n) ** 3
