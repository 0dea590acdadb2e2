"""Gaussian linear density field on the Lagrangian grid (oracle side; test infrastructure only).

Section "Collapse times", eq. deltal: a Gaussian realisation of the linear density contrast,
extrapolated to z = 0, on a cubic grid of N^3 vertices and side L (Mpc/h), with the power
spectrum of ``spectrum`` normalised to sigma_8.

Conventions (readings; the paper fixes neither FFT conventions nor a random-number layout):

* Half-spectrum layout dk[i, j, l] with i, j in [0, N) and l in [0, N/2] (NumPy ``rfftn`` of a
  real field, z fastest).  Integer frequency f(i) = i for i < N/2, i - N otherwise; the physical
  wavenumber is k = 2 pi |f| / L in h/Mpc.
* Forward transform unnormalised (NumPy's), so <|dk|^2> = P(k) N^6 / L^3 and the real field is
  irfftn(dk).
* Each half-space mode draws two uniforms from Philox4x32-10 with counter (i*N + j)*(N/2+1) + l
  and key = seed, turns them into g1 + i g2 by Box-Muller in float64, and takes
  dk = sqrt(P(k) N^6 / (2 L^3)) * (g1 + i g2).
* On the l = 0 plane the member of each (f, -f) pair with the larger i*N + j is drawn and the other
  is its complex conjugate, so the real field is exactly Hermitian-consistent.
* k = 0 and every mode with a Nyquist index (i = N/2, j = N/2 or l = N/2) are zero.
"""

import numpy as np

from . import philox, spectrum


def int_freqs(n):
    """Integer frequencies of the full axis: 0..N/2-1, -N/2..-1 (index N/2 is the Nyquist -N/2)."""
    i = np.arange(n)
    return np.where(i < n // 2, i, i - n).astype(np.float64)


def linear_field(seed, n, box, sigma8=0.8, gamma=0.21, ns=1.0, amplitude=None):
    """Half-spectrum dk (complex128, shape (N, N, N/2+1)) of the sigma_8-normalised BBKS field."""
    if n % 2:
        raise ValueError("N must be even")
    if amplitude is None:
        amplitude = spectrum.amplitude_for_sigma8(sigma8, gamma, ns)
    nh = n // 2 + 1
    f = int_freqs(n)
    fz = np.arange(nh, dtype=np.float64)
    kf = 2.0 * np.pi / box
    norm = float(n) ** 6 / (2.0 * box ** 3)
    dk = np.empty((n, n, nh), dtype=np.complex128)
    j = np.arange(n, dtype=np.int64)
    l = np.arange(nh, dtype=np.int64)
    for i in range(n):
        counter = ((np.int64(i) * n + j)[:, None] * nh + l[None, :]).astype(np.uint64)
        u1, u2 = philox.mode_uniforms(counter, seed)
        rad = np.sqrt(-2.0 * np.log(u1))
        g = rad * np.cos(2.0 * np.pi * u2) + 1j * (rad * np.sin(2.0 * np.pi * u2))
        kmag = kf * np.sqrt(f[i] ** 2 + f[:, None] ** 2 + fz[None, :] ** 2)
        pk = spectrum.power(kmag, amplitude, gamma, ns)
        dk[i] = np.sqrt(pk * norm) * g
    # l = 0 plane: the mode with the larger i*N + j of each (f, -f) pair is drawn, its partner is
    # the conjugate.
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    pi_, pj = (n - ii) % n, (n - jj) % n
    own, partner = ii * n + jj, pi_ * n + pj
    take = partner > own
    plane = dk[:, :, 0].copy()
    plane[take] = np.conj(plane[pi_[take], pj[take]])
    dk[:, :, 0] = plane
    # zero k = 0 and every Nyquist mode
    dk[0, 0, 0] = 0.0
    dk[n // 2, :, :] = 0.0
    dk[:, n // 2, :] = 0.0
    dk[:, :, n // 2] = 0.0
    return dk
