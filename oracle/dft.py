"""Naive discrete Fourier transforms by direct summation (oracle; test infrastructure only).

Used to pin the library FFT the oracle relies on: the 3D transform written out as the sum
X(k) = sum_x x(q) exp(-2 pi i k.q / N) (forward, unnormalised) and its inverse with 1/N^3.
O(N^6); meant for N <= 12.
"""

import numpy as np


def dft3_forward(x):
    """Full complex forward 3D DFT of a cubic array by direct summation."""
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[0]
    idx = np.arange(n)
    out = np.zeros((n, n, n), dtype=np.complex128)
    qx, qy, qz = np.meshgrid(idx, idx, idx, indexing="ij")
    for kx in range(n):
        for ky in range(n):
            for kz in range(n):
                ph = np.exp(-2j * np.pi * (kx * qx + ky * qy + kz * qz) / n)
                out[kx, ky, kz] = np.sum(x * ph)
    return out


def dft3_inverse_half(spec_half, n):
    """Real inverse 3D DFT from a half spectrum (N, N, N/2+1), by direct summation.

    The full spectrum is rebuilt from the half one with X(-k) = conj(X(k)); on the planes l = 0
    and l = N/2 the value stored at index (i, j) is used for (i, j) itself, exactly as a
    Hermitian-consistent input requires.  Returns the real part (the imaginary part vanishes for
    Hermitian-consistent input).
    """
    nh = n // 2 + 1
    full = np.zeros((n, n, n), dtype=np.complex128)
    for i in range(n):
        for j in range(n):
            for l in range(n):
                if l < nh:
                    full[i, j, l] = spec_half[i, j, l]
                else:
                    full[i, j, l] = np.conj(spec_half[(n - i) % n, (n - j) % n, n - l])
    idx = np.arange(n)
    qx, qy, qz = np.meshgrid(idx, idx, idx, indexing="ij")
    out = np.zeros((n, n, n), dtype=np.complex128)
    for kx in range(n):
        for ky in range(n):
            for kz in range(n):
                out += full[kx, ky, kz] * np.exp(2j * np.pi * (kx * qx + ky * qy + kz * qz) / n)
    return out.real / n ** 3, out.imag / n ** 3
