"""Pins of the third-order displacement oracle (oracle.lpt3) against the equations of motion.

A pressureless fluid in an Einstein-de Sitter universe, with the growing mode D as the time
variable and x(q, D) = q + D psi1 + D^2 psi2 + D^3 psi3, obeys two exact Lagrangian equations
(the gravitational acceleration is a gradient, and its divergence is the density contrast):

* irrotational flow: eps_ijk (dx_l/dD)_{,j} x_{l,k} = 0;
* Poisson: sum_ij (D^2 x'' + 3/2 D x')_{i,j} cof(X)_ij = -(3/2) (1 - J), X_ij = x_{i,j}, J = det X.

Order by order in D, these fix psi2 given psi1 and psi3 given both.  The tests take psi1, psi2 and
psi3 from the oracle on random band-limited fields (no mode reaches a third of the Nyquist
frequency, so no product the oracle forms aliases and every derivative taken here is exact),
differentiate them spectrally, and check that the order-D^2 vorticity and the order-D^2 and D^3
Poisson residuals vanish to rounding: a dropped term, a wrong sign or coefficient, a transposed
product or a wrong cross product in the oracle all leave a residual of the size of the terms.
"""

import numpy as np
import pytest

from oracle import hessian, lpt3, run

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

N = 32
BOX = 100.0


def band_limited_field(seed, n=N, fmax=2, amp=1.0):
    """Half spectrum with modes |f_i| <= fmax only, Hermitian-consistent, zero mean."""
    rng = np.random.default_rng(seed)
    fx, fy, fz = hessian.freq_grids(n)
    keep = (np.abs(fx) <= fmax) & (np.abs(fy) <= fmax) & (fz <= fmax)
    dk = (rng.standard_normal(keep.shape) + 1j * rng.standard_normal(keep.shape)) * keep
    dk = np.fft.rfftn(np.fft.irfftn(dk, s=(n, n, n), axes=(0, 1, 2)), axes=(0, 1, 2))
    dk[0, 0, 0] = 0.0
    x = np.fft.irfftn(dk, s=(n, n, n), axes=(0, 1, 2))
    return dk * (amp / np.sqrt(np.mean(x ** 2)))


def gradient_matrix(psi, box=BOX):
    """M[i][j] = d psi_i / d q_j (spectral, q in Mpc/h)."""
    n = psi.shape[1]
    fx, fy, fz = hessian.freq_grids(n)
    k = [2.0 * np.pi * f / box for f in (fx, fy, fz)]
    out = []
    for i in range(3):
        pk = np.fft.rfftn(psi[i], axes=(0, 1, 2))
        out.append([np.fft.irfftn(1j * k[j] * pk, s=(n, n, n), axes=(0, 1, 2)) for j in range(3)])
    return out


def eps(i, j, k):
    return ((i - j) * (j - k) * (k - i)) // 2


def displacements(dk):
    return run.za_displacement(dk, BOX), run.lpt2_displacement(dk, BOX), lpt3.lpt3_displacement(dk, BOX)


# truncated power series in D: lists of 4 coefficient arrays (degrees 0..3)
def pmul(p, q):
    return [sum(p[a] * q[n - a] for a in range(n + 1)) for n in range(4)]


def padd(*ps):
    return [sum(p[n] for p in ps) for n in range(4)]


def pscale(p, c):
    return [c * x for x in p]


def poisson_residual(m1, m2, m3):
    """Coefficients (degrees 0..3) of sum_ij A_ij cof(X)_ij + (3/2)(1 - J)."""
    zero = np.zeros_like(m1[0][0])
    ms = (m1, m2, m3)
    X = [[[np.full_like(zero, float(i == j))] + [ms[n][i][j] for n in range(3)] for j in range(3)]
         for i in range(3)]
    cn = [n * (n - 1) + 1.5 * n for n in range(4)]
    A = [[[zero] + [cn[n + 1] * ms[n][i][j] for n in range(3)] for j in range(3)] for i in range(3)]
    cof = [[None] * 3 for _ in range(3)]
    for i in range(3):
        for j in range(3):
            i1, i2 = (i + 1) % 3, (i + 2) % 3
            j1, j2 = (j + 1) % 3, (j + 2) % 3
            cof[i][j] = padd(pmul(X[i1][j1], X[i2][j2]), pscale(pmul(X[i1][j2], X[i2][j1]), -1.0))
    J = padd(*[pmul(X[0][j], cof[0][j]) for j in range(3)])
    lhs = padd(*[pmul(A[i][j], cof[i][j]) for i in range(3) for j in range(3)])
    one = [np.ones_like(zero), zero, zero, zero]
    res = padd(lhs, pscale(padd(one, pscale(J, -1.0)), 1.5))
    scale = [np.max(np.abs(x)) for x in lhs]
    return res, scale


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_irrotational_to_third_order(seed):
    dk = band_limited_field(seed)
    p1, p2, p3 = displacements(dk)
    m1, m2, m3 = (gradient_matrix(p) for p in (p1, p2, p3))
    for i in range(3):
        curl3 = sum(eps(i, j, k) * m3[k][j] for j in range(3) for k in range(3))
        src = sum(eps(i, j, k) * (m1[l][j] * m2[l][k] + 2.0 * m2[l][j] * m1[l][k])
                  for j in range(3) for k in range(3) for l in range(3))
        scale = np.max(np.abs(src))
        assert scale > 1e-3 * np.max(np.abs(m1[0][0])) ** 3           # the term is really there
        assert np.max(np.abs(3.0 * curl3 + src)) <= 1e-11 * scale
        # lower orders: psi1 and psi2 are gradients
        for m in (m1, m2):
            c = sum(eps(i, j, k) * m[k][j] for j in range(3) for k in range(3))
            assert np.max(np.abs(c)) <= 1e-12 * np.max(np.abs(m[0][0]))


@pytest.mark.parametrize("seed", [4, 5, 6])
def test_poisson_to_third_order(seed):
    dk = band_limited_field(seed)
    p1, p2, p3 = displacements(dk)
    res, scale = poisson_residual(*(gradient_matrix(p) for p in (p1, p2, p3)))
    assert np.max(np.abs(res[0])) == 0.0
    assert scale[2] > 0 and scale[3] > 0
    for n in (1, 2, 3):
        assert np.max(np.abs(res[n])) <= 1e-11 * scale[n], f"order D^{n}"


def helmholtz(psi):
    """(curl-free part, divergence-free part) of a periodic vector field, spectrally."""
    n = psi.shape[1]
    f = hessian.freq_grids(n)
    pk = [np.fft.rfftn(psi[i], axes=(0, 1, 2)) for i in range(3)]
    f2 = sum(fa ** 2 for fa in f)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = np.where(f2 > 0, 1.0 / np.where(f2 > 0, f2, 1.0), 0.0)
    div = sum(f[i] * pk[i] for i in range(3)) * inv
    lon = np.stack([np.fft.irfftn(f[i] * div, s=(n, n, n), axes=(0, 1, 2)) for i in range(3)])
    return lon, psi - lon


def test_equations_detect_wrong_third_order_parts():
    """Both equations are sensitive to the parts they pin: 10% more curl-free part of psi3 leaves
    a Poisson residual, 10% more divergence-free part a vorticity residual, of the size of the
    terms (so the tolerances above are not vacuous)."""
    dk = band_limited_field(7)
    p1, p2, p3 = displacements(dk)
    lon, tra = helmholtz(p3)
    assert np.max(np.abs(tra)) > 1e-2 * np.max(np.abs(lon))        # the transverse part is there
    m1, m2 = gradient_matrix(p1), gradient_matrix(p2)
    res, scale = poisson_residual(m1, m2, gradient_matrix(1.1 * lon + tra))
    assert np.max(np.abs(res[3])) > 1e-3 * scale[3]
    res, scale = poisson_residual(m1, m2, gradient_matrix(lon + 1.1 * tra))
    assert np.max(np.abs(res[3])) <= 1e-11 * scale[3]              # Poisson sees only the divergence
    m3 = gradient_matrix(lon + 1.1 * tra)
    worst = 0.0
    for i in range(3):
        curl3 = sum(eps(i, j, k) * m3[k][j] for j in range(3) for k in range(3))
        src = sum(eps(i, j, k) * (m1[l][j] * m2[l][k] + 2.0 * m2[l][j] * m1[l][k])
                  for j in range(3) for k in range(3) for l in range(3))
        worst = max(worst, np.max(np.abs(3.0 * curl3 + src)) / np.max(np.abs(src)))
    assert worst > 1e-3


def test_one_dimensional_field_has_no_higher_orders():
    """A field varying along one axis is exact at first order: mu2 = mu3 = 0, so psi2 = psi3 = 0."""
    rng = np.random.default_rng(11)
    dk = np.zeros((N, N, N // 2 + 1), dtype=complex)
    for f in (1, 2, 5):
        dk[f, 0, 0] = (rng.standard_normal() + 1j * rng.standard_normal()) * N ** 3
        dk[N - f, 0, 0] = np.conj(dk[f, 0, 0])
    p1, p2, p3 = displacements(dk)
    assert np.max(np.abs(p1)) > 1.0
    assert np.max(np.abs(p2)) <= 1e-12 * np.max(np.abs(p1))
    assert np.max(np.abs(p3)) <= 1e-12 * np.max(np.abs(p1))


def test_cubic_in_the_field():
    dk = band_limited_field(8)
    a = lpt3.lpt3_displacement(dk, BOX)
    b = lpt3.lpt3_displacement(-2.0 * dk, BOX)
    assert np.max(np.abs(b + 8.0 * a)) <= 1e-12 * np.max(np.abs(b))


def test_homogeneous_sphere_and_cylinder_series():
    """Locally homogeneous tensors: the divergence of psi3 per unit length along each compressed
    axis matches the third-order coefficient of the exact EdS collapse of a homogeneous sphere
    (x = q (1 - b D - 3/7 b^2 D^2 - 23/63 b^3 D^3), T1 = b I) and cylinder (T1 = a diag(1, 1, 0),
    x_perp = q_perp (1 - a D - 3/14 a^2 D^2 - 5/42 a^3 D^3)); T2 = mu2(T1) / (number of
    compressed axes) on those axes, the Hessian of the potential of a homogeneous source."""
    b = 0.7
    t1 = [np.array(b), np.array(0.0), np.array(0.0), np.array(b), np.array(0.0), np.array(b)]
    m2 = float(lpt3.mu2(t1))
    t2 = [np.array(m2 / 3.0), np.array(0.0), np.array(0.0), np.array(m2 / 3.0), np.array(0.0), np.array(m2 / 3.0)]
    s, c = lpt3.third_order_sources(t1, t2)
    assert abs(float(s) / 3.0 - (-23.0 / 63.0) * b ** 3) <= 1e-15
    assert all(abs(float(ci)) == 0.0 for ci in c)
    a = 0.4
    t1 = [np.array(a), np.array(0.0), np.array(0.0), np.array(a), np.array(0.0), np.array(0.0)]
    m2 = float(lpt3.mu2(t1))
    t2 = [np.array(m2 / 2.0), np.array(0.0), np.array(0.0), np.array(m2 / 2.0), np.array(0.0), np.array(0.0)]
    s, c = lpt3.third_order_sources(t1, t2)
    assert abs(float(s) / 2.0 - (-5.0 / 42.0) * a ** 3) <= 1e-15
