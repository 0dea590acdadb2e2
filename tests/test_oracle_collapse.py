"""Pins of the oracle's collapse model against exact mathematics.

* delta_c from a numerical integration of the exact EdS spherical-collapse equation;
* the 3rd-order sphere series against the same exact solution (residual scales as x^4);
* planar collapse: the Zel'dovich solution is exact, F = lambda_1;
* the sphere: F = delta/delta_c (the paper's statement for spherical collapse);
* homogeneity of degree 1; the root finder against numpy.roots and a dense scan of J1(D);
* lambda_1 against the closed trigonometric form; invariants against eigenvalues;
* each coefficient of the E3 cubic against the LPT oracles, which the equations of motion pin:
  a = -lambda_1 of the Zel'dovich displacement gradient, b = div(psi2)/3 from the 2LPT
  displacement, c = div(psi3)/3 from the 3LPT source with the second-order potential Hessian
  taken isotropic (mu2/3 on each axis), i.e. every order shared equally by the three axes.
"""

import functools

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import collapse, hessian, lpt3, run


@functools.lru_cache(maxsize=None)
def _eds_shell(delta_i=1e-9):
    """Exact EdS spherical collapse of a top-hat shell, integrated numerically.

    With the unperturbed shell radius t^(2/3) as unit and r = t^(2/3) (1 - u), Newton's
    r'' = -GM/r^2 becomes, in s = ln t, u'' + u'/3 = (2/9) [(1 - u)^-2 - (1 - u)].  The linear
    growing mode is u = delta_L/3 with delta_L = eps t^(2/3); start there at t = 1 with a tiny
    delta_L and integrate until the shell radius falls to 1e-5 of the unperturbed one (the
    remaining time to collapse is then a fraction ~(1e-5)^(3/2) of t).
    """
    eps = delta_i

    def rhs(s, y):
        u, du = y
        return [du, -du / 3 + (2 / 9) * ((1 - u) ** -2 - (1 - u))]

    def crash(s, y):
        return y[0] - (1 - 1e-5)
    crash.terminal = True
    sol = solve_ivp(rhs, [0.0, 60.0], [delta_i / 3, 2 * delta_i / 9], method="DOP853",
                    rtol=1e-12, atol=1e-20, events=crash, dense_output=True)
    return sol, eps


def test_delta_c_from_exact_spherical_collapse():
    sol, eps = _eds_shell()
    t_c = np.exp(sol.t_events[0][0])
    delta_c = eps * t_c ** (2 / 3)
    assert abs(delta_c / collapse.DELTA_C - 1) < 1e-6


def test_third_order_sphere_series_against_exact_solution():
    sol, eps = _eds_shell()
    res = []
    for x in (0.05, 0.1, 0.2):
        s = 1.5 * np.log(x / eps)                     # delta_L(t) = eps t^(2/3) = x
        ratio = 1 - sol.sol(s)[0]                     # R / R_L of the exact solution
        res.append(ratio - collapse._eds_sphere_3lpt(x))
    # the residual is 4th order: doubling x multiplies it by ~16 (a wrong 3rd-order term gives ~8)
    assert 14 < res[1] / res[0] < 18 and 14 < res[2] / res[1] < 19
    assert abs(res[0]) < 1e-6


def test_sphere_root_constant():
    assert abs(collapse._eds_sphere_3lpt(collapse.X3)) < 1e-14
    assert 2.0500 < collapse.X3 < 2.0502


def _iso(d):
    d = np.asarray(d, dtype=float)
    z = np.zeros_like(d)
    return [d / 3, z, z, d / 3, z, d / 3]


def test_sphere_gives_delta_over_delta_c():
    d = np.array([1e-3, 0.1, 1.0, 1.686, 5.0, 40.0])
    f = collapse.inverse_collapse_time(_iso(d))
    assert np.max(np.abs(f * collapse.DELTA_C / d - 1)) < 1e-13
    # underdense spheres never collapse
    assert np.all(collapse.inverse_collapse_time(_iso(-d)) == 0)


def _rot(t6, seed):
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    m = np.array([[t6[0], t6[1], t6[2]], [t6[1], t6[3], t6[4]], [t6[2], t6[4], t6[5]]], dtype=float)
    r = q @ m @ q.T
    return [r[0, 0], r[0, 1], r[0, 2], r[1, 1], r[1, 2], r[2, 2]]


@pytest.mark.parametrize("lam", [0.3, 1.0, 2.5])
def test_planar_collapse_is_zeldovich(lam):
    t6 = _rot([lam, 0, 0, 0, 0, 0], int(lam * 10))
    f = collapse.inverse_collapse_time([np.array([v]) for v in t6])
    assert abs(f[0] - lam) < 1e-12
    t6 = _rot([-lam, 0, 0, 0, 0, 0], 3)
    # rounding in the rotation leaves |lambda_1| ~ 1e-17; the cubic's root then scales like its
    # cube root, so "no collapse" means F negligible against lam
    assert collapse.inverse_collapse_time([np.array([v]) for v in t6])[0] < 1e-5 * lam


def _random_tensors(n, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return [scale * rng.standard_normal(n) for _ in range(6)]


def test_invariants_against_eigenvalues():
    t6 = _random_tensors(2000, 1)
    d, mu2, mu3, p = collapse.invariants(t6)
    m = np.stack([np.stack([t6[0], t6[1], t6[2]], -1), np.stack([t6[1], t6[3], t6[4]], -1),
                  np.stack([t6[2], t6[4], t6[5]], -1)], -2)
    ev = np.linalg.eigvalsh(m)
    assert np.allclose(d, ev.sum(1), atol=1e-12)
    assert np.allclose(mu2, ev[:, 0] * ev[:, 1] + ev[:, 0] * ev[:, 2] + ev[:, 1] * ev[:, 2], atol=1e-11)
    assert np.allclose(mu3, ev.prod(1), atol=1e-11)
    assert np.allclose(p, np.sqrt(np.sum((ev - ev.mean(1, keepdims=True)) ** 2, 1) / 6), atol=1e-12)
    l1 = collapse.largest_eigenvalue(t6)
    assert np.allclose(l1, ev[:, 2], atol=1e-12)
    # closed trigonometric form lambda_1 = m + 2 p cos(acos(det(B)/(2p^3))/3)
    mm = d / 3
    b = m - mm[:, None, None] * np.eye(3)
    r = np.clip(np.linalg.det(b) / (2 * p ** 3), -1, 1)
    assert np.allclose(l1, mm + 2 * p * np.cos(np.arccos(r) / 3), atol=1e-9)


def test_largest_real_root_against_numpy_roots():
    rng = np.random.default_rng(5)
    a, b, c = rng.standard_normal((3, 3000)) * np.array([[1.0], [2.0], [0.5]])
    r = collapse.largest_real_root(a, b, c)
    for k in range(3000):
        roots = np.roots([1.0, a[k], b[k], c[k]])
        real = roots[np.abs(roots.imag) < 1e-7 * max(1.0, np.max(np.abs(roots)))].real
        assert abs(r[k] - real.max()) < 1e-9 * max(1.0, abs(real.max()))


def test_cubic_special_cases():
    # x^3 (triple root 0), (x-1)^2 (x+2) double root at 1, (x-3)(x^2+1)
    a = np.array([0.0, 0.0, -3.0])
    b = np.array([0.0, -3.0, 1.0])
    c = np.array([0.0, 2.0, -3.0])
    r = collapse.largest_real_root(a, b, c)
    assert abs(r[0]) < 1e-12 and abs(r[1] - 1) < 1e-7 and abs(r[2] - 3) < 1e-12


def test_e3_root_is_first_zero_of_j1_by_dense_scan():
    t6 = _random_tensors(300, 9)
    d, mu2, mu3, p = collapse.invariants(t6)
    l1 = collapse.largest_eigenvalue(t6)
    f = collapse.e3_inverse_time(l1, d, mu2, mu3)
    dgrid = np.linspace(1e-6, 50.0, 500001)
    for k in range(300):
        j1 = 1 - l1[k] * dgrid - mu2[k] / 7 * dgrid ** 2 + (mu3[k] / 9 - 10 * d[k] * mu2[k] / 189) * dgrid ** 3
        neg = np.nonzero(j1 <= 0)[0]
        if neg.size == 0:
            assert f[k] == 0 or 1 / f[k] > 49.9
        else:
            dc = dgrid[neg[0]]
            assert f[k] > 0 and abs(1 / f[k] - dc) <= 1.5e-4 * max(1, dc)


def test_homogeneity_and_bounds():
    t6 = _random_tensors(5000, 2)
    f1 = collapse.inverse_collapse_time(t6)
    for s in (0.01, 3.0, 100.0):
        fs = collapse.inverse_collapse_time([s * x for x in t6])
        assert np.allclose(fs, s * f1, rtol=1e-11, atol=1e-14)
    l1 = collapse.largest_eigenvalue(t6)
    # collapse never precedes the Zel'dovich crossing by more than the sphere factor, never negative
    assert np.all(f1 >= 0)
    d, mu2, mu3, p = collapse.invariants(t6)
    assert np.all(f1[l1 <= 0] == 0)


def test_sphericity_limits():
    assert collapse.sphericity(np.array([1.0]), np.array([0.0]))[0] == 1.0
    assert collapse.sphericity(np.array([1.0]), np.array([1 / 3]))[0] == 0.0
    assert collapse.sphericity(np.array([-1.0]), np.array([0.0]))[0] == 0.0


def _band_limited_field(seed, n=32, fmax=2):
    """Half spectrum with |f_i| <= fmax only (no product of two fields reaches the Nyquist
    frequency, so spectral derivatives of the LPT fields are exact), unit rms."""
    rng = np.random.default_rng(seed)
    fx, fy, fz = hessian.freq_grids(n)
    keep = (np.abs(fx) <= fmax) & (np.abs(fy) <= fmax) & (fz <= fmax)
    dk = (rng.standard_normal(keep.shape) + 1j * rng.standard_normal(keep.shape)) * keep
    dk = np.fft.rfftn(np.fft.irfftn(dk, s=(n, n, n), axes=(0, 1, 2)), axes=(0, 1, 2))
    dk[0, 0, 0] = 0.0
    x = np.fft.irfftn(dk, s=(n, n, n), axes=(0, 1, 2))
    return dk / np.sqrt(np.mean(x ** 2))


def _spectral_gradient(psi, box):
    """g[i][j] = d psi_i / d q_j of a periodic vector field (q in the units of box)."""
    n = psi.shape[1]
    f = hessian.freq_grids(n)
    out = []
    for i in range(3):
        pk = np.fft.rfftn(psi[i], axes=(0, 1, 2))
        out.append([np.fft.irfftn(1j * (2 * np.pi / box) * f[j] * pk, s=(n, n, n), axes=(0, 1, 2))
                    for j in range(3)])
    return out


def _lpt_coefficient_residuals(coefficients, seed=12, box=100.0):
    """Largest |residual| / scale of (a, b, c) from `coefficients` against the LPT oracles.

    With the growing mode D as clock and every order >= 2 shared equally by the three axes, the
    stretch of the first axis is J1(D) = 1 + D psi1_{1,1} + D^2 div(psi2)/3 + D^3 div(psi3)/3,
    and F^3 J1(1/F) = F^3 + a F^2 + b F + c.  psi1_{1,1} along the first axis is minus the largest
    eigenvalue of -grad(psi1) (the Zel'dovich displacement's gradient is -T); div(psi2) is taken
    spectrally from the 2LPT displacement (whose k = 0 mode is removed, so both sides lose their
    mean); div(psi3) is the 3LPT divergence source evaluated with T2 = (mu2/3) I.
    """
    dk = _band_limited_field(seed)
    t1 = hessian.deformation_tensor(dk, None)
    delta, mu2, mu3, p = collapse.invariants(t1)
    l1 = collapse.largest_eigenvalue(t1)
    a, b, c = coefficients(l1, delta, mu2, mu3)
    g1 = _spectral_gradient(run.za_displacement(dk, box), box)
    mt = -np.stack([np.stack([0.5 * (g1[i][j] + g1[j][i]) for j in range(3)], -1) for i in range(3)], -2)
    a_lpt = -np.linalg.eigvalsh(mt)[..., 2]
    g2 = _spectral_gradient(run.lpt2_displacement(dk, box), box)
    div2 = g2[0][0] + g2[1][1] + g2[2][2]
    m2 = lpt3.mu2(t1)
    z = np.zeros_like(m2)
    s3, _ = lpt3.third_order_sources(t1, [m2 / 3.0, z, z, m2 / 3.0, z, m2 / 3.0])
    res_a = np.max(np.abs(a - a_lpt)) / np.max(np.abs(a_lpt))
    res_b = np.max(np.abs((3.0 * b - np.mean(3.0 * b)) - div2)) / np.max(np.abs(div2))
    res_c = np.max(np.abs(3.0 * c - s3)) / np.max(np.abs(s3))
    return res_a, res_b, res_c


def test_cubic_coefficients_are_the_lpt_traces():
    res = _lpt_coefficient_residuals(collapse.cubic_coefficients)
    assert max(res) <= 1e-12, res


def test_cubic_constant_term_is_the_isotropic_3lpt_source_on_random_tensors():
    t6 = _random_tensors(20000, 13)
    delta, mu2, mu3, p = collapse.invariants(t6)
    _, b, c = collapse.cubic_coefficients(collapse.largest_eigenvalue(t6), delta, mu2, mu3)
    m2 = lpt3.mu2(t6)
    z = np.zeros_like(m2)
    s3, _ = lpt3.third_order_sources(t6, [m2 / 3.0, z, z, m2 / 3.0, z, m2 / 3.0])
    assert np.max(np.abs(3.0 * c - s3)) <= 1e-14 * np.max(np.abs(s3))
    # the isotropic second-order Hessian has trace mu2, the 2LPT potential's Laplacian
    assert np.max(np.abs(mu2 - m2)) <= 1e-14 * np.max(np.abs(m2))


def _true_plane(lam, seed):
    return [np.array([v]) for v in _rot([lam, 0, 0, 0, 0, 0], seed)]


def test_pins_catch_planted_mistakes(monkeypatch):
    """Each plausible slip in the E3 cubic fails a pin.  The sphere and the plane only fix the sum
    of the higher-order weights at lambda_i = delta/3 and the first-order term; two slips pass
    both (the anisotropic second-order split -(3/7) lambda_2 lambda_3, and a shift of weight
    between mu3 and delta mu2 that keeps the sphere's sum), and the LPT-trace pin catches them."""
    good = collapse.cubic_coefficients
    sphere = _iso(np.array([1.3]))
    plane = _true_plane(0.9, 4)
    # old slips: each moves the sphere or the plane
    visible = [
        lambda l1, d, m2, m3: (-l1, -m2 / 7, m3 / 9),                         # dropped delta mu2
        lambda l1, d, m2, m3: (-l1, +m2 / 7, m3 / 9 - 10 * d * m2 / 189),      # sign of mu2/7
        lambda l1, d, m2, m3: (-l1, -m2 / 7, m3 / 3 - 10 * d * m2 / 189),      # wrong mu3 weight
        lambda l1, d, m2, m3: (-d, -m2 / 7, m3 / 9 - 10 * d * m2 / 189),       # delta for lambda_1
    ]
    # slips the sphere and the plane cannot see
    hidden = [
        # -(3/7) lambda_2 lambda_3 on the first axis, with lambda_2 lambda_3 = mu2 - l1 (delta - l1)
        lambda l1, d, m2, m3: (-l1, -(3.0 / 7.0) * (m2 - l1 * (d - l1)), m3 / 9 - 10 * d * m2 / 189),
        # mu3/9 -> 2 mu3/9 with the delta mu2 weight moved to keep the sphere's sum
        lambda l1, d, m2, m3: (-l1, -m2 / 7, 2 * m3 / 9 - (10.0 / 189 + 1.0 / 81) * d * m2),
    ]
    for bad in visible + hidden:
        monkeypatch.setattr(collapse, "cubic_coefficients", bad)
        f_s = collapse.inverse_collapse_time(sphere)[0]
        f_p = collapse.inverse_collapse_time(plane)[0]
        moved = abs(f_s - 1.3 / collapse.DELTA_C) > 1e-6 or abs(f_p - 0.9) > 1e-6
        assert moved == (bad in visible)
        assert max(_lpt_coefficient_residuals(bad)) > 1e-2
    monkeypatch.setattr(collapse, "cubic_coefficients", good)
    assert max(_lpt_coefficient_residuals(good)) <= 1e-12
