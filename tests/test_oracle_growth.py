"""Pins of the growing-mode clock and of the sigma^2-spaced radius ladder (oracle.growth), and
the native radius ladder (host-only C ABI) against the oracle."""

import numpy as np
import pytest
from scipy import integrate, special

from oracle import growth, spectrum


def _hyp(a, om):
    """Closed form of the flat LambdaCDM growing mode: D ~ a 2F1(1/3, 1; 11/6; -a^3 (1-om)/om)."""
    return a * special.hyp2f1(1.0 / 3.0, 1.0, 11.0 / 6.0, -a ** 3 * (1.0 - om) / om)


@pytest.mark.parametrize("om", [0.25, 0.3, 0.7])
def test_growth_matches_hypergeometric_closed_form(om):
    for a in (1e-3, 0.05, 0.3, 0.7, 1.0, 1.8, 7.0):
        assert abs(growth.growth(a, om) - _hyp(a, om) / _hyp(1.0, om)) <= 1e-12 * growth.growth(a, om)


def test_growth_limits():
    # Einstein-de Sitter: D = a and z_c = F - 1
    for a in (0.37, 3.0, 1e3, 1e6):
        assert abs(growth.growth(a, 1.0) / a - 1.0) <= 1e-13
    F = np.array([0.5, 1.0, 2.0, 7.5])
    assert np.allclose(growth.collapse_redshift(F, 1.0), F - 1.0, rtol=0, atol=1e-13)
    # LambdaCDM: D approaches its limit as D_inf - D ~ a^-2 / (2 (1-om)^(3/2)) * (5 om/2) sqrt(1-om) / D_u(1)
    om = 0.25
    dinf = growth.growth_limit(om)
    c = 2.5 * om / (2.0 * (1.0 - om)) / growth.growth_unnormalised(1.0, om)
    for a in (1e3, 1e4, 1e6):
        assert abs((dinf - growth.growth(a, om)) * a ** 2 / c - 1.0) <= 1e-3
    assert growth.collapse_redshift([1.0 / (dinf * 1.0001)], om)[0] == -1.0
    assert growth.collapse_redshift([0.0, -1.0], om).tolist() == [-1.0, -1.0]


def test_collapse_redshift_inverts_growth():
    om = 0.25
    F = np.array([0.8, 1.0, 1.3, 2.0, 5.0, 30.0])
    z = growth.collapse_redshift(F, om)
    back = np.array([growth.growth(1.0 / (1.0 + zz), om) for zz in z])
    assert np.max(np.abs(back * F - 1.0)) <= 1e-12
    assert abs(z[1]) <= 1e-12


def test_radius_ladder_spacing():
    """sigma^2 of consecutive radii differ by 10^0.15, checked with an independent Simpson rule."""
    n, box = 128, 256.0
    radii = growth.radius_ladder(n, box, 20.0, 1.0)
    amp = spectrum.amplitude_for_sigma8(0.8, 0.21, 1.0)
    cell = box / n

    def s2(r):
        lnk = np.linspace(np.log(1e-7), np.log(60.0 / r), 200001)
        k = np.exp(lnk)
        return integrate.simpson(k ** 3 * spectrum.power(k, amp, 0.21, 1.0) * np.exp(-(k * r) ** 2), x=lnk) / (
            2 * np.pi ** 2)

    v = np.array([s2(r * cell) for r in radii])
    assert np.all(np.diff(radii) < 0) and radii[0] == 20.0 and radii[-1] >= 1.0
    assert np.allclose(np.log10(v[1:] / v[:-1]), 0.15, rtol=0, atol=1e-9)
    assert s2(radii[-1] * cell) * 10 ** 0.15 > s2(1.0 * cell)   # the next step would pass r_min


def test_native_radius_ladder_matches_oracle():
    from paper_1305_1505_amd import binding as B

    for n, box, rmax, rmin in ((512, 1000.0, 60.0, 0.75), (64, 100.0, 20.0, 0.75)):
        ref = growth.radius_ladder(n, box, rmax, rmin)
        got = B.pin_radius_ladder(n, box, rmax, rmin, 0.15, 0.21, 1.0)
        assert len(got) == len(ref)
        assert np.max(np.abs(np.array(got) / np.array(ref) - 1.0)) <= 1e-9
    with pytest.raises(B.PinError):
        B.pin_radius_ladder(64, 100.0, 1.0, 2.0)
