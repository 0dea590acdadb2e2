"""pin_collapse_redshift (growing-mode clock, flat LambdaCDM) vs the oracle, through the C ABI."""

import numpy as np
import pytest

from oracle import growth

pytestmark = pytest.mark.gpu

# 0 and negatives (no collapse), values around the no-collapse limit 1/D_inf (0.7488 for
# omega_m = 0.25), z_c = 0 (F = 1), the table, and F beyond the first node (a < 1e-3)
F_EDGE = [0.0, -2.0, 1e-7, 0.5, 0.7488, 0.74885, 0.749, 0.8, 1.0, 1.0 + 1e-9, 1.5, 3.0, 10.0, 100.0, 999.0,
          1500.0, 5e4]


def _values(seed=5, count=120):
    rng = np.random.default_rng(seed)
    return np.concatenate([np.array(F_EDGE), rng.uniform(0.75, 20.0, count), 10 ** rng.uniform(-3, 3, 40)])


@pytest.mark.parametrize("om", [0.25, 1.0])
def test_redshift_fp64(lib, om):
    import torch

    plan = lib.Plan(16, 10.0, [1.0], prec=lib.PIN_FP64)
    plan.set_growth(om)
    F = _values()
    z = plan.collapse_redshift(torch.tensor(F, dtype=torch.float64, device="cuda")).cpu().numpy()
    ref = growth.collapse_redshift(F, om)
    never = ref == -1.0
    assert np.all(z[never] == -1.0)
    # the table ends at a = 1e6: an F whose collapse lies beyond it reads as never (z_c > -1 + 1e-6)
    late = ~never & (z == -1.0)
    assert np.all(ref[late] < -1.0 + 1e-6)
    ok = ~never & ~late
    # the defining equation D(z_c) F = 1 with the oracle's D (well conditioned, unlike z_c itself
    # near the no-collapse limit where D is flat in a)
    resid = np.array([growth.growth(1.0 / (1.0 + zz), om) * f - 1.0 for zz, f in zip(z[ok], F[ok])])
    assert np.max(np.abs(resid)) <= 1e-12
    assert np.max(np.abs((1.0 + z[ok]) / (1.0 + ref[ok]) - 1.0)) <= 1e-9
    plan.close()


def test_redshift_fp32(lib):
    """float32 plans: F and z_c are float32, the computation float64; z_c is within one float32
    rounding of the oracle's value for the same (float32) F."""
    import torch

    om = 0.25
    plan = lib.Plan(16, 10.0, [1.0], prec=lib.PIN_FP32)
    plan.set_growth(om)
    F = _values(6).astype(np.float32)
    z = plan.collapse_redshift(torch.tensor(F, device="cuda")).cpu().numpy().astype(np.float64)
    ref = growth.collapse_redshift(F.astype(np.float64), om)
    assert np.all(z[ref == -1.0] == -1.0)
    m = ref != -1.0
    assert np.all(np.abs(z[m] - ref[m]) <= 2.0 ** -23 * np.maximum(np.abs(ref[m]), 1e-30) + 1e-12)
    plan.close()


def test_redshift_needs_table(lib):
    import torch

    plan = lib.Plan(16, 10.0, [1.0], prec=lib.PIN_FP32)
    with pytest.raises(lib.PinError):
        plan.collapse_redshift(torch.ones(4, device="cuda"))
    with pytest.raises(lib.PinError):
        plan.set_growth(0.0)
    plan.close()


@pytest.mark.parametrize("om", [1.0, 0.25])
def test_redshift_dense_sweep(lib, om):
    """2^20 values of F log-uniform over the whole table (and beyond its first node), float64.
    Einstein-de Sitter has the closed form D = a, so z_c = F - 1 for every value; for LambdaCDM
    z_c must rise strictly with F (a value searched in the wrong node interval would sit on
    a clamped segment end) and a spread sample solves D(z_c) F = 1 with the oracle's D."""
    import torch

    plan = lib.Plan(16, 10.0, [1.0], prec=lib.PIN_FP64)
    plan.set_growth(om)
    lo = 1e-6 if om == 1.0 else 1.0 / growth.growth_limit(om) * (1.0 + 1e-9)
    F = np.geomspace(lo, 5e3, 1 << 20)
    z = plan.collapse_redshift(torch.tensor(F, dtype=torch.float64, device="cuda")).cpu().numpy()
    plan.close()
    if om == 1.0:
        ok = z != -1.0                       # a = 1e6 ends the table: F < 1e-6 reads as never
        assert np.all(F[~ok] <= 1e-6 * (1.0 + 1e-6)) and ok.sum() > (1 << 20) - 4
        # 1 + z_c to 1e-12 relative, besides the float64 rounding of z_c itself (as z_c -> -1 that
        # rounding and that of F - 1 are each 1e-16 / (1 + z_c) relative to 1 + z_c)
        assert np.all(np.abs(z[ok] - (F[ok] - 1.0)) <= 1e-12 * F[ok] + 2.0 ** -52 * np.abs(z[ok]))
        return
    ok = z != -1.0
    assert np.all(np.diff(z[ok]) > 0.0)
    idx = np.flatnonzero(ok)[np.linspace(0, ok.sum() - 1, 40).astype(int)]
    resid = np.array([growth.growth(1.0 / (1.0 + z[i]), om) * F[i] - 1.0 for i in idx])
    assert np.max(np.abs(resid)) <= 1e-12
