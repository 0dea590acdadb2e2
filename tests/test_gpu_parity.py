"""HIP path vs the FP64 oracle, element by element, through the C ABI (GPU tests).

Tolerances: FP64 plans agree with the oracle to rounding (1e-11 relative to the field's maximum);
FP32 plans (complex64 FFTs) to 2e-6 relative RMS and 1e-5 relative maximum on intermediate
fields, which is the single-precision FFT error ~ eps32 * log2(N) with margin.
"""

import numpy as np
import pytest

from oracle import collapse, field, hessian, metrics, run
from paper_1305_1505_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-11


def _plan(lib, n, radii, prec, box=100.0):
    return lib.Plan(n, box, radii, sigma8=W.SIGMA8, gamma=W.GAMMA, ns=W.NS, prec=prec)


def _to_dev(arr, plan):
    import torch

    return torch.from_numpy(np.ascontiguousarray(arr)).to(device="cuda", dtype=plan.cplx)


def _host(t):
    import torch

    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("n", [8, 12, 16, 24, 32, 64])
def test_field_fp64_matches_oracle(lib, n):
    box, seed = 75.0, 1234 + n
    plan = _plan(lib, n, [1.0], lib.PIN_FP64, box)
    dk = _host(plan.generate_field(seed))
    ref = field.linear_field(seed, n, box, W.SIGMA8, W.GAMMA, W.NS)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(dk - ref)) <= 1e-13 * scale
    # exact zeros and exact conjugate pairs are structural, not rounding
    assert np.array_equal(dk == 0, ref == 0)
    plane = dk[:, :, 0]
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    assert np.array_equal(plane[(n - ii) % n, (n - jj) % n], np.conj(plane))
    plan.close()


def test_field_fp32_matches_oracle(lib):
    n, box, seed = 64, 100.0, 101
    plan = _plan(lib, n, [1.0], lib.PIN_FP32, box)
    dk = _host(plan.generate_field(seed)).astype(np.complex128)
    ref = field.linear_field(seed, n, box, W.SIGMA8, W.GAMMA, W.NS)
    assert np.max(np.abs(dk - ref)) <= 1e-7 * np.max(np.abs(ref))
    plan.close()


SIZES64 = [8, 12, 16, 24, 32, 48, 64, 96]


@pytest.mark.parametrize("n", SIZES64)
@pytest.mark.parametrize("r", [-1, 0])
def test_deformation_tensor_fp64(lib, n, r):
    radius = 1.7
    plan = _plan(lib, n, [radius], lib.PIN_FP64)
    spec = W.random_half_spectrum(n, 50 + n)
    t6 = _host(plan.deformation_tensor(_to_dev(spec, plan), r))
    ref = hessian.deformation_tensor(spec, None if r < 0 else radius)
    scale = max(np.max(np.abs(c)) for c in ref)
    for c in range(6):
        assert np.max(np.abs(t6[c] - ref[c])) <= TOL64 * scale, f"component {c}"
    plan.close()


@pytest.mark.parametrize("n", [16, 32, 64, 128])
def test_deformation_tensor_fp32(lib, n):
    radius = 2.5
    plan = _plan(lib, n, [radius], lib.PIN_FP32)
    spec = W.random_half_spectrum(n, 70 + n)
    t6 = _host(plan.deformation_tensor(_to_dev(spec, plan), 0)).astype(np.float64)
    ref = hessian.deformation_tensor(spec, radius)
    for c in range(6):
        assert metrics.rel_rms(t6[c], ref[c]) <= 2e-6, f"component {c}"
        assert metrics.rel_max(t6[c], ref[c]) <= 1e-5, f"component {c}"
    plan.close()


@pytest.mark.parametrize("n", [16, 24, 32])
def test_collapse_range_fp64_matches_oracle(lib, n):
    import torch

    radii = W.radii_cells(5, 4.0, 0.75)
    box, seed = 50.0, 99 + n
    dk_ref = field.linear_field(seed, n, box, W.SIGMA8, W.GAMMA, W.NS)
    plan = _plan(lib, n, radii, lib.PIN_FP64, box)
    dk = _to_dev(dk_ref, plan)
    F = torch.empty((n, n, n), dtype=torch.float64, device="cuda")
    R = torch.empty((n, n, n), dtype=torch.uint8, device="cuda")
    plan.collapse_reset(F, R)
    plan.collapse_times_range(dk, F, R, 0, 2)
    plan.collapse_times_range(dk, F, R, 2, len(radii))
    f_ref, r_ref = run.collapse_times(dk_ref, radii)
    f, r = _host(F), _host(R)
    assert metrics.rel_rms(f, f_ref) <= 1e-11
    assert metrics.rel_max(f, f_ref) <= 1e-9
    assert np.array_equal(r, r_ref)
    plan.close()


def test_collapse_per_point_function_fp64(lib):
    """Tensors with known answers through the whole path: a triple-cosine field.

    delta = A (cos kx + cos ky + cos kz) gives a diagonal T; at q = 0 it is a sphere, so
    F = 3 A W / delta_c; along the axes the oracle's formula is evaluated on the same tensors.
    """
    import torch

    n, m, amp, radius = 32, 2, 0.6, 1.0
    q = np.arange(n)
    c = np.cos(2 * np.pi * m * q / n)
    x = amp * (c[:, None, None] + c[None, :, None] + c[None, None, :])
    spec = np.fft.rfftn(x, axes=(0, 1, 2))
    plan = _plan(lib, n, [radius], lib.PIN_FP64)
    F, R = plan.collapse_times(_to_dev(spec, plan))
    f = _host(F)
    wk = np.exp(-0.5 * (2 * np.pi * m * radius / n) ** 2)
    assert abs(f[0, 0, 0] - 3 * amp * wk / collapse.DELTA_C) < 1e-12
    t6 = hessian.deformation_tensor(spec, radius)
    ref = np.maximum(collapse.inverse_collapse_time(t6), 0)
    l1 = collapse.largest_eigenvalue(t6)
    # away from lambda_1 = 0 F is well conditioned: compared to rounding, voids (lambda_1 < 0,
    # F = 0) included.  Where lambda_1 = 0 up to FFT rounding (3088 of the 32768 points: a zero
    # tensor or a negative plane, whose cubic has a triple root at F = 0) the root is the cube
    # root of that rounding on both sides (the oracle itself moves by ~1e-6 under 1e-16 input
    # noise), so there F is checked against its exact value 0 within that size.
    good = np.abs(l1) > 1e-8
    assert np.count_nonzero(~good) == 3088
    assert np.max(np.abs(f - ref)[good]) < 1e-11
    assert np.max(f[~good]) < 1e-5
    plan.close()


def test_config_c64_fp64_end_to_end(lib):
    """64^3, 100 Mpc/h, 16 radii 20 -> 0.75 cells, float64: field, F_max, R_max vs the oracle."""
    cfg = W.CONFIGS["c64_fp64"]
    n, box, seed = cfg["n"], cfg["box"], cfg["seed"]
    radii = W.config_radii(cfg)
    plan = _plan(lib, n, radii, lib.PIN_FP64, box)
    dk_ref = field.linear_field(seed, n, box, W.SIGMA8, W.GAMMA, W.NS)
    dk_gpu = plan.generate_field(seed)
    assert np.max(np.abs(_host(dk_gpu) - dk_ref)) <= 1e-13 * np.max(np.abs(dk_ref))
    F, R = plan.collapse_times(_to_dev(dk_ref, plan))
    f_ref, r_ref = run.collapse_times(dk_ref, radii)
    f, r = _host(F), _host(R)
    rep = metrics.report(f, f_ref)
    assert rep["rel_rms"] <= 1e-11 and rep["rel_max"] <= 1e-9
    assert np.array_equal(r, r_ref)
    plan.close()


@pytest.mark.parametrize("n", [16, 24, 32])
def test_displacements_fp64(lib, n):
    box = 40.0
    plan = _plan(lib, n, [1.0], lib.PIN_FP64, box)
    dk_ref = field.linear_field(5 + n, n, box, W.SIGMA8, W.GAMMA, W.NS) * hessian.gaussian_window(n, 1.0)
    p1, p2 = plan.displacements(_to_dev(dk_ref, plan))
    r1, r2 = run.displacements(dk_ref, box)
    p1, p2 = _host(p1), _host(p2)
    for a in range(3):
        assert np.max(np.abs(p1[a] - r1[a])) <= TOL64 * np.max(np.abs(r1)), f"psi1 {a}"
        assert np.max(np.abs(p2[a] - r2[a])) <= TOL64 * np.max(np.abs(r2)), f"psi2 {a}"
    plan.close()


def test_displacements_fp32(lib):
    n, box = 64, 100.0
    plan = _plan(lib, n, [1.0], lib.PIN_FP32, box)
    dk_ref = field.linear_field(77, n, box, W.SIGMA8, W.GAMMA, W.NS)
    p1, p2 = plan.displacements(_to_dev(dk_ref, plan))
    r1, r2 = run.displacements(dk_ref, box)
    assert metrics.rel_rms(_host(p1).astype(np.float64), r1) <= 1e-5
    assert metrics.rel_rms(_host(p2).astype(np.float64), r2) <= 1e-5
    plan.close()


def test_config_c64_fp32_end_to_end(lib):
    """64^3, 100 Mpc/h, 16 radii, float32 FFTs: F within 1e-5 relative RMS of the FP64 oracle and
    the collapse radius unchanged for all but 1e-4 of the points."""
    cfg = W.CONFIGS["c64_fp64"]
    n, box, seed = cfg["n"], cfg["box"], cfg["seed"]
    radii = W.config_radii(cfg)
    plan = _plan(lib, n, radii, lib.PIN_FP32, box)
    dk_ref = field.linear_field(seed, n, box, W.SIGMA8, W.GAMMA, W.NS)
    F, R = plan.collapse_times(_to_dev(dk_ref, plan))
    f_ref, r_ref = run.collapse_times(dk_ref, radii)
    f, r = _host(F).astype(np.float64), _host(R)
    assert metrics.rel_rms(f, f_ref) <= 1e-5
    assert metrics.mismatch_fraction(r, r_ref) <= 1e-4
    plan.close()
