"""Per-point collapse model on the GPU (pin_inverse_collapse_time) vs the oracle, on tensor
families that exercise every branch: random, spheres, planes, exact and near lambda_1 = lambda_2,
axisymmetric, zero, and wide dynamic range.  FP32 plans take float32 inputs; the oracle evaluates
the same float32-rounded tensors in float64."""

import numpy as np
import pytest

from oracle import collapse
from paper_1305_1505_amd import workloads as W

pytestmark = pytest.mark.gpu


def _rot(diag, rng):
    """Random rotations of diagonal tensors; returns the six components (count,) each."""
    q, _ = np.linalg.qr(rng.standard_normal((len(diag), 3, 3)))
    m = np.einsum("nij,nj,nkj->nik", q, diag, q)
    return [m[:, 0, 0], m[:, 0, 1], m[:, 0, 2], m[:, 1, 1], m[:, 1, 2], m[:, 2, 2]]


def families(seed=3, tiny=1e-20):
    rng = np.random.default_rng(seed)
    fam = {}
    fam["random"] = [rng.standard_normal(200000) for _ in range(6)]
    d = rng.uniform(-5, 5, 2000)
    z = np.zeros_like(d)
    fam["sphere"] = [d / 3, z, z, d / 3, z, d / 3]
    lam = rng.uniform(0.01, 3, 2000)
    fam["plane"] = _rot(np.stack([lam, 0 * lam, 0 * lam], 1), rng)
    a, b = rng.uniform(-2, 2, 5000), rng.uniform(-2, 2, 5000)
    fam["l1_eq_l2"] = _rot(np.stack([np.maximum(a, b), np.maximum(a, b), np.minimum(a, b)], 1), rng)
    fam["near_l1_l2"] = _rot(np.stack([np.maximum(a, b) + 1e-6, np.maximum(a, b), np.minimum(a, b)], 1), rng)
    fam["axisym_low"] = _rot(np.stack([np.maximum(a, b), np.minimum(a, b), np.minimum(a, b)], 1), rng)
    fam["zero"] = [np.zeros(64) for _ in range(6)]
    fam["tiny"] = [tiny * rng.standard_normal(1000) for _ in range(6)]
    s = 10.0 ** rng.uniform(-3, 3, 20000)
    fam["scaled"] = [s * rng.standard_normal(20000) for _ in range(6)]
    return fam


def _run(lib, prec, t6):
    plan = lib.Plan(16, 10.0, [1.0], prec=prec)
    import torch

    F = plan.inverse_collapse_time(np.stack(t6)).cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    plan.close()
    return F


@pytest.mark.parametrize("name", list(families().keys()))
def test_fp64_points_match_oracle(lib, name):
    t6 = families()[name]
    F = _run(lib, lib.PIN_FP64, t6)
    ref = collapse.inverse_collapse_time(t6)
    # the oracle's bisection resolves a root to ~1e-33 of its bracket, hence the absolute floor
    scale = np.maximum(1e-20, np.max(np.abs(np.stack(t6)), axis=0))
    err = np.abs(F - ref) / scale
    assert np.max(err) <= 1e-10, f"{name}: worst {np.max(err):.3e}"


@pytest.mark.parametrize("name", list(families().keys()))
def test_fp32_points_match_oracle(lib, name):
    # float32 plans: the invariants are cubic in T, so tensors stay well inside float32 range
    t6 = [c.astype(np.float32).astype(np.float64) for c in families(tiny=1e-5)[name]]
    F = _run(lib, lib.PIN_FP32, t6)
    ref = collapse.inverse_collapse_time(t6)
    scale = np.maximum(1e-20, np.max(np.abs(np.stack(t6)), axis=0))
    err = np.abs(F - ref) / scale
    # float32 inputs and float32 arithmetic: per-point error a few float32 ulps of the tensor scale;
    # the flagged near-degenerate points go through float64
    assert np.quantile(err, 0.999) <= 2e-6, f"{name}: 99.9% {np.quantile(err, 0.999):.3e}"
    assert np.max(err) <= 2e-5, f"{name}: worst {np.max(err):.3e}"


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_negative_planes_do_not_collapse(lib, prec):
    """(-lambda, 0, 0) rotated: the exact answer is F = 0; rounding of the rotated components
    leaves a cubic whose roots scale like the cube root of that rounding, on both sides, so the
    check is |F| small against lambda rather than a match with the oracle."""
    rng = np.random.default_rng(8)
    lam = rng.uniform(0.01, 3, 2000)
    t6 = _rot(np.stack([-lam, 0 * lam, 0 * lam], 1), rng)
    F = _run(lib, lib.PIN_FP64 if prec == "fp64" else lib.PIN_FP32, t6)
    bound = 1e-4 if prec == "fp64" else 2e-2
    assert np.all(F >= 0) and np.all(F <= bound * lam)


def test_empty_count_is_noop(lib):
    import torch

    plan = lib.Plan(16, 10.0, [1.0], prec=lib.PIN_FP32)
    t = torch.zeros((6, 1), dtype=torch.float32, device="cuda")
    F = torch.full((1,), 7.0, dtype=torch.float32, device="cuda")
    lib.pin_inverse_collapse_time(plan.handle, t.data_ptr(), 0, F.data_ptr(), 0)
    torch.cuda.synchronize()
    assert F.item() == 7.0
    plan.close()


def near_cutoff_families(seed=21):
    """Tensor families around the float64 epilogue's switches (float64 plans).

    gap_sweep: lambda_1 - lambda_2 log-spaced from 1e-5 to 1e-1 of the spread lambda_1 - lambda_3,
    across the switch from the closed form (polynomial in sqrt(1 + r) and Newton steps) to Jacobi
    rotations at 1 + r = 1e-5, where the closed form's root is most sensitive to the rounding of
    the characteristic polynomial's coefficients.

    close_roots: the collapse cubic's two largest roots a relative 1e-5 to 1e-1 apart (real and
    distinct), on both sides of its switch from the polynomial to acos/cos at cos(theta) =
    -1 + 1e-8 (a relative gap of about 1e-4).  The largest root then moves by about eps/gap of
    its size under a rounding of the coefficients, on both sides.  Built on the eigenvalues (l1, l2, l3): l3 is found by bisection where
    the discriminant of P vanishes with the upper pair merging, then moved into the three-real
    side and the root gap measured with numpy.roots.
    """
    rng = np.random.default_rng(seed)
    fam = {}
    n = 4000
    l2 = rng.uniform(-2, 2, n)
    l3 = l2 - rng.uniform(0.5, 2, n)
    l1 = l2 + 10.0 ** rng.uniform(-5, -1, n) * (l2 - l3)
    fam["gap_sweep"] = _rot(np.stack([l1, l2, l3], 1), rng)

    def cubic(a, b, c):
        mu2 = a * b + a * c + b * c
        mu3 = a * b * c
        d = a + b + c
        return np.array([1.0, -a, -mu2 / 7.0, mu3 / 9.0 - 10.0 * d * mu2 / 189.0])

    def disc(coef):
        _, p2, p1, p0 = coef
        a3 = p2 / 3.0
        hq = 0.5 * (p0 - a3 * p1 + 2.0 * a3 ** 3)
        p3 = (p1 - p2 * a3) / 3.0
        return hq * hq + p3 ** 3

    rows, gaps = [], []
    while len(rows) < 1500:
        a = rng.uniform(0.3, 2.0)
        b = a * rng.uniform(-0.9, 0.9)
        grid = np.linspace(-3.0 * a, b, 400)
        dv = np.array([disc(cubic(a, b, c)) for c in grid])
        for k in np.nonzero(np.sign(dv[:-1]) != np.sign(dv[1:]))[0]:
            lo, hi = grid[k], grid[k + 1]
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                if np.sign(disc(cubic(a, b, mid))) == np.sign(disc(cubic(a, b, lo))):
                    lo = mid
                else:
                    hi = mid
            c0 = 0.5 * (lo + hi)
            for frac in 10.0 ** rng.uniform(-11, -2, 4):
                for c in (c0 * (1 + frac), c0 * (1 - frac)):
                    if not b >= c:
                        continue
                    r = np.roots(cubic(a, b, c))
                    if np.max(np.abs(r.imag)) > 0:
                        continue
                    r = np.sort(r.real)
                    if r[2] <= 0 or r[1] < r[0] + 0.5 * (r[2] - r[0]):
                        continue                     # the upper pair is the close one
                    gap = (r[2] - r[1]) / r[2]
                    if 1e-5 <= gap <= 1e-1:
                        rows.append((a, b, c))
                        gaps.append(gap)
    lam = np.array(rows)
    fam["close_roots"] = _rot(lam, rng)
    fam["close_roots_gap"] = np.array(gaps)
    return fam


@pytest.mark.parametrize("name", ["gap_sweep", "close_roots"])
def test_fp64_points_near_switches(lib, name):
    """float64 plans at rounding accuracy on both sides of the epilogue's switches."""
    fam = near_cutoff_families()
    t6 = fam[name]
    F = _run(lib, lib.PIN_FP64, t6)
    ref = collapse.inverse_collapse_time(t6)
    scale = np.max(np.abs(np.stack(t6)), axis=0)
    err = np.abs(F - ref) / scale
    # two roots a relative gap apart amplify a rounding of the cubic's coefficients ~1/gap-fold
    bound = 1e-13 + (5e-15 / fam["close_roots_gap"] if name == "close_roots" else 0.0)
    print(f"[points] {name}: fp64 worst {np.max(err):.3g}, worst / bound {np.max(err / bound):.3g}", flush=True)
    assert np.all(err <= bound), name
