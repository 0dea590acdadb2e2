"""Third-order displacement: pin_lpt3_displacement vs the FP64 oracle (oracle.lpt3), through the
C ABI (GPU tests).

Inputs are oracle fields uploaded to the device.  FP64 plans agree with the oracle to rounding
(1e-11 of the field's maximum, per component); the FP32 plan to 1e-5 relative RMS, the bound on
the closing displacements, and 1e-4 of the maximum per point (psi3 is a cubic in the field: three
complex64 FFT chains, each ~eps32 log2 N).  At the benchmark size the result is checked through
properties that hold exactly in floating point (odd in the field, repeatable bit for bit) and
against the second- and first-order displacements' scale; the full-grid comparison with the
oracle at 256^3 runs here, at 512^3 in the accuracy report.
"""

import numpy as np
import pytest

from oracle import field, hessian, lpt3, metrics
from paper_1305_1505_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-11


def _plan(lib, n, prec, box):
    return lib.Plan(n, box, [1.0], sigma8=W.SIGMA8, gamma=W.GAMMA, ns=W.NS, prec=prec)


def _to_dev(arr, plan):
    import torch

    return torch.from_numpy(np.ascontiguousarray(arr)).to(device="cuda", dtype=plan.cplx)


def _host(t):
    import torch

    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("n", [8, 12, 16, 24, 32, 48])
def test_lpt3_fp64_matches_oracle(lib, n):
    box = 2.5 * n
    print(f"[lpt3] fp64 n={n}", flush=True)
    plan = _plan(lib, n, lib.PIN_FP64, box)
    dk = field.linear_field(300 + n, n, box, W.SIGMA8, W.GAMMA, W.NS)
    got = _host(plan.lpt3_displacement(_to_dev(dk, plan)))
    ref = lpt3.lpt3_displacement(dk, box)
    assert np.max(np.abs(ref)) > 0
    for a in range(3):
        assert np.max(np.abs(got[a] - ref[a])) <= TOL64 * np.max(np.abs(ref)), f"component {a}"
    plan.close()


@pytest.mark.parametrize("n", [64, 96])
def test_lpt3_fp32_matches_oracle(lib, n):
    box = 1000.0 * n / 512
    print(f"[lpt3] fp32 n={n}", flush=True)
    plan = _plan(lib, n, lib.PIN_FP32, box)
    dk = field.linear_field(400 + n, n, box, W.SIGMA8, W.GAMMA, W.NS)
    got = _host(plan.lpt3_displacement(_to_dev(dk, plan))).astype(np.float64)
    ref = lpt3.lpt3_displacement(dk, box)
    rms = metrics.rel_rms(got, ref)
    print(f"[lpt3] fp32 n={n}: rel_rms {rms:.3g}, rel_max {metrics.rel_max(got, ref):.3g}", flush=True)
    assert rms <= 1e-5
    assert metrics.rel_max(got, ref) <= 1e-4
    plan.close()


def test_lpt3_band_limited_field_fp64(lib):
    """A field with a few low modes only: no product aliases, the transverse part is large, and
    the result is the exact third-order displacement of that field (oracle pinned to the
    equations of motion on such fields)."""
    n, box = 32, 100.0
    rng = np.random.default_rng(21)
    fx, fy, fz = hessian.freq_grids(n)
    keep = (np.abs(fx) <= 2) & (np.abs(fy) <= 2) & (fz <= 2)
    dk = (rng.standard_normal(keep.shape) + 1j * rng.standard_normal(keep.shape)) * keep * n ** 3
    dk = np.fft.rfftn(np.fft.irfftn(dk, s=(n, n, n), axes=(0, 1, 2)), axes=(0, 1, 2))
    dk[0, 0, 0] = 0.0
    plan = _plan(lib, n, lib.PIN_FP64, box)
    got = _host(plan.lpt3_displacement(_to_dev(dk, plan)))
    ref = lpt3.lpt3_displacement(dk, box)
    assert np.max(np.abs(got - ref)) <= TOL64 * np.max(np.abs(ref))
    plan.close()


@pytest.mark.timeout(900)
def test_lpt3_c256_full_grid(lib):
    name = "c256_fp32"
    cfg = W.CONFIGS[name]
    n, box = cfg["n"], cfg["box"]
    print(f"[lpt3] oracle {name} (full grid)", flush=True)
    dk = field.linear_field(cfg["seed"], n, box, W.SIGMA8, W.GAMMA, W.NS)
    ref = lpt3.lpt3_displacement(dk, box)
    plan = _plan(lib, n, lib.PIN_FP32, box)
    got = _host(plan.lpt3_displacement(_to_dev(dk, plan))).astype(np.float64)
    rms = metrics.rel_rms(got, ref)
    print(f"[lpt3] {name}: rel_rms {rms:.3g}, rel_max {metrics.rel_max(got, ref):.3g}", flush=True)
    assert rms <= 1e-5 and metrics.rel_max(got, ref) <= 1e-4
    plan.close()


@pytest.mark.timeout(600)
def test_lpt3_c512_properties(lib):
    """The benchmark size in the benchmark's launch sequence (generate_field, then psi3): odd in
    the field bit for bit (every operation is symmetric under x -> -x), repeatable bit for bit,
    finite, and of the expected size relative to psi1 (|psi3| / |psi1| ~ (sigma of delta)^2)."""
    import torch

    name = "c512_fp32"
    cfg = W.CONFIGS[name]
    plan = lib.Plan(cfg["n"], cfg["box"], W.config_radii(cfg), sigma8=W.SIGMA8, gamma=W.GAMMA, ns=W.NS,
                    prec=lib.PIN_FP32)
    dk = plan.generate_field(cfg["seed"])
    a = plan.lpt3_displacement(dk)
    b = plan.lpt3_displacement(dk)
    assert bool(torch.equal(a, b))
    assert bool(torch.isfinite(a).all())
    c = plan.lpt3_displacement(-dk)
    assert bool(torch.equal(c, -a))
    del b, c
    p1, _ = plan.displacements(dk, want_psi2=False)
    r3 = float(a.double().pow(2).mean().sqrt())
    r1 = float(p1.double().pow(2).mean().sqrt())
    print(f"[lpt3] {name}: rms psi3 {r3:.4g}, rms psi1 {r1:.4g} Mpc/h", flush=True)
    assert 0.0 < r3 < r1
    plan.close()
