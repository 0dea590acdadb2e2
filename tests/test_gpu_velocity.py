"""v_max (velocity at the trajectory maximum) through the C ABI vs the FP64 oracle."""

import numpy as np
import pytest

from oracle import field, points, run
from paper_1305_1505_amd import workloads as W

pytestmark = pytest.mark.gpu


def _host(t):
    import torch

    torch.cuda.synchronize()
    return t.cpu().numpy()


def _to_dev(arr, plan):
    import torch

    return torch.from_numpy(np.ascontiguousarray(arr)).to(device="cuda", dtype=plan.cplx)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_c64_velocity_matches_oracle(lib, prec):
    """64^3 workload: F and R_max bitwise those of pin_collapse_times; v_max against the oracle
    at every point whose R_max agrees (float64 to 1e-11 of max |v|, float32 1e-5 relative RMS)."""
    cfg = W.CONFIGS["c64_fp64"]
    n, box, seed = cfg["n"], cfg["box"], cfg["seed"]
    radii = W.config_radii(cfg)
    p = lib.PIN_FP64 if prec == "fp64" else lib.PIN_FP32
    plan = lib.Plan(n, box, radii, sigma8=W.SIGMA8, gamma=W.GAMMA, ns=W.NS, prec=p)
    dk_ref = field.linear_field(seed, n, box, W.SIGMA8, W.GAMMA, W.NS)
    dk = _to_dev(dk_ref, plan)
    F, R, V = plan.collapse_times_v(dk)
    F0, R0 = plan.collapse_times(dk)
    assert np.array_equal(_host(F), _host(F0)) and np.array_equal(_host(R), _host(R0))
    f_ref, r_ref, v_ref = run.collapse_times_with_velocity(dk_ref, radii, box)
    r, v = _host(R), _host(V).astype(np.float64)
    same = r == r_ref
    assert np.mean(~same) <= 1e-4
    assert np.all(v[:, r == 255] == 0.0)
    d = (v - v_ref)[:, same]
    if prec == "fp64":
        assert np.max(np.abs(d)) <= 1e-11 * np.max(np.abs(v_ref))
    else:
        assert np.sqrt(np.sum(d ** 2) / np.sum(v_ref[:, same] ** 2)) <= 1e-5
    plan.close()


def test_velocity_range_splitting_is_exact(lib):
    import torch

    n, box = 32, 50.0
    radii = [8.0, 4.0, 2.0, 1.0, 0.75]
    plan = lib.Plan(n, box, radii, prec=lib.PIN_FP32)
    dk = plan.generate_field(11)
    F, R, V = plan.collapse_times_v(dk)
    F2, R2, V2 = torch.empty_like(F), torch.empty_like(R), torch.empty_like(V)
    plan.collapse_reset_v(F2, R2, V2)
    for r0, r1 in ((0, 2), (2, 3), (3, 5)):
        plan.collapse_times_range_v(dk, F2, R2, V2, r0, r1)
    torch.cuda.synchronize()
    assert torch.equal(F, F2) and torch.equal(R, R2) and torch.equal(V, V2)
    plan.close()


@pytest.mark.timeout(600)
def test_fullsize_velocity_at_points(lib):
    """512^3 float32, the benchmark field: v_max at sampled points against oracle.points."""
    import torch

    cfg = W.CONFIGS["c512_fp32"]
    n, box, seed = cfg["n"], cfg["box"], cfg["seed"]
    radii = W.config_radii(cfg)
    plan = lib.Plan(n, box, radii, sigma8=W.SIGMA8, gamma=W.GAMMA, ns=W.NS, prec=lib.PIN_FP32)
    dk = plan.generate_field(seed)
    F, R, V = plan.collapse_times_v(dk)
    pts = [(0, 0, 0), (n - 1, n - 1, n - 1), (n // 2, n // 2 - 1, n // 2 + 1), (17, 300, 451)]
    idx = torch.tensor(pts, device="cuda", dtype=torch.long)
    r = R[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()
    v = V[:, idx[:, 0], idx[:, 1], idx[:, 2]].double().cpu().numpy().T
    dk_ref = field.linear_field(seed, n, box, W.SIGMA8, W.GAMMA, W.NS)
    print("[velocity] oracle v_max at points", flush=True)
    fm, ri, vm, _ = points.collapse_times_with_velocity_at_points(dk_ref, pts, radii, box)
    tol = 2e-5 * max(np.max(np.abs(vm)), 1.0)
    for p in range(len(pts)):
        if r[p] == ri[p]:
            assert np.max(np.abs(v[p] - vm[p])) <= tol, f"point {pts[p]}"
    assert np.mean(r == ri) >= 0.75
    plan.close()
