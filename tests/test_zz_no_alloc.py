"""Allocation-free collapse times (pin_collapse_times_noalloc) against pin_collapse_times on a
plan, through the C ABI: same field, same radii, two calls in a row with the second on a
smaller grid (the shared static workspace keeps the first call's contents), in both
precisions; sizes beyond the static workspace are refused before anything is written."""

import numpy as np
import pytest

from paper_1305_1505_amd import workloads as W

pytestmark = pytest.mark.gpu


def _case(lib, n, box, n_radii, prec, seed):
    import torch

    radii = W.radii_cells(n_radii, 20.0, 0.75)
    plan = lib.Plan(n, box, radii, prec=prec)
    dk = plan.generate_field(seed)
    F_ref, R_ref = plan.collapse_times(dk)
    # outputs start with values the call must overwrite everywhere
    F = torch.full_like(F_ref, 7.0)
    R = torch.full_like(R_ref, 3)
    desc = lib.make_desc(n, box, radii, prec=prec)
    lib.pin_collapse_times_noalloc(desc, dk.data_ptr(), F.data_ptr(), R.data_ptr(),
                                   torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    out = (F.cpu().numpy().astype(np.float64), R.cpu().numpy(), F_ref.cpu().numpy().astype(np.float64),
           R_ref.cpu().numpy())
    plan.close()
    return out


@pytest.mark.parametrize("prec,sizes", [("fp32", [(128, 256.0, 40, 103), (64, 100.0, 16, 101)]),
                                        ("fp64", [(96, 150.0, 24, 104), (32, 50.0, 6, 7)])])
def test_noalloc_matches_plan_path(lib, prec, sizes):
    p = lib.PIN_FP64 if prec == "fp64" else lib.PIN_FP32
    for n, box, n_radii, seed in sizes:
        print(f"noalloc {prec} N={n} radii={n_radii} seed={seed}", flush=True)
        F, R, F_ref, R_ref = _case(lib, n, box, n_radii, p, seed)
        # same kernels on the same inputs; the twiddles are the plan's own values and the window
        # rows are float64 exp on the device instead of the host's, so within rounding
        rel_rms = np.sqrt(np.sum((F - F_ref) ** 2) / np.sum(F_ref ** 2))
        assert rel_rms <= (1e-13 if prec == "fp64" else 1e-6), rel_rms
        assert np.mean(R != R_ref) <= 1e-4
        assert np.all(np.isfinite(F)) and np.all((R == 255) == (F == 0))


def test_noalloc_refuses_sizes_beyond_its_workspace(lib):
    import torch

    for n, prec in ((192, lib.PIN_FP32), (128, lib.PIN_FP64)):
        real = torch.float64 if prec == lib.PIN_FP64 else torch.float32
        cplx = torch.complex128 if prec == lib.PIN_FP64 else torch.complex64
        dk = torch.zeros((n, n, n // 2 + 1), dtype=cplx, device="cuda")
        F = torch.full((n, n, n), 7.0, dtype=real, device="cuda")
        R = torch.full((n, n, n), 3, dtype=torch.uint8, device="cuda")
        desc = lib.make_desc(n, 100.0, [2.0, 1.0], prec=prec)
        with pytest.raises(lib.PinError) as e:
            lib.pin_collapse_times_noalloc(desc, dk.data_ptr(), F.data_ptr(), R.data_ptr(), 0)
        assert e.value.status == lib.PIN_ERR_UNSUPPORTED_SIZE
        torch.cuda.synchronize()
        assert torch.all(F == 7.0).item() and torch.all(R == 3).item()


def test_noalloc_replays_under_graph_capture(lib):
    """The call captured into a HIP graph (after one eager call on the device, which looks up the
    workspace's address) replays to the eager result bit for bit, three times, with an eager call
    on another grid size rewriting the shared workspace before each replay."""
    import torch

    n, box, radii = 64, 100.0, W.radii_cells(16, 20.0, 0.75)
    plan = lib.Plan(n, box, radii, prec=lib.PIN_FP32)
    dk = plan.generate_field(101)
    desc = lib.make_desc(n, box, radii, prec=lib.PIN_FP32)
    F = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
    R = torch.empty((n, n, n), dtype=torch.uint8, device="cuda")
    lib.pin_collapse_times_noalloc(desc, dk.data_ptr(), F.data_ptr(), R.data_ptr(),
                                   torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    F_eager, R_eager = F.clone(), R.clone()
    other = lib.Plan(32, 50.0, W.radii_cells(6, 8.0, 0.75), prec=lib.PIN_FP32)
    dk2 = other.generate_field(7)
    desc2 = lib.make_desc(32, 50.0, W.radii_cells(6, 8.0, 0.75), prec=lib.PIN_FP32)
    F2 = torch.empty((32, 32, 32), dtype=torch.float32, device="cuda")
    R2 = torch.empty((32, 32, 32), dtype=torch.uint8, device="cuda")
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=s, capture_error_mode="thread_local"):
        lib.pin_collapse_times_noalloc(desc, dk.data_ptr(), F.data_ptr(), R.data_ptr(),
                                       torch.cuda.current_stream().cuda_stream)
    for rep in range(3):
        F.fill_(7.0)
        R.fill_(3)
        lib.pin_collapse_times_noalloc(desc2, dk2.data_ptr(), F2.data_ptr(), R2.data_ptr(),
                                       torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(F, F_eager) and torch.equal(R, R_eager), f"replay {rep}"
    del g
    other.close()
    plan.close()
