"""Serving on the GPU: every served result is bitwise identical to the same request computed
alone through the plain entry points, whatever else is in flight; budget-limited admission;
statistics."""

import numpy as np
import pytest

from paper_1305_1505_amd import workloads as W

pytestmark = pytest.mark.gpu


def _plain(lib, req):
    """The same request through a plan and the plain calls (field, collapse times, displacements)."""
    import torch

    plan = lib.Plan(req["n"], req["box"], req["radii"], prec=lib.PIN_FP32)
    dk = plan.generate_field(req["seed"])
    F, R = plan.collapse_times(dk)
    p1, p2 = plan.displacements(dk) if req["disp"] else (None, None)
    torch.cuda.synchronize()
    out = [F.cpu().numpy(), R.cpu().numpy()]
    if req["disp"]:
        out += [p1.cpu().numpy(), p2.cpu().numpy()]
    plan.close()
    return out


def _served(lib, res, req):
    """Copy a served result (server-owned device pointers) to host arrays."""
    import ctypes

    n = req["n"]
    vol = n ** 3

    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip.hipMemcpy.restype = ctypes.c_int

    def grab(ptr, count, dtype):
        host = np.empty(count, dtype=dtype)
        assert hip.hipMemcpy(host.ctypes.data, ptr, host.nbytes, 2) == 0   # device -> host
        return host

    out = [grab(res.F, vol, np.float32).reshape(n, n, n), grab(res.ridx, vol, np.uint8).reshape(n, n, n)]
    if req["disp"]:
        out += [grab(res.psi1, 3 * vol, np.float32).reshape(3, n, n, n),
                grab(res.psi2, 3 * vol, np.float32).reshape(3, n, n, n)]
    return out


REQS = [
    dict(seed=11, n=64, box=128.0, radii=W.radii_cells(12, 20.0, 0.75), disp=1),
    dict(seed=12, n=96, box=192.0, radii=W.radii_cells(9, 30.0, 0.75), disp=1),
    dict(seed=13, n=128, box=256.0, radii=W.radii_cells(14, 60.0, 0.75), disp=0),
    dict(seed=14, n=48, box=96.0, radii=W.radii_cells(5, 10.0, 0.75), disp=1),
    dict(seed=11, n=64, box=128.0, radii=W.radii_cells(12, 20.0, 0.75), disp=1),   # = REQS[0]
    dict(seed=16, n=64, box=100.0, radii=W.radii_cells(7, 20.0, 1.0), disp=0),
    # serving-trace sizes with radix-3 factorisations
    dict(seed=17, n=192, box=384.0, radii=W.radii_cells(10, 60.0, 0.75), disp=1),
    dict(seed=18, n=384, box=768.0, radii=W.radii_cells(6, 60.0, 0.75), disp=0),
]


def test_served_results_bitwise_equal_plain_path_in_a_mix(lib):
    import torch

    B = lib
    cfg = B.make_serve_config(40e9, max_slots_per_class=2)
    srv = B.pin_serve_create(cfg)
    try:
        tickets = [B.pin_serve_submit(srv, B.make_request(r["seed"], r["n"], r["box"], r["radii"], r["disp"]))
                   for r in REQS]
        served = []
        for t, r in zip(tickets, REQS):
            st, res = B.pin_serve_wait(srv, t, 120.0)
            assert st == B.PIN_OK, B.pin_last_error()
            served.append(_served(lib, res, r))
            B.pin_serve_release(srv, t)
        stats = B.pin_serve_stats(srv)
        assert stats["completed"] == len(REQS) and stats["failed"] == 0
        # the same request again, now alone on a warm server (graph replay)
        t = B.pin_serve_submit(srv, B.make_request(REQS[0]["seed"], REQS[0]["n"], REQS[0]["box"],
                                                    REQS[0]["radii"], 1))
        st, res = B.pin_serve_wait(srv, t, 120.0)
        assert st == B.PIN_OK
        alone = _served(lib, res, REQS[0])
        B.pin_serve_release(srv, t)
    finally:
        B.pin_serve_destroy(srv)
    torch.cuda.synchronize()
    for r, got in zip(REQS, served):
        ref = _plain(lib, r)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), f"request seed {r['seed']} differs from the plain path"
    for a, b in zip(alone, served[0]):
        assert np.array_equal(a, b)
    for a, b in zip(served[4], served[0]):      # same request submitted twice in the mix
        assert np.array_equal(a, b)


def test_one_slot_many_boxes(lib):
    """One slot of one size class serves requests of eleven different boxes in turn, the first
    again at the end: the field's mode amplitudes follow each request's box (the plan keeps a
    table per box, at most eight, the oldest dropped), so every result equals the plain path's."""
    import torch

    B = lib
    boxes = [16.0 + 4.0 * i for i in range(11)] + [16.0]
    reqs = [dict(seed=40 + i, n=16, box=bx, radii=W.radii_cells(3, 4.0, 0.75), disp=1) for i, bx in enumerate(boxes)]
    cfg = B.make_serve_config(40e9, max_slots_per_class=1)
    srv = B.pin_serve_create(cfg)
    served = []
    try:
        for r in reqs:
            t = B.pin_serve_submit(srv, B.make_request(r["seed"], r["n"], r["box"], r["radii"], r["disp"]))
            st, res = B.pin_serve_wait(srv, t, 120.0)
            assert st == B.PIN_OK, B.pin_last_error()
            served.append(_served(lib, res, r))
            B.pin_serve_release(srv, t)
    finally:
        B.pin_serve_destroy(srv)
    torch.cuda.synchronize()
    for r, got in zip(reqs, served):
        for a, b in zip(got, _plain(lib, r)):
            assert np.array_equal(a, b), f"box {r['box']} differs from the plain path"


def test_small_budget_serialises_and_completes(lib):
    B = lib
    one = B.pin_serve_slot_bytes(B.make_serve_config(1e12), 64)
    srv = B.pin_serve_create(B.make_serve_config(1.5 * one, max_slots_per_class=4))
    try:
        ts = [B.pin_serve_submit(srv, B.make_request(100 + i, 64, 64.0, W.radii_cells(4, 8.0, 1.0), 0))
              for i in range(5)]
        admits = []
        for t in ts:
            st, res = B.pin_serve_wait(srv, t, 60.0)
            assert st == B.PIN_OK
            admits.append((res.t_admit, res.t_done))
            B.pin_serve_release(srv, t)
        s = B.pin_serve_stats(srv)
        assert s["slots"] == 1 and s["hbm_in_use"] <= 1.5 * one
        admits.sort()
        for (a0, d0), (a1, d1) in zip(admits, admits[1:]):
            assert a1 >= d0
        with pytest.raises(B.PinError) as e:
            B.pin_serve_submit(srv, B.make_request(1, 128, 64.0, [2.0, 1.0], 0))
        assert e.value.status == B.PIN_ERR_BUDGET
    finally:
        B.pin_serve_destroy(srv)
