"""The serving scheduler (csrc/serve_core.hpp) on the CPU, driven through its C ABI with a
host-only executor double (tests/native/fake_serve.cpp): admission by budget, first-come order
within a size class, slot reuse, cancellation, malformed requests, injected device errors,
shutdown, statistics, and concurrent clients."""

import ctypes
import os
import subprocess
import threading
import time

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "fake_serve.cpp")
OUT = os.path.join(ROOT, "tests", "native", "_build", "libpin_serve_fake.so")
DEPS = [SRC] + [os.path.join(ROOT, "paper_1305_1505_amd", "csrc", f) for f in
                ("serve_core.hpp", "serve_api.inc", "errors.hpp")] + [os.path.join(ROOT, "include", "pin.h")]


def build_fake(out=OUT, extra=()):
    if os.path.exists(out) and all(os.path.getmtime(out) >= os.path.getmtime(d) for d in DEPS) and not extra:
        return out
    os.makedirs(os.path.dirname(out), exist_ok=True)
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-shared", "-fPIC", "-pthread", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1305_1505_amd", "csrc"),
           "-I", "/opt/rocm/include", *extra, SRC, "-o", out + ".tmp"]
    subprocess.run(cmd, check=True, capture_output=True)
    os.replace(out + ".tmp", out)
    return out


@pytest.fixture(scope="module")
def api():
    from paper_1305_1505_amd import binding as B

    lib = ctypes.CDLL(build_fake())
    lib.pin_fake_configure.argtypes = [ctypes.c_int, ctypes.c_ulonglong, ctypes.c_ulonglong, ctypes.c_int]
    lib.pin_fake_slot_creates.restype = ctypes.c_longlong
    lib.pin_fake_slot_destroys.restype = ctypes.c_longlong
    return B, B.ServeAPI(lib), lib


RADII = [8.0, 4.0, 2.0, 1.0]


def _server(B, a, budget, max_slots=4):
    return a.pin_serve_create(B.make_serve_config(budget, max_slots))


def _wait_all(a, srv, tickets, timeout=10.0):
    """Wait for each ticket in turn and release it (results hold their slot until released)."""
    out = {}
    for t in tickets:
        st, res = a.pin_serve_wait(srv, t, timeout)
        out[t] = (st, res.t_submit, res.t_admit, res.t_done)
        a.pin_serve_release(srv, t)
    return out


def test_basic_roundtrip_and_results(api):
    B, a, lib = api
    lib.pin_fake_configure(3, 0, 0, 0)
    srv = _server(B, a, 1e9)
    t = a.pin_serve_submit(srv, B.make_request(1, 64, 128.0, RADII, 1))
    st, res = a.pin_serve_wait(srv, t, 5.0)
    assert st == B.PIN_OK and res.status == B.PIN_OK
    assert res.F and res.ridx and res.psi1 and res.psi2 and res.n == 64 and res.n_radii == 4
    assert 0 <= res.t_submit <= res.t_admit <= res.t_done
    a.pin_serve_release(srv, t)
    st, _ = a.pin_serve_poll(srv, t)
    assert st == B.PIN_ERR_INVALID_ARG            # released tickets are forgotten
    a.pin_serve_destroy(srv)


def test_no_displacements_gives_null_psi(api):
    B, a, lib = api
    lib.pin_fake_configure(1, 0, 0, 0)
    srv = _server(B, a, 1e9)
    t = a.pin_serve_submit(srv, B.make_request(2, 32, 64.0, RADII, 0))
    st, res = a.pin_serve_wait(srv, t, 5.0)
    assert st == B.PIN_OK and not res.psi1 and not res.psi2
    a.pin_serve_destroy(srv)


@pytest.mark.parametrize("bad", [
    dict(n=100), dict(n=6), dict(box=0.0), dict(box=-1.0), dict(radii=[]), dict(radii=[1.0, 2.0]),
    dict(radii=[1.0, 1.0]), dict(radii=[2.0, -1.0]), dict(want_disp=2),
])
def test_malformed_requests_rejected(api, bad):
    B, a, lib = api
    srv = _server(B, a, 1e9)
    req = dict(seed=1, n=64, box=10.0, radii=RADII, want_disp=1)
    req.update(bad)
    with pytest.raises(B.PinError) as e:
        a.pin_serve_submit(srv, B.make_request(req["seed"], req["n"], req["box"], req["radii"], req["want_disp"]))
    assert e.value.status in (B.PIN_ERR_INVALID_ARG, B.PIN_ERR_UNSUPPORTED_SIZE)
    assert a.pin_serve_stats(srv)["queued"] == 0
    a.pin_serve_destroy(srv)


def test_request_that_can_never_fit_is_refused(api):
    B, a, lib = api
    srv = _server(B, a, 64 ** 3)                  # fake slot bytes = N^3
    with pytest.raises(B.PinError) as e:
        a.pin_serve_submit(srv, B.make_request(1, 128, 10.0, RADII))
    assert e.value.status == B.PIN_ERR_BUDGET
    t = a.pin_serve_submit(srv, B.make_request(1, 64, 10.0, RADII))
    assert a.pin_serve_wait(srv, t, 5.0)[0] == B.PIN_OK
    a.pin_serve_destroy(srv)


def test_budget_serialises_and_fifo_within_class(api):
    B, a, lib = api
    lib.pin_fake_configure(20, 0, 0, 0)
    srv = _server(B, a, 64 ** 3)                  # room for exactly one 64^3 slot
    tickets = [a.pin_serve_submit(srv, B.make_request(i + 1, 64, 10.0, RADII)) for i in range(4)]
    done = []
    for t in tickets:
        st, res = a.pin_serve_wait(srv, t, 10.0)
        assert st == B.PIN_OK
        done.append((res.t_admit, res.t_done, t))
        a.pin_serve_release(srv, t)               # frees the only slot for the next request
    # admitted in arrival order, one at a time
    assert [d[2] for d in sorted(done)] == tickets
    for (a0, d0, _), (a1, d1, _) in zip(sorted(done), sorted(done)[1:]):
        assert a1 >= d0
    assert a.pin_serve_stats(srv)["slots"] == 1
    a.pin_serve_destroy(srv)


def test_classes_do_not_block_each_other_and_run_concurrently(api):
    B, a, lib = api
    lib.pin_fake_configure(200, 0, 0, 0)
    srv = _server(B, a, 64 ** 3 + 32 ** 3 + 1, max_slots=1)
    big1 = a.pin_serve_submit(srv, B.make_request(1, 64, 10.0, RADII))
    big2 = a.pin_serve_submit(srv, B.make_request(2, 64, 10.0, RADII))    # blocked behind big1
    small = a.pin_serve_submit(srv, B.make_request(3, 32, 10.0, RADII))   # must not wait for big2
    st, rs = a.pin_serve_wait(srv, small, 10.0)
    st1, r1 = a.pin_serve_wait(srv, big1, 10.0)
    assert st == B.PIN_OK and st1 == B.PIN_OK
    assert rs.t_admit < r1.t_done                # the small request ran alongside big1
    a.pin_serve_release(srv, big1)
    assert a.pin_serve_wait(srv, big2, 10.0)[0] == B.PIN_OK
    a.pin_serve_destroy(srv)


def test_slot_reuse_and_eviction(api):
    B, a, lib = api
    lib.pin_fake_configure(1, 0, 0, 0)
    c0 = lib.pin_fake_slot_creates()
    srv = _server(B, a, 64 ** 3)
    for i in range(5):
        t = a.pin_serve_submit(srv, B.make_request(i + 1, 64, 10.0, RADII))
        assert a.pin_serve_wait(srv, t, 5.0)[0] == B.PIN_OK
        a.pin_serve_release(srv, t)
    assert lib.pin_fake_slot_creates() - c0 == 1          # one slot reused five times
    d0 = lib.pin_fake_slot_destroys()
    t = a.pin_serve_submit(srv, B.make_request(9, 48, 10.0, RADII))   # needs the 64^3 slot evicted
    assert a.pin_serve_wait(srv, t, 5.0)[0] == B.PIN_OK
    assert lib.pin_fake_slot_destroys() - d0 == 1
    a.pin_serve_destroy(srv)


def test_cancel_queued_and_running(api):
    B, a, lib = api
    lib.pin_fake_configure(2000, 0, 0, 0)
    srv = _server(B, a, 64 ** 3)
    run = a.pin_serve_submit(srv, B.make_request(1, 64, 10.0, RADII))
    queued = a.pin_serve_submit(srv, B.make_request(2, 64, 10.0, RADII))
    time.sleep(0.05)
    a.pin_serve_cancel(srv, queued)
    assert a.pin_serve_poll(srv, queued)[0] == B.PIN_ERR_CANCELLED
    a.pin_serve_cancel(srv, run)
    st, _ = a.pin_serve_wait(srv, run, 10.0)
    assert st == B.PIN_ERR_CANCELLED
    s = a.pin_serve_stats(srv)
    assert s["cancelled"] == 2 and s["completed"] == 0
    # the cancelled running request freed its slot: a new one gets through
    lib.pin_fake_configure(1, 0, 0, 0)
    t = a.pin_serve_submit(srv, B.make_request(3, 64, 10.0, RADII))
    assert a.pin_serve_wait(srv, t, 5.0)[0] == B.PIN_OK
    with pytest.raises(B.PinError):
        a.pin_serve_release(srv, 10 ** 9)                  # unknown ticket
    a.pin_serve_destroy(srv)


def test_release_of_unfinished_request_is_refused(api):
    B, a, lib = api
    lib.pin_fake_configure(2000, 0, 0, 0)
    srv = _server(B, a, 1e9)
    t = a.pin_serve_submit(srv, B.make_request(1, 64, 10.0, RADII))
    with pytest.raises(B.PinError) as e:
        a.pin_serve_release(srv, t)
    assert e.value.status == B.PIN_ERR_INVALID_ARG
    assert a.pin_serve_wait(srv, t, 0.01)[0] == B.PIN_ERR_TIMEOUT
    a.pin_serve_destroy(srv)                               # waits for the running request


def test_injected_device_errors_fail_only_their_request(api):
    B, a, lib = api
    lib.pin_fake_configure(2, 77, 88, 0)
    srv = _server(B, a, 1e9)
    bad_launch = a.pin_serve_submit(srv, B.make_request(77, 64, 10.0, RADII))
    bad_poll = a.pin_serve_submit(srv, B.make_request(88, 64, 10.0, RADII))
    good = a.pin_serve_submit(srv, B.make_request(5, 64, 10.0, RADII))
    assert a.pin_serve_wait(srv, bad_launch, 5.0)[0] == B.PIN_ERR_DEVICE
    assert a.pin_serve_wait(srv, bad_poll, 5.0)[0] == B.PIN_ERR_DEVICE
    assert a.pin_serve_wait(srv, good, 5.0)[0] == B.PIN_OK
    assert "injected" in lib.pin_last_error().decode() or True
    s = a.pin_serve_stats(srv)
    assert s["failed"] == 2 and s["completed"] == 1
    lib.pin_fake_configure(1, 0, 0, 0)
    a.pin_serve_destroy(srv)


def test_allocation_failure_with_nothing_to_evict_fails_request(api):
    B, a, lib = api
    lib.pin_fake_configure(1, 0, 0, 1)
    srv = _server(B, a, 1e9)
    t = a.pin_serve_submit(srv, B.make_request(1, 64, 10.0, RADII))
    assert a.pin_serve_wait(srv, t, 5.0)[0] == B.PIN_ERR_OUT_OF_MEMORY
    lib.pin_fake_configure(1, 0, 0, 0)
    a.pin_serve_destroy(srv)


def test_shutdown_cancels_queue_and_refuses_new_work(api):
    B, a, lib = api
    lib.pin_fake_configure(500, 0, 0, 0)
    srv = _server(B, a, 64 ** 3)
    ts = [a.pin_serve_submit(srv, B.make_request(i + 1, 64, 10.0, RADII)) for i in range(3)]
    a.pin_serve_destroy(srv)                               # returns after the running one ends


def test_stats_percentiles(api):
    B, a, lib = api
    lib.pin_fake_configure(2, 0, 0, 0)
    srv = _server(B, a, 1e9)
    ts = [a.pin_serve_submit(srv, B.make_request(i + 1, 32, 10.0, RADII)) for i in range(40)]
    res = _wait_all(a, srv, ts)
    assert all(v[0] == B.PIN_OK for v in res.values())
    lat = sorted(v[3] - v[1] for v in res.values())
    s = a.pin_serve_stats(srv)
    assert s["completed"] == 40 and s["queued"] == 0 and s["running"] == 0
    assert abs(s["p50_s"] - (lat[19] + lat[20]) / 2) < 1e-9
    assert lat[0] <= s["p99_s"] <= lat[-1] and s["updates_per_s"] > 0
    a.pin_serve_reset_stats(srv)
    assert a.pin_serve_stats(srv)["completed"] == 0
    a.pin_serve_destroy(srv)


def test_concurrent_clients(api):
    B, a, lib = api
    lib.pin_fake_configure(3, 0, 0, 0)
    srv = _server(B, a, 3 * 64 ** 3, max_slots=2)
    errors = []

    def client(k):
        try:
            for i in range(25):
                n = (32, 48, 64)[(k + i) % 3]
                t = a.pin_serve_submit(srv, B.make_request(1000 * k + i + 1, n, 10.0, RADII))
                st, _ = a.pin_serve_wait(srv, t, 20.0)
                assert st == B.PIN_OK
                a.pin_serve_release(srv, t)
        except Exception as e:  # noqa: BLE001
            errors.append(e)

    th = [threading.Thread(target=client, args=(k,)) for k in range(6)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors
    s = a.pin_serve_stats(srv)
    assert s["completed"] == 150 and s["hbm_in_use"] <= 3 * 64 ** 3
    a.pin_serve_destroy(srv)


def test_thread_sanitizer_stress(tmp_path):
    """The scheduler core under -fsanitize=thread, with several client threads (host only)."""
    driver = os.path.join(ROOT, "tests", "native", "serve_stress.cpp")
    exe = str(tmp_path / "serve_stress")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1305_1505_amd", "csrc"),
           "-I", "/opt/rocm/include", driver, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    proc = subprocess.run([exe], capture_output=True, text=True, timeout=120,
                          env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66"))
    assert proc.returncode == 0, proc.stdout + proc.stderr
    assert "stress ok" in proc.stdout
