"""Benchmark: grid-point x radius collapse updates per second on one MI355X.

One step is one pass of the whole path over one realisation: the seeded Gaussian field, the
collapse times over every radius (per radius: window x Hessian multiply, the three FFT passes,
the per-point eigenvalue / collapse / running maximum), and the closing ZA and 2LPT
displacements.  value = N^3 * n_radii / seconds per step.

Workload (default): 512^3 grid, 1000 Mpc/h box, 40 Gaussian radii log-spaced 60 -> 0.75 cells,
BBKS spectrum (Gamma 0.21, n 1, sigma_8 0.8), complex64 FFTs.  Data are synthetic (seeded).

Prints ONE JSON line.  Extra fields: the dominant kernel's roofline (algorithmic bytes per launch
over its HIP-event-timed average duration; HBM traffic and VALU issue time per launch from the
committed rocprofv3 counter summaries while the kernel sources match them), the collapse-only
rate, the float64 rate of the same workload, and the FP64 CPU oracle timed on a bounded sample
(cpu_baseline).
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(cls, n, real_bytes):
    """Bytes a launch of kernel class `cls` must move at grid size n: its input and output workspace
    slots (a slot is one N x N x N/2 complex array) and, for the collapse pass, F and the radius index."""
    cb = 2 * real_bytes
    slot = n * n * (n // 2) * cb          # one workspace slot (kz = N/2 plane not stored)
    vol = n ** 3
    return {
        "xpass_hessian": slot + 3 * slot,                 # spectrum in (kz < N/2), 3 slots out
        "ypass_hessian": 3 * slot + 6 * slot,             # 3 in, 6 out
        "zpass_collapse": 6 * slot + vol * (2 * real_bytes + 1),   # 6 in; F read + F, ridx written
    }.get(cls)


def measured_traffic(cls, n, prec):
    """HBM bytes per launch (fetch + write) of kernel `cls` from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources at this workload; else None."""
    from paper_1305_1505_amd import binding as B
    from paper_1305_1505_amd import profile_summary

    path = os.path.join(ROOT, "profiles", "traffic_c512_fp32.json")
    if n != 512 or prec != B.PIN_FP32 or not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_sha256") != profile_summary.kernel_source_hash() or cls not in t["kernels"]:
        return None
    k = t["kernels"][cls]
    return {"bytes": k["fetch_bytes"] + k["write_bytes"], "fetch_bytes": k["fetch_bytes"],
            "write_bytes": k["write_bytes"], "source": "profiles/traffic_c512_fp32.json"}


def measured_issue(cls, n, prec):
    """Time the VALU instructions of kernel `cls` take to issue (ns per launch), from the committed
    SQ counter summary, if it was taken on the current kernel sources at this workload; else None."""
    from paper_1305_1505_amd import binding as B
    from paper_1305_1505_amd import profile_summary

    path = os.path.join(ROOT, "profiles", "issue_c512_fp32.json")
    if n != 512 or prec != B.PIN_FP32 or not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_sha256") != profile_summary.kernel_source_hash() or cls not in t["kernels"]:
        return None
    return t["kernels"][cls]["valu_issue_ns"]


def cpu_baseline(sample_n=256, workers=None):
    """The FP64 oracle, as it stands, timed on the host cores on a bounded sample of the workload.

    Sample: a sample_n^3 grid at the workload's cell size (box scaled), the field, the first and
    the last of its radii (their deformation tensors in two threads; the per-point collapse step
    over chunks of points in a thread pool -- NumPy releases the GIL in its FFTs, LAPACK calls and
    array arithmetic), and the ZA and 2LPT displacements (two threads).  The time of the full step
    is extrapolated linearly in the radius count: field + n_radii x (time per radius) +
    displacements.  cores = the threads busy on average (process CPU time / wall time)."""
    import concurrent.futures as cf

    import numpy as np

    from oracle import collapse, field, hessian, run
    from paper_1305_1505_amd import workloads as W

    cfg = W.CONFIGS["c512_fp32"]
    box = cfg["box"] * sample_n / cfg["n"]
    radii = W.config_radii(cfg)
    sample_radii = [radii[0], radii[-1]]
    workers = workers or min(16, os.cpu_count() or 1)
    n3 = sample_n ** 3
    chunk = -(-n3 // (4 * workers))
    with cf.ThreadPoolExecutor(workers) as pool:
        t0, c0 = time.perf_counter(), time.process_time()
        dk = field.linear_field(cfg["seed"], sample_n, box, W.SIGMA8, W.GAMMA, W.NS)
        t1 = time.perf_counter()
        tens = list(pool.map(lambda r: [c.ravel() for c in hessian.deformation_tensor(dk, r)], sample_radii))
        fmax = np.zeros(n3)
        ridx = np.full(n3, run.NEVER, dtype=np.uint8)
        for k, t6 in enumerate(tens):
            f = np.concatenate(list(pool.map(
                lambda s: collapse.inverse_collapse_time([c[s:s + chunk] for c in t6]), range(0, n3, chunk))))
            up = f > fmax
            fmax = np.where(up, f, fmax)
            ridx = np.where(up, np.uint8(k), ridx)
        del tens
        t2 = time.perf_counter()
        list(pool.map(lambda fn: fn(dk, box), (run.za_displacement, run.lpt2_displacement)))
        t3 = time.perf_counter()
        cpu = time.process_time() - c0
    per_radius = (t2 - t1) / len(sample_radii)
    total = (t1 - t0) + len(radii) * per_radius + (t3 - t2)
    return {"value": n3 * len(radii) / total, "unit": "updates/s", "cores": round(cpu / (t3 - t0), 1),
            "kind": "oracle", "measured_s": round(t3 - t0, 2), "extrapolated_step_s": round(total, 1),
            "per_radius_s": round(per_radius, 2), "field_s": round(t1 - t0, 2), "displacements_s": round(t3 - t2, 2),
            "sample": f"{sample_n}^3 grid at the workload's cell size ({box:g} Mpc/h): field, the first and last "
                      f"of its {len(radii)} radii (deformation tensors, collapse, running maximum), ZA + 2LPT; "
                      f"step time extrapolated linearly to {len(radii)} radii; float64 NumPy/SciPy oracle, "
                      f"{workers} threads, {os.cpu_count()} host cores visible ({_cpu_model()})"}


def cpu_baseline_single(sample_n=64):
    """The oracle on one thread on a small grid at the workload's cell size, every radius (the
    figure reported before the threaded sample; kept as a secondary field)."""
    from oracle import field, run
    from paper_1305_1505_amd import workloads as W

    cfg = W.CONFIGS["c512_fp32"]
    box = cfg["box"] * sample_n / cfg["n"]
    radii = W.config_radii(cfg)
    t0 = time.perf_counter()
    dk = field.linear_field(cfg["seed"], sample_n, box, W.SIGMA8, W.GAMMA, W.NS)
    run.collapse_times(dk, radii)
    run.displacements(dk, box)
    dt = time.perf_counter() - t0
    return {"value": sample_n ** 3 * len(radii) / dt, "unit": "updates/s", "cores": 1, "seconds": round(dt, 2),
            "sample": f"{sample_n}^3 grid ({box:g} Mpc/h), all {len(radii)} radii, field + collapse + ZA/2LPT"}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def serve_bench(B, W, full=False):
    """Serving workload: Poisson arrivals (4/s) of mixed-size realizations against a 200 GB budget.

    Phases: warm-up (creates slots and graphs), the measured list replayed at its arrival times
    (p50/p99 latency), the same list submitted at once (served throughput), and the same list run
    one request after another through the plain entry points on one plan per grid size.
    """
    import threading

    import torch

    trace = W.serve_trace(count=None if full else 10 + 60)
    warm = W.SERVE["warmup"] if full else 10
    cfg = B.make_serve_config(W.SERVE["hbm_budget"], max_slots_per_class=4)
    srv = B.pin_serve_create(cfg)

    def run(reqs, paced):
        outstanding, lock, stop = [], threading.Lock(), threading.Event()
        failures = []

        def collector():
            while not stop.is_set() or outstanding:
                with lock:
                    cur = list(outstanding)
                for t in cur:
                    st, _ = B.pin_serve_poll(srv, t)
                    if st == B.PIN_ERR_NOT_READY:
                        continue
                    if st != B.PIN_OK:
                        failures.append((t, st))
                    B.pin_serve_release(srv, t)
                    with lock:
                        outstanding.remove(t)
                time.sleep(0.0005)

        th = threading.Thread(target=collector)
        th.start()
        t0 = time.perf_counter()
        base = reqs[0]["t"]
        for r in reqs:
            if paced:
                delay = (r["t"] - base) - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(delay)
            t = B.pin_serve_submit(srv, B.make_request(r["seed"], r["n"], r["box"], r["radii"], 1))
            with lock:
                outstanding.append(t)
        stop.set()
        th.join()
        if failures:
            raise RuntimeError(f"served requests failed: {failures[:5]}")
        return time.perf_counter() - t0

    run(trace[:warm], paced=True)
    measured = trace[warm:]
    print(f"[bench] serving: {warm} warm-up requests done; {len(measured)} paced at "
          f"{W.SERVE['rate_per_s']:g}/s", file=sys.stderr, flush=True)
    updates = sum(r["n"] ** 3 * len(r["radii"]) for r in measured)
    B.pin_serve_reset_stats(srv)
    wall_paced = run(measured, paced=True)
    paced = B.pin_serve_stats(srv)
    print(f"[bench] serving: paced trace done in {wall_paced:.1f} s; saturated replay", file=sys.stderr, flush=True)
    B.pin_serve_reset_stats(srv)
    wall_sat = run(measured, paced=False)
    sat = B.pin_serve_stats(srv)
    B.pin_serve_destroy(srv)
    torch.cuda.synchronize()

    # plain path: the same list, one request after another, one plan per grid size
    plans = {}
    stream = torch.cuda.current_stream().cuda_stream
    maxr = W.SERVE["n_radii"][1]
    for n in sorted({r["n"] for r in measured}):
        pl = B.Plan(n, 2.0 * n, W.radii_cells(maxr, W.SERVE["r_max"], W.SERVE["r_min"]), prec=B.PIN_FP32)
        bufs = (pl.empty_spectrum(), torch.empty((n, n, n), dtype=torch.float32, device="cuda"),
                torch.empty((n, n, n), dtype=torch.uint8, device="cuda"),
                torch.empty((3, n, n, n), dtype=torch.float32, device="cuda"),
                torch.empty((3, n, n, n), dtype=torch.float32, device="cuda"))
        plans[n] = (pl, bufs)

    def plain_one(r):
        pl, (dk, F, R, p1, p2) = plans[r["n"]]
        assert r["box"] == 2.0 * r["n"]            # the trace's box; the plan was made with it
        B.pin_plan_set_radii(pl.handle, r["radii"], stream)
        B.pin_generate_field(pl.handle, r["seed"], dk.data_ptr(), stream)
        B.pin_collapse_times(pl.handle, dk.data_ptr(), F.data_ptr(), R.data_ptr(), stream)
        B.pin_displacements(pl.handle, dk.data_ptr(), p1.data_ptr(), p2.data_ptr(), stream)

    for r in measured[:5]:
        plain_one(r)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in measured:
        plain_one(r)
    torch.cuda.synchronize()
    wall_plain = time.perf_counter() - t0
    for pl, bufs in plans.values():
        pl.close()
    del plans
    torch.cuda.empty_cache()
    served_rate = updates / wall_sat
    plain_rate = updates / wall_plain
    return {
        "requests": len(measured), "warmup": warm, "latency_samples": int(paced["completed"]),
        "rate_per_s": W.SERVE["rate_per_s"],
        "sizes": list(W.SERVE["sizes"]), "budget_bytes": W.SERVE["hbm_budget"],
        "p50_latency_s": round(paced["p50_s"], 4), "p99_latency_s": round(paced["p99_s"], 4),
        "mean_latency_s": round(paced["mean_s"], 4), "paced_wall_s": round(wall_paced, 2),
        "served_updates_per_s_saturated": served_rate, "plain_updates_per_s": plain_rate,
        "served_over_plain": round(served_rate / plain_rate, 3),
        "saturated_p99_latency_s": round(sat["p99_s"], 4),
        "note": "plain = the same requests one after another through pin_* on one plan per grid size",
    }


def kernel_times(B, plan, fn, repeats):
    """{class name: total_ms, launches, avg_ms} over `repeats` calls of fn with per-launch events."""
    import torch

    B.pin_plan_set_timing(plan.handle, True)
    for _ in range(repeats):
        fn()
    torch.cuda.synchronize()
    out = {}
    for c in range(B.pin_kernel_class_count()):
        ms, cnt = B.pin_plan_kernel_time(plan.handle, c)
        if cnt:
            out[B.pin_kernel_class_name(c)] = {"total_ms": ms, "launches": cnt, "avg_ms": ms / cnt}
    B.pin_plan_set_timing(plan.handle, False)
    return out


def config_leg(B, W, name):
    """Collapse times alone on another workload (collapse_leg)."""
    cfg = W.CONFIGS[name]
    prec = B.PIN_FP64 if cfg["prec"] == "fp64" else B.PIN_FP32
    radii = W.config_radii(cfg)
    out = collapse_leg(B, W, cfg["n"], cfg["box"], radii, prec, cfg["seed"])
    return {"workload": f"{cfg['n']}^3 grid, {cfg['box']:g} Mpc/h, {len(radii)} radii {cfg['r_max']:g}->{cfg['r_min']:g} "
                        f"cells, collapse times only", "precision": cfg["prec"], **out}


def collapse_leg(B, W, n, box, radii, prec, seed):
    """Collapse times alone: median of 5 after 2 warm-ups (HIP events on the plan's stream), then
    one call with per-launch events for the three passes' durations and their algorithmic GB/s."""
    import torch

    plan = B.Plan(n, box, radii, W.SIGMA8, W.GAMMA, W.NS, prec)
    real_bytes = 8 if prec == B.PIN_FP64 else 4
    dk = plan.generate_field(seed)
    F = torch.empty((n, n, n), dtype=plan.real, device="cuda")
    R = torch.empty((n, n, n), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def collapse():
        B.pin_collapse_times(plan.handle, dk.data_ptr(), F.data_ptr(), R.data_ptr(), stream)

    for _ in range(2):
        collapse()
    runs = []
    for _ in range(5):
        ev0.record()
        collapse()
        ev1.record()
        torch.cuda.synchronize()
        runs.append(ev0.elapsed_time(ev1))
    ms = sorted(runs)[2]
    kt = kernel_times(B, plan, collapse, 1)
    passes = {}
    for k in ("xpass_hessian", "ypass_hessian", "zpass_collapse"):
        by = algorithmic_bytes(k, n, real_bytes)
        gbs = by / (kt[k]["avg_ms"] * 1e-3) / 1e9
        passes[k] = {"avg_ms": round(kt[k]["avg_ms"], 4), "bytes_per_launch": by, "GB/s": round(gbs, 1),
                     "frac": round(gbs / HBM_PEAK_GBS, 4)}
    del dk, F, R
    plan.close()
    torch.cuda.empty_cache()
    return {"collapse_ms": round(ms, 2), "updates_per_s": n ** 3 * len(radii) / (ms * 1e-3),
            "runs_ms": [round(x, 2) for x in runs], "passes": passes}


def size_sweep(B, W):
    """Collapse times alone at every supported grid size from 64^3, float32 and float64 plans:
    16 radii from min(60, N/8) to 0.75 cells, 2 Mpc/h cells; one JSON line."""
    import torch

    torch.cuda.set_device(0)
    rows = []
    for prec, name in ((B.PIN_FP32, "fp32"), (B.PIN_FP64, "fp64")):
        for n in [m for m in range(64, 1025) if B.pin_size_supported(m)]:
            radii = W.radii_cells(16, min(60.0, n / 8.0), 0.75)
            r = collapse_leg(B, W, n, 2.0 * n, radii, prec, 11)
            rows.append({"n": n, "precision": name, "radii": len(radii), **r})
            print(f"[bench] sweep {name} N={n}: {r['collapse_ms']} ms, {r['updates_per_s']:.3e} updates/s",
                  file=sys.stderr, flush=True)
    print(json.dumps({"metric": "collapse-only grid-point x radius updates/s by grid size", "unit": "updates/s",
                      "higher_is_better": True, "n_gpus": 1, "data": "synthetic (seeded BBKS Gaussian field)",
                      "sweep": rows}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c512_fp32")
    ap.add_argument("--no-fp64", action="store_true", help="skip the float64 comparison leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--size-sweep", action="store_true",
                    help="only the collapse-only sweep over grid sizes (its own JSON line)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-quick", action="store_true",
                    help="short serving trace (10 + 60 requests) instead of the full 20 + 300")
    ap.add_argument("--no-configs", action="store_true", help="skip the 256^3 and 768^3 collapse legs")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run three plain 1 GiB device copies (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (a realization would shard by "
              "radius with one max-merge of the running state)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1305_1505_amd import binding as B
    from paper_1305_1505_amd import workloads as W

    torch.cuda.set_device(0)
    if args.size_sweep:
        size_sweep(B, W)
        return
    cfg = W.CONFIGS[args.config]
    n, box, seed = cfg["n"], cfg["box"], cfg["seed"]
    radii = W.config_radii(cfg)
    prec = B.PIN_FP64 if cfg["prec"] == "fp64" else B.PIN_FP32
    plan = B.Plan(n, box, radii, W.SIGMA8, W.GAMMA, W.NS, prec)
    real_bytes = 8 if prec == B.PIN_FP64 else 4
    dk = plan.empty_spectrum()
    F = torch.empty((n, n, n), dtype=plan.real, device="cuda")
    R = torch.empty((n, n, n), dtype=torch.uint8, device="cuda")
    p1 = torch.empty((3, n, n, n), dtype=plan.real, device="cuda")
    p2 = torch.empty((3, n, n, n), dtype=plan.real, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream

    def step():
        B.pin_generate_field(plan.handle, seed, dk.data_ptr(), stream)
        B.pin_collapse_times(plan.handle, dk.data_ptr(), F.data_ptr(), R.data_ptr(), stream)
        B.pin_displacements(plan.handle, dk.data_ptr(), p1.data_ptr(), p2.data_ptr(), stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"[bench] warmup done: {args.config} N={n} radii={len(radii)}", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1000.0 * elapsed / args.steps
    updates = n ** 3 * len(radii)
    value = updates / (elapsed / args.steps)
    print(f"[bench] timed {args.steps} steps: {ms_per_step:.2f} ms/step", file=sys.stderr, flush=True)

    # per-kernel durations: HIP events around every launch, on the stream the kernels run on, in
    # steps of their own after the timed region (the events stay out of ms_per_step)
    kernels = kernel_times(B, plan, step, max(1, min(args.steps, 3)))

    # the dominant kernel of the path: largest summed time among the three per-radius passes
    dom = max(("xpass_hessian", "ypass_hessian", "zpass_collapse"), key=lambda k: kernels[k]["total_ms"])
    dom_bytes = algorithmic_bytes(dom, n, real_bytes)
    achieved = dom_bytes / (kernels[dom]["avg_ms"] * 1e-3) / 1e9
    measured = measured_traffic(dom, n, prec)
    # priced against HBM (its bytes are the pass's floor); the z pass is held back by its per-point
    # collapse arithmetic (VALU issue), the x and y passes by their memory pattern
    roofline = {"bound": "hbm", "kernel": dom, "limiter": "valu" if dom == "zpass_collapse" else "hbm",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": round(measured["bytes"]) if measured else None,
                "traffic_detail": measured, "bytes_per_launch": dom_bytes}
    # the VALU side: the time the kernel's VALU instructions take to issue (committed SQ counters,
    # one wave64 instruction per 4 cycles per SIMD at 2.4 GHz) over its measured launch time
    issue_ns = measured_issue(dom, n, prec)
    roofline["valu_issue_frac"] = round(issue_ns / (kernels[dom]["avg_ms"] * 1e6), 4) if issue_ns else None
    per_kernel = {k: {"avg_ms": round(v["avg_ms"], 4), "launches": v["launches"],
                      "GB/s": (round(algorithmic_bytes(k, n, real_bytes) / (v["avg_ms"] * 1e-3) / 1e9, 1)
                               if algorithmic_bytes(k, n, real_bytes) else None)}
                  for k, v in kernels.items()}

    # the path's parts on their own (HIP events on the plan's stream, which is torch's current
    # stream here): collapse times as the median of 5 runs after 2 warm-ups, the field and the
    # displacements once each
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        ev0.record()
        fn()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1)

    def collapse():
        B.pin_collapse_times(plan.handle, dk.data_ptr(), F.data_ptr(), R.data_ptr(), stream)

    for _ in range(2):
        collapse()
    runs = sorted(timed(collapse) for _ in range(5))
    collapse_ms = runs[2]
    field_ms = timed(lambda: B.pin_generate_field(plan.handle, seed, dk.data_ptr(), stream))
    # collapse times with the velocity at the trajectory maximum (v_max), after one warm-up
    vmax = torch.empty((3, n, n, n), dtype=plan.real, device="cuda")

    def collapse_v():
        B.pin_collapse_times_v(plan.handle, dk.data_ptr(), F.data_ptr(), R.data_ptr(), vmax.data_ptr(), stream)

    collapse_v()
    vel_ms = timed(collapse_v)
    # fragmentation at z = 0 (f_min = 1) of that F_max and v_max, after one warm-up call (which
    # allocates its workspace and tables); synchronous, so timed on the host clock too
    label = torch.empty((n, n, n), dtype=torch.int32, device="cuda")
    halo_size = torch.empty((n, n, n), dtype=torch.int32, device="cuda")
    B.pin_fragment(plan.handle, F.data_ptr(), vmax.data_ptr(), 1.0, None, label.data_ptr(), halo_size.data_ptr(), stream)
    t0f = time.perf_counter()
    n_halos = B.pin_fragment(plan.handle, F.data_ptr(), vmax.data_ptr(), 1.0, None, label.data_ptr(),
                             halo_size.data_ptr(), stream)
    frag_ms = 1000.0 * (time.perf_counter() - t0f)
    frag = {"ms": round(frag_ms, 2), "halos": n_halos, "particles_in_halos": int((label >= 0).sum()),
            "filament": int((label == -1).sum()), "collapsed": int((label != -2).sum()),
            "largest_halo": int(halo_size.max())}
    del vmax, label, halo_size
    # collapse redshift of every point (flat LambdaCDM, Omega_m 0.25): 2 x real bytes per point
    zc = torch.empty_like(F)
    B.pin_plan_set_growth(plan.handle, 0.25, stream)
    B.pin_collapse_redshift(plan.handle, F.data_ptr(), n ** 3, zc.data_ptr(), stream)
    z_ms = timed(lambda: B.pin_collapse_redshift(plan.handle, F.data_ptr(), n ** 3, zc.data_ptr(), stream))
    del zc
    disp_ms = timed(lambda: B.pin_displacements(plan.handle, dk.data_ptr(), p1.data_ptr(), p2.data_ptr(), stream))
    # third-order displacement, after one warm-up call (which allocates its workspace)
    p3 = torch.empty((3, n, n, n), dtype=plan.real, device="cuda")
    B.pin_lpt3_displacement(plan.handle, dk.data_ptr(), p3.data_ptr(), stream)
    lpt3_ms = timed(lambda: B.pin_lpt3_displacement(plan.handle, dk.data_ptr(), p3.data_ptr(), stream))
    del p3
    # whole-path roofline at the collapse-only rate: algorithmic bytes per grid-point x radius
    # update of these passes (19 workspace slots of 4 B per point plus F read/write and the
    # index) and the floor of any out-of-core 3D FFT design (spectrum once, one 3-component
    # transpose round trip, F and index: 7 slots + 10 B)
    slot_pp = 2 * real_bytes * (n // 2) / n   # workspace slot bytes per grid point
    per_update = {"three_pass": 19 * slot_pp + 2 * real_bytes + 1, "floor": 7 * slot_pp + 2 * real_bytes + 2}
    rate = updates / (collapse_ms * 1e-3)
    path_roofline = {k: {"bytes_per_update": round(v, 2), "GB/s": round(rate * v / 1e9, 1),
                         "frac": round(rate * v / 1e9 / HBM_PEAK_GBS, 4)} for k, v in per_update.items()}
    del p1, p2, F, R, dk
    plan.close()
    torch.cuda.empty_cache()

    fp64 = None
    if not args.no_fp64 and prec == B.PIN_FP32:
        plan64 = B.Plan(n, box, radii, W.SIGMA8, W.GAMMA, W.NS, B.PIN_FP64)
        dk64 = plan64.generate_field(seed)
        F64 = torch.empty((n, n, n), dtype=torch.float64, device="cuda")
        R64 = torch.empty((n, n, n), dtype=torch.uint8, device="cuda")
        plan64.collapse_times(dk64, F64, R64)
        torch.cuda.synchronize()
        ev0.record()
        plan64.collapse_times(dk64, F64, R64)
        ev1.record()
        torch.cuda.synchronize()
        ms64 = ev0.elapsed_time(ev1)
        fp64 = {"collapse_updates_per_s": updates / (ms64 * 1e-3), "collapse_ms": round(ms64, 2)}
        del dk64, F64, R64
        plan64.close()
        torch.cuda.empty_cache()
        print(f"[bench] fp64 collapse: {ms64:.1f} ms", file=sys.stderr, flush=True)

    if args.copy_probe:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    configs = None
    if not args.no_configs and args.config == "c512_fp32":
        configs = {}
        for name in ("c256_fp32", "c768_fp32"):
            configs[name] = config_leg(B, W, name)
            print(f"[bench] {name}: collapse {configs[name]['collapse_ms']} ms", file=sys.stderr, flush=True)

    serve_out = None
    if not args.no_serve and args.config == "c512_fp32":
        print("[bench] serving leg", file=sys.stderr, flush=True)
        serve_out = serve_bench(B, W, full=not args.serve_quick)
        print(f"[bench] serving: p99 {serve_out['p99_latency_s']} s, served/plain "
              f"{serve_out['served_over_plain']}", file=sys.stderr, flush=True)

    base = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        base = cpu_baseline()
        base["single_thread_64"] = cpu_baseline_single()

    out = {
        "metric": "grid-point x radius collapse updates/s at 512^3 (FP32 vs FP64); p99 serve latency",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == B.PIN_FP32 else "f64",
        "data": "synthetic (seeded BBKS Gaussian field)",
        "config": {"workload": f"{n}^3 grid, {box:g} Mpc/h, {len(radii)} Gaussian radii "
                               f"{cfg['r_max']:g}->{cfg['r_min']:g} cells, field + collapse + ZA/2LPT",
                   "n": n, "box_mpc_h": box, "n_radii": len(radii), "precision": cfg["prec"]},
        "collapse_only": {"updates_per_s": rate, "ms": round(collapse_ms, 2), "runs_ms": [round(x, 2) for x in runs]},
        "collapse_with_velocity": {"updates_per_s": updates / (vel_ms * 1e-3), "ms": round(vel_ms, 2)},
        "collapse_redshift": {"ms": round(z_ms, 3), "GB/s": round(2 * real_bytes * n ** 3 / (z_ms * 1e-3) / 1e9, 1)},
        "field_ms": round(field_ms, 3),
        "displacements_ms": round(disp_ms, 3),
        "lpt3_ms": round(lpt3_ms, 3),
        "fragment": frag,
        "path_roofline": path_roofline,
        "fp64": fp64,
        "roofline": roofline,
        "kernels": per_kernel,
        "configs": configs,
        "serve": serve_out,
        "cpu_baseline": base,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
