"""Benchmark: grid-point x radius collapse updates per second on one MI355X.

One step is one pass of the whole path over one realisation: the seeded Gaussian field, the
collapse times over every radius (per radius: window x Hessian multiply, the three FFT passes,
the per-point eigenvalue / collapse / running maximum), and the closing ZA and 2LPT
displacements.  value = N^3 * n_radii / seconds per step.

Workload (default): 512^3 grid, 1000 Mpc/h box, 40 Gaussian radii log-spaced 60 -> 0.75 cells,
BBKS spectrum (Gamma 0.21, n 1, sigma_8 0.8), complex64 FFTs.  Data are synthetic (seeded).

Prints ONE JSON line.  Extra fields: the dominant kernel's roofline (algorithmic bytes per launch
over its HIP-event-timed average duration), the collapse-only rate, the float64 rate of the same
workload, and the FP64 CPU oracle timed on a bounded sample (cpu_baseline).
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
    """Bytes a launch of kernel class `cls` must move at grid size n (see the design doc table)."""
    cb = 2 * real_bytes
    slot = n * n * (n // 2) * cb          # one workspace slot (kz = N/2 plane not stored)
    vol = n ** 3
    return {
        "xpass_hessian": slot + 3 * slot,                 # spectrum in (kz < N/2), 3 slots out
        "ypass_hessian": 3 * slot + 6 * slot,             # 3 in, 6 out
        "zpass_collapse": 6 * slot + vol * (2 * real_bytes + 1),   # 6 in; F read + F, ridx written
    }.get(cls)


def cpu_baseline(sample_n=64, radius_stride=4):
    """The FP64 oracle on a bounded sample of the workload: a sample_n^3 grid with the same cell
    size (box scaled), every radius_stride-th radius, full step (field, collapse, displacements)."""
    import numpy as np

    from oracle import field, run
    from paper_1305_1505_amd import workloads as W

    cfg = W.CONFIGS["c512_fp32"]
    box = cfg["box"] * sample_n / cfg["n"]
    radii = W.config_radii(cfg)[::radius_stride]
    t0, c0 = time.perf_counter(), time.process_time()
    dk = field.linear_field(cfg["seed"], sample_n, box, W.SIGMA8, W.GAMMA, W.NS)
    run.collapse_times(dk, radii)
    run.displacements(dk, box)
    dt, cpu = time.perf_counter() - t0, time.process_time() - c0
    updates = sample_n ** 3 * len(radii)
    cores = max(1, int(round(cpu / dt)))          # threads actually busy on average
    return {"value": updates / dt, "unit": "updates/s", "cores": cores, "kind": "oracle",
            "seconds": dt,
            "sample": f"{sample_n}^3 grid at the workload's cell size ({box:g} Mpc/h), "
                      f"{len(radii)} of its {cfg['n_radii']} radii, field + collapse + ZA/2LPT, "
                      f"float64 NumPy/SciPy, {os.cpu_count()} host cores visible"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c512_fp32")
    ap.add_argument("--no-fp64", action="store_true", help="skip the float64 comparison leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (see DESIGN.md, sharding)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1305_1505_amd import binding as B
    from paper_1305_1505_amd import workloads as W

    torch.cuda.set_device(0)
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

    B.pin_plan_set_timing(plan.handle, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1000.0 * elapsed / args.steps
    updates = n ** 3 * len(radii)
    value = updates / (elapsed / args.steps)

    kernels = {}
    for c in range(B.pin_kernel_class_count()):
        ms, cnt = B.pin_plan_kernel_time(plan.handle, c)
        if cnt:
            kernels[B.pin_kernel_class_name(c)] = {"total_ms": ms, "launches": cnt, "avg_ms": ms / cnt}
    B.pin_plan_set_timing(plan.handle, False)
    print(f"[bench] timed {args.steps} steps: {ms_per_step:.2f} ms/step", file=sys.stderr, flush=True)

    # the dominant kernel of the path: largest summed time among the three per-radius passes
    dom = max(("xpass_hessian", "ypass_hessian", "zpass_collapse"), key=lambda k: kernels[k]["total_ms"])
    dom_bytes = algorithmic_bytes(dom, n, real_bytes)
    achieved = dom_bytes / (kernels[dom]["avg_ms"] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "bytes_per_launch": dom_bytes}
    per_kernel = {k: {"avg_ms": round(v["avg_ms"], 4), "launches": v["launches"],
                      "GB/s": (round(algorithmic_bytes(k, n, real_bytes) / (v["avg_ms"] * 1e-3) / 1e9, 1)
                               if algorithmic_bytes(k, n, real_bytes) else None)}
                  for k, v in kernels.items()}

    # collapse-only rate (HIP events around pin_collapse_times)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    B.pin_collapse_times(plan.handle, dk.data_ptr(), F.data_ptr(), R.data_ptr(), stream)
    ev1.record()
    torch.cuda.synchronize()
    collapse_ms = ev0.elapsed_time(ev1)
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

    base = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        base = cpu_baseline()

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
        "collapse_only": {"updates_per_s": updates / (collapse_ms * 1e-3), "ms": round(collapse_ms, 2)},
        "fp64": fp64,
        "roofline": roofline,
        "kernels": per_kernel,
        "cpu_baseline": base,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
