"""Accuracy of the HIP path against the FP64 oracle on every workload: max and RMS relative error
of F_max and of the ZA, 2LPT and 3LPT displacements, and the fraction of grid points whose collapse
radius R_max differs (float32 and float64 plans).

    python tests/accuracy_report.py [--workers 16] [--out report.json]

Full grids where the oracle fits the run time (64^3, 256^3; displacements, 3LPT included, also at
512^3);
sampled grid points (oracle.points) for F at 512^3 and 768^3 and psi1 at 768^3.  The oracle runs
in a pool of worker processes started before this process touches the GPU; radii are split
between workers and their partial maxima merged with the rule of the running maximum (larger F
wins, a tie keeps the larger radius).  Metrics as in oracle.metrics: rel_rms = |x - x_o| / |x_o|,
rel_max = max|x - x_o| / max|x_o|, mismatch = fraction of points with a different R_max.
Prints one line per result as it arrives and a markdown table at the end.
"""

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import field, lpt3, metrics, points, run  # noqa: E402
from paper_1305_1505_amd import workloads as W  # noqa: E402

POINTS = {"c512_fp32": 64, "c768_fp32": 32}


def _field(name):
    cfg = W.CONFIGS[name]
    return field.linear_field(cfg["seed"], cfg["n"], cfg["box"], W.SIGMA8, W.GAMMA, W.NS)


def job_radii(name, r0, r1):
    """Running maximum over radii [r0, r1) with fresh state (oracle)."""
    radii = W.config_radii(W.CONFIGS[name])
    return ("radii", name, r0, run.collapse_times(_field(name), radii, r0, r1))


def job_disp(name):
    return ("disp", name, run.displacements(_field(name), W.CONFIGS[name]["box"]))


def job_lpt3(name):
    return ("lpt3", name, lpt3.lpt3_displacement(_field(name), W.CONFIGS[name]["box"]))


def job_points(name, pts):
    cfg = W.CONFIGS[name]
    dk = _field(name)
    fmax, ridx, _ = points.collapse_times_at_points(dk, pts, W.config_radii(cfg))
    return ("points", name, pts, fmax, ridx, points.za_at_points(dk, pts, cfg["box"]))


def sample_points(name):
    n = W.CONFIGS[name]["n"]
    rng = np.random.default_rng(W.CONFIGS[name]["seed"] + 7)
    return [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(POINTS[name])]


def merge(parts):
    """Merge (r0, (fmax, ridx)) partial running maxima in radius order."""
    parts = sorted(parts, key=lambda p: p[0])
    fmax, ridx = parts[0][1]
    for _, (f, r) in parts[1:]:
        up = f > fmax
        fmax = np.where(up, f, fmax)
        ridx = np.where(up, r, ridx)
    return fmax, ridx


def gpu_outputs(lib, name, prec, pts=None, want_disp=True):
    """GPU F, R_max (and psi1, psi2) on the host: full arrays, or only at `pts`."""
    import torch

    cfg = W.CONFIGS[name]
    plan = lib.Plan(cfg["n"], cfg["box"], W.config_radii(cfg), sigma8=W.SIGMA8, gamma=W.GAMMA, ns=W.NS, prec=prec)
    dk = plan.generate_field(cfg["seed"])
    F, R = plan.collapse_times(dk)
    if pts is not None:
        idx = torch.tensor(pts, device="cuda", dtype=torch.long)
        at = lambda t: t[..., idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy().astype(np.float64)
        out = {"F": at(F), "R": at(R)}
    else:
        at = lambda t: t.cpu().numpy()   # native precision (float32 plans: float32)
        out = {"F": at(F), "R": R.cpu().numpy()}
    del F, R
    if want_disp:
        p1, p2 = plan.displacements(dk, want_psi2=pts is None)
        out["psi1"] = at(p1)
        if p2 is not None:
            out["psi2"] = at(p2)
        del p1, p2
        if pts is None:
            p3 = plan.lpt3_displacement(dk)
            out["psi3"] = at(p3)
            del p3
    del dk
    plan.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


CASES = (("c64_fp64", "fp64"), ("c64_fp64", "fp32"), ("c256_fp32", "fp32"), ("c256_fp32", "fp64"),
         ("c512_fp32", "fp32"), ("c768_fp32", "fp32"))
SAMPLED = ("c512_fp32", "c768_fp32")


def gpu_phase(path):
    """Run every case on the GPU and save the outputs (host arrays) to `path` (.npz)."""
    from paper_1305_1505_amd import binding as lib

    t0 = time.time()
    arrays = {}
    for name, precname in CASES:
        prec = lib.PIN_FP64 if precname == "fp64" else lib.PIN_FP32
        if name == "c512_fp32":   # F at the sampled points, displacements on the full grid
            g = gpu_outputs(lib, name, prec, pts=sample_points(name), want_disp=False)
            g.update({k: v for k, v in gpu_outputs(lib, name, prec).items() if k.startswith("psi")})
        elif name in SAMPLED:
            g = gpu_outputs(lib, name, prec, pts=sample_points(name))
        else:
            g = gpu_outputs(lib, name, prec)
        for k, v in g.items():
            arrays[f"{name}|{precname}|{k}"] = v
        print(f"[accuracy] GPU {name} {precname} done {time.time() - t0:.0f} s", flush=True)
    np.savez(path, **arrays)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--out", default=None)
    ap.add_argument("--gpu-phase", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.gpu_phase:
        gpu_phase(args.gpu_phase)
        return
    t0 = time.time()
    # the GPU work runs in a child process first; this process never initialises the GPU
    import subprocess
    import tempfile

    tmp = os.path.join(tempfile.gettempdir(), f"pin_accuracy_{os.getpid()}.npz")
    subprocess.run([sys.executable, "-u", os.path.abspath(__file__), "--gpu-phase", tmp], check=True)
    data = np.load(tmp)
    gpu = {}
    for key in data.files:
        name, precname, k = key.split("|")
        gpu.setdefault((name, precname), {})[k] = data[key]
    os.remove(tmp)

    ctx = mp.get_context("spawn")
    pool = ctx.Pool(args.workers)
    pending = []
    # quick jobs first, then one job per radius at 256^3 (about a minute each)
    pending.append(pool.apply_async(job_radii, ("c64_fp64", 0, len(W.config_radii(W.CONFIGS["c64_fp64"])))))
    for name in ("c64_fp64", "c256_fp32", "c512_fp32"):
        pending.append(pool.apply_async(job_disp, (name,)))
        pending.append(pool.apply_async(job_lpt3, (name,)))
    for r0 in range(len(W.config_radii(W.CONFIGS["c256_fp32"]))):
        pending.append(pool.apply_async(job_radii, ("c256_fp32", r0, r0 + 1)))
    sampled = {name: sample_points(name) for name in SAMPLED}
    for name, pts in sampled.items():
        per = max(1, len(pts) // args.workers)
        for i in range(0, len(pts), per):
            pending.append(pool.apply_async(job_points, (name, pts[i:i + per])))
    print(f"[accuracy] {len(pending)} oracle jobs queued", flush=True)

    radii_parts, disp, pts_res, psi3 = {}, {}, {}, {}
    for job in pending:
        res = job.get()
        if res[0] == "radii":
            radii_parts.setdefault(res[1], []).append((res[2], res[3]))
        elif res[0] == "disp":
            disp[res[1]] = res[2]
        elif res[0] == "lpt3":
            psi3[res[1]] = res[2]
        else:
            pts_res.setdefault(res[1], []).append(res[2:])
        print(f"[accuracy] oracle {res[0]} {res[1]} done {time.time() - t0:.0f} s", flush=True)
    pool.close()

    rows = []
    for (name, precname), g in gpu.items():
        label = f"{name} {precname} plan"
        row = {"config": label}
        if name in radii_parts:
            fmax, ridx = merge(radii_parts[name])
            rep = metrics.report(g["F"], fmax)
            row.update(F_rel_rms=rep["rel_rms"], F_rel_max=rep["rel_max"], F_points="all",
                       R_mismatch=metrics.mismatch_fraction(g["R"], ridx))
        elif name in pts_res:
            # oracle results in the order of `sampled[name]` (chunks were submitted in order)
            pts = [p for chunk in pts_res[name] for p in chunk[0]]
            assert pts == sampled[name]
            fref = np.concatenate([c[1] for c in pts_res[name]])
            rref = np.concatenate([c[2] for c in pts_res[name]])
            row.update(F_rel_rms=metrics.rel_rms(g["F"], fref), F_rel_max=metrics.rel_max(g["F"], fref),
                       F_points=len(pts), R_mismatch=float(np.mean(g["R"] != rref)))
            if name not in disp:
                zref = np.concatenate([c[3] for c in pts_res[name]])
                z = g["psi1"].T
                row.update(psi1_rel_rms=metrics.rel_rms(z, zref), psi1_rel_max=metrics.rel_max(z, zref),
                           psi_points=len(pts))
        if name in disp:
            r1, r2 = disp[name]
            row.update(psi1_rel_rms=metrics.rel_rms(g["psi1"], r1), psi1_rel_max=metrics.rel_max(g["psi1"], r1),
                       psi2_rel_rms=metrics.rel_rms(g["psi2"], r2), psi2_rel_max=metrics.rel_max(g["psi2"], r2),
                       psi_points="all")
        if name in psi3 and "psi3" in g:
            r3 = psi3[name]
            row.update(psi3_rel_rms=metrics.rel_rms(g["psi3"], r3), psi3_rel_max=metrics.rel_max(g["psi3"], r3))
        rows.append(row)
        print("[accuracy] " + json.dumps(row), flush=True)

    keys = ["config", "F_rel_rms", "F_rel_max", "R_mismatch", "F_points", "psi1_rel_rms", "psi1_rel_max",
            "psi2_rel_rms", "psi2_rel_max", "psi3_rel_rms", "psi3_rel_max", "psi_points"]
    fmt = lambda v: f"{v:.2e}" if isinstance(v, float) else str(v)
    print("| " + " | ".join(keys) + " |")
    print("|" + "---|" * len(keys))
    for row in rows:
        print("| " + " | ".join(fmt(row.get(k, "")) for k in keys) + " |")
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(rows, fh, indent=1)


if __name__ == "__main__":
    main()
