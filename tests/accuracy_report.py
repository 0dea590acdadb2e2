"""Accuracy of the HIP path against the FP64 oracle on every workload: max and RMS relative error
of F_max and of the ZA, 2LPT and 3LPT displacements, and the fraction of grid points whose
collapse radius R_max differs (float32 and float64 plans).

Two phases, so that the oracle's hours of host work need no GPU and the GPU's output fits a
bounded transfer:

    python tests/accuracy_report.py gpu <out.npz> [--cases A,B,...] [--part P]   # on the GPU
    python tests/accuracy_report.py oracle <gpu.npz> [<gpu.npz> ...] --out <out.json> [--md out.md]
                                   [--threads 6] [--cache DIR]
    python tests/accuracy_report.py prepare --cases A,B --cache DIR    # oracle side ahead of time

The GPU phase runs each case through the C ABI in the launch configuration bench.py uses (one
plan, pin_generate_field, pin_collapse_times, pin_displacements, pin_lpt3_displacement) and keeps
the outputs on a lattice of grid points: every `stride`-th point along each axis (stride 1 = the
whole grid), one lattice for F_max and R_max and a coarser one for the displacements.  A case
whose F_max/R_max lattice is too large for one transfer is cut into parts of `slab` x-planes:
`--part P` keeps planes [P*slab, (P+1)*slab) (part 0 also keeps the displacements), saved
compressed, and the oracle phase joins the parts of all the files it is given.  The oracle
phase computes the same quantities on the whole grid from the oracle (field, deformation tensors
per radius, collapse model, running maximum, displacements) and reads them at the same lattice
points; nothing in it comes from the GPU.  The 768^3 case runs five of its radii (the first, the
last and three between) on both sides: its full-grid tensors (six 3.6 GB float64 fields per
radius) are the oracle's bottleneck.

Metrics as in oracle.metrics, over the lattice points: rel_rms = |x - x_o| / |x_o|,
rel_max = max|x - x_o| / max|x_o|, R mismatch = fraction of points whose R_max index differs.
F_max is discontinuous where the collapse cubic's two larger roots merge: there F at a radius
jumps between the largest root and a smaller one (or 0), and a rounding of the tensor decides
which.  Every point whose F_max is farther than 1e-4 max|F| from the oracle's is examined with
the oracle alone (its tensors at that point by direct summation, perturbed by one rounding of
the plan's precision): if the GPU's value lies in the range those perturbations give, the point
is a verified jump; the table gives the metrics over all points, the number of verified jumps,
the number of outliers left unexplained (a defect if not 0), and the metrics without the jumps.
"""

import argparse
import collections
import concurrent.futures as cf
import itertools
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import collapse, field, hessian, lpt3, metrics, points, run  # noqa: E402
from paper_1305_1505_amd import workloads as W  # noqa: E402

# name -> (workload, plan precision, F/R lattice stride, displacement lattice stride,
#          displacements compared, radius indices (None = all), x-planes per part (None = one part))
CASES = {
    "c64_fp64": ("c64_fp64", "fp64", 1, 1, ("psi1", "psi2", "psi3"), None, None),
    "c64_fp32": ("c64_fp64", "fp32", 1, 1, ("psi1", "psi2", "psi3"), None, None),
    "c256_fp32": ("c256_fp32", "fp32", 2, 4, ("psi1", "psi2", "psi3"), None, None),
    "c256_fp64": ("c256_fp32", "fp64", 4, 8, ("psi1", "psi2", "psi3"), None, None),
    "c512_fp32": ("c512_fp32", "fp32", 1, 8, ("psi1", "psi2", "psi3"), None, 52),
    "c768_fp32": ("c768_fp32", "fp32", 6, 12, ("psi1",), (0, 11, 22, 33, 44), None),
}


def case_parts(case):
    """Number of GPU parts of a case (lattice x-planes split by `slab`)."""
    wl, _, fs, _, _, _, slab = CASES[case]
    if slab is None:
        return 1
    m = (W.CONFIGS[wl]["n"] + fs - 1) // fs
    return (m + slab - 1) // slab


def case_radii(case):
    wl, _, _, _, _, sel, _ = CASES[case]
    radii = W.config_radii(W.CONFIGS[wl])
    return radii if sel is None else np.array([radii[i] for i in sel])


def lattice(a, stride):
    """The lattice points of a (..., N, N, N) array."""
    return a[..., ::stride, ::stride, ::stride]


# ------------------------------------------------------------------------------------------ GPU
def gpu_case(lib, case, part=0):
    import torch

    wl, precname, fs, ps, disp, _, slab = CASES[case]
    cfg = W.CONFIGS[wl]
    prec = lib.PIN_FP64 if precname == "fp64" else lib.PIN_FP32
    plan = lib.Plan(cfg["n"], cfg["box"], case_radii(case), sigma8=W.SIGMA8, gamma=W.GAMMA, ns=W.NS, prec=prec)
    dk = plan.generate_field(cfg["seed"])
    F, R = plan.collapse_times(dk)
    host = lambda t, s: lattice(t, s).contiguous().cpu().numpy()
    if slab is None:
        out = {"F": host(F, fs), "R": host(R, fs)}
    else:
        lo = part * slab
        out = {f"F@{lo}": host(lattice(F, fs)[lo:lo + slab], 1), f"R@{lo}": host(lattice(R, fs)[lo:lo + slab], 1)}
    del F, R
    if part > 0:
        del dk
        plan.close()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        return out
    p1, p2 = plan.displacements(dk, want_psi2="psi2" in disp)
    out["psi1"] = host(p1, ps)
    if p2 is not None:
        out["psi2"] = host(p2, ps)
    del p1, p2
    if "psi3" in disp:
        p3 = plan.lpt3_displacement(dk)
        out["psi3"] = host(p3, ps)
        del p3
    del dk
    plan.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def gpu_phase(path, cases, part=None):
    from paper_1305_1505_amd import binding as lib

    t0 = time.time()
    arrays = {}
    for case in cases:
        if part is not None and not 0 <= part < case_parts(case):
            raise SystemExit(f"{case} has parts 0..{case_parts(case) - 1}")
        for k, v in gpu_case(lib, case, part or 0).items():
            arrays[f"{case}|{k}"] = v
        print(f"[accuracy] GPU {case} part {part or 0} done {time.time() - t0:.0f} s", flush=True)
    (np.savez if part is None else np.savez_compressed)(path, **arrays)


def load_gpu(paths):
    """The GPU outputs of several files, per case; the parts F@lo / R@lo of a split case are
    joined along x and must cover its whole lattice."""
    gpu = {}
    for path in paths:
        with np.load(path) as data:
            for key in data.files:
                case, k = key.split("|")
                gpu.setdefault(case, {})[k] = data[key]
    for case, g in gpu.items():
        for q in ("F", "R"):
            parts = sorted((int(k.split("@")[1]), k) for k in g if k.startswith(q + "@"))
            if not parts:
                continue
            lo = 0
            for start, k in parts:
                if start != lo:
                    raise SystemExit(f"{case}: {q} parts do not cover planes from {lo}")
                lo += g[k].shape[0]
            g[q] = np.concatenate([g.pop(k) for _, k in parts])
            want = lattice(np.empty((W.CONFIGS[CASES[case][0]]["n"],) * 3, np.uint8), CASES[case][2]).shape
            if g[q].shape != want:
                raise SystemExit(f"{case}: {q} parts cover {g[q].shape}, lattice is {want}")
    return gpu


# --------------------------------------------------------------------------------------- oracle
def bounded_map(ex, fn, items, ahead):
    """fn over items in order, at most `ahead` results computed ahead of the one being used
    (0: one at a time, nothing ahead), so that large results do not pile up in memory."""
    if ahead <= 0:
        for x in items:
            yield fn(x)
        return
    items = iter(items)
    futs = collections.deque(ex.submit(fn, x) for x in itertools.islice(items, ahead))
    while futs:
        res = futs.popleft().result()
        nxt = next(items, None)
        if nxt is not None:
            futs.append(ex.submit(fn, nxt))
        yield res
        del res


def oracle_F(dk, radii, stride, threads, mem_bytes):
    """F_max and R_max index on the lattice: per radius the full-grid tensor (computed ahead in
    threads for as many radii as mem_bytes allows beside the one in use; one component at a time
    above 512^3), read at the lattice points, the collapse model there, and the running maximum
    in radius order."""
    n = dk.shape[0]
    per_radius = (4 if n > 512 else 9) * 8.0 * n ** 3
    ahead = max(0, min(threads, int(mem_bytes // per_radius) - 1))

    def tensor(radius):
        if n > 512:
            return [lattice(hessian.deformation_tensor(dk, radius, components=(ab,))[0], stride).ravel()
                    for ab in hessian.COMPONENTS]
        return [lattice(c, stride).ravel() for c in hessian.deformation_tensor(dk, radius)]

    def model(t6):
        m = t6[0].size
        chunk = min(-(-m // (4 * threads)), 1 << 20)
        with cf.ThreadPoolExecutor(threads) as ex:
            parts = ex.map(lambda s: collapse.inverse_collapse_time([c[s:s + chunk] for c in t6]), range(0, m, chunk))
            return np.concatenate(list(parts))

    fmax = ridx = None
    t0 = time.time()
    with cf.ThreadPoolExecutor(max(1, ahead)) as ex:
        for r, t6 in enumerate(bounded_map(ex, tensor, radii, ahead)):
            f = model(t6)
            del t6
            if fmax is None:
                fmax = np.zeros_like(f)
                ridx = np.full(f.shape, run.NEVER, dtype=np.uint8)
            up = f > fmax
            fmax = np.where(up, f, fmax)
            ridx = np.where(up, np.uint8(r), ridx)
            del f, up
            print(f"[accuracy] oracle N={n} radius {r + 1}/{len(radii)} {time.time() - t0:.0f} s", flush=True)
    m = (n + stride - 1) // stride
    return fmax.reshape(m, m, m), ridx.reshape(m, m, m)


def oracle_case(case, threads, mem_bytes):
    wl, _, fs, ps, disp, _, _ = CASES[case]
    cfg = W.CONFIGS[wl]
    dk = field.linear_field(cfg["seed"], cfg["n"], cfg["box"], W.SIGMA8, W.GAMMA, W.NS)
    out = {}
    out["F"], out["R"] = oracle_F(dk, case_radii(case), fs, threads, mem_bytes)
    box = cfg["box"]
    out["psi1"] = lattice(run.za_displacement(dk, box), ps)
    if "psi2" in disp:
        out["psi2"] = lattice(run.lpt2_displacement(dk, box), ps)
    if "psi3" in disp:
        out["psi3"] = lattice(lpt3.lpt3_displacement(dk, box), ps)
    return out


# Points whose |F - F_oracle| exceeds this fraction of max F_oracle are examined one by one.
OUTLIER = 1e-4
MAX_EXAMINED = 64


def jump_interval(dk, point, radii, precname, samples=200, seed=0):
    """[lo, hi] of F_max at one grid point when each radius's oracle tensor (direct sums,
    oracle.points) is perturbed by Gaussian noise of one rounding of the plan's precision
    (1e-7 of the tensor's norm for float32, 1e-16 for float64), `samples` draws.  Where the
    collapse cubic's two larger roots are about to merge, F at that radius jumps between the
    largest root and a smaller one (or 0) under such noise, and any F_max in this interval is an
    answer the plan's precision cannot tell from the oracle's."""
    t = points.tensor_at_points(dk, np.asarray([point]), radii)[0]          # (n_radii, 6)
    eps = 1e-16 if precname == "fp64" else 1e-7
    rng = np.random.default_rng(seed)
    scale = np.sqrt(np.sum(t ** 2, axis=1, keepdims=True))
    tp = t[None] + rng.normal(size=(samples,) + t.shape) * eps * scale[None]
    f = collapse.inverse_collapse_time([tp[..., c].ravel() for c in range(6)]).reshape(samples, len(radii))
    fmax = np.maximum(f.max(axis=1), 0.0)
    return float(fmax.min()), float(fmax.max())


def examine_outliers(case, g, o):
    """The points where the GPU's F_max is farther than OUTLIER max|F| from the oracle's: each is
    a verified jump if the GPU's value lies in the oracle's jump_interval there (within OUTLIER
    max|F|).  Only the GPU's choice of points to look at comes from the GPU; the interval is the
    oracle's."""
    wl, precname, fs, _, _, _, _ = CASES[case]
    cfg = W.CONFIGS[wl]
    tol = OUTLIER * float(np.max(np.abs(o["F"])))
    d = np.abs(g["F"].astype(np.float64) - o["F"])
    flat = np.flatnonzero(d.ravel() > tol)
    flat = flat[np.argsort(d.ravel()[flat])[::-1]]
    out = {"outliers": int(flat.size), "examined": int(min(flat.size, MAX_EXAMINED)), "jumps": [], "unexplained": []}
    if flat.size == 0:
        return out, np.zeros(d.shape, bool)
    dk = field.linear_field(cfg["seed"], cfg["n"], cfg["box"], W.SIGMA8, W.GAMMA, W.NS)
    radii = case_radii(case)
    jump = np.zeros(d.shape, bool)
    for i in flat[:MAX_EXAMINED]:
        li = np.unravel_index(int(i), d.shape)
        point = tuple(int(v) * fs for v in li)
        lo, hi = jump_interval(dk, point, radii, precname)
        gv, ov = float(g["F"][li]), float(o["F"][li])
        rec = {"point": point, "gpu": gv, "oracle": ov, "interval": [lo, hi]}
        if lo - tol <= gv <= hi + tol:
            out["jumps"].append(rec)
            jump[li] = True
        else:
            out["unexplained"].append(rec)
    return out, jump


def compare(case, g, o):
    wl, precname, fs, ps, disp, sel, _ = CASES[case]
    n = W.CONFIGS[wl]["n"]
    row = {"case": case, "workload": wl, "plan": precname, "n": n,
           "radii": len(case_radii(case)) if sel is None else f"{len(sel)} of {W.CONFIGS[wl]['n_radii']}",
           "F_points": int(g["F"].size), "F_stride": fs,
           "F_rel_rms": metrics.rel_rms(g["F"].astype(np.float64), o["F"]),
           "F_rel_max": metrics.rel_max(g["F"].astype(np.float64), o["F"]),
           "R_mismatch": float(np.mean(g["R"] != o["R"])), "R_mismatch_points": int(np.sum(g["R"] != o["R"])),
           "psi_points": int(g["psi1"][0].size), "psi_stride": ps}
    for k in disp:
        row[f"{k}_rel_rms"] = metrics.rel_rms(g[k].astype(np.float64), o[k])
        row[f"{k}_rel_max"] = metrics.rel_max(g[k].astype(np.float64), o[k])
    ex, jump = examine_outliers(case, g, o)
    row["F_outliers"] = ex["outliers"]
    row["F_jump_points"] = len(ex["jumps"])
    row["F_unexplained"] = ex["outliers"] - len(ex["jumps"])
    keep = ~jump
    row["F_rel_rms_regular"] = float(np.linalg.norm((g["F"].astype(np.float64) - o["F"])[keep]) / np.linalg.norm(o["F"]))
    row["F_rel_max_regular"] = float(np.max(np.abs(g["F"].astype(np.float64) - o["F"])[keep]) / np.max(np.abs(o["F"])))
    row["R_mismatch_regular_points"] = int(np.sum((g["R"] != o["R"]) & keep))
    row["outlier_detail"] = ex
    return row


def cached_oracle_case(case, threads, mem_bytes, cache):
    """oracle_case, kept in `cache` (a directory; None: no cache): the oracle's lattice values do
    not depend on the GPU code, so a later comparison reuses them."""
    if cache is None:
        return oracle_case(case, threads, mem_bytes)
    os.makedirs(cache, exist_ok=True)
    path = os.path.join(cache, f"oracle_{case}.npz")
    if os.path.exists(path):
        with np.load(path) as d:
            return {k: d[k] for k in d.files}
    out = oracle_case(case, threads, mem_bytes)
    np.savez(path, **out)
    return out


def oracle_phase(gpu_paths, out_json, md, threads, mem_bytes, cache=None):
    gpu = load_gpu(gpu_paths)
    rows = []
    t0 = time.time()
    for case in CASES:
        if case not in gpu:
            continue
        row = compare(case, gpu[case], cached_oracle_case(case, threads, mem_bytes, cache))
        rows.append(row)
        print(f"[accuracy] {time.time() - t0:.0f} s " + json.dumps(row), flush=True)
    with open(out_json, "w") as fh:
        json.dump(rows, fh, indent=1)
        fh.write("\n")
    keys = ["case", "radii", "F_points", "F_rel_rms", "F_rel_max", "F_jump_points", "F_unexplained", "F_rel_rms_regular",
            "F_rel_max_regular", "R_mismatch", "R_mismatch_points", "R_mismatch_regular_points", "psi1_rel_rms",
            "psi1_rel_max", "psi2_rel_rms", "psi2_rel_max", "psi3_rel_rms", "psi3_rel_max", "psi_points"]
    fmt = lambda v: f"{v:.2e}" if isinstance(v, float) else str(v)
    table = ["| " + " | ".join(keys) + " |", "|" + "---|" * len(keys)]
    table += ["| " + " | ".join(fmt(r.get(k, "")) for k in keys) + " |" for r in rows]
    print("\n".join(table))
    if md:
        with open(md, "a") as fh:
            fh.write("\n".join(table) + "\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="phase", required=True)
    g = sub.add_parser("gpu")
    g.add_argument("out")
    g.add_argument("--cases", default=",".join(CASES))
    g.add_argument("--part", type=int, default=None, help="part of a case split into x-plane slabs")
    o = sub.add_parser("oracle")
    o.add_argument("gpu", nargs="+")
    o.add_argument("--out", required=True)
    o.add_argument("--md", default=None)
    o.add_argument("--threads", type=int, default=min(6, os.cpu_count() or 1))
    o.add_argument("--mem-gb", type=float, default=30.0, help="host memory for full-grid tensors in flight")
    o.add_argument("--cache", default=None, help="directory keeping the oracle's lattice values per case")
    c = sub.add_parser("prepare", help="fill the oracle cache for some cases, before any GPU output exists")
    c.add_argument("--cases", required=True)
    c.add_argument("--cache", required=True)
    c.add_argument("--threads", type=int, default=min(6, os.cpu_count() or 1))
    c.add_argument("--mem-gb", type=float, default=30.0)
    args = ap.parse_args()
    if args.phase == "prepare":
        for case in (c for c in args.cases.split(",") if c):
            t0 = time.time()
            cached_oracle_case(case, args.threads, args.mem_gb * 1e9, args.cache)
            print(f"[accuracy] oracle {case} cached {time.time() - t0:.0f} s", flush=True)
        return
    if args.phase == "gpu":
        cases = [c for c in args.cases.split(",") if c]
        unknown = [c for c in cases if c not in CASES]
        if unknown:
            raise SystemExit(f"unknown cases {unknown}; known: {list(CASES)}")
        gpu_phase(args.out, cases, args.part)
    else:
        oracle_phase(args.gpu, args.out, args.md, args.threads, args.mem_gb * 1e9, args.cache)


if __name__ == "__main__":
    main()
