"""Write the FP64 oracle's collapse times at sampled grid points of the large workloads, for
tests/test_gpu_fullsize.py: tests/golden/fullsize_points_<workload>.npz.

    python tests/golden/make_fullsize_points.py [workload ...] [--threads 3] [--resume DIR]

Default workloads: s384_fp32, c512_fp32, c768_fp32 (384^3, 512^3 and 768^3 grids).  For each: the
seeded linear field (oracle.field), then per radius the deformation tensor on the full grid
(oracle.hessian, one component at a time so that 768^3 fits in memory, a few radii at once in
threads), read at the points; the collapse model (oracle.collapse) at the points for every
radius and the running maximum (radii largest first, strict '>' to update, 0 and index 255
before any), as oracle.run does on the full grid.  Also stored: the rms of one tensor component
at the smallest radius (Parseval on the oracle field), the scale of the tests' tolerances.

With --resume, each radius's tensor at the points is also kept in DIR and read back on a later
run, so that an interrupted run goes on where it stopped.

Points: the three fixed corner / Nyquist-adjacent indices of the tests, then seeded random ones
(numpy default_rng(seed * 10 + 3)), 1024 in all.  Nothing here reads GPU output.
"""

import argparse
import concurrent.futures as cf
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import collapse, field, hessian  # noqa: E402
from paper_1305_1505_amd import workloads as W  # noqa: E402

NPOINTS = 1024
NEVER = 255


def golden_points(name):
    cfg = W.CONFIGS[name]
    n = cfg["n"]
    rng = np.random.default_rng(cfg["seed"] * 10 + 3)
    fixed = [(0, 0, 0), (n - 1, n - 1, n - 1), (n // 2, n // 2 - 1, n // 2 + 1)]
    rand = rng.integers(0, n, (NPOINTS - len(fixed), 3))
    return np.array(fixed + [tuple(int(v) for v in p) for p in rand], dtype=np.int32)


def component_rms(dk, radius):
    """RMS over the grid of the smoothed density (the trace of T) / sqrt(3), by Parseval."""
    n = dk.shape[0]
    w = hessian.gaussian_window(n, radius) * hessian.nyquist_mask(n)
    wl = np.full(n // 2 + 1, 2.0)
    wl[0] = wl[n // 2] = 1.0
    tot = sum(float(np.sum(wl[None, :] * np.abs(w[i] * dk[i]) ** 2)) for i in range(n))
    return np.sqrt(tot) / float(n) ** 3 / np.sqrt(3.0)


def make(name, threads, resume=None):
    cfg = W.CONFIGS[name]
    n = cfg["n"]
    radii = W.config_radii(cfg)
    pts = golden_points(name)
    t0 = time.time()
    dk = field.linear_field(cfg["seed"], n, cfg["box"], W.SIGMA8, W.GAMMA, W.NS)
    print(f"[golden] {name}: field {time.time() - t0:.0f} s", flush=True)
    ix, iy, iz = pts[:, 0], pts[:, 1], pts[:, 2]

    def tensor_at(r):
        keep = None if resume is None else os.path.join(resume, f"{name}_r{r:03d}.npy")
        if keep is not None and os.path.exists(keep):
            return np.load(keep)
        out = np.empty((len(pts), 6))
        for c, ab in enumerate(hessian.COMPONENTS):
            comp = hessian.deformation_tensor(dk, radii[r], components=(ab,))[0]
            out[:, c] = comp[ix, iy, iz]
            del comp
        if keep is not None:
            np.save(keep + ".tmp.npy", out)
            os.replace(keep + ".tmp.npy", keep)
        return out

    if resume is not None:
        os.makedirs(resume, exist_ok=True)
    with cf.ThreadPoolExecutor(threads) as ex:
        tens = []
        for r, t in enumerate(ex.map(tensor_at, range(len(radii)))):
            tens.append(t)
            print(f"[golden] {name}: radius {r + 1}/{len(radii)} {time.time() - t0:.0f} s", flush=True)
    tens = np.stack(tens, axis=1)                                   # (P, n_radii, 6)
    fr = collapse.inverse_collapse_time([tens[:, :, c].ravel() for c in range(6)]).reshape(len(pts), len(radii))
    fmax = np.zeros(len(pts))
    ridx = np.full(len(pts), NEVER, dtype=np.uint8)
    for r in range(len(radii)):
        up = fr[:, r] > fmax
        fmax = np.where(up, fr[:, r], fmax)
        ridx = np.where(up, np.uint8(r), ridx)
    out = os.path.join(HERE, f"fullsize_points_{name}.npz")
    np.savez_compressed(out, points=pts, fmax=fmax, ridx=ridx, f_per_radius=fr.astype(np.float32),
                        radii=radii, sigma_rmin=component_rms(dk, radii[-1]), n=n, box=cfg["box"], seed=cfg["seed"])
    print(f"[golden] {name}: wrote {out} ({time.time() - t0:.0f} s)", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workloads", nargs="*", default=["s384_fp32", "c512_fp32", "c768_fp32"])
    ap.add_argument("--threads", type=int, default=3)
    ap.add_argument("--resume", default=None, help="directory keeping each radius's tensor at the points")
    args = ap.parse_args()
    for name in args.workloads:
        make(name, args.threads, args.resume)


if __name__ == "__main__":
    main()
