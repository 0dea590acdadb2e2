"""Synthetic workloads: the benchmark configurations and seeded test inputs.

This module holds no arithmetic of the method.  It names the grid sizes, boxes, radii lists and
seeds of the workloads (cubic grids, BBKS spectrum with Gamma = 0.21, n = 1 and sigma_8 = 0.8 at
z = 0, Gaussian smoothing radii log-spaced in cells, largest first), and draws seeded random
half-spectra and request traces for tests and the benchmark.  Both the library's tests and the
oracle's tests take their inputs from here; neither side's arithmetic lives here.
"""

import numpy as np

SIGMA8 = 0.8
GAMMA = 0.21
NS = 1.0


def radii_cells(n_radii, r_max, r_min):
    """n_radii radii log-spaced from r_max down to r_min (cells), strictly decreasing."""
    return np.geomspace(float(r_max), float(r_min), int(n_radii))


#: Plain-method workloads (name -> parameters).  Radii are in grid cells.
CONFIGS = {
    # 64^3 in 100 Mpc/h, 16 radii 20 -> 0.75 cells, float64 path.
    "c64_fp64": dict(n=64, box=100.0, n_radii=16, r_max=20.0, r_min=0.75, prec="fp64", seed=101),
    # 256^3 in 500 Mpc/h, 30 radii 60 -> 0.75 cells, float32 FFTs.
    "c256_fp32": dict(n=256, box=500.0, n_radii=30, r_max=60.0, r_min=0.75, prec="fp32", seed=102),
    # 512^3 in 1000 Mpc/h, 40 radii 60 -> 0.75 cells, float32 FFTs (roofline workload).
    "c512_fp32": dict(n=512, box=1000.0, n_radii=40, r_max=60.0, r_min=0.75, prec="fp32", seed=103),
    # the same workload on the float64 path
    "c512_fp64": dict(n=512, box=1000.0, n_radii=40, r_max=60.0, r_min=0.75, prec="fp64", seed=103),
    # 768^3 in 3072 Mpc/h, 45 radii 60 -> 0.75 cells, float32 FFTs (radix-3 sizes).
    "c768_fp32": dict(n=768, box=3072.0, n_radii=45, r_max=60.0, r_min=0.75, prec="fp32", seed=104),
    # serving-trace grid sizes with their own radix-3 factorisations (2 Mpc/h per cell, 32 radii),
    # float32 FFTs: parity cases
    "s192_fp32": dict(n=192, box=384.0, n_radii=32, r_max=60.0, r_min=0.75, prec="fp32", seed=105),
    "s384_fp32": dict(n=384, box=768.0, n_radii=32, r_max=60.0, r_min=0.75, prec="fp32", seed=106),
}

#: Serving trace: Poisson arrivals, grid sizes, 2 Mpc/h per cell, 24..40 radii, HBM budget.
SERVE = dict(rate_per_s=4.0, sizes=(128, 192, 256, 384, 512), mpc_per_cell=2.0,
             n_radii=(24, 40), r_max=60.0, r_min=0.75, hbm_budget=200e9, seed=4242,
             warmup=20, measured=300)


def config_radii(cfg):
    return radii_cells(cfg["n_radii"], cfg["r_max"], cfg["r_min"])


def random_real_field(n, seed, scale=1.0):
    """A seeded N^3 float64 Gaussian white-noise field."""
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal((n, n, n))


def random_half_spectrum(n, seed, scale=1.0):
    """Half spectrum (N, N, N/2+1) of a seeded real white-noise field (Hermitian-consistent)."""
    return np.fft.rfftn(random_real_field(n, seed, scale), axes=(0, 1, 2))


def serve_trace(seed=SERVE["seed"], count=None):
    """Seeded request trace: list of dicts (t_arrival, seed, n, box, radii) for the serving bench."""
    rng = np.random.default_rng(seed)
    total = SERVE["warmup"] + SERVE["measured"] if count is None else count
    t = 0.0
    out = []
    for _ in range(total):
        t += rng.exponential(1.0 / SERVE["rate_per_s"])
        n = int(rng.choice(SERVE["sizes"]))
        nr = int(rng.integers(SERVE["n_radii"][0], SERVE["n_radii"][1] + 1))
        out.append(dict(t=t, seed=int(rng.integers(1, 2 ** 62)), n=n,
                        box=SERVE["mpc_per_cell"] * n,
                        radii=radii_cells(nr, SERVE["r_max"], SERVE["r_min"])))
    return out
