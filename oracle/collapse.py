"""Inverse collapse time F = 1/D(t_coll) per grid point (oracle side; test infrastructure only).

Section "Collapse times", eq. F.  The paper describes the model but does not print it: the
evolution of a mass element is that of an ellipsoid whose axes come from the deformation tensor;
with the growing mode D as the clock, ellipsoidal collapse is a truncation of 3rd-order LPT in
which all non-locality enters through the deformation tensor; collapse is the orbit crossing of
the first axis; and an empirical correction fixes the slow convergence of LPT for near-spherical
peaks, so that a sphere collapses at F = delta/delta_c.  The formula itself lives in a reference
that is not available, so this module implements the following READING (the GPU path implements
the same reading independently):

E3 -- truncated 3rd-order LPT along the first axis.
    lambda_1 >= lambda_2 >= lambda_3 are the eigenvalues of T, delta = tr T,
    mu2 = sum_{i<j} lambda_i lambda_j, mu3 = lambda_1 lambda_2 lambda_3.  The Lagrangian Poisson
    equation fixes the TRACE of each LPT order locally (2nd order: -(3/7) D^2 mu2; 3rd order:
    D^3 [mu3/3 - (10/63) delta mu2] once the second-order potential Hessian is taken isotropic);
    their traceless parts are non-local and are dropped, i.e. orders >= 2 are shared equally by
    the three axes.  The stretch of the first axis is then
        J1(D) = 1 - lambda_1 D - (mu2/7) D^2 + (mu3/9 - 10 delta mu2/189) D^3,
    and the first axis crosses orbits at the smallest D > 0 with J1(D) = 0.  With D = 1/F this is
    the largest positive real root of the monic cubic
        P(F) = F^3 - lambda_1 F^2 - (mu2/7) F + (mu3/9 - 10 delta mu2/189);
    if P has no positive root the element does not collapse on this scale and F = 0.
    For a sphere (lambda_i = delta/3) J1 is the 3rd-order expansion of the exact EdS spherical
    solution, 1 - x/3 - x^2/21 - 23 x^3/1701 with x = delta D, whose root is X3 = 2.05008...;
    for a plane (lambda_2 = lambda_3 = 0) it is the exact Zel'dovich solution F = lambda_1.

R1 -- quasi-spherical correction.
    F = F_E3 * [1 + (X3/delta_c - 1) * s],  s = clip(1 - 3 p/delta, 0, 1) for delta > 0 else 0,
    p = sqrt(tr(B^2)/6) with B = T - (delta/3) I, delta_c = (3/20)(12 pi)^(2/3) (EdS).
    s = 1 for a sphere, so F = delta/delta_c exactly; s = 0 for a plane, so F = lambda_1 is kept.

Arithmetic: float64 throughout.  lambda_1 comes from LAPACK (numpy.linalg.eigvalsh); the cubic's
largest real root is bracketed with the critical points of P (closed form) and found by
bisection.

Pins (tests/test_oracle_collapse.py): delta_c and the sphere series against the exact EdS
collapse, sphere and plane limits, homogeneity, the root finder against numpy.roots, and each
coefficient of P against the Zel'dovich, 2LPT and 3LPT oracles (which the equations of motion
pin).  Parity unpinned: the paper's own formula for anisotropic tensors (not printed), and the
R1 weight s between its sphere (s = 1) and plane (s = 0) values; a numerically integrated
homogeneous ellipsoid checks its size near the sphere (tests/test_oracle_ellipsoid.py: within
4% for 3p/delta <= 0.07), not its exact form.
"""

import numpy as np


def _eds_sphere_3lpt(x):
    return 1.0 - x / 3.0 - x * x / 21.0 - 23.0 * x ** 3 / 1701.0


def _bisect_scalar(fun, lo, hi, iters=200):
    flo = fun(lo)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if (fun(mid) > 0) == (flo > 0):
            lo, flo = mid, fun(mid)
        else:
            hi = mid
    return 0.5 * (lo + hi)


#: root of the 3rd-order EdS spherical series 1 - x/3 - x^2/21 - 23x^3/1701 (positive, in (1, 3))
X3 = _bisect_scalar(_eds_sphere_3lpt, 1.0, 3.0)
#: linear collapse threshold of the exact EdS spherical collapse, (3/20)(12 pi)^(2/3)
DELTA_C = 0.15 * (12.0 * np.pi) ** (2.0 / 3.0)
#: R1 strength: F_sphere = (delta/X3) * (X3/delta_c) = delta/delta_c
SPHERE_FACTOR = X3 / DELTA_C


def invariants(t6):
    """delta, mu2, mu3 and p of T from its six components (xx, xy, xz, yy, yz, zz), float64."""
    xx, xy, xz, yy, yz, zz = (np.asarray(c, dtype=np.float64) for c in t6)
    delta = xx + yy + zz
    mu2 = xx * yy + xx * zz + yy * zz - xy * xy - xz * xz - yz * yz
    mu3 = xx * (yy * zz - yz * yz) - xy * (xy * zz - yz * xz) + xz * (xy * yz - yy * xz)
    m = delta / 3.0
    bxx, byy, bzz = xx - m, yy - m, zz - m
    p = np.sqrt((bxx * bxx + byy * byy + bzz * bzz + 2.0 * (xy * xy + xz * xz + yz * yz)) / 6.0)
    return delta, mu2, mu3, p


def largest_eigenvalue(t6, chunk=1 << 20):
    """lambda_1 of each symmetric 3x3 T via LAPACK (numpy.linalg.eigvalsh), chunked."""
    comps = [np.asarray(c, dtype=np.float64).ravel() for c in t6]
    n = comps[0].size
    out = np.empty(n, dtype=np.float64)
    xx, xy, xz, yy, yz, zz = comps
    for s in range(0, n, chunk):
        e = slice(s, min(n, s + chunk))
        m = np.empty((e.stop - e.start, 3, 3))
        m[:, 0, 0], m[:, 0, 1], m[:, 0, 2] = xx[e], xy[e], xz[e]
        m[:, 1, 0], m[:, 1, 1], m[:, 1, 2] = xy[e], yy[e], yz[e]
        m[:, 2, 0], m[:, 2, 1], m[:, 2, 2] = xz[e], yz[e], zz[e]
        out[e] = np.linalg.eigvalsh(m)[:, 2]
    return out.reshape(np.shape(t6[0]))


def largest_real_root(a, b, c, iters=110):
    """Largest real root of x^3 + a x^2 + b x + c (arrays), by bracketing and bisection.

    P' = 3x^2 + 2a x + b.  If a^2 <= 3b, P is monotone and has one real root.  Otherwise its
    critical points are c1 < c2 (local max, local min): when P(c2) <= 0 the largest root lies in
    [c2, U] where P increases; when P(c2) > 0 the only real root lies below c1.  U is Cauchy's
    bound 1 + max(|a|, |b|, |c|), which exceeds every root's modulus.
    """
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)

    def poly(x):
        return ((x + a) * x + b) * x + c

    u = 1.0 + np.maximum(np.maximum(np.abs(a), np.abs(b)), np.abs(c))
    disc = a * a - 3.0 * b
    sq = np.sqrt(np.maximum(disc, 0.0))
    c1 = (-a - sq) / 3.0
    c2 = (-a + sq) / 3.0
    has_crit = disc > 0
    upper_branch = has_crit & (poly(c2) <= 0.0)
    lo = np.where(upper_branch, c2, -u)
    hi = np.where(upper_branch, u, np.where(has_crit, c1, u))
    # invariant: P(lo) <= 0 < P(hi), P monotone increasing on [lo, hi]
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        neg = poly(mid) <= 0.0
        lo = np.where(neg, mid, lo)
        hi = np.where(neg, hi, mid)
    return 0.5 * (lo + hi)


def cubic_coefficients(l1, delta, mu2, mu3):
    """(a, b, c) of P(F) = F^3 + a F^2 + b F + c, the E3 first-axis collapse cubic in F = 1/D."""
    return -l1, -mu2 / 7.0, mu3 / 9.0 - 10.0 * delta * mu2 / 189.0


def e3_inverse_time(l1, delta, mu2, mu3):
    """F_E3: largest positive real root of the E3 cubic, 0 where there is none."""
    a, b, c = cubic_coefficients(l1, delta, mu2, mu3)
    r = largest_real_root(a, b, c)
    return np.where(r > 0.0, r, 0.0)


def sphericity(delta, p):
    """s = clip(1 - 3p/delta, 0, 1) for delta > 0, 0 otherwise (1 = sphere, 0 = plane or worse)."""
    delta = np.asarray(delta, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        s = np.clip(1.0 - 3.0 * p / np.where(delta > 0, delta, 1.0), 0.0, 1.0)
    return np.where(delta > 0, s, 0.0)


def inverse_collapse_time(t6):
    """F = R1(E3) per point from the six deformation-tensor components (float64 array)."""
    delta, mu2, mu3, p = invariants(t6)
    l1 = largest_eigenvalue(t6)
    f_e3 = e3_inverse_time(l1, delta, mu2, mu3)
    return f_e3 * (1.0 + (SPHERE_FACTOR - 1.0) * sphericity(delta, p))
