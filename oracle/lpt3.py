"""Third-order Lagrangian displacement (oracle; test infrastructure only).

The conclusions name 3LPT positions as the next extension of the closing displacements (after
2LPT, at about twice the cost of the Zel'dovich step) without printing its terms.  Reading: the
standard third-order Lagrangian perturbation theory of an Einstein-de Sitter growing mode, in the
convention of the other displacements here (lap(phi1) = delta, T1 = Hessian of phi1,
x = q + D psi1 + D^2 psi2 + D^3 psi3, psi1 = -grad(phi1), psi2 = -(3/7) grad(phi2) with
lap(phi2) = mu2(T1), T2 = Hessian of phi2):

    div  psi3 = mu3(T1) / 3 - (10/21) mu2(T1, T2),
    curl psi3 = C / 7,         C_i = eps_ijk (T1 T2)_jk,

with mu3 = det and the mixed invariant mu2(A, B) = ((tr A)(tr B) - tr(A B)) / 2.  In Fourier
space (integer wavevector f, box side L, k = 2 pi f / L):

    psi3(k) = i (L / 2 pi) / f^2 * ( -f S(k) + f x c(k) ),   S = rfftn(s), c = rfftn(C / 7),

s being the divergence above.  Both coefficients follow from the Lagrangian equations of motion
of a pressureless fluid in EdS (irrotational flow and the Poisson equation, order D^3); with them
a homogeneous sphere gets the third-order term -23/1701 delta^3 of its exact collapse and a
homogeneous cylinder -5/42 a^3 (the tests check the equations themselves on random band-limited
fields).  Like 2LPT: unsmoothed tensors, no dealiasing, and k = 0 and every Nyquist mode zeroed in
each spectrum (mu2, S, c).  psi3 is in Mpc/h at D = 1 and scales as D^3.
"""

import numpy as np

from . import hessian

# components of the symmetric tensors, in the order of hessian.COMPONENTS
_IDX = {(a, b): c for c, (a, b) in enumerate(hessian.COMPONENTS)}


def _entry(t6, a, b):
    return t6[_IDX[(a, b) if a <= b else (b, a)]]


def mu2(t6):
    """Second invariant (sum of the 2x2 principal minors) of a symmetric tensor field."""
    xx, xy, xz, yy, yz, zz = t6
    return xx * yy + xx * zz + yy * zz - xy * xy - xz * xz - yz * yz


def mu3(t6):
    """Determinant of a symmetric tensor field."""
    xx, xy, xz, yy, yz, zz = t6
    return xx * (yy * zz - yz * yz) - xy * (xy * zz - yz * xz) + xz * (xy * yz - yy * xz)


def mixed_mu2(a6, b6):
    """((tr A)(tr B) - tr(A B)) / 2 for symmetric A, B."""
    tra = a6[0] + a6[3] + a6[5]
    trb = b6[0] + b6[3] + b6[5]
    trab = sum(_entry(a6, i, j) * _entry(b6, j, i) for i in range(3) for j in range(3))
    return 0.5 * (tra * trb - trab)


def product_curl(a6, b6):
    """C_i = eps_ijk (A B)_jk for symmetric A, B: three real fields."""
    def ab(j, k):
        return sum(_entry(a6, j, l) * _entry(b6, l, k) for l in range(3))
    return [ab(1, 2) - ab(2, 1), ab(2, 0) - ab(0, 2), ab(0, 1) - ab(1, 0)]


def _masked_rfftn(x):
    n = x.shape[0]
    xk = np.fft.rfftn(x, axes=(0, 1, 2)) * hessian.nyquist_mask(n)
    xk[0, 0, 0] = 0.0
    return xk


def second_order_tensor(dk):
    """(T1, T2): the unsmoothed Hessians of phi1 (lap = delta) and of phi2 (lap = mu2(T1))."""
    t1 = hessian.deformation_tensor(dk, None)
    t2 = hessian.deformation_tensor(_masked_rfftn(mu2(t1)), None)
    return t1, t2


def third_order_sources(t1, t2):
    """(s, c): the divergence of psi3 and its curl, four real fields."""
    s = mu3(t1) / 3.0 - (10.0 / 21.0) * mixed_mu2(t1, t2)
    c = [ci / 7.0 for ci in product_curl(t1, t2)]
    return s, c


def lpt3_displacement(dk, box):
    """psi3 at D = 1, shape (3, N, N, N), Mpc/h."""
    n = dk.shape[0]
    s, c = third_order_sources(*second_order_tensor(dk))
    sk = _masked_rfftn(s)
    ck = [_masked_rfftn(ci) for ci in c]
    fx, fy, fz = hessian.freq_grids(n)
    f = (fx, fy, fz)
    f2 = fx ** 2 + fy ** 2 + fz ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = np.where(f2 > 0, 1.0 / np.where(f2 > 0, f2, 1.0), 0.0)
    g = 1j * inv * (box / (2.0 * np.pi))
    out = []
    for a in range(3):
        b, d = (a + 1) % 3, (a + 2) % 3
        spec = g * (-f[a] * sk + f[b] * ck[d] - f[d] * ck[b])
        out.append(np.fft.irfftn(spec, s=(n, n, n), axes=(0, 1, 2)))
    return np.stack(out)
