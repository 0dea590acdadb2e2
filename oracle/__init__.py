"""FP64 CPU oracle for the PINOCCHIO collapse-time path (Monaco et al. 2013, arXiv:1305.1505).

This package is TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark import it; the product library never does, and it shares no code, table or
constant with the HIP path.

What it computes, in the paper's order (section "Collapse times"):

* ``field``       -- the Gaussian linear density field delta_l on an N^3 grid of side L,
                     normalised by sigma_8 (eq. deltal and the paragraph after it).
* ``hessian``     -- per Gaussian smoothing radius R, the deformation tensor T_ij = d_i d_j phi
                     with lap(phi) = delta_l (the "series of FFTs" per radius).
* ``collapse``    -- per grid point, the ellipsoidal collapse time from the truncated 3rd-order
                     LPT with the quasi-spherical correction, as the inverse collapse time
                     F = 1/D(t_coll) (eq. F).  The paper does not print the formula; the reading
                     used is stated in that module's header.
* ``run``         -- F_max and R_max over all radii (the trajectory maximum), and the closing
                     Zel'dovich and 2LPT displacement fields.
* ``lpt3``        -- the third-order displacement named in the conclusions, read as standard EdS
                     3LPT (longitudinal and transverse parts), pinned by the equations of motion.
* ``points``      -- deformation tensor, collapse times and displacements at single grid points
                     by direct summation, for grids too large for the full-grid functions.
* ``growth``      -- the growing mode D(z) of flat LambdaCDM and the sigma^2 radius ladder.
* ``fragment``    -- the sequential fragmentation of the collapsed medium into halos and
                     filaments (section "Fragmentation"), with the readings in its header.
* ``dft``         -- naive O(N^6) discrete Fourier transforms used to pin the library FFT.
* ``philox``      -- the Philox4x32-10 counter-based generator, written from its published
                     definition (Salmon, Moraes, Dror & Shaw, SC'11).

Everything is float64 NumPy/SciPy on CPU cores.
"""

from . import philox, spectrum, field, hessian, collapse, run, dft, metrics, lpt3, fragment  # noqa: F401
