"""FP64 CPU oracle for the compact FAM scheme with single-step OE.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path (the
HIP library and its Python binding) never imports, links or calls it, and this
package imports nothing from the product.

The oracle is plain, slow and written from the paper's definitions:

* ``oracle.exact``   - the reconstruction operators, obtained by solving the
                       moment-matching systems of Sec. 2.4 in exact rational
                       arithmetic and projecting in L2 (not from printed tables);
* ``oracle.physics`` - fluxes, wave speeds, Rusanov flux, 4-point Gauss rule;
* ``oracle.scheme``  - ghost cells, R(U) (eqs. 1dSemi, 11), SSP-RK3 (eqs. 3, 12),
                       OE (Prop. 2.1, eqs. 1dOE_system, 2dOE_system, Tables
                       sigma1d / sigma2d), CFL time step (Sec. 4);
* ``oracle.functional`` - the final-time functional used by the adjoint and its
                       reference gradient by reverse-mode differentiation of the
                       oracle's own step.

All floating-point work is FP64 (torch CPU tensors).  Where the paper is silent
or ambiguous the oracle takes one documented reading (one Lax-Friedrichs wave
speed per direction and stage: the maximum spectral radius over the cell
averages of the stage state; transmissive ghosts copy every moment; the k = 6
two-dimensional OE jumps use p_6 by default).  The optional positivity limiter
(``Config.pp``) is this project's design of the standard safeguard the paper
cites without stating it; it is pinned by invariants (identity on admissible
data, admissible and average-preserving output, tightness of the scaling).
The double Mach reflection boundary data (``Config.dmr``; time-dependent
ghost cells at each RK stage's time) follow the example's statement in Sec. 4
with cell-centre assignment at the shock.  The boundary data are pinned by the
physics they describe (the two states satisfy the Rankine-Hugoniot conditions of a
shock of normal speed 10, the top boundary switches where that shock meets the upper
edge, the wall ghosts are the quadrature moments of the mirrored field); the run
itself has no printed values (the paper prints only a figure), so its results are
pinned by the scheme's invariants only.
The local characteristic-variable stage reconstruction (``Config.char_vars``,
the FAM5 alternative timed in Sec. 4.3) transforms each cell's stencil with the
textbook left eigenvectors of the x-direction flux Jacobian at the cell's own
average and maps the coefficients back with the right eigenvectors (a reading:
the paper names neither the direction nor the averaging state); pinned by the
eigen-decomposition of the Jacobian and by Sec. 2.3's commutation remark.
"""
from .physics import NonPhysicalState, gauss4  # noqa: F401
from .scheme import Config, cfl_dt, oe, residual, rk3, rk3_stage, run, step  # noqa: F401
