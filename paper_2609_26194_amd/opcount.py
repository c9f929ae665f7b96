"""Algorithmic FP64 operation count of one RK-stage launch per cell (2D Euler).

Counts one flop per add, subtract, multiply, divide or square root of the
algorithm (not per hardware instruction), for one cell of one stage:

* reconstruction: the linear map from the 23 (k = 5, 6) or 11 (k = 3, 4) stencil
  moments to the P coefficients of p_k in the orthogonal basis; the coefficient
  formulas of the paper's 2D appendix have NNZ nonzero weights, costing
  2 NNZ - P flops per component (NNZ = 13, 31, 114, 168 for k = 3..6);
* evaluation at the 32 flux points (16 face, 16 volume): contraction over the
  y-degree at the three node magnitudes (GS0, GS1, 1/2) with even/odd splitting,
  3 P multiply-adds, then per point (k multiply-adds plus one combine) per
  component;
* fluxes: 16 volume points with f1 and f2 (shared 1/rho and pressure: 20 flops),
  the 16 face traces of a cell's two owned faces with one flux each (14 flops),
  8 Rusanov combinations (6 flops per component), 4-point face quadratures and
  4x4 volume quadratures (2 flops per multiply-add);
* residual R0, R1, R2 (16 flops per component) and the Shu-Osher update
  (15 flops per component).
"""
NNZ_2D = {3: 13, 4: 31, 5: 114, 6: 168}


def stage_flops(k, ncomp=4):
    P = k * (k + 1) // 2
    rec = 2 * NNZ_2D[k] - P
    contract = 3 * P * 2
    points = 32 * (2 * k + 1)
    per_comp = rec + contract + points
    vol_flux = 16 * 20
    vol_quad = 16 * ncomp * 2 * 2
    face_flux = 16 * 14
    rusanov = 8 * ncomp * 6
    face_quad = 8 * ncomp * 2 * 2
    update = ncomp * (16 + 15)
    return ncomp * per_comp + vol_flux + vol_quad + face_flux + rusanov + face_quad + update


def oe_flops(k, ncomp=4):
    """Per cell: face-centre values (4 per component), jumps, 3x3 sums/maxima, beta, delta."""
    P = k * (k + 1) // 2
    rec = 2 * NNZ_2D[k] - P
    centres = 4 * 2 * k
    denom = 9 + 9 * 2 + 9        # sum, |u - S| and max, max |u|
    speeds = 9 * 12              # spectral radii at 9 averages (x and y)
    return ncomp * (rec + centres + 6 + denom + 4) + speeds + 10
