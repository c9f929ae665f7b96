// fam_char.h - local characteristic variables of the Euler equations for the
// stage reconstruction (the FAM5 alternative the paper times in Sec. 4.3,
// Table runtime-main Panel B).
//
// A cell maps its stencil moments to the characteristic variables of its own
// average with the left eigenvectors of the x-direction flux Jacobian there,
// reconstructs each field with the usual linear operator and maps the
// coefficients back with the right eigenvectors.  The reconstruction is linear,
// so the polynomial is the conservative-variable one up to rounding (Sec. 2.3);
// the variant exists for its cost.
#pragma once

#include "fam_device.h"

namespace fam {

// Textbook eigenvectors at the average a = (rho, rho u[, rho v], E): columns of R
// for u - c, u, u + c (2D: and the shear wave u), rows of L = R^{-1}.  With
// H = (E + p)/rho, q^2 = |velocity|^2, b1 = (gamma - 1)/c^2, b2 = b1 q^2 / 2.
template <int DIM>
__device__ __forceinline__ void char_basis_x(double gamma, const double* a, double (&L)[DIM + 2][DIM + 2],
                                             double (&R)[DIM + 2][DIM + 2]) {
  constexpr int NC = DIM + 2;
  const double inv = 1.0 / a[0];
  const double u = a[1] * inv;
  const double v = DIM == 2 ? a[2] * inv : 0.0;
  const double q2 = u * u + v * v;
  const double p = (gamma - 1.0) * (a[NC - 1] - 0.5 * a[0] * q2);
  const double c2 = gamma * p * inv;
  const double c = sqrt(c2);
  const double ic = 1.0 / c;
  const double H = (a[NC - 1] + p) * inv;
  const double b1 = (gamma - 1.0) / c2;
  const double b2 = 0.5 * b1 * q2;
  R[0][0] = 1.0;
  R[0][1] = 1.0;
  R[0][2] = 1.0;
  R[1][0] = u - c;
  R[1][1] = u;
  R[1][2] = u + c;
  R[NC - 1][0] = H - u * c;
  R[NC - 1][1] = 0.5 * q2;
  R[NC - 1][2] = H + u * c;
  L[0][0] = 0.5 * (b2 + u * ic);
  L[0][1] = -0.5 * (b1 * u + ic);
  L[0][NC - 1] = 0.5 * b1;
  L[1][0] = 1.0 - b2;
  L[1][1] = b1 * u;
  L[1][NC - 1] = -b1;
  L[2][0] = 0.5 * (b2 - u * ic);
  L[2][1] = -0.5 * (b1 * u - ic);
  L[2][NC - 1] = 0.5 * b1;
  if constexpr (DIM == 2) {
    R[2][0] = v;
    R[2][1] = v;
    R[2][2] = v;
    R[0][3] = 0.0;
    R[1][3] = 0.0;
    R[2][3] = 1.0;
    R[3][3] = v;
    L[0][2] = -0.5 * b1 * v;
    L[1][2] = b1 * v;
    L[2][2] = -0.5 * b1 * v;
    L[3][0] = -v;
    L[3][1] = 0.0;
    L[3][2] = 1.0;
    L[3][3] = 0.0;
  }
}

}  // namespace fam
