// fam_device.h - device building blocks of the FAM step on gfx950.
//
// * Reconstruction coefficients: the closed-form solutions of the moment
//   systems, written out from the paper's appendices ("One-dimensional
//   reconstruction coefficients"; "Orthogonal basis functions and polynomial
//   coefficients for the 2D reconstruction").  Coefficients are in the local
//   orthogonal basis built from the scaled Legendre polynomials L0..L5 on
//   [-1/2, 1/2]; the 2D basis function phi^(l) is L_{ax[l]}(xi) L_{ay[l]}(eta).
// * Point evaluation at the 4-point Gauss-Legendre nodes exploits the parity of
//   L_m: values at +s and -s come from one even and one odd partial sum.
// * Physics: linear advection, Burgers, Euler (ideal gas).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fam {

// XCD-aware tile order.  The hardware hands consecutive workgroups to the chip's
// 8 XCDs in turn; tile xcd_tile(L, N) of workgroup L gives each XCD one
// contiguous range of the N tiles (row-major: neighbouring tiles of the same
// rows), so the cache lines that neighbouring tiles share stay in one L2.
// A bijection of [0, N) for any N; only where tiles run changes.
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_tile(int L, int N) {
  const int x = L % NXCD, slot = L / NXCD, q = N / NXCD, r = N % NXCD;
  return x * q + min(x, r) + slot;
}

// ---------------------------------------------------------------------------
// 4-point Gauss-Legendre rule on [-1/2, 1/2] (nodes +-GS0, +-GS1; weights sum
// to one).  Standard tabulated values of the rule on [-1, 1], halved.
// ---------------------------------------------------------------------------
constexpr double GS0 = 0.16999052179242813240;   // inner node
constexpr double GS1 = 0.43056815579702628761;   // outer node
constexpr double GW0 = 0.32607257743127307131;   // inner weight
constexpr double GW1 = 0.17392742256872692868;   // outer weight

// scaled Legendre polynomials of the paper's orthogonal bases
__host__ __device__ constexpr double leg(int m, double t) {
  return m == 0 ? 1.0
       : m == 1 ? t
       : m == 2 ? t * t - 1.0 / 12.0
       : m == 3 ? t * t * t - 3.0 / 20.0 * t
       : m == 4 ? t * t * t * t - 3.0 / 14.0 * t * t + 3.0 / 560.0
       :          t * t * t * t * t - 5.0 / 18.0 * t * t * t + 5.0 / 336.0 * t;
}

// node value L_m(s) for s in {GS0, GS1, 1/2}: index 0, 1, 2
__host__ __device__ constexpr double legn(int m, int which) {
  return leg(m, which == 0 ? GS0 : which == 1 ? GS1 : 0.5);
}

// 2D basis degrees (x-degree, y-degree) of phi^(0..22)
constexpr int AX[23] = {0, 1, 0, 2, 1, 0, 3, 2, 1, 0, 2, 4, 3, 1, 0, 5, 4, 3, 2, 1, 0, 4, 2};
constexpr int AY[23] = {0, 0, 1, 0, 1, 2, 0, 1, 2, 3, 2, 0, 1, 3, 4, 0, 1, 2, 3, 4, 5, 2, 4};

// number of basis terms of p_k (complete degree k-1): 6, 10, 15, 21
__host__ __device__ constexpr int ncoef2d(int k) { return k * (k + 1) / 2; }
__host__ __device__ constexpr int maxdeg(int k) { return k - 1; }

// ---------------------------------------------------------------------------
// 2D coefficients.  Patch cells 1..9 stored at index l-1 (row-major from
// (i-1, j-1)).  u0: averages (9); u1: x-moments; u2: y-moments (9 each, only
// the entries used by the system are read).  NCQ coefficients are produced:
// 11 (k = 3, 4: Q_4) or 23 (k = 5, 6: Q_6); callers keep the ones they need.
// ---------------------------------------------------------------------------
template <int K>
__host__ __device__ constexpr inline void coeffs2d(const double* u0, const double* u1, const double* u2,
                                                   double* c, bool full) {
  // indices 0..8 = patch cells I_1..I_9
  const double a1 = u0[0], a2 = u0[1], a3 = u0[2], a4 = u0[3], a5 = u0[4], a6 = u0[5],
               a7 = u0[6], a8 = u0[7], a9 = u0[8];
  if constexpr (K <= 4) {
    c[0] = a5;
    c[1] = 12.0 * u1[4];
    c[2] = 12.0 * u2[4];
    c[3] = 0.5 * (a4 - 2.0 * a5 + a6);
    c[4] = 0.25 * (a1 - a3 - a7 + a9);
    c[5] = 0.5 * (a2 - 2.0 * a5 + a8);
    if constexpr (K == 4) {
      c[6] = (5.0 / 11.0) * (a6 - a4) - (120.0 / 11.0) * u1[4];
      c[7] = 0.25 * (-a1 + 2.0 * a2 - a3 + a7 - 2.0 * a8 + a9);
      c[8] = 0.25 * (-a1 + a3 + 2.0 * a4 - 2.0 * a6 - a7 + a9);
      c[9] = (5.0 / 11.0) * (a8 - a2) - (120.0 / 11.0) * u2[4];
    }
  } else {
    const double b1 = u1[0], b3 = u1[2], b4 = u1[3], b5 = u1[4], b6 = u1[5], b7 = u1[6],
                 b9 = u1[8];
    const double e1 = u2[0], e2 = u2[1], e3 = u2[2], e5 = u2[4], e7 = u2[6], e8 = u2[7],
                 e9 = u2[8];
    const double dxx = a4 - 2.0 * a5 + a6, dyy = a2 - 2.0 * a5 + a8;
    const double cross = a1 - a3 - a7 + a9;
    c[0] = a5;
    c[1] = 12.0 * b5;
    c[2] = 12.0 * e5;
    c[3] = (73.0 / 56.0) * dxx + (135.0 / 28.0) * (b4 - b6);
    c[4] = (41.0 / 76.0) * cross + (33.0 / 19.0) * (b1 + b3 - b7 - b9 + e1 - e3 + e7 - e9);
    c[5] = (73.0 / 56.0) * dyy + (135.0 / 28.0) * (e2 - e8);
    c[6] = (595.0 / 324.0) * (a6 - a4) - (985.0 / 162.0) * (b4 + b6) - (2585.0 / 81.0) * b5;
    c[7] = (1695.0 / 2128.0) * (-a1 + 2.0 * a2 - a3 + a7 - 2.0 * a8 + a9) +
           (135.0 / 56.0) * (-b1 + b3 + b7 - b9) +
           (33.0 / 19.0) * (-e1 + 2.0 * e2 - e3 - e7 + 2.0 * e8 - e9);
    c[8] = (1695.0 / 2128.0) * (-a1 + a3 + 2.0 * a4 - 2.0 * a6 - a7 + a9) +
           (33.0 / 19.0) * (-b1 - b3 + 2.0 * b4 + 2.0 * b6 - b7 - b9) +
           (135.0 / 56.0) * (-e1 + e3 + e7 - e9);
    c[9] = (595.0 / 324.0) * (a8 - a2) - (985.0 / 162.0) * (e2 + e8) - (2585.0 / 81.0) * e5;
    const double lap2 = a1 - 2.0 * a2 + a3 - 2.0 * a4 + 4.0 * a5 - 2.0 * a6 + a7 - 2.0 * a8 + a9;
    c[10] = (59.0 / 56.0) * lap2 +
            (135.0 / 56.0) * (b1 - b3 - 2.0 * b4 + 2.0 * b6 + b7 - b9 + e1 - 2.0 * e2 + e3 - e7 +
                              2.0 * e8 - e9);
    c[11] = (5.0 / 8.0) * (-dxx) + (15.0 / 4.0) * (b6 - b4);
    c[12] = (5.0 / 38.0) * (-cross) + (30.0 / 19.0) * (-b1 - b3 + b7 + b9);
    c[13] = (5.0 / 38.0) * (-cross) + (30.0 / 19.0) * (-e1 + e3 - e7 + e9);
    c[14] = (5.0 / 8.0) * (-dyy) + (15.0 / 4.0) * (e8 - e2);
    if (K == 6 || full) {
      c[15] = (35.0 / 36.0) * (a4 - a6) + (77.0 / 18.0) * (b4 + b6) + (133.0 / 9.0) * b5;
      c[16] = (5.0 / 16.0) * (a1 - 2.0 * a2 + a3 - a7 + 2.0 * a8 - a9) +
              (15.0 / 8.0) * (b1 - b3 - b7 + b9);
      c[17] = (5.0 / 38.0) * (a1 - a3 - 2.0 * a4 + 2.0 * a6 + a7 - a9) +
              (30.0 / 19.0) * (b1 + b3 - 2.0 * b4 - 2.0 * b6 + b7 + b9);
      c[18] = (5.0 / 38.0) * (a1 - 2.0 * a2 + a3 - a7 + 2.0 * a8 - a9) +
              (30.0 / 19.0) * (e1 - 2.0 * e2 + e3 + e7 - 2.0 * e8 + e9);
      c[19] = (5.0 / 16.0) * (a1 - a3 - 2.0 * a4 + 2.0 * a6 + a7 - a9) +
              (15.0 / 8.0) * (e1 - e3 - e7 + e9);
      c[20] = (35.0 / 36.0) * (a2 - a8) + (77.0 / 18.0) * (e2 + e8) + (133.0 / 9.0) * e5;
    }
    if (full) {
      c[21] = (5.0 / 16.0) * (-lap2) + (15.0 / 8.0) * (-b1 + b3 + 2.0 * b4 - 2.0 * b6 - b7 + b9);
      c[22] = (5.0 / 16.0) * (-lap2) + (15.0 / 8.0) * (-e1 + 2.0 * e2 - e3 + e7 - 2.0 * e8 + e9);
    }
  }
}

// ---------------------------------------------------------------------------
// 1D coefficients (appendix "One-dimensional reconstruction coefficients").
// u0m, u00, u0p: averages of cells i-1, i, i+1; u1*: first moments.
// ---------------------------------------------------------------------------
template <int K>
__device__ __forceinline__ void coeffs1d(double u0m, double u00, double u0p, double u1m, double u10,
                                         double u1p, double* c) {
  c[0] = u00;
  c[1] = 12.0 * u10;
  if constexpr (K <= 4) {
    c[2] = 0.5 * (u0m - 2.0 * u00 + u0p);
    if constexpr (K == 4) c[3] = (5.0 / 11.0) * (u0p - u0m) - (120.0 / 11.0) * u10;
  } else {
    const double d2 = u0m - 2.0 * u00 + u0p;
    c[2] = (73.0 / 56.0) * d2 + (135.0 / 28.0) * (u1m - u1p);
    c[3] = (595.0 / 324.0) * (u0p - u0m) - (985.0 / 162.0) * (u1m + u1p) - (2585.0 / 81.0) * u10;
    c[4] = -(5.0 / 8.0) * d2 - (15.0 / 4.0) * (u1m - u1p);
    if constexpr (K == 6)
      c[5] = (35.0 / 36.0) * (u0m - u0p) + (77.0 / 18.0) * (u1m + u1p) + (133.0 / 9.0) * u10;
  }
}

// 1/x from the hardware reciprocal estimate refined by two Newton steps
// (relative error within a few units in the last place; not IEEE division)
__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// ---------------------------------------------------------------------------
// Physics
// ---------------------------------------------------------------------------
struct Advection {
  static constexpr int NC = 1;
  double ax, ay;
  __device__ __forceinline__ void flux(int d, const double* u, double* f) const {
    f[0] = (d == 0 ? ax : ay) * u[0];
  }
  __device__ __forceinline__ void flux2(const double* u, double* f1, double* f2) const {
    f1[0] = ax * u[0];
    f2[0] = ay * u[0];
  }
  __device__ __forceinline__ double speed(int d, const double* u, bool& bad) const {
    bad |= !(u[0] == u[0]);
    return fabs(d == 0 ? ax : ay);
  }
};

struct Burgers {
  static constexpr int NC = 1;
  double ax, ay;
  __device__ __forceinline__ void flux(int, const double* u, double* f) const {
    f[0] = 0.5 * u[0] * u[0];
  }
  __device__ __forceinline__ void flux2(const double* u, double* f1, double* f2) const {
    f1[0] = 0.5 * u[0] * u[0];
    f2[0] = f1[0];
  }
  __device__ __forceinline__ double speed(int, const double* u, bool& bad) const {
    bad |= !(u[0] == u[0]);
    return fabs(u[0]);
  }
};

// Euler in DIM dimensions: u = (rho, rho u [, rho v], E)
template <int DIM>
struct Euler {
  static constexpr int NC = DIM + 2;
  double g;
  __device__ __forceinline__ double pressure(const double* u, double inv_rho) const {
    double ke = u[1] * u[1];
    if constexpr (DIM == 2) ke += u[2] * u[2];
    return (g - 1.0) * (u[NC - 1] - 0.5 * ke * inv_rho);
  }
  __device__ __forceinline__ void flux(int d, const double* u, double* f) const {
    const double inv = rcp(u[0]);
    const double p = pressure(u, inv);
    const double vel = u[1 + d] * inv;
    f[0] = u[1 + d];
    f[1] = u[1] * vel;
    if constexpr (DIM == 2) f[2] = u[2] * vel;
    f[1 + d] += p;
    f[NC - 1] = (u[NC - 1] + p) * vel;
  }
  // both directional fluxes at one point (shared 1/rho and pressure)
  __device__ __forceinline__ void flux2(const double* u, double* f1, double* f2) const {
    const double inv = rcp(u[0]);
    const double p = pressure(u, inv);
    const double vx = u[1] * inv;
    const double vy = u[DIM == 2 ? 2 : 1] * inv;
    f1[0] = u[1];
    f1[1] = u[1] * vx + p;
    if constexpr (DIM == 2) {
      f1[2] = u[2] * vx;
      f2[0] = u[2];
      f2[1] = u[1] * vy;
      f2[2] = u[2] * vy + p;
      f2[3] = (u[3] + p) * vy;
    }
    f1[NC - 1] = (u[NC - 1] + p) * vx;
  }
  // spectral radius |u_d| + c at a cell average; flags rho <= 0, p <= 0, NaN
  __device__ __forceinline__ double speed(int d, const double* u, bool& bad) const {
    const double inv = 1.0 / u[0];
    const double p = pressure(u, inv);
    bad |= !(u[0] > 0.0) || !(p > 0.0);
    return fabs(u[1 + d] * inv) + sqrt(g * p * inv);
  }
};

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// max of non-negative doubles through their bit patterns (order-preserving)
__device__ __forceinline__ void atomic_max_nonneg(double* addr, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(addr), (unsigned long long)__double_as_longlong(v));
}

// ghost-cell index map: periodic wrap or transmissive clamp
__device__ __forceinline__ int ghost(int i, int n, int bc) {
  if (bc == 0) {
    i %= n;
    return i < 0 ? i + n : i;
  }
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

}  // namespace fam
