// fam_debug.hip - test export: point values of the stage reconstruction.
//
// One thread per cell: the cell's moment stencil (cells i-1, i, i+1 in 1D, the
// 3x3 patch in 2D; ghost cells by periodic wrap or by copying the nearest
// interior cell), the coefficients of p_k from the same closed-form formulas
// that the stage kernels fold into their code (Sec. 2.4 and the appendices of
// reconstruction coefficients), and p_k evaluated in the scaled Legendre basis
// at the cell's flux points:
//   2D, 32 points: right face (1/2, eta_g), left face (-1/2, eta_g), top face
//       (xi_g, 1/2), bottom face (xi_g, -1/2) for g = 0..3, then the volume
//       nodes (xi_a, eta_b) at 16 + 4 b + a;
//   1D, 6 points: right face 1/2, left face -1/2, volume nodes xi_a at 2 + a;
// Gauss nodes in ascending order (-GS1, -GS0, GS0, GS1).  Output layout
// vals[((c * NP) + q) * cells + cell].  The positivity limiter is not applied.
#include <hip/hip_runtime.h>

#include "fam_device.h"
#include "fam_kernels.h"

namespace fam {
namespace {

constexpr int DBG_T = 256;

__device__ __forceinline__ int ghost_index(int i, int n, int bc) {
  if (bc == 0) return i < 0 ? i + n : (i >= n ? i - n : i);
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

__device__ __forceinline__ double gauss_node(int g) {
  return g == 0 ? -GS1 : g == 1 ? -GS0 : g == 2 ? GS0 : GS1;
}

template <int K>
__global__ void __launch_bounds__(DBG_T) dbg_recon2d_kernel(const double* __restrict__ U, Inst in, int nc,
                                                            double* __restrict__ vals) {
  constexpr int NCF = ncoef2d(K);
  const size_t cell = (size_t)blockIdx.x * DBG_T + threadIdx.x;
  if (cell >= in.plane) return;
  const int i = (int)(cell % in.nx), j = (int)(cell / in.nx);
  size_t pid[9];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a)
      pid[b * 3 + a] = (size_t)ghost_index(j - 1 + b, in.ny, in.bcy) * in.nx + ghost_index(i - 1 + a, in.nx, in.bcx);
  for (int c = 0; c < nc; ++c) {
    double u0[9], u1[9], u2[9];
#pragma unroll
    for (int l = 0; l < 9; ++l) {
      u0[l] = U[(size_t)(c * 3 + 0) * in.plane + pid[l]];
      u1[l] = U[(size_t)(c * 3 + 1) * in.plane + pid[l]];
      u2[l] = U[(size_t)(c * 3 + 2) * in.plane + pid[l]];
    }
    double cf[23];
    coeffs2d<K>(u0, u1, u2, cf, false);
#pragma unroll
    for (int q = 0; q < 32; ++q) {
      double x, y;
      if (q < 4) { x = 0.5; y = gauss_node(q); }
      else if (q < 8) { x = -0.5; y = gauss_node(q - 4); }
      else if (q < 12) { x = gauss_node(q - 8); y = 0.5; }
      else if (q < 16) { x = gauss_node(q - 12); y = -0.5; }
      else { x = gauss_node((q - 16) & 3); y = gauss_node((q - 16) >> 2); }
      double v = 0.0;
#pragma unroll
      for (int l = 0; l < NCF; ++l) v = fma(cf[l], leg(AX[l], x) * leg(AY[l], y), v);
      vals[(size_t)(c * 32 + q) * in.plane + cell] = v;
    }
  }
}

template <int K>
__global__ void __launch_bounds__(DBG_T) dbg_recon1d_kernel(const double* __restrict__ U, Inst in, int nc,
                                                            double* __restrict__ vals) {
  const int i = blockIdx.x * DBG_T + threadIdx.x;
  if (i >= in.nx) return;
  const int im = ghost_index(i - 1, in.nx, in.bcx), ip = ghost_index(i + 1, in.nx, in.bcx);
  for (int c = 0; c < nc; ++c) {
    const double* u0 = U + (size_t)(c * 2) * in.plane;
    const double* u1 = U + (size_t)(c * 2 + 1) * in.plane;
    double cf[6];
    coeffs1d<K>(u0[im], u0[i], u0[ip], u1[im], u1[i], u1[ip], cf);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const double x = q == 0 ? 0.5 : q == 1 ? -0.5 : gauss_node(q - 2);
      double v = 0.0;
#pragma unroll
      for (int l = 0; l < K; ++l) v = fma(cf[l], leg(l, x), v);
      vals[(size_t)(c * 6 + q) * in.plane + i] = v;
    }
  }
}

template <int K>
void launch_k(int dim, int nc, const double* U, const Inst& in, double* vals, hipStream_t s) {
  const unsigned blocks = (unsigned)((in.plane + DBG_T - 1) / DBG_T);
  if (dim == 1)
    hipLaunchKernelGGL((dbg_recon1d_kernel<K>), dim3(blocks), dim3(DBG_T), 0, s, U, in, nc, vals);
  else
    hipLaunchKernelGGL((dbg_recon2d_kernel<K>), dim3(blocks), dim3(DBG_T), 0, s, U, in, nc, vals);
}

}  // namespace

void launch_dbg_recon(int dim, int k, int nc, const double* U, const Inst& in, double* vals, hipStream_t s) {
  switch (k) {
    case 3: launch_k<3>(dim, nc, U, in, vals, s); break;
    case 4: launch_k<4>(dim, nc, U, in, vals, s); break;
    case 5: launch_k<5>(dim, nc, U, in, vals, s); break;
    default: launch_k<6>(dim, nc, U, in, vals, s); break;
  }
}

}  // namespace fam
