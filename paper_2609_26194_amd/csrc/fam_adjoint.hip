// fam_adjoint.hip - hand-written reverse mode of the 2D Euler FAM step.
//
// Forward step (fixed dt):  U1 = U0 + dt R(U0);  U2 = 3/4 U0 + 1/4 (U1 + dt R(U1));
// Un = 1/3 U0 + 2/3 (U2 + dt R(U2));  U' = OE(Un)                       (eq. 12)
// Reverse step, given lam = dJ/dU':
//   lamN = OE^T(Un) lam
//   lam2 = 2/3 lamN + R^T(U2) (2/3 dt lamN),   lam0  = 1/3 lamN
//   lam1 = 1/4 lam2 + R^T(U1) (1/4 dt lam2),   lam0 += 3/4 lam2
//   lam0 += lam1 + R^T(U0) (dt lam1)
//
// R^T(U) mu is assembled in gather form, without atomics:
//  (1) adj_coef: for every cell, the adjoint of its reconstruction coefficients.
//      A face flux F = 1/2 (f(uL) + f(uR)) - 1/2 alpha (uR - uL) has dF/duL =
//      1/2 J(uL) + alpha/2 and dF/duR = 1/2 J(uR) - alpha/2, so each cell needs
//      only its own traces and the neighbours' mu.  The volume terms use the
//      flux Jacobians at the 16 Gauss points.  Each cell also adds its share of
//      dJ/dalpha (alpha is the global Lax-Friedrichs speed of the stage state).
//  (2) adj_gather: lam(q) += sum over the 3x3 cells n around q of the transposed
//      reconstruction (compile-time weights) applied to n's coefficient adjoint.
//  (3) alpha route: dJ/dalpha times the gradient of the spectral radius at the
//      cell average that attains the maximum (first index on ties).
// OE^T (Type II) in three gather passes: per cell, the derivative of the damping
// factor with respect to the jump sums, the denominators and the wave-speed
// bounds; per face, the jump adjoints; per cell, the transposed face-centre
// functionals and the denominator / wave-speed routes over the 3x3 patch.
// Non-smooth points: |x|' = sign(x) with sign(0) = 0; maxima pass the derivative
// to the first maximal entry; the zero-denominator branch has zero derivative.
//
// Checkpointing: the forward pass stores U every `checkpoint_every` steps; each
// segment is recomputed from its checkpoint, keeping U0, U1, U2, Un of its
// steps, and then swept in reverse.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <new>
#include <vector>

#include "../../include/fam.h"
#include "fam_ctx.h"
#include "fam_device.h"
#include "fam_eval.h"
#include "fam_kernels.h"

namespace fam {

constexpr int ADJ_TX = 16, ADJ_TY = 16, ADJ_T = ADJ_TX * ADJ_TY;

struct AdjMesh {
  int nx, ny;
  size_t plane;
  double dx, dy, gamma;
};

__device__ __forceinline__ size_t wrap_idx(const AdjMesh& m, int i, int j) {
  i %= m.nx;
  if (i < 0) i += m.nx;
  j %= m.ny;
  if (j < 0) j += m.ny;
  return (size_t)j * m.nx + i;
}

// stencil of component c around cell (i, j) (periodic)
template <int K>
__device__ __forceinline__ void gstencil(const double* __restrict__ U, const AdjMesh& m, int c, int i, int j,
                                         double (&u0)[9], double (&u1)[9], double (&u2)[9]) {
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int l = b * 3 + a;
      const size_t id = wrap_idx(m, i - 1 + a, j - 1 + b);
      u0[l] = U[(c * 3 + 0) * m.plane + id];
      const bool x_used = (K >= 5) ? (l != 1 && l != 7) : (l == 4);
      const bool y_used = (K >= 5) ? (l != 3 && l != 5) : (l == 4);
      u1[l] = x_used ? U[(c * 3 + 1) * m.plane + id] : 0.0;
      u2[l] = y_used ? U[(c * 3 + 2) * m.plane + id] : 0.0;
    }
}

// out = J_d(u)^T w for the 2D Euler flux in direction d
__device__ __forceinline__ void euler_jt(int d, double g, const double* u, const double* w, double* out) {
  const double inv = 1.0 / u[0];
  const double vx = u[1] * inv, vy = u[2] * inv;
  const double q2 = vx * vx + vy * vy;
  const double g1 = g - 1.0;
  const double p = g1 * (u[3] - 0.5 * u[0] * q2);
  const double H = (u[3] + p) * inv;
  const double k = 0.5 * g1 * q2;
  if (d == 0) {
    out[0] = (-vx * vx + k) * w[1] - vx * vy * w[2] + vx * (k - H) * w[3];
    out[1] = w[0] + (3.0 - g) * vx * w[1] + vy * w[2] + (H - g1 * vx * vx) * w[3];
    out[2] = -g1 * vy * w[1] + vx * w[2] - g1 * vx * vy * w[3];
    out[3] = g1 * w[1] + g * vx * w[3];
  } else {
    out[0] = -vx * vy * w[1] + (-vy * vy + k) * w[2] + vy * (k - H) * w[3];
    out[1] = vy * w[1] - g1 * vx * w[2] - g1 * vx * vy * w[3];
    out[2] = w[0] + vx * w[1] + (3.0 - g) * vy * w[2] + (H - g1 * vy * vy) * w[3];
    out[3] = g1 * w[2] + g * vy * w[3];
  }
}

// gradient of |u_d| + sqrt(g p / rho) with respect to (rho, m, n, E)
__device__ __forceinline__ void speed_grad(int d, double g, const double* u, double* gr) {
  const double inv = 1.0 / u[0];
  const double vx = u[1] * inv, vy = u[2] * inv;
  const double g1 = g - 1.0;
  const double p = g1 * (u[3] - 0.5 * (u[1] * u[1] + u[2] * u[2]) * inv);
  const double c = sqrt(g * p * inv);
  const double f = g / (2.0 * c * u[0]);
  const double vd = d == 0 ? vx : vy;
  const double s = vd > 0.0 ? 1.0 : (vd < 0.0 ? -1.0 : 0.0);
  gr[0] = -s * vd * inv + f * (0.5 * g1 * (vx * vx + vy * vy) - p * inv);
  gr[1] = f * (-g1 * vx);
  gr[2] = f * (-g1 * vy);
  gr[3] = f * g1;
  gr[1 + d] += s * inv;
}

__device__ __forceinline__ double sgn(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

// phi_l at (sx * node(gx), sy * node(gy))
template <int L>
__device__ __forceinline__ constexpr double phi_at(int gx, double sx, int gy, double sy) {
  double px = legn(AX[L], gx), py = legn(AY[L], gy);
  if (AX[L] % 2) px *= sx;
  if (AY[L] % 2) py *= sy;
  return px * py;
}

template <int NCF, int... L>
__device__ __forceinline__ void add_phi(double* abar, double ub, int gx, double sx, int gy, double sy,
                                        std::integer_sequence<int, L...>) {
  ((abar[L] = fma(ub, phi_at<L>(gx, sx, gy, sy), abar[L])), ...);
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
  return s;
}

// ---------------------------------------------------------------------------
// (1) coefficient adjoints of R^T(U) mu, mu = scale * lam_out
// ---------------------------------------------------------------------------
template <int K>
__global__ void __launch_bounds__(ADJ_T) adj_coef_kernel(AdjMesh m, const double* __restrict__ U,
                                                         const double* __restrict__ lam, double scale,
                                                         const double* __restrict__ alpha,
                                                         double* __restrict__ abar, double* __restrict__ partial) {
  constexpr int NC = 4, NCF = ncoef2d(K), MD = maxdeg(K);
  __shared__ double red[ADJ_T / 64];
  const int i = blockIdx.x * ADJ_TX + (threadIdx.x % ADJ_TX);
  const int j = blockIdx.y * ADJ_TY + (threadIdx.x / ADJ_TX);
  const bool inside = i < m.nx && j < m.ny;
  double pax = 0.0, pay = 0.0;
  if (inside) {
    const double g = m.gamma;
    const double ax = alpha[0], ay = alpha[1];
    const double idx_ = 1.0 / m.dx, idy = 1.0 / m.dy;
    double cf[NC][NCF];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double u0[9], u1[9], u2[9];
      gstencil<K>(U, m, c, i, j, u0, u1, u2);
      double tmp[23];
      coeffs2d<K>(u0, u1, u2, tmp, false);
#pragma unroll
      for (int l = 0; l < NCF; ++l) cf[c][l] = tmp[l];
    }
    // mu of this cell and of its four neighbours: [self, left, right, bottom, top][c][m]
    double mu[5][NC][3];
    const size_t ids[5] = {wrap_idx(m, i, j), wrap_idx(m, i - 1, j), wrap_idx(m, i + 1, j),
                           wrap_idx(m, i, j - 1), wrap_idx(m, i, j + 1)};
#pragma unroll
    for (int n = 0; n < 5; ++n)
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int r = 0; r < 3; ++r) mu[n][c][r] = scale * lam[(c * 3 + r) * m.plane + ids[n]];
    double ab[NC][NCF];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int l = 0; l < NCF; ++l) ab[c][l] = 0.0;
    using Seq = std::make_integer_sequence<int, NCF>;

    // volume: V1 = sum w f1(u), V2 = sum w f2(u); R1 += V1/dx, R2 += V2/dy
#pragma unroll
    for (int qy = 0; qy < 4; ++qy)
#pragma unroll
      for (int qx = 0; qx < 4; ++qx) {
        double u[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          double E[MD + 1][4], O[MD + 1][3];
          contract_y<NCF, MD>(cf[c], E, O);
          u[c] = eval_pt<MD>(E, O, qnode(qx), qsign(qx), qnode(qy), qsign(qy));
        }
        const double w = qw(qx) * qw(qy);
        double w1[NC], w2[NC], o1[NC], o2[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          w1[c] = w * mu[0][c][1] * idx_;
          w2[c] = w * mu[0][c][2] * idy;
        }
        euler_jt(0, g, u, w1, o1);
        euler_jt(1, g, u, w2, o2);
#pragma unroll
        for (int c = 0; c < NC; ++c)
          add_phi<NCF>(ab[c], o1[c] + o2[c], qnode(qx), qsign(qx), qnode(qy), qsign(qy), Seq{});
      }

    // faces: side 0 right (cell is left state), 1 left (cell is right state),
    //        2 top (cell is lower state), 3 bottom (cell is upper state)
#pragma unroll
    for (int side = 0; side < 4; ++side) {
      const bool xf = side < 2;
      const bool own_left = (side == 0 || side == 2);
      const int nb = side == 0 ? 2 : side == 1 ? 1 : side == 2 ? 4 : 3;   // neighbour slot in mu[]
      double Badj[NC], Tadj[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        // mu of the lower/left cell (L) and upper/right cell (R) of this face
        const double* muL = own_left ? mu[0][c] : mu[nb][c];
        const double* muR = own_left ? mu[nb][c] : mu[0][c];
        if (xf) {
          Badj[c] = -muL[0] * idx_ - 0.5 * muL[1] * idx_ + muR[0] * idx_ - 0.5 * muR[1] * idx_;
          Tadj[c] = -muL[2] * idx_ + muR[2] * idx_;
        } else {
          Badj[c] = -muL[0] * idy - 0.5 * muL[2] * idy + muR[0] * idy - 0.5 * muR[2] * idy;
          Tadj[c] = -muL[1] * idy + muR[1] * idy;
        }
      }
      const double al = xf ? ax : ay;
      const double sgn_side = own_left ? 1.0 : -1.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double u[NC];
        const int gxn = xf ? 2 : qnode(q), gyn = xf ? qnode(q) : 2;
        const double sxv = xf ? (side == 0 ? 1.0 : -1.0) : qsign(q);
        const double syv = xf ? qsign(q) : (side == 2 ? 1.0 : -1.0);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          double E[MD + 1][4], O[MD + 1][3];
          contract_y<NCF, MD>(cf[c], E, O);
          u[c] = eval_pt<MD>(E, O, gxn, sxv, gyn, syv);
        }
        double Fh[NC], jt[NC];
        double dotFu = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          Fh[c] = qw(q) * Badj[c] + qw(q) * qx(q) * Tadj[c];
          dotFu = fma(Fh[c], u[c], dotFu);
        }
        double half[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) half[c] = 0.5 * Fh[c];
        euler_jt(xf ? 0 : 1, g, u, half, jt);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const double ub = jt[c] + sgn_side * 0.5 * al * Fh[c];
          add_phi<NCF>(ab[c], ub, gxn, sxv, gyn, syv, Seq{});
        }
        if (xf)
          pax += sgn_side * 0.5 * dotFu;
        else
          pay += sgn_side * 0.5 * dotFu;
      }
    }
    const size_t id = ids[0];
    const size_t cells = m.plane;
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int l = 0; l < NCF; ++l) abar[(size_t)(c * NCF + l) * cells + id] = ab[c][l];
  }
  const double sx = block_sum(pax, red);
  const double sy = block_sum(pay, red);
  if (threadIdx.x == 0) {
    const int b = blockIdx.y * gridDim.x + blockIdx.x;
    partial[2 * b] = sx;
    partial[2 * b + 1] = sy;
  }
}

// ---------------------------------------------------------------------------
// (2) gather: out(q) = [out(q)] + b lam_out(q) + sum_n RT(q in n) abar_n
// ---------------------------------------------------------------------------
template <int K, int IN>
__device__ __forceinline__ double rt_apply(const double* a) {
  return rt_dot<K, IN>(a, std::make_integer_sequence<int, ncoef2d(K)>{});
}

template <int K, int DX, int DY>
__device__ __forceinline__ void gather_one(const AdjMesh& m, int i, int j, const double* __restrict__ abar,
                                           double (&acc)[4][3]) {
  constexpr int NCF = ncoef2d(K);
  constexpr int L9 = (1 - DX) + 3 * (1 - DY);   // position of q in the patch of n = q + (DX, DY)
  const size_t id = wrap_idx(m, i + DX, j + DY);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double a[NCF];
#pragma unroll
    for (int l = 0; l < NCF; ++l) a[l] = abar[(size_t)(c * NCF + l) * m.plane + id];
    acc[c][0] += rt_apply<K, L9>(a);
    acc[c][1] += rt_apply<K, 9 + L9>(a);
    acc[c][2] += rt_apply<K, 18 + L9>(a);
  }
}

template <int K>
__global__ void __launch_bounds__(ADJ_T) adj_gather_kernel(AdjMesh m, const double* __restrict__ abar,
                                                           const double* __restrict__ lam_out, double b,
                                                           double* __restrict__ out, int accumulate) {
  const int i = blockIdx.x * ADJ_TX + (threadIdx.x % ADJ_TX);
  const int j = blockIdx.y * ADJ_TY + (threadIdx.x / ADJ_TX);
  if (i >= m.nx || j >= m.ny) return;
  double acc[4][3] = {};
  gather_one<K, -1, -1>(m, i, j, abar, acc);
  gather_one<K, 0, -1>(m, i, j, abar, acc);
  gather_one<K, 1, -1>(m, i, j, abar, acc);
  gather_one<K, -1, 0>(m, i, j, abar, acc);
  gather_one<K, 0, 0>(m, i, j, abar, acc);
  gather_one<K, 1, 0>(m, i, j, abar, acc);
  gather_one<K, -1, 1>(m, i, j, abar, acc);
  gather_one<K, 0, 1>(m, i, j, abar, acc);
  gather_one<K, 1, 1>(m, i, j, abar, acc);
  const size_t id = (size_t)j * m.nx + i;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const size_t k = (c * 3 + r) * m.plane + id;
      const double v = b * lam_out[k] + acc[c][r];
      out[k] = accumulate ? out[k] + v : v;
    }
}

__global__ void adj_axpy_kernel(size_t n, double a, const double* __restrict__ x, double* __restrict__ y,
                                int accumulate) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
    y[k] = accumulate ? y[k] + a * x[k] : a * x[k];
}

// ---------------------------------------------------------------------------
// (3) alpha: argmax of the spectral radii at the averages and its route
// ---------------------------------------------------------------------------
constexpr int ALPHA_BLOCKS = 1024;   // partials of the argmax pass
constexpr int RED_T = 1024;          // threads of the single-block final reductions

// (v, i) pairs: larger v wins, equal v -> smaller i (first maximal cell)
__device__ __forceinline__ void argmax_merge(double& v, int& i, double v2, int i2) {
  if (v2 > v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
}

__device__ __forceinline__ void wave_argmax(double& v, int& i) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) argmax_merge(v, i, __shfl_xor(v, off, 64), __shfl_xor(i, off, 64));
}

// block partials of (max speed, first argmax) in x and y
__global__ void __launch_bounds__(256) adj_alpha_part_kernel(AdjMesh m, const double* __restrict__ U,
                                                             double* __restrict__ pv, int* __restrict__ pi) {
  __shared__ double sv[2][4];
  __shared__ int si[2][4];
  const Euler<2> ph{m.gamma};
  bool bad = false;
  double vx = -1.0, vy = -1.0;
  int ix = INT_MAX, iy = INT_MAX;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < m.plane; k += (size_t)gridDim.x * blockDim.x) {
    double a[4] = {U[k], U[3 * m.plane + k], U[6 * m.plane + k], U[9 * m.plane + k]};
    argmax_merge(vx, ix, ph.speed(0, a, bad), (int)k);
    argmax_merge(vy, iy, ph.speed(1, a, bad), (int)k);
  }
  wave_argmax(vx, ix);
  wave_argmax(vy, iy);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sv[0][w] = vx; si[0][w] = ix;
    sv[1][w] = vy; si[1][w] = iy;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int d = threadIdx.x;
    double v = sv[d][0];
    int i = si[d][0];
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q) argmax_merge(v, i, sv[d][q], si[d][q]);
    pv[2 * blockIdx.x + d] = v;
    pi[2 * blockIdx.x + d] = i;
  }
}

__global__ void __launch_bounds__(RED_T) adj_alpha_final_kernel(const double* __restrict__ pv,
                                                                const int* __restrict__ pi, int nparts,
                                                                double* smax, int* sidx) {
  __shared__ double sv[2][RED_T / 64];
  __shared__ int si[2][RED_T / 64];
  double v[2] = {-1.0, -1.0};
  int ix[2] = {INT_MAX, INT_MAX};
  for (int b = threadIdx.x; b < nparts; b += blockDim.x)
    for (int d = 0; d < 2; ++d) argmax_merge(v[d], ix[d], pv[2 * b + d], pi[2 * b + d]);
  for (int d = 0; d < 2; ++d) {
    wave_argmax(v[d], ix[d]);
    if ((threadIdx.x & 63) == 0) {
      sv[d][threadIdx.x >> 6] = v[d];
      si[d][threadIdx.x >> 6] = ix[d];
    }
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int d = threadIdx.x;
    double vv = sv[d][0];
    int ii = si[d][0];
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q) argmax_merge(vv, ii, sv[d][q], si[d][q]);
    smax[d] = vv < 0.0 ? 0.0 : vv;
    sidx[d] = ii;
  }
}

// d alpha_d / d U at the first maximal cell, times the summed alpha adjoints
__global__ void __launch_bounds__(RED_T) adj_alpha_route_kernel(AdjMesh m, const double* __restrict__ U,
                                                                const double* __restrict__ partial, int nblocks,
                                                                const int* sidx, double* __restrict__ out) {
  __shared__ double red[2][RED_T / 64];
  double ab[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
    ab[0] += partial[2 * b];
    ab[1] += partial[2 * b + 1];
  }
  for (int d = 0; d < 2; ++d) {
    ab[d] = wave_sum(ab[d]);
    if ((threadIdx.x & 63) == 0) red[d][threadIdx.x >> 6] = ab[d];
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int d = 0; d < 2; ++d) {
    double tot = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) tot += red[d][q];
    if (sidx[d] < 0 || (size_t)sidx[d] >= m.plane) continue;   // no finite maximum
    const size_t k = (size_t)sidx[d];
    double a[4] = {U[k], U[3 * m.plane + k], U[6 * m.plane + k], U[9 * m.plane + k]};
    double gr[4];
    speed_grad(d, m.gamma, a, gr);
    for (int c = 0; c < 4; ++c) out[(c * 3) * m.plane + k] += tot * gr[c];
  }
}

// ---------------------------------------------------------------------------
// OE adjoint (Type II)
// ---------------------------------------------------------------------------
// per-cell record: [0..3] jump at the left face, [4..7] jump at the bottom face,
// [8..11] dJ/dJx, [12..15] dJ/dJy, [16..19] dJ/dD, [20..23] sign(u_p* - S),
// [24..27] p* (patch index), 28 dJ/dbeta_x, 29 dJ/dbeta_y, 30, 31 argmax patch index
constexpr int OES = 32;

template <int K>
__device__ __forceinline__ void centres_at(const double* __restrict__ U, const AdjMesh& m, int c, int i, int j,
                                           double (&out)[4]) {
  double u0[9], u1[9], u2[9];
  gstencil<K>(U, m, c, i, j, u0, u1, u2);
  double u[27];
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    u[l] = u0[l];
    u[9 + l] = u1[l];
    u[18 + l] = u2[l];
  }
  using Seq = std::make_integer_sequence<int, 27>;
  out[0] = centre_dot<K, false, 0>(u, Seq{});
  out[1] = centre_dot<K, false, 1>(u, Seq{});
  out[2] = centre_dot<K, false, 2>(u, Seq{});
  out[3] = centre_dot<K, false, 3>(u, Seq{});
}

template <int K>
__global__ void __launch_bounds__(ADJ_T) oe_adj_a_kernel(AdjMesh m, const double* __restrict__ Un,
                                                         const double* __restrict__ lam, double dt, double gk,
                                                         double* __restrict__ lamN, double* __restrict__ os) {
  const int i = blockIdx.x * ADJ_TX + (threadIdx.x % ADJ_TX);
  const int j = blockIdx.y * ADJ_TY + (threadIdx.x / ADJ_TX);
  if (i >= m.nx || j >= m.ny) return;
  const Euler<2> ph{m.gamma};
  bool bad = false;
  const size_t id = (size_t)j * m.nx + i;
  double Jx[4], Jy[4], jL[4], jB[4], D[4], eps[4], sD[4];
  int pD[4];
  for (int c = 0; c < 4; ++c) {
    double own[4], lf[4], rt[4], bt[4], tp[4];
    centres_at<K>(Un, m, c, i, j, own);
    centres_at<K>(Un, m, c, i - 1, j, lf);
    centres_at<K>(Un, m, c, i + 1, j, rt);
    centres_at<K>(Un, m, c, i, j - 1, bt);
    centres_at<K>(Un, m, c, i, j + 1, tp);
    jL[c] = own[1] - lf[0];
    const double jR = rt[1] - own[0];
    jB[c] = own[3] - bt[2];
    const double jT = tp[3] - own[2];
    Jx[c] = fabs(jL[c]) + fabs(jR);
    Jy[c] = fabs(jB[c]) + fabs(jT);
    double v[9];
    for (int b = 0; b < 3; ++b)
      for (int a = 0; a < 3; ++a) v[b * 3 + a] = Un[(c * 3) * m.plane + wrap_idx(m, i - 1 + a, j - 1 + b)];
    double S = 0.0, mabs = 0.0;
    for (int p = 0; p < 9; ++p) {
      S += v[p];
      mabs = fmax(mabs, fabs(v[p]));
    }
    double best = -1.0;
    int arg = 0;
    for (int p = 0; p < 9; ++p) {
      const double d = fabs(v[p] - S);
      if (d > best) {
        best = d;
        arg = p;
      }
    }
    D[c] = best;
    pD[c] = arg;
    sD[c] = sgn(v[arg] - S);
    eps[c] = 1e-14 * fmax(mabs, 1.0);
  }
  // wave-speed bounds over the patch (first maximal entry)
  double bx = -1.0, by = -1.0;
  int abx = 0, aby = 0;
  for (int p = 0; p < 9; ++p) {
    const size_t k = wrap_idx(m, i - 1 + p % 3, j - 1 + p / 3);
    double a[4] = {Un[k], Un[3 * m.plane + k], Un[6 * m.plane + k], Un[9 * m.plane + k]};
    const double sx = ph.speed(0, a, bad), sy = ph.speed(1, a, bad);
    if (sx > bx) { bx = sx; abx = p; }
    if (sy > by) { by = sy; aby = p; }
  }
  // sigma per component and its maximum (first maximal component)
  double sgx = -1.0, sgy = -1.0;
  int cx = 0, cy = 0;
  double sigx[4], sigy[4];
  for (int c = 0; c < 4; ++c) {
    const bool small = D[c] < eps[c];
    sigx[c] = small ? 0.0 : gk * Jx[c] / D[c];
    sigy[c] = small ? 0.0 : gk * Jy[c] / D[c];
    if (sigx[c] > sgx) { sgx = sigx[c]; cx = c; }
    if (sigy[c] > sgy) { sgy = sigy[c]; cy = c; }
  }
  const double kx = dt / m.dx, ky = dt / m.dy;
  const double delta = exp(-bx * kx * sgx - by * ky * sgy);
  double dbar = 0.0;
  for (int c = 0; c < 4; ++c) {
    const double l0 = lam[(c * 3) * m.plane + id], l1 = lam[(c * 3 + 1) * m.plane + id],
                 l2 = lam[(c * 3 + 2) * m.plane + id];
    lamN[(c * 3) * m.plane + id] = l0;
    lamN[(c * 3 + 1) * m.plane + id] = delta * l1;
    lamN[(c * 3 + 2) * m.plane + id] = delta * l2;
    dbar += l1 * Un[(c * 3 + 1) * m.plane + id] + l2 * Un[(c * 3 + 2) * m.plane + id];
  }
  const double tbar = -delta * dbar;
  const double bbx = tbar * kx * sgx, bby = tbar * ky * sgy;
  const double sbx = tbar * kx * bx, sby = tbar * ky * by;
  double Jxb[4] = {0, 0, 0, 0}, Jyb[4] = {0, 0, 0, 0}, Db[4] = {0, 0, 0, 0};
  if (!(D[cx] < eps[cx])) {
    Jxb[cx] = gk * sbx / D[cx];
    Db[cx] += -gk * Jx[cx] * sbx / (D[cx] * D[cx]);
  }
  if (!(D[cy] < eps[cy])) {
    Jyb[cy] = gk * sby / D[cy];
    Db[cy] += -gk * Jy[cy] * sby / (D[cy] * D[cy]);
  }
  for (int c = 0; c < 4; ++c) {
    os[(size_t)(0 + c) * m.plane + id] = jL[c];
    os[(size_t)(4 + c) * m.plane + id] = jB[c];
    os[(size_t)(8 + c) * m.plane + id] = Jxb[c];
    os[(size_t)(12 + c) * m.plane + id] = Jyb[c];
    os[(size_t)(16 + c) * m.plane + id] = Db[c];
    os[(size_t)(20 + c) * m.plane + id] = sD[c];
    os[(size_t)(24 + c) * m.plane + id] = (double)pD[c];
  }
  os[(size_t)28 * m.plane + id] = bbx;
  os[(size_t)29 * m.plane + id] = bby;
  os[(size_t)30 * m.plane + id] = (double)abx;
  os[(size_t)31 * m.plane + id] = (double)aby;
}

// face-centre value adjoints of every cell: [c][r, l, t, b]
__global__ void __launch_bounds__(ADJ_T) oe_adj_b_kernel(AdjMesh m, const double* __restrict__ os,
                                                         double* __restrict__ cb) {
  const int i = blockIdx.x * ADJ_TX + (threadIdx.x % ADJ_TX);
  const int j = blockIdx.y * ADJ_TY + (threadIdx.x / ADJ_TX);
  if (i >= m.nx || j >= m.ny) return;
  const size_t id = (size_t)j * m.nx + i;
  const size_t il = wrap_idx(m, i - 1, j), ir = wrap_idx(m, i + 1, j), ib = wrap_idx(m, i, j - 1),
               it = wrap_idx(m, i, j + 1);
  for (int c = 0; c < 4; ++c) {
    const double jL = os[(size_t)c * m.plane + id], jR = os[(size_t)c * m.plane + ir];
    const double jB = os[(size_t)(4 + c) * m.plane + id], jT = os[(size_t)(4 + c) * m.plane + it];
    const double Jxq = os[(size_t)(8 + c) * m.plane + id];
    const double Jyq = os[(size_t)(12 + c) * m.plane + id];
    const double bL = sgn(jL) * (Jxq + os[(size_t)(8 + c) * m.plane + il]);
    const double bR = sgn(jR) * (Jxq + os[(size_t)(8 + c) * m.plane + ir]);
    const double bB = sgn(jB) * (Jyq + os[(size_t)(12 + c) * m.plane + ib]);
    const double bT = sgn(jT) * (Jyq + os[(size_t)(12 + c) * m.plane + it]);
    cb[(size_t)(c * 4 + 0) * m.plane + id] = -bR;
    cb[(size_t)(c * 4 + 1) * m.plane + id] = bL;
    cb[(size_t)(c * 4 + 2) * m.plane + id] = -bT;
    cb[(size_t)(c * 4 + 3) * m.plane + id] = bB;
  }
}

template <int K, int DX, int DY>
__device__ __forceinline__ void oe_gather_one(const AdjMesh& m, int i, int j, const double* __restrict__ Un,
                                              const double* __restrict__ os, const double* __restrict__ cb,
                                              const double* avg, double (&acc)[4][3]) {
  constexpr int L9 = (1 - DX) + 3 * (1 - DY);
  const size_t n = wrap_idx(m, i + DX, j + DY);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double b[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) b[f] = cb[(size_t)(c * 4 + f) * m.plane + n];
    acc[c][0] += cwt_dot<K, false, L9>(b);
    acc[c][1] += cwt_dot<K, false, 9 + L9>(b);
    acc[c][2] += cwt_dot<K, false, 18 + L9>(b);
    const double Db = os[(size_t)(16 + c) * m.plane + n];
    const double s = os[(size_t)(20 + c) * m.plane + n];
    const int ps = (int)os[(size_t)(24 + c) * m.plane + n];
    acc[c][0] += Db * (-s + (ps == L9 ? s : 0.0));
  }
  const int ax = (int)os[(size_t)30 * m.plane + n], ay = (int)os[(size_t)31 * m.plane + n];
  if (ax == L9 || ay == L9) {
    double gr[4];
    if (ax == L9) {
      speed_grad(0, m.gamma, avg, gr);
      const double bb = os[(size_t)28 * m.plane + n];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c][0] += bb * gr[c];
    }
    if (ay == L9) {
      speed_grad(1, m.gamma, avg, gr);
      const double bb = os[(size_t)29 * m.plane + n];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c][0] += bb * gr[c];
    }
  }
}

template <int K>
__global__ void __launch_bounds__(ADJ_T) oe_adj_c_kernel(AdjMesh m, const double* __restrict__ Un,
                                                         const double* __restrict__ os,
                                                         const double* __restrict__ cb, double* __restrict__ lamN) {
  const int i = blockIdx.x * ADJ_TX + (threadIdx.x % ADJ_TX);
  const int j = blockIdx.y * ADJ_TY + (threadIdx.x / ADJ_TX);
  if (i >= m.nx || j >= m.ny) return;
  const size_t id = (size_t)j * m.nx + i;
  double avg[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) avg[c] = Un[(c * 3) * m.plane + id];
  double acc[4][3] = {};
  oe_gather_one<K, -1, -1>(m, i, j, Un, os, cb, avg, acc);
  oe_gather_one<K, 0, -1>(m, i, j, Un, os, cb, avg, acc);
  oe_gather_one<K, 1, -1>(m, i, j, Un, os, cb, avg, acc);
  oe_gather_one<K, -1, 0>(m, i, j, Un, os, cb, avg, acc);
  oe_gather_one<K, 0, 0>(m, i, j, Un, os, cb, avg, acc);
  oe_gather_one<K, 1, 0>(m, i, j, Un, os, cb, avg, acc);
  oe_gather_one<K, -1, 1>(m, i, j, Un, os, cb, avg, acc);
  oe_gather_one<K, 0, 1>(m, i, j, Un, os, cb, avg, acc);
  oe_gather_one<K, 1, 1>(m, i, j, Un, os, cb, avg, acc);
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 3; ++r) lamN[(c * 3 + r) * m.plane + id] += acc[c][r];
}

// ---------------------------------------------------------------------------
// functional J = sum over window cells of dx dy (rho0^2 + 12 rho1^2 + 12 rho2^2)
// and its gradient (the seed of the reverse sweep)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(ADJ_T) adj_seed_kernel(AdjMesh m, double x0, double y0,
                                                         const double* __restrict__ U, double* __restrict__ lam,
                                                         double* __restrict__ partial) {
  __shared__ double red[ADJ_T / 64];
  const int i = blockIdx.x * ADJ_TX + (threadIdx.x % ADJ_TX);
  const int j = blockIdx.y * ADJ_TY + (threadIdx.x / ADJ_TX);
  double part = 0.0;
  if (i < m.nx && j < m.ny) {
    const size_t id = (size_t)j * m.nx + i;
    const double xc = x0 + (i + 0.5) * m.dx, yc = y0 + (j + 0.5) * m.dy;
    const bool win = xc >= 0.25 && xc <= 0.75 && yc >= 0.25 && yc <= 0.75;
    const double a = m.dx * m.dy;
    for (int k = 0; k < 12; ++k) lam[(size_t)k * m.plane + id] = 0.0;
    if (win) {
      const double r0 = U[id], r1 = U[m.plane + id], r2 = U[2 * m.plane + id];
      part = a * (r0 * r0 + 12.0 * r1 * r1 + 12.0 * r2 * r2);
      lam[id] = 2.0 * a * r0;
      lam[m.plane + id] = 24.0 * a * r1;
      lam[2 * m.plane + id] = 24.0 * a * r2;
    }
  }
  const double s = block_sum(part, red);
  if (threadIdx.x == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = s;
}

__global__ void __launch_bounds__(RED_T) adj_sum_kernel(const double* __restrict__ partial, int n, double* out) {
  __shared__ double red[RED_T / 64];
  double v = 0.0;
  for (int b = threadIdx.x; b < n; b += blockDim.x) v += partial[b];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += red[q];
    *out = t;
  }
}

}  // namespace fam

// ===========================================================================
// host driver
// ===========================================================================
struct FamAdjointScratch {
  size_t len = 0, cells = 0;
  int ncp = 0, seg = 0;
  double* ckpt = nullptr;     // ncp checkpoints
  double* segbuf = nullptr;   // seg steps x 4 states (U0, U1, U2, Un)
  double* ucur = nullptr;
  double* lam = nullptr;
  double* lamN = nullptr;
  double* lam1 = nullptr;
  double* lam2 = nullptr;
  double* lam0 = nullptr;
  double* abar = nullptr;     // coefficient adjoints [4][NCF][cells]
  double* os = nullptr;       // OE record [32][cells]
  double* cb = nullptr;       // face-centre adjoints [4][4][cells]
  double* partial = nullptr;  // per-block alpha adjoints / functional sums
  double* smax = nullptr;     // alpha_x, alpha_y
  double* Jd = nullptr;
  double* apv = nullptr;      // argmax partials (values)
  int* sidx = nullptr;        // first maximal cell in x, y
  int* api = nullptr;         // argmax partials (indices)
};

void fam_adjoint_free(fam_ctx* c) {
  if (!c || !c->adj) return;
  FamAdjointScratch* s = c->adj;
  void* bufs[] = {s->ckpt, s->segbuf, s->ucur, s->lam, s->lamN, s->lam1, s->lam2, s->lam0, s->abar,
                  s->os, s->cb, s->partial, s->smax, s->Jd, s->apv, s->sidx, s->api};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  delete s;
  c->adj = nullptr;
}

static fam_status adj_alloc(fam_ctx* c, int ncp, int seg) {
  FamAdjointScratch* s = c->adj;
  if (s && s->ncp >= ncp && s->seg >= seg) return FAM_OK;
  fam_adjoint_free(c);
  s = new (std::nothrow) FamAdjointScratch();
  if (!s) return FAM_ERR_NOMEM;
  c->adj = s;
  s->len = c->len;
  s->cells = c->max_cells;
  s->ncp = ncp;
  s->seg = seg;
  const size_t L = c->len * sizeof(double), D = sizeof(double);
  const size_t nb = ((c->cfg[0].nx + fam::ADJ_TX - 1) / fam::ADJ_TX) * ((c->cfg[0].ny + fam::ADJ_TY - 1) / fam::ADJ_TY);
  struct A {
    void** p;
    size_t bytes;
  } al[] = {{(void**)&s->ckpt, L * ncp}, {(void**)&s->segbuf, L * 4 * seg}, {(void**)&s->ucur, L},
            {(void**)&s->lam, L}, {(void**)&s->lamN, L}, {(void**)&s->lam1, L}, {(void**)&s->lam2, L},
            {(void**)&s->lam0, L}, {(void**)&s->abar, D * 4 * 21 * s->cells},
            {(void**)&s->os, D * fam::OES * s->cells}, {(void**)&s->cb, D * 16 * s->cells},
            {(void**)&s->partial, D * 2 * nb}, {(void**)&s->smax, D * 2}, {(void**)&s->Jd, D},
            {(void**)&s->apv, D * 2 * fam::ALPHA_BLOCKS}, {(void**)&s->sidx, sizeof(int) * 2},
            {(void**)&s->api, sizeof(int) * 2 * fam::ALPHA_BLOCKS}};
  for (auto& a : al)
    if (hipMalloc(a.p, a.bytes) != hipSuccess) {
      fam_adjoint_free(c);
      return FAM_ERR_NOMEM;
    }
  return FAM_OK;
}

template <int K>
static void rT_apply(fam_ctx* c, const fam::AdjMesh& m, const double* Us, const double* lam_out, double b,
                     double dt, double* out, int accumulate, hipStream_t st) {
  FamAdjointScratch* s = c->adj;
  const dim3 grid((m.nx + fam::ADJ_TX - 1) / fam::ADJ_TX, (m.ny + fam::ADJ_TY - 1) / fam::ADJ_TY);
  const int nb = grid.x * grid.y;
  // wave speeds of Us and their first argmax
  hipLaunchKernelGGL(fam::adj_alpha_part_kernel, dim3(fam::ALPHA_BLOCKS), dim3(256), 0, st, m, Us, s->apv, s->api);
  hipLaunchKernelGGL(fam::adj_alpha_final_kernel, dim3(1), dim3(fam::RED_T), 0, st, s->apv, s->api,
                     fam::ALPHA_BLOCKS, s->smax, s->sidx);
  hipLaunchKernelGGL((fam::adj_coef_kernel<K>), grid, dim3(fam::ADJ_T), 0, st, m, Us, lam_out, b * dt, s->smax,
                     s->abar, s->partial);
  hipLaunchKernelGGL((fam::adj_gather_kernel<K>), grid, dim3(fam::ADJ_T), 0, st, m, s->abar, lam_out, b, out,
                     accumulate);
  hipLaunchKernelGGL(fam::adj_alpha_route_kernel, dim3(1), dim3(fam::RED_T), 0, st, m, Us, s->partial, nb, s->sidx, out);
}

template <int K>
static void oe_T_apply(fam_ctx* c, const fam::AdjMesh& m, const double* Un, const double* lam, double dt,
                       double* lamN, hipStream_t st) {
  FamAdjointScratch* s = c->adj;
  const dim3 grid((m.nx + fam::ADJ_TX - 1) / fam::ADJ_TX, (m.ny + fam::ADJ_TY - 1) / fam::ADJ_TY);
  hipLaunchKernelGGL((fam::oe_adj_a_kernel<K>), grid, dim3(fam::ADJ_T), 0, st, m, Un, lam, dt, c->gamma_k, lamN,
                     s->os);
  hipLaunchKernelGGL(fam::oe_adj_b_kernel, grid, dim3(fam::ADJ_T), 0, st, m, s->os, s->cb);
  hipLaunchKernelGGL((fam::oe_adj_c_kernel<K>), grid, dim3(fam::ADJ_T), 0, st, m, Un, s->os, s->cb, lamN);
}

template <int K>
static fam_status adjoint_k(fam_ctx* c, const double* U0, int nsteps, double dt, int every, const double* dJdUT,
                            double* dJdU0, double* J_out) {
  hipStream_t st = c->stream;
  const fam_config& f = c->cfg[0];
  fam::AdjMesh m{f.nx, f.ny, (size_t)f.nx * f.ny, (f.x1 - f.x0) / f.nx, (f.y1 - f.y0) / f.ny, f.gamma};
  const int ncp = (nsteps + every - 1) / every;
  fam_status r = adj_alloc(c, ncp, std::min(every, nsteps));
  if (r != FAM_OK) return r;
  FamAdjointScratch* s = c->adj;
  const size_t L = c->len;
  const size_t bytes = L * sizeof(double);
  if (hipMemcpyAsync(s->ucur, U0, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) return FAM_ERR_DEVICE;

  // forward pass with checkpoints (same kernels and launch path as fam_step)
  reset_steps(c, 0.0, dt);
  enqueue_alpha_full(c, s->ucur, 0);
  for (int n = 0; n < nsteps; ++n) {
    if (n % every == 0)
      if (hipMemcpyAsync(s->ckpt + (size_t)(n / every) * L, s->ucur, bytes, hipMemcpyDeviceToDevice, st) !=
          hipSuccess)
        return FAM_ERR_DEVICE;
    enqueue_step(c, s->ucur, n & 1, dt, 0.0);
  }

  // seed
  const dim3 grid((m.nx + fam::ADJ_TX - 1) / fam::ADJ_TX, (m.ny + fam::ADJ_TY - 1) / fam::ADJ_TY);
  const int nb = grid.x * grid.y;
  if (dJdUT) {
    if (hipMemcpyAsync(s->lam, dJdUT, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) return FAM_ERR_DEVICE;
  } else {
    hipLaunchKernelGGL(fam::adj_seed_kernel, grid, dim3(fam::ADJ_T), 0, st, m, f.x0, f.y0, s->ucur, s->lam,
                       s->partial);
    hipLaunchKernelGGL(fam::adj_sum_kernel, dim3(1), dim3(fam::RED_T), 0, st, s->partial, nb, s->Jd);
  }

  // reverse sweep over the segments
  const size_t aN = std::min<size_t>((L + 255) / 256, 4096);
  for (int sg = ncp - 1; sg >= 0; --sg) {
    const int n0 = sg * every, n1 = std::min(nsteps, n0 + every);
    double* U = s->ucur;
    if (hipMemcpyAsync(U, s->ckpt + (size_t)sg * L, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
      return FAM_ERR_DEVICE;
    reset_steps(c, 0.0, dt);
    enqueue_alpha_full(c, U, 0);
    for (int n = n0; n < n1; ++n) {
      double* S0 = s->segbuf + (size_t)(4 * (n - n0)) * L;
      double *S1 = S0 + L, *S2 = S0 + 2 * L, *SN = S0 + 3 * L;
      const int par = (n - n0) & 1;
      if (hipMemcpyAsync(S0, U, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) return FAM_ERR_DEVICE;
      fam::launch_step_begin(c->st, 1, par, dt, 0.0, st);
      enqueue_stage(c, 0, par, S0, S0, S1, nullptr);
      enqueue_stage(c, 1, par, S0, S1, S2, nullptr);
      enqueue_stage(c, 2, par, S0, S2, SN, nullptr);
      if (c->oe == FAM_OE_OFF) {
        if (hipMemcpyAsync(U, SN, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) return FAM_ERR_DEVICE;
      } else {
        enqueue_oe(c, par, SN, U, nullptr);
      }
    }
    for (int n = n1 - 1; n >= n0; --n) {
      const double* S0 = s->segbuf + (size_t)(4 * (n - n0)) * L;
      const double *S1 = S0 + L, *S2 = S0 + 2 * L, *SN = S0 + 3 * L;
      if (c->oe == FAM_OE_OFF) {
        if (hipMemcpyAsync(s->lamN, s->lam, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) return FAM_ERR_DEVICE;
      } else {
        oe_T_apply<K>(c, m, SN, s->lam, dt, s->lamN, st);
      }
      // stage 2: Un = 1/3 U0 + 2/3 (U2 + dt R(U2))
      rT_apply<K>(c, m, S2, s->lamN, 2.0 / 3.0, dt, s->lam2, 0, st);
      hipLaunchKernelGGL(fam::adj_axpy_kernel, dim3(aN), dim3(256), 0, st, L, 1.0 / 3.0, s->lamN, s->lam0, 0);
      // stage 1: U2 = 3/4 U0 + 1/4 (U1 + dt R(U1))
      rT_apply<K>(c, m, S1, s->lam2, 0.25, dt, s->lam1, 0, st);
      hipLaunchKernelGGL(fam::adj_axpy_kernel, dim3(aN), dim3(256), 0, st, L, 0.75, s->lam2, s->lam0, 1);
      // stage 0: U1 = U0 + dt R(U0)
      rT_apply<K>(c, m, S0, s->lam1, 1.0, dt, s->lam0, 1, st);
      std::swap(s->lam, s->lam0);
    }
  }
  if (hipMemcpyAsync(dJdU0, s->lam, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) return FAM_ERR_DEVICE;
  if (hipGetLastError() != hipSuccess) return FAM_ERR_DEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return FAM_ERR_DEVICE;
  if (J_out) {
    *J_out = 0.0;
    if (!dJdUT && hipMemcpy(J_out, s->Jd, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return FAM_ERR_DEVICE;
  }
  return fam_check(c);
}

extern "C" fam_status fam_adjoint(fam_ctx* c, const double* U0, int nsteps, double dt, int checkpoint_every,
                                  const double* dJdUT, double* dJdU0, double* J_out) {
  if (!c || !U0 || !dJdU0 || nsteps < 1 || !(dt > 0.0) || checkpoint_every < 1) return FAM_ERR_ARG;
  const fam_config& f = c->cfg[0];
  if (c->ninst != 1 || c->dim != 2 || c->sys != FAM_EULER || f.bc_x != FAM_BC_PERIODIC ||
      f.bc_y != FAM_BC_PERIODIC || c->oe == FAM_OE_TYPE1 || c->pp || (c->k == 6 && c->k6t))
    return FAM_ERR_STATE;
  switch (c->k) {
    case 3: return adjoint_k<3>(c, U0, nsteps, dt, checkpoint_every, dJdUT, dJdU0, J_out);
    case 4: return adjoint_k<4>(c, U0, nsteps, dt, checkpoint_every, dJdUT, dJdU0, J_out);
    case 5: return adjoint_k<5>(c, U0, nsteps, dt, checkpoint_every, dJdUT, dJdU0, J_out);
    case 6: return adjoint_k<6>(c, U0, nsteps, dt, checkpoint_every, dJdUT, dJdU0, J_out);
  }
  return FAM_ERR_ARG;
}
