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
// OE^T (Type II) in two LDS-tiled passes: per cell, the derivative of the damping
// factor with respect to the jump sums, the denominators and the wave-speed
// bounds; then per cell, the face adjoints of its 3x3 neighbours, gathered
// through the transposed face-centre functionals, and the denominator /
// wave-speed routes over the 3x3 patch.
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
// a block's cells and a one-cell ring: GT x GT tile positions
constexpr int GT = ADJ_TX + 2;
constexpr int GTC = GT * GT;
constexpr int NLP = (GTC + ADJ_T - 1) / ADJ_T;   // tile positions per thread (at most two)
// the coefficient-adjoint kernel: one wave per block (8 x 8 cells), so that the
// four blocks a CU holds (its registers allow one wave per SIMD) load and compute
// independently
constexpr int CTX = 8, CTY = 8, CT = CTX * CTY;
constexpr int CGX = CTX + 2, CGC = CGX * (CTY + 2);
constexpr int CNLP = (CGC + CT - 1) / CT;

struct AdjMesh {
  int nx, ny;
  size_t plane;
  double dx, dy, gamma;
};

__device__ __forceinline__ int wrap1(int i, int n) {
  if (i < 0) i += n;
  else if (i >= n) i -= n;
  if ((unsigned)i >= (unsigned)n) {   // offsets beyond one period (tiny meshes)
    i %= n;
    if (i < 0) i += n;
  }
  return i;
}

__device__ __forceinline__ size_t wrap_idx(const AdjMesh& m, int i, int j) {
  return (size_t)wrap1(j, m.ny) * m.nx + wrap1(i, m.nx);
}

// this block's tile of the grid in the XCD-aware order (neighbouring tiles,
// which share halo cache lines, run under one L2)
__device__ __forceinline__ int2 block_tile() {
  const int T = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  return make_int2(T % gridDim.x, T / gridDim.x);
}

// periodic image of an index at most one period outside [0, n)
__device__ __forceinline__ int wrap_near(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// the periodic 3x3 patch around the mesh cell (i, j): its three columns and
// three row offsets (a mesh holds at most 2^31 cells); id(l) is the flat index
// of patch cell l, row by row from (i - 1, j - 1): id(4) is the cell, id(3) /
// id(5) its left / right and id(1) / id(7) its bottom / top neighbour
struct Patch {
  unsigned cx[3], ry[3];
  __device__ __forceinline__ unsigned id(int l) const { return ry[l / 3] + cx[l % 3]; }
};

__device__ __forceinline__ Patch patch_of(const AdjMesh& m, int i, int j) {
  Patch P;
  P.cx[0] = wrap_near(i - 1, m.nx);
  P.cx[1] = i;
  P.cx[2] = wrap_near(i + 1, m.nx);
  P.ry[0] = (unsigned)wrap_near(j - 1, m.ny) * (unsigned)m.nx;
  P.ry[1] = (unsigned)j * (unsigned)m.nx;
  P.ry[2] = (unsigned)wrap_near(j + 1, m.ny) * (unsigned)m.nx;
  return P;
}

// stencil of component c over the patch P
template <int K>
__device__ __forceinline__ void gstencil(const double* __restrict__ U, const AdjMesh& m, int c, const Patch& P,
                                         double (&u0)[9], double (&u1)[9], double (&u2)[9]) {
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int l = b * 3 + a;
      const size_t id = P.id(l);
      u0[l] = U[(c * 3 + 0) * m.plane + id];
      const bool x_used = (K >= 5) ? (l != 1 && l != 7) : (l == 4);
      const bool y_used = (K >= 5) ? (l != 3 && l != 5) : (l == 4);
      u1[l] = x_used ? U[(c * 3 + 1) * m.plane + id] : 0.0;
      u2[l] = y_used ? U[(c * 3 + 2) * m.plane + id] : 0.0;
    }
}

// out = J_d(u)^T w for the 2D Euler flux in direction d
__device__ __forceinline__ void euler_jt(int d, double g, const double* u, const double* w, double* out) {
  const double inv = rcp(u[0]);
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

// out = J_1(u)^T w1 + J_2(u)^T w2 (volume points: both directions share the primitives)
__device__ __forceinline__ void euler_jt2(double g, const double* u, const double* w1, const double* w2,
                                          double* out) {
  const double inv = rcp(u[0]);
  const double vx = u[1] * inv, vy = u[2] * inv;
  const double q2 = vx * vx + vy * vy;
  const double g1 = g - 1.0;
  const double p = g1 * (u[3] - 0.5 * u[0] * q2);
  const double H = (u[3] + p) * inv;
  const double k = 0.5 * g1 * q2;
  const double vxy = vx * vy;
  out[0] = (-vx * vx + k) * w1[1] - vxy * (w1[2] + w2[1]) + vx * (k - H) * w1[3] + (-vy * vy + k) * w2[2] +
           vy * (k - H) * w2[3];
  out[1] = w1[0] + (3.0 - g) * vx * w1[1] + vy * (w1[2] + w2[1]) + (H - g1 * vx * vx) * w1[3] -
           g1 * vx * w2[2] - g1 * vxy * w2[3];
  out[2] = -g1 * vy * w1[1] + vx * (w1[2] + w2[1]) - g1 * vxy * w1[3] + w2[0] + (3.0 - g) * vy * w2[2] +
           (H - g1 * vy * vy) * w2[3];
  out[3] = g1 * (w1[1] + w2[2]) + g * (vx * w1[3] + vy * w2[3]);
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
//
// The 32 flux points form 8 groups of 4 sign-symmetric points (sx X, sy Y):
// groups 0, 1: x-faces (X = 1/2, Y = GS0 / GS1; sx = +1 right face, -1 left);
// groups 2, 3: y-faces (X = GS0 / GS1, Y = 1/2; sy = +1 top face, -1 bottom);
// groups 4..7: volume points (X, Y) in {GS0, GS1}^2.
// phi_l(sx X, sy Y) = phi_l(X, Y) sx^(ax_l odd) sy^(ay_l odd), so the point values
// of a group come from four parity sums of the coefficients, and the transposed
// evaluation from four signed sums of the point adjoints.
// ---------------------------------------------------------------------------
// face adjoint weights of the face between cells L (left / below) and R:
// d J / d Fbar and d J / d Ftil (x-face), d J / d Gbar and d J / d Gtil (y-face)
__device__ __forceinline__ void face_adj(bool xface, const double (&muL)[3], const double (&muR)[3], double inv,
                                         double& B, double& T) {
  if (xface) {
    B = (-muL[0] - 0.5 * muL[1] + muR[0] - 0.5 * muR[1]) * inv;
    T = (-muL[2] + muR[2]) * inv;
  } else {
    B = (-muL[0] - 0.5 * muL[2] + muR[0] - 0.5 * muR[2]) * inv;
    T = (-muL[1] + muR[1]) * inv;
  }
}

template <int TC>
__device__ __forceinline__ void tile_mu(const double (&tl)[12][TC], int pos, double (&mu)[4][3]) {
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 3; ++r) mu[c][r] = tl[c * 3 + r][pos];
}

// G: group index; for face groups B/T hold [side][c] for the two faces of the group
// (side 0: sign +1 face, side 1: sign -1 face)
template <int K, int G>
__device__ __forceinline__ void coef_group(double g, const double (&cf)[4][ncoef2d(K)], double (&ab)[4][ncoef2d(K)],
                                           const double (&mu)[4][3], double idx_, double idy,
                                           const double (&B)[2][4], const double (&T)[2][4], double al,
                                           double& pa) {
  constexpr int NCF = ncoef2d(K);
  using Seq = std::make_integer_sequence<int, NCF>;
  constexpr int NXI = G < 2 ? 2 : G < 4 ? (G - 2) : ((G - 4) & 1);
  constexpr int NYI = G < 2 ? G : G < 4 ? 2 : ((G - 4) >> 1);
  constexpr bool XF = G < 2, YF = (G >= 2 && G < 4);
  double u[4][4];   // [point][component]
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double P[4];
    parity_sums<NXI, NYI>(cf[c], P, Seq{});
#pragma unroll
    for (int s = 0; s < 4; ++s) u[s][c] = P[0] + grp_sx(s) * P[1] + grp_sy(s) * P[2] + grp_sx(s) * grp_sy(s) * P[3];
  }
  double ub[4][4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if constexpr (XF || YF) {
      // face point: side by the sign across the face, Gauss node by the sign along it
      const int side = XF ? (grp_sx(s) > 0 ? 0 : 1) : (grp_sy(s) > 0 ? 0 : 1);
      const double eta = XF ? grp_sy(s) * (NYI == 0 ? GS0 : GS1) : grp_sx(s) * (NXI == 0 ? GS0 : GS1);
      const double w = XF ? (NYI == 0 ? GW0 : GW1) : (NXI == 0 ? GW0 : GW1);
      const double sgn = side == 0 ? 1.0 : -1.0;
      double Fh[4], half[4], jt[4];
      double dot = 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        Fh[c] = w * (B[side][c] + eta * T[side][c]);
        half[c] = 0.5 * Fh[c];
        dot = fma(Fh[c], u[s][c], dot);
      }
      euler_jt(XF ? 0 : 1, g, u[s], half, jt);
#pragma unroll
      for (int c = 0; c < 4; ++c) ub[s][c] = jt[c] + sgn * 0.5 * al * Fh[c];
      pa += sgn * 0.5 * dot;
    } else {
      constexpr double w = (NXI == 0 ? GW0 : GW1) * (NYI == 0 ? GW0 : GW1);
      double w1[4], w2[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        w1[c] = w * mu[c][1] * idx_;
        w2[c] = w * mu[c][2] * idy;
      }
      euler_jt2(g, u[s], w1, w2, ub[s]);
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double Q[4];
    Q[0] = ub[0][c] + ub[1][c] + ub[2][c] + ub[3][c];
    Q[1] = ub[0][c] + ub[1][c] - ub[2][c] - ub[3][c];
    Q[2] = ub[0][c] - ub[1][c] + ub[2][c] - ub[3][c];
    Q[3] = ub[0][c] - ub[1][c] - ub[2][c] + ub[3][c];
    parity_scatter<NXI, NYI>(ab[c], Q, Seq{});
  }
}

template <int K>
__global__ void __launch_bounds__(CT) adj_coef_kernel(AdjMesh m, const double* __restrict__ U,
                                                      const double* __restrict__ lam, double scale,
                                                      const double* __restrict__ alpha,
                                                      double* __restrict__ abar, double* __restrict__ partial) {
  constexpr int NC = 4, NCF = ncoef2d(K);
  __shared__ double red[CT / 64];
  // the 12 planes of U and of scale * lam over the block's cells and a one-cell ring
  __shared__ double tu[12][CGC];
  __shared__ double tl[12][CGC];
  const int tx = threadIdx.x % CTX, ty = threadIdx.x / CTX;
  const int2 bt = block_tile();
  const int i0 = bt.x * CTX, j0 = bt.y * CTY;
  const int i = i0 + tx, j = j0 + ty;
  const bool inside = i < m.nx && j < m.ny;
#pragma unroll
  for (int t = 0; t < CNLP; ++t) {
    const int p = threadIdx.x + t * CT;
    if (p < CGC) {
      const int py = p / CGX, px = p - py * CGX;
      const size_t src = wrap_idx(m, i0 - 1 + px, j0 - 1 + py);
#pragma unroll
      for (int q = 0; q < 12; ++q) {
        tu[q][p] = U[(size_t)q * m.plane + src];
        tl[q][p] = scale * lam[(size_t)q * m.plane + src];
      }
    }
  }
  __syncthreads();
  double pax = 0.0, pay = 0.0;
  if (inside) {
    const double g = m.gamma;
    const double ax = alpha[0], ay = alpha[1];
    const double idx_ = 1.0 / m.dx, idy = 1.0 / m.dy;
    const int base = (ty + 1) * CGX + (tx + 1);   // this cell in the tiles
    double cf[NC][NCF];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double u0[9], u1[9], u2[9];
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int l = b * 3 + a, pos = base + (b - 1) * CGX + (a - 1);
          const bool x_used = (K >= 5) ? (l != 1 && l != 7) : (l == 4);
          const bool y_used = (K >= 5) ? (l != 3 && l != 5) : (l == 4);
          u0[l] = tu[c * 3 + 0][pos];
          u1[l] = x_used ? tu[c * 3 + 1][pos] : 0.0;
          u2[l] = y_used ? tu[c * 3 + 2][pos] : 0.0;
        }
      double tmp[23];
      coeffs2d<K>(u0, u1, u2, tmp, false);
#pragma unroll
      for (int l = 0; l < NCF; ++l) cf[c][l] = tmp[l];
      __builtin_amdgcn_sched_barrier(0);
    }
    const size_t id = (size_t)j * m.nx + i;
    double mu[NC][3];
    tile_mu(tl, base, mu);
    double ab[NC][NCF];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int l = 0; l < NCF; ++l) ab[c][l] = 0.0;
    double B[2][4], T[2][4];
    // x-faces: side 0 = right face (this cell on the left), side 1 = left face
    {
      double nb[NC][3];
      tile_mu(tl, base + 1, nb);
#pragma unroll
      for (int c = 0; c < NC; ++c) face_adj(true, mu[c], nb[c], idx_, B[0][c], T[0][c]);
      tile_mu(tl, base - 1, nb);
#pragma unroll
      for (int c = 0; c < NC; ++c) face_adj(true, nb[c], mu[c], idx_, B[1][c], T[1][c]);
    }
    coef_group<K, 0>(g, cf, ab, mu, idx_, idy, B, T, ax, pax);
    __builtin_amdgcn_sched_barrier(0);
    coef_group<K, 1>(g, cf, ab, mu, idx_, idy, B, T, ax, pax);
    __builtin_amdgcn_sched_barrier(0);
    // y-faces: side 0 = top face (this cell below), side 1 = bottom face
    {
      double nb[NC][3];
      tile_mu(tl, base + CGX, nb);
#pragma unroll
      for (int c = 0; c < NC; ++c) face_adj(false, mu[c], nb[c], idy, B[0][c], T[0][c]);
      tile_mu(tl, base - CGX, nb);
#pragma unroll
      for (int c = 0; c < NC; ++c) face_adj(false, nb[c], mu[c], idy, B[1][c], T[1][c]);
    }
    coef_group<K, 2>(g, cf, ab, mu, idx_, idy, B, T, ay, pay);
    __builtin_amdgcn_sched_barrier(0);
    coef_group<K, 3>(g, cf, ab, mu, idx_, idy, B, T, ay, pay);
    __builtin_amdgcn_sched_barrier(0);
    coef_group<K, 4>(g, cf, ab, mu, idx_, idy, B, T, 0.0, pax);
    __builtin_amdgcn_sched_barrier(0);
    coef_group<K, 5>(g, cf, ab, mu, idx_, idy, B, T, 0.0, pax);
    __builtin_amdgcn_sched_barrier(0);
    coef_group<K, 6>(g, cf, ab, mu, idx_, idy, B, T, 0.0, pax);
    __builtin_amdgcn_sched_barrier(0);
    coef_group<K, 7>(g, cf, ab, mu, idx_, idy, B, T, 0.0, pax);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int l = 0; l < NCF; ++l) abar[(size_t)(c * NCF + l) * m.plane + id] = ab[c][l];
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

// LDS tile of one component's coefficient adjoints over the block's cells and a
// one-cell ring (periodic wrap): GT x GT, defined with the block shape

template <int K>
__global__ void __launch_bounds__(ADJ_T) adj_gather_kernel(AdjMesh m, const double* __restrict__ abar,
                                                           const double* __restrict__ lam_out, double b,
                                                           double* __restrict__ out, int accumulate,
                                                           double* __restrict__ out2, double b2, int acc2) {
  constexpr int NCF = ncoef2d(K);
  __shared__ double sh[NCF][GTC];
  const int tx = threadIdx.x % ADJ_TX, ty = threadIdx.x / ADJ_TX;
  const int2 bt = block_tile();
  const int i0 = bt.x * ADJ_TX, j0 = bt.y * ADJ_TY;
  const int i = i0 + tx, j = j0 + ty;
  const bool inside = i < m.nx && j < m.ny;
  double acc[4][3];
  // tile positions this thread loads
  size_t src[NLP];
#pragma unroll
  for (int t = 0; t < NLP; ++t) {
    const int p = threadIdx.x + t * ADJ_T;
    const int py = p / GT, px = p - py * GT;
    src[t] = p < GTC ? wrap_idx(m, i0 - 1 + px, j0 - 1 + py) : 0;
  }
  // component c + 1's tile is loaded into registers while component c is gathered
  double nxt[NLP][NCF];
#pragma unroll
  for (int t = 0; t < NLP; ++t) {
    const int p = threadIdx.x + t * ADJ_T;
#pragma unroll
    for (int l = 0; l < NCF; ++l) nxt[t][l] = p < GTC ? abar[(size_t)l * m.plane + src[t]] : 0.0;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NLP; ++t) {
      const int p = threadIdx.x + t * ADJ_T;
      if (p < GTC) {
#pragma unroll
        for (int l = 0; l < NCF; ++l) sh[l][p] = nxt[t][l];
      }
    }
    __syncthreads();
    if (c < 3) {
#pragma unroll
      for (int t = 0; t < NLP; ++t) {
        const int p = threadIdx.x + t * ADJ_T;
#pragma unroll
        for (int l = 0; l < NCF; ++l)
          nxt[t][l] = p < GTC ? abar[(size_t)((c + 1) * NCF + l) * m.plane + src[t]] : 0.0;
      }
    }
    acc[c][0] = acc[c][1] = acc[c][2] = 0.0;
    if (inside) {
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int pos = (ty + 1 + dy) * GT + (tx + 1 + dx);
          double a[NCF];
#pragma unroll
          for (int l = 0; l < NCF; ++l) a[l] = sh[l][pos];
          // position of this cell in the patch of the neighbour n = q + (dx, dy)
          const int L9 = (1 - dx) + 3 * (1 - dy);
          switch (L9) {
#define FAM_RT3(P)                              \
  case P:                                       \
    acc[c][0] += rt_apply<K, P>(a);             \
    acc[c][1] += rt_apply<K, 9 + P>(a);         \
    acc[c][2] += rt_apply<K, 18 + P>(a);        \
    break;
            FAM_RT3(0) FAM_RT3(1) FAM_RT3(2) FAM_RT3(3) FAM_RT3(4) FAM_RT3(5) FAM_RT3(6) FAM_RT3(7) FAM_RT3(8)
#undef FAM_RT3
          }
        }
    }
  }
  if (!inside) return;
  const size_t id = (size_t)j * m.nx + i;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const size_t k = (c * 3 + r) * m.plane + id;
      const double lo = lam_out[k];
      const double v = b * lo + acc[c][r];
      out[k] = accumulate ? out[k] + v : v;
      // second output: out2 (+)= b2 lam_out (the Shu-Osher U0 terms)
      if (out2) out2[k] = acc2 ? out2[k] + b2 * lo : b2 * lo;
    }
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
// per-cell record (OES planes): [0..3] jump at the left face, [4..7] jump at the
// bottom face, [8..11] dJ/dJx, [12..15] dJ/dJy (read for the face-centre
// adjoints); [16..19] dJ/dD * sign(u_p* - S), 20 packed patch indices (p* of the
// four components, argmax beta_x, argmax beta_y; 4 bits each), 21, 22 dJ/dbeta_x, y
// (read by the gather).
constexpr int OES = 23;

// ---------------------------------------------------------------------------
// OE adjoint in two LDS-tiled passes:
//  rec:    per block, the face-centre values, averages and spectral radii of its
//          cells and a one-cell ring (from a 20 x 20 tile of Un, one component at a
//          time); then per cell the damping factor, lamN = delta lam (first moments),
//          and the record: the derivative of delta with respect to the jump sums,
//          the denominators (routed to the patch cell attaining the maximum) and
//          the wave-speed bounds (first maximal entry);
//  gather: per block and component, the face-centre adjoints of its cells and a
//          one-cell ring (from a 20 x 20 tile of the record's jumps and jump-sum
//          adjoints), gathered through the transposed face-centre functionals, then
//          the denominator and wave-speed routes.
// ---------------------------------------------------------------------------
constexpr int FG = ADJ_TX + 4, FGC = FG * FG;        // a block's cells and a two-cell ring
constexpr int FNLP = (FGC + ADJ_T - 1) / ADJ_T;
static_assert(ADJ_TX == ADJ_TY, "square blocks");

template <int K>
__global__ void __launch_bounds__(ADJ_T) oe_adj_rec_kernel(AdjMesh m, const double* __restrict__ Un,
                                                           const double* __restrict__ lam, double dt, double gk,
                                                           double* __restrict__ lamN, double* __restrict__ os) {
  __shared__ double st[3][FGC];    // one component's three planes over the 20 x 20 region
  __shared__ double cv[16][GTC];   // face-centre values [4c + f] (f: r, l, t, b) over the 18 x 18 region
  __shared__ double av[4][GTC];    // averages over the 18 x 18 region
  __shared__ double sp[2][GTC];    // spectral radii in x and y over the 18 x 18 region
  const int tx = threadIdx.x % ADJ_TX, ty = threadIdx.x / ADJ_TX;
  const int2 bt = block_tile();
  const int i0 = bt.x * ADJ_TX, j0 = bt.y * ADJ_TY;
  const int i = i0 + tx, j = j0 + ty;
  size_t src[FNLP];
#pragma unroll
  for (int t = 0; t < FNLP; ++t) {
    const int p = threadIdx.x + t * ADJ_T;
    const int py = p / FG, px = p - py * FG;
    src[t] = p < FGC ? wrap_idx(m, i0 - 2 + px, j0 - 2 + py) : 0;
  }
  using Seq = std::make_integer_sequence<int, 27>;
#pragma unroll 1
  for (int c = 0; c < 4; ++c) {
    __syncthreads();
#pragma unroll
    for (int t = 0; t < FNLP; ++t) {
      const int p = threadIdx.x + t * ADJ_T;
      if (p < FGC) {
#pragma unroll
        for (int q = 0; q < 3; ++q) st[q][p] = Un[(size_t)(c * 3 + q) * m.plane + src[t]];
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NLP; ++t) {
      const int p = threadIdx.x + t * ADJ_T;
      if (p < GTC) {
        const int py = p / GT, px = p - py * GT;   // region (px, py) = tile (px + 1, py + 1)
        double u[27];
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const int l = b * 3 + a, f = (py + b) * FG + (px + a);
            u[l] = st[0][f];
            u[9 + l] = slot_used<K>(9 + l) ? st[1][f] : 0.0;
            u[18 + l] = slot_used<K>(18 + l) ? st[2][f] : 0.0;
          }
        cv[4 * c + 0][p] = centre_dot<K, false, 0>(u, Seq{});
        cv[4 * c + 1][p] = centre_dot<K, false, 1>(u, Seq{});
        cv[4 * c + 2][p] = centre_dot<K, false, 2>(u, Seq{});
        cv[4 * c + 3][p] = centre_dot<K, false, 3>(u, Seq{});
        av[c][p] = u[4];
      }
    }
  }
  __syncthreads();
  const Euler<2> ph{m.gamma};
  bool bad = false;
#pragma unroll
  for (int t = 0; t < NLP; ++t) {
    const int p = threadIdx.x + t * ADJ_T;
    if (p < GTC) {
      const double a[4] = {av[0][p], av[1][p], av[2][p], av[3][p]};
      sp[0][p] = ph.speed(0, a, bad);
      sp[1][p] = ph.speed(1, a, bad);
    }
  }
  __syncthreads();
  if (i >= m.nx || j >= m.ny) return;
  const int rp = (ty + 1) * GT + (tx + 1);   // this cell in the region
  const size_t id = (size_t)j * m.nx + i;
  double Jx[4], Jy[4], jL[4], jB[4], D[4], eps[4], sD[4];
  int pD[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    jL[c] = cv[4 * c + 1][rp] - cv[4 * c + 0][rp - 1];            // l(i) - r(i-1)
    const double jR = cv[4 * c + 1][rp + 1] - cv[4 * c + 0][rp];   // l(i+1) - r(i)
    jB[c] = cv[4 * c + 3][rp] - cv[4 * c + 2][rp - GT];            // b(j) - t(j-1)
    const double jT = cv[4 * c + 3][rp + GT] - cv[4 * c + 2][rp];  // b(j+1) - t(j)
    Jx[c] = fabs(jL[c]) + fabs(jR);
    Jy[c] = fabs(jB[c]) + fabs(jT);
    double v[9];
    double S = 0.0, mabs = 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      v[q] = av[c][rp + (q / 3 - 1) * GT + (q % 3 - 1)];
      S += v[q];
      mabs = fmax(mabs, fabs(v[q]));
    }
    double best = -1.0;
    int arg = 0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const double d = fabs(v[q] - S);
      if (d > best) {
        best = d;
        arg = q;
      }
    }
    D[c] = best;
    pD[c] = arg;
    sD[c] = sgn(v[arg] - S);
    eps[c] = 1e-14 * fmax(mabs, 1.0);
  }
  double bx = -1.0, by = -1.0;
  int abx = 0, aby = 0;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const int pos = rp + (q / 3 - 1) * GT + (q % 3 - 1);
    const double sx = sp[0][pos], sy = sp[1][pos];
    if (sx > bx) { bx = sx; abx = q; }
    if (sy > by) { by = sy; aby = q; }
  }
  double sgx = -1.0, sgy = -1.0;
  int cx = 0, cy = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const bool small = D[c] < eps[c];
    const double sxc = small ? 0.0 : gk * Jx[c] / D[c];
    const double syc = small ? 0.0 : gk * Jy[c] / D[c];
    if (sxc > sgx) { sgx = sxc; cx = c; }
    if (syc > sgy) { sgy = syc; cy = c; }
  }
  const double kx = dt / m.dx, ky = dt / m.dy;
  const double delta = exp(-bx * kx * sgx - by * ky * sgy);
  double dbar = 0.0;
#pragma unroll
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
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (c == cx && !(D[c] < eps[c])) {
      Jxb[c] = gk * sbx / D[c];
      Db[c] += -gk * Jx[c] * sbx / (D[c] * D[c]);
    }
    if (c == cy && !(D[c] < eps[c])) {
      Jyb[c] = gk * sby / D[c];
      Db[c] += -gk * Jy[c] * sby / (D[c] * D[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    os[(size_t)(0 + c) * m.plane + id] = jL[c];
    os[(size_t)(4 + c) * m.plane + id] = jB[c];
    os[(size_t)(8 + c) * m.plane + id] = Jxb[c];
    os[(size_t)(12 + c) * m.plane + id] = Jyb[c];
    os[(size_t)(16 + c) * m.plane + id] = Db[c] * sD[c];
  }
  const int packed = pD[0] | (pD[1] << 4) | (pD[2] << 8) | (pD[3] << 12) | (abx << 16) | (aby << 20);
  os[(size_t)20 * m.plane + id] = (double)packed;
  os[(size_t)21 * m.plane + id] = bbx;
  os[(size_t)22 * m.plane + id] = bby;
}

template <int K>
__global__ void __launch_bounds__(ADJ_T) oe_adj_gather_kernel(AdjMesh m, const double* __restrict__ Un,
                                                              const double* __restrict__ os,
                                                              double* __restrict__ lamN) {
  __shared__ double t4[4][FGC];    // one component's jL, jB, dJ/dJx, dJ/dJy over the 20 x 20 region
  __shared__ double cbt[4][GTC];   // its face-centre adjoints (r, l, t, b) over the 18 x 18 region
  __shared__ double ex[7][GTC];    // dJ/dD * s (4 components), packed indices, beta adjoints over 18 x 18
  const int tx = threadIdx.x % ADJ_TX, ty = threadIdx.x / ADJ_TX;
  const int2 bt = block_tile();
  const int i0 = bt.x * ADJ_TX, j0 = bt.y * ADJ_TY;
  const int i = i0 + tx, j = j0 + ty;
  const bool inside = i < m.nx && j < m.ny;
  size_t src[FNLP];
#pragma unroll
  for (int t = 0; t < FNLP; ++t) {
    const int p = threadIdx.x + t * ADJ_T;
    const int py = p / FG, px = p - py * FG;
    src[t] = p < FGC ? wrap_idx(m, i0 - 2 + px, j0 - 2 + py) : 0;
  }
#pragma unroll
  for (int t = 0; t < NLP; ++t) {
    const int p = threadIdx.x + t * ADJ_T;
    if (p < GTC) {
      const int py = p / GT, px = p - py * GT;
      const size_t sr = wrap_idx(m, i0 - 1 + px, j0 - 1 + py);
#pragma unroll
      for (int q = 0; q < 7; ++q) ex[q][p] = os[(size_t)(16 + q) * m.plane + sr];
    }
  }
  double acc[4][3] = {};
#pragma unroll 1
  for (int c = 0; c < 4; ++c) {
    __syncthreads();
#pragma unroll
    for (int t = 0; t < FNLP; ++t) {
      const int p = threadIdx.x + t * ADJ_T;
      if (p < FGC) {
        t4[0][p] = os[(size_t)c * m.plane + src[t]];
        t4[1][p] = os[(size_t)(4 + c) * m.plane + src[t]];
        t4[2][p] = os[(size_t)(8 + c) * m.plane + src[t]];
        t4[3][p] = os[(size_t)(12 + c) * m.plane + src[t]];
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NLP; ++t) {
      const int p = threadIdx.x + t * ADJ_T;
      if (p < GTC) {
        const int py = p / GT, px = p - py * GT;
        const int f = (py + 1) * FG + (px + 1);   // the same cell in the 20 x 20 tile
        const double jLv = t4[0][f], jRv = t4[0][f + 1], jBv = t4[1][f], jTv = t4[1][f + FG];
        const double Jxq = t4[2][f], Jyq = t4[3][f];
        const double bL = sgn(jLv) * (Jxq + t4[2][f - 1]);
        const double bR = sgn(jRv) * (Jxq + t4[2][f + 1]);
        const double bB = sgn(jBv) * (Jyq + t4[3][f - FG]);
        const double bT = sgn(jTv) * (Jyq + t4[3][f + FG]);
        cbt[0][p] = -bR;
        cbt[1][p] = bL;
        cbt[2][p] = -bT;
        cbt[3][p] = bB;
      }
    }
    __syncthreads();
    if (inside) {
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int pos = (ty + 1 + dy) * GT + (tx + 1 + dx);
          const int L9 = (1 - dx) + 3 * (1 - dy);   // position of q in the patch of n = q + (dx, dy)
          double b[4];
#pragma unroll
          for (int f = 0; f < 4; ++f) b[f] = cbt[f][pos];
          switch (L9) {
#define FAM_CW3(P)                                    \
  case P:                                             \
    acc[c][0] += cwt_dot<K, false, P>(b);             \
    acc[c][1] += cwt_dot<K, false, 9 + P>(b);         \
    acc[c][2] += cwt_dot<K, false, 18 + P>(b);        \
    break;
            FAM_CW3(0) FAM_CW3(1) FAM_CW3(2) FAM_CW3(3) FAM_CW3(4) FAM_CW3(5) FAM_CW3(6) FAM_CW3(7) FAM_CW3(8)
#undef FAM_CW3
          }
          const int packed = (int)ex[4][pos];
          const int ps = (packed >> (4 * c)) & 15;
          acc[c][0] += ps == L9 ? 0.0 : -ex[c][pos];
        }
    }
  }
  if (!inside) return;
  const size_t id = (size_t)j * m.nx + i;
  double avg[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) avg[c] = Un[(c * 3) * m.plane + id];
  double gx[4], gy[4];
  speed_grad(0, m.gamma, avg, gx);
  speed_grad(1, m.gamma, avg, gy);
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) {
      const int pos = (ty + 1 + dy) * GT + (tx + 1 + dx);
      const int L9 = (1 - dx) + 3 * (1 - dy);
      const int packed = (int)ex[4][pos];
      if (((packed >> 16) & 15) == L9) {
        const double bb = ex[5][pos];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c][0] += bb * gx[c];
      }
      if (((packed >> 20) & 15) == L9) {
        const double bb = ex[6][pos];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c][0] += bb * gy[c];
      }
    }
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
  const int2 bt = block_tile();
  const int i = bt.x * ADJ_TX + (threadIdx.x % ADJ_TX);
  const int j = bt.y * ADJ_TY + (threadIdx.x / ADJ_TX);
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
  double* os = nullptr;       // OE record [OES][cells]
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
                  s->os, s->partial, s->smax, s->Jd, s->apv, s->sidx, s->api};
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
  const int nx = c->cfg[0].nx, ny = c->cfg[0].ny;
  // per-block partials: the coefficient kernel's 8 x 8 blocks outnumber the 16 x 16 ones
  const size_t nb = (size_t)((nx + fam::CTX - 1) / fam::CTX) * ((ny + fam::CTY - 1) / fam::CTY);
  struct A {
    void** p;
    size_t bytes;
  } al[] = {{(void**)&s->ckpt, L * ncp}, {(void**)&s->segbuf, L * 4 * seg}, {(void**)&s->ucur, L},
            {(void**)&s->lam, L}, {(void**)&s->lamN, L}, {(void**)&s->lam1, L}, {(void**)&s->lam2, L},
            {(void**)&s->lam0, L}, {(void**)&s->abar, D * 4 * 21 * s->cells},
            {(void**)&s->os, D * fam::OES * s->cells},
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
                     double dt, double* out, int accumulate, double* out2, double b2, int acc2, hipStream_t st) {
  FamAdjointScratch* s = c->adj;
  const dim3 grid((m.nx + fam::ADJ_TX - 1) / fam::ADJ_TX, (m.ny + fam::ADJ_TY - 1) / fam::ADJ_TY);
  // wave speeds of Us and their first argmax
  hipLaunchKernelGGL(fam::adj_alpha_part_kernel, dim3(fam::ALPHA_BLOCKS), dim3(256), 0, st, m, Us, s->apv, s->api);
  hipLaunchKernelGGL(fam::adj_alpha_final_kernel, dim3(1), dim3(fam::RED_T), 0, st, s->apv, s->api,
                     fam::ALPHA_BLOCKS, s->smax, s->sidx);
  const dim3 cgrid((m.nx + fam::CTX - 1) / fam::CTX, (m.ny + fam::CTY - 1) / fam::CTY);
  const int nb = cgrid.x * cgrid.y;   // blocks of the coefficient kernel: its alpha partials
  hipLaunchKernelGGL((fam::adj_coef_kernel<K>), cgrid, dim3(fam::CT), 0, st, m, Us, lam_out, b * dt, s->smax,
                     s->abar, s->partial);
  hipLaunchKernelGGL((fam::adj_gather_kernel<K>), grid, dim3(fam::ADJ_T), 0, st, m, s->abar, lam_out, b, out,
                     accumulate, out2, b2, acc2);
  hipLaunchKernelGGL(fam::adj_alpha_route_kernel, dim3(1), dim3(fam::RED_T), 0, st, m, Us, s->partial, nb, s->sidx, out);
}

template <int K>
static void oe_T_apply(fam_ctx* c, const fam::AdjMesh& m, const double* Un, const double* lam, double dt,
                       double* lamN, hipStream_t st) {
  FamAdjointScratch* s = c->adj;
  const dim3 grid((m.nx + fam::ADJ_TX - 1) / fam::ADJ_TX, (m.ny + fam::ADJ_TY - 1) / fam::ADJ_TY);
  hipLaunchKernelGGL((fam::oe_adj_rec_kernel<K>), grid, dim3(fam::ADJ_T), 0, st, m, Un, lam, dt, c->gamma_k,
                     lamN, s->os);
  hipLaunchKernelGGL((fam::oe_adj_gather_kernel<K>), grid, dim3(fam::ADJ_T), 0, st, m, Un, s->os, lamN);
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

  // Records steps n0 .. n1-1 from the state in slot 0 of the segment buffer:
  // step n keeps (U0, U1, U2, Un) in slot n - n0 and writes its result into the
  // next slot's U0.  The last step's result (only needed at the end of the run,
  // need_final) goes to ucur.
  auto record_segment = [&](int n0, int n1, bool need_final) {
    reset_steps(c, 0.0, dt);
    enqueue_alpha_full(c, s->segbuf, 0);
    for (int n = n0; n < n1; ++n) {
      double* S0 = s->segbuf + (size_t)(4 * (n - n0)) * L;
      double *S1 = S0 + L, *S2 = S0 + 2 * L, *SN = S0 + 3 * L;
      const bool last = n + 1 == n1;
      double* next = last ? s->ucur : S0 + 4 * L;
      const int par = (n - n0) & 1;
      fam::launch_step_begin(c->st, 1, par, dt, 0.0, st);
      enqueue_stage(c, 0, par, S0, S0, S1, nullptr);
      enqueue_stage(c, 1, par, S0, S1, S2, nullptr);
      if (c->oe == FAM_OE_OFF) {
        if (!last || need_final) enqueue_stage(c, 2, par, S0, S2, next, nullptr);
      } else {
        enqueue_stage(c, 2, par, S0, S2, SN, nullptr);
        if (!last || need_final) enqueue_oe(c, par, SN, next, nullptr);
      }
    }
  };

  // forward pass: checkpoints at the start of every segment but the last, which
  // is recorded directly (same kernels and launch path as fam_step)
  reset_steps(c, 0.0, dt);
  enqueue_alpha_full(c, s->ucur, 0);
  const int last_n0 = (ncp - 1) * every;
  for (int n = 0; n < last_n0; ++n) {
    if (n % every == 0)
      if (hipMemcpyAsync(s->ckpt + (size_t)(n / every) * L, s->ucur, bytes, hipMemcpyDeviceToDevice, st) !=
          hipSuccess)
        return FAM_ERR_DEVICE;
    enqueue_step(c, s->ucur, n & 1, dt, 0.0);
  }
  if (hipMemcpyAsync(s->segbuf, s->ucur, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) return FAM_ERR_DEVICE;
  record_segment(last_n0, nsteps, true);

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
  for (int sg = ncp - 1; sg >= 0; --sg) {
    const int n0 = sg * every, n1 = std::min(nsteps, n0 + every);
    if (sg < ncp - 1) {
      if (hipMemcpyAsync(s->segbuf, s->ckpt + (size_t)sg * L, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return FAM_ERR_DEVICE;
      record_segment(n0, n1, false);
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
      //   lam2 = 2/3 lamN + R^T(U2)(2/3 dt lamN),  lam0 = 1/3 lamN
      rT_apply<K>(c, m, S2, s->lamN, 2.0 / 3.0, dt, s->lam2, 0, s->lam0, 1.0 / 3.0, 0, st);
      // stage 1: U2 = 3/4 U0 + 1/4 (U1 + dt R(U1))
      //   lam1 = 1/4 lam2 + R^T(U1)(1/4 dt lam2),  lam0 += 3/4 lam2
      rT_apply<K>(c, m, S1, s->lam2, 0.25, dt, s->lam1, 0, s->lam0, 0.75, 1, st);
      // stage 0: U1 = U0 + dt R(U0)
      //   lam0 += lam1 + R^T(U0)(dt lam1)
      rT_apply<K>(c, m, S0, s->lam1, 1.0, dt, s->lam0, 1, nullptr, 0.0, 0, st);
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
      f.bc_y != FAM_BC_PERIODIC || f.dmr || f.char_vars || c->oe == FAM_OE_TYPE1 || c->pp || (c->k == 6 && c->k6t))
    return FAM_ERR_STATE;
  // the forward and recomputation passes step the context; its clock is put back
  std::vector<double> clock;
  fam_status r = save_clock(c, &clock);
  if (r != FAM_OK) return r;
  switch (c->k) {
    case 3: r = adjoint_k<3>(c, U0, nsteps, dt, checkpoint_every, dJdUT, dJdU0, J_out); break;
    case 4: r = adjoint_k<4>(c, U0, nsteps, dt, checkpoint_every, dJdUT, dJdU0, J_out); break;
    case 5: r = adjoint_k<5>(c, U0, nsteps, dt, checkpoint_every, dJdUT, dJdU0, J_out); break;
    case 6: r = adjoint_k<6>(c, U0, nsteps, dt, checkpoint_every, dJdUT, dJdU0, J_out); break;
    default: return FAM_ERR_ARG;
  }
  const fam_status rc = restore_clock(c, clock);
  return r != FAM_OK ? r : rc;
}
