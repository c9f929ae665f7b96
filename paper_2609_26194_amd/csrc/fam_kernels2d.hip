// fam_kernels2d.hip - HIP kernels of the 2D FAM step for gfx950.
//
// Work decomposition ("marching strips").  One 64-lane wavefront owns a strip of
// columns: lane l holds column i = i0 - 1 + l.  Lanes 1..62 produce output;
// lanes 0 and 63 are ring columns whose traces feed the strip's two boundary
// faces.  The wave marches upwards over the rows j0-1 .. j0+H (the first and last
// are ring rows), keeping a rolling window of four state rows (12 planes x 66
// columns) in LDS.  Every face flux is evaluated exactly once per strip:
//   x-faces: a lane's right trace is passed to the right neighbour lane by a
//            cross-lane shuffle, and the resulting face flux is passed back;
//   y-faces: the top trace of row r is kept in registers for row r+1.
// The residual of a cell is complete one row later (after its top face), when
// the Shu-Osher update writes the stage result.
//
// Stage s (eq. 12): Uout = a U0 + b (Us + dt R(Us)), R of eq. (11):
//   R0 = -(Fb_{i+1/2} - Fb_{i-1/2})/dx - (Gb_{j+1/2} - Gb_{j-1/2})/dy
//   R1 = V1/dx - (Fb_{i+1/2} + Fb_{i-1/2})/(2dx) - (Gt_{j+1/2} - Gt_{j-1/2})/dy
//   R2 = V2/dy - (Gb_{j+1/2} + Gb_{j-1/2})/(2dy) - (Ft_{i+1/2} - Ft_{i-1/2})/dx
// with Fb = sum_g w_g F(eta_g), Ft = sum_g w_g eta_g F(eta_g) on x-faces (likewise
// Gb, Gt with xi_g on y-faces), V1, V2 the 4x4 Gauss averages of f1, f2, and the
// Lax-Friedrichs flux using one wave speed per direction: the maximum spectral
// radius over the cell averages of Us.  Each stage also max-reduces the wave
// speeds of its output averages for the next stage (and, after the last stage,
// for the next step's time step).
//
// OE (eqs. 2dOE_sol, 2dOE_system, Table sigma2d): per component, face-centre jumps
// of the reconstruction, J^x, J^y, the Type I / Type II denominator over the 3x3
// patch; sigma = max over components; delta = exp(-beta^x dt sigma^x/dx -
// beta^y dt sigma^y/dy); first moments scaled by delta, averages copied.
#include "fam_device.h"
#include "fam_kernels.h"

namespace fam {

constexpr int LANES = 64;
constexpr int SCOLS = LANES + 2;   // LDS columns: i0-2 .. i0+63
constexpr int NPL = 12;            // planes held in LDS for up to 4 components x 3 moments

// Gauss node q = 0..3 at -GS1, -GS0, +GS0, +GS1
__device__ __forceinline__ constexpr int qnode(int q) { return (q == 0 || q == 3) ? 1 : 0; }
__device__ __forceinline__ constexpr double qsign(int q) { return q < 2 ? -1.0 : 1.0; }
__device__ __forceinline__ constexpr double qw(int q) { return (q == 0 || q == 3) ? GW1 : GW0; }
__device__ __forceinline__ constexpr double qx(int q) {
  return q == 0 ? -GS1 : q == 1 ? -GS0 : q == 2 ? GS0 : GS1;
}

// even / odd partial contractions over the y-degree: E[m][w], O[m][w] at
// w = 0 (GS0), 1 (GS1), 2 (1/2), 3 (0; even part only)
template <int NCF, int MD>
__device__ __forceinline__ void contract_y(const double* c, double (&E)[MD + 1][4],
                                           double (&O)[MD + 1][3]) {
#pragma unroll
  for (int m = 0; m <= MD; ++m) {
#pragma unroll
    for (int w = 0; w < 4; ++w) E[m][w] = 0.0;
#pragma unroll
    for (int w = 0; w < 3; ++w) O[m][w] = 0.0;
  }
#pragma unroll
  for (int l = 0; l < NCF; ++l) {
    const int m = AX[l], b = AY[l];
    if (b % 2 == 0) {
#pragma unroll
      for (int w = 0; w < 3; ++w) E[m][w] = fma(c[l], legn(b, w), E[m][w]);
      E[m][3] = fma(c[l], leg(b, 0.0), E[m][3]);
    } else {
#pragma unroll
      for (int w = 0; w < 3; ++w) O[m][w] = fma(c[l], legn(b, w), O[m][w]);
    }
  }
}

// p(xi, eta) with xi = sx * node(gx), eta = sy * node(gy); node 2 = 1/2
template <int MD>
__device__ __forceinline__ double eval_pt(const double (&E)[MD + 1][4], const double (&O)[MD + 1][3],
                                          int gx, double sx, int gy, double sy) {
  double ev = 0.0, od = 0.0;
#pragma unroll
  for (int m = 0; m <= MD; ++m) {
    const double Qm = E[m][gy] + sy * O[m][gy];
    if (m % 2 == 0)
      ev = fma(legn(m, gx), Qm, ev);
    else
      od = fma(legn(m, gx), Qm, od);
  }
  return ev + sx * od;
}

// ---------------------------------------------------------------------------
// LDS row window
// ---------------------------------------------------------------------------
struct Window {
  double v[4][NPL][SCOLS];
};

__device__ __forceinline__ int slot_of(int r) { return r & 3; }

// load row r (BC-mapped) of planes [0, npl) for columns i0-2 .. i0+63 into regs
template <int NPLU>
__device__ __forceinline__ void fetch_row(const double* __restrict__ U, const Inst& in, int i0,
                                          int r, int lane, double (&reg)[2][NPLU]) {
  const int gj = ghost(r, in.ny, in.bcy);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int col = lane + h * LANES;
    if (col < SCOLS) {
      const int gi = ghost(i0 - 2 + col, in.nx, in.bcx);
      const size_t base = (size_t)gj * in.nx + gi;
#pragma unroll
      for (int p = 0; p < NPLU; ++p) reg[h][p] = U[p * in.plane + base];
    }
  }
}

template <int NPLU>
__device__ __forceinline__ void store_row(Window& W, int slot, int lane, const double (&reg)[2][NPLU]) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int col = lane + h * LANES;
    if (col < SCOLS) {
#pragma unroll
      for (int p = 0; p < NPLU; ++p) W.v[slot][p][col] = reg[h][p];
    }
  }
}

// stencil of component c for the cell in LDS column col, row slots sl (r-1), sm, sh
template <int K>
__device__ __forceinline__ void gather(const Window& W, int c, int col, int sl, int sm, int sh,
                                       double (&u0)[9], double (&u1)[9], double (&u2)[9]) {
  const int sr[3] = {sl, sm, sh};
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int l = b * 3 + a;
      u0[l] = W.v[sr[b]][c * 3 + 0][col - 1 + a];
      const bool x_used = (K >= 5) ? (l != 1 && l != 7) : (l == 4);
      const bool y_used = (K >= 5) ? (l != 3 && l != 5) : (l == 4);
      u1[l] = x_used ? W.v[sr[b]][c * 3 + 1][col - 1 + a] : 0.0;
      u2[l] = y_used ? W.v[sr[b]][c * 3 + 2][col - 1 + a] : 0.0;
    }
}

// ---------------------------------------------------------------------------
// stage tile
// ---------------------------------------------------------------------------
template <int K, class P>
__device__ void stage_tile(const P& phys, const StageArgs& A, const Inst& in, int i0, int j0, int H,
                           Window& W, double& amax_x, double& amax_y, bool& bad) {
  constexpr int NC = P::NC;
  constexpr int NCF = ncoef2d(K);
  constexpr int MD = maxdeg(K);
  constexpr int NPLU = NC * 3;
  const int lane = threadIdx.x;
  const int col = lane + 1;
  const int i = i0 - 1 + lane;
  const int rend = min(j0 + H, in.ny);          // exclusive end of output rows
  const bool out_lane = lane >= 1 && lane <= 62 && i < in.nx;
  const double dx = in.dx, dy = in.dy;
  const double ax = in.alpha_in[0], ay = in.alpha_in[1];
  const double dt = *in.dt;
  const double* __restrict__ Us = A.Us + in.offset;
  const double* __restrict__ U0 = A.U0 + in.offset;
  double* __restrict__ Uo = A.Uout + in.offset;

  double reg[2][NPLU];
  // prologue: rows j0-2, j0-1, j0
#pragma unroll 1
  for (int r = j0 - 2; r <= j0; ++r) {
    fetch_row<NPLU>(Us, in, i0, r, lane, reg);
    store_row<NPLU>(W, slot_of(r), lane, reg);
  }
  __syncthreads();

  double prevTop[NC][4];     // top trace of the row below (face j-1/2 of the current row)
  double part[NC][3];        // residual of the row below without its top face
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int q = 0; q < 4; ++q) prevTop[c][q] = 0.0;

#pragma unroll 1
  for (int r = j0 - 1; r <= rend; ++r) {
    const bool pre = (r + 2 <= rend + 1);
    if (pre) fetch_row<NPLU>(Us, in, i0, r + 2, lane, reg);
    const int sl = slot_of(r - 1), sm = slot_of(r), sh = slot_of(r + 1);
    const bool ring_lo = (r == j0 - 1), ring_hi = (r == rend);

    // reconstruction of all components
    double cf[NC][NCF];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double u0[9], u1[9], u2[9];
      gather<K>(W, c, col, sl, sm, sh, u0, u1, u2);
      double tmp[23];
      coeffs2d<K>(u0, u1, u2, tmp, false);
#pragma unroll
      for (int l = 0; l < NCF; ++l) cf[c][l] = tmp[l];
    }

    // traces on the four faces
    double bt[NC][4], tt[NC][4], lt[NC][4], rt[NC][4];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double E[MD + 1][4], O[MD + 1][3];
      contract_y<NCF, MD>(cf[c], E, O);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        rt[c][q] = eval_pt<MD>(E, O, 2, 1.0, qnode(q), qsign(q));
        lt[c][q] = eval_pt<MD>(E, O, 2, -1.0, qnode(q), qsign(q));
        tt[c][q] = eval_pt<MD>(E, O, qnode(q), qsign(q), 2, 1.0);
        bt[c][q] = eval_pt<MD>(E, O, qnode(q), qsign(q), 2, -1.0);
      }
    }

    // y-face below the current row: (i, r-1/2)
    double Gb[NC], Gt[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) Gb[c] = Gt[c] = 0.0;
    if (!ring_lo) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double ul[NC], ur[NC], fl[NC], fr[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) { ul[c] = prevTop[c][q]; ur[c] = bt[c][q]; }
        phys.flux(1, ul, fl);
        phys.flux(1, ur, fr);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const double fh = 0.5 * (fl[c] + fr[c]) - 0.5 * ay * (ur[c] - ul[c]);
          Gb[c] = fma(qw(q), fh, Gb[c]);
          Gt[c] = fma(qw(q) * qx(q), fh, Gt[c]);
        }
      }
    }

    // finish the row below: its top face is this row's bottom face
    if (r - 1 >= j0 && out_lane) {
      const int jj = r - 1;
      const size_t idx = (size_t)jj * in.nx + i;
      double nu[NC][3];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const double R0 = part[c][0] - Gb[c] / dy;
        const double R1 = part[c][1] - Gt[c] / dy;
        const double R2 = part[c][2] - Gb[c] / (2.0 * dy);
        const double Rm[3] = {R0, R1, R2};
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const double us = W.v[sl][c * 3 + m][col];
          const double L = us + dt * Rm[m];
          double v;
          if (A.ca == 0.0)
            v = L;
          else
            v = A.ca * U0[(c * 3 + m) * in.plane + idx] + A.cb * L;
          nu[c][m] = v;
          Uo[(c * 3 + m) * in.plane + idx] = v;
        }
      }
      double avg[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) avg[c] = nu[c][0];
      amax_x = fmax(amax_x, phys.speed(0, avg, bad));
      amax_y = fmax(amax_y, phys.speed(1, avg, bad));
    }
    if (ring_hi) break;

    // carry this row's top trace
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int q = 0; q < 4; ++q) prevTop[c][q] = tt[c][q];

    if (!ring_lo) {
      // x-face left of this lane: (i-1/2, r); left state = right trace of lane-1
      double Fb[NC], Ft[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) Fb[c] = Ft[c] = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double ul[NC], ur[NC], fl[NC], fr[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          ul[c] = __shfl_up(rt[c][q], 1, LANES);
          ur[c] = lt[c][q];
        }
        phys.flux(0, ul, fl);
        phys.flux(0, ur, fr);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const double fh = 0.5 * (fl[c] + fr[c]) - 0.5 * ax * (ur[c] - ul[c]);
          Fb[c] = fma(qw(q), fh, Fb[c]);
          Ft[c] = fma(qw(q) * qx(q), fh, Ft[c]);
        }
      }
      double FbR[NC], FtR[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        FbR[c] = __shfl_down(Fb[c], 1, LANES);
        FtR[c] = __shfl_down(Ft[c], 1, LANES);
      }
      // volume terms: 4x4 Gauss points
      double V1[NC], V2[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) V1[c] = V2[c] = 0.0;
#pragma unroll
      for (int qy = 0; qy < 4; ++qy) {
        double vals[4][NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          double E[MD + 1][4], O[MD + 1][3];
          contract_y<NCF, MD>(cf[c], E, O);
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) vals[qq][c] = eval_pt<MD>(E, O, qnode(qq), qsign(qq), qnode(qy), qsign(qy));
        }
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          double f1[NC], f2[NC];
          phys.flux(0, vals[qq], f1);
          phys.flux(1, vals[qq], f2);
          const double w = qw(qq) * qw(qy);
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            V1[c] = fma(w, f1[c], V1[c]);
            V2[c] = fma(w, f2[c], V2[c]);
          }
        }
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        part[c][0] = -(FbR[c] - Fb[c]) / dx + Gb[c] / dy;
        part[c][1] = V1[c] / dx - (FbR[c] + Fb[c]) / (2.0 * dx) + Gt[c] / dy;
        part[c][2] = V2[c] / dy + Gb[c] * (-1.0 / (2.0 * dy)) - (FtR[c] - Ft[c]) / dx;
      }
    }

    // rotate the window: row r+2 replaces row r-2
    __syncthreads();
    if (pre) store_row<NPLU>(W, slot_of(r + 2), lane, reg);
    __syncthreads();
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// OE tile
// ---------------------------------------------------------------------------
template <int K, class P>
__device__ void oe_tile(const P& phys, const OEArgs& A, const Inst& in, int i0, int j0, int H,
                        Window& W, bool& bad) {
  constexpr int NC = P::NC;
  constexpr int NCF = (K == 6) ? 23 : ncoef2d(K);
  constexpr int MD = (K == 6) ? 5 : maxdeg(K);
  constexpr int NPLU = NC * 3;
  const int lane = threadIdx.x;
  const int col = lane + 1;
  const int i = i0 - 1 + lane;
  const int rend = min(j0 + H, in.ny);
  const bool out_lane = lane >= 1 && lane <= 62 && i < in.nx;
  const double dt = *in.dt;
  const bool full = (K == 6) && A.k6_table;
  const double* __restrict__ Un = A.Un + in.offset;
  double* __restrict__ Uo = A.Uout + in.offset;

  double reg[2][NPLU];
#pragma unroll 1
  for (int r = j0 - 2; r <= j0; ++r) {
    fetch_row<NPLU>(Un, in, i0, r, lane, reg);
    store_row<NPLU>(W, slot_of(r), lane, reg);
  }
  __syncthreads();

  double prevTopC[NC];     // face-centre value at the top of the row below
  double prevJb[NC];       // |jump| at the bottom face of the row below
  double pJx[NC];          // J^x of the row below
  double pD[NC], pEps[NC]; // Type II denominators of the row below
  double pbx = 0.0, pby = 0.0;
#pragma unroll
  for (int c = 0; c < NC; ++c) prevTopC[c] = prevJb[c] = pJx[c] = pD[c] = pEps[c] = 0.0;

#pragma unroll 1
  for (int r = j0 - 1; r <= rend; ++r) {
    const bool pre = (r + 2 <= rend + 1);
    if (pre) fetch_row<NPLU>(Un, in, i0, r + 2, lane, reg);
    const int sl = slot_of(r - 1), sm = slot_of(r), sh = slot_of(r + 1);
    const bool ring_lo = (r == j0 - 1);

    double ctr_r[NC], ctr_l[NC], ctr_t[NC], ctr_b[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double u0[9], u1[9], u2[9];
      gather<K>(W, c, col, sl, sm, sh, u0, u1, u2);
      double cf[23];
      coeffs2d<K>(u0, u1, u2, cf, full);
      if (!full) {
#pragma unroll
        for (int l = ncoef2d(K); l < 23; ++l) cf[l] = 0.0;
      }
      double E[MD + 1][4], O[MD + 1][3];
      contract_y<NCF, MD>(cf, E, O);
      // face centres: (+-1/2, 0) and (0, +-1/2)
      double ev = 0.0, od = 0.0, tv = 0.0, bv = 0.0;
#pragma unroll
      for (int m = 0; m <= MD; ++m) {
        if (m % 2 == 0) {
          ev = fma(legn(m, 2), E[m][3], ev);
          tv = fma(leg(m, 0.0), E[m][2] + O[m][2], tv);
          bv = fma(leg(m, 0.0), E[m][2] - O[m][2], bv);
        } else {
          od = fma(legn(m, 2), E[m][3], od);
        }
      }
      ctr_r[c] = ev + od;
      ctr_l[c] = ev - od;
      ctr_t[c] = tv;
      ctr_b[c] = bv;
    }

    // |jump| at the bottom face of this row (row below's top face)
    double Jb[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) Jb[c] = fabs(ctr_b[c] - prevTopC[c]);

    // finish the row below
    if (r - 1 >= j0 && out_lane) {
      const size_t idx = (size_t)(r - 1) * in.nx + i;
      double sx = 0.0, sy = 0.0;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const double Jy = prevJb[c] + Jb[c];
        double sgx = 0.0, sgy = 0.0;
        if (!(pD[c] < pEps[c])) {
          sgx = A.gamma_k * pJx[c] / pD[c];
          sgy = A.gamma_k * Jy / pD[c];
        }
        sx = fmax(sx, sgx);
        sy = fmax(sy, sgy);
      }
      const double delta = exp(-pbx * dt * sx / in.dx - pby * dt * sy / in.dy);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        Uo[(c * 3 + 0) * in.plane + idx] = W.v[sl][c * 3 + 0][col];
        Uo[(c * 3 + 1) * in.plane + idx] = W.v[sl][c * 3 + 1][col] * delta;
        Uo[(c * 3 + 2) * in.plane + idx] = W.v[sl][c * 3 + 2][col] * delta;
      }
    }
    if (r == rend) break;

    // this row: J^x, denominators and wave-speed bounds over the 3x3 patch
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double jl = ctr_l[c] - __shfl_up(ctr_r[c], 1, LANES);
      const double jr = __shfl_down(jl, 1, LANES);
      pJx[c] = fabs(jl) + fabs(jr);
      prevJb[c] = Jb[c];
      prevTopC[c] = ctr_t[c];
    }
    if (!ring_lo) {
      const int srow[3] = {sl, sm, sh};
      double bx = 0.0, by = 0.0;
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          double avg[NC];
#pragma unroll
          for (int c = 0; c < NC; ++c) avg[c] = W.v[srow[b]][c * 3][col - 1 + a];
          bx = fmax(bx, phys.speed(0, avg, bad));
          by = fmax(by, phys.speed(1, avg, bad));
        }
      pbx = bx;
      pby = by;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        if (A.type == 2) {
          double S = 0.0, mabs = 0.0;
#pragma unroll
          for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              const double v = W.v[srow[b]][c * 3][col - 1 + a];
              S += v;
              mabs = fmax(mabs, fabs(v));
            }
          double D = 0.0;
#pragma unroll
          for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int a = 0; a < 3; ++a) D = fmax(D, fabs(W.v[srow[b]][c * 3][col - 1 + a] - S));
          pD[c] = D;
          pEps[c] = 1e-14 * fmax(mabs, 1.0);
        } else {
          pD[c] = A.stats[in.id * 8 + c];       // D_Omega
          pEps[c] = A.stats[in.id * 8 + 4 + c]; // eps_Omega
        }
      }
    }

    __syncthreads();
    if (pre) store_row<NPLU>(W, slot_of(r + 2), lane, reg);
    __syncthreads();
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// kernels: single instance (grid = strips x row blocks) and batched persistent
// ---------------------------------------------------------------------------
template <class P>
__device__ __forceinline__ P make_phys(const PhysParams& pp);
template <>
__device__ __forceinline__ Advection make_phys<Advection>(const PhysParams& pp) {
  return Advection{pp.ax, pp.ay};
}
template <>
__device__ __forceinline__ Burgers make_phys<Burgers>(const PhysParams& pp) {
  return Burgers{pp.ax, pp.ay};
}
template <>
__device__ __forceinline__ Euler<2> make_phys<Euler<2>>(const PhysParams& pp) {
  return Euler<2>{pp.gamma};
}

__device__ __forceinline__ void flush_wave_results(double amax_x, double amax_y, bool bad,
                                                   double* alpha_out, int* flag) {
  amax_x = wave_max(amax_x);
  amax_y = wave_max(amax_y);
  const bool any_bad = __any(bad);
  if (threadIdx.x == 0) {
    if (alpha_out) {
      atomic_max_nonneg(&alpha_out[0], amax_x);
      atomic_max_nonneg(&alpha_out[1], amax_y);
    }
    if (any_bad) atomicOr(flag, 1);
  }
}

template <int K, class P>
__global__ void __launch_bounds__(LANES) stage2d_kernel(StageArgs A, Inst in, int H) {
  __shared__ Window W;
  if (*A.done) return;
  const P phys = make_phys<P>(A.phys);
  double amx = 0.0, amy = 0.0;
  bool bad = false;
  const int i0 = blockIdx.x * 62;
  const int j0 = blockIdx.y * H;
  stage_tile<K, P>(phys, A, in, i0, j0, H, W, amx, amy, bad);
  flush_wave_results(amx, amy, bad, in.alpha_out, A.flag);
}

template <int K, class P>
__global__ void __launch_bounds__(LANES) stage2d_batched_kernel(StageArgs A, const Inst* __restrict__ insts,
                                                                const int4* __restrict__ work, int nwork) {
  __shared__ Window W;
  const P phys = make_phys<P>(A.phys);
  bool bad = false;
#pragma unroll 1
  for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
    const int4 it = work[w];              // (instance, i0, j0, H)
    const Inst in = insts[it.x];
    if (in.done && *in.done) continue;
    double amx = 0.0, amy = 0.0;
    stage_tile<K, P>(phys, A, in, it.y, it.z, it.w, W, amx, amy, bad);
    flush_wave_results(amx, amy, false, in.alpha_out, A.flag);
  }
  if (__any(bad) && threadIdx.x == 0) atomicOr(A.flag, 1);
}

template <int K, class P>
__global__ void __launch_bounds__(LANES) oe2d_kernel(OEArgs A, Inst in, int H) {
  __shared__ Window W;
  if (*A.done) return;
  const P phys = make_phys<P>(A.phys);
  bool bad = false;
  oe_tile<K, P>(phys, A, in, blockIdx.x * 62, blockIdx.y * H, H, W, bad);
  if (__any(bad) && threadIdx.x == 0) atomicOr(A.flag, 1);
}

template <int K, class P>
__global__ void __launch_bounds__(LANES) oe2d_batched_kernel(OEArgs A, const Inst* __restrict__ insts,
                                                             const int4* __restrict__ work, int nwork) {
  __shared__ Window W;
  const P phys = make_phys<P>(A.phys);
  bool bad = false;
#pragma unroll 1
  for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
    const int4 it = work[w];
    const Inst in = insts[it.x];
    if (in.done && *in.done) continue;
    oe_tile<K, P>(phys, A, in, it.y, it.z, it.w, W, bad);
  }
  if (__any(bad) && threadIdx.x == 0) atomicOr(A.flag, 1);
}

// ---------------------------------------------------------------------------
// reductions over cell averages
// ---------------------------------------------------------------------------
// alpha_out[inst] = max over cells of the spectral radii at the averages
template <class P>
__global__ void __launch_bounds__(256) alpha2d_kernel(PhysParams pp, const double* __restrict__ U,
                                                      const Inst* __restrict__ insts, int ninst, int* flag) {
  const P phys = make_phys<P>(pp);
  constexpr int NC = P::NC;
  bool bad = false;
  for (int inst = blockIdx.y; inst < ninst; inst += gridDim.y) {
    const Inst in = insts[inst];
    const size_t n = (size_t)in.nx * in.ny;
    double mx = 0.0, my = 0.0;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
         idx += (size_t)gridDim.x * blockDim.x) {
      double avg[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) avg[c] = U[in.offset + (c * 3) * in.plane + idx];
      mx = fmax(mx, phys.speed(0, avg, bad));
      my = fmax(my, phys.speed(1, avg, bad));
    }
    mx = wave_max(mx);
    my = wave_max(my);
    if ((threadIdx.x & 63) == 0) {
      atomic_max_nonneg(&in.alpha_out[0], mx);
      atomic_max_nonneg(&in.alpha_out[1], my);
    }
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// Type I statistics, pass 1: per-block partial sums and max |u| of each component
__global__ void __launch_bounds__(256) type1_pass1_kernel(const double* __restrict__ U, Inst in, int nc,
                                                          int nmom, double* __restrict__ partial) {
  __shared__ double red[4][4];
  const size_t n = (size_t)in.nx * in.ny;
  for (int c = 0; c < nc; ++c) {
    double s = 0.0;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
         idx += (size_t)gridDim.x * blockDim.x)
      s += U[in.offset + (c * nmom) * in.plane + idx];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[c][threadIdx.x >> 6] = s;
  }
  __syncthreads();
  if (threadIdx.x < nc) {
    const int c = threadIdx.x;
    partial[blockIdx.x * 4 + c] = ((red[c][0] + red[c][1]) + red[c][2]) + red[c][3];
  }
}

// pass 2 (one block): mean; pass 3: D_Omega = max |u - mean|, eps from max |u|
__global__ void type1_mean_kernel(const double* __restrict__ partial, int nblocks, Inst in, int nc,
                                  double* __restrict__ stats, double* __restrict__ dmax) {
  if (threadIdx.x < 8) dmax[threadIdx.x] = 0.0;
  if (threadIdx.x < nc) {
    const int c = threadIdx.x;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += partial[b * 4 + c];
    stats[in.id * 8 + c] = s / ((double)in.nx * in.ny);   // mean (replaced by D below)
    stats[in.id * 8 + 4 + c] = 0.0;
  }
}

__global__ void __launch_bounds__(256) type1_pass3_kernel(const double* __restrict__ U, Inst in, int nc,
                                                          int nmom, const double* __restrict__ mean,
                                                          double* __restrict__ dmax) {
  const size_t n = (size_t)in.nx * in.ny;
  for (int c = 0; c < nc; ++c) {
    const double mu = mean[in.id * 8 + c];
    double d = 0.0, a = 0.0;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
         idx += (size_t)gridDim.x * blockDim.x) {
      const double v = U[in.offset + (c * nmom) * in.plane + idx];
      d = fmax(d, fabs(v - mu));
      a = fmax(a, fabs(v));
    }
    d = wave_max(d);
    a = wave_max(a);
    if ((threadIdx.x & 63) == 0) {
      atomic_max_nonneg(&dmax[c], d);
      atomic_max_nonneg(&dmax[4 + c], a);
    }
  }
}

__global__ void type1_final_kernel(const double* __restrict__ dmax, Inst in, int nc,
                                   double* __restrict__ stats) {
  if (threadIdx.x < nc) {
    const int c = threadIdx.x;
    stats[in.id * 8 + c] = dmax[c];
    stats[in.id * 8 + 4 + c] = 1e-14 * fmax(dmax[4 + c], 1.0);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int K, class P>
static void launch_stage2d_t(const StageArgs& A, const Inst& in, int H, hipStream_t s) {
  dim3 grid((in.nx + 61) / 62, (in.ny + H - 1) / H);
  hipLaunchKernelGGL((stage2d_kernel<K, P>), grid, dim3(LANES), 0, s, A, in, H);
}
template <int K, class P>
static void launch_oe2d_t(const OEArgs& A, const Inst& in, int H, hipStream_t s) {
  dim3 grid((in.nx + 61) / 62, (in.ny + H - 1) / H);
  hipLaunchKernelGGL((oe2d_kernel<K, P>), grid, dim3(LANES), 0, s, A, in, H);
}
template <int K, class P>
static void launch_stage2d_b(const StageArgs& A, const Inst* insts, const int4* work, int nwork, int nblocks,
                             hipStream_t s) {
  hipLaunchKernelGGL((stage2d_batched_kernel<K, P>), dim3(nblocks), dim3(LANES), 0, s, A, insts, work, nwork);
}
template <int K, class P>
static void launch_oe2d_b(const OEArgs& A, const Inst* insts, const int4* work, int nwork, int nblocks,
                          hipStream_t s) {
  hipLaunchKernelGGL((oe2d_batched_kernel<K, P>), dim3(nblocks), dim3(LANES), 0, s, A, insts, work, nwork);
}

#define FAM_DISPATCH_K(K_, BODY)         \
  switch (K_) {                          \
    case 3: { constexpr int KK = 3; BODY; } break; \
    case 4: { constexpr int KK = 4; BODY; } break; \
    case 5: { constexpr int KK = 5; BODY; } break; \
    case 6: { constexpr int KK = 6; BODY; } break; \
    default: break;                      \
  }

#define FAM_DISPATCH_P(SYS_, BODY)                          \
  switch (SYS_) {                                           \
    case 0: { using PP = Advection; BODY; } break;          \
    case 1: { using PP = Burgers; BODY; } break;            \
    default: { using PP = Euler<2>; BODY; } break;          \
  }

void launch_stage2d(int k, int sys, const StageArgs& A, const Inst& in, int H, hipStream_t s) {
  FAM_DISPATCH_P(sys, FAM_DISPATCH_K(k, (launch_stage2d_t<KK, PP>(A, in, H, s))));
}
void launch_oe2d(int k, int sys, const OEArgs& A, const Inst& in, int H, hipStream_t s) {
  FAM_DISPATCH_P(sys, FAM_DISPATCH_K(k, (launch_oe2d_t<KK, PP>(A, in, H, s))));
}
void launch_stage2d_batched(int k, int sys, const StageArgs& A, const Inst* insts, const int4* work, int nwork,
                            int nblocks, hipStream_t s) {
  FAM_DISPATCH_P(sys, FAM_DISPATCH_K(k, (launch_stage2d_b<KK, PP>(A, insts, work, nwork, nblocks, s))));
}
void launch_oe2d_batched(int k, int sys, const OEArgs& A, const Inst* insts, const int4* work, int nwork,
                         int nblocks, hipStream_t s) {
  FAM_DISPATCH_P(sys, FAM_DISPATCH_K(k, (launch_oe2d_b<KK, PP>(A, insts, work, nwork, nblocks, s))));
}
void launch_alpha2d(int sys, const PhysParams& pp, const double* U, const Inst* insts, int ninst,
                    size_t max_cells, int* flag, hipStream_t s) {
  int bx = (int)std::min<size_t>((max_cells + 255) / 256, 1024);
  dim3 grid(bx < 1 ? 1 : bx, std::min(ninst, 65535));
  FAM_DISPATCH_P(sys, hipLaunchKernelGGL((alpha2d_kernel<PP>), grid, dim3(256), 0, s, pp, U, insts, ninst, flag));
}
void launch_type1_stats(const double* U, const Inst& in, int nc, int nmom, double* partial, int nblocks,
                        double* dmax, double* stats, hipStream_t s) {
  hipLaunchKernelGGL(type1_pass1_kernel, dim3(nblocks), dim3(256), 0, s, U, in, nc, nmom, partial);
  hipLaunchKernelGGL(type1_mean_kernel, dim3(1), dim3(64), 0, s, partial, nblocks, in, nc, stats, dmax);
  hipLaunchKernelGGL(type1_pass3_kernel, dim3(nblocks), dim3(256), 0, s, U, in, nc, nmom, stats, dmax);
  hipLaunchKernelGGL(type1_final_kernel, dim3(1), dim3(64), 0, s, dmax, in, nc, stats);
}

}  // namespace fam
