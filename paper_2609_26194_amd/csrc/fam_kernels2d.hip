// fam_kernels2d.hip - HIP kernels of the 2D FAM step for gfx950.
//
// Work decomposition ("marching strips").  One 64-lane wavefront owns a strip of
// columns: lane l holds column i = i0 - 2 + l.  Lanes 2..61 produce output (60
// columns); lanes 1 and 62 are ring columns whose traces feed the strip's two
// boundary faces; lanes 0 and 63 only load.  The wave marches upwards over the
// rows j0-1 .. j0+H (the first and last are ring rows), keeping a rolling window
// of three state rows (12 planes x 64 columns) in LDS.  Every face flux is evaluated exactly once per strip:
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
#include <algorithm>
#include <type_traits>
#include <utility>

#include "fam_char.h"
#include "fam_device.h"
#include "fam_eval.h"
#include "fam_kernels.h"
#include "fam_strip.h"

namespace fam {

#ifndef FAM_OE_WAVES
#define FAM_OE_WAVES 1
#endif
// occupancy targets (waves per SIMD) handed to the register allocator
#define FAM_STAGE_ATTR __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(FAM_STAGE_WAVES)))
#define FAM_OE_ATTR __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(FAM_OE_WAVES)))

// keeps the scheduler from hoisting the next component's LDS reads above this
// point (bounds the number of live stencil values); used between the OE kernel's
// per-component passes (the stage kernels schedule faster without it)
#ifndef FAM_NO_FENCE
#define FAM_SCHED_FENCE() __builtin_amdgcn_sched_barrier(0)
#else
#define FAM_SCHED_FENCE() ((void)0)
#endif

// ---------------------------------------------------------------------------
// Optional positivity limiter (Euler): the reconstruction p is replaced by
// avg + theta2 (w - avg), w = p with its density scaled by theta1 toward the
// average, theta1 and theta2 the largest values keeping density and pressure
// >= eps = min(1e-13, rho_avg, p(avg)) at all 32 flux points of the cell.
// Both scalings act on the deviation from the average, so they are applied to
// the non-constant coefficients: rho by theta1 theta2, the other components by
// theta2 (the same point values up to rounding).
// ---------------------------------------------------------------------------
// smallest root in (0, 1] of a t^2 + b t + c (c > 0 and value <= 0 at t = 1), else 1
__device__ __forceinline__ double smallest_root_unit(double a, double b, double c) {
  const double disc = fmax(b * b - 4.0 * a * c, 0.0);
  const double sq = sqrt(disc);
  const double q = -0.5 * (b + (b >= 0.0 ? sq : -sq));
  double r1 = (a == 0.0) ? 2.0 : q / a;
  double r2 = c / (q == 0.0 ? 1.0 : q);
  if (!(r1 > 0.0 && r1 <= 1.0)) r1 = 2.0;
  if (!(r2 > 0.0 && r2 <= 1.0)) r2 = 2.0;
  const double r = fmin(r1, r2);
  return r > 1.0 ? 1.0 : r;
}


// min over the 32 lanes of each half of the wave (DPP within rows of 16, then
// one exchange between the two rows of the half)
template <int CTRL>
__device__ __forceinline__ double dpp_min(double v) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(v), __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(v), __double2hiint(v), CTRL, 0xF, 0xF, false);
  return fmin(v, __hiloint2double(hi, lo));
}

__device__ __forceinline__ double half_wave_min(double v) {
  v = dpp_min<0xB1>(v);    // quad_perm [1,0,3,2]
  v = dpp_min<0x4E>(v);    // quad_perm [2,3,0,1]
  v = dpp_min<0x141>(v);   // row_half_mirror
  v = dpp_min<0x140>(v);   // row_mirror: the row minimum in all 16 lanes
  return fmin(v, __shfl_xor(v, 16, 64));
}

// LDS staging of the limiter's exact test: up to CHUNK cells of a wave at a time
// (16; 8 at k = 6, whose kernels also keep their carried traces in LDS and must
// still fit four blocks per CU)
template <int K>
struct PPStage {
  static constexpr int CHUNK = K == 6 ? 8 : 16;
  double cf[CHUNK][4 * ncoef2d(K) + 1];   // coefficients of the 4 components, eps
  double th[CHUNK][2];
  int nwork;                               // cells of this tile that needed the exact test
};

// Called by all 64 lanes of the wave (uniform control flow).  Each lane first
// runs a cheap sufficient test; the few cells that fail it (near
// discontinuities) are then tested exactly and, where needed, limited: their
// coefficients go to LDS, and each half of the wave takes one cell, lane l
// evaluating flux point l mod 32, so a cell costs the wave a few dozen
// instructions instead of a divergent 32-point loop.
template <int K, int NCF, int MD, class P>
__device__ __forceinline__ void pp_limiter(const P& phys, double (&cf)[P::NC][NCF], bool& bad, int lane,
                                           PPStage<K>& S) {
  constexpr int NC = P::NC;
  if constexpr (NC != 4) {
    return;
  } else {
    const double g = phys.g;
    double avg[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) avg[c] = cf[c][0];
    const double inv = 1.0 / avg[0];
    const double pa = phys.pressure(avg, inv);
    const bool adm = (avg[0] > 0.0) && (pa > 0.0);
    if (!adm) bad = true;
    const double eps = fmin(fmin(avg[0], pa), 1e-13);
    // cheap sufficient test: every basis function is bounded by its value at the
    // cell corner (|L_m| <= L_m(1/2) on [-1/2, 1/2]), which bounds each
    // component's deviation from its average; if density and the pressure lower
    // bound built from those deviations stay above eps (with a rounding margin),
    // no point can violate and the limiter is the identity.
    bool need = false;
    if (adm && lane >= 1 && lane <= LANES - 2) {
      double dev[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        dev[c] = 0.0;
#pragma unroll
        for (int l = 1; l < NCF; ++l) dev[c] = fma(fabs(cf[c][l]), leg(AX[l], 0.5) * leg(AY[l], 0.5), dev[c]);
      }
      const double rlo = avg[0] - dev[0];
      const double mm = fabs(avg[1]) + dev[1], nn = fabs(avg[2]) + dev[2];
      const double margin = 1e-12 * (avg[0] + dev[0] + fabs(avg[3]) + dev[3]);
      need = true;
      if (rlo > eps + margin) {
        const double plo = (g - 1.0) * (avg[3] - dev[3] - 0.5 * (mm * mm + nn * nn) / rlo);
        if (plo > eps + margin) need = false;
      }
    }
    unsigned long long todo = __ballot(need);
    if (todo == 0) return;
    if (lane == 0) S.nwork += __popcll(todo);
    // this lane's flux point: right face (1/2, eta_g), left face (-1/2, eta_g),
    // top face (xi_g, 1/2), bottom face (xi_g, -1/2), volume (xi_a, eta_b) at
    // 16 + 4 b + a
    const int pt = lane & 31, half = lane >> 5;
    const double nd[4] = {-GS1, -GS0, GS0, GS1};
    double px, py;
    if (pt < 4) { px = 0.5; py = nd[pt]; }
    else if (pt < 8) { px = -0.5; py = nd[pt - 4]; }
    else if (pt < 12) { px = nd[pt - 8]; py = 0.5; }
    else if (pt < 16) { px = nd[pt - 12]; py = -0.5; }
    else { px = nd[(pt - 16) & 3]; py = nd[(pt - 16) >> 2]; }
    double phi[NCF];
#pragma unroll
    for (int l = 0; l < NCF; ++l) phi[l] = leg(AX[l], px) * leg(AY[l], py);
    const double kk = 2.0 / (g - 1.0);
    double th1 = 1.0, th2 = 1.0;
    while (todo) {
      // the next (up to) CHUNK cells
      unsigned long long chunk = 0, rest = todo;
      int nchunk = 0;
      while (rest && nchunk < PPStage<K>::CHUNK) {
        chunk |= rest & (~rest + 1ull);
        rest &= rest - 1ull;
        ++nchunk;
      }
      todo = rest;
      const bool mine = (chunk >> lane) & 1ull;
      const int slot = __popcll(chunk & ((1ull << lane) - 1ull));
      if (mine) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int l = 0; l < NCF; ++l) S.cf[slot][c * NCF + l] = cf[c][l];
        S.cf[slot][NC * NCF] = eps;
      }
      __syncthreads();
      for (int p = 0; p < nchunk; p += 2) {
        const int cell = min(p + half, nchunk - 1);   // an odd count: both halves take the last cell
        const double* C = S.cf[cell];
        double v[NC], a[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          v[c] = 0.0;
#pragma unroll
          for (int l = 0; l < NCF; ++l) v[c] = fma(C[c * NCF + l], phi[l], v[c]);
          a[c] = C[c * NCF];
        }
        const double e = C[NC * NCF];
        // density: theta1 from the minimum over the 32 points
        const double rmin = half_wave_min(v[0]);
        const double t1 = rmin < e ? (a[0] - e) / (a[0] - rmin) : 1.0;
        // pressure along avg -> density-limited point value
        const double rho0 = a[0], m0 = a[1], n0 = a[2], E0 = a[3];
        const double w0 = rho0 + t1 * (v[0] - rho0);
        const double w[4] = {w0, v[1], v[2], v[3]};
        const double pw = phys.pressure(w, 1.0 / w0);
        double t2 = 1.0;
        if (pw < e) {
          const double qc = 2.0 * rho0 * E0 - (m0 * m0 + n0 * n0) - kk * e * rho0;
          const double rd = w0 - rho0, md = w[1] - m0, nd_ = w[2] - n0, Ed = w[3] - E0;
          const double qa = 2.0 * rd * Ed - (md * md + nd_ * nd_);
          const double qb = 2.0 * (rho0 * Ed + rd * E0) - 2.0 * (m0 * md + n0 * nd_) - kk * e * rd;
          t2 = smallest_root_unit(qa, qb, qc);
        }
        t2 = half_wave_min(t2);
        if (pt == 0) {
          S.th[cell][0] = t1;
          S.th[cell][1] = t2;
        }
      }
      __syncthreads();
      if (mine) {
        th1 = S.th[slot][0];
        th2 = S.th[slot][1];
      }
      __syncthreads();
    }
    if (th1 < 1.0 || th2 < 1.0) {
      const double t0 = th1 * th2;
#pragma unroll
      for (int l = 1; l < NCF; ++l) cf[0][l] *= t0;
#pragma unroll
      for (int c = 1; c < NC; ++c)
#pragma unroll
        for (int l = 1; l < NCF; ++l) cf[c][l] *= th2;
    }
  }
}

// ---------------------------------------------------------------------------
// stage tile
// ---------------------------------------------------------------------------
// The values a row hands to the next (its top traces, the bottom states of the
// next y-face, and its residual without the top face) stay in registers, except
// for the Euler equations at k = 6, whose 4 x 21 coefficients leave no room for
// them: there each lane keeps its own column of them in LDS.
template <int K, int NC>
__host__ __device__ constexpr bool carry_in_lds() { return K == 6 && NC == 4; }

template <bool ON>
struct StageCarry {
  double top[16][LANES];    // [component * 4 + point][lane]
  double part[NPL][LANES];  // [component * 3 + moment][lane]
};
template <>
struct StageCarry<false> {
  char unused;
};
template <int K, class P, bool PP, bool DMR = false, bool CHAR = false>
__device__ void stage_tile(const P& phys, const StageArgs& A, const Inst& in, int i0, int j0, int H,
                           Window& W, PPStage<K>& PS, StageCarry<carry_in_lds<K, P::NC>()>& T, double& amax_x,
                           double& amax_y, bool& bad) {
  constexpr int NC = P::NC;
  constexpr int NCF = ncoef2d(K);
  constexpr int MD = maxdeg(K);
  constexpr int NPLU = NC * 3;
  const int lane = threadIdx.x;
  const int col = lane;
  const int i = i0 - 2 + lane;
  const int rend = min(j0 + H, in.ny);          // exclusive end of output rows
  const bool out_lane = lane >= 2 && lane <= LANES - 3 && i < in.nx;
  const double idx_ = 1.0 / in.dx, idy = 1.0 / in.dy;
  const double i2dx = 0.5 * idx_, i2dy = 0.5 * idy;
  const double ax = in.alpha_in[0], ay = in.alpha_in[1];
  const double dt = *in.dt;
  const double tb = DMR ? *in.t_end - in.t_ofs * dt : 0.0;   // boundary time of this stage
  const bool use_u0 = A.ca != 0.0;
  const double* __restrict__ Us = A.Us + in.offset;
  const double* __restrict__ U0 = A.U0 + in.offset;
  double* __restrict__ Uo = A.Uout + in.offset;
  // moment planes of the output, as an element offset from Uout (0: Uout's own)
  const long long mom_off = A.Uout_mom ? elem_offset(A.Uout, A.Uout_mom) : 0;

  double reg[NPLU];
#pragma unroll 1
  for (int r = j0 - 2; r <= j0; ++r) {
    fetch_row<NPLU, DMR>(Us, in, i0, r, lane, reg, tb);
    store_row<NPLU>(W, slot_of(r), lane, reg);
  }
  __syncthreads();

  constexpr bool CL = carry_in_lds<K, NC>();
  double topR[CL ? 1 : NC][4];    // top trace of the row below (face j-1/2 of the current row)
  double partR[CL ? 1 : NC][3];   // residual of the row below without its top face
  auto prevTop = [&](int c, int q) -> double& {
    if constexpr (CL) return T.top[c * 4 + q][col];
    else return topR[c][q];
  };
  auto part = [&](int c, int m) -> double& {
    if constexpr (CL) return T.part[c * 3 + m][col];
    else return partR[c][m];
  };
#pragma unroll
  for (int c = 0; c < NC; ++c) {
#pragma unroll
    for (int q = 0; q < 4; ++q) prevTop(c, q) = 0.0;
#pragma unroll
    for (int m = 0; m < 3; ++m) part(c, m) = 0.0;
  }

#pragma unroll 1
  for (int r = j0 - 1; r <= rend; ++r) {
    long long t_row = 0;
    if constexpr (PP) {
      if (A.row_cost) t_row = clock64();
    }
    const bool pre = (r + 2 <= rend + 1);
    if (pre) fetch_row<NPLU, DMR>(Us, in, i0, r + 2, lane, reg, tb);
    const bool fin = (r - 1 >= j0) && out_lane;   // this iteration finishes row r-1
    double u0row[NPLU];
    if (fin && use_u0) {
      const size_t idx = (size_t)(r - 1) * in.nx + i;
#pragma unroll
      for (int p = 0; p < NPLU; ++p) u0row[p] = U0[p * in.plane + idx];
    }
    const int sl = slot_of(r - 1), sm = slot_of(r), sh = slot_of(r + 1);
    const bool ring_lo = (r == j0 - 1), ring_hi = (r == rend);

    // reconstruction of all components
    double cf[NC][NCF];
    if constexpr (CHAR) {
      // in the characteristic variables of this cell's average: transform the
      // stencil with L, reconstruct each field, map the coefficients back with R
      double La[NC][NC], Ra[NC][NC];
      {
        double a[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) a[c] = W.v[sm][c * 3][col];
        char_basis_x<2>(phys.g, a, La, Ra);
      }
#pragma unroll
      for (int w = 0; w < NC; ++w) {
        double u0[9], u1[9], u2[9];
#pragma unroll
        for (int l = 0; l < 9; ++l) u0[l] = u1[l] = u2[l] = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          double g0[9], g1[9], g2[9];
          gather<K>(W, c, col, sl, sm, sh, g0, g1, g2);
#pragma unroll
          for (int l = 0; l < 9; ++l) {
            u0[l] = fma(La[w][c], g0[l], u0[l]);
            u1[l] = fma(La[w][c], g1[l], u1[l]);
            u2[l] = fma(La[w][c], g2[l], u2[l]);
          }
        }
        double tmp[23];
        coeffs2d<K>(u0, u1, u2, tmp, false);
#pragma unroll
        for (int l = 0; l < NCF; ++l) cf[w][l] = tmp[l];
      }
#pragma unroll
      for (int l = 0; l < NCF; ++l) {
        double t[NC];
#pragma unroll
        for (int w = 0; w < NC; ++w) t[w] = cf[w][l];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          double v = 0.0;
#pragma unroll
          for (int w = 0; w < NC; ++w) v = fma(Ra[c][w], t[w], v);
          cf[c][l] = v;
        }
      }
    } else {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        double u0[9], u1[9], u2[9];
        gather<K>(W, c, col, sl, sm, sh, u0, u1, u2);
        double tmp[23];
        coeffs2d<K>(u0, u1, u2, tmp, false);
#pragma unroll
        for (int l = 0; l < NCF; ++l) cf[c][l] = tmp[l];
      }
    }

    // optional positivity limiter on this cell's reconstruction
    if constexpr (PP) pp_limiter<K, NCF, MD>(phys, cf, bad, lane, PS);

    // bottom trace -> y-face flux below the current row: (i, r-1/2)
    double Gb[NC], Gt[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) Gb[c] = Gt[c] = 0.0;
    {
      double bt[NC][4];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        double E[MD + 1][4], O[MD + 1][3];
        contract_y<NCF, MD>(cf[c], E, O);
#pragma unroll
        for (int q = 0; q < 4; ++q) bt[c][q] = eval_pt<MD>(E, O, qnode(q), qsign(q), 2, -1.0);
      }
      if (!ring_lo) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          double ul[NC], ur[NC], fl[NC], fr[NC];
#pragma unroll
          for (int c = 0; c < NC; ++c) { ul[c] = prevTop(c, q); ur[c] = bt[c][q]; }
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
    }

    // finish the row below: its top face is this row's bottom face
    if (fin) {
      const size_t idx = (size_t)(r - 1) * in.nx + i;
      double avg[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const double Rm[3] = {part(c, 0) - Gb[c] * idy, part(c, 1) - Gt[c] * idy, part(c, 2) - Gb[c] * i2dy};
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const double L = W.v[sl][c * 3 + m][col] + dt * Rm[m];
          const double v = use_u0 ? fma(A.ca, u0row[c * 3 + m] - L, L) : L;
          Uo[(c * 3 + m) * in.plane + idx + (m == 0 ? 0 : mom_off)] = v;
          if (m == 0) avg[c] = v;
        }
      }
      amax_x = fmax(amax_x, phys.speed(0, avg, bad));
      amax_y = fmax(amax_y, phys.speed(1, avg, bad));
    }
    if (ring_hi) break;

    // top trace of this row (bottom state of the next y-face)
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double E[MD + 1][4], O[MD + 1][3];
      contract_y<NCF, MD>(cf[c], E, O);
#pragma unroll
      for (int q = 0; q < 4; ++q) prevTop(c, q) = eval_pt<MD>(E, O, qnode(q), qsign(q), 2, 1.0);
    }

    if (!ring_lo) {
      // x-face left of this lane: (i-1/2, r); left state = right trace of lane-1
      double Fb[NC], Ft[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) Fb[c] = Ft[c] = 0.0;
      {
        double rt[NC][4], lt[NC][4];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          double E[MD + 1][4], O[MD + 1][3];
          contract_y<NCF, MD>(cf[c], E, O);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            rt[c][q] = eval_pt<MD>(E, O, 2, 1.0, qnode(q), qsign(q));
            lt[c][q] = eval_pt<MD>(E, O, 2, -1.0, qnode(q), qsign(q));
          }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          double ul[NC], ur[NC], fl[NC], fr[NC];
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            ul[c] = from_left(rt[c][q]);
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
      }
      double FbR[NC], FtR[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        FbR[c] = from_right(Fb[c]);
        FtR[c] = from_right(Ft[c]);
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
          phys.flux2(vals[qq], f1, f2);
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
        part(c, 0) = -(FbR[c] - Fb[c]) * idx_ + Gb[c] * idy;
        part(c, 1) = V1[c] * idx_ - (FbR[c] + Fb[c]) * i2dx + Gt[c] * idy;
        part(c, 2) = V2[c] * idy - Gb[c] * i2dy - (FtR[c] - Ft[c]) * idx_;
      }
    }

    // rotate the window: row r+2 replaces row r-1
    __syncthreads();
    if (pre) store_row<NPLU>(W, slot_of(r + 2), lane, reg);
    __syncthreads();
    if constexpr (PP) {
      // the iteration reconstructs (and limits) row r: its cost, for the next
      // launch's partition (rows of this segment only)
      if (A.row_cost && lane == 0 && r >= j0 && r < rend)
        A.row_cost[(size_t)(i0 / STRIP) * in.ny + r] = (float)(clock64() - t_row);
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// OE tile.  The four face-centre values of a cell's reconstruction, p(+-1/2, 0)
// and p(0, +-1/2), are fixed linear functionals of its 3x3 stencil moments
// (weights in fam_eval.h, folded at compile time).
// ---------------------------------------------------------------------------
template <int K, bool FULL>
__device__ __forceinline__ void centre_values(const Window& W, int c, int col, int sl, int sm, int sh,
                                              double (&out)[4]) {
  double u0[9], u1[9], u2[9];
  gather<K>(W, c, col, sl, sm, sh, u0, u1, u2);
  double u[27];
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    u[l] = u0[l];
    u[9 + l] = u1[l];
    u[18 + l] = u2[l];
  }
  using Seq = std::make_integer_sequence<int, 27>;
  out[0] = centre_dot<K, FULL, 0>(u, Seq{});
  out[1] = centre_dot<K, FULL, 1>(u, Seq{});
  out[2] = centre_dot<K, FULL, 2>(u, Seq{});
  out[3] = centre_dot<K, FULL, 3>(u, Seq{});
}

template <int K, class P, bool FULL, bool DMR = false>
__device__ void oe_tile(const P& phys, const OEArgs& A, const Inst& in, int i0, int j0, int H,
                        Window& W, double (&t1s)[8], bool& bad) {
  constexpr int NC = P::NC;
  constexpr int NPLU = NC * 3;
  const int lane = threadIdx.x;
  const int col = lane;
  const int i = i0 - 2 + lane;
  const int rend = min(j0 + H, in.ny);
  const bool out_lane = lane >= 2 && lane <= LANES - 3 && i < in.nx;
  const double dt = *in.dt;
  const double tb = DMR ? *in.t_end : 0.0;   // OE: the end of the step
  const double cx = dt / in.dx, cy = dt / in.dy;
  // averages from Ua (NULL: Un), moments from Un, as an element offset from Ua
  const double* __restrict__ Ua = (A.Ua ? A.Ua : A.Un) + in.offset;
  const long long moff = A.Ua ? elem_offset(A.Ua, A.Un) : 0;
  double* __restrict__ Uo = A.Uout + in.offset;
  const bool write_avg = !A.avg_in_place;

  // Type I: the instance's D_Omega and eps_Omega per component, read once into
  // LDS (a global load inside the row loop would make the compiler wait there
  // for every load in flight, the prefetched rows included, on either type)
  if (A.type != 2 && lane < 2 * NC) {
    const int q = lane < NC ? lane : 4 + lane - NC;   // D_Omega at 0..NC-1, eps_Omega at 4..3+NC
    t1s[q] = A.stats[in.id * 8 + q];
  }

  double reg[NPLU];
#pragma unroll 1
  for (int r = j0 - 2; r <= j0; ++r) {
    fetch_row<NPLU, DMR>(Ua, in, i0, r, lane, reg, tb, moff);
    store_row<NPLU>(W, slot_of(r), lane, reg);
  }
  __syncthreads();
  // rows are fetched two iterations ahead of their store into the window: ra holds
  // row r + 2 during iteration r, rb receives row r + 3
  double ra[NPLU], rb[NPLU];
  if (j0 + 1 <= rend + 1) fetch_row<NPLU, DMR>(Ua, in, i0, j0 + 1, lane, ra, tb, moff);

  double prevTopC[NC];     // face-centre value at the top of the row below
  double prevJb[NC];       // |jump| at the bottom face of the row below
  double pJx[NC];          // J^x of the row below
  double pD[NC], pEps[NC]; // denominators of the row below
  double pbx = 0.0, pby = 0.0;
#pragma unroll
  for (int c = 0; c < NC; ++c) prevTopC[c] = prevJb[c] = pJx[c] = pD[c] = pEps[c] = 0.0;
  // spectral radii of the rows r - 1, r (carried) and r + 1 of the current row r
  double spx[3], spy[3];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    double a1[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) a1[c] = W.v[slot_of(j0 - 2 + q)][c * 3][col];
    spx[q] = phys.speed(0, a1, bad);
    spy[q] = phys.speed(1, a1, bad);
  }
  spx[2] = spy[2] = 0.0;

#pragma unroll 1
  for (int r = j0 - 1; r <= rend; ++r) {
    const bool pre = (r + 2 <= rend + 1);
    const bool pre2 = (r + 3 <= rend + 1);
    if (pre2) fetch_row<NPLU, DMR>(Ua, in, i0, r + 3, lane, rb, tb, moff);
    const int sl = slot_of(r - 1), sm = slot_of(r), sh = slot_of(r + 1);
    const bool ring_lo = (r == j0 - 1);

    // one pass per component: the face-centre values of row r, the sigma of
    // row r - 1 (whose top face is this row's bottom face), then row r's J^x,
    // bottom jump and Type II denominator
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double ctr[4];
      centre_values<K, FULL>(W, c, col, sl, sm, sh, ctr);
      const double Jb = fabs(ctr[3] - prevTopC[c]);
      {
        const double Jy = prevJb[c] + Jb;
        if (!(pD[c] < pEps[c])) {
          const double gD = A.gamma_k / pD[c];
          sx = fmax(sx, gD * pJx[c]);
          sy = fmax(sy, gD * Jy);
        }
      }
      if (r < rend) {
        const double jl = ctr[1] - from_left(ctr[0]);
        const double jr = from_right(jl);
        pJx[c] = fabs(jl) + fabs(jr);
        prevJb[c] = Jb;
        prevTopC[c] = ctr[2];
        if (!ring_lo) {
          if (A.type == 2) {
            // S = sum, M = max, m = min of the 3x3 averages (column-wise, then
            // across the neighbouring lanes); max |v - S| = max(M - S, S - m) and
            // max |v| = max(|M|, |m|) (rounding is monotone)
            const double v0 = W.v[sl][c * 3][col], v1 = W.v[sm][c * 3][col], v2 = W.v[sh][c * 3][col];
            const double cs = v0 + v1 + v2;
            const double cM = fmax(fmax(v0, v1), v2), cmn = fmin(fmin(v0, v1), v2);
            const double S = from_left(cs) + cs + from_right(cs);
            const double M = fmax(cM, fmax(from_left(cM), from_right(cM)));
            const double mn = fmin(cmn, fmin(from_left(cmn), from_right(cmn)));
            pD[c] = fmax(M - S, S - mn);
            pEps[c] = 1e-14 * fmax(fmax(fabs(M), fabs(mn)), 1.0);
          } else {
            pD[c] = t1s[c];        // D_Omega
            pEps[c] = t1s[4 + c];  // eps_Omega
          }
        }
      }
      FAM_SCHED_FENCE();
    }

    // finish the row below
    if (r - 1 >= j0 && out_lane) {
      const size_t idx = (size_t)(r - 1) * in.nx + i;
      const double delta = exp(-pbx * cx * sx - pby * cy * sy);
      if (A.delta_out) A.delta_out[idx] = delta;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        if (write_avg) Uo[(c * 3 + 0) * in.plane + idx] = W.v[sl][c * 3 + 0][col];
        Uo[(c * 3 + 1) * in.plane + idx] = W.v[sl][c * 3 + 1][col] * delta;
        Uo[(c * 3 + 2) * in.plane + idx] = W.v[sl][c * 3 + 2][col] * delta;
      }
    }
    if (r == rend) break;

    // spectral radii of row r + 1 (each cell once; rows r - 1, r carried)
    {
      double a1[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) a1[c] = W.v[sh][c * 3][col];
      spx[2] = phys.speed(0, a1, bad);
      spy[2] = phys.speed(1, a1, bad);
    }
    if (!ring_lo) {
      // wave-speed bounds over the 3x3 patch: column maxima, then the neighbours
      double bx = fmax(fmax(spx[0], spx[1]), spx[2]);
      double by = fmax(fmax(spy[0], spy[1]), spy[2]);
      bx = fmax(bx, fmax(from_left(bx), from_right(bx)));
      by = fmax(by, fmax(from_left(by), from_right(by)));
      pbx = bx;
      pby = by;
    }
    spx[0] = spx[1];
    spx[1] = spx[2];
    spy[0] = spy[1];
    spy[1] = spy[2];

    __syncthreads();
    if (pre) store_row<NPLU>(W, slot_of(r + 2), lane, ra);
    __syncthreads();
#pragma unroll
    for (int p = 0; p < NPLU; ++p) ra[p] = rb[p];
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

// Position in a heavy-first order (nh tiles with limiter work first, then the
// others) that workgroup L of N takes: the heavy tiles in turn over the XCDs,
// the others in the XCD-aware order (each XCD a contiguous range).  A bijection
// of [0, N).
__device__ __forceinline__ int heavy_first_slot(int L, int N, int nh) {
  if (L < nh) return L;
  const int x = L % NXCD;
  int base = 0, first = 0;
  for (int q = 0; q <= x; ++q) {
    const int f = nh + ((q - nh) % NXCD + NXCD) % NXCD;   // first light position on XCD q
    const int cnt = f < N ? (N - 1 - f) / NXCD + 1 : 0;
    if (q < x) base += cnt;
    else first = f;
  }
  return nh + base + (L - first) / NXCD;
}

template <int K, class P, bool PP, bool DMR, bool CHAR = false>
__global__ void FAM_STAGE_ATTR stage2d_kernel(StageArgs A, Inst in, int H) {
  __shared__ Window W;
  __shared__ PPStage<K> PS;
  __shared__ StageCarry<carry_in_lds<K, P::NC>()> T;
  if (*A.done) return;
  const P phys = make_phys<P>(A.phys);
  double amx = 0.0, amy = 0.0;
  bool bad = false;
  int i0, j0, tile = 0;
  if constexpr (PP) {
    // 1D grid: tiles in the order of the previous launch's limiter work
    const int strips = (in.nx + STRIP - 1) / STRIP;
    // tiles with limiter work first (spread over the XCDs in turn), then the
    // others in the XCD-aware order of their row-major index
    const int N = gridDim.x;
    tile = A.tile_perm[heavy_first_slot(blockIdx.x, N, A.tile_perm[N])];
    i0 = (tile % strips) * STRIP;
    j0 = (tile / strips) * H;
    PS.nwork = 0;
  } else {
    const int T = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    i0 = (T % gridDim.x) * STRIP;
    j0 = (T / gridDim.x) * H;
  }
  stage_tile<K, P, PP, DMR, CHAR>(phys, A, in, i0, j0, H, W, PS, T, amx, amy, bad);
  flush_wave_results(amx, amy, bad, in.alpha_out, A.flag);
  if constexpr (PP) {
    if (threadIdx.x == 0) A.tile_work[tile] = PS.nwork;
  }
}

constexpr int ORDER_MIN_TILES = 1024;   // 256 CUs x 4 SIMDs, one stage wave each

// tile_perm := tiles with tile_work > 0 first, then the others, each group in
// index order (one block; each thread owns a contiguous chunk)
__global__ void __launch_bounds__(1024) tile_order_kernel(const int* __restrict__ work, int* __restrict__ perm,
                                                          int n) {
  __shared__ int cnt[1024];
  const int t = threadIdx.x, nt = blockDim.x;
  const int per = (n + nt - 1) / nt;
  const int lo = min(n, t * per), hi = min(n, lo + per);
  int heavy = 0;
  for (int k = lo; k < hi; ++k) heavy += work[k] > 0;
  cnt[t] = heavy;
  __syncthreads();
  // inclusive scan of the per-thread counts (Hillis-Steele)
  for (int off = 1; off < nt; off <<= 1) {
    const int v = t >= off ? cnt[t - off] : 0;
    __syncthreads();
    cnt[t] += v;
    __syncthreads();
  }
  const int total = cnt[nt - 1];
  if (t == 0) perm[n] = total;         // heavy tiles: read by the stage kernel
  int h = cnt[t] - heavy;              // heavy tiles before this chunk
  int l = total + (lo - h);            // light tiles go after all heavy ones
  for (int k = lo; k < hi; ++k) {
    if (work[k] > 0) perm[h++] = k;
    else perm[l++] = k;
  }
}

__global__ void tile_identity_kernel(int* __restrict__ perm, int* __restrict__ work, int n) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k <= n; k += gridDim.x * blockDim.x) {
    perm[k] = k < n ? k : 0;   // perm[n]: no tile with limiter work yet
    if (k < n) work[k] = 0;
  }
}

template <int K, class P, bool DMR, bool CHAR = false>
__global__ void FAM_STAGE_ATTR stage2d_list_kernel(StageArgs A, Inst in, const int4* __restrict__ seg,
                                                    const int* __restrict__ nseg) {
  __shared__ Window W;
  __shared__ PPStage<K> PS;
  __shared__ StageCarry<carry_in_lds<K, P::NC>()> T;
  if (*A.done) return;
  const int n = *nseg;
  if ((int)blockIdx.x >= n) return;
  // the list is ordered by row band: each XCD takes a contiguous share
  const int4 it = seg[xcd_tile(blockIdx.x, n)];
  if (it.w <= 0) return;
  const P phys = make_phys<P>(A.phys);
  double amx = 0.0, amy = 0.0;
  bool bad = false;
  PS.nwork = 0;
  stage_tile<K, P, true, DMR, CHAR>(phys, A, in, it.y, it.z, it.w, W, PS, T, amx, amy, bad);
  flush_wave_results(amx, amy, bad, in.alpha_out, A.flag);
}

// Segment list for the next limiter-on launch.  Each strip's rows are cut into
// n_s segments of equal recorded cost; n_s = ceil(C_s / (tau - R)) with C_s the
// strip's cost, R the cost of a segment's three extra ring rows (three mean
// rows) and tau the smallest per-segment bound (bisection) for which the
// segments fit the budget (one wave slot each).  Two launches:
//   part_scan_kernel (one block per strip): inclusive prefix sums of the row
//     costs and C_s;
//   part_cut_kernel (one block per strip): every block repeats the bisection
//     (same inputs, same operations, same result), takes its strip's n_s and
//     first list index, and starts segment k at the first row whose inclusive
//     prefix exceeds k C_s / n_s.
constexpr int PART_T = 1024;

// strip costs of the partition (device)
struct PartState {
  float Cs[PART_MAX_STRIPS];
};

__global__ void __launch_bounds__(PART_T) part_scan_kernel(const float* __restrict__ cost, float* __restrict__ pref,
                                                          int ny, PartState* __restrict__ ps) {
  __shared__ float sh[PART_T / 64];
  const int t = threadIdx.x, s = blockIdx.x, lane = t & 63, wv = t >> 6;
  const float* __restrict__ C = cost + (size_t)s * ny;
  float* __restrict__ P = pref + (size_t)s * ny;
  // thread t owns rows [t * per, (t + 1) * per)
  const int per = (ny + PART_T - 1) / PART_T;
  const int r0 = min(ny, t * per), r1 = min(ny, r0 + per);
  float own = 0.0f;
  for (int r = r0; r < r1; ++r) own += C[r];
  // inclusive scan of the thread sums: waves, then the wave totals
  float v = own;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const float u = __shfl_up(v, off);
    if (lane >= off) v += u;
  }
  if (lane == 63) sh[wv] = v;
  __syncthreads();
  if (wv == 0) {
    float w = lane < PART_T / 64 ? sh[lane] : 0.0f;
#pragma unroll
    for (int off = 1; off < PART_T / 64; off <<= 1) {
      const float u = __shfl_up(w, off);
      if (lane >= off) w += u;
    }
    if (lane < PART_T / 64) sh[lane] = w;
  }
  __syncthreads();
  const float incl = v + (wv > 0 ? sh[wv - 1] : 0.0f);
  float run = incl - own;
  for (int r = r0; r < r1; ++r) {
    run += C[r];
    P[r] = run;
  }
  if (t == PART_T - 1) ps->Cs[s] = incl;
}

// Segment counts of all strips for the bound tau (lane-strided over the strips,
// summed across the wave): every lane returns the same total.
__device__ __forceinline__ int part_count(const float* sC, int strips, int budget, float R, float tau, int lane) {
  const float inv = 1.0f / (tau - R);
  int c = 0;
  for (int q = lane; q < strips; q += 64) {
    const float x = sC[q] * inv;
    c += x > (float)budget ? budget + 1 : max(1, (int)ceilf(x));
  }
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) c += __shfl_xor(c, m);
  return c;
}

constexpr int PART_CUT_T = 256;
constexpr int PART_LDS_ROWS = 8192;   // strips up to this height search an LDS copy

__global__ void __launch_bounds__(PART_CUT_T) part_cut_kernel(const float* __restrict__ pref, int strips, int ny,
                                                              int budget, const PartState* __restrict__ ps,
                                                              int4* __restrict__ seg, int* __restrict__ nseg) {
  __shared__ float sC[PART_MAX_STRIPS];
  __shared__ int sn[PART_MAX_STRIPS];   // segments per strip
  __shared__ float sp[PART_LDS_ROWS];
  __shared__ int s_all;
  __shared__ float s_Cs;
  const int t = threadIdx.x, s = blockIdx.x, lane = t & 63;
  const float* __restrict__ P = pref + (size_t)s * ny;
  const bool in_lds = ny <= PART_LDS_ROWS;
  if (in_lds)
    for (int r = t; r < ny; r += PART_CUT_T) sp[r] = P[r];
  for (int q = t; q < strips; q += PART_CUT_T) sC[q] = ps->Cs[q];
  __syncthreads();
  if (t < 64) {
    // every block repeats the same bisection (same inputs, same operations)
    float total = 0.0f, cmax = 0.0f;
    for (int q = lane; q < strips; q += 64) {
      total += sC[q];
      cmax = fmaxf(cmax, sC[q]);
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {   // butterfly: every lane ends with the same sums
      total += __shfl_xor(total, m);
      cmax = fmaxf(cmax, __shfl_xor(cmax, m));
    }
    const float R = 3.0f * total / ((float)strips * (float)ny);
    // lo: below any fit (fewer than budget segments cannot hold the total).
    // hi: a bound that fits -- total / (budget - strips) + R fits in exact
    // arithmetic (the ceilings add at most one per strip); if rounding spoils
    // it, one segment per strip (strips <= budget) always fits.
    float lo = total / (float)budget, hi = 2.0f * cmax + R + 1.0f;
    if (strips < budget) {
      const float h1 = 1.001f * total / (float)(budget - strips) + R;
      if (h1 < hi && part_count(sC, strips, budget, R, h1, lane) <= budget) hi = h1;
    }
    for (int it = 0; it < 14; ++it) {
      const float tau = 0.5f * (lo + hi);
      const bool fits = tau > R && part_count(sC, strips, budget, R, tau, lane) <= budget;
      if (fits) hi = tau;
      else lo = tau;
    }
    // every strip's count (<= budget at a bound that fits) and their sum
    const float inv = 1.0f / (hi - R);
    int all = 0;
    for (int q = lane; q < strips; q += 64) {
      const int n = max(1, (int)ceilf(sC[q] * inv));
      sn[q] = n;
      all += n;
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) all += __shfl_xor(all, m);
    if (lane == 0) {
      s_all = all;
      s_Cs = sC[s];
    }
  }
  __syncthreads();
  const int n = sn[s];
  const float Cs = s_Cs;
  if (s == 0 && t == 0) *nseg = s_all;
  for (int k = t; k < n; k += PART_CUT_T) {
    // list position: segments ordered by their index within the strip, then by
    // strip (the k-th segments of all strips cover similar rows, so each XCD's
    // contiguous share of the list is a band of rows across the strips)
    int pos = 0;
    for (int q = 0; q < strips; ++q) pos += min(sn[q], k) + (q < s && sn[q] > k ? 1 : 0);
    int st[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int kk = k + e;
      if (kk == 0) { st[e] = 0; continue; }
      if (kk == n) { st[e] = ny; continue; }
      const float target = Cs * (float)kk / (float)n;
      int x = 0, y = ny;   // first row with P > target
      while (x < y) {
        const int m = (x + y) >> 1;
        if ((in_lds ? sp[m] : P[m]) <= target) x = m + 1;
        else y = m;
      }
      st[e] = x;
    }
    seg[pos] = make_int4(0, s * STRIP, st[0], st[1] - st[0]);
  }
}

__global__ void fill_kernel(float* __restrict__ p, float v, size_t n) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) p[k] = v;
}

template <int K, class P, bool PP>
__global__ void FAM_STAGE_ATTR stage2d_batched_kernel(StageArgs A, const Inst* __restrict__ insts,
                                                                const int4* __restrict__ work, int nwork) {
  __shared__ Window W;
  __shared__ PPStage<K> PS;
  __shared__ StageCarry<carry_in_lds<K, P::NC>()> T;
  const P phys = make_phys<P>(A.phys);
  bool bad = false;
  // one item per workgroup: the XCD-aware order (limiter on: heavy items first)
  const bool one_each = (int)gridDim.x == nwork;
#pragma unroll 1
  for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
    // limiter on: items in the order of the previous launch's limiter work
    int wi;
    if constexpr (PP) wi = A.tile_perm[one_each ? heavy_first_slot(w, nwork, A.tile_perm[nwork]) : w];
    else wi = one_each ? xcd_tile(w, nwork) : w;
    const int4 it = work[wi];             // (instance, i0, j0, H)
    const Inst in = insts[it.x];
    if (in.done && *in.done) continue;
    double amx = 0.0, amy = 0.0;
    if constexpr (PP) PS.nwork = 0;
    stage_tile<K, P, PP>(phys, A, in, it.y, it.z, it.w, W, PS, T, amx, amy, bad);
    flush_wave_results(amx, amy, false, in.alpha_out, A.flag);
    if constexpr (PP) {
      if (threadIdx.x == 0) A.tile_work[wi] = PS.nwork;
    }
  }
  if (__any(bad) && threadIdx.x == 0) atomicOr(A.flag, 1);
}

template <int K, class P, bool DMR>
__global__ void FAM_OE_ATTR oe2d_kernel(OEArgs A, Inst in, int H) {
  __shared__ Window W;
  __shared__ double t1s[8];
  if (*A.done) return;
  const P phys = make_phys<P>(A.phys);
  bool bad = false;
  const int T = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int i0 = (T % gridDim.x) * STRIP, j0 = (T / gridDim.x) * H;
  if (K == 6 && A.k6_table)
    oe_tile<K, P, true, DMR>(phys, A, in, i0, j0, H, W, t1s, bad);
  else
    oe_tile<K, P, false, DMR>(phys, A, in, i0, j0, H, W, t1s, bad);
  if (__any(bad) && threadIdx.x == 0) atomicOr(A.flag, 1);
}

template <int K, class P>
__global__ void FAM_OE_ATTR oe2d_batched_kernel(OEArgs A, const Inst* __restrict__ insts,
                                                             const int4* __restrict__ work, int nwork) {
  __shared__ Window W;
  __shared__ double t1s[8];
  const P phys = make_phys<P>(A.phys);
  bool bad = false;
  const bool one_each = (int)gridDim.x == nwork;   // then the XCD-aware order
#pragma unroll 1
  for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
    const int4 it = work[one_each ? xcd_tile(w, nwork) : w];
    const Inst in = insts[it.x];
    if (in.done && *in.done) continue;
    if (K == 6 && A.k6_table)
      oe_tile<K, P, true>(phys, A, in, it.y, it.z, it.w, W, t1s, bad);
    else
      oe_tile<K, P, false>(phys, A, in, it.y, it.z, it.w, W, t1s, bad);
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
  if ((int)threadIdx.x < nc) {
    const int c = threadIdx.x;
    partial[blockIdx.x * 4 + c] = ((red[c][0] + red[c][1]) + red[c][2]) + red[c][3];
  }
}

// pass 2 (one block): mean; pass 3: D_Omega = max |u - mean|, eps from max |u|
__global__ void type1_mean_kernel(const double* __restrict__ partial, int nblocks, Inst in, int nc,
                                  double* __restrict__ stats, double* __restrict__ dmax) {
  if (threadIdx.x < 8) dmax[threadIdx.x] = 0.0;
  if ((int)threadIdx.x < nc) {
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
  if ((int)threadIdx.x < nc) {
    const int c = threadIdx.x;
    stats[in.id * 8 + c] = dmax[c];
    stats[in.id * 8 + 4 + c] = 1e-14 * fmax(dmax[4 + c], 1.0);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// the double Mach reflection boundaries are an Euler 2D option; other systems
// compile only the plain instantiation
template <class P>
static bool dmr_of(const Inst& in) {
  if constexpr (std::is_same_v<P, Euler<2>>)
    return in.dmr != 0;
  else
    return false;
}
template <int K, class P, bool DMR, bool CHAR = false>
static void launch_stage2d_d(const StageArgs& A, const Inst& in, int H, hipStream_t s) {
  dim3 grid((in.nx + STRIP - 1) / STRIP, (in.ny + H - 1) / H);
  if (A.pp) {
    const int ntiles = grid.x * grid.y;
    hipLaunchKernelGGL((stage2d_kernel<K, P, true, DMR, CHAR>), dim3(ntiles), dim3(LANES), 0, s, A, in, H);
    // up to one tile per wave slot of the chip every tile starts at once: the
    // order stays the identity set with the tile height
    if (ntiles > ORDER_MIN_TILES)
      hipLaunchKernelGGL(tile_order_kernel, dim3(1), dim3(1024), 0, s, A.tile_work, const_cast<int*>(A.tile_perm),
                         ntiles);
  } else {
    hipLaunchKernelGGL((stage2d_kernel<K, P, false, DMR, CHAR>), grid, dim3(LANES), 0, s, A, in, H);
  }
}
template <int K, class P>
static void launch_stage2d_t(const StageArgs& A, const Inst& in, int H, hipStream_t s) {
  if constexpr (std::is_same_v<P, Euler<2>>) {
    // characteristic variables: FAM5 only (the variant the paper times)
    if constexpr (K == 5) {
      if (in.charv) {
        if (dmr_of<P>(in)) return launch_stage2d_d<K, P, true, true>(A, in, H, s);
        return launch_stage2d_d<K, P, false, true>(A, in, H, s);
      }
    }
    if (dmr_of<P>(in)) return launch_stage2d_d<K, P, true>(A, in, H, s);
  }
  launch_stage2d_d<K, P, false>(A, in, H, s);
}
template <int K, class P>
static void launch_oe2d_t(const OEArgs& A, const Inst& in, int H, hipStream_t s) {
  dim3 grid((in.nx + STRIP - 1) / STRIP, (in.ny + H - 1) / H);
  if constexpr (std::is_same_v<P, Euler<2>>) {
    if (dmr_of<P>(in)) {
      hipLaunchKernelGGL((oe2d_kernel<K, P, true>), grid, dim3(LANES), 0, s, A, in, H);
      return;
    }
  }
  hipLaunchKernelGGL((oe2d_kernel<K, P, false>), grid, dim3(LANES), 0, s, A, in, H);
}
template <int K, class P>
static void launch_stage2d_b(const StageArgs& A, const Inst* insts, const int4* work, int nwork, int nblocks,
                             hipStream_t s) {
  if (A.pp) {
    hipLaunchKernelGGL((stage2d_batched_kernel<K, P, true>), dim3(nblocks), dim3(LANES), 0, s, A, insts, work,
                       nwork);
    hipLaunchKernelGGL(tile_order_kernel, dim3(1), dim3(1024), 0, s, A.tile_work, const_cast<int*>(A.tile_perm),
                       nwork);
  } else
    hipLaunchKernelGGL((stage2d_batched_kernel<K, P, false>), dim3(nblocks), dim3(LANES), 0, s, A, insts, work,
                       nwork);
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
template <int K, class P>
static void launch_stage2d_list_t(const StageArgs& A, const Inst& in, const int4* seg, const int* nseg, int budget,
                                  hipStream_t s) {
  if constexpr (std::is_same_v<P, Euler<2>> && K == 5) {
    if (in.charv) {
      if (dmr_of<P>(in))
        hipLaunchKernelGGL((stage2d_list_kernel<K, P, true, true>), dim3(budget), dim3(LANES), 0, s, A, in, seg,
                           nseg);
      else
        hipLaunchKernelGGL((stage2d_list_kernel<K, P, false, true>), dim3(budget), dim3(LANES), 0, s, A, in, seg,
                           nseg);
      return;
    }
  }
  if constexpr (std::is_same_v<P, Euler<2>>) {
    if (dmr_of<P>(in)) {
      hipLaunchKernelGGL((stage2d_list_kernel<K, P, true>), dim3(budget), dim3(LANES), 0, s, A, in, seg, nseg);
      return;
    }
  }
  hipLaunchKernelGGL((stage2d_list_kernel<K, P, false>), dim3(budget), dim3(LANES), 0, s, A, in, seg, nseg);
}
void launch_stage2d_list(int k, int sys, const StageArgs& A, const Inst& in, const int4* seg, const int* nseg,
                         int budget, hipStream_t s) {
  // the limiter is a 2D Euler option
  (void)sys;
  switch (k) {
    case 3: launch_stage2d_list_t<3, Euler<2>>(A, in, seg, nseg, budget, s); break;
    case 4: launch_stage2d_list_t<4, Euler<2>>(A, in, seg, nseg, budget, s); break;
    case 5: launch_stage2d_list_t<5, Euler<2>>(A, in, seg, nseg, budget, s); break;
    default: launch_stage2d_list_t<6, Euler<2>>(A, in, seg, nseg, budget, s); break;
  }
}
size_t partition_state_bytes() { return sizeof(PartState); }
void launch_partition(const float* row_cost, float* pref, void* state, int strips, int ny, int budget, int4* seg,
                      int* nseg, hipStream_t s) {
  PartState* ps = static_cast<PartState*>(state);
  hipLaunchKernelGGL(part_scan_kernel, dim3(strips), dim3(PART_T), 0, s, row_cost, pref, ny, ps);
  hipLaunchKernelGGL(part_cut_kernel, dim3(strips), dim3(PART_CUT_T), 0, s, pref, strips, ny, budget, ps, seg, nseg);
}
void launch_fill(float* p, float v, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)std::min<size_t>(1024, (n + 255) / 256)), dim3(256), 0, s, p, v, n);
}
void launch_tile_identity(int* tile_perm, int* tile_work, int ntiles, hipStream_t s) {
  hipLaunchKernelGGL(tile_identity_kernel, dim3(std::min(1024, (ntiles + 255) / 256)), dim3(256), 0, s, tile_perm,
                     tile_work, ntiles);
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
