// fam_strip.h - the marching-strip machinery shared by the stage, OE and
// adjoint kernels: a 64-lane wave owns a strip of columns and marches up a tile
// of rows, keeping three state rows in an LDS ring.
#pragma once

#include "fam_device.h"
#include "fam_kernels.h"

namespace fam {

constexpr int LANES = 64;
constexpr int NPL = 12;            // planes held in LDS for up to 4 components x 3 moments

// ---------------------------------------------------------------------------
// LDS row window: lane l holds LDS column l = grid column i0 - 2 + l.  Lanes 0
// and 63 only load; lanes 1 and 62 are ring columns; lanes 2..61 write output.
// ---------------------------------------------------------------------------
struct Window {
  double v[3][NPL][LANES];
};

// three row slots used as a ring: row r+2 is fetched into the slot of row r-1
// once every read of row r-1 in the current iteration is done
__device__ __forceinline__ int slot_of(int r) { return ((r % 3) + 3) % 3; }

// the double Mach reflection ghost cells of row r, column ci (at least one
// outside the mesh) at boundary time tb; see fam_config.dmr
template <int NPLU>
__device__ __forceinline__ void dmr_ghost(const double* __restrict__ U, const Inst& in, int r, int ci, double tb,
                                          double (&reg)[NPLU], long long moff) {
  const double xc = in.x0 + (ci + 0.5) * in.dx;
  int which = -1;   // 0: post-shock state, 1: pre-shock state, -1: copy or mirror
  if (r >= in.ny)   // top: the exact shock line at the upper boundary
    which = xc < 1.0 / 6.0 + (in.ytop + 20.0 * tb) * 0.57735026918962576451 ? 0 : 1;
  else if (r < 0 ? xc < 1.0 / 6.0 : ci < 0)   // bottom inflow part, left inflow
    which = 0;
  if (which >= 0) {
    // (rho, u, v, p) = (8, 8.25 cos 30deg, -8.25 sin 30deg, 116.5) behind the shock,
    // (1.4, 0, 0, 1) ahead; conservative, with 1/(gamma - 1) = in.dmr_einv
    constexpr double rl = 8.0, ul = 8.25 * 0.86602540378443864676, vl = -8.25 * 0.5, pl = 116.5;
    const double post[4] = {rl, rl * ul, rl * vl, pl * in.dmr_einv + 0.5 * rl * (ul * ul + vl * vl)};
    const double pre[4] = {1.4, 0.0, 0.0, in.dmr_einv};
#pragma unroll
    for (int p = 0; p < NPLU; ++p) reg[p] = p % 3 == 0 ? (which == 0 ? post[p / 3] : pre[p / 3]) : 0.0;
    return;
  }
  // right outflow (copy of the last column) and, below the mesh, the reflecting
  // wall: mirror image of row -1 - r with rho v and the y-moments of the other
  // components negated
  const int gi = ci >= in.nx ? in.nx - 1 : ci;
  const int gj = r < 0 ? -1 - r : r;
  const size_t base = (size_t)gj * in.nx + gi;
#pragma unroll
  for (int p = 0; p < NPLU; ++p) {
    const double v = U[p * in.plane + base + (p % 3 == 0 ? 0 : moff)];
    const bool neg = r < 0 && ((p / 3 == 2) ? (p % 3 != 2) : (p % 3 == 2));
    reg[p] = neg ? -v : v;
  }
}

// b - a in doubles for two arrays of doubles that may be separate allocations
// (integer addresses: a pointer difference is defined only within one array;
// both are 8-byte aligned, so the byte difference shifts exactly)
__device__ __forceinline__ long long elem_offset(const double* a, const double* b) {
  return ((long long)(uintptr_t)b - (long long)(uintptr_t)a) >> 3;
}

// Row r of the state U; its moment planes (m = 1, 2) lie moff elements after
// the places U's own would have (0: a plain state).  DMR: the instance uses the
// double Mach reflection boundaries (a separate instantiation, so the plain
// kernels carry none of its registers)
template <int NPLU, bool DMR>
__device__ __forceinline__ void fetch_row(const double* __restrict__ U, const Inst& in, int i0, int r,
                                          int lane, double (&reg)[NPLU], double tb, long long moff = 0) {
  const int ci = i0 - 2 + lane;
  if constexpr (DMR) {
    if (r < 0 || r >= in.ny || ci < 0 || ci >= in.nx) {
      dmr_ghost<NPLU>(U, in, r, ci, tb, reg, moff);
      return;
    }
  }
  const int gj = ghost(r, in.ny, in.bcy);
  const int gi = ghost(ci, in.nx, in.bcx);
  const size_t base = (size_t)gj * in.nx + gi;
#pragma unroll
  for (int p = 0; p < NPLU; ++p) reg[p] = U[p * in.plane + base + (p % 3 == 0 ? 0 : moff)];
}

template <int NPLU>
__device__ __forceinline__ void store_row(Window& W, int slot, int lane, const double (&reg)[NPLU]) {
#pragma unroll
  for (int p = 0; p < NPLU; ++p) W.v[slot][p][lane] = reg[p];
}

// stencil of component c around LDS column col (clamped for the load-only lanes)
template <int K>
__device__ __forceinline__ void gather(const Window& W, int c, int col, int sl, int sm, int sh,
                                       double (&u0)[9], double (&u1)[9], double (&u2)[9]) {
  const int sr[3] = {sl, sm, sh};
  const int cm = col > 0 ? col - 1 : 0, cp = col < LANES - 1 ? col + 1 : LANES - 1;
  const int cc[3] = {cm, col, cp};
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int l = b * 3 + a;
      u0[l] = W.v[sr[b]][c * 3 + 0][cc[a]];
      const bool x_used = (K >= 5) ? (l != 1 && l != 7) : (l == 4);
      const bool y_used = (K >= 5) ? (l != 3 && l != 5) : (l == 4);
      u1[l] = x_used ? W.v[sr[b]][c * 3 + 1][cc[a]] : 0.0;
      u2[l] = y_used ? W.v[sr[b]][c * 3 + 2][cc[a]] : 0.0;
    }
}

// neighbour-lane values by DPP whole-wave shifts (GFX9 wave_shr:1 / wave_shl:1):
// from_left(x) in lane l is x of lane l - 1, from_right(x) is x of lane l + 1;
// lane 0 (resp. 63) keeps its own value
__device__ __forceinline__ double from_left(double x) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(x), __double2loint(x), 0x138, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(x), __double2hiint(x), 0x138, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double from_right(double x) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(x), __double2loint(x), 0x130, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(x), __double2hiint(x), 0x130, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

}  // namespace fam
