// fam_kernels.h - argument blocks and launchers shared by the host library and
// the HIP kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include <algorithm>

namespace fam {

constexpr int STRIP = 60;   // output columns per 2D strip (one wavefront)
// waves of the RK stage kernel per SIMD that its register and LDS budget allows
#ifndef FAM_STAGE_WAVES
#define FAM_STAGE_WAVES 1
#endif

struct PhysParams {
  double gamma, ax, ay;
};

// one mesh instance (a batched context holds many)
struct Inst {
  int id;
  int nx, ny;
  size_t plane;            // nx * ny
  size_t offset;           // start of the instance in a batched state (doubles)
  double dx, dy;
  int bcx, bcy;            // 0 periodic, 1 transmissive
  const double* alpha_in;  // [2] wave speeds of the stage input state
  double* alpha_out;       // [2] max-accumulators for the stage output state
  const double* dt;        // time step of the current step
  const int* done;         // instance finished (fam_run), may be null
  // double Mach reflection boundaries (dmr != 0): the boundary time of a launch is
  // *t_end - t_ofs * dt (t_end: the step's end time; t_ofs 1, 0, 1/2 for the RK
  // stages, 0 for OE); x0, ytop: domain; dmr_einv = 1 / (gamma - 1)
  int dmr;
  const double* t_end;
  double t_ofs;
  double x0, ytop, dmr_einv;
  // stage reconstruction in local characteristic variables (Euler, k = 5)
  int charv;
};

struct StageArgs {
  PhysParams phys;
  const double* Us;
  const double* U0;
  double* Uout;
  // moment planes (m = 1, 2) of the output; NULL: those of Uout.  With Uout the
  // state and Uout_mom a stage buffer, the last stage of a step writes its
  // averages in place (each output cell reads only its own U0 value) and leaves
  // its moments for the OE, which then writes only moment planes
  double* Uout_mom;
  // Shu-Osher stage ca U0 + (1 - ca) L with L = Us + dt R(Us), evaluated as
  // L + ca (U0 - L): the rounded 1/3 and 2/3 of the last stage sum to 1 - 2^-54,
  // which as separate weights would shrink every value by that much each step
  double ca;
  int* flag;
  const int* done;
  int pp;                  // positivity limiter on the stage reconstruction (2D Euler)
  // single-instance limiter launches: tiles run in the order tile_perm (cells
  // that needed the exact test in the previous launch first); each tile writes
  // its count of such cells to tile_work
  const int* tile_perm;
  int* tile_work;
  // single-instance limiter launches over a segment list: cycles spent on each
  // row of each strip, row_cost[strip * ny + row] (NULL: not recorded)
  float* row_cost;
};

struct OEArgs {
  PhysParams phys;
  const double* Un;
  // average planes (m = 0) of the input; NULL: those of Un.  When they are
  // Uout's own (avg_in_place = 1) the OE leaves them unwritten: it changes no
  // average, so it then moves 8 planes per cell to HBM instead of 12
  const double* Ua;
  int avg_in_place;
  double* Uout;
  double gamma_k;
  int type;                // 1 or 2
  int k6_table;
  const double* stats;     // Type I: [inst*8 + c] D_Omega, [inst*8 + 4 + c] eps_Omega
  int* flag;
  const int* done;
  double* delta_out;       // single instance, test export: delta per cell (NULL: not written)
};

// per-instance step bookkeeping (device)
struct StepState {
  double alpha[2][3][2];   // [parity][stage input 0..2][x/y]
  double dt;               // time step of the current step
  double t;                // time reached: the context clock (0 at set-up, advanced by every step)
  double t_final;          // <= 0: none
  double dt_fixed;         // > 0: use instead of the CFL rule
  double cfl;
  double hx, hy;           // lengths of the time-step rule: dx, dy or dx^{k/3}, dy^{k/3}
  int dim;
  int done;
  int steps;
  int pad_;
};

void launch_stage2d(int k, int sys, const StageArgs& A, const Inst& in, int H, hipStream_t s);
// tile_perm := tiles with tile_work > 0 first, then the others (both in index order)
void launch_tile_order(const int* tile_work, int* tile_perm, int ntiles, hipStream_t s);
void launch_tile_identity(int* tile_perm, int* tile_work, int ntiles, hipStream_t s);
// limiter-on stage launch over a list of strip segments (x unused, y = first
// column, z = first row, w = rows; w <= 0: empty), one wave per entry; then the
// list for the next launch: each strip cut into segments of equal recorded cost,
// at most `budget` segments in all
void launch_stage2d_list(int k, int sys, const StageArgs& A, const Inst& in, const int4* seg, const int* nseg,
                         int budget, hipStream_t s);
// state: partition_state_bytes() of device memory
size_t partition_state_bytes();
void launch_partition(const float* row_cost, float* pref, void* state, int strips, int ny, int budget, int4* seg,
                      int* nseg, hipStream_t s);
void launch_fill(float* p, float v, size_t n, hipStream_t s);
constexpr int PART_MAX_STRIPS = 1024;
// point values of the stage reconstruction at every cell's flux points (test export)
void launch_dbg_recon(int dim, int k, int nc, const double* U, const Inst& in, double* vals, hipStream_t s);
void launch_oe2d(int k, int sys, const OEArgs& A, const Inst& in, int H, hipStream_t s);
void launch_stage2d_batched(int k, int sys, const StageArgs& A, const Inst* insts, const int4* work, int nwork,
                            int nblocks, hipStream_t s);
void launch_oe2d_batched(int k, int sys, const OEArgs& A, const Inst* insts, const int4* work, int nwork,
                         int nblocks, hipStream_t s);
void launch_alpha2d(int sys, const PhysParams& pp, const double* U, const Inst* insts, int ninst,
                    size_t max_cells, int* flag, hipStream_t s);
// Type I reference quantities of one instance (nmom = moments per component)
void launch_type1_stats(const double* U, const Inst& in, int nc, int nmom, double* partial, int nblocks,
                        double* dmax, double* stats, hipStream_t s);

// 1D
void launch_stage1d(int k, int sys, const StageArgs& A, const Inst& in, hipStream_t s);
void launch_oe1d(int k, int sys, const OEArgs& A, const Inst& in, hipStream_t s);
void launch_alpha1d(int sys, const PhysParams& pp, const double* U, const Inst& in, int* flag, hipStream_t s);

// step bookkeeping: dt, clipping, termination, zeroing of the accumulators
void launch_step_begin(StepState* st, int ninst, int parity, double dt_fixed, double t_final, hipStream_t s);
void launch_zero_alpha(StepState* st, int ninst, int parity, hipStream_t s);
// per run: wave-speed slots, dt, step count and termination back to zero; the
// time (the context clock) is kept
void launch_reset_steps(StepState* st, int ninst, double t_final, double dt_fixed, hipStream_t s);
void launch_set_time(StepState* st, int ninst, double t, hipStream_t s);

}  // namespace fam
