// fam_ctx.h - the library's context object and internal enqueue helpers
// (shared by the host API and the adjoint driver; not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <vector>

#include "../../include/fam.h"
#include "fam_kernels.h"

struct FamAdjointScratch;

struct fam_ctx {
  std::vector<fam_config> cfg;
  int ninst = 0;
  int dim = 2, k = 5, sys = 2, nc = 4, nmom = 3, oe = 2, bcx = 0, bcy = 0, k6t = 0, pp = 0;
  double gamma_k = 15.0;
  fam::PhysParams phys{1.4, 1.0, 0.0};
  hipStream_t stream = nullptr;
  std::vector<size_t> offsets;
  size_t len = 0, max_cells = 0;
  double* W1 = nullptr;
  double* W2 = nullptr;
  fam::StepState* st = nullptr;
  int* flag = nullptr;
  double* stats = nullptr;     // Type I: [inst*8 + ...]
  double* partial = nullptr;   // Type I partial sums
  double* dmax = nullptr;
  int t1_blocks = 256;
  int H = 32;                  // rows per strip tile of the stage kernel (single instance)
  int H_oe = 32;               // rows per strip tile of the OE kernel (single instance)
  // limiter on: order of the stage kernel's tiles (single instance) or work-list
  // items (batch), and the limiter work per tile / item of its last launch
  int* tile_perm = nullptr;
  int* tile_work = nullptr;
  int tile_cap = 0;
  // single instance, limiter on: the stage kernel can run over a list of strip
  // segments cut by the recorded cost of every row (one round of waves)
  bool stage_list = false;
  int seg_budget = 0;          // wave slots of the chip for the stage kernel
  int4* seg = nullptr;         // [seg_budget]
  int* nseg = nullptr;
  float* row_cost = nullptr;   // [strips * ny]
  float* row_pref = nullptr;   // [strips * ny] partition scratch
  void* part_state = nullptr;  // partition counters and per-strip counts
  // batched
  fam::Inst* d_insts[2][4] = {};    // [parity][stage 0..2, 3 = OE]
  fam::Inst* d_ainst[2] = {};       // [parity]: alpha_out = stage-0 input slot
  int4* d_work = nullptr;
  int nwork = 0;
  size_t work_cap = 0;         // allocated work-list entries
  int batch_H = 16;            // tile height of the batched work list
  int pblocks = 0;             // persistent grid size
  std::vector<int> inst_H;
  // graphs (keyed by U pointer, dt_fixed, t_final)
  struct GKey {
    double* U;
    double dt_fixed, t_final;
    bool operator<(const GKey& o) const {
      if (U != o.U) return U < o.U;
      if (dt_fixed != o.dt_fixed) return dt_fixed < o.dt_fixed;
      return t_final < o.t_final;
    }
  };
  std::map<GKey, hipGraphExec_t> graphs;
  bool use_graph = true;
  // adjoint scratch (allocated by the first fam_adjoint call)
  FamAdjointScratch* adj = nullptr;
};


fam_status validate_config(const fam_config& c);
double default_gamma_k(int dim, int k);
int choose_H(int nx, int ny);   // default strip-tile height of a 2D mesh
fam_status set_stage_H(fam_ctx* c, int H);
fam::Inst inst_for(const fam_ctx* c, int i, int parity, int stage);
fam_status reset_steps(fam_ctx* c, double t_final, double dt_fixed);
fam_status save_clock(fam_ctx* c, std::vector<double>* t);
fam_status restore_clock(fam_ctx* c, const std::vector<double>& t);
void enqueue_alpha_full(fam_ctx* c, const double* U, int parity);
// Uout_mom: moment planes of the output (NULL: Uout's own)
void enqueue_stage(fam_ctx* c, int s, int parity, const double* U0, const double* Us, double* Uout,
                   const double* dt_override, bool repartition = true, double* Uout_mom = nullptr);
// Ua: average planes of the input (NULL: Un's own); when Ua == Uout they are left unwritten
void enqueue_oe(fam_ctx* c, int parity, const double* Un, double* Uout, const double* dt_override,
                double* delta_out = nullptr, const double* Ua = nullptr);
void enqueue_step(fam_ctx* c, double* U, int parity, double dt_fixed, double t_final);
