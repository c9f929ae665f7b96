// fam_api.hip - host side of the FAM library: the C ABI of include/fam.h.
//
// A context owns two stage buffers W1, W2 (the SSP-RK3 stage states), one
// StepState per instance (wave-speed maxima per stage, time step, time, step
// count, termination), a non-physical flag, Type I statistics scratch and, for
// batched contexts, device tables of instances and of the work list
// (instance, strip origin, row origin, rows) that the persistent kernels walk.
//
// Step sequence (one stream, no host synchronisation):
//   [alpha reduction of U]  step_begin  stage0: U -> W1  stage1: (W1, U) -> W2
//   stage2: (W2, U) -> W1 (or -> U when OE is off)  [Type I stats]  OE: W1 -> U
// The wave speeds of each stage's output are reduced inside the stage kernel;
// the last stage's are those of the next step's state (OE keeps averages), so
// consecutive steps need no separate reduction pass.  Two consecutive steps
// (stage-slot parity 0 and 1) are captured once into a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "../../include/fam.h"
#include "fam_ctx.h"
#include "fam_kernels.h"

using fam::Inst;
using fam::StepState;

extern "C" const char* fam_status_str(fam_status s) {
  switch (s) {
    case FAM_OK: return "ok";
    case FAM_ERR_ARG: return "invalid argument";
    case FAM_ERR_DEVICE: return "HIP error";
    case FAM_ERR_NOMEM: return "out of device memory";
    case FAM_ERR_NONPHYSICAL: return "non-physical state (rho <= 0 or p <= 0 in a cell average)";
    case FAM_ERR_STATE: return "call not valid for this context";
    case FAM_ERR_SIZE: return "problem larger than the static scratch of fam_step_static";
  }
  return "unknown status";
}

#define HIP_TRY(expr)                       \
  do {                                      \
    if ((expr) != hipSuccess) return FAM_ERR_DEVICE; \
  } while (0)

fam_status validate_config(const fam_config& c) {
  if (c.dim != 1 && c.dim != 2) return FAM_ERR_ARG;
  if (c.nx < 3 || (c.dim == 2 && c.ny < 3)) return FAM_ERR_ARG;
  if (c.k < 3 || c.k > 6) return FAM_ERR_ARG;
  if (c.system < 0 || c.system > 2) return FAM_ERR_ARG;
  if (!(c.x1 > c.x0) || (c.dim == 2 && !(c.y1 > c.y0))) return FAM_ERR_ARG;
  if (c.bc_x < 0 || c.bc_x > 1 || c.bc_y < 0 || c.bc_y > 1) return FAM_ERR_ARG;
  if (c.oe < 0 || c.oe > 2) return FAM_ERR_ARG;
  if (!(c.cfl > 0.0)) return FAM_ERR_ARG;
  if (c.system == FAM_EULER && !(c.gamma > 1.0)) return FAM_ERR_ARG;
  if ((size_t)c.nx * (size_t)(c.dim == 2 ? c.ny : 1) > ((size_t)1 << 31)) return FAM_ERR_ARG;
  if (c.pp && !(c.system == FAM_EULER && c.dim == 2)) return FAM_ERR_ARG;
  if (c.dt_rule != 0 && c.dt_rule != 1) return FAM_ERR_ARG;
  if (c.dmr && !(c.system == FAM_EULER && c.dim == 2)) return FAM_ERR_ARG;
  if (c.char_vars && !(c.system == FAM_EULER && c.k == 5)) return FAM_ERR_ARG;
  return FAM_OK;
}

double default_gamma_k(int dim, int k) {
  if (dim == 1) return k <= 4 ? 25.0 : 12.5;
  return k <= 4 ? 25.0 : 15.0;
}

static Inst make_inst(const fam_ctx* c, int i) {
  const fam_config& f = c->cfg[i];
  Inst in{};
  in.id = i;
  in.nx = f.nx;
  in.ny = c->dim == 2 ? f.ny : 1;
  in.plane = (size_t)in.nx * in.ny;
  in.offset = c->offsets[i];
  in.dx = (f.x1 - f.x0) / f.nx;
  in.dy = c->dim == 2 ? (f.y1 - f.y0) / f.ny : 1.0;
  in.bcx = f.bc_x;
  in.bcy = f.bc_y;
  if (f.dmr) {
    in.dmr = 1;
    in.bcx = in.bcy = FAM_BC_TRANSMISSIVE;
    in.x0 = f.x0;
    in.ytop = f.y1;
    in.dmr_einv = 1.0 / (f.gamma - 1.0);
  }
  in.charv = f.char_vars != 0;
  return in;
}

Inst inst_for(const fam_ctx* c, int i, int parity, int stage) {
  Inst in = make_inst(c, i);
  StepState* s = c->st + i;
  if (stage < 3) {
    in.alpha_in = &s->alpha[parity][stage][0];
    in.alpha_out = stage < 2 ? &s->alpha[parity][stage + 1][0] : &s->alpha[1 - parity][0][0];
  } else {
    in.alpha_in = &s->alpha[parity][0][0];
    in.alpha_out = nullptr;
  }
  in.dt = &s->dt;
  in.done = &s->done;
  in.t_end = &s->t;
  in.t_ofs = stage == 0 ? 1.0 : stage == 2 ? 0.5 : 0.0;   // stage times t_n, t_n + dt, t_n + dt/2; OE t_n + dt
  return in;
}

// rows per strip tile: enough tiles to fill 256 CUs several times over
int choose_H(int nx, int ny) {
  const int strips = (nx + fam::STRIP - 1) / fam::STRIP;
  int H = 32;
  while (H > 8 && (size_t)strips * ((ny + H - 1) / H) < 8 * 256) H /= 2;
  return std::min(H, std::max(ny, 1));
}

static fam_status init_segments(fam_ctx* c);

static fam_status alloc_common(fam_ctx* c) {
  const size_t bytes = c->len * sizeof(double);
  if (hipMalloc(&c->W1, bytes) != hipSuccess) return FAM_ERR_NOMEM;
  if (hipMalloc(&c->W2, bytes) != hipSuccess) return FAM_ERR_NOMEM;
  if (hipMalloc(&c->st, sizeof(StepState) * c->ninst) != hipSuccess) return FAM_ERR_NOMEM;
  if (hipMalloc(&c->flag, sizeof(int) * 4) != hipSuccess) return FAM_ERR_NOMEM;
  if (hipMalloc(&c->stats, sizeof(double) * 8 * c->ninst) != hipSuccess) return FAM_ERR_NOMEM;
  if (hipMalloc(&c->partial, sizeof(double) * 4 * c->t1_blocks) != hipSuccess) return FAM_ERR_NOMEM;
  if (hipMalloc(&c->dmax, sizeof(double) * 8) != hipSuccess) return FAM_ERR_NOMEM;
  std::vector<int> zero(4, 0);
  HIP_TRY(hipMemcpy(c->flag, zero.data(), sizeof(int) * 4, hipMemcpyHostToDevice));
  return FAM_OK;
}

// one-time: the static fields of every instance's StepState (synchronous)
static fam_status init_steps(fam_ctx* c) {
  std::vector<StepState> h(c->ninst);
  for (int i = 0; i < c->ninst; ++i) {
    StepState& s = h[i];
    std::memset(&s, 0, sizeof(s));
    const fam_config& f = c->cfg[i];
    s.cfl = f.cfl;
    const double e = f.dt_rule == 1 ? f.k / 3.0 : 1.0;
    s.hx = std::pow((f.x1 - f.x0) / f.nx, e);
    s.hy = c->dim == 2 ? std::pow((f.y1 - f.y0) / f.ny, e) : 1.0;
    s.dim = c->dim;
  }
  HIP_TRY(hipMemcpy(c->st, h.data(), sizeof(StepState) * c->ninst, hipMemcpyHostToDevice));
  return FAM_OK;
}

// per run: step count, termination and wave-speed slots back to zero; the
// time of every instance (the context clock) is kept
fam_status reset_steps(fam_ctx* c, double t_final, double dt_fixed) {
  fam::launch_reset_steps(c->st, c->ninst, t_final, dt_fixed, c->stream);
  return FAM_OK;
}

// The clock of a synchronous call that steps internally (autotuner, adjoint)
// is put back to what it was on entry.
fam_status save_clock(fam_ctx* c, std::vector<double>* t) {
  std::vector<StepState> h(c->ninst);
  HIP_TRY(hipMemcpyAsync(h.data(), c->st, sizeof(StepState) * c->ninst, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  t->resize(c->ninst);
  for (int i = 0; i < c->ninst; ++i) (*t)[i] = h[i].t;
  return FAM_OK;
}

fam_status restore_clock(fam_ctx* c, const std::vector<double>& t) {
  for (int i = 0; i < c->ninst; ++i) fam::launch_set_time(c->st + i, 1, t[i], c->stream);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(c->stream));
  return FAM_OK;
}

static fam_status build_inst_tables(fam_ctx* c) {
  for (int p = 0; p < 2; ++p) {
    for (int s = 0; s < 4; ++s) {
      std::vector<Inst> h(c->ninst);
      for (int i = 0; i < c->ninst; ++i) h[i] = inst_for(c, i, p, s);
      if (hipMalloc(&c->d_insts[p][s], sizeof(Inst) * c->ninst) != hipSuccess) return FAM_ERR_NOMEM;
      HIP_TRY(hipMemcpy(c->d_insts[p][s], h.data(), sizeof(Inst) * c->ninst, hipMemcpyHostToDevice));
    }
    std::vector<Inst> h(c->ninst);
    for (int i = 0; i < c->ninst; ++i) {
      h[i] = inst_for(c, i, p, 0);
      h[i].alpha_out = const_cast<double*>(h[i].alpha_in);
    }
    if (hipMalloc(&c->d_ainst[p], sizeof(Inst) * c->ninst) != hipSuccess) return FAM_ERR_NOMEM;
    HIP_TRY(hipMemcpy(c->d_ainst[p], h.data(), sizeof(Inst) * c->ninst, hipMemcpyHostToDevice));
  }
  return FAM_OK;
}

static void destroy_graphs(fam_ctx* c) {
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
}

void fam_adjoint_free(fam_ctx* c);

extern "C" void fam_destroy(fam_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  destroy_graphs(c);
  fam_adjoint_free(c);
  void* bufs[] = {c->W1,        c->W2,        c->st,       c->flag, c->stats,    c->partial,  c->dmax,
                  c->d_work,    c->tile_perm, c->tile_work, c->seg,  c->nseg,     c->row_cost, c->row_pref,
                  c->part_state};
  for (void* p : bufs)
    if (p) (void)hipFree(p);
  for (auto& a : c->d_insts)
    for (auto* p : a)
      if (p) (void)hipFree(p);
  for (auto* p : c->d_ainst)
    if (p) (void)hipFree(p);
  delete c;
}

static void set_common(fam_ctx* c, const fam_config& f) {
  c->dim = f.dim;
  c->k = f.k;
  c->sys = f.system;
  c->nc = f.system == FAM_EULER ? f.dim + 2 : 1;
  c->nmom = f.dim == 1 ? 2 : 3;
  c->oe = f.oe;
  c->bcx = f.bc_x;
  c->bcy = f.bc_y;
  c->k6t = f.k6_jump_from_table;
  c->pp = f.pp;
  c->gamma_k = f.oe_gamma_k > 0 ? f.oe_gamma_k : default_gamma_k(f.dim, f.k);
  c->phys = fam::PhysParams{f.gamma, f.ax, f.ay};
}

extern "C" fam_status fam_init(const fam_config* cfg, void* hip_stream, fam_ctx** out) {
  if (!cfg || !out) return FAM_ERR_ARG;
  *out = nullptr;
  fam_status v = validate_config(*cfg);
  if (v != FAM_OK) return v;
  fam_ctx* c = new (std::nothrow) fam_ctx();
  if (!c) return FAM_ERR_NOMEM;
  fam_config f = *cfg;
  if (f.dim == 1) { f.ny = 1; f.y0 = 0.0; f.y1 = 1.0; }
  c->cfg = {f};
  c->ninst = 1;
  set_common(c, f);
  c->stream = (hipStream_t)hip_stream;
  c->use_graph = c->stream != nullptr;
  c->offsets = {0};
  c->max_cells = (size_t)f.nx * (f.dim == 2 ? f.ny : 1);
  c->len = c->max_cells * c->nc * c->nmom;
  c->H = f.dim == 2 ? choose_H(f.nx, f.ny) : 1;
  c->H_oe = c->H;
  fam_status a = alloc_common(c);
  if (a == FAM_OK && f.dim == 2 && c->pp) {
    // tile heights are >= 8 rows (or the whole mesh when ny < 8)
    const int strips = (f.nx + fam::STRIP - 1) / fam::STRIP;
    c->tile_cap = strips * ((f.ny + 7) / 8);
    if (hipMalloc(&c->tile_perm, sizeof(int) * (c->tile_cap + 1)) != hipSuccess ||
        hipMalloc(&c->tile_work, sizeof(int) * c->tile_cap) != hipSuccess)
      a = FAM_ERR_NOMEM;
    if (a == FAM_OK) a = set_stage_H(c, c->H);
    if (a == FAM_OK) a = init_segments(c);
    if (a == FAM_OK && hipStreamSynchronize(c->stream) != hipSuccess) a = FAM_ERR_DEVICE;
  }
  if (a == FAM_OK) a = init_steps(c);
  if (a == FAM_OK) a = build_inst_tables(c);
  if (a != FAM_OK) {
    fam_destroy(c);
    return a;
  }
  *out = c;
  return FAM_OK;
}

// work list of a batch: (instance, i0, j0, H) strip tiles of height min(H, ny),
// largest instances first (the persistent kernels take them round-robin)
static fam_status build_work_list(fam_ctx* c, int Hmax) {
  const int n = c->ninst;
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return (size_t)c->cfg[x].nx * c->cfg[x].ny > (size_t)c->cfg[y].nx * c->cfg[y].ny;
  });
  std::vector<int4> work;
  c->inst_H.assign(n, Hmax);
  for (int i : order) {
    const fam_config& f = c->cfg[i];
    const int H = std::min(Hmax, f.ny);
    c->inst_H[i] = H;
    for (int j0 = 0; j0 < f.ny; j0 += H)
      for (int i0 = 0; i0 < f.nx; i0 += fam::STRIP) work.push_back(make_int4(i, i0, j0, H));
  }
  if (work.size() > c->work_cap) {
    for (void** p : {(void**)&c->d_work, (void**)&c->tile_perm, (void**)&c->tile_work}) {
      if (*p) (void)hipFree(*p);
      *p = nullptr;
    }
    c->work_cap = 0;
    if (hipMalloc(&c->d_work, sizeof(int4) * work.size()) != hipSuccess) return FAM_ERR_NOMEM;
    if (c->pp && (hipMalloc(&c->tile_perm, sizeof(int) * (work.size() + 1)) != hipSuccess ||
                  hipMalloc(&c->tile_work, sizeof(int) * work.size()) != hipSuccess))
      return FAM_ERR_NOMEM;
    c->work_cap = work.size();
  }
  HIP_TRY(hipMemcpy(c->d_work, work.data(), sizeof(int4) * work.size(), hipMemcpyHostToDevice));
  c->nwork = (int)work.size();
  if (c->pp) {
    // the limiter's work order restarts from the list order
    fam::launch_tile_identity(c->tile_perm, c->tile_work, c->nwork, c->stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  c->batch_H = Hmax;
  return FAM_OK;
}

extern "C" fam_status fam_init_batched(const fam_config* per, int n, void* hip_stream, fam_ctx** out) {
  if (!per || !out || n < 1) return FAM_ERR_ARG;
  *out = nullptr;
  for (int i = 0; i < n; ++i) {
    fam_status v = validate_config(per[i]);
    if (v != FAM_OK) return v;
    const fam_config &a = per[0], &b = per[i];
    if (b.dim != 2 || b.k != a.k || b.system != a.system || b.gamma != a.gamma || b.oe != a.oe ||
        b.bc_x != a.bc_x || b.bc_y != a.bc_y || b.cfl != a.cfl || b.oe_gamma_k != a.oe_gamma_k ||
        b.k6_jump_from_table != a.k6_jump_from_table || b.ax != a.ax || b.ay != a.ay || b.pp != a.pp)
      return FAM_ERR_ARG;
  }
  if (per[0].oe == FAM_OE_TYPE1) return FAM_ERR_ARG;   // global statistics per instance: single contexts only
  if (per[0].dmr || per[0].char_vars) return FAM_ERR_ARG;   // single-context options
  fam_ctx* c = new (std::nothrow) fam_ctx();
  if (!c) return FAM_ERR_NOMEM;
  c->cfg.assign(per, per + n);
  c->ninst = n;
  set_common(c, per[0]);
  c->stream = (hipStream_t)hip_stream;
  c->use_graph = c->stream != nullptr;
  size_t off = 0;
  for (int i = 0; i < n; ++i) {
    c->offsets.push_back(off);
    const size_t cells = (size_t)per[i].nx * per[i].ny;
    c->max_cells = std::max(c->max_cells, cells);
    off += cells * c->nc * c->nmom;
  }
  c->len = off;
  fam_status a = alloc_common(c);
  if (a == FAM_OK) a = init_steps(c);
  if (a == FAM_OK) a = build_inst_tables(c);
  if (a != FAM_OK) {
    fam_destroy(c);
    return a;
  }
  fam_status w = build_work_list(c, 16);
  if (w != FAM_OK) {
    fam_destroy(c);
    return w;
  }
  c->pblocks = std::min(c->nwork, 256 * 8);
  *out = c;
  return FAM_OK;
}

extern "C" size_t fam_state_len(const fam_ctx* c) { return c ? c->len : 0; }
extern "C" size_t fam_instance_offset(const fam_ctx* c, int i) {
  return (c && i >= 0 && i < c->ninst) ? c->offsets[i] : 0;
}
extern "C" int fam_num_instances(const fam_ctx* c) { return c ? c->ninst : 0; }

// ---------------------------------------------------------------------------
// enqueue helpers
// ---------------------------------------------------------------------------
void enqueue_alpha_full(fam_ctx* c, const double* U, int parity) {
  fam::launch_zero_alpha(c->st, c->ninst, parity, c->stream);
  if (c->dim == 1) {
    Inst in = inst_for(c, 0, parity, 0);
    in.alpha_out = &c->st[0].alpha[parity][0][0];
    fam::launch_alpha1d(c->sys, c->phys, U, in, c->flag, c->stream);
    return;
  }
  // the reduction writes into the stage-0 input slot of every instance
  fam::launch_alpha2d(c->sys, c->phys, U, c->d_ainst[parity], c->ninst, c->max_cells, c->flag, c->stream);
}

// Segment-list mode of a single limiter-on 2D instance: buffers, uniform row
// costs and the first list.  Not used when the strips outnumber the wave slots.
static fam_status init_segments(fam_ctx* c) {
  const fam_config& f = c->cfg[0];
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    return FAM_ERR_DEVICE;
  const int strips = (f.nx + fam::STRIP - 1) / fam::STRIP;
  c->seg_budget = 4 * FAM_STAGE_WAVES * cus;   // every stage wave slot of the chip
  if (strips > c->seg_budget || strips > fam::PART_MAX_STRIPS) {
    c->seg_budget = 0;
    return FAM_OK;
  }
  const size_t rows = (size_t)strips * f.ny;
  if (hipMalloc(&c->seg, sizeof(int4) * c->seg_budget) != hipSuccess ||
      hipMalloc(&c->nseg, sizeof(int)) != hipSuccess || hipMalloc(&c->row_cost, sizeof(float) * rows) != hipSuccess ||
      hipMalloc(&c->row_pref, sizeof(float) * rows) != hipSuccess ||
      hipMalloc(&c->part_state, fam::partition_state_bytes()) != hipSuccess)
    return FAM_ERR_NOMEM;
  fam::launch_fill(c->row_cost, 1.0f, rows, c->stream);
  fam::launch_partition(c->row_cost, c->row_pref, c->part_state, strips, f.ny, c->seg_budget, c->seg, c->nseg,
                        c->stream);
  return hipGetLastError() == hipSuccess ? FAM_OK : FAM_ERR_DEVICE;
}

// Set the stage kernel's tile height of a single 2D instance; with the limiter
// the tile order restarts from the identity for the new tile count.
fam_status set_stage_H(fam_ctx* c, int H) {
  c->H = H;
  if (!c->tile_perm) return FAM_OK;
  const fam_config& f = c->cfg[0];
  const int ntiles = ((f.nx + fam::STRIP - 1) / fam::STRIP) * ((f.ny + H - 1) / H);
  if (ntiles > c->tile_cap) return FAM_ERR_ARG;
  fam::launch_tile_identity(c->tile_perm, c->tile_work, ntiles, c->stream);
  return hipGetLastError() == hipSuccess ? FAM_OK : FAM_ERR_DEVICE;
}

void enqueue_stage(fam_ctx* c, int s, int parity, const double* U0, const double* Us, double* Uout,
                   const double* dt_override, bool repartition, double* Uout_mom) {
  static const double CA[3] = {0.0, 0.75, 1.0 / 3.0};
  fam::StageArgs A{};
  A.phys = c->phys;
  A.Us = Us;
  A.U0 = U0;
  A.Uout = Uout;
  A.Uout_mom = Uout_mom;
  A.ca = CA[s];
  A.flag = c->flag;
  A.done = &c->st[0].done;
  A.pp = c->pp;
  A.tile_perm = c->tile_perm;
  A.tile_work = c->tile_work;
  A.row_cost = nullptr;
  if (c->ninst == 1) {
    Inst in = inst_for(c, 0, parity, s);
    if (dt_override) in.dt = dt_override;
    if (c->dim == 1) {
      fam::launch_stage1d(c->k, c->sys, A, in, c->stream);
    } else if (c->stage_list) {
      const fam_config& f = c->cfg[0];
      A.row_cost = c->row_cost;
      fam::launch_stage2d_list(c->k, c->sys, A, in, c->seg, c->nseg, c->seg_budget, c->stream);
      if (repartition)
        fam::launch_partition(c->row_cost, c->row_pref, c->part_state, (f.nx + fam::STRIP - 1) / fam::STRIP, f.ny,
                            c->seg_budget, c->seg, c->nseg, c->stream);
    } else {
      fam::launch_stage2d(c->k, c->sys, A, in, c->H, c->stream);
    }
  } else {
    fam::launch_stage2d_batched(c->k, c->sys, A, c->d_insts[parity][s], c->d_work, c->nwork, c->pblocks, c->stream);
  }
}

void enqueue_oe(fam_ctx* c, int parity, const double* Un, double* Uout, const double* dt_override,
                double* delta_out, const double* Ua) {
  fam::OEArgs A{};
  A.delta_out = delta_out;
  A.phys = c->phys;
  A.Un = Un;
  A.Ua = Ua;
  A.avg_in_place = Ua != nullptr && Ua == Uout;
  A.Uout = Uout;
  A.gamma_k = c->gamma_k;
  A.type = c->oe;
  A.k6_table = c->k6t;
  A.stats = c->stats;
  A.flag = c->flag;
  A.done = &c->st[0].done;
  if (c->ninst == 1) {
    Inst in = inst_for(c, 0, parity, 3);
    if (dt_override) in.dt = dt_override;
    if (c->oe == FAM_OE_TYPE1)
      fam::launch_type1_stats(Un, in, c->nc, c->nmom, c->partial, c->t1_blocks, c->dmax, c->stats, c->stream);
    if (c->dim == 1)
      fam::launch_oe1d(c->k, c->sys, A, in, c->stream);
    else
      fam::launch_oe2d(c->k, c->sys, A, in, c->H_oe, c->stream);
  } else {
    fam::launch_oe2d_batched(c->k, c->sys, A, c->d_insts[parity][3], c->d_work, c->nwork, c->pblocks, c->stream);
  }
}

void enqueue_step(fam_ctx* c, double* U, int parity, double dt_fixed, double t_final) {
  fam::launch_step_begin(c->st, c->ninst, parity, dt_fixed, t_final, c->stream);
  // the segment list (limiter on) is re-cut once per step, from stage 0's row costs
  enqueue_stage(c, 0, parity, U, U, c->W1, nullptr, true);
  enqueue_stage(c, 1, parity, U, c->W1, c->W2, nullptr, false);
  if (c->oe == FAM_OE_OFF) {
    enqueue_stage(c, 2, parity, U, c->W2, U, nullptr, false);
  } else if (c->dim == 2 && c->oe == FAM_OE_TYPE2) {
    // the last stage writes its averages into U in place (each output cell reads
    // only its own U0 value) and its moments into W1; the OE, which changes no
    // average, reads both and writes only U's moment planes
    enqueue_stage(c, 2, parity, U, c->W2, U, nullptr, false, c->W1);
    enqueue_oe(c, parity, c->W1, U, nullptr, nullptr, U);
  } else {
    // Type I's global statistics read one whole state: the OE input stays in W1
    enqueue_stage(c, 2, parity, U, c->W2, c->W1, nullptr, false);
    enqueue_oe(c, parity, c->W1, U, nullptr);
  }
}

// ---------------------------------------------------------------------------
// public entry points
// ---------------------------------------------------------------------------
extern "C" fam_status fam_step(fam_ctx* c, double* U, double dt_fixed, double* dt_used_dev) {
  if (!c || !U) return FAM_ERR_ARG;
  fam_status r = reset_steps(c, 0.0, 0.0);
  if (r != FAM_OK) return r;
  enqueue_alpha_full(c, U, 0);
  enqueue_step(c, U, 0, dt_fixed, 0.0);
  if (dt_used_dev) {
    for (int i = 0; i < c->ninst; ++i)
      HIP_TRY(hipMemcpyAsync(dt_used_dev + i, &c->st[i].dt, sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  }
  return hipGetLastError() == hipSuccess ? FAM_OK : FAM_ERR_DEVICE;
}

extern "C" fam_status fam_set_time(fam_ctx* c, double t) {
  if (!c || !std::isfinite(t)) return FAM_ERR_ARG;
  fam::launch_set_time(c->st, c->ninst, t, c->stream);
  return hipGetLastError() == hipSuccess ? FAM_OK : FAM_ERR_DEVICE;
}

extern "C" fam_status fam_dt(fam_ctx* c, const double* U, double dt_fixed, double* dt_dev) {
  if (!c || !U || !dt_dev) return FAM_ERR_ARG;
  fam_status r = reset_steps(c, 0.0, 0.0);
  if (r != FAM_OK) return r;
  enqueue_alpha_full(c, U, 0);
  fam::launch_step_begin(c->st, c->ninst, 0, dt_fixed, 0.0, c->stream);
  for (int i = 0; i < c->ninst; ++i)
    HIP_TRY(hipMemcpyAsync(dt_dev + i, &c->st[i].dt, sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  return hipGetLastError() == hipSuccess ? FAM_OK : FAM_ERR_DEVICE;
}

extern "C" fam_status fam_stage(fam_ctx* c, int s, const double* U0, const double* Us, double* Uout,
                                const double* dt_dev) {
  if (!c || s < 0 || s > 2 || !U0 || !Us || !Uout || !dt_dev || Uout == Us) return FAM_ERR_ARG;
  if (c->ninst != 1) return FAM_ERR_STATE;
  // as in a step, the segment list (limiter on) is re-cut after the stage-0 launch only
  enqueue_stage(c, s, 0, U0, Us, Uout, dt_dev, s == 0);
  return hipGetLastError() == hipSuccess ? FAM_OK : FAM_ERR_DEVICE;
}

extern "C" fam_status fam_oe(fam_ctx* c, const double* Un, double* Uout, const double* dt_dev) {
  if (!c || !Un || !Uout || !dt_dev || Un == Uout) return FAM_ERR_ARG;
  if (c->ninst != 1) return FAM_ERR_STATE;
  if (c->oe == FAM_OE_OFF) {
    HIP_TRY(hipMemcpyAsync(Uout, Un, c->len * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return FAM_OK;
  }
  enqueue_oe(c, 0, Un, Uout, dt_dev);
  return hipGetLastError() == hipSuccess ? FAM_OK : FAM_ERR_DEVICE;
}

extern "C" fam_status fam_set_tiling(fam_ctx* c, int stage_H, int oe_H) {
  if (!c) return FAM_ERR_ARG;
  if (c->dim != 2 || c->ninst != 1) return FAM_ERR_STATE;
  const int ny = c->cfg[0].ny, hmin = std::min(8, ny);
  if (oe_H < hmin || oe_H > ny) return FAM_ERR_ARG;
  if (stage_H == 0 ? c->seg_budget == 0 : (stage_H < hmin || stage_H > ny)) return FAM_ERR_ARG;
  destroy_graphs(c);
  c->stage_list = stage_H == 0;
  if (stage_H > 0) {
    fam_status r = set_stage_H(c, stage_H);
    if (r != FAM_OK) return r;
  }
  c->H_oe = oe_H;
  return hipGetLastError() == hipSuccess ? FAM_OK : FAM_ERR_DEVICE;
}

extern "C" fam_status fam_dbg_recon(fam_ctx* c, const double* U, double* vals) {
  if (!c || !U || !vals) return FAM_ERR_ARG;
  if (c->ninst != 1 || c->cfg[0].dmr) return FAM_ERR_STATE;
  const Inst in = inst_for(c, 0, 0, 0);
  fam::launch_dbg_recon(c->dim, c->k, c->nc, U, in, vals, c->stream);
  return hipGetLastError() == hipSuccess ? FAM_OK : FAM_ERR_DEVICE;
}

extern "C" fam_status fam_dbg_oe_factors(fam_ctx* c, const double* Un, const double* dt_dev, double* delta) {
  if (!c || !Un || !dt_dev || !delta) return FAM_ERR_ARG;
  if (c->ninst != 1 || c->oe == FAM_OE_OFF) return FAM_ERR_STATE;
  if (Un == c->W2) return FAM_ERR_ARG;
  // the OE launch of fam_oe, its output going to the context's second stage buffer
  enqueue_oe(c, 0, Un, c->W2, dt_dev, delta);
  return hipGetLastError() == hipSuccess ? FAM_OK : FAM_ERR_DEVICE;
}

// ---------------------------------------------------------------------------
// autotuner: times the candidate launch shapes on the caller's state and keeps
// the fastest.  Single 2D instance: the strip-tile height of the stage kernel
// and of the OE kernel (the tile count against the 1024 wave slots of the chip
// sets the tail of the last round of waves; shorter tiles add ring rows).
// Batch: the tile height of the work list and the persistent grid size.
// ---------------------------------------------------------------------------
static fam_status time_launches(fam_ctx* c, int reps, const std::function<void()>& body, float* ms) {
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return FAM_ERR_DEVICE;
  }
  body();   // warm-up
  fam_status r = FAM_OK;
  if (hipEventRecord(e0, c->stream) != hipSuccess) r = FAM_ERR_DEVICE;
  for (int i = 0; i < reps && r == FAM_OK; ++i) body();
  if (r == FAM_OK && hipEventRecord(e1, c->stream) != hipSuccess) r = FAM_ERR_DEVICE;
  if (r == FAM_OK && hipEventSynchronize(e1) != hipSuccess) r = FAM_ERR_DEVICE;
  if (r == FAM_OK && hipEventElapsedTime(ms, e0, e1) != hipSuccess) r = FAM_ERR_DEVICE;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (r == FAM_OK && hipGetLastError() != hipSuccess) r = FAM_ERR_DEVICE;
  return r;
}

extern "C" fam_status fam_autotune(fam_ctx* c, const double* U, int reps, int* choice) {
  if (!c || !U || reps < 1) return FAM_ERR_ARG;
  if (c->dim != 2) return FAM_OK;   // 1D launch shapes are fixed
  destroy_graphs(c);                // graphs hold the launch shapes they were captured with
  std::vector<double> clock;
  fam_status r = save_clock(c, &clock);
  if (r != FAM_OK) return r;
  r = reset_steps(c, 0.0, 0.0);
  if (r != FAM_OK) return r;
  enqueue_alpha_full(c, U, 0);
  fam::launch_step_begin(c->st, c->ninst, 0, 0.0, 0.0, c->stream);
  if (c->ninst == 1) {
    c->stage_list = false;
    const int ny = c->cfg[0].ny;
    std::vector<int> cand = {8, 12, 16, 20, 24, 28, 32, 40, 48, 64};
    // plus the heights whose tile count just fits m whole rounds of the chip's
    // wave slots (4 SIMDs per CU, one or two waves per SIMD)
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
    const int strips = (c->cfg[0].nx + fam::STRIP - 1) / fam::STRIP;
    for (int w = 1; w <= 2; ++w)
      for (int m = 1; m <= 3; ++m) {
        const int per = m * cus * 4 * w / strips;   // tiles per strip
        if (per < 1) continue;
        const int H = (ny + per - 1) / per;
        if (H >= 8 && H <= ny && std::find(cand.begin(), cand.end(), H) == cand.end()) cand.push_back(H);
      }
    float best_s = 1e30f, best_o = 1e30f;
    int hs = c->H, ho = c->H_oe;
    for (int H : cand) {
      if (H > ny && H != cand[0]) continue;
      r = set_stage_H(c, H);
      if (r != FAM_OK) return r;
      c->H_oe = H;
      float ms = 0.0f;
      r = time_launches(c, reps, [&] { enqueue_stage(c, 1, 0, U, U, c->W1, nullptr); }, &ms);
      if (r != FAM_OK) return r;
      if (ms < best_s) { best_s = ms; hs = H; }
      if (c->oe != FAM_OE_OFF) {
        r = time_launches(c, reps, [&] { enqueue_oe(c, 0, U, c->W2, nullptr); }, &ms);
        if (r != FAM_OK) return r;
        if (ms < best_o) { best_o = ms; ho = H; }
      }
    }
    // limiter on: the cost-partitioned segment list (reported as height 0)
    c->stage_list = false;
    if (c->seg_budget > 0) {
      c->stage_list = true;
      float ms = 0.0f;
      r = time_launches(c, reps, [&] { enqueue_stage(c, 1, 0, U, U, c->W1, nullptr); }, &ms);
      if (r != FAM_OK) return r;
      if (ms < best_s) {
        best_s = ms;
        hs = 0;
      } else {
        c->stage_list = false;
      }
    }
    if (hs > 0) {
      r = set_stage_H(c, hs);
      if (r != FAM_OK) return r;
    }
    c->H_oe = ho;
    if (choice) {
      choice[0] = hs;
      choice[1] = ho;
    }
  } else {
    const int candH[] = {8, 12, 16, 24, 32};
    float best = 1e30f;
    int bh = c->batch_H, bp = c->pblocks;
    for (int H : candH) {
      r = build_work_list(c, H);
      if (r != FAM_OK) return r;
      const int candP[] = {1024, 2048, 4096, c->nwork};
      for (int P : candP) {
        c->pblocks = std::max(1, std::min(P, c->nwork));
        float ms = 0.0f;
        r = time_launches(c, reps, [&] {
          enqueue_stage(c, 1, 0, U, U, c->W1, nullptr);
          if (c->oe != FAM_OE_OFF) enqueue_oe(c, 0, U, c->W2, nullptr);
        }, &ms);
        if (r != FAM_OK) return r;
        if (ms < best) { best = ms; bh = H; bp = c->pblocks; }
      }
    }
    r = build_work_list(c, bh);
    if (r != FAM_OK) return r;
    c->pblocks = bp;
    if (choice) {
      choice[0] = bh;
      choice[1] = bp;
    }
  }
  // the timing launches may have raised the device flag on the caller's state;
  // the tuned kernels' outputs are discarded, so is the flag
  HIP_TRY(hipStreamSynchronize(c->stream));
  int z = 0;
  HIP_TRY(hipMemcpy(c->flag, &z, sizeof(int), hipMemcpyHostToDevice));
  return restore_clock(c, clock);
}

extern "C" fam_status fam_check(fam_ctx* c) {
  if (!c) return FAM_ERR_ARG;
  HIP_TRY(hipStreamSynchronize(c->stream));
  int h = 0;
  HIP_TRY(hipMemcpy(&h, c->flag, sizeof(int), hipMemcpyDeviceToHost));
  if (h) {
    int z = 0;
    HIP_TRY(hipMemcpy(c->flag, &z, sizeof(int), hipMemcpyHostToDevice));
    return FAM_ERR_NONPHYSICAL;
  }
  return FAM_OK;
}

static fam_status get_graph(fam_ctx* c, double* U, double dt_fixed, double t_final, hipGraphExec_t* out) {
  fam_ctx::GKey key{U, dt_fixed, t_final};
  auto it = c->graphs.find(key);
  if (it != c->graphs.end()) {
    *out = it->second;
    return FAM_OK;
  }
  hipGraph_t g;
  HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  enqueue_step(c, U, 0, dt_fixed, t_final);
  enqueue_step(c, U, 1, dt_fixed, t_final);
  HIP_TRY(hipStreamEndCapture(c->stream, &g));
  hipGraphExec_t ex;
  hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return FAM_ERR_DEVICE;
  c->graphs[key] = ex;
  *out = ex;
  return FAM_OK;
}

extern "C" fam_status fam_run(fam_ctx* c, double* U, double t_final, int max_steps, double dt_fixed,
                              int* steps_done, double* t_done) {
  if (!c || !U || max_steps < 0) return FAM_ERR_ARG;
  if (!(t_final > 0.0) && max_steps == 0) return FAM_ERR_ARG;
  const int limit = max_steps > 0 ? max_steps : 0x7fffffff;
  fam_status r = reset_steps(c, t_final > 0 ? t_final : 0.0, dt_fixed);
  if (r != FAM_OK) return r;
  enqueue_alpha_full(c, U, 0);
  const double tf = t_final > 0 ? t_final : 0.0;
  int launched = 0;
  std::vector<StepState> h(c->ninst);
  int done_steps = 0;
  double tmin = 0.0;
  // With an end time, the first chunk is two steps; each later chunk holds the
  // steps still needed at the last step's dt (at most 64, rounded up to even), so
  // few replays past the end time are no-ops.
  int next = tf > 0 ? 2 : limit;
  while (launched < limit) {
    const int chunk = std::min(limit - launched, next);
    const int pairs = chunk / 2;
    if (c->use_graph && pairs > 0) {
      hipGraphExec_t ex;
      r = get_graph(c, U, dt_fixed, tf, &ex);
      if (r != FAM_OK) return r;
      for (int p = 0; p < pairs; ++p) HIP_TRY(hipGraphLaunch(ex, c->stream));
    } else {
      for (int p = 0; p < pairs; ++p) {
        enqueue_step(c, U, 0, dt_fixed, tf);
        enqueue_step(c, U, 1, dt_fixed, tf);
      }
    }
    if (chunk % 2) enqueue_step(c, U, 0, dt_fixed, tf);
    launched += chunk;
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(h.data(), c->st, sizeof(StepState) * c->ninst, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    bool all_done = true;
    done_steps = 0;
    tmin = 1e300;
    double need = 0.0;
    for (auto& s : h) {
      const bool fin = (s.done != 0) || (tf > 0 && s.t >= tf);
      all_done &= fin;
      done_steps = std::max(done_steps, s.steps);
      tmin = std::min(tmin, s.t);
      if (!fin && s.dt > 0.0) need = std::max(need, std::ceil((tf - s.t) / s.dt));
    }
    int fl = 0;
    HIP_TRY(hipMemcpy(&fl, c->flag, sizeof(int), hipMemcpyDeviceToHost));
    if (fl) {
      if (steps_done) *steps_done = done_steps;
      if (t_done) *t_done = tmin;
      int z = 0;
      HIP_TRY(hipMemcpy(c->flag, &z, sizeof(int), hipMemcpyHostToDevice));
      return FAM_ERR_NONPHYSICAL;
    }
    if (tf > 0 && all_done) break;
    if (chunk % 2) break;   // parity would break on another chunk; odd chunks only end a run
    if (tf > 0) {
      const int want = need > 62.0 ? 64 : std::max(2, (int)need);
      next = want + (want & 1);
    }
  }
  if (steps_done) *steps_done = done_steps;
  if (t_done) *t_done = tmin;
  return FAM_OK;
}
