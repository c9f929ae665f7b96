// fam_static.hip - fam_step_static: one FAM step without a context and without
// any device allocation, for callers that cannot allocate (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).
//
// Its scratch (the two SSP-RK3 stage states, the step bookkeeping, the wave-speed
// and Type I reduction slots, the limiter's tile order) lives in one file-scope
// device array of FAM_STATIC_SCRATCH_BYTES per GPU, held until the process ends.
// Host code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): its device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and kept per device.  Every call
// on one GPU shares that GPU's array, so calls that overlap on one GPU race; each
// call initialises the parts that must start from zero before using them.
//
// The kernels are those of fam_step (same launch shapes as a fresh context's:
// the default strip-tile heights, no segment list), so the result equals
// fam_step's bit for bit.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <mutex>

#include "../../include/fam.h"
#include "fam_ctx.h"
#include "fam_kernels.h"

using fam::Inst;
using fam::StepState;

namespace {

static __device__ __align__(256) double scratch[FAM_STATIC_SCRATCH_BYTES / sizeof(double)];

// byte offsets inside the scratch array
constexpr size_t OFF_ST = 0;              // StepState
constexpr size_t OFF_FLAG = 256;          // internal non-physical flag (int)
constexpr size_t OFF_AINST = 512;         // Inst record of the 2D wave-speed reduction
constexpr size_t OFF_STATS = 1024;        // Type I: D_Omega, eps_Omega per component
constexpr size_t OFF_DMAX = 1280;         // Type I: maxima
constexpr size_t OFF_PARTIAL = 1536;      // Type I: per-block partial sums (4 x T1_BLOCKS)
constexpr int T1_BLOCKS = 256;
constexpr size_t OFF_TILES = 10240;       // limiter: tile order (ntiles + 1) and work (ntiles) ints
constexpr size_t TILE_BYTES = 128 * 1024;
constexpr size_t OFF_W = 256 * 1024;      // W1, W2: two stage states
static_assert(sizeof(StepState) <= OFF_FLAG - OFF_ST, "StepState slot");
static_assert(sizeof(Inst) <= OFF_STATS - OFF_AINST, "Inst slot");
static_assert(OFF_PARTIAL + 4 * T1_BLOCKS * sizeof(double) <= OFF_TILES, "Type I slots");
static_assert(OFF_TILES + TILE_BYTES <= OFF_W, "tile slots");
static_assert(FAM_STATIC_SCRATCH_BYTES % 256 == 0 && OFF_W % 256 == 0, "alignment");

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
char* g_ptr[MAX_DEVICES] = {};

// the scratch array's device address on the current device (looked up once)
fam_status scratch_ptr(char** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return FAM_ERR_DEVICE;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FAM_ERR_DEVICE;
    g_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_ptr[dev];
  return FAM_OK;
}

// every field of the step bookkeeping, the wave-speed Inst record and the
// internal flag, from values passed by value (a kernel: no memset or host copy)
__global__ void static_init_kernel(StepState* st, StepState s0, Inst* ainst, Inst a0, int* flag) {
  if (threadIdx.x == 0) {
    *st = s0;
    *ainst = a0;
    *flag = 0;
  }
}

}  // namespace

// the largest state (doubles) whose two stage copies fit after the fixed slots
constexpr size_t LEN_LIMIT = (FAM_STATIC_SCRATCH_BYTES - OFF_W) / (2 * sizeof(double));

extern "C" fam_status fam_step_static(const fam_config* cfg, void* hip_stream, double* U, double t,
                                      double dt_fixed, double* dt_used_dev, int* flag_dev) {
  if (!cfg || !U || !std::isfinite(t) || std::isnan(dt_fixed)) return FAM_ERR_ARG;
  fam_status v = validate_config(*cfg);
  if (v != FAM_OK) return v;
  fam_config f = *cfg;
  if (f.dim == 1) { f.ny = 1; f.y0 = 0.0; f.y1 = 1.0; }
  const int dim = f.dim;
  const int nc = f.system == FAM_EULER ? dim + 2 : 1;
  const int nmom = dim == 1 ? 2 : 3;
  const size_t cells = (size_t)f.nx * f.ny;
  const size_t len = cells * nc * nmom;
  if (len > LEN_LIMIT) return FAM_ERR_SIZE;
  const int H = dim == 2 ? choose_H(f.nx, f.ny) : 1;
  const int ntiles = dim == 2 ? ((f.nx + fam::STRIP - 1) / fam::STRIP) * ((f.ny + H - 1) / H) : 0;
  if (f.pp && (size_t)(2 * ntiles + 1) * sizeof(int) > TILE_BYTES) return FAM_ERR_SIZE;

  char* base = nullptr;
  fam_status r = scratch_ptr(&base);
  if (r != FAM_OK) return r;
  hipStream_t s = (hipStream_t)hip_stream;
  StepState* st = reinterpret_cast<StepState*>(base + OFF_ST);
  int* flag = flag_dev ? flag_dev : reinterpret_cast<int*>(base + OFF_FLAG);
  Inst* ainst = reinterpret_cast<Inst*>(base + OFF_AINST);
  double* stats = reinterpret_cast<double*>(base + OFF_STATS);
  double* dmax = reinterpret_cast<double*>(base + OFF_DMAX);
  double* partial = reinterpret_cast<double*>(base + OFF_PARTIAL);
  int* tile_perm = reinterpret_cast<int*>(base + OFF_TILES);
  int* tile_work = tile_perm + (ntiles + 1);
  double* W1 = reinterpret_cast<double*>(base + OFF_W);
  double* W2 = W1 + len;

  // the instance and the step bookkeeping a fresh context would hold
  Inst in{};
  in.id = 0;
  in.nx = f.nx;
  in.ny = f.ny;
  in.plane = cells;
  in.offset = 0;
  in.dx = (f.x1 - f.x0) / f.nx;
  in.dy = dim == 2 ? (f.y1 - f.y0) / f.ny : 1.0;
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
  in.dt = &st->dt;
  in.done = &st->done;
  in.t_end = &st->t;
  StepState s0{};
  s0.cfl = f.cfl;
  const double e = f.dt_rule == 1 ? f.k / 3.0 : 1.0;
  s0.hx = std::pow(in.dx, e);
  s0.hy = dim == 2 ? std::pow(in.dy, e) : 1.0;
  s0.dim = dim;
  s0.t = t;
  Inst a0 = in;
  a0.alpha_in = &st->alpha[0][0][0];
  a0.alpha_out = &st->alpha[0][0][0];
  hipLaunchKernelGGL(static_init_kernel, dim3(1), dim3(64), 0, s, st, s0, ainst, a0,
                     reinterpret_cast<int*>(base + OFF_FLAG));
  if (f.pp) fam::launch_tile_identity(tile_perm, tile_work, ntiles, s);

  const fam::PhysParams phys{f.gamma, f.ax, f.ay};
  // wave speeds of U into the stage-0 input slot, then dt and the clock
  if (dim == 1) {
    fam::launch_alpha1d(f.system, phys, U, a0, flag, s);
  } else {
    fam::launch_alpha2d(f.system, phys, U, ainst, 1, cells, flag, s);
  }
  fam::launch_step_begin(st, 1, 0, dt_fixed, 0.0, s);

  static const double CA[3] = {0.0, 0.75, 1.0 / 3.0};
  auto stage = [&](int k_s, const double* Us, double* Uout, double* Uout_mom) {
    fam::StageArgs A{};
    A.phys = phys;
    A.Us = Us;
    A.U0 = U;
    A.Uout = Uout;
    A.Uout_mom = Uout_mom;
    A.ca = CA[k_s];
    A.flag = flag;
    A.done = &st->done;
    A.pp = f.pp;
    A.tile_perm = tile_perm;
    A.tile_work = tile_work;
    A.row_cost = nullptr;
    Inst is = in;
    is.alpha_in = &st->alpha[0][k_s][0];
    is.alpha_out = k_s < 2 ? &st->alpha[0][k_s + 1][0] : &st->alpha[1][0][0];
    is.t_ofs = k_s == 0 ? 1.0 : k_s == 2 ? 0.5 : 0.0;
    if (dim == 1)
      fam::launch_stage1d(f.k, f.system, A, is, s);
    else
      fam::launch_stage2d(f.k, f.system, A, is, H, s);
  };
  stage(0, U, W1, nullptr);
  stage(1, W1, W2, nullptr);
  if (f.oe == FAM_OE_OFF) {
    stage(2, W2, U, nullptr);
  } else {
    // as in fam_step: with Type II in 2D the last stage writes its averages into U
    // in place and its moments into W1, and the OE writes only U's moment planes
    const bool split = dim == 2 && f.oe == FAM_OE_TYPE2;
    if (split)
      stage(2, W2, U, W1);
    else
      stage(2, W2, W1, nullptr);
    fam::OEArgs A{};
    A.delta_out = nullptr;
    A.phys = phys;
    A.Un = W1;
    A.Ua = split ? U : nullptr;
    A.avg_in_place = split;
    A.Uout = U;
    A.gamma_k = f.oe_gamma_k > 0 ? f.oe_gamma_k : default_gamma_k(dim, f.k);
    A.type = f.oe;
    A.k6_table = f.k6_jump_from_table;
    A.stats = stats;
    A.flag = flag;
    A.done = &st->done;
    Inst io = in;
    io.alpha_in = &st->alpha[0][0][0];
    io.alpha_out = nullptr;
    io.t_ofs = 0.0;
    if (f.oe == FAM_OE_TYPE1) fam::launch_type1_stats(W1, io, nc, nmom, partial, T1_BLOCKS, dmax, stats, s);
    if (dim == 1)
      fam::launch_oe1d(f.k, f.system, A, io, s);
    else
      fam::launch_oe2d(f.k, f.system, A, io, H, s);
  }
  if (dt_used_dev && hipMemcpyAsync(dt_used_dev, &st->dt, sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
    return FAM_ERR_DEVICE;
  return hipGetLastError() == hipSuccess ? FAM_OK : FAM_ERR_DEVICE;
}
