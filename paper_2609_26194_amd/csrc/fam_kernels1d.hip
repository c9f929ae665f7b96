// fam_kernels1d.hip - HIP kernels of the 1D FAM step and the per-step
// bookkeeping (time step, clipping, termination) for gfx950.
//
// 1D tile: a block of 256 lanes covers cells i0-1 .. i0+254 (lane t <-> cell
// i0-1+t) and writes cells i0 .. i0+253.  The state of cells i0-2 .. i0+255 is
// staged in LDS; each lane reconstructs its cell (appendix "One-dimensional
// reconstruction coefficients"), publishes its right trace, computes the flux
// of its left interface once, and the Shu-Osher update of eq. (3) uses
//   R0 = -(f_{i+1/2} - f_{i-1/2})/dx,
//   R1 = (sum_g w_g f(p(xi_g)) - (f_{i+1/2} + f_{i-1/2})/2)/dx     (eq. 1dSemi).
// OE (Prop. 2.1, eq. 1dOE_system, Table sigma1d): jumps at both interfaces of the
// cell, Type I / II denominator over Lambda_i = {i-1, i, i+1}, sigma = max over
// components, u^(1) <- u^(1) exp(-beta dt sigma / dx).
#include "fam_char.h"
#include "fam_device.h"
#include "fam_kernels.h"

namespace fam {

constexpr int T1 = 256;           // lanes per block
constexpr int OUT1 = T1 - 2;      // cells written per block
constexpr int NPL1 = 6;           // up to 3 components x 2 moments

// 1D Gauss nodes in the oracle's order: -GS1, -GS0, GS0, GS1
__device__ __forceinline__ constexpr double g1x(int q) {
  return q == 0 ? -GS1 : q == 1 ? -GS0 : q == 2 ? GS0 : GS1;
}
__device__ __forceinline__ constexpr double g1w(int q) { return (q == 0 || q == 3) ? GW1 : GW0; }

template <int K>
__device__ __forceinline__ double poly1d(const double* c, double x) {
  double v = 0.0;
#pragma unroll
  for (int l = 0; l < K; ++l) v = fma(c[l], leg(l, x), v);
  return v;
}

template <class P>
__device__ __forceinline__ P make_phys1(const PhysParams& pp);
template <>
__device__ __forceinline__ Advection make_phys1<Advection>(const PhysParams& pp) { return Advection{pp.ax, pp.ay}; }
template <>
__device__ __forceinline__ Burgers make_phys1<Burgers>(const PhysParams& pp) { return Burgers{pp.ax, pp.ay}; }
template <>
__device__ __forceinline__ Euler<1> make_phys1<Euler<1>>(const PhysParams& pp) { return Euler<1>{pp.gamma}; }

struct Tile1 {
  double u[NPL1][T1 + 2];   // cells i0-2 .. i0+255
  double tr[3][T1];         // right traces
  double fx[3][T1];         // interface fluxes (left interface of lane t)
};

template <int NC>
__device__ __forceinline__ void load_tile1(Tile1& S, const double* __restrict__ U, const Inst& in, int i0) {
  for (int x = threadIdx.x; x < T1 + 2; x += T1) {
    const int gi = ghost(i0 - 2 + x, in.nx, in.bcx);
#pragma unroll
    for (int p = 0; p < NC * 2; ++p) S.u[p][x] = U[in.offset + p * in.plane + gi];
  }
}

template <int K, class P, bool CHAR = false>
__global__ void __launch_bounds__(T1) stage1d_kernel(StageArgs A, Inst in) {
  constexpr int NC = P::NC;
  __shared__ Tile1 S;
  if (*A.done) return;
  const P phys = make_phys1<P>(A.phys);
  const int t = threadIdx.x;
  const int i0 = blockIdx.x * OUT1;
  const int i = i0 - 1 + t;
  const double dx = in.dx, ax = in.alpha_in[0], dt = *in.dt;
  load_tile1<NC>(S, A.Us, in, i0);
  __syncthreads();
  // reconstruction of cell i (LDS column t+1)
  constexpr int NB = (K <= 4) ? (K == 3 ? 3 : 4) : (K == 5 ? 5 : 6);   // coefficients of p
  double cf[NC][6];
  if constexpr (CHAR) {
    // in the characteristic variables of this cell's average (L on the stencil,
    // reconstruction per field, R on the coefficients)
    double La[NC][NC], Ra[NC][NC];
    {
      double a[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) a[c] = S.u[2 * c][t + 1];
      char_basis_x<1>(phys.g, a, La, Ra);
    }
#pragma unroll
    for (int w = 0; w < NC; ++w) {
      double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
          for (int o = 0; o < 3; ++o) v[3 * m + o] = fma(La[w][c], S.u[2 * c + m][t + o], v[3 * m + o]);
      coeffs1d<K>(v[0], v[1], v[2], v[3], v[4], v[5], cf[w]);
    }
#pragma unroll
    for (int l = 0; l < NB; ++l) {
      double tw[NC];
#pragma unroll
      for (int w = 0; w < NC; ++w) tw[w] = cf[w][l];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        double x = 0.0;
#pragma unroll
        for (int w = 0; w < NC; ++w) x = fma(Ra[c][w], tw[w], x);
        cf[c][l] = x;
      }
    }
  } else {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      coeffs1d<K>(S.u[2 * c][t], S.u[2 * c][t + 1], S.u[2 * c][t + 2], S.u[2 * c + 1][t], S.u[2 * c + 1][t + 1],
                  S.u[2 * c + 1][t + 2], cf[c]);
    }
  }
  double lt[NC], rt[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    rt[c] = poly1d<NB>(cf[c], 0.5);
    lt[c] = poly1d<NB>(cf[c], -0.5);
    S.tr[c][t] = rt[c];
  }
  double V[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) V[c] = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double v[NC], f[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = poly1d<NB>(cf[c], g1x(q));
    phys.flux(0, v, f);
#pragma unroll
    for (int c = 0; c < NC; ++c) V[c] = fma(g1w(q), f[c], V[c]);
  }
  __syncthreads();
  if (t >= 1) {
    double ul[NC], fl[NC], fr[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) ul[c] = S.tr[c][t - 1];
    phys.flux(0, ul, fl);
    phys.flux(0, lt, fr);
#pragma unroll
    for (int c = 0; c < NC; ++c) S.fx[c][t] = 0.5 * (fl[c] + fr[c]) - 0.5 * ax * (lt[c] - ul[c]);
  }
  __syncthreads();
  double amax = 0.0;
  bool bad = false;
  if (t >= 1 && t <= OUT1 && i < in.nx) {
    double avg[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double fL = S.fx[c][t], fR = S.fx[c][t + 1];
      const double R0 = -(fR - fL) / dx;
      const double R1 = (V[c] - 0.5 * (fR + fL)) / dx;
      const double Rm[2] = {R0, R1};
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const size_t idx = in.offset + (c * 2 + m) * in.plane + i;
        const double L = S.u[2 * c + m][t + 1] + dt * Rm[m];
        const double v = (A.ca == 0.0) ? L : fma(A.ca, A.U0[idx] - L, L);
        A.Uout[idx] = v;
        if (m == 0) avg[c] = v;
      }
    }
    amax = phys.speed(0, avg, bad);
  }
  amax = wave_max(amax);
  const bool any_bad = __any(bad);
  if ((t & 63) == 0) {
    atomic_max_nonneg(&in.alpha_out[0], amax);
    if (any_bad) atomicOr(A.flag, 1);
  }
}

template <int K, class P>
__global__ void __launch_bounds__(T1) oe1d_kernel(OEArgs A, Inst in) {
  constexpr int NC = P::NC;
  constexpr int NB = (K <= 4) ? (K == 3 ? 3 : 4) : (K == 5 ? 5 : 6);
  __shared__ Tile1 S;
  if (*A.done) return;
  const P phys = make_phys1<P>(A.phys);
  const int t = threadIdx.x;
  const int i0 = blockIdx.x * OUT1;
  const int i = i0 - 1 + t;
  const double dt = *in.dt;
  load_tile1<NC>(S, A.Un, in, i0);
  __syncthreads();
  double lt[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    double cf[6];
    coeffs1d<K>(S.u[2 * c][t], S.u[2 * c][t + 1], S.u[2 * c][t + 2], S.u[2 * c + 1][t], S.u[2 * c + 1][t + 1],
                S.u[2 * c + 1][t + 2], cf);
    S.tr[c][t] = poly1d<NB>(cf, 0.5);
    lt[c] = poly1d<NB>(cf, -0.5);
  }
  __syncthreads();
  if (t >= 1) {
#pragma unroll
    for (int c = 0; c < NC; ++c) S.fx[c][t] = lt[c] - S.tr[c][t - 1];   // jump at i-1/2
  }
  __syncthreads();
  bool bad = false;
  if (t >= 1 && t <= OUT1 && i < in.nx) {
    double sig = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double J = fabs(S.fx[c][t]) + fabs(S.fx[c][t + 1]);
      double D, eps;
      if (A.type == 2) {
        const double a = S.u[2 * c][t], b = S.u[2 * c][t + 1], d = S.u[2 * c][t + 2];
        const double Ssum = (a + b) + d;
        D = fmax(fmax(fabs(a - Ssum), fabs(b - Ssum)), fabs(d - Ssum));
        eps = 1e-14 * fmax(fmax(fmax(fabs(a), fabs(b)), fabs(d)), 1.0);
      } else {
        D = A.stats[in.id * 8 + c];
        eps = A.stats[in.id * 8 + 4 + c];
      }
      const double s = (D < eps) ? 0.0 : A.gamma_k * J / D;
      sig = fmax(sig, s);
    }
    double beta = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double avg[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) avg[c] = S.u[2 * c][t + a];
      beta = fmax(beta, phys.speed(0, avg, bad));
    }
    const double delta = exp(-beta * dt * sig / in.dx);
    if (A.delta_out) A.delta_out[i] = delta;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      A.Uout[in.offset + (c * 2) * in.plane + i] = S.u[2 * c][t + 1];
      A.Uout[in.offset + (c * 2 + 1) * in.plane + i] = S.u[2 * c + 1][t + 1] * delta;
    }
  }
  if (__any(bad) && (t & 63) == 0) atomicOr(A.flag, 1);
}

template <class P>
__global__ void __launch_bounds__(256) alpha1d_kernel(PhysParams pp, const double* __restrict__ U, Inst in,
                                                      int* flag) {
  const P phys = make_phys1<P>(pp);
  constexpr int NC = P::NC;
  bool bad = false;
  double mx = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < in.nx; i += gridDim.x * blockDim.x) {
    double avg[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) avg[c] = U[in.offset + (c * 2) * in.plane + i];
    mx = fmax(mx, phys.speed(0, avg, bad));
  }
  mx = wave_max(mx);
  const bool any_bad = __any(bad);
  if ((threadIdx.x & 63) == 0) {
    atomic_max_nonneg(&in.alpha_out[0], mx);
    if (any_bad) atomicOr(flag, 1);
  }
}

// ---------------------------------------------------------------------------
// step bookkeeping
// ---------------------------------------------------------------------------
__global__ void step_begin_kernel(StepState* st, int ninst, int parity, double dt_fixed, double t_final) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= ninst) return;
  StepState& s = st[id];
  const int q = parity, o = 1 - parity;
  s.alpha[q][1][0] = s.alpha[q][1][1] = 0.0;
  s.alpha[q][2][0] = s.alpha[q][2][1] = 0.0;
  s.alpha[o][0][0] = s.alpha[o][0][1] = 0.0;
  if (s.done) {
    s.dt = 0.0;
    return;
  }
  double dt;
  if (dt_fixed > 0.0) {
    dt = dt_fixed;
  } else {
    const double ax = s.alpha[q][0][0], ay = s.alpha[q][0][1];
    dt = (s.dim == 1) ? s.cfl * s.hx / ax : s.cfl / (ax / s.hx + ay / s.hy);
  }
  double tn = s.t + dt;
  if (t_final > 0.0) {
    if (s.t >= t_final) {
      s.done = 1;
      s.dt = 0.0;
      return;
    }
    if (tn >= t_final) {
      dt = t_final - s.t;
      tn = t_final;
    }
  }
  if (!(dt > 0.0) || !(dt < 1e300)) {
    s.done = 1;
    s.dt = 0.0;
    return;
  }
  s.dt = dt;
  s.t = tn;
  s.steps += 1;
}

__global__ void zero_alpha_kernel(StepState* st, int ninst, int parity) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= ninst) return;
  st[id].alpha[parity][0][0] = 0.0;
  st[id].alpha[parity][0][1] = 0.0;
}

__global__ void reset_steps_kernel(StepState* st, int ninst, double t_final, double dt_fixed) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= ninst) return;
  StepState& s = st[id];
  for (int p = 0; p < 2; ++p)
    for (int q = 0; q < 3; ++q) s.alpha[p][q][0] = s.alpha[p][q][1] = 0.0;
  s.dt = 0.0;
  s.t_final = t_final;
  s.dt_fixed = dt_fixed;
  s.done = 0;
  s.steps = 0;
}

void launch_reset_steps(StepState* st, int ninst, double t_final, double dt_fixed, hipStream_t s) {
  hipLaunchKernelGGL(reset_steps_kernel, dim3((ninst + 63) / 64), dim3(64), 0, s, st, ninst, t_final, dt_fixed);
}

// the context clock: every instance's time set to t (a kernel, not a memset, so a
// captured graph may hold it)
__global__ void set_time_kernel(StepState* st, int ninst, double t) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id < ninst) st[id].t = t;
}

void launch_set_time(StepState* st, int ninst, double t, hipStream_t s) {
  hipLaunchKernelGGL(set_time_kernel, dim3((ninst + 63) / 64), dim3(64), 0, s, st, ninst, t);
}

void launch_step_begin(StepState* st, int ninst, int parity, double dt_fixed, double t_final, hipStream_t s) {
  hipLaunchKernelGGL(step_begin_kernel, dim3((ninst + 63) / 64), dim3(64), 0, s, st, ninst, parity, dt_fixed,
                     t_final);
}
void launch_zero_alpha(StepState* st, int ninst, int parity, hipStream_t s) {
  hipLaunchKernelGGL(zero_alpha_kernel, dim3((ninst + 63) / 64), dim3(64), 0, s, st, ninst, parity);
}

#define FAM_DISPATCH_K1(K_, BODY)                    \
  switch (K_) {                                      \
    case 3: { constexpr int KK = 3; BODY; } break;   \
    case 4: { constexpr int KK = 4; BODY; } break;   \
    case 5: { constexpr int KK = 5; BODY; } break;   \
    case 6: { constexpr int KK = 6; BODY; } break;   \
    default: break;                                  \
  }
#define FAM_DISPATCH_P1(SYS_, BODY)                  \
  switch (SYS_) {                                    \
    case 0: { using PP = Advection; BODY; } break;   \
    case 1: { using PP = Burgers; BODY; } break;     \
    default: { using PP = Euler<1>; BODY; } break;   \
  }

void launch_stage1d(int k, int sys, const StageArgs& A, const Inst& in, hipStream_t s) {
  const dim3 grid((in.nx + OUT1 - 1) / OUT1);
  if (in.charv && sys == 2 && k == 5) {   // characteristic variables: Euler, FAM5
    hipLaunchKernelGGL((stage1d_kernel<5, Euler<1>, true>), grid, dim3(T1), 0, s, A, in);
    return;
  }
  FAM_DISPATCH_P1(sys, FAM_DISPATCH_K1(k, hipLaunchKernelGGL((stage1d_kernel<KK, PP>), grid, dim3(T1), 0, s, A, in)));
}
void launch_oe1d(int k, int sys, const OEArgs& A, const Inst& in, hipStream_t s) {
  const dim3 grid((in.nx + OUT1 - 1) / OUT1);
  FAM_DISPATCH_P1(sys, FAM_DISPATCH_K1(k, hipLaunchKernelGGL((oe1d_kernel<KK, PP>), grid, dim3(T1), 0, s, A, in)));
}
void launch_alpha1d(int sys, const PhysParams& pp, const double* U, const Inst& in, int* flag, hipStream_t s) {
  const int nb = std::max(1, std::min(256, (in.nx + 255) / 256));
  FAM_DISPATCH_P1(sys, hipLaunchKernelGGL((alpha1d_kernel<PP>), dim3(nb), dim3(256), 0, s, pp, U, in, flag));
}

}  // namespace fam
