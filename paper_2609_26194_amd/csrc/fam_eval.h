// fam_eval.h - point evaluation of the 2D reconstruction and compile-time linear
// functionals of the 3x3 stencil, shared by the forward and adjoint kernels.
#pragma once

#include <utility>

#include "fam_device.h"

namespace fam {

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


// Stencil slots that the reconstruction reads: slot 0..8 the averages of the
// 3x3 patch, 9..17 its x-moments, 18..26 its y-moments (patch index b*3 + a).
// For k = 3, 4 only the centre cell's moments enter; for k = 5, 6 the x-moments
// of the cells above and below and the y-moments of the cells left and right
// are not part of the stencil.
template <int K>
__host__ __device__ constexpr bool slot_used(int in) {
  const int l = in % 9;
  if (in < 9) return true;
  if (in < 18) return K >= 5 ? (l != 1 && l != 7) : (l == 4);
  return K >= 5 ? (l != 3 && l != 5) : (l == 4);
}

// ---------------------------------------------------------------------------
// Face-centre values p(1/2, 0), p(-1/2, 0), p(0, 1/2), p(0, -1/2) as linear
// functionals of the stencil inputs u0[1..9], u1[1..9], u2[1..9] (27 slots),
// evaluated at compile time from the coefficient formulas.
// ---------------------------------------------------------------------------
struct CentreWeights {
  double w[4][27];   // [r, l, t, b][u0 1..9, u1 1..9, u2 1..9]
};

template <int K, bool FULL>
__host__ __device__ constexpr CentreWeights make_centre_weights() {
  CentreWeights cw{};
  const double px[4] = {0.5, -0.5, 0.0, 0.0}, py[4] = {0.0, 0.0, 0.5, -0.5};
  const int ncf = FULL ? 23 : ncoef2d(K);
  for (int in = 0; in < 27; ++in) {
    if (!slot_used<K>(in)) continue;
    double u[27] = {};
    u[in] = 1.0;
    double c[23] = {};
    coeffs2d<K>(u, u + 9, u + 18, c, FULL);
    for (int f = 0; f < 4; ++f) {
      double v = 0.0;
      for (int l = 0; l < ncf; ++l) v += c[l] * leg(AX[l], px[f]) * leg(AY[l], py[f]);
      cw.w[f][in] = v;
    }
  }
  return cw;
}

template <int K, bool FULL>
struct CentreTable {
  static constexpr CentreWeights t = make_centre_weights<K, FULL>();
};

// v += w * u[I] with w a compile-time constant (skipped when zero)
template <int K, bool FULL, int F, int I>
__device__ __forceinline__ void centre_acc(double& v, const double (&u)[27]) {
  constexpr double w = CentreTable<K, FULL>::t.w[F][I];
  if constexpr (w != 0.0) v = fma(w, u[I], v);
}

template <int K, bool FULL, int F, int... I>
__device__ __forceinline__ double centre_dot(const double (&u)[27], std::integer_sequence<int, I...>) {
  double v = 0.0;
  (centre_acc<K, FULL, F, I>(v, u), ...);
  return v;
}


// ---------------------------------------------------------------------------
// Transposed reconstruction: RT[in][l] = d c_l / d u_in for the 27 stencil slots
// ---------------------------------------------------------------------------
template <int K>
struct ReconT {
  double w[27][23];
};

template <int K>
__host__ __device__ constexpr ReconT<K> make_recon_t() {
  ReconT<K> r{};
  for (int in = 0; in < 27; ++in) {
    if (!slot_used<K>(in)) continue;
    double u[27] = {};
    u[in] = 1.0;
    double c[23] = {};
    coeffs2d<K>(u, u + 9, u + 18, c, false);
    for (int l = 0; l < 23; ++l) r.w[in][l] = c[l];
  }
  return r;
}

template <int K>
struct ReconTable {
  static constexpr ReconT<K> t = make_recon_t<K>();
};

// acc += sum_l RT[IN][l] a[l] over the p_k coefficients (zeros skipped at compile time)
template <int K, int IN, int L>
__device__ __forceinline__ void rt_acc1(double& acc, const double* a) {
  constexpr double w = ReconTable<K>::t.w[IN][L];
  if constexpr (w != 0.0) acc = fma(w, a[L], acc);
}
template <int K, int IN, int... L>
__device__ __forceinline__ double rt_dot(const double* a, std::integer_sequence<int, L...>) {
  double acc = 0.0;
  (rt_acc1<K, IN, L>(acc, a), ...);
  return acc;
}

// acc += sum_f CW[f][IN] b[f] (transposed face-centre functionals)
template <int K, bool FULL, int IN, int F>
__device__ __forceinline__ void cwt_acc1(double& acc, const double* b) {
  constexpr double w = CentreTable<K, FULL>::t.w[F][IN];
  if constexpr (w != 0.0) acc = fma(w, b[F], acc);
}
template <int K, bool FULL, int IN>
__device__ __forceinline__ double cwt_dot(const double* b) {
  double acc = 0.0;
  cwt_acc1<K, FULL, IN, 0>(acc, b);
  cwt_acc1<K, FULL, IN, 1>(acc, b);
  cwt_acc1<K, FULL, IN, 2>(acc, b);
  cwt_acc1<K, FULL, IN, 3>(acc, b);
  return acc;
}


// ---------------------------------------------------------------------------
// Sign-symmetric point groups.  The 32 flux points of a cell form 8 groups of
// 4 points (sx X, sy Y), sx, sy = +-1, with (X, Y) one of (1/2, GS0), (1/2, GS1)
// (x-faces), (GS0, 1/2), (GS1, 1/2) (y-faces) and {GS0, GS1}^2 (volume).
// phi_l(sx X, sy Y) = phi_l(X, Y) sx^(ax_l odd) sy^(ay_l odd): the values at the
// four points follow from four parity sums of the coefficients, and the
// transposed evaluation from four signed sums.  Node indices: 0 = GS0,
// 1 = GS1, 2 = 1/2.  Point s of a group: 0 (+,+), 1 (+,-), 2 (-,+), 3 (-,-).
// ---------------------------------------------------------------------------
template <int L>
__device__ __forceinline__ constexpr int parity_class() {
  return (AX[L] & 1) + 2 * (AY[L] & 1);
}

template <int L, int NXI, int NYI>
__device__ __forceinline__ constexpr double phi_node() {
  return legn(AX[L], NXI) * legn(AY[L], NYI);
}

template <int NXI, int NYI, int... L>
__device__ __forceinline__ void parity_sums(const double* cf, double (&P)[4], std::integer_sequence<int, L...>) {
  P[0] = P[1] = P[2] = P[3] = 0.0;
  ((P[parity_class<L>()] = fma(cf[L], phi_node<L, NXI, NYI>(), P[parity_class<L>()])), ...);
}

template <int NXI, int NYI, int... L>
__device__ __forceinline__ void parity_scatter(double* ab, const double (&Q)[4], std::integer_sequence<int, L...>) {
  ((ab[L] = fma(phi_node<L, NXI, NYI>(), Q[parity_class<L>()], ab[L])), ...);
}

// point s of a group: s = 0 (+,+), 1 (+,-), 2 (-,+), 3 (-,-)
__device__ __forceinline__ constexpr double grp_sx(int s) { return s < 2 ? 1.0 : -1.0; }
__device__ __forceinline__ constexpr double grp_sy(int s) { return (s & 1) ? -1.0 : 1.0; }

template <int NXI, int NYI, int NCF>
__device__ __forceinline__ void group_values(const double* cf, double (&v)[4]) {
  double P[4];
  parity_sums<NXI, NYI>(cf, P, std::make_integer_sequence<int, NCF>{});
  const double a = P[0] + P[1], b = P[0] - P[1], c = P[2] + P[3], d = P[2] - P[3];
  v[0] = a + c;
  v[1] = a - c;
  v[2] = b + d;
  v[3] = b - d;
}

}  // namespace fam
