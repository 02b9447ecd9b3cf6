// FP64 finalisation of one step's partial sums: totals in a fixed order, the
// observables record of the state the step started from, and the new renormalisation
// factor.  Runs on one block after the step's last pass (one block per instance in the
// batched ensemble).
#pragma once
#include "gp_device.hpp"

namespace gpdbec {

enum : int { FIN_IMAG = 0, FIN_REAL = 1, FIN_OBSERVE = 2, FIN_EKZ = 3 };
constexpr int kRecord = 10;  // norm, mu, energy, e_kin, e_pot, e_int, e_dd, rms x/y/z

struct FinArgs {
  const double* p_x;   // 2 per block: sum |dx psi|^2, sum |d1 psi|^2 (unscaled)
  int nb_x;
  const double* p_nl;  // 7 per block: n, V n, n^2, Phi n, x^2 n, a1^2 n, a2^2 n (scaled)
  int nb_nl;
  const double* p_col; // 2 per block: |u|^2, |d2 u|^2 (new state / unscaled input)
  int nb_col;
  double dV, h0, h1, h2, gc, gdd;
  int geom;            // 0: 3D, 1: XY, 2: XZ
  double* scale;
  double* ekz;         // pending z-kinetic energy of the stored state (3D)
  int* flags;
  double* ring;
  int* ring_pos;
  int ring_cap;
  double* obs;         // FIN_OBSERVE output record
  double* stage;       // two-stage reduction: kStageVals doubles per pre-reduced slice
  int nstage;          // slices (0: the finalize block reads the partials directly)
};

constexpr int kStageVals = 11;   // totals carried per slice (the v[] of finalize_block)
constexpr int kStageMax = 256;   // slices of the two-stage reduction (<= kThreads)

// Sums the partial arrays a block reads, blocks [lo, hi) of each, into v[11] (per
// thread; fixed order).  Each iteration first issues the loads of U blocks of every
// array, then adds them, so a small step's partials arrive in one memory round trip
// (U = 4; U = 1 inside a pass kernel, to stay within the pass's register budget).
template <int U = 4>
__device__ inline void fin_gather(const FinArgs& a, int mode, int slice, int nslice,
                                  double (&v)[11]) {
  const int tid = threadIdx.x;
  const bool xnl = mode != FIN_EKZ;
  const bool col = mode != FIN_OBSERVE || a.geom == 0;
  auto lo_of = [&](int nb) { return (int)((long long)nb * slice / nslice); };
  auto hi_of = [&](int nb) { return (int)((long long)nb * (slice + 1) / nslice); };
  const int lx = lo_of(a.nb_x), nx = xnl ? hi_of(a.nb_x) - lx : 0;
  const int ln = lo_of(a.nb_nl), nn = xnl ? hi_of(a.nb_nl) - ln : 0;
  const int lc = lo_of(a.nb_col), nc = col ? hi_of(a.nb_col) - lc : 0;
  const int span = nx > nn ? (nx > nc ? nx : nc) : (nn > nc ? nn : nc);
  for (int b0 = tid; b0 < span; b0 += U * kThreads) {
    double t[U][11];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = b0 + u * kThreads;
#pragma unroll
      for (int k = 0; k < 2; ++k) t[u][k] = b < nx ? a.p_x[2 * (size_t)(lx + b) + k] : 0.0;
#pragma unroll
      for (int k = 0; k < 7; ++k) t[u][2 + k] = b < nn ? a.p_nl[7 * (size_t)(ln + b) + k] : 0.0;
#pragma unroll
      for (int k = 0; k < 2; ++k) t[u][9 + k] = b < nc ? a.p_col[2 * (size_t)(lc + b) + k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int k = 0; k < 11; ++k) v[k] += t[u][k];
    }
  }
}

// First stage of the two-stage reduction: block g writes the totals of slice g.
template <int U = 4>
__device__ inline void prereduce_block(const FinArgs& a, int mode, int g) {
  __shared__ double red[11 * kWaves];
  double v[11];
#pragma unroll
  for (int k = 0; k < 11; ++k) v[k] = 0.0;
  fin_gather<U>(a, mode, g, a.nstage, v);
  block_sum<11>(v, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kStageVals; ++k) a.stage[g * kStageVals + k] = v[k];
  }
}

// All threads of one block must call this.
template <int U = 4>
__device__ inline void finalize_block(const FinArgs& a, int mode) {
  // no multiply-add contraction: the record rounds the same wherever this is inlined (its
  // own kernel, or folded into a pass kernel)
#pragma clang fp contract(off)
  __shared__ double red[11 * kWaves];
  const int tid = threadIdx.x;
  double v[11];
#pragma unroll
  for (int k = 0; k < 11; ++k) v[k] = 0.0;
  // the scalars thread 0 needs at the end are fetched before the gather
  double s = 1.0, ekz_in = 0.0;
  int pos = 0;
  if (tid == 0) {
    s = *a.scale;
    if (mode != FIN_EKZ && mode != FIN_OBSERVE && a.geom == 0) ekz_in = *a.ekz;
    if (mode != FIN_EKZ && mode != FIN_OBSERVE) pos = *a.ring_pos;
  }
  if (a.nstage > 0) {
    // one pre-reduced slice per thread (nstage <= kStageMax < kThreads), then the
    // fixed-order block sum
    if (tid < a.nstage) {
#pragma unroll
      for (int k = 0; k < kStageVals; ++k) v[k] = a.stage[tid * kStageVals + k];
    }
  } else {
    fin_gather<U>(a, mode, 0, 1, v);
  }
  block_sum<11>(v, red);
  if (tid != 0) return;
  const double s2 = s * s;
  if (mode == FIN_EKZ) {
    *a.ekz = 0.5 * s2 * v[10] / (a.h2 * a.h2) * a.dV;
    return;
  }
  const double dV = a.dV;
  double rec[kRecord];
  const double norm = v[2] * dV;
  double ekin = 0.5 * s2 * (v[0] / (a.h0 * a.h0) + v[1] / (a.h1 * a.h1)) * dV;
  if (a.geom == 0) {
    ekin += (mode == FIN_OBSERVE) ? 0.5 * s2 * v[10] / (a.h2 * a.h2) * dV : ekz_in;
  }
  const double epot = v[3] * dV;
  const double eint = 0.5 * a.gc * v[4] * dV;
  const double edd = 0.5 * a.gdd * v[5] * dV;
  rec[0] = norm;
  rec[1] = ekin + epot + 2.0 * eint + 2.0 * edd;
  rec[2] = ekin + epot + eint + edd;
  rec[3] = ekin;
  rec[4] = epot;
  rec[5] = eint;
  rec[6] = edd;
  const double inv = norm > 0.0 ? 1.0 / norm : 0.0;  // rms of a zero state: 0
  const double r0 = sqrt(v[6] * dV * inv), r1 = sqrt(v[7] * dV * inv), r2 = sqrt(v[8] * dV * inv);
  rec[7] = r0;
  rec[8] = (a.geom == 2) ? 0.0 : r1;
  rec[9] = (a.geom == 0) ? r2 : (a.geom == 2 ? r1 : 0.0);
  double* dst;
  if (mode == FIN_OBSERVE) {
    dst = a.obs;
  } else {
    dst = a.ring + (size_t)(pos % a.ring_cap) * kRecord;
    *a.ring_pos = pos + 1;
  }
#pragma unroll
  for (int k = 0; k < kRecord; ++k) dst[k] = rec[k];
  if (!isfinite(norm)) *a.flags |= 1;
  if (mode == FIN_OBSERVE) return;
  // new state: imaginary time renormalises, real time keeps the physical values
  const double nout = v[9] * dV;
  // imaginary time must renormalise (a zero state cannot be); real time only needs the
  // state to stay finite (zero is a solution)
  if (!isfinite(nout) || (mode == FIN_IMAG && !(nout > 0.0))) {
    *a.flags |= 1;
    *a.scale = 1.0;
    return;
  }
  const double sn = (mode == FIN_IMAG) ? 1.0 / sqrt(nout) : 1.0;
  *a.scale = sn;
  if (a.geom == 0) *a.ekz = 0.5 * sn * sn * v[10] / (a.h2 * a.h2) * dV;
}

}  // namespace gpdbec
