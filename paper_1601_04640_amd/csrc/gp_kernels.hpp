// Pass kernels of one split-step Crank-Nicolson step (templated on precision and on the
// line length of the axis they work along).
//
// Grid: (n2, n1, n0) with x = axis 0 fastest; 3D: n1 = ny, n2 = nz; 2D: n1 = ny (XY) or
// nz (XZ), n2 = 1.  psi is stored "lazily scaled": the physical wave function is
// scale * psi, with scale an FP64 device scalar (1 except after an imaginary-time step,
// whose renormalisation factor is applied by the next pass that reads psi).
//
// Spectrum of the density (after the x real-to-complex transform) is stored
// kx-plane-major, spec[(kx*n2 + k2)*n1 + k1], kx = 0..n0/2, so that the y lines are
// contiguous, the z lines are strided by n1, and one x line of the spectrum is a set
// of n0/2+1 contiguous runs over k1 (coalesced when a block owns several k1).
//
// Pass order of one 3D step (2D: r2c_x, conv_line, c2r_nl_cnx, cn_col(last), finalize):
//   r2c_x        n = s^2|psi|^2, x-R2C (two real lines packed per complex FFT);
//                kinetic x/y difference sums of the incoming state
//   fft_line     y FFT (forward)
//   conv_col     z FFT, multiply by U(k)/N, inverse z FFT
//   fft_line     y FFT (inverse)
//   c2r_nl_cnx   x-C2R -> Phi; norm/V/contact/dipolar/rms sums of the incoming state;
//                psi <- psi exp(-eps dt theta); CN sweep along x
//   cn_col       CN sweep along y
//   cn_col       CN sweep along z; norm and z-kinetic sums of the new state
//   finalize     FP64 totals, observables record, renormalisation factor
#pragma once
#include "gp_device.hpp"
#include "gp_finalize.hpp"

namespace gpdbec {

// Lines per block for passes along x, columns per block for strided passes.
template <typename T, int N>
struct Tiles {
  // x lines per block (even): 16, or 8 when a line of complex T exceeds 4 KiB (LDS)
  static constexpr int TJ = (N * 2 * (int)sizeof(T) > 4096) ? 8 : 16;
  static constexpr int PX = kThreads / TJ;          // lanes per x line in the CN solve
  static constexpr int TC = (sizeof(T) == 8 && N > 256) ? 8 : 16;  // columns per block
  static constexpr int PC = kThreads / TC;
  static constexpr int LB = (2048 / N) < 1 ? 1 : (2048 / N);        // contiguous lines
};

struct StepScalars {
  double dt;        // time step
  double gc;        // contact coupling (2D: includes 1/(sqrt(2 pi) d))
  double gdd;       // dipolar coupling
  double Ar;        // dt/(4 dx^2): A = Ar (imaginary) or i Ar (real time)
  double h0, h1, h2;  // spacings along axes 0, 1, 2
};

// MODE_ADJ: the adjoint sweep of a real-time step (A -> conj(A) = -i Ar).
enum : int { MODE_IMAG = 0, MODE_REAL = 1, MODE_OBSERVE = 2, MODE_PHI = 3, MODE_ADJ = 4 };

// Global-memory phases are statically unrolled over ITERS = ceil(elements/kThreads)
// so that every load of a thread is issued before the first one is consumed.
template <int TOTAL>
struct Iters {
  static constexpr int N = (TOTAL + kThreads - 1) / kThreads;
  __device__ static __forceinline__ bool valid(int u) { return TOTAL % kThreads == 0 || u < TOTAL; }
};

// ---------------------------------------------------------------- pass: r2c_x
// grid: ceil(n1/TJ) * n2 blocks.  partials[b*2 + {0,1}] = sum |dx psi|^2, sum |dy psi|^2
// of the stored psi (unscaled), the y difference reaching one line past the tile.
template <typename T, int N0>
__global__ __launch_bounds__(kThreads) void k_r2c_x(const cpx<T>* __restrict__ psi,
                                                    const double* __restrict__ scale,
                                                    cpx<T>* __restrict__ spec,
                                                    const cpx<T>* __restrict__ tw0,
                                                    double* __restrict__ partials, int n1, int n2) {
  using TL = Tiles<T, N0>;
  constexpr int TJ = TL::TJ, NP = TJ / 2, H = N0 / 2 + 1, LSZ = N0 + 1;
  using IT = Iters<TJ * N0>;
  __shared__ cpx<T> Z[NP * LSZ];
  __shared__ cpx<T> W[N0];
  __shared__ double red[2 * kWaves];
  const int tid = threadIdx.x;
  const int nt1 = (n1 + TJ - 1) / TJ;
  const int k2 = blockIdx.x / nt1;
  const int j0 = (blockIdx.x % nt1) * TJ;
  const cpx<T>* plane = psi + (size_t)k2 * n1 * N0;
  // all loads first: the point, its x neighbour and its y neighbour (mostly cache hits)
  cpx<T> a[IT::N], bx[IT::N], by[IT::N];
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    const int jl = u / N0, i = u % N0, j = j0 + jl;
    const cpx<T> z = {0, 0};
    const bool in = IT::valid(u) && j < n1;
    // clamped indices keep every load in bounds; at the last point of an axis the
    // neighbour is the point itself (zero difference), outside the grid all are zero
    const int jc = min(j, n1 - 1);
    const cpx<T>* line = plane + (size_t)jc * N0;
    const cpx<T> l0 = line[i];
    const cpx<T> l1 = line[min(i + 1, N0 - 1)];
    const cpx<T> l2 = plane[(size_t)min(jc + 1, n1 - 1) * N0 + i];
    a[it] = in ? l0 : z;
    bx[it] = in ? l1 : z;
    by[it] = in ? l2 : z;
  }
  for (int i = tid; i < N0; i += kThreads) W[i] = tw0[i];
  const double s = *scale;
  const T s2 = (T)(s * s);
  double sums[2] = {0.0, 0.0};
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    if (!IT::valid(u)) continue;
    const int jl = u / N0, i = u % N0;
    sums[0] += absdiff2_d(bx[it], a[it]);
    sums[1] += absdiff2_d(by[it], a[it]);
    const T nv = s2 * (a[it].re * a[it].re + a[it].im * a[it].im);
    cpx<T>& zc = Z[(jl >> 1) * LSZ + i];
    if (jl & 1) zc.im = nv;
    else zc.re = nv;
  }
  __syncthreads();
  LdsFFT<T, N0, NP, LSZ, 1, false>::template run<false>(Z, W);
  // untangle the two real lines of each pair and store kx = 0..N0/2
  using IH = Iters<H * NP>;
#pragma unroll
  for (int it = 0; it < IH::N; ++it) {
    const int u = tid + it * kThreads;
    if (!IH::valid(u)) continue;
    const int p = u % NP, kx = u / NP;
    const int j = j0 + 2 * p;
    if (j >= n1) continue;
    const cpx<T> zk = Z[p * LSZ + kx];
    const cpx<T> zm = Z[p * LSZ + ((N0 - kx) % N0)];
    const T hf = (T)0.5;
    const cpx<T> ra = {hf * (zk.re + zm.re), hf * (zk.im - zm.im)};
    const cpx<T> rb = {hf * (zk.im + zm.im), hf * (zm.re - zk.re)};
    cpx<T>* o = spec + ((size_t)kx * n2 + k2) * n1 + j;
    o[0] = ra;
    o[1] = rb;  // n1 is even, so line j+1 exists whenever line j does
  }
  block_sum<2>(sums, red);
  if (tid == 0) {
    partials[blockIdx.x * 2 + 0] = sums[0];
    partials[blockIdx.x * 2 + 1] = sums[1];
  }
}

// Loads LB contiguous lines of length N into LDS rows of stride N + 1.
template <typename T, int N, int LB>
__device__ __forceinline__ void load_lines(cpx<T>* B, const cpx<T>* __restrict__ data, int l0,
                                           int nlines) {
  using IT = Iters<LB * N>;
  cpx<T> v[IT::N];
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = threadIdx.x + it * kThreads;
    const int l = u / N, i = u % N;
    v[it] = (IT::valid(u) && l0 + l < nlines) ? data[(size_t)(l0 + l) * N + i] : cpx<T>{0, 0};
  }
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = threadIdx.x + it * kThreads;
    if (IT::valid(u)) B[(u / N) * (N + 1) + u % N] = v[it];
  }
}

template <typename T, int N, int LB>
__device__ __forceinline__ void store_lines(const cpx<T>* B, cpx<T>* __restrict__ data, int l0,
                                            int nlines) {
  using IT = Iters<LB * N>;
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = threadIdx.x + it * kThreads;
    const int l = u / N, i = u % N;
    if (IT::valid(u) && l0 + l < nlines) data[(size_t)(l0 + l) * N + i] = B[l * (N + 1) + i];
  }
}

// -------------------------------------------------------------- pass: fft_line
// FFT of contiguous lines of length N (count nlines), LB lines per block.
template <typename T, int N, bool INV>
__global__ __launch_bounds__(kThreads) void k_fft_line(cpx<T>* __restrict__ data,
                                                       const cpx<T>* __restrict__ tw, int nlines) {
  constexpr int LB = Tiles<T, N>::LB, LSZ = N + 1;
  __shared__ cpx<T> B[LB * LSZ];
  __shared__ cpx<T> W[N];
  const int l0 = blockIdx.x * LB;
  load_lines<T, N, LB>(B, data, l0, nlines);
  for (int i = threadIdx.x; i < N; i += kThreads) W[i] = tw[i];
  __syncthreads();
  LdsFFT<T, N, LB, LSZ, 1, false>::template run<INV>(B, W);
  store_lines<T, N, LB>(B, data, l0, nlines);
}

// FFT -> multiply by the kernel table -> inverse FFT of contiguous lines (2D: y lines).
template <typename T, int N>
__global__ __launch_bounds__(kThreads) void k_conv_line(cpx<T>* __restrict__ data,
                                                        const T* __restrict__ ktab,
                                                        const cpx<T>* __restrict__ tw, int nlines) {
  constexpr int LB = Tiles<T, N>::LB, LSZ = N + 1;
  using IT = Iters<LB * N>;
  __shared__ cpx<T> B[LB * LSZ];
  __shared__ cpx<T> W[N];
  const int tid = threadIdx.x;
  const int l0 = blockIdx.x * LB;
  load_lines<T, N, LB>(B, data, l0, nlines);
  T kv[IT::N];  // kernel values: loaded now, used after the forward FFT
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    const int l = u / N, i = u % N;
    kv[it] = (IT::valid(u) && l0 + l < nlines) ? ktab[(size_t)(l0 + l) * N + i] : (T)0;
  }
  for (int i = tid; i < N; i += kThreads) W[i] = tw[i];
  __syncthreads();
  LdsFFT<T, N, LB, LSZ, 1, false>::template run<false>(B, W);
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    if (IT::valid(u)) {
      cpx<T>& e = B[(u / N) * LSZ + u % N];
      e = scl(e, kv[it]);
    }
  }
  __syncthreads();
  LdsFFT<T, N, LB, LSZ, 1, false>::template run<true>(B, W);
  store_lines<T, N, LB>(B, data, l0, nlines);
}

// --------------------------------------------------------------- pass: conv_col
// 3D z pass on the spectrum: lines along k2 (stride n1) inside each kx plane; a block
// owns TC consecutive k1 of one kx plane.  grid: ceil(n1/TC) * H blocks.
template <typename T, int N2>
__global__ __launch_bounds__(kThreads) void k_conv_col(cpx<T>* __restrict__ spec,
                                                       const T* __restrict__ ktab,
                                                       const cpx<T>* __restrict__ tw2, int n1) {
  constexpr int TC = Tiles<T, N2>::TC, RS = TC + 1;
  using IT = Iters<N2 * TC>;
  __shared__ cpx<T> B[N2 * RS];
  __shared__ cpx<T> W[N2];
  const int tid = threadIdx.x;
  const int nt = (n1 + TC - 1) / TC;
  const int kx = blockIdx.x / nt;
  const int c0 = (blockIdx.x % nt) * TC;
  const size_t plane = (size_t)kx * N2 * n1;
  cpx<T> v[IT::N];
  T kv[IT::N];
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    const int c = u % TC, r = u / TC;
    const bool in = IT::valid(u) && c0 + c < n1;
    const size_t g = plane + (size_t)r * n1 + c0 + c;
    v[it] = in ? spec[g] : cpx<T>{0, 0};
    kv[it] = in ? ktab[g] : (T)0;
  }
  for (int i = tid; i < N2; i += kThreads) W[i] = tw2[i];
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    if (IT::valid(u)) B[(u / TC) * RS + u % TC] = v[it];
  }
  __syncthreads();
  LdsFFT<T, N2, TC, 1, RS, true>::template run<false>(B, W);
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    if (IT::valid(u)) {
      cpx<T>& e = B[(u / TC) * RS + u % TC];
      e = scl(e, kv[it]);
    }
  }
  __syncthreads();
  LdsFFT<T, N2, TC, 1, RS, true>::template run<true>(B, W);
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    const int c = u % TC, r = u / TC;
    if (IT::valid(u) && c0 + c < n1) spec[plane + (size_t)r * n1 + c0 + c] = B[r * RS + c];
  }
}

// ------------------------------------------------------------ pass: c2r_nl_cnx
// grid: ceil(n1/TJ) * n2 blocks.  MODE_IMAG / MODE_REAL: full step pass (writes psi).
// MODE_OBSERVE: sums only.  MODE_PHI: writes Phi (without g_dd) to phi_out.
// partials[b*7 + ...] = sum n, sum V n, sum n^2, sum Phi n, sum x^2 n, sum y^2 n, sum z^2 n
// of the incoming (scaled) state; axis coordinates (idx - n/2) h.
template <typename T, int N0, int MODE>
__global__ __launch_bounds__(kThreads) void k_c2r_nl_cnx(
    cpx<T>* __restrict__ psi, const T* __restrict__ V, const double* __restrict__ scale,
    const cpx<T>* __restrict__ spec, const cpx<T>* __restrict__ tw0,
    const cpx<T>* __restrict__ cnm, const cpx<T>* __restrict__ cng, StepScalars sc,
    double* __restrict__ partials, T* __restrict__ phi_out, int n1, int n2) {
  using TL = Tiles<T, N0>;
  constexpr int TJ = TL::TJ, NP = TJ / 2, H = N0 / 2 + 1, LSZ = N0 + 1;
  constexpr int PX = TL::PX, SX = (N0 + PX - 1) / PX, LSP = N0 + (N0 + SX - 1) / SX;
  constexpr bool STEP = (MODE == MODE_IMAG || MODE == MODE_REAL);
  constexpr bool NEEDPSI = (MODE != MODE_PHI);
  using IT = Iters<TJ * N0>;
  using IH = Iters<H * NP>;
  __shared__ cpx<T> Z[NP * LSZ];
  __shared__ cpx<T> PS[STEP ? TJ * LSP : 1];
  __shared__ cpx<T> W[N0];
  __shared__ cpx<T> MT[STEP ? N0 : 1], GT[STEP ? N0 : 1];
  __shared__ double red[7 * kWaves];
  const int tid = threadIdx.x;
  const int nt1 = (n1 + TJ - 1) / TJ;
  const int k2 = blockIdx.x / nt1;
  const int j0 = (blockIdx.x % nt1) * TJ;
  const size_t pbase = ((size_t)k2 * n1 + j0) * N0;  // first point of the tile
  // issue every global load of the block up front: spectrum pairs, psi and V tiles
  cpx<T> sa[IH::N], sb[IH::N];
#pragma unroll
  for (int it = 0; it < IH::N; ++it) {
    const int u = tid + it * kThreads;
    const int p = u % NP, kx = u / NP;
    const int j = j0 + 2 * p;
    const bool in = IH::valid(u) && j < n1;
    const cpx<T>* o = spec + ((size_t)kx * n2 + k2) * n1 + j;
    sa[it] = in ? o[0] : cpx<T>{0, 0};
    sb[it] = in ? o[1] : cpx<T>{0, 0};
  }
  cpx<T> pv[NEEDPSI ? IT::N : 1];
  T vv[NEEDPSI ? IT::N : 1];
  if constexpr (NEEDPSI) {
#pragma unroll
    for (int it = 0; it < IT::N; ++it) {
      const int u = tid + it * kThreads;
      const bool in = IT::valid(u) && j0 + u / N0 < n1;
      pv[it] = in ? psi[pbase + u] : cpx<T>{0, 0};
      vv[it] = in ? V[pbase + u] : (T)0;
    }
  }
  for (int i = tid; i < N0; i += kThreads) {
    W[i] = tw0[i];
    if constexpr (STEP) {
      MT[i] = cnm[i];
      GT[i] = cng[i];
    }
  }
  // the Hermitian half spectrum of each line pair -> a full complex line
#pragma unroll
  for (int it = 0; it < IH::N; ++it) {
    const int u = tid + it * kThreads;
    if (!IH::valid(u)) continue;
    const int p = u % NP, kx = u / NP;
    const cpx<T> a = sa[it], b = sb[it];
    cpx<T>* z = Z + p * LSZ;
    if (kx == 0 || kx == N0 / 2) {
      z[kx] = cpx<T>{a.re, b.re};
    } else {
      z[kx] = cpx<T>{a.re - b.im, a.im + b.re};
      z[N0 - kx] = cpx<T>{a.re + b.im, b.re - a.im};
    }
  }
  __syncthreads();
  LdsFFT<T, N0, NP, LSZ, 1, false>::template run<true>(Z, W);

  if constexpr (MODE == MODE_PHI) {
#pragma unroll
    for (int it = 0; it < IT::N; ++it) {
      const int u = tid + it * kThreads;
      const int jl = u / N0, i = u % N0;
      if (IT::valid(u) && j0 + jl < n1)
        phi_out[pbase + u] = reinterpret_cast<const T*>(&Z[(jl >> 1) * LSZ + i])[jl & 1];
    }
    return;
  } else {
    double sums[7] = {0, 0, 0, 0, 0, 0, 0};
    const T ts = (T)(*scale);
    const double h0 = sc.h0, h1 = sc.h1, h2 = sc.h2;
    const double zc = (k2 - n2 / 2) * h2;
#pragma unroll
    for (int it = 0; it < IT::N; ++it) {
      const int u = tid + it * kThreads;
      if (!IT::valid(u)) continue;
      const int jl = u / N0, i = u % N0;
      const int j = j0 + jl;
      if (j >= n1) {
        if constexpr (STEP) PS[jl * LSP + cpad<SX>(i)] = cpx<T>{0, 0};
        continue;
      }
      const T phi = reinterpret_cast<const T*>(&Z[(jl >> 1) * LSZ + i])[jl & 1];
      const cpx<T> p = scl(pv[it], ts);
      const T v = vv[it];
      const double nd = abs2_d(p);
      const double xc = (i - N0 / 2) * h0, yc = (j - n1 / 2) * h1;
      sums[0] += nd;
      sums[1] += (double)v * nd;
      sums[2] += nd * nd;
      sums[3] += (double)phi * nd;
      sums[4] += xc * xc * nd;
      sums[5] += yc * yc * nd;
      sums[6] += zc * zc * nd;
      if constexpr (STEP) {
        const T n = p.re * p.re + p.im * p.im;
        const T th = (T)sc.dt * (v + (T)sc.gc * n + (T)sc.gdd * phi);
        cpx<T> f;
        if constexpr (MODE == MODE_IMAG) {
          f = cpx<T>{exp(-th), (T)0};
        } else {
          f = cpx<T>{cos(th), -sin(th)};
        }
        PS[jl * LSP + cpad<SX>(i)] = p * f;
      }
    }
    block_sum<7>(sums, red);
    if (tid == 0) {
#pragma unroll
      for (int k = 0; k < 7; ++k) partials[blockIdx.x * 7 + k] = sums[k];
    }
    if constexpr (STEP) {
      __syncthreads();
      const cpx<T> A = (MODE == MODE_IMAG) ? cpx<T>{(T)sc.Ar, 0} : cpx<T>{0, (T)sc.Ar};
      const cpx<T> B = (MODE == MODE_IMAG) ? cpx<T>{(T)(1.0 - 2.0 * sc.Ar), 0}
                                           : cpx<T>{(T)1, (T)(-2.0 * sc.Ar)};
      cn_solve_lines<T, N0, TJ, LSP, 1, PX>(PS, MT, GT, A, B);
#pragma unroll
      for (int it = 0; it < IT::N; ++it) {
        const int u = tid + it * kThreads;
        const int jl = u / N0, i = u % N0;
        if (IT::valid(u) && j0 + jl < n1) psi[pbase + u] = PS[jl * LSP + cpad<SX>(i)];
      }
    }
  }
}

// ----------------------------------------------------------------- pass: cn_col
// CN sweep along a strided axis: lines of length N with element stride `estride`;
// a block owns TC consecutive x columns (x0..x0+TC-1) of one "outer" index.
//   y sweep (3D/2D): estride = n0, outer = k2 (n_outer = n2), base = k2*n1*n0
//   z sweep (3D):    estride = n0*n1, outer = k1 (n_outer = n1), base = k1*n0
// SUMS: also partials[b*2+{0,1}] = sum |u|^2, sum |u_{i+1}-u_i|^2 along the line of the
// result (MODE_OBSERVE: of the stored input, nothing written; sums unscaled), and the
// last block to finish runs the step's FP64 finalisation (fin_mode, FinArgs).
// grid: ceil(n0/TC) * n_outer blocks.
template <typename T, int N, int MODE, bool SUMS>
__global__ __launch_bounds__(kThreads) void k_cn_col(cpx<T>* __restrict__ psi,
                                                     const cpx<T>* __restrict__ cnm,
                                                     const cpx<T>* __restrict__ cng,
                                                     double Ar, double* __restrict__ partials,
                                                     int n0, size_t estride, size_t ostride,
                                                     unsigned* counter, FinArgs fa,
                                                     int fin_mode) {
  using TL = Tiles<T, N>;
  constexpr int TC = TL::TC, PC = TL::PC, SC = (N + PC - 1) / PC, RS = TC + 1;
  constexpr int NR = N + (N + SC - 1) / SC;  // padded rows
  constexpr bool SOLVE = (MODE == MODE_IMAG || MODE == MODE_REAL || MODE == MODE_ADJ);
  using IT = Iters<N * TC>;
  __shared__ cpx<T> B[NR * RS];
  __shared__ cpx<T> MT[SOLVE ? N : 1], GT[SOLVE ? N : 1];
  __shared__ double red[2 * kWaves];
  const int tid = threadIdx.x;
  const int nt = (n0 + TC - 1) / TC;
  const int outer = blockIdx.x / nt;
  const int x0 = (blockIdx.x % nt) * TC;
  cpx<T>* base = psi + (size_t)outer * ostride + x0;
  cpx<T> v[IT::N];
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    const int c = u % TC, r = u / TC;
    v[it] = (IT::valid(u) && x0 + c < n0) ? base[(size_t)r * estride + c] : cpx<T>{0, 0};
  }
  if constexpr (SOLVE) {
    for (int i = tid; i < N; i += kThreads) {
      MT[i] = cnm[i];
      GT[i] = cng[i];
    }
  }
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    if (IT::valid(u)) B[cpad<SC>(u / TC) * RS + u % TC] = v[it];
  }
  __syncthreads();
  if constexpr (SOLVE) {
    // A = Ar (imaginary time), i Ar (real time), -i Ar (adjoint); Bc = 1 - 2A
    const cpx<T> A = (MODE == MODE_IMAG) ? cpx<T>{(T)Ar, 0}
                     : (MODE == MODE_REAL) ? cpx<T>{0, (T)Ar} : cpx<T>{0, (T)(-Ar)};
    const cpx<T> Bc = (MODE == MODE_IMAG) ? cpx<T>{(T)(1.0 - 2.0 * Ar), 0}
                      : (MODE == MODE_REAL) ? cpx<T>{(T)1, (T)(-2.0 * Ar)}
                                            : cpx<T>{(T)1, (T)(2.0 * Ar)};
    cn_solve_lines<T, N, TC, 1, RS, PC>(B, MT, GT, A, Bc);
  }
  double sums[2] = {0.0, 0.0};
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    const int c = u % TC, r = u / TC;
    if (!IT::valid(u) || x0 + c >= n0) continue;
    const cpx<T> val = B[cpad<SC>(r) * RS + c];
    if constexpr (SOLVE) base[(size_t)r * estride + c] = val;
    if constexpr (SUMS) {
      sums[0] += abs2_d(val);
      if (r + 1 < N) sums[1] += absdiff2_d(B[cpad<SC>(r + 1) * RS + c], val);
    }
  }
  if constexpr (SUMS) {
    block_sum<2>(sums, red);
    publish_and_finalize(sums, partials, counter, fa, fin_mode);
  }
}

}  // namespace gpdbec

// ========================================================= adjoint (real time)
// Backpropagation through one real-time step (costate lambda = dL/d conj(psi)):
//   lambda_a = C_x(-dt) C_y(-dt) C_z(-dt) lambda      (adjoint of each CN factor)
//   mu = exp(+i dt theta) lambda_a,  theta = V + g_c n + g_dd Phi  (of psi_n)
//   s  = 2 dt Im(conj(mu) psi_n);   dL/dV += s;  sums s n, s Phi -> dL/dg_c, dL/dg_dd
//   lambda_n = mu + (g_c s + g_dd K s) psi_n,  K s = F^-1[U F[s]]
namespace gpdbec {

// Real-to-complex x pass of a real field f (the adjoint's second convolution input).
// grid: ceil(n1/TJ) * n2 blocks; writes the same kx-plane-major half spectrum.
template <typename T, int N0>
__global__ __launch_bounds__(kThreads) void k_r2c_real(const T* __restrict__ f,
                                                       cpx<T>* __restrict__ spec,
                                                       const cpx<T>* __restrict__ tw0, int n1,
                                                       int n2) {
  using TL = Tiles<T, N0>;
  constexpr int TJ = TL::TJ, NP = TJ / 2, H = N0 / 2 + 1, LSZ = N0 + 1;
  using IT = Iters<TJ * N0>;
  using IH = Iters<H * NP>;
  __shared__ cpx<T> Z[NP * LSZ];
  __shared__ cpx<T> W[N0];
  const int tid = threadIdx.x;
  const int nt1 = (n1 + TJ - 1) / TJ;
  const int k2 = blockIdx.x / nt1;
  const int j0 = (blockIdx.x % nt1) * TJ;
  const size_t pbase = ((size_t)k2 * n1 + j0) * N0;
  T fv[IT::N];
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    fv[it] = (IT::valid(u) && j0 + u / N0 < n1) ? f[pbase + u] : (T)0;
  }
  for (int i = tid; i < N0; i += kThreads) W[i] = tw0[i];
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    if (!IT::valid(u)) continue;
    const int jl = u / N0, i = u % N0;
    cpx<T>& zc = Z[(jl >> 1) * LSZ + i];
    if (jl & 1) zc.im = fv[it];
    else zc.re = fv[it];
  }
  __syncthreads();
  LdsFFT<T, N0, NP, LSZ, 1, false>::template run<false>(Z, W);
#pragma unroll
  for (int it = 0; it < IH::N; ++it) {
    const int u = tid + it * kThreads;
    if (!IH::valid(u)) continue;
    const int p = u % NP, kx = u / NP;
    const int j = j0 + 2 * p;
    if (j >= n1) continue;
    const cpx<T> zk = Z[p * LSZ + kx];
    const cpx<T> zm = Z[p * LSZ + ((N0 - kx) % N0)];
    const T hf = (T)0.5;
    cpx<T>* o = spec + ((size_t)kx * n2 + k2) * n1 + j;
    o[0] = cpx<T>{hf * (zk.re + zm.re), hf * (zk.im - zm.im)};
    o[1] = cpx<T>{hf * (zk.im + zm.im), hf * (zm.re - zk.re)};
  }
}

// Gathers the Hermitian half spectrum of the tile's line pairs into full complex lines
// (issued loads first) and runs the inverse x FFT: afterwards line jl of the tile holds
// the real field in component (jl & 1) of Z[(jl >> 1) * (N0 + 1) + i].
template <typename T, int N0, int NP>
__device__ __forceinline__ void c2r_tile(cpx<T>* Z, const cpx<T>* W,
                                         const cpx<T>* __restrict__ spec, int j0, int k2,
                                         int n1, int n2, const cpx<T> (&sa)[Iters<(N0 / 2 + 1) * NP>::N],
                                         const cpx<T> (&sb)[Iters<(N0 / 2 + 1) * NP>::N]) {
  constexpr int LSZ = N0 + 1, H = N0 / 2 + 1;
  using IH = Iters<H * NP>;
#pragma unroll
  for (int it = 0; it < IH::N; ++it) {
    const int u = threadIdx.x + it * kThreads;
    if (!IH::valid(u)) continue;
    const int p = u % NP, kx = u / NP;
    const cpx<T> a = sa[it], b = sb[it];
    cpx<T>* z = Z + p * LSZ;
    if (kx == 0 || kx == N0 / 2) {
      z[kx] = cpx<T>{a.re, b.re};
    } else {
      z[kx] = cpx<T>{a.re - b.im, a.im + b.re};
      z[N0 - kx] = cpx<T>{a.re + b.im, b.re - a.im};
    }
  }
  __syncthreads();
  LdsFFT<T, N0, NP, LSZ, 1, false>::template run<true>(Z, W);
}

template <typename T, int N0, int NP>
__device__ __forceinline__ void load_spec_pairs(const cpx<T>* __restrict__ spec, int j0, int k2,
                                                int n1, int n2,
                                                cpx<T> (&sa)[Iters<(N0 / 2 + 1) * NP>::N],
                                                cpx<T> (&sb)[Iters<(N0 / 2 + 1) * NP>::N]) {
  using IH = Iters<(N0 / 2 + 1) * NP>;
#pragma unroll
  for (int it = 0; it < IH::N; ++it) {
    const int u = threadIdx.x + it * kThreads;
    const int p = u % NP, kx = u / NP;
    const int j = j0 + 2 * p;
    const bool in = IH::valid(u) && j < n1;
    const cpx<T>* o = spec + ((size_t)kx * n2 + k2) * n1 + j;
    sa[it] = in ? o[0] : cpx<T>{0, 0};
    sb[it] = in ? o[1] : cpx<T>{0, 0};
  }
}

// Adjoint x pass: lambda_a = C_x(-dt) lambda (conj tables), Phi of psi_n from the
// spectrum, mu = exp(i dt theta) lambda_a -> lam, s -> sfield, gradV += s (FP64),
// partials[b*2 + {0,1}] = sum s n, sum s Phi.  grid: ceil(n1/TJ) * n2 blocks.
template <typename T, int N0>
__global__ __launch_bounds__(kThreads) void k_adj_x(
    cpx<T>* __restrict__ lam, const cpx<T>* __restrict__ psin, const T* __restrict__ V,
    const cpx<T>* __restrict__ spec, const cpx<T>* __restrict__ tw0,
    const cpx<T>* __restrict__ cnm, const cpx<T>* __restrict__ cng, StepScalars sc,
    T* __restrict__ sfield, double* __restrict__ gradV, double* __restrict__ partials, int n1,
    int n2) {
  using TL = Tiles<T, N0>;
  constexpr int TJ = TL::TJ, NP = TJ / 2, LSZ = N0 + 1;
  constexpr int PX = TL::PX, SX = (N0 + PX - 1) / PX, LSP = N0 + (N0 + SX - 1) / SX;
  using IT = Iters<TJ * N0>;
  using IH = Iters<(N0 / 2 + 1) * NP>;
  __shared__ cpx<T> Z[NP * LSZ];
  __shared__ cpx<T> PS[TJ * LSP];
  __shared__ cpx<T> W[N0];
  __shared__ cpx<T> MT[N0], GT[N0];
  __shared__ double red[2 * kWaves];
  const int tid = threadIdx.x;
  const int nt1 = (n1 + TJ - 1) / TJ;
  const int k2 = blockIdx.x / nt1;
  const int j0 = (blockIdx.x % nt1) * TJ;
  const size_t pbase = ((size_t)k2 * n1 + j0) * N0;
  cpx<T> sa[IH::N], sb[IH::N];
  load_spec_pairs<T, N0, NP>(spec, j0, k2, n1, n2, sa, sb);
  cpx<T> lv[IT::N], pv[IT::N];
  T vv[IT::N];
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    const bool in = IT::valid(u) && j0 + u / N0 < n1;
    lv[it] = in ? lam[pbase + u] : cpx<T>{0, 0};
    pv[it] = in ? psin[pbase + u] : cpx<T>{0, 0};
    vv[it] = in ? V[pbase + u] : (T)0;
  }
  for (int i = tid; i < N0; i += kThreads) {
    W[i] = tw0[i];
    MT[i] = cnm[i];
    GT[i] = cng[i];
  }
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    if (IT::valid(u)) PS[(u / N0) * LSP + cpad<SX>(u % N0)] = lv[it];
  }
  c2r_tile<T, N0, NP>(Z, W, spec, j0, k2, n1, n2, sa, sb);  // ends with a barrier
  const cpx<T> A = {0, (T)(-sc.Ar)};
  const cpx<T> B = {(T)1, (T)(2.0 * sc.Ar)};
  cn_solve_lines<T, N0, TJ, LSP, 1, PX>(PS, MT, GT, A, B);
  double sums[2] = {0.0, 0.0};
  const T dt = (T)sc.dt;
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    if (!IT::valid(u)) continue;
    const int jl = u / N0, i = u % N0;
    if (j0 + jl >= n1) continue;
    const T phi = (jl & 1) ? Z[(jl >> 1) * LSZ + i].im : Z[(jl >> 1) * LSZ + i].re;
    const cpx<T> p = pv[it];
    const T n = p.re * p.re + p.im * p.im;
    const T th = dt * (vv[it] + (T)sc.gc * n + (T)sc.gdd * phi);
    const cpx<T> la = PS[jl * LSP + cpad<SX>(i)];
    const cpx<T> mu = la * cpx<T>{cos(th), sin(th)};
    const T s = (T)2 * dt * (mu.re * p.im - mu.im * p.re);
    lam[pbase + u] = mu;
    sfield[pbase + u] = s;
    gradV[pbase + u] += (double)s;
    sums[0] += (double)s * (double)n;
    sums[1] += (double)s * (double)phi;
  }
  block_sum<2>(sums, red);
  if (tid == 0) {
    partials[blockIdx.x * 2 + 0] = sums[0];
    partials[blockIdx.x * 2 + 1] = sums[1];
  }
}

// Adjoint closing x pass: K s from the spectrum; lambda = mu + (g_c s + g_dd K s) psi_n.
template <typename T, int N0>
__global__ __launch_bounds__(kThreads) void k_adj_fin(cpx<T>* __restrict__ lam,
                                                      const cpx<T>* __restrict__ psin,
                                                      const T* __restrict__ sfield,
                                                      const cpx<T>* __restrict__ spec,
                                                      const cpx<T>* __restrict__ tw0,
                                                      StepScalars sc, int n1, int n2) {
  using TL = Tiles<T, N0>;
  constexpr int TJ = TL::TJ, NP = TJ / 2, LSZ = N0 + 1;
  using IT = Iters<TJ * N0>;
  using IH = Iters<(N0 / 2 + 1) * NP>;
  __shared__ cpx<T> Z[NP * LSZ];
  __shared__ cpx<T> W[N0];
  const int tid = threadIdx.x;
  const int nt1 = (n1 + TJ - 1) / TJ;
  const int k2 = blockIdx.x / nt1;
  const int j0 = (blockIdx.x % nt1) * TJ;
  const size_t pbase = ((size_t)k2 * n1 + j0) * N0;
  cpx<T> sa[IH::N], sb[IH::N];
  load_spec_pairs<T, N0, NP>(spec, j0, k2, n1, n2, sa, sb);
  cpx<T> mv[IT::N], pv[IT::N];
  T sv[IT::N];
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    const bool in = IT::valid(u) && j0 + u / N0 < n1;
    mv[it] = in ? lam[pbase + u] : cpx<T>{0, 0};
    pv[it] = in ? psin[pbase + u] : cpx<T>{0, 0};
    sv[it] = in ? sfield[pbase + u] : (T)0;
  }
  for (int i = tid; i < N0; i += kThreads) W[i] = tw0[i];
  c2r_tile<T, N0, NP>(Z, W, spec, j0, k2, n1, n2, sa, sb);
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    if (!IT::valid(u)) continue;
    const int jl = u / N0, i = u % N0;
    if (j0 + jl >= n1) continue;
    const T ks = (jl & 1) ? Z[(jl >> 1) * LSZ + i].im : Z[(jl >> 1) * LSZ + i].re;
    const T w = (T)sc.gc * sv[it] + (T)sc.gdd * ks;
    lam[pbase + u] = mv[it] + scl(pv[it], w);
  }
}

}  // namespace gpdbec
