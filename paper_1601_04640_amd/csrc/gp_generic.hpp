// Pass kernels for axis lengths with no compile-time specialisation: any even length
// whose prime factors are at most 31.  The line length, the FFT's radix plan and the
// tile shapes are kernel arguments, so one set of kernels serves every such grid.
//
// The step is the same split-step as the specialised passes ("Solution method": the
// dipolar term by the convolution theorem, then the Crank-Nicolson sweeps; "Summary of
// revisions": calcpsidd2, calcnu, calclux, calcluy, calcluz, calcnorm), in more and
// simpler launches:
//   kg_r2c_x        n = |psi|^2 of the stored state, x real-to-complex FFT (two real
//                   lines per complex line), x / axis-1 difference sums
//   kg_lines        line FFTs of the half spectrum (forward, inverse, or forward + U(k)
//                   product + inverse, the convolution along the last axis)
//   kg_c2r_x        x complex-to-real FFT -> Phi (a real grid)
//   kg_nl_transpose psi <- scale psi exp(-eps dt (V + g_c n + g_dd Phi)) with the
//                   norm / potential / contact / dipolar / rms sums, written x-major
//                   (transposed), so that the x lines become columns
//   kg_cn_cols      Crank-Nicolson sweep of columns (one thread per line, Thomas
//                   recurrences through a scratch array), optionally with the norm and
//                   difference sums of the new state
//   kg_transpose    back to the psi layout
// The partial sums have the meaning the FP64 finalisation reads (gp_finalize.hpp).
#pragma once
#include "gp_device.hpp"
#include "gp_kernels.hpp"  // pass modes

namespace gpdbec {

constexpr int kGenMaxStages = 24;
// The LDS-FFT kernels run up to 1024 threads per block (launched with as many 64-lane
// waves as their lines need), each holding a few values per FFT stage.
constexpr int kGenThreads = 1024;

// Sum over the block's waves (any multiple of 64 threads up to kGenThreads) in a fixed
// order; the total is valid in thread 0.  red: NV * 16 doubles of LDS.
template <int NV>
__device__ __forceinline__ void gblock_sum(double (&v)[NV], double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum_to_last(v[k]);
  if (lane == 63) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k * 16 + wave] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double acc = red[k * 16];
      for (int w = 1; w < nw; ++w) acc += red[k * 16 + w];
      v[k] = acc;
    }
  }
}
constexpr int kGenMaxPrime = 31;

// Radices of an N-point FFT: factors 8, 4, 2, then the odd primes up to 31.
struct GPlan {
  int n;
  int nst;
  int rad[kGenMaxStages];
};

__host__ __device__ inline bool gen_plan(int n, GPlan* p) {
  p->n = n;
  p->nst = 0;
  int m = n;
  const int order[] = {8, 4, 2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31};
  for (int r : order) {
    while (m % r == 0) {
      if (p->nst >= kGenMaxStages) return false;
      p->rad[p->nst++] = r;
      m /= r;
    }
  }
  return m == 1;
}

// ---------------------------------------------------------------- radix butterflies
// Odd prime P: X[r] = sum_s x[s] W_P^(r s), with w[k] = W_P^k (conjugated for INV).
template <typename T, int P>
__device__ __forceinline__ void dft_prime(cpx<T>* x, const cpx<T>* w) {
  cpx<T> y[P];
#pragma unroll
  for (int r = 0; r < P; ++r) {
    cpx<T> acc = x[0];
#pragma unroll
    for (int s = 1; s < P; ++s) acc = acc + x[s] * w[(r * s) % P];
    y[r] = acc;
  }
#pragma unroll
  for (int r = 0; r < P; ++r) x[r] = y[r];
}

template <typename T, bool INV>
__device__ __forceinline__ cpx<T> twid(const cpx<T>* __restrict__ tw, long long k) {
  const cpx<T> w = tw[k];
  return INV ? cpx<T>{w.re, -w.im} : w;
}

// One Stockham stage of radix R over NL lines of length N held in LDS (line l at
// buf[l*N]).  Butterfly i of a line (i < N/R) reads x[i + r N/R], applies the twiddles
// W_(L R)^(r k), k = i mod L (L: product of the earlier radices), and writes
// y[(i/L) L R + k + r L].  Every butterfly's inputs are read into registers before any
// output is written (all threads, across a barrier), so the stage runs in place.
// Each thread holds at most QM butterflies: NL*N/R <= QM*blockDim.
template <typename T, int R, bool INV, int QM>
__device__ __forceinline__ void gstage(cpx<T>* buf, int NL, int N, int L,
                                       const cpx<T>* __restrict__ tw) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int NB = N / R;
  const int tot = NL * NB;
  const int tstride = N / (L * R);
  cpx<T> w[R];
  if constexpr (R == 7 || R > 8) {
#pragma unroll
    for (int k = 0; k < R; ++k) w[k] = twid<T, INV>(tw, (long long)k * (N / R));
  }
  cpx<T> v[QM][R];
#pragma unroll
  for (int q = 0; q < QM; ++q) {
    const int b = tid + q * nt;
    if (b < tot) {
      const int line = b / NB, i = b - line * NB;
      const int k = i % L;
      cpx<T>* x = buf + (size_t)line * N;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = x[i + r * NB];
      if (L > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[q][r] = v[q][r] * twid<T, INV>(tw, (long long)r * k * tstride);
      }
      if constexpr (R == 7 || R > 8) {
        dft_prime<T, R>(v[q], w);
      } else {
        dft<T, R, INV>(v[q]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < QM; ++q) {
    const int b = tid + q * nt;
    if (b < tot) {
      const int line = b / NB, i = b - line * NB;
      const int k = i % L;
      cpx<T>* y = buf + (size_t)line * N + (i / L) * L * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) y[r * L] = v[q][r];
    }
  }
  __syncthreads();
}

// All stages of the plan over NL lines in LDS; EMAX bounds the values per thread
// (NL*N <= EMAX*blockDim).  Every thread of the block must call it.  SMALL kernels carry
// only the radices 2, 3, 4, 5, 8 (lengths 2^a 3^b 5^c): the prime stages' registers
// would otherwise be charged to every launch.
template <typename T, bool INV, int EMAX, bool SMALL>
__device__ inline void gfft(cpx<T>* buf, int NL, const GPlan& p, const cpx<T>* __restrict__ tw) {
  int L = 1;
  for (int s = 0; s < p.nst; ++s) {
    const int R = p.rad[s];
    switch (R) {
#define GSTAGE(RR)                                                   \
  case RR:                                                           \
    gstage<T, RR, INV, (EMAX + RR - 1) / RR>(buf, NL, p.n, L, tw);   \
    break;
      GSTAGE(2) GSTAGE(3) GSTAGE(4) GSTAGE(5) GSTAGE(7) GSTAGE(8)
#undef GSTAGE
#define GSTAGE(RR)                                                               \
  case RR:                                                                       \
    if constexpr (!SMALL) gstage<T, RR, INV, (EMAX + RR - 1) / RR>(buf, NL, p.n, L, tw); \
    break;
      GSTAGE(11) GSTAGE(13) GSTAGE(17) GSTAGE(19) GSTAGE(23) GSTAGE(29) GSTAGE(31)
#undef GSTAGE
      default:
        break;
    }
    L *= R;
  }
}

// Whether a plan uses only the radices of the SMALL kernels.
__host__ __device__ inline bool gen_plan_small(const GPlan& p) {
  for (int s = 0; s < p.nst; ++s)
    if (p.rad[s] > 8) return false;
  return true;
}

// Line l, element e of a strided batch: (l / G) so + (l mod G) si + e se.
struct GLines {
  int n, nlines, nl;   // line length, lines, lines per block
  int G;
  long long so, si, se;
  __device__ __forceinline__ long long addr(int l, int e) const {
    return (long long)(l / G) * so + (long long)(l % G) * si + (long long)e * se;
  }
};

// Kernel-table index of a spectrum line element for the convolution pass.
//   3D (q3): lines along z, l = kx n1 + k1, e = k2; quadrant table (U is even in k1, k2)
//            ktab[(kx (n2/2+1) + min(k2, n2-k2)) (n1/2+1) + min(k1, n1-k1)]
//   2D:      lines along axis 1, l = kx, e = k1; ktab[kx n1 + k1]
struct GKtab {
  int q3, n1, n2;
  __device__ __forceinline__ long long index(int l, int e) const {
    if (q3) {
      const int kx = l / n1, k1 = l - kx * n1;
      const int m1 = k1 <= n1 - k1 ? k1 : n1 - k1;
      const int m2 = e <= n2 - e ? e : n2 - e;
      return ((long long)kx * (n2 / 2 + 1) + m2) * (n1 / 2 + 1) + m1;
    }
    return (long long)l * n1 + e;
  }
};

enum : int { GL_FWD = 0, GL_INV = 1, GL_CONV = 2 };

// Line FFTs of the half spectrum.  KIND GL_CONV: forward FFT, product with
// U(k) scale^2 / N (the table holds U/N), inverse FFT.
template <typename T, int KIND, int EMAX, bool SMALL>
__global__ void __launch_bounds__(kGenThreads) kg_lines(cpx<T>* __restrict__ data, GLines g,
                                                     GPlan p, const cpx<T>* __restrict__ tw,
                                                     const T* __restrict__ ktab, GKtab km,
                                                     const double* __restrict__ scale) {
  extern __shared__ __align__(16) char lds_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lds_raw);
  const int l0 = blockIdx.x * g.nl;
  const int nl = min(g.nl, g.nlines - l0);
  const int N = g.n;
  const int tot = nl * N;
  const bool contig = g.se == 1;
  for (int t = threadIdx.x; t < tot; t += blockDim.x) {
    const int line = contig ? t / N : t % nl;
    const int e = contig ? t - line * N : t / nl;
    buf[line * N + e] = data[g.addr(l0 + line, e)];
  }
  __syncthreads();
  if constexpr (KIND == GL_CONV) {
    gfft<T, false, EMAX, SMALL>(buf, nl, p, tw);
    const double s = *scale;
    const T s2 = (T)(s * s);
    for (int t = threadIdx.x; t < tot; t += blockDim.x) {
      const int line = t / N, e = t - line * N;
      buf[t] = scl(buf[t], ktab[km.index(l0 + line, e)] * s2);
    }
    __syncthreads();
    gfft<T, true, EMAX, SMALL>(buf, nl, p, tw);
  } else {
    gfft<T, KIND == GL_INV, EMAX, SMALL>(buf, nl, p, tw);
  }
  for (int t = threadIdx.x; t < tot; t += blockDim.x) {
    const int line = contig ? t / N : t % nl;
    const int e = contig ? t - line * N : t / nl;
    data[g.addr(l0 + line, e)] = buf[line * N + e];
  }
}

// Grid of the x passes: block b covers the line pairs (j, j+1), j = j0, j0 + 2, ...,
// j0 + 2 np - 2 (j0 = 2 np (b mod nbj)) of the plane k = b / nbj.  Spectrum layout
// spec[(kx n2 + k) n1 + j], kx = 0..n0/2.
struct GXTile {
  int n0, n1, n2, np, nbj;
  __device__ __forceinline__ void locate(int b, int* k, int* j0, int* npairs) const {
    *k = b / nbj;
    *j0 = 2 * np * (b - *k * nbj);
    const int left = (n1 - *j0) / 2;
    *npairs = left < np ? left : np;
  }
};

// |psi|^2 of two x lines packed as one complex line (line j real, j+1 imaginary), FFT,
// and untangled: A_k = (Z_k + conj Z_(N-k))/2, B_k = (Z_k - conj Z_(N-k))/(2i).  The
// difference sums of the stored state: part[2b] = sum |psi(i+1) - psi(i)|^2 along x,
// part[2b+1] along axis 1 (both over the block's lines).
template <typename T, int EMAX, bool SMALL>
__global__ void __launch_bounds__(kGenThreads) kg_r2c_x(const cpx<T>* __restrict__ psi,
                                                     cpx<T>* __restrict__ spec, GXTile xt,
                                                     GPlan p, const cpx<T>* __restrict__ tw,
                                                     double* __restrict__ part) {
  extern __shared__ __align__(16) char lds_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lds_raw);
  int k, j0, npairs;
  xt.locate(blockIdx.x, &k, &j0, &npairs);
  const int N = xt.n0, n1 = xt.n1;
  const int tot = npairs * N;
  double dx = 0.0, dy = 0.0;  // reduced at the end, through the same LDS
  for (int t = threadIdx.x; t < tot; t += blockDim.x) {
    const int q = t / N, i = t - q * N;
    const int j = j0 + 2 * q;
    const long long a = ((long long)k * n1 + j) * N + i;
    const cpx<T> u = psi[a], v = psi[a + N];
    buf[q * N + i] = cpx<T>{u.re * u.re + u.im * u.im, v.re * v.re + v.im * v.im};
    if (i + 1 < N) dx += absdiff2_d(psi[a + 1], u) + absdiff2_d(psi[a + N + 1], v);
    dy += absdiff2_d(v, u);
    if (j + 2 < n1) dy += absdiff2_d(psi[a + 2 * N], v);
  }
  __syncthreads();
  gfft<T, false, EMAX, SMALL>(buf, npairs, p, tw);
  const int H = N / 2 + 1;
  const int tot2 = H * 2 * npairs;
  for (int t = threadIdx.x; t < tot2; t += blockDim.x) {
    const int kx = t / (2 * npairs), r = t - kx * 2 * npairs;
    const int q = r >> 1, which = r & 1;
    const cpx<T> zk = buf[q * N + kx];
    const cpx<T> zm = buf[q * N + (kx == 0 ? 0 : N - kx)];
    cpx<T> o;
    if (which == 0) {  // (Z_k + conj Z_(N-k)) / 2
      o = cpx<T>{(T)0.5 * (zk.re + zm.re), (T)0.5 * (zk.im - zm.im)};
    } else {           // (Z_k - conj Z_(N-k)) / (2i)
      o = cpx<T>{(T)0.5 * (zk.im + zm.im), (T)0.5 * (zm.re - zk.re)};
    }
    spec[((long long)kx * xt.n2 + k) * n1 + j0 + 2 * q + which] = o;
  }
  __syncthreads();  // the line buffer is free: its first bytes hold the reduction
  double s[2] = {dx, dy};
  gblock_sum<2>(s, reinterpret_cast<double*>(lds_raw));
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s[0];
    part[2 * blockIdx.x + 1] = s[1];
  }
}

// Inverse of kg_r2c_x for the half spectrum of two real lines: Z_k = A_k + i B_k for
// k <= N/2 and Z_(N-k) = conj A_k + i conj B_k, inverse FFT, line j = Re, j+1 = Im.
template <typename T, int EMAX, bool SMALL>
__global__ void __launch_bounds__(kGenThreads) kg_c2r_x(const cpx<T>* __restrict__ spec,
                                                     T* __restrict__ phi, GXTile xt, GPlan p,
                                                     const cpx<T>* __restrict__ tw) {
  extern __shared__ __align__(16) char lds_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lds_raw);
  int k, j0, npairs;
  xt.locate(blockIdx.x, &k, &j0, &npairs);
  const int N = xt.n0, n1 = xt.n1;
  const int H = N / 2 + 1;
  const int tot = H * npairs;
  for (int t = threadIdx.x; t < tot; t += blockDim.x) {
    const int kx = t / npairs, q = t - kx * npairs;
    const long long a = ((long long)kx * xt.n2 + k) * n1 + j0 + 2 * q;
    const cpx<T> A = spec[a], B = spec[a + 1];
    buf[q * N + kx] = cpx<T>{A.re - B.im, A.im + B.re};
    if (kx > 0 && kx < N - kx) buf[q * N + N - kx] = cpx<T>{A.re + B.im, B.re - A.im};
  }
  __syncthreads();
  gfft<T, true, EMAX, SMALL>(buf, npairs, p, tw);
  const int tot2 = npairs * N;
  for (int t = threadIdx.x; t < tot2; t += blockDim.x) {
    const int q = t / N, i = t - q * N;
    const long long a = ((long long)k * n1 + j0 + 2 * q) * N + i;
    const cpx<T> z = buf[t];
    phi[a] = z.re;
    phi[a + N] = z.im;
  }
}

struct GStep {
  double dt, gc, gdd, h0, h1, h2;
};

// Nonlinear sub-step of 32 x 32 (x, axis 1) tiles of one plane, written transposed
// (dst[(k n0 + i) n1 + j]) unless MODE is MODE_OBSERVE.  part[7 b ...]: sum n, V n,
// n^2, Phi n, x^2 n, a1^2 n, a2^2 n of the physical incoming state (scale psi).
template <typename T, int MODE>
__global__ void __launch_bounds__(kThreads) kg_nl_transpose(const cpx<T>* __restrict__ psi,
                                                            const T* __restrict__ V,
                                                            const T* __restrict__ phi,
                                                            const double* __restrict__ scale,
                                                            cpx<T>* __restrict__ dst, GStep sc,
                                                            int n0, int n1, int n2,
                                                            double* __restrict__ part) {
  __shared__ cpx<T> tile[32][33];
  __shared__ double red[7 * kWaves];
  const int tx = (n0 + 31) / 32, ty = (n1 + 31) / 32;
  const int b = blockIdx.x;
  const int k = b / (tx * ty);
  const int rem = b - k * tx * ty;
  const int i0 = (rem % tx) * 32, jt0 = (rem / tx) * 32;
  const T ts = (T)(*scale);
  double ps[7] = {0, 0, 0, 0, 0, 0, 0};
  const double a2 = (k - n2 / 2) * sc.h2;
  const int li = threadIdx.x & 31;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int lj = (threadIdx.x >> 5) + 8 * r;
    const int i = i0 + li, j = jt0 + lj;
    if (i < n0 && j < n1) {
      const long long a = ((long long)k * n1 + j) * n0 + i;
      const cpx<T> pv = scl(psi[a], ts);
      const T v = V[a], ph = phi[a];
      const T n = pv.re * pv.re + pv.im * pv.im;
      const double nd = (double)n;
      const double x = (i - n0 / 2) * sc.h0, y = (j - n1 / 2) * sc.h1;
      ps[0] += nd;
      ps[1] += (double)v * nd;
      ps[2] += nd * nd;
      ps[3] += (double)ph * nd;
      ps[4] += x * x * nd;
      ps[5] += y * y * nd;
      ps[6] += a2 * a2 * nd;
      if constexpr (MODE == MODE_IMAG || MODE == MODE_REAL) {
        const T th = (T)sc.dt * (v + (T)sc.gc * n + (T)sc.gdd * ph);
        cpx<T> f;
        if constexpr (MODE == MODE_IMAG) {
          f = cpx<T>{exp(-th), (T)0};
        } else {
          T sn, cs;
          sincos_phase(th, sn, cs);
          f = cpx<T>{cs, -sn};
        }
        tile[lj][li] = pv * f;
      }
    }
  }
  block_sum<7>(ps, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < 7; ++q) part[7 * (long long)b + q] = ps[q];
  }
  if constexpr (MODE == MODE_IMAG || MODE == MODE_REAL) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int li2 = (threadIdx.x >> 5) + 8 * r;   // x within the tile
      const int lj2 = threadIdx.x & 31;             // axis 1 within the tile
      const int i = i0 + li2, j = jt0 + lj2;
      if (i < n0 && j < n1) dst[((long long)k * n0 + i) * n1 + j] = tile[lj2][li2];
    }
  }
}

// dst[(k a + x) b + y] = src[(k b + y) a + x]: the two fastest axes of nz planes swapped.
template <typename T>
__global__ void __launch_bounds__(kThreads) kg_transpose(const cpx<T>* __restrict__ src,
                                                         cpx<T>* __restrict__ dst, int a, int b,
                                                         int nz) {
  __shared__ cpx<T> tile[32][33];
  const int tx = (a + 31) / 32, ty = (b + 31) / 32;
  const int blk = blockIdx.x;
  const int k = blk / (tx * ty);
  const int rem = blk - k * tx * ty;
  const int x0 = (rem % tx) * 32, y0 = (rem / tx) * 32;
  const int l = threadIdx.x & 31;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int yy = (threadIdx.x >> 5) + 8 * r;
    if (x0 + l < a && y0 + yy < b) tile[yy][l] = src[((long long)k * b + y0 + yy) * a + x0 + l];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int xx = (threadIdx.x >> 5) + 8 * r;
    if (x0 + xx < a && y0 + l < b) dst[((long long)k * a + x0 + xx) * b + y0 + l] = tile[l][xx];
  }
}

// Crank-Nicolson sweep of columns, one thread per line (line l: element e at
// (l / G) so + (l mod G) + e se, consecutive lines adjacent in memory).  In increment
// form: with Delta_i = psi_(i-1) + psi_(i+1) - 2 psi_i and the factor table f_i = 2 A m_i
// (Thomas factors m of (1 + 2A) u_i - A (u_(i-1) + u_(i+1)), zero on the boundary rows),
//   d_i = f_i Delta_i + (f_i/2) d_(i-1)      i = 1 .. N-2   (forward, d kept in dscr)
//   e_i = d_i + (f_i/2) e_(i+1)              i = N-2 .. 1   (backward)
//   u_i = psi_i + e_i.
// SUMS: part[2b] = sum |u|^2, part[2b+1] = sum_(i < N-1) |u_(i+1) - u_i|^2 of the new
// state; OBS: the same sums of the stored state, nothing written.
template <typename T, bool SUMS, bool OBS>
__global__ void __launch_bounds__(kThreads) kg_cn_cols(cpx<T>* __restrict__ u,
                                                       cpx<T>* __restrict__ dscr,
                                                       const cpx<T>* __restrict__ f, int N,
                                                       int G, long long so, long long se,
                                                       int nlines, double* __restrict__ part) {
  __shared__ double red[2 * kWaves];
  const int l = blockIdx.x * kThreads + threadIdx.x;
  double s0 = 0.0, s1 = 0.0;
  if (l < nlines) {
    const long long base = (long long)(l / G) * so + (l % G);
    if constexpr (OBS) {
      cpx<T> prev = u[base];
      s0 += abs2_d(prev);
      for (int i = 1; i < N; ++i) {
        const cpx<T> cur = u[base + i * se];
        s0 += abs2_d(cur);
        s1 += absdiff2_d(cur, prev);
        prev = cur;
      }
    } else {
      cpx<T> pm = u[base], pc = u[base + se];
      cpx<T> d = cpx<T>{0, 0};
      for (int i = 1; i <= N - 2; ++i) {
        const cpx<T> pn = u[base + (long long)(i + 1) * se];
        const cpx<T> del = (pm + pn) - (pc + pc);
        const cpx<T> fi = f[i];
        d = fi * del + scl(fi, (T)0.5) * d;
        dscr[base + (long long)i * se] = d;
        pm = pc;
        pc = pn;
      }
      cpx<T> e = cpx<T>{0, 0};
      cpx<T> unext = u[base + (long long)(N - 1) * se];
      if constexpr (SUMS) s0 += abs2_d(unext);
      for (int i = N - 2; i >= 1; --i) {
        const long long a = base + (long long)i * se;
        const cpx<T> fi = f[i];
        e = dscr[a] + scl(fi, (T)0.5) * e;
        const cpx<T> ui = u[a] + e;
        u[a] = ui;
        if constexpr (SUMS) {
          s0 += abs2_d(ui);
          s1 += absdiff2_d(unext, ui);
        }
        unext = ui;
      }
      if constexpr (SUMS) {
        const cpx<T> u0 = u[base];
        s0 += abs2_d(u0);
        s1 += absdiff2_d(unext, u0);
      }
    }
  }
  if constexpr (SUMS || OBS) {
    double s[2] = {s0, s1};
    block_sum<2>(s, red);
    if (threadIdx.x == 0) {
      part[2 * blockIdx.x] = s[0];
      part[2 * blockIdx.x + 1] = s[1];
    }
  }
}

}  // namespace gpdbec
