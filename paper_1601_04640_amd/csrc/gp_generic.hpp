// Pass kernels for axis lengths with no compile-time specialisation: any length of at
// least 4 whose FFT line (the length, or Bluestein's M for a prime factor above 31) fits
// one LDS buffer; longer 2D axes add the four-step passes of gp_long.hpp.  The line
// length, the FFT's radix plan and the tile shapes are kernel arguments, so one set of
// kernels serves every such grid.
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
//   kg_nonlinear    the norm / potential / contact / dipolar / rms sums of the stored
//                   state (observables; it can also apply the sub-step in place)
//   kg_cn_tile      Crank-Nicolson sweep of a tile of lines held in LDS, one or more
//                   waves per line (a chunked scan of the Thomas recurrences with the
//                   chunks' values in registers); the x sweep with the nonlinear
//                   sub-step applied as it loads; optionally with the norm and
//                   difference sums of the new state
//   kg_cn_cols      the same sweep, one thread per strided line with the recurrence
//                   values in a scratch grid: strided axes of more than 1024 points with
//                   many lines, where consecutive threads read consecutive addresses
// The partial sums have the meaning the FP64 finalisation reads (gp_finalize.hpp).
#pragma once
#include "gp_device.hpp"
#include "gp_fdiv.hpp"
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
// Copy loops between global memory and LDS move kGenU values per thread per round, all
// loads issued before the first is used, so a block waits on one memory latency per
// round rather than one per value.
constexpr int kGenU = 8;

// The FFT kernels of the radices 2..8 copy the twiddle table (N values) into LDS beside
// their lines, so the stages read it at LDS latency.  The first values are fetched into
// registers before the lines' loads are issued and stored after them (one memory latency
// for both).  The kernels that also carry the radices 11..31 read the table from global
// memory: their LDS-table build gave wrong FP32 convolutions for lines with a factor 17
// or 19 (parity test), with no cause found in the source.
template <typename T>
constexpr int tw_pre() { return sizeof(T) == 4 ? 8 : 4; }
template <typename T, bool SMALL, int UT>
__device__ __forceinline__ void tw_fetch(cpx<T> (&v)[UT], const cpx<T>* __restrict__ tw, int N) {
  if constexpr (!SMALL) return;
#pragma unroll
  for (int u = 0; u < UT; ++u) {
    const int t = threadIdx.x + u * blockDim.x;
    v[u] = tw[t < N ? t : 0];
  }
}
// returns the table the stages read: twl (radices up to 8) or tw
template <typename T, bool SMALL, int UT>
__device__ __forceinline__ const cpx<T>* tw_store(cpx<T>* twl, const cpx<T> (&v)[UT],
                                                  const cpx<T>* __restrict__ tw, int N) {
  if constexpr (!SMALL) return tw;
#pragma unroll
  for (int u = 0; u < UT; ++u) {
    const int t = threadIdx.x + u * blockDim.x;
    if (t < N) twl[t] = v[u];
  }
  for (int t = threadIdx.x + UT * blockDim.x; t < N; t += blockDim.x) twl[t] = tw[t];
  return twl;
}

// Plan of an N-point FFT.  Lengths whose prime factors are at most 31 run Stockham
// stages of radices 8, 4, 2, then the odd primes; per stage the divisors of its
// butterfly indexing (M / R butterflies per line, L = the product of the earlier
// radices).  Other lengths run Bluestein's algorithm (Bluestein, "A linear filtering
// approach to the computation of discrete Fourier transform", 1970): with the chirp
// c_j = exp(-i pi j^2 / N), the DFT is X_k = c_k sum_j (x_j c_j) conj(c_(k-j)), a
// convolution evaluated by FFTs of a length M >= 2N - 1 whose factors are 2, 3, 5, 7; the
// stages are then those of M.  A line occupies m values of LDS (m = M, or N).
struct GPlan {
  int n;      // transform length
  int m;      // stage length and LDS line stride (N, or Bluestein's M)
  int blue;   // Bluestein's algorithm
  int nst;
  int rad[kGenMaxStages];
  FDiv nb[kGenMaxStages], l[kGenMaxStages];
  FDiv fm;                  // divisor by m
  const void* chirp;        // Bluestein: c_j, j < N (cpx<T>, set with the tables)
  const void* filt;         // Bluestein: FFT_M of conj(c) wrapped to M, over M (cpx<T>)
};

// Stockham stages of an m-point FFT; false if m has a prime factor above 31.
__host__ __device__ inline bool gen_stages(int m, GPlan* p) {
  p->nst = 0;
  int r_ = m;
  const int order[] = {8, 4, 2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31};
  int L = 1;
  for (int r : order) {
    while (r_ % r == 0) {
      if (p->nst >= kGenMaxStages) return false;
      p->nb[p->nst] = fdiv_make((uint32_t)(m / r));
      p->l[p->nst] = fdiv_make((uint32_t)L);
      p->rad[p->nst++] = r;
      L *= r;
      r_ /= r;
    }
  }
  return r_ == 1;
}

// Bluestein's convolution length for n: the smallest M >= 2n - 1 with factors 2, 3, 5, 7.
__host__ __device__ inline int gen_blue_len(int n) {
  for (int M = 2 * n - 1;; ++M) {
    int r = M;
    for (int q : {2, 3, 5, 7})
      while (r % q == 0) r /= q;
    if (r == 1) return M;
  }
}

__host__ __device__ inline bool gen_plan(int n, GPlan* p) {
  p->n = n;
  p->chirp = nullptr;
  p->filt = nullptr;
  if (n >= 1 && gen_stages(n, p)) {
    p->m = n;
    p->blue = 0;
  } else {
    if (n < 2) return false;
    p->m = gen_blue_len(n);
    p->blue = 1;
    if (!gen_stages(p->m, p)) return false;
  }
  p->fm = fdiv_make((uint32_t)p->m);
  return true;
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
__device__ __forceinline__ cpx<T> twid(const cpx<T>* __restrict__ tw, int k) {
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
__device__ __forceinline__ void gstage(cpx<T>* buf, int NL, int N, int L, FDiv fnb, FDiv fl,
                                       const cpx<T>* __restrict__ tw) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int NB = N / R;
  const int tot = NL * NB;
  const int tstride = N / (L * R);
  cpx<T> w[R];
  if constexpr (R == 7 || R > 8) {
#pragma unroll
    for (int k = 0; k < R; ++k) w[k] = twid<T, INV>(tw, k * (N / R));
  }
  cpx<T> v[QM][R];
  int dst[QM];
#pragma unroll
  for (int q = 0; q < QM; ++q) {
    const int b = tid + q * nt;
    dst[q] = -1;
    if (b < tot) {
      const int line = (int)fdiv((uint32_t)b, fnb), i = b - line * NB;
      const int hi = (int)fdiv((uint32_t)i, fl), k = i - hi * L;
      dst[q] = line * N + hi * L * R + k;
      cpx<T>* x = buf + (size_t)line * N;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = x[i + r * NB];
      if (L > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[q][r] = v[q][r] * twid<T, INV>(tw, r * k * tstride);
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
    if (dst[q] >= 0) {
      cpx<T>* y = buf + dst[q];
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
__device__ inline void gstages(cpx<T>* buf, int NL, const GPlan& p,
                               const cpx<T>* __restrict__ tw) {
  int L = 1;
  for (int s = 0; s < p.nst; ++s) {
    const int R = p.rad[s];
    switch (R) {
#define GSTAGE(RR)                                                   \
  case RR:                                                           \
    gstage<T, RR, INV, (EMAX + RR - 1) / RR>(buf, NL, p.m, L, p.nb[s], p.l[s], tw); \
    break;
      GSTAGE(2) GSTAGE(3) GSTAGE(4) GSTAGE(5) GSTAGE(7) GSTAGE(8)
#undef GSTAGE
#define GSTAGE(RR)                                                               \
  case RR:                                                                       \
    if constexpr (!SMALL)                                                        \
      gstage<T, RR, INV, (EMAX + RR - 1) / RR>(buf, NL, p.m, L, p.nb[s], p.l[s], tw); \
    break;
      GSTAGE(11) GSTAGE(13) GSTAGE(17) GSTAGE(19) GSTAGE(23) GSTAGE(29) GSTAGE(31)
#undef GSTAGE
      default:
        break;
    }
    L *= R;
  }
}

// The N-point transform of NL lines at LDS stride p.m (unnormalised; INV: exponent +).
// BLUE (plans with p.blue; compiled separately, so the other kernels keep their
// registers): a = x c (the conjugate input for INV), zero-padded to M; FFT_M; times the
// filter (which carries 1/M); inverse FFT_M; times c (conjugated back for INV).  The
// element loops read the chirp and the filter from global memory.
template <typename T, bool INV, int EMAX, bool SMALL, bool BLUE>
__device__ inline void gfft(cpx<T>* buf, int NL, const GPlan& p, const cpx<T>* __restrict__ tw) {
  if constexpr (!BLUE) {
    gstages<T, INV, EMAX, SMALL>(buf, NL, p, tw);
    return;
  }
  const cpx<T>* __restrict__ ch = reinterpret_cast<const cpx<T>*>(p.chirp);
  const cpx<T>* __restrict__ fl = reinterpret_cast<const cpx<T>*>(p.filt);
  const int N = p.n, M = p.m, tot = NL * M;
  for (int t = threadIdx.x; t < tot; t += blockDim.x) {
    const int j = t - (int)fdiv((uint32_t)t, p.fm) * M;
    cpx<T> v{0, 0};
    if (j < N) {
      v = buf[t];
      if (INV) v = conjg(v);
      v = v * ch[j];
    }
    buf[t] = v;
  }
  __syncthreads();
  gstages<T, false, EMAX, SMALL>(buf, NL, p, tw);
  for (int t = threadIdx.x; t < tot; t += blockDim.x) {
    const int j = t - (int)fdiv((uint32_t)t, p.fm) * M;
    buf[t] = buf[t] * fl[j];
  }
  __syncthreads();
  gstages<T, true, EMAX, SMALL>(buf, NL, p, tw);
  for (int t = threadIdx.x; t < tot; t += blockDim.x) {
    const int j = t - (int)fdiv((uint32_t)t, p.fm) * M;
    if (j < N) {
      cpx<T> v = buf[t] * ch[j];
      if (INV) v = conjg(v);
      buf[t] = v;
    }
  }
  __syncthreads();
}

// Whether a plan uses only the radices of the SMALL kernels.
__host__ __device__ inline bool gen_plan_small(const GPlan& p) {
  for (int s = 0; s < p.nst; ++s)
    if (p.rad[s] > 8) return false;
  return true;
}

// Line l, element e of a strided batch: (l / G) so + (l mod G) si + e se.  fn, fnl, fg:
// divisors by n, nl and G.
struct GLines {
  int n, nlines, nl;   // line length, lines, lines per block
  int G;
  long long so, si, se;
  FDiv fn, fnl, fg;
  // the lines are consecutive runs of n values (G = 1, so = n, se = 1): a block's tile is
  // one contiguous range
  __device__ __forceinline__ bool packed() const { return G == 1 && se == 1 && so == n; }
  __device__ __forceinline__ long long addr(int l, int e) const {
    const int hi = (int)fdiv((uint32_t)l, fg);
    return (long long)hi * so + (long long)(l - hi * G) * si + (long long)e * se;
  }
  // element t of a block's tile of nl lines as (line, element): line-major when the lines
  // are contiguous, element-major when strided, so that consecutive threads touch
  // consecutive addresses (value selects: no pointer into registers)
  __device__ __forceinline__ int2 tile_index(int t) const {
    const bool c = se == 1;
    const int q = (int)fdiv((uint32_t)t, c ? fn : fnl);
    const int r = t - q * (c ? n : nl);
    return c ? make_int2(q, r) : make_int2(r, q);
  }
};

// Kernel-table index of a spectrum line element for the convolution pass.
//   3D (q3): lines along z, l = kx n1 + k1, e = k2; quadrant table (U is even in k1, k2)
//            ktab[(kx (n2/2+1) + min(k2, n2-k2)) (n1/2+1) + min(k1, n1-k1)]
//   2D:      lines along axis 1, l = kx, e = k1; ktab[kx n1 + k1]
// 2D grids with a split axis (slot != 0): the table is laid out like the spectrum, and
// an element's entry is at its own spectrum offset.
struct GKtab {
  int q3, n1, n2;
  FDiv fn1;
  int slot;
  __device__ __forceinline__ long long index(int l, int e) const {
    if (q3) {
      const int kx = (int)fdiv((uint32_t)l, fn1), k1 = l - kx * n1;
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
// FP32: at most 64 VGPRs, so that two full 16-wave blocks share a CU (not asked of the
// Bluestein variants, which would spill)
template <typename T, bool BLUE>
constexpr int gen_waves_per_eu() { return sizeof(T) == 4 && !BLUE ? 8 : 1; }

// The four-step FFT's outer passes (w4 != null): GL_FWD multiplies element k of line l by
// w4[c k] after its transform, GL_INV by conj(w4[c k]) before it, with the line's column
// c = l / G (w4hi) or l mod G; w4[m] = W_N^m of the split axis.
template <typename T, int KIND, int EMAX, bool SMALL, bool BLUE = false>
__global__ void __launch_bounds__(kGenThreads, (gen_waves_per_eu<T, BLUE>())) kg_lines(cpx<T>* __restrict__ data, GLines g,
                                                     GPlan p, const cpx<T>* __restrict__ tw,
                                                     const T* __restrict__ ktab, GKtab km,
                                                     const double* __restrict__ scale,
                                                     const cpx<T>* __restrict__ w4, int w4hi) {
  extern __shared__ __align__(16) char lds_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lds_raw);
  // tiles numbered XCD-contiguously (blocks run on the XCDs round-robin): neighbouring
  // tiles, which share 128-byte lines of strided data, share an L2
  const int l0 = xcd_tile(blockIdx.x, gridDim.x) * g.nl;
  const int nl = min(g.nl, g.nlines - l0);
  const int N = g.n;
  const int LS = BLUE ? p.m : N;   // LDS line stride: N, or Bluestein's M
  const int nt = blockDim.x;
  const int tot = g.nl * N;  // the full tile's indexing; lines past nl are skipped
  cpx<T>* twl = buf + g.nl * LS;   // the twiddle table (of the stage length)
  constexpr int UT = tw_pre<T>() / 2;
  cpx<T> twv[UT];
  tw_fetch<T, SMALL, UT>(twv, tw, LS);
  const bool packed = g.packed();
  // LDS slot of element t of a packed tile (line-major, lines at stride LS)
  auto pslot = [&](int t) { return LS == N ? t : t + (int)fdiv((uint32_t)t, g.fn) * (LS - N); };
  cpx<T>* const run = data + (long long)l0 * N;  // the tile when packed
  for (int t0 = threadIdx.x; t0 < tot; t0 += kGenU * nt) {
    T vr[kGenU], vi[kGenU];  // separate parts: arrays of the aligned pair type stay in memory
    int at[kGenU];
#pragma unroll
    for (int u = 0; u < kGenU; ++u) {
      const int t = t0 + u * nt;
      if (packed) {
        at[u] = t < nl * N ? pslot(t) : -1;
        const cpx<T> v = run[at[u] >= 0 ? t : 0];
        vr[u] = v.re;
        vi[u] = v.im;
      } else {
        const int2 le = g.tile_index(t);
        const int line = le.x, e = le.y;
        at[u] = (t < tot && line < nl) ? line * LS + e : -1;
        const cpx<T> v = data[at[u] >= 0 ? g.addr(l0 + line, e) : 0];
        vr[u] = v.re;
        vi[u] = v.im;
      }
    }
#pragma unroll
    for (int u = 0; u < kGenU; ++u)
      if (at[u] >= 0) buf[at[u]] = cpx<T>{vr[u], vi[u]};
  }
  const cpx<T>* twu = tw_store<T, SMALL, UT>(twl, twv, tw, LS);
  __syncthreads();
  // the four-step twiddle of line l, element e
  auto w4_of = [&](int line, int e) {
    const int l = l0 + line;
    const int hi = (int)fdiv((uint32_t)l, g.fg);
    return w4[(w4hi ? hi : l - hi * g.G) * e];
  };
  if constexpr (KIND == GL_INV) {
    if (w4 != nullptr) {
      for (int t = threadIdx.x; t < nl * N; t += nt) {
        const int line = (int)fdiv((uint32_t)t, g.fn), e = t - line * N;
        buf[line * LS + e] = buf[line * LS + e] * conjg(w4_of(line, e));
      }
      __syncthreads();
    }
  }
  if constexpr (KIND == GL_CONV) {
    gfft<T, false, EMAX, SMALL, BLUE>(buf, nl, p, twu);
    const double s = *scale;
    const T s2 = (T)(s * s);
    // the tile's order of the loads (element-major for strided lines): the table reads of
    // adjacent lines are adjacent
    for (int t0 = threadIdx.x; t0 < tot; t0 += kGenU * nt) {
      T kv[kGenU];
      int at[kGenU];
#pragma unroll
      for (int u = 0; u < kGenU; ++u) {
        const int t = t0 + u * nt;
        const int2 le = g.tile_index(t);
        at[u] = (t < tot && le.x < nl) ? le.x * LS + le.y : -1;
        long long ki = 0;
        if (at[u] >= 0) ki = km.slot ? g.addr(l0 + le.x, le.y) : km.index(l0 + le.x, le.y);
        kv[u] = ktab[ki];
      }
#pragma unroll
      for (int u = 0; u < kGenU; ++u)
        if (at[u] >= 0) buf[at[u]] = scl(buf[at[u]], kv[u] * s2);
    }
    __syncthreads();
    gfft<T, true, EMAX, SMALL, BLUE>(buf, nl, p, twu);
  } else {
    gfft<T, KIND == GL_INV, EMAX, SMALL, BLUE>(buf, nl, p, twu);
    if constexpr (KIND == GL_FWD) {
      if (w4 != nullptr) {
        for (int t = threadIdx.x; t < nl * N; t += nt) {
          const int line = (int)fdiv((uint32_t)t, g.fn), e = t - line * N;
          buf[line * LS + e] = buf[line * LS + e] * w4_of(line, e);
        }
        __syncthreads();
      }
    }
  }
  if (packed) {
    for (int t = threadIdx.x; t < nl * N; t += nt) run[t] = buf[pslot(t)];
  } else {
    for (int t = threadIdx.x; t < tot; t += nt) {
      const int2 le = g.tile_index(t);
      if (le.x < nl) data[g.addr(l0 + le.x, le.y)] = buf[le.x * LS + le.y];
    }
  }
}

// Grid of the x passes: block b covers the line pairs (j, j+1), j = j0, j0 + 2, ...,
// j0 + 2 np - 2 (j0 = 2 np (b mod nbj)) of the plane k = b / nbj; with an odd n1 the
// last pair of a plane has no line j + 1 (packed as a zero line).  Spectrum layout
// spec[(kx n2 + k) n1 + j], kx = 0..n0/2.  fn0, fnp, f2np, fnbj: divisors by n0, np, 2 np
// and nbj.
struct GXTile {
  int n0, n1, n2, np, nbj;
  FDiv fn0, fnp, f2np, fnbj;
  __device__ __forceinline__ void locate(int b, int* k, int* j0, int* npairs) const {
    *k = (int)fdiv((uint32_t)b, fnbj);
    *j0 = 2 * np * (b - *k * nbj);
    const int left = (n1 - *j0 + 1) / 2;  // an odd n1 leaves a last pair of one line
    *npairs = left < np ? left : np;
  }
};

// |psi|^2 of two x lines packed as one complex line (line j real, j+1 imaginary), FFT,
// and untangled: A_k = (Z_k + conj Z_(N-k))/2, B_k = (Z_k - conj Z_(N-k))/(2i).  The
// difference sums of the stored state: part[2b] = sum |psi(i+1) - psi(i)|^2 along x,
// part[2b+1] along axis 1 (both over the block's lines).
template <typename T, int EMAX, bool SMALL, bool BLUE = false>
__global__ void __launch_bounds__(kGenThreads) kg_r2c_x(const cpx<T>* __restrict__ psi,
                                                     cpx<T>* __restrict__ spec, GXTile xt,
                                                     GPlan p, const cpx<T>* __restrict__ tw,
                                                     double* __restrict__ part) {
  // five loads per value: fewer values per round than the plain copy loops
  constexpr int U = sizeof(T) == 4 ? 4 : 2;
  extern __shared__ __align__(16) char lds_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lds_raw);
  int k, j0, npairs;
  xt.locate(xcd_tile(blockIdx.x, gridDim.x), &k, &j0, &npairs);  // XCD-contiguous tiles
  const int N = xt.n0, n1 = xt.n1;
  const int LS = BLUE ? p.m : N;  // LDS line stride: N, or Bluestein's M
  const int nt = blockDim.x;
  const int tot = npairs * N;
  cpx<T>* twl = buf + xt.np * LS;  // the twiddle table (a shorter prefetch: five loads a value)
  constexpr int UT = tw_pre<T>() / 2;
  cpx<T> twv[UT];
  tw_fetch<T, SMALL, UT>(twv, tw, LS);
  double dx = 0.0, dy = 0.0;  // reduced at the end, through the same LDS
  for (int t0 = threadIdx.x; t0 < tot; t0 += U * nt) {
    // |psi|^2 needs the two values; the differences their x and axis-1 neighbours
    T n0v[U], n1v[U];
    double ddx[U], ddy[U];
    int jj[U], ss[U];
    cpx<T> a0[U], a1[U], b0[U], b1[U], c1[U];
    bool hh[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * nt;
      const int q = (int)fdiv((uint32_t)t, xt.fn0);
      const int i = t - q * N;
      jj[u] = t < tot ? j0 + 2 * q : -1;
      ss[u] = q * LS + i;
      // loads from in-range addresses only, selected afterwards (a select between a
      // load and a constant would be turned into a load through a stack slot)
      const bool ok = jj[u] >= 0;
      const bool has1 = ok && jj[u] + 1 < n1;  // line j + 1 exists
      hh[u] = has1;
      const long long a = ok ? ((long long)k * n1 + j0 + 2 * q) * N + i : 0;
      a0[u] = psi[a];
      a1[u] = psi[has1 ? a + N : a];  // without line j + 1: line j again (no difference)
      b0[u] = psi[ok && i + 1 < N ? a + 1 : a];
      b1[u] = psi[has1 && i + 1 < N ? a + N + 1 : (has1 ? a + N : a)];
      c1[u] = psi[has1 && jj[u] + 2 < n1 ? a + 2 * N : (has1 ? a + N : a)];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      n0v[u] = a0[u].re * a0[u].re + a0[u].im * a0[u].im;
      n1v[u] = hh[u] ? a1[u].re * a1[u].re + a1[u].im * a1[u].im : (T)0;
      ddx[u] = absdiff2_d(b0[u], a0[u]) + absdiff2_d(b1[u], a1[u]);
      ddy[u] = absdiff2_d(a1[u], a0[u]) + absdiff2_d(c1[u], a1[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (jj[u] >= 0) {
        buf[ss[u]] = cpx<T>{n0v[u], n1v[u]};
        dx += ddx[u];
        dy += ddy[u];
      }
    }
  }
  const cpx<T>* twu = tw_store<T, SMALL, UT>(twl, twv, tw, LS);
  __syncthreads();
  gfft<T, false, EMAX, SMALL, BLUE>(buf, npairs, p, twu);
  const int H = N / 2 + 1;
  const int tot2 = H * 2 * xt.np;  // the full tile's indexing; pairs past npairs skipped
  for (int t = threadIdx.x; t < tot2; t += nt) {
    const int kx = (int)fdiv((uint32_t)t, xt.f2np), r = t - kx * 2 * xt.np;
    const int q = r >> 1, which = r & 1;
    if (q >= npairs || j0 + 2 * q + which >= n1) continue;
    const cpx<T> zk = buf[q * LS + kx];
    const cpx<T> zm = buf[q * LS + (kx == 0 ? 0 : N - kx)];
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
template <typename T, int EMAX, bool SMALL, bool BLUE = false>
__global__ void __launch_bounds__(kGenThreads) kg_c2r_x(const cpx<T>* __restrict__ spec,
                                                     T* __restrict__ phi, GXTile xt, GPlan p,
                                                     const cpx<T>* __restrict__ tw) {
  constexpr int U = kGenU / 2;  // two loads per value
  extern __shared__ __align__(16) char lds_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lds_raw);
  int k, j0, npairs;
  xt.locate(xcd_tile(blockIdx.x, gridDim.x), &k, &j0, &npairs);  // XCD-contiguous tiles
  const int N = xt.n0, n1 = xt.n1;
  const int LS = BLUE ? p.m : N;  // LDS line stride: N, or Bluestein's M
  const int H = N / 2 + 1;
  const int nt = blockDim.x;
  const int tot = H * xt.np;  // the full tile's indexing; pairs past npairs skipped
  cpx<T>* twl = buf + xt.np * LS;  // the twiddle table
  cpx<T> twv[tw_pre<T>()];
  tw_fetch<T, SMALL, tw_pre<T>()>(twv, tw, LS);
  for (int t0 = threadIdx.x; t0 < tot; t0 += U * nt) {
    cpx<T> A[U], B[U];
    int kk[U], qq[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * nt;
      kk[u] = (int)fdiv((uint32_t)t, xt.fnp);
      qq[u] = t - kk[u] * xt.np;
      if (t >= tot || qq[u] >= npairs) qq[u] = -1;
      // in-range addresses only (see kg_r2c_x); no line j + 1: B = 0
      const long long a =
          qq[u] >= 0 ? ((long long)kk[u] * xt.n2 + k) * n1 + j0 + 2 * qq[u] : 0;
      const bool has1 = qq[u] >= 0 && j0 + 2 * qq[u] + 1 < n1;
      A[u] = spec[a];
      B[u] = spec[has1 ? a + 1 : a];
      if (!has1) B[u] = cpx<T>{0, 0};
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (qq[u] >= 0) {
        const int kx = kk[u], q = qq[u];
        buf[q * LS + kx] = cpx<T>{A[u].re - B[u].im, A[u].im + B[u].re};
        if (kx > 0 && kx < N - kx)
          buf[q * LS + N - kx] = cpx<T>{A[u].re + B[u].im, B[u].re - A[u].im};
      }
    }
  }
  const cpx<T>* twu = tw_store<T, SMALL, tw_pre<T>()>(twl, twv, tw, LS);
  __syncthreads();
  gfft<T, true, EMAX, SMALL, BLUE>(buf, npairs, p, twu);
  const int tot2 = npairs * N;
  for (int t = threadIdx.x; t < tot2; t += nt) {
    const int q = (int)fdiv((uint32_t)t, xt.fn0), i = t - q * N;
    const long long a = ((long long)k * n1 + j0 + 2 * q) * N + i;
    const cpx<T> z = buf[q * LS + i];
    phi[a] = z.re;
    if (j0 + 2 * q + 1 < n1) phi[a + N] = z.im;
  }
}

// Step scalars of the nonlinear pass; f0, f1: divisors by n0 and n1.
struct GStep {
  double dt, gc, gdd, h0, h1, h2;
  FDiv f0, f1;
};

// Nonlinear sub-step in place: psi <- scale psi exp(-eps dt (V + g_c n + g_dd Phi)),
// eps = 1 (MODE_IMAG) or i (MODE_REAL); MODE_OBSERVE only sums.  part[7 b ...]: sum n,
// V n, n^2, Phi n, x^2 n, a1^2 n, a2^2 n of the physical incoming state (scale psi).
// Each thread walks its points kThreads apart, U at a time with their loads in flight;
// the point's row r = a / n0 and column i advance by the divisor of n0.
template <typename T, int MODE>
__global__ void __launch_bounds__(kThreads) kg_nonlinear(cpx<T>* __restrict__ psi,
                                                         const T* __restrict__ V,
                                                         const T* __restrict__ phi,
                                                         const double* __restrict__ scale,
                                                         GStep sc, int n0, int n1, int n2,
                                                         double* __restrict__ part) {
  constexpr int U = 4;
  __shared__ double red[7 * kWaves];
  const long long npts = (long long)n0 * n1 * n2;
  const long long per = (npts + gridDim.x - 1) / gridDim.x;
  const long long lo = per * blockIdx.x;
  const long long hi = lo + per < npts ? lo + per : npts;
  const T ts = (T)(*scale);
  double ps[7] = {0, 0, 0, 0, 0, 0, 0};
  long long a = lo + threadIdx.x;
  // row and column of a (a < 2^31 n0: one 64-bit division per thread)
  uint32_t r = 0;
  int i = 0;
  if (a < hi) {
    r = (uint32_t)(a / n0);
    i = (int)(a - (long long)r * n0);
  }
  for (; a < hi; a += U * kThreads) {
    cpx<T> pv[U];
    T vv[U], ph[U];
    int ii[U];
    uint32_t rr[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long au = a + (long long)u * kThreads;
      ok[u] = au < hi;
      ii[u] = i;
      rr[u] = r;
      const long long as = ok[u] ? au : lo;  // in-range addresses only (see kg_r2c_x)
      pv[u] = psi[as];
      vv[u] = V[as];
      ph[u] = phi[as];
      i += kThreads;
      const uint32_t dq = fdiv((uint32_t)i, sc.f0);
      r += dq;
      i -= (int)dq * n0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!ok[u]) continue;
      const int k = (int)fdiv(rr[u], sc.f1), j = (int)rr[u] - k * n1;
      const cpx<T> p = scl(pv[u], ts);
      const T v = vv[u];
      const T n = p.re * p.re + p.im * p.im;
      const double nd = (double)n;
      const double x = (ii[u] - n0 / 2) * sc.h0, y = (j - n1 / 2) * sc.h1,
                   z = (k - n2 / 2) * sc.h2;
      ps[0] += nd;
      ps[1] += (double)v * nd;
      ps[2] += nd * nd;
      ps[3] += (double)ph[u] * nd;
      ps[4] += x * x * nd;
      ps[5] += y * y * nd;
      ps[6] += z * z * nd;
      if constexpr (MODE == MODE_IMAG || MODE == MODE_REAL) {
        const T th = (T)sc.dt * (v + (T)sc.gc * n + (T)sc.gdd * ph[u]);
        cpx<T> f;
        if constexpr (MODE == MODE_IMAG) {
          f = cpx<T>{exp(-th), (T)0};
        } else {
          T sn, cs;
          sincos_phase(th, sn, cs);
          f = cpx<T>{cs, -sn};
        }
        psi[a + (long long)u * kThreads] = p * f;
      }
    }
  }
  block_sum<7>(ps, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < 7; ++q) part[7 * (long long)blockIdx.x + q] = ps[q];
  }
}

template <typename T>
__device__ __forceinline__ cpx<T> shfl_up_c(cpx<T> v, int off) {
  return cpx<T>{__shfl_up(v.re, off, 64), __shfl_up(v.im, off, 64)};
}
template <typename T>
__device__ __forceinline__ cpx<T> shfl_down_c(cpx<T> v, int off) {
  return cpx<T>{__shfl_down(v.re, off, 64), __shfl_down(v.im, off, 64)};
}

// Crank-Nicolson sweeps of lines.  In increment form, with
// Delta_i = psi_(i-1) + psi_(i+1) - 2 psi_i and the factor table f_i = 2 A m_i (Thomas
// factors m of (1 + 2A) u_i - A (u_(i-1) + u_(i+1)); f = 0 on the two boundary rows),
// g_i = f_i / 2:
//   forward  d_i = f_i Delta_i + g_i d_(i-1)      backward  e_i = d_i + g_i e_(i+1)
//   u_i = psi_i + e_i.
// Both are first-order linear recurrences.  Each lane takes a chunk of S consecutive
// rows, runs the recurrence from a zero carry, and the chunks are joined by a scan of the
// affine maps c -> (prod g) c + (local result); each lane then adds its carry times the
// running product of g.  The result equals the sequential recurrence up to rounding
// order.
// LDS layout of a line spread over `lanes` lanes (S = ceil(N/lanes)): lane q's rows sit
// at [q Sp, q Sp + S) with Sp = S | 1 (odd), so lanes reading the j-th rows of their
// chunks touch distinct bank pairs; a line takes ceil(N/S) Sp values (lanes past the
// last chunk own none).
__host__ __device__ inline int cn_line_slots(int n, int lanes = 64) {
  const int S = (n + lanes - 1) / lanes;
  return ((n + S - 1) / S) * (S | 1);
}

// Crank-Nicolson sweep of a tile of lines: the recurrences and chunked scans above, with
// wpl waves per line (64 wpl lanes; wpl = 1 for lines of up to 1024
// points, up to 16 for 8192), the chunk's recurrence values in registers (S <= TS rows
// per lane) and the factor table in LDS, laid out like the lines.  With wpl > 1 the waves'
// affine maps are composed through LDS after the in-wave scans: the carry into wave w of
// a line is the composition of the totals of waves 0..w-1 (forward) or w+1..wpl-1
// (backward).  Strided tiles take adjacent lines (64-byte runs).
// MODE 0: solve; 1: solve with the new-state sums part[2b], part[2b+1]; 2: those sums of
// the stored state, no solve.
// NLM = MODE_IMAG or MODE_REAL (x lines only: G = 1, so = n0, se = 1): the nonlinear
// sub-step of kg_nonlinear applied to each value as it is loaded, with its seven sums of
// the incoming state in pnl[7b ...]; NLM < 0: none.
constexpr int kTileS = 16;
constexpr int kTileMaxN = 64 * kTileS;   // longest line at one wave per line
constexpr int kTileMaxWaves = 16;
// waves per tile block: 16 FP32, 8 FP64 (whose recurrence values need up to 256 VGPRs)
template <typename T>
constexpr int tile_max_waves() { return sizeof(T) == 4 ? 16 : 8; }

// Lines longer than one tile are swept in segments of n rows (SEG): line l of the tile is
// segment s = l mod nseg of the long line l / nseg, its factor rows f[s n ..] (read from
// global memory).  The recurrences are linear, so a segment's results follow from its own
// solve started from two carries: C, the true d entering the segment (at its row -1), and
// E, the true e entering from the right (at its row n).  With d0, e0 the zero-carry
// results and R_i = g_a ... g_i (a: the first row),
//   d_i = d0_i + R_i C,   e_a = e0_a + Q C + P E,   P = R_(last row),
//   Q = sum_m (g_a ... g_(m-1)) R_m
// (P, Q fixed by the factor table).  The carries run along each long line from the
// segments' summaries (k_seg_summary, k_seg_carry); the sweep starts its scans from
// car[4l] = C and car[4l+1] = E, with car[4l+2], car[4l+3] = psi of the rows before and
// after the segment (values before the sweep: the neighbouring segments are rewritten by
// other blocks).
// Segment lines are numbered line-major, l = L nseg + s (contiguous long lines: the tile's
// lines are consecutive segments), or segment-major, l = s nlong + L (cols: strided long
// lines, so that a tile holds the same segment of adjacent lines; fseg then divides by
// nlong).
struct GSeg {
  int nseg;
  FDiv fseg;
  const void* car;
  int cols;
};

struct GNl {  // the nonlinear sub-step's inputs for the fused x sweep
  const void* V;
  const void* phi;
  const double* scale;
  GStep sc;
  int n0, n1, n2;
  double* part;
};

// LDS writes of a wave made visible to the wave's other lanes (no block barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// WI (contiguous lines, one wave per line): each wave loads, solves and stores its own
// line, lanes along it (coalesced), with the factor rows read from global memory, so the
// waves of a block run independently up to the final reduction of the sums.
template <typename T, int MODE, int NLM, int TS, bool SEG = false, bool WI = false>
__global__ void __launch_bounds__(64 * tile_max_waves<T>()) kg_cn_tile(cpx<T>* __restrict__ data,
                                                                GLines g, int wpl, FDiv fs,
                                                                const cpx<T>* __restrict__ f,
                                                                double* __restrict__ part,
                                                                GNl nlz, GSeg sg) {
  static_assert(!SEG || NLM < 0, "segments carry no nonlinear sub-step");
  extern __shared__ __align__(16) char lds_raw[];
  __shared__ double red[7 * kTileMaxWaves];
  __shared__ cpx<T> wP[kTileMaxWaves], wB[kTileMaxWaves];  // the waves' composed maps
  const int N = g.n;
  const int S = (int)fs.d, Sp = S | 1, LS = cn_line_slots(N, 64 * wpl);
  // tiles numbered XCD-contiguously (blocks run on the XCDs round-robin): neighbouring
  // tiles, which share 128-byte lines of strided data, share an L2
  const int l0 = xcd_tile(blockIdx.x, gridDim.x) * g.nl;
  const int nl = min(g.nl, g.nlines - l0);
  const int nt = blockDim.x;
  const int tot = g.nl * N;  // the full tile's indexing; lines past nl are skipped
  cpx<T>* ps = reinterpret_cast<cpx<T>*>(lds_raw);   // nl lines of psi (then u)
  cpx<T>* fl = ps + (size_t)g.nl * LS;                // the factor table, one line (not SEG)
  // values per thread per load round (FP64: half, a quarter with the nonlinear sub-step,
  // for the registers)
  constexpr int U = sizeof(T) == 4 ? kGenU : (NLM >= 0 ? kGenU / 4 : kGenU / 2);
  constexpr int UF = 4;  // factor-table values per thread fetched ahead of the tile
  double q7[7] = {0, 0, 0, 0, 0, 0, 0};
  [[maybe_unused]] T ts = (T)1;
  if constexpr (NLM >= 0) ts = (T)(*nlz.scale);
  // the factor table's first UF nt values are loaded with the tile and stored after it
  cpx<T> fpre[UF];
  if constexpr (MODE != 2 && !SEG && !WI) {
#pragma unroll
    for (int u = 0; u < UF; ++u) {
      const int t = threadIdx.x + u * nt;
      fpre[u] = f[t < N ? t : 0];
    }
  }
  // packed tiles are one contiguous range; in strided tiles (element-major, blockDim a
  // multiple of nl) thread tid keeps line tid mod nl and walks its elements nt/nl apart,
  // so its line's base address is computed once
  const bool packed = g.packed();
  const int sl = threadIdx.x % g.nl, se0 = threadIdx.x / g.nl, sstep = nt / g.nl;
  const long long sbase = !packed && sl < nl ? g.addr(l0 + sl, 0) : 0;
  const long long pbase = (long long)l0 * N;
  // WI: wave wv walks its own line wv, lanes 64 apart
  const int wv = threadIdx.x >> 6;
  const int tstart = WI ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
  const int tstep = WI ? 64 : nt;
  const int tlim = WI ? N : tot;
  for (int t0 = tstart, r0 = 0; t0 < tlim; t0 += U * tstep, r0 += U) {
    T vr[U], vi[U];
    [[maybe_unused]] T vv[U], ph[U];
    int at[U], ee[U], ll[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * tstep;
      int line, e;
      long long a;
      if (WI) {
        line = wv;
        e = t;
        a = pbase + (long long)line * N + t;
      } else if (packed) {
        line = (int)fdiv((uint32_t)t, g.fn);
        e = t - line * N;
        a = pbase + t;
      } else {
        line = sl;
        e = se0 + sstep * (r0 + u);
        a = sbase + (long long)e * g.se;
      }
      const int c = (int)fdiv((uint32_t)e, fs);
      at[u] = (t < tlim && line < nl) ? line * LS + c * Sp + (e - c * S) : -1;
      ee[u] = e;
      ll[u] = l0 + line;
      if (at[u] < 0) a = 0;  // in range only
      const cpx<T> v = data[a];
      vr[u] = v.re;
      vi[u] = v.im;
      if constexpr (NLM >= 0) {
        vv[u] = reinterpret_cast<const T*>(nlz.V)[a];
        ph[u] = reinterpret_cast<const T*>(nlz.phi)[a];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (at[u] < 0) continue;
      cpx<T> v{vr[u], vi[u]};
      if constexpr (NLM >= 0) {
        // psi <- scale psi exp(-eps dt (V + g_c n + g_dd Phi)) and the sums of scale psi
        const GStep& sc = nlz.sc;
        const cpx<T> pv = scl(v, ts);
        const T n = pv.re * pv.re + pv.im * pv.im;
        const double nd = (double)n;
        const int k = (int)fdiv((uint32_t)ll[u], sc.f1), j = ll[u] - k * nlz.n1;
        const double x = (ee[u] - nlz.n0 / 2) * sc.h0, y = (j - nlz.n1 / 2) * sc.h1,
                     z = (k - nlz.n2 / 2) * sc.h2;
        q7[0] += nd;
        q7[1] += (double)vv[u] * nd;
        q7[2] += nd * nd;
        q7[3] += (double)ph[u] * nd;
        q7[4] += x * x * nd;
        q7[5] += y * y * nd;
        q7[6] += z * z * nd;
        const T th = (T)sc.dt * (vv[u] + (T)sc.gc * n + (T)sc.gdd * ph[u]);
        cpx<T> fz;
        if constexpr (NLM == MODE_IMAG) {
          fz = cpx<T>{exp(-th), (T)0};
        } else {
          T sn, cs;
          sincos_phase(th, sn, cs);
          fz = cpx<T>{cs, -sn};
        }
        v = pv * fz;
      }
      ps[at[u]] = v;
    }
  }
  // segments and WI tiles read their factor rows from global memory (each lane its
  // chunk's S rows, contiguous; the table is small and stays in L2), not through LDS
  if constexpr (MODE != 2 && !SEG && !WI) {
#pragma unroll
    for (int u = 0; u < UF; ++u) {
      const int t = threadIdx.x + u * nt;
      if (t < N) {
        const int c = (int)fdiv((uint32_t)t, fs);
        fl[c * Sp + (t - c * S)] = fpre[u];
      }
    }
    for (int t = threadIdx.x + UF * nt; t < N; t += nt) {
      const int c = (int)fdiv((uint32_t)t, fs);
      fl[c * Sp + (t - c * S)] = f[t];
    }
  }
  if constexpr (WI) wave_sync(); else __syncthreads();
  // wave w works on line w / wpl, lanes q = 64 (w mod wpl) + lane of it
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int line = wave / wpl, sub = wave - line * wpl;
  const bool act = line < nl;
  const int q = sub * 64 + lane;
  const int i0 = q * S;
  const int cnt = act ? min(S, N - i0) : 0;  // rows of this lane's chunk (<= 0: none)
  const int slot = cnt > 0 ? q * Sp : 0;     // lanes with no chunk point at the line start
  const cpx<T> zero{0, 0};
  double s0 = 0.0, s1 = 0.0;
  cpx<T>* p = ps + (act ? line : 0) * LS + slot;
  cpx<T> d[TS];
  // segments: the line's index, its segment, the rows beside it and the carries entering
  [[maybe_unused]] const int lg = l0 + (act ? line : 0);
  [[maybe_unused]] int sgi = 0;
  [[maybe_unused]] cpx<T> eL = zero, eR = zero, cC = zero, cE = zero;
  if constexpr (SEG) {
    const int q = (int)fdiv((uint32_t)lg, sg.fseg);
    sgi = sg.cols ? q : lg - q * sg.nseg;
    const cpx<T>* car = reinterpret_cast<const cpx<T>*>(sg.car) + 4LL * lg;
    cC = car[0];
    cE = car[1];
    eL = car[2];
    eR = car[3];
  }
  if constexpr (MODE != 2) {
    const cpx<T>* fq =
        (SEG || WI) ? f + (long long)sgi * N + (cnt > 0 ? i0 : 0) : fl + slot;
    // forward, zero carry: local d and the chunk's product of g
    cpx<T> acc = zero, prod = {1, 0};
    cpx<T> pm = p[q > 0 && cnt > 0 ? -Sp + S - 1 : 0];   // row i0 - 1
    if (!(i0 > 0 && cnt > 0)) pm = SEG ? eL : zero;      // a segment's row -1: its neighbour
    cpx<T> pc = p[0];
#pragma unroll
    for (int j = 0; j < TS; ++j) {
      if (j < cnt) {
        cpx<T> pn = p[j + 1 < cnt ? j + 1 : Sp];  // row N is none: zero (a segment's: eR)
        if (i0 + j + 1 >= N) pn = SEG ? eR : zero;
        const cpx<T> fi = fq[j];
        acc = fi * ((pm + pn) - (pc + pc)) + scl(fi, (T)0.5) * acc;
        prod = scl(fi, (T)0.5) * prod;
        d[j] = acc;
        pm = pc;
        pc = pn;
      }
    }
    // inclusive scan of the maps c -> prod c + acc over the wave's lanes
    cpx<T> P = prod, B = acc;
    for (int off = 1; off < 64; off <<= 1) {
      const cpx<T> Pp = shfl_up_c(P, off), Bp = shfl_up_c(B, off);
      if (lane >= off) {
        B = P * Bp + B;
        P = P * Pp;
      }
    }
    // d entering the wave: the earlier waves' totals composed in order (on a segment's
    // carry)
    cpx<T> C = SEG ? cC : zero;
    if (wpl > 1) {
      if (lane == 63) {
        wP[wave] = P;
        wB[wave] = B;
      }
      __syncthreads();
      for (int s2 = 0; s2 < sub; ++s2) C = wP[wave - sub + s2] * C + wB[wave - sub + s2];
      __syncthreads();  // the totals are read before the backward pass writes its own
    }
    const cpx<T> Pu = shfl_up_c(P, 1), Bu = shfl_up_c(B, 1);
    cpx<T> carry = lane == 0 ? C : Pu * C + Bu;   // d at the end of the previous chunk
#pragma unroll
    for (int j = 0; j < TS; ++j) {
      if (j < cnt) {
        carry = scl(fq[j], (T)0.5) * carry;
        d[j] = d[j] + carry;
      }
    }
    // backward, zero carry from the right: local e (kept in d)
    acc = zero;
#pragma unroll
    for (int j = TS - 1; j >= 0; --j) {
      if (j < cnt) {
        acc = d[j] + scl(fq[j], (T)0.5) * acc;
        d[j] = acc;
      }
    }
    P = prod;
    B = acc;
    for (int off = 1; off < 64; off <<= 1) {
      const cpx<T> Pn = shfl_down_c(P, off), Bn = shfl_down_c(B, off);
      if (lane + off < 64) {
        B = P * Bn + B;
        P = P * Pn;
      }
    }
    // e entering the wave from the right: the later waves' totals composed in order
    cpx<T> E = SEG ? cE : zero;
    if (wpl > 1) {
      if (lane == 0) {
        wP[wave] = P;
        wB[wave] = B;
      }
      __syncthreads();
      for (int s2 = wpl - 1; s2 > sub; --s2) E = wP[wave - sub + s2] * E + wB[wave - sub + s2];
    }
    const cpx<T> Pd = shfl_down_c(P, 1), Bd = shfl_down_c(B, 1);
    carry = lane == 63 ? E : Pd * E + Bd;         // e at the start of the next chunk
#pragma unroll
    for (int j = TS - 1; j >= 0; --j) {
      if (j < cnt) {
        carry = scl(fq[j], (T)0.5) * carry;
        d[j] = p[j] + (d[j] + carry);   // u
        p[j] = d[j];
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < TS; ++j)
      if (j < cnt) d[j] = p[j];
  }
  if constexpr (MODE != 0) {
    // sums of u (or of the stored state): |u|^2 and the differences, the last one with
    // the next chunk's first row (the next lane's, or the next wave's lane 0 through LDS;
    // after a segment's last row: the next segment's first, psi + e there)
    if constexpr (WI) wave_sync(); else __syncthreads();
    cpx<T> unext = shfl_down_c(d[0], 1);
    if (lane == 63 && cnt > 0 && i0 + cnt < N) unext = p[Sp];
    cpx<T> prev = zero;
#pragma unroll
    for (int j = 0; j < TS; ++j) {
      if (j < cnt) {
        s0 += abs2_d(d[j]);
        if (j > 0) s1 += absdiff2_d(d[j], prev);
        prev = d[j];
      }
    }
    if (cnt > 0 && i0 + cnt < N) s1 += absdiff2_d(unext, prev);
    if constexpr (SEG) {
      if (cnt > 0 && i0 + cnt == N && sgi + 1 < sg.nseg) s1 += absdiff2_d(eR + cE, prev);
    }
    double sv[2] = {s0, s1};
    gblock_sum<2>(sv, red);
    if (threadIdx.x == 0) {
      part[2 * blockIdx.x] = sv[0];
      part[2 * blockIdx.x + 1] = sv[1];
    }
  }
  if constexpr (NLM >= 0) {
    __syncthreads();  // red is reused
    gblock_sum<7>(q7, red);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < 7; ++k) nlz.part[7 * (long long)blockIdx.x + k] = q7[k];
    }
  }
  if constexpr (MODE != 2 && WI) {
    wave_sync();
    if (wv < nl) {
      for (int t = (int)(threadIdx.x & 63); t < N; t += 64) {
        const int c = (int)fdiv((uint32_t)t, fs);
        data[pbase + (long long)wv * N + t] = ps[wv * LS + c * Sp + (t - c * S)];
      }
    }
  } else if constexpr (MODE != 2) {
    __syncthreads();
    for (int t = threadIdx.x, r = 0; t < tot; t += nt, ++r) {
      int ln, e;
      long long a;
      if (packed) {
        ln = (int)fdiv((uint32_t)t, g.fn);
        e = t - ln * N;
        a = pbase + t;
      } else {
        ln = sl;
        e = se0 + sstep * r;
        a = sbase + (long long)e * g.se;
      }
      if (ln < nl) {
        const int c = (int)fdiv((uint32_t)e, fs);
        data[a] = ps[ln * LS + c * Sp + (e - c * S)];
      }
    }
  }
}

// Transpose of a rows x cols grid of complex values, out[c rows + r] = in[r cols + c],
// through TT x TT LDS tiles padded by one column (reads and writes both along rows).
template <typename T, int TT>
__global__ void __launch_bounds__(kThreads) kg_transpose(const cpx<T>* __restrict__ in,
                                                         cpx<T>* __restrict__ out, int rows,
                                                         int cols) {
  __shared__ cpx<T> tile[TT][TT + 1];
  constexpr int RY = kThreads / TT;
  const int c0 = blockIdx.x * TT, r0 = blockIdx.y * TT;
  const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;
#pragma unroll
  for (int k = ty; k < TT; k += RY) {
    const int r = r0 + k, c = c0 + tx;
    if (r < rows && c < cols) tile[k][tx] = in[(long long)r * cols + c];
  }
  __syncthreads();
#pragma unroll
  for (int k = ty; k < TT; k += RY) {
    const int c = c0 + k, r = r0 + tx;
    if (r < rows && c < cols) out[(long long)c * rows + r] = tile[tx][k];
  }
}

// Crank-Nicolson sweep of strided lines with many lines per sweep (3D y and z lines of
// more than 1024 points), one thread per line (line l: element e at
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
