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
// of n0/2+1 contiguous runs over k1 (coalesced when a tile owns several k1).
//
// Pass order of one 3D step (2D: r2c_x, conv_line, c2r_nl_cnx, cn_col, finalize):
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
//
// Every pass is a __device__ body working on one tile (index `bid`) with its LDS carved
// from a byte pointer, so the same body serves a single-grid kernel (one block per tile)
// and a persistent multi-instance kernel (blocks looping over tiles of many grids).
// lds_bytes<T, N, pass>() gives the bytes a body needs.
#pragma once
#include "gp_device.hpp"
#include "gp_finalize.hpp"

namespace gpdbec {

// Lines per tile for passes along x, columns per tile for strided passes.
// Tile-shape thresholds (compile-time; the defaults are the measured choice).
#ifndef GP_TJ_SPLIT_N
#define GP_TJ_SPLIT_N 256
#endif
#ifndef GP_TC_SPLIT_FP32
#define GP_TC_SPLIT_FP32 24
#endif
#ifndef GP_TC_SPLIT_FP64
#define GP_TC_SPLIT_FP64 8
#endif
#ifndef GP_LB_POINTS
#define GP_LB_POINTS 1024
#endif
#ifndef GP_TV_SPLIT_BYTES
#define GP_TV_SPLIT_BYTES 65536
#endif
#ifndef GP_R2C_WIDE
#define GP_R2C_WIDE 1
#endif

// S selects a tile-shape variant (the batched ensemble's autotuner chooses per pass and
// size class; the single-grid passes use S = 0):
//   S = 1: x tiles and CN column tiles of 8 lines (32 lanes per line) where the default
//          is 16, and line-FFT blocks of twice the default points.
// A variant only ever goes from 16 to 32 lanes per line: 32-lane solves compose the scan
// gains on the fly, so the factor table (whose gains are stored for the default lane
// count) serves both.
template <typename T, int N, int S = 0>
struct Tiles {
  // x lines per tile (even): 16, or 8 from GP_TJ_SPLIT_N points on (32 lanes per line:
  // half the serial chunk of the CN solve, twice the tiles)
  static constexpr int TJ0 = (N >= GP_TJ_SPLIT_N) ? 8 : 16;
  static constexpr int TJ = S == 1 ? 8 : TJ0;
  // x lines per tile of the single-grid R2C pass: FP64 256-point lines go 16 to a tile
  // (spectrum rows written in 256-byte runs) where the other x passes keep 8
  static constexpr int TJW = (GP_R2C_WIDE && sizeof(T) == 8 && N == 256 && S == 0) ? 16 : TJ;
  static constexpr int PX = kThreads / TJ;          // lanes per x line in the CN solve
  // columns per tile: 16, or 8 (32 lanes per line) when the 16-lane chunk would exceed
  // GP_TC_SPLIT_* elements
  static constexpr int TC0 =
      ((N + 15) / 16 > (sizeof(T) == 8 ? GP_TC_SPLIT_FP64 : GP_TC_SPLIT_FP32)) ? 8 : 16;
  static constexpr int TC = S == 1 ? 8 : TC0;
  static constexpr int PC = kThreads / TC;
  // columns per tile of the z convolution: 16, or 8 when a 16-column tile would take more
  // than GP_TV_SPLIT_BYTES of LDS (more resident blocks per CU).  256-point columns are
  // always 16 per tile: each thread keeps 16 points in registers (two 16-point stages
  // around one LDS exchange per direction).  In FP64 (CONV_SPLIT) the exchange moves the
  // real parts and then the imaginary parts through one real-valued buffer: 38.9 KB of
  // LDS instead of 73.7 KB, so that 16-column tiles (256-byte row runs) keep three
  // blocks per CU (registers bound them there) instead of two.
  static constexpr bool CONV_REG = (N == 256);
  static constexpr bool CONV_SPLIT = CONV_REG && sizeof(T) == 8;
  static constexpr int TV =
      (CONV_REG || (size_t)N * 17 * 2 * sizeof(T) <= (size_t)GP_TV_SPLIT_BYTES) ? 16 : 8;
  // contiguous lines per block of the line FFT passes
  static constexpr int LB0 = (GP_LB_POINTS / N) < 1 ? 1 : (GP_LB_POINTS / N);
  static constexpr int LB = S == 1 ? ((2 * GP_LB_POINTS / N) < 1 ? 1 : (2 * GP_LB_POINTS / N))
                                   : LB0;
  // lines per block of the y FFT pass: 16 for FP32 lines of 16 x 16 points (one 16-point
  // stage in registers on each side of a single LDS exchange), else LB
  static constexpr bool FFT16 = (N == 256 && sizeof(T) == 4);
  static constexpr int LBF = FFT16 ? 16 : LB;
};

// Workgroups are dispatched to the 8 XCDs round-robin (block b runs on XCD b % 8), and
// each XCD has its own L2.  The x passes and the z convolution renumber their tiles so
// that every XCD works through one contiguous range: neighbouring tiles, which read the
// two halves of the same 128-byte lines (spectrum lines of 8-line FP32 x tiles, kernel
// table rows of 16-column z tiles), then share an L2.
constexpr int kXcds = 8;
constexpr int kFinLead = kXcds;  // leading blocks that carry a folded finalisation
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int x = b % kXcds, i = b / kXcds, per = nb / kXcds, rem = nb % kXcds;
  return x * per + (x < rem ? x : rem) + i;
}

struct StepScalars {
  double dt;        // time step
  double gc;        // contact coupling (2D: includes 1/(sqrt(2 pi) d))
  double gdd;       // dipolar coupling
  double h0, h1, h2;  // spacings along axes 0, 1, 2
};

// MODE_ADJ: the adjoint sweep of a real-time step (A -> conj(A) = -i Ar).
enum : int { MODE_IMAG = 0, MODE_REAL = 1, MODE_OBSERVE = 2, MODE_PHI = 3, MODE_ADJ = 4 };

// CN coupling of one sweep: A = Ar (imaginary time) or A = i Ar (real time; its adjoint
// sweep: A = -i Ar).  The factor tables carry A; the sweep only needs to know whether it
// is complex.
template <int MODE>
constexpr bool cn_imag_a() { return MODE != MODE_IMAG; }

// Global-memory phases are statically unrolled over ITERS = ceil(elements/kThreads)
// so that every load of a thread is issued before the first one is consumed.
template <int TOTAL>
struct Iters {
  static constexpr int N = (TOTAL + kThreads - 1) / kThreads;
  __device__ static __forceinline__ bool valid(int u) { return TOTAL % kThreads == 0 || u < TOTAL; }
};

// ------------------------------------------------------------------ LDS carving
constexpr size_t a16(size_t b) { return (b + 15) & ~(size_t)15; }
struct Carve {
  char* p;
  template <typename X>
  __device__ __forceinline__ X* take(size_t n) {
    X* r = reinterpret_cast<X*>(p);
    p += a16(n * sizeof(X));
    return r;
  }
};

// Element `idx` of an array whose byte offset from `base` fits in 32 bits (every
// workspace array does: at most 512^3 complex doubles).  The 64-bit tile base is
// uniform, the 32-bit offset per lane, which maps onto scalar-base + vector-offset
// addressing instead of a 64-bit address computation per access.
template <typename X>
__device__ __forceinline__ X& at32(X* base, unsigned idx) {
  return *reinterpret_cast<X*>(reinterpret_cast<char*>(base) + idx * (unsigned)sizeof(X));
}
template <typename X>
__device__ __forceinline__ const X& at32(const X* base, unsigned idx) {
  return *reinterpret_cast<const X*>(reinterpret_cast<const char*>(base) +
                                     idx * (unsigned)sizeof(X));
}

// Two neighbouring complex values (the lines j, j + 1 of a packed pair), moved as one
// aligned access: j is even, so a pair starts on a 2 * sizeof(cpx<T>) boundary.
template <typename T>
struct alignas(2 * sizeof(cpx<T>)) cpx2 {
  cpx<T> a, b;
};

// Geometry of an x-line tile (TJ lines of N0 points; NP packed complex pairs).
template <typename T, int N0, int S = 0>
struct XT {
  static constexpr int TJ = Tiles<T, N0, S>::TJ, NP = TJ / 2, H = N0 / 2 + 1, LSZ = N0 + 1;
  static constexpr int PX = Tiles<T, N0, S>::PX, SX = (N0 + PX - 1) / PX;
  static constexpr int LSP = N0 + (N0 + SX - 1) / SX;  // chunk-padded line for CN
  static constexpr size_t C = sizeof(cpx<T>);
  static constexpr size_t Z = a16(NP * LSZ * C), W = a16(N0 * C), PS = a16(TJ * LSP * C),
                          MT = a16(cn_table_len<N0, PX>() * C),
                          RED = a16(8 * kWaves * sizeof(double)),
                          RED8 = a16(32 * kWaves * sizeof(double));  // block_sum_store8
  static constexpr size_t mx(size_t a, size_t b) { return a > b ? a : b; }
};

// Geometry of a strided-column CN tile (TC columns of N points).
template <typename T, int N, int S = 0>
struct CT {
  static constexpr int TC = Tiles<T, N, S>::TC, PC = Tiles<T, N, S>::PC, SC = (N + PC - 1) / PC;
  static constexpr int RS = TC + 1, NR = N + (N + SC - 1) / SC;  // padded rows
  static constexpr size_t C = sizeof(cpx<T>);
  static constexpr size_t B = a16(NR * RS * C), MT = a16(cn_table_len<N, PC>() * C),
                          RED = a16(8 * kWaves * sizeof(double));
};

// -------------------------------------------------------------------- LDS sizes
enum : int { P_R2C = 0, P_R2C_REAL, P_FFT_LINE, P_CONV_LINE, P_CONV_COL, P_C2R_STEP, P_C2R_OBS,
             P_CN_COL, P_ADJ_X, P_ADJ_FIN, P_R2C_W };
template <typename T, int N, int PASS, int S = 0>
constexpr size_t lds_bytes() {
  using X = XT<T, N, S>;
  using G = CT<T, N, S>;
  constexpr size_t C = sizeof(cpx<T>);
  constexpr int LB = Tiles<T, N, S>::LB, TC = Tiles<T, N, S>::TC;
  if (PASS == P_R2C) return X::Z + X::W + X::RED;
  if (PASS == P_R2C_W)
    return a16(Tiles<T, N, S>::TJW / 2 * X::LSZ * C) + X::W + X::RED;
  if (PASS == P_R2C_REAL) return X::Z + X::W;
  if (PASS == P_FFT_LINE)
    return Tiles<T, N>::FFT16 ? a16(16 * (N + N / 16) * C) + a16(N * C)
                              : a16(LB * (N + 1) * C) + a16(N * C);
  if (PASS == P_CONV_LINE) return a16(LB * (N + 1) * C) + a16(N * C);
  if (PASS == P_CONV_COL)
    return a16(N * (Tiles<T, N>::TV + 1) * (Tiles<T, N>::CONV_SPLIT ? sizeof(T) : C)) +
           a16(N * C);
  if (PASS == P_C2R_STEP) return X::mx(X::mx(X::Z, X::PS), X::RED8) + X::W + X::MT;
  if (PASS == P_ADJ_X) return X::Z + X::PS + X::W + X::MT + X::RED;
  if (PASS == P_C2R_OBS) return X::mx(X::Z, X::RED8) + X::W;
  if (PASS == P_CN_COL) return G::B + G::MT + G::RED;
  if (PASS == P_ADJ_FIN) return X::Z + X::W;
  return 0;
}

// ================================================================ pass bodies
// ---------------------------------------------------------------- r2c_x
// tiles: ceil(n1/TJ) * n2 (TJ = Tiles::TJW in the single-grid pass, Tiles::TJ in the
// batched one).  Spectrum of the stored |psi|^2 (unscaled: the convolution
// applies scale^2).  partials[bid*2 + {0,1}] = sum |dx psi|^2, sum |dy psi|^2 of the
// stored psi (unscaled), the y difference reaching one line past the tile.
// WIDE: the single-grid pass, with Tiles::TJW lines per tile.
template <typename T, int N0, int S = 0, bool WIDE = false>
__device__ __forceinline__ void r2c_x_body(const cpx<T>* __restrict__ psi,
                                           cpx<T>* __restrict__ spec,
                                           const cpx<T>* __restrict__ tw0,
                                           double* __restrict__ partials, int n1, int n2, int bid,
                                           char* lds) {
  using X = XT<T, N0, S>;
  constexpr int TJ = WIDE ? Tiles<T, N0, S>::TJW : X::TJ, NP = TJ / 2, H = X::H,
                LSZ = X::LSZ;
  using IT = Iters<TJ * N0>;
  Carve cv{lds};
  cpx<T>* Z = cv.take<cpx<T>>(NP * LSZ);
  cpx<T>* W = cv.take<cpx<T>>(N0);
  double* red = cv.take<double>(8 * kWaves);
  const int tid = thread_idx();
  const int nt1 = (n1 + TJ - 1) / TJ;
  const int k2 = bid / nt1;
  const int j0 = (bid % nt1) * TJ;
  const cpx<T>* plane = psi + (size_t)k2 * n1 * N0;
  // all loads first: the point, its x neighbour and its y neighbour (mostly cache hits)
  constexpr bool LANE_X = N0 == kThreads && sizeof(T) == 8;
  cpx<T> a[IT::N], bx[LANE_X ? 1 : IT::N], by[LANE_X ? 1 : IT::N];
  // per-thread partials in T (at most 16 points), FP64 above
  T ps[2] = {0, 0};
  if constexpr (LANE_X) {
    // lane = x index, register it = line j0 + it: the y neighbour is the next register
    // (one halo line loaded past the tile), the x neighbour the next lane (a wave shift;
    // the last lane of each wave loads its own, or reads it from LDS in 16-line tiles).
    // In FP64 this frees the registers that held the neighbours (8-line tiles: 3 -> 4
    // waves per SIMD); FP32 is faster with the plain loads.
    const cpx<T> z = {0, 0};
    const int i = tid;
    const bool last_lane = (tid & 63) == 63;
    // 16-line tiles keep rows past the grid as loaded (clamped) and mask what they feed,
    // and take the last lane's x neighbour from the next wave's first lane through LDS
    // (the twiddle buffer, filled afterwards) instead of loading it again
    constexpr bool EDGE_LDS = IT::N > 8;
#pragma unroll
    for (int it = 0; it < IT::N; ++it) {
      const int j = j0 + it;
      const int jc = min(j, n1 - 1);
      const cpx<T> l0 = at32(plane, (unsigned)(jc * N0 + i));
      a[it] = (EDGE_LDS || j < n1) ? l0 : z;
    }
    const cpx<T> halo = at32(plane, (unsigned)(min(j0 + IT::N, n1 - 1) * N0 + i));
    const int wv = tid >> 6;
    if constexpr (EDGE_LDS) {
      if ((tid & 63) == 0) {
#pragma unroll
        for (int it = 0; it < IT::N; ++it) W[wv * IT::N + it] = a[it];
      }
      __syncthreads();
    }
#pragma unroll
    for (int it = 0; it < IT::N; ++it) {
      const int j = j0 + it;
      const bool in = j < n1;
      // min(j + 1, n1 - 1): the next line if there is one, else the point itself
      const cpx<T> nxt = (it + 1 < IT::N) ? a[it + 1 < IT::N ? it + 1 : it] : halo;
      const cpx<T> byv = in ? csel(j + 1 <= n1 - 1, nxt, a[it]) : z;
      const cpx<T> sh = dpp<DPP_WAVE_SHL1>(a[it]);
      cpx<T> nb = sh;
      if (last_lane && i < N0 - 1) {
        // (rows past the grid are zeroed below whatever nb holds)
        if constexpr (EDGE_LDS) nb = W[(wv + 1) * IT::N + it];
        else nb = at32(plane, (unsigned)(min(j, n1 - 1) * N0 + i + 1));
      }
      const cpx<T> bxv = in ? csel(i < N0 - 1, nb, a[it]) : z;
      // the differences, partial sums and density of register it (line it, point i),
      // in the order of the general path below
      const cpx<T> dx = bxv - a[it], dy = byv - a[it];
      const T sx = dx.re * dx.re + dx.im * dx.im, sy = dy.re * dy.re + dy.im * dy.im;
      const T n2v = a[it].re * a[it].re + a[it].im * a[it].im;
      ps[0] += EDGE_LDS ? (in ? sx : (T)0) : sx;
      ps[1] += EDGE_LDS ? (in ? sy : (T)0) : sy;
      const T nv = EDGE_LDS ? (in ? n2v : (T)0) : n2v;
      cpx<T>& zc = Z[(it >> 1) * LSZ + i];
      if (it & 1) zc.im = nv;
      else zc.re = nv;
      // 16-line tiles: a scheduling fence between registers
      if constexpr (EDGE_LDS) __builtin_amdgcn_sched_barrier(0);
    }
  } else {
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    const int jl = u / N0, i = u % N0, j = j0 + jl;
    const cpx<T> z = {0, 0};
    const bool in = IT::valid(u) && j < n1;
    // clamped indices keep every load in bounds; at the last point of an axis the
    // neighbour is the point itself (zero difference), outside the grid all are zero
    const int jc = min(j, n1 - 1);
    const cpx<T> l0 = at32(plane, (unsigned)(jc * N0 + i));
    const cpx<T> l1 = at32(plane, (unsigned)(jc * N0 + min(i + 1, N0 - 1)));
    const cpx<T> l2 = at32(plane, (unsigned)(min(jc + 1, n1 - 1) * N0 + i));
    a[it] = in ? l0 : z;
    bx[it] = in ? l1 : z;
    by[it] = in ? l2 : z;
  }
  }
  if constexpr (LANE_X && IT::N > 8) __syncthreads();  // the edge values are read
  for (int i = tid; i < N0; i += kThreads) W[i] = tw0[i];
#pragma unroll
  for (int it = 0; it < (LANE_X ? 0 : IT::N); ++it) {
    const int u = tid + it * kThreads;
    if (!IT::valid(u)) continue;
    const int jl = u / N0, i = u % N0;
    const cpx<T> dx = bx[it] - a[it], dy = by[it] - a[it];
    ps[0] += dx.re * dx.re + dx.im * dx.im;
    ps[1] += dy.re * dy.re + dy.im * dy.im;
    const T nv = a[it].re * a[it].re + a[it].im * a[it].im;
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
    cpx<T>* sp = spec + (size_t)k2 * n1 + j0;  // uniform; + kx n2 n1 + 2p per lane
    const unsigned off = (unsigned)(kx * n2 * n1 + 2 * p);
    *reinterpret_cast<cpx2<T>*>(&at32(sp, off)) =
        cpx2<T>{{hf * (zk.re + zm.re), hf * (zk.im - zm.im)},
                {hf * (zk.im + zm.im), hf * (zm.re - zk.re)}};  // n1 even: line j+1 exists
  }
  double sums[2] = {(double)ps[0], (double)ps[1]};
  block_sum_store<2>(sums, red, partials + bid * 2);
}

// Real-to-complex x pass of a real field f (the adjoint's second convolution input).
template <typename T, int N0>
__device__ __forceinline__ void r2c_real_body(const T* __restrict__ f, cpx<T>* __restrict__ spec,
                                              const cpx<T>* __restrict__ tw0, int n1, int n2,
                                              int bid, char* lds) {
  using X = XT<T, N0>;
  constexpr int TJ = X::TJ, NP = X::NP, H = X::H, LSZ = X::LSZ;
  using IT = Iters<TJ * N0>;
  using IH = Iters<H * NP>;
  Carve cv{lds};
  cpx<T>* Z = cv.take<cpx<T>>(NP * LSZ);
  cpx<T>* W = cv.take<cpx<T>>(N0);
  const int tid = thread_idx();
  const int nt1 = (n1 + TJ - 1) / TJ;
  const int k2 = bid / nt1;
  const int j0 = (bid % nt1) * TJ;
  const size_t pbase = ((size_t)k2 * n1 + j0) * N0;
  T fv[IT::N];
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    fv[it] = (IT::valid(u) && j0 + u / N0 < n1) ? at32(f + pbase, (unsigned)u) : (T)0;
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
    cpx<T>* sp = spec + (size_t)k2 * n1 + j0;  // uniform; + kx n2 n1 + 2p per lane
    const unsigned off = (unsigned)(kx * n2 * n1 + 2 * p);
    *reinterpret_cast<cpx2<T>*>(&at32(sp, off)) =
        cpx2<T>{{hf * (zk.re + zm.re), hf * (zk.im - zm.im)},
                {hf * (zk.im + zm.im), hf * (zm.re - zk.re)}};  // n1 even: line j+1 exists
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
    const int u = thread_idx() + it * kThreads;
    const int l = u / N, i = u % N;
    v[it] = (IT::valid(u) && l0 + l < nlines) ? at32(data + (size_t)l0 * N, (unsigned)(l * N + i)) : cpx<T>{0, 0};
  }
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = thread_idx() + it * kThreads;
    if (IT::valid(u)) B[(u / N) * (N + 1) + u % N] = v[it];
  }
}

template <typename T, int N, int LB>
__device__ __forceinline__ void store_lines(const cpx<T>* B, cpx<T>* __restrict__ data, int l0,
                                            int nlines) {
  using IT = Iters<LB * N>;
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = thread_idx() + it * kThreads;
    const int l = u / N, i = u % N;
    if (IT::valid(u) && l0 + l < nlines) at32(data + (size_t)l0 * N, (unsigned)(l * N + i)) = B[l * (N + 1) + i];
  }
}

// ------------------------------------------------------------------ fft_line
// FFT of contiguous lines of length N (count nlines), LB lines per tile.
template <typename T, int N, bool INV>
__device__ __forceinline__ void fft_line_body(cpx<T>* __restrict__ data,
                                              const cpx<T>* __restrict__ tw, int nlines, int bid,
                                              char* lds) {
  if constexpr (Tiles<T, N>::FFT16) {
    // 16 lines of 16 x 16 points; thread (line l, g) holds points g + 16 m of its line.
    // First 16-point stage on the loaded values, one LDS exchange (line pitch 272: one
    // spare slot per 16 points keeps the stride-16 writes on distinct banks), second
    // stage with twiddles W^(g m), stored from registers: point g + 16 m again.
    constexpr int R = 16, LP = N + N / R;
    Carve cv{lds};
    cpx<T>* B = cv.take<cpx<T>>(R * LP);
    cpx<T>* W = cv.take<cpx<T>>(N);
    const int tid = thread_idx();
    const int l = tid / R, g = tid % R;
    const int line = bid * R + l;
    const bool in = line < nlines;
    cpx<T>* src = data + (size_t)bid * R * N;
    cpx<T> v[R];
#pragma unroll
    for (int m = 0; m < R; ++m)
      v[m] = in ? at32(src, (unsigned)(l * N + g + R * m)) : cpx<T>{0, 0};
    for (int i = tid; i < N; i += kThreads) W[i] = tw[i];
    dft<T, R, INV>(v);
    cpx<T>* b = B + l * LP;
#pragma unroll
    for (int m = 0; m < R; ++m) b[g * (R + 1) + m] = v[m];  // point R g + m, padded
    __syncthreads();
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const cpx<T> e = b[g + (R + 1) * m];  // point g + R m, padded
      const cpx<T> w = INV ? conjg(W[g * m]) : W[g * m];
      v[m] = (m == 0) ? e : e * w;
    }
    dft<T, R, INV>(v);
#pragma unroll
    for (int m = 0; m < R; ++m)
      if (in) at32(src, (unsigned)(l * N + g + R * m)) = v[m];
    return;
  }
  constexpr int LB = Tiles<T, N>::LB, LSZ = N + 1;
  Carve cv{lds};
  cpx<T>* B = cv.take<cpx<T>>(LB * LSZ);
  cpx<T>* W = cv.take<cpx<T>>(N);
  const int l0 = bid * LB;
  load_lines<T, N, LB>(B, data, l0, nlines);
  for (int i = thread_idx(); i < N; i += kThreads) W[i] = tw[i];
  __syncthreads();
  LdsFFT<T, N, LB, LSZ, 1, false>::template run<INV>(B, W);
  store_lines<T, N, LB>(B, data, l0, nlines);
}

// FFT -> multiply by the kernel table -> inverse FFT of contiguous lines (2D: y lines).
template <typename T, int N, int S = 0>
__device__ __forceinline__ void conv_line_body(cpx<T>* __restrict__ data,
                                               const T* __restrict__ ktab,
                                               const double* __restrict__ scale,
                                               const cpx<T>* __restrict__ tw, int nlines, int bid,
                                               char* lds) {
  constexpr int LB = Tiles<T, N, S>::LB, LSZ = N + 1;
  using IT = Iters<LB * N>;
  Carve cv{lds};
  cpx<T>* B = cv.take<cpx<T>>(LB * LSZ);
  cpx<T>* W = cv.take<cpx<T>>(N);
  const int tid = thread_idx();
  const int l0 = bid * LB;
  load_lines<T, N, LB>(B, data, l0, nlines);
  T kv[IT::N];  // kernel values: loaded now, used after the forward FFT
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    const int l = u / N, i = u % N;
    kv[it] = (IT::valid(u) && l0 + l < nlines) ? at32(ktab + (size_t)l0 * N, (unsigned)(l * N + i)) : (T)0;
  }
  const double sc = *scale;
  const T s2 = (T)(sc * sc);  // the density was transformed unscaled
  for (int i = tid; i < N; i += kThreads) W[i] = tw[i];
  __syncthreads();
  LdsFFT<T, N, LB, LSZ, 1, false>::template run<false>(B, W);
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    if (IT::valid(u)) {
      cpx<T>& e = B[(u / N) * LSZ + u % N];
      e = scl(e, kv[it] * s2);
    }
  }
  __syncthreads();
  LdsFFT<T, N, LB, LSZ, 1, false>::template run<true>(B, W);
  store_lines<T, N, LB>(B, data, l0, nlines);
}

// ------------------------------------------------------------------ conv_col
// The LDS exchange of the register path: register m of thread (column c, group g) is
// row g R + m of its column on the way in and row g + R m on the way out.  SPLIT sends
// the real parts and then the imaginary parts through one real-valued buffer (half the
// LDS, two more barriers).  The caller fences earlier reads of the buffer.
template <typename T, int R, int RS, bool SPLIT>
__device__ __forceinline__ void col_exchange(cpx<T> (&v)[R], char* buf, int c, int g) {
  if constexpr (SPLIT) {
    T* Br = reinterpret_cast<T*>(buf);
#pragma unroll
    for (int m = 0; m < R; ++m) Br[(g * R + m) * RS + c] = v[m].re;
    __syncthreads();
#pragma unroll
    for (int m = 0; m < R; ++m) v[m].re = Br[(g + R * m) * RS + c];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < R; ++m) Br[(g * R + m) * RS + c] = v[m].im;
    __syncthreads();
#pragma unroll
    for (int m = 0; m < R; ++m) v[m].im = Br[(g + R * m) * RS + c];
  } else {
    cpx<T>* B = reinterpret_cast<cpx<T>*>(buf);
#pragma unroll
    for (int m = 0; m < R; ++m) B[(g * R + m) * RS + c] = v[m];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = B[(g + R * m) * RS + c];
  }
}

// 3D z pass on the spectrum: lines along k2 (stride n1) inside each kx plane; a tile is
// TC consecutive k1 of one kx plane.  tiles: ceil(n1/TC) * H.
template <typename T, int N2>
__device__ __forceinline__ void conv_col_body(cpx<T>* __restrict__ spec,
                                              const T* __restrict__ ktab,
                                              const double* __restrict__ scale,
                                              const cpx<T>* __restrict__ tw2, int n1, int bid,
                                              char* lds) {
  constexpr int TC = Tiles<T, N2>::TV, RS = TC + 1;
  constexpr bool SPLIT = Tiles<T, N2>::CONV_SPLIT;
  using IT = Iters<N2 * TC>;
  Carve cv{lds};
  char* buf = cv.take<char>(N2 * RS * (SPLIT ? sizeof(T) : sizeof(cpx<T>)));
  cpx<T>* W = cv.take<cpx<T>>(N2);
  cpx<T>* B = reinterpret_cast<cpx<T>*>(buf);
  const int tid = thread_idx();
  const int nt = (n1 + TC - 1) / TC;
  const int kx = bid / nt;
  const int c0 = (bid % nt) * TC;
  const size_t plane = (size_t)kx * N2 * n1;
  // the kernel table holds the quadrant k1 <= n1/2, k2 <= N2/2 (U is even in both)
  const int H1 = n1 / 2 + 1;
  const T* kq = ktab + (size_t)kx * (N2 / 2 + 1) * H1;
  using FFT = LdsFFT<T, N2, TC, 1, RS, true>;
  constexpr int R = IT::N;
  constexpr bool REG = FFT::P.n == 2 && FFT::P.r[0] == R && FFT::P.r[1] == R &&
                      kThreads / TC == R && IT::N * kThreads == N2 * TC;
  static_assert(REG || !SPLIT, "the split exchange exists only on the register path");
  // kernel value of element `it` of this thread (row u / TC, column u % TC)
  auto kernel_value = [&](int it) -> T {
    const int u = tid + it * kThreads;
    const int c = u % TC, r = u / TC;
    const int k1 = c0 + c;
    const int k1r = min(k1, n1 - k1), k2r = min(r, N2 - r);
    return (IT::valid(u) && k1 < n1) ? at32(kq, (unsigned)(k2r * H1 + k1r)) : (T)0;
  };
  cpx<T> v[IT::N];
  T kv[IT::N];
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    const int c = u % TC, r = u / TC;
    const bool in = IT::valid(u) && c0 + c < n1;
    v[it] = in ? at32(spec + plane + c0, (unsigned)(r * n1 + c)) : cpx<T>{0, 0};
    kv[it] = kernel_value(it);
  }
  for (int i = tid; i < N2; i += kThreads) W[i] = tw2[i];
  {
    const double sc = *scale;
    const T s2 = (T)(sc * sc);  // the density was transformed unscaled
#pragma unroll
    for (int it = 0; it < IT::N; ++it) kv[it] *= s2;
  }
  if constexpr (REG) {
    // N2 = R * R with R points per thread at stride R (rows g + R m of column c): the
    // first forward stage works on the loaded registers, the second leaves spectrum
    // index g + R m in register m, where the kernel multiply and the first inverse stage
    // follow; the last inverse stage leaves row g + R m in register m for the store.
    // Two LDS exchanges per tile.
    const int c = tid % TC, g = tid / TC;
    dft<T, R, false>(v);
    col_exchange<T, R, RS, SPLIT>(v, buf, c, g);
#pragma unroll
    for (int m = 1; m < R; ++m) v[m] = v[m] * W[g * m];
    dft<T, R, false>(v);
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = scl(v[m], kv[m]);
    dft<T, R, true>(v);
    __syncthreads();  // every forward read of the buffer is done
    col_exchange<T, R, RS, SPLIT>(v, buf, c, g);
#pragma unroll
    for (int m = 1; m < R; ++m) v[m] = v[m] * conjg(W[g * m]);
    dft<T, R, true>(v);
#pragma unroll
    for (int m = 0; m < R; ++m)
      if (c0 + c < n1) at32(spec + plane + c0, (unsigned)((g + R * m) * n1 + c)) = v[m];
    return;
  }
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    if (IT::valid(u)) B[(u / TC) * RS + u % TC] = v[it];
  }
  __syncthreads();
  FFT::template run<false>(B, W);
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    if (IT::valid(u)) {
      cpx<T>& e = B[(u / TC) * RS + u % TC];
      e = scl(e, kv[it]);
    }
  }
  __syncthreads();
  FFT::template run<true>(B, W);
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    const int c = u % TC, r = u / TC;
    if (IT::valid(u) && c0 + c < n1) at32(spec + plane + c0, (unsigned)(r * n1 + c)) = B[r * RS + c];
  }
}

// ------------------------------------------------- spectrum of a line pair tile
template <typename T, int N0, int NP>
__device__ __forceinline__ void load_spec_pairs(const cpx<T>* __restrict__ spec, int j0, int k2,
                                                int n1, int n2,
                                                cpx<T> (&sa)[Iters<(N0 / 2 + 1) * NP>::N],
                                                cpx<T> (&sb)[Iters<(N0 / 2 + 1) * NP>::N]) {
  using IH = Iters<(N0 / 2 + 1) * NP>;
#pragma unroll
  for (int it = 0; it < IH::N; ++it) {
    const int u = thread_idx() + it * kThreads;
    const int p = u % NP, kx = u / NP;
    const int j = j0 + 2 * p;
    const bool in = IH::valid(u) && j < n1;
    const cpx2<T> v = in ? *reinterpret_cast<const cpx2<T>*>(
                               &at32(spec + (size_t)k2 * n1 + j0, (unsigned)(kx * n2 * n1 + 2 * p)))
                         : cpx2<T>{{0, 0}, {0, 0}};
    sa[it] = v.a;
    sb[it] = v.b;
  }
}

// Hermitian half spectra of the tile's line pairs -> full complex lines -> inverse x
// FFT: line jl of the tile then holds its real field in component (jl & 1) of
// Z[(jl >> 1) * (N0 + 1) + i].  Every thread must call this (block barriers inside).
template <typename T, int N0, int NP>
__device__ __forceinline__ void c2r_tile(cpx<T>* Z, const cpx<T>* W,
                                         const cpx<T> (&sa)[Iters<(N0 / 2 + 1) * NP>::N],
                                         const cpx<T> (&sb)[Iters<(N0 / 2 + 1) * NP>::N]) {
  constexpr int LSZ = N0 + 1, H = N0 / 2 + 1;
  using IH = Iters<H * NP>;
#pragma unroll
  for (int it = 0; it < IH::N; ++it) {
    const int u = thread_idx() + it * kThreads;
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

template <typename T>
__device__ __forceinline__ T tile_real(const cpx<T>* Z, int LSZ, int jl, int i) {
  const cpx<T> z = Z[(jl >> 1) * LSZ + i];
  return (jl & 1) ? z.im : z.re;
}

// ------------------------------------------------------------------ c2r_nl_cnx
// tiles: ceil(n1/TJ) * n2.  MODE_IMAG / MODE_REAL: full step pass (writes psi).
// MODE_OBSERVE: sums only.  MODE_PHI: writes Phi (without g_dd) to phi_out.
// partials[bid*7 + ...] = sum n, sum V n, sum n^2, sum Phi n, sum x^2 n, sum y^2 n,
// sum z^2 n of the incoming (scaled) state; axis coordinates (idx - n/2) h.
template <typename T, int N0, int MODE, int S = 0>
__device__ __forceinline__ void c2r_nl_cnx_body(
    cpx<T>* __restrict__ psi, const T* __restrict__ V, const double* __restrict__ scale,
    const cpx<T>* __restrict__ spec, const cpx<T>* __restrict__ tw0,
    const cpx<T>* __restrict__ cnm, const StepScalars& sc, double* __restrict__ partials,
    T* __restrict__ phi_out, int n1, int n2, int bid, char* lds) {
  using X = XT<T, N0, S>;
  constexpr int TJ = X::TJ, NP = X::NP, LSZ = X::LSZ, PX = X::PX, SX = X::SX, LSP = X::LSP;
  constexpr bool STEP = (MODE == MODE_IMAG || MODE == MODE_REAL);
  constexpr bool NEEDPSI = (MODE != MODE_PHI);
  using IT = Iters<TJ * N0>;
  using IH = Iters<(N0 / 2 + 1) * NP>;
  Carve cv{lds};
  // The step modes keep the CN lines in the FFT tile's memory (Phi is read into registers
  // before the first CN write): the smaller footprint lets more blocks share a CU.
  constexpr int ZL = NP * LSZ, PL = STEP ? TJ * LSP : 0;
  constexpr int RL = (int)(X::RED8 / sizeof(cpx<T>));  // the reduction's 32 per wave
  constexpr int TL = ZL > PL ? ZL : PL;
  cpx<T>* Z = cv.take<cpx<T>>(TL > RL ? TL : RL);
  cpx<T>* PS = STEP ? Z : nullptr;
  cpx<T>* W = cv.take<cpx<T>>(N0);
  cpx<T>* MT = STEP ? cv.take<cpx<T>>(cn_table_len<N0, PX>()) : nullptr;
  // the observables reduction at the end reuses the tile's memory
  double* red = reinterpret_cast<double*>(Z);
  const int tid = thread_idx();
  const int nt1 = (n1 + TJ - 1) / TJ;
  const int k2 = bid / nt1;
  const int j0 = (bid % nt1) * TJ;
  const size_t pbase = ((size_t)k2 * n1 + j0) * N0;  // first point of the tile
  // issue every global load of the tile up front: spectrum pairs, psi and V
  cpx<T> sa[IH::N], sb[IH::N];
  load_spec_pairs<T, N0, NP>(spec, j0, k2, n1, n2, sa, sb);
  cpx<T> pv[NEEDPSI ? IT::N : 1];
  T vv[NEEDPSI ? IT::N : 1];
  if constexpr (NEEDPSI) {
#pragma unroll
    for (int it = 0; it < IT::N; ++it) {
      const int u = tid + it * kThreads;
      const bool in = IT::valid(u) && j0 + u / N0 < n1;
      pv[it] = in ? at32(psi + pbase, (unsigned)u) : cpx<T>{0, 0};
      vv[it] = in ? at32(V + pbase, (unsigned)u) : (T)0;
    }
  }
  for (int i = tid; i < N0; i += kThreads) W[i] = tw0[i];
  if constexpr (STEP) load_cn_table<T, N0, PX>(MT, cnm);
  c2r_tile<T, N0, NP>(Z, W, sa, sb);

  if constexpr (MODE == MODE_PHI) {
#pragma unroll
    for (int it = 0; it < IT::N; ++it) {
      const int u = tid + it * kThreads;
      const int jl = u / N0, i = u % N0;
      if (IT::valid(u) && j0 + jl < n1) at32(phi_out + pbase, (unsigned)u) = tile_real(Z, LSZ, jl, i);
    }
  } else {
    // Each thread's partials over its IT::N points (at most 16) are formed in T, then
    // widened: the block and grid sums are FP64.  In FP32 an 8- or 16-term partial
    // carries an unbiased rounding of ~1e-7 of itself, far below the observables' bar.
    T ps[6] = {0, 0, 0, 0, 0, 0};
    // when N0 divides the block size every point of a thread has the same x index
    constexpr bool XFIX = kThreads % N0 == 0;
    const T ts = (T)(*scale);
    const T h0 = (T)sc.h0, h1 = (T)sc.h1;
    const double zc = (k2 - n2 / 2) * sc.h2;
    T phv[IT::N];
#pragma unroll
    for (int it = 0; it < IT::N; ++it) {
      const int u = tid + it * kThreads;
      phv[it] = IT::valid(u) ? tile_real(Z, LSZ, u / N0, u % N0) : (T)0;
    }
    if constexpr (STEP) __syncthreads();  // every Phi read before PS (= Z) is written
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
      const T phi = phv[it];
      const cpx<T> p = scl(pv[it], ts);
      const T v = vv[it];
      const T n = p.re * p.re + p.im * p.im;
      const T xc = (T)(i - N0 / 2) * h0, yc = (T)(j - n1 / 2) * h1;
      ps[0] += n;
      ps[1] += v * n;
      ps[2] += n * n;
      ps[3] += phi * n;
      if constexpr (!XFIX) ps[4] += xc * xc * n;
      ps[5] += yc * yc * n;
      if constexpr (STEP) {
        const T th = (T)sc.dt * (v + (T)sc.gc * n + (T)sc.gdd * phi);
        cpx<T> f;
        if constexpr (MODE == MODE_IMAG) {
          f = cpx<T>{exp(-th), (T)0};
        } else {
          T sn, cs;
          sincos_phase(th, sn, cs);
          f = cpx<T>{cs, -sn};
        }
        PS[jl * LSP + cpad<SX>(i)] = p * f;
      }
    }
    if constexpr (STEP) {
      __syncthreads();
      cn_solve_lines<T, N0, TJ, LSP, 1, PX, cn_imag_a<MODE>()>(PS, MT, cnm + N0);
#pragma unroll
      for (int it = 0; it < IT::N; ++it) {
        const int u = tid + it * kThreads;
        const int jl = u / N0, i = u % N0;
        if (IT::valid(u) && j0 + jl < n1) at32(psi + pbase, (unsigned)u) = PS[jl * LSP + cpad<SX>(i)];
      }
    }
    if constexpr (XFIX) {  // one x per thread: sum x^2 n = x^2 sum n
      const T xc = (T)(tid % N0 - N0 / 2) * h0;
      ps[4] = xc * xc * ps[0];
    }
    // the block reduction of the observables sums comes last, off the solve's path; the
    // tile (the reduction's LDS) is free once every thread has passed the barrier, and
    // sum z^2 n is zc^2 times the block's sum n (zc is one value per tile)
    double sums[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) sums[k] = (double)ps[k];
    __syncthreads();
    const double total = block_sum_store8<6>(sums, red, partials + bid * 7);
    if (tid == 0) partials[bid * 7 + 6] = zc * zc * total;  // thread 0 holds sum n
  }
}

// --------------------------------------------------------------------- cn_col
// CN sweep along a strided axis: lines of length N with element stride `estride`; a
// tile is TC consecutive x columns (x0..x0+TC-1) of one "outer" index.
//   y sweep (3D/2D): estride = n0, outer = k2 (n_outer = n2), ostride = n1*n0
//   z sweep (3D):    estride = n0*n1, outer = k1 (n_outer = n1), ostride = n0
// SUMS: also partials[bid*2+{0,1}] = sum |u|^2, sum |u_{i+1}-u_i|^2 along the line of
// the result (MODE_OBSERVE: of the stored input, nothing written; sums unscaled).
// tiles: ceil(n0/TC) * n_outer.
template <typename T, int N, int MODE, bool SUMS, int S = 0>
__device__ __forceinline__ void cn_col_body(cpx<T>* __restrict__ psi,
                                            const cpx<T>* __restrict__ cnm,
                                            double* __restrict__ partials, int n0,
                                            size_t estride, size_t ostride, int bid, char* lds) {
  using G = CT<T, N, S>;
  constexpr int TC = G::TC, PC = G::PC, SC = G::SC, RS = G::RS;
  constexpr bool SOLVE = (MODE == MODE_IMAG || MODE == MODE_REAL || MODE == MODE_ADJ);
  using IT = Iters<N * TC>;
  Carve cv{lds};
  cpx<T>* B = cv.take<cpx<T>>(G::NR * RS);
  cpx<T>* MT = cv.take<cpx<T>>(cn_table_len<N, PC>());
  double* red = cv.take<double>(8 * kWaves);
  const int tid = thread_idx();
  const int nt = (n0 + TC - 1) / TC;
  const int outer = bid / nt;
  const int x0 = (bid % nt) * TC;
  cpx<T>* base = psi + (size_t)outer * ostride + x0;
  cpx<T> v[IT::N];
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    const int c = u % TC, r = u / TC;
    const unsigned es = (unsigned)estride;
    v[it] = (IT::valid(u) && x0 + c < n0) ? at32(base, r * es + c) : cpx<T>{0, 0};
  }
  if constexpr (SOLVE) load_cn_table<T, N, PC>(MT, cnm);
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    if (IT::valid(u)) B[cpad<SC>(u / TC) * RS + u % TC] = v[it];
  }
  __syncthreads();
  if constexpr (SOLVE) {
    cn_solve_lines<T, N, TC, 1, RS, PC, cn_imag_a<MODE>()>(B, MT, cnm + N);
  }
  double sums[2] = {0.0, 0.0};
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    const int c = u % TC, r = u / TC;
    if (!IT::valid(u) || x0 + c >= n0) continue;
    const cpx<T> val = B[cpad<SC>(r) * RS + c];
    if constexpr (SOLVE) at32(base, r * (unsigned)estride + c) = val;
    if constexpr (SUMS) {
      sums[0] += abs2_d(val);
      if (r + 1 < N) sums[1] += absdiff2_d(B[cpad<SC>(r + 1) * RS + c], val);
    }
  }
  if constexpr (SUMS) block_sum_store<2>(sums, red, partials + bid * 2);
}

// ============================================================ adjoint bodies
// Backpropagation through one real-time step (costate lambda = dL/d conj(psi)):
//   lambda_a = C_x(-dt) C_y(-dt) C_z(-dt) lambda      (adjoint of each CN factor)
//   mu = exp(+i dt theta) lambda_a,  theta = V + g_c n + g_dd Phi  (of psi_n)
//   s  = 2 dt Im(conj(mu) psi_n);   dL/dV += s;  sums s n, s Phi -> dL/dg_c, dL/dg_dd
//   lambda_n = mu + (g_c s + g_dd K s) psi_n,  K s = F^-1[U F[s]]

// Adjoint x pass: lambda_a = C_x(-dt) lambda (conjugate factors), Phi of psi_n from the
// spectrum, mu -> lam, s -> sfield, gradV += s (FP64), partials[bid*2 + {0,1}] =
// sum s n, sum s Phi.  tiles: ceil(n1/TJ) * n2.
template <typename T, int N0>
__device__ __forceinline__ void adj_x_body(
    cpx<T>* __restrict__ lam, const cpx<T>* __restrict__ psin, const T* __restrict__ V,
    const cpx<T>* __restrict__ spec, const cpx<T>* __restrict__ tw0,
    const cpx<T>* __restrict__ cnm, const StepScalars& sc, T* __restrict__ sfield,
    double* __restrict__ gradV, double* __restrict__ partials, int n1, int n2, int bid,
    char* lds) {
  using X = XT<T, N0>;
  constexpr int TJ = X::TJ, NP = X::NP, LSZ = X::LSZ, PX = X::PX, SX = X::SX, LSP = X::LSP;
  using IT = Iters<TJ * N0>;
  using IH = Iters<(N0 / 2 + 1) * NP>;
  Carve cv{lds};
  cpx<T>* Z = cv.take<cpx<T>>(NP * LSZ);
  cpx<T>* PS = cv.take<cpx<T>>(TJ * LSP);
  cpx<T>* W = cv.take<cpx<T>>(N0);
  cpx<T>* MT = cv.take<cpx<T>>(cn_table_len<N0, PX>());
  double* red = cv.take<double>(8 * kWaves);
  const int tid = thread_idx();
  const int nt1 = (n1 + TJ - 1) / TJ;
  const int k2 = bid / nt1;
  const int j0 = (bid % nt1) * TJ;
  const size_t pbase = ((size_t)k2 * n1 + j0) * N0;
  cpx<T> sa[IH::N], sb[IH::N];
  load_spec_pairs<T, N0, NP>(spec, j0, k2, n1, n2, sa, sb);
  cpx<T> lv[IT::N], pv[IT::N];
  T vv[IT::N];
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    const bool in = IT::valid(u) && j0 + u / N0 < n1;
    lv[it] = in ? at32(lam + pbase, (unsigned)u) : cpx<T>{0, 0};
    pv[it] = in ? at32(psin + pbase, (unsigned)u) : cpx<T>{0, 0};
    vv[it] = in ? at32(V + pbase, (unsigned)u) : (T)0;
  }
  for (int i = tid; i < N0; i += kThreads) W[i] = tw0[i];
  load_cn_table<T, N0, PX>(MT, cnm);
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    if (IT::valid(u)) PS[(u / N0) * LSP + cpad<SX>(u % N0)] = lv[it];
  }
  c2r_tile<T, N0, NP>(Z, W, sa, sb);  // ends with a barrier
  cn_solve_lines<T, N0, TJ, LSP, 1, PX, true>(PS, MT, cnm + N0);
  double sums[2] = {0.0, 0.0};
  const T dt = (T)sc.dt;
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    if (!IT::valid(u)) continue;
    const int jl = u / N0, i = u % N0;
    if (j0 + jl >= n1) continue;
    const T phi = tile_real(Z, LSZ, jl, i);
    const cpx<T> p = pv[it];
    const T n = p.re * p.re + p.im * p.im;
    const T th = dt * (vv[it] + (T)sc.gc * n + (T)sc.gdd * phi);
    const cpx<T> la = PS[jl * LSP + cpad<SX>(i)];
    T sn, cs;
    sincos_phase(th, sn, cs);
    const cpx<T> mu = la * cpx<T>{cs, sn};
    const T s = (T)2 * dt * (mu.re * p.im - mu.im * p.re);
    at32(lam + pbase, (unsigned)u) = mu;
    at32(sfield + pbase, (unsigned)u) = s;
    at32(gradV + pbase, (unsigned)u) += (double)s;
    sums[0] += (double)s * (double)n;
    sums[1] += (double)s * (double)phi;
  }
  block_sum_store<2>(sums, red, partials + bid * 2);
}

// Adjoint closing x pass: K s from the spectrum; lambda = mu + (g_c s + g_dd K s) psi_n.
template <typename T, int N0>
__device__ __forceinline__ void adj_fin_body(cpx<T>* __restrict__ lam,
                                             const cpx<T>* __restrict__ psin,
                                             const T* __restrict__ sfield,
                                             const cpx<T>* __restrict__ spec,
                                             const cpx<T>* __restrict__ tw0,
                                             const StepScalars& sc, int n1, int n2, int bid,
                                             char* lds) {
  using X = XT<T, N0>;
  constexpr int TJ = X::TJ, NP = X::NP, LSZ = X::LSZ;
  using IT = Iters<TJ * N0>;
  using IH = Iters<(N0 / 2 + 1) * NP>;
  Carve cv{lds};
  cpx<T>* Z = cv.take<cpx<T>>(NP * LSZ);
  cpx<T>* W = cv.take<cpx<T>>(N0);
  const int tid = thread_idx();
  const int nt1 = (n1 + TJ - 1) / TJ;
  const int k2 = bid / nt1;
  const int j0 = (bid % nt1) * TJ;
  const size_t pbase = ((size_t)k2 * n1 + j0) * N0;
  cpx<T> sa[IH::N], sb[IH::N];
  load_spec_pairs<T, N0, NP>(spec, j0, k2, n1, n2, sa, sb);
  cpx<T> mv[IT::N], pv[IT::N];
  T sv[IT::N];
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    const bool in = IT::valid(u) && j0 + u / N0 < n1;
    mv[it] = in ? at32(lam + pbase, (unsigned)u) : cpx<T>{0, 0};
    pv[it] = in ? at32(psin + pbase, (unsigned)u) : cpx<T>{0, 0};
    sv[it] = in ? at32(sfield + pbase, (unsigned)u) : (T)0;
  }
  for (int i = tid; i < N0; i += kThreads) W[i] = tw0[i];
  c2r_tile<T, N0, NP>(Z, W, sa, sb);
#pragma unroll
  for (int it = 0; it < IT::N; ++it) {
    const int u = tid + it * kThreads;
    if (!IT::valid(u)) continue;
    const int jl = u / N0, i = u % N0;
    if (j0 + jl >= n1) continue;
    const T w = (T)sc.gc * sv[it] + (T)sc.gdd * tile_real(Z, LSZ, jl, i);
    at32(lam + pbase, (unsigned)u) = mv[it] + scl(pv[it], w);
  }
}

// ========================================================= single-grid kernels
// One block per tile; static LDS sized for the pass.
#define GP_LDS(T, N, PASS) __shared__ __attribute__((aligned(16))) char lds[lds_bytes<T, N, PASS>()]

template <typename T, int N0>
__global__ __launch_bounds__(kThreads) void k_r2c_x(const cpx<T>* __restrict__ psi,
                                                    cpx<T>* __restrict__ spec,
                                                    const cpx<T>* __restrict__ tw0,
                                                    double* __restrict__ partials, int n1, int n2) {
  GP_LDS(T, N0, P_R2C_W);
  r2c_x_body<T, N0, 0, true>(psi, spec, tw0, partials, n1, n2, xcd_tile(blockIdx.x, gridDim.x),
                             lds);
}

// The x R2C of a step with the previous step's finalisation folded in: that finalisation
// reads the previous step's partials, which this pass does not write, and writes the
// scale, which this pass does not read (the convolution applies it).  The first nlead
// blocks (a multiple of 8, so that the tiles keep their XCD placement) carry it: nfin of
// them run the finalize block or the first-stage slices, the others return; the
// remaining blocks are the tiles.
template <typename T, int N0, int FIN_MODE>
__global__ __launch_bounds__(kThreads) void k_r2c_x_fin(const cpx<T>* __restrict__ psi,
                                                        cpx<T>* __restrict__ spec,
                                                        const cpx<T>* __restrict__ tw0,
                                                        double* __restrict__ partials, int n1,
                                                        int n2, FinArgs fa, int nfin,
                                                        int nlead) {
  GP_LDS(T, N0, P_R2C_W);
  const int b = blockIdx.x;
  if (b < nlead) {
    if (b < nfin) {
      if (fa.nstage > 0) prereduce_block<1>(fa, FIN_MODE, b);
      else finalize_block<1>(fa, FIN_MODE);
    }
    return;
  }
  r2c_x_body<T, N0, 0, true>(psi, spec, tw0, partials, n1, n2,
                             xcd_tile(b - nlead, gridDim.x - nlead), lds);
}

template <typename T, int N0>
__global__ __launch_bounds__(kThreads) void k_r2c_real(const T* __restrict__ f,
                                                       cpx<T>* __restrict__ spec,
                                                       const cpx<T>* __restrict__ tw0, int n1,
                                                       int n2) {
  GP_LDS(T, N0, P_R2C_REAL);
  r2c_real_body<T, N0>(f, spec, tw0, n1, n2, xcd_tile(blockIdx.x, gridDim.x), lds);
}

template <typename T, int N, bool INV>
__global__ __launch_bounds__(kThreads) void k_fft_line(cpx<T>* __restrict__ data,
                                                       const cpx<T>* __restrict__ tw, int nlines) {
  GP_LDS(T, N, P_FFT_LINE);
  fft_line_body<T, N, INV>(data, tw, nlines, blockIdx.x, lds);
}

// Forward y FFT with the second stage of a two-stage folded finalisation (see
// k_r2c_x_fin) in its first block; blocks 1-7 return, the rest are the lines.
template <typename T, int N, int FIN_MODE>
__global__ __launch_bounds__(kThreads) void k_fft_line_fin(cpx<T>* __restrict__ data,
                                                           const cpx<T>* __restrict__ tw,
                                                           int nlines, FinArgs fa) {
  GP_LDS(T, N, P_FFT_LINE);
  const int b = blockIdx.x;
  if (b < kFinLead) {
    if (b == 0) finalize_block<1>(fa, FIN_MODE);
    return;
  }
  fft_line_body<T, N, false>(data, tw, nlines, b - kFinLead, lds);
}

template <typename T, int N>
__global__ __launch_bounds__(kThreads) void k_conv_line(cpx<T>* __restrict__ data,
                                                        const T* __restrict__ ktab,
                                                        const double* __restrict__ scale,
                                                        const cpx<T>* __restrict__ tw, int nlines) {
  GP_LDS(T, N, P_CONV_LINE);
  conv_line_body<T, N>(data, ktab, scale, tw, nlines, blockIdx.x, lds);
}

template <typename T, int N2>
__global__ __launch_bounds__(kThreads) void k_conv_col(cpx<T>* __restrict__ spec,
                                                       const T* __restrict__ ktab,
                                                       const double* __restrict__ scale,
                                                       const cpx<T>* __restrict__ tw2, int n1) {
  GP_LDS(T, N2, P_CONV_COL);
  conv_col_body<T, N2>(spec, ktab, scale, tw2, n1, xcd_tile(blockIdx.x, gridDim.x), lds);
}

template <typename T, int N0, int MODE>
__global__ __launch_bounds__(kThreads) void k_c2r_nl_cnx(
    cpx<T>* __restrict__ psi, const T* __restrict__ V, const double* __restrict__ scale,
    const cpx<T>* __restrict__ spec, const cpx<T>* __restrict__ tw0,
    const cpx<T>* __restrict__ cnm, StepScalars sc, double* __restrict__ partials,
    T* __restrict__ phi_out, int n1, int n2, unsigned long long* __restrict__ stamps) {
  GP_LDS(T, N0, ((MODE == MODE_IMAG || MODE == MODE_REAL) ? P_C2R_STEP : P_C2R_OBS));
  // optional wall-clock stamps of the block's start and end (kernel-span timing)
  if (stamps != nullptr && threadIdx.x == 0) stamps[2 * blockIdx.x] = wall_clock64();
  c2r_nl_cnx_body<T, N0, MODE>(psi, V, scale, spec, tw0, cnm, sc, partials, phi_out, n1, n2,
                               xcd_tile(blockIdx.x, gridDim.x), lds);
  if (stamps != nullptr) {
    __syncthreads();
    if (threadIdx.x == 0) stamps[2 * blockIdx.x + 1] = wall_clock64();
  }
}

template <typename T, int N, int MODE, bool SUMS>
__global__ __launch_bounds__(kThreads) void k_cn_col(cpx<T>* __restrict__ psi,
                                                     const cpx<T>* __restrict__ cnm,
                                                     double* __restrict__ partials,
                                                     int n0, size_t estride, size_t ostride) {
  GP_LDS(T, N, P_CN_COL);
  cn_col_body<T, N, MODE, SUMS>(psi, cnm, partials, n0, estride, ostride, blockIdx.x, lds);
}

template <typename T, int N0>
__global__ __launch_bounds__(kThreads) void k_adj_x(
    cpx<T>* __restrict__ lam, const cpx<T>* __restrict__ psin, const T* __restrict__ V,
    const cpx<T>* __restrict__ spec, const cpx<T>* __restrict__ tw0,
    const cpx<T>* __restrict__ cnm, StepScalars sc, T* __restrict__ sfield,
    double* __restrict__ gradV, double* __restrict__ partials, int n1, int n2) {
  GP_LDS(T, N0, P_ADJ_X);
  adj_x_body<T, N0>(lam, psin, V, spec, tw0, cnm, sc, sfield, gradV, partials, n1, n2,
                    xcd_tile(blockIdx.x, gridDim.x), lds);
}

template <typename T, int N0>
__global__ __launch_bounds__(kThreads) void k_adj_fin(cpx<T>* __restrict__ lam,
                                                      const cpx<T>* __restrict__ psin,
                                                      const T* __restrict__ sfield,
                                                      const cpx<T>* __restrict__ spec,
                                                      const cpx<T>* __restrict__ tw0,
                                                      StepScalars sc, int n1, int n2) {
  GP_LDS(T, N0, P_ADJ_FIN);
  adj_fin_body<T, N0>(lam, psin, sfield, spec, tw0, sc, n1, n2, xcd_tile(blockIdx.x, gridDim.x),
                      lds);
}

#undef GP_LDS

}  // namespace gpdbec
