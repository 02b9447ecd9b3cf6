// Device building blocks for the dipolar GP split-step Crank-Nicolson step on gfx950:
//   * cpx<T>            interleaved complex value (float or double)
//   * LdsFFT            batched mixed-radix (2, 3, 4, 5) Stockham FFT of lines held in LDS
//   * cn_solve_lines    constant-coefficient tridiagonal Crank-Nicolson solves of lines in
//                       LDS, several lanes per line, exact chunked scan of the two Thomas
//                       recurrences across the lanes (DPP lane moves)
//   * block_sum         deterministic FP64 block reductions
// All kernels run with 256 threads per block (4 wave64s).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace gpdbec {

constexpr int kThreads = 256;

// Thread index in the block.  The translation unit of the persistent batched kernels
// (which loop over work items) defines GP_ITEM_LOOP_KERNELS: there every use goes through
// an empty volatile asm and yields a fresh value, so each item recomputes its index
// arithmetic instead of the compiler hoisting all of it out of the item loop, where it
// would stay live across items and exhaust the registers.  Elsewhere it is plain, and
// the index arithmetic is shared across a kernel.
__device__ __forceinline__ int thread_idx() {
  int t = (int)threadIdx.x;
#ifdef GP_ITEM_LOOP_KERNELS
  asm volatile("" : "+v"(t));
#endif
  return t;
}

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cpx<T> mk(T r, T i) { return cpx<T>{r, i}; }
template <typename T>
__device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cpx<T> operator*(cpx<T> a, cpx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cpx<T> scl(cpx<T> a, T s) { return {a.re * s, a.im * s}; }
template <typename T>
__device__ __forceinline__ cpx<T> conjg(cpx<T> a) { return {a.re, -a.im}; }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__device__ __forceinline__ cpx<T> mul_mi(cpx<T> a) {
  return INV ? cpx<T>{-a.im, a.re} : cpx<T>{a.im, -a.re};
}

// |a|^2 with the operands widened to double first (reductions accumulate in FP64).
template <typename T>
__device__ __forceinline__ double abs2_d(cpx<T> a) {
  const double r = (double)a.re, i = (double)a.im;
  return r * r + i * i;
}
template <typename T>
__device__ __forceinline__ double absdiff2_d(cpx<T> a, cpx<T> b) {
  const double r = (double)a.re - (double)b.re, i = (double)a.im - (double)b.im;
  return r * r + i * i;
}

// ------------------------------------------------------------------ radix plan
struct RadixPlan {
  int n;
  int r[16];
};
// Radices of a Stockham plan for length N: powers of two up to RMAX (16, 8 or 4) first,
// then 2, 3, 5.
constexpr RadixPlan make_plan(int N, int RMAX = 4) {
  RadixPlan p{0, {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}};
  int m = N;
  if (RMAX >= 16)
    while (m % 16 == 0) { p.r[p.n++] = 16; m /= 16; }
  if (RMAX >= 8)
    while (m % 8 == 0) { p.r[p.n++] = 8; m /= 8; }
  while (m % 4 == 0) { p.r[p.n++] = 4; m /= 4; }
  while (m % 2 == 0) { p.r[p.n++] = 2; m /= 2; }
  while (m % 3 == 0) { p.r[p.n++] = 3; m /= 3; }
  while (m % 5 == 0) { p.r[p.n++] = 5; m /= 5; }
  return p;
}
constexpr bool plan_ok(int N) {
  int m = N;
  while (m % 2 == 0) m /= 2;
  while (m % 3 == 0) m /= 3;
  while (m % 5 == 0) m /= 5;
  return m == 1;
}
constexpr int plan_span(int N, int s, int RMAX = 4) {  // product of the radices before stage s
  RadixPlan p = make_plan(N, RMAX);
  int L = 1;
  for (int i = 0; i < s; ++i) L *= p.r[i];
  return L;
}

// -------------------------------------------------------------- small DFTs
template <typename T, bool INV>
__device__ __forceinline__ void dft2(cpx<T>* x) {
  const cpx<T> a = x[0], b = x[1];
  x[0] = a + b;
  x[1] = a - b;
}
template <typename T, bool INV>
__device__ __forceinline__ void dft4(cpx<T>* x) {
  const cpx<T> s02 = x[0] + x[2], d02 = x[0] - x[2];
  const cpx<T> s13 = x[1] + x[3], d13 = mul_mi<T, INV>(x[1] - x[3]);
  x[0] = s02 + s13;
  x[2] = s02 - s13;
  x[1] = d02 + d13;
  x[3] = d02 - d13;
}
template <typename T, bool INV>
__device__ __forceinline__ void dft3(cpx<T>* x) {
  // W3 = exp(-2 pi i/3) = -1/2 - i sqrt(3)/2 (forward)
  const T h = (T)0.5;
  const T s = INV ? (T)-0.86602540378443864676 : (T)0.86602540378443864676;
  const cpx<T> t1 = x[1] + x[2], t2 = x[1] - x[2];
  const cpx<T> m = x[0] - scl(t1, h);
  const cpx<T> r = {s * t2.im, -s * t2.re};  // -i s t2
  x[0] = x[0] + t1;
  x[1] = m + r;
  x[2] = m - r;
}
template <typename T, bool INV>
__device__ __forceinline__ void dft5(cpx<T>* x) {
  const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
  const T s1 = INV ? (T)-0.95105651629515357212 : (T)0.95105651629515357212;
  const T s2 = INV ? (T)-0.58778525229247312917 : (T)0.58778525229247312917;
  const cpx<T> t1 = x[1] + x[4], t2 = x[2] + x[3];
  const cpx<T> t3 = x[1] - x[4], t4 = x[2] - x[3];
  const cpx<T> a1 = x[0] + scl(t1, c1) + scl(t2, c2);
  const cpx<T> a2 = x[0] + scl(t1, c2) + scl(t2, c1);
  const cpx<T> u1 = scl(t3, s1) + scl(t4, s2);   // multiplied by -i below
  const cpx<T> u2 = scl(t3, s2) - scl(t4, s1);
  const cpx<T> b1 = {u1.im, -u1.re};
  const cpx<T> b2 = {u2.im, -u2.re};
  x[0] = x[0] + t1 + t2;
  x[1] = a1 + b1;
  x[4] = a1 - b1;
  x[2] = a2 + b2;
  x[3] = a2 - b2;
}
// exp(-2 pi i e/16) for 0 <= e < 16 (forward sign; INV conjugates).
template <typename T, bool INV>
__device__ __forceinline__ cpx<T> w16(int e) {
  constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173;  // pi/8
  constexpr double h = 0.70710678118654752440;                                // pi/4
  constexpr double cs[16] = {1, c1, h, s1, 0, -s1, -h, -c1, -1, -c1, -h, -s1, 0, s1, h, c1};
  const double c = cs[e & 15], sn = cs[(e + 12) & 15];  // sin(a) = cos(a - pi/2)
  return cpx<T>{(T)c, INV ? (T)sn : (T)-sn};
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dft(cpx<T>* x);

// DFT of length R = R1 R2 from DFTs of lengths R1 and R2 (R divides 16): with
// n = R2 n1 + n2 and k = k1 + R1 k2,
//   X[k1 + R1 k2] = sum_n2 W_R2^(n2 k2) W_R^(n2 k1) sum_n1 W_R1^(n1 k1) x[R2 n1 + n2].
template <typename T, int R1, int R2, bool INV>
__device__ __forceinline__ void dft_split(cpx<T>* x) {
  constexpr int R = R1 * R2;
  cpx<T> y[R2][R1];
#pragma unroll
  for (int n2 = 0; n2 < R2; ++n2) {
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) y[n2][n1] = x[R2 * n1 + n2];
    dft<T, R1, INV>(y[n2]);
#pragma unroll
    for (int k1 = 1; k1 < R1; ++k1)
      if (n2 > 0) y[n2][k1] = y[n2][k1] * w16<T, INV>((16 / R) * n2 * k1);
  }
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) {
    cpx<T> b[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) b[n2] = y[n2][k1];
    dft<T, R2, INV>(b);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) x[k1 + R1 * k2] = b[k2];
  }
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dft(cpx<T>* x) {
  if constexpr (R == 2) dft2<T, INV>(x);
  else if constexpr (R == 3) dft3<T, INV>(x);
  else if constexpr (R == 4) dft4<T, INV>(x);
  else if constexpr (R == 5) dft5<T, INV>(x);
  else if constexpr (R == 8) dft_split<T, 4, 2, INV>(x);
  else dft_split<T, 4, 4, INV>(x);
}

// --------------------------------------------------------------- LDS FFT
// NL lines of length N live in LDS; element (line l, index i) at buf[l*LS + i*ES].
// tw[k] = exp(-2 pi i k/N), k < N, in LDS.  LINE_FAST selects which of (line,
// butterfly) varies fastest across threads: true for column tiles (LS = 1), false for
// contiguous rows (ES = 1), so that neighbouring lanes touch neighbouring addresses.
// Every thread of the block must call run(); it synchronises the block internally and
// returns after a final barrier.  Forward: unnormalised exp(-i...); INV: exp(+i...).
template <typename T, int N, int NL, int LS, int ES, bool LINE_FAST>
struct LdsFFT {
  // Radices up to 16 while every thread still has a butterfly of each stage (a block of
  // NL lines of N points); never below 4.
  static constexpr int RMAX = (NL * N >= 16 * kThreads) ? 16 : (NL * N >= 8 * kThreads) ? 8 : 4;
  static constexpr RadixPlan P = make_plan(N, RMAX);
  static_assert(plan_ok(N), "FFT length must factor into 2, 3, 5");

  template <int S, bool INV>
  __device__ static __forceinline__ void stage(cpx<T>* buf, const cpx<T>* tw) {
    if constexpr (S < P.n) {
      constexpr int R = P.r[S];
      constexpr int L = plan_span(N, S, RMAX);
      constexpr int NB = N / R;                 // butterflies per line
      constexpr int TOT = NL * NB;
      constexpr int IT = (TOT + kThreads - 1) / kThreads;
      constexpr int TWS = N / (L * R);
      cpx<T> v[IT][R];
      const int tid = thread_idx();
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int u = tid + it * kThreads;
        if (TOT % kThreads == 0 || u < TOT) {
          const int l = LINE_FAST ? (u % NL) : (u / NB);
          const int t = LINE_FAST ? (u / NL) : (u % NB);
          const int j = t % L;
          cpx<T>* base = buf + l * LS;
#pragma unroll
          for (int m = 0; m < R; ++m) v[it][m] = base[(t + m * NB) * ES];
          if (L > 1) {
#pragma unroll
            for (int m = 1; m < R; ++m) {
              cpx<T> w = tw[j * m * TWS];
              if (INV) w.im = -w.im;
              v[it][m] = v[it][m] * w;
            }
          }
          dft<T, R, INV>(v[it]);
        }
      }
      __syncthreads();
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int u = tid + it * kThreads;
        if (TOT % kThreads == 0 || u < TOT) {
          const int l = LINE_FAST ? (u % NL) : (u / NB);
          const int t = LINE_FAST ? (u / NL) : (u % NB);
          const int j = t % L;
          cpx<T>* base = buf + l * LS;
          const int o = (t - j) * R + j;
#pragma unroll
          for (int m = 0; m < R; ++m) base[(o + m * L) * ES] = v[it][m];
        }
      }
      __syncthreads();
      stage<S + 1, INV>(buf, tw);
    }
  }

  template <bool INV>
  __device__ __forceinline__ static void run(cpx<T>* buf, const cpx<T>* tw) {
    stage<0, INV>(buf, tw);
  }
};

// ------------------------------------------------------------------ lane moves
// DPP moves: a lane reads another lane's register directly, without the LDS crossbar.
// A wave64 is four rows of 16 lanes.  Lanes whose source lies outside their row
// (row_shl / row_shr), or outside the wave, receive an unspecified value, which callers
// select away.  Every lane of the wave must be active.
enum : int {
  DPP_QUAD_1032 = 0xB1,        // quad_perm [1,0,3,2]
  DPP_QUAD_2301 = 0x4E,        // quad_perm [2,3,0,1]
  DPP_ROW_SHL = 0x100,         // + k: lane reads lane + k of its row
  DPP_ROW_SHR = 0x110,         // + k: lane reads lane - k of its row
  DPP_WAVE_SHL1 = 0x130,       // lane reads lane + 1
  DPP_WAVE_SHR1 = 0x138,       // lane reads lane - 1
  DPP_ROW_MIRROR = 0x140,      // lane reads lane 15 - l of its row
  DPP_ROW_HALF_MIRROR = 0x141, // the same within each half row of 8
  DPP_ROW_BCAST15 = 0x142,     // row r reads lane 15 of row r - 1
  DPP_ROW_BCAST31 = 0x143,     // rows 2 and 3 read lane 31
};
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned)lo));
}
template <int CTRL, typename T>
__device__ __forceinline__ cpx<T> dpp(cpx<T> v) {
  return cpx<T>{dpp<CTRL>(v.re), dpp<CTRL>(v.im)};
}
// The value of lane LANE, in every lane.
template <int LANE>
__device__ __forceinline__ float lane_val(float v) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), LANE));
}
template <int LANE>
__device__ __forceinline__ double lane_val(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)b, LANE);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), LANE);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned)lo));
}
template <int LANE, typename T>
__device__ __forceinline__ cpx<T> lane_val(cpx<T> v) {
  return cpx<T>{lane_val<LANE>(v.re), lane_val<LANE>(v.im)};
}

// ---------------------------------------------------- Crank-Nicolson line solves
// Chunk-padded position of element i for a line split into chunks of S elements: one
// spare slot after every chunk keeps the P lanes of a line on distinct LDS banks.
template <int S>
__device__ __forceinline__ int cpad(int i) { return i + i / S; }


// Solve, for NL lines of N points (two Dirichlet end points included) held in LDS at
// buf[l*LS + cpad<S>(i)*ES] with S = ceil(N/P):
//     -A u_{i-1} + (1+2A) u_i - A u_{i+1} = A p_{i-1} + (1-2A) p_i + A p_{i+1},  0 < i < N-1,
//     u_0 = u_{N-1} = 0,
// and overwrite the line with u.  A = a (IMAG_A false: imaginary-time step, all factors
// real) or A = i a (IMAG_A true: real-time step, a > 0, or its adjoint, a < 0).
// Thomas elimination with the data-independent factors precomputed per axis:
// m_i = 1/(b - a c_{i-1}) and g_i = A m_i (= -c_i), so that
//     forward   d_i = m_i r_i + g_i d_{i-1}
//     backward  u_i = d_i + g_i u_{i+1}
// (m = 0 on the two boundary rows makes them u = 0).  Each recurrence is an affine map
// per chunk, composed across the P lanes of a line by a Hillis-Steele scan of (gain,
// offset) pairs through DPP lane moves, then re-run with the exact carry-in.  P divides
// 64, so one line never spans two waves.  mt holds f_i = 2 A m_i in LDS at cpad<S>(i)
// (the same chunk padding as the data, so the P lanes of a line read distinct banks):
// the right-hand side 2 A (p_{i-1} + p_{i+1} - 2 p_i) enters as m_i r_i = f_i (p_{i-1} +
// p_{i+1} - 2 p_i), and g_i = f_i / 2.  Each lane reads its chunk, its two neighbours and
// its f_i once into registers.  Every thread
// must call this; it ends with a block barrier.
// Gains g = A m of the recurrences: complex when A = i a, real when A = a (then m is
// real too).  mulg(g, x) = g x for a complex x; gg(g, h) = g h.
template <typename T>
__device__ __forceinline__ cpx<T> mulg(cpx<T> g, cpx<T> x) { return g * x; }
template <typename T>
__device__ __forceinline__ cpx<T> mulg(T g, cpx<T> x) { return {g * x.re, g * x.im}; }

template <typename T, bool IMAG_A>
struct CnArith {
  using G = typename std::conditional<IMAG_A, cpx<T>, T>::type;
  static __device__ __forceinline__ G one() {
    if constexpr (IMAG_A) return cpx<T>{1, 0};
    else return (T)1;
  }
  // The table holds f = 2 A m (complex when A = i a, real when A = a).
  // g = A m = f / 2
  __device__ __forceinline__ G gain(cpx<T> f) const {
    if constexpr (IMAG_A) return cpx<T>{(T)0.5 * f.re, (T)0.5 * f.im};
    else return (T)0.5 * f.re;
  }
  // f x = m * (2 A x)
  __device__ __forceinline__ cpx<T> mulm(cpx<T> f, cpx<T> x) const {
    return IMAG_A ? f * x : cpx<T>{f.re * x.re, f.re * x.im};
  }
  // the right-hand side of the increment system without its factor 2 A (which the
  // table carries): p_{i-1} + p_{i+1} - 2 p_i
  __device__ __forceinline__ cpx<T> inc(cpx<T> pm, cpx<T> p0, cpx<T> pp) const {
    return cpx<T>{pm.re + pp.re - (T)2 * p0.re, pm.im + pp.im - (T)2 * p0.im};
  }
};

// Component-wise select of two complex values (a select of whole structs can be lowered
// through scratch memory).
template <typename T>
__device__ __forceinline__ cpx<T> csel(bool c, cpx<T> a, cpx<T> b) {
  return cpx<T>{c ? a.re : b.re, c ? a.im : b.im};
}
template <typename T>
__device__ __forceinline__ T csel(bool c, T a, T b) {
  return c ? a : b;
}

// One step of the scan of chunk maps x -> V + G x with the gains composed on the fly:
// where `take`, compose the lane's map with the map (Gs, Vs) of the lane CTRL reads,
// V + G (Vs + Gs x).
template <int CTRL, typename T, typename GT>
__device__ __forceinline__ void cn_scan_step(GT& G, cpx<T>& V, bool take) {
  const GT Gs = dpp<CTRL>(G);
  const cpx<T> Vs = dpp<CTRL>(V);
  const cpx<T> Vn = mulg(G, Vs) + V;
  const GT Gn = G * Gs;
  V = csel(take, Vn, V);
  G = csel(take, Gn, G);
}
// One step of the scan with the lane's gain w for this step precomputed: where `take`,
// V + w Vs with Vs the offset of the lane CTRL reads.
template <int CTRL, typename T, typename GT>
__device__ __forceinline__ void cn_scan_w(GT w, cpx<T>& V, bool take) {
  const cpx<T> Vs = dpp<CTRL>(V);
  V = csel(take, mulg(w, Vs) + V, V);
}
// A scan weight as the gain type (real gains keep the real part).
template <typename GT, typename T>
__device__ __forceinline__ GT scan_weight(const cpx<T>* __restrict__ w) {
  if constexpr (std::is_same<GT, T>::value) return w->re;
  else return *w;
}
constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

template <typename T, int N, int NL, int LS, int ES, int P, bool IMAG_A>
__device__ __forceinline__ void cn_solve_lines(cpx<T>* buf, const cpx<T>* mt,
                                               const cpx<T>* __restrict__ wt) {
  static_assert(64 % P == 0 && P <= 32 && NL * P == kThreads, "lanes per line");
  constexpr int S = (N + P - 1) / P;
  constexpr bool FULL = (N % P == 0);  // every lane's chunk lies inside the line
  using AR = CnArith<T, IMAG_A>;
  using GT = typename AR::G;
  const AR ar{};
  const int tid = thread_idx();
  const int l = tid / P, q = tid % P;
  const int lo = q * S;          // first element of the lane's chunk
  const int base = lo + q;       // its chunk-padded position: cpad<S>(lo + e) = base + e
  cpx<T>* line = buf + l * LS;
  cpx<T> r[S];
  GT g[S];
  const cpx<T> zero = {0, 0};
  // The system is solved for the increment delta = u - p:
  //   (1 + A T) delta = 2 A (p_{i-1} + p_{i+1} - 2 p_i),   u = p + delta,
  // which equals (1 + A T) u = (1 - A T) p.  Rounding of the factor table then scales
  // only the O(A) increment, not p itself: with the table in FP32 the direct form loses
  // norm coherently (every interior factor carries the same rounding), the increment
  // form about fifty times less.  Boundary values enter as zero (Dirichlet); the table
  // holds m = 0 on the two boundary rows, so those rows get delta = 0 and g = 0, and
  // elements past the line end (chunks that overhang it) are zero as well, which makes
  // the recurrences below need no per-element guards.
  // Neighbours of the chunk (interior elements only) and the chunk, read once with
  // indices clamped into the line.
  // (lanes past the end of a line that the chunks overhang have lo >= N: neither
  // neighbour is an interior element, and every index below is clamped into the line)
  constexpr int last = (N - 1) + (N - 1) / S;  // padded position of element N - 1
  const bool has_l = lo - 1 >= 1 && lo - 1 <= N - 2;
  const bool has_r = lo + S <= N - 2;
  const cpx<T> tl = line[(has_l ? base - 2 : 0) * ES];
  const cpx<T> tr = line[(has_r ? base + S + 1 : 0) * ES];
  const cpx<T> pl = csel(has_l, tl, zero);
  const cpx<T> pr = csel(has_r, tr, zero);
#pragma unroll
  for (int e = 0; e < S; ++e) {
    if constexpr (FULL) {
      r[e] = line[(base + e) * ES];
    } else {
      const int i = lo + e;
      const cpx<T> v = line[(i < N ? base + e : last) * ES];
      r[e] = csel(i < N - 1, v, zero);
    }
  }
  r[0] = csel(q == 0, zero, r[0]);                // element 0
  if constexpr (FULL) {
    r[S - 1] = csel(q == P - 1, zero, r[S - 1]);  // element N - 1
  }
  // r <- m * rhs = f * (p_{i-1} + p_{i+1} - 2 p_i), g = A m = f / 2 (f = 2 A m from the
  // table; 0 on the boundary rows and past the line end)
  {
    cpx<T> prev = pl;
#pragma unroll
    for (int e = 0; e < S; ++e) {
      cpx<T> m;
      if constexpr (FULL) {
        m = mt[base + e];
      } else {
        const cpx<T> f = mt[lo + e < N ? base + e : last];
        m = csel(lo + e < N, f, zero);
      }
      const cpx<T> cur = r[e];
      const cpx<T> next = (e + 1 < S) ? r[e + 1] : pr;
      r[e] = ar.mulm(m, ar.inc(prev, cur, next));
      g[e] = ar.gain(m);
      prev = cur;
    }
  }
  // forward recurrence d_i = r_i + g_i d_{i-1}: the chunk's affine map (Gc, D), an
  // inclusive scan of the maps across the P lanes, then the chunk from its true input.
  // The gains of the scan (Gc and its compositions) depend on the factors only.  Lines of
  // up to 16 lanes read the gain lane q carries into step s from the table (wt[s P + q],
  // backward wt[(NS + s) P + q]) and move only the offsets between lanes; 32-lane lines
  // compose the gains as they go (ten table gains in flight would cost a wave of
  // occupancy, or expose their load latency at three waves per SIMD).
  constexpr int NS = ilog2(P);
  constexpr bool WTAB = P <= 16;
  GT Gc = AR::one();
  cpx<T> D = {0, 0};
#pragma unroll
  for (int e = 0; e < S; ++e) {
    D = r[e] + mulg(g[e], D);
    if constexpr (!WTAB) Gc = g[e] * Gc;
  }
  // Lines of P <= 16 lanes lie inside one row of 16 lanes; a line of 32 lanes spans two
  // rows.  The scans move values with DPP: row shifts inside a row, then one step across
  // the row pair.
  constexpr int PR = P < 16 ? P : 16;
  const int rq = tid & (PR - 1);  // lane within the line's part of its row
  cpx<T> din = {0, 0};
  if constexpr (P > 1 && WTAB) {
    GT w[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) w[k] = scan_weight<GT>(wt + k * P + q);
    if constexpr (PR > 1) cn_scan_w<DPP_ROW_SHR + 1>(w[0], D, rq >= 1);
    if constexpr (PR > 2) cn_scan_w<DPP_ROW_SHR + 2>(w[1], D, rq >= 2);
    if constexpr (PR > 4) cn_scan_w<DPP_ROW_SHR + 4>(w[2], D, rq >= 4);
    if constexpr (PR > 8) cn_scan_w<DPP_ROW_SHR + 8>(w[3], D, rq >= 8);
    din = csel(q == 0, zero, dpp<DPP_WAVE_SHR1>(D));
  } else if constexpr (P > 1) {
    GT Gn = Gc;
    cn_scan_step<DPP_ROW_SHR + 1>(Gn, D, rq >= 1);
    cn_scan_step<DPP_ROW_SHR + 2>(Gn, D, rq >= 2);
    cn_scan_step<DPP_ROW_SHR + 4>(Gn, D, rq >= 4);
    cn_scan_step<DPP_ROW_SHR + 8>(Gn, D, rq >= 8);
    // the upper row of a 32-lane line takes the total of the lower row (its lane 15)
    cn_scan_step<DPP_ROW_BCAST15>(Gn, D, (tid & 16) != 0);
    din = csel(q == 0, zero, dpp<DPP_WAVE_SHR1>(D));
  }
  {
    cpx<T> d = din;
#pragma unroll
    for (int e = 0; e < S; ++e) {
      d = r[e] + mulg(g[e], d);
      r[e] = d;
    }
  }
  // backward recurrence u_i = d_i + g_i u_{i+1}: the chunk's map is (Gc, X) with the same
  // product of factors
  cpx<T> X = {0, 0};
#pragma unroll
  for (int e = S - 1; e >= 0; --e) X = r[e] + mulg(g[e], X);
  cpx<T> xin = {0, 0};
  if constexpr (P > 1 && WTAB) {
    GT w[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) w[k] = scan_weight<GT>(wt + (NS + k) * P + q);
    if constexpr (PR > 1) cn_scan_w<DPP_ROW_SHL + 1>(w[0], X, rq + 1 < PR);
    if constexpr (PR > 2) cn_scan_w<DPP_ROW_SHL + 2>(w[1], X, rq + 2 < PR);
    if constexpr (PR > 4) cn_scan_w<DPP_ROW_SHL + 4>(w[2], X, rq + 4 < PR);
    if constexpr (PR > 8) cn_scan_w<DPP_ROW_SHL + 8>(w[3], X, rq + 8 < PR);
    xin = csel(q == P - 1, zero, dpp<DPP_WAVE_SHL1>(X));
  } else if constexpr (P > 1) {
    GT Gn = Gc;
    cn_scan_step<DPP_ROW_SHL + 1>(Gn, X, rq + 1 < PR);
    cn_scan_step<DPP_ROW_SHL + 2>(Gn, X, rq + 2 < PR);
    cn_scan_step<DPP_ROW_SHL + 4>(Gn, X, rq + 4 < PR);
    cn_scan_step<DPP_ROW_SHL + 8>(Gn, X, rq + 8 < PR);
    // the lower row of a 32-lane line takes the total of the upper row, held by the
    // upper row's first lane (16 or 48)
    const bool second = (tid & 32) != 0;
    const cpx<T> Xs = csel(second, lane_val<48>(X), lane_val<16>(X));
    X = csel((tid & 16) == 0, mulg(Gn, Xs) + X, X);
    xin = csel(q == P - 1, zero, dpp<DPP_WAVE_SHL1>(X));
  }
  {
    cpx<T> x = xin;
#pragma unroll
    for (int e = S - 1; e >= 0; --e) {
      x = r[e] + mulg(g[e], x);
      r[e] = x;
    }
  }
  __syncthreads();  // every lane has read its neighbours
  // u = p + delta on the interior, 0 on the boundary rows
#pragma unroll
  for (int e = 0; e < S; ++e) {
    const int i = lo + e;
    if constexpr (FULL) {
      cpx<T>& dst = line[(base + e) * ES];
      cpx<T> u = dst + r[e];
      if (e == 0) u = csel(q == 0, zero, u);
      if (e == S - 1) u = csel(q == P - 1, zero, u);
      dst = u;
    } else if (i < N) {
      cpx<T>& dst = line[(base + e) * ES];
      dst = csel(i >= 1 && i <= N - 2, dst + r[e], zero);
    }
  }
  __syncthreads();
}

// exp(-i x) as (cos x, sin x): Taylor series in Horner form for |x| <= pi/4 (truncation
// below 1e-9 relative in float, 1e-19 in double), the library sincos beyond.
__device__ __forceinline__ void sincos_taylor(float x, float& s, float& c) {
  const float x2 = x * x;
  s = x * (1.f + x2 * (-1.f / 6.f + x2 * (1.f / 120.f + x2 * (-1.f / 5040.f + x2 * (1.f / 362880.f)))));
  c = 1.f + x2 * (-0.5f + x2 * (1.f / 24.f + x2 * (-1.f / 720.f + x2 * (1.f / 40320.f +
      x2 * (-1.f / 3628800.f)))));
}
// Beyond pi/4 the argument is reduced modulo pi/2 in double precision, x = k pi/2 + r,
// |r| <= pi/4 (the error of pi/2 rounded to double, 6e-17, times k stays far below
// float resolution for any |x| < 1e7), and the quadrant k mod 4 rotates (sin r, cos r).
__device__ __forceinline__ void sincos_phase(float x, float& s, float& c) {
  if (fabsf(x) <= 0.78539816339744831f) {
    sincos_taylor(x, s, c);
  } else {
    const double xd = (double)x;
    const double k = rint(xd * 0.63661977236758134);          // 2/pi
    const float r = (float)fma(-k, 1.5707963267948966, xd);    // pi/2
    float sr, cr;
    sincos_taylor(r, sr, cr);
    const int q = (int)(long long)k & 3;
    s = (q == 0) ? sr : (q == 1) ? cr : (q == 2) ? -sr : -cr;
    c = (q == 0) ? cr : (q == 1) ? -sr : (q == 2) ? -cr : sr;
  }
}
__device__ __forceinline__ void sincos_phase(double x, double& s, double& c) {
  if (fabs(x) <= 0.78539816339744831) {
    const double x2 = x * x;
    // sum_{k=0}^{8} (-1)^k x^(2k+1)/(2k+1)!  and  sum_{k=0}^{9} (-1)^k x^(2k)/(2k)!
    double ps = 1.0 / 355687428096000.0;            // 1/17!
    ps = -1.0 / 1307674368000.0 + x2 * ps;           // 1/15!
    ps = 1.0 / 6227020800.0 + x2 * ps;               // 1/13!
    ps = -1.0 / 39916800.0 + x2 * ps;                // 1/11!
    ps = 1.0 / 362880.0 + x2 * ps;                   // 1/9!
    ps = -1.0 / 5040.0 + x2 * ps;
    ps = 1.0 / 120.0 + x2 * ps;
    ps = -1.0 / 6.0 + x2 * ps;
    s = x * (1.0 + x2 * ps);
    double pc = -1.0 / 6402373705728000.0;           // 1/18!
    pc = 1.0 / 20922789888000.0 + x2 * pc;           // 1/16!
    pc = -1.0 / 87178291200.0 + x2 * pc;             // 1/14!
    pc = 1.0 / 479001600.0 + x2 * pc;                // 1/12!
    pc = -1.0 / 3628800.0 + x2 * pc;                 // 1/10!
    pc = 1.0 / 40320.0 + x2 * pc;
    pc = -1.0 / 720.0 + x2 * pc;
    pc = 1.0 / 24.0 + x2 * pc;
    pc = -0.5 + x2 * pc;
    c = 1.0 + x2 * pc;
  } else {
    sincos(x, &s, &c);
  }
}

// Stores the factor table m (N entries) in LDS at the chunk-padded positions used by
// cn_solve_lines with P lanes per line.
template <typename T, int N, int P>
__device__ __forceinline__ void load_cn_table(cpx<T>* mt, const cpx<T>* __restrict__ m) {
  constexpr int S = (N + P - 1) / P;
  for (int i = thread_idx(); i < N; i += kThreads) mt[cpad<S>(i)] = m[i];
}
template <int N, int P>
constexpr int cn_table_len() {
  return N + (N + (N + P - 1) / P - 1) / ((N + P - 1) / P);
}

// ------------------------------------------------------------- reductions
// Sum over the 64 lanes of a wave, valid in lane 63 only, in a fixed order: pairs, quads,
// half rows and rows of 16 (every lane of a row then holds the row total), then row 2
// into row 3 (and row 0 into row 1), then rows 0-1 (lane 31) into row 3.  Lanes of
// rows 0-2 end with partial or unspecified values.
__device__ __forceinline__ double wave_sum_to_last(double v) {
  v += dpp<DPP_QUAD_1032>(v);
  v += dpp<DPP_QUAD_2301>(v);
  v += dpp<DPP_ROW_HALF_MIRROR>(v);
  v += dpp<DPP_ROW_MIRROR>(v);
  v += dpp<DPP_ROW_BCAST15>(v);
  v += dpp<DPP_ROW_BCAST31>(v);
  return v;
}

// Deterministic FP64 block sum of NV values per thread; result valid in thread 0.
// Each wave sums in registers (wave_sum_to_last), then the kThreads/64 wave totals are
// added in wave order: one barrier, fixed summation order.
constexpr int kWaves = kThreads / 64;
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red /* LDS NV*kWaves */) {
  const int lane = thread_idx() & 63, wave = thread_idx() >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum_to_last(v[k]);
  if (lane == 63) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k * kWaves + wave] = v[k];
  }
  __syncthreads();
  if (thread_idx() == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double acc = red[k * kWaves];
#pragma unroll
      for (int w = 1; w < kWaves; ++w) acc += red[k * kWaves + w];
      v[k] = acc;
    }
  }
}

// Block totals of NV per-thread doubles written to out[0..NV) (global): the wave totals
// are combined by NV threads in parallel, each in wave order (the same summation order as
// block_sum), so no thread waits on a serial tail.
template <int NV>
__device__ __forceinline__ void block_sum_store(double (&v)[NV], double* red /* LDS NV*kWaves */,
                                                double* __restrict__ out) {
  static_assert(NV <= kThreads, "one thread per total");
  const int t = thread_idx();
  const int lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum_to_last(v[k]);
  if (lane == 63) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k * kWaves + wave] = v[k];
  }
  __syncthreads();
  if (t < NV) {
    double acc = red[t * kWaves];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) acc += red[t * kWaves + w];
    out[t] = acc;
  }
}

// Block totals of NV <= 8 per-thread doubles written to out[0..NV) (global), for the
// larger sets: partner lanes first split the values between them (lane pairs 1 apart
// keep values 0-3 and 4-7, then pairs 2 apart keep half of those), so that each lane
// goes on summing two values only; row shifts by 4 and 8 leave each row of 16 lanes
// with its totals in lanes 12-15, and the 16 row totals of every value (4 waves x 4
// rows) are added in a fixed order by NV threads.  red: LDS of 128 doubles, free for
// this call (the caller has synchronised the block if it aliases other data).  Returns
// total t to thread t < NV (0 elsewhere).
template <int NV>
__device__ __forceinline__ double block_sum_store8(double (&v)[NV], double* red,
                                                   double* __restrict__ out) {
  static_assert(NV > 2 && NV <= 8, "two to eight values");
  const int t = thread_idx();
  const int lane = t & 63, wave = t >> 6;
  double x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = k < NV ? v[k] : 0.0;
  const bool odd = lane & 1, hi2 = lane & 2;
  double a[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double send = odd ? x[k] : x[k + 4];
    const double keep = odd ? x[k + 4] : x[k];
    a[k] = keep + dpp<DPP_QUAD_1032>(send);
  }
  double b[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double send = hi2 ? a[k] : a[k + 2];
    const double keep = hi2 ? a[k + 2] : a[k];
    b[k] = keep + dpp<DPP_QUAD_2301>(send);
  }
  // lane holds values 4 (lane & 1) + 2 ((lane >> 1) & 1) + k, k < 2
#pragma unroll
  for (int k = 0; k < 2; ++k) b[k] += dpp<DPP_ROW_SHR + 4>(b[k]);
#pragma unroll
  for (int k = 0; k < 2; ++k) b[k] += dpp<DPP_ROW_SHR + 8>(b[k]);
  if ((lane & 15) >= 12) {
    const int base = 4 * (lane & 1) + 2 * ((lane >> 1) & 1);
    const int row = (wave << 2) | (lane >> 4);
#pragma unroll
    for (int k = 0; k < 2; ++k) red[row * 8 + base + k] = b[k];
  }
  __syncthreads();
  double acc = 0.0;
  if (t < NV) {
    acc = red[t];
#pragma unroll
    for (int r = 1; r < 4 * kWaves; ++r) acc += red[r * 8 + t];
    out[t] = acc;
  }
  return acc;
}

}  // namespace gpdbec
