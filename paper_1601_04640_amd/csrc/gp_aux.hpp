// Set-up, I/O and reduction kernels: FFT twiddles, Crank-Nicolson factor tables, the
// dipolar kernel table U(k)/N, the harmonic trap, wave-function conversion with the
// Dirichlet boundary, and the FP64 finalisation of one step's partial sums.
#pragma once
#include "gp_device.hpp"
#include "gp_finalize.hpp"

namespace gpdbec {

// tw[k] = exp(-2 pi i k/N), evaluated in FP64 and rounded to T.
template <typename T>
__global__ void k_twiddles(cpx<T>* tw, int N) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  double s, c;
  sincospi(2.0 * (double)k / (double)N, &s, &c);
  tw[k] = cpx<T>{(T)c, (T)(-s)};
}

// Bluestein tables of an n-point axis with convolution length m, in FP64 rounded to T:
// the chirp c_j = exp(-i pi j^2 / n), j < n (j^2 taken mod 2n), and the filter
// F_k = (1/m) sum_q w_q exp(-2 pi i q k / m) of w_q = conj(c_q) (q < n), w_(m-q) = w_q
// (0 < q < n), zero elsewhere; w is even, so F_k = (1/m) (1 + 2 sum_(q=1)^(n-1) conj(c_q)
// cos(2 pi q k / m)).  One thread per k < m.
template <typename T>
__global__ void k_bluestein(cpx<T>* chirp, cpx<T>* filt, int n, int m) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) {
    const long long r = ((long long)k * k) % (2LL * n);
    double s, c;
    sincospi((double)r / n, &s, &c);
    chirp[k] = cpx<T>{(T)c, (T)(-s)};
  }
  if (k >= m) return;
  double fr = 1.0, fi = 0.0;
  for (int q = 1; q < n; ++q) {
    const long long r = ((long long)q * q) % (2LL * n);
    double s, c;
    sincospi((double)r / n, &s, &c);            // conj(c_q) = c + i s
    const long long u = ((long long)q * k) % m;
    const double w = 2.0 * cospi(2.0 * (double)u / m);
    fr += w * c;
    fi += w * s;
  }
  filt[k] = cpx<T>{(T)(fr / m), (T)(fi / m)};
}

// Thomas factors of (1 + 2A) u_i - A (u_{i-1} + u_{i+1}) with Dirichlet ends, for
// A = Ar (imaginary time) and A = i Ar (real time), evaluated sequentially in FP64:
//   m_1 = 1/b,  m_i = 1/(b - a c_{i-1}),  c_i = a m_i,  g_i = -c_i = A m_i,
// with a = -A, b = 1 + 2A; m = g = 0 on the two boundary rows.
struct zd {
  double re, im;
};
__device__ inline zd zmul(zd a, zd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline zd zsub(zd a, zd b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline zd zinv(zd a) {
  const double d = a.re * a.re + a.im * a.im;
  return {a.re / d, -a.im / d};
}

// Each table holds f_i = 2 A m_i for i = 0..N-1 (the factor the solve multiplies the
// right-hand side p_{i-1} + p_{i+1} - 2 p_i by; g_i = f_i / 2), then the scan weights of the line solve that sweeps
// this axis with P lanes per line (chunks of S = ceil(N/P) points; cn_solve_lines):
// per lane q, the gain its (gain, offset) map carries into each step of the forward
// scan (entries s P + q) and of the backward scan (entries (NS + s) P + q), NS = log2 P.
// They depend on the factors only: the products g of every chunk, composed across the
// lanes in the solve's own step order.
constexpr int kScanWeights = 2 * 5 * 32;  // 2 NS P for P <= 32
template <typename T>
__device__ inline void cn_scan_weights(const zd* gc, int P, cpx<T>* w) {
  const int PR = P < 16 ? P : 16;  // lanes of a line inside one row of 16
  int NS = 0;
  while ((1 << NS) < P) ++NS;
  zd G[32], H[32];
  for (int dir = 0; dir < 2; ++dir) {
    for (int q = 0; q < P; ++q) G[q] = gc[q];
    int s = 0;
    for (int off = 1; off < PR; off <<= 1, ++s) {
      for (int q = 0; q < P; ++q) {
        w[(dir * NS + s) * P + q] = cpx<T>{(T)G[q].re, (T)G[q].im};
        const int rq = q % PR;
        const bool take = dir == 0 ? rq >= off : rq + off < PR;
        H[q] = take ? zmul(G[q], G[dir == 0 ? q - off : q + off]) : G[q];
      }
      for (int q = 0; q < P; ++q) G[q] = H[q];
    }
    if (P == 32)  // the step across the two rows of a 32-lane line
      for (int q = 0; q < P; ++q) w[(dir * NS + s) * P + q] = cpx<T>{(T)G[q].re, (T)G[q].im};
  }
}

// Third set: A = -i Ar, the adjoint sweep of a real-time step (conjugate factors).
template <typename T>
__global__ void k_cn_tables(cpx<T>* m_im, cpx<T>* m_re, cpx<T>* m_adj, int N, double Ar, int P) {
  if (blockIdx.x != 0 || threadIdx.x > 2) return;
  const int set = threadIdx.x;
  cpx<T>* mt = set == 0 ? m_im : (set == 1 ? m_re : m_adj);
  const zd A = set == 0 ? zd{Ar, 0.0} : (set == 1 ? zd{0.0, Ar} : zd{0.0, -Ar});
  const zd a = {-A.re, -A.im};
  const zd b = {1.0 + 2.0 * A.re, 2.0 * A.im};
  const int S = (N + P - 1) / P;
  // chunk products of g; a chunk holding a boundary row or reaching past the line end
  // has a zero factor
  zd gc[32];
  for (int q = 0; q < P; ++q) {
    const bool zero = q == 0 || (q + 1) * S > N - 1;
    gc[q] = zero ? zd{0.0, 0.0} : zd{1.0, 0.0};
  }
  zd c = {0.0, 0.0};
  mt[0] = cpx<T>{0, 0};
  for (int i = 1; i <= N - 2; ++i) {
    const zd m = zinv(zsub(b, zmul(a, c)));
    c = zmul(a, m);
    const zd f = zmul(zd{2.0 * A.re, 2.0 * A.im}, m);  // the solve's factor 2 A m
    mt[i] = cpx<T>{(T)f.re, (T)f.im};
    const int q = i / S;
    gc[q] = zmul(gc[q], zd{-c.re, -c.im});
  }
  mt[N - 1] = cpx<T>{0, 0};
  cn_scan_weights(gc, P, mt + N);
}

// Spherical-cutoff factor b(s) = 1 + 3 cos s/s^2 - 3 sin s/s^3 (s = kR); for s < 1 the
// alternating series sum_{k>=2} (-1)^k 6k s^(2k-2)/(2k+1)! avoids the cancellation.
__device__ inline double cutoff_b(double s) {
  if (s < 1.0) {
    const double s2 = s * s;
    double term = s2 / 10.0;  // k = 2
    double acc = term;
    for (int k = 2; k < 15; ++k) {
      term *= -s2 * (double)(k + 1) / ((double)k * (2.0 * k + 2.0) * (2.0 * k + 3.0));
      acc += term;
    }
    return acc;
  }
  double sn, cs;
  sincos(s, &sn, &cs);
  return 1.0 + 3.0 * cs / (s * s) - 3.0 * sn / (s * s * s);
}

struct KernelGeom {
  int geom;          // 0: 3D, 1: 2D XY, 2: 2D XZ
  int n0, n1, n2;    // grid axes (x fastest)
  double h0, h1, h2;
  double R;          // 3D cutoff radius (<= 0: none)
  double d;          // 2D transverse width
  // 2D axes split for the four-step FFT (x: Ax Bx, y: Ay By; 0 when not split): the table
  // is laid out like the spectrum, one value per slot (rows of rs slots for a split x)
  int Ax, Bx, Ay, By, rs;
};

// ktab[(kx*n2 + k2)*n1 + k1] = U(k)/(n0 n1 n2), kx = 0..n0/2, in FP64 rounded to T.
//  3D:  U = (3 kz^2/k^2 - 1) b(kR), U(0) = 0   (axis 1 = y, axis 2 = z)
//  XY:  U = [2 - 3 sqrt(pi) xi erfcx(xi)]/(sqrt(2 pi) d),  xi = q d/sqrt 2
//  XZ:  U = [-1 + 3 sqrt(pi) (kz^2/q^2) xi erfcx(xi)]/(sqrt(2 pi) d)   (axis 1 = z)
template <typename T>
__global__ void k_kernel_table(T* ktab, KernelGeom kg) {
  // 3D: U depends on k1 and k2 through their squares only, so the table holds the
  // quadrant k1 <= n1/2, k2 <= n2/2 (ktab[(kx (n2/2+1) + k2) (n1/2+1) + k1]); the z
  // convolution reads index min(k, n - k).  2D: the full [kx][k1] table, or with a split
  // axis the spectrum's slots: a split x keeps rows y of rs slots p holding
  // kx = Bx (p mod Ax) + p / Ax (U is even in kx: folded to n0 - kx past n0/2); a split y
  // slot y = kb Ay + ka holds k1 = By ka + kb.
  const int H = kg.n0 / 2 + 1;
  const bool q3 = kg.geom == 0;
  const int m1n = q3 ? kg.n1 / 2 + 1 : kg.n1, m2n = q3 ? kg.n2 / 2 + 1 : kg.n2;
  const size_t total = kg.Ax ? (size_t)kg.rs * kg.n1 : (size_t)H * m1n * m2n;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  int k1, k2, kx;
  if (kg.Ax) {
    const int y = (int)(idx / kg.rs), p = (int)(idx % kg.rs);
    kx = kg.Bx * (p % kg.Ax) + p / kg.Ax;
    if (kx > kg.n0 - kx) kx = kg.n0 - kx;
    k1 = y;
    k2 = 0;
  } else {
    k1 = (int)(idx % m1n);
    k2 = (int)((idx / m1n) % m2n);
    kx = (int)(idx / ((size_t)m1n * m2n));
  }
  if (kg.Ay) k1 = kg.By * (k1 % kg.Ay) + k1 / kg.Ay;
  const double pi = 3.14159265358979323846;
  const double qx = 2.0 * pi * kx / (kg.n0 * kg.h0);
  // signed frequency of index k: k below n/2, k - n from n/2 on (odd n: every k <= n/2
  // of the quadrant is a non-negative frequency)
  const int m1 = (2 * k1 < kg.n1) ? k1 : k1 - kg.n1;
  const int m2 = (2 * k2 < kg.n2) ? k2 : k2 - kg.n2;
  const double q1 = 2.0 * pi * m1 / (kg.n1 * kg.h1);
  const double q2 = (kg.n2 > 1) ? 2.0 * pi * m2 / (kg.n2 * kg.h2) : 0.0;
  double u;
  if (kg.geom == 0) {
    const double k2s = qx * qx + q1 * q1 + q2 * q2;
    if (k2s == 0.0) {
      u = 0.0;
    } else {
      u = 3.0 * q2 * q2 / k2s - 1.0;
      if (kg.R > 0.0) u *= cutoff_b(sqrt(k2s) * kg.R);
    }
  } else {
    const double pref = 1.0 / (sqrt(2.0 * pi) * kg.d);
    const double qq = qx * qx + q1 * q1;
    const double q = sqrt(qq);
    const double xi = q * kg.d / sqrt(2.0);
    const double ex = 3.0 * sqrt(pi) * xi * erfcx(xi);
    if (kg.geom == 1) {
      u = pref * (2.0 - ex);
    } else {
      const double ratio = (qq > 0.0) ? q1 * q1 / qq : 0.0;
      u = pref * (-1.0 + ratio * ex);
    }
  }
  ktab[idx] = (T)(u / ((double)kg.n0 * (double)kg.n1 * (double)kg.n2));
}

// Harmonic trap V = (w0^2 a0^2 + w1^2 a1^2 + w2^2 a2^2)/2 with a = (idx - n/2) h.
template <typename T>
__global__ void k_harmonic(T* V, int n0, int n1, int n2, double h0, double h1, double h2,
                           double w0, double w1, double w2) {
  const size_t total = (size_t)n0 * n1 * n2;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int i = (int)(idx % n0);
  const int j = (int)((idx / n0) % n1);
  const int k = (int)(idx / ((size_t)n0 * n1));
  const double x = (i - n0 / 2) * h0, y = (j - n1 / 2) * h1, z = (k - n2 / 2) * h2;
  V[idx] = (T)(0.5 * (w0 * w0 * x * x + w1 * w1 * y * y + w2 * w2 * z * z));
}

__device__ inline bool on_boundary(size_t idx, int n0, int n1, int n2) {
  const int i = (int)(idx % n0);
  const int j = (int)((idx / n0) % n1);
  const int k = (int)(idx / ((size_t)n0 * n1));
  return i == 0 || i == n0 - 1 || j == 0 || j == n1 - 1 || (n2 > 1 && (k == 0 || k == n2 - 1));
}

// psi[off + e] = src[e] (converted), boundary points zeroed.
template <typename T, typename S>
__global__ void k_psi_in(cpx<T>* psi, const cpx<S>* src, size_t off, size_t cnt, int n0, int n1,
                         int n2) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cnt) return;
  const size_t idx = off + e;
  const cpx<S> v = src[e];
  psi[idx] = on_boundary(idx, n0, n1, n2) ? cpx<T>{0, 0} : cpx<T>{(T)v.re, (T)v.im};
}

// dst[e] = scale * psi[off + e] (converted).
template <typename T, typename D>
__global__ void k_psi_out(cpx<D>* dst, const cpx<T>* psi, const double* scale, size_t off,
                          size_t cnt) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cnt) return;
  const double s = *scale;
  const cpx<T> v = psi[off + e];
  dst[e] = cpx<D>{(D)(s * (double)v.re), (D)(s * (double)v.im)};
}

template <typename D, typename S>
__global__ void k_real_convert(D* dst, const S* src, size_t cnt) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < cnt) dst[e] = (D)src[e];
}

// ------------------------------------------------------------------ finalisation
// Standalone finalize (used where no column pass ends the sequence: 2D observables).
__global__ __launch_bounds__(kThreads) void k_finalize(FinArgs a, int mode) {
  finalize_block(a, mode);
}

// First stage of the two-stage finalisation (one block per slice).
__global__ __launch_bounds__(kThreads) void k_prereduce(FinArgs a, int mode) {
  prereduce_block(a, mode, blockIdx.x);
}

// dL/dg += cfac * sum(s n), dL/dg_dd += sum(s Phi) over the k_adj_x partials (one block,
// fixed summation order).
__global__ __launch_bounds__(kThreads) void k_adj_reduce(const double* __restrict__ partials,
                                                         int nb, double cfac, double* grad_g,
                                                         double* grad_gdd) {
  __shared__ double red[2 * kWaves];
  double v[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < nb; b += kThreads) {
    v[0] += partials[2 * b];
    v[1] += partials[2 * b + 1];
  }
  block_sum<2>(v, red);
  if (threadIdx.x == 0) {
    *grad_g += cfac * v[0];
    *grad_gdd += v[1];
  }
}

__global__ void k_reset_state(double* scale, double* one, double* ekz, int* flags,
                              int* ring_pos) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *scale = 1.0;
    *one = 1.0;
    *ekz = 0.0;
    *flags = 0;
    *ring_pos = 0;
  }
}

__global__ void k_set_scale_one(double* scale) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *scale = 1.0;
}

// Span of one stamped launch (last block end - first block start, wall-clock ticks),
// added to acc[0]; acc[1] counts launches.  One block.
__global__ __launch_bounds__(kThreads) void k_span_reduce(const unsigned long long* stamps,
                                                          int nb, unsigned long long* acc) {
  __shared__ unsigned long long lo[kThreads], hi[kThreads];
  unsigned long long mn = ~0ull, mx = 0ull;
  for (int b = threadIdx.x; b < nb; b += kThreads) {
    mn = min(mn, stamps[2 * b]);
    mx = max(mx, stamps[2 * b + 1]);
  }
  lo[threadIdx.x] = mn;
  hi[threadIdx.x] = mx;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      lo[threadIdx.x] = min(lo[threadIdx.x], lo[threadIdx.x + w]);
      hi[threadIdx.x] = max(hi[threadIdx.x], hi[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    acc[0] += (hi[0] > lo[0]) ? hi[0] - lo[0] : 0ull;
    acc[1] += 1ull;
  }
}

__global__ void k_clear_u64(unsigned long long* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0ull;
}

// Fixed numbers of the Crank-Nicolson segments of a long line (segment s: rows a = s n ..
// b = a + n - 1; g = f / 2 of the factor table), in FP64, one thread per segment.  The
// zero-carry recurrences are linear in Delta:
//   d0_b = sum_i w_i Delta_i,  w_i = f_i g_(i+1) ... g_b
//   e0_a = sum_i u_i Delta_i,  u_i = f_i S_i,  S_i = G_(i-1) + g_(i+1) S_(i+1),  S_b = G_(b-1)
// with G_(i-1) = g_a ... g_(i-1); the carries need P = g_a ... g_b and
// Q = sum_m G_(m-1) G_m = g_a S_a.  pq[2s], pq[2s+1] = P, Q; wu[2i], wu[2i+1] = w_i, u_i
// (G is parked in wu[2i+1] between the two passes).
template <typename T>
__global__ void k_seg_tables(const cpx<T>* __restrict__ f, int n, int nseg, cpx<T>* pq,
                             cpx<T>* wu) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  const int a = s * n, b = a + n - 1;
  auto gof = [&](int i) { return zd{0.5 * (double)f[i].re, 0.5 * (double)f[i].im}; };
  zd G{1.0, 0.0};
  for (int i = a; i <= b; ++i) {
    wu[2 * i + 1] = cpx<T>{(T)G.re, (T)G.im};
    G = zmul(G, gof(i));
  }
  zd S{0.0, 0.0}, R{1.0, 0.0};
  for (int i = b; i >= a; --i) {
    const zd Gm{(double)wu[2 * i + 1].re, (double)wu[2 * i + 1].im};
    const zd gn = i < b ? gof(i + 1) : zd{0.0, 0.0};
    const zd gS = zmul(gn, S);
    S = zd{Gm.re + gS.re, Gm.im + gS.im};
    const zd fi{(double)f[i].re, (double)f[i].im};
    const zd w = zmul(fi, R), u = zmul(fi, S);
    wu[2 * i] = cpx<T>{(T)w.re, (T)w.im};
    wu[2 * i + 1] = cpx<T>{(T)u.re, (T)u.im};
    R = zmul(R, gof(i));
  }
  const zd Q = zmul(gof(a), S);
  pq[2 * s] = cpx<T>{(T)G.re, (T)G.im};
  pq[2 * s + 1] = cpx<T>{(T)Q.re, (T)Q.im};
}

}  // namespace gpdbec
