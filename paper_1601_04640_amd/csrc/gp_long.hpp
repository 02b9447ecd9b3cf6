// Pass kernels of 2D grids with an axis longer than one LDS line (more than 8192 FP32 /
// 4096 FP64 points), e.g. the 13000^2 and 15000^2 grids of the paper's 2D runs.
//
// FFT.  An N-point axis is split N = A B, both factors at most one LDS line.  With
// x = a + A b and k = B ka + kb,
//   X_k = sum_a W_A^(a ka) [ W_N^(a kb) sum_b x_(a + A b) W_B^(b kb) ]
// (the four-step factorisation; Bailey, "FFTs in external or hierarchical memory",
// J. Supercomputing 4, 1990): B-point FFTs down the columns a (stride A), the twiddle
// W_N^(a kb), A-point FFTs along the rows kb.  Wavenumber k lands in row kb, column ka, and
// the spectrum keeps that order: the kernel product only needs to know which wavenumber a
// slot holds, and the inverse runs the same steps backwards (conjugate exponents).  Along
// a long y axis the outer steps are kg_lines with the twiddle option and the inner one its
// convolution with the split index (GKtab m4); a long x axis, whose lines are real,
// has the kernels below.
//
// Long x axis.  The densities of lines j and j + 1 are packed as one complex line (j real,
// j + 1 imaginary).  After the row FFTs the two real spectra are untangled with the value
// at N - k, which sits in row (B - kb) mod B, column A - 1 - ka (kb > 0) or (A - ka) mod A
// (kb = 0).  Rows 0 .. B/2 are kept: spec[j rs + kb A + ka], rs = (B/2 + 1) A (rows 0 and,
// for an even B, B/2 hold both k and N - k); the other rows are their conjugates.
//   kg_lx_cols_fwd   |psi|^2 of a line pair, B-point column FFTs, twiddle -> w (pair-major
//                    [pair][kb][a] grid), with the x / y difference sums of kg_r2c_x
//   kg_lx_rows_fwd   A-point row FFTs of rows kb and B - kb, untangled -> spec
//   kg_lx_rows_inv   the rows of Z = A + i B rebuilt from spec (rows past B/2 from their
//                    conjugates), inverse A-point FFTs, conjugate twiddle -> w
//   kg_lx_cols_inv   inverse B-point column FFTs -> Phi of lines j (Re) and j + 1 (Im)
//
// Crank-Nicolson sweeps of long lines run in segments: k_seg_summary (two weighted sums
// per segment), k_seg_carry along each line, and the sweep proper (kg_cn_tile with SEG,
// GSeg); the weights and the carry products P, Q come from k_seg_tables.
#pragma once
#include "gp_generic.hpp"

namespace gpdbec {

// Long-x geometry: x = a + A b, k = B ka + kb; spectrum rows of rs = Bh A slots (Bh = B/2+1);
// n1 lines in np = ceil(n1/2) pairs.  Column kernels: ta columns per block, nat tiles per
// pair.  Row kernels: ipf items of two rows (pair, kb <= B/2) per block forward, ipi items of
// one row (pair, kb) inverse.  f*: divisors.
struct GLX {
  int N, A, B, Bh, rs;
  int n1, np;
  int ta, nat, ipf, ipi;
  FDiv fA, fB, fBh, fta, fnat;
};

template <typename T, int EMAX, bool SMALL, bool BLUE>
__global__ void __launch_bounds__(kGenThreads) kg_lx_cols_fwd(const cpx<T>* __restrict__ psi,
                                                           cpx<T>* __restrict__ w, GLX x,
                                                           GPlan p,
                                                           const cpx<T>* __restrict__ tw,
                                                           const cpx<T>* __restrict__ w4,
                                                           double* __restrict__ part) {
  constexpr int U = sizeof(T) == 4 ? 4 : 2;  // five loads per value
  extern __shared__ __align__(16) char lds_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lds_raw);
  const int bt = xcd_tile(blockIdx.x, gridDim.x);
  const int jp = (int)fdiv((uint32_t)bt, x.fnat);
  const int a0 = (bt - jp * x.nat) * x.ta;
  const int na = min(x.ta, x.A - a0);
  const int j = 2 * jp;
  const bool has1 = j + 1 < x.n1;
  const int N = x.N, A = x.A, B = x.B;
  const int LS = BLUE ? p.m : B;
  const int nt = blockDim.x;
  const int tot = B * x.ta;  // element-major: (b, column c), consecutive threads along a
  cpx<T>* twl = buf + x.ta * LS;
  constexpr int UT = tw_pre<T>() / 2;
  cpx<T> twv[UT];
  tw_fetch<T, SMALL, UT>(twv, tw, LS);
  const long long r0 = (long long)j * N;
  double dx = 0.0, dy = 0.0;
  for (int t0 = threadIdx.x; t0 < tot; t0 += U * nt) {
    cpx<T> v0[U], v1[U], b0[U], b1[U], c1[U];
    int ss[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * nt;
      const int b = (int)fdiv((uint32_t)t, x.fta), c = t - b * x.ta;
      ok[u] = t < tot && c < na;
      ss[u] = c * LS + b;
      const int xi = a0 + c + A * b;
      const bool nx = ok[u] && xi + 1 < N;
      // in-range addresses only; a missing neighbour reads the value itself (no difference)
      const long long ad = ok[u] ? r0 + xi : 0;
      v0[u] = psi[ad];
      v1[u] = psi[has1 ? ad + N : ad];
      b0[u] = psi[nx ? ad + 1 : ad];
      b1[u] = psi[has1 ? (nx ? ad + N + 1 : ad + N) : ad];
      c1[u] = psi[has1 ? (j + 2 < x.n1 ? ad + 2 * N : ad + N) : ad];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!ok[u]) continue;
      const T d0 = v0[u].re * v0[u].re + v0[u].im * v0[u].im;
      const T d1 = has1 ? v1[u].re * v1[u].re + v1[u].im * v1[u].im : (T)0;
      buf[ss[u]] = cpx<T>{d0, d1};
      dx += absdiff2_d(b0[u], v0[u]) + absdiff2_d(b1[u], v1[u]);
      dy += absdiff2_d(v1[u], v0[u]) + absdiff2_d(c1[u], v1[u]);
    }
  }
  const cpx<T>* twu = tw_store<T, SMALL, UT>(twl, twv, tw, LS);
  __syncthreads();
  gfft<T, false, EMAX, SMALL, BLUE>(buf, na, p, twu);
  const long long wb = (long long)jp * B * A;
  for (int t = threadIdx.x; t < tot; t += nt) {
    const int kb = (int)fdiv((uint32_t)t, x.fta), c = t - kb * x.ta;
    if (c < na) {
      const int a = a0 + c;
      w[wb + (long long)kb * A + a] = buf[c * LS + kb] * w4[a * kb];
    }
  }
  __syncthreads();  // the line buffer is free: its first bytes hold the reduction
  double s[2] = {dx, dy};
  gblock_sum<2>(s, reinterpret_cast<double*>(lds_raw));
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s[0];
    part[2 * blockIdx.x + 1] = s[1];
  }
}

// Row slot of the partner N - k of row kb, column ka (row kb's slot q, its pair row's q+1).
__device__ __forceinline__ int lx_partner(int kb, int B, int A, int ka, int q, int LS) {
  if (kb == 0) return q * LS + (ka == 0 ? 0 : A - ka);
  if (2 * kb == B) return q * LS + (A - 1 - ka);
  return (q + 1) * LS + (A - 1 - ka);
}

template <typename T, int EMAX, bool SMALL, bool BLUE>
__global__ void __launch_bounds__(kGenThreads) kg_lx_rows_fwd(const cpx<T>* __restrict__ w,
                                                           cpx<T>* __restrict__ spec, GLX x,
                                                           GPlan p,
                                                           const cpx<T>* __restrict__ tw) {
  extern __shared__ __align__(16) char lds_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lds_raw);
  const int it0 = xcd_tile(blockIdx.x, gridDim.x) * x.ipf;  // items (pair, kb), kb < Bh
  const int nit = min(x.ipf, x.np * x.Bh - it0);
  const int A = x.A, B = x.B;
  const int LS = BLUE ? p.m : A;
  const int nt = blockDim.x;
  const int tot = 2 * x.ipf * A;  // line slot 2 item + (0: row kb, 1: row B - kb)
  cpx<T>* twl = buf + 2 * x.ipf * LS;
  constexpr int UT = tw_pre<T>() / 2;
  cpx<T> twv[UT];
  tw_fetch<T, SMALL, UT>(twv, tw, LS);
  for (int t0 = threadIdx.x; t0 < tot; t0 += kGenU * nt) {
    cpx<T> v[kGenU];
    int at[kGenU];
#pragma unroll
    for (int u = 0; u < kGenU; ++u) {
      const int t = t0 + u * nt;
      const int sl = (int)fdiv((uint32_t)t, x.fA), e = t - sl * A;
      const int item = sl >> 1;
      const bool ok = t < tot && item < nit;
      const int it = it0 + item;
      const int jp = (int)fdiv((uint32_t)it, x.fBh), kb = it - jp * x.Bh;
      const int row = (sl & 1) && kb > 0 ? B - kb : kb;
      at[u] = ok ? sl * LS + e : -1;
      v[u] = w[ok ? ((long long)jp * B + row) * A + e : 0];
    }
#pragma unroll
    for (int u = 0; u < kGenU; ++u)
      if (at[u] >= 0) buf[at[u]] = v[u];
  }
  const cpx<T>* twu = tw_store<T, SMALL, UT>(twl, twv, tw, LS);
  __syncthreads();
  gfft<T, false, EMAX, SMALL, BLUE>(buf, 2 * nit, p, twu);
  // A_k = (Z_k + conj Z_(N-k)) / 2 (line j), B_k = (Z_k - conj Z_(N-k)) / (2i) (line j+1)
  for (int t = threadIdx.x; t < x.ipf * A; t += nt) {
    const int item = (int)fdiv((uint32_t)t, x.fA), ka = t - item * A;
    if (item >= nit) continue;
    const int it = it0 + item;
    const int jp = (int)fdiv((uint32_t)it, x.fBh), kb = it - jp * x.Bh;
    const cpx<T> zk = buf[2 * item * LS + ka];
    const cpx<T> zm = buf[lx_partner(kb, B, A, ka, 2 * item, LS)];
    const int j = 2 * jp;
    const long long o = (long long)j * x.rs + (long long)kb * A + ka;
    spec[o] = cpx<T>{(T)0.5 * (zk.re + zm.re), (T)0.5 * (zk.im - zm.im)};
    if (j + 1 < x.n1) spec[o + x.rs] = cpx<T>{(T)0.5 * (zk.im + zm.im), (T)0.5 * (zm.re - zk.re)};
  }
}

template <typename T, int EMAX, bool SMALL, bool BLUE>
__global__ void __launch_bounds__(kGenThreads) kg_lx_rows_inv(const cpx<T>* __restrict__ spec,
                                                           cpx<T>* __restrict__ w, GLX x,
                                                           GPlan p,
                                                           const cpx<T>* __restrict__ tw,
                                                           const cpx<T>* __restrict__ w4) {
  constexpr int U = kGenU / 2;  // two loads per value
  extern __shared__ __align__(16) char lds_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lds_raw);
  const int it0 = xcd_tile(blockIdx.x, gridDim.x) * x.ipi;  // items (pair, kb), kb < B
  const int nit = min(x.ipi, x.np * x.B - it0);
  const int A = x.A, B = x.B;
  const int LS = BLUE ? p.m : A;
  const int nt = blockDim.x;
  const int tot = x.ipi * A;
  cpx<T>* twl = buf + x.ipi * LS;
  constexpr int UT = tw_pre<T>() / 2;
  cpx<T> twv[UT];
  tw_fetch<T, SMALL, UT>(twv, tw, LS);
  for (int t0 = threadIdx.x; t0 < tot; t0 += U * nt) {
    cpx<T> va[U], vb[U];
    int at[U];
    bool mir[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * nt;
      const int item = (int)fdiv((uint32_t)t, x.fA), ka = t - item * A;
      const bool ok = t < tot && item < nit;
      const int it = it0 + item;
      const int jp = (int)fdiv((uint32_t)it, x.fB), kb = it - jp * B;
      // rows past B/2: the conjugates of row B - kb, columns reversed
      mir[u] = kb >= x.Bh;
      const long long src = mir[u] ? (long long)(B - kb) * A + (A - 1 - ka)
                                   : (long long)kb * A + ka;
      const int j = 2 * jp;
      const bool has1 = ok && j + 1 < x.n1;
      const long long o = ok ? (long long)j * x.rs + src : 0;
      at[u] = ok ? item * LS + ka : -1;
      va[u] = spec[o];
      vb[u] = spec[has1 ? o + x.rs : o];
      if (!has1) vb[u] = cpx<T>{0, 0};
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (at[u] < 0) continue;
      const cpx<T> a = va[u], b = vb[u];
      buf[at[u]] = mir[u] ? cpx<T>{a.re + b.im, b.re - a.im} : cpx<T>{a.re - b.im, a.im + b.re};
    }
  }
  const cpx<T>* twu = tw_store<T, SMALL, UT>(twl, twv, tw, LS);
  __syncthreads();
  gfft<T, true, EMAX, SMALL, BLUE>(buf, nit, p, twu);
  for (int t = threadIdx.x; t < tot; t += nt) {
    const int item = (int)fdiv((uint32_t)t, x.fA), a = t - item * A;
    if (item >= nit) continue;
    const int it = it0 + item;
    const int jp = (int)fdiv((uint32_t)it, x.fB), kb = it - jp * B;
    w[((long long)jp * B + kb) * A + a] = buf[item * LS + a] * conjg(w4[a * kb]);
  }
}

template <typename T, int EMAX, bool SMALL, bool BLUE>
__global__ void __launch_bounds__(kGenThreads) kg_lx_cols_inv(const cpx<T>* __restrict__ w,
                                                           T* __restrict__ phi, GLX x, GPlan p,
                                                           const cpx<T>* __restrict__ tw) {
  extern __shared__ __align__(16) char lds_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lds_raw);
  const int bt = xcd_tile(blockIdx.x, gridDim.x);
  const int jp = (int)fdiv((uint32_t)bt, x.fnat);
  const int a0 = (bt - jp * x.nat) * x.ta;
  const int na = min(x.ta, x.A - a0);
  const int j = 2 * jp;
  const bool has1 = j + 1 < x.n1;
  const int N = x.N, A = x.A, B = x.B;
  const int LS = BLUE ? p.m : B;
  const int nt = blockDim.x;
  const int tot = B * x.ta;
  cpx<T>* twl = buf + x.ta * LS;
  constexpr int UT = tw_pre<T>() / 2;
  cpx<T> twv[UT];
  tw_fetch<T, SMALL, UT>(twv, tw, LS);
  const long long wb = (long long)jp * B * A;
  for (int t0 = threadIdx.x; t0 < tot; t0 += kGenU * nt) {
    cpx<T> v[kGenU];
    int at[kGenU];
#pragma unroll
    for (int u = 0; u < kGenU; ++u) {
      const int t = t0 + u * nt;
      const int kb = (int)fdiv((uint32_t)t, x.fta), c = t - kb * x.ta;
      const bool ok = t < tot && c < na;
      at[u] = ok ? c * LS + kb : -1;
      v[u] = w[ok ? wb + (long long)kb * A + a0 + c : 0];
    }
#pragma unroll
    for (int u = 0; u < kGenU; ++u)
      if (at[u] >= 0) buf[at[u]] = v[u];
  }
  const cpx<T>* twu = tw_store<T, SMALL, UT>(twl, twv, tw, LS);
  __syncthreads();
  gfft<T, true, EMAX, SMALL, BLUE>(buf, na, p, twu);
  const long long r0 = (long long)j * N;
  for (int t = threadIdx.x; t < tot; t += nt) {
    const int b = (int)fdiv((uint32_t)t, x.fta), c = t - b * x.ta;
    if (c < na) {
      const long long o = r0 + a0 + c + (long long)A * b;
      const cpx<T> z = buf[c * LS + b];
      phi[o] = z.re;
      if (has1) phi[o + N] = z.im;
    }
  }
}

// Segment summaries by the fixed weights of k_seg_tables: sum[4l ..] = d0 at the last row
// (sum_i w_i Delta_i), e0 at the first row (sum_i u_i Delta_i), psi at the first and the
// last row, for the nlines = nlong nseg contiguous segment lines l = L nseg + s of sn rows
// (Delta from the long line's neighbours; none past its ends).  One wave per segment line,
// lanes over its rows.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_seg_summary(const cpx<T>* __restrict__ data,
                                                          cpx<T>* __restrict__ sum,
                                                          const cpx<T>* __restrict__ wu,
                                                          int sn, int nseg, FDiv fseg,
                                                          int nlines) {
  constexpr int U = 4;
  const int lane = threadIdx.x & 63;
  const int l = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (l >= nlines) return;  // whole waves
  const int s = l - (int)fdiv((uint32_t)l, fseg) * nseg;
  const long long base = (long long)l * sn;
  const int r0 = s * sn;                 // the segment's first row in its long line
  const int N = nseg * sn;
  T wr = 0, wi = 0, ur = 0, ui = 0;
  for (int i0 = lane; i0 < sn; i0 += 64 * U) {
    cpx<T> pm[U], pc[U], pn[U], w[U], u[U];
    bool ok[U], hm[U], hn[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int i = i0 + 64 * q;
      ok[q] = i < sn;
      const int r = r0 + (ok[q] ? i : 0);
      hm[q] = ok[q] && r > 0;
      hn[q] = ok[q] && r + 1 < N;
      const long long ad = base + (ok[q] ? i : 0);
      pc[q] = data[ad];
      pm[q] = data[hm[q] ? ad - 1 : ad];
      pn[q] = data[hn[q] ? ad + 1 : ad];
      w[q] = wu[2LL * r];
      u[q] = wu[2LL * r + 1];
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      if (!ok[q]) continue;
      const cpx<T> zero{0, 0};
      const cpx<T> dl = (hm[q] ? pm[q] : zero) + (hn[q] ? pn[q] : zero) - (pc[q] + pc[q]);
      wr += w[q].re * dl.re - w[q].im * dl.im;
      wi += w[q].re * dl.im + w[q].im * dl.re;
      ur += u[q].re * dl.re - u[q].im * dl.im;
      ui += u[q].re * dl.im + u[q].im * dl.re;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    wr += __shfl_down(wr, off, 64);
    wi += __shfl_down(wi, off, 64);
    ur += __shfl_down(ur, off, 64);
    ui += __shfl_down(ui, off, 64);
  }
  if (lane == 0) {
    sum[4LL * l] = cpx<T>{wr, wi};
    sum[4LL * l + 1] = cpx<T>{ur, ui};
    sum[4LL * l + 2] = data[base];
    sum[4LL * l + 3] = data[base + sn - 1];
  }
}

// The same summaries for strided long lines (segment-major numbering l = s nlong + L, row
// r of line L at L + r ld): one thread per segment line walking its rows, adjacent
// threads on adjacent lines (coalesced).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_seg_summary_cols(const cpx<T>* __restrict__ data,
                                                               cpx<T>* __restrict__ sum,
                                                               const cpx<T>* __restrict__ wu,
                                                               int sn, int nseg, int nlong,
                                                               long long ld) {
  constexpr int U = 8;
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= nseg * nlong) return;
  const int s = gid / nlong, L = gid - s * nlong;
  const int r0 = s * sn;
  const long long base = (long long)L + (long long)r0 * ld;
  // rows r0 - 1 and r0 (the long line's row -1 is none); in-range loads, values selected
  // afterwards, real and imaginary parts apart (no arrays of the aligned pair type)
  const cpx<T> first = data[base];
  const cpx<T> before = data[s > 0 ? base - ld : base];
  cpx<T> pm{s > 0 ? before.re : (T)0, s > 0 ? before.im : (T)0}, pc = first;
  T wr = 0, wi = 0, ur = 0, ui = 0;
  const int N = nseg * sn;
  for (int e0 = 0; e0 < sn; e0 += U) {
    T nr[U], ni[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = r0 + e0 + u + 1;  // the next row of each of the U rows
      ok[u] = e0 + u < sn && r < N;
      const cpx<T> v = data[ok[u] ? base + (long long)(e0 + u + 1) * ld : base];
      nr[u] = v.re;
      ni[u] = v.im;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (e0 + u < sn) {
        const int r = r0 + e0 + u;
        const cpx<T> nxu{ok[u] ? nr[u] : (T)0, ok[u] ? ni[u] : (T)0};
        const cpx<T> dl = (pm + nxu) - (pc + pc);
        const cpx<T> w = wu[2LL * r], uu = wu[2LL * r + 1];
        wr += w.re * dl.re - w.im * dl.im;
        wi += w.re * dl.im + w.im * dl.re;
        ur += uu.re * dl.re - uu.im * dl.im;
        ui += uu.re * dl.im + uu.im * dl.re;
        pm = pc;
        pc = nxu;
      }
    }
  }
  sum[4LL * gid] = cpx<T>{wr, wi};
  sum[4LL * gid + 1] = cpx<T>{ur, ui};
  sum[4LL * gid + 2] = first;
  sum[4LL * gid + 3] = data[base + (long long)(sn - 1) * ld];
}

// Carries along each long line (one thread per line of nseg segments; segment lines
// l = L nseg + s, or s nlong + L with cols): C_0 = 0, C_(s+1) = P_s C_s + d0_s;
// E_nseg = 0, E_s = e0_s + Q_s C_s + P_s E_(s+1); car[4l ..] = C_s, E_(s+1), psi before the
// segment, psi after it.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_seg_carry(const cpx<T>* __restrict__ sum,
                                                        cpx<T>* __restrict__ car,
                                                        const cpx<T>* __restrict__ pq,
                                                        int nseg, int nlong, int cols) {
  const int L = blockIdx.x * blockDim.x + threadIdx.x;
  if (L >= nlong) return;
  // segment s of line L: l0 + s dl
  const long long l0 = cols ? (long long)L : (long long)L * nseg;
  const long long dl = cols ? (long long)nlong : 1;
  cpx<T> C{0, 0};
  for (int s = 0; s < nseg; ++s) {
    const long long l = l0 + s * dl;
    car[4 * l] = C;
    // in-range loads, values selected afterwards
    const cpx<T> before = sum[4 * (s > 0 ? l - dl : l) + 3];
    const cpx<T> after = sum[4 * (s + 1 < nseg ? l + dl : l) + 2];
    car[4 * l + 2] = cpx<T>{s > 0 ? before.re : (T)0, s > 0 ? before.im : (T)0};
    car[4 * l + 3] = cpx<T>{s + 1 < nseg ? after.re : (T)0, s + 1 < nseg ? after.im : (T)0};
    C = pq[2 * s] * C + sum[4 * l];
  }
  cpx<T> E{0, 0};
  for (int s = nseg - 1; s >= 0; --s) {
    const long long l = l0 + s * dl;
    car[4 * l + 1] = E;
    E = sum[4 * l + 1] + pq[2 * s + 1] * car[4 * l] + pq[2 * s] * E;
  }
}

}  // namespace gpdbec
