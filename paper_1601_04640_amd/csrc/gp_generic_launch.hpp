// Host-side launchers of the run-time-length pass kernels (gp_generic.hpp), one
// instantiation per precision in gp_generic_inst.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "gp_generic.hpp"
#include "gp_long.hpp"

namespace gpdbec {

// Longest line one block transforms in LDS: 64 KiB of complex values (8 per thread of
// a 1024-thread block in FP32, 4 in FP64).
template <typename T>
constexpr int gen_max_line() {
  return (int)(65536 / (2 * sizeof(T)));
}

// An axis the run-time-length kernels accept: at least 4 points, with its FFT's LDS line
// (N, or Bluestein's M for lengths with a prime factor above 31) at most gen_max_line.
template <typename T>
inline bool gen_size_ok(int n) {
  GPlan p;
  return n >= 4 && n <= gen_max_line<T>() && gen_plan(n, &p) && p.m <= gen_max_line<T>();
}

// An axis of a 2D grid longer than one LDS line: the four-step FFT split n = A B (A >= B,
// the smallest such A; both transforms within one LDS line, two rows of A for the
// untangling of real lines) and the Crank-Nicolson segments (nseg segments of sn rows: the
// largest divisor of n from 64 to 512, one wave per segment with at most 8 rows per lane
// and several segments per block; failing that the largest one tile sweep holds).
struct GLong {
  int A, B;
  int sn, nseg;
};

// Plan of a factor of a split axis: a factor with a prime above 7 runs Bluestein's
// algorithm through a 2-3-5-7 length when that fits `lim` (the radix 11-31 kernels keep
// values in scratch memory), else its own stages.
inline bool gen_long_subplan(int n, int lim, GPlan* p) {
  if (!gen_plan(n, p)) return false;
  if (p->blue || gen_plan_small(*p)) return true;
  GPlan q = *p;
  q.m = gen_blue_len(n);
  q.blue = 1;
  if (q.m <= lim && gen_stages(q.m, &q)) {
    q.fm = fdiv_make((uint32_t)q.m);
    *p = q;
  }
  return true;
}

// Crank-Nicolson segments of a line: the largest divisor of n from 64 to 512 with at
// least two segments (one wave per segment, at most 8 rows per lane).
inline bool gen_seg_split(int n, int* sn, int* nseg) {
  for (int s = 512; s >= 64; --s) {
    if (n % s == 0 && n / s >= 2) {
      *sn = s;
      *nseg = n / s;
      return true;
    }
  }
  return false;
}

template <typename T>
inline bool gen_long_plan(int n, GLong* lp) {
  const int lim = gen_max_line<T>();
  if (n <= lim) return false;
  lp->A = lp->B = lp->sn = lp->nseg = 0;
  int a = 1;
  while ((long long)a * a < n) ++a;
  for (; a <= lim; ++a) {
    if (n % a) continue;
    GPlan pa, pb;
    const int b = n / a;
    if (b >= 2 && gen_long_subplan(a, lim / 2, &pa) && gen_long_subplan(b, lim, &pb) &&
        2 * pa.m <= lim && pb.m <= lim) {
      lp->A = a;
      lp->B = b;
      break;
    }
  }
  if (lp->A == 0) return false;
  if (gen_seg_split(n, &lp->sn, &lp->nseg)) return true;
  for (int s = lim; s >= 64; --s) {
    if (n % s == 0 && n / s >= 2) {
      lp->sn = s;
      lp->nseg = n / s;
      return true;
    }
  }
  return false;
}

// LDS line stride of an axis's FFT: N, or Bluestein's M.
inline int gen_stride(int n) {
  GPlan p;
  return gen_plan(n, &p) ? p.m : n;
}

template <typename T>
struct GLaunch {
  // raises the dynamic LDS limit of the LDS-FFT kernels to 128 KiB and of the CN sweeps to
  // 159 KiB (once per process; called when a context is created, never inside a graph
  // capture)
  static hipError_t prepare();
  // x passes: tile of the grid (line pairs per block) and its block count
  static GXTile xtile(int n0, int n1, int n2);
  static int x_blocks(int n0, int n1, int n2);
  // blocks of the nonlinear pass (partial-sum slots) and of a CN sweep over nlines lines
  // (the x sweep's, which carries the nonlinear sub-step and its sums)
  static int nl_blocks(int n0, int n1, int n2) {
    if (n0 > gen_max_line<T>()) {  // a long x axis: the nonlinear pass runs on its own
      const long long b = (long long)n0 * n1 * n2 / 4096;
      return (int)(b < 256 ? 256 : (b > 16384 ? 16384 : b));
    }
    return cn_blocks(n0, n1 * n2, false);
  }
  // CN sweeps: kg_cn_tile with wpl waves per line (1 up to kTileMaxN points, then one
  // lane per 8 rows) and cn_tile_lines lines per block, except strided sweeps of many
  // lines longer than kTileMaxN, which run one thread per line (kg_cn_cols)
  static int cn_tile_wpl(int n) {
    int w = 1;
    while (n > kTileMaxN && 64 * 8 * w < n) w *= 2;
    return w;
  }
  static int cn_tile_lines(int n, int nlines, bool strided);
  static constexpr int kColLines = 32768;
  static bool cn_by_columns(int n, bool strided, int nlines) {
    return n > kTileMaxN && strided && nlines >= kColLines;
  }
  static int cn_blocks(int n, int nlines, bool strided) {
    if (cn_by_columns(n, strided, nlines)) return (nlines + kThreads - 1) / kThreads;
    const int nl = cn_tile_lines(n, nlines, strided);
    return (nlines + nl - 1) / nl;
  }
  // 2D y sweeps of lines longer than kTileMaxN run on a transposed copy of the state
  // (lines of the copy are contiguous), through the scratch grid
  static bool y2d_transposed(int n1) { return n1 > kTileMaxN; }

  static hipError_t r2c_x(hipStream_t st, const cpx<T>* psi, cpx<T>* spec, const GPlan& p,
                          const cpx<T>* tw, double* part, int n0, int n1, int n2);
  static hipError_t c2r_x(hipStream_t st, const cpx<T>* spec, T* phi, const GPlan& p,
                          const cpx<T>* tw, int n0, int n1, int n2);
  // kind: GL_FWD, GL_INV, GL_CONV (ktab, km, scale used by GL_CONV only); w4: the
  // four-step twiddle of the outer passes of a split axis (GL_FWD after, GL_INV before the
  // transform; the line's column l / G if w4hi, else l mod G)
  static hipError_t lines(int kind, hipStream_t st, cpx<T>* data, int n, int nlines, int G,
                          long long so, long long si, long long se, const GPlan& p,
                          const cpx<T>* tw, const T* ktab, GKtab km, const double* scale,
                          const cpx<T>* w4 = nullptr, int w4hi = 0);
  // long x axis (2D): geometry, blocks of the forward column pass (its x-partial slots),
  // and the two passes each way: psi -> w (grid of ceil(n1/2) n0 values) -> spec, and
  // spec -> w -> phi; pa, pb: plans of the A- and B-point transforms, twa, twb their
  // stage twiddles, w4 = W_N^m
  static GLX lx_geom(int n0, int n1, const GLong& lp, const GPlan& pa, const GPlan& pb);
  static int lx_blocks(const GLX& x) { return x.np * x.nat; }
  static hipError_t lx_r2c(hipStream_t st, const cpx<T>* psi, cpx<T>* w, cpx<T>* spec,
                           const GLX& x, const GPlan& pa, const GPlan& pb, const cpx<T>* twa,
                           const cpx<T>* twb, const cpx<T>* w4, double* part);
  static hipError_t lx_c2r(hipStream_t st, const cpx<T>* spec, cpx<T>* w, T* phi,
                           const GLX& x, const GPlan& pa, const GPlan& pb, const cpx<T>* twa,
                           const cpx<T>* twb, const cpx<T>* w4);
  // segmented CN sweep of nlong contiguous lines of nseg segments of sn rows (mode 0:
  // solve, 1: solve with the new-state sums in part over seg_blocks blocks); f: the long
  // line's factor table, pq: the segments' carry products P, Q (2 nseg values) followed by
  // the rows' summary weights (2 per row); sum, car: 4 values per segment
  // ld = 0: contiguous long lines (line L at L nseg sn); ld > 0: strided long lines,
  // line L at L, row r at r ld (consecutive lines adjacent), swept in place
  static int seg_lines(int sn, int nlines, bool cols = false);
  static int seg_blocks(int sn, int nlines, bool cols = false) {
    const int nl = seg_lines(sn, nlines, cols);
    return (nlines + nl - 1) / nl;
  }
  static hipError_t seg_sweep(int mode, hipStream_t st, cpx<T>* data, int sn, int nseg,
                              int nlong, const cpx<T>* f, const cpx<T>* pq, cpx<T>* sum,
                              cpx<T>* car, double* part, long long ld = 0);
  // the nonlinear sub-step's sums of the stored state (mode MODE_OBSERVE; MODE_IMAG and
  // MODE_REAL also apply it in place), over nl_blocks blocks
  static hipError_t nonlinear(int mode, hipStream_t st, cpx<T>* psi, const T* V, const T* phi,
                              const double* scale, const GStep& sc, int n0, int n1, int n2,
                              double* part);
  // CN sweep of nlines lines (addressing as `lines`); mode 0 solve, 1 solve + new-state
  // sums, 2 sums of the stored state only (strided sweeps of many long lines run
  // kg_cn_cols, with dscr: a grid of scratch values)
  static hipError_t cn_lines(int mode, hipStream_t st, cpx<T>* data, int n, int nlines, int G,
                             long long so, long long si, long long se, const cpx<T>* f,
                             double* part, cpx<T>* dscr);
  // out[c rows + r] = in[r cols + c]: a rows x cols grid of complex values transposed
  static hipError_t transpose(hipStream_t st, const cpx<T>* in, cpx<T>* out, int rows,
                              int cols);
  // the x sweep (lines (j, k) of n0 points) with the nonlinear sub-step of MODE_IMAG /
  // MODE_REAL fused into its loads; nlz.part: the nl_blocks seven-sum slots
  static hipError_t cn_x_nonlinear(int mode, hipStream_t st, cpx<T>* psi, int n0, int lines,
                                   const cpx<T>* f, const GNl& nlz);
};

#define GP_DECLARE_GLAUNCH(T)                                                                  \
  template <> hipError_t GLaunch<T>::prepare();                                                \
  template <> GXTile GLaunch<T>::xtile(int, int, int);                                         \
  template <> int GLaunch<T>::x_blocks(int, int, int);                                         \
  template <> int GLaunch<T>::cn_tile_lines(int, int, bool);                                   \
  template <> hipError_t GLaunch<T>::r2c_x(hipStream_t, const cpx<T>*, cpx<T>*, const GPlan&, \
                                           const cpx<T>*, double*, int, int, int);             \
  template <> hipError_t GLaunch<T>::c2r_x(hipStream_t, const cpx<T>*, T*, const GPlan&,      \
                                           const cpx<T>*, int, int, int);                      \
  template <> hipError_t GLaunch<T>::lines(int, hipStream_t, cpx<T>*, int, int, int,          \
                                           long long, long long, long long, const GPlan&,     \
                                           const cpx<T>*, const T*, GKtab, const double*,     \
                                           const cpx<T>*, int);                               \
  template <> GLX GLaunch<T>::lx_geom(int, int, const GLong&, const GPlan&, const GPlan&);    \
  template <> hipError_t GLaunch<T>::lx_r2c(hipStream_t, const cpx<T>*, cpx<T>*, cpx<T>*,    \
                                            const GLX&, const GPlan&, const GPlan&,          \
                                            const cpx<T>*, const cpx<T>*, const cpx<T>*,     \
                                            double*);                                          \
  template <> hipError_t GLaunch<T>::lx_c2r(hipStream_t, const cpx<T>*, cpx<T>*, T*,         \
                                            const GLX&, const GPlan&, const GPlan&,          \
                                            const cpx<T>*, const cpx<T>*, const cpx<T>*);    \
  template <> int GLaunch<T>::seg_lines(int, int, bool);                                       \
  template <> hipError_t GLaunch<T>::seg_sweep(int, hipStream_t, cpx<T>*, int, int, int,      \
                                               const cpx<T>*, const cpx<T>*, cpx<T>*,         \
                                               cpx<T>*, double*, long long);                   \
  template <> hipError_t GLaunch<T>::nonlinear(int, hipStream_t, cpx<T>*, const T*, const T*, \
                                               const double*, const GStep&, int, int, int,    \
                                               double*);                                       \
  template <> hipError_t GLaunch<T>::cn_lines(int, hipStream_t, cpx<T>*, int, int, int,       \
                                              long long, long long, long long, const cpx<T>*, \
                                              double*, cpx<T>*);                               \
  template <> hipError_t GLaunch<T>::cn_x_nonlinear(int, hipStream_t, cpx<T>*, int, int,     \
                                                    const cpx<T>*, const GNl&);              \
  template <> hipError_t GLaunch<T>::transpose(hipStream_t, const cpx<T>*, cpx<T>*, int, int);
GP_DECLARE_GLAUNCH(float)
GP_DECLARE_GLAUNCH(double)
#undef GP_DECLARE_GLAUNCH

}  // namespace gpdbec
