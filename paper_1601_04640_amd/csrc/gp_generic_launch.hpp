// Host-side launchers of the run-time-length pass kernels (gp_generic.hpp), one
// instantiation per precision in gp_generic_inst.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "gp_generic.hpp"

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
  static int nl_blocks(int n0, int n1, int n2) { return cn_blocks(n0, n1 * n2, false); }
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
  // kind: GL_FWD, GL_INV, GL_CONV (ktab, km, scale used by GL_CONV only)
  static hipError_t lines(int kind, hipStream_t st, cpx<T>* data, int n, int nlines, int G,
                          long long so, long long si, long long se, const GPlan& p,
                          const cpx<T>* tw, const T* ktab, GKtab km, const double* scale);
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
                                           const cpx<T>*, const T*, GKtab, const double*);    \
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
