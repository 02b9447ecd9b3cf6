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

// An axis the run-time-length kernels accept: even, at least 4, at most gen_max_line,
// and every prime factor at most 31.
template <typename T>
inline bool gen_size_ok(int n) {
  GPlan p;
  return n >= 4 && n % 2 == 0 && n <= gen_max_line<T>() && gen_plan(n, &p);
}

template <typename T>
struct GLaunch {
  // raises the dynamic LDS limit of the LDS-FFT kernels to 64 KiB (once per process;
  // called when a context is created, never inside a graph capture)
  static hipError_t prepare();
  // x passes: tile of the grid (line pairs per block) and its block count
  static GXTile xtile(int n0, int n1, int n2);
  static int x_blocks(int n0, int n1, int n2);
  // nonlinear / transpose tiles (32 x 32 of the two fastest axes)
  static int nl_blocks(int n0, int n1, int n2);
  static int col_blocks(int nlines) { return (nlines + kThreads - 1) / kThreads; }

  static hipError_t r2c_x(hipStream_t st, const cpx<T>* psi, cpx<T>* spec, const GPlan& p,
                          const cpx<T>* tw, double* part, int n0, int n1, int n2);
  static hipError_t c2r_x(hipStream_t st, const cpx<T>* spec, T* phi, const GPlan& p,
                          const cpx<T>* tw, int n0, int n1, int n2);
  // kind: GL_FWD, GL_INV, GL_CONV (ktab, km, scale used by GL_CONV only)
  static hipError_t lines(int kind, hipStream_t st, cpx<T>* data, int n, int nlines, int G,
                          long long so, long long si, long long se, const GPlan& p,
                          const cpx<T>* tw, const T* ktab, GKtab km, const double* scale);
  // mode: MODE_IMAG, MODE_REAL (write dst), MODE_OBSERVE (sums only)
  static hipError_t nl_transpose(int mode, hipStream_t st, const cpx<T>* psi, const T* V,
                                 const T* phi, const double* scale, cpx<T>* dst,
                                 const GStep& sc, int n0, int n1, int n2, double* part);
  static hipError_t transpose(hipStream_t st, const cpx<T>* src, cpx<T>* dst, int a, int b,
                              int nz);
  // sums: 0 none, 1 new-state sums, 2 observe only (no solve)
  static hipError_t cn_cols(int sums, hipStream_t st, cpx<T>* u, cpx<T>* dscr, const cpx<T>* f,
                            int n, int G, long long so, long long se, int nlines, double* part);
};

#define GP_DECLARE_GLAUNCH(T)                                                                  \
  template <> hipError_t GLaunch<T>::prepare();                                                \
  template <> GXTile GLaunch<T>::xtile(int, int, int);                                         \
  template <> int GLaunch<T>::x_blocks(int, int, int);                                         \
  template <> int GLaunch<T>::nl_blocks(int, int, int);                                        \
  template <> hipError_t GLaunch<T>::r2c_x(hipStream_t, const cpx<T>*, cpx<T>*, const GPlan&, \
                                           const cpx<T>*, double*, int, int, int);             \
  template <> hipError_t GLaunch<T>::c2r_x(hipStream_t, const cpx<T>*, T*, const GPlan&,      \
                                           const cpx<T>*, int, int, int);                      \
  template <> hipError_t GLaunch<T>::lines(int, hipStream_t, cpx<T>*, int, int, int,          \
                                           long long, long long, long long, const GPlan&,     \
                                           const cpx<T>*, const T*, GKtab, const double*);    \
  template <> hipError_t GLaunch<T>::nl_transpose(int, hipStream_t, const cpx<T>*, const T*,  \
                                                  const T*, const double*, cpx<T>*,           \
                                                  const GStep&, int, int, int, double*);      \
  template <> hipError_t GLaunch<T>::transpose(hipStream_t, const cpx<T>*, cpx<T>*, int, int, \
                                               int);                                           \
  template <> hipError_t GLaunch<T>::cn_cols(int, hipStream_t, cpx<T>*, cpx<T>*,              \
                                             const cpx<T>*, int, int, long long, long long,   \
                                             int, double*);
GP_DECLARE_GLAUNCH(float)
GP_DECLARE_GLAUNCH(double)
#undef GP_DECLARE_GLAUNCH

}  // namespace gpdbec
