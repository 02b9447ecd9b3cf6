// Host-side launchers: map a runtime line length onto the compile-time specialised
// pass kernels.  Supported line lengths (every axis): even N = 2^a 3^b 5^c with
// b, c <= 1 and 8 <= N <= 512.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "gp_device.hpp"
#include "gp_finalize.hpp"

#define GP_FOR_SIZES(X) \
  X(8) X(10) X(12) X(16) X(20) X(24) X(30) X(32) X(40) X(48) X(60) X(64) X(80) X(96) X(120) \
  X(128) X(160) X(192) X(240) X(256) X(320) X(384) X(480) X(512)

namespace gpdbec {

struct StepScalars;

bool size_supported(int n);

template <typename T>
struct Launch {
  // tile geometry of the pass kernels for line length n
  static int tj(int n);  // x lines per block
  static int tjw(int n); // x lines per block of the single-grid R2C pass
  static int tc(int n);  // columns per block (strided passes)
  static int tv(int n);  // columns per block (z convolution)
  static int lb(int n);  // contiguous lines per block
  static int lbf(int n); // contiguous lines per block of the y FFT pass

  static hipError_t r2c_x(int n0, int blocks, hipStream_t st, const cpx<T>* psi, cpx<T>* spec,
                          const cpx<T>* tw0, double* part, int n1, int n2);
  static hipError_t fft_line(int n, bool inv, int blocks, hipStream_t st, cpx<T>* data,
                             const cpx<T>* tw, int nlines);
  // a step's x R2C / forward y FFT carrying the previous step's finalisation (mode
  // fin_mode; nfin blocks: 1 finalize block, or the first-stage slices)
  static hipError_t r2c_x_fin(int n0, int blocks, hipStream_t st, const cpx<T>* psi,
                              cpx<T>* spec, const cpx<T>* tw0, double* part, int n1, int n2,
                              const FinArgs& fa, int fin_mode, int nfin);
  static hipError_t fft_line_fin(int n, int blocks, hipStream_t st, cpx<T>* data,
                                 const cpx<T>* tw, int nlines, const FinArgs& fa, int fin_mode);
  static hipError_t conv_line(int n, int blocks, hipStream_t st, cpx<T>* data, const T* ktab,
                              const double* scale, const cpx<T>* tw, int nlines);
  static hipError_t conv_col(int n2, int blocks, hipStream_t st, cpx<T>* spec, const T* ktab,
                             const double* scale, const cpx<T>* tw2, int n1);
  static hipError_t c2r_nl_cnx(int n0, int mode, int blocks, hipStream_t st, cpx<T>* psi,
                               const T* V, const double* scale, const cpx<T>* spec,
                               const cpx<T>* tw0, const cpx<T>* cnm, const StepScalars& sc,
                               double* part, T* phi_out, int n1, int n2,
                               unsigned long long* stamps = nullptr, hipEvent_t ev0 = nullptr,
                               hipEvent_t ev1 = nullptr);
  // adjoint x passes
  static hipError_t r2c_real(int n0, int blocks, hipStream_t st, const T* f, cpx<T>* spec,
                             const cpx<T>* tw0, int n1, int n2);
  static hipError_t adj_x(int n0, int blocks, hipStream_t st, cpx<T>* lam, const cpx<T>* psin,
                          const T* V, const cpx<T>* spec, const cpx<T>* tw0, const cpx<T>* cnm,
                          const StepScalars& sc, T* sfield, double* gradV, double* part, int n1,
                          int n2);
  static hipError_t adj_fin(int n0, int blocks, hipStream_t st, cpx<T>* lam,
                            const cpx<T>* psin, const T* sfield, const cpx<T>* spec,
                            const cpx<T>* tw0, const StepScalars& sc, int n1, int n2);
  static hipError_t cn_col(int n, int mode, bool sums, int blocks, hipStream_t st, cpx<T>* psi,
                           const cpx<T>* cnm, double* part, int n0, size_t estride,
                           size_t ostride);
};

// The members are defined (explicitly specialised) per precision in gp_inst.hip.
#define GP_DECLARE_LAUNCH(T)                                                                  \
  template <> int Launch<T>::tj(int);                                                         \
  template <> int Launch<T>::tjw(int);                                                        \
  template <> int Launch<T>::tc(int);                                                         \
  template <> int Launch<T>::tv(int);                                                         \
  template <> int Launch<T>::lb(int);                                                         \
  template <> int Launch<T>::lbf(int);                                                        \
  template <> hipError_t Launch<T>::r2c_x(int, int, hipStream_t, const cpx<T>*, cpx<T>*,      \
                                          const cpx<T>*, double*, int, int);                   \
  template <> hipError_t Launch<T>::fft_line(int, bool, int, hipStream_t, cpx<T>*,             \
                                             const cpx<T>*, int);                              \
  template <> hipError_t Launch<T>::r2c_x_fin(int, int, hipStream_t, const cpx<T>*, cpx<T>*,  \
                                              const cpx<T>*, double*, int, int, const FinArgs&, \
                                              int, int);                                      \
  template <> hipError_t Launch<T>::fft_line_fin(int, int, hipStream_t, cpx<T>*,              \
                                                 const cpx<T>*, int, const FinArgs&, int);     \
  template <> hipError_t Launch<T>::conv_line(int, int, hipStream_t, cpx<T>*, const T*,       \
                                              const double*, const cpx<T>*, int);              \
  template <> hipError_t Launch<T>::conv_col(int, int, hipStream_t, cpx<T>*, const T*,        \
                                             const double*, const cpx<T>*, int);               \
  template <> hipError_t Launch<T>::c2r_nl_cnx(int, int, int, hipStream_t, cpx<T>*, const T*, \
                                               const double*, const cpx<T>*, const cpx<T>*,    \
                                               const cpx<T>*, const StepScalars&, double*, T*, \
                                               int, int, unsigned long long*, hipEvent_t,      \
                                               hipEvent_t);                                    \
  template <> hipError_t Launch<T>::r2c_real(int, int, hipStream_t, const T*, cpx<T>*,        \
                                             const cpx<T>*, int, int);                          \
  template <> hipError_t Launch<T>::adj_x(int, int, hipStream_t, cpx<T>*, const cpx<T>*,       \
                                          const T*, const cpx<T>*, const cpx<T>*,               \
                                          const cpx<T>*, const StepScalars&, T*, double*,       \
                                          double*, int, int);                                   \
  template <> hipError_t Launch<T>::adj_fin(int, int, hipStream_t, cpx<T>*, const cpx<T>*,     \
                                            const T*, const cpx<T>*, const cpx<T>*,             \
                                            const StepScalars&, int, int);                      \
  template <> hipError_t Launch<T>::cn_col(int, int, bool, int, hipStream_t, cpx<T>*,         \
                                           const cpx<T>*, double*, int, size_t, size_t);
GP_DECLARE_LAUNCH(float)
GP_DECLARE_LAUNCH(double)
#undef GP_DECLARE_LAUNCH

}  // namespace gpdbec
