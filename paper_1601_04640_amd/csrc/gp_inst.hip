// Instantiations of the pass kernels for one precision (GP_REAL) and one family of
// passes (GP_FAMILY), compiled once per combination so the build parallelises:
//   GP_FAMILY 0: x passes (r2c_x, c2r_nl_cnx)
//   GP_FAMILY 1: spectrum passes (fft_line, conv_line, conv_col)
//   GP_FAMILY 2: strided CN sweeps (cn_col) and tile queries
#include <hip/hip_ext.h>

#include "gp_kernels.hpp"
#include "gp_launch.hpp"

#ifndef GP_REAL
#error "GP_REAL must be float or double"
#endif
#ifndef GP_FAMILY
#error "GP_FAMILY must be 0, 1 or 2"
#endif

namespace gpdbec {
using T = GP_REAL;

#define GP_LAUNCH(kern, blocks, st, ...) \
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(kThreads), 0, st, __VA_ARGS__)

#if GP_FAMILY == 0
template <>
hipError_t Launch<T>::r2c_x_fin(int n0, int blocks, hipStream_t st, const cpx<T>* psi,
                                cpx<T>* spec, const cpx<T>* tw0, double* part, int n1, int n2,
                                const FinArgs& fa, int fin_mode, int nfin) {
  if (nfin < 1 || nfin > kStageMax) return hipErrorInvalidValue;
  if (fin_mode != FIN_IMAG && fin_mode != FIN_REAL) return hipErrorInvalidValue;
  const int nlead = (nfin + kFinLead - 1) / kFinLead * kFinLead;
  switch (n0) {
#define X(N)                                                                              \
  case N:                                                                                 \
    if (fin_mode == FIN_IMAG)                                                             \
      GP_LAUNCH((k_r2c_x_fin<T, N, FIN_IMAG>), blocks + nlead, st, psi, spec, tw0, part,  \
                n1, n2, fa, nfin, nlead);                                                 \
    else                                                                                  \
      GP_LAUNCH((k_r2c_x_fin<T, N, FIN_REAL>), blocks + nlead, st, psi, spec, tw0, part,  \
                n1, n2, fa, nfin, nlead);                                                 \
    break;
    GP_FOR_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <>
hipError_t Launch<T>::r2c_x(int n0, int blocks, hipStream_t st, const cpx<T>* psi,
                            cpx<T>* spec, const cpx<T>* tw0, double* part, int n1, int n2) {
  switch (n0) {
#define X(N)                                                                        \
  case N:                                                                           \
    GP_LAUNCH((k_r2c_x<T, N>), blocks, st, psi, spec, tw0, part, n1, n2);           \
    break;
    GP_FOR_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <>
hipError_t Launch<T>::c2r_nl_cnx(int n0, int mode, int blocks, hipStream_t st, cpx<T>* psi,
                                 const T* V, const double* scale, const cpx<T>* spec,
                                 const cpx<T>* tw0, const cpx<T>* cnm, const StepScalars& sc,
                                 double* part, T* phi_out, int n1, int n2,
                                 unsigned long long* stamps, hipEvent_t ev0, hipEvent_t ev1) {
  // with events: the launch records them from its own dispatch start/end timestamps
#define CASE_MODE(N, M)                                                                      \
  case M:                                                                                    \
    if (ev0 != nullptr) {                                                                    \
      hipExtLaunchKernelGGL((k_c2r_nl_cnx<T, N, M>), dim3(blocks), dim3(kThreads), 0, st,    \
                            ev0, ev1, 0, psi, V, scale, spec, tw0, cnm, sc, part, phi_out,   \
                            n1, n2, stamps);                                                 \
    } else {                                                                                 \
      GP_LAUNCH((k_c2r_nl_cnx<T, N, M>), blocks, st, psi, V, scale, spec, tw0, cnm, sc,     \
                part, phi_out, n1, n2, stamps);                                              \
    }                                                                                        \
    break;
  switch (n0) {
#define X(N)                               \
  case N:                                  \
    switch (mode) {                        \
      CASE_MODE(N, MODE_IMAG)              \
      CASE_MODE(N, MODE_REAL)              \
      CASE_MODE(N, MODE_OBSERVE)           \
      CASE_MODE(N, MODE_PHI)               \
      default:                             \
        return hipErrorInvalidValue;       \
    }                                      \
    break;
    GP_FOR_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
#undef CASE_MODE
  return hipGetLastError();
}

template <>
hipError_t Launch<T>::r2c_real(int n0, int blocks, hipStream_t st, const T* f, cpx<T>* spec,
                               const cpx<T>* tw0, int n1, int n2) {
  switch (n0) {
#define X(N)                                                                 \
  case N:                                                                    \
    GP_LAUNCH((k_r2c_real<T, N>), blocks, st, f, spec, tw0, n1, n2);         \
    break;
    GP_FOR_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <>
hipError_t Launch<T>::adj_x(int n0, int blocks, hipStream_t st, cpx<T>* lam, const cpx<T>* psin,
                            const T* V, const cpx<T>* spec, const cpx<T>* tw0,
                            const cpx<T>* cnm, const StepScalars& sc, T* sfield, double* gradV,
                            double* part, int n1, int n2) {
  switch (n0) {
#define X(N)                                                                          \
  case N:                                                                             \
    GP_LAUNCH((k_adj_x<T, N>), blocks, st, lam, psin, V, spec, tw0, cnm, sc, sfield, \
              gradV, part, n1, n2);                                                   \
    break;
    GP_FOR_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <>
hipError_t Launch<T>::adj_fin(int n0, int blocks, hipStream_t st, cpx<T>* lam,
                              const cpx<T>* psin, const T* sfield, const cpx<T>* spec,
                              const cpx<T>* tw0, const StepScalars& sc, int n1, int n2) {
  switch (n0) {
#define X(N)                                                                              \
  case N:                                                                                 \
    GP_LAUNCH((k_adj_fin<T, N>), blocks, st, lam, psin, sfield, spec, tw0, sc, n1, n2);  \
    break;
    GP_FOR_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
#endif

#if GP_FAMILY == 1
template <>
hipError_t Launch<T>::fft_line_fin(int n, int blocks, hipStream_t st, cpx<T>* data,
                                   const cpx<T>* tw, int nlines, const FinArgs& fa,
                                   int fin_mode) {
  switch (n) {
#define X(N)                                                                               \
  case N:                                                                                  \
    if (fin_mode == FIN_IMAG)                                                              \
      GP_LAUNCH((k_fft_line_fin<T, N, FIN_IMAG>), blocks + kFinLead, st, data, tw, nlines, fa); \
    else                                                                                   \
      GP_LAUNCH((k_fft_line_fin<T, N, FIN_REAL>), blocks + kFinLead, st, data, tw, nlines, fa); \
    break;
    GP_FOR_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <>
hipError_t Launch<T>::fft_line(int n, bool inv, int blocks, hipStream_t st, cpx<T>* data,
                               const cpx<T>* tw, int nlines) {
  switch (n) {
#define X(N)                                                                    \
  case N:                                                                       \
    if (inv)                                                                    \
      GP_LAUNCH((k_fft_line<T, N, true>), blocks, st, data, tw, nlines);        \
    else                                                                        \
      GP_LAUNCH((k_fft_line<T, N, false>), blocks, st, data, tw, nlines);       \
    break;
    GP_FOR_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <>
hipError_t Launch<T>::conv_line(int n, int blocks, hipStream_t st, cpx<T>* data, const T* ktab,
                                const double* scale, const cpx<T>* tw, int nlines) {
  switch (n) {
#define X(N)                                                                    \
  case N:                                                                       \
    GP_LAUNCH((k_conv_line<T, N>), blocks, st, data, ktab, scale, tw, nlines);  \
    break;
    GP_FOR_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <>
hipError_t Launch<T>::conv_col(int n2, int blocks, hipStream_t st, cpx<T>* spec, const T* ktab,
                               const double* scale, const cpx<T>* tw2, int n1) {
  switch (n2) {
#define X(N)                                                                    \
  case N:                                                                       \
    GP_LAUNCH((k_conv_col<T, N>), blocks, st, spec, ktab, scale, tw2, n1);      \
    break;
    GP_FOR_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
#endif

#if GP_FAMILY == 2
template <>
hipError_t Launch<T>::cn_col(int n, int mode, bool sums, int blocks, hipStream_t st,
                             cpx<T>* psi, const cpx<T>* cnm, double* part, int n0,
                             size_t estride, size_t ostride) {
#define CN(N, M, S) \
  GP_LAUNCH((k_cn_col<T, N, M, S>), blocks, st, psi, cnm, part, n0, estride, ostride)
  switch (n) {
#define X(N)                                        \
  case N:                                           \
    if (mode == MODE_OBSERVE) {                     \
      CN(N, MODE_OBSERVE, true);                    \
    } else if (mode == MODE_ADJ) {                  \
      CN(N, MODE_ADJ, false);                       \
    } else if (mode == MODE_IMAG) {                 \
      if (sums) CN(N, MODE_IMAG, true);             \
      else CN(N, MODE_IMAG, false);                 \
    } else if (mode == MODE_REAL) {                 \
      if (sums) CN(N, MODE_REAL, true);             \
      else CN(N, MODE_REAL, false);                 \
    } else {                                        \
      return hipErrorInvalidValue;                  \
    }                                               \
    break;
    GP_FOR_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
#undef CN
  return hipGetLastError();
}

template <>
int Launch<T>::tj(int n) {
  switch (n) {
#define X(N) \
  case N:    \
    return Tiles<T, N>::TJ;
    GP_FOR_SIZES(X)
#undef X
  }
  return 0;
}
template <>
int Launch<T>::tjw(int n) {
  switch (n) {
#define X(N) \
  case N:    \
    return Tiles<T, N>::TJW;
    GP_FOR_SIZES(X)
#undef X
  }
  return 0;
}
template <>
int Launch<T>::tc(int n) {
  switch (n) {
#define X(N) \
  case N:    \
    return Tiles<T, N>::TC;
    GP_FOR_SIZES(X)
#undef X
  }
  return 0;
}
template <>
int Launch<T>::tv(int n) {
  switch (n) {
#define X(N) \
  case N:    \
    return Tiles<T, N>::TV;
    GP_FOR_SIZES(X)
#undef X
  }
  return 0;
}
template <>
int Launch<T>::lbf(int n) {
  switch (n) {
#define X(N) \
  case N:    \
    return Tiles<T, N>::LBF;
    GP_FOR_SIZES(X)
#undef X
  }
  return 0;
}
template <>
int Launch<T>::lb(int n) {
  switch (n) {
#define X(N) \
  case N:    \
    return Tiles<T, N>::LB;
    GP_FOR_SIZES(X)
#undef X
  }
  return 0;
}
#endif

}  // namespace gpdbec
