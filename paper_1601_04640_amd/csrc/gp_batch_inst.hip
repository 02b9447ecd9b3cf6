// Persistent multi-instance kernels for one precision (GP_REAL) and their launcher.
// (Item-loop kernels: see thread_idx.)
#define GP_ITEM_LOOP_KERNELS
#include "gp_batch.hpp"
#include "gp_batch_launch.hpp"

#include <mutex>

#ifndef GP_REAL
#error "GP_REAL must be float or double"
#endif

namespace gpdbec {
using T = GP_REAL;

template <>
bool batch_size_ok<T>(int n) {
  switch (n) {
#define X(N) case N:
    GP_BATCH_SIZES(X)
#undef X
    return true;
    default:
      return false;
  }
}

template <int S>
static size_t lds_of_shape(int pass, int n, int mode) {
  switch (n) {
#define X(N)                                                                   \
  case N:                                                                      \
    switch (pass) {                                                            \
      case BP_R2C: return lds_bytes<T, N, P_R2C, S>();                         \
      case BP_CONV: return lds_bytes<T, N, P_CONV_LINE, S>();                  \
      case BP_C2R:                                                             \
        return (mode == MODE_OBSERVE) ? lds_bytes<T, N, P_C2R_OBS, S>()        \
                                      : lds_bytes<T, N, P_C2R_STEP, S>();      \
      case BP_CN: return lds_bytes<T, N, P_CN_COL, S>();                       \
      default: return 0;                                                       \
    }
    GP_BATCH_SIZES(X)
#undef X
    default:
      return 0;
  }
}

template <>
size_t batch_lds<T>(int pass, int n, int mode, int shape) {
  return shape == 1 ? lds_of_shape<1>(pass, n, mode) : lds_of_shape<0>(pass, n, mode);
}

template <int S>
static int tiles_of_shape(int pass, int n0, int n1) {
  int tj = 0, lb = 0, tc = 0;
  switch (n0) {
#define X(N)                     \
  case N:                        \
    tj = Tiles<T, N, S>::TJ;     \
    break;
    GP_BATCH_SIZES(X)
#undef X
  }
  switch (n1) {
#define X(N)                     \
  case N:                        \
    lb = Tiles<T, N, S>::LB;     \
    tc = Tiles<T, N, S>::TC;     \
    break;
    GP_BATCH_SIZES(X)
#undef X
  }
  if (tj == 0 || lb == 0 || tc == 0) return 0;
  switch (pass) {
    case BP_R2C:
    case BP_C2R: return (n1 + tj - 1) / tj;          // x tiles
    case BP_CONV: return (n0 / 2 + 1 + lb - 1) / lb; // y-line blocks of the half spectrum
    case BP_CN: return (n0 + tc - 1) / tc;           // y column tiles
    default: return 0;
  }
}

template <>
int batch_tiles<T>(int pass, int n0, int n1, int shape) {
  return shape == 1 ? tiles_of_shape<1>(pass, n0, n1) : tiles_of_shape<0>(pass, n0, n1);
}

template <typename K>
static hipError_t launch_dyn(K kern, int grid, size_t lds, hipStream_t st, char* base,
                             const BDesc<T>* D, const WorkItem* work, int nwork) {
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), lds, st, base, D, work, nwork);
  return hipGetLastError();
}

// The kernel behind (pass, mode, class, shape), as an untyped function pointer.
template <int CLS, int S>
static const void* kernel_of(int pass, int mode) {
  switch (pass) {
    case BP_R2C: return reinterpret_cast<const void*>(kb_r2c_x<T, 0, CLS, S>);
    case BP_CONV: return reinterpret_cast<const void*>(kb_conv_y<T, 0, CLS, S>);
    case BP_C2R:
      if (mode == MODE_IMAG) return reinterpret_cast<const void*>(kb_c2r_nl_cnx<T, MODE_IMAG, CLS, S>);
      if (mode == MODE_REAL) return reinterpret_cast<const void*>(kb_c2r_nl_cnx<T, MODE_REAL, CLS, S>);
      return reinterpret_cast<const void*>(kb_c2r_nl_cnx<T, MODE_OBSERVE, CLS, S>);
    case BP_CN:
      if (mode == MODE_IMAG) return reinterpret_cast<const void*>(kb_cn_y<T, MODE_IMAG, CLS, S>);
      return reinterpret_cast<const void*>(kb_cn_y<T, MODE_REAL, CLS, S>);
    default: return nullptr;
  }
}

template <>
hipError_t batch_reserve_lds<T>(int pass, int mode, int cls, int shape, size_t lds) {
  // Raise (never lower) the kernel's dynamic-LDS limit; called outside stream capture.
  static std::mutex mu;
  static size_t have[BP_COUNT][3][kBatchClasses][kBatchShapes] = {};
  if (pass < 0 || pass >= BP_COUNT || mode < 0 || mode > MODE_OBSERVE || cls < 0 ||
      cls >= kBatchClasses || shape < 0 || shape >= kBatchShapes)
    return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lock(mu);
  size_t& h = have[pass][mode][cls][shape];
  if (lds <= h) return hipSuccess;
  const void* k = cls == 0 ? (shape == 0 ? kernel_of<0, 0>(pass, mode) : kernel_of<0, 1>(pass, mode))
                           : (shape == 0 ? kernel_of<1, 0>(pass, mode) : kernel_of<1, 1>(pass, mode));
  const hipError_t e =
      hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess) h = lds;
  return e;
}

template <int CLS, int S>
static hipError_t launch_class(int pass, int mode, int grid, size_t lds, hipStream_t st,
                               char* base, const BDesc<T>* D, const WorkItem* work, int nwork) {
  switch (pass) {
    case BP_R2C:
      return launch_dyn(kb_r2c_x<T, 0, CLS, S>, grid, lds, st, base, D, work, nwork);
    case BP_CONV:
      return launch_dyn(kb_conv_y<T, 0, CLS, S>, grid, lds, st, base, D, work, nwork);
    case BP_C2R:
      if (mode == MODE_IMAG)
        return launch_dyn(kb_c2r_nl_cnx<T, MODE_IMAG, CLS, S>, grid, lds, st, base, D, work, nwork);
      if (mode == MODE_REAL)
        return launch_dyn(kb_c2r_nl_cnx<T, MODE_REAL, CLS, S>, grid, lds, st, base, D, work, nwork);
      return launch_dyn(kb_c2r_nl_cnx<T, MODE_OBSERVE, CLS, S>, grid, lds, st, base, D, work, nwork);
    case BP_CN:
      if (mode == MODE_IMAG)
        return launch_dyn(kb_cn_y<T, MODE_IMAG, CLS, S>, grid, lds, st, base, D, work, nwork);
      return launch_dyn(kb_cn_y<T, MODE_REAL, CLS, S>, grid, lds, st, base, D, work, nwork);
    default:
      return hipErrorInvalidValue;
  }
}

template <>
hipError_t batch_launch<T>(int pass, int mode, int cls, int shape, int grid, size_t lds,
                           hipStream_t st, char* base, const BDesc<T>* D, const WorkItem* work,
                           int nwork) {
  if (grid <= 0 || nwork <= 0) return hipSuccess;
  if (cls == 0)
    return shape == 0 ? launch_class<0, 0>(pass, mode, grid, lds, st, base, D, work, nwork)
                      : launch_class<0, 1>(pass, mode, grid, lds, st, base, D, work, nwork);
  return shape == 0 ? launch_class<1, 0>(pass, mode, grid, lds, st, base, D, work, nwork)
                    : launch_class<1, 1>(pass, mode, grid, lds, st, base, D, work, nwork);
}

template <>
hipError_t batch_finalize<T>(int count, int mode, hipStream_t st, const BDesc<T>* D) {
  hipLaunchKernelGGL(kb_finalize<T>, dim3(count), dim3(kThreads), 0, st, D, mode);
  return hipGetLastError();
}

}  // namespace gpdbec
