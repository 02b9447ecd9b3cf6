// Host-side entry points of the persistent multi-instance kernels (per precision).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "gp_batch.hpp"

namespace gpdbec {

template <typename T>
bool batch_size_ok(int n);
// LDS of pass `pass` (BP_*) for line length n (the pass's axis), mode, shape variant
template <typename T>
size_t batch_lds(int pass, int n, int mode, int shape);
// Work items (tiles) of one instance (axes n0, n1) in pass `pass` with shape variant
template <typename T>
int batch_tiles(int pass, int n0, int n1, int shape);
template <typename T>
hipError_t batch_launch(int pass, int mode, int cls, int shape, int grid, size_t lds,
                        hipStream_t st, char* base, const BDesc<T>* D, const WorkItem* work,
                        int nwork);
template <typename T>
hipError_t batch_reserve_lds(int pass, int mode, int cls, int shape, size_t lds);
template <typename T>
hipError_t batch_finalize(int count, int mode, hipStream_t st, const BDesc<T>* D);

#define GP_DECLARE_BATCH(T)                                                                \
  template <> bool batch_size_ok<T>(int);                                                  \
  template <> size_t batch_lds<T>(int, int, int, int);                                     \
  template <> int batch_tiles<T>(int, int, int, int);                                      \
  template <> hipError_t batch_launch<T>(int, int, int, int, int, size_t, hipStream_t,     \
                                         char*, const BDesc<T>*, const WorkItem*, int);    \
  template <> hipError_t batch_reserve_lds<T>(int, int, int, int, size_t);                 \
  template <> hipError_t batch_finalize<T>(int, int, hipStream_t, const BDesc<T>*);
GP_DECLARE_BATCH(float)
GP_DECLARE_BATCH(double)
#undef GP_DECLARE_BATCH

}  // namespace gpdbec
