// Host-side entry points of the persistent multi-instance kernels (per precision).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "gp_batch.hpp"

namespace gpdbec {

template <typename T>
bool batch_size_ok(int n);
template <typename T>
size_t batch_lds(int pass, int n, int mode);
template <typename T>
void batch_tiles(int n0, int n1, int* nb_x, int* nb_conv, int* nb_col);
template <typename T>
hipError_t batch_launch(int pass, int mode, int cls, int grid, size_t lds, hipStream_t st,
                        char* base, const BDesc<T>* D, const WorkItem* work, int nwork);
template <typename T>
hipError_t batch_reserve_lds(int pass, int mode, int cls, size_t lds);
template <typename T>
hipError_t batch_finalize(int count, int mode, hipStream_t st, const BDesc<T>* D);

#define GP_DECLARE_BATCH(T)                                                              \
  template <> bool batch_size_ok<T>(int);                                                \
  template <> size_t batch_lds<T>(int, int, int);                                        \
  template <> void batch_tiles<T>(int, int, int*, int*, int*);                           \
  template <> hipError_t batch_launch<T>(int, int, int, int, size_t, hipStream_t, char*, \
                                         const BDesc<T>*, const WorkItem*, int);         \
  template <> hipError_t batch_reserve_lds<T>(int, int, int, size_t);                    \
  template <> hipError_t batch_finalize<T>(int, int, hipStream_t, const BDesc<T>*);
GP_DECLARE_BATCH(float)
GP_DECLARE_BATCH(double)
#undef GP_DECLARE_BATCH

}  // namespace gpdbec
