// Batched ensemble of independent quasi-2D instances (XY or XZ planes) of uneven sizes:
// one persistent launch per pass covers every instance.  Each launch walks a work list
// of (instance, tile) items sorted by decreasing cost; block b takes items b, b + G,
// b + 2G, ... (G = launched blocks, chosen by the autotuner).  The per-instance
// descriptor points into that instance's own workspace region, laid out exactly like a
// single-grid context, so the tile bodies are the single-grid ones.
#pragma once
#include "gp_kernels.hpp"

// Line lengths the batched kernels are specialised for (every axis of every instance);
// the kernel switches below list the same sizes.
#define GP_BATCH_SIZES(X) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512)

namespace gpdbec {

// Tile-shape variants per pass and size class (Tiles<T, N, S>), chosen by the autotuner.
constexpr int kBatchShapes = 2;

// Per-instance descriptor.  Arrays are byte offsets from the batch workspace base, which
// the kernels receive as an argument: pointers formed from a kernel argument keep the
// global address space (pointers loaded from memory would fall back to flat accesses with
// 64-bit per-lane addresses).
template <typename T>
struct BDesc {
  size_t psi, V, spec, ktab, tw0, tw1;
  size_t cn0[2];  // x-axis factor tables: [imaginary, real time]
  size_t cn1[2];  // second-axis factor tables
  size_t p_x, p_nl, p_col, scale;
  StepScalars sc;  // step scalars (dt, couplings, spacings)
  int n0, n1;
  FinArgs fa;      // FP64 finalisation of this instance
};

template <typename X>
__device__ __forceinline__ X* bptr(char* base, size_t off) {
  return reinterpret_cast<X*>(base + off);
}

struct WorkItem {
  int inst;
  int tile;
};

enum : int { BP_R2C = 0, BP_CONV = 1, BP_C2R = 2, BP_CN = 3, BP_COUNT = 4 };

// Size classes: a single switch over all nine sizes exceeds the register allocator's
// budget when the 384/512 bodies sit beside the smaller ones, so each pass has one
// persistent kernel per class (<= 256 and 384/512), each over its own work list.
#define GP_BATCH_CLASS0(X) X(32) X(48) X(64) X(96) X(128) X(192) X(256)
#define GP_BATCH_CLASS1(X) X(384) X(512)
constexpr int kBatchClasses = 2;
__host__ __device__ constexpr int batch_class(int n) { return n > 256 ? 1 : 0; }

// Dynamic LDS: the largest body of the pass and class present is requested at launch.
// Every block walks items blockIdx.x + k gridDim.x of the work list.
#define GP_BATCH_KERNEL(NAME, AXIS, BODY)                                              \
  template <typename T, int MODE, int CLS, int S>                                      \
  __global__ __launch_bounds__(kThreads) void NAME(char* __restrict__ base,             \
                                                   const BDesc<T>* __restrict__ D,     \
                                                   const WorkItem* __restrict__ work,  \
                                                   int nwork) {                        \
    extern __shared__ __attribute__((aligned(16))) char lds[];                         \
    constexpr int K = (MODE == MODE_REAL) ? 1 : 0;                                     \
    (void)K;                                                                           \
    for (int w = blockIdx.x; w < nwork; w += gridDim.x) {                              \
      const WorkItem item = work[w];                                                   \
      const BDesc<T>& d = D[item.inst];                                                \
      if constexpr (CLS == 0) {                                                        \
        switch (d.AXIS) { GP_BATCH_CLASS0(BODY) default: break; }                      \
      } else {                                                                         \
        switch (d.AXIS) { GP_BATCH_CLASS1(BODY) default: break; }                      \
      }                                                                                \
      __syncthreads();                                                                 \
    }                                                                                  \
  }

#define GP_BODY_R2C(N)                                                                  \
  case N:                                                                               \
    r2c_x_body<T, N, S>(bptr<cpx<T>>(base, d.psi), bptr<cpx<T>>(base, d.spec),           \
                     bptr<cpx<T>>(base, d.tw0), bptr<double>(base, d.p_x), d.n1, 1,      \
                     item.tile, lds);                                                     \
    break;
#define GP_BODY_CONV(N)                                                                 \
  case N:                                                                               \
    conv_line_body<T, N, S>(bptr<cpx<T>>(base, d.spec), bptr<T>(base, d.ktab),           \
                         bptr<double>(base, d.scale), bptr<cpx<T>>(base, d.tw1),         \
                         d.n0 / 2 + 1, item.tile, lds);                                  \
    break;
#define GP_BODY_C2R(N)                                                                  \
  case N:                                                                               \
    c2r_nl_cnx_body<T, N, MODE, S>(bptr<cpx<T>>(base, d.psi), bptr<T>(base, d.V),        \
                                bptr<double>(base, d.scale), bptr<cpx<T>>(base, d.spec), \
                                bptr<cpx<T>>(base, d.tw0), bptr<cpx<T>>(base, d.cn0[K]), \
                                d.sc, bptr<double>(base, d.p_nl), nullptr, d.n1, 1,      \
                                item.tile, lds);                                         \
    break;
#define GP_BODY_CN(N)                                                                   \
  case N:                                                                               \
    cn_col_body<T, N, MODE, true, S>(bptr<cpx<T>>(base, d.psi), bptr<cpx<T>>(base, d.cn1[K]), \
                                  bptr<double>(base, d.p_col), d.n0, (size_t)d.n0,        \
                                  (size_t)d.n0 * d.n1, item.tile, lds);                   \
    break;
GP_BATCH_KERNEL(kb_r2c_x, n0, GP_BODY_R2C)
GP_BATCH_KERNEL(kb_conv_y, n1, GP_BODY_CONV)
GP_BATCH_KERNEL(kb_c2r_nl_cnx, n0, GP_BODY_C2R)
GP_BATCH_KERNEL(kb_cn_y, n1, GP_BODY_CN)
#undef GP_BODY_R2C
#undef GP_BODY_CONV
#undef GP_BODY_C2R
#undef GP_BODY_CN
#undef GP_BATCH_KERNEL

// One block per instance.
template <typename T>
__global__ __launch_bounds__(kThreads) void kb_finalize(const BDesc<T>* __restrict__ D,
                                                        int mode) {
  finalize_block(D[blockIdx.x].fa, mode);
}

}  // namespace gpdbec
