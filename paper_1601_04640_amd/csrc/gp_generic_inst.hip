// Instantiations of the run-time-length pass kernels for one precision (GP_REAL).
#include <mutex>

#include "gp_generic.hpp"
#include "gp_generic_launch.hpp"

#ifndef GP_REAL
#error "GP_REAL must be float or double"
#endif

namespace gpdbec {
using T = GP_REAL;

// values of a block's lines per thread: 8 (FP32) or 4 (FP64) at 1024 threads, i.e. 64 KiB
constexpr int kEmax = (int)(65536 / (2 * sizeof(T))) / kGenThreads;
static_assert(kEmax * kGenThreads == gen_max_line<T>(), "one block holds the longest line");

namespace {
// lines per block of a line-FFT pass: about 2048 values, at most what 64 KiB of LDS
// holds, halved while the pass would have fewer than 512 blocks
int lines_per_block(int n, int nlines) {
  const int cap = gen_max_line<T>() / n;
  int nl = 2048 / n;
  if (nl < 1) nl = 1;
  if (nl > cap) nl = cap;
  while (nl > 1 && (nlines + nl - 1) / nl < 512) nl /= 2;
  return nl;
}
size_t lds_of(int values) { return (size_t)values * sizeof(cpx<T>); }
// threads of an LDS-FFT block holding `values`: whole waves, kEmax values each
dim3 threads_for(int values) {
  int w = (values + 64 * kEmax - 1) / (64 * kEmax);
  if (w < 1) w = 1;
  if (w > kGenThreads / 64) w = kGenThreads / 64;
  return dim3(64 * w);
}
}  // namespace

template <>
hipError_t GLaunch<T>::prepare() {
  static std::mutex mu;
  static bool done = false;
  std::lock_guard<std::mutex> lock(mu);
  if (done) return hipSuccess;
  const int lds = (int)lds_of(gen_max_line<T>());
  const void* ks[] = {
      reinterpret_cast<const void*>(&kg_lines<T, GL_FWD, kEmax, true>),
      reinterpret_cast<const void*>(&kg_lines<T, GL_INV, kEmax, true>),
      reinterpret_cast<const void*>(&kg_lines<T, GL_CONV, kEmax, true>),
      reinterpret_cast<const void*>(&kg_r2c_x<T, kEmax, true>),
      reinterpret_cast<const void*>(&kg_c2r_x<T, kEmax, true>),
      reinterpret_cast<const void*>(&kg_lines<T, GL_FWD, kEmax, false>),
      reinterpret_cast<const void*>(&kg_lines<T, GL_INV, kEmax, false>),
      reinterpret_cast<const void*>(&kg_lines<T, GL_CONV, kEmax, false>),
      reinterpret_cast<const void*>(&kg_r2c_x<T, kEmax, false>),
      reinterpret_cast<const void*>(&kg_c2r_x<T, kEmax, false>)};
  for (const void* k : ks) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
  }
  // the CN sweeps hold two buffers of up to 64 KiB
  const void* kc[] = {reinterpret_cast<const void*>(&kg_cn_lines<T, 0>),
                      reinterpret_cast<const void*>(&kg_cn_lines<T, 1>),
                      reinterpret_cast<const void*>(&kg_cn_lines<T, 2>)};
  for (const void* k : kc) {
    const hipError_t e =
        hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 2 * lds);
    if (e != hipSuccess) return e;
  }
  done = true;
  return hipSuccess;
}

template <>
GXTile GLaunch<T>::xtile(int n0, int n1, int n2) {
  GXTile xt{};
  xt.n0 = n0;
  xt.n1 = n1;
  xt.n2 = n2;
  const int pairs = n1 / 2;
  int np = gen_max_line<T>() / n0;   // pairs whose packed lines fit in LDS
  if (np > 8) np = 8;                // 16 consecutive y lines: 128-byte spectrum runs (FP64)
  if (np > pairs) np = pairs;
  if (np < 1) np = 1;
  // keep at least 512 blocks where the grid allows it
  while (np > 1 && (long long)n2 * ((pairs + np - 1) / np) < 512) np /= 2;
  xt.np = np;
  xt.nbj = (pairs + np - 1) / np;
  return xt;
}

template <>
int GLaunch<T>::x_blocks(int n0, int n1, int n2) {
  const GXTile xt = xtile(n0, n1, n2);
  return xt.nbj * n2;
}

template <>
int GLaunch<T>::cn_lines_per_block(int n, int nlines) {
  // two LDS buffers (psi and the recurrence values) of nl lines within 128 KiB; about
  // 4096 values per block, halved while the sweep would have fewer than 512 blocks
  const int cap = 2 * gen_max_line<T>() / (2 * n);
  int nl = 4096 / n;
  if (nl < 1) nl = 1;
  if (nl > cap) nl = cap;
  while (nl > 1 && (nlines + nl - 1) / nl < 512) nl /= 2;
  return nl;
}

template <>
hipError_t GLaunch<T>::r2c_x(hipStream_t st, const cpx<T>* psi, cpx<T>* spec, const GPlan& p,
                             const cpx<T>* tw, double* part, int n0, int n1, int n2) {
  const GXTile xt = xtile(n0, n1, n2);
  if (xt.np * n0 > gen_max_line<T>()) return hipErrorInvalidValue;
  // the block's reduction reuses the line buffer: at least 32 doubles
  const size_t lds_r2c = lds_of(xt.np * n0) < 256 ? 256 : lds_of(xt.np * n0);
  if (gen_plan_small(p))
    hipLaunchKernelGGL((kg_r2c_x<T, kEmax, true>), dim3(xt.nbj * n2), threads_for(xt.np * n0),
                       lds_r2c, st, psi, spec, xt, p, tw, part);
  else
    hipLaunchKernelGGL((kg_r2c_x<T, kEmax, false>), dim3(xt.nbj * n2), threads_for(xt.np * n0),
                       lds_r2c, st, psi, spec, xt, p, tw, part);
  return hipGetLastError();
}

template <>
hipError_t GLaunch<T>::c2r_x(hipStream_t st, const cpx<T>* spec, T* phi, const GPlan& p,
                             const cpx<T>* tw, int n0, int n1, int n2) {
  const GXTile xt = xtile(n0, n1, n2);
  if (xt.np * n0 > gen_max_line<T>()) return hipErrorInvalidValue;
  if (gen_plan_small(p))
    hipLaunchKernelGGL((kg_c2r_x<T, kEmax, true>), dim3(xt.nbj * n2), threads_for(xt.np * n0),
                       lds_of(xt.np * n0), st, spec, phi, xt, p, tw);
  else
    hipLaunchKernelGGL((kg_c2r_x<T, kEmax, false>), dim3(xt.nbj * n2), threads_for(xt.np * n0),
                       lds_of(xt.np * n0), st, spec, phi, xt, p, tw);
  return hipGetLastError();
}

template <>
hipError_t GLaunch<T>::lines(int kind, hipStream_t st, cpx<T>* data, int n, int nlines, int G,
                             long long so, long long si, long long se, const GPlan& p,
                             const cpx<T>* tw, const T* ktab, GKtab km, const double* scale) {
  if (n > gen_max_line<T>() || nlines < 1) return hipErrorInvalidValue;
  GLines g{};
  g.n = n;
  g.nlines = nlines;
  g.nl = lines_per_block(n, nlines);
  g.G = G;
  g.so = so;
  g.si = si;
  g.se = se;
  const int blocks = (nlines + g.nl - 1) / g.nl;
  const size_t lds = lds_of(g.nl * n);
  const bool small = gen_plan_small(p);
  switch (kind * 2 + (small ? 1 : 0)) {
#define GLINES(K, S)                                                                      \
  case K * 2 + (S ? 1 : 0):                                                               \
    hipLaunchKernelGGL((kg_lines<T, K, kEmax, S>), dim3(blocks), threads_for(g.nl * n), lds, st, \
                       data, g, p, tw, ktab, km, scale);                                  \
    break;
    GLINES(GL_FWD, true) GLINES(GL_FWD, false) GLINES(GL_INV, true) GLINES(GL_INV, false)
    GLINES(GL_CONV, true) GLINES(GL_CONV, false)
#undef GLINES
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <>
hipError_t GLaunch<T>::nonlinear(int mode, hipStream_t st, cpx<T>* psi, const T* V,
                                 const T* phi, const double* scale, const GStep& sc, int n0,
                                 int n1, int n2, double* part) {
  const int blocks = nl_blocks(n0, n1, n2);
  switch (mode) {
    case MODE_IMAG:
      hipLaunchKernelGGL((kg_nonlinear<T, MODE_IMAG>), dim3(blocks), dim3(kThreads), 0, st,
                         psi, V, phi, scale, sc, n0, n1, n2, part);
      break;
    case MODE_REAL:
      hipLaunchKernelGGL((kg_nonlinear<T, MODE_REAL>), dim3(blocks), dim3(kThreads), 0, st,
                         psi, V, phi, scale, sc, n0, n1, n2, part);
      break;
    case MODE_OBSERVE:
      hipLaunchKernelGGL((kg_nonlinear<T, MODE_OBSERVE>), dim3(blocks), dim3(kThreads), 0, st,
                         psi, V, phi, scale, sc, n0, n1, n2, part);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <>
hipError_t GLaunch<T>::cn_lines(int mode, hipStream_t st, cpx<T>* data, int n, int nlines,
                                int G, long long so, long long si, long long se,
                                const cpx<T>* f, double* part, cpx<T>* dscr) {
  if (n > gen_max_line<T>() || nlines < 1) return hipErrorInvalidValue;
  if (cn_by_columns(se != 1, nlines)) {
    // consecutive lines adjacent (si = 1): one thread per line
    if (si != 1) return hipErrorInvalidValue;
    const int blocks = (nlines + kThreads - 1) / kThreads;
    switch (mode) {
      case 0:
        hipLaunchKernelGGL((kg_cn_cols<T, false, false>), dim3(blocks), dim3(kThreads), 0, st,
                           data, dscr, f, n, G, so, se, nlines, part);
        break;
      case 1:
        hipLaunchKernelGGL((kg_cn_cols<T, true, false>), dim3(blocks), dim3(kThreads), 0, st,
                           data, dscr, f, n, G, so, se, nlines, part);
        break;
      case 2:
        hipLaunchKernelGGL((kg_cn_cols<T, false, true>), dim3(blocks), dim3(kThreads), 0, st,
                           data, dscr, f, n, G, so, se, nlines, part);
        break;
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  GLines g{};
  g.n = n;
  g.nlines = nlines;
  g.nl = cn_lines_per_block(n, nlines);
  g.G = G;
  g.so = so;
  g.si = si;
  g.se = se;
  const int blocks = (nlines + g.nl - 1) / g.nl;
  // psi lines, then the recurrence values (at least the block reduction's 64 bytes)
  const size_t one = lds_of(g.nl * n);
  const size_t lds = one + (one < 64 ? 64 : one);
  switch (mode) {
    case 0:
      hipLaunchKernelGGL((kg_cn_lines<T, 0>), dim3(blocks), dim3(kThreads), lds, st, data, g,
                         f, part);
      break;
    case 1:
      hipLaunchKernelGGL((kg_cn_lines<T, 1>), dim3(blocks), dim3(kThreads), lds, st, data, g,
                         f, part);
      break;
    case 2:
      hipLaunchKernelGGL((kg_cn_lines<T, 2>), dim3(blocks), dim3(kThreads), lds, st, data, g,
                         f, part);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace gpdbec
