// Instantiations of the run-time-length pass kernels for one precision (GP_REAL).
#include <algorithm>
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
constexpr int kCnLds = 163840;  // LDS limit of the CN sweeps (160 KiB)
constexpr int kTileLds = kCnLds - 2048;  // dynamic LDS of the tile sweeps (static: 1408 B)

// lines per block of a line-FFT pass whose lines take ls values of LDS (the plan's
// stride): about 2048 values (contiguous lines) or as many lines as 64 KiB of LDS holds
// (strided lines: the longest contiguous runs), halved while the pass would have fewer
// than 512 blocks
int lines_per_block(int ls, int nlines, bool strided) {
  const int cap = gen_max_line<T>() / ls;
  int nl = strided ? cap : 2048 / ls;
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
  // lines of up to gen_max_line values and the twiddle table
  const int lds = (int)lds_of(2 * gen_max_line<T>());
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
      reinterpret_cast<const void*>(&kg_c2r_x<T, kEmax, false>),
      reinterpret_cast<const void*>(&kg_lines<T, GL_FWD, kEmax, true, true>),
      reinterpret_cast<const void*>(&kg_lines<T, GL_INV, kEmax, true, true>),
      reinterpret_cast<const void*>(&kg_lines<T, GL_CONV, kEmax, true, true>),
      reinterpret_cast<const void*>(&kg_r2c_x<T, kEmax, true, true>),
      reinterpret_cast<const void*>(&kg_c2r_x<T, kEmax, true, true>),
#define GLX_KERNELS(S, B)                                                        \
  reinterpret_cast<const void*>(&kg_lx_cols_fwd<T, kEmax, S, B>),               \
      reinterpret_cast<const void*>(&kg_lx_rows_fwd<T, kEmax, S, B>),           \
      reinterpret_cast<const void*>(&kg_lx_rows_inv<T, kEmax, S, B>),           \
      reinterpret_cast<const void*>(&kg_lx_cols_inv<T, kEmax, S, B>)
      GLX_KERNELS(true, false), GLX_KERNELS(false, false), GLX_KERNELS(true, true)
#undef GLX_KERNELS
  };
  for (const void* k : ks) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
  }
  // the tile sweeps: up to 16 padded lines (or one line of 8192 FP32 / 4096 FP64 points)
  // and the factor table, beside the static reduction and scan space
#define GP_TILE_K(M, NL, TSV, SG, WIV) reinterpret_cast<const void*>(&kg_cn_tile<T, M, NL, TSV, SG, WIV>)
#define GP_TILE_TS(M, NL, SG, WIV) GP_TILE_K(M, NL, 8, SG, WIV), GP_TILE_K(M, NL, kTileS, SG, WIV)
#define GP_TILE_ALL(WIV)                                                                    \
  GP_TILE_TS(0, -1, false, WIV), GP_TILE_TS(1, -1, false, WIV), GP_TILE_TS(2, -1, false, WIV), \
      GP_TILE_TS(0, MODE_IMAG, false, WIV), GP_TILE_TS(0, MODE_REAL, false, WIV),           \
      GP_TILE_TS(0, -1, true, WIV), GP_TILE_TS(1, -1, true, WIV)
  const void* kt[] = {GP_TILE_ALL(false), GP_TILE_K(0, -1, kTileS, false, true),
                      GP_TILE_K(1, -1, kTileS, false, true), GP_TILE_K(2, -1, kTileS, false, true),
                      GP_TILE_K(0, MODE_IMAG, kTileS, false, true),
                      GP_TILE_K(0, MODE_REAL, kTileS, false, true),
                      GP_TILE_K(0, -1, kTileS, true, true), GP_TILE_K(1, -1, kTileS, true, true)};
#undef GP_TILE_ALL
#undef GP_TILE_TS
#undef GP_TILE_K
  for (const void* k : kt) {
    const hipError_t e =
        hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, kTileLds);
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
  const int pairs = (n1 + 1) / 2;  // an odd n1: the last pair has one line
  int np = gen_max_line<T>() / gen_stride(n0);   // pairs whose packed lines fit in LDS
  if (np > 8) np = 8;                // 16 consecutive y lines: 128-byte spectrum runs (FP64)
  if (np > pairs) np = pairs;
  if (np < 1) np = 1;
  // keep at least 512 blocks where the grid allows it
  while (np > 1 && (long long)n2 * ((pairs + np - 1) / np) < 512) np /= 2;
  xt.np = np;
  xt.nbj = (pairs + np - 1) / np;
  xt.fn0 = fdiv_make((uint32_t)n0);
  xt.fnp = fdiv_make((uint32_t)np);
  xt.f2np = fdiv_make((uint32_t)(2 * np));
  xt.fnbj = fdiv_make((uint32_t)xt.nbj);
  return xt;
}

template <>
int GLaunch<T>::x_blocks(int n0, int n1, int n2) {
  const GXTile xt = xtile(n0, n1, n2);
  return xt.nbj * n2;
}

template <>
int GLaunch<T>::cn_tile_lines(int n, int nlines, bool strided) {
  // wpl waves per line; strided tiles: 64-byte runs (8 FP32 or 4 FP64 lines, kept),
  // contiguous lines: 8 lines, at most 52 KiB of LDS (two blocks per CU at the kernels'
  // register use); at most tile_max_waves waves per block; halved while the sweep would
  // have fewer than 512 blocks; the tile and the factor table fit the LDS
  const int wpl = cn_tile_wpl(n);
  const int per_line = cn_line_slots(n, 64 * wpl) * (int)sizeof(cpx<T>);
  int nl = strided ? 64 / (int)sizeof(cpx<T>) : 53248 / per_line;
  if (!strided && nl > 8) nl = 8;
  const int cap = kTileLds / per_line - 1;
  if (nl > cap) nl = cap;
  if (nl > tile_max_waves<T>() / wpl) nl = tile_max_waves<T>() / wpl;
  if (nl < 1) nl = 1;
  while (nl > (strided ? 4 : 1) && (nlines + nl - 1) / nl < 512) nl /= 2;
  if (nl * wpl > tile_max_waves<T>()) nl = 1;
  return nl;
}

namespace {
constexpr int kTransTile = 32;  // transpose tiles of 32 x 32 values, 256 threads

// SEG: segments of long lines (factor rows from global memory).  Contiguous FP64 lines
// of one wave with more than 8 rows per lane run the wave-independent variant (WI: no
// factor line in LDS either; it frees registers of the 16-row bodies: 600^3 FP64 step
// 16.1 -> 14.4 ms, while FP32 and the 8-row bodies ran 2-5 % slower with it).
template <int MODE, int NLM, bool SEG = false>
hipError_t launch_tile(hipStream_t st, cpx<T>* data, const GLines& g, int wpl,
                       const cpx<T>* f, double* part, const GNl& nlz, const GSeg& sg = GSeg{}) {
  const int blocks = (g.nlines + g.nl - 1) / g.nl;
  const int S = (g.n + 64 * wpl - 1) / (64 * wpl);
  const bool wi =
      sizeof(T) == 8 && S > 8 && wpl == 1 && g.G == 1 && g.se == 1 && g.so == g.n;
  const size_t lds = lds_of((SEG || wi ? g.nl : g.nl + 1) * cn_line_slots(g.n, 64 * wpl));
  if (lds > (size_t)kTileLds || g.nl * wpl > tile_max_waves<T>() || S > kTileS)
    return hipErrorInvalidValue;
  const FDiv fs = fdiv_make((uint32_t)S);
  const dim3 threads(64 * wpl * g.nl);
  // at most 8 rows per lane: fewer registers
#define GP_TILE(TSV, WIV)                                                                   \
  hipLaunchKernelGGL((kg_cn_tile<T, MODE, NLM, TSV, SEG, WIV>), dim3(blocks), threads, lds, st, \
                     data, g, wpl, fs, f, part, nlz, sg)
  if (S <= 8)
    GP_TILE(8, false);
  else if (wi)
    GP_TILE(kTileS, true);
  else
    GP_TILE(kTileS, false);
#undef GP_TILE
  return hipGetLastError();
}

GLines tile_lines(int n, int nlines, int nl, int G, long long so, long long si, long long se) {
  GLines g{};
  g.n = n;
  g.nlines = nlines;
  g.nl = nl;
  g.G = G;
  g.so = so;
  g.si = si;
  g.se = se;
  g.fn = fdiv_make((uint32_t)n);
  g.fnl = fdiv_make((uint32_t)nl);
  g.fg = fdiv_make((uint32_t)G);
  return g;
}
}  // namespace

template <>
hipError_t GLaunch<T>::transpose(hipStream_t st, const cpx<T>* in, cpx<T>* out, int rows,
                                 int cols) {
  if (rows < 1 || cols < 1) return hipErrorInvalidValue;
  const dim3 grid((cols + kTransTile - 1) / kTransTile, (rows + kTransTile - 1) / kTransTile);
  hipLaunchKernelGGL((kg_transpose<T, kTransTile>), grid, dim3(kThreads), 0, st, in, out,
                     rows, cols);
  return hipGetLastError();
}

template <>
hipError_t GLaunch<T>::cn_x_nonlinear(int mode, hipStream_t st, cpx<T>* psi, int n0, int lines,
                                      const cpx<T>* f, const GNl& nlz) {
  if (n0 > gen_max_line<T>() || lines < 1) return hipErrorInvalidValue;
  const GLines g = tile_lines(n0, lines, cn_tile_lines(n0, lines, false), 1, n0, 0, 1);
  const int wpl = cn_tile_wpl(n0);
  if (mode == MODE_IMAG) return launch_tile<0, MODE_IMAG>(st, psi, g, wpl, f, nullptr, nlz);
  if (mode == MODE_REAL) return launch_tile<0, MODE_REAL>(st, psi, g, wpl, f, nullptr, nlz);
  return hipErrorInvalidValue;
}

template <>
hipError_t GLaunch<T>::r2c_x(hipStream_t st, const cpx<T>* psi, cpx<T>* spec, const GPlan& p,
                             const cpx<T>* tw, double* part, int n0, int n1, int n2) {
  const GXTile xt = xtile(n0, n1, n2);
  if (xt.np * p.m > gen_max_line<T>()) return hipErrorInvalidValue;
  // the lines and the twiddle table; the block's reduction reuses the line buffer (at
  // least 32 doubles)
  const int ls = p.m;
  const size_t lds_r2c = lds_of(xt.np * ls + ls) < 256 ? 256 : lds_of(xt.np * ls + ls);
  if (p.blue)  // Bluestein: stages of M, radices 2..8
    hipLaunchKernelGGL((kg_r2c_x<T, kEmax, true, true>), dim3(xt.nbj * n2),
                       threads_for(xt.np * ls), lds_r2c, st, psi, spec, xt, p, tw, part);
  else if (gen_plan_small(p))
    hipLaunchKernelGGL((kg_r2c_x<T, kEmax, true>), dim3(xt.nbj * n2), threads_for(xt.np * ls),
                       lds_r2c, st, psi, spec, xt, p, tw, part);
  else
    hipLaunchKernelGGL((kg_r2c_x<T, kEmax, false>), dim3(xt.nbj * n2), threads_for(xt.np * ls),
                       lds_r2c, st, psi, spec, xt, p, tw, part);
  return hipGetLastError();
}

template <>
hipError_t GLaunch<T>::c2r_x(hipStream_t st, const cpx<T>* spec, T* phi, const GPlan& p,
                             const cpx<T>* tw, int n0, int n1, int n2) {
  const GXTile xt = xtile(n0, n1, n2);
  if (xt.np * p.m > gen_max_line<T>()) return hipErrorInvalidValue;
  if (p.blue)
    hipLaunchKernelGGL((kg_c2r_x<T, kEmax, true, true>), dim3(xt.nbj * n2),
                       threads_for(xt.np * p.m), lds_of(xt.np * p.m + p.m), st, spec, phi, xt, p,
                       tw);
  else if (gen_plan_small(p))
    hipLaunchKernelGGL((kg_c2r_x<T, kEmax, true>), dim3(xt.nbj * n2), threads_for(xt.np * p.m),
                       lds_of(xt.np * p.m + p.m), st, spec, phi, xt, p, tw);
  else
    hipLaunchKernelGGL((kg_c2r_x<T, kEmax, false>), dim3(xt.nbj * n2), threads_for(xt.np * p.m),
                       lds_of(xt.np * p.m + p.m), st, spec, phi, xt, p, tw);
  return hipGetLastError();
}

template <>
hipError_t GLaunch<T>::lines(int kind, hipStream_t st, cpx<T>* data, int n, int nlines, int G,
                             long long so, long long si, long long se, const GPlan& p,
                             const cpx<T>* tw, const T* ktab, GKtab km, const double* scale,
                             const cpx<T>* w4, int w4hi) {
  if (p.m > gen_max_line<T>() || nlines < 1) return hipErrorInvalidValue;
  GLines g{};
  g.n = n;
  g.nlines = nlines;
  g.nl = lines_per_block(p.m, nlines, se != 1);
  // the stages hold at most kEmax values per thread of a 1024-thread block
  if (g.nl * p.m > gen_max_line<T>() || p.n != n) return hipErrorInvalidValue;
  g.G = G;
  g.so = so;
  g.si = si;
  g.se = se;
  g.fn = fdiv_make((uint32_t)n);
  g.fnl = fdiv_make((uint32_t)g.nl);
  g.fg = fdiv_make((uint32_t)G);
  const int blocks = (nlines + g.nl - 1) / g.nl;
  const size_t lds = lds_of(g.nl * p.m + p.m);  // the lines and the twiddle table
  const bool small = gen_plan_small(p);
  if (p.blue) {
    switch (kind) {
#define GLINESB(K)                                                                           \
  case K:                                                                                    \
    hipLaunchKernelGGL((kg_lines<T, K, kEmax, true, true>), dim3(blocks),                    \
                       threads_for(g.nl * p.m), lds, st, data, g, p, tw, ktab, km, scale,    \
                       w4, w4hi);                                                            \
    break;
      GLINESB(GL_FWD) GLINESB(GL_INV) GLINESB(GL_CONV)
#undef GLINESB
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  switch (kind * 2 + (small ? 1 : 0)) {
#define GLINES(K, S)                                                                      \
  case K * 2 + (S ? 1 : 0):                                                               \
    hipLaunchKernelGGL((kg_lines<T, K, kEmax, S>), dim3(blocks), threads_for(g.nl * p.m), lds, st, \
                       data, g, p, tw, ktab, km, scale, w4, w4hi);                        \
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
  if (cn_by_columns(n, se != 1, nlines)) {
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
  const GLines g = tile_lines(n, nlines, cn_tile_lines(n, nlines, se != 1), G, so, si, se);
  const int wpl = cn_tile_wpl(n);
  const GNl none{};
  switch (mode) {
    case 0: return launch_tile<0, -1>(st, data, g, wpl, f, part, none);
    case 1: return launch_tile<1, -1>(st, data, g, wpl, f, part, none);
    case 2: return launch_tile<2, -1>(st, data, g, wpl, f, part, none);
    default: return hipErrorInvalidValue;
  }
}

template <>
GLX GLaunch<T>::lx_geom(int n0, int n1, const GLong& lp, const GPlan& pa, const GPlan& pb) {
  GLX x{};
  x.N = n0;
  x.A = lp.A;
  x.B = lp.B;
  x.Bh = lp.B / 2 + 1;
  x.rs = x.Bh * lp.A;
  x.n1 = n1;
  x.np = (n1 + 1) / 2;
  const int lim = gen_max_line<T>();
  // column tiles of about 4096 values (ta consecutive columns: runs of ta values)
  int ta = 4096 / pb.m;
  if (ta > lim / pb.m) ta = lim / pb.m;
  if (ta > lp.A) ta = lp.A;
  if (ta < 1) ta = 1;
  x.ta = ta;
  x.nat = (lp.A + ta - 1) / ta;
  // row items of about 4096 values
  int ipf = 4096 / (2 * pa.m);
  if (ipf > lim / (2 * pa.m)) ipf = lim / (2 * pa.m);
  x.ipf = ipf < 1 ? 1 : ipf;
  int ipi = 4096 / pa.m;
  if (ipi > lim / pa.m) ipi = lim / pa.m;
  x.ipi = ipi < 1 ? 1 : ipi;
  x.fA = fdiv_make((uint32_t)lp.A);
  x.fB = fdiv_make((uint32_t)lp.B);
  x.fBh = fdiv_make((uint32_t)x.Bh);
  x.fta = fdiv_make((uint32_t)ta);
  x.fnat = fdiv_make((uint32_t)x.nat);
  return x;
}

namespace {
// one launch of a long-x kernel in the variant its plan needs (Bluestein, radices up to 8,
// or all radices)
#define GLX_LAUNCH(KERNEL, plan, grid, values, lds, ...)                                     \
  do {                                                                                        \
    if ((plan).blue)                                                                          \
      hipLaunchKernelGGL((KERNEL<T, kEmax, true, true>), dim3(grid), threads_for(values), lds, \
                         st, __VA_ARGS__);                                                    \
    else if (gen_plan_small(plan))                                                            \
      hipLaunchKernelGGL((KERNEL<T, kEmax, true, false>), dim3(grid), threads_for(values),    \
                         lds, st, __VA_ARGS__);                                               \
    else                                                                                      \
      hipLaunchKernelGGL((KERNEL<T, kEmax, false, false>), dim3(grid), threads_for(values),   \
                         lds, st, __VA_ARGS__);                                               \
  } while (0)
}  // namespace

template <>
hipError_t GLaunch<T>::lx_r2c(hipStream_t st, const cpx<T>* psi, cpx<T>* w, cpx<T>* spec,
                              const GLX& x, const GPlan& pa, const GPlan& pb,
                              const cpx<T>* twa, const cpx<T>* twb, const cpx<T>* w4,
                              double* part) {
  const int lim = gen_max_line<T>();
  if (x.ta * pb.m > lim || 2 * x.ipf * pa.m > lim || pa.n != x.A || pb.n != x.B)
    return hipErrorInvalidValue;
  // the reduction reuses the line buffer (at least 32 doubles)
  const size_t lds1 = std::max<size_t>(256, lds_of(x.ta * pb.m + pb.m));
  GLX_LAUNCH(kg_lx_cols_fwd, pb, x.np * x.nat, x.ta * pb.m, lds1, psi, w, x, pb, twb, w4,
             part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int items = x.np * x.Bh;
  GLX_LAUNCH(kg_lx_rows_fwd, pa, (items + x.ipf - 1) / x.ipf, 2 * x.ipf * pa.m,
             lds_of(2 * x.ipf * pa.m + pa.m), w, spec, x, pa, twa);
  return hipGetLastError();
}

template <>
hipError_t GLaunch<T>::lx_c2r(hipStream_t st, const cpx<T>* spec, cpx<T>* w, T* phi,
                              const GLX& x, const GPlan& pa, const GPlan& pb,
                              const cpx<T>* twa, const cpx<T>* twb, const cpx<T>* w4) {
  const int lim = gen_max_line<T>();
  if (x.ta * pb.m > lim || x.ipi * pa.m > lim || pa.n != x.A || pb.n != x.B)
    return hipErrorInvalidValue;
  const int items = x.np * x.B;
  GLX_LAUNCH(kg_lx_rows_inv, pa, (items + x.ipi - 1) / x.ipi, x.ipi * pa.m,
             lds_of(x.ipi * pa.m + pa.m), spec, w, x, pa, twa, w4);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  GLX_LAUNCH(kg_lx_cols_inv, pb, x.np * x.nat, x.ta * pb.m, lds_of(x.ta * pb.m + pb.m), w,
             phi, x, pb, twb);
  return hipGetLastError();
}
#undef GLX_LAUNCH

template <>
int GLaunch<T>::seg_lines(int sn, int nlines, bool cols) {
  // the tile sweep's lines per block (segments keep no factor line in LDS); strided
  // segments take the strided tiles of adjacent lines
  return cn_tile_lines(sn, nlines, cols);
}

template <>
hipError_t GLaunch<T>::seg_sweep(int mode, hipStream_t st, cpx<T>* data, int sn, int nseg,
                                 int nlong, const cpx<T>* f, const cpx<T>* pq, cpx<T>* sum,
                                 cpx<T>* car, double* part, long long ld) {
  if (sn > gen_max_line<T>() || nseg < 2 || nlong < 1 || (mode != 0 && mode != 1) ||
      (ld != 0 && ld < nlong))
    return hipErrorInvalidValue;
  const bool cols = ld != 0;
  const int nlines = nlong * nseg;
  // contiguous: line l = L nseg + s at l sn; strided: l = s nlong + L at s sn ld + L
  const GLines g = cols ? tile_lines(sn, nlines, seg_lines(sn, nlines, true), nlong, sn * ld,
                                     1, ld)
                        : tile_lines(sn, nlines, seg_lines(sn, nlines), 1, sn, 0, 1);
  const int wpl = cn_tile_wpl(sn);
  const GNl none{};
  const GSeg sg{nseg, fdiv_make((uint32_t)(cols ? nlong : nseg)), car, cols ? 1 : 0};
  const cpx<T>* wu = pq + 2 * nseg;
  if (cols) {
    hipLaunchKernelGGL(k_seg_summary_cols<T>, dim3((nlines + kThreads - 1) / kThreads),
                       dim3(kThreads), 0, st, data, sum, wu, sn, nseg, nlong, ld);
  } else {
    constexpr int kWavesPerBlock = kThreads / 64;
    hipLaunchKernelGGL(k_seg_summary<T>, dim3((nlines + kWavesPerBlock - 1) / kWavesPerBlock),
                       dim3(kThreads), 0, st, data, sum, wu, sn, nseg, sg.fseg, nlines);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_seg_carry<T>, dim3((nlong + kThreads - 1) / kThreads), dim3(kThreads), 0,
                     st, sum, car, pq, nseg, nlong, cols ? 1 : 0);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (mode == 0) return launch_tile<0, -1, true>(st, data, g, wpl, f, nullptr, none, sg);
  return launch_tile<1, -1, true>(st, data, g, wpl, f, part, none, sg);
}

}  // namespace gpdbec
