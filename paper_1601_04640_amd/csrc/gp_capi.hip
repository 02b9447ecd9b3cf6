// C ABI of libgpdbec (see include/gp.h): context set-up, workspace carving, state I/O
// and the per-step pass schedule on the caller's HIP stream.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "../../include/gp.h"
#include "gp_aux.hpp"
#include "gp_batch_launch.hpp"
#include "gp_generic_launch.hpp"
#include "gp_kernels.hpp"
#include "gp_launch.hpp"

using namespace gpdbec;

namespace {

constexpr int kRingCap = 4096;
constexpr long long kStageThreshold = 16384;  // partial values above which the finalize
constexpr long long kStageSlice = 512;        // runs in two stages, ~kStageSlice per slice
constexpr int kGraphSteps = 8;  // steps per captured graph
constexpr size_t kIoChunk = (size_t)1 << 22;  // points per host-transfer chunk (64 MiB FP64)

// Axis lengths with compile-time specialised passes.
bool fast_size(int n) {
  switch (n) {
#define X(N) case N:
    GP_FOR_SIZES(X)
#undef X
    return true;
    default:
      return false;
  }
}

// Every axis length a context accepts: a specialised one, one the run-time-length passes
// take (n >= 4, its FFT line within 64 KiB of LDS), or, in a 2D grid (plane), a longer one
// with a four-step split and Crank-Nicolson segments.
bool long_size(int n, bool fp64) {
  GLong lp;
  return fp64 ? gen_long_plan<double>(n, &lp) : gen_long_plan<float>(n, &lp);
}
bool size_ok(int n, bool fp64, bool plane = false) {
  return fast_size(n) || (fp64 ? gen_size_ok<double>(n) : gen_size_ok<float>(n)) ||
         (plane && long_size(n, fp64));
}

// The axes a geometry uses: (n0, n1, n2) with n2 = 1 in 2D.
void plane_axes(const gp_params* p, int* n0, int* n1, int* n2) {
  *n0 = p->nx;
  *n1 = p->geom == GP_2D_XZ ? p->nz : p->ny;
  *n2 = p->geom == GP_3D ? p->nz : 1;
}

bool is_generic(const gp_params* p) {
  int n0, n1, n2;
  plane_axes(p, &n0, &n1, &n2);
  return !fast_size(n0) || !fast_size(n1) || (p->geom == GP_3D && !fast_size(n2));
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

struct Layout {
  int n0, n1, n2;       // grid axes, x fastest
  double h0, h1, h2;
  size_t npts, nspec, nktab;  // grid points, half-spectrum values, kernel-table values
  size_t esz;           // bytes of one real value
  int nb_x, nb_nl, nb_col, nb_colobs;
  int nb_r2c;           // tiles of the single-grid R2C pass (nb_x unless its tiles are wider)
  // axes without a compile-time specialisation run the run-time-length passes; gscr: their
  // one-thread-per-line sweeps need a grid of scratch values (o_gscr)
  bool generic, gscr;
  // 2D axes longer than one LDS line (x, y): four-step FFT and segmented sweeps; the
  // intermediate grid of the x transforms uses o_gscr.  sy: the 2D y sweep runs in
  // segments over the strided columns (a long y axis, or one-line y axes past a tile
  // with a segment length dividing them; others run on a transposed copy in o_gscr)
  bool lx, ly, sy;
  GLong lg[2];
  GLX lxg;  // the long-x passes' geometry (host side; the plans' strides from lg)
  // byte offsets inside the workspace
  size_t o_psi, o_V, o_spec, o_ktab, o_tw[3], o_blue[3], o_cn[3][3], o_px[2], o_pnl, o_pcol, o_padj, o_sfield,
      o_scalars, o_ring, o_obs, o_io, o_stamps, o_stage, o_gscr, total;
  // long axes: stage twiddles of the A- and B-point plans and W_N^m, their Bluestein
  // tables, the segments' carry products per factor set, segment summaries and carries
  size_t o_ltw[2][3], o_lblue[2][2], o_seg[2][3], o_ssum, o_scar;
};

struct Scalars {  // device-side scalars (one 256-byte block)
  double scale;
  double one;        // constant 1 (scale of an externally supplied psi)
  double ekz;
  double obs_pad;
  int flags;
  int ring_pos;
  unsigned long long span[2];  // c2r kernel-span timing: ticks, launches
};

gp_status validate(const gp_params* p) {
  if (!p) return GP_E_ARG;
  if (p->geom < GP_3D || p->geom > GP_2D_XZ) return GP_E_ARG;
  if (p->prec != GP_FP64 && p->prec != GP_FP32_MIXED) return GP_E_ARG;
  if (!(p->dt > 0) || !isfinite(p->dt)) return GP_E_ARG;
  if (!(p->dx > 0) || !isfinite(p->dx)) return GP_E_ARG;
  if (!isfinite(p->g) || !isfinite(p->gdd) || !isfinite(p->gamma) || !isfinite(p->nu) ||
      !isfinite(p->lambda) || !isfinite(p->cutoff_R))
    return GP_E_ARG;
  const bool fp64 = p->prec == GP_FP64;
  if (!size_ok(p->nx, fp64, p->geom != GP_3D)) return GP_E_SIZE;
  if (p->geom == GP_3D) {
    if (!(p->dy > 0) || !(p->dz > 0)) return GP_E_ARG;
    if (!size_ok(p->ny, fp64) || !size_ok(p->nz, fp64)) return GP_E_SIZE;
  } else if (p->geom == GP_2D_XY) {
    if (!(p->dy > 0) || !(p->lambda > 0)) return GP_E_ARG;
    if (!size_ok(p->nx, fp64, true) || !size_ok(p->ny, fp64, true)) return GP_E_SIZE;
  } else {
    if (!(p->dz > 0) || !(p->nu > 0)) return GP_E_ARG;
    if (!size_ok(p->nx, fp64, true) || !size_ok(p->nz, fp64, true)) return GP_E_SIZE;
  }
  // the run-time-length passes address the grid with 32-bit line offsets
  int n0, n1, n2;
  plane_axes(p, &n0, &n1, &n2);
  if (is_generic(p) && (double)n0 * n1 * n2 > 2147483647.0) return GP_E_SIZE;
  return GP_OK;
}

int tj_of(bool fp64, int n) { return fp64 ? Launch<double>::tj(n) : Launch<float>::tj(n); }
int tjw_of(bool fp64, int n) { return fp64 ? Launch<double>::tjw(n) : Launch<float>::tjw(n); }
int tc_of(bool fp64, int n) { return fp64 ? Launch<double>::tc(n) : Launch<float>::tc(n); }
int tv_of(bool fp64, int n) { return fp64 ? Launch<double>::tv(n) : Launch<float>::tv(n); }

Layout make_layout(const gp_params* p, unsigned host = 0) {
  Layout L{};
  const bool fp64 = p->prec == GP_FP64;
  L.n0 = p->nx;
  L.h0 = p->dx;
  if (p->geom == GP_3D) {
    L.n1 = p->ny; L.h1 = p->dy; L.n2 = p->nz; L.h2 = p->dz;
  } else if (p->geom == GP_2D_XY) {
    L.n1 = p->ny; L.h1 = p->dy; L.n2 = 1; L.h2 = 1.0;
  } else {
    L.n1 = p->nz; L.h1 = p->dz; L.n2 = 1; L.h2 = 1.0;
  }
  L.esz = fp64 ? 8 : 4;
  L.npts = (size_t)L.n0 * L.n1 * L.n2;
  const int H = L.n0 / 2 + 1;
  L.nspec = (size_t)H * L.n1 * L.n2;
  L.generic = is_generic(p);
  const int ns0[2] = {L.n0, L.n1};
  bool lng[2] = {false, false};
  for (int a = 0; a < 2 && p->geom != GP_3D; ++a)
    lng[a] = fp64 ? gen_long_plan<double>(ns0[a], &L.lg[a])
                  : gen_long_plan<float>(ns0[a], &L.lg[a]);
  L.lx = lng[0];
  L.ly = lng[1];
  // one-line y axes past a tile: segmented when there are enough column segments to fill
  // the GPU (the summary walks each with one thread; fewer ran slower than the transposed
  // sweep: 1500^2 FP32 0.12 -> 0.22 ms, while 8192^2 went 3.07 -> 2.75 ms)
  if (!L.ly && p->geom != GP_3D && L.generic && L.n1 > kTileMaxN) {
    GLong sg{};
    if (gen_seg_split(L.n1, &sg.sn, &sg.nseg) &&
        (long long)L.n0 * sg.nseg >= (fp64 ? 16384 : 40960)) {
      L.lg[1] = sg;
      L.sy = true;
    }
  }
  L.sy = L.sy || L.ly;
  GPlan lpa[2], lpb[2];
  const int lim = fp64 ? gen_max_line<double>() : gen_max_line<float>();
  for (int a = 0; a < 2; ++a)
    if (lng[a]) {
      gen_long_subplan(L.lg[a].A, lim / 2, &lpa[a]);
      gen_long_subplan(L.lg[a].B, lim, &lpb[a]);
    }
  if (L.lx) {
    L.lxg = fp64 ? GLaunch<double>::lx_geom(L.n0, L.n1, L.lg[0], lpa[0], lpb[0])
                 : GLaunch<float>::lx_geom(L.n0, L.n1, L.lg[0], lpa[0], lpb[0]);
    L.nspec = (size_t)L.n1 * L.lxg.rs;   // rows of kept four-step slots
  }
  if (L.generic) {
    L.nb_x = fp64 ? GLaunch<double>::x_blocks(L.n0, L.n1, L.n2)
                  : GLaunch<float>::x_blocks(L.n0, L.n1, L.n2);
    if (L.lx) L.nb_x = GLaunch<float>::lx_blocks(L.lxg);
    L.nb_r2c = L.nb_x;
    L.nb_nl = fp64 ? GLaunch<double>::nl_blocks(L.n0, L.n1, L.n2)
                   : GLaunch<float>::nl_blocks(L.n0, L.n1, L.n2);
    // blocks of the last sweep (z in 3D, y in 2D), which the z observe shares
    L.nb_col = p->geom == GP_3D
                   ? (fp64 ? GLaunch<double>::cn_blocks(L.n2, L.n0 * L.n1, true)
                           : GLaunch<float>::cn_blocks(L.n2, L.n0 * L.n1, true))
                   : (fp64 ? GLaunch<double>::cn_blocks(
                                     L.n1, L.n0, !GLaunch<double>::y2d_transposed(L.n1))
                           : GLaunch<float>::cn_blocks(
                                     L.n1, L.n0, !GLaunch<float>::y2d_transposed(L.n1)));
    // a scratch grid for the one-thread-per-line sweeps (3D grids whose y or z sweep has
    // many lines longer than a tile) and for the transposed 2D y sweep of long lines
    L.gscr = p->geom == GP_3D
                 ? (GLaunch<float>::cn_by_columns(L.n1, true, L.n0 * L.n2) ||
                    GLaunch<float>::cn_by_columns(L.n2, true, L.n0 * L.n1))
                 : ((GLaunch<float>::y2d_transposed(L.n1) && !L.sy) || L.lx);
    // a segmented y sweep (the last in 2D) runs over the strided columns
    if (L.sy)
      L.nb_col = fp64 ? GLaunch<double>::seg_blocks(L.lg[1].sn, L.n0 * L.lg[1].nseg, true)
                      : GLaunch<float>::seg_blocks(L.lg[1].sn, L.n0 * L.lg[1].nseg, true);
  } else {
    const int tj = tj_of(fp64, L.n0), tjw = tjw_of(fp64, L.n0);
    L.nb_x = ((L.n1 + tj - 1) / tj) * L.n2;
    L.nb_nl = L.nb_x;   // the x pass writes both
    L.nb_r2c = ((L.n1 + tjw - 1) / tjw) * L.n2;
    if (p->geom == GP_3D) {
      const int tcz = tc_of(fp64, L.n2);
      L.nb_col = ((L.n0 + tcz - 1) / tcz) * L.n1;   // z sweep / z observe
    } else {
      const int tcy = tc_of(fp64, L.n1);
      L.nb_col = ((L.n0 + tcy - 1) / tcy) * L.n2;   // y sweep (last pass in 2D)
    }
  }
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o += align_up(bytes);
    return r;
  };
  L.o_psi = take(2 * L.esz * L.npts);
  L.o_V = take((host & GP_HOST_V) ? 0 : L.esz * L.npts);
  L.o_spec = take(2 * L.esz * L.nspec);
  // kernel table: 3D holds the quadrant k1 <= n1/2, k2 <= n2/2 of the half spectrum; 2D
  // every k1 of kx <= n0/2, in the spectrum's slot order when an axis is split
  L.nktab = (p->geom == GP_3D) ? (size_t)H * (L.n1 / 2 + 1) * (L.n2 / 2 + 1) : L.nspec;
  L.o_ktab = take((host & GP_HOST_KTAB) ? 0 : L.esz * L.nktab);
  const int ns[3] = {L.n0, L.n1, L.n2};
  for (int a = 0; a < 3; ++a) {
    // twiddles of the stage length (Bluestein's M for a run-time-length axis with a prime
    // factor above 31), then that axis's chirp (n) and filter (M)
    const bool la = a < 2 && lng[a];
    const int ms = la ? 0 : (L.generic ? gen_stride(ns[a]) : ns[a]);
    L.o_tw[a] = take(2 * L.esz * ms);
    L.o_blue[a] = take(!la && ms != ns[a] ? 2 * L.esz * (size_t)(ns[a] + ms) : 0);
    // factor table and scan weights per set (imaginary time, real time, adjoint)
    for (int t = 0; t < 3; ++t) L.o_cn[a][t] = take(2 * L.esz * (ns[a] + kScanWeights));
  }
  // Partial-sum slots: one per tile, for the largest tile count any shape variant of the
  // batched passes can use (x and column tiles of 8 lines).
  int cap_x = L.nb_x, cap_nl = L.nb_nl, cap_col = L.nb_col;
  if (!L.generic) {
    cap_x = std::max(cap_x, ((L.n1 + 7) / 8) * L.n2);
    cap_nl = std::max(cap_nl, cap_x);
    cap_col = std::max(cap_col, ((L.n0 + 7) / 8) * (p->geom == GP_3D ? L.n1 : L.n2));
  }
  // two x-partial buffers: a real-time step's x pass writes one while the previous
  // step's folded finalisation reads the other
  for (int k = 0; k < 2; ++k) L.o_px[k] = take(sizeof(double) * 2 * cap_x);
  L.o_pnl = take(sizeof(double) * 7 * cap_nl);
  L.o_pcol = take(sizeof(double) * 2 * cap_col);
  L.o_padj = take(sizeof(double) * 2 * L.nb_x);
  L.o_sfield = take(L.esz * L.npts);
  L.o_scalars = take(sizeof(Scalars));
  L.o_ring = take(sizeof(double) * kRecord * kRingCap);
  L.o_obs = take(sizeof(double) * kRecord);
  L.o_io = take(16 * std::min(L.npts, kIoChunk));
  L.o_stamps = take(16 * (size_t)L.nb_x);
  L.o_stage = take(sizeof(double) * kStageVals * kStageMax);
  L.o_gscr = take(L.generic && L.gscr ? 2 * L.esz * L.npts : 0);
  size_t nsegl = 0;  // segment lines of the longer segmented sweep
  for (int a = 0; a < 2; ++a) {
    const GPlan* pl[2] = {&lpa[a], &lpb[a]};
    for (int q = 0; q < 2; ++q) {
      L.o_ltw[a][q] = take(lng[a] ? 2 * L.esz * pl[q]->m : 0);
      L.o_lblue[a][q] =
          take(lng[a] && pl[q]->blue ? 2 * L.esz * (size_t)(pl[q]->n + pl[q]->m) : 0);
    }
    L.o_ltw[a][2] = take(lng[a] ? 2 * L.esz * ns0[a] : 0);
    // per factor set: P, Q of each segment, then the summary weights w, u of each row
    const bool seg = a == 0 ? L.lx : L.sy;  // this axis's sweep runs in segments
    for (int t = 0; t < 3; ++t)
      L.o_seg[a][t] = take(seg ? 4 * L.esz * ((size_t)L.lg[a].nseg + ns0[a]) : 0);
    if (seg) nsegl = std::max(nsegl, (size_t)ns0[1 - a] * L.lg[a].nseg);
  }
  L.o_ssum = take(8 * L.esz * nsegl);
  L.o_scar = take(8 * L.esz * nsegl);
  L.total = o;
  return L;
}

}  // namespace

struct gp_ctx {
  // Step loops replay captured HIP graphs of 8, 4, 2 and 1 steps (a run of n steps is
  // the binary decomposition of n, eights first), captured once per
  // [time direction imaginary/real][start state: nothing outstanding, or a finalisation of
  // that direction outstanding in x-partial buffer 0 / 1][length]; each records the state
  // its steps leave behind.
  bool use_graphs = true;
  hipStream_t cap_st = nullptr;
  struct GraphRec {
    hipGraphExec_t ex = nullptr;
    bool end_pending = false;
    int end_sel = 0;
  };
  GraphRec gexec[2][3][4];
  // Steps defer their finalisation into the next step's first pass: fin_pending marks
  // one outstanding (mode pend_mode, its x partials in buffer pend_sel); px_sel is the
  // buffer the x pass writes next.
  bool fin_pending = false;
  int pend_sel = 0;
  int pend_mode = FIN_REAL;
  int px_sel = 0;
  // optional per-pass timing: event pairs recorded around selected pass launches
  unsigned tmask = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> tev[GP_PASS_COUNT];
  std::vector<hipEvent_t> tpool;
  gp_params p;
  Layout L;
  hipStream_t st;
  char* ws;
  bool fp64;
  bool psi_set;
  bool ekz_valid;
  double gc;
  int clock_khz = 0;  // device wall clock (kernel-span timing)
  GPlan gplan[3] = {};  // radix plans of the run-time-length passes (axes 0, 1, 2)
  GPlan lplan[2][2] = {};  // long 2D axes: plans of the A- and B-point transforms
  // device addresses of caller-owned pinned host memory holding V / the kernel table
  // (gp_init_ex with GP_HOST_V / GP_HOST_KTAB), else null
  char* hostV = nullptr;
  char* hostK = nullptr;
  template <typename X>
  X* at(size_t off) const { return reinterpret_cast<X*>(ws + off); }
  Scalars* sc() const { return at<Scalars>(L.o_scalars); }
};

namespace {

thread_local char g_last_error[256] = "";

gp_status dev(hipError_t e) {
  if (e == hipSuccess) return GP_OK;
  snprintf(g_last_error, sizeof(g_last_error), "%s (%d)", hipGetErrorString(e), (int)e);
  return GP_E_DEVICE;
}

// Discard an error left in HIP's per-thread slot by earlier, unrelated runtime calls, so
// that a launch check reports only this library's launches.
void clear_stale_error() { (void)hipGetLastError(); }
#define GP_TRY(expr)                     \
  do {                                   \
    const gp_status _s = (expr);         \
    if (_s != GP_OK) return _s;          \
  } while (0)
#define GP_HIP(expr) GP_TRY(dev(expr))

hipEvent_t take_event(gp_ctx* c) {
  if (!c->tpool.empty()) {
    hipEvent_t e = c->tpool.back();
    c->tpool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Records the start event of a timed pass; returns false when timing is off.
gp_status pass_begin(gp_ctx* c, int pass) {
  if (!(c->tmask & (1u << pass))) return GP_OK;
  hipEvent_t a = take_event(c), b = take_event(c);
  if (!a || !b) return GP_E_DEVICE;
  c->tev[pass].emplace_back(a, b);
  return dev(hipEventRecord(a, c->st));
}

gp_status pass_end(gp_ctx* c, int pass) {
  if (!(c->tmask & (1u << pass))) return GP_OK;
  return dev(hipEventRecord(c->tev[pass].back().second, c->st));
}

#define GP_PASS(c, id, expr)        \
  do {                              \
    GP_TRY(pass_begin((c), (id)));  \
    GP_HIP(expr);                   \
    GP_TRY(pass_end((c), (id)));    \
  } while (0)

unsigned blocks_for(size_t n, int per = kThreads) { return (unsigned)((n + per - 1) / per); }

double d_perp(const gp_params& p) {
  return p.geom == GP_2D_XY ? 1.0 / sqrt(p.lambda) : 1.0 / sqrt(p.nu);
}

double contact(const gp_params& p) {
  if (p.geom == GP_3D) return p.g;
  return p.g / (sqrt(2.0 * M_PI) * d_perp(p));
}

StepScalars step_scalars(const gp_ctx* c) {
  StepScalars s{};
  s.dt = c->p.dt;
  s.gc = c->gc;
  s.gdd = c->p.gdd;
  s.h0 = c->L.h0;
  s.h1 = c->L.h1;
  s.h2 = c->L.h2;
  return s;
}

// Partials of the pass sequence whose x pass wrote buffer `sel`.
FinArgs fin_args(const gp_ctx* c, int sel) {
  FinArgs a{};
  a.p_x = c->at<double>(c->L.o_px[sel]);
  a.nb_x = c->L.nb_r2c;
  a.p_nl = c->at<double>(c->L.o_pnl);
  a.nb_nl = c->L.nb_nl;
  a.p_col = c->at<double>(c->L.o_pcol);
  a.nb_col = c->L.nb_col;
  a.dV = c->L.h0 * c->L.h1 * (c->p.geom == GP_3D ? c->L.h2 : 1.0);
  a.h0 = c->L.h0;
  a.h1 = c->L.h1;
  a.h2 = c->L.h2;
  a.gc = c->gc;
  a.gdd = c->p.gdd;
  a.geom = c->p.geom;
  Scalars* s = c->sc();
  a.scale = &s->scale;
  a.ekz = &s->ekz;
  a.flags = &s->flags;
  a.ring = c->at<double>(c->L.o_ring);
  a.ring_pos = &s->ring_pos;
  a.ring_cap = kRingCap;
  a.obs = c->at<double>(c->L.o_obs);
  // many partials: a first stage of up to kStageMax blocks sums slices of ~512 values
  const long long nvals = 2LL * c->L.nb_r2c + 7LL * c->L.nb_nl + 2LL * c->L.nb_col;
  a.stage = c->at<double>(c->L.o_stage);
  a.nstage = nvals > kStageThreshold
                 ? (int)std::min<long long>(kStageMax, (nvals + kStageSlice - 1) / kStageSlice)
                 : 0;
  return a;
}

// The outstanding real-time finalisation, if any, as its own launch(es).  Every entry
// point other than the real-time step calls this first.
gp_status settle(gp_ctx* c) {
  if (!c->fin_pending) return GP_OK;
  c->fin_pending = false;
  const FinArgs a = fin_args(c, c->pend_sel);
  if (a.nstage > 0)
    hipLaunchKernelGGL(k_prereduce, dim3(a.nstage), dim3(kThreads), 0, c->st, a, c->pend_mode);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, c->st, a, c->pend_mode);
  return dev(hipGetLastError());
}

// ------------------------------------------------------------- pass schedule
template <typename T>
struct Passes {
  static cpx<T>* psi(gp_ctx* c) { return c->at<cpx<T>>(c->L.o_psi); }
  static cpx<T>* spec(gp_ctx* c) { return c->at<cpx<T>>(c->L.o_spec); }
  // the trap potential and the kernel table: in the workspace, or in caller-owned pinned
  // host memory read through its device mapping (gp_init_ex)
  static T* Vp(gp_ctx* c) { return c->hostV ? reinterpret_cast<T*>(c->hostV) : c->at<T>(c->L.o_V); }
  static T* Kp(gp_ctx* c) {
    return c->hostK ? reinterpret_cast<T*>(c->hostK) : c->at<T>(c->L.o_ktab);
  }
  static const cpx<T>* tw(gp_ctx* c, int a) { return c->at<cpx<T>>(c->L.o_tw[a]); }
  // factor table of axis a, set k (0: imaginary time, 1: real time, 2: adjoint sweep)
  static const cpx<T>* cn(gp_ctx* c, int a, int k) { return c->at<cpx<T>>(c->L.o_cn[a][k]); }

  // ------------------------------------------- run-time-length passes (gp_generic.hpp)
  // The same step as the specialised passes, in simpler launches: the x R2C, the y FFT,
  // the z convolution and the inverse y FFT (2D: the y convolution), the x C2R into a
  // real Phi grid, the phase in place, then the x, y and z sweeps; the finalisation runs
  // after every step.
  // long 2D axes: stage twiddles of the A- (q = 0) and B-point (q = 1) plans, W_N^m (q = 2)
  static const cpx<T>* ltw(gp_ctx* c, int a, int q) { return c->at<cpx<T>>(c->L.o_ltw[a][q]); }
  static cpx<T>* gscr(gp_ctx* c) { return c->at<cpx<T>>(c->L.o_gscr); }

  // 2D convolution along y of a spectrum whose x axis or y axis is split (four-step):
  // spectrum [kx][y] (x in one line) or rows [y][rs] of four-step slots (long x)
  static gp_status g_conv_y_long(gp_ctx* c, const double* scale) {
    const Layout& L = c->L;
    const int H = L.n0 / 2 + 1;
    // the kernel table is in the spectrum's slot order
    GKtab km{0, L.n1, 1, fdiv_make((uint32_t)L.n1), 1};
    if (!L.ly) {  // long x only: columns p of the rows, the whole y line in LDS
      const int rs = L.lxg.rs;
      GP_PASS(c, GP_PASS_CONV_Y,
              GLaunch<T>::lines(GL_CONV, c->st, spec(c), L.n1, rs, rs, 0, 1, rs, c->gplan[1],
                                tw(c, 1), Kp(c), km, scale));
      return GP_OK;
    }
    // y = a + Ay b: B-point transforms over b with the twiddle of column a, the A-point
    // convolution over a (wavenumber By ka + kb), the inverse steps
    const int Ay = L.lg[1].A, By = L.lg[1].B;
    const GPlan& pa = c->lplan[1][0];
    const GPlan& pb = c->lplan[1][1];
    GP_TRY(pass_begin(c, GP_PASS_CONV_Y));
    if (!L.lx) {  // spectrum [kx][y]: lines (kx, a) of stride Ay; inner lines contiguous
      GP_HIP(GLaunch<T>::lines(GL_FWD, c->st, spec(c), By, H * Ay, Ay, L.n1, 1, Ay, pb,
                               ltw(c, 1, 1), nullptr, km, scale, ltw(c, 1, 2), 0));
      GP_HIP(GLaunch<T>::lines(GL_CONV, c->st, spec(c), Ay, H * By, 1, Ay, 0, 1, pa,
                               ltw(c, 1, 0), Kp(c), km, scale));
      GP_HIP(GLaunch<T>::lines(GL_INV, c->st, spec(c), By, H * Ay, Ay, L.n1, 1, Ay, pb,
                               ltw(c, 1, 1), nullptr, km, scale, ltw(c, 1, 2), 0));
    } else {      // rows [y][rs]: lines (a, p) and (kb, p), consecutive p adjacent
      const long long rs = L.lxg.rs;
      GP_HIP(GLaunch<T>::lines(GL_FWD, c->st, spec(c), By, (int)(Ay * rs), (int)rs, rs, 1,
                               Ay * rs, pb, ltw(c, 1, 1), nullptr, km, scale, ltw(c, 1, 2), 1));
      GP_HIP(GLaunch<T>::lines(GL_CONV, c->st, spec(c), Ay, (int)(By * rs), (int)rs, Ay * rs, 1,
                               rs, pa, ltw(c, 1, 0), Kp(c), km, scale));
      GP_HIP(GLaunch<T>::lines(GL_INV, c->st, spec(c), By, (int)(Ay * rs), (int)rs, rs, 1,
                               Ay * rs, pb, ltw(c, 1, 1), nullptr, km, scale, ltw(c, 1, 2), 1));
    }
    return pass_end(c, GP_PASS_CONV_Y);
  }

  static gp_status g_convolution(gp_ctx* c, const cpx<T>* src, const double* scale) {
    const Layout& L = c->L;
    const int H = L.n0 / 2 + 1;
    if (L.lx) {
      GP_PASS(c, GP_PASS_R2C_X,
              GLaunch<T>::lx_r2c(c->st, src, gscr(c), spec(c), L.lxg, c->lplan[0][0],
                                 c->lplan[0][1], ltw(c, 0, 0), ltw(c, 0, 1), ltw(c, 0, 2),
                                 c->at<double>(L.o_px[0])));
    } else {
      GP_PASS(c, GP_PASS_R2C_X,
              GLaunch<T>::r2c_x(c->st, src, spec(c), c->gplan[0], tw(c, 0),
                                c->at<double>(L.o_px[0]), L.n0, L.n1, L.n2));
    }
    if (L.lx || L.ly) return g_conv_y_long(c, scale);
    const GKtab none{0, L.n1, L.n2, fdiv_make((uint32_t)L.n1)};
    if (c->p.geom == GP_3D) {
      // y lines l = kx n2 + k2 (contiguous); z lines l = kx n1 + k1 (stride n1)
      GP_PASS(c, GP_PASS_FFT_Y_FWD,
              GLaunch<T>::lines(GL_FWD, c->st, spec(c), L.n1, H * L.n2, 1, L.n1, 0, 1,
                                c->gplan[1], tw(c, 1), nullptr, none, scale));
      GP_PASS(c, GP_PASS_CONV_Z,
              GLaunch<T>::lines(GL_CONV, c->st, spec(c), L.n2, H * L.n1, L.n1,
                                (long long)L.n1 * L.n2, 1, L.n1, c->gplan[2], tw(c, 2),
                                Kp(c), GKtab{1, L.n1, L.n2, fdiv_make((uint32_t)L.n1)}, scale));
      GP_PASS(c, GP_PASS_FFT_Y_INV,
              GLaunch<T>::lines(GL_INV, c->st, spec(c), L.n1, H * L.n2, 1, L.n1, 0, 1,
                                c->gplan[1], tw(c, 1), nullptr, none, scale));
    } else {
      GP_PASS(c, GP_PASS_CONV_Y,
              GLaunch<T>::lines(GL_CONV, c->st, spec(c), L.n1, H, 1, L.n1, 0, 1, c->gplan[1],
                                tw(c, 1), Kp(c), GKtab{0, L.n1, 1, fdiv_make((uint32_t)L.n1)},
                                scale));
    }
    return GP_OK;
  }

  static GStep g_scalars(gp_ctx* c) {
    return GStep{c->p.dt, c->gc, c->p.gdd, c->L.h0, c->L.h1, c->L.h2,
                 fdiv_make((uint32_t)c->L.n0), fdiv_make((uint32_t)c->L.n1)};
  }

  // the x C2R of the convolved spectrum into phi
  static gp_status g_c2r(gp_ctx* c, T* phi) {
    const Layout& L = c->L;
    if (L.lx)
      return dev(GLaunch<T>::lx_c2r(c->st, spec(c), gscr(c), phi, L.lxg, c->lplan[0][0],
                                    c->lplan[0][1], ltw(c, 0, 0), ltw(c, 0, 1), ltw(c, 0, 2)));
    return dev(GLaunch<T>::c2r_x(c->st, spec(c), phi, c->gplan[0], tw(c, 0), L.n0, L.n1, L.n2));
  }

  // Phi of src into phi (the convolution, then the x C2R)
  static gp_status g_phi(gp_ctx* c, const cpx<T>* src, const double* scale, T* phi) {
    GP_TRY(g_convolution(c, src, scale));
    return g_c2r(c, phi);
  }

  // CN sweep of axis a (0: x, 1: y, 2: z) of the stored state; mode 0: solve, 1: solve
  // with the new-state sums, 2: the sums of the stored state only
  static gp_status g_sweep(gp_ctx* c, int axis, int k, int mode) {
    const Layout& L = c->L;
    double* pc = mode == 0 ? nullptr : c->at<double>(L.o_pcol);
    const cpx<T>* f = mode == 2 ? nullptr : cn(c, axis, k);
    const long long plane = (long long)L.n0 * L.n1;
    cpx<T>* dscr = c->at<cpx<T>>(L.o_gscr);
    if (axis == 0 && L.lx)  // long x lines: segmented
      return dev(GLaunch<T>::seg_sweep(mode, c->st, psi(c), L.lg[0].sn, L.lg[0].nseg, L.n1, f,
                                       c->at<cpx<T>>(L.o_seg[0][k]), c->at<cpx<T>>(L.o_ssum),
                                       c->at<cpx<T>>(L.o_scar), pc));
    if (axis == 0)  // lines (j, k2), contiguous
      return dev(GLaunch<T>::cn_lines(mode, c->st, psi(c), L.n0, L.n1 * L.n2, 1, L.n0, 0, 1,
                                      f, pc, dscr));
    if (axis == 1 && L.sy)  // segmented, in place over the strided columns
      return dev(GLaunch<T>::seg_sweep(mode, c->st, psi(c), L.lg[1].sn, L.lg[1].nseg, L.n0, f,
                                       c->at<cpx<T>>(L.o_seg[1][k]), c->at<cpx<T>>(L.o_ssum),
                                       c->at<cpx<T>>(L.o_scar), pc, L.n0));
    if (axis == 1 && c->p.geom != GP_3D && GLaunch<T>::y2d_transposed(L.n1)) {
      // 2D lines longer than a tile: the sweep runs along the rows of the transposed state
      // (scratch grid, n0 rows of n1) and the result is transposed back
      GP_HIP(GLaunch<T>::transpose(c->st, psi(c), dscr, L.n1, L.n0));
      GP_HIP(GLaunch<T>::cn_lines(mode, c->st, dscr, L.n1, L.n0, 1, L.n1, 0, 1, f, pc, nullptr));
      return dev(GLaunch<T>::transpose(c->st, dscr, psi(c), L.n0, L.n1));
    }
    if (axis == 1)  // lines (i, k2) along y: base k2 n0 n1 + i, stride n0
      return dev(GLaunch<T>::cn_lines(mode, c->st, psi(c), L.n1, L.n0 * L.n2, L.n0, plane, 1,
                                      L.n0, f, pc, dscr));
    // lines (i, j) along z: base j n0 + i, stride n0 n1
    return dev(GLaunch<T>::cn_lines(mode, c->st, psi(c), L.n2, L.n0 * L.n1, L.n0 * L.n1, 0, 1,
                                    plane, f, pc, dscr));
  }

  static gp_status g_step(gp_ctx* c, bool imag) {
    const Layout& L = c->L;
    const int mode = imag ? MODE_IMAG : MODE_REAL;
    const int k = imag ? 0 : 1;
    T* phi = c->at<T>(L.o_sfield);
    GP_TRY(settle(c));
    GP_TRY(g_convolution(c, psi(c), &c->sc()->scale));
    GP_TRY(pass_begin(c, GP_PASS_C2R_NL_CNX));
    GP_TRY(g_c2r(c, phi));
    if (L.lx) {
      // long x lines: the nonlinear sub-step in place, then the segmented sweep
      GP_HIP(GLaunch<T>::nonlinear(mode, c->st, psi(c), Vp(c), phi, &c->sc()->scale,
                                   g_scalars(c), L.n0, L.n1, L.n2, c->at<double>(L.o_pnl)));
      GP_TRY(g_sweep(c, 0, k, 0));
    } else {
      // the nonlinear sub-step rides in the x sweep's loads
      const GNl nlz{Vp(c), phi, &c->sc()->scale, g_scalars(c), L.n0, L.n1, L.n2,
                    c->at<double>(L.o_pnl)};
      GP_HIP(GLaunch<T>::cn_x_nonlinear(mode, c->st, psi(c), L.n0, L.n1 * L.n2, cn(c, 0, k),
                                        nlz));
    }
    GP_TRY(pass_end(c, GP_PASS_C2R_NL_CNX));
    if (c->p.geom == GP_3D) {
      GP_TRY(pass_begin(c, GP_PASS_CN_Y));
      GP_TRY(g_sweep(c, 1, k, 0));
      GP_TRY(pass_end(c, GP_PASS_CN_Y));
      GP_TRY(pass_begin(c, GP_PASS_CN_Z));
      GP_TRY(g_sweep(c, 2, k, 1));
      GP_TRY(pass_end(c, GP_PASS_CN_Z));
    } else {
      GP_TRY(pass_begin(c, GP_PASS_CN_Y));
      GP_TRY(g_sweep(c, 1, k, 1));
      GP_TRY(pass_end(c, GP_PASS_CN_Y));
    }
    return finalize(c, imag ? (int)FIN_IMAG : (int)FIN_REAL);
  }

  static gp_status g_observe(gp_ctx* c) {
    const Layout& L = c->L;
    T* phi = c->at<T>(L.o_sfield);
    GP_TRY(g_phi(c, psi(c), &c->sc()->scale, phi));
    GP_HIP(GLaunch<T>::nonlinear(MODE_OBSERVE, c->st, psi(c), Vp(c), phi,
                                 &c->sc()->scale, g_scalars(c), L.n0, L.n1, L.n2,
                                 c->at<double>(L.o_pnl)));
    if (c->p.geom == GP_3D) return z_observe(c, FIN_OBSERVE);
    return finalize(c, FIN_OBSERVE);
  }

  // y/z transforms of the x-half spectrum, U(k)/N product, inverse y/z transforms
  // y/z transforms of the x-half spectrum of the stored density, U(k) scale^2/N product,
  // inverse transforms; fin2: a two-stage folded finalisation (mode fin_mode) whose
  // second stage rides in the forward y FFT
  static gp_status spectrum_passes(gp_ctx* c, const double* scale,
                                   const FinArgs* fin2 = nullptr, int fin_mode = FIN_REAL) {
    const Layout& L = c->L;
    const int H = L.n0 / 2 + 1;
    if (c->p.geom == GP_3D) {
      const int nl = H * L.n2;
      const int lb = c->fp64 ? Launch<double>::lbf(L.n1) : Launch<float>::lbf(L.n1);
      const int tc = tv_of(c->fp64, L.n2);
      if (fin2) {
        GP_HIP(Launch<T>::fft_line_fin(L.n1, (nl + lb - 1) / lb, c->st, spec(c), tw(c, 1), nl,
                                       *fin2, fin_mode));
      } else {
        GP_PASS(c, GP_PASS_FFT_Y_FWD,
                Launch<T>::fft_line(L.n1, false, (nl + lb - 1) / lb, c->st, spec(c), tw(c, 1),
                                    nl));
      }
      GP_PASS(c, GP_PASS_CONV_Z,
              Launch<T>::conv_col(L.n2, ((L.n1 + tc - 1) / tc) * H, c->st, spec(c),
                                  Kp(c), scale, tw(c, 2), L.n1));
      GP_PASS(c, GP_PASS_FFT_Y_INV,
              Launch<T>::fft_line(L.n1, true, (nl + lb - 1) / lb, c->st, spec(c), tw(c, 1), nl));
    } else {
      const int lb = c->fp64 ? Launch<double>::lb(L.n1) : Launch<float>::lb(L.n1);
      GP_PASS(c, GP_PASS_CONV_Y,
              Launch<T>::conv_line(L.n1, (H + lb - 1) / lb, c->st, spec(c), Kp(c),
                                   scale, tw(c, 1), H));
    }
    return GP_OK;
  }

  // density of `src` (times scale^2) -> spectrum -> U(k) product -> x-half spectrum;
  // `fold`: the previous step's finalisation (mode fin_mode) rides in the x pass (one
  // block, or the first-stage slices there and the finalize block in the forward y FFT)
  static gp_status convolution(gp_ctx* c, const cpx<T>* src, const double* scale,
                               const FinArgs* fold = nullptr, int fin_mode = FIN_REAL) {
    const Layout& L = c->L;
    double* px = c->at<double>(L.o_px[c->px_sel]);
    if (fold) {
      GP_HIP(Launch<T>::r2c_x_fin(L.n0, L.nb_r2c, c->st, src, spec(c), tw(c, 0), px, L.n1, L.n2,
                                  *fold, fin_mode, fold->nstage > 0 ? fold->nstage : 1));
    } else {
      GP_PASS(c, GP_PASS_R2C_X,
              Launch<T>::r2c_x(L.n0, L.nb_r2c, c->st, src, spec(c), tw(c, 0), px, L.n1, L.n2));
    }
    return spectrum_passes(c, scale, fold && fold->nstage > 0 ? fold : nullptr, fin_mode);
  }
  static gp_status convolution(gp_ctx* c) {
    if (c->L.generic) return g_convolution(c, psi(c), &c->sc()->scale);
    return convolution(c, psi(c), &c->sc()->scale);
  }

  // Backpropagation through one real-time step (see gp_step_real_adjoint).
  static gp_status adjoint(gp_ctx* c, const cpx<T>* psin, cpx<T>* lam, double* gradV,
                           double* grad_g, double* grad_gdd) {
    const Layout& L = c->L;
    if (L.generic) {
      snprintf(g_last_error, sizeof(g_last_error),
               "the adjoint step needs axis lengths with specialised passes");
      return GP_E_SIZE;
    }
    const int tcy = tc_of(c->fp64, L.n1);
    const int nb_y = ((L.n0 + tcy - 1) / tcy) * L.n2;
    if (c->p.geom == GP_3D) {
      GP_HIP(Launch<T>::cn_col(L.n2, MODE_ADJ, false, L.nb_col, c->st, lam, cn(c, 2, 2), nullptr, L.n0, (size_t)L.n0 * L.n1,
                               (size_t)L.n0));
    }
    GP_HIP(Launch<T>::cn_col(L.n1, MODE_ADJ, false, nb_y, c->st, lam, cn(c, 1, 2), nullptr, L.n0, (size_t)L.n0,
                             (size_t)L.n0 * L.n1));
    GP_TRY(convolution(c, psin, &c->sc()->one));
    const StepScalars sx = step_scalars(c);
    T* sf = c->at<T>(L.o_sfield);
    double* pa = c->at<double>(L.o_padj);
    GP_HIP(Launch<T>::adj_x(L.n0, L.nb_x, c->st, lam, psin, Vp(c), spec(c), tw(c, 0),
                            cn(c, 0, 2), sx, sf, gradV, pa, L.n1, L.n2));
    GP_HIP(Launch<T>::r2c_real(L.n0, L.nb_x, c->st, sf, spec(c), tw(c, 0), L.n1, L.n2));
    GP_TRY(spectrum_passes(c, &c->sc()->one));
    GP_HIP(Launch<T>::adj_fin(L.n0, L.nb_x, c->st, lam, psin, sf, spec(c), tw(c, 0), sx, L.n1,
                              L.n2));
    const double cfac = (c->p.geom == GP_3D) ? 1.0 : 1.0 / (sqrt(2.0 * M_PI) * d_perp(c->p));
    hipLaunchKernelGGL(k_adj_reduce, dim3(1), dim3(kThreads), 0, c->st, pa, L.nb_x, cfac,
                       grad_g, grad_gdd);
    return dev(hipGetLastError());
  }

  // FP64 finalisation of the partial sums (fin_mode: FIN_IMAG/REAL after a step,
  // FIN_OBSERVE for gp_energy, FIN_EKZ for the pending z-kinetic part)
  static gp_status finalize(gp_ctx* c, int fin_mode) {
    GP_TRY(pass_begin(c, GP_PASS_FINALIZE));
    const FinArgs a = fin_args(c, c->px_sel);
    if (a.nstage > 0)
      hipLaunchKernelGGL(k_prereduce, dim3(a.nstage), dim3(kThreads), 0, c->st, a, fin_mode);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, c->st, a, fin_mode);
    GP_HIP(hipGetLastError());
    return pass_end(c, GP_PASS_FINALIZE);
  }

  // z-difference sums of the stored state (3D), for the kinetic energy, then finalise
  // with fin_mode (FIN_EKZ: pending z-kinetic part; FIN_OBSERVE: full record)
  static gp_status z_observe(gp_ctx* c, int fin_mode) {
    const Layout& L = c->L;
    if (L.generic) {
      GP_TRY(g_sweep(c, 2, 0, 2));
      return finalize(c, fin_mode);
    }
    GP_HIP(Launch<T>::cn_col(L.n2, MODE_OBSERVE, true, L.nb_col, c->st, psi(c), nullptr,
                             c->at<double>(L.o_pcol), L.n0, (size_t)L.n0 * L.n1,
                             (size_t)L.n0));
    return finalize(c, fin_mode);
  }

  static gp_status step(gp_ctx* c, bool imag) {
    if (c->L.generic) return g_step(c, imag);
    const Layout& L = c->L;
    const int mode = imag ? MODE_IMAG : MODE_REAL;
    const int fin = imag ? (int)FIN_IMAG : (int)FIN_REAL;
    const int k = imag ? 0 : 1;  // factor table: imaginary or real time
    // Without per-pass timing a step defers its finalisation: the next step's x pass (or
    // its forward y FFT) carries it while writing the other x-partial buffer.  The x pass
    // does not read the scale the finalisation writes (the convolution and the x CN pass
    // apply it, after it).  The record and non-finite flag of a step therefore land one
    // launch later; every other entry point settles an outstanding one first.
    const bool defer = c->tmask == 0;
    FinArgs prev{};
    bool fold = false;
    const int prev_mode = c->pend_mode;
    if (defer && c->fin_pending) {
      prev = fin_args(c, c->pend_sel);
      fold = c->p.geom == GP_3D || prev.nstage == 0;
      if (fold) {
        c->fin_pending = false;
        c->px_sel = 1 - c->pend_sel;
      }
    }
    GP_TRY(settle(c));
    GP_TRY(convolution(c, psi(c), &c->sc()->scale, fold ? &prev : nullptr, prev_mode));
    const StepScalars sx = step_scalars(c);
    // timed: the launch's own dispatch timestamps fill the event pair (no separate event
    // packets around it), and every block stamps its start and end
    const bool span = (c->tmask >> GP_PASS_C2R_NL_CNX) & 1u;
    unsigned long long* stamps = span ? c->at<unsigned long long>(L.o_stamps) : nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (span) {
      e0 = take_event(c);
      e1 = take_event(c);
      if (!e0 || !e1) {
        if (e0) c->tpool.push_back(e0);
        if (e1) c->tpool.push_back(e1);
        return GP_E_DEVICE;
      }
      c->tev[GP_PASS_C2R_NL_CNX].emplace_back(e0, e1);
    }
    GP_HIP(Launch<T>::c2r_nl_cnx(L.n0, mode, L.nb_x, c->st, psi(c), Vp(c),
                                 &c->sc()->scale, spec(c), tw(c, 0), cn(c, 0, k), sx,
                                 c->at<double>(L.o_pnl), nullptr, L.n1, L.n2, stamps, e0, e1));
    if (span) {
      hipLaunchKernelGGL(k_span_reduce, dim3(1), dim3(kThreads), 0, c->st, stamps, L.nb_x,
                         c->sc()->span);
      GP_HIP(hipGetLastError());
    }
    const int tcy = tc_of(c->fp64, L.n1);
    if (c->p.geom == GP_3D) {
      GP_PASS(c, GP_PASS_CN_Y,
              Launch<T>::cn_col(L.n1, mode, false, ((L.n0 + tcy - 1) / tcy) * L.n2, c->st,
                                psi(c), cn(c, 1, k), nullptr, L.n0, (size_t)L.n0,
                                (size_t)L.n0 * L.n1));
      GP_PASS(c, GP_PASS_CN_Z,
              Launch<T>::cn_col(L.n2, mode, true, L.nb_col, c->st, psi(c), cn(c, 2, k),
                                c->at<double>(L.o_pcol), L.n0, (size_t)L.n0 * L.n1,
                                (size_t)L.n0));
    } else {
      GP_PASS(c, GP_PASS_CN_Y,
              Launch<T>::cn_col(L.n1, mode, true, L.nb_col, c->st, psi(c), cn(c, 1, k),
                                c->at<double>(L.o_pcol), L.n0, (size_t)L.n0,
                                (size_t)L.n0 * L.n1));
    }
    if (defer) {
      c->fin_pending = true;
      c->pend_sel = c->px_sel;
      c->pend_mode = fin;
      return GP_OK;
    }
    return finalize(c, fin);
  }

  // One launch of a pass exactly as inside a real-time step (burst timing).
  static gp_status launch_pass(gp_ctx* c, int pass) {
    const Layout& L = c->L;
    if (L.generic) return GP_E_ARG;
    const int tcy = tc_of(c->fp64, L.n1);
    switch (pass) {
      case GP_PASS_R2C_X:
        return dev(Launch<T>::r2c_x(L.n0, L.nb_r2c, c->st, psi(c), spec(c),
                                    tw(c, 0), c->at<double>(L.o_px[c->px_sel]), L.n1, L.n2));
      case GP_PASS_C2R_NL_CNX:
        return dev(Launch<T>::c2r_nl_cnx(L.n0, MODE_REAL, L.nb_x, c->st, psi(c),
                                         Vp(c), &c->sc()->scale, spec(c), tw(c, 0),
                                         cn(c, 0, 1), step_scalars(c), c->at<double>(L.o_pnl),
                                         nullptr, L.n1, L.n2));
      case GP_PASS_CN_Y:
        if (c->p.geom == GP_3D)
          return dev(Launch<T>::cn_col(L.n1, MODE_REAL, false, ((L.n0 + tcy - 1) / tcy) * L.n2,
                                       c->st, psi(c), cn(c, 1, 1), nullptr,
                                       L.n0, (size_t)L.n0, (size_t)L.n0 * L.n1));
        return dev(Launch<T>::cn_col(L.n1, MODE_REAL, true, L.nb_col, c->st, psi(c), cn(c, 1, 1),
                                     c->at<double>(L.o_pcol), L.n0,
                                     (size_t)L.n0, (size_t)L.n0 * L.n1));
      case GP_PASS_CN_Z:
        if (c->p.geom != GP_3D) return GP_E_ARG;
        return dev(Launch<T>::cn_col(L.n2, MODE_REAL, true, L.nb_col, c->st, psi(c), cn(c, 2, 1),
                                     c->at<double>(L.o_pcol), L.n0,
                                     (size_t)L.n0 * L.n1, (size_t)L.n0));
      default:
        return GP_E_ARG;
    }
  }

  static gp_status observe(gp_ctx* c) {
    if (c->L.generic) return g_observe(c);
    const Layout& L = c->L;
    GP_TRY(convolution(c));
    const StepScalars sx = step_scalars(c);
    GP_HIP(Launch<T>::c2r_nl_cnx(L.n0, MODE_OBSERVE, L.nb_x, c->st, psi(c), Vp(c),
                                 &c->sc()->scale, spec(c), tw(c, 0), nullptr, sx,
                                 c->at<double>(L.o_pnl), nullptr, L.n1, L.n2));
    if (c->p.geom == GP_3D) return z_observe(c, FIN_OBSERVE);
    return finalize(c, FIN_OBSERVE);
  }

  static gp_status phi(gp_ctx* c, T* out) {
    if (c->L.generic) return g_phi(c, psi(c), &c->sc()->scale, out);
    const Layout& L = c->L;
    GP_TRY(convolution(c));
    const StepScalars sx = step_scalars(c);
    GP_HIP(Launch<T>::c2r_nl_cnx(L.n0, MODE_PHI, L.nb_x, c->st, psi(c), Vp(c),
                                 &c->sc()->scale, spec(c), tw(c, 0), nullptr, sx,
                                 c->at<double>(L.o_pnl), out, L.n1, L.n2));
    return GP_OK;
  }

  static gp_status init_tables(gp_ctx* c) {
    const Layout& L = c->L;
    const bool lng[3] = {L.lx, L.ly, false};
    if (L.generic) {
      const int ns3[3] = {L.n0, L.n1, L.n2};
      for (int a = 0; a < (c->p.geom == GP_3D ? 3 : 2); ++a) {
        if (lng[a]) {
          if (!gen_long_subplan(L.lg[a].A, gen_max_line<T>() / 2, &c->lplan[a][0]) ||
              !gen_long_subplan(L.lg[a].B, gen_max_line<T>(), &c->lplan[a][1]))
            return GP_E_SIZE;
        } else if (!gen_plan(ns3[a], &c->gplan[a])) {
          return GP_E_SIZE;
        }
      }
      GP_HIP(GLaunch<T>::prepare());
    }
    const int ns[3] = {L.n0, L.n1, L.n2};
    const double hs[3] = {L.h0, L.h1, L.h2};
    const int naxes = (c->p.geom == GP_3D) ? 3 : 2;
    // twiddles of a stage length m and, for a Bluestein plan, its chirp and filter
    auto plan_tables = [&](GPlan& pl, size_t o_tw, size_t o_blue) {
      hipLaunchKernelGGL(k_twiddles<T>, dim3(blocks_for(pl.m)), dim3(kThreads), 0, c->st,
                         c->at<cpx<T>>(o_tw), pl.m);
      if (pl.blue) {
        cpx<T>* ch = c->at<cpx<T>>(o_blue);
        cpx<T>* fl = ch + pl.n;
        hipLaunchKernelGGL(k_bluestein<T>, dim3(blocks_for(pl.m)), dim3(kThreads), 0, c->st, ch,
                           fl, pl.n, pl.m);
        pl.chirp = ch;
        pl.filt = fl;
      }
    };
    for (int a = 0; a < naxes; ++a) {
      if (lng[a]) {
        plan_tables(c->lplan[a][0], L.o_ltw[a][0], L.o_lblue[a][0]);
        plan_tables(c->lplan[a][1], L.o_ltw[a][1], L.o_lblue[a][1]);
        hipLaunchKernelGGL(k_twiddles<T>, dim3(blocks_for(ns[a])), dim3(kThreads), 0, c->st,
                           c->at<cpx<T>>(L.o_ltw[a][2]), ns[a]);   // W_N^m
      } else if (L.generic) {
        plan_tables(c->gplan[a], L.o_tw[a], L.o_blue[a]);
      } else {
        hipLaunchKernelGGL(k_twiddles<T>, dim3(blocks_for(ns[a])), dim3(kThreads), 0, c->st,
                           c->at<cpx<T>>(L.o_tw[a]), ns[a]);
      }
      const double Ar = c->p.dt / (4.0 * hs[a] * hs[a]);
      // lanes per line of the solve that sweeps this axis: x lines in the x pass, columns
      // in the strided sweeps
      const int P = L.generic ? 1
                              : kThreads / (a == 0 ? Launch<T>::tj(ns[a]) : Launch<T>::tc(ns[a]));
      hipLaunchKernelGGL(k_cn_tables<T>, dim3(1), dim3(64), 0, c->st,
                         c->at<cpx<T>>(L.o_cn[a][0]), c->at<cpx<T>>(L.o_cn[a][1]),
                         c->at<cpx<T>>(L.o_cn[a][2]), ns[a], Ar, P);
      if (a == 0 ? L.lx : (a == 1 && L.sy)) {  // the segments' fixed numbers per factor set
        for (int t = 0; t < 3; ++t)
          hipLaunchKernelGGL(k_seg_tables<T>, dim3(blocks_for(L.lg[a].nseg)), dim3(kThreads), 0,
                             c->st, c->at<cpx<T>>(L.o_cn[a][t]), L.lg[a].sn, L.lg[a].nseg,
                             c->at<cpx<T>>(L.o_seg[a][t]),
                             c->at<cpx<T>>(L.o_seg[a][t]) + 2 * L.lg[a].nseg);
      }
    }
    KernelGeom kg{};
    kg.geom = c->p.geom;
    kg.n0 = L.n0;
    kg.n1 = L.n1;
    kg.n2 = L.n2;
    kg.h0 = L.h0;
    kg.h1 = L.h1;
    kg.h2 = L.h2;
    kg.R = c->p.cutoff_R;
    kg.d = (c->p.geom == GP_3D) ? 0.0 : d_perp(c->p);
    if (L.lx) {
      kg.Ax = L.lg[0].A;
      kg.Bx = L.lg[0].B;
      kg.rs = L.lxg.rs;
    }
    if (L.ly) {
      kg.Ay = L.lg[1].A;
      kg.By = L.lg[1].B;
    }
    hipLaunchKernelGGL(k_kernel_table<T>, dim3(blocks_for(L.nktab)), dim3(kThreads), 0, c->st,
                       Kp(c), kg);
    double w0 = c->p.gamma, w1, w2 = 0.0;
    if (c->p.geom == GP_3D) {
      w1 = c->p.nu;
      w2 = c->p.lambda;
    } else if (c->p.geom == GP_2D_XY) {
      w1 = c->p.nu;
    } else {
      w1 = c->p.lambda;
    }
    hipLaunchKernelGGL(k_harmonic<T>, dim3(blocks_for(L.npts)), dim3(kThreads), 0, c->st,
                       Vp(c), L.n0, L.n1, L.n2, L.h0, L.h1, L.h2, w0, w1, w2);
    Scalars* s = c->sc();
    hipLaunchKernelGGL(k_reset_state, dim3(1), dim3(64), 0, c->st, &s->scale, &s->one, &s->ekz,
                       &s->flags, &s->ring_pos);
    hipLaunchKernelGGL(k_clear_u64, dim3(1), dim3(64), 0, c->st, s->span, 2);
    return dev(hipGetLastError());
  }

  // Host transfers go through the io staging area in chunks of at most kIoChunk points
  // (FP64 values), so the workspace holds 16 B x min(points, kIoChunk) for them.
  static gp_status set_psi(gp_ctx* c, const void* src, int on_device) {
    const Layout& L = c->L;
    if (on_device) {
      hipLaunchKernelGGL((k_psi_in<T, T>), dim3(blocks_for(L.npts)), dim3(kThreads), 0, c->st,
                         psi(c), reinterpret_cast<const cpx<T>*>(src), (size_t)0, L.npts, L.n0,
                         L.n1, L.n2);
      GP_HIP(hipGetLastError());
    } else {
      cpx<double>* io = c->at<cpx<double>>(L.o_io);
      const cpx<double>* h = reinterpret_cast<const cpx<double>*>(src);
      for (size_t off = 0; off < L.npts; off += kIoChunk) {
        const size_t cnt = std::min(kIoChunk, L.npts - off);
        GP_HIP(hipMemcpyAsync(io, h + off, 16 * cnt, hipMemcpyHostToDevice, c->st));
        hipLaunchKernelGGL((k_psi_in<T, double>), dim3(blocks_for(cnt)), dim3(kThreads), 0,
                           c->st, psi(c), io, off, cnt, L.n0, L.n1, L.n2);
        GP_HIP(hipGetLastError());
      }
      GP_HIP(hipStreamSynchronize(c->st));
    }
    hipLaunchKernelGGL(k_set_scale_one, dim3(1), dim3(64), 0, c->st, &c->sc()->scale);
    return dev(hipGetLastError());
  }

  static gp_status get_psi(gp_ctx* c, void* dst, int on_device) {
    const Layout& L = c->L;
    if (on_device) {
      hipLaunchKernelGGL((k_psi_out<T, T>), dim3(blocks_for(L.npts)), dim3(kThreads), 0, c->st,
                         reinterpret_cast<cpx<T>*>(dst), psi(c), &c->sc()->scale, (size_t)0,
                         L.npts);
      return dev(hipGetLastError());
    }
    cpx<double>* io = c->at<cpx<double>>(L.o_io);
    cpx<double>* h = reinterpret_cast<cpx<double>*>(dst);
    for (size_t off = 0; off < L.npts; off += kIoChunk) {
      const size_t cnt = std::min(kIoChunk, L.npts - off);
      hipLaunchKernelGGL((k_psi_out<T, double>), dim3(blocks_for(cnt)), dim3(kThreads), 0,
                         c->st, io, psi(c), &c->sc()->scale, off, cnt);
      GP_HIP(hipGetLastError());
      GP_HIP(hipMemcpyAsync(h + off, io, 16 * cnt, hipMemcpyDeviceToHost, c->st));
    }
    GP_HIP(hipStreamSynchronize(c->st));
    return GP_OK;
  }

  static gp_status set_potential(gp_ctx* c, const void* src, int on_device) {
    const Layout& L = c->L;
    if (on_device) {
      GP_HIP(hipMemcpyAsync(Vp(c), src, L.esz * L.npts, hipMemcpyDefault, c->st));
      return GP_OK;
    }
    double* io = c->at<double>(L.o_io);
    const double* h = reinterpret_cast<const double*>(src);
    for (size_t off = 0; off < L.npts; off += kIoChunk) {
      const size_t cnt = std::min(kIoChunk, L.npts - off);
      GP_HIP(hipMemcpyAsync(io, h + off, 8 * cnt, hipMemcpyHostToDevice, c->st));
      hipLaunchKernelGGL((k_real_convert<T, double>), dim3(blocks_for(cnt)), dim3(kThreads), 0,
                         c->st, Vp(c) + off, io, cnt);
      GP_HIP(hipGetLastError());
    }
    GP_HIP(hipStreamSynchronize(c->st));
    return GP_OK;
  }

  static gp_status dipolar(gp_ctx* c, void* dst, int on_device) {
    const Layout& L = c->L;
    if (on_device) return phi(c, reinterpret_cast<T*>(dst));
    T* tmp = c->at<T>(L.o_sfield);  // free outside the adjoint step
    GP_TRY(phi(c, tmp));
    double* io = c->at<double>(L.o_io);
    double* h = reinterpret_cast<double*>(dst);
    for (size_t off = 0; off < L.npts; off += kIoChunk) {
      const size_t cnt = std::min(kIoChunk, L.npts - off);
      hipLaunchKernelGGL((k_real_convert<double, T>), dim3(blocks_for(cnt)), dim3(kThreads), 0,
                         c->st, io, tmp + off, cnt);
      GP_HIP(hipGetLastError());
      GP_HIP(hipMemcpyAsync(h + off, io, 8 * cnt, hipMemcpyDeviceToHost, c->st));
    }
    GP_HIP(hipStreamSynchronize(c->st));
    return GP_OK;
  }
};

gp_status check_flags(gp_ctx* c) {
  int flags = 0;
  GP_HIP(hipMemcpyAsync(&flags, &c->sc()->flags, sizeof(int), hipMemcpyDeviceToHost, c->st));
  GP_HIP(hipStreamSynchronize(c->st));
  return (flags & 1) ? GP_E_NONFINITE : GP_OK;
}

void drop_graphs(gp_ctx* c) {
  for (auto& dir : c->gexec)
    for (auto& st : dir)
      for (auto& g : st) {
        if (g.ex) hipGraphExecDestroy(g.ex);
        g = gp_ctx::GraphRec{};
      }
}

gp_status one_step(gp_ctx* c, bool imag) {
  return c->fp64 ? Passes<double>::step(c, imag) : Passes<float>::step(c, imag);
}

// Capture `len` steps on a private stream (the caller's stream may be the null stream,
// which cannot be captured); the graph is launched on the caller's stream.  Capturing
// runs the host side of the steps, so the context's finalisation state afterwards is the
// one the graph leaves behind; it is recorded with the graph for later replays.
gp_status build_graph(gp_ctx* c, bool imag, int len, gp_ctx::GraphRec* rec) {
  if (!c->cap_st) GP_HIP(hipStreamCreateWithFlags(&c->cap_st, hipStreamNonBlocking));
  const hipStream_t user = c->st;
  c->st = c->cap_st;
  hipGraph_t g = nullptr;
  gp_status s = dev(hipStreamBeginCapture(c->cap_st, hipStreamCaptureModeThreadLocal));
  if (s == GP_OK) {
    for (int i = 0; i < len && s == GP_OK; ++i) s = one_step(c, imag);
    const gp_status e = dev(hipStreamEndCapture(c->cap_st, &g));
    if (s == GP_OK) s = e;
  }
  c->st = user;
  if (s != GP_OK) {
    if (g) hipGraphDestroy(g);
    return s;
  }
  hipGraphExec_t ex = nullptr;
  s = dev(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
  hipGraphDestroy(g);
  if (s != GP_OK) return s;
  rec->ex = ex;
  rec->end_pending = c->fin_pending;
  rec->end_sel = c->pend_sel;
  return GP_OK;
}

gp_status run_steps(gp_ctx* c, int nsteps, bool imag) {
  if (!c) return GP_E_ARG;
  clear_stale_error();
  if (nsteps < 0) return GP_E_ARG;
  if (!c->psi_set) return GP_E_STATE;
  if (!c->ekz_valid) GP_TRY(settle(c));
  if (c->p.geom == GP_3D && !c->ekz_valid) {
    if (c->fp64) {
      GP_TRY(Passes<double>::z_observe(c, FIN_EKZ));
    } else {
      GP_TRY(Passes<float>::z_observe(c, FIN_EKZ));
    }
    c->ekz_valid = true;
  }
  if (!c->use_graphs || c->tmask != 0) {
    for (int done = 0; done < nsteps; ++done) GP_TRY(one_step(c, imag));
    return GP_OK;
  }
  // a finalisation of the other time direction is completed first, so that every graph
  // starts from nothing outstanding or from one of its own direction
  const int fmode = imag ? (int)FIN_IMAG : (int)FIN_REAL;
  if (c->fin_pending && c->pend_mode != fmode) GP_TRY(settle(c));
  for (int done = 0; done < nsteps;) {
    int li = 3;
    while ((1 << li) > nsteps - done) --li;
    const int start = c->fin_pending ? 1 + c->pend_sel : 0;
    gp_ctx::GraphRec& g = c->gexec[imag ? 0 : 1][start][li];
    if (!g.ex) {
      GP_TRY(build_graph(c, imag, 1 << li, &g));   // leaves the host state at g's end
    } else {
      c->fin_pending = g.end_pending;
      c->pend_sel = g.end_sel;
      c->px_sel = g.end_sel;
      c->pend_mode = fmode;
    }
    GP_HIP(hipGraphLaunch(g.ex, c->st));
    done += 1 << li;
  }
  return GP_OK;
}

// ------------------------------------------------ allocation-free dipolar potential
// Library-owned scratch for gp_dipolar_potential_noalloc: the half spectrum, the kernel
// table, the twiddles, the x-pass partial sums and the device scalars of one call.  Each
// device holds its own copy for the life of the process.  In host code `scratch` only
// names the symbol; the device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

gp_status scratch_for_current_device(char** out) {
  int devid = 0;
  GP_HIP(hipGetDevice(&devid));
  if (devid < 0 || devid >= kMaxDevices) return GP_E_ARG;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[devid]) {
    void* ptr = nullptr;
    GP_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return GP_E_DEVICE;
    g_scratch_ptr[devid] = reinterpret_cast<char*>(ptr);
  }
  *out = g_scratch_ptr[devid];
  return GP_OK;
}

// The arrays one dipolar-potential evaluation touches, carved from offset 0: the pass
// kernels address them through the context exactly as in a workspace.
Layout scratch_layout(const gp_params* p) {
  Layout L = make_layout(p);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o += align_up(bytes);
    return r;
  };
  L.o_spec = take(2 * L.esz * L.nspec);
  L.o_ktab = take(L.esz * L.nktab);
  const int ns[3] = {L.n0, L.n1, L.n2};
  for (int a = 0; a < 3; ++a) L.o_tw[a] = take(2 * L.esz * ns[a]);
  L.o_px[0] = L.o_px[1] = take(sizeof(double) * 2 * L.nb_x);
  L.o_scalars = take(sizeof(Scalars));
  L.total = o;
  return L;
}

template <typename T>
gp_status dipolar_noalloc_t(gp_ctx* c, const cpx<T>* psi, T* phi) {
  const Layout& L = c->L;
  // tables of this call's grid (the scratch keeps whatever the last call left)
  const int ns[3] = {L.n0, L.n1, L.n2};
  const int naxes = (c->p.geom == GP_3D) ? 3 : 2;
  for (int a = 0; a < naxes; ++a)
    hipLaunchKernelGGL(k_twiddles<T>, dim3(blocks_for(ns[a])), dim3(kThreads), 0, c->st,
                       c->at<cpx<T>>(L.o_tw[a]), ns[a]);
  KernelGeom kg{};
  kg.geom = c->p.geom;
  kg.n0 = L.n0;
  kg.n1 = L.n1;
  kg.n2 = L.n2;
  kg.h0 = L.h0;
  kg.h1 = L.h1;
  kg.h2 = L.h2;
  kg.R = c->p.cutoff_R;
  kg.d = (c->p.geom == GP_3D) ? 0.0 : d_perp(c->p);
  hipLaunchKernelGGL(k_kernel_table<T>, dim3(blocks_for(L.nktab)), dim3(kThreads), 0, c->st,
                     c->at<T>(L.o_ktab), kg);
  Scalars* sc = c->sc();
  hipLaunchKernelGGL(k_reset_state, dim3(1), dim3(64), 0, c->st, &sc->scale, &sc->one,
                     &sc->ekz, &sc->flags, &sc->ring_pos);
  GP_HIP(hipGetLastError());
  // |psi|^2 of the caller's (physical) psi -> spectrum -> U(k)/N product -> inverse
  GP_TRY(Passes<T>::convolution(c, psi, &sc->one));
  GP_HIP(Launch<T>::c2r_nl_cnx(L.n0, MODE_PHI, L.nb_x, c->st, nullptr, nullptr, &sc->one,
                               Passes<T>::spec(c), Passes<T>::tw(c, 0), nullptr,
                               step_scalars(c), nullptr, phi, L.n1, L.n2));
  return GP_OK;
}

gp_status dipolar_noalloc(const gp_params* p, const void* psi, void* phi, hipStream_t st) {
  if (is_generic(p)) {
    snprintf(g_last_error, sizeof(g_last_error),
             "the allocation-free call needs axis lengths with specialised passes");
    return GP_E_SIZE;
  }
  const Layout L = scratch_layout(p);
  if (L.total > kScratchBytes) {
    snprintf(g_last_error, sizeof(g_last_error),
             "grid needs %zu bytes of scratch; the allocation-free call holds %zu",
             L.total, kScratchBytes);
    return GP_E_SIZE;
  }
  char* base = nullptr;
  GP_TRY(scratch_for_current_device(&base));
  // a context on the stack over the scratch: no host or device allocation
  gp_ctx c;
  c.p = *p;
  c.L = L;
  c.st = st;
  c.ws = base;
  c.fp64 = p->prec == GP_FP64;
  c.psi_set = true;
  c.ekz_valid = true;
  c.gc = contact(c.p);
  return c.fp64 ? dipolar_noalloc_t<double>(&c, reinterpret_cast<const cpx<double>*>(psi),
                                            reinterpret_cast<double*>(phi))
                : dipolar_noalloc_t<float>(&c, reinterpret_cast<const cpx<float>*>(psi),
                                           reinterpret_cast<float*>(phi));
}

}  // namespace

// =============================================================== batched ensemble
struct gp_batch {
  int count = 0;
  bool fp64 = false;
  hipStream_t st = nullptr;
  std::vector<gp_ctx*> inst;
  std::vector<gp_params> params;
  char* ws = nullptr;
  void* desc = nullptr;                       // device BDesc<T>[count]
  WorkItem* work[BP_COUNT][kBatchClasses] = {};
  int nwork[BP_COUNT][kBatchClasses] = {};
  // tile-shape variant per (pass, class) (Tiles<T, N, S>) and the persistent block count
  // asked for (0: the default, min(items, 1024))
  int shape[BP_COUNT][kBatchClasses] = {};
  int grid_req[BP_COUNT][kBatchClasses] = {};
  WorkItem* work_base = nullptr;  // device work-list region (per-(pass, class) capacities)
  size_t lds[BP_COUNT][kBatchClasses][3] = {};  // [pass][class][mode imag/real/observe]
  int grid[BP_COUNT][kBatchClasses] = {};
  bool use_graphs = true;
  hipStream_t cap_st = nullptr;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  std::vector<double> cpl;                    // (g, g_dd) per instance in the descriptors
  // The two size-class kernels of one pass touch disjoint work items.  With
  // two_streams set, the larger class runs on a second stream (default priority),
  // forked from and joined back to the step's stream around each pass; by default both
  // run in order on the step's stream, so a captured step graph is one linear chain.
  bool two_streams = false;
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

namespace {

constexpr int kBatchDefaultGrid = 1024;

gp_status batch_validate(const gp_params* arr, int count) {
  if (!arr || count <= 0) return GP_E_ARG;
  for (int i = 0; i < count; ++i) {
    GP_TRY(validate(&arr[i]));
    if (arr[i].geom == GP_3D) return GP_E_ARG;
    if (arr[i].prec != arr[0].prec) return GP_E_ARG;
    const int n1 = arr[i].geom == GP_2D_XY ? arr[i].ny : arr[i].nz;
    const bool ok = arr[i].prec == GP_FP64
                        ? (batch_size_ok<double>(arr[i].nx) && batch_size_ok<double>(n1))
                        : (batch_size_ok<float>(arr[i].nx) && batch_size_ok<float>(n1));
    if (!ok) return GP_E_SIZE;
  }
  return GP_OK;
}

// Workspace: descriptors, work lists, then one single-grid workspace per instance.
struct BatchLayout {
  size_t o_desc, o_work, o_inst0, total;
  std::vector<size_t> o_inst;
  int total_items;
};

// The class (size class of the pass's line length) and work items of instance (n0, n1)
// in pass p with shape variant sh.
int batch_pass_class(int p, int n0, int n1) {
  return batch_class((p == BP_R2C || p == BP_C2R) ? n0 : n1);
}
template <typename T>
int batch_item_cap(int p, int n0, int n1) {
  int m = 0;
  for (int sh = 0; sh < kBatchShapes; ++sh) m = std::max(m, batch_tiles<T>(p, n0, n1, sh));
  return m;
}

// Work-list capacity per (pass, class): every instance's largest tile count over the
// shape variants, so a variant change rebuilds a list in place.
template <typename T>
void batch_caps(const gp_params* arr, int count, int cap[BP_COUNT][kBatchClasses]) {
  for (int p = 0; p < BP_COUNT; ++p)
    for (int k = 0; k < kBatchClasses; ++k) cap[p][k] = 0;
  for (int i = 0; i < count; ++i) {
    const int n0 = arr[i].nx, n1 = arr[i].geom == GP_2D_XY ? arr[i].ny : arr[i].nz;
    for (int p = 0; p < BP_COUNT; ++p)
      cap[p][batch_pass_class(p, n0, n1)] += batch_item_cap<T>(p, n0, n1);
  }
}

BatchLayout batch_layout(const gp_params* arr, int count) {
  BatchLayout B{};
  const bool fp64 = arr[0].prec == GP_FP64;
  const size_t dsz = fp64 ? sizeof(BDesc<double>) : sizeof(BDesc<float>);
  int cap[BP_COUNT][kBatchClasses];
  if (fp64) batch_caps<double>(arr, count, cap);
  else batch_caps<float>(arr, count, cap);
  B.total_items = 0;
  for (int p = 0; p < BP_COUNT; ++p)
    for (int k = 0; k < kBatchClasses; ++k) B.total_items += cap[p][k];
  size_t o = 0;
  B.o_desc = o;
  o += align_up(dsz * count);
  B.o_work = o;
  o += align_up(sizeof(WorkItem) * (size_t)B.total_items);
  for (int i = 0; i < count; ++i) {
    B.o_inst.push_back(o);
    o += align_up(make_layout(&arr[i]).total);
  }
  B.total = o;
  return B;
}

void batch_drop_graphs(gp_batch* b) {
  for (auto& g : b->gexec) {
    if (g) hipGraphExecDestroy(g);
    g = nullptr;
  }
}

// Per-instance descriptors (pointers into the instance workspaces, step scalars and
// couplings); rewritten when an instance's couplings change.
template <typename T>
gp_status batch_write_desc(gp_batch* b) {
  std::vector<BDesc<T>> D(b->count);
  b->cpl.assign(2 * (size_t)b->count, 0.0);
  for (int i = 0; i < b->count; ++i) {
    gp_ctx* c = b->inst[i];
    const Layout& L = c->L;
    BDesc<T>& d = D[i];
    // byte offsets from the batch workspace base
    const size_t o = (size_t)(c->ws - b->ws);
    d.psi = o + L.o_psi;
    d.V = o + L.o_V;
    d.spec = o + L.o_spec;
    d.ktab = o + L.o_ktab;
    d.tw0 = o + L.o_tw[0];
    d.tw1 = o + L.o_tw[1];
    d.cn0[0] = o + L.o_cn[0][0];
    d.cn0[1] = o + L.o_cn[0][1];
    d.cn1[0] = o + L.o_cn[1][0];
    d.cn1[1] = o + L.o_cn[1][1];
    d.p_x = o + L.o_px[0];
    d.p_nl = o + L.o_pnl;
    d.p_col = o + L.o_pcol;
    d.scale = o + L.o_scalars + offsetof(Scalars, scale);
    d.sc = step_scalars(c);
    d.n0 = L.n0;
    d.n1 = L.n1;
    d.fa = fin_args(c, 0);
    d.fa.nstage = 0;  // the per-instance finalize blocks read their partials directly
    // partial sums written by the batch passes: one slot per tile of the shape in use
    // (the instance workspace holds slots for the largest tile count of any shape)
    const int cx = batch_class(L.n0), cy = batch_class(L.n1);
    d.fa.nb_x = batch_tiles<T>(BP_R2C, L.n0, L.n1, b->shape[BP_R2C][cx]);
    d.fa.nb_nl = batch_tiles<T>(BP_C2R, L.n0, L.n1, b->shape[BP_C2R][cx]);
    d.fa.nb_col = batch_tiles<T>(BP_CN, L.n0, L.n1, b->shape[BP_CN][cy]);
    b->cpl[2 * i] = c->p.g;
    b->cpl[2 * i + 1] = c->p.gdd;
  }
  GP_HIP(hipMemcpyAsync(b->desc, D.data(), sizeof(BDesc<T>) * b->count, hipMemcpyHostToDevice,
                        b->st));
  return dev(hipStreamSynchronize(b->st));
}

// Work lists per (pass, class) for the current shape variants (instances by decreasing
// size, then their tiles), the dynamic LDS of each launch, and the descriptors.  Called
// at set-up and after a shape change, never inside a capture.
template <typename T>
gp_status batch_build(gp_batch* b) {
  GP_TRY(batch_write_desc<T>(b));
  std::vector<int> n0(b->count), n1(b->count);
  for (int i = 0; i < b->count; ++i) {
    n0[i] = b->inst[i]->L.n0;
    n1[i] = b->inst[i]->L.n1;
  }
  std::vector<int> order(b->count);
  for (int i = 0; i < b->count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return (size_t)n0[x] * n1[x] > (size_t)n0[y] * n1[y];
  });
  std::vector<WorkItem> lists[BP_COUNT][kBatchClasses];
  for (int p = 0; p < BP_COUNT; ++p)
    for (int k = 0; k < kBatchClasses; ++k)
      for (int m = 0; m < 3; ++m) b->lds[p][k][m] = 0;
  const int modes[3] = {MODE_IMAG, MODE_REAL, MODE_OBSERVE};
  for (int i : order) {
    for (int p = 0; p < BP_COUNT; ++p) {
      const int k = batch_pass_class(p, n0[i], n1[i]);
      const int sh = b->shape[p][k];
      const int nt = batch_tiles<T>(p, n0[i], n1[i], sh);
      for (int t = 0; t < nt; ++t) lists[p][k].push_back({i, t});
      const int n = (p == BP_R2C || p == BP_C2R) ? n0[i] : n1[i];
      for (int m = 0; m < 3; ++m)
        b->lds[p][k][m] = std::max(b->lds[p][k][m], batch_lds<T>(p, n, modes[m], sh));
    }
  }
  int cap[BP_COUNT][kBatchClasses];
  batch_caps<T>(b->params.data(), b->count, cap);
  size_t off = 0;
  for (int p = 0; p < BP_COUNT; ++p) {
    for (int k = 0; k < kBatchClasses; ++k) {
      if ((int)lists[p][k].size() > cap[p][k]) return GP_E_ARG;  // cannot happen
      b->work[p][k] = b->work_base + off;
      b->nwork[p][k] = (int)lists[p][k].size();
      const int req = b->grid_req[p][k];
      b->grid[p][k] = std::min(b->nwork[p][k], req > 0 ? req : kBatchDefaultGrid);
      if (!lists[p][k].empty())
        GP_HIP(hipMemcpyAsync(b->work[p][k], lists[p][k].data(),
                              sizeof(WorkItem) * lists[p][k].size(), hipMemcpyHostToDevice,
                              b->st));
      off += cap[p][k];
      for (int m = 0; m < 3; ++m)
        if (b->lds[p][k][m] > 0)
          GP_HIP(batch_reserve_lds<T>(p, m, k, b->shape[p][k], b->lds[p][k][m]));
    }
  }
  GP_HIP(hipStreamSynchronize(b->st));
  return GP_OK;
}

template <typename T>
gp_status batch_step(gp_batch* b, hipStream_t st, bool imag) {
  const int mode = imag ? MODE_IMAG : MODE_REAL;
  const int mi = imag ? 0 : 1;
  const BDesc<T>* D = reinterpret_cast<const BDesc<T>*>(b->desc);
  const int passes[4] = {BP_R2C, BP_CONV, BP_C2R, BP_CN};
  for (int p : passes) {
    // an instance's class can differ between passes (x length vs y length), so the two
    // classes of one pass run side by side and the pass ends with both joined
    const bool two =
        b->two_streams && b->side != nullptr && b->nwork[p][0] > 0 && b->nwork[p][1] > 0;
    if (two) {
      GP_HIP(hipEventRecord(b->ev_fork, st));
      GP_HIP(hipStreamWaitEvent(b->side, b->ev_fork, 0));
    }
    for (int k = 0; k < kBatchClasses; ++k) {
      const hipStream_t sk = (two && k == 1) ? b->side : st;
      GP_HIP(batch_launch<T>(p, mode, k, b->shape[p][k], b->grid[p][k], b->lds[p][k][mi], sk,
                             b->ws, D, b->work[p][k], b->nwork[p][k]));
    }
    if (two) {
      GP_HIP(hipEventRecord(b->ev_join, b->side));
      GP_HIP(hipStreamWaitEvent(st, b->ev_join, 0));
    }
  }
  return dev(batch_finalize<T>(b->count, imag ? (int)FIN_IMAG : (int)FIN_REAL, st, D));
}

gp_status batch_one_step(gp_batch* b, hipStream_t st, bool imag) {
  return b->fp64 ? batch_step<double>(b, st, imag) : batch_step<float>(b, st, imag);
}

gp_status batch_build_graph(gp_batch* b, bool imag) {
  if (!b->cap_st) GP_HIP(hipStreamCreateWithFlags(&b->cap_st, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  gp_status s = dev(hipStreamBeginCapture(b->cap_st, hipStreamCaptureModeThreadLocal));
  if (s == GP_OK) {
    for (int i = 0; i < kGraphSteps && s == GP_OK; ++i) s = batch_one_step(b, b->cap_st, imag);
    const gp_status e = dev(hipStreamEndCapture(b->cap_st, &g));
    if (s == GP_OK) s = e;
  }
  if (s != GP_OK) {
    if (g) hipGraphDestroy(g);
    return s;
  }
  hipGraphExec_t ex = nullptr;
  s = dev(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
  hipGraphDestroy(g);
  if (s != GP_OK) return s;
  b->gexec[imag ? 0 : 1] = ex;
  return GP_OK;
}

gp_status batch_run(gp_batch* b, int nsteps, bool imag) {
  if (!b || nsteps < 0) return GP_E_ARG;
  clear_stale_error();
  bool stale = false;
  for (int i = 0; i < b->count; ++i) {
    const gp_ctx* c = b->inst[i];
    if (!c->psi_set) return GP_E_STATE;
    stale |= c->p.g != b->cpl[2 * i] || c->p.gdd != b->cpl[2 * i + 1];
  }
  if (stale) {  // gp_set_couplings on an instance context since the descriptors were written
    batch_drop_graphs(b);
    GP_TRY(b->fp64 ? batch_write_desc<double>(b) : batch_write_desc<float>(b));
  }
  // An instance context stepped on its own (gp_step_imag/real on it) may hold a deferred
  // finalisation: complete it, so its scale and record are current before the batch
  // kernels read them, and return its x-partial selection to buffer 0, which the batch
  // descriptors name.
  for (int i = 0; i < b->count; ++i) {
    gp_ctx* c = b->inst[i];
    GP_TRY(settle(c));
    c->px_sel = 0;
    c->pend_sel = 0;
  }
  int done = 0;
  if (b->use_graphs && nsteps >= kGraphSteps) {
    const int gi = imag ? 0 : 1;
    if (!b->gexec[gi]) GP_TRY(batch_build_graph(b, imag));
    for (; nsteps - done >= kGraphSteps; done += kGraphSteps)
      GP_HIP(hipGraphLaunch(b->gexec[gi], b->st));
  }
  for (; done < nsteps; ++done) GP_TRY(batch_one_step(b, b->st, imag));
  return GP_OK;
}

}  // namespace

extern "C" {

gp_status gp_workspace_bytes(const gp_params* params, size_t* bytes) {
  if (!bytes) return GP_E_ARG;
  GP_TRY(validate(params));
  *bytes = make_layout(params).total;
  return GP_OK;
}

gp_status gp_workspace_bytes_ex(const gp_params* params, unsigned host, size_t* bytes) {
  if (!bytes || (host & ~(GP_HOST_V | GP_HOST_KTAB))) return GP_E_ARG;
  GP_TRY(validate(params));
  *bytes = make_layout(params, host).total;
  return GP_OK;
}

gp_status gp_host_bytes(const gp_params* params, size_t* v_bytes, size_t* ktab_bytes) {
  if (!v_bytes || !ktab_bytes) return GP_E_ARG;
  GP_TRY(validate(params));
  const Layout L = make_layout(params);
  *v_bytes = L.esz * L.npts;
  *ktab_bytes = L.esz * L.nktab;
  return GP_OK;
}

gp_status gp_init_ex(const gp_params* params, unsigned host, void* dev_workspace,
                     size_t ws_bytes, void* host_v, void* host_ktab, void* hip_stream,
                     gp_ctx** out) {
  clear_stale_error();
  if (!out || !dev_workspace || (host & ~(GP_HOST_V | GP_HOST_KTAB))) return GP_E_ARG;
  *out = nullptr;
  GP_TRY(validate(params));
  const Layout L = make_layout(params, host);
  if (ws_bytes < L.total) return GP_E_ARG;
  if ((reinterpret_cast<uintptr_t>(dev_workspace) & 255) != 0) return GP_E_ARG;
  // host-resident arrays: pinned host memory, mapped into the device's address space
  void* maps[2] = {nullptr, nullptr};
  void* const hp[2] = {host_v, host_ktab};
  const unsigned fl[2] = {GP_HOST_V, GP_HOST_KTAB};
  for (int k = 0; k < 2; ++k) {
    if (!(host & fl[k])) continue;
    if (!hp[k] || (reinterpret_cast<uintptr_t>(hp[k]) & 15) != 0) return GP_E_ARG;
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, hp[k]) != hipSuccess || at.type != hipMemoryTypeHost) {
      clear_stale_error();
      snprintf(g_last_error, sizeof(g_last_error),
               "host array %d is not pinned host memory (hipHostMalloc)", k);
      return GP_E_ARG;
    }
    GP_HIP(hipHostGetDevicePointer(&maps[k], hp[k], 0));
  }
  gp_ctx* c = new (std::nothrow) gp_ctx();
  if (!c) return GP_E_NOMEM;
  c->p = *params;
  c->L = L;
  c->st = reinterpret_cast<hipStream_t>(hip_stream);
  c->ws = reinterpret_cast<char*>(dev_workspace);
  c->fp64 = params->prec == GP_FP64;
  c->psi_set = false;
  c->ekz_valid = false;
  c->gc = contact(c->p);
  c->hostV = reinterpret_cast<char*>(maps[0]);
  c->hostK = reinterpret_cast<char*>(maps[1]);
  int devid = 0;
  if (hipGetDevice(&devid) != hipSuccess ||
      hipDeviceGetAttribute(&c->clock_khz, hipDeviceAttributeWallClockRate, devid) != hipSuccess)
    c->clock_khz = 0;
  clear_stale_error();
  gp_status s = c->fp64 ? Passes<double>::init_tables(c) : Passes<float>::init_tables(c);
  // the tables written through a host mapping are complete before the call returns
  if (s == GP_OK && host) s = dev(hipStreamSynchronize(c->st));
  if (s != GP_OK) {
    delete c;
    return s;
  }
  *out = c;
  return GP_OK;
}

gp_status gp_init(const gp_params* params, void* dev_workspace, size_t ws_bytes, void* hip_stream,
                  gp_ctx** out) {
  return gp_init_ex(params, 0u, dev_workspace, ws_bytes, nullptr, nullptr, hip_stream, out);
}

gp_status gp_destroy(gp_ctx* ctx) {
  if (!ctx) return GP_E_ARG;
  const hipError_t e = hipStreamSynchronize(ctx->st);
  for (int k = 0; k < GP_PASS_COUNT; ++k) {
    for (auto& ev : ctx->tev[k]) {
      hipEventDestroy(ev.first);
      hipEventDestroy(ev.second);
    }
  }
  for (auto ev : ctx->tpool) hipEventDestroy(ev);
  drop_graphs(ctx);
  if (ctx->cap_st) hipStreamDestroy(ctx->cap_st);
  delete ctx;
  return dev(e);
}

const char* gp_status_string(gp_status s) {
  switch (s) {
    case GP_OK: return "ok";
    case GP_E_ARG: return "invalid argument";
    case GP_E_SIZE: return "unsupported grid size (an axis < 4, an FFT line longer than 8192 FP32 / 4096 FP64 points in 3D, or a longer 2D axis with no four-step split)";
    case GP_E_DEVICE: return "HIP runtime error";
    case GP_E_NONFINITE: return "wave function became non-finite";
    case GP_E_STATE: return "call out of order (set psi first)";
    case GP_E_NOMEM: return "host allocation failed";
    case GP_E_IO: return "state file could not be written or read, or is not a state file";
    default: return "unknown status";
  }
}

gp_status gp_set_psi(gp_ctx* c, const void* psi, int on_device) {
  clear_stale_error();
  if (!c || !psi) return GP_E_ARG;
  GP_TRY(settle(c));
  GP_TRY(c->fp64 ? Passes<double>::set_psi(c, psi, on_device)
                 : Passes<float>::set_psi(c, psi, on_device));
  c->psi_set = true;
  c->ekz_valid = false;
  // nothing is outstanding after settle(): restart the x-partial double buffer, so that
  // a step loop after a new state always starts from the same buffer (and replays the
  // same captured graph)
  c->px_sel = 0;
  c->pend_sel = 0;
  return GP_OK;
}

gp_status gp_get_psi(gp_ctx* c, void* psi, int on_device) {
  clear_stale_error();
  if (!c || !psi) return GP_E_ARG;
  if (!c->psi_set) return GP_E_STATE;
  GP_TRY(settle(c));
  GP_TRY(c->fp64 ? Passes<double>::get_psi(c, psi, on_device)
                 : Passes<float>::get_psi(c, psi, on_device));
  return on_device ? GP_OK : check_flags(c);
}

gp_status gp_set_potential(gp_ctx* c, const void* V, int on_device) {
  clear_stale_error();
  if (!c || !V) return GP_E_ARG;
  GP_TRY(settle(c));
  return c->fp64 ? Passes<double>::set_potential(c, V, on_device)
                 : Passes<float>::set_potential(c, V, on_device);
}

gp_status gp_set_couplings(gp_ctx* c, double g, double gdd) {
  if (!c || !isfinite(g) || !isfinite(gdd)) return GP_E_ARG;
  GP_TRY(settle(c));
  c->p.g = g;
  c->p.gdd = gdd;
  c->gc = contact(c->p);
  drop_graphs(c);  // the couplings are launch arguments of the captured kernels
  return GP_OK;
}

gp_status gp_step_imag(gp_ctx* c, int nsteps) { return run_steps(c, nsteps, true); }

gp_status gp_step_real_adjoint(gp_ctx* c, const void* psi_n, void* lam, double* gradV,
                               double* grad_g, double* grad_gdd) {
  if (!c || !psi_n || !lam || !gradV || !grad_g || !grad_gdd) return GP_E_ARG;
  clear_stale_error();
  GP_TRY(settle(c));
  if (c->fp64) {
    return Passes<double>::adjoint(c, reinterpret_cast<const cpx<double>*>(psi_n),
                                   reinterpret_cast<cpx<double>*>(lam), gradV, grad_g, grad_gdd);
  }
  return Passes<float>::adjoint(c, reinterpret_cast<const cpx<float>*>(psi_n),
                                reinterpret_cast<cpx<float>*>(lam), gradV, grad_g, grad_gdd);
}
gp_status gp_step_real(gp_ctx* c, int nsteps) { return run_steps(c, nsteps, false); }

gp_status gp_energy(gp_ctx* c, gp_observables* out) {
  clear_stale_error();
  if (!c || !out) return GP_E_ARG;
  if (!c->psi_set) return GP_E_STATE;
  GP_TRY(settle(c));
  GP_TRY(c->fp64 ? Passes<double>::observe(c) : Passes<float>::observe(c));
  double rec[kRecord];
  GP_HIP(hipMemcpyAsync(rec, c->at<double>(c->L.o_obs), sizeof(rec), hipMemcpyDeviceToHost, c->st));
  GP_HIP(hipStreamSynchronize(c->st));
  out->norm = rec[0];
  out->mu = rec[1];
  out->energy = rec[2];
  out->e_kin = rec[3];
  out->e_pot = rec[4];
  out->e_int = rec[5];
  out->e_dd = rec[6];
  out->rms[0] = rec[7];
  out->rms[1] = rec[8];
  out->rms[2] = rec[9];
  return check_flags(c);
}

gp_status gp_dipolar_potential(gp_ctx* c, void* phi, int on_device) {
  clear_stale_error();
  if (!c || !phi) return GP_E_ARG;
  if (!c->psi_set) return GP_E_STATE;
  GP_TRY(settle(c));
  return c->fp64 ? Passes<double>::dipolar(c, phi, on_device)
                 : Passes<float>::dipolar(c, phi, on_device);
}

int gp_history_capacity(void) { return kRingCap; }

const char* gp_last_error(void) { return g_last_error; }

gp_status gp_use_graphs(gp_ctx* c, int enable) {
  if (!c) return GP_E_ARG;
  c->use_graphs = enable != 0;
  return GP_OK;
}

gp_status gp_timing_enable(gp_ctx* c, unsigned mask) {
  if (!c) return GP_E_ARG;
  clear_stale_error();
  GP_TRY(settle(c));
  GP_HIP(hipStreamSynchronize(c->st));
  for (int k = 0; k < GP_PASS_COUNT; ++k) {
    for (auto& e : c->tev[k]) {
      c->tpool.push_back(e.first);
      c->tpool.push_back(e.second);
    }
    c->tev[k].clear();
  }
  c->tmask = mask & ((1u << GP_PASS_COUNT) - 1);
  hipLaunchKernelGGL(k_clear_u64, dim3(1), dim3(64), 0, c->st, c->sc()->span, 2);
  return dev(hipGetLastError());
}

gp_status gp_timing_span(gp_ctx* c, int pass, double* total_ms, int* launches) {
  if (!c || !total_ms || !launches) return GP_E_ARG;
  if (pass != GP_PASS_C2R_NL_CNX) return GP_E_ARG;
  clear_stale_error();
  GP_TRY(settle(c));
  unsigned long long acc[2] = {0ull, 0ull};
  GP_HIP(hipMemcpyAsync(acc, c->sc()->span, sizeof(acc), hipMemcpyDeviceToHost, c->st));
  GP_HIP(hipStreamSynchronize(c->st));
  *total_ms = c->clock_khz > 0 ? (double)acc[0] / (double)c->clock_khz : 0.0;
  *launches = (int)acc[1];
  return GP_OK;
}

gp_status gp_timing_read(gp_ctx* c, double* total_ms, int* launches) {
  if (!c || !total_ms || !launches) return GP_E_ARG;
  clear_stale_error();
  GP_TRY(settle(c));
  GP_HIP(hipStreamSynchronize(c->st));
  for (int k = 0; k < GP_PASS_COUNT; ++k) {
    double acc = 0.0;
    for (auto& e : c->tev[k]) {
      float ms = 0.f;
      GP_HIP(hipEventElapsedTime(&ms, e.first, e.second));
      acc += ms;
    }
    total_ms[k] = acc;
    launches[k] = (int)c->tev[k].size();
  }
  return GP_OK;
}

gp_status gp_timing_burst(gp_ctx* c, int pass, int reps, double* ms_per_launch) {
  clear_stale_error();
  if (!c || !ms_per_launch || reps < 1 || reps > 4096) return GP_E_ARG;
  if (!c->psi_set) return GP_E_STATE;
  GP_TRY(settle(c));
  if (pass != GP_PASS_R2C_X && pass != GP_PASS_C2R_NL_CNX && pass != GP_PASS_CN_Y &&
      pass != GP_PASS_CN_Z)
    return GP_E_ARG;
  if (pass == GP_PASS_CN_Z && c->p.geom != GP_3D) return GP_E_ARG;
  if (!c->cap_st) GP_HIP(hipStreamCreateWithFlags(&c->cap_st, hipStreamNonBlocking));
  GP_HIP(hipStreamSynchronize(c->st));
  const hipStream_t user = c->st;
  c->st = c->cap_st;
  hipGraph_t g = nullptr;
  gp_status s = dev(hipStreamBeginCapture(c->cap_st, hipStreamCaptureModeThreadLocal));
  if (s == GP_OK) {
    for (int i = 0; i < reps && s == GP_OK; ++i)
      s = c->fp64 ? Passes<double>::launch_pass(c, pass) : Passes<float>::launch_pass(c, pass);
    const gp_status e = dev(hipStreamEndCapture(c->cap_st, &g));
    if (s == GP_OK) s = e;
  }
  c->st = user;
  if (s != GP_OK) {
    if (g) hipGraphDestroy(g);
    return s;
  }
  hipGraphExec_t ex = nullptr;
  s = dev(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
  hipGraphDestroy(g);
  if (s != GP_OK) return s;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float ms = 0.f;
  s = dev(hipEventCreate(&e0));
  if (s == GP_OK) s = dev(hipEventCreate(&e1));
  if (s == GP_OK) s = dev(hipGraphLaunch(ex, c->st));  // warm-up
  if (s == GP_OK) s = dev(hipEventRecord(e0, c->st));
  if (s == GP_OK) s = dev(hipGraphLaunch(ex, c->st));
  if (s == GP_OK) s = dev(hipEventRecord(e1, c->st));
  if (s == GP_OK) s = dev(hipEventSynchronize(e1));
  if (s == GP_OK) s = dev(hipEventElapsedTime(&ms, e0, e1));
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipGraphExecDestroy(ex);
  if (s != GP_OK) return s;
  *ms_per_launch = (double)ms / reps;
  c->ekz_valid = false;  // the stored state was advanced by partial steps
  return GP_OK;
}

gp_status gp_history(gp_ctx* c, gp_observables* out, int max_records, int* count) {
  clear_stale_error();
  if (!c || !count || max_records < 0 || (max_records > 0 && !out)) return GP_E_ARG;
  GP_TRY(settle(c));
  int pos = 0;
  GP_HIP(hipMemcpyAsync(&pos, &c->sc()->ring_pos, sizeof(int), hipMemcpyDeviceToHost, c->st));
  GP_HIP(hipStreamSynchronize(c->st));
  int avail = pos < kRingCap ? pos : kRingCap;
  int n = avail < max_records ? avail : max_records;
  if (n > 0) {
    double* ring = new (std::nothrow) double[(size_t)kRecord * kRingCap];
    if (!ring) return GP_E_NOMEM;
    const hipError_t e = hipMemcpyAsync(ring, c->at<double>(c->L.o_ring),
                                        sizeof(double) * kRecord * kRingCap,
                                        hipMemcpyDeviceToHost, c->st);
    const hipError_t e2 = (e == hipSuccess) ? hipStreamSynchronize(c->st) : e;
    if (e2 != hipSuccess) {
      delete[] ring;
      return GP_E_DEVICE;
    }
    for (int r = 0; r < n; ++r) {
      const double* rec = ring + (size_t)((pos - n + r) % kRingCap) * kRecord;
      out[r].norm = rec[0];
      out[r].mu = rec[1];
      out[r].energy = rec[2];
      out[r].e_kin = rec[3];
      out[r].e_pot = rec[4];
      out[r].e_int = rec[5];
      out[r].e_dd = rec[6];
      out[r].rms[0] = rec[7];
      out[r].rms[1] = rec[8];
      out[r].rms[2] = rec[9];
    }
    delete[] ring;
  }
  *count = n;
  return check_flags(c);
}

gp_status gp_batch_workspace_bytes(const gp_params* params, int count, size_t* bytes) {
  if (!bytes) return GP_E_ARG;
  GP_TRY(batch_validate(params, count));
  *bytes = batch_layout(params, count).total;
  return GP_OK;
}

gp_status gp_batch_init(const gp_params* params, int count, void* dev_workspace, size_t ws_bytes,
                        void* hip_stream, gp_batch** out) {
  if (!out || !dev_workspace) return GP_E_ARG;
  *out = nullptr;
  clear_stale_error();
  GP_TRY(batch_validate(params, count));
  const BatchLayout BL = batch_layout(params, count);
  if (ws_bytes < BL.total) return GP_E_ARG;
  if ((reinterpret_cast<uintptr_t>(dev_workspace) & 255) != 0) return GP_E_ARG;
  gp_batch* b = new (std::nothrow) gp_batch();
  if (!b) return GP_E_NOMEM;
  b->count = count;
  b->fp64 = params[0].prec == GP_FP64;
  b->st = reinterpret_cast<hipStream_t>(hip_stream);
  b->ws = reinterpret_cast<char*>(dev_workspace);
  b->desc = b->ws + BL.o_desc;
  b->params.assign(params, params + count);
  gp_status s = GP_OK;
  for (int i = 0; i < count && s == GP_OK; ++i) {
    gp_ctx* c = nullptr;
    s = gp_init(&params[i], b->ws + BL.o_inst[i], make_layout(&params[i]).total, hip_stream, &c);
    if (s == GP_OK) b->inst.push_back(c);
  }
  b->work_base = reinterpret_cast<WorkItem*>(b->ws + BL.o_work);
  if (s == GP_OK) s = b->fp64 ? batch_build<double>(b) : batch_build<float>(b);
  if (s == GP_OK) s = dev(hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking));
  if (s == GP_OK) s = dev(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
  if (s == GP_OK) s = dev(hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming));
  if (s != GP_OK) {
    gp_batch_destroy(b);
    return s;
  }
  *out = b;
  return GP_OK;
}

gp_status gp_batch_destroy(gp_batch* b) {
  if (!b) return GP_E_ARG;
  const hipError_t e = hipStreamSynchronize(b->st);
  if (b->side) hipStreamSynchronize(b->side);
  batch_drop_graphs(b);
  if (b->cap_st) hipStreamDestroy(b->cap_st);
  if (b->side) hipStreamDestroy(b->side);
  if (b->ev_fork) hipEventDestroy(b->ev_fork);
  if (b->ev_join) hipEventDestroy(b->ev_join);
  for (gp_ctx* c : b->inst) gp_destroy(c);
  delete b;
  return dev(e);
}

gp_ctx* gp_batch_context(gp_batch* b, int idx) {
  if (!b || idx < 0 || idx >= b->count) return nullptr;
  return b->inst[idx];
}

gp_status gp_batch_step_imag(gp_batch* b, int nsteps) { return batch_run(b, nsteps, true); }
gp_status gp_batch_step_real(gp_batch* b, int nsteps) { return batch_run(b, nsteps, false); }

gp_status gp_batch_energy(gp_batch* b, gp_observables* out) {
  if (!b || !out) return GP_E_ARG;
  for (int i = 0; i < b->count; ++i) GP_TRY(gp_energy(b->inst[i], &out[i]));
  return GP_OK;
}

gp_status gp_batch_plan(gp_batch* b, int* items, int* blocks) {
  if (!b || !items || !blocks) return GP_E_ARG;
  for (int p = 0; p < BP_COUNT; ++p)
    for (int k = 0; k < kBatchClasses; ++k) {
      items[p * kBatchClasses + k] = b->nwork[p][k];
      blocks[p * kBatchClasses + k] = b->grid[p][k];
    }
  return GP_OK;
}

gp_status gp_batch_set_blocks(gp_batch* b, int pass, int size_class, int blocks) {
  if (!b || pass < 0 || pass >= BP_COUNT || size_class < 0 || size_class >= kBatchClasses)
    return GP_E_ARG;
  const int n = b->nwork[pass][size_class];
  b->grid_req[pass][size_class] = blocks <= 0 ? 0 : blocks;
  b->grid[pass][size_class] = blocks <= 0 ? std::min(n, kBatchDefaultGrid) : std::min(blocks, n);
  batch_drop_graphs(b);  // the grid sizes are captured launch parameters
  return GP_OK;
}

gp_status gp_batch_set_shape(gp_batch* b, int pass, int size_class, int shape) {
  if (!b || pass < 0 || pass >= BP_COUNT || size_class < 0 || size_class >= kBatchClasses ||
      shape < 0 || shape >= kBatchShapes)
    return GP_E_ARG;
  clear_stale_error();
  if (b->shape[pass][size_class] == shape) return GP_OK;
  // the batch's partial sums of the previous shape must be consumed first
  for (gp_ctx* c : b->inst) GP_TRY(settle(c));
  GP_HIP(hipStreamSynchronize(b->st));
  b->shape[pass][size_class] = shape;
  batch_drop_graphs(b);
  return b->fp64 ? batch_build<double>(b) : batch_build<float>(b);
}

gp_status gp_batch_shapes(gp_batch* b, int* shapes) {
  if (!b || !shapes) return GP_E_ARG;
  for (int p = 0; p < BP_COUNT; ++p)
    for (int k = 0; k < kBatchClasses; ++k) shapes[p * kBatchClasses + k] = b->shape[p][k];
  return GP_OK;
}

gp_status gp_batch_use_graphs(gp_batch* b, int enable) {
  if (!b) return GP_E_ARG;
  b->use_graphs = enable != 0;
  return GP_OK;
}

gp_status gp_batch_use_streams(gp_batch* b, int enable) {
  if (!b) return GP_E_ARG;
  if (b->two_streams != (enable != 0)) batch_drop_graphs(b);  // a different graph shape
  b->two_streams = enable != 0;
  return GP_OK;
}

gp_status gp_batch_set_psi(gp_batch* b, int idx, const void* psi, int on_device) {
  if (!b || idx < 0 || idx >= b->count) return GP_E_ARG;
  return gp_set_psi(b->inst[idx], psi, on_device);
}

gp_status gp_batch_get_psi(gp_batch* b, int idx, void* psi, int on_device) {
  if (!b || idx < 0 || idx >= b->count) return GP_E_ARG;
  return gp_get_psi(b->inst[idx], psi, on_device);
}

int gp_axis_kind(int n, int prec) {
  if (prec != GP_FP64 && prec != GP_FP32_MIXED) return 0;
  if (fast_size(n)) return 1;
  if (size_ok(n, prec == GP_FP64)) return 2;
  return long_size(n, prec == GP_FP64) ? 3 : 0;
}

gp_status gp_get_params(gp_ctx* c, gp_params* out) {
  if (!c || !out) return GP_E_ARG;
  *out = c->p;
  return GP_OK;
}

gp_status gp_sync(gp_ctx* c) {
  clear_stale_error();
  if (!c) return GP_E_ARG;
  GP_TRY(settle(c));
  return check_flags(c);
}

gp_status gp_dipolar_potential_noalloc(const gp_params* params, const void* psi, void* phi,
                                       void* hip_stream) {
  clear_stale_error();
  g_last_error[0] = '\0';
  if (!params || !psi || !phi) return GP_E_ARG;
  GP_TRY(validate(params));
  return dipolar_noalloc(params, psi, phi, reinterpret_cast<hipStream_t>(hip_stream));
}

}  // extern "C"
