// Saved states and output cadence around the step loop (host code over the public C ABI).
//
// The paper's programs hand a stationary state from the imaginary-time run to the
// real-time run through a file (program summaries of the real-time programs: with no
// imaginary-time steps of its own, a run reads the output of an imaginary-time run), and
// they write the chemical potential, energy, rms sizes and density profiles at chosen
// steps (calcmuen, calcrms; "Summary of revisions": only the wave function returns to
// the host, for output).  The file layout is not given there; this one is the library's
// own and is documented with the declarations in gp.h.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <vector>

#include "../../include/gp.h"

namespace {

constexpr char kMagic[8] = {'G', 'P', 'D', 'B', 'E', 'C', 'S', '1'};
constexpr uint32_t kVersion = 1;
constexpr size_t kHeaderBytes = 256;

static_assert(sizeof(double) == 8 && sizeof(int32_t) == 4, "fixed-width header fields");

// FNV-1a over the payload bytes (64-bit variant: offset basis 0xcbf29ce484222325, prime
// 0x100000001b3).
struct Fnv {
  uint64_t h = 0xcbf29ce484222325ull;
  void add(const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
      h ^= b[i];
      h *= 0x100000001b3ull;
    }
  }
};

// Header fields at fixed byte offsets (little-endian host).
struct HeaderView {
  unsigned char* b;
  template <typename X>
  void put(size_t off, X v) { memcpy(b + off, &v, sizeof(X)); }
  template <typename X>
  X get(size_t off) const {
    X v;
    memcpy(&v, b + off, sizeof(X));
    return v;
  }
};

enum : size_t {
  H_MAGIC = 0, H_VERSION = 8, H_KIND = 12, H_GEOM = 16, H_NX = 20, H_NY = 24, H_NZ = 28,
  H_DX = 32, H_DY = 40, H_DZ = 48, H_DT = 56, H_GAMMA = 64, H_NU = 72, H_LAMBDA = 80,
  H_G = 88, H_GDD = 96, H_R = 104, H_PREC = 112, H_STEP = 120, H_TIME = 128,
  H_NPOINTS = 136, H_CHECKSUM = 144
};

size_t plane_points(const gp_params& p) {
  if (p.geom == GP_3D) return (size_t)p.nx * p.ny * p.nz;
  return (size_t)p.nx * (p.geom == GP_2D_XY ? p.ny : p.nz);
}

void encode(unsigned char* b, int kind, const gp_params& p, long long step, double time,
            uint64_t npoints, uint64_t checksum) {
  memset(b, 0, kHeaderBytes);
  HeaderView h{b};
  memcpy(b + H_MAGIC, kMagic, sizeof(kMagic));
  h.put<uint32_t>(H_VERSION, kVersion);
  h.put<uint32_t>(H_KIND, (uint32_t)kind);
  h.put<int32_t>(H_GEOM, p.geom);
  h.put<int32_t>(H_NX, p.nx);
  h.put<int32_t>(H_NY, p.ny);
  h.put<int32_t>(H_NZ, p.nz);
  h.put<double>(H_DX, p.dx);
  h.put<double>(H_DY, p.dy);
  h.put<double>(H_DZ, p.dz);
  h.put<double>(H_DT, p.dt);
  h.put<double>(H_GAMMA, p.gamma);
  h.put<double>(H_NU, p.nu);
  h.put<double>(H_LAMBDA, p.lambda);
  h.put<double>(H_G, p.g);
  h.put<double>(H_GDD, p.gdd);
  h.put<double>(H_R, p.cutoff_R);
  h.put<int32_t>(H_PREC, p.prec);
  h.put<int64_t>(H_STEP, (int64_t)step);
  h.put<double>(H_TIME, time);
  h.put<uint64_t>(H_NPOINTS, npoints);
  h.put<uint64_t>(H_CHECKSUM, checksum);
}

gp_status decode(const unsigned char* b, gp_state_info* out) {
  if (memcmp(b + H_MAGIC, kMagic, sizeof(kMagic)) != 0) return GP_E_IO;
  HeaderView h{const_cast<unsigned char*>(b)};
  if (h.get<uint32_t>(H_VERSION) != kVersion) return GP_E_IO;
  const uint32_t kind = h.get<uint32_t>(H_KIND);
  if (kind != GP_STATE_PSI && kind != GP_STATE_DENSITY) return GP_E_IO;
  gp_state_info s;
  memset(&s, 0, sizeof(s));
  s.kind = (int)kind;
  gp_params& p = s.params;
  p.geom = h.get<int32_t>(H_GEOM);
  p.nx = h.get<int32_t>(H_NX);
  p.ny = h.get<int32_t>(H_NY);
  p.nz = h.get<int32_t>(H_NZ);
  p.dx = h.get<double>(H_DX);
  p.dy = h.get<double>(H_DY);
  p.dz = h.get<double>(H_DZ);
  p.dt = h.get<double>(H_DT);
  p.gamma = h.get<double>(H_GAMMA);
  p.nu = h.get<double>(H_NU);
  p.lambda = h.get<double>(H_LAMBDA);
  p.g = h.get<double>(H_G);
  p.gdd = h.get<double>(H_GDD);
  p.cutoff_R = h.get<double>(H_R);
  p.prec = h.get<int32_t>(H_PREC);
  s.step = (long long)h.get<int64_t>(H_STEP);
  s.time = h.get<double>(H_TIME);
  s.npoints = h.get<uint64_t>(H_NPOINTS);
  s.checksum = h.get<uint64_t>(H_CHECKSUM);
  if (p.geom < GP_3D || p.geom > GP_2D_XZ || p.nx < 1 || p.ny < 1 || p.nz < 1) return GP_E_IO;
  if (s.npoints != (uint64_t)plane_points(p)) return GP_E_IO;
  *out = s;
  return GP_OK;
}

size_t value_doubles(int kind) { return kind == GP_STATE_PSI ? 2 : 1; }

gp_status write_file(const char* path, int kind, const gp_params& p, long long step,
                     double time, const double* data) {
  const size_t n = plane_points(p) * value_doubles(kind);
  Fnv f;
  f.add(data, n * sizeof(double));
  unsigned char hdr[kHeaderBytes];
  encode(hdr, kind, p, step, time, plane_points(p), f.h);
  FILE* fp = fopen(path, "wb");
  if (!fp) return GP_E_IO;
  bool ok = fwrite(hdr, 1, kHeaderBytes, fp) == kHeaderBytes;
  ok = ok && fwrite(data, sizeof(double), n, fp) == n;
  ok = (fclose(fp) == 0) && ok;
  if (!ok) remove(path);  // no partial state files
  return ok ? GP_OK : GP_E_IO;
}

bool same_grid(const gp_params& a, const gp_params& b) {
  auto close = [](double x, double y) { return fabs(x - y) <= 1e-12 * fmax(fabs(x), fabs(y)); };
  if (a.geom != b.geom || a.nx != b.nx) return false;
  if (!close(a.dx, b.dx)) return false;
  if (a.geom != GP_2D_XZ && (a.ny != b.ny || !close(a.dy, b.dy))) return false;
  if (a.geom != GP_2D_XY && (a.nz != b.nz || !close(a.dz, b.dz))) return false;
  return true;
}

}  // namespace

extern "C" {

gp_status gp_state_read_info(const char* path, gp_state_info* info) {
  if (!path || !info) return GP_E_ARG;
  FILE* fp = fopen(path, "rb");
  if (!fp) return GP_E_IO;
  unsigned char hdr[kHeaderBytes];
  const bool ok = fread(hdr, 1, kHeaderBytes, fp) == kHeaderBytes;
  fclose(fp);
  if (!ok) return GP_E_IO;
  return decode(hdr, info);
}

gp_status gp_state_read(const char* path, gp_state_info* info, double* data, size_t max_doubles) {
  if (!path || !info || !data) return GP_E_ARG;
  FILE* fp = fopen(path, "rb");
  if (!fp) return GP_E_IO;
  unsigned char hdr[kHeaderBytes];
  gp_status s = fread(hdr, 1, kHeaderBytes, fp) == kHeaderBytes ? decode(hdr, info) : GP_E_IO;
  if (s == GP_OK) {
    const size_t n = (size_t)info->npoints * value_doubles(info->kind);
    if (n > max_doubles) {
      s = GP_E_ARG;
    } else if (fread(data, sizeof(double), n, fp) != n || fgetc(fp) != EOF) {
      s = GP_E_IO;  // short payload, or bytes beyond it
    } else {
      Fnv f;
      f.add(data, n * sizeof(double));
      if (f.h != info->checksum) s = GP_E_IO;
    }
  }
  fclose(fp);
  return s;
}

gp_status gp_save_state(gp_ctx* ctx, const char* path, long long step, double time) {
  if (!ctx || !path) return GP_E_ARG;
  gp_params p;
  gp_status s = gp_get_params(ctx, &p);
  if (s != GP_OK) return s;
  std::vector<double> psi;
  try {
    psi.resize(2 * plane_points(p));
  } catch (const std::bad_alloc&) {
    return GP_E_NOMEM;
  }
  s = gp_get_psi(ctx, psi.data(), 0);
  if (s != GP_OK) return s;
  return write_file(path, GP_STATE_PSI, p, step, time, psi.data());
}

gp_status gp_save_density(gp_ctx* ctx, const char* path, long long step, double time) {
  if (!ctx || !path) return GP_E_ARG;
  gp_params p;
  gp_status s = gp_get_params(ctx, &p);
  if (s != GP_OK) return s;
  const size_t n = plane_points(p);
  std::vector<double> psi, den;
  try {
    psi.resize(2 * n);
    den.resize(n);
  } catch (const std::bad_alloc&) {
    return GP_E_NOMEM;
  }
  s = gp_get_psi(ctx, psi.data(), 0);
  if (s != GP_OK) return s;
  for (size_t i = 0; i < n; ++i) den[i] = psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];
  return write_file(path, GP_STATE_DENSITY, p, step, time, den.data());
}

gp_status gp_load_state(gp_ctx* ctx, const char* path, gp_state_info* info) {
  if (!ctx || !path) return GP_E_ARG;
  gp_params p;
  gp_status s = gp_get_params(ctx, &p);
  if (s != GP_OK) return s;
  gp_state_info in;
  s = gp_state_read_info(path, &in);
  if (s != GP_OK) return s;
  if (in.kind != GP_STATE_PSI || !same_grid(in.params, p)) return GP_E_ARG;
  std::vector<double> psi;
  try {
    psi.resize(2 * plane_points(p));
  } catch (const std::bad_alloc&) {
    return GP_E_NOMEM;
  }
  s = gp_state_read(path, &in, psi.data(), psi.size());
  if (s != GP_OK) return s;
  s = gp_set_psi(ctx, psi.data(), 0);
  if (s == GP_OK && info) *info = in;
  return s;
}

gp_status gp_evolve(gp_ctx* ctx, int imag, int nsteps, int every, gp_output_fn fn, void* user,
                    int* steps_done) {
  if (!ctx || nsteps < 0 || every < 0) return GP_E_ARG;
  int done = 0;
  if (steps_done) *steps_done = 0;
  gp_observables obs;
  bool stop = false;
  if (fn) {
    const gp_status s = gp_energy(ctx, &obs);
    if (s != GP_OK) return s;
    stop = fn(user, ctx, 0, &obs) != 0;
  }
  while (!stop && done < nsteps) {
    const int k = (every > 0 && every < nsteps - done) ? every : nsteps - done;
    gp_status s = imag ? gp_step_imag(ctx, k) : gp_step_real(ctx, k);
    if (s != GP_OK) return s;
    done += k;
    if (steps_done) *steps_done = done;
    if (fn) {
      s = gp_energy(ctx, &obs);
      if (s != GP_OK) return s;
      stop = fn(user, ctx, done, &obs) != 0;
    }
  }
  return fn ? GP_OK : gp_sync(ctx);
}

}  // extern "C"
