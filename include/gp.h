/*
 * gp.h -- C ABI of libgpdbec: one split-step semi-implicit Crank-Nicolson time step
 * of the dipolar Gross-Pitaevskii equation on an AMD Instinct MI355X (gfx950).
 *
 * Method (Loncar et al., CPC, arXiv:1601.04640, program summary "Nature of problem"
 * and "Solution method"; function roles from "Summary of revisions"):
 *   the GP equation with contact and dipolar interactions in a harmonic anisotropic
 *   trap, in 2D (x-y or x-z plane) or 3D, propagated in imaginary time (stationary
 *   states) or real time (dynamics) by split-step Crank-Nicolson; the dipolar
 *   potential is a momentum-space product (convolution theorem).  One step is
 *     n = |psi|^2;  Phi = F^-1[U(k) F[n]]                      (calcpsidd2)
 *     psi <- psi exp(-eps dt (V + g_c n + g_dd Phi))            (calcnu)
 *     CN sweeps along x, y, z, A = eps dt/(4 h^2), Dirichlet    (calclux/y/z)
 *     imaginary time: psi <- psi/sqrt(sum|psi|^2 dV)           (calcnorm)
 *   with eps = 1 (imaginary time) or i (real time), and norm, energy, chemical
 *   potential and rms sizes reduced in FP64 (calcnorm, calcmuen, calcrms).
 *   U(k) = (3 kz^2/k^2 - 1) b(kR) in 3D (dipoles along z, spherical cutoff R);
 *   quasi-2D kernels are its transverse Gaussian averages; g_c = g in 3D and
 *   g/(sqrt(2 pi) d) in 2D with d = 1/sqrt(omega_perp).
 *
 * Layout: every grid is stored x fastest.  3D index (k*ny + j)*nx + i, 2D XY
 *   j*nx + i, 2D XZ k*nx + i.  Complex values are interleaved (re, im).  Grid
 *   coordinates are x_i = (i - n/2) h; the first and last point of every axis are
 *   Dirichlet boundary points (zero).
 *
 * Memory ownership: the caller allocates one device workspace of at least
 *   gp_workspace_bytes() bytes (256-byte aligned) and owns the HIP stream; the library
 *   allocates no device memory, owns only the host-side context, and never frees
 *   the workspace.  All device work of a context is enqueued on its stream.
 *
 * Precision: GP_FP64 keeps every field in double.  GP_FP32_MIXED keeps psi, V, the
 *   spectrum, the kernel table and all bulk arithmetic (FFT, multiply, phase, CN) in
 *   float; norm/energy/mu/rms reductions and the imaginary-time renormalisation
 *   factor are accumulated and computed in double.
 *
 * Errors: every call returns a gp_status; no call prints, throws or aborts.  Steps
 *   are asynchronous: a non-finite norm detected on the device sets a sticky flag
 *   that the next synchronous call (gp_energy, gp_get_psi to host, gp_sync,
 *   gp_history) reports as GP_E_NONFINITE.  A context is not thread-safe; distinct
 *   contexts may be used from distinct threads.
 */
#ifndef GPDBEC_GP_H
#define GPDBEC_GP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int gp_status;
#define GP_OK            0
#define GP_E_ARG        -1  /* bad pointer, non-positive dt/h, bad enum, workspace too small */
#define GP_E_SIZE       -2  /* an axis is < 4; or a 3D axis's FFT line is longer than 8192
                               points (FP32) / 4096 (FP64): N, or for a length with a prime
                               factor above 31 Bluestein's M >= 2N - 1; or a longer 2D axis
                               has no four-step split; see gp_axis_kind */
#define GP_E_DEVICE     -3  /* a HIP runtime call or kernel launch failed */
#define GP_E_NONFINITE  -4  /* the wave function became NaN/Inf (or its norm underflowed to 0) */
#define GP_E_STATE      -5  /* call out of order (e.g. stepping before gp_set_psi) */
#define GP_E_NOMEM      -6  /* host-side allocation failed */
#define GP_E_IO         -7  /* a state file could not be written or read, or is not one */

typedef enum { GP_3D = 0, GP_2D_XY = 1, GP_2D_XZ = 2 } gp_geom;
typedef enum { GP_FP64 = 0, GP_FP32_MIXED = 1 } gp_prec;

/* Problem parameters.  In 2D XY the grid is (ny, nx) and nz, dz are ignored; lambda is
 * the frozen transverse frequency (d = 1/sqrt(lambda)).  In 2D XZ the grid is (nz, nx)
 * and ny, dy are ignored; nu is the frozen transverse frequency (d = 1/sqrt(nu)).
 * cutoff_R <= 0 disables the spherical cutoff (3D only).  The trap is
 * V = (gamma^2 x^2 + nu^2 y^2 + lambda^2 z^2)/2 restricted to the plane in 2D, unless
 * replaced by gp_set_potential. */
typedef struct gp_params {
  int geom;                 /* gp_geom */
  int nx, ny, nz;
  double dx, dy, dz;
  double dt;                /* > 0; the sign of time is set by the step call */
  double gamma, nu, lambda; /* trap frequencies along x, y, z */
  double g, gdd;            /* contact and dipolar couplings (3D units) */
  double cutoff_R;
  int prec;                 /* gp_prec */
} gp_params;

/* FP64 observables of one wave function.  rms[] = (x, y, z); the frozen axis of a 2D
 * geometry reports 0.  e_int and e_dd already contain the 1/2; mu doubles them. */
typedef struct gp_observables {
  double norm, mu, energy, e_kin, e_pot, e_int, e_dd;
  double rms[3];
} gp_observables;

typedef struct gp_ctx gp_ctx;

/* Bytes of device workspace a context with these parameters needs.  Validates params
 * exactly as gp_init does.  (The paper's programs allocate the wave function, one complex
 * temporary and up to two real grids on the device once, before any computation:
 * "Summary of revisions" and Fig. 1; here the caller allocates that memory as one
 * block.) */
gp_status gp_workspace_bytes(const gp_params* params, size_t* bytes);

/* How an axis of n points runs (no GPU work): 1 = passes specialised at compile time
 * for this length (even n = 2^a 3^b 5^c, b, c <= 1, 8 <= n <= 512), 2 = the run-time-length
 * passes (any other n >= 4, even or odd: prime factors up to 31 by Stockham stages,
 * larger ones by Bluestein's algorithm through an FFT of length M >= 2n - 1 whose factors
 * are 2, 3, 5, 7; the FFT line, n or M, up to 8192 points in GP_FP32_MIXED and 4096 in
 * GP_FP64), 3 = longer than one such line, in 2D grids only (the paper's 2D runs reach
 * 15000^2): the FFT by the four-step split n = A B (A >= B the smallest such factor whose
 * A- and B-point transforms fit the line, and two A-point rows fit it together) through
 * the workspace, the Crank-Nicolson sweeps in segments of up to 512 rows joined by their
 * carries; 0 = unsupported (GP_E_SIZE; for kind 3 a length with no such split, e.g. a
 * prime).  A grid with any axis of kind 2 or 3 runs every pass with the run-time-length
 * kernels, which take more launches per step; gp_step_real_adjoint, the batched ensemble
 * and the allocation-free call need axes of kind 1.  (The paper's programs enlarge an
 * unsuitable grid silently, "Unusual features"; here every accepted size runs as given.) */
int gp_axis_kind(int n, int prec);

/* Create a context ("Summary of revisions": the host initialises the variables, which
 * are copied to the device once and stay there).  dev_workspace: device pointer,
 * >= gp_workspace_bytes, 256-byte aligned, owned by the caller and kept alive until
 * gp_destroy.  hip_stream: a hipStream_t (NULL = the null stream).  Builds the FFT
 * twiddles, the kernel table U(k)/N (the momentum-space dipolar term of "Solution
 * method"), the CN factor tables and the harmonic V ("Nature of problem") on the device;
 * psi is unset.  Errors: GP_E_ARG (null pointer, misaligned or small workspace, bad
 * parameter), GP_E_SIZE (see above), GP_E_NOMEM, GP_E_DEVICE. */
gp_status gp_init(const gp_params* params, void* dev_workspace, size_t ws_bytes,
                  void* hip_stream, gp_ctx** out);
gp_status gp_destroy(gp_ctx* ctx);
const char* gp_status_string(gp_status status);

/* Host-resident arrays (the paper's POTMEM choice, Fig. 1 and "Summary of revisions":
 * the potentials may stay in host memory mapped into the GPU's address space, so that
 * larger grids fit on the device).  GP_HOST_V keeps the trap potential V, GP_HOST_KTAB
 * the dipolar kernel table U(k)/N, in caller-owned pinned host memory (hipHostMalloc;
 * torch's pin_memory) instead of the device workspace; the kernels read them through the
 * host mapping at every step, over the host link.  gp_workspace_bytes_ex gives the
 * smaller workspace; gp_host_bytes the sizes of the two host arrays (V: one real value
 * per grid point, in the context precision; the table: its own layout).  gp_init_ex is
 * gp_init with these flags: host_v / host_ktab must be pinned host memory (16-byte
 * aligned) of at least those sizes when their flag is set (else GP_E_ARG), are written
 * at init (the harmonic V, the table) and by gp_set_potential, and must stay alive and
 * untouched by the caller until gp_destroy.  Results are bit for bit those of a context
 * with the arrays resident. */
#define GP_HOST_V    1u
#define GP_HOST_KTAB 2u
gp_status gp_workspace_bytes_ex(const gp_params* params, unsigned host, size_t* bytes);
gp_status gp_host_bytes(const gp_params* params, size_t* v_bytes, size_t* ktab_bytes);
gp_status gp_init_ex(const gp_params* params, unsigned host, void* dev_workspace,
                     size_t ws_bytes, void* host_v, void* host_ktab, void* hip_stream,
                     gp_ctx** out);

/* Wave function I/O ("Summary of revisions": only the wave function returns to the
 * host, when output is written).  on_device = 0: host buffer of interleaved complex
 * double.  on_device = 1: device buffer of interleaved complex in the context precision
 * (double for GP_FP64, float for GP_FP32_MIXED).  The caller owns the buffer; it must
 * hold nx*ny*nz (3D) or the plane's point count values.  set: boundary points are
 * zeroed; the input is otherwise used as is (not renormalised).  get to host
 * synchronises and reports GP_E_NONFINITE if the sticky flag is set. */
gp_status gp_set_psi(gp_ctx* ctx, const void* psi, int on_device);
gp_status gp_get_psi(gp_ctx* ctx, void* psi, int on_device);

/* Replace the trap ("Nature of problem": the harmonic anisotropic trap; the paper's pot
 * array, Fig. 1) by an arbitrary real grid V (host: double; device: context precision),
 * same layout as psi.  The caller keeps ownership; the values are copied. */
gp_status gp_set_potential(gp_ctx* ctx, const void* V, int on_device);

/* Change the contact and dipolar couplings ("Nature of problem": contact and dipolar
 * interactions), e.g. a quench g -> g'.  Takes effect for later steps.  GP_E_ARG for a
 * non-finite value. */
gp_status gp_set_couplings(gp_ctx* ctx, double g, double gdd);

/* nsteps >= 0 steps in imaginary time (with renormalisation) / real time ("Solution
 * method": propagation in imaginary or real time over small time steps; one step runs
 * calcpsidd2, calcnu, calclux, calcluy, calcluz and, in imaginary time, calcnorm, in the
 * order "Summary of revisions" lists them).  Asynchronous.  GP_E_STATE before
 * gp_set_psi, GP_E_ARG for nsteps < 0.  Each step also reduces the FP64 observables of the state it starts
 * from (kept in a history ring, see gp_history).  Each step leaves its final FP64
 * reduction (the record, the non-finite check and, in imaginary time, the new
 * renormalisation factor) to the next step's first launch; every other call on the
 * context (gp_history, gp_sync, gp_energy, gp_get_psi, ...) completes an outstanding
 * one before it does anything else, so what those calls see is unchanged. */
gp_status gp_step_imag(gp_ctx* ctx, int nsteps);
gp_status gp_step_real(gp_ctx* ctx, int nsteps);

/* Backpropagation through one real-time step (gp_step_real with nsteps = 1).
 * All pointers are device pointers.  psi_n: the forward state at the START of the step
 * (interleaved complex, context precision, physical values).  lam: in: the costate
 * dL/d conj(psi) at the end of the step; out: at its start (context precision, in
 * place).  gradV: double grid (psi layout), accumulated += dL/dV of this step.
 * grad_g, grad_gdd: one double each, accumulated += dL/dg (3D units; the quasi-2D
 * contact factor 1/(sqrt(2 pi) d) is applied) and += dL/dg_dd.  With the convention
 * dL = 2 Re sum conj(lam) dpsi:
 *   lam_a = C_x(-dt) C_y(-dt) C_z(-dt) lam     (adjoint CN sweeps)
 *   mu = exp(+i dt theta) lam_a,  s = 2 dt Im(conj(mu) psi_n),  theta of psi_n
 *   dL/dV += s, dL/dg_c += sum s n, dL/dg_dd += sum s Phi
 *   lam_n = mu + (g_c s + g_dd F^-1[U F[s]]) psi_n
 * Uses the context's workspace (spectrum, scratch field) and couplings/potential; the
 * context's own psi is left unchanged.  Asynchronous on the context's stream. */
gp_status gp_step_real_adjoint(gp_ctx* ctx, const void* psi_n, void* lam, double* gradV,
                               double* grad_g, double* grad_gdd);

/* Observables of the current psi: norm (calcnorm), energy, chemical potential and their
 * parts (calcmuen, with the forward-difference kinetic term that calcmuen's partial
 * derivatives stand for) and rms sizes (calcrms), all accumulated in FP64 ("Summary of
 * revisions").  Computes Phi of this psi.  Synchronous; GP_E_NONFINITE if the sticky flag
 * is set, GP_E_STATE before gp_set_psi. */
gp_status gp_energy(gp_ctx* ctx, gp_observables* out);

/* Phi = F^-1[U F[|psi|^2]] of the current psi, WITHOUT the g_dd factor: the dipolar
 * potential that calcpsidd2 evaluates by the convolution theorem ("Solution method";
 * real-to-complex and complex-to-real transforms of the real density, "Summary of
 * revisions").  on_device = 0: host buffer of double (synchronous); 1: device buffer in
 * context precision (asynchronous).  The caller owns the buffer. */
gp_status gp_dipolar_potential(gp_ctx* ctx, void* phi, int on_device);

/* Observables of the states the most recent steps started from, oldest first.
 * Copies min(max_records, available) records (at most gp_history_capacity()) to host
 * memory; *count receives the number copied.  Synchronous. */
gp_status gp_history(gp_ctx* ctx, gp_observables* out, int max_records, int* count);
int gp_history_capacity(void);

/* Wait for the context's stream; reports the sticky non-finite flag. */
gp_status gp_sync(gp_ctx* ctx);

/* Step loops of at least 8 steps replay a captured HIP graph of 8 steps (captured once
 * per time direction, re-captured after gp_set_couplings); enable = 0 launches every
 * pass directly.  Default: enabled.  Timing (below) always launches directly. */
gp_status gp_use_graphs(gp_ctx* ctx, int enable);

/* Optional per-pass timing (profiling and benchmarks).  With a non-zero mask, every
 * launch of a selected pass (bit 1 << gp_pass) inside a step is timed with a pair of HIP
 * events on the context's stream: GP_PASS_C2R_NL_CNX is launched with
 * hipExtLaunchKernelGGL, whose events take the kernel dispatch's own start and end
 * timestamps; the other passes are bracketed by event records.  gp_timing_read
 * synchronises, returns the summed durations (ms) and launch counts of every pass since
 * the last enable, and keeps timing on.  Mask 0 turns timing off.  Steps run without
 * graph replay while timing is on.  Events are host-side objects; no device memory is
 * allocated. */
typedef enum {
  GP_PASS_R2C_X = 0,      /* |psi|^2, x real-to-complex FFT, x/y kinetic sums      */
  GP_PASS_FFT_Y_FWD = 1,  /* 3D: forward y FFT of the half spectrum                */
  GP_PASS_CONV_Z = 2,     /* 3D: z FFT, U(k)/N product, inverse z FFT              */
  GP_PASS_FFT_Y_INV = 3,  /* 3D: inverse y FFT                                     */
  GP_PASS_CONV_Y = 4,     /* 2D: y FFT, U(k)/N product, inverse y FFT              */
  GP_PASS_C2R_NL_CNX = 5, /* x C2R -> Phi, observables sums, phase, CN sweep x     */
  GP_PASS_CN_Y = 6,       /* CN sweep y (2D: with the new-state norm sum)          */
  GP_PASS_CN_Z = 7,       /* 3D: CN sweep z with new-state norm / z-kinetic sums   */
  GP_PASS_FINALIZE = 8,   /* single-block FP64 finalisation of the block partials   */
                          /* (norm, observables, next lazy scale, history record)   */
  GP_PASS_COUNT = 9
} gp_pass;
gp_status gp_timing_enable(gp_ctx* ctx, unsigned pass_mask);
gp_status gp_timing_read(gp_ctx* ctx, double* total_ms, int* launches);
/* In-kernel span of a timed pass: while timing is enabled for GP_PASS_C2R_NL_CNX, every
 * launch of that pass inside a step also stamps each block's start and end with the
 * device wall clock, and a one-block kernel adds (last end - first start) to a device
 * accumulator.  Returns the summed spans (ms) and launch count since gp_timing_enable;
 * unlike the event pairs it excludes the events' own latency.  Synchronous.  GP_E_ARG for
 * any other pass. */
gp_status gp_timing_span(gp_ctx* ctx, int pass, double* total_ms, int* launches);
/* Duration of one pass alone: `reps` (1..4096) back-to-back launches of the pass, on the
 * current state exactly as inside a real-time step, are captured into a HIP graph and
 * replayed twice; the second replay is bracketed by one pair of events on the context's
 * stream and *ms_per_launch = its duration / reps.  Passes: GP_PASS_R2C_X,
 * GP_PASS_C2R_NL_CNX, GP_PASS_CN_Y, GP_PASS_CN_Z (3D).  Synchronous.  The stored state is
 * advanced by the repeated partial steps: set psi again before using the context for a
 * run.  GP_E_ARG for another pass or reps out of range, GP_E_STATE before gp_set_psi. */
gp_status gp_timing_burst(gp_ctx* ctx, int pass, int reps, double* ms_per_launch);

/* ------------------------------------------------------------ batched ensemble
 * Many independent quasi-2D instances (GP_2D_XY / GP_2D_XZ, any mix) of uneven sizes
 * and parameters, stepped together: each pass of a step is one persistent launch per
 * size class (lines <= 256 points, and 384/512) over a work list of (instance, tile)
 * items from every instance, sorted by decreasing instance size; one FP64 finalisation
 * block per instance.  Steps replay a captured HIP graph (8 steps) when nsteps >= 8.
 * All instances share one precision; every axis must be one of 32, 48, 64, 96, 128, 192,
 * 256, 384, 512 (else GP_E_SIZE).  The caller-owned workspace holds one single-grid
 * workspace per instance plus descriptors and work lists. */
typedef struct gp_batch gp_batch;
gp_status gp_batch_workspace_bytes(const gp_params* params, int count, size_t* bytes);
gp_status gp_batch_init(const gp_params* params, int count, void* dev_workspace,
                        size_t ws_bytes, void* hip_stream, gp_batch** out);
gp_status gp_batch_destroy(gp_batch* batch);
/* The single-grid context of instance idx (owned by the batch; NULL if out of range):
 * use it for gp_set_psi / gp_get_psi / gp_energy / gp_history of that instance. */
gp_ctx* gp_batch_context(gp_batch* batch, int idx);
/* gp_set_psi / gp_get_psi of instance idx (GP_E_ARG if idx is out of range). */
gp_status gp_batch_set_psi(gp_batch* batch, int idx, const void* psi, int on_device);
gp_status gp_batch_get_psi(gp_batch* batch, int idx, void* psi, int on_device);
/* nsteps imaginary- / real-time steps of every instance (all psi must be set;
 * GP_E_STATE otherwise).  An instance context stepped on its own since the last batch
 * step is brought up to date first. */
gp_status gp_batch_step_imag(gp_batch* batch, int nsteps);
gp_status gp_batch_step_real(gp_batch* batch, int nsteps);
/* Observables of every instance's current psi (count records).  Synchronous. */
gp_status gp_batch_energy(gp_batch* batch, gp_observables* out);
/* Launch plan (autotuner interface).  items/blocks: arrays of 4 passes x 2 size classes
 * (r2c, conv, c2r, cn; class 0 = lines <= 256): work items and persistent blocks.
 * gp_batch_set_blocks sets the persistent block count of one (pass, class); 0 restores
 * the default (min(items, 1024)). */
gp_status gp_batch_plan(gp_batch* batch, int* items, int* blocks);
gp_status gp_batch_set_blocks(gp_batch* batch, int pass, int size_class, int blocks);
/* Tile shape of one (pass, class), for the autotuner: 0 = the default tiles; 1 = x tiles
 * and CN column tiles of 8 lines (32 lanes per line) where the default is 16, and
 * line-FFT blocks of twice the default points.  The work lists, the launches' LDS and the
 * captured graphs are rebuilt (outstanding finalisations are completed first); results
 * change only by rounding order.  gp_batch_shapes copies the 4 x 2 shapes in use. */
gp_status gp_batch_set_shape(gp_batch* batch, int pass, int size_class, int shape);
gp_status gp_batch_shapes(gp_batch* batch, int* shapes);
gp_status gp_batch_use_graphs(gp_batch* batch, int enable);
/* enable = 1: the larger size class of every pass runs on a second stream, forked from
 * and joined back to the batch stream around the pass (so the two classes overlap; a
 * captured step graph then has two branches per pass).  Default 0: one stream, one
 * linear chain of launches. */
gp_status gp_batch_use_streams(gp_batch* batch, int enable);

/* ------------------------------------------------------ saved states and output
 * The imaginary-time run hands its stationary state to the real-time run through a file
 * (program summaries of the real-time programs: a run with no imaginary-time steps of its
 * own reads the imaginary-time program's output), and runs report the chemical
 * potential, energy, rms sizes (calcmuen, calcrms) and the density at chosen steps; only
 * the wave function returns to the host, for output ("Summary of revisions").
 *
 * State file (the library's own layout; little-endian):
 *   bytes   0..7    magic "GPDBECS1"
 *           8       uint32 version (1)
 *          12       uint32 kind: 1 = wave function, 2 = density |psi|^2
 *          16..31   int32 geom, nx, ny, nz
 *          32..111  double dx, dy, dz, dt, gamma, nu, lambda, g, gdd, cutoff_R
 *         112       int32 prec of the context that wrote it
 *         120       int64 step (the caller's label)     128  double time (the caller's label)
 *         136       uint64 npoints (the grid's point count: nx*ny*nz, or the plane's)
 *         144       uint64 FNV-1a 64 of the payload bytes; the rest of the 256 bytes is zero
 *   payload from byte 256: npoints complex doubles (re, im) for kind 1, npoints doubles
 *   for kind 2, in the psi layout (x fastest).  Values are FP64 whatever the context
 *   precision (an FP32 context's values widened exactly). */
#define GP_STATE_PSI     1
#define GP_STATE_DENSITY 2
typedef struct gp_state_info {
  int kind;                 /* GP_STATE_PSI or GP_STATE_DENSITY */
  gp_params params;         /* the writing context's parameters */
  long long step;
  double time;
  unsigned long long npoints;
  unsigned long long checksum;
} gp_state_info;

/* The parameters the context runs with (those of gp_init, with the couplings of the last
 * gp_set_couplings).  Host only. */
gp_status gp_get_params(gp_ctx* ctx, gp_params* out);

/* Write the current wave function (kind 1) or its density (kind 2) to `path`, labelled
 * with step and time.  Synchronous (the values come to the host through gp_get_psi, so
 * GP_E_NONFINITE is reported as there).  A failed write removes the file: GP_E_IO. */
gp_status gp_save_state(gp_ctx* ctx, const char* path, long long step, double time);
gp_status gp_save_density(gp_ctx* ctx, const char* path, long long step, double time);

/* Read a wave-function file into the context (as gp_set_psi from a host buffer: the
 * boundary points are zeroed, the values are otherwise used as they are).  The file's grid
 * (geometry, point counts, spacings to 1e-12 relative) must be the context's: else
 * GP_E_ARG; the trap, couplings, dt and precision may differ (a quench, a real-time run
 * from an imaginary-time state).  GP_E_IO for a missing, short, over-long or corrupt file
 * (checksum).  info (may be NULL) receives the header. */
gp_status gp_load_state(gp_ctx* ctx, const char* path, gp_state_info* info);

/* Header of a state file (no GPU work).  GP_E_IO if it is not a state file. */
gp_status gp_state_read_info(const char* path, gp_state_info* info);
/* Header and payload: data receives npoints * (2 for kind 1, 1 for kind 2) doubles;
 * GP_E_ARG if that exceeds max_doubles, GP_E_IO for a short, over-long or corrupt file. */
gp_status gp_state_read(const char* path, gp_state_info* info, double* data,
                        size_t max_doubles);

/* Step loop with output cadence: nsteps imaginary-time (imag != 0) or real-time steps,
 * in runs of `every` steps (every = 0: one run).  When fn is not NULL it is called on the
 * host with the observables of the state after 0, every, 2 every, ... and nsteps steps
 * (gp_energy of that state, FP64); inside the call the context may be used (gp_get_psi,
 * gp_save_state, gp_save_density, ...).  A non-zero return stops the loop after that
 * output.  *steps_done (may be NULL) receives the steps taken.  Errors as gp_step_* and
 * gp_energy. */
typedef int (*gp_output_fn)(void* user, gp_ctx* ctx, int step, const gp_observables* obs);
gp_status gp_evolve(gp_ctx* ctx, int imag, int nsteps, int every, gp_output_fn fn, void* user,
                    int* steps_done);

/* ------------------------------------------------------------ allocation-free call
 * For callers that cannot allocate device memory, and cannot hand the library a
 * workspace either: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Computes the same Phi = F^-1[U F[|psi|^2]] as gp_dipolar_potential
 * (without the g_dd factor), for a device psi, with no context: psi and phi are device
 * buffers in the precision of params->prec (interleaved complex / real, the layout of
 * gp_set_psi), owned by the caller; work is enqueued on hip_stream (a hipStream_t, NULL =
 * the null stream) and the call returns without waiting.  The half spectrum, the kernel
 * table, the twiddles and the partial sums live in a library-owned static device array of
 * 64 MiB per device (held until the process ends; enough for 128^3 in FP64, about 200^3
 * in FP32); the call allocates no host or device memory.  Every call on one device
 * shares that array and overwrites it, so calls that overlap on one device (two streams,
 * two threads) race: serialise them.  Errors: GP_E_ARG (null pointer, bad parameter),
 * GP_E_SIZE (unsupported axis, or a grid whose arrays exceed the 64 MiB; gp_last_error
 * then gives the bytes needed), GP_E_DEVICE. */
gp_status gp_dipolar_potential_noalloc(const gp_params* params, const void* psi, void* phi,
                                       void* hip_stream);

/* Text of the HIP error behind the calling thread's most recent GP_E_DEVICE, or of the
 * size limit behind a GP_E_SIZE of gp_dipolar_potential_noalloc ("" if none).  The
 * pointer stays valid until the thread's next failing call. */
const char* gp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GPDBEC_GP_H */
