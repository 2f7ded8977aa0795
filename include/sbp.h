/*
 * sbp.h - shearing-box Poisson solver for AMD MI355X (gfx950): C ABI.
 *
 * Solves the Poisson equation  lap(Phi) = 4 pi G rho  (Eq. 1 of Rendon Restrepo & Gressel,
 * "An efficient spectral Poisson solver for the NIRVANA code: the shearing-box case with
 * vertical vacuum boundary conditions") on a cell-centred Nx x Ny x Nz box that is
 * shear-periodic in x, periodic in y and vacuum-bounded in z.  One solve performs:
 *
 *   a0  shear parameters: Delta_y0 = fmod(q Omega Lx t, Ly) in [0, Ly), s = Delta_y0/Lx, and
 *       the sheared wave vector k(t) = (Kx + s Ky, Ky, kz) (Sect. 2.1);
 *   a1  map to the periodic frame (spectral y-shift by exp(-i Ky s x)) and the forward
 *       horizontal transforms (Sect. 2.1);
 *   a2  Hockney zero padding of z from Nz to M = P Nz cells (Sect. 2.2, Sect. 2.4);
 *   a3  forward z transform of each padded pencil;
 *   a4  multiplication by the Green's function: VGF-HybridBC uses the regularised
 *       G^L(k, kz) with L = alpha Lz (Sect. 2.3, equation "Green's function regularized in
 *       Fourier", App. A); SASHA uses -1/|k|^2 with the zero mode removed (Eq. 2, Sect. 2.2);
 *   a5  inverse z transform and extraction of the Nz physical cells;
 *   a6  inverse horizontal transforms, reverse mapping exp(+i Ky s x), scaling by 4 pi G
 *       (Sect. 2.3), plus Phi_0(z) = 4 pi G <rho> z (z/2 - z0) for SASHA (Sect. 2.2);
 *   a7  (SASHA) the reductions sum(rho) and sum(z rho) that give <rho> and z0.
 *
 * Conventions (the paper leaves them open):
 *   - lab fields satisfy f(x + Lx, y) = f(x, y + Delta_y0); q is a parameter (3/2 in the paper);
 *   - cell centres x_i = (i+1/2) Lx/Nx, y_j = (j+1/2) Ly/Ny, z_k = -Lz/2 + (k+1/2) Lz/Nz;
 *   - the y-Nyquist row is dropped; x and z mode numbers run 0..n/2-1, -n/2..-1;
 *   - discrete normalisation Phi = 4 pi G IDFT(G DFT(rho_padded));
 *   - SASHA's mean is over the padded domain, <rho> = sum(rho)/(Nx Ny M);
 *   - linear remap: row x_i is shifted by s x_i / dy y cells, interpolated between floor and
 *     floor + 1 of the sampled position.
 *
 * Memory: rho and phi are caller-owned DEVICE buffers in C order [nx][ny][nz] (z fastest),
 * element type float for SBP_FP32 plans and double for SBP_FP64 plans.  rho is only read;
 * phi must not overlap rho or the workspace.  All entry points return an sbp_status; no
 * C++ exception crosses this interface.  A plan is not thread-safe and serves one stream at
 * a time.
 */
#ifndef SBP_H
#define SBP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sbp_plan_s* sbp_plan;

typedef enum {
  SBP_OK = 0,
  SBP_E_ARG = 1,       /* null/aliased pointer, bad enum or flag, non-positive length */
  SBP_E_SIZE = 2,      /* grid size outside the supported set (see sbp_plan_create)   */
  SBP_E_NOMEM = 3,     /* host or device allocation failed                            */
  SBP_E_WORKSPACE = 4, /* workspace pointer null/misaligned or smaller than required  */
  SBP_E_HIP = 5,       /* a HIP runtime call failed (also reports earlier async errors)*/
  SBP_E_STATE = 6      /* call not valid in the plan's current state                  */
} sbp_status;

typedef enum { SBP_FP64 = 0, SBP_FP32 = 1 } sbp_precision;
typedef enum { SBP_VGF = 0, SBP_SASHA = 1 } sbp_method;
/* Mapping to the periodic frame (Sect. 2.1 names both): the periodic field at (x, y) is the lab
 * field at (x, y - s x).  SPECTRAL multiplies the y spectrum by exp(-i Ky s x) (Fourier
 * interpolation); LINEAR samples the lab field at y - s x by linear interpolation between the
 * two neighbouring y cells (periodic in y) before the y transform, and the potential back at
 * y + s x after it.  Both use the sheared wave vector kx = Kx + s Ky in the Green's function. */
typedef enum { SBP_REMAP_SPECTRAL = 0, SBP_REMAP_LINEAR = 1 } sbp_remap;

/* Plan flags. */
#define SBP_FLAG_GRAPH 0x1u    /* capture the solve once into a HIP graph; replay per call      */
#define SBP_FLAG_AUTOTUNE 0x2u /* time the tile variants at plan creation and keep the fastest
                                  (five-pass kernels, fused passes A and C); results are cached in
                                  the file named by SBP_TUNE_CACHE ($HOME/.cache/sbp_tune.txt) */
#define SBP_FLAG_PLAIN 0x4u    /* unfused reference path: padded spectrum in HBM, one kernel per
                                  step (pad, each axis transform, Green multiply, extract, ...) */
#define SBP_FLAG_FIVE_PASS 0x8u /* one streaming pass per axis and direction: five HBM round trips
                                   of the half spectrum */
#define SBP_FLAG_FUSED 0x10u    /* fused three-pass schedule (x split into 16 x nx/16, four-step):
                                   three HBM round trips of the half spectrum.  It applies to
                                   power-of-two 16 <= nx <= 256, 16 <= ny <= 512 and
                                   32 <= pad*nz <= 512, and, with this flag only, to FP32 boxes
                                   with nx and ny in {512, 1024}, pad 2 and 64 <= 2*nz <= 512 (x
                                   split into 64 x nx/64); other boxes of the plan run five-pass.
                                   Without either schedule flag a plan takes the fused schedule
                                   wherever it is the faster on gfx950: the narrow boxes above in
                                   both precisions, not the wide FP32 ones (there five-pass is
                                   1.2-1.5 x faster).  Both flags together are SBP_E_ARG. */

/* Geometry, method and remap of one box.
 *   nx, ny: horizontal cells, each in {8,12,16,24,32,48,64,96,128,192,256,384,512,768,1024};
 *   nz:     vertical cells, even, >= 4, with pad*nz in the same set;
 *   lx, ly, lz: box lengths, > 0 and finite;
 *   pad:    z padding factor P in {2, 4}; 0 selects 2;
 *   alpha:  truncation L = alpha*lz of the VGF kernel (Sect. 2.3); 0 selects pad/2 (the padded
 *           half-period, so periodic images of the truncated kernel never reach the box);
 *           must satisfy 1 <= alpha <= pad/2 otherwise;
 *   method: sbp_method;
 *   remap:  sbp_remap (the plain path supports SBP_REMAP_SPECTRAL only). */
typedef struct {
  int32_t nx, ny, nz;
  double lx, ly, lz;
  int32_t pad;
  double alpha;
  int32_t method;
  int32_t remap;
} sbp_box;

/* Per-solve parameters of one box: shear rate q, rotation Omega, time t, constant G.
 * q*omega*lx*t must be finite. */
typedef struct {
  double q, omega, t, G;
} sbp_shear;

/* Create a plan for nbox (1..4096) boxes, solved together by each sbp_solve call.
 * precision: sbp_precision.  SBP_FP32 computes the transforms in float with twiddles,
 *   Green's-function scalars, shear phases and the k = 0 pencil evaluated in double.
 * device: HIP device ordinal; the plan's tables are allocated there.
 * flags: SBP_FLAG_*; SBP_FLAG_PLAIN requires SBP_FP64 and nbox == 1 and excludes the
 *   schedule flags.
 * On success *out receives the plan; on failure *out is set to NULL.
 * Returns SBP_E_ARG / SBP_E_SIZE for invalid descriptors before any HIP call is made. */
sbp_status sbp_plan_create(const sbp_box* boxes, int32_t nbox, int32_t precision, int32_t device,
                           uint32_t flags, sbp_plan* out);

/* Bytes of device workspace a solve needs (intermediate spectra of all boxes). */
sbp_status sbp_workspace_size(sbp_plan plan, size_t* bytes);

/* Hand the plan a caller-owned device workspace of at least sbp_workspace_size bytes,
 * 256-byte aligned.  The caller keeps ownership and must keep it alive while solves that
 * use it are in flight.  Without this call the plan allocates its own workspace on the
 * first solve.  Passing NULL reverts to plan-owned workspace. */
sbp_status sbp_set_workspace(sbp_plan plan, void* device_ptr, size_t bytes);

/* Enqueue one solve of every box on `stream` (a hipStream_t; NULL = default stream).
 * rho[b], phi[b]: device pointers of box b (see layout above); params[b]: host memory,
 * read before the call returns.  Returns SBP_OK once the work is enqueued; the result is
 * ready when the stream reaches that point.  Asynchronous kernel faults surface as
 * SBP_E_HIP from a later call. */
sbp_status sbp_solve(sbp_plan plan, const void* const* rho, void* const* phi,
                     const sbp_shear* params, void* stream);

/* Size of the fixed device workspace that sbp_solve_static uses: 128 MiB, enough for a
 * 256 x 256 x 256 box in either precision (a plan's need is sbp_workspace_size). */
#define SBP_STATIC_WORKSPACE_BYTES (128u << 20)

/* For callers that cannot allocate device memory while they solve: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same arguments, layout and result as
 * sbp_solve, but the workspace is a fixed array of SBP_STATIC_WORKSPACE_BYTES that the library
 * holds on each device until the process ends (set up by sbp_plan_create on that device), so the
 * call makes no hipMalloc, hipFree or other allocating call; the plan's own workspace and one set
 * by sbp_set_workspace are not used.  It records no profiling events.
 *   - SBP_E_SIZE if the plan needs more workspace than the array holds;
 *   - SBP_E_STATE for an SBP_FLAG_GRAPH plan whose graph has not been captured yet (its first
 *     sbp_solve captures it);
 *   - SBP_E_HIP if the array's device address could not be obtained on the plan's device;
 *   - SBP_E_ARG as sbp_solve, and if rho or phi overlaps the array.
 * Every call on one device shares that device's array and leaves its contents behind; nothing in
 * it needs to start at zero (a solve writes every workspace value before it reads it).  Calls that
 * overlap in time on one device (other streams, or other host threads) race on the array and
 * must be serialised by the caller. */
sbp_status sbp_solve_static(sbp_plan plan, const void* const* rho, void* const* phi, const sbp_shear* params,
                            void* stream);

/* Potential with ng ghost layers below and above the box (Sect. 2.4): in the ghost cells the
 * vertical gradient equals that of the last active cell, i.e. Phi continues linearly with the
 * slope between the two outermost active cells.
 * phi[b]: device, [nx][ny][nz] (as written by sbp_solve); out[b]: device, [nx][ny][nz + 2 ng],
 * the active cells at z offset ng; element type of the plan's precision; out must not overlap
 * phi.  1 <= ng <= 16, else SBP_E_ARG.  Enqueued on `stream`. */
sbp_status sbp_ghosts(sbp_plan plan, const void* const* phi, void* const* out, int32_t ng, void* stream);

/* Gravitational acceleration g = -grad Phi of every box at the cell centres, by second-order
 * centred differences: periodic in y; in z the values beyond the edges follow the ghost rule
 * above (so the edge cells take the one-sided difference); shear-periodic in x, where the
 * neighbour beyond the last x row is the first row sampled at y + Delta_y0 and the one before
 * the first row is the last row sampled at y - Delta_y0, by linear interpolation in y.
 * phi[b]: device, [nx][ny][nz]; gx[b], gy[b], gz[b]: device outputs of the same layout and
 * type, not overlapping each other or phi; params[b]: the shear parameters of the solve (only
 * Delta_y0 = fmod(q Omega Lx t, Ly) is used).  Enqueued on `stream`. */
sbp_status sbp_gravity(sbp_plan plan, const void* const* phi, void* const* gx, void* const* gy, void* const* gz,
                       const sbp_shear* params, void* stream);

/* Free the plan and everything it allocated.  It first waits for all work on the plan's device
 * (hipDeviceSynchronize), so that nothing still queued reads what it frees; it must therefore
 * not be called while a stream of that device is being captured.  NULL is accepted and ignored. */
sbp_status sbp_plan_destroy(sbp_plan plan);

/* Static description of a status code. */
const char* sbp_status_str(sbp_status status);

/* Detail message of the last failing call on this thread ("" if none). */
const char* sbp_last_error(void);

/* Instrumentation: when enabled, sbp_solve records HIP events around each kernel it launches
 * (on the solve's stream) and accumulates their durations.  sbp_profile_read copies up to
 * `cap` records {name, launches, total milliseconds} into the caller's arrays, returns the
 * number of distinct kernels in *count, and resets the accumulators.  Graph plans are timed
 * as a whole ("graph").  names[i] points to static strings owned by the library. */
sbp_status sbp_profile_enable(sbp_plan plan, int32_t enable);
sbp_status sbp_profile_read(sbp_plan plan, const char** names, int64_t* launches, double* total_ms,
                            int32_t cap, int32_t* count);

/* One-line JSON description of the plan's schedule (passes, tile variants, bytes moved per
 * solve) written into buf (NUL-terminated, truncated to len). */
sbp_status sbp_plan_describe(sbp_plan plan, char* buf, size_t len);

#ifdef __cplusplus
}
#endif

#endif /* SBP_H */
