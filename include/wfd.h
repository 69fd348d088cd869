/*
 * wfd.h — C ABI of the MI355X acoustic finite-difference library.
 *
 * The library time-steps the 3-D acoustic wave equation (arXiv 2502.12350,
 * §2.1, Eq. 1): constant density p_tt = c^2 lap(p) + S, or variable density
 * q_tt = c^2 (lap(q) - m^2 q) + S / sqrt(rho) with q = p / sqrt(rho) and
 * m^2 = lap(sqrt(rho)) / sqrt(rho), S = f(t) delta(x - x_S).  The scheme is
 * second order in time (leapfrog) and eighth order in space (§2.1), with an
 * absorbing boundary of `border` cells (§2.1; §2.2.1 parameter table): a
 * damping sponge, or a CPML layer; optionally a free surface on top.  It
 * serves forward modeling (Alg. 1) and the per-shot body of the FWI gradient
 * (Alg. 3): forward sweep with receiver recording and wavefield saving,
 * misfit, backward (adjoint) sweep with the cross-correlation imaging
 * condition, and the chain rule to the velocity gradient.  Forward-wavefield
 * management follows the paper's three options (§2.1): keep every state in
 * memory, keep it in secondary (here host) storage, or optimal checkpointing
 * with recomputation.  Gradient smoothing, time resampling and the layers of
 * a learned gradient preconditioner are separate calls below.
 *
 * Conventions (§2.2.2, data format)
 *   - volumes are C-order [z][y][x], x fastest, FP32;
 *   - positions are metres, (x, y, z) order, FP64, host memory; a position
 *     maps to the nearest node, i = floor((x - o) / h + 1/2); a position
 *     outside the model is an error (WFD_E_RANGE);
 *   - seismograms are trace-major [nrec][nt] FP32: sample n of a trace is
 *     the recorded pressure at time (n + 1) dt, wavelet sample n is the
 *     source value at time n dt;
 *   - the border is added outside the model on all six faces (with a free
 *     surface the top one holds zeros and absorbs nothing); the padded grid
 *     is Nd = nd + 2 border, with the model's edge values replicated into
 *     the border; each Nd is at most 2^24 and a pitched x-y plane (Nx
 *     rounded up to a multiple of 64, times Ny) holds fewer than 2^30 points
 *     (WFD_E_ARG otherwise).
 *
 * Ownership and ordering
 *   - the caller owns every device buffer (model buffer, workspace, inputs,
 *     outputs); the library owns only the opaque context.  All device
 *     pointers must belong to the context's device.  The library never
 *     calls hipMalloc.
 *   - every call that launches work is stream-ordered on the context's
 *     stream and returns without synchronising, except wfd_set_model (it
 *     waits for its CFL reduction) and wfd_kernel_stats.
 *   - outputs named "accumulated" are added to (+=), so several shots sum,
 *     as the paper's all-reduce over shots does (Alg. 3).
 *
 * Errors: every call returns a wfd_status; nothing aborts or throws across
 * the ABI.  wfd_last_error() returns a thread-local description of the last
 * failure on the calling thread.
 */
#ifndef WFD_H
#define WFD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WFD_OK = 0,
  WFD_E_ARG = -1,    /* bad size, null required pointer, inconsistent arguments   */
  WFD_E_CFL = -2,    /* dt violates the stability bound (ValidConditions, §2.2)    */
  WFD_E_RANGE = -3,  /* a source / receiver position lies outside the model        */
  WFD_E_NOMEM = -4,  /* caller buffer smaller than the size the library asked for  */
  WFD_E_HIP = -5,    /* a HIP runtime call failed                                   */
  WFD_E_STATE = -6   /* call out of order (e.g. forward before set_model)          */
} wfd_status;

/* Model grid, sponge and time axis (§2.2.1: nx ny nz, dx dy dz, ox oy oz,
 * border, dt, ns).  nt is the number of time steps = samples per trace. */
typedef struct {
  int32_t nx, ny, nz; /* model points per axis (>= 1)                          */
  double dx, dy, dz;  /* spacing, m (> 0)                                      */
  double ox, oy, oz;  /* position of model node (0,0,0), m                      */
  int32_t border;     /* sponge cells on every face (>= 0; 0 = no sponge)      */
  double dt;          /* time step, s (> 0)                                    */
  int32_t nt;         /* number of time steps (>= 1)                           */
  int32_t free_surface; /* 1: pressure-release free surface at the top model
                           plane (z index 0; the image method: planes above it
                           read as the negated mirror, sqrt(rho) mirrored
                           evenly, no sponge on that side; the field is zero
                           on and above it); 0: sponge on all six faces      */
  int32_t cpml;       /* absorbing boundary in the border cells (§2.1):
                         0: damping (the Cerjan sponge);
                         1: CPML (Roden and Gedney's convolutional PML) with
                         d(delta) = d0 (delta/N)^2, d0 = -3 vmax ln(1e-3) /
                         (2 N h), alpha = pi fpeak (1 - delta/N), kappa = 1,
                         delta the depth into the layer in cells; no layer on
                         the free-surface side                             */
  double fpeak;       /* CPML: source peak frequency, Hz (>= 0; 0 = alpha 0)  */
  double cpml_vmax;   /* CPML: velocity of d0, m/s (> 0), or 0 = the model's
                         largest velocity.  The layer's coefficients are held
                         fixed in the gradient (like dt).                  */
} wfd_grid;

/* Forward-wavefield management for the gradient (§2.1, the three options:
 * the whole wavefield in memory, the whole wavefield in secondary storage,
 * optimal checkpointing).  The secondary store here is host RAM reached over
 * PCIe (WFD_CKPT_HOST); writing it to a file is left to the caller. */
enum {
  WFD_CKPT_FULL = 0,    /* keep w^1 .. w^nt in the device workspace            */
  WFD_CKPT_REVOLVE = 1, /* keep n_snapshots leapfrog pairs, recompute the rest */
  WFD_CKPT_HOST = 2     /* keep w^1 .. w^nt in caller-owned pinned host memory;
                           the device workspace holds a ring of 4 staging
                           volumes.  Copies run on a second stream of the
                           context, overlapped with the step kernels, and are
                           complete when the caller's stream reaches the end of
                           the call.  The gradient is bitwise that of FULL.   */
};
typedef struct {
  int32_t mode;         /* WFD_CKPT_FULL, WFD_CKPT_REVOLVE or WFD_CKPT_HOST     */
  int32_t n_snapshots;  /* REVOLVE: pairs kept (>= 1); 0 = derive from
                           mem_fraction of the device's free memory            */
  double mem_fraction;  /* (0, 1]; like the paper's check_mem (default 0.8)    */
  void *host_store;     /* HOST: page-locked host buffer (hipHostMalloc, or a
                           torch tensor made with pin_memory=True) of at least
                           wfd_host_store_bytes(); slot m-1 receives 2^e w^m
                           (e: the call's field exponent, wfd_gradient_opts) on
                           the padded grid as [Nz][Ny][pitch] FP32, pitch = Nx
                           rounded up to a multiple of 64 (the columns past
                           Nx are padding).  Other modes: ignored.            */
  uint64_t host_bytes;  /* HOST: size of host_store in bytes                   */
} wfd_ckpt;

typedef struct wfd_ctx wfd_ctx;

/* Create a context on HIP device `device` that launches on `hip_stream`
 * (a hipStream_t; NULL = the legacy default stream). */
wfd_status wfd_create(wfd_ctx **ctx, int32_t device, void *hip_stream);

/* Change the stream later calls launch on. */
wfd_status wfd_set_stream(wfd_ctx *ctx, void *hip_stream);

/* Release the context (not the caller's buffers).  NULL is accepted. */
wfd_status wfd_destroy(wfd_ctx *ctx);

/* Bytes of the caller-owned device buffer that holds the precomputed model
 * (coefficient volumes and sponge tables) for this grid.  Host only. */
wfd_status wfd_model_bytes(const wfd_grid *grid, int32_t variable_density, size_t *bytes);

/* Prepare a model (Eq. 1 coefficients, ValidConditions):
 *   k = dt^2 v^2 on the padded grid (edge-replicated v),
 *   VD only: m^2 = L8(sqrt(rho)) / sqrt(rho) in FP64 (sqrt(rho) replicated
 *   past the padded grid as well), sqrt(rho) kept for source/receiver scales,
 *   1-D sponge tables g[i] = exp(-(0.4 delta_i / border)^2),
 * and check dt^2 vmax^2 (Lambda_max + max(m^2, 0)) < 4 with Lambda_max =
 * (2048/315) sum_d 1/h_d^2 (returns WFD_E_CFL otherwise).
 *   vel_dev           [nz][ny][nx] FP32 velocity, m/s (> 0), device;
 *   rho_dev_or_null   [nz][ny][nx] FP32 density (> 0) or NULL = constant density;
 *   model_dev, bytes  caller buffer of at least wfd_model_bytes(); it must stay
 *                     allocated and unmodified while the context uses the model.
 * vel and rho are read during this call only.  Waits on the stream once. */
wfd_status wfd_set_model(wfd_ctx *ctx, const wfd_grid *grid, const float *vel_dev,
                         const float *rho_dev_or_null, void *model_dev, size_t model_bytes);

/* Workspace bytes for one shot with nrec receivers: ckpt_or_null == NULL for
 * wfd_forward, else for wfd_gradient with that checkpoint policy. */
wfd_status wfd_workspace_bytes(const wfd_ctx *ctx, int32_t nrec, const wfd_ckpt *ckpt_or_null,
                               size_t *bytes);

/* Bytes of the host store that WFD_CKPT_HOST needs for the context's model:
 * nt pitched padded volumes of FP32 (nt * Nz * Ny * pitch * 4). */
wfd_status wfd_host_store_bytes(const wfd_ctx *ctx, size_t *bytes);

/* Forward modeling of one shot (Alg. 1 body; ModelingStep + ReadReceiver).
 *   wavelet_dev   [nt] FP32 source signature f(n dt), device;
 *   src_xyz       host [3] source position, m;
 *   nrec, rec_xyz host [nrec][3] receiver positions, m (nrec >= 0);
 *   seis_dev      [nrec][nt] FP32 output pressure traces, device (may be NULL
 *                 when nrec == 0);
 *   final_dev_or_null  [2][Nz][Ny][Nx] FP32 output: w^nt then w^(nt-1) on the
 *                 padded grid (q for variable density), device, or NULL;
 *   work_dev, work_bytes  workspace of at least wfd_workspace_bytes(NULL). */
wfd_status wfd_forward(wfd_ctx *ctx, const float *wavelet_dev, const double src_xyz[3],
                       int32_t nrec, const double *rec_xyz, float *seis_dev,
                       float *final_dev_or_null, void *work_dev, size_t work_bytes);

/* wfd_forward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation, bitwise, with the workspace taken from the library's
 * own static device array of WFD_NOALLOC_SCRATCH_BYTES instead of a caller
 * buffer.  Nothing is allocated.  The array is per GPU (each device that
 * loads the library holds one until the process ends) and shared by every
 * call on that GPU: calls that overlap on one GPU (several host threads, or
 * several streams in flight) race and must be serialised by the caller.  A
 * shot whose workspace (wfd_workspace_bytes with a NULL policy) exceeds the
 * array returns WFD_E_NOMEM before anything is launched.  Arguments as for
 * wfd_forward. */
#define WFD_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
wfd_status wfd_forward_noalloc(wfd_ctx *ctx, const float *wavelet_dev, const double src_xyz[3],
                               int32_t nrec, const double *rec_xyz, float *seis_dev,
                               float *final_dev_or_null);

/* Forward sweep of one shot and its misfit only (SeismicData::Misfit of
 * Alg. 3 without the backward sweep; line searches of the FWI loop need it):
 *   dobs_dev          [nrec][nt] FP32 observed traces, device;
 *   seis_or_null      [nrec][nt] FP32 output synthetic traces, or NULL;
 *   misfit_dev        device FP64 scalar, accumulated (+= 1/2 sum (d - d_obs)^2);
 *   work_dev, work_bytes  workspace of at least wfd_misfit_workspace_bytes(). */
wfd_status wfd_forward_misfit(wfd_ctx *ctx, const float *wavelet_dev, const double src_xyz[3],
                              int32_t nrec, const double *rec_xyz, const float *dobs_dev,
                              float *seis_or_null, double *misfit_dev, void *work_dev,
                              size_t work_bytes);

/* Workspace bytes of wfd_forward_misfit for nrec receivers. */
wfd_status wfd_misfit_workspace_bytes(const wfd_ctx *ctx, int32_t nrec, size_t *bytes);

/* Misfit and velocity gradient of one shot (Alg. 3 body for one shot).
 * With the CPML boundary WFD_CKPT_FULL keeps the layer's correction of every
 * step (on the shell of points the layer reaches) for the imaging condition;
 * WFD_CKPT_REVOLVE keeps the six memory variables with each checkpoint
 * (stored near the layer only: 4 W / N of a volume per axis, W = B + 8 for
 * a layer of B cells on an axis of N padded cells) and recomputes a visited step's
 * correction; WFD_CKPT_HOST returns WFD_E_ARG.  The steps:
 * forward sweep with recording and wavefield saving, res = d - d_obs,
 * J = 1/2 sum res^2, discrete adjoint sweep (exact transpose of the forward
 * recursion) with the zero-lag cross-correlation imaging condition, then
 * dJ/dv = 2 g / v with the sponge cells folded into the model-edge cells
 * they replicate.
 *   dobs_dev          [nrec][nt] FP32 observed traces, device;
 *   ckpt              forward-wavefield policy (non-NULL);
 *   seis_dev_or_null  [nrec][nt] FP32 output synthetic traces, or NULL;
 *   misfit_dev        device FP64 scalar, accumulated (+= J);
 *   grad_dev          [nz][ny][nx] FP32 device, accumulated (+= dJ/dv);
 *   illum_dev_or_null [nz][ny][nx] FP32 device, accumulated (+= sum_{n=1..nt}
 *                     (w^n)^2 on the model grid), or NULL. */
wfd_status wfd_gradient(wfd_ctx *ctx, const float *wavelet_dev, const double src_xyz[3],
                        int32_t nrec, const double *rec_xyz, const float *dobs_dev,
                        const wfd_ckpt *ckpt, float *seis_dev_or_null, double *misfit_dev,
                        float *grad_dev, float *illum_dev_or_null, void *work_dev,
                        size_t work_bytes);

/* Options of wfd_gradient_ex (a zeroed struct gives wfd_gradient's behaviour).
 *
 * Field scaling.  The step kernels carry every field times 2^e, an exact
 * power of two chosen per call on the device so that the source term
 * sigma max|f| 2^e lies in [1, 2) (sigma = dt^2 / (hx hy hz sqrt(rho_src)),
 * Eq. 1 source term; |e| <= 120).  The time stepping is linear in the field,
 * so the mantissas are those of an unscaled run, while a quiet source or a
 * coarse grid no longer drives FP32 products into the subnormal range.
 * Seismograms, final states and the misfit are returned in physical units.
 * The gradient and the illumination are quadratic in the source amplitude
 * and can lie below FP32's range on their own; they are returned times
 * 2^out_exp2 (exact). */
typedef struct {
  float *wavelet_grad_dev;  /* [nt] FP32 device, accumulated (+=) 2^out_exp2 dJ/df[n],
                               the gradient of the misfit with respect to wavelet
                               sample n (the transpose of the wavelet -> data map
                               applied to the residual: sigma psi^(n+1)[src] /
                               k_src), or NULL                                    */
  int32_t out_exp2;         /* grad_dev, illum_dev_or_null and wavelet_grad_dev
                               accumulate 2^out_exp2 times their quantity; 0 =
                               physical units; |out_exp2| <= 240 (else WFD_E_ARG) */
  int32_t *field_exp2_dev;  /* device int32 that receives the call's field
                               exponent e, or NULL                                */
} wfd_gradient_opts;

/* wfd_gradient with options (NULL = wfd_gradient).  With WFD_CKPT_HOST the
 * host store holds the scaled states 2^e w^m (e as in field_exp2_dev). */
wfd_status wfd_gradient_ex(wfd_ctx *ctx, const float *wavelet_dev, const double src_xyz[3],
                           int32_t nrec, const double *rec_xyz, const float *dobs_dev,
                           const wfd_ckpt *ckpt, float *seis_dev_or_null, double *misfit_dev,
                           float *grad_dev, float *illum_dev_or_null,
                           const wfd_gradient_opts *opts_or_null, void *work_dev,
                           size_t work_bytes);

/* ZeroesNearSurface (Alg. 3; zeroes_nplanes_gradient in §3): set the top
 * `zero_top_planes` z-planes of grad_dev [nz][ny][nx] to zero. */
wfd_status wfd_gradient_finish(wfd_ctx *ctx, float *grad_dev, int32_t zero_top_planes);

/* ---- launch tuning and batched shots ------------------------------------ */

/* Launch shapes of the context's step kernels: the GPU counterpart of the
 * paper's autotuning of the OpenMP chunk size of its time-step loop (PATSMA,
 * Alg. 1 and Alg. 3).  The choices are CDNA4 tiles and z chunkings:
 *   fwd_variant  forward tiles (rows per thread x wavefronts per block x
 *                64-column groups per thread):
 *                0: 2x8x1 = 64x16 tiles [default]  1: 2x16x1 = 64x32
 *                2: 2x4x1 = 64x8                     3: 4x4x1 = 64x16
 *                4: 1x16x3 = 192x16
 *   adj_variant  adjoint tiles: 0: 2x16x1 = 64x32 [default]
 *                1: 2x8x1 = 64x16 with a two-plane halo delay
 *                2: 2x4x1 = 64x8  3: 2x8x1 = 64x16, halo loaded one plane ahead
 *   *_rounds     z chunking aims at this many rounds of resident blocks per
 *                launch (at most 64); 0 = automatic: the chunk count that
 *                minimises a model of the launch time (rounds of resident
 *                blocks, a partly filled last round, z-halo re-reads).
 * Every shape computes bitwise the same result; only speed differs. */
typedef struct {
  int32_t fwd_variant, fwd_rounds;
  int32_t adj_variant, adj_rounds;
} wfd_tuning;

wfd_status wfd_set_tuning(wfd_ctx *ctx, const wfd_tuning *tuning);
wfd_status wfd_get_tuning(const wfd_ctx *ctx, wfd_tuning *tuning);

/* Time `steps` steps of every forward shape, then of every adjoint shape,
 * each with rounds in {0 (automatic), 2, 3, 4, 6, 8}, on the context's model (no source, no
 * receivers) with HIP events; keep the fastest in the context.
 *   work_dev, work_bytes  workspace of at least wfd_workspace_bytes(nrec = 0,
 *                 binomial checkpointing with 1 stored pair); overwritten;
 *   best_or_null  the chosen shapes;
 *   us_or_null    [2] microseconds per forward and per adjoint step.
 * Waits on the stream. */
wfd_status wfd_autotune(wfd_ctx *ctx, int32_t steps, void *work_dev, size_t work_bytes,
                        wfd_tuning *best_or_null, double *us_or_null);

/* A batch of shots whose forward sweeps (Alg. 1) run together: each time
 * step is ONE kernel launch over the tiles of every shot, so small grids
 * (windowed shots, a sub-volume per source) fill the device.  Each shot has
 * its own context (model on its own grid, e.g. the window around its source)
 * and its own workspace; results are bitwise those of wfd_forward on each
 * context.
 *   nshot            1..64;
 *   ctxs[i]          contexts with a model, all on one device and stream,
 *                    with equal nt and the same density mode (all constant
 *                    or all variable), each used once;
 *   wavelet_dev      [nt] FP32 source signature shared by all shots, device;
 *   src_xyz          host [nshot][3] source positions (in shot i's grid);
 *   nrec, rec_xyz    host per-shot receiver counts and [nrec[i]][3] arrays;
 *   seis_dev         per-shot [nrec[i]][nt] FP32 output traces, device;
 *   work_dev[i], work_bytes[i]  per-shot workspace of at least
 *                    wfd_workspace_bytes(ctxs[i], nrec[i], NULL), 256-byte
 *                    aligned; shot 0's also holds the batch's step
 *                    descriptors.
 * Receiver tables are built and uploaded here, so a run repeats the same
 * acquisition.  Contexts, models, wavelet, workspaces and outputs must stay
 * allocated until wfd_batch_destroy; shot 0's forward tile shape at creation
 * time is used for every shot (each shot keeps its own z chunking). */
typedef struct wfd_batch wfd_batch;
wfd_status wfd_batch_create(wfd_batch **batch, int32_t nshot, wfd_ctx *const *ctxs,
                            const float *wavelet_dev, const double *src_xyz,
                            const int32_t *nrec, const double *const *rec_xyz,
                            float *const *seis_dev, void *const *work_dev,
                            const size_t *work_bytes);

/* Enqueue the whole batch (clear states, nt steps, trace transposes) on the
 * stream.  use_graph != 0: the first call captures the sequence into a HIP
 * graph (the stream must not be the legacy NULL stream and profiling must be
 * off); every call launches that graph.  Asynchronous.  WFD_E_STATE if a
 * member context's model was set again after wfd_batch_create (the batch
 * holds the coefficient pointers of the model it was created with). */
wfd_status wfd_batch_run(wfd_batch *batch, int32_t use_graph);

/* Wait for the stream if a graph exists, release the batch (not the
 * caller's buffers).  NULL is accepted. */
wfd_status wfd_batch_destroy(wfd_batch *batch);

/* A batch of shots whose whole gradients (Alg. 3 body for each shot) run
 * together: every forward step and every adjoint step of the binomial
 * checkpointing schedule is ONE kernel launch over the tiles of every shot,
 * and the whole sequence can be captured once into a HIP graph.  The shots
 * share the schedule (equal nt and n_snapshots), so their stored states and
 * recomputations line up.  Each shot has its own context (model on its own
 * grid, e.g. the window around its source) and workspace; results are
 * bitwise those of wfd_gradient on each context with WFD_CKPT_REVOLVE and
 * n_snapshots pairs.
 *   nshot            1..64;
 *   ctxs[i]          contexts with a model on one device and stream, equal nt,
 *                    one density mode, sponge boundaries (no CPML), each used
 *                    once; shot 0's tile shapes (wfd_set_tuning) are used for
 *                    every shot;
 *   wavelet_dev      [nt] FP32 source signature shared by all shots;
 *   src_xyz          host [nshot][3]; nrec, rec_xyz per shot as in wfd_batch_create;
 *   dobs_dev[i]      [nrec[i]][nt] FP32 observed traces of shot i;
 *   n_snapshots      checkpoint pairs per shot (>= 1);
 *   misfit_dev[i]    device FP64 scalar, accumulated (+= J_i);
 *   grad_dev[i]      [nz][ny][nx] of shot i's grid, accumulated (+= dJ_i/dv);
 *   illum_dev_or_null  NULL, or per-shot [nz][ny][nx] accumulated illumination
 *                    (given for every shot or for none);
 *   work_dev[i], work_bytes[i]  per-shot workspace of at least
 *                    wfd_workspace_bytes(ctxs[i], nrec[i], REVOLVE n_snapshots),
 *                    256-byte aligned; shot 0's also holds the descriptors.
 * Receiver tables and scales are built here.  Everything must stay allocated
 * until wfd_gbatch_destroy; a context whose model is set again makes
 * wfd_gbatch_run return WFD_E_STATE. */
typedef struct wfd_gbatch wfd_gbatch;
wfd_status wfd_gbatch_create(wfd_gbatch **batch, int32_t nshot, wfd_ctx *const *ctxs,
                             const float *wavelet_dev, const double *src_xyz,
                             const int32_t *nrec, const double *const *rec_xyz,
                             const float *const *dobs_dev, int32_t n_snapshots,
                             double *const *misfit_dev, float *const *grad_dev,
                             float *const *illum_dev_or_null, void *const *work_dev,
                             const size_t *work_bytes);

/* Enqueue the batched gradients (as wfd_batch_run: use_graph != 0 captures the
 * sequence into a HIP graph on the first call and replays it). */
wfd_status wfd_gbatch_run(wfd_gbatch *batch, int32_t use_graph);

/* Wait for the stream if a graph exists and release the batch.  NULL is accepted. */
wfd_status wfd_gbatch_destroy(wfd_gbatch *batch);

/* ---- host-only helpers (no GPU needed) --------------------------------- */

/* Padded-grid node (ix, iy, iz) of a position in metres (rule above). */
wfd_status wfd_map_position(const wfd_grid *grid, const double xyz[3], int32_t ijk[3]);

/* Stability ratio dt^2 vmax^2 (Lambda_max + max(m2max, 0)) / 4; the scheme is
 * stable when the ratio is below 1 (ValidConditions, §2.2). */
wfd_status wfd_cfl_ratio(const wfd_grid *grid, double vmax, double m2max, double *ratio);

/* Checkpoint schedule for reversing nt steps with n_snapshots stored pairs
 * (plus the zero initial state, which needs no storage).  Actions are
 * written as int32 triples (op, a, b):
 *   op 0 ADVANCE  a = from state, b = to state    (b - a forward steps)
 *   op 1 STORE    a = state,      b = slot
 *   op 2 VISIT    a = state (the backward sweep consumes w^a)
 *   op 3 FREE     a = state,      b = slot
 * Visits run a = nt down to 1.  The forward-step count is minimal
 * (Griewank & Walther binomial bound).  actions may be NULL to query sizes. */
wfd_status wfd_checkpoint_plan(int32_t nt, int32_t n_snapshots, int32_t *actions,
                               int64_t capacity, int64_t *n_actions, int64_t *n_forward_steps);

/* ---- learned gradient preconditioner (BF16 3-D CNN) ----------------------
 *
 * Replaces the paper's fixed gradient smoothing (GradientPreconditioning,
 * Bessel or Laplace filters) by a small network of 3 x 3 x 3 convolutions
 * with "same" zero padding: 2 -> 16 -> 16 -> 16 -> 1 channels, ReLU after the
 * first three, and the first input channel added to the output.  Stateless calls on device buffers, enqueued on `stream` (a
 * hipStream_t, NULL = legacy default stream) on the current device.
 *
 * Layouts: BF16 values are passed as uint16_t bit patterns.  Volumes are
 * channels-last [nz][ny][nx][C].  Master weights are FP32 W[27][cin][cout]
 * with tap = 9 kz + 3 ky + kx reading the input at (z + kz - 1, y + ky - 1,
 * x + kx - 1).  Convolutions take weights packed for the matrix cores by
 * wfd_cnn_pack_weights.  All buffers are caller-owned; no call allocates.
 * Supported layers: (cin, cout) = (2, 16), (16, 16), (16, 1). */

#define WFD_CNN_REDUCE_BYTES 8192  /* workspace of wfd_cnn_mse / wfd_cnn_pack_input */

/* Number of uint16_t of a packed weight matrix: flip = 0 for the forward
 * convolution, 1 for the data-gradient convolution of the same layer. */
wfd_status wfd_cnn_packed_elems(int32_t cin, int32_t cout, int32_t flip, int64_t *elems);

/* Pack FP32 master weights w[27][cin][cout] into BF16 matrix-core operands:
 *   flip = 0: A[16][K], A[co][tap * cin + ci] = bf16(w[tap][ci][co]);
 *   flip = 1: A[16][K], A[ci][tap * cout + co] = bf16(w[26 - tap][ci][co])
 * (rounded to nearest even; rows and columns past the layer are zero). */
wfd_status wfd_cnn_pack_weights(const float *w_dev, int32_t cin, int32_t cout, int32_t flip,
                                uint16_t *packed_dev, void *stream);

/* out[p][co] = sum_{tap, ci} in[p + offset(tap)][ci] * A[co][tap * cin + ci]
 * (+ bias[co]), then max(., 0) if relu, then 0 where mask[p][co] <= 0 if a
 * mask is given, then (cout = 1 only) + residual[p][0] of a BF16
 * residual[p][residual_channels] if given; BF16 products, FP32 sums.  With the flip-packed weights of a
 * layer (cin, cout) this is the data gradient of that layer: call it with
 * cin' = cout and cout' = cin.  (cin, cout) in {(2,16), (16,16), (16,1),
 * (1,16)}.  Written as BF16 (rounded to nearest even) and/or FP32
 * channels-last; in, packed and outputs 16-byte aligned, a 16-channel mask
 * 8-byte aligned.  WFD_E_ARG for another layer shape, an empty volume, an
 * x-y plane of more than 2^24 voxels, a misaligned or missing buffer, or a
 * residual with more than one output or outside 1 to 16 channels. */
wfd_status wfd_cnn_conv(const uint16_t *in_dev, int32_t nx, int32_t ny, int32_t nz, int32_t cin,
                        int32_t cout, const uint16_t *packed_dev, const float *bias_or_null,
                        int32_t relu, const uint16_t *mask_or_null,
                        const uint16_t *residual_or_null, int32_t residual_channels,
                        uint16_t *out_bf16_or_null, float *out_f32_or_null, void *stream);

/* Workspace of wfd_cnn_wgrad for an nx x ny x nz volume. */
wfd_status wfd_cnn_wgrad_workspace_bytes(int32_t nx, int32_t ny, int32_t nz, size_t *bytes);

/* Weight and bias gradients of layer (cin, cout) from its input `in` and the
 * gradient dz of its output (before the layer's ReLU, i.e. already masked):
 *   dw[tap][ci][co] = sum_p in[p + offset(tap)][ci] dz[p][co]   (FP32, written)
 *   db[co] = sum_p dz[p][co]                                     (if non-NULL)
 * BF16 products, FP32 sums in a fixed order (deterministic).  in and (for
 * 16 output channels) dz 16-byte aligned; work (device, caller-owned) at
 * least wfd_cnn_wgrad_workspace_bytes, else WFD_E_NOMEM.  An x-y plane holds
 * at most 2^24 voxels (WFD_E_ARG otherwise). */
wfd_status wfd_cnn_wgrad(const uint16_t *in_dev, const uint16_t *dz_dev, int32_t nx, int32_t ny,
                         int32_t nz, int32_t cin, int32_t cout, float *dw_dev,
                         float *db_dev_or_null, void *work_dev, size_t work_bytes, void *stream);

/* Mean squared error of y against t (n FP32 values each): loss_dev (FP64
 * scalar, written) = mean((y - t)^2), dy_dev = bf16(2 (y - t) / n). */
wfd_status wfd_cnn_mse(const float *y_dev, const float *t_dev, int64_t n, uint16_t *dy_dev,
                       double *loss_dev, void *work_dev, size_t work_bytes, void *stream);

/* One Adam step (Kingma & Ba 2015) on n FP32 parameters; step counts from 1. */
wfd_status wfd_cnn_adam(float *w_dev, const float *g_dev, float *m_dev, float *v_dev, int32_t n,
                        float lr, float beta1, float beta2, float eps, int32_t step,
                        void *stream);

/* Network input [n][2]: c = grad / (illum + eps max|illum|) (the plain
 * illumination-compensated gradient) scaled by max|c|, and illum scaled by
 * max|illum|, both rounded to BF16; a channel whose maximum is 0 is left
 * unscaled (with max|illum| = 0, c = grad).  eps > 0. */
wfd_status wfd_cnn_pack_input(const float *grad_dev, const float *illum_dev, int64_t n, float eps,
                              uint16_t *out_dev, void *work_dev, size_t work_bytes, void *stream);

/* ---- gradient smoothing (GradientPreconditioning, §2.2) --------------------
 *
 * The paper smooths every gradient with a Bessel or a Laplace filter of
 * lengths l_x, l_y, l_z (default twice the spacing).  Readings:
 *   WFD_SMOOTH_LAPLACE  separable exponential kernel: along x, then y, then
 *                       z, u = T^-1 g with T = [(1 + a^2) I - a (S + S^-1)]
 *                       / (1 - a)^2, a = exp(-h / l), zero-flux (mirror) ends;
 *                       its interior impulse response is (1-a)/(1+a) a^|n|;
 *   WFD_SMOOTH_BESSEL   u = B^-1 g, B = I - sum_d l_d^2 D_dd with 3-point
 *                       second differences and zero-flux ends (a K_1/2 Bessel
 *                       kernel), by conjugate gradients to a relative residual
 *                       tol (at most max_iter iterations; WFD_E_RANGE if not
 *                       reached).
 * Both keep constants.  A length of 0 leaves that axis unsmoothed (Laplace)
 * or drops its term (Bessel). */
enum { WFD_SMOOTH_LAPLACE = 1, WFD_SMOOTH_BESSEL = 2 };

/* Workspace bytes of wfd_smooth. */
wfd_status wfd_smooth_workspace_bytes(int32_t mode, int32_t nx, int32_t ny, int32_t nz,
                                      size_t *bytes);

/* Smooth in_dev [nz][ny][nx] FP32 into out_dev (may equal in_dev for the
 * Laplace filter; must differ for Bessel).  lengths and spacing are (x, y, z)
 * in metres.  Enqueued on `stream` (a hipStream_t); returns after the stream
 * has drained (the Bessel solver reads its inner products on the host).
 * iterations_or_null receives the conjugate-gradient iteration count. */
wfd_status wfd_smooth(int32_t mode, const float *in_dev, float *out_dev, int32_t nx, int32_t ny,
                      int32_t nz, const double lengths[3], const double spacing[3], double tol,
                      int32_t max_iter, void *work_dev, size_t work_bytes,
                      int32_t *iterations_or_null, void *stream);

/* ---- time resampling of seismic data (§2.1) ---------------------------------
 * Traces [nrec][nt] with sample k at time (k + 1) dt (the trace convention of
 * wfd_forward).  WFD_RESAMPLE_NEAREST: out[m] = in[n] with n = round-half-up
 * (t_m / dt_in) - 1 clamped to the trace; WFD_RESAMPLE_SINC: out[m] =
 * sum_n in[n] sinc((t_m - t_n) / dt_in) over the whole trace (FP64 sums).
 * in and out are distinct device buffers; enqueued on `stream`. */
enum { WFD_RESAMPLE_NEAREST = 1, WFD_RESAMPLE_SINC = 2 };
wfd_status wfd_resample(int32_t mode, const float *in_dev, int32_t nrec, int32_t nt_in,
                        double dt_in, float *out_dev, int32_t nt_out, double dt_out,
                        void *stream);

/* ---- measurement ---------------------------------------------------------- */

enum {
  WFD_K_FORWARD = 0,   /* forward step (fd_step, incl. source + receivers)     */
  WFD_K_ADJOINT = 1,   /* adjoint step fused with imaging                       */
  WFD_K_OTHER = 2,     /* setup, misfit, copies, gradient finish                */
  WFD_K_COUNT = 3
};

/* Enable (1) or disable (0) per-launch HIP-event timing on the context's
 * stream; enabling clears the counters. */
wfd_status wfd_set_profiling(wfd_ctx *ctx, int32_t enable);

/* Launch count and summed kernel time (ms) of one kernel class since
 * profiling was enabled.  Waits for the stream. */
wfd_status wfd_kernel_stats(wfd_ctx *ctx, int32_t kernel_class, int64_t *launches, double *total_ms);

/* Thread-local text of the last error ("" if none). */
const char *wfd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* WFD_H */
