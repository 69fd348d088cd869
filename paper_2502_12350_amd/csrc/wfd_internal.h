// Internal interfaces between the host orchestrator (wfd_api.cpp) and the
// HIP kernels (wfd_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wfd.h"

namespace wfd {

// Context queries and the thread-local error text, for the library's other
// translation units (wfd_api.cpp owns both).
int ctx_device(const wfd_ctx *c);
wfd_status set_error(wfd_status status, const char *message);

// Padded-grid geometry and coefficient volumes seen by every step kernel.
// Volumes are [Nz][Ny][pitch] FP32 with pitch >= Nx (rows 256-byte aligned).
struct StepGrid {
  int nx, ny, nz;        // padded extents Nx, Ny, Nz
  int pitch;             // floats per row
  int64_t plane;         // pitch * Ny
  float cx, cy, cz;      // 1 / h^2 per axis
  const float *gx, *gy, *gz;  // 1-D sponge tables
  const float *k;        // dt^2 v^2
  const float *m2;       // mass term (variable density) or nullptr
  int zs;                // free-surface plane (planes above read as its negated
                         // mirror, planes at and above it stay zero), or
                         // kNoSurface, below every plane a kernel touches
};
constexpr int kNoSurface = -(1 << 24);

// Receivers grouped by (y, x) column of the padded grid.  Entry e is one
// distinct receiver node at depth ent_z[e]; the receivers sharing it are
// perm[ent_rp[e] .. ent_rp[e+1]).  col_start has Ny*Nx + 1 entries.
struct RecTable {
  const int *col_start;
  const int *ent_z;
  const int *ent_rp;
  const int *perm;
  int nrec;
};

// Per-shot scales, computed on the device from the wavelet (no host sync).
// The step kernels carry the field times 2^e, an exact power of two chosen so
// that the source term sigma max|f| 2^e lies in [1, 2): the fields stay far
// from FP32's subnormal range whatever the source amplitude and grid spacing.
// Every operation of the time stepping is linear in the field, so the scaled
// run has bitwise the mantissas of the unscaled one; recordings, final states,
// the gradient and the illumination undo the factor on output.
struct ShotScale {
  float sigma;       // injection factor sigma 2^e (first member: Source::sigma)
  float sigma_phys;  // sigma = dt^2 / (hx hy hz sqrt(rho_src))
  int e;             // field exponent
  int pad;
};
constexpr int kMaxFieldExp = 120;  // |e| bound: 2^-120 sqrt(rho) stays a normal FP32

// Source: padded node (linear index into a pitched volume), device scalar
// sigma 2^e (the first member of the shot's ShotScale) and the wavelet.
struct Source {
  int64_t idx;
  const float *sigma;
  const float *wavelet;
};

// How a step kernel's blocks cover a grid: 64-wide tiles of `ty` rows,
// z split into nchunks chunks of zc planes.
struct TileMap {
  int tiles_x, tiles_y, nchunks, zc, nblocks;
};

// Step-kernel tuning.  Tile shapes (rows per thread x wavefronts per block
// x 64-column groups per thread):
//   forward  0: 2x8x1 (64x16 tiles)  1: 2x16x1 (64x32)  2: 2x4x1 (64x8)
//            3: 4x4x1 (64x16)        4: 1x16x3 (192x16)
//   adjoint  0: 2x16x1 (64x32)       1: 2x8x1 (64x16, 2-plane halo delay)
//            2: 2x4x1 (64x8)         3: 2x8x1 (64x16, halo one plane ahead)
// and the number of rounds of resident blocks the z chunking aims for
// (0 = chosen by the launch cost model).  Every shape computes bitwise the
// same values.
constexpr int kFwdVariants = 5, kAdjVariants = 4;
struct Tuning {
  int variant = 0;
  int rounds = 0;
  int adj_variant = 0;
  int adj_rounds = 0;
};

// One shot's forward step inside a multi-window launch.
struct WindowStep {
  StepGrid g;
  TileMap map;
  const float *cur;
  const float *prev;
  float *out;
  Source src;
  RecTable rec;
  const float *rec_scale;
  float *seis_tm;
  int block_begin, block_end;
};

// Illumination output of the adjoint step: illum[model cell] += 2^(out_exp2 -
// 2 e) (w^m)^2 with e from the shot's scale (the field kernels carry 2^e w).
struct IllumOut {
  float *p;  // [mnz][mny][mnx] or nullptr
  int border, mnx, mny, mnz;
  const ShotScale *sc;
  int out_exp2;
};

// One shot of a batched gradient (wfd_gbatch): its grid, tile maps of the
// forward and adjoint launches, source, receivers, and the buffers.  The
// forward states live in a pool: W1, W2, then the checkpoint store; every
// shot uses the same pool indices at every step (one plan for all shots).
struct GradWindow {
  StepGrid g;
  TileMap fmap, amap;
  Source src;
  RecTable rec;
  const float *rec_scale;
  float *seis_tm;        // [nt][nrec] recorded traces
  const float *res_tm;   // [nt][nrec] scaled residuals
  float *W1, *W2, *store;
  int64_t vol;           // floats per pitched volume
  float *P1, *P2, *gimg;  // adjoint pair and imaging sum
  IllumOut il;
  int fblock_begin, fblock_end, ablock_begin, ablock_end;
};

// Kernel launchers; all enqueue on `stream` and return the launch status.
hipError_t launch_forward_step(const StepGrid &g, const float *cur, const float *prev, float *out,
                               const Source &src, int n, const RecTable *rec,
                               const float *rec_scale, float *seis_tm, const Tuning &tu,
                               hipStream_t stream);

// z chunks at least this deep: single launches, and batches of several shots
// (whose windows fill the device together).
constexpr int kSingleMinZc = 4, kBatchMinZc = 16;

// Blocks of one window's share of a batched forward launch over g with tuning
// tu, z chunks at least min_zc planes deep (and its tile map).
int forward_tile_map(const StepGrid &g, const Tuning &tu, int min_zc, TileMap *map);

// One step of every window in wins[0..nwin) (device array), nblocks blocks.
// fs: some window has a free surface (selects the kernels with image loads).
hipError_t launch_forward_multi(const WindowStep *wins, int nwin, int nblocks, int n, int variant,
                                bool vd, bool fs, hipStream_t stream);

hipError_t launch_adjoint_step(const Tuning &tu, const StepGrid &g, const float *cur,
                               const float *prev, float *out,
                               const RecTable &rec, const float *res_tm, int m,
                               const float *wm, float *grad, const IllumOut &illum,
                               hipStream_t stream);

// Blocks of one window's share of a batched adjoint launch over g with
// tuning tu, z chunks at least min_zc planes deep (and its tile map).
int adjoint_tile_map(const StepGrid &g, const Tuning &tu, bool illum, int min_zc, TileMap *map);

// Batched gradient: one forward step of every window (pool buffers cur_k,
// prev_k -> out_k; receivers recorded when record != 0), and one adjoint step
// of every window (psi^{m+1} in P1 for parity 0 else P2; w^m = pool buffer
// wm_k).  variant / adj_variant: the tile shapes of the windows' maps.
hipError_t launch_forward_pool(const GradWindow *wins, int nwin, int nblocks, int n, int cur_k,
                               int prev_k, int out_k, int record, int variant, bool vd, bool fs,
                               hipStream_t stream);
hipError_t launch_adjoint_multi(const GradWindow *wins, int nwin, int nblocks, int m, int parity,
                                int wm_k, int adj_variant, bool vd, bool illum, bool fs,
                                hipStream_t stream);

// Model preparation.
hipError_t launch_precompute_k(const float *vel, int mnx, int mny, int mnz, int border, double dt,
                               float *k, int pitch, int ny, int nz, float *partial_max,
                               int n_partial, hipStream_t stream);
hipError_t launch_precompute_m2(const float *rho, int mnx, int mny, int mnz, int border,
                                int free_surface, double idx2, double idy2, double idz2,
                                float *m2, int pitch, int ny, int nz, float *sqrt_rho,
                                float *partial_max, int n_partial, hipStream_t stream);

// Per-shot scales: the ShotScale (sigma, field exponent e from max|wavelet|)
// and per-receiver recording scales sqrt(rho_r) 2^-e (physical pressure out
// of the scaled field) and adjoint injection scales k_r sqrt(rho_r) (the
// residual kernel applies 2^e).
hipError_t launch_shot_setup(const float *k, const float *sqrt_rho, int64_t src_idx,
                             int src_model_idx, double dt2_over_h3, const float *wavelet, int nt,
                             const int64_t *rec_idx, const int *rec_model_idx, int nrec,
                             ShotScale *sc, float *rec_scale, float *rec_adj, hipStream_t stream);

// dst[z][y][x] (dense Nz x Ny x Nx) = 2^-e src[z][y][pitch x]: a field of the
// step kernels in physical units.
hipError_t launch_unscale_copy(const float *src, float *dst, int nx, int ny, int nz, int pitch,
                               const ShotScale *sc, hipStream_t stream);

// wg[m - 1] += 2^(out_exp2 - e) sigma psi[src_idx] / k[src_idx]: sample m - 1
// of the misfit's gradient with respect to the wavelet, from the adjoint
// state psi^m of the step that was just taken.
hipError_t launch_source_gradient(const float *psi, const float *k, int64_t src_idx,
                                  const ShotScale *sc, int out_exp2, int m, float *wg,
                                  hipStream_t stream);

// Residual + misfit: res_tm[n][r] = 2^e adj[r] (seis_tm[n][r] - dobs[r][n]),
// partial[b] = 1/2 sum (seis - dobs)^2 (FP64) per block; then misfit += sum partial.
hipError_t launch_residual(const float *seis_tm, const float *dobs, const float *rec_adj,
                           const ShotScale *sc, int nrec, int nt, float *res_tm, double *partial,
                           int *n_partial, hipStream_t stream);
int residual_partial_count(int nrec, int nt);
hipError_t launch_sum_partials(const double *partial, int n, double *misfit, hipStream_t stream);

// [nt][nrec] -> [nrec][nt]
hipError_t launch_transpose(const float *src_tm, float *dst_rm, int nrec, int nt,
                            hipStream_t stream);

// grad[m] += 2^(out_exp2 - 2 e) 2 / v * sum of g over the padded cells that
// replicate model cell m (g carries the factor 2^(2 e) of the two scaled
// fields it correlates).
hipError_t launch_grad_fold(const float *g, const float *k, int pitch, int pny, int border,
                            int mnx, int mny, int mnz, double dt, const ShotScale *sc,
                            int out_exp2, float *grad, hipStream_t stream);

hipError_t launch_fill_zero(float *p, int64_t n, hipStream_t stream);

// ---- CNN preconditioner kernels (wfd_cnn.hip) ----
// BF16 values travel as uint16_t bit patterns.
int cnn_conv_blocks(int nx, int ny, int nz);
int cnn_wgrad_blocks(int nx, int ny, int nz);
size_t cnn_wgrad_workspace_floats(int nx, int ny, int nz);
constexpr int kCnnReduceBlocks = 512;  // partials of the loss and input-scale reductions
hipError_t launch_conv(int cin, int cout, const uint16_t *in, int nx, int ny, int nz,
                       const uint16_t *apk, const float *bias, int relu, const uint16_t *mask,
                       const uint16_t *res, int res_c, uint16_t *out_bf, float *out_f,
                       hipStream_t stream);
hipError_t launch_wgrad(int cin, int cout, const uint16_t *in, const uint16_t *dz, int nx, int ny,
                        int nz, float *work, float *dw, float *db, hipStream_t stream);
hipError_t launch_pack_weights(const float *w, int cin, int cout, int flip, uint16_t *apk,
                               hipStream_t stream);
hipError_t launch_mse(const float *y, const float *t, int64_t n, uint16_t *dy, double *partial,
                      int npart, double *loss, hipStream_t stream);
hipError_t launch_adam(float *w, const float *g, float *m, float *v, int n, float lr, float b1,
                       float b2, float eps, int step, hipStream_t stream);
hipError_t launch_pack_input(const float *grad, const float *illum, int64_t n, float eps,
                             float *partial, int npart, uint16_t *out, hipStream_t stream);

// ---- gradient smoothing kernels (wfd_smooth.hip) ----
hipError_t launch_tri_lines(float *u, int axis, int n, int64_t nlines, int nx, int ny,
                            const double *cp, const double *inv_den, double a, double scale,
                            hipStream_t stream);
hipError_t launch_bessel_apply(const float *x, float *y, int nx, int ny, int nz, float cx,
                               float cy, float cz, double *part, int npart, hipStream_t stream);
hipError_t launch_cg_update(float *x, float *r, const float *p, const float *ap, int64_t n,
                            float alpha, double *part, int npart, hipStream_t stream);
hipError_t launch_cg_direction(float *p, const float *r, int64_t n, float beta, int npart,
                               hipStream_t stream);
hipError_t launch_cg_start(const float *g, float *r, float *x, int64_t n, double *part, int npart,
                           hipStream_t stream);
hipError_t launch_resample(const float *in, int nrec, int nt_in, double dt_in, float *out,
                           int nt_out, double dt_out, int sinc, hipStream_t stream);

// ---- CPML absorbing layer (wfd_cpml.hip) ----
constexpr int kStencilRadius = 4;  // reach of the eighth-order differences
// Recursive-convolution coefficients a, b per padded index of each axis.
struct CpmlTables {
  const float *ax, *bx, *ay, *by, *az, *bz;
  float ihx, ihy, ihz;  // 1 / h per axis
  // Compact memory variables (layout in wfd_cpml.hip): per axis x, y, z the
  // slab width W (cells [0, W) and [N - W, N) are stored) and the stored
  // length L of the axis (2 W, or N when the two slabs would meet).
  int half[3], len[3];
};
// Stored slab width of an axis of N padded cells with a layer of B cells: the
// layer plus the 8 cells that points within reach of it (4) see through their
// own reach (4), so every memory-variable read of the layer kernels lands in
// the slab; the whole axis when the two slabs would meet.
inline int cpml_slab_half(int N, int B) { return 2 * (B + 8) >= N ? N : B + 8; }
inline int cpml_slab_len(int N, int B) { return 2 * (B + 8) >= N ? N : 2 * (B + 8); }
// Floats of one compact memory variable of axis d (0, 1, 2 = x, y, z).
inline int64_t cpml_mem_len(int d, int Nx, int Ny, int Nz, int B) {
  return d == 0   ? (int64_t)Nz * Ny * cpml_slab_len(Nx, B)
         : d == 1 ? (int64_t)Nz * cpml_slab_len(Ny, B) * Nx
                  : (int64_t)cpml_slab_len(Nz, B) * Ny * Nx;
}
// The points the layer's terms reach: the padded grid minus the inner box
// more than 4 cells from every layer, as up to 6 boxes [lo, hi) in (z, y, x).
// Point q of the shell lies in the box b with start[b] <= q < start[b + 1],
// at offset q - start[b] in x-fastest order, then the box's thinner of z and
// y (so the z or y neighbours of a row are a few rows away and stay in L2);
// every box holds fewer than 2^31 points.  lo/hi are the inner box (inclusive) per axis x, y, z: a point
// outside [lo, hi] along an axis is within reach of that axis' layer.
constexpr int kShellBoxes = 6;
struct Shell {
  int nbox;
  int z0[kShellBoxes], z1[kShellBoxes], y0[kShellBoxes], y1[kShellBoxes];
  int x0[kShellBoxes], x1[kShellBoxes];
  int64_t start[kShellBoxes + 1];
  int zfirst[kShellBoxes];  // 1: order x, z, y (z before y), for boxes thin in z
  int lo[3], hi[3];
  // Column marching: a block of 64 x 4 threads owns one (x, y) tile of a box
  // and marches a chunk of cz planes; tx, ty, nch tile counts per box, bstart
  // the first block of each box, zq whether the box reaches z-derivative terms
  // (then each thread keeps nine-plane queues along z and the chunks are long,
  // kShellChunkZ; other boxes take short chunks, kShellChunk, for parallelism).
  int tx[kShellBoxes], ty[kShellBoxes], nch[kShellBoxes], zq[kShellBoxes], cz[kShellBoxes];
  int64_t bstart[kShellBoxes + 1];
};
constexpr int kShellTileX = 64, kShellTileY = 4, kShellChunkZ = 16, kShellChunk = 8;
// Forward: psi_d = b psi_d + a D1_d w (cur) on the layer.
hipError_t launch_cpml_psi(const StepGrid &g, const CpmlTables &t, const Shell &sh,
                           const float *cur, float *psi_x, float *psi_y, float *psi_z,
                           hipStream_t stream);
// Forward: zeta_d = b zeta_d + a (D2_d w + D1_d psi_d) on the layer; C = sum_d
// (D1_d psi_d + zeta_d); out += k C below the free surface; C to cstore[q]
// when cstore is given.
hipError_t launch_cpml_zeta(const StepGrid &g, const CpmlTables &t, const Shell &sh,
                            const float *cur, const float *psi_x, const float *psi_y,
                            const float *psi_z, float *zeta_x, float *zeta_y, float *zeta_z,
                            float *out, float *cstore, hipStream_t stream);
// Adjoint: nu_d = phi1 + b nu_d on the layer.
hipError_t launch_cpml_nu(const StepGrid &g, const CpmlTables &t, const Shell &sh,
                          const float *phi1, float *nu_x, float *nu_y, float *nu_z,
                          hipStream_t stream);
// Adjoint: mu_d = b mu_d - D1_d (a nu_d + phi1) on the layer.
hipError_t launch_cpml_mu(const StepGrid &g, const CpmlTables &t, const Shell &sh,
                          const float *phi1, const float *nu_x, const float *nu_y,
                          const float *nu_z, float *mu_x, float *mu_y, float *mu_z,
                          hipStream_t stream);
// Adjoint: phi += k sum_d [D2_d (a nu_d) - D1_d (a mu_d)] below the free
// surface; g += phi1 C (C from cstore) when cstore is given.
hipError_t launch_cpml_adjoint(const StepGrid &g, const CpmlTables &t, const Shell &sh,
                               const float *nu_x, const float *nu_y, const float *nu_z,
                               const float *mu_x, const float *mu_y, const float *mu_z,
                               float *phi, const float *phi1, const float *cstore, float *grad,
                               hipStream_t stream);
// seis_tm[n][r] = scale[r] field[idx[r]] (receivers read after the layer's
// correction).
hipError_t launch_record(const float *field, const int64_t *idx, const float *scale, int nrec,
                         int n, float *seis_tm, hipStream_t stream);

}  // namespace wfd
