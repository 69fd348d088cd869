// HIP kernels for gfx950 (MI355X) around the step kernels (wfd_step.hip):
// model preparation (Eq. 1 coefficients, in FP64 where it matters), per-shot
// source / receiver scales with the field's power-of-two exponent, the misfit
// with a deterministic FP64 reduction (Alg. 3, SeismicData::Misfit),
// seismogram transposes and the gradient finish (chain rule to dJ/dv with the
// sponge fold).
//
// Block reductions run as a butterfly of cross-lane shuffles inside each
// 64-lane wavefront (every lane ends with the same value, since a + b and
// b + a round alike), then over the four wavefront results in a fixed order:
// the result does not depend on scheduling.
#include "wfd_internal.h"

namespace wfd {
namespace {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

constexpr int kBlock = 256;                 // threads of every reducing block
constexpr int kWaves = kBlock / 64;

template <class T, class Op>
__device__ __forceinline__ T wave_reduce(T v, Op op) {
  for (int o = 32; o > 0; o >>= 1) v = op(v, __shfl_xor(v, o, 64));
  return v;
}

// Reduction over a 256-thread block, returned to every thread; t is the
// thread's linear index in the block.
template <class T, class Op>
__device__ __forceinline__ T block_reduce(T v, Op op, int t) {
  __shared__ T part[kWaves];
  v = wave_reduce(v, op);
  if ((t & 63) == 0) part[t >> 6] = v;
  __syncthreads();
  T r = part[0];
  for (int w = 1; w < kWaves; ++w) r = op(r, part[w]);
  return r;
}

struct MaxOp {
  __device__ float operator()(float a, float b) const { return fmaxf(a, b); }
};
struct SumOp {
  __device__ double operator()(double a, double b) const { return a + b; }
};

// k = dt^2 v^2 over the padded grid (v edge-replicated); per-block max of v.
__global__ void __launch_bounds__(256)
    k_precompute_k(const float *__restrict__ vel, int mnx, int mny, int mnz, int border, double dt,
                   float *__restrict__ k, int pitch, int ny, int nz, float *__restrict__ part) {
  const int nx = mnx + 2 * border;
  const int64_t total = (int64_t)nx * ny * nz;
  float vmax = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % nx);
    const int y = (int)((i / nx) % ny);
    const int z = (int)(i / ((int64_t)nx * ny));
    const int mx = clampi(x - border, 0, mnx - 1);
    const int my = clampi(y - border, 0, mny - 1);
    const int mz = clampi(z - border, 0, mnz - 1);
    const double v = vel[((int64_t)mz * mny + my) * mnx + mx];
    k[(int64_t)z * pitch * ny + (int64_t)y * pitch + x] = (float)(dt * dt * v * v);
    vmax = fmaxf(vmax, (float)v);
  }
  const float r = block_reduce(vmax, MaxOp(), threadIdx.x);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

// sqrt(rho) at model node (x, y, z), edge-replicated beyond the model; with a
// free surface, mirrored evenly about the top plane first.
__device__ __forceinline__ double sqrt_rho_at(const float *rho, int mnx, int mny, int mnz,
                                              int x, int y, int z, bool fs) {
  if (fs && z < 0) z = -z;
  const int mx = clampi(x, 0, mnx - 1), my = clampi(y, 0, mny - 1), mz = clampi(z, 0, mnz - 1);
  return sqrt((double)rho[((int64_t)mz * mny + my) * mnx + mx]);
}

// m^2 = L8(s) / s with s = sqrt(rho) edge-replicated beyond the model, mirrored
// evenly above a free surface (FP64);
// also s on the model grid for source / receiver scales; per-block max m^2.
__global__ void __launch_bounds__(256)
    k_precompute_m2(const float *__restrict__ rho, int mnx, int mny, int mnz, int border, int fs,
                    double idx2, double idy2, double idz2, float *__restrict__ m2, int pitch,
                    int ny, int nz, float *__restrict__ sqrt_rho, float *__restrict__ part) {
  const int nx = mnx + 2 * border;
  const int64_t total = (int64_t)nx * ny * nz;
  const double w[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};
  float mmax = -3.0e38f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % nx);
    const int y = (int)((i / nx) % ny);
    const int z = (int)(i / ((int64_t)nx * ny));
    const int mx = x - border, my = y - border, mz = z - border;
    const double s = sqrt_rho_at(rho, mnx, mny, mnz, mx, my, mz, fs != 0);
    double lx = w[0] * s, ly = w[0] * s, lz = w[0] * s;
    for (int j = 1; j <= 4; ++j) {
      lx += w[j] * (sqrt_rho_at(rho, mnx, mny, mnz, mx + j, my, mz, fs != 0) +
                    sqrt_rho_at(rho, mnx, mny, mnz, mx - j, my, mz, fs != 0));
      ly += w[j] * (sqrt_rho_at(rho, mnx, mny, mnz, mx, my + j, mz, fs != 0) +
                    sqrt_rho_at(rho, mnx, mny, mnz, mx, my - j, mz, fs != 0));
      lz += w[j] * (sqrt_rho_at(rho, mnx, mny, mnz, mx, my, mz + j, fs != 0) +
                    sqrt_rho_at(rho, mnx, mny, mnz, mx, my, mz - j, fs != 0));
    }
    const double val = (lx * idx2 + ly * idy2 + lz * idz2) / s;
    m2[(int64_t)z * pitch * ny + (int64_t)y * pitch + x] = (float)val;
    mmax = fmaxf(mmax, (float)val);
    if (mx >= 0 && mx < mnx && my >= 0 && my < mny && mz >= 0 && mz < mnz)
      sqrt_rho[((int64_t)mz * mny + my) * mnx + mx] = (float)s;
  }
  const float r = block_reduce(mmax, MaxOp(), threadIdx.x);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

// Field exponent e of a source term of size x = sigma max|f|: x 2^e in [1, 2),
// clamped to [-kMaxFieldExp, kMaxFieldExp]; 0 for a silent (or non-finite) source.
__device__ __forceinline__ int field_exponent(double x) {
  if (!(x > 0.0) || !(x < 1.0e300)) return 0;
  const int e = -ilogb(x);
  return e < -kMaxFieldExp ? -kMaxFieldExp : (e > kMaxFieldExp ? kMaxFieldExp : e);
}

// Every block reduces max|f| itself (nt values), so that all of them take the
// same exponent without a second launch.
__global__ void __launch_bounds__(256)
    k_shot_setup(const float *__restrict__ k, const float *__restrict__ sqrt_rho, int64_t src_idx,
                 int src_model_idx, double dt2_over_h3, const float *__restrict__ wavelet, int nt,
                 const int64_t *__restrict__ rec_idx, const int *__restrict__ rec_model_idx,
                 int nrec, ShotScale *__restrict__ sc, float *__restrict__ rec_scale,
                 float *__restrict__ rec_adj) {
  (void)src_idx;
  float fm = 0.0f;
  for (int n = threadIdx.x; n < nt; n += kBlock) fm = fmaxf(fm, fabsf(wavelet[n]));
  fm = block_reduce(fm, MaxOp(), threadIdx.x);
  const double s_src = sqrt_rho ? (double)sqrt_rho[src_model_idx] : 1.0;
  const double sigma = dt2_over_h3 / s_src;
  const int e = field_exponent(sigma * (double)fm);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    sc->sigma = (float)ldexp(sigma, e);
    sc->sigma_phys = (float)sigma;
    sc->e = e;
    sc->pad = 0;
  }
  if (i < nrec) {
    const float s = sqrt_rho ? sqrt_rho[rec_model_idx[i]] : 1.0f;
    rec_scale[i] = ldexpf(s, -e);
    rec_adj[i] = k[rec_idx[i]] * s;
  }
}

__global__ void __launch_bounds__(256)
    k_unscale_copy(const float *__restrict__ src, float *__restrict__ dst, int nx, int ny, int nz,
                   int pitch, const ShotScale *__restrict__ sc) {
  const int e = sc->e;
  const int64_t total = (int64_t)nx * ny * nz;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = i / nx;
    const int x = (int)(i - row * nx);
    dst[i] = ldexpf(src[row * pitch + x], -e);
  }
}

__global__ void k_source_gradient(const float *__restrict__ psi, const float *__restrict__ k,
                                  int64_t src_idx, const ShotScale *__restrict__ sc, int out_exp2,
                                  int m, float *__restrict__ wg) {
  if (threadIdx.x != 0) return;
  const double v = (double)sc->sigma_phys * (double)psi[src_idx] / (double)k[src_idx];
  wg[m - 1] += (float)ldexp(v, out_exp2 - sc->e);
}

constexpr int TT = 32;  // transpose tile

// res_tm[n][r] = 2^e adj[r] (seis_tm[n][r] - dobs[r][n]) (the adjoint field
// carries 2^e like the forward one); per-block 1/2 sum res^2 (physical).
__global__ void __launch_bounds__(256)
    k_residual(const float *__restrict__ seis_tm, const float *__restrict__ dobs,
               const float *__restrict__ adj, const ShotScale *__restrict__ sc, int nrec, int nt,
               float *__restrict__ res_tm, double *__restrict__ partial) {
  const int e = sc->e;
  __shared__ float tile[TT][TT + 1];
  const int r0 = blockIdx.y * TT, n0 = blockIdx.x * TT;
  const int tx = threadIdx.x, ty = threadIdx.y;  // 32 x 8
  for (int j = ty; j < TT; j += 8) {
    const int r = r0 + j, n = n0 + tx;
    tile[j][tx] = (r < nrec && n < nt) ? dobs[(int64_t)r * nt + n] : 0.0f;
  }
  __syncthreads();
  double acc = 0.0;
  for (int j = ty; j < TT; j += 8) {
    const int n = n0 + j, r = r0 + tx;
    if (r < nrec && n < nt) {
      const float res = seis_tm[(int64_t)n * nrec + r] - tile[tx][j];
      res_tm[(int64_t)n * nrec + r] = ldexpf(adj[r] * res, e);
      acc += 0.5 * (double)res * (double)res;
    }
  }
  const int t = ty * TT + tx;
  acc = block_reduce(acc, SumOp(), t);
  if (t == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = acc;
}

__global__ void __launch_bounds__(256)
    k_sum_partials(const double *__restrict__ partial, int n, double *misfit) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kBlock) acc += partial[i];
  acc = block_reduce(acc, SumOp(), threadIdx.x);
  if (threadIdx.x == 0) misfit[0] += acc;
}

__global__ void __launch_bounds__(256)
    k_transpose(const float *__restrict__ src_tm, float *__restrict__ dst_rm, int nrec, int nt) {
  __shared__ float tile[TT][TT + 1];
  const int r0 = blockIdx.x * TT, n0 = blockIdx.y * TT;
  const int tx = threadIdx.x, ty = threadIdx.y;
  for (int j = ty; j < TT; j += 8) {
    const int n = n0 + j, r = r0 + tx;
    tile[j][tx] = (r < nrec && n < nt) ? src_tm[(int64_t)n * nrec + r] : 0.0f;
  }
  __syncthreads();
  for (int j = ty; j < TT; j += 8) {
    const int r = r0 + j, n = n0 + tx;
    if (r < nrec && n < nt) dst_rm[(int64_t)r * nt + n] = tile[tx][j];
  }
}

// Padded range that folds into model index i along an axis of n cells.
__device__ __forceinline__ void fold_range(int i, int n, int border, int &lo, int &hi) {
  lo = (i == 0) ? 0 : i + border;
  hi = (i == n - 1) ? n - 1 + 2 * border : i + border;
}

__global__ void __launch_bounds__(256)
    k_grad_fold(const float *__restrict__ g, const float *__restrict__ k, int pitch, int pny,
                int border, int mnx, int mny, int mnz, double dt,
                const ShotScale *__restrict__ sc, int out_exp2, float *__restrict__ grad) {
  const int64_t total = (int64_t)mnx * mny * mnz;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int ix = (int)(i % mnx);
  const int iy = (int)((i / mnx) % mny);
  const int iz = (int)(i / ((int64_t)mnx * mny));
  int x0, x1, y0, y1, z0, z1;
  fold_range(ix, mnx, border, x0, x1);
  fold_range(iy, mny, border, y0, y1);
  fold_range(iz, mnz, border, z0, z1);
  const int64_t plane = (int64_t)pitch * pny;
  double s = 0.0;
  for (int z = z0; z <= z1; ++z)
    for (int y = y0; y <= y1; ++y)
      for (int x = x0; x <= x1; ++x) s += g[(int64_t)z * plane + (int64_t)y * pitch + x];
  const float kc = k[(int64_t)(iz + border) * plane + (int64_t)(iy + border) * pitch + ix + border];
  const double v = sqrt((double)kc) / dt;
  grad[i] += (float)ldexp(2.0 * s / v, out_exp2 - 2 * sc->e);
}

__global__ void __launch_bounds__(256) k_fill_zero(float *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

}  // namespace

hipError_t launch_precompute_k(const float *vel, int mnx, int mny, int mnz, int border, double dt,
                               float *k, int pitch, int ny, int nz, float *partial_max,
                               int n_partial, hipStream_t stream) {
  hipLaunchKernelGGL(k_precompute_k, dim3(n_partial), dim3(256), 0, stream, vel, mnx, mny, mnz,
                     border, dt, k, pitch, ny, nz, partial_max);
  return hipGetLastError();
}

hipError_t launch_precompute_m2(const float *rho, int mnx, int mny, int mnz, int border,
                                int free_surface, double idx2, double idy2, double idz2,
                                float *m2, int pitch, int ny, int nz, float *sqrt_rho,
                                float *partial_max, int n_partial, hipStream_t stream) {
  hipLaunchKernelGGL(k_precompute_m2, dim3(n_partial), dim3(256), 0, stream, rho, mnx, mny, mnz,
                     border, free_surface, idx2, idy2, idz2, m2, pitch, ny, nz, sqrt_rho,
                     partial_max);
  return hipGetLastError();
}

hipError_t launch_shot_setup(const float *k, const float *sqrt_rho, int64_t src_idx,
                             int src_model_idx, double dt2_over_h3, const float *wavelet, int nt,
                             const int64_t *rec_idx, const int *rec_model_idx, int nrec,
                             ShotScale *sc, float *rec_scale, float *rec_adj, hipStream_t stream) {
  const int n = nrec > 1 ? nrec : 1;
  hipLaunchKernelGGL(k_shot_setup, dim3((n + 255) / 256), dim3(256), 0, stream, k, sqrt_rho,
                     src_idx, src_model_idx, dt2_over_h3, wavelet, nt, rec_idx, rec_model_idx,
                     nrec, sc, rec_scale, rec_adj);
  return hipGetLastError();
}

hipError_t launch_unscale_copy(const float *src, float *dst, int nx, int ny, int nz, int pitch,
                               const ShotScale *sc, hipStream_t stream) {
  const int64_t total = (int64_t)nx * ny * nz;
  if (total <= 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_unscale_copy, dim3((unsigned)blocks), dim3(256), 0, stream, src, dst, nx,
                     ny, nz, pitch, sc);
  return hipGetLastError();
}

hipError_t launch_source_gradient(const float *psi, const float *k, int64_t src_idx,
                                  const ShotScale *sc, int out_exp2, int m, float *wg,
                                  hipStream_t stream) {
  hipLaunchKernelGGL(k_source_gradient, dim3(1), dim3(64), 0, stream, psi, k, src_idx, sc,
                     out_exp2, m, wg);
  return hipGetLastError();
}

int residual_partial_count(int nrec, int nt) {
  return ((nt + TT - 1) / TT) * ((nrec + TT - 1) / TT);
}

hipError_t launch_residual(const float *seis_tm, const float *dobs, const float *rec_adj,
                           const ShotScale *sc, int nrec, int nt, float *res_tm, double *partial,
                           int *n_partial, hipStream_t stream) {
  dim3 grid((nt + TT - 1) / TT, (nrec + TT - 1) / TT);
  *n_partial = (int)(grid.x * grid.y);
  hipLaunchKernelGGL(k_residual, grid, dim3(TT, 8), 0, stream, seis_tm, dobs, rec_adj, sc, nrec,
                     nt, res_tm, partial);
  return hipGetLastError();
}

hipError_t launch_sum_partials(const double *partial, int n, double *misfit, hipStream_t stream) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, stream, partial, n, misfit);
  return hipGetLastError();
}

hipError_t launch_transpose(const float *src_tm, float *dst_rm, int nrec, int nt,
                            hipStream_t stream) {
  dim3 grid((nrec + TT - 1) / TT, (nt + TT - 1) / TT);
  hipLaunchKernelGGL(k_transpose, grid, dim3(TT, 8), 0, stream, src_tm, dst_rm, nrec, nt);
  return hipGetLastError();
}

hipError_t launch_grad_fold(const float *g, const float *k, int pitch, int pny, int border,
                            int mnx, int mny, int mnz, double dt, const ShotScale *sc,
                            int out_exp2, float *grad, hipStream_t stream) {
  const int64_t total = (int64_t)mnx * mny * mnz;
  hipLaunchKernelGGL(k_grad_fold, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, g,
                     k, pitch, pny, border, mnx, mny, mnz, dt, sc, out_exp2, grad);
  return hipGetLastError();
}

hipError_t launch_fill_zero(float *p, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, stream, p, n);
  return hipGetLastError();
}

}  // namespace wfd
