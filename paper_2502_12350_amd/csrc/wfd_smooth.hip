// Gradient smoothing (the paper's GradientPreconditioning: Laplace or Bessel
// filter with lengths l_x, l_y, l_z).  Volumes are [z][y][x] FP32.
//
// Laplace filter: along each axis, solve the tridiagonal system
//   [(1 + a^2) I - a (S + S^-1)] u = (1 - a)^2 g,  a = exp(-h / l),
// whose inverse is the exponential kernel (1 - a)/(1 + a) a^|n|; the end rows
// use a mirror (zero-flux) condition so constants are kept.  One thread solves
// one line by the Thomas algorithm in FP64 with per-axis coefficients
// computed on the host.
//
// Bessel filter: u = B^-1 g with B = I - sum_d l_d^2 D_dd (3-point second
// differences, zero-flux ends), symmetric positive definite; conjugate
// gradients with this matrix-vector product and FP64 inner products.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "wfd_internal.h"

namespace wfd {
namespace {

// Line L of an axis: first point and stride between consecutive points.
__device__ __forceinline__ void line_of(int axis, int64_t L, int nx, int ny, int64_t &base,
                                        int64_t &stride) {
  if (axis == 0) {  // x lines
    base = L * nx;
    stride = 1;
  } else if (axis == 1) {  // y lines: L = z * nx + x
    const int64_t x = L % nx, z = L / nx;
    base = z * (int64_t)ny * nx + x;
    stride = nx;
  } else {  // z lines: L = y * nx + x
    base = L;
    stride = (int64_t)nx * ny;
  }
}

// cp[i] and inv_den[i] of the Thomas recursion for the line length n
// (precomputed); rhs scale (1 - a)^2, off-diagonal -a.
__global__ void k_tri_lines(float *__restrict__ u, int axis, int n, int64_t nlines, int nx,
                            int ny, const double *__restrict__ cp,
                            const double *__restrict__ inv_den, double a, double scale) {
  const int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (L >= nlines) return;
  int64_t base, stride;
  line_of(axis, L, nx, ny, base, stride);
  // forward sweep: d'_i = (scale g_i + a d'_{i-1}) / den_i, kept in u
  double d = 0.0;
  for (int i = 0; i < n; ++i) {
    float *p = u + base + (int64_t)i * stride;
    d = (scale * (double)*p + a * d) * inv_den[i];
    *p = (float)d;
  }
  // back substitution: x_i = d'_i - cp_i x_{i+1}
  double x = d;
  for (int i = n - 2; i >= 0; --i) {
    float *p = u + base + (int64_t)i * stride;
    x = (double)*p - cp[i] * x;
    *p = (float)x;
  }
}

// y = B x and a per-block partial of <p, y> when p is given.
__global__ void k_bessel_apply(const float *__restrict__ x, float *__restrict__ y, int nx, int ny,
                               int nz, float cx, float cy, float cz, double *__restrict__ part) {
  __shared__ double red[256];
  const int64_t n = (int64_t)nx * ny * nz;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int ix = (int)(i % nx), iy = (int)((i / nx) % ny), iz = (int)(i / ((int64_t)nx * ny));
    const float c = x[i];
    // zero-flux ends: a missing neighbour contributes no difference
    float dxx = 0.0f, dyy = 0.0f, dzz = 0.0f;
    if (ix > 0) dxx += x[i - 1] - c;
    if (ix < nx - 1) dxx += x[i + 1] - c;
    if (iy > 0) dyy += x[i - nx] - c;
    if (iy < ny - 1) dyy += x[i + nx] - c;
    if (iz > 0) dzz += x[i - (int64_t)nx * ny] - c;
    if (iz < nz - 1) dzz += x[i + (int64_t)nx * ny] - c;
    const float v = c - (cx * dxx + cy * dyy + cz * dzz);
    y[i] = v;
    s += (double)c * (double)v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// x += alpha p; r -= alpha Ap; per-block partial of <r, r>.
__global__ void k_cg_update(float *__restrict__ x, float *__restrict__ r,
                            const float *__restrict__ p, const float *__restrict__ ap, int64_t n,
                            float alpha, double *__restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    x[i] += alpha * p[i];
    const float ri = r[i] - alpha * ap[i];
    r[i] = ri;
    s += (double)ri * (double)ri;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// p = r + beta p (beta = 0: p = r); optionally also x = 0 and r = g first.
__global__ void k_cg_direction(float *__restrict__ p, const float *__restrict__ r, int64_t n,
                               float beta) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = r[i] + beta * p[i];
}

__global__ void k_copy_zero(const float *__restrict__ g, float *__restrict__ r,
                            float *__restrict__ x, int64_t n, double *__restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float v = g[i];
    r[i] = v;
    x[i] = 0.0f;
    s += (double)v * (double)v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

}  // namespace

hipError_t launch_tri_lines(float *u, int axis, int n, int64_t nlines, int nx, int ny,
                            const double *cp, const double *inv_den, double a, double scale,
                            hipStream_t stream) {
  const int64_t blocks = (nlines + 255) / 256;
  hipLaunchKernelGGL(k_tri_lines, dim3((unsigned)blocks), dim3(256), 0, stream, u, axis, n,
                     nlines, nx, ny, cp, inv_den, a, scale);
  return hipGetLastError();
}

hipError_t launch_bessel_apply(const float *x, float *y, int nx, int ny, int nz, float cx,
                               float cy, float cz, double *part, int npart, hipStream_t stream) {
  hipLaunchKernelGGL(k_bessel_apply, dim3(npart), dim3(256), 0, stream, x, y, nx, ny, nz, cx, cy,
                     cz, part);
  return hipGetLastError();
}

hipError_t launch_cg_update(float *x, float *r, const float *p, const float *ap, int64_t n,
                            float alpha, double *part, int npart, hipStream_t stream) {
  hipLaunchKernelGGL(k_cg_update, dim3(npart), dim3(256), 0, stream, x, r, p, ap, n, alpha, part);
  return hipGetLastError();
}

hipError_t launch_cg_direction(float *p, const float *r, int64_t n, float beta, int npart,
                               hipStream_t stream) {
  hipLaunchKernelGGL(k_cg_direction, dim3(npart), dim3(256), 0, stream, p, r, n, beta);
  return hipGetLastError();
}

hipError_t launch_cg_start(const float *g, float *r, float *x, int64_t n, double *part, int npart,
                           hipStream_t stream) {
  hipLaunchKernelGGL(k_copy_zero, dim3(npart), dim3(256), 0, stream, g, r, x, n, part);
  return hipGetLastError();
}

}  // namespace wfd

// ---- time resampling of traces -------------------------------------------------
// Trace sample k sits at (k + 1) dt.  nearest: round half up, clamped.  sinc:
// out[m] = sum_n in[n] sinc(a_m - n) with a_m = t_m / dt_in - 1; using
// sin(pi (a - n)) = (-1)^n sin(pi a) each term is one division (FP64 sums);
// an integer a_m selects the input sample.
namespace wfd {
namespace {

__global__ void k_resample(const float *__restrict__ in, int nrec, int nt_in, double dt_in,
                           float *__restrict__ out, int nt_out, double dt_out, int sinc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nrec * nt_out) return;
  const int r = (int)(i / nt_out), m = (int)(i % nt_out);
  const float *tr = in + (int64_t)r * nt_in;
  const double a = (double)(m + 1) * dt_out / dt_in - 1.0;
  if (!sinc) {
    int n = (int)floor(a + 1.0 + 0.5) - 1;
    n = n < 0 ? 0 : (n > nt_in - 1 ? nt_in - 1 : n);
    out[i] = tr[n];
    return;
  }
  const double an = rint(a);
  if (fabs(a - an) < 1e-12) {  // on an input sample
    const int n = (int)an;
    out[i] = (n >= 0 && n < nt_in) ? tr[n] : 0.0f;
    return;
  }
  double s = 0.0;
  for (int n = 0; n < nt_in; ++n) {
    const double term = (double)tr[n] / (a - (double)n);
    s += (n & 1) ? -term : term;
  }
  out[i] = (float)(s * sin(M_PI * a) / M_PI);
}

}  // namespace

hipError_t launch_resample(const float *in, int nrec, int nt_in, double dt_in, float *out,
                           int nt_out, double dt_out, int sinc, hipStream_t stream) {
  const int64_t n = (int64_t)nrec * nt_out;
  hipLaunchKernelGGL(k_resample, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, in, nrec,
                     nt_in, dt_in, out, nt_out, dt_out, sinc);
  return hipGetLastError();
}

}  // namespace wfd
