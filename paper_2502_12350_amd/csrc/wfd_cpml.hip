// CPML absorbing layer (§2.1: the convolutional PML of Roden and Gedney, the
// paper's alternative to damping), on the second-order equation.
//
// In the layer each second derivative is taken in stretched coordinates,
// d2/dx~2 w = D2 w + D1 psi + zeta, with the recursive convolutions
//   psi_d  = b_d psi_d  + a_d D1_d w
//   zeta_d = b_d zeta_d + a_d (D2_d w + D1_d psi_d)
// so the leapfrog step gains k C with C = sum_d (D1_d psi_d + zeta_d).  The
// step kernels do everything else (with unit sponge tables); these kernels
// add the layer's terms on the shell, the points within reach of them.  The
// adjoint is the exact transpose:
//   nu_d = phi^{m+1} + b_d nu_d,   mu_d = b_d mu_d - D1_d (a_d nu_d + phi^{m+1}),
//   phi^m += k sum_d [D2_d (a_d nu_d) - D1_d (a_d mu_d)],
// and the imaging condition gains phi^{m+1} C^m.
//
// D1 is the eighth-order central first difference (4/5, -1/5, 4/105, -1/280)
// and D2 the second difference of L; cells outside the padded grid are zero,
// and D2 along z reads the free surface's negated image like L does.  A block
// of 64 x 4 threads owns an (x, y) tile of one shell box and marches a chunk
// of planes; where the box is within reach of a z layer each thread keeps
// nine-plane queues along z, and x and y neighbours come through the caches.
// The point-wise nu update runs one thread per shell point.
//
// A memory variable of axis d is nonzero only on that axis' layer, the B
// border cells at each end of the padded axis, and is stored as two slabs of
// W = B + 8 cells, [0, W) and [N - W, N) (the whole axis when they would
// meet): x as [Nz][Ny][2W], y as [Nz][2W][Nx], z as [2W][Ny][Nx].  A point
// within reach of the layer (4 cells) reads the variable at most 4 cells
// further, so every read lands in the point's own slab and a line of the
// variable is addressed like a line of a full volume.  Psi and zeta (or mu
// and nu) of an axis take 4 W / N of a volume rather than two volumes, and
// every checkpoint of the gradient's forward sweep holds a set of six.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "wfd_internal.h"

namespace wfd {
namespace {

__device__ __forceinline__ float d1c(int j) {
  return j == 1 ? 0.8f : j == 2 ? -0.2f : j == 3 ? (float)(4.0 / 105.0) : (float)(-1.0 / 280.0);
}
__device__ __forceinline__ float d2c(int j) {
  return j == 0   ? (float)(-205.0 / 72.0)
         : j == 1 ? 1.6f
         : j == 2 ? -0.2f
         : j == 3 ? (float)(8.0 / 315.0)
                  : (float)(-1.0 / 560.0);
}

__device__ __forceinline__ int64_t lin(const StepGrid &g, int x, int y, int z) {
  return (int64_t)z * g.plane + (int64_t)y * g.pitch + x;
}

// Compact memory variables (above): stored index of cell i on an axis of n
// cells with slab width `half` and stored length `len`, whether it is stored,
// and the element of (x, y, z) in the x, y or z variable.
__device__ __forceinline__ int cidx(int i, int half, int len, int n) {
  return i < half ? i : i - (n - len);
}
__device__ __forceinline__ bool stored(int i, int half, int len, int n) {
  return i < half || i >= n - (len - half);
}
__device__ __forceinline__ int64_t mem_x(const StepGrid &g, const CpmlTables &t, int x, int y,
                                         int z) {
  return ((int64_t)z * g.ny + y) * t.len[0] + cidx(x, t.half[0], t.len[0], g.nx);
}
__device__ __forceinline__ int64_t mem_y(const StepGrid &g, const CpmlTables &t, int x, int y,
                                         int z) {
  return ((int64_t)z * t.len[1] + cidx(y, t.half[1], t.len[1], g.ny)) * g.nx + x;
}
__device__ __forceinline__ int64_t mem_z(const StepGrid &g, const CpmlTables &t, int x, int y,
                                         int z) {
  return ((int64_t)cidx(z, t.half[2], t.len[2], g.nz) * g.ny + y) * g.nx + x;
}
__device__ __forceinline__ bool stored_z(const StepGrid &g, const CpmlTables &t, int z) {
  return z >= 0 && z < g.nz && stored(z, t.half[2], t.len[2], g.nz);
}

// Shell point q -> (x, y, z).  Offsets inside a box fit 32 bits (the host
// checks), so the divisions are 32-bit: 64-bit ones are long software
// sequences and dominated these kernels.
__device__ __forceinline__ void decode(const Shell &sh, int64_t q, int &x, int &y, int &z) {
  int b = 0;
  while (b + 1 < sh.nbox && q >= sh.start[b + 1]) ++b;
  const uint32_t l = (uint32_t)(q - sh.start[b]);
  const uint32_t nxb = (uint32_t)(sh.x1[b] - sh.x0[b]);
  const uint32_t r = l / nxb;
  x = sh.x0[b] + (int)(l - r * nxb);
  if (sh.zfirst[b]) {
    const uint32_t nzb = (uint32_t)(sh.z1[b] - sh.z0[b]);
    const uint32_t yy = r / nzb;
    z = sh.z0[b] + (int)(r - yy * nzb);
    y = sh.y0[b] + (int)yy;
  } else {
    const uint32_t nyb = (uint32_t)(sh.y1[b] - sh.y0[b]);
    const uint32_t zz = r / nyb;
    y = sh.y0[b] + (int)(r - zz * nyb);
    z = sh.z0[b] + (int)zz;
  }
}

// Within reach (4 cells) of the layer of axis d = 0, 1, 2 (x, y, z).
__device__ __forceinline__ bool near(const Shell &sh, int d, int i) {
  return i < sh.lo[d] || i > sh.hi[d];
}

// A field along one axis through (x, y, z), optionally weighted by that axis'
// a table, zero outside the grid.
struct Line {
  const float *p;  // the point
  const float *a;  // weight per index along the axis, or nullptr
  int64_t stride;  // elements between neighbours along the axis
  int i, n;        // index along the axis and the axis length
  bool inner;      // i - 4 .. i + 4 all inside [0, n): no bounds tests
  __device__ __forceinline__ Line(const float *u, const float *a_, int64_t base, int64_t stride_,
                                  int i_, int n_)
      : p(u + base), a(a_), stride(stride_), i(i_), n(n_),
        inner(i_ >= kStencilRadius && i_ + kStencilRadius < n_) {}
  __device__ __forceinline__ float operator()(int j) const {  // value at offset j
    if (!inner) {
      const int ii = i + j;
      if (ii < 0 || ii >= n) return 0.0f;
    }
    const float v = p[j * stride];
    return a ? a[i + j] * v : v;
  }
};

__device__ __forceinline__ float first_diff(const Line &f) {
  float s = 0.0f;
#pragma unroll
  for (int j = 1; j <= 4; ++j) s += d1c(j) * (f(j) - f(-j));
  return s;
}

// Second difference along the line (x or y: no image planes).
__device__ __forceinline__ float second_diff(const Line &f) {
  float s = d2c(0) * f(0);
#pragma unroll
  for (int j = 1; j <= 4; ++j) s += d2c(j) * (f(j) + f(-j));
  return s;
}

constexpr int kThreads = 256;
static_assert(kThreads == kShellTileX * kShellTileY, "a column block is one x-y tile");

// The (x, y) column and z chunk of this thread (column marching).  Returns
// false for lanes past the box's x or y extent.
struct Column {
  int b, x, y, z0, z1;
  uint32_t nxb, nyb, nzb;
  int64_t pxy;  // offset of (x, y) in a plane
  __device__ __forceinline__ bool init(const Shell &sh, const StepGrid &g) {
    const int64_t blk = blockIdx.x;
    b = 0;
    while (b + 1 < sh.nbox && blk >= sh.bstart[b + 1]) ++b;
    uint32_t l = (uint32_t)(blk - sh.bstart[b]);
    const uint32_t ch = l % (uint32_t)sh.nch[b];
    l /= (uint32_t)sh.nch[b];
    const uint32_t ty = l % (uint32_t)sh.ty[b], tx = l / (uint32_t)sh.ty[b];
    x = sh.x0[b] + (int)tx * kShellTileX + (int)(threadIdx.x % kShellTileX);
    y = sh.y0[b] + (int)ty * kShellTileY + (int)(threadIdx.x / kShellTileX);
    z0 = sh.z0[b] + (int)ch * sh.cz[b];
    z1 = min(z0 + sh.cz[b], sh.z1[b]);
    nxb = (uint32_t)(sh.x1[b] - sh.x0[b]);
    nyb = (uint32_t)(sh.y1[b] - sh.y0[b]);
    nzb = (uint32_t)(sh.z1[b] - sh.z0[b]);
    pxy = (int64_t)y * g.pitch + x;
    return x < sh.x1[b] && y < sh.y1[b];
  }
  // index of (x, y, z) in the shell's point order (the correction store)
  __device__ __forceinline__ int64_t q(const Shell &sh, int z) const {
    const uint32_t xo = (uint32_t)(x - sh.x0[b]), yo = (uint32_t)(y - sh.y0[b]),
                   zo = (uint32_t)(z - sh.z0[b]);
    const uint32_t l = sh.zfirst[b] ? xo + nxb * (zo + nzb * yo) : xo + nxb * (yo + nyb * zo);
    return sh.start[b] + (int64_t)l;
  }
};

// Nine planes z-4 .. z+4 of a quantity along the thread's column; f(z') gives
// plane z'.  prime() at the chunk's first plane, then advance() per plane.
struct ZWin {
  float v[9];
  template <class F>
  __device__ __forceinline__ void prime(F f, int z) {
#pragma unroll
    for (int i = 0; i < 9; ++i) v[i] = f(z - 4 + i);
  }
  template <class F>
  __device__ __forceinline__ void advance(F f, int z) {  // to plane z + 1
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = v[i + 1];
    v[8] = f(z + 5);
  }
  __device__ __forceinline__ float d1() const {
    float s = 0.0f;
#pragma unroll
    for (int j = 1; j <= 4; ++j) s += d1c(j) * (v[4 + j] - v[4 - j]);
    return s;
  }
  __device__ __forceinline__ float d2() const {
    float s = d2c(0) * v[4];
#pragma unroll
    for (int j = 1; j <= 4; ++j) s += d2c(j) * (v[4 + j] + v[4 - j]);
    return s;
  }
};

// Plane z' of a column of u (offset pxy): zero outside the grid; with `image`,
// planes above the free surface read the negated mirror (as L does).
__device__ __forceinline__ float zval(const float *u, const StepGrid &g, int64_t pxy, int zz,
                                      bool image) {
  if (image && zz < g.zs) {
    const int zm = 2 * g.zs - zz;
    return zm < g.nz ? -u[(int64_t)zm * g.plane + pxy] : 0.0f;
  }
  return (zz >= 0 && zz < g.nz) ? u[(int64_t)zz * g.plane + pxy] : 0.0f;
}

__global__ void __launch_bounds__(kThreads)
    k_cpml_psi(StepGrid g, CpmlTables t, Shell sh, const float *__restrict__ w, float *px,
               float *py, float *pz) {
  Column c;
  if (!c.init(sh, g)) return;
  const bool zq = sh.zq[c.b];
  const float ax = t.ax[c.x], bx = t.bx[c.x], ay = t.ay[c.y], by = t.by[c.y];
  auto wz = [&](int zz) { return zval(w, g, c.pxy, zz, false); };
  ZWin qw;
  if (zq) qw.prime(wz, c.z0);
  for (int z = c.z0; z < c.z1; ++z) {
    const int64_t p = (int64_t)z * g.plane + c.pxy;
    if (ax != 0.0f) {
      float &v = px[mem_x(g, t, c.x, c.y, z)];
      v = bx * v + ax * (first_diff(Line{w, nullptr, p, 1, c.x, g.nx}) * t.ihx);
    }
    if (ay != 0.0f) {
      float &v = py[mem_y(g, t, c.x, c.y, z)];
      v = by * v + ay * (first_diff(Line{w, nullptr, p, g.pitch, c.y, g.ny}) * t.ihy);
    }
    if (zq) {
      const float az = t.az[z];
      if (az != 0.0f) {
        float &v = pz[mem_z(g, t, c.x, c.y, z)];
        v = t.bz[z] * v + az * (qw.d1() * t.ihz);
      }
      qw.advance(wz, z);
    }
  }
}

__global__ void __launch_bounds__(kThreads)
    k_cpml_zeta(StepGrid g, CpmlTables t, Shell sh, const float *__restrict__ w,
                const float *__restrict__ px, const float *__restrict__ py,
                const float *__restrict__ pz, float *zx, float *zy, float *zz_, float *out,
                float *cstore) {
  Column c;
  if (!c.init(sh, g)) return;
  const bool zq = sh.zq[c.b];
  const bool nx = near(sh, 0, c.x), ny = near(sh, 1, c.y);
  const float ax = t.ax[c.x], bx = t.bx[c.x], ay = t.ay[c.y], by = t.by[c.y];
  auto wz = [&](int zz) { return zval(w, g, c.pxy, zz, true); };
  auto pzz = [&](int zz) { return stored_z(g, t, zz) ? pz[mem_z(g, t, c.x, c.y, zz)] : 0.0f; };
  ZWin qw, qp;
  if (zq) {
    qw.prime(wz, c.z0);
    qp.prime(pzz, c.z0);
  }
  for (int z = c.z0; z < c.z1; ++z) {
    const int64_t p = (int64_t)z * g.plane + c.pxy;
    float C = 0.0f;
    if (nx) {
      const int64_t q = mem_x(g, t, c.x, c.y, z);
      const float d1p = first_diff(Line{px, nullptr, q, 1, c.x, g.nx}) * t.ihx;
      C += d1p;
      if (ax != 0.0f) {
        const float v =
            bx * zx[q] + ax * (second_diff(Line{w, nullptr, p, 1, c.x, g.nx}) * g.cx + d1p);
        zx[q] = v;
        C += v;
      }
    }
    if (ny) {
      const int64_t q = mem_y(g, t, c.x, c.y, z);
      const float d1p = first_diff(Line{py, nullptr, q, g.nx, c.y, g.ny}) * t.ihy;
      C += d1p;
      if (ay != 0.0f) {
        const float v = by * zy[q] +
                        ay * (second_diff(Line{w, nullptr, p, g.pitch, c.y, g.ny}) *
                                  g.cy + d1p);
        zy[q] = v;
        C += v;
      }
    }
    if (zq) {
      if (near(sh, 2, z)) {
        const float d1p = qp.d1() * t.ihz;
        C += d1p;
        const float az = t.az[z];
        if (az != 0.0f) {
          float &zv = zz_[mem_z(g, t, c.x, c.y, z)];
          const float v = t.bz[z] * zv + az * (qw.d2() * g.cz + d1p);
          zv = v;
          C += v;
        }
      }
      qw.advance(wz, z);
      qp.advance(pzz, z);
    }
    if (out && z > g.zs) out[p] += g.k[p] * C;
    if (cstore) cstore[c.q(sh, z)] = C;
  }
}

__global__ void __launch_bounds__(kThreads)
    k_cpml_nu(StepGrid g, CpmlTables t, Shell sh, const float *__restrict__ phi1, float *nx_,
              float *ny_, float *nz_) {
  const int64_t total = sh.start[sh.nbox];
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    int x, y, z;
    decode(sh, q, x, y, z);
    const float f = phi1[lin(g, x, y, z)];
    if (t.ax[x] != 0.0f) {
      float &v = nx_[mem_x(g, t, x, y, z)];
      v = f + t.bx[x] * v;
    }
    if (t.ay[y] != 0.0f) {
      float &v = ny_[mem_y(g, t, x, y, z)];
      v = f + t.by[y] * v;
    }
    if (t.az[z] != 0.0f) {
      float &v = nz_[mem_z(g, t, x, y, z)];
      v = f + t.bz[z] * v;
    }
  }
}

__global__ void __launch_bounds__(kThreads)
    k_cpml_mu(StepGrid g, CpmlTables t, Shell sh, const float *__restrict__ phi1,
              const float *__restrict__ nx_, const float *__restrict__ ny_,
              const float *__restrict__ nz_, float *mx, float *my, float *mz) {
  Column c;
  if (!c.init(sh, g)) return;
  const bool zq = sh.zq[c.b];
  const float ax = t.ax[c.x], bx = t.bx[c.x], ay = t.ay[c.y], by = t.by[c.y];
  // D1 of (a nu + phi1); along z from a queue of a_z nu_z + phi1
  auto fz = [&](int zz) {
    if (zz < 0 || zz >= g.nz) return 0.0f;
    const float f = phi1[(int64_t)zz * g.plane + c.pxy];
    return stored_z(g, t, zz) ? t.az[zz] * nz_[mem_z(g, t, c.x, c.y, zz)] + f : f;
  };
  ZWin qf;
  if (zq) qf.prime(fz, c.z0);
  for (int z = c.z0; z < c.z1; ++z) {
    const int64_t p = (int64_t)z * g.plane + c.pxy;
    if (ax != 0.0f) {
      const int64_t q = mem_x(g, t, c.x, c.y, z);
      const float d = first_diff(Line{nx_, t.ax, q, 1, c.x, g.nx}) +
                      first_diff(Line{phi1, nullptr, p, 1, c.x, g.nx});
      mx[q] = bx * mx[q] - d * t.ihx;
    }
    if (ay != 0.0f) {
      const int64_t q = mem_y(g, t, c.x, c.y, z);
      const float d = first_diff(Line{ny_, t.ay, q, g.nx, c.y, g.ny}) +
                      first_diff(Line{phi1, nullptr, p, g.pitch, c.y, g.ny});
      my[q] = by * my[q] - d * t.ihy;
    }
    if (zq) {
      const float az = t.az[z];
      if (az != 0.0f) {
        float &v = mz[mem_z(g, t, c.x, c.y, z)];
        v = t.bz[z] * v - qf.d1() * t.ihz;
      }
      qf.advance(fz, z);
    }
  }
}

__global__ void __launch_bounds__(kThreads)
    k_cpml_adjoint(StepGrid g, CpmlTables t, Shell sh, const float *__restrict__ nx_,
                   const float *__restrict__ ny_, const float *__restrict__ nz_,
                   const float *__restrict__ mx, const float *__restrict__ my,
                   const float *__restrict__ mz, float *phi, const float *__restrict__ phi1,
                   const float *__restrict__ cstore, float *grad) {
  Column c;
  if (!c.init(sh, g)) return;
  const bool zq = sh.zq[c.b];
  const bool nx = near(sh, 0, c.x), ny = near(sh, 1, c.y);
  // along z: a_z nu_z (image planes above a free surface, for D2) and a_z mu_z
  auto nuz = [&](int zz) {
    int z2 = zz;
    float sgn = 1.0f;
    if (zz < g.zs) {
      z2 = 2 * g.zs - zz;
      sgn = -1.0f;
    }
    return stored_z(g, t, z2) ? sgn * t.az[z2] * nz_[mem_z(g, t, c.x, c.y, z2)] : 0.0f;
  };
  auto muz = [&](int zz) {
    return stored_z(g, t, zz) ? t.az[zz] * mz[mem_z(g, t, c.x, c.y, zz)] : 0.0f;
  };
  ZWin qn, qm;
  if (zq) {
    qn.prime(nuz, c.z0);
    qm.prime(muz, c.z0);
  }
  for (int z = c.z0; z < c.z1; ++z) {
    const int64_t p = (int64_t)z * g.plane + c.pxy;
    float corr = 0.0f;
    if (nx) {
      const int64_t q = mem_x(g, t, c.x, c.y, z);
      corr += second_diff(Line{nx_, t.ax, q, 1, c.x, g.nx}) * g.cx -
              first_diff(Line{mx, t.ax, q, 1, c.x, g.nx}) * t.ihx;
    }
    if (ny) {
      const int64_t q = mem_y(g, t, c.x, c.y, z);
      corr += second_diff(Line{ny_, t.ay, q, g.nx, c.y, g.ny}) * g.cy -
              first_diff(Line{my, t.ay, q, g.nx, c.y, g.ny}) * t.ihy;
    }
    if (zq) {
      if (near(sh, 2, z)) corr += qn.d2() * g.cz - qm.d1() * t.ihz;
      qn.advance(nuz, z);
      qm.advance(muz, z);
    }
    if (z > g.zs) phi[p] += g.k[p] * corr;
    if (cstore) grad[p] += phi1[p] * cstore[c.q(sh, z)];
  }
}

__global__ void k_record(const float *__restrict__ field, const int64_t *__restrict__ idx,
                         const float *__restrict__ scale, int nrec, int n,
                         float *__restrict__ seis_tm) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nrec) seis_tm[(int64_t)n * nrec + r] = scale[r] * field[idx[r]];
}

unsigned blocks_for(const Shell &sh) {
  const int64_t total = sh.start[sh.nbox];
  const int64_t b = (total + kThreads - 1) / kThreads;
  return (unsigned)(b < 1 ? 1 : (b > 16384 ? 16384 : b));
}

unsigned columns_for(const Shell &sh) { return (unsigned)sh.bstart[sh.nbox]; }

}  // namespace

hipError_t launch_cpml_psi(const StepGrid &g, const CpmlTables &t, const Shell &sh,
                           const float *cur, float *psi_x, float *psi_y, float *psi_z,
                           hipStream_t stream) {
  if (sh.start[sh.nbox] == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cpml_psi, dim3(columns_for(sh)), dim3(kThreads), 0, stream, g, t, sh, cur,
                     psi_x, psi_y, psi_z);
  return hipGetLastError();
}

hipError_t launch_cpml_zeta(const StepGrid &g, const CpmlTables &t, const Shell &sh,
                            const float *cur, const float *psi_x, const float *psi_y,
                            const float *psi_z, float *zeta_x, float *zeta_y, float *zeta_z,
                            float *out, float *cstore, hipStream_t stream) {
  if (sh.start[sh.nbox] == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cpml_zeta, dim3(columns_for(sh)), dim3(kThreads), 0, stream, g, t, sh, cur,
                     psi_x, psi_y, psi_z, zeta_x, zeta_y, zeta_z, out, cstore);
  return hipGetLastError();
}

hipError_t launch_cpml_nu(const StepGrid &g, const CpmlTables &t, const Shell &sh,
                          const float *phi1, float *nu_x, float *nu_y, float *nu_z,
                          hipStream_t stream) {
  if (sh.start[sh.nbox] == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cpml_nu, dim3(blocks_for(sh)), dim3(kThreads), 0, stream, g, t, sh, phi1,
                     nu_x, nu_y, nu_z);
  return hipGetLastError();
}

hipError_t launch_cpml_mu(const StepGrid &g, const CpmlTables &t, const Shell &sh,
                          const float *phi1, const float *nu_x, const float *nu_y,
                          const float *nu_z, float *mu_x, float *mu_y, float *mu_z,
                          hipStream_t stream) {
  if (sh.start[sh.nbox] == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cpml_mu, dim3(columns_for(sh)), dim3(kThreads), 0, stream, g, t, sh, phi1,
                     nu_x, nu_y, nu_z, mu_x, mu_y, mu_z);
  return hipGetLastError();
}

hipError_t launch_cpml_adjoint(const StepGrid &g, const CpmlTables &t, const Shell &sh,
                               const float *nu_x, const float *nu_y, const float *nu_z,
                               const float *mu_x, const float *mu_y, const float *mu_z,
                               float *phi, const float *phi1, const float *cstore, float *grad,
                               hipStream_t stream) {
  if (sh.start[sh.nbox] == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cpml_adjoint, dim3(columns_for(sh)), dim3(kThreads), 0, stream, g, t, sh,
                     nu_x, nu_y, nu_z, mu_x, mu_y, mu_z, phi, phi1, cstore, grad);
  return hipGetLastError();
}

hipError_t launch_record(const float *field, const int64_t *idx, const float *scale, int nrec,
                         int n, float *seis_tm, hipStream_t stream) {
  if (nrec <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_record, dim3((unsigned)((nrec + 255) / 256)), dim3(256), 0, stream, field,
                     idx, scale, nrec, n, seis_tm);
  return hipGetLastError();
}

}  // namespace wfd
