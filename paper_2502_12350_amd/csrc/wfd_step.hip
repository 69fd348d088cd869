// Leapfrog step kernels for gfx950 (MI355X): the eighth-order 25-point star
// (arXiv 2502.12350, §2.1) in a z-marching, LDS-tiled form.
//
// A block of NW wavefronts owns a 64 x TY column tile (TY = NW * RY) of the
// padded grid and a chunk of z planes (defaults: forward 8 wavefronts of 2
// rows, 64 x 16 tiles; adjoint 16 wavefronts of 2 rows, 64 x 32 tiles).
// Lane = x, so every global access is a 256-byte row per wavefront.  Each
// thread keeps, for each of its RY rows, the nine z-neighbours of the current
// point in a register queue; the current plane with a 4-cell x/y halo is
// staged in LDS (double-buffered: one barrier per plane).  The next plane's
// queue entries and pointwise streams are fetched one iteration ahead, the
// halo five planes ahead through a register delay line (below).  Blocks are
// mapped XCD-aware: the
// dispatcher places block b on XCD b mod 8, so each XCD receives a
// contiguous range of tiles and neighbouring tiles share halos in one L2.
//
// HBM traffic per point: forward 16 B (constant density) / 20 B (variable
// density); adjoint + imaging 28 B / 32 B (+ 8 B with illumination).
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdlib>

#include "wfd_internal.h"

namespace wfd {
namespace {

constexpr float W0 = -205.0f / 72.0f;
constexpr float W1 = 8.0f / 5.0f;
constexpr float W2 = -1.0f / 5.0f;
constexpr float W3 = 8.0f / 315.0f;
constexpr float W4 = -1.0f / 560.0f;

constexpr int TX = 64;  // tile width = one wavefront

// A tile is NW wavefronts, each owning RY consecutive rows of 64 points.
template <int RY, int NW>
struct Tile {
  static constexpr int NTHREADS = TX * NW;
  static constexpr int TY = NW * RY;
  static constexpr int LX = TX + 8;
  static constexpr int LY = TY + 8;
  static constexpr int NHALO = 8 * TX + 8 * TY;  // y-halo rows + x-halo columns
  static constexpr int HPT = (NHALO + NTHREADS - 1) / NTHREADS;
};

// Block -> (tile x, tile y, z chunk).  Logical tiles are numbered x fastest,
// then y, then z chunk; XCD k (= blockIdx mod 8) gets one contiguous range.
__device__ __forceinline__ void tile_of(const TileMap &m, int b, int &tx, int &ty, int &tz) {
  const int nb = m.nblocks;
  const int per = nb / 8, rem = nb % 8;
  const int xcd = b % 8, slot = b / 8;
  const int logical =
      xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
  tx = logical % m.tiles_x;
  const int r = logical / m.tiles_x;
  ty = r % m.tiles_y;
  tz = r / m.tiles_y;
}

// Halo element h of a tile plane: global (gx, gy) and its LDS row / column.
template <int RY, int NW, int K>
__device__ __forceinline__ void halo_slot(int h, int x0, int y0, int &gx, int &gy, int &lrow,
                                          int &lcol) {
  constexpr int TY = Tile<RY, NW>::TY;
  if (h < 8 * TX) {  // four rows above and four below the tile
    const int r = h / TX, col = h % TX;
    gx = x0 + col;
    lcol = 4 + col;
    if (r < 4) {
      gy = y0 - 4 + r;
      lrow = r;
    } else {
      gy = y0 + TY + (r - 4);
      lrow = TY + r;
    }
  } else {  // four columns left and four right of each tile row
    const int hh = h - 8 * TX;
    const int row = hh / 8, c = hh % 8;
    gy = y0 + row;
    lrow = 4 + row;
    if (c < 4) {
      gx = x0 - 4 + c;
      lcol = c;
    } else {
      gx = x0 + TX + (c - 4);
      lcol = TX + c;
    }
  }
}

// Single-use streams (previous state, coefficients, gradient) bypass the
// cache's normal retention so that L2 keeps the stenciled planes.
__device__ __forceinline__ float ld_stream(const float *f, const StepGrid &g, int z, uint32_t o,
                                           bool ok) {
  return ok ? __builtin_nontemporal_load(f + (int64_t)z * g.plane + o) : 0.0f;
}
__device__ __forceinline__ void st_stream(float *f, int64_t p, float v) {
  __builtin_nontemporal_store(v, f + p);
}

// Per-thread view of one stenciled field: register queue + halo staging.
// The halo of a plane is loaded together with the plane's interior (five
// planes ahead of its use), when the neighbouring tiles load the same lines
// as their interior, and waits in a register delay line; loading it one plane
// ahead instead needed L2 to keep four planes of every resident tile, and the
// adjoint (two stenciled fields) then re-read its halo from HBM.
// DL is the delay-line depth: the halo of plane z is loaded DL planes before
// it is staged (5: with the interior of that plane; 1: one plane ahead).
// K tags the kernel family (0 forward, 1 adjoint): each family gets its own
// instantiations of the tile helpers.  With shared ones, hipcc allocated the
// adjoint 137 VGPRs instead of 123 once a forward shape used the same tile,
// dropping it from 4 to 3 waves per SIMD.
// FS: the grid may have a free surface.  Without one, plane loads carry no
// image branch: a uniform branch in every load cost 7 % of the step time.
template <int RY, int NW, int K, bool FS, int DL = 5>
struct Marcher {
  using T = Tile<RY, NW>;
  float q[RY][9];        // planes z-4 .. z+4 of the thread's RY points
  float nxt[RY];         // plane z+5 (in flight)
  float hq[DL][T::HPT];  // halo of planes z .. z+DL-1 (hq[0] is staged next)

  // Plane z of the field at offset o: zero past the grid, and above a free
  // surface the negated mirror image about it.
  __device__ __forceinline__ static float ld(const float *f, const StepGrid &g, int z, uint32_t o,
                                             bool ok) {
    if (FS && z < g.zs) {
      const int zm = 2 * g.zs - z;
      return (ok && zm < g.nz) ? -f[(int64_t)zm * g.plane + o] : 0.0f;
    }
    return (ok && z >= 0 && z < g.nz) ? f[(int64_t)z * g.plane + o] : 0.0f;
  }
  __device__ __forceinline__ void prime(const float *f, const StepGrid &g, int z0,
                                        const uint32_t *off, const bool *in,
                                        const uint32_t *hoff, const bool *hin) {
#pragma unroll
    for (int j = 0; j < RY; ++j)
#pragma unroll
      for (int i = 0; i < 9; ++i) q[j][i] = ld(f, g, z0 - 4 + i, off[j], in[j]);
#pragma unroll
    for (int d = 0; d < DL; ++d)
#pragma unroll
      for (int i = 0; i < T::HPT; ++i) hq[d][i] = ld(f, g, z0 + d, hoff[i], hin[i]);
  }
  __device__ __forceinline__ void stage(float (*s)[T::LX], int wave, int lane,
                                        const int *hslot) {
#pragma unroll
    for (int j = 0; j < RY; ++j) s[4 + wave * RY + j][4 + lane] = q[j][4];
#pragma unroll
    for (int i = 0; i < T::HPT; ++i)
      if (hslot[i] >= 0) (&s[0][0])[hslot[i]] = hq[0][i];
  }
  // After stage(): the interior of plane z+5 and the halo of plane z+DL.
  __device__ __forceinline__ void fetch(const float *f, const StepGrid &g, int z,
                                        const uint32_t *off, const bool *in,
                                        const uint32_t *hoff, const bool *hin) {
#pragma unroll
    for (int j = 0; j < RY; ++j) nxt[j] = ld(f, g, z + 5, off[j], in[j]);
#pragma unroll
    for (int d = 0; d < DL - 1; ++d)
#pragma unroll
      for (int i = 0; i < T::HPT; ++i) hq[d][i] = hq[d + 1][i];
#pragma unroll
    for (int i = 0; i < T::HPT; ++i) hq[DL - 1][i] = ld(f, g, z + DL, hoff[i], hin[i]);
  }
  __device__ __forceinline__ void shift() {
#pragma unroll
    for (int j = 0; j < RY; ++j) {
#pragma unroll
      for (int i = 0; i < 8; ++i) q[j][i] = q[j][i + 1];
      q[j][8] = nxt[j];
    }
  }
  // Sum of the x, y and z second differences (before 1/h^2 weights) of row j.
  template <int J>
  __device__ __forceinline__ void diffs(const float (*s)[T::LX], int wave, int lane, float &sx,
                                        float &sy, float &sz) const {
    const int ly = 4 + wave * RY + J, lx = 4 + lane;
    const float *row = s[ly];
    sx = W1 * (row[lx - 1] + row[lx + 1]) + W2 * (row[lx - 2] + row[lx + 2]) +
         W3 * (row[lx - 3] + row[lx + 3]) + W4 * (row[lx - 4] + row[lx + 4]);
    float up[4], dn[4];
#pragma unroll
    for (int k = 1; k <= 4; ++k) {
      up[k - 1] = (J - k >= 0) ? q[(J - k >= 0) ? J - k : 0][4] : s[ly - k][lx];
      dn[k - 1] = (J + k < RY) ? q[(J + k < RY) ? J + k : 0][4] : s[ly + k][lx];
    }
    sy = W1 * (up[0] + dn[0]) + W2 * (up[1] + dn[1]) + W3 * (up[2] + dn[2]) +
         W4 * (up[3] + dn[3]);
    sz = W1 * (q[J][3] + q[J][5]) + W2 * (q[J][2] + q[J][6]) + W3 * (q[J][1] + q[J][7]) +
         W4 * (q[J][0] + q[J][8]);
  }
};

// Common per-thread tile geometry.
template <int RY, int NW, int K>
struct Geo {
  using T = Tile<RY, NW>;
  int lane, wave, x0, y0, x, z0, z1;
  bool in[RY];
  uint32_t off[RY];
  int yv[RY];
  uint32_t hoff[T::HPT];
  bool hin[T::HPT];
  int hslot[T::HPT];

  __device__ __forceinline__ bool init(const StepGrid &g, const TileMap &map, int b) {
    int tx, ty, tz;
    tile_of(map, b, tx, ty, tz);
    z0 = tz * map.zc;
    z1 = min(z0 + map.zc, g.nz);
    lane = threadIdx.x % TX;
    wave = threadIdx.x / TX;
    x0 = tx * TX;
    y0 = ty * T::TY;
    x = x0 + lane;
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      yv[j] = y0 + wave * RY + j;
      in[j] = x < g.nx && yv[j] < g.ny;
      off[j] = in[j] ? (uint32_t)yv[j] * (uint32_t)g.pitch + (uint32_t)x : 0u;
    }
#pragma unroll
    for (int i = 0; i < T::HPT; ++i) {
      const int h = threadIdx.x + i * T::NTHREADS;
      if (h < T::NHALO) {
        int gx, gy, lrow, lcol;
        halo_slot<RY, NW, K>(h, x0, y0, gx, gy, lrow, lcol);
        hin[i] = gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny;
        hoff[i] = hin[i] ? (uint32_t)gy * (uint32_t)g.pitch + (uint32_t)gx : 0u;
        hslot[i] = lrow * T::LX + lcol;
      } else {
        hin[i] = false;
        hoff[i] = 0u;
        hslot[i] = -1;
      }
    }
    return z0 < g.nz;
  }
};

// Receiver entries of one column, walked in z order.
struct ColCursor {
  int e, ee, ez;
  __device__ __forceinline__ void init(const RecTable &rec, int col, int z0, bool ok) {
    e = ee = 0;
    ez = INT_MAX;
    if (!ok) return;
    e = rec.col_start[col];
    ee = rec.col_start[col + 1];
    while (e < ee && rec.ent_z[e] < z0) ++e;
    ez = e < ee ? rec.ent_z[e] : INT_MAX;
  }
  __device__ __forceinline__ void advance(const RecTable &rec) {
    ++e;
    ez = e < ee ? rec.ent_z[e] : INT_MAX;
  }
};

// One LDS plane of a tile with its halo.
template <int RY, int NW>
using LdsPlane = float[Tile<RY, NW>::LY][Tile<RY, NW>::LX];

// One leapfrog step over tile block b of a grid; records the receivers of
// step n when seis_tm is set (recomputation sweeps pass none).
template <int RY, int NW, bool VD, bool FS>
__device__ __forceinline__ void forward_tile(
    LdsPlane<RY, NW> *sm, const StepGrid &g,
    const float *__restrict__ cur, const float *prev, float *out, const Source &src, int n,
    const RecTable &rec, const float *__restrict__ rec_scale, float *__restrict__ seis_tm,
    const TileMap &map, int b) {
  using T = Tile<RY, NW>;
  Geo<RY, NW, 0> geo;
  if (!geo.init(g, map, b)) return;
  Marcher<RY, NW, 0, FS> f;
  f.prime(cur, g, geo.z0, geo.off, geo.in, geo.hoff, geo.hin);
  const float gxv = geo.x < g.nx ? g.gx[geo.x] : 0.0f;
  float gyv[RY];
  ColCursor cc[RY];
#pragma unroll
  for (int j = 0; j < RY; ++j) {
    gyv[j] = geo.in[j] ? g.gy[geo.yv[j]] : 0.0f;
    cc[j].init(rec, geo.yv[j] * g.nx + geo.x, geo.z0, geo.in[j] && seis_tm != nullptr);
  }
  const float c0 = W0 * (g.cx + g.cy + g.cz);
  float pv[RY], kv[RY], mv[RY];  // pointwise streams of the current plane
#pragma unroll
  for (int j = 0; j < RY; ++j) {
    pv[j] = ld_stream(prev, g, geo.z0, geo.off[j], geo.in[j]);
    kv[j] = ld_stream(g.k, g, geo.z0, geo.off[j], geo.in[j]);
    mv[j] = VD ? ld_stream(g.m2, g, geo.z0, geo.off[j], geo.in[j]) : 0.0f;
  }
  for (int z = geo.z0; z < geo.z1; ++z) {
    float(*s)[T::LX] = sm[z & 1];
    f.stage(s, geo.wave, geo.lane, geo.hslot);
    f.fetch(cur, g, z, geo.off, geo.in, geo.hoff, geo.hin);
    const bool more = z + 1 < geo.z1;
    float pn[RY], kn[RY], mn[RY];  // next plane, in flight during this one
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      pn[j] = ld_stream(prev, g, z + 1, geo.off[j], geo.in[j] && more);
      kn[j] = ld_stream(g.k, g, z + 1, geo.off[j], geo.in[j] && more);
      mn[j] = VD ? ld_stream(g.m2, g, z + 1, geo.off[j], geo.in[j] && more) : 0.0f;
    }
    __syncthreads();
    const float gzv = g.gz[z];
    const int64_t zoff = (int64_t)z * g.plane;
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      float sx, sy, sz;
      switch (j) {  // compile-time row index for the register / LDS choice
        case 0: f.template diffs<0>(s, geo.wave, geo.lane, sx, sy, sz); break;
        case 1: f.template diffs<(RY > 1 ? 1 : 0)>(s, geo.wave, geo.lane, sx, sy, sz); break;
        case 2: f.template diffs<(RY > 2 ? 2 : 0)>(s, geo.wave, geo.lane, sx, sy, sz); break;
        default: f.template diffs<(RY > 3 ? 3 : 0)>(s, geo.wave, geo.lane, sx, sy, sz); break;
      }
      const float c = f.q[j][4];
      const float lap = c0 * c + g.cx * sx + g.cy * sy + g.cz * sz;
      float acc = VD ? 2.0f * c + kv[j] * (lap - mv[j] * c) : 2.0f * c + kv[j] * lap;
      const int64_t p = zoff + geo.off[j];
      if (geo.in[j] && p == src.idx) acc += src.sigma[0] * src.wavelet[n];
      const float G = gxv * gyv[j] * gzv;
      const float o = (!FS || z > g.zs) ? G * (acc - G * pv[j]) : 0.0f;  // zero at/above a free surface
      if (geo.in[j]) st_stream(out, p, o);
      if (cc[j].ez == z) {
        for (int r = rec.ent_rp[cc[j].e]; r < rec.ent_rp[cc[j].e + 1]; ++r) {
          const int id = rec.perm[r];
          seis_tm[(int64_t)n * rec.nrec + id] = rec_scale[id] * o;
        }
        cc[j].advance(rec);
      }
    }
    f.shift();
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      pv[j] = pn[j];
      kv[j] = kn[j];
      mv[j] = mn[j];
    }
  }
}

template <int RY, int NW, bool VD, bool FS>
__global__ void __launch_bounds__(TX * NW)
    k_forward(StepGrid g, const float *__restrict__ cur, const float *prev, float *out,
              Source src, int n, RecTable rec, const float *__restrict__ rec_scale,
              float *__restrict__ seis_tm, TileMap map) {
  using T = Tile<RY, NW>;
  __shared__ float sm[2][T::LY][T::LX];
  forward_tile<RY, NW, VD, FS>(sm, g, cur, prev, out, src, n, rec, rec_scale, seis_tm, map,
                           blockIdx.x);
}

// Several grids (one per shot) advanced by one launch: block b belongs to the
// window whose [block_begin, block_end) contains it.  Window ranges start at
// multiples of 8 so that each window keeps the XCD-aware tile order.
template <int RY, int NW, bool VD, bool FS>
__global__ void __launch_bounds__(TX * NW)
    k_forward_multi(const WindowStep *__restrict__ wins, int nwin, int n) {
  using T = Tile<RY, NW>;
  __shared__ float sm[2][T::LY][T::LX];
  const int b = blockIdx.x;
  int w = 0;
  while (w + 1 < nwin && b >= wins[w + 1].block_begin) ++w;
  const WindowStep &d = wins[w];
  if (b >= d.block_end) return;
  forward_tile<RY, NW, VD, FS>(sm, d.g, d.cur, d.prev, d.out, d.src, n, d.rec, d.rec_scale,
                           d.seis_tm, d.map, b - d.block_begin);
}

// Halo delay-line depths of the adjoint's two fields.
constexpr int kDelayPsi = 5, kDelayW = 5;

template <int RY, int NW, bool VD, bool ILLUM, bool FS>
__global__ void __launch_bounds__(TX * NW)
    k_adjoint(StepGrid g, const float *__restrict__ cur, const float *prev, float *out,
              RecTable rec, const float *__restrict__ res_tm, int m,
              const float *__restrict__ wm, float *__restrict__ grad, IllumOut il,
              TileMap map) {
  using T = Tile<RY, NW>;
  __shared__ float sm[2][2][T::LY][T::LX];  // [field][buffer]
  Geo<RY, NW, 1> geo;
  if (!geo.init(g, map, blockIdx.x)) return;
  Marcher<RY, NW, 1, FS, kDelayPsi> fa;  // adjoint state psi^{m+1}
  Marcher<RY, NW, 1, FS, kDelayW> fw;    // forward state w^m
  fa.prime(cur, g, geo.z0, geo.off, geo.in, geo.hoff, geo.hin);
  fw.prime(wm, g, geo.z0, geo.off, geo.in, geo.hoff, geo.hin);
  const float gxv = geo.x < g.nx ? g.gx[geo.x] : 0.0f;
  float gyv[RY];
  ColCursor cc[RY];
#pragma unroll
  for (int j = 0; j < RY; ++j) {
    gyv[j] = geo.in[j] ? g.gy[geo.yv[j]] : 0.0f;
    cc[j].init(rec, geo.yv[j] * g.nx + geo.x, geo.z0, geo.in[j]);
  }
  const float c0 = W0 * (g.cx + g.cy + g.cz);
  const float *res_row = res_tm + (int64_t)(m - 1) * rec.nrec;
  const int iexp = ILLUM ? il.out_exp2 - 2 * il.sc->e : 0;  // (2^e w)^2 -> 2^out_exp2 w^2
  float pv[RY], kv[RY], mv[RY], gv[RY];
#pragma unroll
  for (int j = 0; j < RY; ++j) {
    pv[j] = ld_stream(prev, g, geo.z0, geo.off[j], geo.in[j]);
    kv[j] = ld_stream(g.k, g, geo.z0, geo.off[j], geo.in[j]);
    mv[j] = VD ? ld_stream(g.m2, g, geo.z0, geo.off[j], geo.in[j]) : 0.0f;
    gv[j] = ld_stream(grad, g, geo.z0, geo.off[j], geo.in[j]);
  }
  for (int z = geo.z0; z < geo.z1; ++z) {
    float(*sa)[T::LX] = sm[0][z & 1];
    float(*sw)[T::LX] = sm[1][z & 1];
    fa.stage(sa, geo.wave, geo.lane, geo.hslot);
    fw.stage(sw, geo.wave, geo.lane, geo.hslot);
    fa.fetch(cur, g, z, geo.off, geo.in, geo.hoff, geo.hin);
    fw.fetch(wm, g, z, geo.off, geo.in, geo.hoff, geo.hin);
    const bool more = z + 1 < geo.z1;
    float pn[RY], kn[RY], mn[RY], gn[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      pn[j] = ld_stream(prev, g, z + 1, geo.off[j], geo.in[j] && more);
      kn[j] = ld_stream(g.k, g, z + 1, geo.off[j], geo.in[j] && more);
      mn[j] = VD ? ld_stream(g.m2, g, z + 1, geo.off[j], geo.in[j] && more) : 0.0f;
      gn[j] = ld_stream(grad, g, z + 1, geo.off[j], geo.in[j] && more);
    }
    __syncthreads();
    const float gzv = g.gz[z];
    const int64_t zoff = (int64_t)z * g.plane;
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      float ax, ay, az, wx, wy, wz;
      switch (j) {
        case 0:
          fa.template diffs<0>(sa, geo.wave, geo.lane, ax, ay, az);
          fw.template diffs<0>(sw, geo.wave, geo.lane, wx, wy, wz);
          break;
        case 1:
          fa.template diffs<(RY > 1 ? 1 : 0)>(sa, geo.wave, geo.lane, ax, ay, az);
          fw.template diffs<(RY > 1 ? 1 : 0)>(sw, geo.wave, geo.lane, wx, wy, wz);
          break;
        case 2:
          fa.template diffs<(RY > 2 ? 2 : 0)>(sa, geo.wave, geo.lane, ax, ay, az);
          fw.template diffs<(RY > 2 ? 2 : 0)>(sw, geo.wave, geo.lane, wx, wy, wz);
          break;
        default:
          fa.template diffs<(RY > 3 ? 3 : 0)>(sa, geo.wave, geo.lane, ax, ay, az);
          fw.template diffs<(RY > 3 ? 3 : 0)>(sw, geo.wave, geo.lane, wx, wy, wz);
          break;
      }
      const float ca = fa.q[j][4], cw = fw.q[j][4];
      const float lap_a = c0 * ca + g.cx * ax + g.cy * ay + g.cz * az;
      const float lap_w = c0 * cw + g.cx * wx + g.cy * wy + g.cz * wz;
      float acc = VD ? 2.0f * ca + kv[j] * (lap_a - mv[j] * ca) : 2.0f * ca + kv[j] * lap_a;
      if (cc[j].ez == z) {  // receiver residuals injected at this node
        float sum = 0.0f;
        for (int r = rec.ent_rp[cc[j].e]; r < rec.ent_rp[cc[j].e + 1]; ++r)
          sum += res_row[rec.perm[r]];
        acc += sum;
        cc[j].advance(rec);
      }
      const float G = gxv * gyv[j] * gzv;
      const int64_t p = zoff + geo.off[j];
      if (geo.in[j]) {
        const bool live = !FS || z > g.zs;  // at and above a free surface psi and w stay zero
        st_stream(out, p, live ? G * (acc - G * pv[j]) : 0.0f);
        st_stream(grad, p, live ? gv[j] + ca * (VD ? lap_w - mv[j] * cw : lap_w) : gv[j]);
        if (ILLUM) {
          const int ix = geo.x - il.border, iy = geo.yv[j] - il.border, iz = z - il.border;
          if (ix >= 0 && ix < il.mnx && iy >= 0 && iy < il.mny && iz >= 0 && iz < il.mnz)
            il.p[((int64_t)iz * il.mny + iy) * il.mnx + ix] += ldexpf(cw * cw, iexp);
        }
      }
    }
    fa.shift();
    fw.shift();
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      pv[j] = pn[j];
      kv[j] = kn[j];
      mv[j] = mn[j];
      gv[j] = gn[j];
    }
  }
}

int env_int(const char *name, int dflt) {
  const char *v = std::getenv(name);
  if (!v || !*v) return dflt;
  return std::atoi(v);
}

int device_cus() {
  static const int cus = [] {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0)
      n = 256;
    return n;
  }();
  return cus;
}

template <class K>
int blocks_per_cu(K kernel, int threads) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
      per_cu <= 0)
    per_cu = 4;
  return per_cu;
}

// Tile map: the grid's (x, y) tiles times nch z chunks.  With `rounds` > 0 the
// chunk count aims at that many rounds of resident blocks.  Otherwise it
// minimises a cost model of the launch with R = blocks / resident slots:
//   R <= 1:  one round, as long as one block (an under-filled device runs no
//            faster per block);
//   R > 1:   floor(R) full rounds plus a last round that costs its fill
//            fraction but at least kTailFloor of a round,
// each round lasting zc planes plus `halo` plane-equivalents for re-reading
// the 8-plane z halo of the stencil fields.  Fitted to step times measured at
// 576^3 (forward 64x16 and adjoint 64x8 tiles, 2 to 19 chunks): time / cost
// was constant to within 3 per cent, with a last round of few blocks taking
// about half a full one.
constexpr double kTailFloor = 0.47;

double launch_cost(double R, int zc, double halo) {
  if (R <= 1.0) return zc + halo;
  const double full = std::floor(R), f = R - full;
  return (full + (f > 0.0 ? std::max(f, kTailFloor) : 0.0)) * (zc + halo);
}

TileMap make_map(const StepGrid &g, int ty, int per_cu, int nch_override, int rounds,
                 double halo) {
  TileMap m;
  m.tiles_x = (g.nx + TX - 1) / TX;
  m.tiles_y = (g.ny + ty - 1) / ty;
  const int64_t tiles = (int64_t)m.tiles_x * m.tiles_y;
  const int64_t slots = (int64_t)per_cu * device_cus();
  const int max_nch = std::max(1, (g.nz + 15) / 16);
  int nch = nch_override;
  if (nch <= 0 && rounds > 0) nch = (int)((rounds * slots + tiles / 2) / tiles);
  if (nch <= 0) {
    double best = 1e300;
    for (int c = 1; c <= max_nch; ++c) {
      const int zc = (g.nz + c - 1) / c;
      if ((g.nz + zc - 1) / zc != c) continue;  // same chunks as a smaller count
      const double cost = launch_cost((double)(c * tiles) / (double)slots, zc, halo);
      if (cost < best) {
        best = cost;
        nch = c;
      }
    }
  }
  nch = std::max(1, std::min(nch, max_nch));
  m.zc = (g.nz + nch - 1) / nch;
  m.nchunks = (g.nz + m.zc - 1) / m.zc;
  m.nblocks = (int)(tiles * m.nchunks);
  return m;
}

// Halo cost of the step kernels in plane-equivalents: 8 planes times the
// stencil fields' share of the bytes per point (forward: 4 of 20 B with
// variable density; adjoint: 8 of 32 B).
constexpr double kFwdHalo = 8.0 * 4.0 / 20.0, kAdjHalo = 8.0 * 8.0 / 32.0;

// Forward tile shapes selectable at run time: (rows per thread, wavefronts).
// Variant 0 was the fastest at 576^3 (694 us per step against 793 us for
// 64 x 32 tiles and 745 us for 4 x 4 with the same chunking rule).
template <int V>
struct FwdShape;
template <>
struct FwdShape<0> {
  static constexpr int RY = 2, NW = 8;  // 64 x 16
};
template <>
struct FwdShape<1> {
  static constexpr int RY = 2, NW = 16;  // 64 x 32
};
template <>
struct FwdShape<2> {
  static constexpr int RY = 2, NW = 4;  // 64 x 8
};
template <>
struct FwdShape<3> {
  static constexpr int RY = 4, NW = 4;  // 64 x 16
};

// Adjoint tile shapes selectable at run time.  With two stenciled fields and
// their halo delay lines, only the 64 x 32 tile (one halo value per thread
// per plane) stays within 128 VGPRs (4 waves per SIMD): 1213 us per step at
// 576^3 against 1432 us (64 x 8) and 1654 us (64 x 16).
template <int V>
struct AdjShape;
template <>
struct AdjShape<0> {
  static constexpr int RY = 2, NW = 16;  // 64 x 32
};
template <>
struct AdjShape<1> {
  static constexpr int RY = 2, NW = 8;  // 64 x 16
};
template <>
struct AdjShape<2> {
  static constexpr int RY = 2, NW = 4;  // 64 x 8
};

template <int V, bool VD, bool FS>
int fwd_per_cu() {
  using S = FwdShape<V>;
  static const int per_cu =
      blocks_per_cu(k_forward<S::RY, S::NW, VD, FS>, Tile<S::RY, S::NW>::NTHREADS);
  return per_cu;
}

template <int V>
int fwd_rows() {
  return Tile<FwdShape<V>::RY, FwdShape<V>::NW>::TY;
}

template <int V, bool VD, bool FS>
hipError_t fwd_launch(const StepGrid &g, const float *cur, const float *prev, float *out,
                      const Source &src, int n, const RecTable &rec, const float *rec_scale,
                      float *seis_tm, const Tuning &tu, hipStream_t stream) {
  using S = FwdShape<V>;
  static const int nch_env = env_int("WFD_ZCHUNKS_FWD", 0);  // 0 = automatic
  const TileMap map =
      make_map(g, fwd_rows<V>(), fwd_per_cu<V, VD, FS>(), nch_env, tu.rounds, kFwdHalo);
  hipLaunchKernelGGL((k_forward<S::RY, S::NW, VD, FS>), dim3(map.nblocks),
                     dim3(Tile<S::RY, S::NW>::NTHREADS), 0, stream, g, cur, prev, out, src, n,
                     rec, rec_scale, seis_tm, map);
  return hipGetLastError();
}

template <int V, bool VD, bool FS>
hipError_t fwd_multi_launch(const WindowStep *wins, int nwin, int nblocks, int n,
                            hipStream_t stream) {
  using S = FwdShape<V>;
  hipLaunchKernelGGL((k_forward_multi<S::RY, S::NW, VD, FS>), dim3(nblocks),
                     dim3(Tile<S::RY, S::NW>::NTHREADS), 0, stream, wins, nwin, n);
  return hipGetLastError();
}

template <int V, bool VD, bool ILLUM, bool FS>
hipError_t adj_launch(const Tuning &tu, const StepGrid &g, const float *cur, const float *prev,
                      float *out, const RecTable &rec, const float *res_tm, int m,
                      const float *wm, float *grad, const IllumOut &illum, hipStream_t stream) {
  using S = AdjShape<V>;
  using T = Tile<S::RY, S::NW>;
  static const int per_cu = blocks_per_cu(k_adjoint<S::RY, S::NW, VD, ILLUM, FS>, T::NTHREADS);
  static const int nch = env_int("WFD_ZCHUNKS_ADJ", 0);  // 0 = automatic
  const TileMap map = make_map(g, T::TY, per_cu, nch, tu.adj_rounds, kAdjHalo);
  hipLaunchKernelGGL((k_adjoint<S::RY, S::NW, VD, ILLUM, FS>), dim3(map.nblocks), dim3(T::NTHREADS),
                     0, stream, g, cur, prev, out, rec, res_tm, m, wm, grad, illum, map);
  return hipGetLastError();
}

template <int V>
hipError_t adj_dispatch(const Tuning &tu, const StepGrid &g, const float *cur, const float *prev,
                        float *out, const RecTable &rec, const float *res_tm, int m,
                        const float *wm, float *grad, const IllumOut &illum, hipStream_t stream) {
  const bool vd = g.m2 != nullptr, fs = g.zs != kNoSurface;
#define WFD_ADJ(VD_, IL_)                                                                       \
  return fs ? adj_launch<V, VD_, IL_, true>(tu, g, cur, prev, out, rec, res_tm, m, wm, grad,    \
                                            illum, stream)                                      \
            : adj_launch<V, VD_, IL_, false>(tu, g, cur, prev, out, rec, res_tm, m, wm, grad,   \
                                             illum, stream)
  if (vd) {
    if (illum.p) WFD_ADJ(true, true);
    WFD_ADJ(true, false);
  }
  if (illum.p) WFD_ADJ(false, true);
  WFD_ADJ(false, false);
#undef WFD_ADJ
}

}  // namespace

hipError_t launch_forward_step(const StepGrid &g, const float *cur, const float *prev, float *out,
                               const Source &src, int n, const RecTable *rec,
                               const float *rec_scale, float *seis_tm, const Tuning &tu,
                               hipStream_t stream) {
  const bool vd = g.m2 != nullptr, fs = g.zs != kNoSurface;
  const RecTable none{};
  const RecTable &r = rec ? *rec : none;
  float *rec_out = rec ? seis_tm : nullptr;
#define WFD_FWD1(V, VD_)                                                                     \
  (fs ? fwd_launch<V, VD_, true>(g, cur, prev, out, src, n, r, rec_scale, rec_out, tu, stream) \
      : fwd_launch<V, VD_, false>(g, cur, prev, out, src, n, r, rec_scale, rec_out, tu, stream))
#define WFD_FWD(V) return vd ? WFD_FWD1(V, true) : WFD_FWD1(V, false)
  switch (tu.variant) {
    case 1: WFD_FWD(1);
    case 2: WFD_FWD(2);
    case 3: WFD_FWD(3);
    default: WFD_FWD(0);
  }
#undef WFD_FWD
#undef WFD_FWD1
}

int forward_tile_map(const StepGrid &g, const Tuning &tu, TileMap *map) {
  const bool vd = g.m2 != nullptr, fs = g.zs != kNoSurface;
  int ty = 16, per_cu = 4;
#define WFD_PCU(V)                                                                 \
  (vd ? (fs ? fwd_per_cu<V, true, true>() : fwd_per_cu<V, true, false>())          \
      : (fs ? fwd_per_cu<V, false, true>() : fwd_per_cu<V, false, false>()))
  switch (tu.variant) {
    case 1: ty = fwd_rows<1>(); per_cu = WFD_PCU(1); break;
    case 2: ty = fwd_rows<2>(); per_cu = WFD_PCU(2); break;
    case 3: ty = fwd_rows<3>(); per_cu = WFD_PCU(3); break;
    default: ty = fwd_rows<0>(); per_cu = WFD_PCU(0); break;
  }
#undef WFD_PCU
  *map = make_map(g, ty, per_cu, 0, tu.rounds, kFwdHalo);
  return map->nblocks;
}

hipError_t launch_forward_multi(const WindowStep *wins, int nwin, int nblocks, int n, int variant,
                                bool vd, bool fs, hipStream_t stream) {
#define WFD_MULTI(V)                                                                       \
  return vd ? (fs ? fwd_multi_launch<V, true, true>(wins, nwin, nblocks, n, stream)         \
                  : fwd_multi_launch<V, true, false>(wins, nwin, nblocks, n, stream))       \
            : (fs ? fwd_multi_launch<V, false, true>(wins, nwin, nblocks, n, stream)        \
                  : fwd_multi_launch<V, false, false>(wins, nwin, nblocks, n, stream))
  switch (variant) {
    case 1: WFD_MULTI(1);
    case 2: WFD_MULTI(2);
    case 3: WFD_MULTI(3);
    default: WFD_MULTI(0);
  }
#undef WFD_MULTI
}

hipError_t launch_adjoint_step(const Tuning &tu, const StepGrid &g, const float *cur,
                               const float *prev, float *out, const RecTable &rec,
                               const float *res_tm, int m, const float *wm, float *grad,
                               const IllumOut &illum, hipStream_t stream) {
  switch (tu.adj_variant) {
    case 1: return adj_dispatch<1>(tu, g, cur, prev, out, rec, res_tm, m, wm, grad, illum, stream);
    case 2: return adj_dispatch<2>(tu, g, cur, prev, out, rec, res_tm, m, wm, grad, illum, stream);
    default: return adj_dispatch<0>(tu, g, cur, prev, out, rec, res_tm, m, wm, grad, illum, stream);
  }
}

}  // namespace wfd
