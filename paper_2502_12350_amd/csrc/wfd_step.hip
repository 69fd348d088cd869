// Leapfrog step kernels for gfx950 (MI355X): the eighth-order 25-point star
// (arXiv 2502.12350, §2.1) in a z-marching, LDS-tiled form.
//
// A block of NW wavefronts owns a TX x TY column tile of the padded grid
// (TX = 64 NI, TY = NW RY) and a chunk of z planes: each thread holds NI
// column groups (x = x0 + lane + 64 i) of RY consecutive rows, so every
// global access is a 256-byte row segment per wavefront instruction.  Each
// thread keeps, for each of its points, the nine z-neighbours in a register
// queue; the current plane with a 4-cell x/y halo is staged in LDS
// (double-buffered: one barrier per plane).  The next plane's queue entries
// and pointwise streams are fetched one iteration ahead, the halo five planes
// ahead through a register delay line (below).  Blocks are mapped XCD-aware:
// the dispatcher places block b on XCD b mod 8, so each XCD receives a
// contiguous range of tiles and neighbouring tiles share halos in one L2.
//
// HBM traffic per point: forward 16 B (constant density) / 20 B (variable
// density); adjoint + imaging 28 B / 32 B (+ 8 B with illumination).
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <type_traits>

#include "wfd_internal.h"

namespace wfd {
namespace {

constexpr float W0 = -205.0f / 72.0f;
constexpr float W1 = 8.0f / 5.0f;
constexpr float W2 = -1.0f / 5.0f;
constexpr float W3 = 8.0f / 315.0f;
constexpr float W4 = -1.0f / 560.0f;

constexpr int WAVE = 64;  // lanes per wavefront = width of one column group

// Calls f(integral_constant<int, 0>), ..., f(integral_constant<int, N - 1>):
// a compile-time index for register-array access in unrolled loops.
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (N > 0) {
    static_for<N - 1>(f);
    f(std::integral_constant<int, N - 1>{});
  }
}

// A tile is NW wavefronts; each thread owns NI column groups of RY rows.
template <int RY, int NW, int NI>
struct Tile {
  static constexpr int NTHREADS = WAVE * NW;
  static constexpr int TX = WAVE * NI;
  static constexpr int TY = NW * RY;
  static constexpr int NP = RY * NI;  // points per thread: p = j * NI + i
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
template <int RY, int NW, int NI, int K>
__device__ __forceinline__ void halo_slot(int h, int x0, int y0, int &gx, int &gy, int &lrow,
                                          int &lcol) {
  constexpr int TX = Tile<RY, NW, NI>::TX;
  constexpr int TY = Tile<RY, NW, NI>::TY;
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
// The adjoint's form: a lane outside the grid (or a plane past the chunk)
// reads the field's first element and drops the value instead of skipping
// the load.  Together with the branch-free stores below and the sponge factor
// read a plane ahead this took the 576^3 adjoint step from 1218 to 1158 us;
// the same changes made the forward step slower (688 -> 713 us), so it keeps
// the branches.
__device__ __forceinline__ float ld_stream_nb(const float *f, const StepGrid &g, int z,
                                              uint32_t o, bool ok) {
  const float v = __builtin_nontemporal_load(f + (ok ? (int64_t)z * g.plane + o : 0));
  return ok ? v : 0.0f;
}
// Nontemporal store of one value per lane into plane z of a field through a
// buffer resource over that plane (under 2^32 bytes: the host caps a pitched
// plane below 2^30 points).  A lane outside the grid passes kDropOffset, past
// every plane, and the hardware drops its store, so the store needs no
// branch (the adjoint's stores).
constexpr uint32_t kDropOffset = 0xFFFFFFF0u;
__device__ __forceinline__ void st_plane(float *f, const StepGrid &g, int z, uint32_t ob,
                                         float v) {
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
      f + (int64_t)z * g.plane, (short)0, (int)(uint32_t)(g.plane * 4), 0x00020000);
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, ob, 0, 2 /* nt */);
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
template <int RY, int NW, int NI, int K, bool FS, int DL = 5>
struct Marcher {
  using T = Tile<RY, NW, NI>;
  static constexpr int NP = T::NP;
  float q[NP][9];        // planes z-4 .. z+4 of the thread's points
  float nxt[NP];         // plane z+5 (in flight)
  float hq[DL][T::HPT];  // halo of planes z .. z+DL-1 (hq[0] is staged next)

  // Plane z of the field at offset o: zero past the grid, and above a free
  // surface the negated mirror image about it.
  __device__ __forceinline__ static float ld(const float *f, const StepGrid &g, int z, uint32_t o,
                                             bool ok) {
    if (FS && z < g.zs) {
      const int zm = 2 * g.zs - z;
      return (ok && zm < g.nz) ? -f[(int64_t)zm * g.plane + o] : 0.0f;
    }
    const bool in = ok && z >= 0 && z < g.nz;
    if (K == 0) return in ? f[(int64_t)z * g.plane + o] : 0.0f;
    const float v = f[in ? (int64_t)z * g.plane + o : 0];  // adjoint: as ld_stream_nb
    return in ? v : 0.0f;
  }
  __device__ __forceinline__ void prime(const float *f, const StepGrid &g, int z0,
                                        const uint32_t *off, const bool *in,
                                        const uint32_t *hoff, const bool *hin) {
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int i = 0; i < 9; ++i) q[p][i] = ld(f, g, z0 - 4 + i, off[p], in[p]);
#pragma unroll
    for (int d = 0; d < DL; ++d)
#pragma unroll
      for (int i = 0; i < T::HPT; ++i) hq[d][i] = ld(f, g, z0 + d, hoff[i], hin[i]);
  }
  __device__ __forceinline__ void stage(float (*s)[T::LX], int wave, int lane,
                                        const int *hslot) {
#pragma unroll
    for (int j = 0; j < RY; ++j)
#pragma unroll
      for (int i = 0; i < NI; ++i) s[4 + wave * RY + j][4 + WAVE * i + lane] = q[j * NI + i][4];
#pragma unroll
    for (int i = 0; i < T::HPT; ++i)
      if (hslot[i] >= 0) (&s[0][0])[hslot[i]] = hq[0][i];
  }
  // After stage(): the interior of plane z+5 and the halo of plane z+DL.
  __device__ __forceinline__ void fetch(const float *f, const StepGrid &g, int z,
                                        const uint32_t *off, const bool *in,
                                        const uint32_t *hoff, const bool *hin) {
#pragma unroll
    for (int p = 0; p < NP; ++p) nxt[p] = ld(f, g, z + 5, off[p], in[p]);
#pragma unroll
    for (int d = 0; d < DL - 1; ++d)
#pragma unroll
      for (int i = 0; i < T::HPT; ++i) hq[d][i] = hq[d + 1][i];
#pragma unroll
    for (int i = 0; i < T::HPT; ++i) hq[DL - 1][i] = ld(f, g, z + DL, hoff[i], hin[i]);
  }
  __device__ __forceinline__ void shift() {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
#pragma unroll
      for (int i = 0; i < 8; ++i) q[p][i] = q[p][i + 1];
      q[p][8] = nxt[p];
    }
  }
  // Sum of the x, y and z second differences (before 1/h^2 weights) of the
  // point in row J, column group I of the thread.
  template <int J, int I>
  __device__ __forceinline__ void diffs(const float (*s)[T::LX], int wave, int lane, float &sx,
                                        float &sy, float &sz) const {
    const int ly = 4 + wave * RY + J, lx = 4 + WAVE * I + lane;
    const float *row = s[ly];
    sx = W1 * (row[lx - 1] + row[lx + 1]) + W2 * (row[lx - 2] + row[lx + 2]) +
         W3 * (row[lx - 3] + row[lx + 3]) + W4 * (row[lx - 4] + row[lx + 4]);
    float up[4], dn[4];
#pragma unroll
    for (int k = 1; k <= 4; ++k) {
      up[k - 1] = (J - k >= 0) ? q[((J - k >= 0) ? J - k : 0) * NI + I][4] : s[ly - k][lx];
      dn[k - 1] = (J + k < RY) ? q[((J + k < RY) ? J + k : 0) * NI + I][4] : s[ly + k][lx];
    }
    sy = W1 * (up[0] + dn[0]) + W2 * (up[1] + dn[1]) + W3 * (up[2] + dn[2]) +
         W4 * (up[3] + dn[3]);
    constexpr int P = J * NI + I;
    sz = W1 * (q[P][3] + q[P][5]) + W2 * (q[P][2] + q[P][6]) + W3 * (q[P][1] + q[P][7]) +
         W4 * (q[P][0] + q[P][8]);
  }
};

// Common per-thread tile geometry.
template <int RY, int NW, int NI, int K>
struct Geo {
  using T = Tile<RY, NW, NI>;
  static constexpr int NP = T::NP;
  int lane, wave, x0, y0, z0, z1;
  int xs[NI];     // x of column group i
  int yv[RY];     // y of row j
  bool in[NP];
  uint32_t off[NP];
  uint32_t hoff[T::HPT];
  bool hin[T::HPT];
  int hslot[T::HPT];

  __device__ __forceinline__ bool init(const StepGrid &g, const TileMap &map, int b) {
    int tx, ty, tz;
    tile_of(map, b, tx, ty, tz);
    z0 = tz * map.zc;
    z1 = min(z0 + map.zc, g.nz);
    lane = threadIdx.x % WAVE;
    wave = threadIdx.x / WAVE;
    x0 = tx * T::TX;
    y0 = ty * T::TY;
#pragma unroll
    for (int i = 0; i < NI; ++i) xs[i] = x0 + WAVE * i + lane;
#pragma unroll
    for (int j = 0; j < RY; ++j) yv[j] = y0 + wave * RY + j;
#pragma unroll
    for (int j = 0; j < RY; ++j)
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        const int p = j * NI + i;
        in[p] = xs[i] < g.nx && yv[j] < g.ny;
        off[p] = in[p] ? (uint32_t)yv[j] * (uint32_t)g.pitch + (uint32_t)xs[i] : 0u;
      }
#pragma unroll
    for (int i = 0; i < T::HPT; ++i) {
      const int h = threadIdx.x + i * T::NTHREADS;
      if (h < T::NHALO) {
        int gx, gy, lrow, lcol;
        halo_slot<RY, NW, NI, K>(h, x0, y0, gx, gy, lrow, lcol);
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
template <int RY, int NW, int NI>
using LdsPlane = float[Tile<RY, NW, NI>::LY][Tile<RY, NW, NI>::LX];

// One leapfrog step over tile block b of a grid; records the receivers of
// step n when seis_tm is set (recomputation sweeps pass none).
template <int RY, int NW, int NI, bool VD, bool FS>
__device__ __forceinline__ void forward_tile(
    LdsPlane<RY, NW, NI> *sm, const StepGrid &g,
    const float *__restrict__ cur, const float *prev, float *out, const Source &src, int n,
    const RecTable &rec, const float *__restrict__ rec_scale, float *__restrict__ seis_tm,
    const TileMap &map, int b) {
  using T = Tile<RY, NW, NI>;
  constexpr int NP = T::NP;
  Geo<RY, NW, NI, 0> geo;
  if (!geo.init(g, map, b)) return;
  Marcher<RY, NW, NI, 0, FS> f;
  f.prime(cur, g, geo.z0, geo.off, geo.in, geo.hoff, geo.hin);
  float gxv[NI], gyv[RY];
#pragma unroll
  for (int i = 0; i < NI; ++i) gxv[i] = geo.xs[i] < g.nx ? g.gx[geo.xs[i]] : 0.0f;
#pragma unroll
  for (int j = 0; j < RY; ++j) gyv[j] = geo.yv[j] < g.ny ? g.gy[geo.yv[j]] : 0.0f;
  ColCursor cc[NP];
#pragma unroll
  for (int j = 0; j < RY; ++j)
#pragma unroll
    for (int i = 0; i < NI; ++i)
      cc[j * NI + i].init(rec, geo.yv[j] * g.nx + geo.xs[i], geo.z0,
                          geo.in[j * NI + i] && seis_tm != nullptr);
  const float c0 = W0 * (g.cx + g.cy + g.cz);
  float pv[NP], kv[NP], mv[NP];  // pointwise streams of the current plane
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    pv[p] = ld_stream(prev, g, geo.z0, geo.off[p], geo.in[p]);
    kv[p] = ld_stream(g.k, g, geo.z0, geo.off[p], geo.in[p]);
    mv[p] = VD ? ld_stream(g.m2, g, geo.z0, geo.off[p], geo.in[p]) : 0.0f;
  }
  for (int z = geo.z0; z < geo.z1; ++z) {
    float(*s)[T::LX] = sm[z & 1];
    f.stage(s, geo.wave, geo.lane, geo.hslot);
    f.fetch(cur, g, z, geo.off, geo.in, geo.hoff, geo.hin);
    const bool more = z + 1 < geo.z1;
    float pn[NP], kn[NP], mn[NP];  // next plane, in flight during this one
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      pn[p] = ld_stream(prev, g, z + 1, geo.off[p], geo.in[p] && more);
      kn[p] = ld_stream(g.k, g, z + 1, geo.off[p], geo.in[p] && more);
      mn[p] = VD ? ld_stream(g.m2, g, z + 1, geo.off[p], geo.in[p] && more) : 0.0f;
    }
    __syncthreads();
    const float gzv = g.gz[z];
    const int64_t zoff = (int64_t)z * g.plane;
    static_for<RY>([&](auto Jc) {
      constexpr int J = decltype(Jc)::value;
      static_for<NI>([&](auto Ic) {
        constexpr int I = decltype(Ic)::value;
        constexpr int P = J * NI + I;
        float sx, sy, sz;
        f.template diffs<J, I>(s, geo.wave, geo.lane, sx, sy, sz);
        const float c = f.q[P][4];
        const float lap = c0 * c + g.cx * sx + g.cy * sy + g.cz * sz;
        float acc = VD ? 2.0f * c + kv[P] * (lap - mv[P] * c) : 2.0f * c + kv[P] * lap;
        const int64_t p = zoff + geo.off[P];
        if (geo.in[P] && p == src.idx) acc += src.sigma[0] * src.wavelet[n];
        const float G = gxv[I] * gyv[J] * gzv;
        const float o = (!FS || z > g.zs) ? G * (acc - G * pv[P]) : 0.0f;  // zero at/above a free surface
        if (geo.in[P]) __builtin_nontemporal_store(o, out + p);
        if (cc[P].ez == z) {
          for (int r = rec.ent_rp[cc[P].e]; r < rec.ent_rp[cc[P].e + 1]; ++r) {
            const int id = rec.perm[r];
            seis_tm[(int64_t)n * rec.nrec + id] = rec_scale[id] * o;
          }
          cc[P].advance(rec);
        }
      });
    });
    f.shift();
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      pv[p] = pn[p];
      kv[p] = kn[p];
      mv[p] = mn[p];
    }
  }
}

template <int RY, int NW, int NI, bool VD, bool FS>
__global__ void __launch_bounds__(WAVE * NW)
    k_forward(StepGrid g, const float *__restrict__ cur, const float *prev, float *out,
              Source src, int n, RecTable rec, const float *__restrict__ rec_scale,
              float *__restrict__ seis_tm, TileMap map) {
  using T = Tile<RY, NW, NI>;
  __shared__ float sm[2][T::LY][T::LX];
  forward_tile<RY, NW, NI, VD, FS>(sm, g, cur, prev, out, src, n, rec, rec_scale, seis_tm, map,
                                   blockIdx.x);
}

// Several grids (one per shot) advanced by one launch: block b belongs to the
// window whose [block_begin, block_end) contains it.  Window ranges start at
// multiples of 8 so that each window keeps the XCD-aware tile order.
template <int RY, int NW, int NI, bool VD, bool FS>
__global__ void __launch_bounds__(WAVE * NW)
    k_forward_multi(const WindowStep *__restrict__ wins, int nwin, int n) {
  using T = Tile<RY, NW, NI>;
  __shared__ float sm[2][T::LY][T::LX];
  const int b = blockIdx.x;
  int w = 0;
  while (w + 1 < nwin && b >= wins[w + 1].block_begin) ++w;
  const WindowStep &d = wins[w];
  if (b >= d.block_end) return;
  forward_tile<RY, NW, NI, VD, FS>(sm, d.g, d.cur, d.prev, d.out, d.src, n, d.rec, d.rec_scale,
                                   d.seis_tm, d.map, b - d.block_begin);
}

// DL: halo delay-line depth of the adjoint's two fields (the tile shapes
// below choose it: each delay stage costs two registers per halo value).
// One adjoint step fused with the imaging condition over tile block b of a
// grid: psi^m (out, in place over psi^{m+2} = prev) from psi^{m+1} (cur), the
// residuals of sample m-1 injected at the receivers, and
// g += psi^{m+1} (L w^m - m2 w^m) (+ the illumination).  sm[0] stages psi,
// sm[1] w.
template <int RY, int NW, int NI, int DL, bool VD, bool ILLUM, bool FS>
__device__ __forceinline__ void adjoint_tile(
    const StepGrid g, const float *__restrict__ cur, const float *prev,
    float *out, const RecTable rec, const float *__restrict__ res_tm, int m,
    const float *__restrict__ wm, float *__restrict__ grad, const IllumOut il,
    const TileMap map, int b) {
  using T = Tile<RY, NW, NI>;
  constexpr int NP = T::NP;
  __shared__ float sm[2][2][T::LY][T::LX];  // [field][buffer]
  Geo<RY, NW, NI, 1> geo;
  if (!geo.init(g, map, b)) return;
  Marcher<RY, NW, NI, 1, FS, DL> fa;  // adjoint state psi^{m+1}
  Marcher<RY, NW, NI, 1, FS, DL> fw;  // forward state w^m
  fa.prime(cur, g, geo.z0, geo.off, geo.in, geo.hoff, geo.hin);
  fw.prime(wm, g, geo.z0, geo.off, geo.in, geo.hoff, geo.hin);
  float gxv[NI], gyv[RY];
#pragma unroll
  for (int i = 0; i < NI; ++i) gxv[i] = geo.xs[i] < g.nx ? g.gx[geo.xs[i]] : 0.0f;
#pragma unroll
  for (int j = 0; j < RY; ++j) gyv[j] = geo.yv[j] < g.ny ? g.gy[geo.yv[j]] : 0.0f;
  ColCursor cc[NP];
#pragma unroll
  for (int j = 0; j < RY; ++j)
#pragma unroll
    for (int i = 0; i < NI; ++i)
      cc[j * NI + i].init(rec, geo.yv[j] * g.nx + geo.xs[i], geo.z0, geo.in[j * NI + i]);
  const float c0 = W0 * (g.cx + g.cy + g.cz);
  const float *res_row = res_tm + (int64_t)(m - 1) * rec.nrec;
  const int iexp = ILLUM ? il.out_exp2 - 2 * il.sc->e : 0;  // (2^e w)^2 -> 2^out_exp2 w^2
  float gzv = g.gz[geo.z0];  // the z sponge factor, read one plane ahead
  float pv[NP], kv[NP], mv[NP], gv[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    pv[p] = ld_stream_nb(prev, g, geo.z0, geo.off[p], geo.in[p]);
    kv[p] = ld_stream_nb(g.k, g, geo.z0, geo.off[p], geo.in[p]);
    mv[p] = VD ? ld_stream_nb(g.m2, g, geo.z0, geo.off[p], geo.in[p]) : 0.0f;
    gv[p] = ld_stream_nb(grad, g, geo.z0, geo.off[p], geo.in[p]);
  }
  for (int z = geo.z0; z < geo.z1; ++z) {
    float(*sa)[T::LX] = sm[0][z & 1];
    float(*sw)[T::LX] = sm[1][z & 1];
    fa.stage(sa, geo.wave, geo.lane, geo.hslot);
    fw.stage(sw, geo.wave, geo.lane, geo.hslot);
    const float gzn = g.gz[z + 1 < g.nz ? z + 1 : z];
    fa.fetch(cur, g, z, geo.off, geo.in, geo.hoff, geo.hin);
    fw.fetch(wm, g, z, geo.off, geo.in, geo.hoff, geo.hin);
    const bool more = z + 1 < geo.z1;
    float pn[NP], kn[NP], mn[NP], gn[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      pn[p] = ld_stream_nb(prev, g, z + 1, geo.off[p], geo.in[p] && more);
      kn[p] = ld_stream_nb(g.k, g, z + 1, geo.off[p], geo.in[p] && more);
      mn[p] = VD ? ld_stream_nb(g.m2, g, z + 1, geo.off[p], geo.in[p] && more) : 0.0f;
      gn[p] = ld_stream_nb(grad, g, z + 1, geo.off[p], geo.in[p] && more);
    }
    __syncthreads();
    static_for<RY>([&](auto Jc) {
      constexpr int J = decltype(Jc)::value;
      static_for<NI>([&](auto Ic) {
        constexpr int I = decltype(Ic)::value;
        constexpr int P = J * NI + I;
        float ax, ay, az, wx, wy, wz;
        fa.template diffs<J, I>(sa, geo.wave, geo.lane, ax, ay, az);
        fw.template diffs<J, I>(sw, geo.wave, geo.lane, wx, wy, wz);
        const float ca = fa.q[P][4], cw = fw.q[P][4];
        const float lap_a = c0 * ca + g.cx * ax + g.cy * ay + g.cz * az;
        const float lap_w = c0 * cw + g.cx * wx + g.cy * wy + g.cz * wz;
        float acc = VD ? 2.0f * ca + kv[P] * (lap_a - mv[P] * ca) : 2.0f * ca + kv[P] * lap_a;
        if (cc[P].ez == z) {  // receiver residuals injected at this node
          float sum = 0.0f;
          for (int r = rec.ent_rp[cc[P].e]; r < rec.ent_rp[cc[P].e + 1]; ++r)
            sum += res_row[rec.perm[r]];
          acc += sum;
          cc[P].advance(rec);
        }
        const float G = gxv[I] * gyv[J] * gzv;
        const bool live = !FS || z > g.zs;  // at and above a free surface psi and w stay zero
        const uint32_t ob = geo.in[P] ? 4u * geo.off[P] : kDropOffset;
        st_plane(out, g, z, ob, live ? G * (acc - G * pv[P]) : 0.0f);
        st_plane(grad, g, z, ob, live ? gv[P] + ca * (VD ? lap_w - mv[P] * cw : lap_w) : gv[P]);
        if (ILLUM && geo.in[P]) {
          const int ix = geo.xs[I] - il.border, iy = geo.yv[J] - il.border, iz = z - il.border;
          if (ix >= 0 && ix < il.mnx && iy >= 0 && iy < il.mny && iz >= 0 && iz < il.mnz)
            il.p[((int64_t)iz * il.mny + iy) * il.mnx + ix] += ldexpf(cw * cw, iexp);
        }
      });
    });
    fa.shift();
    fw.shift();
    gzv = gzn;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      pv[p] = pn[p];
      kv[p] = kn[p];
      mv[p] = mn[p];
      gv[p] = gn[p];
    }
  }
}

// The single-shot kernel keeps its own copy of the tile body: sharing the
// device function with the batched kernel cost two VGPR spills in the plane
// loop (1238 against 1220 us per step at 576^3).
template <int RY, int NW, int NI, int DL, bool VD, bool ILLUM, bool FS>
__global__ void __launch_bounds__(WAVE * NW)
    k_adjoint(StepGrid g, const float *__restrict__ cur, const float *prev, float *out,
              RecTable rec, const float *__restrict__ res_tm, int m,
              const float *__restrict__ wm, float *__restrict__ grad, IllumOut il,
              TileMap map) {
  using T = Tile<RY, NW, NI>;
  constexpr int NP = T::NP;
  __shared__ float sm[2][2][T::LY][T::LX];  // [field][buffer]
  Geo<RY, NW, NI, 1> geo;
  if (!geo.init(g, map, blockIdx.x)) return;
  Marcher<RY, NW, NI, 1, FS, DL> fa;  // adjoint state psi^{m+1}
  Marcher<RY, NW, NI, 1, FS, DL> fw;  // forward state w^m
  fa.prime(cur, g, geo.z0, geo.off, geo.in, geo.hoff, geo.hin);
  fw.prime(wm, g, geo.z0, geo.off, geo.in, geo.hoff, geo.hin);
  float gxv[NI], gyv[RY];
#pragma unroll
  for (int i = 0; i < NI; ++i) gxv[i] = geo.xs[i] < g.nx ? g.gx[geo.xs[i]] : 0.0f;
#pragma unroll
  for (int j = 0; j < RY; ++j) gyv[j] = geo.yv[j] < g.ny ? g.gy[geo.yv[j]] : 0.0f;
  ColCursor cc[NP];
#pragma unroll
  for (int j = 0; j < RY; ++j)
#pragma unroll
    for (int i = 0; i < NI; ++i)
      cc[j * NI + i].init(rec, geo.yv[j] * g.nx + geo.xs[i], geo.z0, geo.in[j * NI + i]);
  const float c0 = W0 * (g.cx + g.cy + g.cz);
  const float *res_row = res_tm + (int64_t)(m - 1) * rec.nrec;
  const int iexp = ILLUM ? il.out_exp2 - 2 * il.sc->e : 0;  // (2^e w)^2 -> 2^out_exp2 w^2
  float gzv = g.gz[geo.z0];  // the z sponge factor, read one plane ahead
  float pv[NP], kv[NP], mv[NP], gv[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    pv[p] = ld_stream_nb(prev, g, geo.z0, geo.off[p], geo.in[p]);
    kv[p] = ld_stream_nb(g.k, g, geo.z0, geo.off[p], geo.in[p]);
    mv[p] = VD ? ld_stream_nb(g.m2, g, geo.z0, geo.off[p], geo.in[p]) : 0.0f;
    gv[p] = ld_stream_nb(grad, g, geo.z0, geo.off[p], geo.in[p]);
  }
  for (int z = geo.z0; z < geo.z1; ++z) {
    float(*sa)[T::LX] = sm[0][z & 1];
    float(*sw)[T::LX] = sm[1][z & 1];
    fa.stage(sa, geo.wave, geo.lane, geo.hslot);
    fw.stage(sw, geo.wave, geo.lane, geo.hslot);
    const float gzn = g.gz[z + 1 < g.nz ? z + 1 : z];
    fa.fetch(cur, g, z, geo.off, geo.in, geo.hoff, geo.hin);
    fw.fetch(wm, g, z, geo.off, geo.in, geo.hoff, geo.hin);
    const bool more = z + 1 < geo.z1;
    float pn[NP], kn[NP], mn[NP], gn[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      pn[p] = ld_stream_nb(prev, g, z + 1, geo.off[p], geo.in[p] && more);
      kn[p] = ld_stream_nb(g.k, g, z + 1, geo.off[p], geo.in[p] && more);
      mn[p] = VD ? ld_stream_nb(g.m2, g, z + 1, geo.off[p], geo.in[p] && more) : 0.0f;
      gn[p] = ld_stream_nb(grad, g, z + 1, geo.off[p], geo.in[p] && more);
    }
    __syncthreads();
    static_for<RY>([&](auto Jc) {
      constexpr int J = decltype(Jc)::value;
      static_for<NI>([&](auto Ic) {
        constexpr int I = decltype(Ic)::value;
        constexpr int P = J * NI + I;
        float ax, ay, az, wx, wy, wz;
        fa.template diffs<J, I>(sa, geo.wave, geo.lane, ax, ay, az);
        fw.template diffs<J, I>(sw, geo.wave, geo.lane, wx, wy, wz);
        const float ca = fa.q[P][4], cw = fw.q[P][4];
        const float lap_a = c0 * ca + g.cx * ax + g.cy * ay + g.cz * az;
        const float lap_w = c0 * cw + g.cx * wx + g.cy * wy + g.cz * wz;
        float acc = VD ? 2.0f * ca + kv[P] * (lap_a - mv[P] * ca) : 2.0f * ca + kv[P] * lap_a;
        if (cc[P].ez == z) {  // receiver residuals injected at this node
          float sum = 0.0f;
          for (int r = rec.ent_rp[cc[P].e]; r < rec.ent_rp[cc[P].e + 1]; ++r)
            sum += res_row[rec.perm[r]];
          acc += sum;
          cc[P].advance(rec);
        }
        const float G = gxv[I] * gyv[J] * gzv;
        const bool live = !FS || z > g.zs;  // at and above a free surface psi and w stay zero
        const uint32_t ob = geo.in[P] ? 4u * geo.off[P] : kDropOffset;
        st_plane(out, g, z, ob, live ? G * (acc - G * pv[P]) : 0.0f);
        st_plane(grad, g, z, ob, live ? gv[P] + ca * (VD ? lap_w - mv[P] * cw : lap_w) : gv[P]);
        if (ILLUM && geo.in[P]) {
          const int ix = geo.xs[I] - il.border, iy = geo.yv[J] - il.border, iz = z - il.border;
          if (ix >= 0 && ix < il.mnx && iy >= 0 && iy < il.mny && iz >= 0 && iz < il.mnz)
            il.p[((int64_t)iz * il.mny + iy) * il.mnx + ix] += ldexpf(cw * cw, iexp);
        }
      });
    });
    fa.shift();
    fw.shift();
    gzv = gzn;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      pv[p] = pn[p];
      kv[p] = kn[p];
      mv[p] = mn[p];
      gv[p] = gn[p];
    }
  }
}

// Buffer k of a batched gradient's forward pool: W1, W2, then the stored
// checkpoint volumes.
__device__ __forceinline__ float *pool_buffer(const GradWindow &d, int k) {
  return k == 0 ? d.W1 : (k == 1 ? d.W2 : d.store + (int64_t)(k - 2) * d.vol);
}

// One forward step of every window of a batched gradient: block b belongs to
// the window whose [fblock_begin, fblock_end) contains it; the step reads pool
// buffers cur_k (w^n) and prev_k (w^{n-1}) and writes out_k, recording the
// receivers when `record` is set.
template <int RY, int NW, int NI, bool VD, bool FS>
__global__ void __launch_bounds__(WAVE * NW)
    k_forward_pool(const GradWindow *__restrict__ wins, int nwin, int n, int cur_k, int prev_k,
                   int out_k, int record) {
  using T = Tile<RY, NW, NI>;
  __shared__ float sm[2][T::LY][T::LX];
  const int b = blockIdx.x;
  int w = 0;
  while (w + 1 < nwin && b >= wins[w + 1].fblock_begin) ++w;
  const GradWindow &d = wins[w];
  if (b >= d.fblock_end) return;
  const RecTable none{};
  forward_tile<RY, NW, NI, VD, FS>(sm, d.g, pool_buffer(d, cur_k), pool_buffer(d, prev_k),
                                   pool_buffer(d, out_k), d.src, n, record ? d.rec : none,
                                   d.rec_scale, record ? d.seis_tm : nullptr, d.fmap,
                                   b - d.fblock_begin);
}

// One adjoint step (with imaging) of every window: psi^{m+1} is P1 (parity 0)
// or P2 (parity 1) and psi^m overwrites the other; w^m is pool buffer wm_k.
template <int RY, int NW, int NI, int DL, bool VD, bool ILLUM, bool FS>
__global__ void __launch_bounds__(WAVE * NW)
    k_adjoint_multi(const GradWindow *__restrict__ wins, int nwin, int m, int parity, int wm_k) {
  const int b = blockIdx.x;
  int w = 0;
  while (w + 1 < nwin && b >= wins[w + 1].ablock_begin) ++w;
  const GradWindow &d = wins[w];
  if (b >= d.ablock_end) return;
  float *a1 = parity ? d.P2 : d.P1, *a2 = parity ? d.P1 : d.P2;
  adjoint_tile<RY, NW, NI, DL, VD, ILLUM, FS>(d.g, a1, a2, a2, d.rec, d.res_tm, m,
                                              pool_buffer(d, wm_k), d.gimg, d.il, d.amap,
                                              b - d.ablock_begin);
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
// about half a full one.  Chunks are at least min_zc planes deep.  A single
// launch takes min_zc = 4: a grid too small to fill the device even then
// (R <= 1) gets the shortest marches, since its step time is the latency of
// one block's march (80^3 forward: 21 us per step with 16-plane chunks, 11 us
// with 4-plane ones; 2 planes gave 11.2).  The windows of a batch of several
// shots take 16: together they fill the device, and 4-plane chunks of small
// windows only added halo re-reads (24 windows of 50-69 cells: gradients
// 0.182 s against 0.162 s).
constexpr double kTailFloor = 0.47;

double launch_cost(double R, int zc, double halo) {
  if (R <= 1.0) return zc + halo;
  const double full = std::floor(R), f = R - full;
  return (full + (f > 0.0 ? std::max(f, kTailFloor) : 0.0)) * (zc + halo);
}

TileMap make_map(const StepGrid &g, int tx, int ty, int per_cu, int nch_override, int rounds,
                 double halo, int min_zc) {
  TileMap m;
  m.tiles_x = (g.nx + tx - 1) / tx;
  m.tiles_y = (g.ny + ty - 1) / ty;
  const int64_t tiles = (int64_t)m.tiles_x * m.tiles_y;
  const int64_t slots = (int64_t)per_cu * device_cus();
  const int max_nch = std::max(1, (g.nz + min_zc - 1) / min_zc);
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

// Forward tile shapes selectable at run time: (rows per thread, wavefronts,
// column groups per thread).  Variant 0 was the fastest of the 64-wide tiles
// at 576^3 (694 us per step against 793 us for 64 x 32 tiles and 745 us for
// 4 x 4 with the same chunking rule).
template <int V>
struct FwdShape;
template <>
struct FwdShape<0> {
  static constexpr int RY = 2, NW = 8, NI = 1;  // 64 x 16
};
template <>
struct FwdShape<1> {
  static constexpr int RY = 2, NW = 16, NI = 1;  // 64 x 32
};
template <>
struct FwdShape<2> {
  static constexpr int RY = 2, NW = 4, NI = 1;  // 64 x 8
};
template <>
struct FwdShape<3> {
  static constexpr int RY = 4, NW = 4, NI = 1;  // 64 x 16
};
template <>
struct FwdShape<4> {
  static constexpr int RY = 1, NW = 16, NI = 3;  // 192 x 16
};

// Adjoint tile shapes selectable at run time, with their halo delay-line
// depth.  With two stenciled fields, the 64 x 32 tile (one halo value per
// thread per plane, five-plane delay) stays within 128 VGPRs (4 waves per
// SIMD): 1213 us per step at 576^3 against 1432 us (64 x 8) and 1654 us
// (64 x 16, five-plane delay: 137 VGPRs, 3 waves per SIMD).  A two-plane delay
// keeps the 64 x 16 tile at 125 VGPRs: two blocks per CU.
template <int V>
struct AdjShape;
template <>
struct AdjShape<0> {
  static constexpr int RY = 2, NW = 16, NI = 1, DL = 5;  // 64 x 32
};
template <>
struct AdjShape<1> {
  static constexpr int RY = 2, NW = 8, NI = 1, DL = 2;  // 64 x 16
};
template <>
struct AdjShape<2> {
  static constexpr int RY = 2, NW = 4, NI = 1, DL = 5;  // 64 x 8
};
template <>
struct AdjShape<3> {
  static constexpr int RY = 2, NW = 8, NI = 1, DL = 1;  // 64 x 16, halo one plane ahead
};

template <int V, bool VD, bool FS>
int fwd_per_cu() {
  using S = FwdShape<V>;
  static const int per_cu =
      blocks_per_cu(k_forward<S::RY, S::NW, S::NI, VD, FS>, Tile<S::RY, S::NW, S::NI>::NTHREADS);
  return per_cu;
}

template <int V>
using FwdTile = Tile<FwdShape<V>::RY, FwdShape<V>::NW, FwdShape<V>::NI>;

template <int V, bool VD, bool FS>
hipError_t fwd_launch(const StepGrid &g, const float *cur, const float *prev, float *out,
                      const Source &src, int n, const RecTable &rec, const float *rec_scale,
                      float *seis_tm, const Tuning &tu, hipStream_t stream) {
  using S = FwdShape<V>;
  static const int nch_env = env_int("WFD_ZCHUNKS_FWD", 0);  // 0 = automatic
  const TileMap map = make_map(g, FwdTile<V>::TX, FwdTile<V>::TY, fwd_per_cu<V, VD, FS>(),
                               nch_env, tu.rounds, kFwdHalo, kSingleMinZc);
  hipLaunchKernelGGL((k_forward<S::RY, S::NW, S::NI, VD, FS>), dim3(map.nblocks),
                     dim3(FwdTile<V>::NTHREADS), 0, stream, g, cur, prev, out, src, n, rec,
                     rec_scale, seis_tm, map);
  return hipGetLastError();
}

template <int V, bool VD, bool FS>
hipError_t fwd_multi_launch(const WindowStep *wins, int nwin, int nblocks, int n,
                            hipStream_t stream) {
  using S = FwdShape<V>;
  hipLaunchKernelGGL((k_forward_multi<S::RY, S::NW, S::NI, VD, FS>), dim3(nblocks),
                     dim3(FwdTile<V>::NTHREADS), 0, stream, wins, nwin, n);
  return hipGetLastError();
}

template <int V, bool VD, bool ILLUM, bool FS>
hipError_t adj_launch(const Tuning &tu, const StepGrid &g, const float *cur, const float *prev,
                      float *out, const RecTable &rec, const float *res_tm, int m,
                      const float *wm, float *grad, const IllumOut &illum, hipStream_t stream) {
  using S = AdjShape<V>;
  using T = Tile<S::RY, S::NW, S::NI>;
  static const int per_cu =
      blocks_per_cu(k_adjoint<S::RY, S::NW, S::NI, S::DL, VD, ILLUM, FS>, T::NTHREADS);
  static const int nch = env_int("WFD_ZCHUNKS_ADJ", 0);  // 0 = automatic
  const TileMap map =
      make_map(g, T::TX, T::TY, per_cu, nch, tu.adj_rounds, kAdjHalo, kSingleMinZc);
  hipLaunchKernelGGL((k_adjoint<S::RY, S::NW, S::NI, S::DL, VD, ILLUM, FS>), dim3(map.nblocks),
                     dim3(T::NTHREADS), 0, stream, g, cur, prev, out, rec, res_tm, m, wm, grad,
                     illum, map);
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

template <int V, bool VD, bool FS>
hipError_t fwd_pool_launch(const GradWindow *wins, int nwin, int nblocks, int n, int ck, int pk,
                           int ok, int record, hipStream_t stream) {
  using S = FwdShape<V>;
  hipLaunchKernelGGL((k_forward_pool<S::RY, S::NW, S::NI, VD, FS>), dim3(nblocks),
                     dim3(FwdTile<V>::NTHREADS), 0, stream, wins, nwin, n, ck, pk, ok, record);
  return hipGetLastError();
}

template <int V, bool VD, bool ILLUM, bool FS>
hipError_t adj_multi_launch(const GradWindow *wins, int nwin, int nblocks, int m, int parity,
                            int wk, hipStream_t stream) {
  using S = AdjShape<V>;
  hipLaunchKernelGGL((k_adjoint_multi<S::RY, S::NW, S::NI, S::DL, VD, ILLUM, FS>), dim3(nblocks),
                     dim3(WAVE * S::NW), 0, stream, wins, nwin, m, parity, wk);
  return hipGetLastError();
}

template <int V>
hipError_t adj_multi_dispatch(const GradWindow *wins, int nwin, int nblocks, int m, int parity,
                              int wk, bool vd, bool illum, bool fs, hipStream_t stream) {
#define WFD_AM(VD_, IL_)                                                                     \
  return fs ? adj_multi_launch<V, VD_, IL_, true>(wins, nwin, nblocks, m, parity, wk, stream) \
            : adj_multi_launch<V, VD_, IL_, false>(wins, nwin, nblocks, m, parity, wk, stream)
  if (vd) {
    if (illum) WFD_AM(true, true);
    WFD_AM(true, false);
  }
  if (illum) WFD_AM(false, true);
  WFD_AM(false, false);
#undef WFD_AM
}

template <int V>
int adj_map(const StepGrid &g, const Tuning &tu, bool illum, int min_zc, TileMap *map) {
  using S = AdjShape<V>;
  using T = Tile<S::RY, S::NW, S::NI>;
  const bool vd = g.m2 != nullptr, fs = g.zs != kNoSurface;
  int per_cu;
#define WFD_PC(VD_, IL_, FS_) \
  blocks_per_cu(k_adjoint<S::RY, S::NW, S::NI, S::DL, VD_, IL_, FS_>, T::NTHREADS)
  if (vd)
    per_cu = illum ? (fs ? WFD_PC(true, true, true) : WFD_PC(true, true, false))
                   : (fs ? WFD_PC(true, false, true) : WFD_PC(true, false, false));
  else
    per_cu = illum ? (fs ? WFD_PC(false, true, true) : WFD_PC(false, true, false))
                   : (fs ? WFD_PC(false, false, true) : WFD_PC(false, false, false));
#undef WFD_PC
  *map = make_map(g, T::TX, T::TY, per_cu, 0, tu.adj_rounds, kAdjHalo, min_zc);
  return map->nblocks;
}

}  // namespace

int adjoint_tile_map(const StepGrid &g, const Tuning &tu, bool illum, int min_zc, TileMap *map) {
  switch (tu.adj_variant) {
    case 1: return adj_map<1>(g, tu, illum, min_zc, map);
    case 2: return adj_map<2>(g, tu, illum, min_zc, map);
    case 3: return adj_map<3>(g, tu, illum, min_zc, map);
    default: return adj_map<0>(g, tu, illum, min_zc, map);
  }
}

hipError_t launch_forward_pool(const GradWindow *wins, int nwin, int nblocks, int n, int cur_k,
                               int prev_k, int out_k, int record, int variant, bool vd, bool fs,
                               hipStream_t stream) {
#define WFD_FP(V)                                                                              \
  return vd ? (fs ? fwd_pool_launch<V, true, true>(wins, nwin, nblocks, n, cur_k, prev_k, out_k, \
                                                   record, stream)                             \
                  : fwd_pool_launch<V, true, false>(wins, nwin, nblocks, n, cur_k, prev_k,     \
                                                    out_k, record, stream))                    \
            : (fs ? fwd_pool_launch<V, false, true>(wins, nwin, nblocks, n, cur_k, prev_k,     \
                                                    out_k, record, stream)                     \
                  : fwd_pool_launch<V, false, false>(wins, nwin, nblocks, n, cur_k, prev_k,    \
                                                     out_k, record, stream))
  switch (variant) {
    case 1: WFD_FP(1);
    case 2: WFD_FP(2);
    case 3: WFD_FP(3);
    case 4: WFD_FP(4);
    default: WFD_FP(0);
  }
#undef WFD_FP
}

hipError_t launch_adjoint_multi(const GradWindow *wins, int nwin, int nblocks, int m, int parity,
                                int wm_k, int adj_variant, bool vd, bool illum, bool fs,
                                hipStream_t stream) {
  switch (adj_variant) {
    case 1: return adj_multi_dispatch<1>(wins, nwin, nblocks, m, parity, wm_k, vd, illum, fs, stream);
    case 2: return adj_multi_dispatch<2>(wins, nwin, nblocks, m, parity, wm_k, vd, illum, fs, stream);
    case 3: return adj_multi_dispatch<3>(wins, nwin, nblocks, m, parity, wm_k, vd, illum, fs, stream);
    default: return adj_multi_dispatch<0>(wins, nwin, nblocks, m, parity, wm_k, vd, illum, fs, stream);
  }
}

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
    case 4: WFD_FWD(4);
    default: WFD_FWD(0);
  }
#undef WFD_FWD
#undef WFD_FWD1
}

int forward_tile_map(const StepGrid &g, const Tuning &tu, int min_zc, TileMap *map) {
  const bool vd = g.m2 != nullptr, fs = g.zs != kNoSurface;
  int tx = 64, ty = 16, per_cu = 4;
#define WFD_PCU(V)                                                                 \
  tx = FwdTile<V>::TX;                                                              \
  ty = FwdTile<V>::TY;                                                              \
  per_cu = (vd ? (fs ? fwd_per_cu<V, true, true>() : fwd_per_cu<V, true, false>())  \
               : (fs ? fwd_per_cu<V, false, true>() : fwd_per_cu<V, false, false>()))
  switch (tu.variant) {
    case 1: WFD_PCU(1); break;
    case 2: WFD_PCU(2); break;
    case 3: WFD_PCU(3); break;
    case 4: WFD_PCU(4); break;
    default: WFD_PCU(0); break;
  }
#undef WFD_PCU
  *map = make_map(g, tx, ty, per_cu, 0, tu.rounds, kFwdHalo, min_zc);
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
    case 4: WFD_MULTI(4);
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
    case 3: return adj_dispatch<3>(tu, g, cur, prev, out, rec, res_tm, m, wm, grad, illum, stream);
    default: return adj_dispatch<0>(tu, g, cur, prev, out, rec, res_tm, m, wm, grad, illum, stream);
  }
}

}  // namespace wfd
