// Kernels of the learned gradient preconditioner: a 3-D CNN of 3x3x3
// convolutions ("same" zero padding) with BF16 weights and activations and
// FP32 accumulation on the CDNA4 matrix cores.
//
// Layouts.  Activations are channels-last BF16 [z][y][x][C] with C in
// {1, 2, 16}.  Master weights are FP32 W[tap][ci][co] with tap = 9 kz + 3 ky +
// kx reading the input at offset (kz - 1, ky - 1, kx - 1).  For the matrix
// cores they are packed as A[16][K] BF16: row = output channel (rows past the
// layer's outputs are zero), k = tap * CIN + ci, K = 27 CIN rounded up to a
// multiple of 32 with zeros.
//
// Matrix-core mapping (v_mfma_f32_16x16x32_bf16, one wavefront, lane l,
// element e; checked on the device): A[i][k] sits in lane i + 16 (k / 8),
// element k % 8; B[k][j] in lane j + 16 (k / 8), element k % 8; the 16 x 16
// FP32 result D[i][j] in lane j + 16 (i / 4), element i % 4.
//
// Convolution as an implicit GEMM: for a row of 16 output voxels,
// D[co][voxel] = sum_k A[co][k] X[k][voxel] with X[tap * CIN + ci][voxel] =
// input[voxel + offset(tap)][ci].  A convolution block marches a 64 x 4
// output tile along z with a ring of input planes in LDS; each of its 4
// wavefronts computes one 64-voxel output row as four 16 x 16 tiles (k_conv
// for one or two input channels, k_conv16 for 16, input-plane major).  The
// data gradient is the same kernel on flipped, transposed weights; the weight
// gradient marches the same tiles and reduces over voxels with the voxel
// index as the matrix-core K dimension (k_wgrad, and k_wgrad_pack for the
// layers with one output or two input channels).
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>

#include "wfd_internal.h"

namespace wfd {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ bool bf16_pos(uint16_t b) { return b != 0 && !(b & 0x8000u); }

constexpr int kpad(int cin) { return (27 * cin + 31) / 32 * 32; }

// Convolution (forward or data gradient).  out = conv(in; A) [+ bias], then
// relu, then * (mask > 0), then (single output channel only) + channel 0 of
// res[voxel][res_c]; written as BF16 and/or FP32 channels-last with COUT
// channels.  Every output voxel of the tile is computed by exactly one lane.
//
// A block owns a 64 x 4 output tile in x-y and marches CM_ZC output planes
// along z.  Input planes (the tile plus a one-voxel halo, 66 x 6 voxels) go
// through an LDS ring; each of the 4 wavefronts computes one 64-voxel output
// row as four 16 x 16 tiles with the packed weights held in registers.  With
// one or two input channels (k_conv) all 27 taps of an output voxel fit in one
// or two K chunks: output plane z reads planes z - 1 .. z + 1 from a four-slot
// ring (plane p in slot p & 3) while plane z + 2 is fetched, into registers
// before the matrix-core work and into its slot after it, so one barrier per
// plane suffices (the slot written held plane z - 2, read only before the
// previous barrier).  With 16 input channels, k_conv16 below.
constexpr int CM_TY = 4, CM_ZC = 16, CM_THR = 256;
constexpr int CM_LX = 66, CM_LY = CM_TY + 2, CM_PLANE = CM_LX * CM_LY, CM_SLOTS = 4;
// CIN = 16: a plane is CM_PLANE * 2 sixteen-byte items, at most CM_PF per thread
constexpr int CM_PF = (CM_PLANE * 2 + CM_THR - 1) / CM_THR;

// Block b runs on XCD b mod 8, and each XCD has its own L2: tiles are
// numbered so that XCD k gets one contiguous range of them, and neighbouring
// columns (which fetch each other's halo) share an L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int per = nb / 8, rem = nb % 8, xcd = b % 8, slot = b / 8;
  return xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
}

inline int cm_tiles(int nx, int ny, int nz) {
  return ((nx + 63) / 64) * ((ny + CM_TY - 1) / CM_TY) * ((nz + CM_ZC - 1) / CM_ZC);
}

// CIN = 16: fetch plane gz into registers, then store it into its slot.
__device__ __forceinline__ void cm_fetch16(u32x4 *pf, const uint16_t *__restrict__ in, int nx,
                                           int ny, int nz, int x0, int y0, int gz) {
#pragma unroll
  for (int i = 0; i < CM_PF; ++i) {
    const int q = threadIdx.x + i * CM_THR;
    const int v = q >> 1, half = q & 1;
    const int lx = v % CM_LX, ly = v / CM_LX;
    const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
    u32x4 d = {0u, 0u, 0u, 0u};
    if (q < CM_PLANE * 2 && gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz)
      d = *reinterpret_cast<const u32x4 *>(in + (((int64_t)gz * ny + gy) * nx + gx) * 16 +
                                           8 * half);
    pf[i] = d;
  }
}
__device__ __forceinline__ void cm_store16(uint16_t *lds, int slot, const u32x4 *pf) {
#pragma unroll
  for (int i = 0; i < CM_PF; ++i) {
    const int q = threadIdx.x + i * CM_THR;
    if (q < CM_PLANE * 2)
      *reinterpret_cast<u32x4 *>(lds + (slot * CM_PLANE + (q >> 1)) * 16 + 8 * (q & 1)) = pf[i];
  }
}

// CIN = 1 or 2: fetch plane gz into registers (one voxel's channels per item),
// then store it into its slot.
constexpr int CM_PFS = (CM_PLANE + CM_THR - 1) / CM_THR;
template <int CIN>
__device__ __forceinline__ void cm_fetch_small(uint32_t *pf, const uint16_t *__restrict__ in,
                                               int nx, int ny, int nz, int x0, int y0, int gz) {
#pragma unroll
  for (int i = 0; i < CM_PFS; ++i) {
    const int v = threadIdx.x + i * CM_THR;
    const int lx = v % CM_LX, ly = v / CM_LX;
    const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
    uint32_t d = 0u;
    if (v < CM_PLANE && gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz) {
      const int64_t g = ((int64_t)gz * ny + gy) * nx + gx;
      d = CIN == 2 ? *reinterpret_cast<const uint32_t *>(in + g * 2) : (uint32_t)in[g];
    }
    pf[i] = d;
  }
}
template <int CIN>
__device__ __forceinline__ void cm_store_small(uint16_t *lds, int slot, const uint32_t *pf) {
#pragma unroll
  for (int i = 0; i < CM_PFS; ++i) {
    const int v = threadIdx.x + i * CM_THR;
    if (v >= CM_PLANE) continue;
    if (CIN == 2)
      *reinterpret_cast<uint32_t *>(lds + (slot * CM_PLANE + v) * 2) = pf[i];
    else
      lds[slot * CM_PLANE + v] = (uint16_t)pf[i];
  }
}

// B fragment of chunk c (one or two input channels) for output voxel lx of
// row ly and lane group g; sl[d] is the slot of input plane z - 1 + d.
template <int CIN>
__device__ __forceinline__ bf16x8 cm_gather(const uint16_t *lds, int c, int lx, int ly,
                                            const int *sl, int g) {
  if (CIN == 2) {  // elements (2u, 2u + 1) are both channels of tap 4 (c, g) + u
    u32x4 d;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = 16 * c + 4 * g + u;
      uint32_t val = 0u;
      if (t < 27) {
        const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
        val = *reinterpret_cast<const uint32_t *>(
            lds + (sl[dz] * CM_PLANE + (ly + dy) * CM_LX + lx + dx) * 2);
      }
      d[u] = val;
    }
    return __builtin_bit_cast(bf16x8, d);
  } else {
    u16x8 d;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 32 * c + 8 * g + e;
      const int t = k / CIN, ci = k % CIN;
      uint16_t val = 0;
      if (t < 27) {
        const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
        val = lds[(sl[dz] * CM_PLANE + (ly + dy) * CM_LX + lx + dx) * CIN + ci];
      }
      d[e] = val;
    }
    return __builtin_bit_cast(bf16x8, d);
  }
}

// Epilogue of one output row of 4 x 16 voxels: lane holds D[co = 4 g + e][voxel
// j] of each tile.  Bias, relu, the mask and (single output channel only) the
// residual, then BF16 and/or FP32 stores.
template <int COUT>
__device__ __forceinline__ void cm_epilogue(const f32x4 *acc, int nx, int ny, int z, int x0,
                                            int gy, int j, int g, const float *__restrict__ bias,
                                            int relu, const uint16_t *__restrict__ mask,
                                            const uint16_t *__restrict__ res, int res_c,
                                            uint16_t *__restrict__ out_bf,
                                            float *__restrict__ out_f) {
  if (gy >= ny) return;
#pragma unroll
  for (int tl = 0; tl < 4; ++tl) {
    const int gx = x0 + 16 * tl + j;
    if (gx >= nx) continue;
    const int64_t vox = ((int64_t)z * ny + gy) * nx + gx;
    uint16_t mk[4] = {1, 1, 1, 1};  // positive bits unless a mask is given
    if (mask) {
      if (COUT == 16) {  // the lane's four channels 4g .. 4g + 3 in one load
        const uint2 m2 = *reinterpret_cast<const uint2 *>(mask + vox * 16 + 4 * g);
        mk[0] = (uint16_t)m2.x, mk[1] = (uint16_t)(m2.x >> 16);
        mk[2] = (uint16_t)m2.y, mk[3] = (uint16_t)(m2.y >> 16);
      } else if (g == 0) {
        mk[0] = mask[vox * COUT];
      }
    }
    float v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int co = 4 * g + e;
      float s = acc[tl][e];
      if (bias && co < COUT) s += bias[co];
      if (relu) s = fmaxf(s, 0.0f);
      if (mask && co < COUT && !bf16_pos(mk[e])) s = 0.0f;
      v[e] = s;
    }
    if (COUT == 16) {
      if (out_bf) {
        const uint32_t lo = (uint32_t)to_bf16(v[0]) | ((uint32_t)to_bf16(v[1]) << 16);
        const uint32_t hi = (uint32_t)to_bf16(v[2]) | ((uint32_t)to_bf16(v[3]) << 16);
        *reinterpret_cast<uint2 *>(out_bf + vox * 16 + 4 * g) = make_uint2(lo, hi);
      }
      if (out_f)
        *reinterpret_cast<float4 *>(out_f + vox * 16 + 4 * g) =
            make_float4(v[0], v[1], v[2], v[3]);
    } else if (g == 0) {  // single output channel: co = 0 is element 0 of group 0
      if (res) v[0] += from_bf16(res[vox * res_c]);
      if (out_bf) out_bf[vox] = to_bf16(v[0]);
      if (out_f) out_f[vox] = v[0];
    }
  }
}

template <int CIN, int COUT>
__global__ void __launch_bounds__(CM_THR, 4)  // 4 waves per SIMD fit without spills; 5 spill
    k_conv(const uint16_t *__restrict__ in, int nx, int ny, int nz,
           const uint16_t *__restrict__ apk, const float *__restrict__ bias, int relu,
           const uint16_t *__restrict__ mask, const uint16_t *__restrict__ res, int res_c,
           uint16_t *__restrict__ out_bf, float *__restrict__ out_f) {
  static_assert(CIN == 1 || CIN == 2, "16 input channels: k_conv16");
  constexpr int K = kpad(CIN), NC = K / 32;
  __shared__ __attribute__((aligned(16))) uint16_t lds[CM_SLOTS * CM_PLANE * CIN + 8];
  const int tx = (nx + 63) / 64, ty = (ny + CM_TY - 1) / CM_TY;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int x0 = (tile % tx) * 64, y0 = ((tile / tx) % ty) * CM_TY;
  const int zs = (tile / (tx * ty)) * CM_ZC, ze = min(zs + CM_ZC, nz);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, g = lane >> 4;
  // weights: A fragment of every chunk (row co = j, k = 32 c + 8 g + e)
  bf16x8 a[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c)
    a[c] = __builtin_bit_cast(
        bf16x8, *reinterpret_cast<const u32x4 *>(apk + (size_t)j * K + 32 * c + 8 * g));
  // prologue: planes zs - 1 .. zs + 1
  for (int p = zs - 1; p <= zs + 1; ++p) {
    uint32_t pf[CM_PFS];
    cm_fetch_small<CIN>(pf, in, nx, ny, nz, x0, y0, p);
    cm_store_small<CIN>(lds, p & 3, pf);
  }
  __syncthreads();
  const int ly = wave, gy = y0 + ly;  // this wave's output row
#pragma unroll 1
  for (int z = zs; z < ze; ++z) {
    const bool more = z + 1 < ze;  // plane z + 2 is needed for output plane z + 1
    uint32_t pfs[CM_PFS];
    if (more) cm_fetch_small<CIN>(pfs, in, nx, ny, nz, x0, y0, z + 2);
    const int sl[3] = {(z - 1) & 3, z & 3, (z + 1) & 3};
    f32x4 acc[4];
#pragma unroll
    for (int tl = 0; tl < 4; ++tl) acc[tl] = f32x4{0.f, 0.f, 0.f, 0.f};
    // chunk-major: the four tiles' fragments of one chunk are in flight together
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      bf16x8 b[4];
#pragma unroll
      for (int tl = 0; tl < 4; ++tl) b[tl] = cm_gather<CIN>(lds, c, 16 * tl + j, ly, sl, g);
#pragma unroll
      for (int tl = 0; tl < 4; ++tl)
        acc[tl] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[c], b[tl], acc[tl], 0, 0, 0);
    }
    cm_epilogue<COUT>(acc, nx, ny, z, x0, gy, j, g, bias, relu, mask, res, res_c, out_bf, out_f);
    if (more) cm_store_small<CIN>(lds, (z + 2) & 3, pfs);
    __syncthreads();
  }
}
// Convolution with 16 input channels, input-plane major.  An input plane p
// feeds output planes p + 1, p and p - 1 through the taps kz = 0, 1, 2, so
// the K dimension is split as k = 144 kz + k' with k' = 16 (3 ky + kx) + ci
// (five chunks of 32, the last half zero): each B fragment of plane p is read
// from LDS once and used by the three kz slices of the weights, and the
// matrix-core work per output plane is 15 instead of 14 products while the
// LDS fragment reads drop from 14 to 5.  With 16 output channels the three
// kz products go to three rotating accumulators (output planes p + 1, p,
// p - 1); with one output channel the rows of A are the three kz slices of
// the single weight row, one product per chunk leaves the three partial sums
// in rows 0..2, and two running sums per voxel complete the output.  Output
// plane p - 1 is complete after input plane p.  Input planes go through a
// two-slot LDS ring (the next plane is fetched into registers during the
// matrix-core work and stored after it, one barrier per plane).
template <int COUT>
__global__ void __launch_bounds__(CM_THR, COUT == 16 ? 3 : 1)
    k_conv16(const uint16_t *__restrict__ in, int nx, int ny, int nz,
             const uint16_t *__restrict__ apk, const float *__restrict__ bias, int relu,
             const uint16_t *__restrict__ mask, const uint16_t *__restrict__ res, int res_c,
             uint16_t *__restrict__ out_bf, float *__restrict__ out_f) {
  constexpr int K = kpad(16), NC = 5, KP = 144;  // K' = 9 taps x 16 channels
  constexpr int NA = COUT == 16 ? 3 : 1;         // A fragments per chunk
  __shared__ __attribute__((aligned(16))) uint16_t lds[2 * CM_PLANE * 16 + 8];
  const int tx = (nx + 63) / 64, ty = (ny + CM_TY - 1) / CM_TY;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int x0 = (tile % tx) * 64, y0 = ((tile / tx) % ty) * CM_TY;
  const int zs = (tile / (tx * ty)) * CM_ZC, ze = min(zs + CM_ZC, nz);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, g = lane >> 4;
  // A fragments: lane (i + 16 g) holds k' = 32 c + 8 g .. + 7 of row i.
  // COUT = 16: fragment (kz, c), row i = co, kept in LDS (read once per chunk,
  // a conflict-free 16-byte read per lane), so that the kernel fits 128
  // registers and 4 waves per SIMD hide the plane loads' latency.
  // COUT = 1: a[0][c] in registers, row i = kz (rows 3..15 zero).
  __shared__ __attribute__((aligned(16))) u32x4 alds[COUT == 16 ? NA * NC * 64 : 1];
  bf16x8 a[COUT == 16 ? 1 : NA][NC];
  if (COUT == 16) {
    for (int idx = threadIdx.x; idx < NA * NC * 64; idx += CM_THR) {
      const int q = idx / (NC * 64), c = (idx / 64) % NC, ln = idx % 64;
      const int kp = 32 * c + 8 * (ln >> 4);
      u32x4 d = {0u, 0u, 0u, 0u};
      if (kp < KP) d = *reinterpret_cast<const u32x4 *>(apk + (size_t)(ln & 15) * K + KP * q + kp);
      alds[idx] = d;
    }
  } else {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int kp = 32 * c + 8 * g;
      u32x4 d = {0u, 0u, 0u, 0u};
      if (kp < KP && j < 3) d = *reinterpret_cast<const u32x4 *>(apk + KP * j + kp);
      a[0][c] = __builtin_bit_cast(bf16x8, d);
    }
  }
  {  // prologue: input plane zs - 1
    u32x4 pf[CM_PF];
    cm_fetch16(pf, in, nx, ny, nz, x0, y0, zs - 1);
    cm_store16(lds, (zs - 1) & 1, pf);
  }
  __syncthreads();
  const int ly = wave, gy = y0 + ly;  // this wave's output row
  // COUT = 16: acc[0] -> output p + 1, acc[1] -> p, acc[2] -> p - 1 (per tile)
  // COUT = 1: s1 = partial of output p, s2 = partial of output p - 1
  f32x4 acc[3][4];
  float s1[4], s2[4];
#pragma unroll
  for (int tl = 0; tl < 4; ++tl) {
    s1[tl] = s2[tl] = 0.0f;
#pragma unroll
    for (int q = 0; q < 3; ++q) acc[q][tl] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
#pragma unroll 1
  for (int p = zs - 1; p <= ze; ++p) {
    const bool more = p + 1 <= ze;
    u32x4 pf[CM_PF];
    if (more) cm_fetch16(pf, in, nx, ny, nz, x0, y0, p + 1);
    const uint16_t *pl = lds + (p & 1) * CM_PLANE * 16;
    // every input plane feeds three accumulators; those of output planes
    // outside [zs, ze) (at the first two and last two input planes) are never
    // written out, and branch-free products schedule better than skipping them
    const bool to_prev = p - 1 >= zs;
    f32x4 d[4];
#pragma unroll
    for (int tl = 0; tl < 4; ++tl) d[tl] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int t = 2 * c + (g >> 1);  // tap ky * 3 + kx of this lane's k'
      bf16x8 b[4];
#pragma unroll
      for (int tl = 0; tl < 4; ++tl) {
        u32x4 v = {0u, 0u, 0u, 0u};
        if (t < 9) {
          const int vox = (ly + t / 3) * CM_LX + 16 * tl + j + t % 3;
          v = *reinterpret_cast<const u32x4 *>(pl + vox * 16 + 8 * (g & 1));
        }
        b[tl] = __builtin_bit_cast(bf16x8, v);
      }
      if (COUT == 16) {
        const bf16x8 a0 = __builtin_bit_cast(bf16x8, alds[(0 * NC + c) * 64 + lane]);
        const bf16x8 a1 = __builtin_bit_cast(bf16x8, alds[(1 * NC + c) * 64 + lane]);
        const bf16x8 a2 = __builtin_bit_cast(bf16x8, alds[(2 * NC + c) * 64 + lane]);
#pragma unroll
        for (int tl = 0; tl < 4; ++tl) {
          acc[0][tl] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b[tl], acc[0][tl], 0, 0, 0);
          acc[1][tl] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b[tl], acc[1][tl], 0, 0, 0);
          acc[2][tl] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b[tl], acc[2][tl], 0, 0, 0);
        }
      } else {
#pragma unroll
        for (int tl = 0; tl < 4; ++tl)
          d[tl] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][c], b[tl], d[tl], 0, 0, 0);
      }
    }
    if (to_prev) {  // output plane p - 1 is complete
      if (COUT == 16) {
        cm_epilogue<COUT>(acc[2], nx, ny, p - 1, x0, gy, j, g, bias, relu, mask, res, res_c,
                          out_bf, out_f);
      } else {  // lanes of group 0 hold (P0, P1, P2) of voxel j in elements 0..2
        f32x4 o[4];
#pragma unroll
        for (int tl = 0; tl < 4; ++tl) o[tl] = f32x4{s2[tl] + d[tl][2], 0.f, 0.f, 0.f};
        cm_epilogue<COUT>(o, nx, ny, p - 1, x0, gy, j, g, bias, relu, mask, res, res_c, out_bf,
                          out_f);
      }
    }
    // rotate: output p becomes p - 1 for the next plane, p + 1 becomes p
#pragma unroll
    for (int tl = 0; tl < 4; ++tl) {
      if (COUT == 16) {
        acc[2][tl] = acc[1][tl];
        acc[1][tl] = acc[0][tl];
        acc[0][tl] = f32x4{0.f, 0.f, 0.f, 0.f};
      } else {
        s2[tl] = s1[tl] + d[tl][1];
        s1[tl] = d[tl][0];
      }
    }
    if (more) cm_store16(lds, (p + 1) & 1, pf);
    __syncthreads();
  }
}

// Weight gradient: dW[tap][ci][co] = sum over voxels v of dz[v][co] *
// in[v + offset(tap)][ci], and db[co] = sum of dz[v][co], with the voxel index
// as the matrix-core K dimension: A[co][k] = dz[voxel k][co], B[k][ci] =
// in[voxel k + offset][ci], k = 32 consecutive voxels of one output row.
//
// A block marches a 64 x 4 output tile along z like the convolution, with a
// four-slot ring of input planes and a two-slot ring of dz planes in LDS.  In
// LDS the planes are channel-planar, [row][channel][x] with rows of 80, so
// the eight consecutive voxels of one channel that a lane contributes to a
// fragment are one aligned 16-byte read.  A row stride of 40 dwords makes
// these reads free of bank conflicts (measured: strides of 36, 44 and 52
// dwords cost 4 extra cycles per read); the two plane rings then take 80 KB,
// and two blocks still fit a CU's LDS.  For the three x taps of a
// (kz, ky) pair a lane reads 10 elements once and shifts them in registers.
// Each wavefront owns one output row and accumulates all 27 taps (and the
// bias, as a product with a ones fragment) over every plane of every tile it
// visits; the grid is persistent, and each wavefront writes one row of
// partial sums that two fixed-order passes reduce.
constexpr int WG_TY = 4, WG_ZC = 16, WG_THR = 256, WG_RX = 80, WG_LY = WG_TY + 2;
constexpr int WG_ROW = 27 * 256 + 16;  // partial sums of a wavefront: [tap][co][ci], then db[co]
constexpr int WG_MAXB = 512, WG_SEG = 32;

inline int wg_tiles(int nx, int ny, int nz) {
  return ((nx + 63) / 64) * ((ny + WG_TY - 1) / WG_TY) * ((nz + WG_ZC - 1) / WG_ZC);
}

// The two channel values of voxels a (low half) and b (high half).
__device__ __forceinline__ uint32_t wg_lo(uint32_t a, uint32_t b) { return (a & 0xFFFFu) | (b << 16); }
__device__ __forceinline__ uint32_t wg_hi(uint32_t a, uint32_t b) {
  return (a >> 16) | (b & 0xFFFF0000u);
}

// Input plane gz (66 x 6 voxels from (x0 - 1, y0 - 1)) in pairs of voxels
// (lx = 2p, 2p + 1): item = (row, channel half, pair).  Fetched into
// registers, then stored as one dword per channel.
template <int CIN>
struct WgIn {
  static constexpr int HALVES = CIN == 16 ? 2 : 1;
  static constexpr int ITEMS = WG_LY * HALVES * 33;
  static constexpr int PER = (ITEMS + WG_THR - 1) / WG_THR;
  static constexpr int SLOT = WG_LY * CIN * WG_RX;  // elements per slot
  u32x4 a[PER], b[PER];
  __device__ __forceinline__ void fetch(const uint16_t *__restrict__ in, int nx, int ny, int nz,
                                        int x0, int y0, int gz) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int q = threadIdx.x + i * WG_THR;
      const int pr = q % 33, h = (q / 33) % HALVES, ly = q / (33 * HALVES);
      const int gy = y0 - 1 + ly, xa = x0 - 1 + 2 * pr;
      const bool row = q < ITEMS && gy >= 0 && gy < ny && gz >= 0 && gz < nz;
      const int64_t base = ((int64_t)gz * ny + gy) * nx;
      u32x4 va = {0u, 0u, 0u, 0u}, vb = {0u, 0u, 0u, 0u};
      if (CIN == 16) {
        if (row && xa >= 0 && xa < nx)
          va = *reinterpret_cast<const u32x4 *>(in + (base + xa) * 16 + 8 * h);
        if (row && xa + 1 < nx)
          vb = *reinterpret_cast<const u32x4 *>(in + (base + xa + 1) * 16 + 8 * h);
      } else if (CIN == 2) {  // one dword per voxel
        if (row && xa >= 0 && xa < nx) va[0] = *reinterpret_cast<const uint32_t *>(in + (base + xa) * 2);
        if (row && xa + 1 < nx) vb[0] = *reinterpret_cast<const uint32_t *>(in + (base + xa + 1) * 2);
      } else {  // CIN = 1: one element per voxel
        if (row && xa >= 0 && xa < nx) va[0] = in[base + xa];
        if (row && xa + 1 < nx) vb[0] = in[base + xa + 1];
      }
      a[i] = va;
      b[i] = vb;
    }
  }
  __device__ __forceinline__ void store(uint32_t *lds, int slot) const {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int q = threadIdx.x + i * WG_THR;
      if (q >= ITEMS) continue;
      const int pr = q % 33, h = (q / 33) % HALVES, ly = q / (33 * HALVES);
      uint32_t *d = lds + (slot * SLOT + (ly * CIN + 8 * h) * WG_RX) / 2 + pr;
      if (CIN == 16) {
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          d[(2 * w) * (WG_RX / 2)] = wg_lo(a[i][w], b[i][w]);
          d[(2 * w + 1) * (WG_RX / 2)] = wg_hi(a[i][w], b[i][w]);
        }
      } else {
        d[0] = wg_lo(a[i][0], b[i][0]);
        if (CIN == 2) d[WG_RX / 2] = wg_hi(a[i][0], b[i][0]);
      }
    }
  }
};

// dz plane gz of the output tile (64 x 4 voxels from (x0, y0)), same scheme.
template <int COUT>
struct WgDz {
  static constexpr int HALVES = COUT == 16 ? 2 : 1;
  static constexpr int ITEMS = WG_TY * HALVES * 32;
  static constexpr int PER = (ITEMS + WG_THR - 1) / WG_THR;
  static constexpr int SLOT = WG_TY * COUT * WG_RX;
  u32x4 a[PER], b[PER];
  __device__ __forceinline__ void fetch(const uint16_t *__restrict__ dz, int nx, int ny, int x0,
                                        int y0, int gz) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int q = threadIdx.x + i * WG_THR;
      const int pr = q % 32, h = (q / 32) % HALVES, r = q / (32 * HALVES);
      const int gy = y0 + r, xa = x0 + 2 * pr;
      const bool row = q < ITEMS && gy < ny;
      const int64_t base = ((int64_t)gz * ny + gy) * nx;
      u32x4 va = {0u, 0u, 0u, 0u}, vb = {0u, 0u, 0u, 0u};
      if (COUT == 16) {
        if (row && xa < nx) va = *reinterpret_cast<const u32x4 *>(dz + (base + xa) * 16 + 8 * h);
        if (row && xa + 1 < nx)
          vb = *reinterpret_cast<const u32x4 *>(dz + (base + xa + 1) * 16 + 8 * h);
      } else {  // COUT = 1: one element per voxel
        if (row && xa < nx) va[0] = dz[base + xa];
        if (row && xa + 1 < nx) vb[0] = dz[base + xa + 1];
      }
      a[i] = va;
      b[i] = vb;
    }
  }
  __device__ __forceinline__ void store(uint32_t *lds, int slot) const {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int q = threadIdx.x + i * WG_THR;
      if (q >= ITEMS) continue;
      const int pr = q % 32, h = (q / 32) % HALVES, r = q / (32 * HALVES);
      uint32_t *d = lds + (slot * SLOT + (r * COUT + 8 * h) * WG_RX) / 2 + pr;
      if (COUT == 16) {
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          d[(2 * w) * (WG_RX / 2)] = wg_lo(a[i][w], b[i][w]);
          d[(2 * w + 1) * (WG_RX / 2)] = wg_hi(a[i][w], b[i][w]);
        }
      } else {
        d[0] = wg_lo(a[i][0], b[i][0]);
      }
    }
  }
};

template <int CIN, int COUT>
__global__ void __launch_bounds__(WG_THR)
    k_wgrad(const uint16_t *__restrict__ in, const uint16_t *__restrict__ dz, int nx, int ny,
            int nz, int ntiles, float *__restrict__ partial) {
  using In = WgIn<CIN>;
  using Dz = WgDz<COUT>;
  __shared__ __attribute__((aligned(16))) uint32_t lin[4 * In::SLOT / 2];
  __shared__ __attribute__((aligned(16))) uint32_t ldz[2 * Dz::SLOT / 2];
  const uint16_t *lin16 = reinterpret_cast<const uint16_t *>(lin);
  const uint16_t *ldz16 = reinterpret_cast<const uint16_t *>(ldz);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, g = lane >> 4;
  const int tx = (nx + 63) / 64, ty = (ny + WG_TY - 1) / WG_TY;
  f32x4 acc[27];
#pragma unroll
  for (int t = 0; t < 27; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  f32x4 accb = {0.f, 0.f, 0.f, 0.f};
  const uint32_t one2 = 0x3F803F80u;  // two BF16 ones
  const bf16x8 ones = __builtin_bit_cast(bf16x8, u32x4{one2, one2, one2, one2});
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int x0 = (tile % tx) * 64, y0 = ((tile / tx) % ty) * WG_TY;
    const int zs = (tile / (tx * ty)) * WG_ZC, ze = min(zs + WG_ZC, nz);
    {  // prologue: input planes zs - 1 .. zs + 1 and dz plane zs
      In pin;
      for (int p = zs - 1; p <= zs + 1; ++p) {
        pin.fetch(in, nx, ny, nz, x0, y0, p);
        pin.store(lin, p & 3);
      }
      Dz pdz;
      pdz.fetch(dz, nx, ny, x0, y0, zs);
      pdz.store(ldz, zs & 1);
    }
    __syncthreads();
    const bool row_live = y0 + wave < ny;
#pragma unroll 1
    for (int z = zs; z < ze; ++z) {
      const bool more = z + 1 < ze;
      In nin;
      Dz ndz;
      if (more) {
        nin.fetch(in, nx, ny, nz, x0, y0, z + 2);
        ndz.fetch(dz, nx, ny, x0, y0, z + 1);
      }
      if (row_live) {
#pragma unroll
        for (int xb = 0; xb < 64; xb += 32) {
          if (x0 + xb >= nx) break;  // the chunk's dz are all zero
          u32x4 av = {0u, 0u, 0u, 0u};
          if (j < COUT)
            av = *reinterpret_cast<const u32x4 *>(
                ldz16 + (z & 1) * Dz::SLOT + (wave * COUT + j) * WG_RX + xb + 8 * g);
          const bf16x8 A = __builtin_bit_cast(bf16x8, av);
          accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, ones, accb, 0, 0, 0);
#pragma unroll
          for (int kz = 0; kz < 3; ++kz) {
            const uint16_t *pl = lin16 + ((z - 1 + kz) & 3) * In::SLOT;
#pragma unroll
            for (int ky = 0; ky < 3; ++ky) {
              u32x4 w = {0u, 0u, 0u, 0u};
              uint32_t w4 = 0u;
              if (j < CIN) {
                const uint16_t *r = pl + ((wave + ky) * CIN + j) * WG_RX + xb + 8 * g;
                w = *reinterpret_cast<const u32x4 *>(r);
                w4 = *reinterpret_cast<const uint32_t *>(r + 8);
              }
              // keep the shifted fragments in registers: without this the
              // compiler re-reads w1..w4 from LDS as dwords (bank conflicts)
              asm volatile("" : "+v"(w), "+v"(w4));
              const u32x4 s1 = {__builtin_amdgcn_alignbyte(w[1], w[0], 2),
                                __builtin_amdgcn_alignbyte(w[2], w[1], 2),
                                __builtin_amdgcn_alignbyte(w[3], w[2], 2),
                                __builtin_amdgcn_alignbyte(w4, w[3], 2)};
              const u32x4 s2 = {w[1], w[2], w[3], w4};
              const int t = 9 * kz + 3 * ky;
              acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, __builtin_bit_cast(bf16x8, w),
                                                               acc[t], 0, 0, 0);
              acc[t + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                  A, __builtin_bit_cast(bf16x8, s1), acc[t + 1], 0, 0, 0);
              acc[t + 2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                  A, __builtin_bit_cast(bf16x8, s2), acc[t + 2], 0, 0, 0);
            }
          }
        }
      }
      if (more) {
        nin.store(lin, (z + 2) & 3);
        ndz.store(ldz, (z + 1) & 1);
      }
      __syncthreads();
    }
  }
  // lane holds D[co = 4 g + e][ci = j] of every tap: each wavefront writes
  // its own partial row; the bias sums D_b[co][j] are the same for every j
  float *row = partial + ((size_t)blockIdx.x * 4 + wave) * WG_ROW;
#pragma unroll
  for (int t = 0; t < 27; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) row[t * 256 + (4 * g + e) * 16 + j] = acc[t][e];
  if (j == 0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) row[27 * 256 + 4 * g + e] = accb[e];
  }
}

// Eight consecutive elements starting s = 0, 1 or 2 elements past an aligned
// position, from the ten read there (w0..w3 and w4).
__device__ __forceinline__ u32x4 wg_shift(const u32x4 &w, uint32_t w4, int s) {
  const uint32_t sh = 2u * (uint32_t)(s & 1);
  const uint32_t n[5] = {w[0], w[1], w[2], w[3], w4};
  u32x4 r;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    r[i] = s == 2 ? n[i + 1] : __builtin_amdgcn_alignbyte(n[i + 1], n[i], sh);
  return r;
}

// Weight gradients of the layers with a single output channel (MODE 0: 16
// -> 1) or two input channels (MODE 1: 2 -> 16).  In k_wgrad these run
// 16 x 16 tiles with 15 of 16 rows (or 14 of 16 columns) zero.  Here the idle
// rows or columns carry other taps, each lane reading its operand at its own
// tap's offset:
//   MODE 0: A[tap][k] = dz[voxel k - offset(tap)], B[k][ci] = in[voxel k][ci]
//           (D = dW[tap][ci] summed over voxels k; 16 taps per product, 2
//           products per chunk, the centre tap's row of A against ones gives
//           db);
//   MODE 1: A[co][k] = dz[voxel k][co], B[k][(tap, ci)] = in[voxel k +
//           offset(tap)][ci] (8 taps x 2 channels per product, 4 products).
// The shifted operand is marched with its one-voxel halo in a four-slot ring
// (planes z - 1 .. z + 1 and the next), the other one plane at a time, as in
// k_wgrad; a lane's eight voxels of a tap are read as ten aligned elements and
// shifted in registers by its tap's x offset.
template <int MODE>
__global__ void __launch_bounds__(WG_THR)
    k_wgrad_pack(const uint16_t *__restrict__ in, const uint16_t *__restrict__ dz, int nx, int ny,
                 int nz, int ntiles, float *__restrict__ partial) {
  constexpr int RC = MODE == 0 ? 1 : 2;  // channels of the shifted (ringed) operand
  constexpr int NQ = MODE == 0 ? 2 : 4;  // shifted fragments per chunk
  using Ring = WgIn<RC>;
  using Flat = WgDz<16>;
  const uint16_t *ring_src = MODE == 0 ? dz : in;
  const uint16_t *flat_src = MODE == 0 ? in : dz;
  __shared__ __attribute__((aligned(16))) uint32_t lring[4 * Ring::SLOT / 2];
  __shared__ __attribute__((aligned(16))) uint32_t lflat[2 * Flat::SLOT / 2];
  const uint16_t *ring16 = reinterpret_cast<const uint16_t *>(lring);
  const uint16_t *flat16 = reinterpret_cast<const uint16_t *>(lflat);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, g = lane >> 4;
  const int tx = (nx + 63) / 64, ty = (ny + WG_TY - 1) / WG_TY;
  // the lane's tap and channel in each shifted fragment
  int tk[NQ], ch[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    tk[q] = MODE == 0 ? 16 * q + j : 8 * q + (j >> 1);
    ch[q] = MODE == 0 ? 0 : (j & 1);
  }
  f32x4 acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
  f32x4 accb = {0.f, 0.f, 0.f, 0.f};
  const uint32_t one2 = 0x3F803F80u;  // two BF16 ones
  const bf16x8 ones = __builtin_bit_cast(bf16x8, u32x4{one2, one2, one2, one2});
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int x0 = (tile % tx) * 64, y0 = ((tile / tx) % ty) * WG_TY;
    const int zs = (tile / (tx * ty)) * WG_ZC, ze = min(zs + WG_ZC, nz);
    {  // prologue: ring planes zs - 1 .. zs + 1 and flat plane zs
      Ring pr;
      for (int p = zs - 1; p <= zs + 1; ++p) {
        pr.fetch(ring_src, nx, ny, nz, x0, y0, p);
        pr.store(lring, p & 3);
      }
      Flat pf;
      pf.fetch(flat_src, nx, ny, x0, y0, zs);
      pf.store(lflat, zs & 1);
    }
    __syncthreads();
    const bool row_live = y0 + wave < ny;
#pragma unroll 1
    for (int z = zs; z < ze; ++z) {
      const bool more = z + 1 < ze;
      Ring nr;
      Flat nf;
      if (more) {
        nr.fetch(ring_src, nx, ny, nz, x0, y0, z + 2);
        nf.fetch(flat_src, nx, ny, x0, y0, z + 1);
      }
      if (row_live) {
#pragma unroll
        for (int xb = 0; xb < 64; xb += 32) {
          if (x0 + xb >= nx) break;  // the chunk's voxels are all outside
          const bf16x8 F = __builtin_bit_cast(
              bf16x8, *reinterpret_cast<const u32x4 *>(flat16 + (z & 1) * Flat::SLOT +
                                                       (wave * 16 + j) * WG_RX + xb + 8 * g));
          if (MODE == 1) accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F, ones, accb, 0, 0, 0);
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            u32x4 sv = {0u, 0u, 0u, 0u};
            const int t = tk[q];
            if (t < 27) {
              const int kz = t / 9, ky = (t / 3) % 3, kx = t % 3;
              const int pl = MODE == 0 ? z + 1 - kz : z - 1 + kz;
              const int row = MODE == 0 ? wave + 2 - ky : wave + ky;
              const uint16_t *r =
                  ring16 + (pl & 3) * Ring::SLOT + (row * RC + ch[q]) * WG_RX + xb + 8 * g;
              sv = wg_shift(*reinterpret_cast<const u32x4 *>(r),
                            *reinterpret_cast<const uint32_t *>(r + 8), MODE == 0 ? 2 - kx : kx);
            }
            const bf16x8 S = __builtin_bit_cast(bf16x8, sv);
            if (MODE == 0) {
              acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(S, F, acc[q], 0, 0, 0);
              if (q == 0) accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(S, ones, accb, 0, 0, 0);
            } else {
              acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F, S, acc[q], 0, 0, 0);
            }
          }
        }
      }
      if (more) {
        nr.store(lring, (z + 2) & 3);
        nf.store(lflat, (z + 1) & 1);
      }
      __syncthreads();
    }
  }
  // lane holds D[i = 4 g + e][j] of each product; one partial row per wavefront
  float *row = partial + ((size_t)blockIdx.x * 4 + wave) * WG_ROW;
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = 4 * g + e;
      if (MODE == 0) {  // D[tap = 16 q + i][ci = j]
        const int t = 16 * q + i;
        if (t < 27) row[t * 256 + j] = acc[q][e];
      } else {          // D[co = i][(tap, ci) = j]
        const int t = 8 * q + (j >> 1);
        if (t < 27) row[t * 256 + i * 16 + (j & 1)] = acc[q][e];
      }
    }
  if (MODE == 0) {  // db from the centre tap's row (13 = 4 * 3 + 1)
    if (j == 0 && g == 3) row[27 * 256] = accb[1];
  } else if (j == 0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) row[27 * 256 + 4 * g + e] = accb[e];
  }
}

// Fixed-order reduction of the wavefronts' partial rows: pass 1 sums each
// segment of WG_SEG rows in order, pass 2 sums the segment totals in order
// and scatters them into dW[tap][ci][co] and db[co].
__global__ void k_wgrad_seg(const float *__restrict__ partial, int nrows,
                            float *__restrict__ seg) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= WG_ROW) return;
  const int r0 = blockIdx.y * WG_SEG, r1 = min(r0 + WG_SEG, nrows);
  float s = 0.0f;
  for (int r = r0; r < r1; ++r) s += partial[(size_t)r * WG_ROW + col];
  seg[(size_t)blockIdx.y * WG_ROW + col] = s;
}

__global__ void k_wgrad_final(const float *__restrict__ seg, int nseg, int cin, int cout,
                              float *__restrict__ dw, float *__restrict__ db) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= WG_ROW) return;
  float s = 0.0f;
  for (int k = 0; k < nseg; ++k) s += seg[(size_t)k * WG_ROW + i];
  if (i < 27 * 256) {
    const int t = i / 256, co = (i / 16) % 16, ci = i % 16;
    if (co < cout && ci < cin) dw[(t * cin + ci) * cout + co] = s;
  } else {
    const int co = i - 27 * 256;
    if (co < cout && db) db[co] = s;
  }
}

// Pack FP32 master weights W[tap][ci][co] into the matrix-core layout.
// flip = 0: A[co][tap * cin + ci] = W[tap][ci][co]            (forward)
// flip = 1: A[ci][tap * cout + co] = W[26 - tap][ci][co]      (data gradient)
__global__ void k_pack_weights(const float *__restrict__ w, int cin, int cout, int flip,
                               uint16_t *__restrict__ apk) {
  const int rows_in = flip ? cout : cin;  // input channels of the packed conv
  const int rows_out = flip ? cin : cout;
  const int K = (27 * rows_in + 31) / 32 * 32;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 16 * K) return;
  const int r = i / K, k = i % K;
  float v = 0.0f;
  if (r < rows_out && k < 27 * rows_in) {
    const int t = k / rows_in, c = k % rows_in;
    v = flip ? w[((26 - t) * cin + r) * cout + c] : w[(t * cin + c) * cout + r];
  }
  apk[i] = to_bf16(v);
}

// Residual of the output against the target: loss partials (FP64, fixed
// order inside a block) and dy = bf16(2 (y - t) / n).
__global__ void k_mse(const float *__restrict__ y, const float *__restrict__ t, int64_t n,
                      uint16_t *__restrict__ dy, double *__restrict__ partial) {
  __shared__ double red[256];
  double s = 0.0;
  const double inv = 2.0 / (double)n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double d = (double)y[i] - (double)t[i];  // exact
    s += d * d;
    dy[i] = to_bf16((float)(inv * d));
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_sum_f64(const double *__restrict__ partial, int n, double scale,
                          double *__restrict__ out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += partial[i];
    *out = s * scale;
  }
}

// Adam (Kingma & Ba, Alg. 1) on FP32 parameters.
__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Largest |x| per block; with illum set, of x / (illum + eps * max|illum|),
// the maximum of illum being reduced from the np entries of pmax first.
__global__ void k_absmax(const float *__restrict__ x, const float *__restrict__ illum,
                         const float *__restrict__ pmax, int np, float eps, int64_t n,
                         float *__restrict__ partial) {
  __shared__ float red[256];
  __shared__ float shift;
  if (illum) {
    if (threadIdx.x == 0) {
      float m = 0.0f;
      for (int i = 0; i < np; ++i) m = fmaxf(m, pmax[i]);
      shift = eps * m;
    }
    __syncthreads();
  }
  float s = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float v = illum ? (shift > 0.0f ? x[i] / (illum[i] + shift) : x[i]) : x[i];
    s = fmaxf(s, fabsf(v));
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Network input [voxel][2]: c = grad / (illum + eps max|illum|) scaled by
// max|c|, and illum scaled by max|illum| (a channel with maximum 0 is left
// unscaled).  pi, pc: per-block maxima of |illum| and |c|.
__global__ void k_pack_input(const float *__restrict__ grad, const float *__restrict__ illum,
                             int64_t n, float eps, const float *__restrict__ pi,
                             const float *__restrict__ pc, int np, uint16_t *__restrict__ out) {
  __shared__ float mi, mc;
  if (threadIdx.x == 0) {
    float a = 0.0f, b = 0.0f;
    for (int i = 0; i < np; ++i) {
      a = fmaxf(a, pi[i]);
      b = fmaxf(b, pc[i]);
    }
    mi = a;
    mc = b;
  }
  __syncthreads();
  const float shift = eps * mi;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float c = mi > 0.0f ? grad[i] / (illum[i] + shift) : grad[i];
    out[2 * i] = to_bf16(mc > 0.0f ? c / mc : c);
    out[2 * i + 1] = to_bf16(mi > 0.0f ? illum[i] / mi : illum[i]);
  }
}


}  // namespace

int cnn_conv_blocks(int nx, int ny, int nz) { return cm_tiles(nx, ny, nz); }

hipError_t launch_conv(int cin, int cout, const uint16_t *in, int nx, int ny, int nz,
                       const uint16_t *apk, const float *bias, int relu, const uint16_t *mask,
                       const uint16_t *res, int res_c, uint16_t *out_bf, float *out_f,
                       hipStream_t stream) {
  const dim3 grid(cm_tiles(nx, ny, nz)), block(CM_THR);
#define WFD_CONV(CI, CO)                                                                      \
  hipLaunchKernelGGL((k_conv<CI, CO>), grid, block, 0, stream, in, nx, ny, nz, apk, bias, relu, \
                     mask, res, res_c, out_bf, out_f)
#define WFD_CONV16(CO)                                                                        \
  hipLaunchKernelGGL((k_conv16<CO>), grid, block, 0, stream, in, nx, ny, nz, apk, bias, relu,  \
                     mask, res, res_c, out_bf, out_f)
  if (cin == 16 && cout == 16) WFD_CONV16(16);
  else if (cin == 2 && cout == 16) WFD_CONV(2, 16);
  else if (cin == 1 && cout == 16) WFD_CONV(1, 16);
  else if (cin == 16 && cout == 1) WFD_CONV16(1);
  else return hipErrorInvalidValue;
#undef WFD_CONV16
#undef WFD_CONV
  return hipGetLastError();
}

int cnn_wgrad_blocks(int nx, int ny, int nz) { return std::min(wg_tiles(nx, ny, nz), WG_MAXB); }

// partial rows (four per block) followed by the segment totals
size_t cnn_wgrad_workspace_floats(int nx, int ny, int nz) {
  const int rows = 4 * cnn_wgrad_blocks(nx, ny, nz);
  return (size_t)(rows + (rows + WG_SEG - 1) / WG_SEG) * WG_ROW;
}

hipError_t launch_wgrad(int cin, int cout, const uint16_t *in, const uint16_t *dz, int nx, int ny,
                        int nz, float *work, float *dw, float *db, hipStream_t stream) {
  const int ntiles = wg_tiles(nx, ny, nz);
  const int nb = cnn_wgrad_blocks(nx, ny, nz), rows = 4 * nb;
  const int nseg = (rows + WG_SEG - 1) / WG_SEG;
  float *partial = work, *seg = work + (size_t)rows * WG_ROW;
#define WFD_WG(CI, CO)                                                                          \
  hipLaunchKernelGGL((k_wgrad<CI, CO>), dim3(nb), dim3(WG_THR), 0, stream, in, dz, nx, ny, nz, \
                     ntiles, partial)
#define WFD_WGP(M)                                                                            \
  hipLaunchKernelGGL((k_wgrad_pack<M>), dim3(nb), dim3(WG_THR), 0, stream, in, dz, nx, ny, nz, \
                     ntiles, partial)
  if (cin == 16 && cout == 16) WFD_WG(16, 16);
  else if (cin == 2 && cout == 16) WFD_WGP(1);
  else if (cin == 16 && cout == 1) WFD_WGP(0);
  else return hipErrorInvalidValue;
#undef WFD_WG
#undef WFD_WGP
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int cb = (WG_ROW + 255) / 256;
  hipLaunchKernelGGL(k_wgrad_seg, dim3(cb, nseg), dim3(256), 0, stream, partial, rows, seg);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_wgrad_final, dim3(cb), dim3(256), 0, stream, seg, nseg, cin, cout, dw, db);
  return hipGetLastError();
}

hipError_t launch_pack_weights(const float *w, int cin, int cout, int flip, uint16_t *apk,
                               hipStream_t stream) {
  const int rows_in = flip ? cout : cin;
  const int n = 16 * ((27 * rows_in + 31) / 32 * 32);
  hipLaunchKernelGGL(k_pack_weights, dim3((n + 255) / 256), dim3(256), 0, stream, w, cin, cout,
                     flip, apk);
  return hipGetLastError();
}

hipError_t launch_mse(const float *y, const float *t, int64_t n, uint16_t *dy, double *partial,
                      int npart, double *loss, hipStream_t stream) {
  hipLaunchKernelGGL(k_mse, dim3(npart), dim3(256), 0, stream, y, t, n, dy, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(64), 0, stream, partial, npart, 1.0 / (double)n,
                     loss);
  return hipGetLastError();
}

hipError_t launch_adam(float *w, const float *g, float *m, float *v, int n, float lr, float b1,
                       float b2, float eps, int step, hipStream_t stream) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, stream, w, g, m, v, n, lr, b1,
                     b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_pack_input(const float *grad, const float *illum, int64_t n, float eps,
                             float *partial, int npart, uint16_t *out, hipStream_t stream) {
  float *pi = partial, *pc = partial + npart;
  hipLaunchKernelGGL(k_absmax, dim3(npart), dim3(256), 0, stream, illum, nullptr, nullptr, 0, 0.0f,
                     n, pi);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_absmax, dim3(npart), dim3(256), 0, stream, grad, illum, pi, npart, eps, n,
                     pc);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pack_input, dim3(npart), dim3(256), 0, stream, grad, illum, n, eps, pi, pc,
                     npart, out);
  return hipGetLastError();
}

}  // namespace wfd
