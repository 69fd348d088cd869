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
#include <type_traits>

#include "wfd_internal.h"

namespace wfd {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

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
// ring (plane p in slot p & 3); plane z + 2 was fetched into registers during
// iteration z - 1 and goes into its slot after the matrix-core work, so one
// barrier per plane suffices (the slot written held plane z - 2, read only
// before the previous barrier), and each load has a whole iteration of other
// work before it is waited for.  With 16 input channels, k_conv16 below.
//
// The march issues little besides its loads, LDS reads and matrix-core
// products: global memory is addressed through raw buffer resources, one per
// plane, and an access at an offset past a resource's size reads zero (a
// store is dropped).  Halo voxels outside the volume and output voxels past
// its edge get an offset beyond every plane (kFarVox) once, before the march,
// so the march has no per-lane bounds branches; every per-lane address is
// likewise computed once, and the fragments of taps past the last one read a
// zeroed LDS pad.  Offsets are 32-bit: a plane holds at most 2^24 voxels (the
// host checks).
constexpr int CM_TY = 4, CM_ZC = 16, CM_THR = 256;
constexpr int CM_LX = 66, CM_LY = CM_TY + 2, CM_PLANE = CM_LX * CM_LY, CM_SLOTS = 4;
// CIN = 16: a plane is CM_PLANE * 2 sixteen-byte items, at most CM_PF per thread
constexpr int CM_PF = (CM_PLANE * 2 + CM_THR - 1) / CM_THR;
// CIN = 1 or 2: a plane is CM_PLANE voxels, at most CM_PFS per thread
constexpr int CM_PFS = (CM_PLANE + CM_THR - 1) / CM_THR;
constexpr uint32_t kFarVox = 1u << 25;  // voxel index of "outside": every offset from it misses

// Calls f(integral_constant<int, 0>), ..., f(integral_constant<int, N - 1>).
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (N > 0) {
    static_for<N - 1>(f);
    f(std::integral_constant<int, N - 1>{});
  }
}

typedef __amdgpu_buffer_rsrc_t Rsrc;

// Raw buffer resource over `bytes` bytes from p (stride 0, 32-bit data format).
__device__ __forceinline__ Rsrc buf(const void *p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes,
                                           0x00020000);
}

// Plane gz of a channels-last BF16 volume with c channels and pv voxels per
// plane; an empty resource for a plane outside [0, nz).
__device__ __forceinline__ Rsrc plane_buf(const uint16_t *v, int64_t pv, int c, int nz, int gz) {
  const bool ok = gz >= 0 && gz < nz;
  return buf(v + (ok ? (int64_t)gz * pv * c : 0), ok ? (uint32_t)(pv * c * 2) : 0u);
}

// Two floats -> two BF16 (round to nearest even) in one dword, low first.
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){lo, hi}, bf16x2));
}

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

// Byte offset within an input plane of the halo voxel v of the tile at
// (x0, y0) (v = 66 ly + lx), times `bytes` per voxel; far outside the volume.
__device__ __forceinline__ uint32_t halo_offset(int v, int nx, int ny, int x0, int y0,
                                                uint32_t bytes, int nvox = CM_PLANE) {
  const int lx = v % CM_LX, ly = v / CM_LX;
  const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
  const bool ok = v < nvox && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
  return (ok ? (uint32_t)(gy * nx + gx) : kFarVox) * bytes;
}

// Output voxel indices within a plane of this lane's four tiles (x0 + 16 tl +
// j, row gy); kFarVox past the volume, and (single output channel) for lanes
// outside group 0, which hold no output.
template <int COUT>
__device__ __forceinline__ void out_voxels(uint32_t *vo, int nx, int ny, int x0, int gy, int j,
                                           int g) {
#pragma unroll
  for (int tl = 0; tl < 4; ++tl) {
    const int gx = x0 + 16 * tl + j;
    const bool ok = gx < nx && gy < ny && (COUT == 16 || g == 0);
    vo[tl] = ok ? (uint32_t)(gy * nx + gx) : kFarVox;
  }
}

// Per-voxel inputs of the epilogue of one output row: COUT = 16: the mask of
// the lane's channels 4 g .. 4 g + 3 per tile; COUT = 1: the mask (m[tl].x)
// and the residual.  Loaded early (epi_load) so that the march does not wait
// on them at the epilogue.
//
// BF (branch-free; the 16 -> 16 convolution): loads and stores go through
// resources that are empty for an absent option or an unwanted plane (ok
// false) instead of being skipped by a branch.  The compiler can then count
// the accesses in flight exactly instead of waiting for all of them; that
// took the 16 -> 16 convolution at 256^3 from 330 to 294 us, but made the
// one- and two-channel marches and the 16 -> 1 layer slower (148 -> 175 and
// 176 -> 222 us), which keep the branches.
struct EpiIn {
  u32x2 m[4];
  float r[4];
};

template <int COUT, bool BF = false>
__device__ __forceinline__ void epi_load(EpiIn &ei, int z, bool ok, int64_t pv,
                                         const uint32_t *vo, int g,
                                         const uint16_t *__restrict__ mask,
                                         const uint16_t *__restrict__ res, int res_c) {
  const int64_t zo = (int64_t)z * pv;
  const uint32_t n = (uint32_t)pv;
  const bool has_m = ok && mask, has_r = ok && res;
  if (BF || has_m) {
    const Rsrc rm = buf(has_m ? mask + zo * COUT : nullptr, has_m ? n * COUT * 2 : 0u);
#pragma unroll
    for (int tl = 0; tl < 4; ++tl)
      ei.m[tl] = COUT == 16 ? __builtin_amdgcn_raw_buffer_load_b64(rm, vo[tl] * 32u + 8u * (uint32_t)g, 0, 0)
                            : u32x2{(uint32_t)__builtin_amdgcn_raw_buffer_load_b16(rm, vo[tl] * 2u, 0, 0), 0u};
  }
  if (COUT == 1 && (BF || has_r)) {
    const Rsrc rr = buf(has_r ? res + zo * res_c : nullptr, has_r ? n * (uint32_t)res_c * 2 : 0u);
#pragma unroll
    for (int tl = 0; tl < 4; ++tl)
      ei.r[tl] = from_bf16(__builtin_amdgcn_raw_buffer_load_b16(rr, vo[tl] * (uint32_t)res_c * 2u, 0, 0));
  }
}

// Epilogue of one output row of 4 x 16 voxels in plane z: lane holds D[co =
// 4 g + e][voxel j] of each tile (single output channel: co = 0 in element 0
// of group 0).  Bias (bco: the lane's channels), relu, the mask and (single
// output channel) the residual from ei, then BF16 and/or FP32 stores.
template <int COUT, bool BF = false>
__device__ __forceinline__ void cm_epilogue(const f32x4 *acc, int z, bool ok, int64_t pv,
                                            const uint32_t *vo, const float *bco, int g,
                                            int relu, bool mask, bool res, const EpiIn &ei,
                                            uint16_t *__restrict__ out_bf,
                                            float *__restrict__ out_f) {
  const int64_t zo = (int64_t)z * pv;
  const uint32_t n = (uint32_t)pv;
  const bool has_bf = ok && out_bf, has_f = ok && out_f;
  const Rsrc rb = buf(has_bf ? out_bf + zo * COUT : nullptr, has_bf ? n * COUT * 2 : 0u);
  const Rsrc rf = buf(has_f ? out_f + zo * COUT : nullptr, has_f ? n * COUT * 4 : 0u);
#pragma unroll
  for (int tl = 0; tl < 4; ++tl) {
    float v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = acc[tl][e] + bco[e];
    if (relu) {
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = fmaxf(v[e], 0.0f);
    }
    if (COUT == 16) {
      const uint32_t ob = vo[tl] * 32u + 8u * (uint32_t)g;  // channels 4g .. 4g + 3, BF16
      if (mask) {
        const u32x2 m = ei.m[tl];
        v[0] = bf16_pos((uint16_t)m.x) ? v[0] : 0.0f;
        v[1] = bf16_pos((uint16_t)(m.x >> 16)) ? v[1] : 0.0f;
        v[2] = bf16_pos((uint16_t)m.y) ? v[2] : 0.0f;
        v[3] = bf16_pos((uint16_t)(m.y >> 16)) ? v[3] : 0.0f;
      }
      if (BF || has_bf)
        __builtin_amdgcn_raw_buffer_store_b64((u32x2){pack_bf16(v[0], v[1]), pack_bf16(v[2], v[3])},
                                              rb, ob, 0, 0);
      if (BF || has_f)
        __builtin_amdgcn_raw_buffer_store_b128(
            (u32x4){__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]),
                    __float_as_uint(v[3])},
            rf, vo[tl] * 64u + 16u * (uint32_t)g, 0, 0);
    } else {
      const uint32_t o = vo[tl];
      if (mask) v[0] = bf16_pos((uint16_t)ei.m[tl].x) ? v[0] : 0.0f;
      if (res) v[0] += ei.r[tl];
      if (BF || has_bf)
        __builtin_amdgcn_raw_buffer_store_b16((uint16_t)pack_bf16(v[0], 0.0f), rb, o * 2u, 0, 0);
      if (BF || has_f) __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v[0]), rf, o * 4u, 0, 0);
    }
  }
}

// Bias of the lane's output channels (4 g + e; single output channel: 0).
template <int COUT>
__device__ __forceinline__ void lane_bias(float *bco, const float *__restrict__ bias, int g) {
#pragma unroll
  for (int e = 0; e < 4; ++e) bco[e] = bias ? bias[COUT == 16 ? 4 * g + e : 0] : 0.0f;
}

// CIN = 1 or 2 (k_conv): a block owns a 64 x 8 output tile, each wavefront
// two consecutive rows, so that every plane load and barrier is shared by
// twice the matrix-core work (these marches wait on load latency, not on
// bandwidth).  A ring slot holds one halo plane, 66 x 10 voxels of CIN BF16
// channels; the zeroed pad after the four slots serves taps past 26 (offsets
// up to one row and 3 tiles of 16 voxels on).
constexpr int KC_RW = 2, KC_TY = 4 * KC_RW, KC_LY = KC_TY + 2, KC_PLANE = CM_LX * KC_LY;
constexpr int KC_PFS = (KC_PLANE + CM_THR - 1) / CM_THR;
template <int CIN>
struct SmallRing {
  static constexpr uint32_t ROW = CM_LX * CIN * 2;  // bytes of a halo row
  static constexpr uint32_t SLOT = KC_PLANE * CIN * 2;
  static constexpr uint32_t PAD = CM_SLOTS * SLOT;
  static constexpr uint32_t PAD_BYTES = ROW + 3 * 16 * CIN * 2 + 16;
  static constexpr uint32_t BYTES = PAD + PAD_BYTES;
};

inline int kc_tiles(int nx, int ny, int nz) {
  return ((nx + 63) / 64) * ((ny + KC_TY - 1) / KC_TY) * ((nz + CM_ZC - 1) / CM_ZC);
}

template <int CIN, int COUT>
__global__ void __launch_bounds__(CM_THR, 3)
    k_conv(const uint16_t *__restrict__ in, int nx, int ny, int nz,
           const uint16_t *__restrict__ apk, const float *__restrict__ bias, int relu,
           const uint16_t *__restrict__ mask, const uint16_t *__restrict__ res, int res_c,
           uint16_t *__restrict__ out_bf, float *__restrict__ out_f) {
  static_assert(CIN == 1 || CIN == 2, "16 input channels: k_conv16");
  using RG = SmallRing<CIN>;
  constexpr int K = kpad(CIN), NC = K / 32;
  constexpr int NE = CIN == 2 ? 4 : 8;  // LDS reads per fragment: one per tap
  __shared__ __attribute__((aligned(16))) char lds[(RG::BYTES + 15) / 16 * 16];
  const int tx = (nx + 63) / 64, ty = (ny + KC_TY - 1) / KC_TY;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int x0 = (tile % tx) * 64, y0 = ((tile / tx) % ty) * KC_TY;
  const int zs = (tile / (tx * ty)) * CM_ZC, ze = min(zs + CM_ZC, nz);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, g = lane >> 4;
  const int64_t pv = (int64_t)nx * ny;
  // weights: A fragment of every chunk (row co = j, k = 32 c + 8 g + e)
  bf16x8 a[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c)
    a[c] = __builtin_bit_cast(
        bf16x8, *reinterpret_cast<const u32x4 *>(apk + (size_t)j * K + 32 * c + 8 * g));
  // (loaded before the prologue, whose stores wait for them too: the march
  // then never waits on a load older than its own)
  float bco[4];
  lane_bias<COUT>(bco, bias, g);
  for (uint32_t i = threadIdx.x * 4; i < RG::PAD_BYTES; i += CM_THR * 4)
    *reinterpret_cast<uint32_t *>(lds + RG::PAD + i) = 0u;
  uint32_t fo[KC_PFS];
#pragma unroll
  for (int i = 0; i < KC_PFS; ++i)
    fo[i] = halo_offset(threadIdx.x + i * CM_THR, nx, ny, x0, y0, CIN * 2, KC_PLANE);
  auto fetch = [&](uint32_t *pf, int gz) {
    const Rsrc r = plane_buf(in, pv, CIN, nz, gz);
#pragma unroll
    for (int i = 0; i < KC_PFS; ++i)
      pf[i] = CIN == 2 ? __builtin_amdgcn_raw_buffer_load_b32(r, fo[i], 0, 0)
                       : (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, fo[i], 0, 0);
  };
  auto store = [&](int gz, const uint32_t *pf) {
    char *s = lds + (gz & 3) * RG::SLOT;
#pragma unroll
    for (int i = 0; i < KC_PFS; ++i) {
      const int v = threadIdx.x + i * CM_THR;
      if (i + 1 < KC_PFS || v < KC_PLANE) {
        if (CIN == 2)
          *reinterpret_cast<uint32_t *>(s + v * 4) = pf[i];
        else
          *reinterpret_cast<uint16_t *>(s + v * 2) = (uint16_t)pf[i];
      }
    }
  };
  for (int p = zs - 1; p <= zs + 1; ++p) {  // prologue: planes zs - 1 .. zs + 1
    uint32_t pf[KC_PFS];
    fetch(pf, p);
    store(p, pf);
  }
  // planes are loaded an iteration before their use, into register sets A and
  // B that alternate (the loop is unrolled twice, so that no register copy
  // waits on a load in flight)
  uint32_t pfA[KC_PFS], pfB[KC_PFS];
  fetch(pfA, zs + 2);
  const int ly = KC_RW * wave;  // this wave's first output row in the tile
  // The LDS read of tap element (c, e) of this lane for the first row: plane
  // z - 1 + dz[c][e] at byte offset to[c][e] (tile 0; tile tl is 16 tl voxels
  // on, the second row one halo row on), or the pad (dz = 3) past the last
  // tap.  CIN = 2: element e is the channel pair of tap 16 c + 4 g + e;
  // CIN = 1: the channel of tap 32 c + 8 g + e.
  int dz[NC][NE];
  uint32_t to[NC][NE];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int t = CIN == 2 ? 16 * c + 4 * g + e : 32 * c + 8 * g + e;
      const int kz = t / 9, ky = (t / 3) % 3, kx = t % 3;
      dz[c][e] = t < 27 ? kz : 3;
      to[c][e] = t < 27 ? (uint32_t)(((ly + ky) * CM_LX + j + kx) * CIN * 2) : 0u;
    }
  uint32_t vo[KC_RW][4];
#pragma unroll
  for (int r = 0; r < KC_RW; ++r) out_voxels<COUT>(vo[r], nx, ny, x0, y0 + ly + r, j, g);
  __syncthreads();
  // output plane z from planes z - 1 .. z + 1; cur holds plane z + 2, nxt
  // receives plane z + 3
  auto step = [&](int z, uint32_t *cur, uint32_t *nxt) {
    const bool more = z + 1 < ze;  // plane z + 2 is needed for output plane z + 1
    if (z + 2 < ze) fetch(nxt, z + 3);
    EpiIn ei[KC_RW];
#pragma unroll
    for (int r = 0; r < KC_RW; ++r)
      epi_load<COUT>(ei[r], z, true, pv, vo[r], g, mask, res, res_c);
    const uint32_t sb0 = ((z - 1) & 3) * RG::SLOT, sb1 = (z & 3) * RG::SLOT,
                   sb2 = ((z + 1) & 3) * RG::SLOT;
    f32x4 acc[KC_RW][4];
    // chunk-major: the tiles' fragments of one chunk are in flight together
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      uint32_t ad[NE];
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const int d = dz[c][e];
        ad[e] = to[c][e] + (d == 0 ? sb0 : d == 1 ? sb1 : d == 2 ? sb2 : RG::PAD);
      }
#pragma unroll
      for (int r = 0; r < KC_RW; ++r) {
        bf16x8 b[4];
#pragma unroll
        for (int tl = 0; tl < 4; ++tl) {
          if (CIN == 2) {
            u32x4 d;
#pragma unroll
            for (int e = 0; e < 4; ++e)
              d[e] = *reinterpret_cast<const uint32_t *>(lds + ad[e] + r * RG::ROW + 64 * tl);
            b[tl] = __builtin_bit_cast(bf16x8, d);
          } else {
            u16x8 d;
#pragma unroll
            for (int e = 0; e < 8; ++e)
              d[e] = *reinterpret_cast<const uint16_t *>(lds + ad[e] + r * RG::ROW + 32 * tl);
            b[tl] = __builtin_bit_cast(bf16x8, d);
          }
        }
#pragma unroll
        for (int tl = 0; tl < 4; ++tl)
          acc[r][tl] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              a[c], b[tl], c == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : acc[r][tl], 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < KC_RW; ++r)
      cm_epilogue<COUT>(acc[r], z, true, pv, vo[r], bco, g, relu, mask, res, ei[r], out_bf,
                        out_f);
    if (more) store(z + 2, cur);
    __syncthreads();
  };
#pragma unroll 1
  for (int z = zs; z < ze; z += 2) {
    step(z, pfA, pfB);
    if (z + 1 < ze) step(z + 1, pfB, pfA);
  }
}

// Convolution with 16 input channels, input-plane major.  An input plane p
// feeds output planes p + 1, p and p - 1 through the taps kz = 0, 1, 2, so
// the K dimension is split as k = 144 kz + k' with k' = 16 (3 ky + kx) + ci
// (five chunks of 32, the last half zero): each B fragment of plane p is read
// from LDS once and used by the three kz slices of the weights, and the
// matrix-core work per output plane is 15 instead of 14 products while the
// LDS fragment reads drop from 14 to 5.  With 16 output channels the three
// kz products go to three accumulators whose roles (output planes p + 1, p,
// p - 1) rotate with p: the plane loop is unrolled three times so that the
// rotation is a renaming, and the accumulator of output p + 1 starts from
// its first product.  With one output channel the rows of A are the three kz
// slices of the single weight row, one product per chunk leaves the three
// partial sums in rows 0..2, and two running sums per voxel complete the
// output.  Output plane p - 1 is complete after input plane p.  Input planes
// go through a two-slot LDS ring (the next plane is fetched into registers
// during the matrix-core work and stored after it, one barrier per plane);
// each slot is followed by a zeroed pad that the fragments of k' >= 144 read.
//
// RW output rows per wavefront: a block owns a 64 x 4 RW tile and every
// plane load, LDS weight-fragment read and barrier serves RW rows of
// products.
template <int RW>
struct C16 {
  static constexpr int TY = 4 * RW, LY = TY + 2, VOX = CM_LX * LY;  // halo plane
  static constexpr int ITEMS = VOX * 2;                             // 16-byte halves
  static constexpr int PF = (ITEMS + CM_THR - 1) / CM_THR;
  static constexpr uint32_t ROW = CM_LX * 32;                       // bytes of a halo row
  static constexpr uint32_t PLANE = VOX * 32;
  // zeroed pad read by the fragments of k' >= 144: up to RW - 1 rows and
  // three tiles on, one item
  static constexpr uint32_t PAD = (RW - 1) * ROW + 3 * 16 * 32 + 16;
  static constexpr uint32_t SLOT = PLANE + PAD;
};
constexpr int C16_RW16 = 2;  // rows per wavefront with 16 output channels
template <int COUT>
constexpr int c16_rw() { return COUT == 16 ? C16_RW16 : 1; }

inline int c16_tiles(int rw, int nx, int ny, int nz) {
  return ((nx + 63) / 64) * ((ny + 4 * rw - 1) / (4 * rw)) * ((nz + CM_ZC - 1) / CM_ZC);
}

// Occupancy: 16 output channels, 2 waves per SIMD (two rows per wavefront
// take about 230 registers); one output channel, 4 (110 registers; with no
// bound the compiler took 120 and the 16 -> 1 layer ran 164 against 157 us).
template <int COUT>
__global__ void __launch_bounds__(CM_THR, COUT == 16 ? 2 : 4)
    k_conv16(const uint16_t *__restrict__ in, int nx, int ny, int nz,
             const uint16_t *__restrict__ apk, const float *__restrict__ bias, int relu,
             const uint16_t *__restrict__ mask, const uint16_t *__restrict__ res, int res_c,
             uint16_t *__restrict__ out_bf, float *__restrict__ out_f) {
  constexpr int RW = c16_rw<COUT>();
  using G = C16<RW>;
  constexpr int K = kpad(16), NC = 5, KP = 144;  // K' = 9 taps x 16 channels
  constexpr int NA = COUT == 16 ? 3 : 1;         // A fragments per chunk
  __shared__ __attribute__((aligned(16))) char lds[2 * G::SLOT];
  const int tx = (nx + 63) / 64, ty = (ny + G::TY - 1) / G::TY;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int x0 = (tile % tx) * 64, y0 = ((tile / tx) % ty) * G::TY;
  const int zs = (tile / (tx * ty)) * CM_ZC, ze = min(zs + CM_ZC, nz);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, g = lane >> 4;
  const int64_t pv = (int64_t)nx * ny;
  // A fragments: lane (i + 16 g) holds k' = 32 c + 8 g .. + 7 of row i.
  // COUT = 16: fragment (kz, c), row i = co, kept in LDS (read once per chunk,
  // a conflict-free 16-byte read per lane) to leave registers for the
  // accumulators.  COUT = 1: a[0][c] in registers, row i = kz (rows 3..15 zero).
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
  float bco[4];  // before the prologue, whose stores wait for it too
  lane_bias<COUT>(bco, bias, g);
  for (uint32_t i = threadIdx.x * 16; i < 2 * G::PAD; i += CM_THR * 16) {
    const uint32_t s = i / G::PAD, o = i % G::PAD;
    *reinterpret_cast<u32x4 *>(lds + s * G::SLOT + G::PLANE + o) = u32x4{0u, 0u, 0u, 0u};
  }
  // this thread's items (16-byte halves of halo voxels) of a plane
  uint32_t fo[G::PF];
#pragma unroll
  for (int i = 0; i < G::PF; ++i) {
    const int q = threadIdx.x + i * CM_THR;
    fo[i] = halo_offset(q >> 1, nx, ny, x0, y0, 32, G::VOX) + 16u * (q & 1);
  }
  auto fetch = [&](u32x4 *pf, int gz, bool ok) {  // ok false: zeros, no traffic
    const Rsrc r = plane_buf(in, pv, 16, ok ? nz : 0, gz);
#pragma unroll
    for (int i = 0; i < G::PF; ++i) pf[i] = __builtin_amdgcn_raw_buffer_load_b128(r, fo[i], 0, 0);
  };
  auto store = [&](int gz, const u32x4 *pf) {
    char *s = lds + (gz & 1) * G::SLOT;
#pragma unroll
    for (int i = 0; i < G::PF; ++i) {
      const int q = threadIdx.x + i * CM_THR;
      if (i + 1 < G::PF || q < G::ITEMS) *reinterpret_cast<u32x4 *>(s + q * 16) = pf[i];
    }
  };
  {  // prologue: input plane zs - 1
    u32x4 pf[G::PF];
    fetch(pf, zs - 1, true);
    store(zs - 1, pf);
  }
  const int ly = RW * wave;  // this wave's first output row in the tile
  // B fragment of chunk c for the first row: taps t = 2 c + (g >> 1) (ky =
  // t / 3, kx = t % 3), channels 8 (g & 1) .. + 7, at byte bo[c] of a slot
  // (tile 0; tile tl is 16 voxels on, row r one halo row on); t = 9 (the zero
  // half of chunk 4) reads the pad.
  uint32_t bo[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int t = 2 * c + (g >> 1);
    bo[c] = t < 9 ? (uint32_t)(((ly + t / 3) * CM_LX + j + t % 3) * 32 + 16 * (g & 1)) : G::PLANE;
  }
  uint32_t vo[RW][4];
#pragma unroll
  for (int r = 0; r < RW; ++r) out_voxels<COUT>(vo[r], nx, ny, x0, y0 + ly + r, j, g);
  __syncthreads();
  // COUT = 16: acc[r][s] accumulates output plane o of row r with
  // (o - zs + 1) mod 3 = s.  COUT = 1: s1 = partial of output p, s2 = partial
  // of output p - 1.
  f32x4 acc[RW][3][4];
  float s1[RW][4], s2[RW][4];
#pragma unroll
  for (int r = 0; r < RW; ++r)
#pragma unroll
    for (int tl = 0; tl < 4; ++tl) {
      s1[r][tl] = s2[r][tl] = 0.0f;
#pragma unroll
      for (int q = 0; q < 3; ++q) acc[r][q][tl] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  // Input plane p (p = zs - 1 .. ze); R = (p - zs + 1) mod 3 fixes the
  // accumulators' roles.  BF (16 output channels, see EpiIn): no memory
  // access is skipped by a branch, the epilogue's loads go first, and the
  // loop below runs whole groups of three planes.
  constexpr bool BF = COUT == 16;
  auto sub = [&](auto Rc, int p) {
    constexpr int R = decltype(Rc)::value;
    constexpr int SN = (R + 1) % 3, SC = R, SP = (R + 2) % 3;  // outputs p + 1, p, p - 1
    const bool more = p + 1 <= ze;
    const bool done = p - 1 >= zs;  // output plane p - 1 is complete after this plane
    u32x4 pf[G::PF];
    if (!BF && more) fetch(pf, p + 1, true);
    EpiIn ei[RW];
    if (BF || done) {
#pragma unroll
      for (int r = 0; r < RW; ++r)
        epi_load<COUT, BF>(ei[r], p - 1, done, pv, vo[r], g, mask, res, res_c);
    }
    if (BF) fetch(pf, p + 1, more);
    const char *pl = lds + (p & 1) * G::SLOT;
    // every input plane feeds three accumulators; those of output planes
    // outside [zs, ze) (at the first two and last two input planes) are
    // never written out, and branch-free products schedule better than
    // skipping them
    f32x4 d[RW][4];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      bf16x8 a0, a1, a2;
      if (COUT == 16) {
        a0 = __builtin_bit_cast(bf16x8, alds[(0 * NC + c) * 64 + lane]);
        a1 = __builtin_bit_cast(bf16x8, alds[(1 * NC + c) * 64 + lane]);
        a2 = __builtin_bit_cast(bf16x8, alds[(2 * NC + c) * 64 + lane]);
      }
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        bf16x8 b[4];
#pragma unroll
        for (int tl = 0; tl < 4; ++tl)
          b[tl] = __builtin_bit_cast(
              bf16x8, *reinterpret_cast<const u32x4 *>(pl + bo[c] + r * G::ROW + 512 * tl));
        if (COUT == 16) {
#pragma unroll
          for (int tl = 0; tl < 4; ++tl) {
            acc[r][SN][tl] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                a0, b[tl], c == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : acc[r][SN][tl], 0, 0, 0);
            acc[r][SC][tl] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b[tl], acc[r][SC][tl], 0, 0, 0);
            acc[r][SP][tl] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b[tl], acc[r][SP][tl], 0, 0, 0);
          }
        } else {
#pragma unroll
          for (int tl = 0; tl < 4; ++tl)
            d[r][tl] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                a[0][c], b[tl], c == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : d[r][tl], 0, 0, 0);
        }
      }
    }
    if (BF || done) {  // output plane p - 1 (BF: its stores are dropped unless done)
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        if (COUT == 16) {
          cm_epilogue<COUT, BF>(acc[r][SP], p - 1, done, pv, vo[r], bco, g, relu, mask, res,
                                ei[r], out_bf, out_f);
        } else {  // lanes of group 0 hold (P0, P1, P2) of voxel j in elements 0..2
          f32x4 o[4];
#pragma unroll
          for (int tl = 0; tl < 4; ++tl) o[tl] = f32x4{s2[r][tl] + d[r][tl][2], 0.f, 0.f, 0.f};
          cm_epilogue<COUT, BF>(o, p - 1, done, pv, vo[r], bco, g, relu, mask, res, ei[r],
                                out_bf, out_f);
        }
      }
    }
    if (COUT == 1) {
#pragma unroll
      for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int tl = 0; tl < 4; ++tl) {
          s2[r][tl] = s1[r][tl] + d[r][tl][1];
          s1[r][tl] = d[r][tl][0];
        }
    }
    if (more) store(p + 1, pf);
    __syncthreads();
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  int p0 = zs - 1;
  if (BF) {  // whole groups in the loop, the last one or two planes after it
#pragma unroll 1
    for (; p0 + 2 <= ze; p0 += 3) {
      sub(I0{}, p0);
      sub(I1{}, p0 + 1);
      sub(I2{}, p0 + 2);
    }
    if (p0 <= ze) sub(I0{}, p0);
    if (p0 + 1 <= ze) sub(I1{}, p0 + 1);
  } else {
#pragma unroll 1
    for (; p0 <= ze; p0 += 3) {
      sub(I0{}, p0);
      if (p0 + 1 <= ze) sub(I1{}, p0 + 1);
      if (p0 + 2 <= ze) sub(I2{}, p0 + 2);
    }
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
// registers, then stored as one dword per channel.  init() computes, once per
// tile, each item's byte offsets in a plane (kFarVox-based past the volume,
// so that the buffer loads read zero) and its LDS position.
template <int CIN>
struct WgIn {
  static constexpr int HALVES = CIN == 16 ? 2 : 1;
  static constexpr int ITEMS = WG_LY * HALVES * 33;
  static constexpr int PER = (ITEMS + WG_THR - 1) / WG_THR;
  static constexpr int SLOT = WG_LY * CIN * WG_RX;  // elements per slot
  static constexpr uint32_t VB = CIN * 2;           // bytes per voxel
  struct Data {
    u32x4 a[PER], b[PER];
  };
  uint32_t oa[PER], ob[PER];  // byte offsets of voxels xa and xa + 1
  int ld[PER];                // dword offset in a slot, -1 past the items
  __device__ __forceinline__ void init(int nx, int ny, int x0, int y0) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int q = threadIdx.x + i * WG_THR;
      const int pr = q % 33, h = (q / 33) % HALVES, ly = q / (33 * HALVES);
      const int gy = y0 - 1 + ly, xa = x0 - 1 + 2 * pr;
      const bool row = q < ITEMS && gy >= 0 && gy < ny;
      const uint32_t hb = CIN == 16 ? 16u * h : 0u;
      oa[i] = (row && xa >= 0 && xa < nx ? (uint32_t)(gy * nx + xa) : kFarVox) * VB + hb;
      ob[i] = (row && xa + 1 < nx ? (uint32_t)(gy * nx + xa + 1) : kFarVox) * VB + hb;
      ld[i] = q < ITEMS ? ((ly * CIN + 8 * h) * WG_RX) / 2 + pr : -1;
    }
  }
  __device__ __forceinline__ void fetch(Data &d, const uint16_t *__restrict__ in, int64_t pv,
                                        int nz, int gz) const {
    const Rsrc r = plane_buf(in, pv, CIN, nz, gz);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      if (CIN == 16) {
        d.a[i] = __builtin_amdgcn_raw_buffer_load_b128(r, oa[i], 0, 0);
        d.b[i] = __builtin_amdgcn_raw_buffer_load_b128(r, ob[i], 0, 0);
      } else if (CIN == 2) {  // one dword per voxel
        d.a[i] = u32x4{__builtin_amdgcn_raw_buffer_load_b32(r, oa[i], 0, 0), 0u, 0u, 0u};
        d.b[i] = u32x4{__builtin_amdgcn_raw_buffer_load_b32(r, ob[i], 0, 0), 0u, 0u, 0u};
      } else {  // CIN = 1: one element per voxel
        d.a[i] = u32x4{(uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, oa[i], 0, 0), 0u, 0u, 0u};
        d.b[i] = u32x4{(uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, ob[i], 0, 0), 0u, 0u, 0u};
      }
    }
  }
  __device__ __forceinline__ void store(uint32_t *lds, int slot, const Data &dd) const {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      if (i + 1 == PER && ld[i] < 0) continue;
      uint32_t *d = lds + slot * (SLOT / 2) + ld[i];
      if (CIN == 16) {
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          d[(2 * w) * (WG_RX / 2)] = wg_lo(dd.a[i][w], dd.b[i][w]);
          d[(2 * w + 1) * (WG_RX / 2)] = wg_hi(dd.a[i][w], dd.b[i][w]);
        }
      } else {
        d[0] = wg_lo(dd.a[i][0], dd.b[i][0]);
        if (CIN == 2) d[WG_RX / 2] = wg_hi(dd.a[i][0], dd.b[i][0]);
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
  static constexpr uint32_t VB = COUT * 2;
  struct Data {
    u32x4 a[PER], b[PER];
  };
  uint32_t oa[PER], ob[PER];
  int ld[PER];
  __device__ __forceinline__ void init(int nx, int ny, int x0, int y0) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int q = threadIdx.x + i * WG_THR;
      const int pr = q % 32, h = (q / 32) % HALVES, r = q / (32 * HALVES);
      const int gy = y0 + r, xa = x0 + 2 * pr;
      const bool row = q < ITEMS && gy < ny;
      const uint32_t hb = COUT == 16 ? 16u * h : 0u;
      oa[i] = (row && xa < nx ? (uint32_t)(gy * nx + xa) : kFarVox) * VB + hb;
      ob[i] = (row && xa + 1 < nx ? (uint32_t)(gy * nx + xa + 1) : kFarVox) * VB + hb;
      ld[i] = q < ITEMS ? ((r * COUT + 8 * h) * WG_RX) / 2 + pr : -1;
    }
  }
  __device__ __forceinline__ void fetch(Data &d, const uint16_t *__restrict__ dz, int64_t pv,
                                        int nz, int gz) const {
    const Rsrc r = plane_buf(dz, pv, COUT, nz, gz);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      if (COUT == 16) {
        d.a[i] = __builtin_amdgcn_raw_buffer_load_b128(r, oa[i], 0, 0);
        d.b[i] = __builtin_amdgcn_raw_buffer_load_b128(r, ob[i], 0, 0);
      } else {  // COUT = 1: one element per voxel
        d.a[i] = u32x4{(uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, oa[i], 0, 0), 0u, 0u, 0u};
        d.b[i] = u32x4{(uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, ob[i], 0, 0), 0u, 0u, 0u};
      }
    }
  }
  __device__ __forceinline__ void store(uint32_t *lds, int slot, const Data &dd) const {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      if (i + 1 == PER && ld[i] < 0) continue;
      uint32_t *d = lds + slot * (SLOT / 2) + ld[i];
      if (COUT == 16) {
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          d[(2 * w) * (WG_RX / 2)] = wg_lo(dd.a[i][w], dd.b[i][w]);
          d[(2 * w + 1) * (WG_RX / 2)] = wg_hi(dd.a[i][w], dd.b[i][w]);
        }
      } else {
        d[0] = wg_lo(dd.a[i][0], dd.b[i][0]);
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
  const int64_t pv = (int64_t)nx * ny;
  f32x4 acc[27];
#pragma unroll
  for (int t = 0; t < 27; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  f32x4 accb = {0.f, 0.f, 0.f, 0.f};
  const uint32_t one2 = 0x3F803F80u;  // two BF16 ones
  const bf16x8 ones = __builtin_bit_cast(bf16x8, u32x4{one2, one2, one2, one2});
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int x0 = (tile % tx) * 64, y0 = ((tile / tx) % ty) * WG_TY;
    const int zs = (tile / (tx * ty)) * WG_ZC, ze = min(zs + WG_ZC, nz);
    In fin;
    Dz fdz;
    fin.init(nx, ny, x0, y0);
    fdz.init(nx, ny, x0, y0);
    {  // prologue: input planes zs - 1 .. zs + 1 and dz plane zs
      typename In::Data d;
      for (int p = zs - 1; p <= zs + 1; ++p) {
        fin.fetch(d, in, pv, nz, p);
        fin.store(lin, p & 3, d);
      }
      typename Dz::Data e;
      fdz.fetch(e, dz, pv, nz, zs);
      fdz.store(ldz, zs & 1, e);
    }
    __syncthreads();
    const bool row_live = y0 + wave < ny;
#pragma unroll 1
    for (int z = zs; z < ze; ++z) {
      const bool more = z + 1 < ze;
      typename In::Data nin;
      typename Dz::Data ndz;
      if (more) {
        fin.fetch(nin, in, pv, nz, z + 2);
        fdz.fetch(ndz, dz, pv, nz, z + 1);
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
        fin.store(lin, (z + 2) & 3, nin);
        fdz.store(ldz, (z + 1) & 1, ndz);
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
  const int64_t pv = (int64_t)nx * ny;
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
    Ring fr;
    Flat ff;
    fr.init(nx, ny, x0, y0);
    ff.init(nx, ny, x0, y0);
    {  // prologue: ring planes zs - 1 .. zs + 1 and flat plane zs
      typename Ring::Data d;
      for (int p = zs - 1; p <= zs + 1; ++p) {
        fr.fetch(d, ring_src, pv, nz, p);
        fr.store(lring, p & 3, d);
      }
      typename Flat::Data e;
      ff.fetch(e, flat_src, pv, nz, zs);
      ff.store(lflat, zs & 1, e);
    }
    __syncthreads();
    const bool row_live = y0 + wave < ny;
#pragma unroll 1
    for (int z = zs; z < ze; ++z) {
      const bool more = z + 1 < ze;
      typename Ring::Data nr;
      typename Flat::Data nf;
      if (more) {
        fr.fetch(nr, ring_src, pv, nz, z + 2);
        ff.fetch(nf, flat_src, pv, nz, z + 1);
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
        fr.store(lring, (z + 2) & 3, nr);
        ff.store(lflat, (z + 1) & 1, nf);
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
  const dim3 grid(cm_tiles(nx, ny, nz)), grid_kc(kc_tiles(nx, ny, nz)), block(CM_THR);
#define WFD_CONV(CI, CO)                                                                      \
  hipLaunchKernelGGL((k_conv<CI, CO>), grid_kc, block, 0, stream, in, nx, ny, nz, apk, bias,   \
                     relu, mask, res, res_c, out_bf, out_f)
#define WFD_CONV16(CO)                                                                         \
  hipLaunchKernelGGL((k_conv16<CO>), dim3(c16_tiles(c16_rw<CO>(), nx, ny, nz)), block, 0,      \
                     stream, in, nx, ny, nz, apk, bias, relu, mask, res, res_c, out_bf, out_f)
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
