// Streaming probes for bench.py (measurement only; not part of the library):
// plain kernels that read R arrays and write W arrays of float4 with a
// grid-stride loop and no reuse, giving the achievable-bandwidth reference
// beside the step kernels' rooflines.  (R, W) = (1, 1), (3, 1), (4, 1) and
// (6, 2) match a copy, the forward step's streams without the stencil reuse,
// and the adjoint's.  The tile-march probes walk the step kernels' tiles and
// z chunks instead.  Built by __graft_entry__.build() into bench_probe.so.
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

template <int R, int W, bool NT>
__global__ void __launch_bounds__(256)
    k_stream(const v4f *__restrict__ in, v4f *__restrict__ out, int64_t n4) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
       i += (int64_t)gridDim.x * blockDim.x) {
    v4f s = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const v4f *p = in + (int64_t)r * n4 + i;
      s += NT ? __builtin_nontemporal_load(p) : *p;
    }
#pragma unroll
    for (int w = 0; w < W; ++w) {
      v4f *p = out + (int64_t)w * n4 + i;
      if (NT)
        __builtin_nontemporal_store(s, p);
      else
        *p = s;
    }
  }
}

template <int R, int W>
hipError_t stream_launch(bool nt, float *buf, int64_t n, int blocks, hipStream_t stream) {
  const int64_t n4 = n / 4;
  const v4f *in = reinterpret_cast<const v4f *>(buf);
  v4f *out = reinterpret_cast<v4f *>(buf) + (int64_t)R * n4;
  if (nt)
    hipLaunchKernelGGL((k_stream<R, W, true>), dim3(blocks), dim3(256), 0, stream, in, out, n4);
  else
    hipLaunchKernelGGL((k_stream<R, W, false>), dim3(blocks), dim3(256), 0, stream, in, out, n4);
  return hipGetLastError();
}

// Tile-march probes: the step kernels' access pattern without the stencil.
// A block of NW wavefronts owns a 64 x 2 NW column tile of an nx x ny plane
// (one lane per column, two rows per wavefront) and marches zc planes of it,
// reading R arrays and writing W arrays at each point as one 256-byte row
// segment per wavefront and array.  The first array is read through the
// cache (the stenciled field), the others and the stores are nontemporal, as
// in the step kernels.  Blocks are numbered x fastest, then y, then z chunk.
template <int R, int W, int NW>
__global__ void __launch_bounds__(64 * NW)
    k_march(const float *__restrict__ in, float *__restrict__ out, int nx, int ny, int nz,
            int zc, int64_t n) {
  constexpr int RY = 2, TY = NW * RY;
  const int tx = (nx + 63) / 64, ty = (ny + TY - 1) / TY;
  const int b = blockIdx.x;
  const int x = (b % tx) * 64 + (int)(threadIdx.x % 64);
  const int y0 = ((b / tx) % ty) * TY + (int)(threadIdx.x / 64) * RY;
  const int z0 = (b / (tx * ty)) * zc, z1 = min(z0 + zc, nz);
  if (x >= nx) return;
  for (int z = z0; z < z1; ++z) {
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      if (y0 + j >= ny) continue;
      const int64_t p = ((int64_t)z * ny + y0 + j) * nx + x;
      float s = in[p];
#pragma unroll
      for (int r = 1; r < R; ++r) s += __builtin_nontemporal_load(in + (int64_t)r * n + p);
#pragma unroll
      for (int w = 0; w < W; ++w) __builtin_nontemporal_store(s, out + (int64_t)w * n + p);
    }
  }
}

template <int R, int W, int NW>
hipError_t march_launch(float *buf, int nx, int ny, int nz, int zc, hipStream_t stream) {
  const int64_t n = (int64_t)nx * ny * nz;
  const int64_t blocks = (int64_t)((nx + 63) / 64) * ((ny + 2 * NW - 1) / (2 * NW)) *
                         ((nz + zc - 1) / zc);
  hipLaunchKernelGGL((k_march<R, W, NW>), dim3((unsigned)blocks), dim3(64 * NW), 0, stream, buf,
                     buf + (int64_t)R * n, nx, ny, nz, zc, n);
  return hipGetLastError();
}

}  // namespace

// One tile-march launch over buf = reads + writes arrays of nx * ny * nz
// floats: (reads, writes) = (4, 1) on 64 x 16 tiles (the variable-density
// forward step's streams and tile) or (6, 2) on 64 x 32 tiles (the adjoint's);
// zc planes per z chunk.  Returns 0 or a hipError_t code (hipErrorInvalidValue
// for another pair or a bad size).
extern "C" int bench_march_probe(int reads, int writes, float *buf, int nx, int ny, int nz,
                                 int zc, void *stream) {
  if (!buf || nx <= 0 || ny <= 0 || nz <= 0 || zc <= 0 || (uintptr_t)buf % 16 != 0 ||
      (int64_t)nx * ny * nz > ((int64_t)1 << 31))
    return (int)hipErrorInvalidValue;
  hipStream_t s = (hipStream_t)stream;
  if (reads == 4 && writes == 1) return (int)march_launch<4, 1, 8>(buf, nx, ny, nz, zc, s);
  if (reads == 6 && writes == 2) return (int)march_launch<6, 2, 16>(buf, nx, ny, nz, zc, s);
  return (int)hipErrorInvalidValue;
}

// One launch over buf = reads + writes arrays of n floats (inputs first, then
// outputs); n a positive multiple of 4, buf 16-byte aligned.  Returns 0 or a
// hipError_t code (hipErrorInvalidValue for another (reads, writes) pair or a
// bad size).
extern "C" int bench_stream_probe(int reads, int writes, int nontemporal, float *buf, int64_t n,
                                  int blocks, void *stream) {
  if (!buf || n <= 0 || n % 4 != 0 || blocks <= 0 || (uintptr_t)buf % 16 != 0)
    return (int)hipErrorInvalidValue;
  hipStream_t s = (hipStream_t)stream;
  const bool nt = nontemporal != 0;
  if (reads == 1 && writes == 1) return (int)stream_launch<1, 1>(nt, buf, n, blocks, s);
  if (reads == 3 && writes == 1) return (int)stream_launch<3, 1>(nt, buf, n, blocks, s);
  if (reads == 4 && writes == 1) return (int)stream_launch<4, 1>(nt, buf, n, blocks, s);
  if (reads == 6 && writes == 2) return (int)stream_launch<6, 2>(nt, buf, n, blocks, s);
  return (int)hipErrorInvalidValue;
}
