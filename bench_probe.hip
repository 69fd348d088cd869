// Streaming probes for bench.py (measurement only; not part of the library):
// plain kernels that read R arrays and write W arrays of float4 with a
// grid-stride loop and no reuse, giving the achievable-bandwidth reference
// beside the step kernels' rooflines.  (R, W) = (1, 1), (3, 1), (4, 1) and
// (6, 2) match a copy, the forward step's streams without the stencil reuse,
// and the adjoint's.  Built by __graft_entry__.build() into bench_probe.so.
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

}  // namespace

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
