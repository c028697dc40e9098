// Memory ceilings of the GPU, for the measurement of the propagation passes against what HBM
// delivers in practice (not part of the method). Three streaming kernels over one buffer:
//   mode 0: in place, read and write every byte (x <- s x, s = 1 at run time): the access pattern of
//           an in-place pass (16 B per complex64 element per sweep);
//   mode 1: write only (the source builder's pattern);
//   mode 2: read only (the pattern of the observables-only passes).
// Each thread moves 64 contiguous bytes as four 16-byte vectors, all loads issued before the first
// store, and consecutive threads take consecutive 64-byte blocks, so that every wavefront covers
// 4 KB of contiguous memory.
#include "wolf_internal.hpp"

namespace wolf {

__global__ __launch_bounds__(256) void k_ceiling_rmw(float4* __restrict__ p, long long nvec, float s) {
  const long long base = ((long long)blockIdx.x * 256 + threadIdx.x) * 4;
  if (base + 4 > nvec) return;
  float4 v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = p[base + k];
#pragma unroll
  for (int k = 0; k < 4; ++k) p[base + k] = make_float4(v[k].x * s, v[k].y * s, v[k].z * s, v[k].w * s);
}

__global__ __launch_bounds__(256) void k_ceiling_fill(float4* __restrict__ p, long long nvec, float s) {
  const long long base = ((long long)blockIdx.x * 256 + threadIdx.x) * 4;
  if (base + 4 > nvec) return;
#pragma unroll
  for (int k = 0; k < 4; ++k) p[base + k] = make_float4(s, s, s, s);
}

__global__ __launch_bounds__(256) void k_ceiling_read(float4* __restrict__ p, long long nvec, float s) {
  const long long base = ((long long)blockIdx.x * 256 + threadIdx.x) * 4;
  if (base + 4 > nvec) return;
  float4 v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = p[base + k];
  float acc = 0.f;
#pragma unroll
  for (int k = 0; k < 4; ++k) acc += v[k].x + v[k].y + v[k].z + v[k].w;
  // s is never NaN, so this store never happens; it keeps the loads.
  if (acc == s && s != s) p[base] = make_float4(acc, acc, acc, acc);
}

hipError_t launch_ceiling(void* buf, long long bytes, int mode, hipStream_t st) {
  const long long nvec = bytes / 16;
  const long long blocks = nvec / (256 * 4);
  if (blocks <= 0 || blocks > 0x7fffffffll || bytes % (256 * 64) != 0) return hipErrorInvalidValue;
  float4* p = static_cast<float4*>(buf);
  switch (mode) {
    case 0: hipLaunchKernelGGL(k_ceiling_rmw, dim3((unsigned)blocks), dim3(256), 0, st, p, nvec, 1.0f); break;
    case 1: hipLaunchKernelGGL(k_ceiling_fill, dim3((unsigned)blocks), dim3(256), 0, st, p, nvec, 0.0f); break;
    case 2: hipLaunchKernelGGL(k_ceiling_read, dim3((unsigned)blocks), dim3(256), 0, st, p, nvec, 1.0f); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace wolf
