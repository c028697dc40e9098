// Memory ceilings of the GPU, for the measurement of the propagation passes against what HBM
// delivers in practice (not part of the method). Three streaming kernels over one buffer:
//   mode 0: in place, read and write every byte (x <- s x, s = 1 at run time): the access pattern of
//           an in-place pass (16 B per complex64 element per sweep);
//   mode 1: write only (the source builder's pattern);
//   mode 2: read only (the pattern of the observables-only passes);
//   modes 3, 4, 5: the same with the nontemporal hint on every load and store.
// A workgroup moves 16 KB: each of its four 16-byte vector loads (or stores) per thread covers 4 KB
// of contiguous memory across the 256 threads, all loads issued before the first store.
#include "wolf_internal.hpp"

namespace wolf {

constexpr int kCeilVec = 4;  // 16-byte vectors per thread
typedef float ceil_v4f __attribute__((ext_vector_type(4)));

// NT: the loads and stores carry the nontemporal hint (the data is touched once).
template <bool NT> __device__ __forceinline__ ceil_v4f ld(const ceil_v4f* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT> __device__ __forceinline__ void st(ceil_v4f* p, ceil_v4f v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

template <bool NT>
__global__ __launch_bounds__(256) void k_ceiling_rmw(ceil_v4f* __restrict__ p, float s) {
  ceil_v4f* q = p + (long long)blockIdx.x * (256 * kCeilVec) + threadIdx.x;
  ceil_v4f v[kCeilVec];
#pragma unroll
  for (int k = 0; k < kCeilVec; ++k) v[k] = ld<NT>(&q[k * 256]);
#pragma unroll
  for (int k = 0; k < kCeilVec; ++k) st<NT>(&q[k * 256], v[k] * s);
}

template <bool NT>
__global__ __launch_bounds__(256) void k_ceiling_fill(ceil_v4f* __restrict__ p, float s) {
  ceil_v4f* q = p + (long long)blockIdx.x * (256 * kCeilVec) + threadIdx.x;
  const ceil_v4f v = {s, s, s, s};
#pragma unroll
  for (int k = 0; k < kCeilVec; ++k) st<NT>(&q[k * 256], v);
}

// `never` is a value the data cannot sum to (the caller passes -1e38): the store keeps the loads.
template <bool NT>
__global__ __launch_bounds__(256) void k_ceiling_read(ceil_v4f* __restrict__ p, float never) {
  ceil_v4f* q = p + (long long)blockIdx.x * (256 * kCeilVec) + threadIdx.x;
  ceil_v4f v[kCeilVec];
#pragma unroll
  for (int k = 0; k < kCeilVec; ++k) v[k] = ld<NT>(&q[k * 256]);
  float acc = 0.f;
#pragma unroll
  for (int k = 0; k < kCeilVec; ++k) acc += (v[k].x + v[k].y) + (v[k].z + v[k].w);
  if (acc == never) q[0] = ceil_v4f{acc, acc, acc, acc};
}

hipError_t launch_ceiling(void* buf, long long bytes, int mode, hipStream_t st) {
  const long long per_block = 256ll * kCeilVec * 16;  // 16 KB
  const long long blocks = bytes / per_block;
  if (blocks <= 0 || blocks > 0x7fffffffll || bytes % per_block != 0) return hipErrorInvalidValue;
  ceil_v4f* p = static_cast<ceil_v4f*>(buf);
  const dim3 g((unsigned)blocks), b(256);
  switch (mode) {
    case 0: hipLaunchKernelGGL(k_ceiling_rmw<false>, g, b, 0, st, p, 1.0f); break;
    case 1: hipLaunchKernelGGL(k_ceiling_fill<false>, g, b, 0, st, p, 0.0f); break;
    case 2: hipLaunchKernelGGL(k_ceiling_read<false>, g, b, 0, st, p, -1e38f); break;
    case 3: hipLaunchKernelGGL(k_ceiling_rmw<true>, g, b, 0, st, p, 1.0f); break;
    case 4: hipLaunchKernelGGL(k_ceiling_fill<true>, g, b, 0, st, p, 0.0f); break;
    case 5: hipLaunchKernelGGL(k_ceiling_read<true>, g, b, 0, st, p, -1e38f); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace wolf
