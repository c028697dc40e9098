// Source CSD builder (Sec. 3.2, eq. GSM_source; Algorithms 6-7; eq. W_def; Sec. 2.2 thin lens).
//
// One workgroup writes one contiguous slab p1 = (i1, j1) of W0[i1][j1][i2][j2]. The array is
// write-only, so the kernel is bound by HBM writes (8 B/element in complex64). The models and
// their factorisation are in wolf_source.hpp: the workgroup builds its two axis rows in FP64,
// rounds them once, then forms each element with one complex multiply.
#include "wolf_source.hpp"

namespace wolf {

template <class T>
__global__ __launch_bounds__(256) void k_build_source(T* __restrict__ w, int n, SourceParams sp) {
  using R = typename real_of<T>::type;
  __shared__ T fx[256], fy[256];
  __shared__ R m2[1];
  const int p1 = blockIdx.x;
  const int i1 = p1 / n, j1 = p1 - (p1 / n) * n;
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    fx[t] = axis_factor<T>(sp, i1, t, n);
    fy[t] = axis_factor<T>(sp, j1, t, n);
  }
  if (threadIdx.x == 0) m2[0] = slab_scale<R>(sp, i1, j1, n);
  __syncthreads();
  const R am1 = m2[0];
  const long long nn = (long long)n * n;
  T* slab = w + (long long)p1 * nn;
  if (sp.model == 3) {  // incoherent: Kronecker delta in (p1, p2)
    for (long long e = threadIdx.x; e < nn; e += blockDim.x) slab[e] = T{(R)0, (R)0};
    __syncthreads();  // every zero of this slab is written before the diagonal entry
    if (threadIdx.x == 0) {
      __threadfence_block();
      slab[p1] = T{am1, (R)0};
    }
    return;
  }
  // Element e = i2 N + j2 advances by the block size each step: (i2, j2) advance by (bs / N, bs % N) with
  // a carry, so the loop needs no division.
  const int bs = (int)blockDim.x, di = bs / n, dj = bs - di * n;
  int i2 = (int)threadIdx.x / n, j2 = (int)threadIdx.x - i2 * n;
  for (int e = (int)threadIdx.x; e < (int)nn; e += bs) {
    slab[e] = source_entry<T>(sp, fx, fy, am1, i2, j2, n);
    i2 += di;
    j2 += dj;
    if (j2 >= n) {
      j2 -= n;
      ++i2;
    }
  }
}

template <class T>
hipError_t launch_build_source(int n, const SourceParams& sp, T* w, hipStream_t st) {
  const int threads = n * n < 256 ? n * n : 256;
  hipLaunchKernelGGL(k_build_source<T>, dim3((unsigned)(n * n)), dim3(threads), 0, st, w, n, sp);
  return hipGetLastError();
}

template hipError_t launch_build_source<float2>(int, const SourceParams&, float2*, hipStream_t);
template hipError_t launch_build_source<double2>(int, const SourceParams&, double2*, hipStream_t);

}  // namespace wolf
