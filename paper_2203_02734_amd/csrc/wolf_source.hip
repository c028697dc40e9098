// Source CSD builder (Sec. 3.2, eq. GSM_source; Algorithms 6-7; eq. W_def; Sec. 2.2 thin lens).
//
// One workgroup writes one contiguous slab p1 = (i1, j1) of W0[i1][j1][i2][j2]. The array is
// write-only, so the kernel is bound by HBM writes (8 B/element in complex64).
// In pixel units (d = pitch), every model factorises as
//   W0[p1; p2] = A * fx(i1, i2) * fy(j1, j2) * m(p1) * m(p2)
//   f(a, b)    = exp(-(a'^2 + b'^2) pitch^2 / (4 sS^2) - (a - b)^2 pitch^2 / (2 sg^2))
//              * exp(i pi (a'^2 - b'^2) pitch^2 / (lambda f_lens)),   a' = a - N/2, b' = b - N/2
//   m(p)       = Y(p) * sqrt(I(p)) for the MAP model, Y(p) otherwise.
// The y flip of eq. (n12) drops out: only squares and squared differences of the coordinates
// appear. The workgroup builds its two axis rows fx(i1, .) and fy(j1, .) in FP64, rounds them
// once, then forms each element with one complex multiply.
#include "wolf_internal.hpp"

namespace wolf {

__device__ __forceinline__ bool inside(const SourceParams& sp, int di, int dj, int n, int i, int j) {
  const long long a = (long long)di * di, b = (long long)dj * dj;
  switch (sp.geometry) {
    case 1: return a + b <= sp.t0;
    case 2: return a <= sp.t0 && b <= sp.t0;
    case 3: return a + b <= sp.t0 && a + b > sp.t1;
    case 4: return sp.mask[(long long)i * n + j] != 0;
    default: return true;
  }
}

template <class T>
__device__ __forceinline__ T axis_factor(const SourceParams& sp, int a, int b, int n) {
  using R = typename real_of<T>::type;
  const long long da = a - n / 2, db = b - n / 2;
  const double e = -(double)(da * da + db * db) * sp.inv4s2_px - (double)((da - db) * (da - db)) * sp.inv2g2_px;
  const double mag = exp(e);
  if (sp.lens_alpha == 0.0) return T{(R)mag, (R)0};
  const double ph = reduce_mod2((double)(da * da - db * db) * sp.lens_alpha);
  double s, c;
  sincospi(ph, &s, &c);
  return T{(R)(mag * c), (R)(mag * s)};
}

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
  if (threadIdx.x == 0) {
    R m1 = inside(sp, i1 - n / 2, j1 - n / 2, n, i1, j1) ? (R)1 : (R)0;
    if (sp.model == 1) m1 *= sqrt((R)sp.imap[(long long)i1 * n + j1]);
    m2[0] = m1 * (R)sp.amplitude;
  }
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
    R m = inside(sp, i2 - n / 2, j2 - n / 2, n, i2, j2) ? am1 : (R)0;
    if (sp.model == 1) m *= sqrt((R)sp.imap[e]);
    slab[e] = cscale(cmul(fx[i2], fy[j2]), m);
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
