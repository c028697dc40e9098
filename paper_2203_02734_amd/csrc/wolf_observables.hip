// Observables of a CSD array (Sec. 3.5): the spectral density (Algorithm 4, eq. defS) and the
// spectral degree of coherence (Algorithm 5, eq. defMu). Also the chirp-table export.
//
// S[m] = Re W[m; m] is a gather at stride N^2 + 1 (N^2 values). mu reads one contiguous slab W[P1; .]
// (slice) or the whole array (full mu), and S.
// The floor tau = floor_rel * max S masks points with no light (mu = 0 there). max S is an
// order-independent reduction, done with an atomic max on order-preserving integer keys.
#include <map>
#include <mutex>

#include "wolf_internal.hpp"

namespace wolf {

// Scratch of the allocation-free degree-of-coherence entry point: the order key of max S (at
// offset 0) and the N^2 values of S (at offset 256), up to N = 256 in FP64. One copy per GPU, held
// until the process ends, shared by every call on that GPU.
constexpr size_t kMuStaticBytes = 256 + (size_t)256 * 256 * 8;
static __device__ __align__(256) unsigned char scratch[kMuStaticBytes];

hipError_t mu_static_scratch(void** out, size_t* bytes) {
  static std::mutex mu;
  static std::map<int, void*> ptrs;  // device -> address of that device's copy of `scratch`
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  auto it = ptrs.find(dev);
  if (it == ptrs.end()) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));  // the device address; `scratch` itself is a host stand-in
    if (e != hipSuccess) return e;
    it = ptrs.emplace(dev, p).first;
  }
  *out = it->second;
  *bytes = kMuStaticBytes;
  return hipSuccess;
}

template <class T>
__global__ __launch_bounds__(256) void k_sdiag(const T* __restrict__ w, int n, typename real_of<T>::type* __restrict__ s) {
  const long long nn = (long long)n * n;
  const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m < nn) s[m] = w[m * (nn + 1)].x;
}

__global__ void k_clear_key(unsigned long long* key) { *key = 0ull; }

template <class T>
__global__ __launch_bounds__(256) void k_sdiag_max(const T* __restrict__ w, int n, typename real_of<T>::type* __restrict__ s,
                                                   unsigned long long* key) {
  __shared__ unsigned long long red[256];
  const long long nn = (long long)n * n;
  const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long k = 0ull;
  if (m < nn) {
    const auto v = w[m * (nn + 1)].x;
    s[m] = v;
    k = order_key((double)v);
  }
  red[threadIdx.x] = k;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h && red[threadIdx.x + h] > red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(key, red[0]);
}

template <class T>
__global__ __launch_bounds__(256) void k_mu_slice(const T* __restrict__ w, int n, int p1, double floor_rel,
                                                  const typename real_of<T>::type* __restrict__ s,
                                                  const unsigned long long* __restrict__ key, T* __restrict__ mu) {
  using R = typename real_of<T>::type;
  const long long nn = (long long)n * n;
  const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nn) return;
  const R tau = (R)(floor_rel * key_value(*key));
  const R s1 = s[p1], s2 = s[m];
  T out{(R)0, (R)0};
  if (s1 > tau && s2 > tau) {
    const R d = sqrt(s1) * sqrt(s2);
    const T v = w[(long long)p1 * nn + m];
    out = T{v.x / d, v.y / d};
  }
  mu[m] = out;
}

template <class T>
__global__ __launch_bounds__(256) void k_mu_full(const T* __restrict__ w, int n, double floor_rel,
                                                 const typename real_of<T>::type* __restrict__ s,
                                                 const unsigned long long* __restrict__ key, T* __restrict__ mu) {
  using R = typename real_of<T>::type;
  const long long nn = (long long)n * n;
  const long long p1 = blockIdx.x;
  const R tau = (R)(floor_rel * key_value(*key));
  const R s1 = s[p1];
  const bool ok1 = s1 > tau;
  const R r1 = ok1 ? sqrt(s1) : (R)1;
  const T* row = w + p1 * nn;
  T* out = mu + p1 * nn;
  for (long long e = threadIdx.x; e < nn; e += blockDim.x) {
    const R s2 = s[e];
    T o{(R)0, (R)0};
    if (ok1 && s2 > tau) {
      const R d = r1 * sqrt(s2);
      const T v = row[e];
      o = T{v.x / d, v.y / d};
    }
    out[e] = o;
  }
}

template <class T>
hipError_t launch_spectral_density(int n, const T* w, typename real_of<T>::type* s, hipStream_t st) {
  const long long nn = (long long)n * n;
  hipLaunchKernelGGL(k_sdiag<T>, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, w, n, s);
  return hipGetLastError();
}

template <class T>
hipError_t launch_coherence(int n, const T* w, int ip, int jp, double floor_rel, T* mu, void* scratch,
                            hipStream_t st) {
  using R = typename real_of<T>::type;
  const long long nn = (long long)n * n;
  auto* key = reinterpret_cast<unsigned long long*>(scratch);
  auto* s = reinterpret_cast<R*>(reinterpret_cast<char*>(scratch) + 256);
  hipLaunchKernelGGL(k_clear_key, dim3(1), dim3(1), 0, st, key);
  hipLaunchKernelGGL(k_sdiag_max<T>, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, w, n, s, key);
  if (ip >= 0) {
    hipLaunchKernelGGL(k_mu_slice<T>, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, w, n, ip * n + jp,
                       floor_rel, (const R*)s, (const unsigned long long*)key, mu);
  } else {
    hipLaunchKernelGGL(k_mu_full<T>, dim3((unsigned)nn), dim3(256), 0, st, w, n, floor_rel, (const R*)s,
                       (const unsigned long long*)key, mu);
  }
  return hipGetLastError();
}

template <class T>
__global__ void k_chirp_table(int n, Chirp ch, T* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = chirp_entry<T>(ch, i, n);
}

template <class T>
hipError_t launch_chirp_table(int n, const Chirp& ch, T* out, hipStream_t st) {
  hipLaunchKernelGGL(k_chirp_table<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, ch, out);
  return hipGetLastError();
}

template hipError_t launch_spectral_density<float2>(int, const float2*, float*, hipStream_t);
template hipError_t launch_spectral_density<double2>(int, const double2*, double*, hipStream_t);
template hipError_t launch_coherence<float2>(int, const float2*, int, int, double, float2*, void*, hipStream_t);
template hipError_t launch_coherence<double2>(int, const double2*, int, int, double, double2*, void*, hipStream_t);
template hipError_t launch_chirp_table<float2>(int, const Chirp&, float2*, hipStream_t);
template hipError_t launch_chirp_table<double2>(int, const Chirp&, double2*, hipStream_t);

}  // namespace wolf
