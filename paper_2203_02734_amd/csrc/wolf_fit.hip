// Gradient kernels for fitting a source to an observed spectral density.
//
// Model (eq. W_def with a Gaussian degree of coherence): W_A[p1; p2] = a(p1) a(p2) mu_g(p1, p2),
// with a = sqrt(I) and mu_g = exp(-|xi1 - xi2|^2 / (2 sg^2)). The loss depends on S_B = Re diag(W_B)
// (Algorithm 4). With g = dL/dS_B, the gradient with respect to W_B is diag(g)
// (k_diag_embed). The adjoint propagation maps it to G_A (wolf_propagate_adjoint). For each real
// parameter theta, dL/dtheta = sum Re(conj(G_A) dW_A/dtheta):
//   dL/dI(p) = [R(p) + K(p)] / (2 a(p)),  R(p) = sum_q Re(conj(G_A[p; q])) a(q) mu_g(p, q)
//                                          K(p) = sum_q Re(conj(G_A[q; p])) a(q) mu_g(q, p)
//   dL/dsg   = sum_{p, q} Re(conj(G_A[p; q]) W_A[p; q]) |xi_p - xi_q|^2 / sg^3
// The row sums R come from one workgroup per slab. The column sums K are accumulated by workgroups
// that each own a group of slabs, then reduced over the groups.
#include "wolf_internal.hpp"

namespace wolf {

template <class T>
__global__ __launch_bounds__(256) void k_diag_embed(const typename real_of<T>::type* __restrict__ g, int n,
                                                    T* __restrict__ out) {
  using R = typename real_of<T>::type;
  const long long nn = (long long)n * n;
  const long long p1 = blockIdx.x;
  T* slab = out + p1 * nn;
  for (long long e = threadIdx.x; e < nn; e += blockDim.x) slab[e] = T{e == p1 ? g[p1] : (R)0, (R)0};
}

// Per-group partials: rows[p1] (one per slab), colpart[group][q], sgpart[group].
template <class T, int COLS_PER_THREAD>
__global__ __launch_bounds__(256) void k_fit_partials(const T* __restrict__ ga, const float* __restrict__ imap, int n,
                                                      double inv2g2_px, int slabs_per_group,
                                                      typename real_of<T>::type* __restrict__ rows,
                                                      typename real_of<T>::type* __restrict__ colpart,
                                                      double* __restrict__ sgpart) {
  using R = typename real_of<T>::type;
  __shared__ R red[256];
  __shared__ double redd[256];
  __shared__ R gx[256];  // exp(-d^2 pitch^2 / (2 sg^2)) for d = 0..N-1; mu_g = gx[|di|] gx[|dj|]
  const long long nn = (long long)n * n;
  const int tid = threadIdx.x;
  for (int d = tid; d < n; d += blockDim.x) gx[d] = (R)exp(-(double)d * (double)d * inv2g2_px);
  __syncthreads();
  R colacc[COLS_PER_THREAD];
#pragma unroll
  for (int k = 0; k < COLS_PER_THREAD; ++k) colacc[k] = (R)0;
  double sgacc = 0.0;
  const long long group = blockIdx.x;
  for (int s = 0; s < slabs_per_group; ++s) {
    const long long p = group * slabs_per_group + s;
    const int pi = (int)(p / n), pj = (int)(p % n);
    const R ap = sqrt((R)imap[p]);
    const T* row = ga + p * nn;
    R racc = (R)0;
#pragma unroll
    for (int k = 0; k < COLS_PER_THREAD; ++k) {
      const long long q = (long long)k * 256 + tid;
      if (q < nn) {
        const int qi = (int)(q / n), qj = (int)(q % n);
        const int di = pi - qi, dj = pj - qj;
        const double d2 = (double)(di * di + dj * dj);
        const R mu = gx[di < 0 ? -di : di] * gx[dj < 0 ? -dj : dj];
        const R aq = sqrt((R)imap[q]);
        const T gv = row[q];
        const R w = gv.x * aq * mu;                  // Re(conj(G) a(q) mu), a and mu real
        racc += w;
        colacc[k] += gv.x * ap * mu;                 // contribution to K(q)
        sgacc += (double)(w * ap) * d2;              // Re(conj(G) W_A) |d|^2 in pixel units
      }
    }
    red[tid] = racc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (tid < h) red[tid] += red[tid + h];
      __syncthreads();
    }
    if (tid == 0) rows[p] = red[0];
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < COLS_PER_THREAD; ++k) {
    const long long q = (long long)k * 256 + tid;
    if (q < nn) colpart[group * nn + q] = colacc[k];
  }
  redd[tid] = sgacc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) redd[tid] += redd[tid + h];
    __syncthreads();
  }
  if (tid == 0) sgpart[group] = redd[0];
}

template <class T>
__global__ __launch_bounds__(256) void k_fit_finish(const float* __restrict__ imap, int n, int groups,
                                                    const typename real_of<T>::type* __restrict__ rows,
                                                    const typename real_of<T>::type* __restrict__ colpart,
                                                    const double* __restrict__ sgpart, double sg_scale,
                                                    float* __restrict__ d_imap, double* __restrict__ d_sigma) {
  using R = typename real_of<T>::type;
  const long long nn = (long long)n * n;
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nn) {
    R k = (R)0;
    for (int g = 0; g < groups; ++g) k += colpart[(long long)g * nn + q];
    const R a = sqrt((R)imap[q]);
    d_imap[q] = (float)((rows[q] + k) / ((R)2 * a));
  }
  if (q == 0) {
    double t = 0.0;
    for (int g = 0; g < groups; ++g) t += sgpart[g];
    *d_sigma = t * sg_scale;
  }
}

template <class T>
hipError_t launch_diag_embed(int n, const typename real_of<T>::type* g, T* out, hipStream_t st) {
  hipLaunchKernelGGL(k_diag_embed<T>, dim3((unsigned)(n * n)), dim3(256), 0, st, g, n, out);
  return hipGetLastError();
}

template <class T>
hipError_t launch_fit_gradient(int n, const T* ga, const float* imap, double inv2g2_px, double sg_scale, void* work,
                               float* d_imap, double* d_sigma, hipStream_t st) {
  using R = typename real_of<T>::type;
  const long long nn = (long long)n * n;
  const int slabs_per_group = fit_slabs_per_group(n);
  const int groups = (int)(nn / slabs_per_group);
  R* rows = reinterpret_cast<R*>(work);
  R* colpart = rows + nn;
  double* sgpart = reinterpret_cast<double*>(colpart + (long long)groups * nn + 1) ;
  sgpart = reinterpret_cast<double*>((reinterpret_cast<uintptr_t>(sgpart) + 7) & ~(uintptr_t)7);
  switch ((nn + 255) / 256) {
    case 1: hipLaunchKernelGGL((k_fit_partials<T, 1>), dim3(groups), dim3(256), 0, st, ga, imap, n, inv2g2_px, slabs_per_group, rows, colpart, sgpart); break;
    case 4: hipLaunchKernelGGL((k_fit_partials<T, 4>), dim3(groups), dim3(256), 0, st, ga, imap, n, inv2g2_px, slabs_per_group, rows, colpart, sgpart); break;
    case 16: hipLaunchKernelGGL((k_fit_partials<T, 16>), dim3(groups), dim3(256), 0, st, ga, imap, n, inv2g2_px, slabs_per_group, rows, colpart, sgpart); break;
    case 64: hipLaunchKernelGGL((k_fit_partials<T, 64>), dim3(groups), dim3(256), 0, st, ga, imap, n, inv2g2_px, slabs_per_group, rows, colpart, sgpart); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fit_finish<T>, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, imap, n, groups,
                     (const R*)rows, (const R*)colpart, (const double*)sgpart, sg_scale, d_imap, d_sigma);
  return hipGetLastError();
}

int fit_slabs_per_group(int n) {
  const long long nn = (long long)n * n;
  // About 512 groups of slabs: two workgroups per CU, and a partial buffer of 512 x N^2 reals.
  long long s = nn / 512;
  return (int)(s < 1 ? 1 : s);
}

size_t fit_work_bytes(int n, int real_bytes) {
  const long long nn = (long long)n * n;
  const long long groups = nn / fit_slabs_per_group(n);
  return (size_t)(nn + groups * nn + 1) * real_bytes + 8 + (size_t)groups * 8;
}

template hipError_t launch_diag_embed<float2>(int, const float*, float2*, hipStream_t);
template hipError_t launch_diag_embed<double2>(int, const double*, double2*, hipStream_t);
template hipError_t launch_fit_gradient<float2>(int, const float2*, const float*, double, double, void*, float*,
                                                double*, hipStream_t);
template hipError_t launch_fit_gradient<double2>(int, const double2*, const float*, double, double, void*, float*,
                                                 double*, hipStream_t);

}  // namespace wolf
