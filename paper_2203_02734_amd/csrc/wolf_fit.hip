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
// Workgroups own a group of slabs and a part of the N^2 columns (at most 4096 of them: one part below
// N = 128, four at N = 128). Each gives a partial row sum R per slab and part, a partial column sum K
// per column and group, and a partial of dL/dsg; the finishing kernel adds the parts in a fixed order.
#include "wolf_device.hpp"
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

// Partials of one (group of slabs, part of the columns): rows[part][p] (a slab's row sum over the
// part's columns), colpart[group][q] (q in the part), sgpart[group][part]. A thread owns the columns
// q = part * COLS_PER_THREAD * 256 + k 256 + tid, k < COLS_PER_THREAD (at most 16, so that the column
// sums stay in registers), issues their loads before it uses any, and computes a(q) of its columns once.
// N divides 256 (both powers of two, N <= 128 here), so q has the fixed second index qj = tid mod N.
// The row sum of a slab is reduced by a butterfly within each wavefront and then over the four
// wavefronts in order.
template <class T, int COLS_PER_THREAD>
__global__ __launch_bounds__(256) void k_fit_partials(const T* __restrict__ ga, const float* __restrict__ imap, int n,
                                                      double inv2g2_px, int slabs_per_group, int parts,
                                                      typename real_of<T>::type* __restrict__ rows,
                                                      typename real_of<T>::type* __restrict__ colpart,
                                                      double* __restrict__ sgpart) {
  using R = typename real_of<T>::type;
  constexpr int CPT = COLS_PER_THREAD;
  __shared__ R red[2][4];  // wavefront sums of the row, double-buffered by slab parity
  __shared__ double redd[256];
  __shared__ R gx[256];  // exp(-d^2 pitch^2 / (2 sg^2)) for d = 0..N-1; mu_g = gx[|di|] gx[|dj|]
  const int nn = n * n;
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  for (int d = tid; d < n; d += 256) gx[d] = (R)exp(-(double)d * (double)d * inv2g2_px);
  const long long group = blockIdx.x / parts;
  const int part = (int)(blockIdx.x - group * parts);
  const int q0 = part * CPT * 256;
  const int qj = tid % n, qi0 = (q0 + tid) / n, qstep = 256 / n;
  R aqs[CPT];  // a(q) = sqrt(I(q)) of this thread's columns, the same for every slab
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int q = q0 + k * 256 + tid;
    aqs[k] = q < nn ? sqrt((R)imap[q]) : (R)0;
  }
  __syncthreads();
  R colacc[CPT];
#pragma unroll
  for (int k = 0; k < CPT; ++k) colacc[k] = (R)0;
  double sgacc = 0.0;
  for (int s = 0; s < slabs_per_group; ++s) {
    const long long p = group * slabs_per_group + s;
    const int pi = (int)(p / n), pj = (int)(p % n);
    const R ap = sqrt((R)imap[p]);
    const T* row = ga + p * nn + q0;
    const int dj = pj - qj;
    const R muj = gx[dj < 0 ? -dj : dj];
    T gv[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) gv[k] = load_or_first(row, q0 + k * 256 + tid < nn, k * 256 + tid);
    R racc = (R)0;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const bool ok = q0 + k * 256 + tid < nn;
      const int di = pi - (qi0 + k * qstep);
      const int ai = di < 0 ? -di : di;
      const double d2 = (double)(di * di + dj * dj);
      const R mu = gx[ok ? ai : 0] * muj;
      const R gre = ok ? gv[k].x : (R)0;
      const R w = gre * aqs[k] * mu;               // Re(conj(G) a(q) mu), a and mu real
      racc += w;
      colacc[k] += gre * ap * mu;                  // contribution to K(q)
      sgacc += (double)(w * ap) * d2;              // Re(conj(G) W_A) |d|^2 in pixel units
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) racc += __shfl_xor(racc, off);
    if (lane == 0) red[s & 1][wave] = racc;
    __syncthreads();
    if (tid == 0) rows[(long long)part * nn + p] = ((red[s & 1][0] + red[s & 1][1]) + red[s & 1][2]) + red[s & 1][3];
  }
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int q = q0 + k * 256 + tid;
    if (q < nn) colpart[group * nn + q] = colacc[k];
  }
  redd[tid] = sgacc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) redd[tid] += redd[tid + h];
    __syncthreads();
  }
  if (tid == 0) sgpart[blockIdx.x] = redd[0];
}

// dL/dI from the row sums (added over the column parts) and the column partials, and dL/dsg from the
// group partials. A workgroup
// owns 32 columns; its eight slices of 32 threads each add every eighth group in order, and the slices
// are combined in order. Workgroup 0 also adds the sg partials: 256 strided sums, then a fixed tree.
template <class T>
__global__ __launch_bounds__(256) void k_fit_finish(const float* __restrict__ imap, int n, int groups, int parts,
                                                    const typename real_of<T>::type* __restrict__ rows,
                                                    const typename real_of<T>::type* __restrict__ colpart,
                                                    const double* __restrict__ sgpart, double sg_scale,
                                                    float* __restrict__ d_imap, double* __restrict__ d_sigma) {
  using R = typename real_of<T>::type;
  __shared__ R part[8][32];
  __shared__ double sred[256];
  const long long nn = (long long)n * n;
  const int cx = threadIdx.x % 32, sl = threadIdx.x / 32;
  const long long q = (long long)blockIdx.x * 32 + cx;
  R k = (R)0;
  if (q < nn) {
#pragma unroll 8
    for (int g = sl; g < groups; g += 8) k += colpart[(long long)g * nn + q];  // loads in flight, sums in order
  }
  part[sl][cx] = k;
  if (blockIdx.x == 0) {
    double t = 0.0;
    for (int g = threadIdx.x; g < groups * parts; g += 256) t += sgpart[g];
    sred[threadIdx.x] = t;
  }
  __syncthreads();
  if (sl == 0 && q < nn) {
    R kk = part[0][cx];
#pragma unroll
    for (int j = 1; j < 8; ++j) kk += part[j][cx];
    R rsum = rows[q];
    for (int j = 1; j < parts; ++j) rsum += rows[(long long)j * nn + q];
    const R a = sqrt((R)imap[q]);
    d_imap[q] = (float)((rsum + kk) / ((R)2 * a));
  }
  if (blockIdx.x == 0) {
    for (int h = 128; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) sred[threadIdx.x] += sred[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) *d_sigma = sred[0] * sg_scale;
  }
}

template <class T>
hipError_t launch_diag_embed(int n, const typename real_of<T>::type* g, T* out, hipStream_t st) {
  hipLaunchKernelGGL(k_diag_embed<T>, dim3((unsigned)(n * n)), dim3(256), 0, st, g, n, out);
  return hipGetLastError();
}

// Columns per part: 256 threads x at most 16 columns each.
static int fit_parts(int n) {
  const long long nn = (long long)n * n;
  return nn > 4096 ? (int)(nn / 4096) : 1;
}

template <class T>
hipError_t launch_fit_gradient(int n, const T* ga, const float* imap, double inv2g2_px, double sg_scale, void* work,
                               float* d_imap, double* d_sigma, hipStream_t st) {
  using R = typename real_of<T>::type;
  const long long nn = (long long)n * n;
  const int slabs_per_group = fit_slabs_per_group(n);
  const int groups = (int)(nn / slabs_per_group);
  const int parts = fit_parts(n);
  R* rows = reinterpret_cast<R*>(work);
  R* colpart = rows + parts * nn;
  double* sgpart = reinterpret_cast<double*>(colpart + (long long)groups * nn + 1);
  sgpart = reinterpret_cast<double*>((reinterpret_cast<uintptr_t>(sgpart) + 7) & ~(uintptr_t)7);
  const dim3 grid((unsigned)(groups * parts));
  switch (nn / parts > 256 ? (nn / parts + 255) / 256 : 1) {
    case 1: hipLaunchKernelGGL((k_fit_partials<T, 1>), grid, dim3(256), 0, st, ga, imap, n, inv2g2_px, slabs_per_group, parts, rows, colpart, sgpart); break;
    case 4: hipLaunchKernelGGL((k_fit_partials<T, 4>), grid, dim3(256), 0, st, ga, imap, n, inv2g2_px, slabs_per_group, parts, rows, colpart, sgpart); break;
    case 16: hipLaunchKernelGGL((k_fit_partials<T, 16>), grid, dim3(256), 0, st, ga, imap, n, inv2g2_px, slabs_per_group, parts, rows, colpart, sgpart); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fit_finish<T>, dim3((unsigned)((nn + 31) / 32)), dim3(256), 0, st, imap, n, groups, parts,
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
  const long long parts = fit_parts(n);
  return (size_t)(parts * nn + groups * nn + 1) * real_bytes + 8 + (size_t)(groups * parts) * 8;
}

template hipError_t launch_diag_embed<float2>(int, const float*, float2*, hipStream_t);
template hipError_t launch_diag_embed<double2>(int, const double*, double2*, hipStream_t);
template hipError_t launch_fit_gradient<float2>(int, const float2*, const float*, double, double, void*, float*,
                                                double*, hipStream_t);
template hipError_t launch_fit_gradient<double2>(int, const double2*, const float*, double, double, void*, float*,
                                                 double*, hipStream_t);

}  // namespace wolf
