// Propagation with the exact free-space kernel (eq. h_free), summed directly: the check of the
// approximation Lambda/r ~ Lambda/R (eq. approx_L) and of the Fresnel expansion (eq. W_fresnel).
//
// h(x, xi) = Lambda(r) exp(i k r) / r with r = sqrt(z^2 + |x - xi|^2). A secondary source at normal
// incidence has Lambda = (k / (4 pi i)) (1 + z / r); a primary one Lambda = 1 / (4 pi). The factor 1/i
// and the common phase exp(i k z) cancel between h* and h and are left out, so
//   H[m][p] = |Lambda(r)| exp(2 pi i (r - z) / lambda) / r,   r - z = rho^2 / (r + z)  (no cancellation),
// on the output grid of the Fresnel operator (pitch lambda z / (N pitch)) and the source grid.
// The kernel does not factorise over x and y, so the sum is a dense contraction over N^2 source
// points for each point: W_B = pitch^4 conj(H) W_A H^T, two complex GEMMs of size N^2.
#include "wolf_device.hpp"
#include "wolf_internal.hpp"
#include "wolf_mfma.hpp"

namespace wolf {

template <class T>
__global__ __launch_bounds__(256) void k_rs_kernel(T* __restrict__ h, int n, double pitch, double dx, double z,
                                                   double lam, int primary) {
  using R = typename real_of<T>::type;
  const long long nn = (long long)n * n, total = nn * nn;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long m = e / nn, p = e - m * nn;
    const int mi = (int)(m / n), mj = (int)(m % n), pi = (int)(p / n), pj = (int)(p % n);
    // x = d (i - N/2), y = d (N/2 - j) on both grids (the y flip enters both coordinates alike).
    const double ddx = dx * (mi - n / 2) - pitch * (pi - n / 2);
    const double ddy = dx * (n / 2 - mj) - pitch * (n / 2 - pj);
    const double rho2 = ddx * ddx + ddy * ddy;
    const double r = sqrt(z * z + rho2);
    const double cyc = rho2 / ((r + z) * lam);  // (r - z) / lambda
    const double red = cyc - rint(cyc);          // cycles mod 1, exact
    double s, c;
    sincospi(2.0 * red, &s, &c);
    const double amp = (primary ? 1.0 / (4.0 * M_PI) : (1.0 + z / r) / (2.0 * lam)) / r;
    h[e] = T{(R)(amp * c), (R)(amp * s)};
  }
}

// C = alpha op(A) op(B), complex, square NN x NN, row-major. op(A) = A or conj(A) (CONJ_A).
// B_TRANS: op(B)[k][j] = B[j][k]; else op(B)[k][j] = B[k][j].
// On the matrix cores (FP32 for complex64, FP64 for complex128) in the 3M form: 64 x 64 outputs per
// workgroup of four wavefronts (32 x 32 blocks), k staged through double-buffered LDS 16 at a time, the
// HBM loads of step s + 1 issued before the products of step s. Out-of-range elements load as zero and
// are not stored (NN < 64).
template <class T, bool CONJ_A, bool B_TRANS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 3 : 2))) void k_cgemm(
    const T* __restrict__ A, const T* __restrict__ B, T* __restrict__ C, int nn, double alpha) {
  using R = typename real_of<T>::type;
  using G = MTile<64>;
  constexpr int TK = 16;
  __shared__ R ar[2][TK][G::LDA], ai[2][TK][G::LDA], br[2][TK][G::LDB], bi[2][TK][G::LDB];
  const int tid = threadIdx.x, lane = tid % 64;
  const int wv = __builtin_amdgcn_readfirstlane(tid / 64);  // wavefront-uniform
  const int row0 = (wv / G::WC) * 32, col0 = (wv % G::WC) * 32;
  const long long i0 = (long long)blockIdx.y * 64, j0 = (long long)blockIdx.x * 64;
  // Element q of thread tid in a step: rows of A (and of B when B_TRANS) as (row e / 16, k e % 16): 16
  // consecutive k of one row; B otherwise as (k e / 64, column e % 64): 64 consecutive columns.
  T ra[4], rb[4];
  auto fetch = [&](long long k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const long long gi = i0 + e / TK, gk = k0 + e % TK;
      ra[q] = load_or_first(A, gi < nn && gk < nn, gi * nn + gk);
      if constexpr (B_TRANS) {
        const long long gj = j0 + e / TK;
        rb[q] = load_or_first(B, gj < nn && gk < nn, gj * nn + gk);
      } else {
        const long long gj = j0 + e % 64, gkb = k0 + e / 64;
        rb[q] = load_or_first(B, gj < nn && gkb < nn, gkb * nn + gj);
      }
    }
  };
  auto stage = [&](int buf, long long k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int ii = e / TK, kk = e % TK;
      T v = keep_or_zero(i0 + ii < nn && k0 + kk < nn, ra[q]);
      if constexpr (CONJ_A) v.y = -v.y;
      ar[buf][kk][ii] = v.x;
      ai[buf][kk][ii] = v.y;
      const int jj = B_TRANS ? e / TK : e % 64, kb = B_TRANS ? e % TK : e / 64;
      const T u = keep_or_zero(j0 + jj < nn && k0 + kb < nn, rb[q]);
      br[buf][kb][jj] = u.x;
      bi[buf][kb][jj] = u.y;
    }
  };
  CTile<T> acc;
  ctile_zero(acc);
  fetch(0);
  stage(0, 0);
  __syncthreads();
  int buf = 0;
  for (long long k0 = 0; k0 < nn; k0 += TK) {
    const bool more = k0 + TK < nn;
    if (more) fetch(k0 + TK);
    ctile_mfma16<T, G::LDA, G::LDB>(acc, ar[buf], ai[buf], br[buf], bi[buf], row0, col0, lane);
    if (more) stage(buf ^ 1, k0 + TK);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const long long gi = i0 + row0 + 16 * r + Mfma<T>::row(lane, i), gj = j0 + col0 + 16 * q + lane % 16;
        if (gi < nn && gj < nn)
          C[gi * nn + gj] = T{(R)(alpha * acc.re(r, q, i)), (R)(alpha * acc.im(r, q, i))};
      }
}

template <class T>
hipError_t launch_direct(int n, const T* in, T* out, void* work, double pitch, double lam, double z, int primary,
                         hipStream_t st) {
  const long long nn = (long long)n * n, total = nn * nn;
  T* h = reinterpret_cast<T*>(work);
  T* t1 = h + total;
  const double dx = lam * z / ((double)n * pitch);
  long long blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_rs_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, st, h, n, pitch, dx, z, lam, primary);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned tiles = (unsigned)((nn + 63) / 64);
  // T1[p1][m2] = sum_p2 W[p1][p2] H[m2][p2]
  hipLaunchKernelGGL((k_cgemm<T, false, true>), dim3(tiles, tiles), dim3(256), 0, st, in, (const T*)h, t1, (int)nn,
                     1.0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // W_B[m1][m2] = pitch^4 sum_p1 conj(H[m1][p1]) T1[p1][m2]
  const double s = pitch * pitch * pitch * pitch;
  hipLaunchKernelGGL((k_cgemm<T, true, false>), dim3(tiles, tiles), dim3(256), 0, st, (const T*)h, (const T*)t1, out,
                     (int)nn, s);
  return hipGetLastError();
}

size_t direct_work_bytes(int n, int elem) { return 2 * (size_t)n * n * n * n * (size_t)elem; }

template hipError_t launch_direct<float2>(int, const float2*, float2*, void*, double, double, double, int, hipStream_t);
template hipError_t launch_direct<double2>(int, const double2*, double2*, void*, double, double, double, int,
                                           hipStream_t);

}  // namespace wolf
