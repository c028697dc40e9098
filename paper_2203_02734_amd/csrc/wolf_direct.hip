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
// Tiles of 64 x 64 outputs per workgroup of 256 threads; thread (tx, ty) owns rows ty + 16 r and
// columns tx + 16 c (r, c < 4), so that the LDS reads of a wavefront are broadcasts (A) or
// consecutive (B), and the stores are 16 consecutive elements. The k dimension is staged through
// LDS 16 at a time. Out-of-range elements load as zero and are not stored (NN < 64).
// complex128 tiles need about 200 registers: at most two waves per SIMD, rather than spills.
template <class T> constexpr int cgemm_max_waves() { return sizeof(T) == 16 ? 2 : 8; }

template <class T, bool CONJ_A, bool B_TRANS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, cgemm_max_waves<T>()))) void k_cgemm(const T* __restrict__ A, const T* __restrict__ B, T* __restrict__ C,
                                               int nn, double alpha) {
  using R = typename real_of<T>::type;
  constexpr int TM = 64, TN = 64, TK = 16;
  __shared__ T As[TK][TM + 1];
  __shared__ T Bs[TK][TN + 1];
  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;
  const long long i0 = (long long)blockIdx.y * TM, j0 = (long long)blockIdx.x * TN;
  T acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = T{(R)0, (R)0};
  const T zero{(R)0, (R)0};
  for (long long k0 = 0; k0 < nn; k0 += TK) {
    // All eight loads are issued before any is used (out-of-range lanes read element 0, then zero).
    T ra[4], rb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int ii = e / TK, kk = e % TK;
      const long long gi = i0 + ii, gk = k0 + kk;
      ra[q] = load_or_first(A, gi < nn && gk < nn, gi * nn + gk);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      if constexpr (B_TRANS) {
        const int jj = e / TK, kk = e % TK;
        const long long gj = j0 + jj, gk = k0 + kk;
        rb[q] = load_or_first(B, gj < nn && gk < nn, gj * nn + gk);
      } else {
        const int kk = e / TN, jj = e % TN;
        const long long gj = j0 + jj, gk = k0 + kk;
        rb[q] = load_or_first(B, gj < nn && gk < nn, gk * nn + gj);
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int ii = e / TK, kk = e % TK;
      T v = keep_or_zero(i0 + ii < nn && k0 + kk < nn, ra[q]);
      if constexpr (CONJ_A) v.y = -v.y;
      As[kk][ii] = v;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      if constexpr (B_TRANS) {
        const int jj = e / TK, kk = e % TK;
        Bs[kk][jj] = keep_or_zero(j0 + jj < nn && k0 + kk < nn, rb[q]);
      } else {
        const int kk = e / TN, jj = e % TN;
        Bs[kk][jj] = keep_or_zero(j0 + jj < nn && k0 + kk < nn, rb[q]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      T a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = As[kk][ty + 16 * r];
#pragma unroll
      for (int c = 0; c < 4; ++c) b[c] = Bs[kk][tx + 16 * c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          acc[r][c].x += a[r].x * b[c].x - a[r].y * b[c].y;
          acc[r][c].y += a[r].x * b[c].y + a[r].y * b[c].x;
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const long long gi = i0 + ty + 16 * r;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const long long gj = j0 + tx + 16 * c;
      if (gi < nn && gj < nn) C[gi * nn + gj] = T{(R)(alpha * acc[r][c].x), (R)(alpha * acc[r][c].y)};
    }
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
