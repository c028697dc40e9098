// Axis-FFT kernels of the CSD propagation operator, and the operator itself as a sequence of
// axis passes.
//
// The 4D array W[i1][j1][i2][j2] (Sec. 3.1) lives in HBM as one contiguous block with j2
// fastest. Every pass transforms one axis of length N for the whole array. It reads each element
// once and writes it once, and fuses the per-axis diagonal factors into its load and store.
//
// Length-N DFT across threads (N = N1 N2, N1 >= N2). Thread t of an FFT loads x[N2 a + t],
// a = 0..N1-1, and does an N1-point DFT in registers. It then multiplies by w_N^{t k1} and passes
// the values through LDS. After the exchange each thread holds, for its k1 values, the N2 inputs
// of an N2-point DFT in registers, and the outputs land at X[k1 + N1 k2].
#include "wolf_device.hpp"
#include "wolf_internal.hpp"

namespace wolf {

// ---------------------------------------------------------------------------------------------
// Strided axis: element (o, n, c) at o * outer_stride + n * axis_stride + c, c in [0, inner_len).
// A workgroup takes one outer index and C consecutive c (coalesced runs of C elements).
// ---------------------------------------------------------------------------------------------
template <class T, int N, int C, int SIGN>
__global__ __launch_bounds__(Split<N>::N2 * C) void k_axis_fft(const T* src, T* dst,
                                                              long long outer_stride, long long axis_stride,
                                                              long long tiles_per_outer, Chirp pre, Chirp post) {
  using S = Split<N>;
  constexpr int N1 = S::N1, N2 = S::N2, Q = S::Q;
  constexpr int NT = N2 * C;
  __shared__ T xch[N * C];
  __shared__ T tpre[N], tpost[N], tw[N];

  for (int i = threadIdx.x; i < N; i += NT) {
    tpre[i] = chirp_entry<T>(pre, i, N);
    tpost[i] = chirp_entry<T>(post, i, N);
    tw[i] = twiddle_entry<T, SIGN>(i, N);
  }
  __syncthreads();

  const int c = threadIdx.x % C;
  const int t = threadIdx.x / C;
  const long long bid = blockIdx.x;
  const long long o = bid / tiles_per_outer;
  const long long c0 = (bid - o * tiles_per_outer) * C;
  const long long base = o * outer_stride + c0 + c;

  T v[N1];
#pragma unroll
  for (int a = 0; a < N1; ++a) {
    const int n = N2 * a + t;
    v[a] = cmul(src[base + (long long)n * axis_stride], tpre[n]);
  }
  dft_reg<N1, SIGN>(v);
#pragma unroll
  for (int k1 = 0; k1 < N1; ++k1) {
    xch[(k1 * N2 + t) * C + c] = cmul(v[k1], tw[(t * k1) & (N - 1)]);
  }
  __syncthreads();
  T u[N1];
#pragma unroll
  for (int r = 0; r < Q; ++r) {
    const int k1 = t * Q + r;
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) u[r * N2 + n2] = xch[(k1 * N2 + n2) * C + c];
    dft_reg<N2, SIGN>(&u[r * N2]);
  }
#pragma unroll
  for (int r = 0; r < Q; ++r) {
    const int k1 = t * Q + r;
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      const int k = k1 + N1 * k2;
      dst[base + (long long)k * axis_stride] = cmul(u[r * N2 + k2], tpost[k]);
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Contiguous axis (rows of N elements). A workgroup takes B consecutive rows.
// ---------------------------------------------------------------------------------------------
template <class T, int N, int B, int SIGN>
__global__ __launch_bounds__(Split<N>::N2 * B) void k_row_fft(const T* src, T* dst,
                                                             Chirp pre, Chirp post) {
  using S = Split<N>;
  constexpr int N1 = S::N1, N2 = S::N2, Q = S::Q;
  constexpr int NT = N2 * B;
  constexpr int LD = N2 + 1;  // padded stride of one k1 group in LDS
  __shared__ T xch[B * N1 * LD];
  __shared__ T tpre[N], tpost[N], tw[N];

  for (int i = threadIdx.x; i < N; i += NT) {
    tpre[i] = chirp_entry<T>(pre, i, N);
    tpost[i] = chirp_entry<T>(post, i, N);
    tw[i] = twiddle_entry<T, SIGN>(i, N);
  }
  __syncthreads();

  const int t = threadIdx.x % N2;
  const int r = threadIdx.x / N2;
  const long long row = (long long)blockIdx.x * B + r;
  const T* in = src + row * N;
  T* out = dst + row * N;

  T v[N1];
#pragma unroll
  for (int a = 0; a < N1; ++a) {
    const int n = N2 * a + t;
    v[a] = cmul(in[n], tpre[n]);
  }
  dft_reg<N1, SIGN>(v);
#pragma unroll
  for (int k1 = 0; k1 < N1; ++k1) xch[(r * N1 + k1) * LD + t] = cmul(v[k1], tw[(t * k1) & (N - 1)]);
  __syncthreads();
  T u[N1];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int k1 = t * Q + q;
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) u[q * N2 + n2] = xch[(r * N1 + k1) * LD + n2];
    dft_reg<N2, SIGN>(&u[q * N2]);
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int k1 = t * Q + q;
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      const int k = k1 + N1 * k2;
      out[k] = cmul(u[q * N2 + k2], tpost[k]);
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------------------------
template <int N> constexpr int axis_cols() {
  constexpr int c = 256 / Split<N>::N2;
  return c < N ? c : N;
}
template <int N> constexpr int row_batch() {
  constexpr int b = 256 / Split<N>::N2;
  return b < N * N * N ? b : N * N * N;
}

template <class T, int N, int SIGN>
static hipError_t launch_axis_n(const T* src, T* dst, int axis, const Chirp& pre, const Chirp& post,
                                hipStream_t st) {
  // axis 0 = i1, 1 = j1, 2 = i2 (the strided axes of [i1][j1][i2][j2]).
  constexpr int C = axis_cols<N>();
  const long long n = N;
  long long outer_count, outer_stride, axis_stride, inner_len;
  if (axis == 0) { outer_count = 1; outer_stride = 0; axis_stride = n * n * n; inner_len = n * n * n; }
  else if (axis == 1) { outer_count = n; outer_stride = n * n * n; axis_stride = n * n; inner_len = n * n; }
  else { outer_count = n * n; outer_stride = n * n; axis_stride = n; inner_len = n; }
  const long long tiles = inner_len / C;
  const long long blocks = outer_count * tiles;
  hipLaunchKernelGGL((k_axis_fft<T, N, C, SIGN>), dim3((unsigned)blocks), dim3(Split<N>::N2 * C), 0, st, src, dst,
                     outer_stride, axis_stride, tiles, pre, post);
  return hipGetLastError();
}

template <class T, int N, int SIGN>
static hipError_t launch_row_n(const T* src, T* dst, const Chirp& pre, const Chirp& post, hipStream_t st) {
  constexpr int B = row_batch<N>();
  const long long rows = (long long)N * N * N;
  const long long blocks = rows / B;   // N^3 is a multiple of B for every supported N
  hipLaunchKernelGGL((k_row_fft<T, N, B, SIGN>), dim3((unsigned)blocks), dim3(Split<N>::N2 * B), 0, st, src, dst,
                     pre, post);
  return hipGetLastError();
}

template <class T, int SIGN>
static hipError_t launch_axis_sign(int n, const T* src, T* dst, int axis, const Chirp& pre, const Chirp& post,
                                   hipStream_t st) {
  switch (n) {
#define WOLF_CASE(NN)                                                                  \
  case NN:                                                                             \
    return axis == 3 ? launch_row_n<T, NN, SIGN>(src, dst, pre, post, st)             \
                     : launch_axis_n<T, NN, SIGN>(src, dst, axis, pre, post, st);
    WOLF_CASE(2) WOLF_CASE(4) WOLF_CASE(8) WOLF_CASE(16) WOLF_CASE(32) WOLF_CASE(64) WOLF_CASE(128) WOLF_CASE(256)
#undef WOLF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <class T>
hipError_t launch_axis_pass(int n, const T* src, T* dst, int axis, int sign, const Chirp& pre, const Chirp& post,
                            hipStream_t st) {
  return sign < 0 ? launch_axis_sign<T, -1>(n, src, dst, axis, pre, post, st)
                  : launch_axis_sign<T, +1>(n, src, dst, axis, pre, post, st);
}

template hipError_t launch_axis_pass<float2>(int, const float2*, float2*, int, int, const Chirp&, const Chirp&,
                                             hipStream_t);
template hipError_t launch_axis_pass<double2>(int, const double2*, double2*, int, int, const Chirp&, const Chirp&,
                                              hipStream_t);

}  // namespace wolf
