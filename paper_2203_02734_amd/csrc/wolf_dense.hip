// The propagation operator for any even N and any transform length N_z >= N: zero padding of
// the N-point axes to N_z points and cropping back to N (Sec. 3.3), and N that are not powers of two.
//
// Along one axis the operator is
//   y[k] = post[k] sum_n e^{SIGN 2 pi i (k - N/2)(n - N/2) / N_z} pre[n] x[n],   k, n in [0, N),
// the N central outputs of the centred N_z-point DFT of the N inputs embedded in N_z - N zeros. The
// index (k - N/2)(n - N/2) mod N_z is exact in integers, and the table of the N_z roots of unity is
// built in FP64. There is no FFT here: each axis is a dense product of the N x N matrix (generated
// from the table, never stored) with the N-point lines of the array, tiled like a GEMM (64 x 64
// outputs per tile, 4 x 4 per thread, 16 inputs per LDS stage) on a persistent grid that builds
// the tables once per workgroup. The four axes run as four passes that alternate between the
// output and a work buffer.
//   COLS: a strided axis (stride S); the lines of one batch o are S contiguous columns:
//         out[o N S + k S + c] from in[o N S + n S + c], tiles of 64 k x 64 c.
//   !COLS: the contiguous axis: out[r N + k] from in[r N + n], tiles of 64 r x 64 k.
#include "wolf_device.hpp"
#include "wolf_internal.hpp"

namespace wolf {

constexpr int kDenseMaxNz = 2048;
constexpr int kDenseMaxN = 256;

struct DenseAxis {
  long long S;       // stride of the axis (COLS), columns per batch
  long long outer;   // batches (COLS)
  long long rows;    // lines (!COLS)
  long long ctiles;  // column tiles per batch (COLS)
  int n, nz;
};

__device__ __forceinline__ int dense_index(int k, int n, int c, int nz) {
  int m = ((k - c) * (n - c)) % nz;
  return m < 0 ? m + nz : m;
}

template <class T, bool COLS, int SIGN>
__global__ __launch_bounds__(256) void k_dense_axis(const T* __restrict__ in, T* __restrict__ out, DenseAxis d,
                                                    Chirp pre, Chirp post, double scale) {
  using R = typename real_of<T>::type;
  constexpr int TM = 64, TN = 64, TK = 16;
  __shared__ T tw[kDenseMaxNz];
  __shared__ T tpre[kDenseMaxN], tpost[kDenseMaxN];
  __shared__ T As[TK][TM + 1];
  __shared__ T Bs[TK][TN + 1];
  const int tid = threadIdx.x;
  const int n = d.n, nz = d.nz, c0 = n / 2;
  for (int i = tid; i < nz; i += 256) tw[i] = twiddle_entry<T, SIGN>(i, nz);
  for (int i = tid; i < n; i += 256) {
    tpre[i] = chirp_entry<T>(pre, i, n);
    tpost[i] = chirp_entry<T>(post, i, n);
  }
  __syncthreads();
  const int tx = tid % 16, ty = tid / 16;
  const T zero{(R)0, (R)0};
  const long long ktiles = (n + TM - 1) / TM;
  const long long tiles = COLS ? d.outer * d.ctiles * ktiles : ((d.rows + TM - 1) / TM) * ktiles;
  // Persistent grid: the tables above are built once per workgroup, then it takes every
  // gridDim-th tile.
  for (long long t = blockIdx.x; t < tiles; t += gridDim.x) {
    long long o = 0, i0, j0;
    if constexpr (COLS) {
      const long long kt = t % ktiles, rest = t / ktiles;
      o = rest / d.ctiles;
      j0 = (rest - o * d.ctiles) * TN;  // columns c
      i0 = kt * TM;                      // outputs k
    } else {
      i0 = (t / ktiles) * TM;            // lines r
      j0 = (t % ktiles) * TN;            // outputs k
    }
    const long long base = o * (long long)n * d.S;
    T acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[r][c] = zero;
    for (int n0 = 0; n0 < n; n0 += TK) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = tid + 256 * q;
        const int ii = e / TK, kk = e % TK;
        const long long gi = i0 + ii;
        const int gn = n0 + kk;
        T v = zero;
        if constexpr (COLS) {
          if (gi < n && gn < n) v = tw[dense_index((int)gi, gn, c0, nz)];
        } else {
          if (gi < d.rows && gn < n) v = cmul(in[gi * n + gn], tpre[gn]);
        }
        As[kk][ii] = v;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = tid + 256 * q;
        T v = zero;
        if constexpr (COLS) {
          const int kk = e / TN, jj = e % TN;
          const long long gc = j0 + jj;
          const int gn = n0 + kk;
          if (gc < d.S && gn < n) v = cmul(in[base + (long long)gn * d.S + gc], tpre[gn]);
          Bs[kk][jj] = v;
        } else {
          const int jj = e / TK, kk = e % TK;
          const long long gk = j0 + jj;
          const int gn = n0 + kk;
          if (gk < n && gn < n) v = tw[dense_index((int)gk, gn, c0, nz)];
          Bs[kk][jj] = v;
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
        if constexpr (COLS) {
          if (gi < n && gj < d.S) {
            const T v = cmul(acc[r][c], tpost[gi]);
            out[base + gi * d.S + gj] = T{(R)(scale * v.x), (R)(scale * v.y)};
          }
        } else {
          if (gi < d.rows && gj < n) {
            const T v = cmul(acc[r][c], tpost[gj]);
            out[gi * n + gj] = T{(R)(scale * v.x), (R)(scale * v.y)};
          }
        }
      }
    }
  }
}

template <class T, bool COLS>
static hipError_t launch_dense_axis(const T* in, T* out, const DenseAxis& d, int sign, const Chirp& pre,
                                    const Chirp& post, double scale, hipStream_t st) {
  const long long ktiles = (d.n + 63) / 64;
  const long long tiles = COLS ? d.outer * d.ctiles * ktiles : ((d.rows + 63) / 64) * ktiles;
  const long long grid = tiles < 2048 ? tiles : 2048;  // a few resident workgroups per CU
  if (grid < 1) return hipSuccess;
  if (sign < 0)
    hipLaunchKernelGGL((k_dense_axis<T, COLS, -1>), dim3((unsigned)grid), dim3(256), 0, st, in, out, d, pre, post,
                       scale);
  else
    hipLaunchKernelGGL((k_dense_axis<T, COLS, +1>), dim3((unsigned)grid), dim3(256), 0, st, in, out, d, pre, post,
                       scale);
  return hipGetLastError();
}

bool dense_supported(int n, int nz) { return n >= 2 && n <= kDenseMaxN && n % 2 == 0 && nz >= n && nz <= kDenseMaxNz; }

// in -> (j2) work -> (i2) out -> (j1) work -> (i1) out. in == out is allowed (the first pass reads in
// completely before the second writes out); work must not overlap either.
template <class T>
hipError_t launch_operator_dense(int n, int nz, const T* in, T* out, T* work, const OperatorTables& op,
                                 hipStream_t st) {
  if (!dense_supported(n, nz)) return hipErrorInvalidValue;
  const long long N = n, NN = N * N, NNN = NN * N;
  hipError_t e;
  DenseAxis d{};
  d.n = n;
  d.nz = nz;
  d.rows = NNN;
  if ((e = launch_dense_axis<T, false>(in, work, d, op.sign2, op.pre2, op.post2, 1.0, st)) != hipSuccess) return e;
  d = DenseAxis{N, NN, 0, (N + 63) / 64, n, nz};  // i2: stride N, N^2 batches
  if ((e = launch_dense_axis<T, true>(work, out, d, op.sign2, op.pre2, op.post2, 1.0, st)) != hipSuccess) return e;
  d = DenseAxis{NN, N, 0, (NN + 63) / 64, n, nz};  // j1: stride N^2, N batches
  if ((e = launch_dense_axis<T, true>(out, work, d, op.sign1, op.pre1, op.post1, 1.0, st)) != hipSuccess) return e;
  d = DenseAxis{NNN, 1, 0, (NNN + 63) / 64, n, nz};  // i1: stride N^3, one batch
  return launch_dense_axis<T, true>(work, out, d, op.sign1, op.pre1, op.post1, op.scale, st);
}

template hipError_t launch_operator_dense<float2>(int, int, const float2*, float2*, float2*, const OperatorTables&,
                                                  hipStream_t);
template hipError_t launch_operator_dense<double2>(int, int, const double2*, double2*, double2*,
                                                   const OperatorTables&, hipStream_t);

}  // namespace wolf
