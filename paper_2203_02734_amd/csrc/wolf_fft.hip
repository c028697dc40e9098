// Axis-FFT kernels of the CSD propagation operator, and the operator as a schedule of passes.
//
// The 4D array W[i1][j1][i2][j2] (Sec. 3.1) is one contiguous block in HBM, j2 fastest. The
// operator of eqs. (W_general)/(W_fresnel) factorises over the four axes. Along each axis it is a
// diagonal pre-factor, a length-N centred DFT and a diagonal post-factor (see wolf_device.hpp).
// All four axis operations commute, so the passes may be grouped and ordered freely:
//   slab pass   : both second-point axes (i2, j2) of one contiguous N x N slab, in LDS (one sweep).
//                 It also applies the first-point pre-factor, which is a scalar per slab.
//   axis passes : one strided axis (j1 or i1, or i2 when the slab pass does not fit), over a tile of
//                 C consecutive columns. It runs over column chunks, so that the two first-point
//                 passes can reuse the chunk from the 256 MB Infinity Cache.
//   row pass    : the contiguous axis j2 on its own (when the slab pass does not fit).
//
// Length-N DFT across threads (N = N1 N2, N1 >= N2). Thread t of one FFT loads x[N2 a + t],
// a = 0..N1-1, does an N1-point DFT in registers and multiplies by w_N^{t k1}. One exchange
// through LDS follows. Thread t then owns k1 = t + N2 r (r < N1/N2), does the N2-point DFTs over
// n2 and writes X[k1 + N1 k2]. With this ownership the outputs of the N2 threads are contiguous.
#include "wolf_device.hpp"
#include "wolf_internal.hpp"
#include "wolf_source.hpp"

namespace wolf {

// ---------------------------------------------------------------------------------------------
// Strided axis: element (o, n, c) at o * outer_stride + n * axis_stride + inner_offset + c.
// A workgroup takes one outer index and C consecutive columns c (coalesced runs of C elements).
// ---------------------------------------------------------------------------------------------
// NTL: the loads carry the nontemporal hint (data read once from HBM: the grouped schedule's final i1
// pass, and every axis pass in complex128; measured faster there, slower where the input comes from the
// memory-side cache).
template <class T, int N, int C, int SIGN, bool NTL = false>
__global__ __launch_bounds__(Split<N>::N2 * C) void k_axis_fft(const T* src, T* dst, AxisJob ja, AxisJob jb) {
  using S = Split<N>;
  constexpr int N1 = S::N1, N2 = S::N2, Q = S::Q;
  constexpr int NT = N2 * C;
  __shared__ T xch[N * C];
  __shared__ T tpre[N], tpost[N], tw[N];

  // Two independent jobs may share one launch (the j1 pass of one column chunk and the i1 pass of
  // the previous one). With equal sizes they interleave block by block.
  long long bid = blockIdx.x;
  bool second;
  if (jb.blocks == ja.blocks) {
    second = (bid & 1) != 0;
    bid >>= 1;
  } else {
    second = bid >= ja.blocks;
    if (second) bid -= ja.blocks;
  }
  const AxisJob& j = second ? jb : ja;

  for (int i = threadIdx.x; i < N; i += NT) {
    tpre[i] = chirp_entry<T>(j.pre, i, N);
    tpost[i] = chirp_entry<T>(j.post, i, N);
    tw[i] = twiddle_entry<T, SIGN>(i, N);
  }
  __syncthreads();

  const int c = threadIdx.x % C;
  const int t = threadIdx.x / C;
  const long long o = bid / j.tiles_per_outer;
  const long long c0 = (bid - o * j.tiles_per_outer) * C;
  const long long base = o * j.outer_stride + j.inner_offset + c0 + c;
  const long long as = j.axis_stride;

  T v[N1];
#pragma unroll
  for (int a = 0; a < N1; ++a) {
    const int n = N2 * a + t;
    if constexpr (NTL) {
      typedef typename real_of<T>::type R;
      typedef R r2 __attribute__((ext_vector_type(2)));
      const r2 x = __builtin_nontemporal_load(reinterpret_cast<const r2*>(src + base + (long long)n * as));
      v[a] = cmul(T{x.x, x.y}, tpre[n]);
    } else {
      v[a] = cmul(src[base + (long long)n * as], tpre[n]);
    }
  }
  dft_reg<N1, SIGN>(v);
#pragma unroll
  for (int k1 = 0; k1 < N1; ++k1) xch[(k1 * N2 + t) * C + c] = cmul(v[k1], tw[(t * k1) & (N - 1)]);
  __syncthreads();
  T u[N1];
#pragma unroll
  for (int r = 0; r < Q; ++r) {
    const int k1 = t + N2 * r;
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) u[r * N2 + n2] = xch[(k1 * N2 + n2) * C + c];
    dft_reg<N2, SIGN>(&u[r * N2]);
  }
#pragma unroll
  for (int r = 0; r < Q; ++r) {
    const int k1 = t + N2 * r;
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      const int k = k1 + N1 * k2;
      dst[base + (long long)k * as] = cmul(u[r * N2 + k2], tpost[k]);
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Contiguous axis (rows of N elements). A workgroup takes B consecutive rows.
// GEN > 0 (B <= N, so that the rows of a workgroup lie in one slab p1 = (i1, j1)): the input rows are
// the source W0 of `sp` (as in the slab pass: GEN = 1 without an aperture or a lens, 2 with a circle,
// square, annulus or lens), formed from the slab's row fy(j1, .) and the scalars fx(i1, i2) of its B
// rows; row0 is the global index of the launch's first row. W0 is never stored.
// ---------------------------------------------------------------------------------------------
template <class T, int N, int B, int SIGN, int GEN>
__global__ __launch_bounds__(Split<N>::N2 * B) void k_row_fft(const T* src, T* dst, Chirp pre, Chirp post,
                                                             long long row0, SourceParams sp) {
  using S = Split<N>;
  using R = typename real_of<T>::type;
  constexpr int N1 = S::N1, N2 = S::N2, Q = S::Q;
  constexpr int NT = N2 * B;
  constexpr int LD = N2 + 1;  // padded stride of one k1 group in LDS
  static_assert(GEN == 0 || B <= N, "generated rows of one workgroup lie in one slab");
  __shared__ T xch[B * N1 * LD];
  __shared__ T tpre[N], tpost[N], tw[N];
  __shared__ T gy[GEN ? N : 1], gx[GEN ? B : 1];  // GEN: fy(j1, .) and fx(i1, i2) of the B rows

  const long long first = row0 + (long long)blockIdx.x * B;  // GEN: global index of the first row
  const int i1 = (int)(first / ((long long)N * N)), j1 = (int)((first / N) % N);
  for (int i = threadIdx.x; i < N; i += NT) {
    tpre[i] = chirp_entry<T>(pre, i, N);
    tpost[i] = chirp_entry<T>(post, i, N);
    tw[i] = twiddle_entry<T, SIGN>(i, N);
    if constexpr (GEN > 0) gy[i] = axis_factor<T>(sp, j1, i, N);
  }
  if constexpr (GEN > 0) {
    for (int i = threadIdx.x; i < B; i += NT) gx[i] = axis_factor<T>(sp, i1, (int)((first + i) % N), N);
  }
  __syncthreads();

  const int t = threadIdx.x % N2;
  const int r = threadIdx.x / N2;
  const long long row = (long long)blockIdx.x * B + r;
  const T* in = src + row * N;
  T* out = dst + row * N;

  T v[N1];
  if constexpr (GEN > 0) {
    const int i2 = (int)((first + r) % N);
    const R am1 = GEN == 1 ? (R)sp.amplitude : slab_scale<R>(sp, i1, j1, N);  // A m(p1)
    const T fx = gx[r];
#pragma unroll
    for (int a = 0; a < N1; ++a) {
      const int n = N2 * a + t;
      R m = am1;
      if constexpr (GEN == 2) m = inside_coords(sp, i2 - N / 2, n - N / 2) ? am1 : (R)0;
      v[a] = cmul_exact(source_value(fx, gy[n], m), tpre[n]);
    }
  } else {
#pragma unroll
    for (int a = 0; a < N1; ++a) {
      const int n = N2 * a + t;
      v[a] = cmul_exact(in[n], tpre[n]);
    }
  }
  dft_reg<N1, SIGN>(v);
#pragma unroll
  for (int k1 = 0; k1 < N1; ++k1) xch[(r * N1 + k1) * LD + t] = cmul(v[k1], tw[(t * k1) & (N - 1)]);
  __syncthreads();
  T u[N1];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int k1 = t + N2 * q;
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) u[q * N2 + n2] = xch[(r * N1 + k1) * LD + n2];
    dft_reg<N2, SIGN>(&u[q * N2]);
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int k1 = t + N2 * q;
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      const int k = k1 + N1 * k2;
      out[k] = cmul(u[q * N2 + k2], tpost[k]);
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Slab pass: 2D DFT over (i2, j2) of one contiguous N x N slab per workgroup, N2 * N threads.
// Phase 1 transforms the columns (i2, stride N): the loads are coalesced along j2. Phase 2
// transforms the rows (j2) after a transpose through LDS. The LDS row stride SP keeps the 16-lane
// groups of both phases on distinct banks.
// ---------------------------------------------------------------------------------------------
template <int N> constexpr int slab_stride() {
  constexpr int need = Split<N>::N1 * (Split<N>::N2 + 1);
  constexpr int s = need > N ? need : N;
  return N >= 64 ? ((s % 16 == 8) ? s : s + ((8 - s % 16) + 16) % 16) : s;
}

template <class T, int N> constexpr size_t slab_lds_bytes() {
  return sizeof(T) * ((size_t)N * slab_stride<N>() + 3 * N + 2);
}

// The 2D transform of one slab, shared by the slab passes. The work is
// laid out for N2 N virtual threads; each real thread runs VT of them (virtual id = tid + vt NT / VT).
// `tid` is the real thread id. On return, virtual thread (t, r) = (id % N2, id / N2) holds in u[vt N1 + q N2 + k2] the transformed
// value of row r at column k = t + N2 q + N1 k2, before the column post-factor tpost[k]. The row
// post-factor tpost[r] is applied only if ROW_POST.

// Raw loads of one slab for the column phase: virtual thread (t, c) takes rows n = N2 a + t of
// column c into v[vt N1 + a].
template <class T, int N, int VT = 1>
__device__ __forceinline__ void slab_load(const T* in, T* v, int tid) {
  using S = Split<N>;
  constexpr int N1 = S::N1, N2 = S::N2;
  constexpr int NTR = N2 * N / VT;
#pragma unroll
  for (int vt = 0; vt < VT; ++vt) {
    const int id = tid + vt * NTR;
    const int c = id % N;
    const int t = id / N;
#pragma unroll
    for (int a = 0; a < N1; ++a) v[vt * N1 + a] = in[(N2 * a + t) * N + c];
  }
}

// Zero the loaded values outside the pupil (pu.geo != 0), in the layout of slab_load.
template <class T, int N, int VT = 1>
__device__ __forceinline__ void slab_mask(const Pupil& pu, T* v, int tid) {
  using S = Split<N>;
  using R = typename real_of<T>::type;
  constexpr int N1 = S::N1, N2 = S::N2;
  constexpr int NTR = N2 * N / VT;
  if (pu.geo == 0) return;
#pragma unroll
  for (int vt = 0; vt < VT; ++vt) {
    const int id = tid + vt * NTR;
    const int c = id % N;
    const int t = id / N;
#pragma unroll
    for (int a = 0; a < N1; ++a)
      if (!pupil_pass(pu, N2 * a + t, c, N)) v[vt * N1 + a] = T{(R)0, (R)0};
  }
}

// The transform of a slab whose raw values slab_load put in v (v is overwritten).
template <class T, int N, int SIGN, bool ROW_POST, int VT>
__device__ __forceinline__ void slab_transform_loaded(T* v, T* buf, const T* tpre, const T* tpost, const T* tw,
                                                      const T scal, T* u, int tid) {
  using S = Split<N>;
  constexpr int N1 = S::N1, N2 = S::N2, Q = S::Q;
  constexpr int SP = slab_stride<N>();
  constexpr int NTR = N2 * N / VT;  // real threads
  // Phase 1: columns. Virtual thread (t, c); c is the j2 column.
  {
#pragma unroll
    for (int vt = 0; vt < VT; ++vt) {
      const int id = tid + vt * NTR;
      const int c = id % N;
      const int t = id / N;
#pragma unroll
      for (int a = 0; a < N1; ++a) v[vt * N1 + a] = cmul(v[vt * N1 + a], tpre[N2 * a + t]);
      dft_reg<N1, SIGN>(&v[vt * N1]);
#pragma unroll
      for (int k1 = 0; k1 < N1; ++k1) buf[(k1 * N2 + t) * N + c] = cmul(v[vt * N1 + k1], tw[(t * k1) & (N - 1)]);
    }
    __syncthreads();
    T w[VT * N1];
#pragma unroll
    for (int vt = 0; vt < VT; ++vt) {
      const int id = tid + vt * NTR;
      const int c = id % N;
      const int t = id / N;
#pragma unroll
      for (int r = 0; r < Q; ++r) {
        const int k1 = t + N2 * r;
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) w[vt * N1 + r * N2 + n2] = buf[(k1 * N2 + n2) * N + c];
        dft_reg<N2, SIGN>(&w[vt * N1 + r * N2]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int vt = 0; vt < VT; ++vt) {
      const int id = tid + vt * NTR;
      const int c = id % N;
      const int t = id / N;
      const T cst = cmul(tpre[c], scal);  // j2 pre-factor and the slab's first-point factor
#pragma unroll
      for (int r = 0; r < Q; ++r) {
        const int k1 = t + N2 * r;
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) {
          const int k = k1 + N1 * k2;
          if constexpr (ROW_POST) buf[k * SP + c] = cmul(w[vt * N1 + r * N2 + k2], cmul(tpost[k], cst));
          else buf[k * SP + c] = cmul(w[vt * N1 + r * N2 + k2], cst);
        }
      }
    }
  }
  __syncthreads();
  // Phase 2: rows. Virtual thread (t, r); r is the i2 row.
  {
    T v[VT * N1];
#pragma unroll
    for (int vt = 0; vt < VT; ++vt) {
      const int id = tid + vt * NTR;
      const int t = id % N2;
      const int r = id / N2;
#pragma unroll
      for (int a = 0; a < N1; ++a) v[vt * N1 + a] = buf[r * SP + N2 * a + t];
      dft_reg<N1, SIGN>(&v[vt * N1]);
    }
    __syncthreads();
#pragma unroll
    for (int vt = 0; vt < VT; ++vt) {
      const int id = tid + vt * NTR;
      const int t = id % N2;
      const int r = id / N2;
#pragma unroll
      for (int k1 = 0; k1 < N1; ++k1)
        buf[r * SP + k1 * (N2 + 1) + t] = cmul(v[vt * N1 + k1], tw[(t * k1) & (N - 1)]);
    }
    __syncthreads();
#pragma unroll
    for (int vt = 0; vt < VT; ++vt) {
      const int id = tid + vt * NTR;
      const int t = id % N2;
      const int r = id / N2;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int k1 = t + N2 * q;
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) u[vt * N1 + q * N2 + n2] = buf[r * SP + k1 * (N2 + 1) + n2];
        dft_reg<N2, SIGN>(&u[vt * N1 + q * N2]);
      }
    }
  }
}

template <class T, int N, int SIGN>
__global__ __launch_bounds__(Split<N>::N2 * N) void k_slab_fft2(const T* src, T* dst, Chirp pre, Chirp post,
                                                               Chirp slab_pre, Pupil pu, long long slab0) {
  using S = Split<N>;
  using R = typename real_of<T>::type;
  constexpr int N1 = S::N1, N2 = S::N2, Q = S::Q;
  constexpr int NT = N2 * N;
  constexpr int SP = slab_stride<N>();
  __shared__ T buf[N * SP];
  __shared__ T tpre[N], tpost[N], tw[N], sc[2];

  const long long p1 = slab0 + blockIdx.x;
  const int a1 = (int)(p1 / N), b1 = (int)(p1 % N);
  for (int i = threadIdx.x; i < N; i += NT) {
    tpre[i] = chirp_entry<T>(pre, i, N);
    tpost[i] = chirp_entry<T>(post, i, N);
    tw[i] = twiddle_entry<T, SIGN>(i, N);
  }
  if (threadIdx.x < 2) sc[threadIdx.x] = chirp_entry<T>(slab_pre, threadIdx.x == 0 ? a1 : b1, N);
  __syncthreads();
  T v[N1];
  slab_load<T, N>(src + p1 * N * N, v, (int)threadIdx.x);
  slab_mask<T, N>(pu, v, (int)threadIdx.x);
  T scal = cmul(sc[0], sc[1]);
  if (!pupil_pass(pu, a1, b1, N)) scal = T{(R)0, (R)0};
  T u[N1];
  slab_transform_loaded<T, N, SIGN, true, 1>(v, buf, tpre, tpost, tw, scal, u, (int)threadIdx.x);
  T* out = dst + p1 * N * N;
  const int t = threadIdx.x % N2;
  const int r = threadIdx.x / N2;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int k1 = t + N2 * q;
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      const int k = k1 + N1 * k2;
      out[r * N + k] = cmul(u[q * N2 + k2], tpost[k]);
    }
  }
}

// Slab pass with half the LDS of k_slab_fft2. The column exchange runs for the two column halves in
// turn, and the transposition to rows plus the row exchange for the two row halves in turn, each
// through a buffer of N/2 rows. At N = 128 that buffer is 70 KB in complex64, so two workgroups are
// resident per CU (one loads while the other computes), and 139 KB in complex128, which fits where
// the whole slab (256 KB) does not. Thread tid plays (t1, c) = (tid / H, tid % H + H vt) in the column
// phase and (t2, r) = (tid % N2, tid / N2 + H h) in the row phase, with H = N/2.
template <class T, int N> constexpr size_t half_lds_bytes() {
  return sizeof(T) * ((size_t)(N / 2) * slab_stride<N>() + 3 * N + 2);
}

// Two resident workgroups per CU where the LDS allows it (complex64): waves per SIMD for the register
// budget (512 VGPRs per SIMD lane shared by the resident waves).
template <class T, int N> constexpr int half_waves_per_simd() {
  constexpr int waves = (Split<N>::N2 * N / 2 + 63) / 64 / 4;
  return (2 * half_lds_bytes<T, N>() <= kMaxLds ? 2 : 1) * (waves < 1 ? 1 : waves);
}

// GEN > 0: the slab's input is the source W0 of `sp` (wolf_source.hpp), formed where it would be
// loaded, so W0 is never stored; the values are the builder's, bit for bit. Sources decided by the
// coordinates alone (GSM and coherent models, a lens): GEN = 1 without an aperture or a lens (real
// rows: the builder's complex product is then (fx fy A, +0) exactly), GEN = 2 otherwise. The column phase uses the first N H entries of the buffer; the two
// source rows sit behind them until the row phase.
// NTL: the input loads carry the nontemporal hint (the grouped schedule's slab pass in complex64, whose
// input is read once from HBM while the memory-side cache holds the previous group for its j1 pass).
template <class T, int N, int SIGN, int GEN, bool NTL = false>
__global__ __launch_bounds__(Split<N>::N2 * N / 2) __attribute__((amdgpu_waves_per_eu(half_waves_per_simd<T, N>())))
void k_slab_half(const T* src, T* dst, Chirp pre, Chirp post, Chirp slab_pre, Pupil pu, SourceParams sp,
                 long long slab0) {
  using S = Split<N>;
  using R = typename real_of<T>::type;
  constexpr int N1 = S::N1, N2 = S::N2, Q = S::Q;
  constexpr int H = N / 2;
  constexpr int NT = N2 * H;
  constexpr int SP = slab_stride<N>();
  static_assert(H % N1 == 0 && SP >= N, "half slab layout");
  __shared__ T buf[H * SP];
  __shared__ T tpre[N], tpost[N], tw[N], sc[2];
  static_assert(H * SP - N * H >= 2 * N, "source rows behind the column-phase buffer");
  T* const gx = buf + N * H;  // GEN: the source rows fx(i1, .), fy(j1, .)
  T* const gy = gx + N;

  const long long p1 = slab0 + blockIdx.x;
  const int a1 = (int)(p1 / N), b1 = (int)(p1 % N);
  for (int i = threadIdx.x; i < N; i += NT) {
    tpre[i] = chirp_entry<T>(pre, i, N);
    tpost[i] = chirp_entry<T>(post, i, N);
    tw[i] = twiddle_entry<T, SIGN>(i, N);
    if constexpr (GEN > 0) {
      gx[i] = axis_factor<T>(sp, a1, i, N);
      gy[i] = axis_factor<T>(sp, b1, i, N);
    }
  }
  if (threadIdx.x < 2) sc[threadIdx.x] = chirp_entry<T>(slab_pre, threadIdx.x == 0 ? a1 : b1, N);
  const int tid = threadIdx.x;
  const int t1 = tid / H, cl = tid % H;
  const T* in = src + p1 * N * N;
  __syncthreads();  // tables
  T scal = cmul(sc[0], sc[1]);
  if (!pupil_pass(pu, a1, b1, N)) scal = T{(R)0, (R)0};

  // Column phase, one column half at a time: buffer X[(k1 N2 + t1)][cl] of N x H entries. The loads
  // of a half are issued when it starts; the other resident workgroup hides their latency.
  T w[2][N1];
#pragma unroll
  for (int vt = 0; vt < 2; ++vt) {
    const int c = cl + H * vt;
    T v[N1];
    if constexpr (GEN == 1) {
      const R am1 = (R)sp.amplitude;  // A m(p1) with no aperture and no map
      const R fy = gy[c].x;
#pragma unroll
      for (int a = 0; a < N1; ++a) v[a] = T{(gx[N2 * a + t1].x * fy) * am1, (R)0};
    } else if constexpr (GEN == 2) {
      const R am1 = slab_scale<R>(sp, a1, b1, N);
#pragma unroll
      for (int a = 0; a < N1; ++a) v[a] = source_entry_coords<T>(sp, gx, gy, am1, N2 * a + t1, c, N);
    } else {
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        if constexpr (NTL) {
          typedef R r2 __attribute__((ext_vector_type(2)));
          const r2 x = __builtin_nontemporal_load(reinterpret_cast<const r2*>(in + (N2 * a + t1) * N + c));
          v[a] = T{x.x, x.y};
        } else {
          v[a] = in[(N2 * a + t1) * N + c];
        }
      }
    }
    if (pu.geo != 0) {
#pragma unroll
      for (int a = 0; a < N1; ++a)
        if (!pupil_pass(pu, N2 * a + t1, c, N)) v[a] = T{(R)0, (R)0};
    }
    const T cst = cmul(tpre[c], scal);
#pragma unroll
    for (int a = 0; a < N1; ++a) v[a] = cmul_exact(v[a], tpre[N2 * a + t1]);
    dft_reg<N1, SIGN>(v);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) buf[(k1 * N2 + t1) * H + cl] = cmul(v[k1], tw[(t1 * k1) & (N - 1)]);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int k1 = t1 + N2 * q;
#pragma unroll
      for (int n2 = 0; n2 < N2; ++n2) w[vt][q * N2 + n2] = buf[(k1 * N2 + n2) * H + cl];
      dft_reg<N2, SIGN>(&w[vt][q * N2]);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) {
        const int k = t1 + N2 * q + N1 * k2;
        w[vt][q * N2 + k2] = cmul(w[vt][q * N2 + k2], cmul(tpost[k], cst));
      }
  }

  // Row phase, one row half at a time: rows k in [H h, H h + H) are written to the buffer (row
  // k - H h, stride SP), transformed by threads (t2, rl), and stored.
  const int t2 = tid % N2, rl = tid / N2;
  T* out = dst + p1 * N * N;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int vt = 0; vt < 2; ++vt)
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) {
          // k = t1 + N2 q + N1 k2 with t1 + N2 q < N1, so k / H = k2 / (H / N1): fixed at compile time.
          if ((k2 * N1) / H != h) continue;
          const int k = t1 + N2 * q + N1 * k2;
          buf[(k - H * h) * SP + cl + H * vt] = w[vt][q * N2 + k2];
        }
    __syncthreads();
    T x[N1];
#pragma unroll
    for (int a = 0; a < N1; ++a) x[a] = buf[rl * SP + N2 * a + t2];
    dft_reg<N1, SIGN>(x);
    __syncthreads();
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) buf[rl * SP + k1 * (N2 + 1) + t2] = cmul(x[k1], tw[(t2 * k1) & (N - 1)]);
    __syncthreads();
    T u[N1];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int k1 = t2 + N2 * q;
#pragma unroll
      for (int n2 = 0; n2 < N2; ++n2) u[q * N2 + n2] = buf[rl * SP + k1 * (N2 + 1) + n2];
      dft_reg<N2, SIGN>(&u[q * N2]);
    }
    const int r = rl + H * h;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int k1 = t2 + N2 * q;
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) {
        const int k = k1 + N1 * k2;
        out[r * N + k] = cmul(u[q * N2 + k2], tpost[k]);
      }
    }
    __syncthreads();  // the next half reuses the buffer
  }
}

// Persistent form of the slab pass: each workgroup takes every gridDim-th slab and keeps its
// tables. The raw values of its next slab are loaded into registers while it transforms the
// current one, so the loads of one slab overlap the arithmetic of the previous one.
template <class T, int N, int SIGN>
__global__ __launch_bounds__(Split<N>::N2 * N) void k_slab_fft2p(const T* src, T* dst, long long slab0, long long slab_end,
                                                                Chirp pre, Chirp post, Chirp slab_pre, Pupil pu) {
  using S = Split<N>;
  using R = typename real_of<T>::type;
  constexpr int N1 = S::N1, N2 = S::N2, Q = S::Q;
  constexpr int NT = N2 * N;
  constexpr int SP = slab_stride<N>();
  __shared__ T buf[N * SP];
  __shared__ T tpre[N], tpost[N], tw[N], tpre1[N];
  for (int i = threadIdx.x; i < N; i += NT) {
    tpre[i] = chirp_entry<T>(pre, i, N);
    tpost[i] = chirp_entry<T>(post, i, N);
    tw[i] = twiddle_entry<T, SIGN>(i, N);
    tpre1[i] = chirp_entry<T>(slab_pre, i, N);
  }
  __syncthreads();
  const long long nn = (long long)N * N;
  long long p1 = slab0 + blockIdx.x;
  if (p1 >= slab_end) return;
  T cur[N1];
  slab_load<T, N>(src + p1 * nn, cur, (int)threadIdx.x);
  for (; p1 < slab_end; p1 += gridDim.x) {
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));  // recompute thread-derived addresses per slab
    const long long pn = p1 + gridDim.x;
    T nxt[N1];
    if (pn < slab_end) slab_load<T, N>(src + pn * nn, nxt, tid);
    T u[N1];
    const int a1 = (int)(p1 / N), b1 = (int)(p1 % N);
    slab_mask<T, N>(pu, cur, tid);
    T scal = cmul(tpre1[a1], tpre1[b1]);
    if (!pupil_pass(pu, a1, b1, N)) scal = T{(R)0, (R)0};
    slab_transform_loaded<T, N, SIGN, true, 1>(cur, buf, tpre, tpost, tw, scal, u, tid);
    __syncthreads();  // buf is reused by the next slab
    T* out = dst + p1 * nn;
    const int t = tid % N2;
    const int r = tid / N2;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int k1 = t + N2 * q;
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) {
        const int k = k1 + N1 * k2;
        out[r * N + k] = cmul(u[q * N2 + k2], tpost[k]);
      }
    }
#pragma unroll
    for (int i = 0; i < N1; ++i) cur[i] = nxt[i];
  }
}


// ---------------------------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------------------------

// Columns of an axis-pass tile: 256 threads' worth (256 / N2), except at N = 256, whose strided rows
// are 512 KB or more apart, so that each row access opens its own DRAM page: 32 columns there (256 B
// per row in complex64) instead of 16. Measured at N = 256 complex64: 16 columns 65 ms, 32 columns
// 51 ms, 64 columns 54 ms for the propagation.
template <class T, int N> constexpr int axis_cols() {
  constexpr int c = N == 256 ? 32 : 256 / Split<N>::N2;
  return c < N ? c : N;
}
template <int N> constexpr int row_batch() {
  constexpr int b = 256 / Split<N>::N2;
  return b < N * N * N ? b : N * N * N;
}

// One or two strided-axis blocks in one launch (see AxisRange); `b` may be null.
template <class T, int N>
static bool make_job(const AxisRange& ar, const Chirp& pre, const Chirp& post, AxisJob* j) {
  constexpr int C = axis_cols<T, N>();
  if (ar.ncols % C != 0 || ar.ncols <= 0 || ar.outer_count <= 0) return false;
  j->outer_stride = ar.outer_stride;
  j->axis_stride = ar.axis_stride;
  j->inner_offset = ar.inner_offset;
  j->tiles_per_outer = ar.ncols / C;
  j->blocks = ar.outer_count * j->tiles_per_outer;
  j->pre = pre;
  j->post = post;
  return true;
}

template <class T, int N, int SIGN>
static hipError_t launch_axis_n(const T* src, T* dst, const AxisRange& a, const Chirp& pre_a, const Chirp& post_a,
                                const AxisRange* b, const Chirp& pre_b, const Chirp& post_b, bool nt_loads,
                                hipStream_t st) {
  constexpr int C = axis_cols<T, N>();
  AxisJob ja{}, jb{};
  if (!make_job<T, N>(a, pre_a, post_a, &ja)) return hipErrorInvalidValue;
  if (b != nullptr && !make_job<T, N>(*b, pre_b, post_b, &jb)) return hipErrorInvalidValue;
  const long long blocks = ja.blocks + jb.blocks;
  if (blocks > 0x7fffffffll) return hipErrorInvalidValue;
  if (nt_loads)
    hipLaunchKernelGGL((k_axis_fft<T, N, C, SIGN, true>), dim3((unsigned)blocks), dim3(Split<N>::N2 * C), 0, st, src,
                       dst, ja, jb);
  else
    hipLaunchKernelGGL((k_axis_fft<T, N, C, SIGN>), dim3((unsigned)blocks), dim3(Split<N>::N2 * C), 0, st, src, dst,
                       ja, jb);
  return hipGetLastError();
}

template <class T, int N, int SIGN>
static hipError_t launch_row_n(const T* src, T* dst, long long rows, const Chirp& pre, const Chirp& post,
                               const SourceParams* gen, long long row0, hipStream_t st) {
  constexpr int B = row_batch<N>();
  if (rows % B != 0) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(rows / B)), block(Split<N>::N2 * B);
  if (gen) {
    if constexpr (B <= N) {
      if (row0 % B != 0) return hipErrorInvalidValue;
      if (gen->geometry == 0)
        hipLaunchKernelGGL((k_row_fft<T, N, B, SIGN, 1>), grid, block, 0, st, dst, dst, pre, post, row0, *gen);
      else
        hipLaunchKernelGGL((k_row_fft<T, N, B, SIGN, 2>), grid, block, 0, st, dst, dst, pre, post, row0, *gen);
    } else {
      return hipErrorInvalidValue;
    }
  } else {
    hipLaunchKernelGGL((k_row_fft<T, N, B, SIGN, 0>), grid, block, 0, st, src, dst, pre, post, 0ll, SourceParams{});
  }
  return hipGetLastError();
}

// Workgroups of the persistent slab pass: as many as fit on the 256 CUs at once (LDS and waves).
template <class T, int N> constexpr long long slab_resident_wgs() {
  constexpr long long by_lds = (long long)(kMaxLds / slab_lds_bytes<T, N>());
  constexpr long long by_waves = 32 / ((Split<N>::N2 * N + 63) / 64);
  constexpr long long k = by_lds < by_waves ? by_lds : by_waves;
  return 256 * (k < 1 ? 1 : k);
}

template <class T, int N, int SIGN>
static hipError_t launch_slab_n(const T* src, T* dst, long long slab0, long long slabs, const Chirp& pre,
                                const Chirp& post, const Chirp& slab_pre, const Pupil& pu, int mode,
                                const SourceParams* gen, bool nt_loads, hipStream_t st) {
  if (slabs <= 0 || slabs > 0x7fffffffll || slab0 < 0 || slab0 + slabs > (long long)N * N) return hipErrorInvalidValue;
  if (mode == 3) {
    if constexpr (N >= 32 && N <= 128 && half_lds_bytes<T, N>() <= kMaxLds) {
      const dim3 grid((unsigned)slabs), block(Split<N>::N2 * N / 2);
      if (gen && gen->geometry == 0 && gen->lens_alpha == 0.0)
        hipLaunchKernelGGL((k_slab_half<T, N, SIGN, 1>), grid, block, 0, st, dst, dst, pre, post, slab_pre, pu, *gen,
                           slab0);
      else if (gen)
        hipLaunchKernelGGL((k_slab_half<T, N, SIGN, 2>), grid, block, 0, st, dst, dst, pre, post, slab_pre, pu, *gen,
                           slab0);
      else if (nt_loads && sizeof(T) == 8)
        hipLaunchKernelGGL((k_slab_half<T, N, SIGN, 0, true>), grid, block, 0, st, src, dst, pre, post, slab_pre, pu,
                           SourceParams{}, slab0);
      else
        hipLaunchKernelGGL((k_slab_half<T, N, SIGN, 0>), grid, block, 0, st, src, dst, pre, post, slab_pre, pu,
                           SourceParams{}, slab0);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  if (gen) return hipErrorInvalidValue;  // only the half-buffer pass generates its input
  if constexpr (slab_lds_bytes<T, N>() > kMaxLds) {
    return hipErrorInvalidValue;
  } else {
    if (mode == 2) {
      const long long g = slabs < slab_resident_wgs<T, N>() ? slabs : slab_resident_wgs<T, N>();
      hipLaunchKernelGGL((k_slab_fft2p<T, N, SIGN>), dim3((unsigned)g), dim3(Split<N>::N2 * N), 0, st, src, dst,
                         slab0, slab0 + slabs, pre, post, slab_pre, pu);
    } else {
      hipLaunchKernelGGL((k_slab_fft2<T, N, SIGN>), dim3((unsigned)slabs), dim3(Split<N>::N2 * N), 0, st, src, dst,
                         pre, post, slab_pre, pu, slab0);
    }
    return hipGetLastError();
  }
}

#define WOLF_DISPATCH_N(n, CALL)                   \
  switch (n) {                                     \
    case 2: { constexpr int NN = 2; return CALL; }     \
    case 4: { constexpr int NN = 4; return CALL; }     \
    case 8: { constexpr int NN = 8; return CALL; }     \
    case 16: { constexpr int NN = 16; return CALL; }   \
    case 32: { constexpr int NN = 32; return CALL; }   \
    case 64: { constexpr int NN = 64; return CALL; }   \
    case 128: { constexpr int NN = 128; return CALL; } \
    case 256: { constexpr int NN = 256; return CALL; } \
    default: return hipErrorInvalidValue;          \
  }

template <class T>
hipError_t launch_axis_range(int n, const T* src, T* dst, int sign, const AxisRange& a, const Chirp& pre_a,
                             const Chirp& post_a, const AxisRange* b, const Chirp& pre_b, const Chirp& post_b,
                             hipStream_t st, bool nt_loads = sizeof(T) == 16) {
  if (sign < 0) {
    WOLF_DISPATCH_N(n, (launch_axis_n<T, NN, -1>(src, dst, a, pre_a, post_a, b, pre_b, post_b, nt_loads, st)))
  }
  WOLF_DISPATCH_N(n, (launch_axis_n<T, NN, +1>(src, dst, a, pre_a, post_a, b, pre_b, post_b, nt_loads, st)))
}

template <class T>
hipError_t launch_row_pass(int n, const T* src, T* dst, long long rows, int sign, const Chirp& pre,
                           const Chirp& post, hipStream_t st, const SourceParams* gen = nullptr, long long row0 = 0) {
  if (sign < 0) { WOLF_DISPATCH_N(n, (launch_row_n<T, NN, -1>(src, dst, rows, pre, post, gen, row0, st))) }
  WOLF_DISPATCH_N(n, (launch_row_n<T, NN, +1>(src, dst, rows, pre, post, gen, row0, st)))
}

template <class T>
hipError_t launch_slab_pass(int n, const T* src, T* dst, long long slab0, long long slabs, int sign, const Chirp& pre,
                            const Chirp& post, const Chirp& slab_pre, const Pupil& pu, int mode, const SourceParams* gen,
                            hipStream_t st, bool nt_loads = false) {
  if (sign < 0) {
    WOLF_DISPATCH_N(n, (launch_slab_n<T, NN, -1>(src, dst, slab0, slabs, pre, post, slab_pre, pu, mode, gen, nt_loads,
                                                 st)))
  }
  WOLF_DISPATCH_N(n, (launch_slab_n<T, NN, +1>(src, dst, slab0, slabs, pre, post, slab_pre, pu, mode, gen, nt_loads,
                                               st)))
}

// Plain 2D DFTs of `count` N x N arrays in place (no chirps, no centring):
//   X[m1][m2] = sum_{i, p} e^{SIGN 2 pi i (m1 i + m2 p) / N} x[i][p],
// a row pass over p, then an axis pass over i (stride N). count N must be whole row-pass workgroups.
bool dft2_batch_ok(int n, long long count) {
  return n >= 2 && n <= 256 && (n & (n - 1)) == 0 && count > 0 && (count * n) % row_pass_rows(n) == 0;
}

template <class T>
hipError_t launch_dft2_batch(int n, T* data, long long count, int sign, hipStream_t st) {
  if (!dft2_batch_ok(n, count)) return hipErrorInvalidValue;
  const Chirp ident{0.0, 1.0, +1, 0};
  hipError_t e = launch_row_pass<T>(n, data, data, count * n, sign, ident, ident, st);
  if (e != hipSuccess) return e;
  const AxisRange ar{count, (long long)n * n, n, 0, n};
  return launch_axis_range<T>(n, data, data, sign, ar, ident, ident, nullptr, ident, ident, st);
}
template hipError_t launch_dft2_batch<float2>(int, float2*, long long, int, hipStream_t);
template hipError_t launch_dft2_batch<double2>(int, double2*, long long, int, hipStream_t);

template <class T>
__global__ __launch_bounds__(256) void k_apply_pupil(const T* in, T* out, int n, Pupil pu) {
  using R = typename real_of<T>::type;
  const long long nn = (long long)n * n, total = nn * nn;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long p1 = e / nn, p2 = e - p1 * nn;
    const bool keep = pupil_pass(pu, (int)(p1 / n), (int)(p1 % n), n) && pupil_pass(pu, (int)(p2 / n), (int)(p2 % n), n);
    out[e] = keep ? in[e] : T{(R)0, (R)0};
  }
}

template <class T>
hipError_t launch_apply_pupil(int n, const T* in, T* out, const Pupil& pu, hipStream_t st) {
  const long long total = (long long)n * n * n * n;
  long long blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_apply_pupil<T>, dim3((unsigned)blocks), dim3(256), 0, st, in, out, n, pu);
  return hipGetLastError();
}
template hipError_t launch_apply_pupil<float2>(int, const float2*, float2*, const Pupil&, hipStream_t);
template hipError_t launch_apply_pupil<double2>(int, const double2*, double2*, const Pupil&, hipStream_t);

template <class T> bool slab_pass_supported(int n) {
  switch (n) {
    case 2: return slab_lds_bytes<T, 2>() <= kMaxLds;
    case 4: return slab_lds_bytes<T, 4>() <= kMaxLds;
    case 8: return slab_lds_bytes<T, 8>() <= kMaxLds;
    case 16: return slab_lds_bytes<T, 16>() <= kMaxLds;
    case 32: return slab_lds_bytes<T, 32>() <= kMaxLds;
    case 64: return slab_lds_bytes<T, 64>() <= kMaxLds;
    case 128: return slab_lds_bytes<T, 128>() <= kMaxLds;
    case 256: return slab_lds_bytes<T, 256>() <= kMaxLds;
    default: return false;
  }
}

template <class T> bool gen_source_supported(int n, const SourceParams& sp, int fused_slab) {
  if ((sp.model != 0 && sp.model != 2) || sp.geometry < 0 || sp.geometry > 3) return false;
  if (fused_slab == 3) return half_slab_supported<T>(n);
  return fused_slab == 0 && n >= 64 && n <= 256;  // the row pass: a workgroup's rows lie in one slab
}
template bool gen_source_supported<float2>(int, const SourceParams&, int);
template bool gen_source_supported<double2>(int, const SourceParams&, int);

template <class T> bool half_slab_supported(int n) {
  switch (n) {
    case 32: return half_lds_bytes<T, 32>() <= kMaxLds;
    case 64: return half_lds_bytes<T, 64>() <= kMaxLds;
    case 128: return half_lds_bytes<T, 128>() <= kMaxLds;
    default: return false;
  }
}
template bool half_slab_supported<float2>(int);
template bool half_slab_supported<double2>(int);

int row_pass_rows(int n) {
  switch (n) {
    case 2: return row_batch<2>();
    case 4: return row_batch<4>();
    case 8: return row_batch<8>();
    case 16: return row_batch<16>();
    case 32: return row_batch<32>();
    case 64: return row_batch<64>();
    case 128: return row_batch<128>();
    case 256: return row_batch<256>();
    default: return 1;
  }
}

template <class T> static int axis_tile_cols_t(int n) {
  switch (n) {
    case 2: return axis_cols<T, 2>();
    case 4: return axis_cols<T, 4>();
    case 8: return axis_cols<T, 8>();
    case 16: return axis_cols<T, 16>();
    case 32: return axis_cols<T, 32>();
    case 64: return axis_cols<T, 64>();
    case 128: return axis_cols<T, 128>();
    case 256: return axis_cols<T, 256>();
    default: return 1;
  }
}
int axis_tile_cols(int n, int elem_bytes) {
  return elem_bytes == 8 ? axis_tile_cols_t<float2>(n) : axis_tile_cols_t<double2>(n);
}

// ---------------------------------------------------------------------------------------------
// The operator: a schedule of passes (see Plan).
// ---------------------------------------------------------------------------------------------
template <class T>
hipError_t launch_operator(int n, const T* in, T* out, const OperatorTables& op, const Plan& plan, void* counters,
                           hipStream_t st, const SourceParams* gen) {
  const long long N = n, NN = N * N, NNN = NN * N;
  hipError_t e;
  const Chirp ident{0.0, 1.0, +1, 0};
  // A formed source: the half-buffer slab pass or the row pass (N >= 64), with no input pupil.
  if (gen && (op.pupil.geo != 0 || !(plan.fused_slab == 3 || (plan.fused_slab == 0 && n >= 64))))
    return hipErrorInvalidValue;
  // An input pupil is applied while the slab pass loads; the other schedules apply it first.
  if (op.pupil.geo != 0 && !plan.fused_slab) {
    e = launch_apply_pupil<T>(n, in, out, op.pupil, st);
    if (e != hipSuccess) return e;
    in = out;
  }
  const Chirp pre1 = plan.fused_slab ? ident : op.pre1;
  Chirp post_last = op.post1;
  post_last.scale = op.scale;
  // Grouped schedule (in place, or a formed source): the slab pass over a group of whole i1 planes
  // (slab_chunk slabs), then at once the j1 pass of those planes, while they are still in the 256 MB
  // memory-side cache; the i1 pass follows in one launch. Out of place the paired column chunks below
  // measured faster, so an out-of-place call with a grouped plan takes them.
  if (plan.fused_slab && !plan.coop && plan.slab_chunk > 0 && plan.slab_chunk < NN && (in == out || gen)) {
    const long long g = plan.slab_chunk;
    if (g % N != 0) return hipErrorInvalidValue;
    for (long long s0 = 0; s0 < NN; s0 += g) {
      // Nontemporal input loads in complex64: 2.33 ms against 2.37 ms in place at N = 128 (complex128: slower).
      e = launch_slab_pass<T>(n, in, out, s0, g, op.sign2, op.pre2, op.post2, op.pre1, op.pupil, plan.fused_slab, gen,
                              st, sizeof(T) == 8);
      if (e != hipSuccess) return e;
      const AxisRange aj{g / N, NNN, NN, 0, NN};  // j1 of the group's planes: outer i1, stride N^2
      e = launch_axis_range<T>(n, out + s0 * NN, out + s0 * NN, op.sign1, aj, pre1, op.post1, nullptr, ident, ident,
                               st);
      if (e != hipSuccess) return e;
    }
    const AxisRange ai{N, NN, NNN, 0, NN};  // i1 over all columns: outer j1, stride N^3
    return launch_axis_range<T>(n, out, out, op.sign1, ai, pre1, post_last, nullptr, ident, ident, st, true);
  }
  // Second-point axes (i2, j2).
  if (plan.fused_slab) {
    e = launch_slab_pass<T>(n, in, out, 0, NN, op.sign2, op.pre2, op.post2, op.pre1, op.pupil, plan.fused_slab, gen,
                            st);
    if (e != hipSuccess) return e;
  } else {
    const long long g = plan.slab_chunk > 0 ? plan.slab_chunk : NN;  // slabs per chunk
    // In place, chunks of whole i1 planes also take their j1 pass at once (as the grouped slab-pass
    // schedule), while the chunk is still in the memory-side cache; the i1 pass then runs alone.
    const bool grouped_j1 = !plan.coop && (in == out || gen) && g < NN && g % N == 0;
    for (long long s0 = 0; s0 < NN; s0 += g) {
      const long long gs = (s0 + g <= NN) ? g : NN - s0;
      e = launch_row_pass<T>(n, gen ? out + s0 * NN : in + s0 * NN, out + s0 * NN, gs * N, op.sign2, op.pre2, op.post2,
                             st, gen, s0 * N);
      if (e != hipSuccess) return e;
      const AxisRange ar{gs, NN, N, 0, N};  // axis i2 inside each slab of the chunk
      e = launch_axis_range<T>(n, out + s0 * NN, out + s0 * NN, op.sign2, ar, op.pre2, op.post2, nullptr, ident,
                               ident, st);
      if (e != hipSuccess) return e;
      if (grouped_j1) {
        const AxisRange aj{gs / N, NNN, NN, 0, NN};  // j1 of the chunk's planes: outer i1, stride N^2
        e = launch_axis_range<T>(n, out + s0 * NN, out + s0 * NN, op.sign1, aj, op.pre1, op.post1, nullptr, ident,
                                 ident, st);
        if (e != hipSuccess) return e;
      }
    }
    if (grouped_j1) {
      const AxisRange ai{N, NN, NNN, 0, NN};  // i1 over all columns: outer j1, stride N^3
      return launch_axis_range<T>(n, out, out, op.sign1, ai, op.pre1, post_last, nullptr, ident, ident, st, true);
    }
  }
  if (plan.coop) return launch_first_point_coop<T>(n, out, op, pre1, plan.coop_cols, plan.coop_lookahead, counters, st);
  // First-point axes (j1, i1) over column chunks of the N^2 columns m2. The i1 pass of chunk k - 1
  // shares a launch with the j1 pass of chunk k: they touch disjoint columns.
  const long long m = plan.col_chunk > 0 ? plan.col_chunk : NN;
  const long long chunks = (NN + m - 1) / m;
  for (long long k = 0; k <= chunks; ++k) {
    const bool has_j = k < chunks, has_i = k > 0;
    const long long cj = k * m, ci = (k - 1) * m;
    const AxisRange aj{N, NNN, NN, cj, has_j ? ((cj + m <= NN) ? m : NN - cj) : 0};  // j1: outer i1, stride N^2
    const AxisRange ai{N, NN, NNN, ci, has_i ? ((ci + m <= NN) ? m : NN - ci) : 0};  // i1: outer j1, stride N^3
    if (has_j && has_i)
      e = launch_axis_range<T>(n, out, out, op.sign1, aj, pre1, op.post1, &ai, pre1, post_last, st);
    else if (has_j)
      e = launch_axis_range<T>(n, out, out, op.sign1, aj, pre1, op.post1, nullptr, ident, ident, st);
    else
      e = launch_axis_range<T>(n, out, out, op.sign1, ai, pre1, post_last, nullptr, ident, ident, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------------------------
// Operator applied to a diagonal input diag(g) (e.g. the gradient of a loss of S = Re diag W).
// The second-point 2D DFT of row m1 = (a, b) of diag(g) is a plane wave:
//   Y[m1; (p, q)] = g(m1) pre1[a] pre1[b] pre2[a] pre2[b] w^{a p} w^{b q} post2[p] post2[q],
// with w = e^{sign2 2 pi i / N}. A write-only kernel makes it without reading an N^4 input.
// ---------------------------------------------------------------------------------------------
template <class T, int SIGN>
__global__ __launch_bounds__(256) void k_slab_from_diag(const typename real_of<T>::type* __restrict__ g, T* dst, int n,
                                                        Chirp pre1, Chirp pre2, Chirp post2) {
  __shared__ T tp[256], tw[256];
  __shared__ T sc[1];
  const long long m1 = blockIdx.x;
  const int a = (int)(m1 / n), b = (int)(m1 % n);
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    tp[i] = chirp_entry<T>(post2, i, n);
    tw[i] = twiddle_entry<T, SIGN>(i, n);
  }
  if (threadIdx.x == 0) {
    using R = typename real_of<T>::type;
    const T f = cmul(cmul(chirp_entry<T>(pre1, a, n), chirp_entry<T>(pre1, b, n)),
                     cmul(chirp_entry<T>(pre2, a, n), chirp_entry<T>(pre2, b, n)));
    sc[0] = cscale(f, (R)g[m1]);
  }
  __syncthreads();
  const T s = sc[0];
  const long long nn = (long long)n * n;
  T* out = dst + m1 * nn;
  for (long long e = threadIdx.x; e < nn; e += blockDim.x) {
    const int p = (int)(e / n), q = (int)(e % n);
    const T row = cmul(tw[(a * p) & (n - 1)], tp[p]);
    const T col = cmul(tw[(b * q) & (n - 1)], tp[q]);
    out[e] = cmul(s, cmul(row, col));
  }
}

template <class T>
hipError_t launch_operator_diag(int n, const typename real_of<T>::type* g, T* out, const OperatorTables& op,
                                const Plan& plan, void* counters, hipStream_t st) {
  const long long N = n, NN = N * N, NNN = NN * N;
  const Chirp ident{0.0, 1.0, +1, 0};
  if (op.sign2 < 0)
    hipLaunchKernelGGL((k_slab_from_diag<T, -1>), dim3((unsigned)NN), dim3(256), 0, st, g, out, n, op.pre1, op.pre2,
                       op.post2);
  else
    hipLaunchKernelGGL((k_slab_from_diag<T, +1>), dim3((unsigned)NN), dim3(256), 0, st, g, out, n, op.pre1, op.pre2,
                       op.post2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (plan.coop) return launch_first_point_coop<T>(n, out, op, ident, plan.coop_cols, plan.coop_lookahead, counters, st);
  const long long m = plan.col_chunk > 0 ? plan.col_chunk : NN;
  Chirp post_last = op.post1;
  post_last.scale = op.scale;
  const long long chunks = (NN + m - 1) / m;
  for (long long k = 0; k <= chunks; ++k) {
    const bool has_j = k < chunks, has_i = k > 0;
    const long long cj = k * m, ci = (k - 1) * m;
    const AxisRange aj{N, NNN, NN, cj, has_j ? ((cj + m <= NN) ? m : NN - cj) : 0};
    const AxisRange ai{N, NN, NNN, ci, has_i ? ((ci + m <= NN) ? m : NN - ci) : 0};
    if (has_j && has_i)
      e = launch_axis_range<T>(n, out, out, op.sign1, aj, ident, op.post1, &ai, ident, post_last, st);
    else if (has_j)
      e = launch_axis_range<T>(n, out, out, op.sign1, aj, ident, op.post1, nullptr, ident, ident, st);
    else
      e = launch_axis_range<T>(n, out, out, op.sign1, ai, ident, post_last, nullptr, ident, ident, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template hipError_t launch_operator_diag<float2>(int, const float*, float2*, const OperatorTables&, const Plan&, void*,
                                                 hipStream_t);
template hipError_t launch_operator_diag<double2>(int, const double*, double2*, const OperatorTables&, const Plan&,
                                                  void*, hipStream_t);

template hipError_t launch_operator<float2>(int, const float2*, float2*, const OperatorTables&, const Plan&, void*,
                                            hipStream_t, const SourceParams*);
template hipError_t launch_operator<double2>(int, const double2*, double2*, const OperatorTables&, const Plan&, void*,
                                             hipStream_t, const SourceParams*);
template bool slab_pass_supported<float2>(int);
template bool slab_pass_supported<double2>(int);

}  // namespace wolf
