// The propagation operator for any even N and any transform length N_z >= N: zero padding of
// the N-point axes to N_z points and cropping back to N (Sec. 3.3), and N that are not powers of two.
//
// Along one axis the operator is
//   y[k] = post[k] sum_n e^{SIGN 2 pi i (k - N/2)(n - N/2) / N_z} pre[n] x[n],   k, n in [0, N),
// the N central outputs of the centred N_z-point DFT of the N inputs embedded in N_z - N zeros. The
// index (k - N/2)(n - N/2) mod N_z is exact in integers, and the table of the N_z roots of unity is
// built in FP64. There is no FFT here: each axis is a dense product of the N x N matrix (generated
// from the table, never stored) with the N-point lines of the array, tiled like a GEMM (64 x 64
// outputs per tile on the matrix cores in the 3M form, 16 inputs per LDS stage) on a persistent grid
// that builds the tables once per workgroup. The four axes run as four passes that alternate between the
// output and a work buffer.
//   COLS: a strided axis (stride S); the lines of one batch o are S contiguous columns:
//         out[o N S + k S + c] from in[o N S + n S + c], tiles of 64 k x 64 c.
//   !COLS: the contiguous axis: out[r N + k] from in[r N + n], tiles of 64 r x 64 k.
#include "wolf_device.hpp"
#include "wolf_internal.hpp"
#include "wolf_mfma.hpp"

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
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 4 : 2))) void k_dense_axis(
    const T* __restrict__ in, T* __restrict__ out, DenseAxis d, Chirp pre, Chirp post, double scale) {
  using R = typename real_of<T>::type;
  using G = MTile<64>;
  constexpr int TM = 64, TN = 64, TK = 16;
  __shared__ T tw[kDenseMaxNz];
  __shared__ T tpre[kDenseMaxN], tpost[kDenseMaxN];
  __shared__ R ar[TK][G::LDA], ai[TK][G::LDA], br[TK][G::LDB], bi[TK][G::LDB];
  const int tid = threadIdx.x, lane = tid % 64;
  const int wv = __builtin_amdgcn_readfirstlane(tid / 64);  // wavefront-uniform
  const int row0 = (wv / G::WC) * 32, col0 = (wv % G::WC) * 32;
  const int n = d.n, nz = d.nz, c0 = n / 2;
  for (int i = tid; i < nz; i += 256) tw[i] = twiddle_entry<T, SIGN>(i, nz);
  for (int i = tid; i < n; i += 256) {
    tpre[i] = chirp_entry<T>(pre, i, n);
    tpost[i] = chirp_entry<T>(post, i, n);
  }
  __syncthreads();
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
    CTile<T> acc;
    ctile_zero(acc);
    for (int n0 = 0; n0 < n; n0 += TK) {
      T raw[4];  // this thread's four elements of the array tile, all loads issued first
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = tid + 256 * q;
        if constexpr (COLS) {
          const int kk = e / TN, jj = e % TN;
          const long long gc = j0 + jj;
          const int gn = n0 + kk;
          raw[q] = load_or_first(in, gc < d.S && gn < n, base + (long long)gn * d.S + gc);
        } else {
          const int ii = e / TK, kk = e % TK;
          const long long gi = i0 + ii;
          const int gn = n0 + kk;
          raw[q] = load_or_first(in, gi < d.rows && gn < n, gi * n + gn);
        }
      }
      // A (TM x TK): the DFT matrix (COLS) or the pre-multiplied lines (!COLS); B (TK x TN): the
      // pre-multiplied columns (COLS) or the DFT matrix (!COLS). Staged as re / im planes.
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
          const T x = cmul(raw[q], tpre[gn < n ? gn : 0]);
          v = keep_or_zero(gi < d.rows && gn < n, x);
        }
        ar[kk][ii] = v.x;
        ai[kk][ii] = v.y;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = tid + 256 * q;
        T v = zero;
        int kk, jj;
        if constexpr (COLS) {
          kk = e / TN;
          jj = e % TN;
          const long long gc = j0 + jj;
          const int gn = n0 + kk;
          const T x = cmul(raw[q], tpre[gn < n ? gn : 0]);
          v = keep_or_zero(gc < d.S && gn < n, x);
        } else {
          jj = e / TK;
          kk = e % TK;
          const long long gk = j0 + jj;
          const int gn = n0 + kk;
          if (gk < n && gn < n) v = tw[dense_index((int)gk, gn, c0, nz)];
        }
        br[kk][jj] = v.x;
        bi[kk][jj] = v.y;
      }
      __syncthreads();
      ctile_mfma16<T, G::LDA, G::LDB>(acc, ar, ai, br, bi, row0, col0, lane);
      __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const long long gi = i0 + row0 + 16 * r + Mfma<T>::row(lane, i), gj = j0 + col0 + 16 * q + lane % 16;
          const T a{acc.re(r, q, i), acc.im(r, q, i)};
          if constexpr (COLS) {
            if (gi < n && gj < d.S) {
              const T v = cmul(a, tpost[gi]);
              out[base + gi * d.S + gj] = T{(R)(scale * v.x), (R)(scale * v.y)};
            }
          } else {
            if (gi < d.rows && gj < n) {
              const T v = cmul(a, tpost[gj]);
              out[gi * n + gj] = T{(R)(scale * v.x), (R)(scale * v.y)};
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

// ---------------------------------------------------------------------------------------------
// The same operator with a zero-padded FFT when N_z is a power of two (<= 1024). Per line, the N
// inputs sit at positions n + s (s = (N_z - N)/2) of an N_z-point transform, the rest are zeros,
// and the outputs at positions k + s are kept. With the centring factors on the padded indices,
//   e^{SIGN 2 pi i (k - N/2)(n - N/2)/N_z} = e^{SIGN 2 pi i k' n'/N_z} (-1)^{k'} (-1)^{n'} (-1)^{N_z/2},
// k' = k + s, n' = n + s; (-1)^{n'} (-1)^{k'} = (-1)^{n + k}, which the checkerboarded chirps on the
// N-point grids carry, and (-1)^{N_z/2} cancels over the four axes. The transform is the split
// N_z = N1 N2 of the slab and axis passes. A workgroup owns C lines (one LDS exchange) and loops
// over tiles of lines; it reads its lines before a barrier and writes them after, so dst may be src.
// ---------------------------------------------------------------------------------------------
// Lines of one pass: `outer` blocks (stride outer_stride) of ncols lines each (stride col_stride);
// the transformed axis has stride axis_stride. tiles_per_outer and tiles are filled at launch.
struct PadJob {
  long long outer, outer_stride, axis_stride, col_stride, ncols;
  int n, s;
  Chirp pre, post;
  long long tiles_per_outer, tiles;
};

// Split of an N_z-point line transform over L2 threads that hold L1 = Q L2 elements each
// (N_z = Q L2^2), and the C lines of a workgroup (L2 C <= 256 threads, at most one wavefront per
// SIMD). Powers of two take the split of the slab and axis passes and C = 256 / L2. Other lengths
// take the largest L2 with L1 <= 32 (the register DFTs); C is a multiple of 16 lines in complex64
// (16 max(1, floor(16 / L2))) and of 8 lines in complex128 (8 floor(32 / L2)), so that a tile of
// neighbouring lines spans whole 128-byte memory lines (tiles that split lines between workgroups,
// which run on different XCDs, took 27 ms instead of 23 ms at N = 200 in complex64).
__host__ __device__ constexpr int line_l2(int lz) {
  if (is_pow2(lz)) return lz >> ((ilog2(lz) + 1) / 2);  // Split<lz>::N2
  for (int l2 = 32; l2 >= 1; --l2)
    if (lz % (l2 * l2) == 0 && (lz / (l2 * l2)) * l2 <= 32) return l2;
  return 0;
}
__host__ __device__ constexpr int line_cols(int l2, int elem_bytes) {
  return elem_bytes == 8 ? 16 * (16 / l2 > 1 ? 16 / l2 : 1) : 8 * (32 / l2);
}
template <class T, int NZ> struct LineCfg {
  static constexpr int L2 = line_l2(NZ);
  static constexpr int L1 = NZ / L2;
  static constexpr int Q = L1 / L2;
  static constexpr int C = is_pow2(NZ) ? 256 / L2 : line_cols(L2, (int)sizeof(T));
  static constexpr int kThreads = L2 * C;
  static_assert(L2 >= 1 && L1 == Q * L2 && L1 <= 32 && kThreads <= 256, "line split");
};

// Lane layout and exchange buffer of a pass. The exchange runs in Q / G phases: in phase p the
// buffer holds the first-stage outputs k1 in [p G N2, (p + 1) G N2) of the C lines, G N2 x N2 x C
// entries. G = Q is one exchange; G = 1 takes a factor Q less LDS (more workgroups per CU) for
// Q - 1 more barriers and registers that hold the inputs across the phases.
//   !CONTIG (a strided axis; neighbouring lines are contiguous): lanes run across the C lines,
//           c = tid % C; entry (k1l, n2, c) at k1l (N2 C + C) + n2 C + c.
//   CONTIG (the contiguous axis): lanes run along the line, t = tid % N2, so each load and store
//           covers whole lines of memory; entry at c G N2 (N2 + 1) + k1l (N2 + 1) + n2.
// The paddings (C entries per k1l, one per N2) keep the writes and the reads of a phase free of
// bank conflicts beyond the two passes that 64 eight-byte accesses need.
template <class T, int NZ, bool CONTIG, int G, int CC = LineCfg<T, NZ>::C> struct PadLayout {
  static constexpr int N2 = LineCfg<T, NZ>::L2;
  static constexpr int C = CC;
  static constexpr int kSize = CONTIG ? C * G * N2 * (N2 + 1) : G * N2 * (N2 * C + C);
  static __device__ __forceinline__ int at(int k1l, int n2, int c) {
    return CONTIG ? c * (G * N2 * (N2 + 1)) + k1l * (N2 + 1) + n2 : k1l * (N2 * C + C) + n2 * C + c;
  }
};

template <class T, int NZ, int G> constexpr size_t pad_lds_bytes() {
  return (PadLayout<T, NZ, false, G>::kSize + 2 * kDenseMaxN + NZ) * sizeof(T);
}

// One exchange unless phases let more workgroups share a CU and the inputs are few enough (L1 <= 16)
// to stay in registers across the phases; with complex64 the single exchange already fits as many
// workgroups as the registers allow (measured register counts of the unrolled kernels).
template <class T, int NZ> constexpr int pad_groups() {
  using S = LineCfg<T, NZ>;
  constexpr bool phases_fit_more = kMaxLds / pad_lds_bytes<T, NZ, S::Q>() < kMaxLds / pad_lds_bytes<T, NZ, 1>();
  return (sizeof(T) == 16 && S::L1 <= 16 && phases_fit_more) ? 1 : S::Q;
}

// Tiles of a pass in XCD order. The hardware deals consecutive workgroups to the 8 XCDs in turn, and with
// the plain grid-stride order neighbouring tiles ran on different XCDs: where a line's rows are not
// 128-byte aligned (N = 200: 1600 B), two neighbouring tiles share the cache lines at their boundary, and
// each XCD fetched those lines again. Here XCD x takes a contiguous share of the tiles, in proportion to
// its workgroups (b < G with b mod 8 = x), and its workgroups stride through that share, so neighbouring
// tiles run at the same time on one XCD and meet in its L2. A partition of [0, tiles) for any grid size.
struct TileRange {
  long long first, end, step;
};
__device__ __forceinline__ TileRange xcd_tiles(long long tiles) {
  const long long G = gridDim.x, x = blockIdx.x % 8, r = G % 8;
  const long long below = (G / 8) * x + (r < x ? r : x);             // workgroups on XCDs 0 .. x-1
  const long long upto = (G / 8) * (x + 1) + (r < x + 1 ? r : x + 1);  // ... on XCDs 0 .. x
  return TileRange{tiles * below / G + blockIdx.x / 8, tiles * upto / G, upto - below};
}

template <class T, int NZ, int SIGN, bool CONTIG>
__global__ __launch_bounds__((LineCfg<T, NZ>::kThreads)) void k_axis_pad(const T* src, T* dst, PadJob j) {
  using S = LineCfg<T, NZ>;
  constexpr int N1 = S::L1, N2 = S::L2, Q = S::Q, C = S::C, NT = S::kThreads, G = pad_groups<T, NZ>();
  using L = PadLayout<T, NZ, CONTIG, G>;
  __shared__ T xch[L::kSize];
  __shared__ T tpre[kDenseMaxN], tpost[kDenseMaxN], tw[NZ];
  const int n = j.n, sft = j.s;
  for (int i = threadIdx.x; i < n; i += NT) {
    tpre[i] = chirp_entry<T>(j.pre, i, n);
    tpost[i] = chirp_entry<T>(j.post, i, n);
  }
  for (int i = threadIdx.x; i < NZ; i += NT) tw[i] = twiddle_entry<T, SIGN>(i, NZ);
  __syncthreads();
  const int t = CONTIG ? (int)threadIdx.x % N2 : (int)threadIdx.x / C;
  const int c = CONTIG ? (int)threadIdx.x / N2 : (int)threadIdx.x % C;
  // Per-element offsets m * stride (the compiler keeps them across tiles): one start and
  // wave-uniform steps took fewer registers but ran slower here (N = 200: 25.4 ms instead of 22.7 ms).
  const long long as = j.axis_stride;
  const TileRange tr = xcd_tiles(j.tiles);
  for (long long tile = tr.first; tile < tr.end; tile += tr.step) {
    const long long o = tile / j.tiles_per_outer;
    const long long col = (tile - o * j.tiles_per_outer) * C + c;
    const bool valid = col < j.ncols;
    const long long base = o * j.outer_stride + col * j.col_stride;
    T v[N1];
#pragma unroll
    for (int a = 0; a < N1; ++a) {
      const int m = N2 * a + t - sft;
      v[a] = load_or_first(src, valid && m >= 0 && m < n, base + (long long)m * as);
    }
#pragma unroll
    for (int a = 0; a < N1; ++a) {
      const int m = N2 * a + t - sft;
      const bool ok = valid && m >= 0 && m < n;
      const T x = cmul(v[a], tpre[ok ? m : 0]);
      v[a] = keep_or_zero(ok, x);
    }
    dft_any<N1, SIGN>(v);
#pragma unroll
    for (int k1 = 1; k1 < N1; ++k1) v[k1] = cmul(v[k1], tw[t * k1]);  // t k1 < N_z
    // Every load of the tile has been consumed here, so the stores below may overwrite src.
#pragma unroll
    for (int p = 0; p < Q / G; ++p) {
#pragma unroll
      for (int k1l = 0; k1l < G * N2; ++k1l) xch[L::at(k1l, t, c)] = v[p * G * N2 + k1l];
      __syncthreads();
      T u[G][N2];
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) u[g][n2] = xch[L::at(t + N2 * g, n2, c)];
      __syncthreads();  // the buffer is rewritten by the next phase or tile
#pragma unroll
      for (int g = 0; g < G; ++g) {
        dft_any<N2, SIGN>(u[g]);
        const int k1 = t + N2 * (p * G + g);
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) {
          const int m = k1 + N1 * k2 - sft;
          if (valid && m >= 0 && m < n) dst[base + (long long)m * as] = cmul(u[g][k2], tpost[m]);
        }
      }
    }
  }
}

// Padding to N_z >= 2N with N_z = 2 L2^2 (8, 32, 128, 512; L1 = 2 L2). Thread t's inputs are the rows
// a of the first stage with s <= L2 a + t < s + N: at most N / L2 <= L1 / 2 consecutive rows
// a = a0 + r, r in [0, L1/2). With z[r] = x(a0 + r) and k1 = 2 kappa + p (p = 0, 1),
//   V[k1] = sum_a x(a) e^{SIGN 2 pi i a k1 / L1}
//         = e^{SIGN 2 pi i a0 k1 / L1} sum_r [z[r] e^{SIGN 2 pi i r p / L1}] e^{SIGN 2 pi i r kappa / (L1/2)},
// two L1/2-point transforms; the factor of a0 joins the first-stage twiddle e^{SIGN 2 pi i t k1 / N_z}
// as e^{SIGN 2 pi i (t + L2 a0) k1 / N_z}. The even and the odd outputs are the two phases of the
// exchange (second-stage thread t takes k1 = 2t + p). A thread holds L1/2 inputs instead of L1, and
// its addresses are one per-lane start plus wave-uniform steps (input r at start + r L2 stride,
// output k2 at start + k2 L1 stride), so no per-element offsets stay live across tiles. The register
// budget is held to the waves per SIMD that the LDS allows. A workgroup owns C lines of 128 bytes
// across (16 in complex64, 8 in complex128, whose exchange then takes half the LDS).
template <class T, int NZ> struct FoldCfg {
  static constexpr int N2 = LineCfg<T, NZ>::L2;
  static constexpr int C = (sizeof(T) == 16 ? 128 : 256) / N2;
  static constexpr int kThreads = N2 * C;
  static constexpr size_t kLds = (PadLayout<T, NZ, false, 1, C>::kSize + 2 * kDenseMaxN + NZ) * sizeof(T);
  // Waves per SIMD: what the LDS allows, at most 5 (the 8 + 8 register DFTs of N_z = 128 need about 90
  // VGPRs; at the 80 of six waves they spill).
  static constexpr int kWaves = [] {
    const int w = (int)((kMaxLds / kLds) * (kThreads / 64) + 3) / 4;  // workgroups per CU over 4 SIMDs
    return w < 1 ? 1 : (w > 5 ? 5 : w);
  }();
};

// KW > 0 instantiates a band of N for the centred crop s = (N_z - N)/2: 4 L2 KW <= N < 4 L2 (KW + 1).
// Input row r (data indices m0 + L2 r, m0 in [0, L2) over the lanes) is then in the data on every lane
// for r < 4 KW and on none for r >= 4 KW + 4. Output k2 = L2/2 + d of phase p has data index
// 2 t + p + N/2 + 2 L2 d (t in [0, L2)): in the data on every lane for d in [-KW, KW), on none for
// d < -KW - 1 or d > KW. Those rows skip their per-lane range tests or are dropped at compile time
// (with the arithmetic that only feeds them). KW = 0 tests every row.
template <class T, int NZ, int SIGN, bool CONTIG, int KW>
__global__ __launch_bounds__((FoldCfg<T, NZ>::kThreads)) __attribute__((amdgpu_waves_per_eu(FoldCfg<T, NZ>::kWaves)))
void k_axis_pad_fold(const T* src, T* dst, PadJob j) {
  using S = LineCfg<T, NZ>;
  using F = FoldCfg<T, NZ>;
  constexpr int N1 = S::L1, N2 = S::L2, H = N1 / 2, C = F::C, NT = F::kThreads;
  static_assert(is_pow2(NZ) && S::Q == 2 && H == N2, "folded split");
  using L = PadLayout<T, NZ, CONTIG, 1, C>;
  __shared__ T xch[L::kSize];
  __shared__ T tpre[kDenseMaxN], tpost[kDenseMaxN], tw[NZ];
  const int n = j.n, sft = j.s;
  for (int i = threadIdx.x; i < n; i += NT) {
    tpre[i] = chirp_entry<T>(j.pre, i, n);
    tpost[i] = chirp_entry<T>(j.post, i, n);
  }
  for (int i = threadIdx.x; i < NZ; i += NT) tw[i] = twiddle_entry<T, SIGN>(i, NZ);
  __syncthreads();
  const int t = CONTIG ? (int)threadIdx.x % N2 : (int)threadIdx.x / C;
  const int c = CONTIG ? (int)threadIdx.x / N2 : (int)threadIdx.x % C;
  const int a0 = (sft - t + N2 - 1) / N2;  // s >= L2 > t (checked at launch): a positive numerator
  const int m0 = N2 * a0 + t - sft;        // data index of input r = 0, in [0, L2)
  const int tk = t + N2 * a0;              // first-stage twiddle factor t + L2 a0
  const long long as = j.axis_stride, in_step = (long long)N2 * as, out_step = (long long)N1 * as;
  constexpr int RA = 4 * KW, RZ = KW > 0 ? 4 * KW + 4 : H;  // rows below RA: all lanes; from RZ: none
  static_assert(KW >= 0 && RA <= H && (KW == 0 || KW < N2 / 2), "bands of N within N_z / 2");
  const TileRange tr = xcd_tiles(j.tiles);
  for (long long tile = tr.first; tile < tr.end; tile += tr.step) {
    const long long o = tile / j.tiles_per_outer;
    const long long col0 = (tile - o * j.tiles_per_outer) * C;
    const long long col = col0 + c;
    const bool valid = col < j.ncols;
    // With RA > 0, lanes of columns past the end of a ragged tile work on the tile's first column (in
    // bounds; their results are not stored), so the unconditional rows need no column test.
    const long long base = o * j.outer_stride + (RA > 0 && !valid ? col0 : col) * j.col_stride;
    const bool lane_ok = RA > 0 || valid;
    T z[H];
    {
      long long at = base + (long long)m0 * as;
#pragma unroll
      for (int r = 0; r < H; ++r, at += in_step) {
        if (r < RA)
          z[r] = src[at];
        else if (r < RZ)
          z[r] = load_or_first(src, lane_ok && m0 + N2 * r < n, at);
      }
    }
#pragma unroll
    for (int r = 0; r < H; ++r) {
      const int m = m0 + N2 * r;
      if (r < RA) {
        z[r] = cmul(z[r], tpre[m]);
      } else if (r >= RZ) {
        z[r] = T{(typename real_of<T>::type)0, (typename real_of<T>::type)0};
      } else {
        const bool ok = lane_ok && m < n;
        z[r] = keep_or_zero(ok, cmul(z[r], tpre[ok ? m : 0]));
      }
    }
    // Every load of the tile has been consumed here, so the stores below may overwrite src.
    // Output k2 of phase p: data index 2 t + p - s + L1 k2, stored where it is in the data.
    const long long at0 = base + (long long)(2 * t - sft) * as;  // output k2 = 0 of phase 0
    auto store = [&](int p, int k2, const T& val) {
      const int m = 2 * t + p - sft + N1 * k2, d = k2 - N2 / 2;
      const long long at = at0 + p * as + k2 * out_step;
      if (KW > 0 && d >= -KW && d < KW) {
        if (valid) dst[at] = cmul(val, tpost[m]);
      } else if (KW == 0 || (d >= -KW - 1 && d <= KW)) {
        if (valid && m >= 0 && m < n) dst[at] = cmul(val, tpost[m]);
      }
    };
    // Along a contiguous line the two phases fill alternate elements of the same memory lines: phase 0's
    // outputs wait in registers and both phases store together, so that no line leaves the L2 half written.
    // Where the registers allow it (N_z <= 128; at N_z = 512 the complex64 bands KW = 1 .. 3; elsewhere they
    // spill).
    constexpr bool kDefer = CONTIG && (NZ < 512 || (sizeof(T) == 8 && KW >= 1 && KW <= 3));
    T u0[N2];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      T v[H];
#pragma unroll
      for (int r = 0; r < H; ++r) v[r] = (p == 0 || r == 0) ? z[r] : cmul(z[r], tw[N2 * r]);
      dft_any<H, SIGN>(v);
#pragma unroll
      for (int kp = 0; kp < H; ++kp) {
        const int k1 = 2 * kp + p;
        xch[L::at(kp, t, c)] = k1 == 0 ? v[kp] : cmul(v[kp], tw[(tk * k1) & (NZ - 1)]);
      }
      __syncthreads();
      T u[N2];
#pragma unroll
      for (int n2 = 0; n2 < N2; ++n2) u[n2] = xch[L::at(t, n2, c)];
      __syncthreads();  // the buffer is rewritten by the next phase or tile
      dft_any<N2, SIGN>(u);
      if constexpr (kDefer) {
        if (p == 0) {
#pragma unroll
          for (int k2 = 0; k2 < N2; ++k2) u0[k2] = u[k2];
        } else {
#pragma unroll
          for (int k2 = 0; k2 < N2; ++k2) {
            store(0, k2, u0[k2]);
            store(1, k2, u[k2]);
          }
        }
      } else {
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) store(p, k2, u[k2]);
      }
    }
  }
}

template <class T, int NZ, bool CONTIG, int KW>
static hipError_t launch_fold_nzcb(const T* src, T* dst, const PadJob& j, int sign, unsigned grid, hipStream_t st) {
  constexpr int NT = FoldCfg<T, NZ>::kThreads;
  if (sign < 0)
    hipLaunchKernelGGL((k_axis_pad_fold<T, NZ, -1, CONTIG, KW>), dim3(grid), dim3(NT), 0, st, src, dst, j);
  else
    hipLaunchKernelGGL((k_axis_pad_fold<T, NZ, +1, CONTIG, KW>), dim3(grid), dim3(NT), 0, st, src, dst, j);
  return hipGetLastError();
}

// A centred crop with N >= 4 L2 takes the instantiated band of N, KW = N / (4 L2): at N_z = 512 (L2 = 16)
// KW = 1 .. 4 (N = 64 .. 256), at N_z = 128 (L2 = 8) KW = 1, 2 (N = 32 .. 64); other cases test every row.
template <class T, int NZ, bool CONTIG, int KW>
static hipError_t launch_fold_band(const T* src, T* dst, const PadJob& j, int sign, unsigned grid, hipStream_t st,
                                   bool& done) {
  constexpr int N2 = LineCfg<T, NZ>::L2;
  if constexpr (4 * KW <= N2) {
    if (j.n / (4 * N2) == KW) {
      done = true;
      return launch_fold_nzcb<T, NZ, CONTIG, KW>(src, dst, j, sign, grid, st);
    }
  }
  return hipSuccess;
}

template <class T, int NZ, bool CONTIG>
static hipError_t launch_fold_nzc(const T* src, T* dst, const PadJob& j, int sign, unsigned grid, hipStream_t st) {
  if constexpr (NZ == 128 || NZ == 512) {
    if (2 * j.s == NZ - j.n) {
      bool done = false;
      hipError_t e = launch_fold_band<T, NZ, CONTIG, 1>(src, dst, j, sign, grid, st, done);
      if (!done) e = launch_fold_band<T, NZ, CONTIG, 2>(src, dst, j, sign, grid, st, done);
      if (!done) e = launch_fold_band<T, NZ, CONTIG, 3>(src, dst, j, sign, grid, st, done);
      if (!done) e = launch_fold_band<T, NZ, CONTIG, 4>(src, dst, j, sign, grid, st, done);
      if (done) return e;
    }
  }
  return launch_fold_nzcb<T, NZ, CONTIG, 0>(src, dst, j, sign, grid, st);
}

template <class T, int NZ, bool CONTIG>
static hipError_t launch_pad_nzc(const T* src, T* dst, const PadJob& j, int sign, unsigned grid, hipStream_t st) {
  constexpr int NT = LineCfg<T, NZ>::kThreads;
  if (sign < 0)
    hipLaunchKernelGGL((k_axis_pad<T, NZ, -1, CONTIG>), dim3(grid), dim3(NT), 0, st, src, dst, j);
  else
    hipLaunchKernelGGL((k_axis_pad<T, NZ, +1, CONTIG>), dim3(grid), dim3(NT), 0, st, src, dst, j);
  return hipGetLastError();
}

template <class T, int NZ>
static hipError_t launch_pad_nz(const T* src, T* dst, PadJob j, int sign, hipStream_t st) {
  if constexpr (is_pow2(NZ) && NZ >= 8 && LineCfg<T, NZ>::Q == 2) {
    if (2 * j.n <= NZ) {  // then s = (N_z - N)/2 >= N_z/4 >= L2, as the folded kernel assumes
      constexpr int C = FoldCfg<T, NZ>::C;
      j.tiles_per_outer = (j.ncols + C - 1) / C;
      j.tiles = j.outer * j.tiles_per_outer;
      const long long grid = j.tiles < 4096 ? j.tiles : 4096;
      if (grid < 1) return hipSuccess;
      return j.axis_stride == 1 ? launch_fold_nzc<T, NZ, true>(src, dst, j, sign, (unsigned)grid, st)
                                : launch_fold_nzc<T, NZ, false>(src, dst, j, sign, (unsigned)grid, st);
    }
  }
  constexpr int C = LineCfg<T, NZ>::C;
  j.tiles_per_outer = (j.ncols + C - 1) / C;
  j.tiles = j.outer * j.tiles_per_outer;
  const long long grid = j.tiles < 4096 ? j.tiles : 4096;
  if (grid < 1) return hipSuccess;
  return j.axis_stride == 1 ? launch_pad_nzc<T, NZ, true>(src, dst, j, sign, (unsigned)grid, st)
                            : launch_pad_nzc<T, NZ, false>(src, dst, j, sign, (unsigned)grid, st);
}

// Transform lengths of the FFT passes besides the powers of two 2 .. 1024: even N_z = Q L2^2 with
// odd factors 3, 5, 7 and L1 = Q L2 <= 32 (N_z = 200 is the 20 x 10 split).
#define WOLF_MIXED_LINES(X) X(6) X(10) X(12) X(20) X(24) X(36) X(48) X(72) X(80) X(96) X(100) X(144) X(192) X(200)

template <class T>
static hipError_t launch_pad_axis(int nz, const T* src, T* dst, const PadJob& j, int sign, hipStream_t st) {
#define WOLF_LINE_CASE(L) \
  case L: return launch_pad_nz<T, L>(src, dst, j, sign, st);
  switch (nz) {
    WOLF_LINE_CASE(2) WOLF_LINE_CASE(4) WOLF_LINE_CASE(8) WOLF_LINE_CASE(16) WOLF_LINE_CASE(32) WOLF_LINE_CASE(64)
    WOLF_LINE_CASE(128) WOLF_LINE_CASE(256) WOLF_LINE_CASE(512) WOLF_LINE_CASE(1024)
    WOLF_MIXED_LINES(WOLF_LINE_CASE)
    default: return hipErrorInvalidValue;
  }
#undef WOLF_LINE_CASE
}

static bool line_length_supported(int nz) {
  if (nz >= 2 && nz <= 1024 && is_pow2(nz)) return true;
#define WOLF_LINE_MATCH(L) if (nz == L) return true;
  WOLF_MIXED_LINES(WOLF_LINE_MATCH)
#undef WOLF_LINE_MATCH
  return false;
}

bool pad_fft_supported(int n, int nz) {
  return n >= 2 && n <= kDenseMaxN && n % 2 == 0 && nz >= n && line_length_supported(nz);
}

// Four passes: j2 (lines along the contiguous axis, line stride N), i2, j1, i1. The first reads `in`
// and writes `out`; the others work in place on `out`. The tables carry the (-1)^n centring.
template <class T>
hipError_t launch_operator_padfft(int n, int nz, const T* in, T* out, const OperatorTables& op, hipStream_t st) {
  if (!pad_fft_supported(n, nz)) return hipErrorInvalidValue;
  const long long N = n, NN = N * N, NNN = NN * N;
  const int sft = (nz - n) / 2;
  Chirp post1 = op.post1;
  post1.scale = op.scale;
  hipError_t e;
  // PadJob{outer, outer_stride, axis_stride, col_stride, ncols, n, s, pre, post}
  const PadJob j2{1, 0, 1, N, NNN, n, sft, op.pre2, op.post2, 0, 0};     // contiguous axis: lines of N
  const PadJob i2{NN, NN, N, 1, N, n, sft, op.pre2, op.post2, 0, 0};    // stride N, N^2 blocks of N lines
  const PadJob j1{N, NNN, NN, 1, NN, n, sft, op.pre1, op.post1, 0, 0};  // stride N^2, N blocks of N^2 lines
  const PadJob i1{1, 0, NNN, 1, NNN, n, sft, op.pre1, post1, 0, 0};     // stride N^3, N^3 lines
  // The j2, i2 and j1 passes run over groups of whole i1 planes of at most 256 MB, one group after the other,
  // so that each group's second and third passes find it in the memory-side cache; the i1 pass then runs over
  // the whole array. N = 200 padded to 512: 24.7 -> 23.1 ms in complex64 (groups of 4 planes); N = 256 to 512:
  // 66.4 -> 58.3 ms (1 plane); N = 200 to 512 in complex128: 47.5 -> 44.6 ms; N = 200 unpadded (with the tiles
  // in XCD order): 22.29 -> 22.03 ms.
  const long long P = (256ll << 20) / (NNN * (long long)sizeof(T));  // planes per group
  if (P < N) {
    const long long pg = P < 1 ? 1 : P;
    for (long long i0 = 0; i0 < N; i0 += pg) {
      const long long pp = i0 + pg <= N ? pg : N - i0, off = i0 * NNN;
      const PadJob gj2{1, 0, 1, N, pp * NN, n, sft, op.pre2, op.post2, 0, 0};    // the group's lines of N
      const PadJob gi2{pp * N, NN, N, 1, N, n, sft, op.pre2, op.post2, 0, 0};   // pp N blocks of N lines
      const PadJob gj1{pp, NNN, NN, 1, NN, n, sft, op.pre1, op.post1, 0, 0};    // pp blocks of N^2 lines
      if ((e = launch_pad_axis<T>(nz, in + off, out + off, gj2, op.sign2, st)) != hipSuccess) return e;
      if ((e = launch_pad_axis<T>(nz, out + off, out + off, gi2, op.sign2, st)) != hipSuccess) return e;
      if ((e = launch_pad_axis<T>(nz, out + off, out + off, gj1, op.sign1, st)) != hipSuccess) return e;
    }
    return launch_pad_axis<T>(nz, out, out, i1, op.sign1, st);
  }
  if ((e = launch_pad_axis<T>(nz, in, out, j2, op.sign2, st)) != hipSuccess) return e;
  if ((e = launch_pad_axis<T>(nz, out, out, i2, op.sign2, st)) != hipSuccess) return e;
  if ((e = launch_pad_axis<T>(nz, out, out, j1, op.sign1, st)) != hipSuccess) return e;
  return launch_pad_axis<T>(nz, out, out, i1, op.sign1, st);
}

template hipError_t launch_operator_padfft<float2>(int, int, const float2*, float2*, const OperatorTables&,
                                                   hipStream_t);
template hipError_t launch_operator_padfft<double2>(int, int, const double2*, double2*, const OperatorTables&,
                                                    hipStream_t);

template hipError_t launch_operator_dense<float2>(int, int, const float2*, float2*, float2*, const OperatorTables&,
                                                  hipStream_t);
template hipError_t launch_operator_dense<double2>(int, int, const double2*, double2*, double2*,
                                                   const OperatorTables&, hipStream_t);

}  // namespace wolf
