// First-point transform (axes j1 and i1) in one pass over HBM, by workgroups that cooperate
// through the L2 of their XCD.
//
// After the second-point pass, each column m2 of W[p1; m2] still needs a 2D DFT over p1 = (i1, j1):
// N^2 elements spread over the whole array at stride N^2. A tile of C adjacent columns and all N^2
// rows (C N^2 elements: 1 MB for C = 8 at N = 128 in complex64) is more than a CU holds but fits in
// the 4 MB L2 of one XCD, so a tile is transformed in two phases by workgroups of one XCD:
//   phase A: items of R rows i1; each does the j1 DFT of its rows (stride N^2) for the tile's columns;
//   phase B: items of R rows j1; each does the i1 DFT (stride N^3). It starts once every phase-A item
//            of the tile is done (a per-tile counter).
// Phase B reads what phase A wrote from the XCD's L2, so the pair can cost one HBM read and one HBM
// write per element instead of two of each.
//
// Scheduling. Every workgroup takes exactly one item, from the queue of the XCD it runs on (its XCD
// id is read from the hardware register XCC_ID), so the items of a tile run on the XCD whose L2 holds
// the tile. Tiles are dealt round-robin to the 8 queues. A queue lists A(0..L-1), then B(k) A(k+L) for
// each k, then the last L B items. The items a phase-B workgroup waits for come earlier in its queue,
// so they were taken by workgroups that are already running and that never wait themselves: the
// waits end whatever the residency. Each wait is also bounded in wall time (the 100 MHz real-time
// clock); a wait that runs out sets an error flag, and later waits then do not wait at all, so the
// kernel ends soon after.
//
// Control flow. There is no loop around a barrier: one item per workgroup, taken once. The wait is a
// loop of wave 0 alone whose condition is made wave-uniform (readfirstlane), so it compiles to a
// scalar loop with the full execution mask, and the barrier follows it. (A persistent form that took
// items in a loop, with the item fetch and the counter update under `threadIdx.x == 0`, was compiled
// into a loop in which the other lanes returned to the item barrier while lane 0's fetch of the next
// item waited for that loop to end: the workgroup repeated one item without end.)
//
// Memory ordering. A phase-A workgroup drains its stores to the L2 (s_waitcnt 0) before the counter
// update (an agent-scope atomic: atomics are coherent across XCDs). The L1 is write-through and per
// CU, and tiles do not share cache lines (C columns are 64 to 256 bytes). A CU that reads a row
// segment in phase B either wrote it itself in phase A or never touched it, so no stale L1 line is
// hit. Plain stores of one workgroup are visible to the plain loads of another workgroup of the same
// XCD once written to their shared L2; stores made on another XCD are not (its L2 is separate), which
// is why a tile never leaves its XCD.
#include "wolf_device.hpp"
#include "wolf_internal.hpp"

namespace wolf {

__device__ __forceinline__ unsigned xcc_id() {
  // s_getreg_b32 hwreg(HW_REG_XCC_ID, 0, 4): id 20, offset 0, size 4 (the XCD of this wave, 0..7).
  return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 7u;
}

__global__ void k_coop_clear(unsigned* p, int count) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// Phase and tile of queue position `item` (K tiles per XCD, IA items per phase, lookahead L).
__device__ __forceinline__ void coop_decode(int item, int K, int L, int IA, bool* phase_b, int* k, int* r) {
  const int slot = item / IA;
  *r = item - slot * IA;
  if (slot < L) {
    *k = slot;
    *phase_b = false;
  } else {
    const int q = slot - L;
    if (q < 2 * (K - L)) {
      *phase_b = (q & 1) == 0;
      *k = (q >> 1) + (*phase_b ? 0 : L);
    } else {
      *phase_b = true;
      *k = (K - L) + (q - 2 * (K - L));
    }
  }
}

template <class T, int N, int C, int SIGN>
__global__ __launch_bounds__(256) void k_first_point_coop(T* data, CoopParams cp) {
  using S = Split<N>;
  constexpr int N1 = S::N1, N2 = S::N2, Q = S::Q;
  constexpr int G = N2 * C;   // threads per row group
  constexpr int R = 256 / G;  // rows per item
  static_assert(R >= 1 && R * G == 256 && R <= N, "row groups");
  __shared__ T xch[R * N * C];
  __shared__ T tpre[N], tpost[N], tw[N];
  __shared__ int s_item;

  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const unsigned xcd = xcc_id();
  if (tid == 0) s_item = (int)atomicAdd(&cp.head[xcd], 1u);
  __syncthreads();
  const int item = __builtin_amdgcn_readfirstlane(s_item);  // uniform: the branches below are scalar
  const int K = cp.tiles_per_xcd, IA = cp.items_per_phase;
  if (item >= 2 * K * IA) return;  // a queue holds exactly its XCD's share of the grid; never taken
  bool phase_b;
  int k, r;
  coop_decode(item, K, cp.lookahead, IA, &phase_b, &k, &r);
  const long long tile = (long long)k * 8 + xcd;

  const Chirp pre = phase_b ? cp.b_pre : cp.a_pre;
  const Chirp post = phase_b ? cp.b_post : cp.a_post;
  for (int i = tid; i < N; i += 256) {
    tpre[i] = chirp_entry<T>(pre, i, N);
    tpost[i] = chirp_entry<T>(post, i, N);
    tw[i] = twiddle_entry<T, SIGN>(i, N);
  }
  if (phase_b && wave == 0) {
    // Wait for the tile's phase A. Every lane of wave 0 runs the loop; the atomic is issued once for
    // the wave and its value made uniform, so the loop is a scalar loop.
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    for (;;) {
      const unsigned done = __builtin_amdgcn_readfirstlane(
          __hip_atomic_fetch_add(&cp.done_a[tile], cp.zero, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      if (done >= (unsigned)IA) break;
      const unsigned failed = __builtin_amdgcn_readfirstlane(
          __hip_atomic_fetch_add(cp.err, cp.zero, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      if (failed != 0u) break;
      if (__builtin_amdgcn_s_memrealtime() - t0 > cp.max_ticks) {
        __hip_atomic_fetch_or(cp.err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
  }
  __syncthreads();

  const int rg = tid / G, lt = tid - rg * G;
  const int c = lt % C, t = lt / C;
  T* xr = xch + rg * N * C;
  const long long col0 = tile * C;
  const long long row = (long long)r * R + rg;
  const long long base = (phase_b ? row * cp.NN : row * cp.NNN) + col0 + c;
  const long long stride = phase_b ? cp.NNN : cp.NN;

  T v[N1];
#pragma unroll
  for (int a = 0; a < N1; ++a) {
    const int n = N2 * a + t;
    v[a] = cmul(data[base + (long long)n * stride], tpre[n]);
  }
  dft_reg<N1, SIGN>(v);
#pragma unroll
  for (int k1 = 0; k1 < N1; ++k1) xr[(k1 * N2 + t) * C + c] = cmul(v[k1], tw[(t * k1) & (N - 1)]);
  __syncthreads();
  T u[N1];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int k1 = t + N2 * q;
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) u[q * N2 + n2] = xr[(k1 * N2 + n2) * C + c];
    dft_reg<N2, SIGN>(&u[q * N2]);
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int k1 = t + N2 * q;
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      const int kk = k1 + N1 * k2;
      data[base + (long long)kk * stride] = cmul(u[q * N2 + k2], tpost[kk]);
    }
  }
  if (!phase_b) {
    __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have reached the L2
    __syncthreads();
    if (tid == 0) __hip_atomic_fetch_add(&cp.done_a[tile], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Tile widths (columns) that the pass is built for: 64, 128 or 256 bytes of each row.
template <class T> constexpr int coop_min_cols() { return 64 / (int)sizeof(T); }

template <class T, int N, int C, int SIGN>
static hipError_t launch_coop_c(T* data, const CoopParams& cp, long long wgs, hipStream_t st) {
  if constexpr (256 % (Split<N>::N2 * C) != 0 || 256 / (Split<N>::N2 * C) > N) {
    return hipErrorInvalidValue;
  } else {
    hipLaunchKernelGGL((k_first_point_coop<T, N, C, SIGN>), dim3((unsigned)wgs), dim3(256), 0, st, data, cp);
    return hipGetLastError();
  }
}

template <class T, int N, int SIGN>
static hipError_t launch_coop_n(T* data, const CoopParams& cp, int cols, long long wgs, hipStream_t st) {
  constexpr int c0 = coop_min_cols<T>();
  if (cols == c0) return launch_coop_c<T, N, c0, SIGN>(data, cp, wgs, st);
  if (cols == 2 * c0) return launch_coop_c<T, N, 2 * c0, SIGN>(data, cp, wgs, st);
  if (cols == 4 * c0) return launch_coop_c<T, N, 4 * c0, SIGN>(data, cp, wgs, st);
  return hipErrorInvalidValue;
}

bool coop_supported(int n, int elem_bytes, int cols) {
  if (n < 32 || n > 128 || (n & (n - 1)) != 0) return false;
  const int c0 = 64 / elem_bytes;
  if (cols != c0 && cols != 2 * c0 && cols != 4 * c0) return false;
  const long long nn = (long long)n * n;
  const long long tile_bytes = nn * cols * (long long)elem_bytes;
  const long long tiles = nn / cols;
  // A tile must fit well inside one XCD's 4 MB L2, and the tiles must split evenly over the 8 XCDs.
  return tile_bytes <= (2ll << 20) && tiles % 8 == 0;
}

static int coop_rows_per_item(int n, int cols) {
  const int n2 = n / (1 << ((ilog2(n) + 1) / 2));  // Split<N>::N2
  return 256 / (n2 * cols);
}

template <class T>
hipError_t launch_first_point_coop(int n, T* data, const OperatorTables& op, const Chirp& pre1, int cols,
                                   int lookahead, void* counters, hipStream_t st) {
  if (!coop_supported(n, (int)sizeof(T), cols)) return hipErrorInvalidValue;
  const long long nn = (long long)n * n;
  const int tiles = (int)(nn / cols);
  CoopParams cp{};
  cp.NN = nn;
  cp.NNN = nn * n;
  cp.tiles_per_xcd = tiles / 8;
  cp.lookahead = lookahead < cp.tiles_per_xcd ? lookahead : cp.tiles_per_xcd;
  if (cp.lookahead < 1) cp.lookahead = 1;
  cp.items_per_phase = n / coop_rows_per_item(n, cols);
  cp.max_ticks = 2000000ull;  // 20 ms at the 100 MHz real-time clock
  cp.zero = 0u;
  unsigned* base = static_cast<unsigned*>(counters);
  cp.err = base;            // [0]
  cp.head = base + 8;       // [8, 16)
  cp.done_a = base + 16;    // [16, 16 + tiles)
  cp.a_pre = pre1;
  cp.a_post = op.post1;
  // The first-point factors are products of one table per axis: j1 (phase A) and i1 (phase B) each
  // apply theirs; the scale is applied once, with i1's post-factor.
  cp.b_pre = pre1;
  cp.b_post = op.post1;
  cp.b_post.scale = op.scale;
  const long long wgs = 2ll * tiles * cp.items_per_phase;  // one workgroup per item, all 8 queues
  const int count = 16 + tiles;
  hipLaunchKernelGGL(k_coop_clear, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, base, count);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (op.sign1 < 0) {
    switch (n) {
      case 32: return launch_coop_n<T, 32, -1>(data, cp, cols, wgs, st);
      case 64: return launch_coop_n<T, 64, -1>(data, cp, cols, wgs, st);
      case 128: return launch_coop_n<T, 128, -1>(data, cp, cols, wgs, st);
    }
  } else {
    switch (n) {
      case 32: return launch_coop_n<T, 32, +1>(data, cp, cols, wgs, st);
      case 64: return launch_coop_n<T, 64, +1>(data, cp, cols, wgs, st);
      case 128: return launch_coop_n<T, 128, +1>(data, cp, cols, wgs, st);
    }
  }
  return hipErrorInvalidValue;
}

size_t coop_counter_bytes(int n) { return (size_t)(16 + (long long)n * n) * sizeof(unsigned); }

template hipError_t launch_first_point_coop<float2>(int, float2*, const OperatorTables&, const Chirp&, int, int, void*,
                                                    hipStream_t);
template hipError_t launch_first_point_coop<double2>(int, double2*, const OperatorTables&, const Chirp&, int, int,
                                                     void*, hipStream_t);

}  // namespace wolf
