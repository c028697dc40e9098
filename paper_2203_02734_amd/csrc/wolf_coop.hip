// First-point transform (axes j1 and i1) in one pass over HBM, by workgroups that cooperate
// through the L2 of their XCD.
//
// After the slab pass, each column m2 of W[p1; m2] still needs a 2D DFT over p1 = (i1, j1): N^2
// elements spread over the whole array at stride N^2. A coalesced unit is a tile of C adjacent
// columns (one 128 B line per row segment) and all N^2 rows. That is 2 MB at N = 128, more than a
// CU holds, but half of one XCD's 4 MB L2. So a tile is transformed in two phases by the
// workgroups of one XCD:
//   phase A: items of R rows i1; each does the j1 DFT of its rows (stride N^2) for the tile's columns;
//   phase B: items of R rows j1; each does the i1 DFT (stride N^3). It starts once all phase-A
//            items of the tile are done (a per-tile counter).
// Phase B reads what phase A wrote from the XCD's L2, so the pair costs one HBM read and one HBM
// write per element instead of two of each.
//
// Scheduling: every XCD has its own queue (its XCD id is read from the hardware register XCC_ID),
// so all items of a tile run on the XCD whose L2 holds the tile. Tiles are dealt round-robin to
// the queues. A queue lists A(0..L-1), then B(k) A(k+L) for each k, then the last B items.
// Every item a workgroup waits for was taken from the queue before its own, by a workgroup that is
// already running and that never waits itself. The waits therefore end whatever the residency.
// Each wait is also bounded: after max_ticks of the real-time clock the workgroup sets an error flag
// and moves on, so every wave exits.
//
// Memory ordering: a phase-A item drains its stores to the L2 (s_waitcnt 0) before it bumps the
// counter. The L1 is write-through and per CU, and tiles do not share cache lines. So a CU that
// reads a row segment in phase B has never read that segment's old contents (only the CU that wrote
// the segment in phase A touched it earlier). No stale L1 line can be hit.
#include "wolf_device.hpp"
#include "wolf_internal.hpp"

namespace wolf {

__device__ __forceinline__ unsigned xcc_id() {
  // s_getreg_b32 hwreg(HW_REG_XCC_ID, 0, 4): id 20, offset 0, size 4.
  return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 7u;
}

__global__ void k_coop_clear(unsigned* p, int count) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = 0u;
}

template <class T, int N, int C, int SIGN>
__global__ __launch_bounds__(256) void k_first_point_coop(T* data, CoopParams cp) {
  using S = Split<N>;
  constexpr int N1 = S::N1, N2 = S::N2, Q = S::Q;
  constexpr int G = N2 * C;  // threads per row group
  constexpr int R = 256 / G; // rows per item
  static_assert(R >= 1 && R * G == 256, "row groups");
  __shared__ T xch[R * N * C];
  __shared__ T apre[N], apost[N], bpre[N], bpost[N], tw[N];
  __shared__ int s_item;

  for (int i = threadIdx.x; i < N; i += 256) {
    apre[i] = chirp_entry<T>(cp.a_pre, i, N);
    apost[i] = chirp_entry<T>(cp.a_post, i, N);
    bpre[i] = chirp_entry<T>(cp.b_pre, i, N);
    bpost[i] = chirp_entry<T>(cp.b_post, i, N);
    tw[i] = twiddle_entry<T, SIGN>(i, N);
  }
  __syncthreads();

  const unsigned xcd = xcc_id();
  const int tid = threadIdx.x;
  const int rg = tid / G, lt = tid - rg * G;
  const int c = lt % C, t = lt / C;
  T* xr = xch + rg * N * C;
  const int K = cp.tiles_per_xcd, L = cp.lookahead, IA = cp.items_per_phase;
  const int total = 2 * K * IA;

  for (;;) {
    if (tid == 0) s_item = (int)atomicAdd(&cp.head[xcd], 1u);
    __syncthreads();
    const int item = s_item;
    __syncthreads();
    if (item >= total) break;
    const int slot = item / IA, r = item - slot * IA;
    int k;
    bool phase_b;
    if (slot < L) {
      k = slot;
      phase_b = false;
    } else {
      const int q = slot - L;
      if (q < 2 * (K - L)) {
        phase_b = (q & 1) == 0;
        k = (q >> 1) + (phase_b ? 0 : L);
      } else {
        phase_b = true;
        k = (K - L) + (q - 2 * (K - L));
      }
    }
    const long long tile = (long long)k * 8 + xcd;
    if (phase_b) {
      if (tid == 0) {
        // Poll with a read-modify-write (adding an opaque zero), which is served where the
        // increments are: the L2 of this XCD. A plain device-scope load bypasses that L2 and would
        // not see them. The wait is bounded in wall time (s_memrealtime, 100 MHz).
        const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
        while (__hip_atomic_fetch_add(&cp.done_a[tile], cp.zero, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
               (unsigned)IA) {
          __builtin_amdgcn_s_sleep(4);
          if (__builtin_amdgcn_s_memrealtime() - t0 > cp.max_ticks) {
            atomicOr(cp.err, 1u);
            break;
          }
        }
      }
      __syncthreads();
    }
    const long long col0 = tile * C;
    const long long row = (long long)r * R + rg;
    const long long base = (phase_b ? row * cp.NN : row * cp.NNN) + col0 + c;
    const long long stride = phase_b ? cp.NNN : cp.NN;
    const T* tpre = phase_b ? bpre : apre;
    const T* tpost = phase_b ? bpost : apost;

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
}

template <class T> constexpr int coop_cols() { return 128 / (int)sizeof(T); }  // one 128 B line

template <class T, int N, int SIGN>
static hipError_t launch_coop_n(T* data, const CoopParams& cp, int wgs, hipStream_t st) {
  constexpr int C = coop_cols<T>();
  if constexpr (256 % (Split<N>::N2 * C) != 0 || 256 / (Split<N>::N2 * C) > N) {
    return hipErrorInvalidValue;
  } else {
    hipLaunchKernelGGL((k_first_point_coop<T, N, C, SIGN>), dim3((unsigned)wgs), dim3(256), 0, st, data, cp);
    return hipGetLastError();
  }
}

template <class T> bool coop_supported(int n) {
  if (n < 32 || n > 128) return false;
  const long long nn = (long long)n * n;
  const long long tile_bytes = nn * coop_cols<T>() * (long long)sizeof(T);
  const long long tiles = nn / coop_cols<T>();
  return tile_bytes <= (2ll << 20) && tiles % 8 == 0;
}

template <class T> int coop_rows_per_item(int n) {
  const int n2 = n == 32 ? 4 : (n == 64 ? 8 : 8);
  return 256 / (n2 * coop_cols<T>());
}

template <class T>
hipError_t launch_first_point_coop(int n, T* data, const OperatorTables& op, const Chirp& pre1, int wgs,
                                   int lookahead, void* counters, hipStream_t st) {
  if (!coop_supported<T>(n)) return hipErrorInvalidValue;
  const long long nn = (long long)n * n;
  const int tiles = (int)(nn / coop_cols<T>());
  CoopParams cp{};
  cp.NN = nn;
  cp.NNN = nn * n;
  cp.tiles_per_xcd = tiles / 8;
  cp.lookahead = lookahead < cp.tiles_per_xcd ? lookahead : cp.tiles_per_xcd;
  if (cp.lookahead < 1) cp.lookahead = 1;
  cp.items_per_phase = n / coop_rows_per_item<T>(n);
  cp.max_ticks = 10000000ull;  // 100 ms at the 100 MHz real-time clock
  cp.zero = 0u;
  unsigned* base = static_cast<unsigned*>(counters);
  cp.err = base;            // [0]
  cp.head = base + 8;       // [8, 16)
  cp.done_a = base + 16;    // [16, 16 + tiles)
  cp.a_pre = pre1;
  cp.a_post = op.post1;
  cp.b_pre = pre1;
  cp.b_post = op.post1;
  cp.b_post.scale = op.scale;
  const int count = 16 + tiles;
  hipLaunchKernelGGL(k_coop_clear, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, base, count);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // cp.err keeps its value from the clear above: the flag reports this launch only.
  if (op.sign1 < 0) {
    switch (n) {
      case 32: return launch_coop_n<T, 32, -1>(data, cp, wgs, st);
      case 64: return launch_coop_n<T, 64, -1>(data, cp, wgs, st);
      case 128: return launch_coop_n<T, 128, -1>(data, cp, wgs, st);
    }
  } else {
    switch (n) {
      case 32: return launch_coop_n<T, 32, +1>(data, cp, wgs, st);
      case 64: return launch_coop_n<T, 64, +1>(data, cp, wgs, st);
      case 128: return launch_coop_n<T, 128, +1>(data, cp, wgs, st);
    }
  }
  return hipErrorInvalidValue;
}

size_t coop_counter_bytes(int n) { return (size_t)(16 + (long long)n * n) * sizeof(unsigned); }

template bool coop_supported<float2>(int);
template bool coop_supported<double2>(int);
template hipError_t launch_first_point_coop<float2>(int, float2*, const OperatorTables&, const Chirp&, int, int, void*,
                                                    hipStream_t);
template hipError_t launch_first_point_coop<double2>(int, double2*, const OperatorTables&, const Chirp&, int, int,
                                                     void*, hipStream_t);

}  // namespace wolf
