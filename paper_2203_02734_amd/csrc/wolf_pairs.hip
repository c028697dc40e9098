// Observables of many (lambda, z) pairs without a propagated N^4 array: the sums that S and the row
// W_B[P; .] need are contractions over the first point that the pairs of a group share (eq. W_fresnel).
//
// With the operator's checkerboarded tables u1 = pre1, u2 = pre2 (per axis; they carry the source
// chirp of each pair and the (-1)^n centring), the raw sums of S and of the row are
//   s0[m] = Re sum_d e^{+2 pi i <m, d>/N} D[d],  D[d] = sum_{p1} u1(p1) u2(p1 - d) W[p1; p1 - d]
//   b0[m] = sum_{p2} e^{-2 pi i <m, p2>/N} u2(p2) R[p2],  R[p2] = sum_{p1} e^{+2 pi i <P, p1>/N} u1(p1) W[p1; p2]
// (indices mod N, 2D products of the axis tables). S = s w s0 and W_B[P; m] = s w post1(P) post2(m) b0[m]:
// on the diagonal m1 = m2 = m the post-factors cancel and the two exponentials depend on p1 - p2 only.
// Both sums are dense contractions over p1 with pair-dependent weights:
//   R = C W with C[k][p1] = ci_k[a] cj_k[b] (a complex GEMM, pairs x N^2 x N^2), and
//   D[k][(di, dj)] = sum_b B_k^{dj}[b] sum_a A_k^{di}[a] W[a, b; a - di, b - dj] with A = u1[a] u2[a - di],
//   B = u1[b] u2[b - dj]: for each di and b a GEMM over a (pairs x N x N).
// The source is read twice per group of up to 64 pairs (once for a group of one entry), then two N x N
// DFTs per pair. The polychromatic sum on a common grid (below) uses the same contractions.
#include "wolf_device.hpp"
#include "wolf_internal.hpp"
#include "wolf_mfma.hpp"

namespace wolf {

constexpr int kPairTile = kPairGroup;  // pairs per group (rows of the GEMM tiles)
constexpr int kPairSplitK = 16;  // chunks of p1 in the row sums R (partials summed in FP64)
constexpr int kOneThreads = 256, kOneCols = 8;  // the one-pass sums of a group of one entry

struct PairGroup {
  int count;                 // pairs in this group (<= kPairTile)
  double a_src[kPairTile];   // source chirp rate of each pair (0 in the far field)
};

// Tables of one group, FP64-built: u1, u2 (pre1, pre2 of each pair), ci = e^{2 pi i P_i a/N} u1[a],
// cj = e^{2 pi i P_j b/N} u1[b]; each kPairTile x N. Pairs beyond the count get zero tables. The
// matrix-core kernels read the same four tables transposed (tr: [4][N][kPairTile]), so that the 64
// pairs of one index are 512 contiguous bytes.
template <class T>
__device__ __forceinline__ void store_tables(T* u1, T* u2, T* ci, T* cj, T* tr, int n, int k, int a, T v1, T v2,
                                             T vi, T vj) {
  const int e = k * n + a;
  const long long t = (long long)a * kPairTile + k, q = (long long)n * kPairTile;
  u1[e] = v1; u2[e] = v2; ci[e] = vi; cj[e] = vj;
  tr[t] = v1; tr[q + t] = v2; tr[2 * q + t] = vi; tr[3 * q + t] = vj;
}

template <class T>
__global__ __launch_bounds__(256) void k_pair_tables(PairGroup g, int n, int pi, int pj, T* u1, T* u2, T* ci, T* cj,
                                                     T* tr) {
  using R = typename real_of<T>::type;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kPairTile * n) return;
  const int k = e / n, a = e % n;
  if (k >= g.count) {
    const T z{(R)0, (R)0};
    store_tables(u1, u2, ci, cj, tr, n, k, a, z, z, z, z);
    return;
  }
  const Chirp c1{g.a_src[k], 1.0, -1, 1}, c2{g.a_src[k], 1.0, +1, 1};
  const double2 v1 = chirp_entry<double2>(c1, a, n), v2 = chirp_entry<double2>(c2, a, n);
  double si, co, sj, cjx;
  sincospi(2.0 * (double)((pi * a) % n) / (double)n, &si, &co);
  sincospi(2.0 * (double)((pj * a) % n) / (double)n, &sj, &cjx);
  const double2 wi = cmul(double2{co, si}, v1), wj = cmul(double2{cjx, sj}, v1);
  store_tables(u1, u2, ci, cj, tr, n, k, a, T{(R)v1.x, (R)v1.y}, T{(R)v2.x, (R)v2.y}, T{(R)wi.x, (R)wi.y},
               T{(R)wj.x, (R)wj.y});
}

// Staged element q of thread tid in one step of 16 contraction rows kk: the B operand (TN columns) and
// the A operand (TM pairs). For TM = 64 the row of both is one per wavefront (wavefront-uniform, so its
// index math runs on the scalar unit); for TM = 32 the B row is, and the A row is per lane.
template <int TM> struct MStage {
  static constexpr int TN = MTile<TM>::TN;
  __device__ __forceinline__ static int b_row(int wv, int q) { return (wv * 64) / TN + (256 / TN) * q; }
  __device__ __forceinline__ static int b_col(int wv, int lane) { return (wv * 64) % TN + lane; }
  __device__ __forceinline__ static int a_row(int tid, int wv, int q) {
    if constexpr (TM == 64) return wv + 4 * q;
    else return (tid + 256 * q) / TM;
  }
  __device__ __forceinline__ static int a_pair(int tid, int lane) {
    if constexpr (TM == 64) return lane;
    else return tid % TM;
  }
};

// Row sums: part[s][k][p2] = sum_{p1 in chunk s} ci[k][a] cj[k][b] W[p1][p2] (p1 = a N + b), for the
// first TM pairs k. A workgroup computes a tile of TM pairs x TN columns p2; p1 runs through the chunk 16
// at a time: the A operand is generated from the tables, the W rows are TN contiguous elements. The
// operands of step s + 1 are loaded from HBM while the matrix cores work on step s, and staged into the
// second LDS buffer after it: one barrier per step.
template <class T, int TM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 4 : 2))) void k_pair_rows_mfma(
    const T* __restrict__ w, int n, const T* __restrict__ cit, const T* __restrict__ cjt, long long chunk,
    T* __restrict__ part) {
  using R = typename real_of<T>::type;
  using G = MTile<TM>;
  using M = MStage<TM>;
  constexpr int TK = 16, TN = G::TN;
  __shared__ R ar[2][TK][G::LDA], ai[2][TK][G::LDA], br[2][TK][G::LDB], bi[2][TK][G::LDB];
  const long long nn = (long long)n * n;
  const int tid = threadIdx.x, lane = tid % 64;
  const int wv = __builtin_amdgcn_readfirstlane(tid / 64);  // wavefront-uniform
  const int row0 = (wv / G::WC) * 32, col0 = (wv % G::WC) * 32;
  const long long j0 = (long long)blockIdx.x * TN;
  const long long s = blockIdx.y;
  const long long p_begin = s * chunk, p_end = (p_begin + chunk < nn) ? p_begin + chunk : nn;
  const int lg = __builtin_ctz((unsigned)n);
  T rb[G::QB], ca[G::QA], cb[G::QA];
  auto fetch = [&](long long k0) {
#pragma unroll
    for (int q = 0; q < G::QB; ++q) {  // W[p1][p2], p1 = k0 + row, p2 = j0 + column
      const long long p1 = k0 + M::b_row(wv, q), p2 = j0 + M::b_col(wv, lane);
      rb[q] = load_or_first(w, p1 < p_end && p2 < nn, p1 * nn + p2);
    }
#pragma unroll
    for (int q = 0; q < G::QA; ++q) {  // A[kk][k] = ci[k][a] cj[k][b], p1 = k0 + kk = a N + b
      const long long p1 = k0 + M::a_row(tid, wv, q);
      const int k = M::a_pair(tid, lane);
      const int pi = p1 < p_end ? (int)p1 : 0;  // p1 < N^2, N a power of two
      ca[q] = cit[(pi >> lg) * kPairTile + k];
      cb[q] = cjt[(pi & (n - 1)) * kPairTile + k];
    }
  };
  auto stage = [&](int buf, long long k0) {
#pragma unroll
    for (int q = 0; q < G::QB; ++q) {
      const int kk = M::b_row(wv, q), jj = M::b_col(wv, lane);
      const T v = keep_or_zero(k0 + kk < p_end && j0 + jj < nn, rb[q]);
      br[buf][kk][jj] = v.x;
      bi[buf][kk][jj] = v.y;
    }
#pragma unroll
    for (int q = 0; q < G::QA; ++q) {
      const int kk = M::a_row(tid, wv, q), k = M::a_pair(tid, lane);
      const T a = keep_or_zero(k0 + kk < p_end, cmul(ca[q], cb[q]));
      ar[buf][kk][k] = a.x;
      ai[buf][kk][k] = a.y;
    }
  };
  CTile<T> acc;
  ctile_zero(acc);
  fetch(p_begin);
  stage(0, p_begin);
  __syncthreads();
  int buf = 0;
  for (long long k0 = p_begin; k0 < p_end; k0 += TK) {
    const bool more = k0 + TK < p_end;
    if (more) fetch(k0 + TK);
    ctile_mfma16<T, G::LDA, G::LDB>(acc, ar[buf], ai[buf], br[buf], bi[buf], row0, col0, lane);
    if (more) stage(buf ^ 1, k0 + TK);
    __syncthreads();
    buf ^= 1;
  }
  T* out = part + s * kPairTile * nn;
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const long long k = row0 + 16 * r + Mfma<T>::row(lane, i);
        const long long j = j0 + col0 + 16 * q + lane % 16;
        if (j < nn) out[k * nn + j] = T{acc.re(r, q, i), acc.im(r, q, i)};
      }
}

// Row sums of a complex64 group at N = 64 or 128, with the W stream kept deep in flight:
// part[s][k][p2] = sum_{a} ci[k][a] G_a[k][p2], G_a[k][p2] = sum_b cj[k][b] W[a N + b][p2], over the
// whole rows a of chunk s, for the first 16 R pairs k (R = 4: groups of more than 32 pairs; 2: 17-32; 1: up
// to 16; the rows of the other pairs are not written). The tables cj and ci of the group sit in LDS for the
// whole launch (2 x N x 64 complex, one workgroup per CU), so the only memory loads of the loop are the W
// operand: a wavefront owns the 16 R pairs and 32 columns p2 and keeps eight steps of 16 rows of W in
// registers (one wavefront per SIMD, up to 512 registers). Each step is 24 R MFMAs into G (R x 2 tiles of
// 16 x 16 in the 3M form, A = cj from LDS); after the N / 16 steps of a row a, G is folded into the output
// sums with ci[k][a] and cleared. Every load is unconditional (the ring's last loads re-read the chunk's last step) and the
// scheduling barriers keep each step's loads ahead of the matrix-core block they precede, so that the
// waits leave the seven later steps in flight.
struct RingStep {
  float2 v[4][2];  // W[k0 + 4 ks + l / 16][j0 + 16 q + l % 16]
};

template <int N, int R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_pair_rows_ring(
    const float2* __restrict__ w, const float2* __restrict__ cit, const float2* __restrict__ cjt, long long chunk,
    int items, float2* __restrict__ part) {
  constexpr long long NN = (long long)N * N;
  constexpr int SPA = N / 16;  // steps per row a
  constexpr int RING = 8;
  constexpr int TILES = (int)(NN / 128);  // 128-column tiles per chunk
  static_assert(SPA <= RING && RING % SPA == 0, "ring of whole rows");
  static_assert(R >= 1 && 16 * R <= kPairTile, "tiles of 16 pairs");
  __shared__ float2 cjs[N * kPairTile], cis[N * kPairTile];
  const int tid = threadIdx.x, lane = tid % 64, l16 = lane % 16, kq = lane / 16;
  const int wv = __builtin_amdgcn_readfirstlane(tid / 64);
  // cj[b][k] at b 64 + (k ^ 16 (b & 1)): the four rows of an MFMA step fall on alternate bank halves.
  for (int e = tid; e < N * kPairTile; e += 256) {
    const int b = e / kPairTile, k = e % kPairTile;
    cjs[b * kPairTile + (k ^ ((b & 1) << 4))] = cjt[e];
    cis[e] = cit[e];
  }
  __syncthreads();
  // Items (column tile, chunk) item = blockIdx.x + i gridDim.x, i < mine, run back to back as one
  // sequence of steps t = i steps + step, so the ring stays full across items.
  const int steps = (int)(chunk / 16);
  const int mine = (items - (int)blockIdx.x + (int)gridDim.x - 1) / (int)gridDim.x;
  const int total = mine * steps;
  auto item_of = [&](int i) { return (int)blockIdx.x + i * (int)gridDim.x; };
  auto load = [&](RingStep& r, int t) {
    const int tc = t < total ? t : total - 1;
    const int it = item_of(tc / steps), step = tc % steps;
    const long long j0 = (long long)(it % TILES) * 128 + 32 * wv;
    const long long p1 = (long long)(it / TILES) * chunk + 16 * step + kq;
    const float2* q0 = w + p1 * NN + j0 + l16;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
      for (int q = 0; q < 2; ++q) r.v[ks][q] = q0[(long long)ks * 4 * NN + 16 * q];
  };
  v4f t1[R][2], t2[R][2], t3[R][2];
  float2 f[R][2][4];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      t1[r][q] = t2[r][q] = t3[r][q] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int i = 0; i < 4; ++i) f[r][q][i] = float2{0.f, 0.f};
    }
  // A operand of one step (cj rows b0 .. b0 + 15 of this lane's pairs), read from LDS one step ahead.
  auto read_a = [&](float2 (&av)[4][R], int b0) {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int b = b0 + 4 * ks + kq;
#pragma unroll
      for (int r = 0; r < R; ++r) av[ks][r] = cjs[b * kPairTile + ((16 * r + l16) ^ ((b & 1) << 4))];
    }
  };
  auto step_mfma = [&](const float2 (&av)[4][R], const RingStep& bw) {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      float xs[R], ys[2];
#pragma unroll
      for (int r = 0; r < R; ++r) xs[r] = av[ks][r].x + av[ks][r].y;
#pragma unroll
      for (int q = 0; q < 2; ++q) ys[q] = bw.v[ks][q].x + bw.v[ks][q].y;
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          t1[r][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ks][r].x, bw.v[ks][q].x, t1[r][q], 0, 0, 0);
          t2[r][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ks][r].y, bw.v[ks][q].y, t2[r][q], 0, 0, 0);
          t3[r][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(xs[r], ys[q], t3[r][q], 0, 0, 0);
        }
    }
  };
  RingStep ring[RING];
#pragma unroll
  for (int u = 0; u < RING - 1; ++u) {
    load(ring[u], u);
    __builtin_amdgcn_sched_barrier(0);
  }
  float2 avs[2][4][R];
  read_a(avs[0], 0);
  for (int t0 = 0; t0 < total; t0 += RING) {  // steps is a multiple of RING: t0 is a multiple of SPA
#pragma unroll
    for (int u = 0; u < RING; ++u) {
      load(ring[(u + RING - 1) % RING], t0 + u + RING - 1);
      read_a(avs[(u + 1) % 2], ((u + 1) % SPA) * 16);  // the next step's operand
      __builtin_amdgcn_sched_barrier(0);
      step_mfma(avs[u % 2], ring[u]);
      if ((u + 1) % SPA == 0) {  // the last step of row a: fold G into the sums with ci[k][a]
        const int t = t0 + u, it = item_of(t / steps);
        const int a = (int)(((long long)(it / TILES) * chunk + 16 * (t % steps)) / N);
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float2 c = cis[a * kPairTile + 16 * r + Mfma<float2>::row(lane, i)];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
              const float gr = t1[r][q][i] - t2[r][q][i], gi = t3[r][q][i] - t1[r][q][i] - t2[r][q][i];
              f[r][q][i].x += c.x * gr - c.y * gi;
              f[r][q][i].y += c.x * gi + c.y * gr;
            }
          }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int q = 0; q < 2; ++q) t1[r][q] = t2[r][q] = t3[r][q] = v4f{0.f, 0.f, 0.f, 0.f};
        if ((t + 1) % steps == 0) {  // the item's last step: store its sums and start the next item
          float2* out = part + (long long)(it / TILES) * kPairTile * NN;
          const long long j0 = (long long)(it % TILES) * 128 + 32 * wv;
#pragma unroll
          for (int r = 0; r < R; ++r)
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                out[(16 * r + Mfma<float2>::row(lane, i)) * NN + j0 + 16 * q + l16] = f[r][q][i];
                f[r][q][i] = float2{0.f, 0.f};
              }
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// Difference sums: part[z][k][di N + dj] = sum_{b in chunk z} B_k^{dj}[b] sum_a A_k^{di}[a]
// W[a, b; a - di, b - dj] (indices mod N), A = u1[a] u2[a - di], B = u1[b] u2[b - dj], for the first TM
// pairs k. A workgroup owns di, TN values of dj and a chunk of b; for each b the inner sum is a GEMM over
// a (TM x TN x N) whose W operand is TN consecutive columns of one row, read backwards and wrapping. The
// steps (b, a0) run in one sequence, double-buffered like k_pair_rows_mfma; after the last a0 of each b
// the wavefront block folds its G tile into D.
template <class T, int TM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 3 : 2))) void k_pair_diffs_mfma(
    const T* __restrict__ w, int n, const T* __restrict__ u1, const T* __restrict__ u2,
    const T* __restrict__ u1t, const T* __restrict__ u2t, int bchunk, T* __restrict__ part) {
  using R = typename real_of<T>::type;
  using G = MTile<TM>;
  using M = MStage<TM>;
  constexpr int TK = 16;
  __shared__ R ar[2][TK][G::LDA], ai[2][TK][G::LDA], br[2][TK][G::LDB], bi[2][TK][G::LDB];
  const long long nn = (long long)n * n;
  const int tid = threadIdx.x, lane = tid % 64;
  const int wv = __builtin_amdgcn_readfirstlane(tid / 64);  // wavefront-uniform
  const int row0 = (wv / G::WC) * 32, col0 = (wv % G::WC) * 32;
  const int dj0 = blockIdx.x * G::TN, di = blockIdx.y, nm = n - 1;  // N is a power of two
  const int b_begin = blockIdx.z * bchunk, b_end = (b_begin + bchunk < n) ? b_begin + bchunk : n;
  R dre[2][2][4], dim[2][2][4];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) dre[r][q][i] = dim[r][q][i] = (R)0;
  T rb[G::QB], ca[G::QA], cb[G::QA];
  auto fetch = [&](int b, int a0) {  // W[a, b; a - di, b - dj] and the tables of A = u1[a] u2[a - di]
#pragma unroll
    for (int q = 0; q < G::QB; ++q) {
      const int a = a0 + M::b_row(wv, q), dj = dj0 + M::b_col(wv, lane);
      rb[q] = load_or_first(w, a < n && dj < n,
                            ((long long)a * n + b) * nn + (long long)((a - di) & nm) * n + ((b - dj) & nm));
    }
#pragma unroll
    for (int q = 0; q < G::QA; ++q) {
      const int a = a0 + M::a_row(tid, wv, q), k = M::a_pair(tid, lane);
      const int ac = a < n ? a : 0;
      ca[q] = u1t[ac * kPairTile + k];
      cb[q] = u2t[((ac - di) & nm) * kPairTile + k];
    }
  };
  auto stage = [&](int buf, int a0) {
#pragma unroll
    for (int q = 0; q < G::QB; ++q) {
      const int kk = M::b_row(wv, q), jj = M::b_col(wv, lane);
      const T v = keep_or_zero(a0 + kk < n && dj0 + jj < n, rb[q]);
      br[buf][kk][jj] = v.x;
      bi[buf][kk][jj] = v.y;
    }
#pragma unroll
    for (int q = 0; q < G::QA; ++q) {
      const int kk = M::a_row(tid, wv, q), k = M::a_pair(tid, lane);
      const T a = keep_or_zero(a0 + kk < n, cmul(ca[q], cb[q]));
      ar[buf][kk][k] = a.x;
      ai[buf][kk][k] = a.y;
    }
  };
  if (b_begin < b_end) {
    fetch(b_begin, 0);
    stage(0, 0);
  }
  __syncthreads();
  CTile<T> g;
  ctile_zero(g);
  int buf = 0;
  for (int b = b_begin, a0 = 0; b < b_end;) {
    const bool last_a = a0 + TK >= n;
    const int nb = last_a ? b + 1 : b, na = last_a ? 0 : a0 + TK;
    const bool more = nb < b_end;
    if (more) fetch(nb, na);
    ctile_mfma16<T, G::LDA, G::LDB>(g, ar[buf], ai[buf], br[buf], bi[buf], row0, col0, lane);
    if (last_a) {
      // D += B_k^{dj}[b] G, B = u1[k][b] u2[k][b - dj], on the outputs this lane holds
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int k = row0 + 16 * r + Mfma<T>::row(lane, i);
          const T ub = u1[k * n + b];
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int dj = dj0 + col0 + 16 * q + lane % 16;
            const T f = cmul(ub, u2[k * n + ((b - dj) & nm)]);
            const R gr = g.re(r, q, i), gi = g.im(r, q, i);
            dre[r][q][i] += f.x * gr - f.y * gi;
            dim[r][q][i] += f.x * gi + f.y * gr;
          }
        }
      ctile_zero(g);
    }
    if (more) stage(buf ^ 1, na);
    __syncthreads();
    buf ^= 1;
    b = nb;
    a0 = na;
  }
  T* out = part + (long long)blockIdx.z * kPairTile * nn;
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const long long k = row0 + 16 * r + Mfma<T>::row(lane, i);
        const int dj = dj0 + col0 + 16 * q + lane % 16;
        if (dj < n) out[k * nn + (long long)di * n + dj] = T{dre[r][q][i], dim[r][q][i]};
      }
}

// Difference sums of a complex64 group at N = 128, with the W stream kept deep
// in flight (the ring of k_pair_rows_ring): part[z][k][di N + dj] = sum_{b in chunk z} B_k^{dj}[b] G_b[k][dj],
// G_b[k][dj] = sum_a A^{di}[a][k] W[a, b; a - di, b - dj], A^{di}[a][k] = u1[k][a] u2[k][a - di],
// B_k^{dj}[b] = u1[k][b] u2[k][b - dj] (indices mod N). A workgroup owns one di and 256 / N chunks of b
// (z = blockIdx.x % (256 / N)), the first 16 R pairs (R = 4, 2, 1 for groups of more than 32, 17-32 and
// up to 16 pairs; the other pairs' sums are not written) and all N values of dj (a wavefront: 32 of them). A^{di}
// (formed once) and u2 sit in LDS; u1[k][b] is loaded at the start of each b. Each step is 16 values of a
// (24 R MFMAs into G); after the N / 16 steps of one b, G is folded into the sums. Only N = 128 fills the
// four wavefronts' 128 columns; at N = 64 wavefronts 2 and 3 hold no columns and stay idle.
template <int N, int R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_pair_diffs_ring(
    const float2* __restrict__ w, const float2* __restrict__ u1t, const float2* __restrict__ u2t,
    float2* __restrict__ part) {
  constexpr long long NN = (long long)N * N;
  constexpr int SPB = N / 16;  // steps per b
  constexpr int RING = 8, BSPLIT = 256 / N, BCH = N / BSPLIT;
  constexpr int NM = N - 1;
  static_assert(SPB <= RING && RING % SPB == 0, "ring of whole b");
  static_assert(R >= 1 && 16 * R <= kPairTile, "tiles of 16 pairs");
  __shared__ float2 as_[N * kPairTile], u2s[N * kPairTile];
  const int tid = threadIdx.x, lane = tid % 64, l16 = lane % 16, kq = lane / 16;
  const int wv = __builtin_amdgcn_readfirstlane(tid / 64);
  const int di = (int)blockIdx.x / BSPLIT, z = (int)blockIdx.x % BSPLIT;
  const int b_lo = z * BCH;
  // A^{di}[a][k] at a 64 + (k ^ 16 (a & 1)); u2[m][k] at m 64 + (k ^ 2 (m & 15)) (the fold's 16 lanes of one
  // k read 16 consecutive m).
  for (int e = tid; e < N * kPairTile; e += 256) {
    const int m = e / kPairTile, k = e % kPairTile;
    as_[m * kPairTile + (k ^ ((m & 1) << 4))] = cmul(u1t[e], u2t[((m - di) & NM) * kPairTile + k]);
    u2s[m * kPairTile + (k ^ ((m & 15) << 1))] = u2t[e];
  }
  __syncthreads();
  if (wv * 32 >= N) return;  // no columns for this wavefront (N = 64); no barrier follows
  const int dj0 = 32 * wv;
  constexpr int total = BCH * SPB;
  auto load = [&](RingStep& r, int t) {
    const int tc = t < total ? t : total - 1;
    const int b = b_lo + tc / SPB, a0 = (tc % SPB) * 16;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int a = a0 + 4 * ks + kq;
      const float2* row = w + ((long long)a * N + b) * NN + (long long)((a - di) & NM) * N;
#pragma unroll
      for (int q = 0; q < 2; ++q) r.v[ks][q] = row[(b - dj0 - 16 * q - l16) & NM];
    }
  };
  v4f t1[R][2], t2[R][2], t3[R][2];
  float2 f[R][2][4], u1v[R][4];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      t1[r][q] = t2[r][q] = t3[r][q] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int i = 0; i < 4; ++i) f[r][q][i] = float2{0.f, 0.f};
    }
  auto read_a = [&](float2 (&av)[4][R], int a0) {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int a = a0 + 4 * ks + kq;
#pragma unroll
      for (int r = 0; r < R; ++r) av[ks][r] = as_[a * kPairTile + ((16 * r + l16) ^ ((a & 1) << 4))];
    }
  };
  auto step_mfma = [&](const float2 (&av)[4][R], const RingStep& bw) {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      float xs[R], ys[2];
#pragma unroll
      for (int r = 0; r < R; ++r) xs[r] = av[ks][r].x + av[ks][r].y;
#pragma unroll
      for (int q = 0; q < 2; ++q) ys[q] = bw.v[ks][q].x + bw.v[ks][q].y;
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          t1[r][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ks][r].x, bw.v[ks][q].x, t1[r][q], 0, 0, 0);
          t2[r][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ks][r].y, bw.v[ks][q].y, t2[r][q], 0, 0, 0);
          t3[r][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(xs[r], ys[q], t3[r][q], 0, 0, 0);
        }
    }
  };
  RingStep ring[RING];
#pragma unroll
  for (int u = 0; u < RING - 1; ++u) {
    load(ring[u], u);
    __builtin_amdgcn_sched_barrier(0);
  }
  float2 avs[2][4][R];
  read_a(avs[0], 0);
  for (int t0 = 0; t0 < total; t0 += RING) {  // t0 is a multiple of SPB
#pragma unroll
    for (int u = 0; u < RING; ++u) {
      const int b = b_lo + (t0 + u) / SPB;
      load(ring[(u + RING - 1) % RING], t0 + u + RING - 1);
      if (u % SPB == 0) {  // u1[k][b] of this b, behind the ring's load (it is needed at the fold)
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int i = 0; i < 4; ++i) u1v[r][i] = u1t[b * kPairTile + 16 * r + Mfma<float2>::row(lane, i)];
      }
      read_a(avs[(u + 1) % 2], ((u + 1) % SPB) * 16);  // the next step's operand
      __builtin_amdgcn_sched_barrier(0);
      step_mfma(avs[u % 2], ring[u]);
      if ((u + 1) % SPB == 0) {  // the last step of b: D += u1[k][b] u2[k][b - dj] G
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int k = 16 * r + Mfma<float2>::row(lane, i);
#pragma unroll
            for (int q = 0; q < 2; ++q) {
              const int m = (b - dj0 - 16 * q - l16) & NM;
              const float2 c = cmul(u1v[r][i], u2s[m * kPairTile + (k ^ ((m & 15) << 1))]);
              const float gr = t1[r][q][i] - t2[r][q][i], gi = t3[r][q][i] - t1[r][q][i] - t2[r][q][i];
              f[r][q][i].x += c.x * gr - c.y * gi;
              f[r][q][i].y += c.x * gi + c.y * gr;
            }
          }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int q = 0; q < 2; ++q) t1[r][q] = t2[r][q] = t3[r][q] = v4f{0.f, 0.f, 0.f, 0.f};
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  float2* out = part + (long long)z * kPairTile * NN;
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        out[(16 * r + Mfma<float2>::row(lane, i)) * NN + (long long)di * N + dj0 + 16 * q + l16] = f[r][q][i];
}

// The polychromatic difference sums without wrap (the bins of k_poly_diffs_mfma) on the register ring of
// k_pair_diffs_ring, for the pairs k0 .. k0 + 16 R - 1 of a complex64 group at N = 128: one tile of 16 pairs
// with eight steps of the source in flight (R = 1, RING = 8), or two tiles with four steps (R = 2, RING = 4:
// with eight, the two bins' sums of two tiles exceed the registers of one wavefront per SIMD and spill). A
// workgroup owns one folded d_i, 256 / N chunks of b (z = blockIdx.x % (256 / N)) and every a: a step of 16
// values of a adds into the G of bin d_i (a >= d_i) or of bin d_i - N (a < d_i); the one step that holds d_i
// runs twice, with the A rows of the other bin zeroed. After the N / 16 steps of one b both G are folded into
// their sums. On the second point a lane's column d_j switches bin once as b rises, so the lane stores its
// lower bin's sums when b passes d_j - 1 and writes each of its four bins (two of d_i, two of d_j) exactly once
// per chunk of b, zeros where the chunk holds no term.
template <int N, int R, int RING>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_poly_diffs_ring(
    const float2* __restrict__ w, const float2* __restrict__ u1t, const float2* __restrict__ u2t, int k0,
    float2* __restrict__ part) {
  constexpr long long NN = (long long)N * N, BINS = 4 * NN;
  constexpr int SPB = N / 16;  // steps per b
  constexpr int BSPLIT = 256 / N, BCH = N / BSPLIT;
  constexpr int NM = N - 1;
  static_assert((SPB <= RING && RING % SPB == 0) || (RING < SPB && SPB % RING == 0), "ring and steps per b nest");
  static_assert((R == 1 && RING == 8) || (R == 2 && RING == 4), "the register budgets measured");
  __shared__ float2 as_[N * kPairTile], u2s[N * kPairTile];
  const int tid = threadIdx.x, lane = tid % 64, l16 = lane % 16, kq = lane / 16;
  const int wv = __builtin_amdgcn_readfirstlane(tid / 64);
  const int di = (int)blockIdx.x / BSPLIT, z = (int)blockIdx.x % BSPLIT;
  const int b_lo = z * BCH, b_hi = b_lo + BCH;
  // A^{di}[a][k] at a 64 + (k ^ 16 (a & 1)); u2[m][k] at m 64 + (k ^ 2 (m & 15)), as in k_pair_diffs_ring.
  for (int e = tid; e < N * kPairTile; e += 256) {
    const int m = e / kPairTile, k = e % kPairTile;
    as_[m * kPairTile + (k ^ ((m & 1) << 4))] = cmul(u1t[e], u2t[((m - di) & NM) * kPairTile + k]);
    u2s[m * kPairTile + (k ^ ((m & 15) << 1))] = u2t[e];
  }
  __syncthreads();
  if (wv * 32 >= N) return;  // no columns for this wavefront; no barrier follows
  const int dj0 = 32 * wv;
  constexpr int total = BCH * SPB;
  auto load = [&](RingStep& r, int t) {
    const int tc = t < total ? t : total - 1;
    const int b = b_lo + tc / SPB, a0 = (tc % SPB) * 16;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int a = a0 + 4 * ks + kq;
      const float2* row = w + ((long long)a * N + b) * NN + (long long)((a - di) & NM) * N;
#pragma unroll
      for (int q = 0; q < 2; ++q) r.v[ks][q] = row[(b - dj0 - 16 * q - l16) & NM];
    }
  };
  // [h]: h = 0 the bin d_i (a >= d_i), h = 1 the bin d_i - N (a < d_i).
  v4f t1[2][R][2], t2[2][R][2], t3[2][R][2];
  float2 f[2][R][2][4], u1v[R][4];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        t1[h][r][q] = t2[h][r][q] = t3[h][r][q] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < 4; ++i) f[h][r][q][i] = float2{0.f, 0.f};
      }
  auto read_a = [&](float2 (&av)[4][R], int a0) {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int a = a0 + 4 * ks + kq;
#pragma unroll
      for (int r = 0; r < R; ++r) av[ks][r] = as_[a * kPairTile + ((k0 + 16 * r + l16) ^ ((a & 1) << 4))];
    }
  };
  auto step_mfma = [&](const float2 (&av)[4][R], const RingStep& bw, v4f (&s1)[R][2], v4f (&s2)[R][2],
                       v4f (&s3)[R][2]) {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      float xs[R], ys[2];
#pragma unroll
      for (int r = 0; r < R; ++r) xs[r] = av[ks][r].x + av[ks][r].y;
#pragma unroll
      for (int q = 0; q < 2; ++q) ys[q] = bw.v[ks][q].x + bw.v[ks][q].y;
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          s1[r][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ks][r].x, bw.v[ks][q].x, s1[r][q], 0, 0, 0);
          s2[r][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ks][r].y, bw.v[ks][q].y, s2[r][q], 0, 0, 0);
          s3[r][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(xs[r], ys[q], s3[r][q], 0, 0, 0);
        }
    }
  };
  // The lane's four bins of pair k: d_i bin h (row di + N, or di), d_j bin dj (upper) or dj - N (lower).
  float2* const out = part + (long long)z * kPairTile * BINS;
  auto bin_at = [&](int k, int h, int dj_bin) {
    return (long long)(k0 + k) * BINS + (long long)(h == 0 ? di + N : di) * (2 * N) + dj_bin + N;
  };
  RingStep ring[RING];
#pragma unroll
  for (int u = 0; u < RING - 1; ++u) {
    load(ring[u], u);
    __builtin_amdgcn_sched_barrier(0);
  }
  float2 avs[2][4][R];
  read_a(avs[0], 0);
  for (int t0 = 0; t0 < total; t0 += RING) {
#pragma unroll
    for (int u = 0; u < RING; ++u) {
      // Step of this b: known at compile time when the ring holds whole b (t0 a multiple of SPB), else
      // wavefront-uniform.
      const int sb = RING % SPB == 0 ? u % SPB : (t0 + u) % SPB;
      const int b = b_lo + (t0 + u) / SPB, a0 = sb * 16;
      load(ring[(u + RING - 1) % RING], t0 + u + RING - 1);
      if (sb == 0) {  // u1[k][b] of this b, behind the ring's load (it is needed at the fold)
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int i = 0; i < 4; ++i) u1v[r][i] = u1t[b * kPairTile + k0 + 16 * r + Mfma<float2>::row(lane, i)];
      }
      read_a(avs[(u + 1) % 2], ((sb + 1) % SPB) * 16);  // the next step's operand
      __builtin_amdgcn_sched_barrier(0);
      if (a0 >= di) {  // workgroup-uniform: every a of the step is in the bin d_i
        step_mfma(avs[u % 2], ring[u], t1[0], t2[0], t3[0]);
      } else if (a0 + 16 <= di) {  // every a is in the bin d_i - N
        step_mfma(avs[u % 2], ring[u], t1[1], t2[1], t3[1]);
      } else {  // the step holds d_i: each bin with the other bin's rows of A zeroed
        float2 am[4][R];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const bool upper = a0 + 4 * ks + kq >= di;
#pragma unroll
          for (int r = 0; r < R; ++r) am[ks][r] = upper ? avs[u % 2][ks][r] : float2{0.f, 0.f};
        }
        step_mfma(am, ring[u], t1[0], t2[0], t3[0]);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const bool upper = a0 + 4 * ks + kq >= di;
#pragma unroll
          for (int r = 0; r < R; ++r) am[ks][r] = upper ? float2{0.f, 0.f} : avs[u % 2][ks][r];
        }
        step_mfma(am, ring[u], t1[1], t2[1], t3[1]);
      }
      if (sb == SPB - 1) {  // the last step of b: D_h += u1[k][b] u2[k][b - dj] G_h, then the d_j switch
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int k = 16 * r + Mfma<float2>::row(lane, i);
#pragma unroll
            for (int q = 0; q < 2; ++q) {
              const int dj = dj0 + 16 * q + l16;
              const int m = (b - dj) & NM;
              const float2 c = cmul(u1v[r][i], u2s[m * kPairTile + ((k0 + k) ^ ((m & 15) << 1))]);
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                const float gr = t1[h][r][q][i] - t2[h][r][q][i];
                const float gi = t3[h][r][q][i] - t1[h][r][q][i] - t2[h][r][q][i];
                f[h][r][q][i].x += c.x * gr - c.y * gi;
                f[h][r][q][i].y += c.x * gi + c.y * gr;
              }
              if (b == dj - 1 && dj < b_hi) {  // every b below d_j is summed: the lower d_j bin is complete
                // (at dj = b_hi the sums stay held: the chunk ends there and stores them in the lower bin)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                  out[bin_at(k, h, dj - N)] = f[h][r][q][i];
                  f[h][r][q][i] = float2{0.f, 0.f};
                }
              }
            }
          }
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int r = 0; r < R; ++r)
#pragma unroll
            for (int q = 0; q < 2; ++q) t1[h][r][q] = t2[h][r][q] = t3[h][r][q] = v4f{0.f, 0.f, 0.f, 0.f};
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // The sums still held belong to the d_j bin of the chunk's last b; the other d_j bin was stored at the
  // switch, or has no term in this chunk (zero).
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = 16 * r + Mfma<float2>::row(lane, i);
        const int dj = dj0 + 16 * q + l16;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (dj >= b_hi) {  // every b of the chunk is below d_j
            out[bin_at(k, h, dj - N)] = f[h][r][q][i];
            out[bin_at(k, h, dj)] = float2{0.f, 0.f};
          } else {
            out[bin_at(k, h, dj)] = f[h][r][q][i];
            if (dj <= b_lo) out[bin_at(k, h, dj - N)] = float2{0.f, 0.f};  // no b of the chunk is below d_j
          }
        }
      }
}

// out[k][i] = f(k, i) sum_s part[s][k][i] (k < kcount), summed in FP64 in the order of s;
// f = u2[k][i / n] u2[k][i % n] when u2 is given (the row sums), else 1.
template <class T>
__global__ __launch_bounds__(256) void k_pair_sum(const T* __restrict__ part, int parts, int n, int kcount,
                                                  const T* __restrict__ u2, T* __restrict__ out) {
  using R = typename real_of<T>::type;
  const long long nn = (long long)n * n, total = (long long)kcount * nn;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  double2 acc{0.0, 0.0};
#pragma unroll 8
  for (int s = 0; s < parts; ++s) {
    const T v = part[(long long)s * total + e];
    acc.x += (double)v.x;
    acc.y += (double)v.y;
  }
  if (u2 != nullptr) {
    const long long k = e / nn, i = e - k * nn;
    const T f = cmul(u2[k * n + i / n], u2[k * n + i % n]);
    acc = cmul(acc, double2{(double)f.x, (double)f.y});
  }
  out[e] = T{(R)acc.x, (R)acc.y};
}

// One axis of the 2D DFT of every pair's N x N array, stored transposed:
// out[k][m][i] = sum_p e^{SIGN 2 pi i m p / N} in[k][i][p]. Applied twice it gives the 2D DFT in natural
// order. One workgroup per row (k, i): the row and the N roots (FP64-built) are staged in LDS.
template <class T, int SIGN>
__global__ __launch_bounds__(256) void k_pair_dft(const T* __restrict__ in, int n, T* __restrict__ out) {
  using R = typename real_of<T>::type;
  __shared__ T row[256], tw[256];
  const long long nn = (long long)n * n;
  const long long k = blockIdx.x / n, i = blockIdx.x % n;
  for (int p = threadIdx.x; p < n; p += blockDim.x) {
    row[p] = in[k * nn + i * n + p];
    tw[p] = twiddle_entry<T, SIGN>(p, n);
  }
  __syncthreads();
  for (int m = threadIdx.x; m < n; m += blockDim.x) {
    T acc{(R)0, (R)0};
    int idx = 0;
    for (int p = 0; p < n; ++p) {
      const T t = cmul(tw[idx], row[p]);
      acc.x += t.x;
      acc.y += t.y;
      idx += m;
      if (idx >= n) idx -= n;
    }
    out[k * nn + (long long)m * n + i] = acc;
  }
}

// S and mu(P, .) of up to kPairTile pairs in one launch (emit_observables), from the raw sums of pair
// k (shared: the same sums for every pair, in the far field).
struct PairEmit {
  int count;
  double c[kPairTile];      // s * weight of each pair
  double a_out[kPairTile];  // output chirp rate of each pair
};

template <class T>
__global__ __launch_bounds__(256) void k_pair_emit(const typename real_of<T>::type* __restrict__ s0,
                                                   const T* __restrict__ b0, const unsigned long long* key, int shared,
                                                   int n, int pi, int pj, PairEmit pe, double floor_rel,
                                                   typename real_of<T>::type* __restrict__ s_out, T* __restrict__ mu_out) {
  const long long nn = (long long)n * n;
  const int k = blockIdx.y;
  const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nn || k >= pe.count) return;
  const long long so = shared ? 0 : k * nn;
  const Chirp post1{pe.a_out[k], 1.0, -1, 1}, post2{pe.a_out[k], 1.0, +1, 1};
  emit_observables(s0 + so, b0 + so, key[shared ? 0 : k], n, pi, pj, m, pe.c[k], post1, post2, floor_rel,
                   s_out + k * nn, mu_out + k * nn);
}

// s0[k][m] = Re z[k][m] and key[k] = order key of max_m s0[k][m]: blockIdx.y is the pair, blockIdx.x one of
// gridDim.x ranges of m; the ranges' maxima meet in an atomic max on the order keys (order-independent),
// which k_pair_clear_keys has zeroed.
__global__ void k_pair_clear_keys(unsigned long long* key, int count) {
  if ((int)threadIdx.x < count) key[threadIdx.x] = 0ull;
}

template <class T>
__global__ __launch_bounds__(256) void k_pair_s0(const T* __restrict__ z, int n, typename real_of<T>::type* s0,
                                                 unsigned long long* key) {
  using R = typename real_of<T>::type;
  __shared__ double red[256];
  const long long nn = (long long)n * n;
  const long long k = blockIdx.y;
  const long long len = (nn + gridDim.x - 1) / gridDim.x, m0 = blockIdx.x * len;
  const long long m1 = m0 + len < nn ? m0 + len : nn;
  double mx = -INFINITY;
  for (long long m = m0 + threadIdx.x; m < m1; m += blockDim.x) {
    const R v = z[k * nn + m].x;
    s0[k * nn + m] = v;
    mx = fmax(mx, (double)v);
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0 && m0 < m1) atomicMax(&key[k], order_key(red[0]));
}

// Ranges of m per pair in k_pair_s0: about 4096 elements each.
static unsigned s0_ranges(int n) {
  const long long nn = (long long)n * n;
  return (unsigned)((nn + 4095) / 4096);
}

// ---------------------------------------------------------------------------------------------
// Polychromatic sums on a common output grid of any pitch (the chirp-z form of the same sums).
// With the plain chirp t_k[a] = e^{i pi alpha_k (a - c)^2} (alpha_k = pitch^2 / (lambda_k z_k), 0 in the far
// field) and the DFT frequency beta_k = out_pitch pitch / (lambda_k z_k) (1/N on the FFT grid):
//   S_k(m)     = s_k Re sum_{d in [-N, N)^2} e^{+2 pi i beta_k <m - c, d>} D_k[d],
//   D_k[d]     = sum_{p1 : p1 - d in [0, N)^2} conj(T_k[p1]) T_k[p1 - d] W[p1; p1 - d]   (no wrap),
//   W_k[P; m]  = s_k conj(tau_k(P)) tau_k(m) sum_{p2} e^{-2 pi i beta_k <m - c, p2 - c>} T_k[p2] R_k[p2],
//   R_k[p2]    = sum_{p1} e^{+2 pi i beta_k <P - c, p1 - c>} conj(T_k[p1]) W[p1; p2],
// tau_k(m) = e^{i pi gamma_k (m - c)^2}, gamma_k = out_pitch^2 / (lambda_k z_k); then S = sum_k w_k S_k and
// W[P; .] = sum_k w_k W_k[P; .] (R17). The output grid no longer has the period N of the DFT, so the
// difference sums keep both signs of d: bins d in [-N, N), index d + N.
// ---------------------------------------------------------------------------------------------
struct PolyGroup {
  int count;
  double alpha[kPairTile];  // source chirp rate of each pair
  double beta[kPairTile];   // DFT frequency of each pair on the common grid
  double gamma[kPairTile];  // output chirp rate of each pair on the common grid
  double c[kPairTile];      // weight * s of each pair
};

// u1 = conj(t), u2 = t, ci = e^{2 pi i beta (P_i - c)(a - c)} conj(t[a]), cj likewise with P_j (FP64-built).
template <class T>
__global__ __launch_bounds__(256) void k_poly_tables(PolyGroup g, int n, int pi, int pj, T* u1, T* u2, T* ci, T* cj,
                                                     T* tr) {
  using R = typename real_of<T>::type;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kPairTile * n) return;
  const int k = e / n, a = e % n, c = n / 2;
  if (k >= g.count) {
    const T z{(R)0, (R)0};
    store_tables(u1, u2, ci, cj, tr, n, k, a, z, z, z, z);
    return;
  }
  const double2 t = chirp_entry<double2>(Chirp{g.alpha[k], 1.0, +1, 0}, a, n);
  const double2 tc{t.x, -t.y};
  double pr = g.beta[k] * (double)(pi - c) * (double)(a - c);
  double ps = g.beta[k] * (double)(pj - c) * (double)(a - c);
  pr -= rint(pr);
  ps -= rint(ps);
  double si, co, sj, cjx;
  sincospi(2.0 * pr, &si, &co);
  sincospi(2.0 * ps, &sj, &cjx);
  const double2 wi = cmul(double2{co, si}, tc), wj = cmul(double2{cjx, sj}, tc);
  store_tables(u1, u2, ci, cj, tr, n, k, a, T{(R)tc.x, (R)tc.y}, T{(R)t.x, (R)t.y}, T{(R)wi.x, (R)wi.y},
               T{(R)wj.x, (R)wj.y});
}

// Difference sums without wrap: part[z][k][(di + N) 2N + dj + N] = sum_b B_k^{dj}[b] sum_a A_k^{di}[a]
// W[a, b; a - di, b - dj] over a - di, b - dj in [0, N), A = u1[a] u2[a - di], B = u1[b] u2[b - dj]
// (di, dj in [-N, N)). They are taken in the folded order of k_pair_diffs_mfma, with no wasted rows: for a
// folded offset
// (d_i, d_j) in [0, N)^2 the folded sum over a and b splits exactly into the unfolded bins. On the first
// point, a >= d_i belongs to bin d_i and a < d_i to bin d_i - N (the workgroup's half h takes one of the
// two a ranges); on the second point, b >= d_j belongs to bin d_j and b < d_j to bin d_j - N. As b rises
// through the workgroup's chunk, a lane's column d_j switches bin once: the lane stores the lower bin's
// sum when b passes d_j - 1 and writes each of its two bins exactly once. For the first TM pairs.
template <class T, int TM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 3 : 2))) void k_poly_diffs_mfma(
    const T* __restrict__ w, int n, const T* __restrict__ u1, const T* __restrict__ u2,
    const T* __restrict__ u1t, const T* __restrict__ u2t, int bchunk, T* __restrict__ part) {
  using R = typename real_of<T>::type;
  using G = MTile<TM>;
  using M = MStage<TM>;
  constexpr int TK = 16;
  __shared__ R ar[2][TK][G::LDA], ai[2][TK][G::LDA], br[2][TK][G::LDB], bi[2][TK][G::LDB];
  const long long nn = (long long)n * n, bins = 4 * nn;
  const int tid = threadIdx.x, lane = tid % 64;
  const int wv = __builtin_amdgcn_readfirstlane(tid / 64);  // wavefront-uniform
  const int row0 = (wv / G::WC) * 32, col0 = (wv % G::WC) * 32;
  const int dj0 = blockIdx.x * G::TN, nm = n - 1;             // N is a power of two
  const int h = (int)blockIdx.y & 1, di = (int)blockIdx.y >> 1;  // h = 0: a >= d_i; h = 1: a < d_i
  const int a_lo = h ? 0 : di, a_hi = h ? di : n;
  const int b_lo = blockIdx.z * bchunk, b_hi = (b_lo + bchunk < n) ? b_lo + bchunk : n;
  T* out = part + (long long)blockIdx.z * kPairTile * bins + (long long)(h ? di : di + n) * (2 * n) + n;
  R dre[2][2][4], dim[2][2][4];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) dre[r][q][i] = dim[r][q][i] = (R)0;
  T rb[G::QB], ca[G::QA], cb[G::QA];
  auto fetch = [&](int b, int a0) {  // W[a, b; a - di, b - dj] (indices mod N) and the tables of A
#pragma unroll
    for (int q = 0; q < G::QB; ++q) {
      const int a = a0 + M::b_row(wv, q), dj = dj0 + M::b_col(wv, lane);
      rb[q] = load_or_first(w, a < a_hi && dj < n,
                            ((long long)a * n + b) * nn + (long long)((a - di) & nm) * n + ((b - dj) & nm));
    }
#pragma unroll
    for (int q = 0; q < G::QA; ++q) {  // A[kk][k] = u1[k][a] u2[k][a - di]
      const int a = a0 + M::a_row(tid, wv, q), k = M::a_pair(tid, lane);
      const int ac = a < a_hi ? a : a_lo;
      ca[q] = u1t[ac * kPairTile + k];
      cb[q] = u2t[((ac - di) & nm) * kPairTile + k];
    }
  };
  auto stage = [&](int buf, int a0) {
#pragma unroll
    for (int q = 0; q < G::QB; ++q) {
      const int kk = M::b_row(wv, q), jj = M::b_col(wv, lane);
      const T v = keep_or_zero(a0 + kk < a_hi && dj0 + jj < n, rb[q]);
      br[buf][kk][jj] = v.x;
      bi[buf][kk][jj] = v.y;
    }
#pragma unroll
    for (int q = 0; q < G::QA; ++q) {
      const int kk = M::a_row(tid, wv, q), k = M::a_pair(tid, lane);
      const T a = keep_or_zero(a0 + kk < a_hi, cmul(ca[q], cb[q]));
      ar[buf][kk][k] = a.x;
      ai[buf][kk][k] = a.y;
    }
  };
  const bool any = a_lo < a_hi && b_lo < b_hi;
  if (any) {
    fetch(b_lo, a_lo);
    stage(0, a_lo);
  }
  __syncthreads();
  CTile<T> g;
  ctile_zero(g);
  int buf = 0;
  for (int b = b_lo, a0 = a_lo; any && b < b_hi;) {
    const bool last_a = a0 + TK >= a_hi;
    const int nb = last_a ? b + 1 : b, na = last_a ? a_lo : a0 + TK;
    const bool more = nb < b_hi;
    if (more) fetch(nb, na);
    ctile_mfma16<T, G::LDA, G::LDB>(g, ar[buf], ai[buf], br[buf], bi[buf], row0, col0, lane);
    if (last_a) {
      // D += B_k^{dj}[b] G, B = u1[k][b] u2[k][b - dj]; at b = dj - 1 the lower bin d_j - N is complete.
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int k = row0 + 16 * r + Mfma<T>::row(lane, i);
          const T ub = u1[k * n + b];
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int dj = dj0 + col0 + 16 * q + lane % 16;
            const T f = cmul(ub, u2[k * n + ((b - dj) & nm)]);
            const R gr = g.re(r, q, i), gi = g.im(r, q, i);
            dre[r][q][i] += f.x * gr - f.y * gi;
            dim[r][q][i] += f.x * gi + f.y * gr;
            if (b == dj - 1 && dj < b_hi && dj < n) {
              out[(long long)k * bins + dj - n] = T{dre[r][q][i], dim[r][q][i]};
              dre[r][q][i] = dim[r][q][i] = (R)0;
            }
          }
        }
      ctile_zero(g);
    }
    if (more) stage(buf ^ 1, na);
    __syncthreads();
    buf ^= 1;
    b = nb;
    a0 = na;
  }
  // Each lane writes both of its bins once: the sum it holds goes to the bin of the chunk's last b; the
  // other bin was stored at the switch, or has no term in this chunk.
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const long long k = row0 + 16 * r + Mfma<T>::row(lane, i);
        const int dj = dj0 + col0 + 16 * q + lane % 16;
        if (dj >= n) continue;
        const T v{dre[r][q][i], dim[r][q][i]}, z{(R)0, (R)0};
        if (!any || dj >= b_hi) {  // every b of the chunk is below dj (or there is no term at all)
          out[k * bins + dj - n] = v;
          out[k * bins + dj] = z;
        } else {
          out[k * bins + dj] = v;
          if (dj <= b_lo) out[k * bins + dj - n] = z;  // no b of the chunk is below dj
        }
      }
}

// Block of the one-pass sums: (column tile, slab range). The hardware deals consecutive workgroups to the
// 8 XCDs in turn, so the linear index is remapped to put every column tile of one slab range on one XCD:
// the slab's rows that a tile gathers for D were read for R by another tile of the same range, and are
// then found in that XCD's L2 (with the x-fastest order each XCD held one column tile of every range, and
// the gathered rows came from the other XCDs' reads). Identity where the ranges are not a multiple of 8.
struct OneBlock {
  int x, y;
};
__device__ __forceinline__ OneBlock one_block() {
  const int gx = (int)gridDim.x, gy = (int)gridDim.y;
  if (gy % 8 != 0) return OneBlock{(int)blockIdx.x, (int)blockIdx.y};
  const int l = (int)blockIdx.x + gx * (int)blockIdx.y;
  return OneBlock{(l / 8) % gx, l % 8 + 8 * (l / (8 * gx))};
}

// The polychromatic sums of a group of one pair in one pass over the source, as k_one_sums: R as there,
// and the unfolded difference sums D[d], d in [-N, N)^2. The element W[p1; p1 - d] of a thread's folded
// column d = (d_i, d_j) belongs to the unfolded bin (a >= d_i ? d_i : d_i - N, b >= d_j ? d_j : d_j - N);
// each thread keeps the four bins of each of its columns. part_d[y][(d_i + N) 2N + d_j + N].
template <class T>
__global__ __launch_bounds__(kOneThreads) void k_one_poly_sums(const T* __restrict__ w, int n,
                                                              const T* __restrict__ u1, const T* __restrict__ u2,
                                                              const T* __restrict__ ci, const T* __restrict__ cj,
                                                              int slabs, T* __restrict__ part_r,
                                                              T* __restrict__ part_d) {
  using R = typename real_of<T>::type;
  __shared__ T su2[256];
  const int nn = n * n, nm = n - 1, lg = __builtin_ctz((unsigned)n);  // N is a power of two
  const int tid = threadIdx.x;
  for (int i = tid; i < n; i += kOneThreads) su2[i] = u2[i];
  __syncthreads();
  const OneBlock ob = one_block();
  const int c0 = ob.x * kOneThreads * kOneCols + tid;
  const int di0 = c0 >> lg, dj0 = c0 & nm, step = kOneThreads >> lg;
  const int p_lo = ob.y * slabs, p_hi = p_lo + slabs < nn ? p_lo + slabs : nn;
  const T zero{(R)0, (R)0};
  T r[kOneCols], d[4][kOneCols];  // d[2 (a < d_i) + (b < d_j)][j]
#pragma unroll
  for (int j = 0; j < kOneCols; ++j) r[j] = d[0][j] = d[1][j] = d[2][j] = d[3][j] = zero;
  for (int p1 = p_lo; p1 < p_hi; ++p1) {
    const int a = p1 >> lg, b = p1 & nm;
    const T cr = cmul(ci[a], cj[b]), cu = cmul(u1[a], u1[b]);
    const T* slab = w + (long long)p1 * nn;
    const int b2 = (b - dj0) & nm;
    T xr[kOneCols], xd[kOneCols];
#pragma unroll
    for (int j = 0; j < kOneCols; ++j) {
      const int i = c0 + kOneThreads * j;
      xr[j] = load_or_first(slab, i < nn, i);
      xd[j] = load_or_first(slab, i < nn, ((a - di0 - step * j) & nm) * n + b2);
    }
#pragma unroll
    for (int j = 0; j < kOneCols; ++j) {
      const T t = cmul(cr, xr[j]);
      r[j].x += t.x;
      r[j].y += t.y;
    }
    const T ub = cmul(cu, su2[b2]);
    const int lb = b < dj0 ? 1 : 0;
#pragma unroll
    for (int j = 0; j < kOneCols; ++j) {
      const int a2 = (a - di0 - step * j) & nm;
      const T t = cmul(cmul(ub, su2[a2]), xd[j]);
      const int qd = (a < di0 + step * j ? 2 : 0) + lb;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        d[q][j].x += q == qd ? t.x : (R)0;
        d[q][j].y += q == qd ? t.y : (R)0;
      }
    }
  }
  T* orr = part_r + (long long)ob.y * nn;
  T* odd = part_d + (long long)ob.y * 4 * nn;
#pragma unroll
  for (int j = 0; j < kOneCols; ++j) {
    const int i = c0 + kOneThreads * j;
    if (i >= nn) continue;
    orr[i] = r[j];
    const int di = di0 + step * j;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int du = (q & 2) ? di - n : di, ju = (q & 1) ? dj0 - n : dj0;
      odd[(long long)(du + n) * (2 * n) + ju + n] = d[q][j];
    }
  }
}

// One axis of a chirp-z transform of every pair's array, stored transposed:
// out[k][m][i] = sum_{p < len} e^{SIGN 2 pi i beta_k (m - c)(p - off)} in[k][i][p], m < N, i < rows. The
// factors come from an FP64 recurrence along p (one FP64 product per term); sums in FP64.
template <class T, int SIGN>
__global__ __launch_bounds__(256) void k_poly_czt(const T* __restrict__ in, int n, int rows, int len, int off,
                                                  PolyGroup g, T* __restrict__ out) {
  using R = typename real_of<T>::type;
  __shared__ T row[512];
  const int k = blockIdx.x / rows, i = blockIdx.x % rows, c = n / 2;
  const long long inb = ((long long)k * rows + i) * len;
  for (int p = threadIdx.x; p < len; p += blockDim.x) row[p] = in[inb + p];
  __syncthreads();
  const double beta = k < g.count ? g.beta[k] : 0.0;
  for (int m = threadIdx.x; m < n; m += blockDim.x) {
    double f0 = (double)SIGN * beta * (double)(m - c) * (double)(0 - off);
    double fs = (double)SIGN * beta * (double)(m - c);
    f0 -= rint(f0);
    fs -= rint(fs);
    double s0, c0, s1, c1;
    sincospi(2.0 * f0, &s0, &c0);
    sincospi(2.0 * fs, &s1, &c1);
    double2 wv{c0, s0};
    const double2 rot{c1, s1};
    double2 acc{0.0, 0.0};
    for (int p = 0; p < len; ++p) {
      const T v = row[p];
      acc.x += wv.x * (double)v.x - wv.y * (double)v.y;
      acc.y += wv.x * (double)v.y + wv.y * (double)v.x;
      wv = cmul(wv, rot);
    }
    out[((long long)k * n + m) * rows + i] = T{(R)acc.x, (R)acc.y};
  }
}

// S(m) (+)= sum_k c_k Re zd_k[m]; W(m) (+)= sum_k c_k conj(tau_k(P)) tau_k(m) zr_k[m], in FP64, pairs in order.
template <class T>
__global__ __launch_bounds__(256) void k_poly_combine(const T* __restrict__ zd, const T* __restrict__ zr, int n,
                                                      int pi, int pj, PolyGroup g, int first, double* s_acc,
                                                      double2* w_acc) {
  const long long nn = (long long)n * n;
  const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nn) return;
  const int mi = (int)(m / n), mj = (int)(m % n);
  double s = 0.0;
  double2 wr{0.0, 0.0};
  for (int k = 0; k < g.count; ++k) {
    const Chirp ch{g.gamma[k], 1.0, +1, 0};
    const double2 tp = cmul(chirp_entry<double2>(ch, pi, n), chirp_entry<double2>(ch, pj, n));
    const double2 tm = cmul(chirp_entry<double2>(ch, mi, n), chirp_entry<double2>(ch, mj, n));
    const double2 ph = cmul(double2{tp.x, -tp.y}, tm);
    const T d = zd[k * nn + m], r = zr[k * nn + m];
    s += g.c[k] * (double)d.x;
    const double2 v = cmul(ph, double2{(double)r.x, (double)r.y});
    wr.x += g.c[k] * v.x;
    wr.y += g.c[k] * v.y;
  }
  if (first) {
    s_acc[m] = s;
    w_acc[m] = wr;
  } else {
    s_acc[m] += s;
    w_acc[m] = double2{w_acc[m].x + wr.x, w_acc[m].y + wr.y};
  }
}

// S and mu(P, .) from the sums: one workgroup, the maximum of S by a fixed tree.
template <class T>
__global__ __launch_bounds__(1024) void k_poly_mu(const double* __restrict__ s_acc, const double2* __restrict__ w_acc,
                                                  int n, int pi, int pj, double floor_rel,
                                                  typename real_of<T>::type* __restrict__ s_out, T* __restrict__ mu_out) {
  using R = typename real_of<T>::type;
  __shared__ double red[1024];
  const long long nn = (long long)n * n;
  double mx = -INFINITY;
  for (long long m = threadIdx.x; m < nn; m += blockDim.x) mx = fmax(mx, s_acc[m]);
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  const double tau = floor_rel * red[0], sp = s_acc[(long long)pi * n + pj];
  for (long long m = threadIdx.x; m < nn; m += blockDim.x) {
    const double sm = s_acc[m];
    s_out[m] = (R)sm;
    T o{(R)0, (R)0};
    if (sp > tau && sm > tau) {
      const double d = sqrt(sp) * sqrt(sm);
      o = T{(R)(w_acc[m].x / d), (R)(w_acc[m].y / d)};
    }
    mu_out[m] = o;
  }
}

// ---------------------------------------------------------------------------------------------
// One set of sums (a group of one entry: the far field, whose sums every pair shares, or a single
// pair). With one row the two contractions are matrix-vector products, bound by HBM, and both come
// from one pass over the source. A workgroup takes a range of slabs p1 and a block of columns; each
// thread keeps kOneCols columns i of both raw sums in registers:
//   R[i] += ci[a] cj[b] W[p1; i]                                  (the row sums with one row)
//   D[i] += u1[a] u1[b] u2[a - d_i] u2[b - d_j] W[p1; p1 - d], d = i  (the difference sums; indices mod N)
// The read of a slab for D finds it in the caches after the read for R.
// ---------------------------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(kOneThreads) void k_one_sums(const T* __restrict__ w, int n, const T* __restrict__ u1,
                                                         const T* __restrict__ u2, const T* __restrict__ ci,
                                                         const T* __restrict__ cj, int slabs, T* __restrict__ part_r,
                                                         T* __restrict__ part_d) {
  using R = typename real_of<T>::type;
  __shared__ T su2[256];
  const int nn = n * n, nm = n - 1, lg = __builtin_ctz((unsigned)n);  // N is a power of two
  const int tid = threadIdx.x;
  for (int i = tid; i < n; i += kOneThreads) su2[i] = u2[i];
  __syncthreads();
  const OneBlock ob = one_block();
  const int c0 = ob.x * kOneThreads * kOneCols + tid;
  // Column i = c0 + kOneThreads j is d = (di0 + step j, dj0): kOneThreads is a multiple of N.
  const int di0 = c0 >> lg, dj0 = c0 & nm, step = kOneThreads >> lg;
  const int p_lo = ob.y * slabs, p_hi = p_lo + slabs < nn ? p_lo + slabs : nn;
  const T zero{(R)0, (R)0};
  T r[kOneCols], d[kOneCols];
#pragma unroll
  for (int j = 0; j < kOneCols; ++j) r[j] = d[j] = zero;
  for (int p1 = p_lo; p1 < p_hi; ++p1) {
    const int a = p1 >> lg, b = p1 & nm;
    const T cr = cmul(ci[a], cj[b]), cu = cmul(u1[a], u1[b]);
    const T* slab = w + (long long)p1 * nn;
    const int b2 = (b - dj0) & nm;
    T xr[kOneCols], xd[kOneCols];  // both reads of the slab in flight together
#pragma unroll
    for (int j = 0; j < kOneCols; ++j) {
      const int i = c0 + kOneThreads * j;
      xr[j] = load_or_first(slab, i < nn, i);
      xd[j] = load_or_first(slab, i < nn, ((a - di0 - step * j) & nm) * n + b2);
    }
#pragma unroll
    for (int j = 0; j < kOneCols; ++j) {
      const T t = cmul(cr, xr[j]);
      r[j].x += t.x;
      r[j].y += t.y;
    }
    const T ub = cmul(cu, su2[b2]);
#pragma unroll
    for (int j = 0; j < kOneCols; ++j) {
      const int a2 = (a - di0 - step * j) & nm;
      const T t = cmul(cmul(ub, su2[a2]), xd[j]);
      d[j].x += t.x;
      d[j].y += t.y;
    }
  }
  T* orr = part_r + (long long)ob.y * nn;
  T* odd = part_d + (long long)ob.y * nn;
#pragma unroll
  for (int j = 0; j < kOneCols; ++j) {
    const int i = c0 + kOneThreads * j;
    if (i < nn) {
      orr[i] = r[j];
      odd[i] = d[j];
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Work layout (per group of kPairTile pairs), in elements of T unless noted.
// ---------------------------------------------------------------------------------------------
static int pair_tiles_j(int n) { return (n + 63) / 64; }
// Chunks of b in the difference sums: about 3072 workgroups (a few rounds of the resident slots, so that
// the last round does not run on a fraction of the chip; measured 2 % faster than 1024 at N = 128).
static int pair_bsplit(int n) {
  int sb = (3072 + pair_tiles_j(n) * n - 1) / (pair_tiles_j(n) * n);
  if (sb < 4) sb = 4;
  if (sb > n) sb = n;
  return sb;
}

// The matrix-core contractions of one group: tiles of 32 pairs x 128 columns when a complex64 group has
// at most 32 pairs, else 64 x 64 (complex128 always; its FP64 operands fill the LDS twice as fast). kind 0:
// row sums; 1: Fresnel difference sums; 2: the polychromatic (unfolded) difference sums. The tables tr are
// [4][N][kPairTile] (u1, u2, ci, cj).
template <class T, int TM>
static hipError_t launch_mfma_tm(int kind, int n, const T* w, const T* u1, const T* u2, const T* tr, long long chunk,
                                 int bchunk, int sb, T* part, hipStream_t st) {
  constexpr int TN = MTile<TM>::TN;
  const long long nn = (long long)n * n, tq = (long long)kPairTile * n;
  const unsigned tiles_j = (unsigned)((n + TN - 1) / TN);
  if (kind == 0)
    hipLaunchKernelGGL((k_pair_rows_mfma<T, TM>), dim3((unsigned)((nn + TN - 1) / TN), kPairSplitK), dim3(256), 0, st,
                       w, n, tr + 2 * tq, tr + 3 * tq, chunk, part);
  else if (kind == 1)
    hipLaunchKernelGGL((k_pair_diffs_mfma<T, TM>), dim3(tiles_j, (unsigned)n, (unsigned)sb), dim3(256), 0, st, w, n,
                       u1, u2, tr, tr + tq, bchunk, part);
  else  // folded offsets: (tiles of d_j in [0, N)) x (d_i in [0, N), two halves of the a range) x (b chunks)
    hipLaunchKernelGGL((k_poly_diffs_mfma<T, TM>), dim3(tiles_j, (unsigned)(2 * n), (unsigned)sb), dim3(256), 0, st,
                       w, n, u1, u2, tr, tr + tq, bchunk, part);
  return hipGetLastError();
}

// The ring form of the row sums (complex64, N = 64 or 128, any count): the number of chunks of p1 it writes
// (256 workgroups over the N^2 / 128 column tiles), or 0 where it does not apply.
static int rows_ring_parts(int n, int count) {
  if (count < 1 || (n != 64 && n != 128)) return 0;
  return 256 / (n * n / 128);
}

// The ring form of the Fresnel difference sums (complex64, N = 128, any count) writes 256 / N chunks of b.
static bool diffs_ring_ok(int n, int count) { return n == 128 && count >= 1; }

// The ring form of the polychromatic difference sums (complex64, N = 128, any count) writes 256 / N chunks
// of b.
static bool poly_diffs_ring_ok(int n, int count) { return n == 128 && count >= 1; }

template <class T>
static hipError_t launch_mfma(int count, int kind, int n, const T* w, const T* u1, const T* u2, const T* tr,
                              long long chunk, int bchunk, int sb, T* part, hipStream_t st) {
  if constexpr (sizeof(T) == 8) {
    const long long nn = (long long)n * n, tq = (long long)kPairTile * n;
    if (kind == 0 && rows_ring_parts(n, count) > 0) {
      // One workgroup per CU (the tables take 2 x N x 64 complex of LDS): 256 items of one 128-column tile
      // and one of rows_ring_parts chunks of p1, so the chunk sums are few partials.
      const int parts = rows_ring_parts(n, count);
      const long long ring_chunk = nn / parts;
      using RowsRing = void (*)(const float2*, const float2*, const float2*, long long, int, float2*);
      const RowsRing rows = n == 64 ? (count > 32 ? k_pair_rows_ring<64, 4>
                                                  : count > 16 ? k_pair_rows_ring<64, 2> : k_pair_rows_ring<64, 1>)
                                    : (count > 32 ? k_pair_rows_ring<128, 4>
                                                  : count > 16 ? k_pair_rows_ring<128, 2> : k_pair_rows_ring<128, 1>);
      hipLaunchKernelGGL(rows, dim3(256), dim3(256), 0, st, w, tr + 2 * tq, tr + 3 * tq, ring_chunk, 256, part);
      return hipGetLastError();
    }
    if (kind == 1 && diffs_ring_ok(n, count)) {
      using DiffsRing = void (*)(const float2*, const float2*, const float2*, float2*);
      const DiffsRing diffs = count > 32   ? k_pair_diffs_ring<128, 4>
                              : count > 16 ? k_pair_diffs_ring<128, 2>
                                           : k_pair_diffs_ring<128, 1>;
      hipLaunchKernelGGL(diffs, dim3(256), dim3(256), 0, st, w, tr, tr + tq, part);
      return hipGetLastError();
    }
    if (kind == 2 && poly_diffs_ring_ok(n, count)) {
      if (count <= 16) {
        hipLaunchKernelGGL((k_poly_diffs_ring<128, 1, 8>), dim3(256), dim3(256), 0, st, w, tr, tr + tq, 0, part);
      } else {  // tiles of 32 pairs, one launch each
        for (int k0 = 0; k0 < count; k0 += 32)
          hipLaunchKernelGGL((k_poly_diffs_ring<128, 2, 4>), dim3(256), dim3(256), 0, st, w, tr, tr + tq, k0, part);
      }
      return hipGetLastError();
    }
    if (count <= 32) return launch_mfma_tm<T, 32>(kind, n, w, u1, u2, tr, chunk, bchunk, sb, part, st);
  }
  return launch_mfma_tm<T, 64>(kind, n, w, u1, u2, tr, chunk, bchunk, sb, part, st);
}

template <class T> size_t pair_work_bytes(int n) {
  using R = typename real_of<T>::type;
  const size_t nn = (size_t)n * n, g = (size_t)kPairTile * nn;
  const size_t elems = 8 * (size_t)kPairTile * n + (size_t)kPairSplitK * g + (size_t)pair_bsplit(n) * g + 3 * g;
  return elems * sizeof(T) + g * sizeof(R) + kPairTile * sizeof(unsigned long long) + 256;
}

template <class T>
hipError_t launch_pair_sums(int n, const T* w, const double* a_src, int count, int pi, int pj, void* work,
                            ObsSums<T>* out, hipStream_t st) {
  using R = typename real_of<T>::type;
  if (count < 1 || count > kPairTile) return hipErrorInvalidValue;
  const long long nn = (long long)n * n, g = (long long)kPairTile * nn;
  T* base = reinterpret_cast<T*>(work);
  T* u1 = base;
  T* u2 = u1 + kPairTile * n;
  T* ci = u2 + kPairTile * n;
  T* cj = ci + kPairTile * n;
  T* tr = cj + kPairTile * n;  // u1, u2, ci, cj transposed
  const long long tq = (long long)kPairTile * n;
  T* part_r = tr + 4 * tq;
  const int sb = pair_bsplit(n);
  T* part_d = part_r + (long long)kPairSplitK * g;
  T* buf_d = part_d + (long long)sb * g;  // D, then the 2D DFT of D
  T* buf_t = buf_d + g;                   // transposed intermediate of the DFTs
  T* buf_r = buf_t + g;                   // u2 R, then b0
  R* s0 = reinterpret_cast<R*>(buf_r + g);
  unsigned long long* key = reinterpret_cast<unsigned long long*>(
      (reinterpret_cast<uintptr_t>(s0 + g) + 7) & ~(uintptr_t)7);

  PairGroup pg{};
  pg.count = count;
  for (int k = 0; k < count; ++k) pg.a_src[k] = a_src[k];
  hipLaunchKernelGGL(k_pair_tables<T>, dim3((unsigned)((kPairTile * n + 255) / 256)), dim3(256), 0, st, pg, n, pi, pj,
                     u1, u2, ci, cj, tr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (count == 1) {  // one row: both sums in one pass, HBM-bound
    const int ranges = nn < 256 ? (int)nn : 256;  // slab ranges; partials fit: 64 sb >= 256 or nn
    const int slabs = (int)((nn + ranges - 1) / ranges);
    const dim3 grid((unsigned)((nn + kOneThreads * kOneCols - 1) / (kOneThreads * kOneCols)), (unsigned)ranges);
    hipLaunchKernelGGL(k_one_sums<T>, grid, dim3(kOneThreads), 0, st, w, n, (const T*)u1, (const T*)u2,
                       (const T*)ci, (const T*)cj, slabs, part_r, part_d);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const unsigned blocks = (unsigned)((nn + 255) / 256);
    hipLaunchKernelGGL(k_pair_sum<T>, dim3(blocks), dim3(256), 0, st, (const T*)part_r, ranges, n, 1, (const T*)u2,
                       buf_r);
    hipLaunchKernelGGL(k_pair_sum<T>, dim3(blocks), dim3(256), 0, st, (const T*)part_d, ranges, n, 1,
                       (const T*)nullptr, buf_d);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((k_pair_dft<T, +1>), dim3((unsigned)n), dim3(256), 0, st, (const T*)buf_d, n, buf_t);
    hipLaunchKernelGGL((k_pair_dft<T, +1>), dim3((unsigned)n), dim3(256), 0, st, (const T*)buf_t, n, buf_d);
    hipLaunchKernelGGL((k_pair_dft<T, -1>), dim3((unsigned)n), dim3(256), 0, st, (const T*)buf_r, n, buf_t);
    hipLaunchKernelGGL((k_pair_dft<T, -1>), dim3((unsigned)n), dim3(256), 0, st, (const T*)buf_t, n, buf_r);
    hipLaunchKernelGGL(k_pair_clear_keys, dim3(1), dim3(64), 0, st, key, 1);
    hipLaunchKernelGGL(k_pair_s0<T>, dim3(s0_ranges(n), 1), dim3(256), 0, st, (const T*)buf_d, n, s0, key);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    out[0] = ObsSums<T>{s0, buf_r, key};
    return hipSuccess;
  }
  const long long chunk = (nn + kPairSplitK - 1) / kPairSplitK;
  const int bchunk = (n + sb - 1) / sb;
  if ((e = launch_mfma<T>(count, 0, n, w, u1, u2, tr, chunk, bchunk, sb, part_r, st)) != hipSuccess) return e;
  e = launch_mfma<T>(count, 1, n, w, u1, u2, tr, chunk, bchunk, sb, part_d, st);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const unsigned sum_blocks = (unsigned)((g + 255) / 256);
  const int sr = (sizeof(T) == 8 && rows_ring_parts(n, count) > 0) ? rows_ring_parts(n, count) : kPairSplitK;
  hipLaunchKernelGGL(k_pair_sum<T>, dim3(sum_blocks), dim3(256), 0, st, (const T*)part_r, sr, n, kPairTile,
                     (const T*)u2, buf_r);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int sd = (sizeof(T) == 8 && diffs_ring_ok(n, count)) ? 256 / n : sb;  // chunks of b written
  hipLaunchKernelGGL(k_pair_sum<T>, dim3(sum_blocks), dim3(256), 0, st, (const T*)part_d, sd, n, kPairTile,
                     (const T*)nullptr, buf_d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const unsigned rows = (unsigned)(count * n);  // the group's pairs only
  // s0 = Re F D F^T with the + sign; b0 = F* (u2 R) F*^T: FFT passes in place where the group's rows fill
  // whole row-pass workgroups, else the direct DFT kernel (transposed twice).
  if (dft2_batch_ok(n, count)) {
    if ((e = launch_dft2_batch<T>(n, buf_d, count, +1, st)) != hipSuccess) return e;
    if ((e = launch_dft2_batch<T>(n, buf_r, count, -1, st)) != hipSuccess) return e;
  } else {
    hipLaunchKernelGGL((k_pair_dft<T, +1>), dim3(rows), dim3(256), 0, st, (const T*)buf_d, n, buf_t);
    hipLaunchKernelGGL((k_pair_dft<T, +1>), dim3(rows), dim3(256), 0, st, (const T*)buf_t, n, buf_d);
    hipLaunchKernelGGL((k_pair_dft<T, -1>), dim3(rows), dim3(256), 0, st, (const T*)buf_r, n, buf_t);
    hipLaunchKernelGGL((k_pair_dft<T, -1>), dim3(rows), dim3(256), 0, st, (const T*)buf_t, n, buf_r);
  }
  hipLaunchKernelGGL(k_pair_clear_keys, dim3(1), dim3(64), 0, st, key, count);
  hipLaunchKernelGGL(k_pair_s0<T>, dim3(s0_ranges(n), (unsigned)count), dim3(256), 0, st, (const T*)buf_d, n, s0,
                     key);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int k = 0; k < count; ++k) out[k] = ObsSums<T>{s0 + k * nn, buf_r + k * nn, key + k};
  return hipSuccess;
}

template <class T>
hipError_t launch_pair_emit(int n, const ObsSums<T>& sums, bool shared, int count, const double* c,
                            const double* a_out, int pi, int pj, double floor_rel, typename real_of<T>::type* s_out,
                            T* mu_out, hipStream_t st) {
  if (count < 1 || count > kPairTile) return hipErrorInvalidValue;
  PairEmit pe{};
  pe.count = count;
  for (int k = 0; k < count; ++k) {
    pe.c[k] = c[k];
    pe.a_out[k] = a_out[k];
  }
  const long long nn = (long long)n * n;
  hipLaunchKernelGGL(k_pair_emit<T>, dim3((unsigned)((nn + 255) / 256), (unsigned)count), dim3(256), 0, st,
                     (const typename real_of<T>::type*)sums.s0, (const T*)sums.b0,
                     (const unsigned long long*)sums.key, shared ? 1 : 0, n, pi, pj, pe, floor_rel, s_out, mu_out);
  return hipGetLastError();
}

// Work of the polychromatic sums, per group (elements of T unless noted): tables 8 x 64 N, row-sum
// partials 16 x 64 N^2, difference-sum partials sb x 64 x 4N^2, D 64 x 4N^2, T R 64 N^2, transform
// intermediate 64 x 2N^2, the two transformed arrays 64 N^2 each; then S and W[P; .] in FP64 (N^2 each).
static int poly_bsplit(int n) {
  int sb = (3072 + 2 * n - 1) / (2 * n);  // chunks of b: about 3072 workgroups per column tile (unequal a ranges)
  if (sb < 4) sb = 4;
  if (sb > n) sb = n;
  return sb;
}

template <class T> size_t poly_work_bytes(int n) {
  const size_t nn = (size_t)n * n, g = (size_t)kPairTile * nn;
  const size_t elems = 8 * (size_t)kPairTile * n + (size_t)kPairSplitK * g + (size_t)poly_bsplit(n) * 4 * g + 4 * g +
                       g + 2 * g + 2 * g;
  return elems * sizeof(T) + nn * (sizeof(double) + sizeof(double2)) + 512;
}

template <class T>
hipError_t launch_poly(int n, const T* w, int n_pairs, const double* alpha, const double* beta, const double* gamma,
                       const double* coef, int pi, int pj, double floor_rel, void* work,
                       typename real_of<T>::type* s_out, T* mu_out, hipStream_t st) {
  const long long nn = (long long)n * n, g = (long long)kPairTile * nn;
  T* base = reinterpret_cast<T*>(work);
  T* u1 = base;
  T* u2 = u1 + kPairTile * n;
  T* ci = u2 + kPairTile * n;
  T* cj = ci + kPairTile * n;
  T* tr = cj + kPairTile * n;  // u1, u2, ci, cj transposed
  const long long tq = (long long)kPairTile * n;
  T* part_r = tr + 4 * tq;
  const int sb = poly_bsplit(n);
  T* part_d = part_r + (long long)kPairSplitK * g;
  T* dfull = part_d + (long long)sb * 4 * g;
  T* rr = dfull + 4 * g;
  T* tmp = rr + g;
  T* zd = tmp + 2 * g;
  T* zr = zd + g;
  double* s_acc = reinterpret_cast<double*>((reinterpret_cast<uintptr_t>(zr + g) + 15) & ~(uintptr_t)15);
  double2* w_acc = reinterpret_cast<double2*>(s_acc + nn);
  hipError_t e = hipSuccess;
  for (int k0 = 0; k0 < n_pairs; k0 += kPairTile) {
    PolyGroup pg{};
    pg.count = n_pairs - k0 < kPairTile ? n_pairs - k0 : kPairTile;
    for (int k = 0; k < pg.count; ++k) {
      pg.alpha[k] = alpha[k0 + k];
      pg.beta[k] = beta[k0 + k];
      pg.gamma[k] = gamma[k0 + k];
      pg.c[k] = coef[k0 + k];
    }
    hipLaunchKernelGGL(k_poly_tables<T>, dim3((unsigned)((kPairTile * n + 255) / 256)), dim3(256), 0, st, pg, n, pi,
                       pj, u1, u2, ci, cj, tr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (pg.count == 1) {  // one pair: both sums in one pass, HBM-bound
      const int ranges = nn < 256 ? (int)nn : 256;  // slab ranges; partials fit: 64 sb >= 256 or nn
      const int slabs = (int)((nn + ranges - 1) / ranges);
      const dim3 grid((unsigned)((nn + kOneThreads * kOneCols - 1) / (kOneThreads * kOneCols)), (unsigned)ranges);
      hipLaunchKernelGGL(k_one_poly_sums<T>, grid, dim3(kOneThreads), 0, st, w, n, (const T*)u1, (const T*)u2,
                         (const T*)ci, (const T*)cj, slabs, part_r, part_d);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      const unsigned blocks = (unsigned)((nn + 255) / 256);
      hipLaunchKernelGGL(k_pair_sum<T>, dim3(blocks), dim3(256), 0, st, (const T*)part_r, ranges, n, 1,
                         (const T*)u2, rr);
      hipLaunchKernelGGL(k_pair_sum<T>, dim3(4 * blocks), dim3(256), 0, st, (const T*)part_d, ranges, 2 * n, 1,
                         (const T*)nullptr, dfull);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    } else {
      const long long chunk = (nn + kPairSplitK - 1) / kPairSplitK;
      const int bchunk = (n + sb - 1) / sb;
      if ((e = launch_mfma<T>(pg.count, 0, n, w, u1, u2, tr, chunk, bchunk, sb, part_r, st)) != hipSuccess) return e;
      if ((e = launch_mfma<T>(pg.count, 2, n, w, u1, u2, tr, chunk, bchunk, sb, part_d, st)) != hipSuccess) return e;
      const int rp = sizeof(T) == 8 ? rows_ring_parts(n, pg.count) : 0;
      const int sr = rp > 0 ? rp : kPairSplitK;
      hipLaunchKernelGGL(k_pair_sum<T>, dim3((unsigned)((g + 255) / 256)), dim3(256), 0, st, (const T*)part_r, sr, n,
                         kPairTile, (const T*)u2, rr);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      const int sdp = (sizeof(T) == 8 && poly_diffs_ring_ok(n, pg.count)) ? 256 / n : sb;  // chunks of b written
      hipLaunchKernelGGL(k_pair_sum<T>, dim3((unsigned)((4 * g + 255) / 256)), dim3(256), 0, st, (const T*)part_d,
                         sdp, 2 * n, kPairTile, (const T*)nullptr, dfull);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // S: the + transform of D over [-N, N)^2 (offset N); the row: the - transform of T R (offset N/2). Only
    // the group's pairs are transformed.
    hipLaunchKernelGGL((k_poly_czt<T, +1>), dim3((unsigned)(pg.count * 2 * n)), dim3(256), 0, st, (const T*)dfull, n,
                       2 * n, 2 * n, n, pg, tmp);
    hipLaunchKernelGGL((k_poly_czt<T, +1>), dim3((unsigned)(pg.count * n)), dim3(256), 0, st, (const T*)tmp, n, n,
                       2 * n, n, pg, zd);
    hipLaunchKernelGGL((k_poly_czt<T, -1>), dim3((unsigned)(pg.count * n)), dim3(256), 0, st, (const T*)rr, n, n, n,
                       n / 2, pg, tmp);
    hipLaunchKernelGGL((k_poly_czt<T, -1>), dim3((unsigned)(pg.count * n)), dim3(256), 0, st, (const T*)tmp, n, n, n,
                       n / 2, pg, zr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_poly_combine<T>, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, (const T*)zd,
                       (const T*)zr, n, pi, pj, pg, k0 == 0 ? 1 : 0, s_acc, w_acc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_poly_mu<T>, dim3(1), dim3(1024), 0, st, (const double*)s_acc, (const double2*)w_acc, n, pi, pj,
                     floor_rel, s_out, mu_out);
  return hipGetLastError();
}

template size_t poly_work_bytes<float2>(int);
template size_t poly_work_bytes<double2>(int);
template hipError_t launch_poly<float2>(int, const float2*, int, const double*, const double*, const double*,
                                        const double*, int, int, double, void*, float*, float2*, hipStream_t);
template hipError_t launch_poly<double2>(int, const double2*, int, const double*, const double*, const double*,
                                         const double*, int, int, double, void*, double*, double2*, hipStream_t);

template size_t pair_work_bytes<float2>(int);
template size_t pair_work_bytes<double2>(int);
template hipError_t launch_pair_sums<float2>(int, const float2*, const double*, int, int, int, void*, ObsSums<float2>*,
                                             hipStream_t);
template hipError_t launch_pair_sums<double2>(int, const double2*, const double*, int, int, int, void*,
                                              ObsSums<double2>*, hipStream_t);
template hipError_t launch_pair_emit<float2>(int, const ObsSums<float2>&, bool, int, const double*, const double*, int,
                                             int, double, float*, float2*, hipStream_t);
template hipError_t launch_pair_emit<double2>(int, const ObsSums<double2>&, bool, int, const double*, const double*,
                                              int, int, double, double*, double2*, hipStream_t);

}  // namespace wolf
