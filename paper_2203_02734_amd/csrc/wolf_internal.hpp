// Internal declarations shared by the kernel translation units and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wolf_device.hpp"

namespace wolf {

// The propagation operator along its four axes. Axis of the first point (i1, j1) and of the
// second point (i2, j2): diagonal pre-factor, DFT of sign `sign` (-1 direct, +1 inverse,
// unnormalised), diagonal post-factor. The real `scale` multiplies the result.
// `pupil` multiplies the input by P(p1) P(p2) (real 0/1) before the transforms.
struct OperatorTables {
  Chirp pre1, post1, pre2, post2;
  int sign1, sign2;
  double scale;
  Pupil pupil;
};

// Schedule of the passes. fused_slab: one slab pass for (i2, j2); with 0 < slab_chunk < N^2 (whole
// i1 planes), an in-place call runs it over groups of slab_chunk slabs, each followed at once by the
// j1 pass of its planes, and the i1 pass follows in one launch. Otherwise a row pass and an i2 pass
// run over chunks of `slab_chunk` slabs (in place, chunks of whole planes take their j1 pass at once
// too). Without groups (and out of place), the j1 and i1 passes run
// over chunks of `col_chunk` columns m2 (0 = all), the i1 pass of one chunk beside the j1 pass of the next.
struct Plan {
  int fused_slab;  // 0: row pass + i2 axis pass; 1: one slab per workgroup; 2: persistent slab pass;
                   // 3: one slab per workgroup through a half-size LDS buffer
  long long slab_chunk;
  long long col_chunk;
  int coop;        // 1: first-point axes in one cooperative pass (wolf_coop.hip); col_chunk unused
  int coop_cols;   // columns of a cooperative tile (64, 128 or 256 bytes of each row)
  int coop_lookahead;
};

// Parameters of the cooperative first-point pass (see wolf_coop.hip).
struct CoopParams {
  long long NN, NNN;
  int tiles_per_xcd, lookahead, items_per_phase;
  unsigned long long max_ticks;  // bound of one wait, in ticks of the 100 MHz real-time clock
  unsigned zero;                 // 0, opaque to the compiler (keeps the poll a read-modify-write)
  unsigned* head;
  unsigned* done_a;
  unsigned* err;
  Chirp a_pre, a_post, b_pre, b_post;
};

// A strided-axis block: outer_count blocks (stride outer_stride); per block, columns
// [inner_offset, inner_offset + ncols) at unit stride; the transformed axis has stride axis_stride.
struct AxisRange {
  long long outer_count, outer_stride, axis_stride, inner_offset, ncols;
};

// Kernel-side form of an AxisRange: tiles of C columns, `blocks` workgroups.
struct AxisJob {
  long long outer_stride, axis_stride, inner_offset, tiles_per_outer, blocks;
  Chirp pre, post;
};

struct SourceParams;

// `counters`: per-stream device scratch of at least coop_counter_bytes(n) (used when plan.coop).
// `gen` (plan.fused_slab == 3, or 0 at N >= 64 with no input pupil): the input is the source
// described by *gen, formed inside the first pass; `in` is not read.
template <class T>
hipError_t launch_operator(int n, const T* in, T* out, const OperatorTables& op, const Plan& plan, void* counters,
                           hipStream_t st, const SourceParams* gen = nullptr);
// The operator applied to diag(g), g an N*N real array (no N^4 input is read).
template <class T>
hipError_t launch_operator_diag(int n, const typename real_of<T>::type* g, T* out, const OperatorTables& op,
                                const Plan& plan, void* counters, hipStream_t st);
// Raw sums of the observables S and mu(P, .) of one pair, with no N^4 output (wolf_pairs.hip).
template <class T> struct ObsSums {
  typename real_of<T>::type* s0;  // raw sums for S, N^2
  T* b0;                          // raw sums for the row W_B[P; .], N^2
  unsigned long long* key;        // order key of max s0
};
// The sums for groups of up to kPairGroup pairs at once: the first-point contractions are shared by the
// pairs of a group, so the source is read twice per group (once for a group of one). a_src[k] is
// the source chirp rate pitch^2 / (lambda z) of pair k (0 in the far field); out[k] receives pair k's
// sums, which live in `work` (pair_work_bytes) until the next call.
constexpr int kPairGroup = 64;
template <class T> size_t pair_work_bytes(int n);
template <class T>
hipError_t launch_pair_sums(int n, const T* w, const double* a_src, int count, int pi, int pj, void* work,
                            ObsSums<T>* out, hipStream_t st);
// S and mu(P, .) of `count` (<= kPairGroup) pairs in one launch from the sums of launch_pair_sums (pair
// k reads sums + k N^2, or the first pair's sums for all when shared): c[k] = s weight, a_out[k] the
// output chirp rate; pair k writes s_out + k N^2 and mu_out + k N^2.
template <class T>
hipError_t launch_pair_emit(int n, const ObsSums<T>& sums, bool shared, int count, const double* c,
                            const double* a_out, int pi, int pj, double floor_rel, typename real_of<T>::type* s_out,
                            T* mu_out, hipStream_t st);
// Polychromatic S and mu(P, .) on a common output grid (wolf_pairs.hip): alpha[k], beta[k], gamma[k] are the
// source chirp rate, the DFT frequency and the output chirp rate of pair k on that grid, coef[k] its weight
// times s; the pairs run in groups of kPairGroup, and the sums are written to s_out, mu_out (N^2 each).
template <class T> size_t poly_work_bytes(int n);
template <class T>
hipError_t launch_poly(int n, const T* w, int n_pairs, const double* alpha, const double* beta, const double* gamma,
                       const double* coef, int pi, int pj, double floor_rel, void* work,
                       typename real_of<T>::type* s_out, T* mu_out, hipStream_t st);
bool coop_supported(int n, int elem_bytes, int cols);
template <class T>
hipError_t launch_first_point_coop(int n, T* data, const OperatorTables& op, const Chirp& pre1, int cols,
                                   int lookahead, void* counters, hipStream_t st);
size_t coop_counter_bytes(int n);
template <class T> bool slab_pass_supported(int n);
template <class T> bool half_slab_supported(int n);  // plan fused_slab = 3
// out[p1; p2] = P(p1) P(p2) in[p1; p2] (in == out allowed).
template <class T>
hipError_t launch_apply_pupil(int n, const T* in, T* out, const Pupil& pu, hipStream_t st);

// In-place plain 2D DFTs (sign of the exponent `sign`) of `count` N x N arrays: a row pass and an axis
// pass of the operator's FFT kernels. dft2_batch_ok: count N is a whole number of row-pass workgroups.
bool dft2_batch_ok(int n, long long count);
template <class T>
hipError_t launch_dft2_batch(int n, T* data, long long count, int sign, hipStream_t st);
int axis_tile_cols(int n, int elem_bytes);  // columns of an axis-pass tile
int row_pass_rows(int n);  // rows per workgroup of the row pass

// The operator for any even N and transform length N_z >= N (zero padding and crop), as four dense
// axis passes (wolf_dense.hip). work: N^4 elements. Tables without the (-1)^n centring factor.
bool dense_supported(int n, int nz);
// The same operator with zero-padded FFTs, for a power-of-two N_z <= 1024 (in -> out, then in place).
// Tables with the (-1)^n centring factor.
bool pad_fft_supported(int n, int nz);
template <class T>
hipError_t launch_operator_padfft(int n, int nz, const T* in, T* out, const OperatorTables& op, hipStream_t st);
template <class T>
hipError_t launch_operator_dense(int n, int nz, const T* in, T* out, T* work, const OperatorTables& op,
                                 hipStream_t st);

// Direct sum with the exact free-space kernel (wolf_direct.hip). work: direct_work_bytes(n, elem).
template <class T>
hipError_t launch_direct(int n, const T* in, T* out, void* work, double pitch, double lam, double z, int primary,
                         hipStream_t st);
size_t direct_work_bytes(int n, int elem);

// Source description after host-side validation and unit conversion.
struct SourceParams {
  int model;
  int geometry;
  double amplitude;
  double inv4s2;        // 1 / (4 sS^2), 0 for uniform S
  double inv2g2_px;     // pitch^2 / (2 sg^2), 0 for full coherence (pixel units)
  double inv4s2_px;     // pitch^2 / (4 sS^2) (pixel units)
  long long t0, t1;     // squared pixel radii thresholds, floor((r/pitch)^2 (1 + 1e-9))
  const float* imap;
  const uint8_t* mask;
  double lens_alpha;    // pitch^2 / (lambda f), 0 = no lens
};

template <class T>
hipError_t launch_build_source(int n, const SourceParams& sp, T* w, hipStream_t st);
// The first pass of the schedule `fused_slab` (3: the half-buffer slab pass; 0: the row pass) can
// form this source itself at this N (launch_operator's `gen`).
template <class T> bool gen_source_supported(int n, const SourceParams& sp, int fused_slab);

template <class T>
hipError_t launch_spectral_density(int n, const T* w, typename real_of<T>::type* s, hipStream_t st);

// mu slice (ip >= 0) or full mu (ip < 0). scratch: at least 16 + N*N*sizeof(real) bytes.
template <class T>
hipError_t launch_coherence(int n, const T* w, int ip, int jp, double floor_rel, T* mu, void* scratch,
                            hipStream_t st);

// Device address and size of the static scratch of the allocation-free mu entry point on the current
// device (looked up once per device; allocates nothing).
hipError_t mu_static_scratch(void** out, size_t* bytes);

template <class T>
hipError_t launch_chirp_table(int n, const Chirp& ch, T* out, hipStream_t st);

// Fit gradients (wolf_fit.hip).
template <class T>
hipError_t launch_diag_embed(int n, const typename real_of<T>::type* g, T* out, hipStream_t st);
template <class T>
hipError_t launch_fit_gradient(int n, const T* ga, const float* imap, double inv2g2_px, double sg_scale, void* work,
                               float* d_imap, double* d_sigma, hipStream_t st);
int fit_slabs_per_group(int n);
size_t fit_work_bytes(int n, int real_bytes);

// Memory ceilings (wolf_measure.hip): mode 0 in-place read-modify-write, 1 write only, 2 read only,
// over `bytes` (a multiple of 16 KB) of `buf`.
hipError_t launch_ceiling(void* buf, long long bytes, int mode, hipStream_t st);

}  // namespace wolf
