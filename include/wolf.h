/*
 * libwolf: MI355X (gfx950) propagation of the cross-spectral density (CSD) of a planar source.
 *
 * The method is that of Magalhaes & Rebordao, "PyWolf: A PyOpenCL implementation for simulating
 * the propagation of partially coherent light" (arXiv 2203.02734).
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - CSD layout: one contiguous array W[i1][j1][i2][j2] of N^4 complex numbers, j2 fastest. The
 *    real and imaginary parts are interleaved, as torch.complex64 / torch.complex128 of shape
 *    (N, N, N, N) store them. Index (i, j) is the point
 *    (pitch (i - N/2), pitch (N/2 - j)) (Sec. 3.1, eqs. point and n12).
 *  - N is a power of two from 2 to 256. Other values return WOLF_EUNSUPPORTED.
 *  - dtype WOLF_C64 computes in FP32 (complex64 data); WOLF_C128 computes in FP64
 *    (complex128 data). In both, the quadratic-phase tables and the FFT twiddles are built in
 *    FP64 with argument reduction.
 *  - Every buffer argument is device memory, allocated and owned by the caller. The library
 *    checks that each buffer lies in one device allocation large enough for the call. A host
 *    pointer or a too-small buffer returns WOLF_EINVAL before anything is launched.
 *  - Calls are asynchronous on `stream`, a hipStream_t passed as void*. NULL is the default
 *    stream. There is no implicit synchronisation.
 *  - Arguments are validated before any launch, and a call that fails validation has no side
 *    effect. A launch failure, or a sticky error from earlier GPU work, returns WOLF_EDEVICE.
 *    wolf_last_error_message() gives details. No C++ exception crosses this interface.
 *  - Input and output may be the same buffer (in place). Buffers that partly overlap return
 *    WOLF_EINVAL.
 *  - Units are SI (metres).
 */
#ifndef WOLF_H
#define WOLF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WOLF_API __attribute__((visibility("default")))

typedef int32_t wolf_status;
enum {
  WOLF_OK = 0,
  WOLF_EINVAL = -1,       /* invalid argument (null, range, overlap, buffer too small, host pointer) */
  WOLF_EUNSUPPORTED = -2, /* valid but not supported (N not a power of two in [2, 256]) */
  WOLF_ENOMEM = -3,       /* the library could not allocate its own small device scratch */
  WOLF_EDEVICE = -4       /* HIP error at launch, or a sticky error from earlier GPU work */
};

enum { WOLF_C64 = 0, WOLF_C128 = 1 };

/* Obliquity factor Lambda of eq. (h_free): a secondary source (an aperture, Lambda = 1/(i lambda)
 * at normal incidence) or a primary source (Lambda = 1/(4 pi)). C = Lambda1* Lambda2 / R^2, eq. (C). */
enum { WOLF_SECONDARY = 0, WOLF_PRIMARY = 1 };

/* Source models (Sec. 3.2; eq. W_def; Sec. 5.1, 5.2, 5.4; Algorithm 7). */
enum {
  WOLF_MODEL_GSM = 0,       /* A exp(-(xi1^2+xi2^2)/(4 sS^2)) exp(-|xi1-xi2|^2/(2 sg^2)); sS or sg may be +inf */
  WOLF_MODEL_MAP = 1,       /* A sqrt(I(p1)) sqrt(I(p2)) exp(-|xi1-xi2|^2/(2 sg^2)), I a device N*N map */
  WOLF_MODEL_COHERENT = 2,  /* A (mu = 1, uniform S) */
  WOLF_MODEL_INCOHERENT = 3 /* A delta(p1, p2) (Kronecker delta on the grid) */
};

/* Geometry Y(xi) in {0,1} of eq. (GSM_source); W0 = Y(xi1) Y(xi2) W_rho (Sec. 3.2, eq. circle). */
enum {
  WOLF_GEO_NONE = 0,
  WOLF_GEO_CIRCLE = 1,  /* |xi| <= r0 */
  WOLF_GEO_SQUARE = 2,  /* |x| <= r0 and |y| <= r0 (r0 = half side) */
  WOLF_GEO_ANNULUS = 3, /* r1 < |xi| <= r0 */
  WOLF_GEO_MASK = 4     /* caller's device N*N uint8 mask, nonzero = inside */
};

typedef struct wolf_source {
  int32_t model;             /* WOLF_MODEL_* */
  int32_t geometry;          /* WOLF_GEO_* */
  double amplitude;          /* A >= 0 */
  double sigma_s_m;          /* GSM r.m.s. width of S (> 0, +inf = uniform) */
  double sigma_g_m;          /* GSM/MAP r.m.s. width of mu (> 0, +inf = coherent) */
  double geo_r0_m;           /* circle / annulus outer radius, square half side (> 0) */
  double geo_r1_m;           /* annulus inner radius (0 <= r1 < r0) */
  const float* intensity_map;/* MAP only: device, N*N float32 [i][j], >= 0 */
  const uint8_t* mask;       /* MASK only: device, N*N uint8 [i][j] */
  double lens_focal_m;       /* thin lens in the source plane, 0 = none; Sec. 2.2 */
  double wavelength_m;       /* needed iff lens_focal_m != 0 */
} wolf_source;

/*
 * wolf_build_source -- source CSD array W0 (Algorithm 1 steps 1-3; Sec. 3.2, eq. GSM_source).
 *
 * W0[p1; p2] = Y(p1) Y(p2) W_rho(xi1, xi2), with W_rho set by src->model. With a lens, W0 is then
 * multiplied by q(f, xi1) q*(f, xi2), where q(R, xi) = exp(i pi |xi|^2 / (lambda R)) (eq. q_factor).
 * This is the thin lens T = q*(f, x) of Sec. 2.2, applied as T*(x1) W T(x2).
 * The geometry test runs in pixel units: d2 <= floor((r/pitch)^2 (1 + 1e-9)), with d2 an exact integer.
 *   src      host pointer to the description. The device pointers it holds are read by the kernel.
 *   n, pitch_m   grid size and sample pitch (> 0).
 *   w_out    device, N^4 complex of `dtype`, written in full (write-only).
 */
WOLF_API wolf_status wolf_build_source(const wolf_source* src, int32_t n, double pitch_m, int32_t dtype,
                                       void* w_out, void* stream);

/*
 * wolf_propagate_source -- the source of wolf_build_source propagated over z_m in one call
 * (Algorithm 1: build the source, then Algorithms 2-3; Sec. 2.1 eqs. W_fresnel, W_farfield).
 *
 * The result is wolf_build_source(src, ..., w_out) followed by wolf_propagate_fresnel (far_field = 0)
 * or wolf_propagate_farfield (far_field = 1) in place on w_out, bit for bit. Where the propagation
 * runs the half-buffer slab pass (the default plan at N = 128; N = 32 or 64 with that pass set by
 * wolf_set_plan) and the source is decided by the coordinates alone (WOLF_MODEL_GSM or
 * WOLF_MODEL_COHERENT with WOLF_GEO_NONE, CIRCLE, SQUARE or ANNULUS, with or without a lens), that
 * pass forms each W0 entry where it would load it, so W0 is never written to memory: one write and
 * one read of the N^4 array less. So does the row pass of the four-sweep schedule (the default at
 * N = 256; N = 64 or 128 when set) for the same sources. Other sources and schedules build W0 in
 * w_out first.
 *   src, n, pitch_m   as wolf_build_source (N a power of two in [2, 256]).
 *   wavelength_m, z_m, kind, out_pitch_m   as wolf_propagate_fresnel.
 *   far_field         0 (Fresnel) or 1 (far field).
 *   w_out             device, N^4 complex of `dtype`, written in full.
 */
WOLF_API wolf_status wolf_propagate_source(const wolf_source* src, int32_t n, double pitch_m, double wavelength_m,
                                           double z_m, int32_t far_field, int32_t kind, int32_t dtype, void* w_out,
                                           double* out_pitch_m, void* stream);

/*
 * wolf_propagate_fresnel -- free-space Fresnel propagation of W over distance z
 * (Sec. 2.1 eq. W_fresnel; Sec. 3.4 Algorithms 2-3).
 *
 * W_B(x1, x2) = C pitch^4 sum_{xi1, xi2} h*(x1, xi1) W_A(xi1, xi2) h(x2, xi2),
 * with h(x, xi) = exp(i pi |x - xi|^2 / (lambda z)) (eqs. h_free, approx_L) and C from eq. (C).
 * The output lies on the same index grid with pitch dx = lambda z / (N pitch) (eq. spatial_resolution).
 * The direct DFT runs over the second point and the inverse DFT over the first (h* on xi1).
 *   w_in, w_out   device, N^4 complex of `dtype`. They may be equal (in place).
 *   kind          WOLF_SECONDARY or WOLF_PRIMARY.
 *   out_pitch_m   optional host pointer that receives dx.
 */
WOLF_API wolf_status wolf_propagate_fresnel(const void* w_in, void* w_out, int32_t n, double pitch_m,
                                            double wavelength_m, double z_m, int32_t kind, int32_t dtype,
                                            double* out_pitch_m, void* stream);

/*
 * wolf_propagate_farfield -- far-field propagation (Sec. 2.1 eq. W_farfield).
 * Same as wolf_propagate_fresnel with the source-plane propagator q(z, xi) set to 1, so
 * h(x, xi) = exp(i pi |x|^2 / (lambda z)) exp(-2 pi i x.xi / (lambda z)). The output propagator is kept.
 */
WOLF_API wolf_status wolf_propagate_farfield(const void* w_in, void* w_out, int32_t n, double pitch_m,
                                             double wavelength_m, double z_m, int32_t kind, int32_t dtype,
                                             double* out_pitch_m, void* stream);

/*
 * wolf_propagate_lens -- a thin lens at the input plane, then Fresnel propagation by z_m
 * (Sec. 2.2: lens transmission T(x) = P(x) q*(f, x), W+ = T*(x1) W- T(x2); the second stage of
 * eq. WC_imaging). With wolf_propagate_fresnel from the source plane A to the lens plane B (distance
 * R1) and this call from B (its pitch is the out_pitch of the first call) to C (distance R2), the
 * pair is the two-stage imaging system of eqs. WA_imaging and WC_imaging, with no approximation.
 *   focal_m          focal length f (negative: diverging lens); 0 = no lens phase (pupil only).
 *   pupil_geometry   WOLF_GEO_NONE (P = 1), WOLF_GEO_CIRCLE (P = 1 for |x| <= r) or WOLF_GEO_SQUARE
 *                    (P = 1 for |x|, |y| <= r), decided on the input grid in pixel units with the
 *                    rule of the source geometry. P is real (no aberration phase).
 *   pupil_radius_m   r (> 0) when pupil_geometry != WOLF_GEO_NONE.
 * Other arguments, layout, in-place use and errors as wolf_propagate_fresnel. The lens phase only
 * changes the source-side chirp of the operator (q*(f) q(z) is one chirp), and the pupil is applied
 * while the first pass loads its input, so the call costs one propagation.
 */
WOLF_API wolf_status wolf_propagate_lens(const void* w_in, void* w_out, int32_t n, double pitch_m,
                                         double wavelength_m, double focal_m, int32_t pupil_geometry,
                                         double pupil_radius_m, double z_m, int32_t kind, int32_t dtype,
                                         double* out_pitch_m, void* stream);

/*
 * wolf_propagate_direct -- the validity check of the Fresnel propagation: eq. (W_general) with the
 * exact free-space kernel of eq. (h_free), h = Lambda(r) exp(i k r) / r, r = sqrt(z^2 + |x - xi|^2),
 * summed directly over the grids, without the approximation Lambda/r ~ Lambda/R (eq. approx_L) and
 * without the Fresnel expansion of r. Secondary source: Lambda = (k / 4 pi i)(1 + z / r) (normal
 * incidence); primary: Lambda = 1 / (4 pi). The output grid is that of wolf_propagate_fresnel with
 * the same arguments (pitch lambda z / (N pitch_m)), so the two results compare element by element;
 * their difference is the error of the Fresnel approximation for this source and distance.
 * The kernel does not separate into x and y: the cost is two dense complex products of size N^2
 * (2 N^6 complex multiply-adds), meant for N <= 64 (N = 128 is accepted).
 *   w_in, w_out   device N^4 complex of `dtype`; w_in == w_out is allowed (partial overlap is not).
 *   work          device scratch of wolf_direct_work_bytes(n, dtype) bytes (two N^4 arrays),
 *                 overwritten, not overlapping w_in or w_out.
 *   out_pitch_m   optional host output.
 * Returns WOLF_EUNSUPPORTED for N > 128.
 */
WOLF_API wolf_status wolf_propagate_direct(const void* w_in, void* w_out, int32_t n, double pitch_m,
                                           double wavelength_m, double z_m, int32_t kind, int32_t dtype, void* work,
                                           double* out_pitch_m, void* stream);

/* Bytes of the work buffer of wolf_propagate_direct; -1 if (n, dtype) is not supported. */
WOLF_API int64_t wolf_direct_work_bytes(int32_t n, int32_t dtype);

/*
 * wolf_propagate_padded -- Fresnel or far-field propagation (eqs. W_fresnel, W_farfield) for any
 * even N and with zero padding (Sec. 3.3): the N-point axes are padded to n_fft points for the
 * transform and the result is cropped back to the central N points, so the output pitch is
 * lambda z / (n_fft pitch_m) (eq. spatial_resolution with n_fft in place of N). n_fft = N gives the
 * plain operator for N that are not powers of two (e.g. the paper's N = 200 examples, padded to
 * n_fft = 512). Four passes, one per axis. An n_fft that is a power of two (<= 1024) or one of 6, 10,
 * 12, 20, 24, 36, 48, 72, 80, 96, 100, 144, 192, 200 takes zero-padded FFTs of n_fft points per line
 * (the N inputs at the centre, the N central outputs kept; mixed radices 2, 3, 5 for the listed
 * lengths). Any other n_fft takes dense N x N products with the exact centred kernel
 * e^{-+2 pi i (k - N/2)(n - N/2) / n_fft} (32 N real flops per element).
 *   n          even, 2..256.   n_fft   N..2048.
 *   w_in, w_out   device N^4 complex; w_in == w_out allowed (partial overlap is not).
 *   work       device N^4 complex of `dtype` (used by the dense passes), overwritten; must not
 *              overlap w_in or w_out.
 *   farfield   0 Fresnel, 1 far field.   kind, dtype, out_pitch_m as wolf_propagate_fresnel.
 * The source builder and the observables accept any even N as well.
 */
WOLF_API wolf_status wolf_propagate_padded(const void* w_in, void* w_out, int32_t n, int32_t n_fft, double pitch_m,
                                           double wavelength_m, double z_m, int32_t farfield, int32_t kind, int32_t dtype,
                                           void* work, double* out_pitch_m, void* stream);

/*
 * wolf_propagate_adjoint -- adjoint of the Fresnel (farfield = 0) or far-field (farfield = 1)
 * propagation, for the real inner product Re sum conj(a) b. It is the derivative operator of the
 * paper's propagation (eq. W_general).
 * For P(W) = C pitch^4 conj(H) W H^T: g_in = C pitch^4 H^T g_out conj(H), i.e.
 * G_A(xi1, xi2) = C pitch^4 sum_{x1, x2} h(x1, xi1) G_B(x1, x2) h*(x2, xi2).
 * With torch's convention for complex gradients (dL/dRe + i dL/dIm), this maps the gradient with
 * respect to W_B to the gradient with respect to W_A.
 *   g_out   device, N^4, gradient on the output grid (pitch lambda z / (N pitch)).
 *   g_in    device, N^4, written. It may equal g_out.
 */
WOLF_API wolf_status wolf_propagate_adjoint(const void* g_out, void* g_in, int32_t n, double pitch_m,
                                            double wavelength_m, double z_m, int32_t farfield, int32_t kind,
                                            int32_t dtype, void* stream);

/*
 * wolf_propagate_adjoint_diag -- wolf_propagate_adjoint applied to diag(g), without reading an N^4
 * input: g_in = P^H(G_B) with G_B[x1; x2] = g(x1) delta(x1, x2). This is the gradient with respect
 * to W_A of a loss that depends on the propagated CSD only through S_B = Re diag W_B
 * (Algorithm 4), given g = dL/dS_B.
 *   g_diag   device, N*N real (float32 for WOLF_C64, float64 for WOLF_C128), on the output grid.
 *   g_in     device, N^4 complex, written in full.
 */
WOLF_API wolf_status wolf_propagate_adjoint_diag(const void* g_diag, void* g_in, int32_t n, double pitch_m,
                                                 double wavelength_m, double z_m, int32_t farfield, int32_t kind,
                                                 int32_t dtype, void* stream);

/*
 * wolf_spectral_density -- S[i][j] = Re W[i][j; i][j] (Sec. 3.5, Algorithm 4, eq. defS).
 *   s_out   device, N*N real (float32 for WOLF_C64, float64 for WOLF_C128).
 */
WOLF_API wolf_status wolf_spectral_density(const void* w, int32_t n, int32_t dtype, void* s_out, void* stream);

/*
 * wolf_degree_of_coherence -- mu(P1, x) = W(P1, x) / sqrt(S(P1) S(x)) (Sec. 3.5, Algorithm 5,
 * eq. defMu; the printed numerator W(xi, xi) is read as W(xi1, xi2)).
 * Where S(P1) <= tau or S(x) <= tau, with tau = s_floor_rel * max S, mu = 0.
 *   ip, jp   index of P1 in [0, N): mu_out is N*N complex [i][j] (the slice mu(P1, .)).
 *            ip = jp = -1: mu_out is the full N^4 mu[p1; p2].
 *   s_floor_rel   >= 0 (1e-12 is a good default).
 * Uses a small per-device scratch owned by the library. Calls that use it on one device must be
 * ordered (same stream, or synchronised).
 */
WOLF_API wolf_status wolf_degree_of_coherence(const void* w, int32_t n, int32_t dtype, int32_t ip, int32_t jp,
                                              double s_floor_rel, void* mu_out, void* stream);

/*
 * wolf_degree_of_coherence_noalloc -- wolf_degree_of_coherence (same arguments, same kernels, the same
 * result bit for bit) for callers that cannot allocate device memory: code under hipGraph stream
 * capture, tight serving loops, harnesses that forbid hipMalloc. It allocates nothing: its scratch
 * (the maximum of S and the N^2 values of S) is a static device array of 256 + 256*256*8 bytes
 * (enough for any N <= 256 in either dtype), one copy per GPU, looked up on the first call on each
 * device and held until the process ends. Sizes beyond that array return WOLF_EINVAL.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU (on different
 * streams, or from different threads without ordering) race and give wrong results. Order them
 * (one stream, or synchronise).
 */
WOLF_API wolf_status wolf_degree_of_coherence_noalloc(const void* w, int32_t n, int32_t dtype, int32_t ip, int32_t jp,
                                                      double s_floor_rel, void* mu_out, void* stream);

/*
 * wolf_propagate_batch -- many (lambda, z) pairs of one source (polychromatic light; the paper's
 * Sec. 7 names it as future work). For pair k, weight[k] * w_src is propagated to distance z[k]
 * at wavelength lambda[k] (Sec. 2.1, eqs. W_fresnel / W_farfield), and S_k (Algorithm 4) and
 * mu_k(P1, .) (Algorithm 5) are written to s_out[k] and mu_out[k]. No propagated N^4 array is
 * returned.
 * The propagated CSD is never stored. On the diagonal it depends on the source only through sums
 * along the difference coordinate p1 - p2, and the row W_B[P1; .] through a weighted sum over the
 * first point; with the source chirps of the pairs as weights both are dense contractions that
 * groups of up to 64 pairs share (two reads of w_src per group, then two N x N DFTs per pair). In the
 * far field the source-side factors do not depend on (lambda, z): one set of sums serves every pair,
 * and a group of one entry (the far field, or a single pair) takes one pass over w_src.
 * The first call for a given shape records the sequence of launches in a hipGraph; later calls
 * with the same shape replay it.
 *   w_src          device N^4, read only.
 *   wavelength_m, z_m, weight   host arrays of n_pairs (> 0, > 0, >= 0).
 *   work           device scratch owned by the caller, at least wolf_batch_work_bytes(n, dtype)
 *                  bytes (overwritten).
 *   s_out          device n_pairs * N*N real; mu_out: device n_pairs * N*N complex.
 */
WOLF_API wolf_status wolf_propagate_batch(const void* w_src, int32_t n, double pitch_m, int32_t n_pairs,
                                          const double* wavelength_m, const double* z_m, const double* weight,
                                          int32_t farfield, int32_t kind, int32_t dtype, int32_t ip, int32_t jp,
                                          double s_floor_rel, void* work, void* s_out, void* mu_out, void* stream);

/*
 * wolf_propagate_polychromatic -- polychromatic light from one source on a common output grid
 * (the paper's Sec. 7 names polychromatic light as future work). The CSD at each frequency
 * propagates on its own (eq. W_general at wavelength_m[k] and distance z_m[k], Fresnel or far
 * field); on the output grid x = out_pitch_m (i - N/2), y = out_pitch_m (N/2 - j), which need not be
 * any pair's FFT grid, the weighted CSDs add: W = sum_k weight[k] W_k. s_out receives S of the sum
 * (Algorithm 4) and mu_out mu(P1, .) of the sum (Algorithm 5, floor s_floor_rel * max S).
 * The sums over the first point are shared by groups of 64 pairs as in wolf_propagate_batch, and
 * the DFTs of the FFT grid become chirp-z transforms at frequency out_pitch pitch / (lambda z);
 * the difference-coordinate sums then keep both signs of the offset.
 *   w_src          device N^4, read only.
 *   wavelength_m, z_m, weight   host arrays of n_pairs (> 0, > 0, >= 0); out_pitch_m > 0.
 *   work           device scratch of wolf_polychromatic_work_bytes(n, dtype) bytes (overwritten).
 *   s_out          device N*N real; mu_out: device N*N complex.
 */
WOLF_API wolf_status wolf_propagate_polychromatic(const void* w_src, int32_t n, double pitch_m, int32_t n_pairs,
                                                  const double* wavelength_m, const double* z_m, const double* weight,
                                                  double out_pitch_m, int32_t farfield, int32_t kind, int32_t dtype,
                                                  int32_t ip, int32_t jp, double s_floor_rel, void* work, void* s_out,
                                                  void* mu_out, void* stream);

/* Bytes of the work buffer of wolf_propagate_polychromatic (about 250 MB at N = 128 complex64); -1
 * if (n, dtype) is not supported. */
WOLF_API int64_t wolf_polychromatic_work_bytes(int32_t n, int32_t dtype);

/*
 * wolf_batch_work_bytes -- bytes of the `work` buffer that wolf_propagate_batch needs for (n, dtype):
 * the partial sums of one group of 64 pairs (16 + up to 48 N^2 x 64 complex chunks), three N^2 x 64
 * buffers and the tables (about 265 MB at N = 128 complex64); never an N^4 array. -1 if (n, dtype)
 * is not supported.
 */
WOLF_API int64_t wolf_batch_work_bytes(int32_t n, int32_t dtype);

/*
 * wolf_diag_embed -- out[p1; p2] = g[p1] if p1 == p2 else 0: the gradient with respect to W of a
 * loss that depends on W only through S = Re diag(W) (Algorithm 4), given g = dL/dS.
 *   g     device, N*N real (float32 for WOLF_C64, float64 for WOLF_C128).
 *   out   device, N^4 complex, written in full.
 */
WOLF_API wolf_status wolf_diag_embed(const void* g, int32_t n, int32_t dtype, void* out, void* stream);

/*
 * wolf_fit_gradient -- gradients of a loss with respect to the parameters of the custom-map source
 * W_A[p1; p2] = sqrt(I(p1)) sqrt(I(p2)) exp(-|xi1 - xi2|^2 / (2 sg^2)) (eq. W_def with a Gaussian
 * degree of coherence, amplitude 1, no geometry, no lens), given G_A = dL/dW_A in torch's complex
 * convention (dL/dRe + i dL/dIm), e.g. from wolf_propagate_adjoint:
 *   d_imap[p] = sum_q Re(conj(G_A[p;q]) + conj(G_A[q;p])) sqrt(I(q)) mu_g(p,q) / (2 sqrt(I(p)))
 *   d_sigma   = sum_{p,q} Re(conj(G_A[p;q]) W_A[p;q]) |xi_p - xi_q|^2 / sg^3
 *   ga       device N^4 complex of `dtype`.   imap: device N*N float32, every entry > 0.
 *   work     device scratch of at least wolf_fit_work_bytes(n, dtype) bytes (overwritten).
 *   d_imap   device N*N float32.   d_sigma: device, one float64.
 * N <= 128 (WOLF_EUNSUPPORTED above).
 */
WOLF_API wolf_status wolf_fit_gradient(const void* ga, const float* imap, int32_t n, double pitch_m, double sigma_g_m,
                                       int32_t dtype, void* work, float* d_imap, double* d_sigma, void* stream);
WOLF_API int64_t wolf_fit_work_bytes(int32_t n, int32_t dtype);

/*
 * wolf_chirp_table -- the FP64-built table of the quadratic-phase propagator q(z, xi) of
 * eq. (q_factor), along one axis: out[i] = exp(i pi (pitch (i - N/2))^2 / (lambda z)), i in [0, N).
 * The 2D propagator is out[i] * out[j]. It is the same table the propagation kernels build, minus
 * their (-1)^i centring factor.
 *   out   device, N complex of `dtype`.
 */
WOLF_API wolf_status wolf_chirp_table(int32_t n, double pitch_m, double wavelength_m, double z_m, int32_t dtype,
                                      void* out, void* stream);

/*
 * Schedule of the propagation passes for one (n, dtype). The operator factorises over the four
 * axes (see wolf_propagate_fresnel), so its passes can be grouped and ordered freely.
 *   fused_slab  1: one pass does both second-point axes, one N x N slab per workgroup in LDS
 *                  (needs N^2 elements <= 160 KB of LDS). 2: the same pass on a persistent grid
 *                  (as many workgroups as are resident), each loading the next slab into the L2
 *                  while it transforms the current one. 3: one slab per workgroup with its exchanges
 *                  through a buffer of N/2 rows (32 <= N <= 128; two resident workgroups per CU in
 *                  complex64, and it fits complex128 at N = 128). 0: a row pass and an i2 pass instead.
 *   slab_chunk  fused_slab = 0: slabs per chunk of the row + i2 pass pair (0 = all), a power-of-two
 *               divisor of N^2; in place, chunks of whole i1 planes also take their j1 pass at once, and
 *               the i1 pass then runs over all columns in one launch. fused_slab > 0: 0 or N^2 runs the slab pass over all slabs at once; a
 *               smaller power-of-two multiple of N makes in-place calls (and wolf_propagate_source) run it
 *               over groups of that many slabs (whole i1 planes), each followed at once by the j1 pass of
 *               its planes while they are still in the 256 MB Infinity Cache, and then the i1 pass over
 *               all columns in one launch; out-of-place calls keep the paired passes over col_chunk
 *               chunks. Ignored by the cooperative pass.
 *   col_chunk   columns m2 per chunk of the j1 + i1 pass pair (0 = all). A power-of-two divisor
 *               of N^2 and a multiple of the axis tile. Chunks of tens of MB let the second pass of
 *               a pair read the first pass's output from the Infinity Cache instead of HBM.
 *   coop_cols   > 0: the first-point axes (j1, i1) run as one cooperative pass (one HBM sweep instead
 *               of two). The N^2 columns are cut into tiles of coop_cols columns (64, 128 or 256 bytes
 *               of each row: 8, 16 or 32 columns in complex64, 4, 8 or 16 in complex128), and each tile
 *               is transformed along j1 and then along i1 by the workgroups of one XCD, through that
 *               XCD's L2. Needs N = 32, 64 or 128 and a tile of at most 2 MB. 0: two passes over
 *               column chunks (col_chunk).
 *   coop_lookahead  tiles whose j1 phase may run ahead of their i1 phase on an XCD (1..8).
 * wolf_set_plan with fused_slab = slab_chunk = col_chunk = -1 restores the built-in default.
 * A plan that is not valid for (n, dtype) returns WOLF_EINVAL. Plans are per process.
 */
WOLF_API wolf_status wolf_set_plan(int32_t n, int32_t dtype, int32_t fused_slab, int64_t slab_chunk,
                                   int64_t col_chunk, int32_t coop_cols, int32_t coop_lookahead);
WOLF_API wolf_status wolf_get_plan(int32_t n, int32_t dtype, int32_t* fused_slab, int64_t* slab_chunk,
                                   int64_t* col_chunk, int32_t* coop_cols, int32_t* coop_lookahead);

/*
 * wolf_coop_error_flag -- 1 if the last cooperative pass on `stream` gave up waiting for a tile (a
 * wait is bounded to 20 ms; the result of that call is then wrong), else 0. Synchronises the stream.
 * The flag is cleared at the start of every cooperative pass.
 */
WOLF_API wolf_status wolf_coop_error_flag(void* stream, int32_t* flag);

/*
 * Autotuner: times every candidate schedule for (n, dtype) on `work` with HIP events on `stream`.
 * Each candidate gets one warm-up run and `reps` timed runs. The fastest is kept for later calls.
 * `work` is device memory of N^4 elements, overwritten (its contents do not matter).
 * Blocks the calling thread until the timing is done. best_ms (optional) receives the best time.
 */
WOLF_API wolf_status wolf_autotune(int32_t n, int32_t dtype, void* work, int32_t reps, double* best_ms,
                                   void* stream);

/*
 * wolf_memory_ceiling -- a measurement aid, not an operation of the paper: one streaming pass over
 * `bytes` of `buf`, to compare the propagation passes with what HBM delivers in practice.
 *   mode 0: in place, every byte read and written back (the access pattern of an in-place pass);
 *   mode 1: every byte written (the builder's pattern);
 *   mode 2: every byte read (the observables-only passes);
 *   modes 3, 4, 5: the same three with the nontemporal hint on every load and store.
 *   buf     device memory owned by the caller; modes 0, 2, 3, 5 leave its contents unchanged, 1 and 4
 *           write zeros.
 *   bytes   a positive multiple of 16384. WOLF_EINVAL otherwise.
 */
WOLF_API wolf_status wolf_memory_ceiling(void* buf, int64_t bytes, int32_t mode, void* stream);

/* Output pitch dx = lambda z / (N pitch) of eq. (spatial_resolution). Pure host arithmetic. */
WOLF_API double wolf_output_pitch(int32_t n, double pitch_m, double wavelength_m, double z_m);

WOLF_API const char* wolf_status_string(wolf_status s);
/* Details of the last failed call on this host thread (empty if none). */
WOLF_API const char* wolf_last_error_message(void);
WOLF_API int32_t wolf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WOLF_H */
