// C-ABI layer of libwolf: argument validation, buffer checks, per-device scratch and dispatch.
// No exception crosses this layer. Every entry point returns a wolf_status.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/wolf.h"
#include "wolf_internal.hpp"

namespace {

thread_local std::string g_last_error;

wolf_status fail(wolf_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
wolf_status fail(wolf_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

bool supported_n(int32_t n) { return n >= 2 && n <= 256 && (n & (n - 1)) == 0; }
// Sizes that the source builder, the observables and wolf_propagate_padded accept: any even N.
bool even_n(int32_t n) { return n >= 2 && n <= 256 && n % 2 == 0; }
bool pos_finite(double v) { return std::isfinite(v) && v > 0.0; }
size_t elem_bytes(int32_t dtype) { return dtype == WOLF_C64 ? 8 : 16; }
size_t real_bytes(int32_t dtype) { return dtype == WOLF_C64 ? 4 : 8; }
size_t n4(int32_t n) { return (size_t)n * n * n * n; }

// A device buffer of at least `bytes`, inside one allocation on the current device.
wolf_status check_buf(const void* p, size_t bytes, const char* what) {
  if (p == nullptr) return fail(WOLF_EINVAL, "%s: null pointer", what);
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof attr);
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(WOLF_EINVAL, "%s: not a device pointer (%s)", what, hipGetErrorString(e));
  }
  if (attr.type != hipMemoryTypeDevice) return fail(WOLF_EINVAL, "%s: not device memory", what);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != attr.device)
    return fail(WOLF_EINVAL, "%s: buffer is on device %d, current device is %d", what, attr.device, dev);
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  e = hipMemGetAddressRange(&base, &size, const_cast<void*>(p));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(WOLF_EINVAL, "%s: cannot query the allocation (%s)", what, hipGetErrorString(e));
  }
  const char* b = static_cast<const char*>(base);
  const char* q = static_cast<const char*>(p);
  if (q < b || (size_t)(q - b) + bytes > size)
    return fail(WOLF_EINVAL, "%s: buffer too small (%zu bytes needed past the pointer, allocation has %zu)", what,
                bytes, size - (size_t)(q - b));
  return WOLF_OK;
}

// [a, a + na) and [b, b + nb) share a byte.
bool intervals_overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + nb && y < x + na;
}

bool partial_overlap(const void* a, const void* b, size_t bytes) {
  if (a == b) return false;
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + bytes && y < x + bytes;
}

wolf_status launched(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(WOLF_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  g_last_error.clear();
  return WOLF_OK;
}

// Per-stream scratch owned by the library (one per (device, stream) pair, never freed):
// reduction keys and N^2 reals for mu, or the tile counters of the cooperative pass. Work on one
// stream is ordered, so its calls can share the block. Work on other streams uses other blocks.
constexpr size_t kScratchBytes = 256 + (size_t)256 * 256 * 8;
std::mutex g_scratch_mu;
std::map<std::pair<int, uintptr_t>, void*> g_scratch;

wolf_status stream_scratch(void* stream, void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(WOLF_EDEVICE, "hipGetDevice failed");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  const auto key = std::make_pair(dev, (uintptr_t)stream);
  auto it = g_scratch.find(key);
  if (it != g_scratch.end()) {
    *out = it->second;
    return WOLF_OK;
  }
  // The library allocates only outside graph capture: a stream's first call that needs the scratch
  // must not be captured.
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(static_cast<hipStream_t>(stream), &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    return fail(WOLF_EINVAL,
                "the first call on a stream that needs the library's scratch (mu, the cooperative pass) must run "
                "outside graph capture; call it once before capturing");
  void* p = nullptr;
  static_assert(kScratchBytes >= (16 + 256 * 256) * sizeof(unsigned), "coop counters fit");
  if (hipMalloc(&p, kScratchBytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(WOLF_ENOMEM, "cannot allocate %zu bytes of device scratch", kScratchBytes);
  }
  g_scratch[key] = p;
  *out = p;
  return WOLF_OK;
}

// ---------------------------------------------------------------------------------------------
// The propagation operator and its schedule.
// ---------------------------------------------------------------------------------------------
wolf::OperatorTables make_op(int32_t n, double pitch, double lam, double z, bool farfield, int32_t kind,
                             bool adjoint) {
  using wolf::Chirp;
  const double dx = lam * z / ((double)n * pitch);
  const double c = kind == WOLF_PRIMARY ? 1.0 / ((4.0 * M_PI * z) * (4.0 * M_PI * z)) : 1.0 / ((lam * z) * (lam * z));
  const double a_src = farfield ? 0.0 : pitch * pitch / (lam * z);
  const double a_out = dx * dx / (lam * z);
  wolf::OperatorTables op;
  if (!adjoint) {
    // Second point: q(xi) (-1)^n, direct DFT, q(x) (-1)^k. First point: conjugates, inverse DFT.
    op.pre2 = Chirp{a_src, 1.0, +1, 1};
    op.post2 = Chirp{a_out, 1.0, +1, 1};
    op.sign2 = -1;
    op.pre1 = Chirp{a_src, 1.0, -1, 1};
    op.post1 = Chirp{a_out, 1.0, -1, 1};
    op.sign1 = +1;
  } else {
    // Adjoint: first point q(x) (-1)^k, direct DFT, q(xi) (-1)^n; second point conjugates, inverse.
    op.pre1 = Chirp{a_out, 1.0, +1, 1};
    op.post1 = Chirp{a_src, 1.0, +1, 1};
    op.sign1 = -1;
    op.pre2 = Chirp{a_out, 1.0, -1, 1};
    op.post2 = Chirp{a_src, 1.0, -1, 1};
    op.sign2 = +1;
  }
  op.scale = c * pitch * pitch * pitch * pitch;
  op.pupil = wolf::Pupil{0, 0};
  return op;
}

// A thin lens T = P q*(f, x) at the input plane (Sec. 2.2): W+ = T*(x1) W T(x2) before a Fresnel
// propagation. q*(f) times the source chirp q(z) is one chirp q(z f / (f - z)) (eqs. qprop), so the
// lens only changes the source-side chirp rate; the pupil is applied while the input is loaded.
struct LensSpec {
  double focal_m;  // 0: no lens phase
  int32_t pupil_geometry;
  double pupil_radius_m;
};

// The batch extracts S and mu(P, .) without an N^4 output: the sums over the first point are shared
// contractions of all pairs of a group (wolf_pairs.hip); a group of one entry (the far field, whose
// sums every pair shares, or a single pair) takes one HBM-bound pass.
size_t batch_work_bytes(int32_t n, int32_t dtype) {
  return dtype == WOLF_C64 ? wolf::pair_work_bytes<float2>(n) : wolf::pair_work_bytes<double2>(n);
}

// Groups of up to 64 pairs: their raw sums from one pair-sums pass, then one emit per pair. In the far
// field the sums do not depend on (lambda, z): one group of one chirp-free entry serves every pair.
template <class T>
hipError_t record_pair_groups(int32_t n, const T* w_src, double pitch, int32_t n_pairs, const double* lam,
                              const double* z, const double* weight, bool farfield, int32_t kind, int32_t ip, int32_t jp,
                              double floor_rel, void* work, typename wolf::real_of<T>::type* s_out, T* mu_out,
                              hipStream_t st) {
  const size_t nn = (size_t)n * n;
  constexpr int G = wolf::kPairGroup;
  std::vector<wolf::ObsSums<T>> sums(G);
  double a_src[G];
  hipError_t e = hipSuccess;
  for (int k0 = 0; k0 < n_pairs && e == hipSuccess; k0 += G) {
    const int cnt = farfield ? 1 : std::min(G, n_pairs - k0);
    for (int k = 0; k < cnt; ++k) a_src[k] = farfield ? 0.0 : pitch * pitch / (lam[k0 + k] * z[k0 + k]);
    if (k0 == 0 || !farfield) e = wolf::launch_pair_sums<T>(n, w_src, a_src, cnt, ip, jp, work, sums.data(), st);
    // In the far field every pair reads the one set of sums; emit in launches of up to G pairs.
    const int last = farfield ? n_pairs : std::min(n_pairs, k0 + G);
    for (int e0 = k0; e0 < last && e == hipSuccess; e0 += G) {
      const int ecnt = std::min(G, last - e0);
      double c[G], a_out[G];
      for (int k = 0; k < ecnt; ++k) {
        const wolf::OperatorTables op = make_op(n, pitch, lam[e0 + k], z[e0 + k], farfield, kind, false);
        c[k] = op.scale * weight[e0 + k];
        a_out[k] = op.post2.alpha;
      }
      e = wolf::launch_pair_emit<T>(n, sums[farfield ? 0 : e0 - k0], farfield, ecnt, c, a_out, ip, jp, floor_rel,
                                    s_out + e0 * nn, mu_out + e0 * nn, st);
    }
    if (farfield) break;
  }
  return e;
}

hipError_t record_batch_pairs(int32_t n, const void* w_src, double pitch, int32_t n_pairs, const double* lam,
                              const double* z, const double* weight, bool farfield, int32_t kind, int32_t dtype,
                              int32_t ip, int32_t jp, double floor_rel, void* work, void* s_out, void* mu_out,
                              hipStream_t st) {
  if (dtype == WOLF_C64)
    return record_pair_groups<float2>(n, (const float2*)w_src, pitch, n_pairs, lam, z, weight, farfield, kind, ip, jp,
                                      floor_rel, work, (float*)s_out, (float2*)mu_out, st);
  return record_pair_groups<double2>(n, (const double2*)w_src, pitch, n_pairs, lam, z, weight, farfield, kind, ip, jp,
                                     floor_rel, work, (double*)s_out, (double2*)mu_out, st);
}

struct BatchGraph {
  std::vector<double> key;
  hipGraphExec_t exec;
};
std::mutex g_batch_mu;
std::vector<BatchGraph> g_batch_graphs;  // recorded batch graphs (most recent last, at most 8)


std::mutex g_plan_mu;
std::map<std::pair<int, int>, wolf::Plan> g_plans;  // (n, dtype) -> plan chosen by wolf_set_plan / autotune

bool plan_valid(int32_t n, int32_t dtype, const wolf::Plan& p) {
  const long long nn = (long long)n * n;
  const int c = wolf::axis_tile_cols(n, (int)elem_bytes(dtype));
  if (p.fused_slab < 0 || p.fused_slab > 3) return false;
  if (p.fused_slab == 3) {
    if (!(dtype == WOLF_C64 ? wolf::half_slab_supported<float2>(n) : wolf::half_slab_supported<double2>(n))) return false;
  } else if (p.fused_slab &&
             !(dtype == WOLF_C64 ? wolf::slab_pass_supported<float2>(n) : wolf::slab_pass_supported<double2>(n))) {
    return false;
  }
  if (p.col_chunk < 0 || p.col_chunk > nn || (p.col_chunk > 0 && (p.col_chunk % c != 0 || nn % p.col_chunk != 0)))
    return false;
  if (p.slab_chunk < 0 || p.slab_chunk > nn || (p.slab_chunk > 0 && nn % p.slab_chunk != 0)) return false;
  // The row pass over a chunk of slabs needs whole workgroups of rows; a group of the slab pass is
  // whole i1 planes.
  if (!p.fused_slab && p.slab_chunk > 0 && (p.slab_chunk * n) % wolf::row_pass_rows(n) != 0) return false;
  if (p.fused_slab && p.slab_chunk > 0 && p.slab_chunk % n != 0) return false;
  if (p.coop != 0 && p.coop != 1) return false;
  if (p.coop) {
    if (!wolf::coop_supported(n, (int)elem_bytes(dtype), p.coop_cols)) return false;
    if (p.coop_lookahead < 1 || p.coop_lookahead > 8) return false;
  }
  return true;
}

// Slabs per chunk of the row + i2 pass pair: about 64 MB, so that the i2 pass reads the row pass's
// output from the Infinity Cache.
long long row_chunk_slabs(int32_t n, int32_t dtype) {
  const long long nn = (long long)n * n, eb = (long long)elem_bytes(dtype);
  long long slabs = nn;
  while (slabs > 1 && slabs * nn * eb > (64ll << 20) && ((slabs >> 1) * n) % wolf::row_pass_rows(n) == 0) slabs >>= 1;
  return slabs;
}

wolf::Plan default_plan(int32_t n, int32_t dtype) {
  wolf::Plan p{};
  p.fused_slab = dtype == WOLF_C64 ? wolf::slab_pass_supported<float2>(n) : wolf::slab_pass_supported<double2>(n);
  // Where the whole slab does not fit the LDS, the half-buffer slab pass still saves a sweep.
  if (!p.fused_slab && (dtype == WOLF_C64 ? wolf::half_slab_supported<float2>(n) : wolf::half_slab_supported<double2>(n)))
    p.fused_slab = 3;
  const long long nn = (long long)n * n;
  const long long eb = (long long)elem_bytes(dtype);
  // Chunks of about 64 MB, so that the pass pair reuses the chunk from the 256 MB Infinity Cache.
  const long long target = 64ll << 20;
  const int c = wolf::axis_tile_cols(n, (int)elem_bytes(dtype));
  long long cols = nn;
  while (cols > c && cols * nn * eb > target) cols >>= 1;
  p.col_chunk = cols;
  p.slab_chunk = p.fused_slab ? 0 : row_chunk_slabs(n, dtype);
  p.coop = 0;  // opt in through wolf_set_plan / wolf_autotune
  p.coop_cols = 0;
  p.coop_lookahead = 1;
  if (n == 128) {
    // Measured on MI355X (in-place propagation, N = 128): the half-buffer slab pass is the fastest in
    // both precisions; complex64 with 1024-column chunks of the first-point pair (2.38 ms against
    // 2.48 ms for the whole-slab pass), complex128 unchunked (4.94 ms against 6.49 ms for the row pass).
    p.fused_slab = 3;
    p.col_chunk = dtype == WOLF_C64 ? 1024 : nn;
    if (dtype == WOLF_C64) {
      // In place, the grouped schedule: the slab pass and the j1 pass over groups of 16 i1 planes (256 MB),
      // then the i1 pass in one launch: 2.31-2.37 ms against 2.39-2.40 ms for the paired chunks (groups of
      // 4 planes: 2.80 ms, launch-bound). Out of place the paired 1024-column chunks: 2.43 ms against 2.50.
      p.slab_chunk = 16 * (long long)n;
    }
  }
  if (n == 64 && dtype == WOLF_C64) {
    // Measured on the N = 64 top-hat + lens workload (build + in-place propagation): the half-buffer slab
    // pass (two workgroups per CU) and unchunked first-point passes, 0.148 ms, against 0.154 ms for the
    // whole-slab pass with 2048-column chunks; the whole 134 MB array sits in the memory-side cache anyway.
    p.fused_slab = 3;
    p.slab_chunk = 0;
    p.col_chunk = nn;
  }
  if (n == 256) {
    // Measured at N = 256 complex64, in place: row, i2 and j1 passes over chunks of 512 slabs (two i1 planes,
    // 256 MB, in the memory-side cache), then the i1 pass: 45.8 ms, against 49.1 ms (512) and 50.8 ms (256)
    // with the j1 pass after all chunks, 54.8 ms with 1024-slab chunks, and 58 ms with 64 MB chunks of both.
    p.slab_chunk = 512;
    p.col_chunk = nn;
  }
  return p;
}

// Column chunk of the paired j1/i1 passes that the grouped candidates of the autotuner carry (their
// out-of-place schedule): the built-in one for (n, dtype).
long long c_best_paired(int32_t n, int32_t dtype) { return default_plan(n, dtype).col_chunk; }

wolf::Plan plan_for(int32_t n, int32_t dtype) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  auto it = g_plans.find({n, dtype});
  return it != g_plans.end() ? it->second : default_plan(n, dtype);
}

template <class T>
wolf_status run_operator(const T* in, T* out, int32_t n, int32_t dtype, const wolf::OperatorTables& op,
                         hipStream_t st) {
  const wolf::Plan plan = plan_for(n, dtype);
  void* scratch = nullptr;
  if (plan.coop) {
    const wolf_status s = stream_scratch(st, &scratch);
    if (s != WOLF_OK) return s;
  }
  const hipError_t e = wolf::launch_operator<T>(n, in, out, op, plan, scratch, st);
  if (e != hipSuccess) return fail(WOLF_EDEVICE, "propagation launch: %s", hipGetErrorString(e));
  g_last_error.clear();
  return WOLF_OK;
}

wolf_status propagate_common(const void* w_in, void* w_out, int32_t n, double pitch, double lam, double z,
                             bool farfield, int32_t kind, int32_t dtype, bool adjoint, double* out_pitch,
                             void* stream, const char* who, const LensSpec* lens = nullptr) {
  if (!supported_n(n)) return fail(WOLF_EUNSUPPORTED, "%s: N=%d is not a power of two in [2, 256]", who, n);
  if (dtype != WOLF_C64 && dtype != WOLF_C128) return fail(WOLF_EINVAL, "%s: bad dtype %d", who, dtype);
  if (!pos_finite(pitch) || !pos_finite(lam) || !pos_finite(z))
    return fail(WOLF_EINVAL, "%s: pitch, wavelength and z must be finite and > 0", who);
  if (kind != WOLF_SECONDARY && kind != WOLF_PRIMARY) return fail(WOLF_EINVAL, "%s: bad kind %d", who, kind);
  if (lens) {
    if (!std::isfinite(lens->focal_m)) return fail(WOLF_EINVAL, "%s: focal_m must be finite (0 = no lens phase)", who);
    if (lens->pupil_geometry != WOLF_GEO_NONE && lens->pupil_geometry != WOLF_GEO_CIRCLE &&
        lens->pupil_geometry != WOLF_GEO_SQUARE)
      return fail(WOLF_EINVAL, "%s: pupil_geometry must be NONE, CIRCLE or SQUARE", who);
    if (lens->pupil_geometry != WOLF_GEO_NONE &&
        (!pos_finite(lens->pupil_radius_m) || lens->pupil_radius_m / pitch > 1e6))
      return fail(WOLF_EINVAL, "%s: pupil_radius_m must be finite, > 0 and < 1e6 pixels", who);
  }
  const size_t bytes = n4(n) * elem_bytes(dtype);
  wolf_status s;
  if ((s = check_buf(w_in, bytes, "input")) != WOLF_OK) return s;
  if ((s = check_buf(w_out, bytes, "output")) != WOLF_OK) return s;
  if (partial_overlap(w_in, w_out, bytes)) return fail(WOLF_EINVAL, "%s: input and output partly overlap", who);
  wolf::OperatorTables op = make_op(n, pitch, lam, z, farfield, kind, adjoint);
  if (lens) {
    if (lens->focal_m != 0.0) {
      const double a = pitch * pitch * (1.0 / z - 1.0 / lens->focal_m) / lam;
      op.pre1.alpha = a;
      op.pre2.alpha = a;
    }
    if (lens->pupil_geometry != WOLF_GEO_NONE) {
      const double rho = lens->pupil_radius_m / pitch;
      op.pupil = wolf::Pupil{lens->pupil_geometry, (long long)std::floor(rho * rho * (1.0 + 1e-9))};
    }
  }
  if (out_pitch) *out_pitch = lam * z / ((double)n * pitch);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype == WOLF_C64)
    return run_operator<float2>(static_cast<const float2*>(w_in), static_cast<float2*>(w_out), n, dtype, op, st);
  return run_operator<double2>(static_cast<const double2*>(w_in), static_cast<double2*>(w_out), n, dtype, op, st);
}

// Validates a source description and converts it to pixel units (shared by the builder and the
// propagation of a source).
wolf_status source_params(const wolf_source* src, int32_t n, double pitch_m, wolf::SourceParams* out, const char* who) {
  if (src == nullptr) return fail(WOLF_EINVAL, "%s: null source", who);
  if (!pos_finite(pitch_m)) return fail(WOLF_EINVAL, "%s: pitch must be finite and > 0", who);
  if (src->model < 0 || src->model > 3) return fail(WOLF_EINVAL, "%s: bad model %d", who, src->model);
  if (src->geometry < 0 || src->geometry > 4) return fail(WOLF_EINVAL, "%s: bad geometry", who);
  if (!std::isfinite(src->amplitude) || src->amplitude < 0) return fail(WOLF_EINVAL, "amplitude must be >= 0");
  const bool uses_s = src->model == WOLF_MODEL_GSM;
  const bool uses_g = src->model == WOLF_MODEL_GSM || src->model == WOLF_MODEL_MAP;
  if (uses_s && !(src->sigma_s_m > 0)) return fail(WOLF_EINVAL, "sigma_s_m must be > 0 (or +inf)");
  if (uses_g && !(src->sigma_g_m > 0)) return fail(WOLF_EINVAL, "sigma_g_m must be > 0 (or +inf)");
  wolf::SourceParams sp{};
  sp.model = src->model;
  sp.geometry = src->geometry;
  sp.amplitude = src->amplitude;
  sp.inv4s2_px = (uses_s && !std::isinf(src->sigma_s_m)) ? pitch_m * pitch_m / (4.0 * src->sigma_s_m * src->sigma_s_m) : 0.0;
  sp.inv2g2_px = (uses_g && !std::isinf(src->sigma_g_m)) ? pitch_m * pitch_m / (2.0 * src->sigma_g_m * src->sigma_g_m) : 0.0;
  sp.inv4s2 = 0.0;
  auto thresh = [&](double r) {
    const double rho = r / pitch_m;
    return (long long)std::floor(rho * rho * (1.0 + 1e-9));
  };
  if (src->geometry == WOLF_GEO_CIRCLE || src->geometry == WOLF_GEO_SQUARE || src->geometry == WOLF_GEO_ANNULUS) {
    if (!pos_finite(src->geo_r0_m)) return fail(WOLF_EINVAL, "geo_r0_m must be finite and > 0");
    if (src->geo_r0_m / pitch_m > 1e6) return fail(WOLF_EINVAL, "geo_r0_m too large");
    sp.t0 = thresh(src->geo_r0_m);
  }
  if (src->geometry == WOLF_GEO_ANNULUS) {
    if (!(src->geo_r1_m >= 0 && src->geo_r1_m < src->geo_r0_m)) return fail(WOLF_EINVAL, "need 0 <= geo_r1_m < geo_r0_m");
    sp.t1 = thresh(src->geo_r1_m);
  }
  wolf_status s;
  if (src->model == WOLF_MODEL_MAP) {
    if ((s = check_buf(src->intensity_map, (size_t)n * n * 4, "intensity_map")) != WOLF_OK) return s;
    sp.imap = src->intensity_map;
  }
  if (src->geometry == WOLF_GEO_MASK) {
    if ((s = check_buf(src->mask, (size_t)n * n, "mask")) != WOLF_OK) return s;
    sp.mask = src->mask;
  }
  if (src->lens_focal_m != 0.0) {
    if (!std::isfinite(src->lens_focal_m) || !pos_finite(src->wavelength_m))
      return fail(WOLF_EINVAL, "lens needs a finite focal length and a wavelength > 0");
    sp.lens_alpha = pitch_m * pitch_m / (src->wavelength_m * src->lens_focal_m);
  }
  *out = sp;
  return WOLF_OK;
}

// Arguments of the degree of coherence (both entry points): validated, and the buffers checked.
wolf_status coherence_args(const void* w, int32_t n, int32_t dtype, int32_t ip, int32_t jp, double s_floor_rel,
                           void* mu_out, const char* who) {
  if (!even_n(n)) return fail(WOLF_EUNSUPPORTED, "%s: N=%d (even, 2..256)", who, n);
  if (dtype != WOLF_C64 && dtype != WOLF_C128) return fail(WOLF_EINVAL, "%s: bad dtype", who);
  const bool full = ip == -1 && jp == -1;
  if (!full && (ip < 0 || ip >= n || jp < 0 || jp >= n))
    return fail(WOLF_EINVAL, "%s: (ip, jp) must be in [0, N) or both -1", who);
  if (!std::isfinite(s_floor_rel) || s_floor_rel < 0) return fail(WOLF_EINVAL, "%s: s_floor_rel must be >= 0", who);
  const size_t eb = elem_bytes(dtype);
  wolf_status s;
  if ((s = check_buf(w, n4(n) * eb, "w")) != WOLF_OK) return s;
  const size_t out_bytes = full ? n4(n) * eb : (size_t)n * n * eb;
  if ((s = check_buf(mu_out, out_bytes, "mu_out")) != WOLF_OK) return s;
  if (intervals_overlap(w, n4(n) * eb, mu_out, out_bytes))
    return fail(WOLF_EINVAL, "%s: mu_out overlaps w (mu is never computed in place)", who);
  return WOLF_OK;
}

wolf_status coherence_launch(const void* w, int32_t n, int32_t dtype, int32_t ip, int32_t jp, double s_floor_rel,
                             void* mu_out, void* scratch, void* stream, const char* who) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool full = ip == -1 && jp == -1;
  const int i = full ? -1 : ip, j = full ? -1 : jp;
  hipError_t e = dtype == WOLF_C64
                     ? wolf::launch_coherence<float2>(n, static_cast<const float2*>(w), i, j, s_floor_rel,
                                                      static_cast<float2*>(mu_out), scratch, st)
                     : wolf::launch_coherence<double2>(n, static_cast<const double2*>(w), i, j, s_floor_rel,
                                                       static_cast<double2*>(mu_out), scratch, st);
  return launched(e, who);
}

}  // namespace

extern "C" {

WOLF_API int32_t wolf_version(void) { return 1; }

WOLF_API const char* wolf_status_string(wolf_status s) {
  switch (s) {
    case WOLF_OK: return "WOLF_OK";
    case WOLF_EINVAL: return "WOLF_EINVAL: invalid argument";
    case WOLF_EUNSUPPORTED: return "WOLF_EUNSUPPORTED: unsupported size";
    case WOLF_ENOMEM: return "WOLF_ENOMEM: device scratch allocation failed";
    case WOLF_EDEVICE: return "WOLF_EDEVICE: HIP error";
    default: return "unknown wolf_status";
  }
}

WOLF_API const char* wolf_last_error_message(void) { return g_last_error.c_str(); }

WOLF_API double wolf_output_pitch(int32_t n, double pitch_m, double wavelength_m, double z_m) {
  return wavelength_m * z_m / ((double)n * pitch_m);
}

WOLF_API wolf_status wolf_propagate_fresnel(const void* w_in, void* w_out, int32_t n, double pitch_m,
                                            double wavelength_m, double z_m, int32_t kind, int32_t dtype,
                                            double* out_pitch_m, void* stream) {
  return propagate_common(w_in, w_out, n, pitch_m, wavelength_m, z_m, false, kind, dtype, false, out_pitch_m,
                          stream, "wolf_propagate_fresnel");
}

WOLF_API wolf_status wolf_propagate_farfield(const void* w_in, void* w_out, int32_t n, double pitch_m,
                                             double wavelength_m, double z_m, int32_t kind, int32_t dtype,
                                             double* out_pitch_m, void* stream) {
  return propagate_common(w_in, w_out, n, pitch_m, wavelength_m, z_m, true, kind, dtype, false, out_pitch_m,
                          stream, "wolf_propagate_farfield");
}

WOLF_API wolf_status wolf_propagate_lens(const void* w_in, void* w_out, int32_t n, double pitch_m,
                                         double wavelength_m, double focal_m, int32_t pupil_geometry,
                                         double pupil_radius_m, double z_m, int32_t kind, int32_t dtype,
                                         double* out_pitch_m, void* stream) {
  const LensSpec lens{focal_m, pupil_geometry, pupil_radius_m};
  return propagate_common(w_in, w_out, n, pitch_m, wavelength_m, z_m, false, kind, dtype, false, out_pitch_m,
                          stream, "wolf_propagate_lens", &lens);
}

WOLF_API int64_t wolf_direct_work_bytes(int32_t n, int32_t dtype) {
  if (!supported_n(n) || n > 128 || (dtype != WOLF_C64 && dtype != WOLF_C128)) return -1;
  return (int64_t)wolf::direct_work_bytes(n, (int)elem_bytes(dtype));
}

WOLF_API wolf_status wolf_propagate_direct(const void* w_in, void* w_out, int32_t n, double pitch_m,
                                           double wavelength_m, double z_m, int32_t kind, int32_t dtype, void* work,
                                           double* out_pitch_m, void* stream) {
  const char* who = "wolf_propagate_direct";
  if (!supported_n(n) || n > 128) return fail(WOLF_EUNSUPPORTED, "%s: N=%d (powers of two up to 128)", who, n);
  if (dtype != WOLF_C64 && dtype != WOLF_C128) return fail(WOLF_EINVAL, "%s: bad dtype", who);
  if (!pos_finite(pitch_m) || !pos_finite(wavelength_m) || !pos_finite(z_m))
    return fail(WOLF_EINVAL, "%s: pitch, wavelength and z must be finite and > 0", who);
  if (kind != WOLF_SECONDARY && kind != WOLF_PRIMARY) return fail(WOLF_EINVAL, "%s: bad kind", who);
  const size_t bytes = n4(n) * elem_bytes(dtype), wb = wolf::direct_work_bytes(n, (int)elem_bytes(dtype));
  wolf_status s;
  if ((s = check_buf(w_in, bytes, "w_in")) != WOLF_OK) return s;
  if ((s = check_buf(w_out, bytes, "w_out")) != WOLF_OK) return s;
  if ((s = check_buf(work, wb, "work")) != WOLF_OK) return s;
  if (partial_overlap(w_in, w_out, bytes) || intervals_overlap(work, wb, w_in, bytes) ||
      intervals_overlap(work, wb, w_out, bytes))
    return fail(WOLF_EINVAL, "%s: buffers overlap", who);
  if (out_pitch_m) *out_pitch_m = wavelength_m * z_m / ((double)n * pitch_m);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int primary = kind == WOLF_PRIMARY ? 1 : 0;
  const hipError_t e =
      dtype == WOLF_C64
          ? wolf::launch_direct<float2>(n, (const float2*)w_in, (float2*)w_out, work, pitch_m, wavelength_m, z_m,
                                        primary, st)
          : wolf::launch_direct<double2>(n, (const double2*)w_in, (double2*)w_out, work, pitch_m, wavelength_m, z_m,
                                         primary, st);
  return launched(e, who);
}

WOLF_API wolf_status wolf_propagate_padded(const void* w_in, void* w_out, int32_t n, int32_t n_fft, double pitch_m,
                                           double wavelength_m, double z_m, int32_t farfield, int32_t kind, int32_t dtype,
                                           void* work, double* out_pitch_m, void* stream) {
  const char* who = "wolf_propagate_padded";
  if (!even_n(n)) return fail(WOLF_EUNSUPPORTED, "%s: N=%d (even, 2..256)", who, n);
  if (!wolf::dense_supported(n, n_fft)) return fail(WOLF_EUNSUPPORTED, "%s: n_fft=%d (N..2048)", who, n_fft);
  if (dtype != WOLF_C64 && dtype != WOLF_C128) return fail(WOLF_EINVAL, "%s: bad dtype", who);
  if (!pos_finite(pitch_m) || !pos_finite(wavelength_m) || !pos_finite(z_m))
    return fail(WOLF_EINVAL, "%s: pitch, wavelength and z must be finite and > 0", who);
  if (farfield != 0 && farfield != 1) return fail(WOLF_EINVAL, "%s: farfield must be 0 or 1", who);
  if (kind != WOLF_SECONDARY && kind != WOLF_PRIMARY) return fail(WOLF_EINVAL, "%s: bad kind", who);
  const size_t bytes = n4(n) * elem_bytes(dtype);
  wolf_status s;
  if ((s = check_buf(w_in, bytes, "w_in")) != WOLF_OK) return s;
  if ((s = check_buf(w_out, bytes, "w_out")) != WOLF_OK) return s;
  if ((s = check_buf(work, bytes, "work")) != WOLF_OK) return s;
  if (partial_overlap(w_in, w_out, bytes) || intervals_overlap(work, bytes, w_in, bytes) ||
      intervals_overlap(work, bytes, w_out, bytes))
    return fail(WOLF_EINVAL, "%s: buffers overlap", who);
  // Tables of the dense passes: chirps on the N-point grids, no (-1)^n (the centring is exact in
  // the kernel index), output pitch lambda z / (n_fft pitch).
  const double dx = wavelength_m * z_m / ((double)n_fft * pitch_m);
  const double c = kind == WOLF_PRIMARY ? 1.0 / ((4.0 * M_PI * z_m) * (4.0 * M_PI * z_m))
                                        : 1.0 / ((wavelength_m * z_m) * (wavelength_m * z_m));
  const double a_src = farfield ? 0.0 : pitch_m * pitch_m / (wavelength_m * z_m);
  const double a_out = dx * dx / (wavelength_m * z_m);
  // A power-of-two n_fft takes zero-padded FFTs (the centring as (-1)^n in the tables); any other
  // n_fft the dense passes (the centring exact in the kernel index, no (-1)^n).
  const bool fft = wolf::pad_fft_supported(n, n_fft);
  const int chk = fft ? 1 : 0;
  wolf::OperatorTables op;
  op.pre2 = wolf::Chirp{a_src, 1.0, +1, chk};
  op.post2 = wolf::Chirp{a_out, 1.0, +1, chk};
  op.sign2 = -1;
  op.pre1 = wolf::Chirp{a_src, 1.0, -1, chk};
  op.post1 = wolf::Chirp{a_out, 1.0, -1, chk};
  op.sign1 = +1;
  op.scale = c * pitch_m * pitch_m * pitch_m * pitch_m;
  op.pupil = wolf::Pupil{0, 0};
  if (out_pitch_m) *out_pitch_m = dx;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (fft)
    e = dtype == WOLF_C64 ? wolf::launch_operator_padfft<float2>(n, n_fft, (const float2*)w_in, (float2*)w_out, op, st)
                          : wolf::launch_operator_padfft<double2>(n, n_fft, (const double2*)w_in, (double2*)w_out, op,
                                                                  st);
  else
    e = dtype == WOLF_C64
            ? wolf::launch_operator_dense<float2>(n, n_fft, (const float2*)w_in, (float2*)w_out, (float2*)work, op, st)
            : wolf::launch_operator_dense<double2>(n, n_fft, (const double2*)w_in, (double2*)w_out, (double2*)work, op,
                                                   st);
  return launched(e, who);
}

WOLF_API wolf_status wolf_propagate_adjoint(const void* g_out, void* g_in, int32_t n, double pitch_m,
                                            double wavelength_m, double z_m, int32_t farfield, int32_t kind,
                                            int32_t dtype, void* stream) {
  if (farfield != 0 && farfield != 1) return fail(WOLF_EINVAL, "wolf_propagate_adjoint: farfield must be 0 or 1");
  return propagate_common(g_out, g_in, n, pitch_m, wavelength_m, z_m, farfield == 1, kind, dtype, true, nullptr,
                          stream, "wolf_propagate_adjoint");
}

WOLF_API wolf_status wolf_build_source(const wolf_source* src, int32_t n, double pitch_m, int32_t dtype, void* w_out,
                                       void* stream) {
  if (!even_n(n)) return fail(WOLF_EUNSUPPORTED, "wolf_build_source: N=%d (even, 2..256)", n);
  if (dtype != WOLF_C64 && dtype != WOLF_C128) return fail(WOLF_EINVAL, "wolf_build_source: bad dtype");
  wolf::SourceParams sp{};
  wolf_status s;
  if ((s = source_params(src, n, pitch_m, &sp, "wolf_build_source")) != WOLF_OK) return s;
  if ((s = check_buf(w_out, n4(n) * elem_bytes(dtype), "w_out")) != WOLF_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = dtype == WOLF_C64 ? wolf::launch_build_source<float2>(n, sp, static_cast<float2*>(w_out), st)
                                   : wolf::launch_build_source<double2>(n, sp, static_cast<double2*>(w_out), st);
  return launched(e, "wolf_build_source");
}

WOLF_API wolf_status wolf_propagate_source(const wolf_source* src, int32_t n, double pitch_m, double wavelength_m,
                                           double z_m, int32_t far_field, int32_t kind, int32_t dtype, void* w_out,
                                           double* out_pitch_m, void* stream) {
  const char* who = "wolf_propagate_source";
  if (!supported_n(n)) return fail(WOLF_EUNSUPPORTED, "%s: N=%d is not a power of two in [2, 256]", who, n);
  if (dtype != WOLF_C64 && dtype != WOLF_C128) return fail(WOLF_EINVAL, "%s: bad dtype %d", who, dtype);
  if (far_field != 0 && far_field != 1) return fail(WOLF_EINVAL, "%s: far_field must be 0 or 1", who);
  if (!pos_finite(pitch_m) || !pos_finite(wavelength_m) || !pos_finite(z_m))
    return fail(WOLF_EINVAL, "%s: pitch, wavelength and z must be finite and > 0", who);
  if (kind != WOLF_SECONDARY && kind != WOLF_PRIMARY) return fail(WOLF_EINVAL, "%s: bad kind %d", who, kind);
  wolf::SourceParams sp{};
  wolf_status s;
  if ((s = source_params(src, n, pitch_m, &sp, who)) != WOLF_OK) return s;
  if ((s = check_buf(w_out, n4(n) * elem_bytes(dtype), "w_out")) != WOLF_OK) return s;
  const wolf::Plan plan = plan_for(n, dtype);
  const bool gen = dtype == WOLF_C64 ? wolf::gen_source_supported<float2>(n, sp, plan.fused_slab)
                                     : wolf::gen_source_supported<double2>(n, sp, plan.fused_slab);
  if (!gen) {  // build the array, then propagate it in place
    if ((s = wolf_build_source(src, n, pitch_m, dtype, w_out, stream)) != WOLF_OK) return s;
    return propagate_common(w_out, w_out, n, pitch_m, wavelength_m, z_m, far_field == 1, kind, dtype, false,
                            out_pitch_m, stream, who);
  }
  const wolf::OperatorTables op = make_op(n, pitch_m, wavelength_m, z_m, far_field == 1, kind, false);
  void* scratch = nullptr;
  if (plan.coop && (s = stream_scratch(stream, &scratch)) != WOLF_OK) return s;
  if (out_pitch_m) *out_pitch_m = wavelength_m * z_m / ((double)n * pitch_m);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const hipError_t e =
      dtype == WOLF_C64
          ? wolf::launch_operator<float2>(n, nullptr, static_cast<float2*>(w_out), op, plan, scratch, st, &sp)
          : wolf::launch_operator<double2>(n, nullptr, static_cast<double2*>(w_out), op, plan, scratch, st, &sp);
  return launched(e, who);
}

WOLF_API wolf_status wolf_spectral_density(const void* w, int32_t n, int32_t dtype, void* s_out, void* stream) {
  if (!even_n(n)) return fail(WOLF_EUNSUPPORTED, "wolf_spectral_density: N=%d (even, 2..256)", n);
  if (dtype != WOLF_C64 && dtype != WOLF_C128) return fail(WOLF_EINVAL, "wolf_spectral_density: bad dtype");
  wolf_status s;
  if ((s = check_buf(w, n4(n) * elem_bytes(dtype), "w")) != WOLF_OK) return s;
  if ((s = check_buf(s_out, (size_t)n * n * real_bytes(dtype), "s_out")) != WOLF_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = dtype == WOLF_C64
                     ? wolf::launch_spectral_density<float2>(n, static_cast<const float2*>(w), static_cast<float*>(s_out), st)
                     : wolf::launch_spectral_density<double2>(n, static_cast<const double2*>(w), static_cast<double*>(s_out), st);
  return launched(e, "wolf_spectral_density");
}

WOLF_API wolf_status wolf_degree_of_coherence(const void* w, int32_t n, int32_t dtype, int32_t ip, int32_t jp,
                                              double s_floor_rel, void* mu_out, void* stream) {
  const char* who = "wolf_degree_of_coherence";
  wolf_status s;
  if ((s = coherence_args(w, n, dtype, ip, jp, s_floor_rel, mu_out, who)) != WOLF_OK) return s;
  void* scratch = nullptr;
  if ((s = stream_scratch(stream, &scratch)) != WOLF_OK) return s;
  return coherence_launch(w, n, dtype, ip, jp, s_floor_rel, mu_out, scratch, stream, who);
}

WOLF_API wolf_status wolf_degree_of_coherence_noalloc(const void* w, int32_t n, int32_t dtype, int32_t ip, int32_t jp,
                                                      double s_floor_rel, void* mu_out, void* stream) {
  const char* who = "wolf_degree_of_coherence_noalloc";
  wolf_status s;
  if ((s = coherence_args(w, n, dtype, ip, jp, s_floor_rel, mu_out, who)) != WOLF_OK) return s;
  void* scratch = nullptr;
  size_t cap = 0;
  const hipError_t e = wolf::mu_static_scratch(&scratch, &cap);
  if (e != hipSuccess) return fail(WOLF_EDEVICE, "%s: cannot find the static scratch: %s", who, hipGetErrorString(e));
  const size_t need = 256 + (size_t)n * n * real_bytes(dtype);
  if (need > cap)
    return fail(WOLF_EINVAL, "%s: N=%d needs %zu bytes of scratch, more than the %zu of the static scratch", who, n,
                need, cap);
  return coherence_launch(w, n, dtype, ip, jp, s_floor_rel, mu_out, scratch, stream, who);
}

WOLF_API wolf_status wolf_chirp_table(int32_t n, double pitch_m, double wavelength_m, double z_m, int32_t dtype,
                                      void* out, void* stream) {
  if (!even_n(n)) return fail(WOLF_EUNSUPPORTED, "wolf_chirp_table: N=%d (even, 2..256)", n);
  if (dtype != WOLF_C64 && dtype != WOLF_C128) return fail(WOLF_EINVAL, "wolf_chirp_table: bad dtype");
  if (!pos_finite(pitch_m) || !pos_finite(wavelength_m) || !pos_finite(z_m))
    return fail(WOLF_EINVAL, "wolf_chirp_table: pitch, wavelength and z must be finite and > 0");
  wolf_status s;
  if ((s = check_buf(out, (size_t)n * elem_bytes(dtype), "out")) != WOLF_OK) return s;
  const wolf::Chirp ch{pitch_m * pitch_m / (wavelength_m * z_m), 1.0, +1, 0};
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = dtype == WOLF_C64 ? wolf::launch_chirp_table<float2>(n, ch, static_cast<float2*>(out), st)
                                   : wolf::launch_chirp_table<double2>(n, ch, static_cast<double2*>(out), st);
  return launched(e, "wolf_chirp_table");
}

WOLF_API wolf_status wolf_propagate_batch(const void* w_src, int32_t n, double pitch_m, int32_t n_pairs,
                                          const double* wavelength_m, const double* z_m, const double* weight,
                                          int32_t farfield, int32_t kind, int32_t dtype, int32_t ip, int32_t jp,
                                          double s_floor_rel, void* work, void* s_out, void* mu_out, void* stream) {
  const char* who = "wolf_propagate_batch";
  if (!supported_n(n)) return fail(WOLF_EUNSUPPORTED, "%s: N=%d unsupported", who, n);
  if (dtype != WOLF_C64 && dtype != WOLF_C128) return fail(WOLF_EINVAL, "%s: bad dtype", who);
  if (!pos_finite(pitch_m)) return fail(WOLF_EINVAL, "%s: pitch must be finite and > 0", who);
  if (n_pairs < 1 || n_pairs > 4096) return fail(WOLF_EINVAL, "%s: n_pairs must be in [1, 4096]", who);
  if (!wavelength_m || !z_m || !weight) return fail(WOLF_EINVAL, "%s: null parameter array", who);
  for (int k = 0; k < n_pairs; ++k) {
    if (!pos_finite(wavelength_m[k]) || !pos_finite(z_m[k]) || !std::isfinite(weight[k]) || weight[k] < 0)
      return fail(WOLF_EINVAL, "%s: pair %d needs lambda > 0, z > 0, weight >= 0", who, k);
  }
  if (farfield != 0 && farfield != 1) return fail(WOLF_EINVAL, "%s: farfield must be 0 or 1", who);
  if (kind != WOLF_SECONDARY && kind != WOLF_PRIMARY) return fail(WOLF_EINVAL, "%s: bad kind", who);
  if (ip < 0 || ip >= n || jp < 0 || jp >= n) return fail(WOLF_EINVAL, "%s: (ip, jp) out of range", who);
  if (!std::isfinite(s_floor_rel) || s_floor_rel < 0) return fail(WOLF_EINVAL, "%s: s_floor_rel must be >= 0", who);
  const size_t eb = elem_bytes(dtype), big = n4(n) * eb, nn = (size_t)n * n;
  wolf_status s;
  const size_t wb = batch_work_bytes(n, dtype);
  if ((s = check_buf(w_src, big, "w_src")) != WOLF_OK) return s;
  if ((s = check_buf(work, wb, "work")) != WOLF_OK) return s;
  if ((s = check_buf(s_out, (size_t)n_pairs * nn * real_bytes(dtype), "s_out")) != WOLF_OK) return s;
  if ((s = check_buf(mu_out, (size_t)n_pairs * nn * eb, "mu_out")) != WOLF_OK) return s;
  const size_t s_bytes = (size_t)n_pairs * nn * real_bytes(dtype), mu_bytes = (size_t)n_pairs * nn * eb;
  if (intervals_overlap(w_src, big, work, wb) || intervals_overlap(s_out, s_bytes, mu_out, mu_bytes) ||
      intervals_overlap(s_out, s_bytes, w_src, big) || intervals_overlap(s_out, s_bytes, work, wb) ||
      intervals_overlap(mu_out, mu_bytes, w_src, big) || intervals_overlap(mu_out, mu_bytes, work, wb))
    return fail(WOLF_EINVAL, "%s: buffers overlap", who);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(WOLF_EDEVICE, "%s: hipGetDevice failed", who);

  // Key of the recorded graph: every argument that a kernel sees.
  std::vector<double> key = {(double)dev, (double)n, pitch_m, (double)n_pairs, (double)farfield, (double)kind,
                             (double)dtype, (double)ip, (double)jp, s_floor_rel,
                             (double)(uintptr_t)w_src, (double)(uintptr_t)work, (double)(uintptr_t)s_out,
                             (double)(uintptr_t)mu_out};
  for (int k = 0; k < n_pairs; ++k) {
    key.push_back(wavelength_m[k]);
    key.push_back(z_m[k]);
    key.push_back(weight[k]);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(g_batch_mu);
  BatchGraph* hit = nullptr;
  for (auto& g : g_batch_graphs)
    if (g.key == key) hit = &g;
  if (hit == nullptr) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
      return fail(WOLF_EINVAL, "%s: the first call for a shape records its own graph; call it once outside capture",
                  who);
    hipStream_t cap = nullptr;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
      return fail(WOLF_EDEVICE, "%s: cannot create the capture stream", who);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) e = record_batch_pairs(n, w_src, pitch_m, n_pairs, wavelength_m, z_m, weight, farfield == 1,
                                                kind, dtype, ip, jp, s_floor_rel, work, s_out, mu_out, cap);
    const hipError_t e_end = hipStreamEndCapture(cap, &graph);
    if (e == hipSuccess) e = e_end;
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) hipGraphDestroy(graph);
    hipStreamDestroy(cap);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(WOLF_EDEVICE, "%s: graph capture failed: %s", who, hipGetErrorString(e));
    }
    if (g_batch_graphs.size() >= 8) {
      hipGraphExecDestroy(g_batch_graphs.front().exec);
      g_batch_graphs.erase(g_batch_graphs.begin());
    }
    g_batch_graphs.push_back(BatchGraph{key, exec});
    hit = &g_batch_graphs.back();
  }
  return launched(hipGraphLaunch(hit->exec, st), who);
}

WOLF_API wolf_status wolf_propagate_polychromatic(const void* w_src, int32_t n, double pitch_m, int32_t n_pairs,
                                                  const double* wavelength_m, const double* z_m, const double* weight,
                                                  double out_pitch_m, int32_t farfield, int32_t kind, int32_t dtype,
                                                  int32_t ip, int32_t jp, double s_floor_rel, void* work, void* s_out,
                                                  void* mu_out, void* stream) {
  const char* who = "wolf_propagate_polychromatic";
  if (!supported_n(n)) return fail(WOLF_EUNSUPPORTED, "%s: N=%d unsupported", who, n);
  if (dtype != WOLF_C64 && dtype != WOLF_C128) return fail(WOLF_EINVAL, "%s: bad dtype", who);
  if (!pos_finite(pitch_m) || !pos_finite(out_pitch_m)) return fail(WOLF_EINVAL, "%s: pitches must be finite and > 0", who);
  if (n_pairs < 1 || n_pairs > 4096) return fail(WOLF_EINVAL, "%s: n_pairs must be in [1, 4096]", who);
  if (!wavelength_m || !z_m || !weight) return fail(WOLF_EINVAL, "%s: null parameter array", who);
  for (int k = 0; k < n_pairs; ++k) {
    if (!pos_finite(wavelength_m[k]) || !pos_finite(z_m[k]) || !std::isfinite(weight[k]) || weight[k] < 0)
      return fail(WOLF_EINVAL, "%s: pair %d needs lambda > 0, z > 0, weight >= 0", who, k);
  }
  if (farfield != 0 && farfield != 1) return fail(WOLF_EINVAL, "%s: farfield must be 0 or 1", who);
  if (kind != WOLF_SECONDARY && kind != WOLF_PRIMARY) return fail(WOLF_EINVAL, "%s: bad kind", who);
  if (ip < 0 || ip >= n || jp < 0 || jp >= n) return fail(WOLF_EINVAL, "%s: (ip, jp) out of range", who);
  if (!std::isfinite(s_floor_rel) || s_floor_rel < 0) return fail(WOLF_EINVAL, "%s: s_floor_rel must be >= 0", who);
  const size_t eb = elem_bytes(dtype), big = n4(n) * eb, nn = (size_t)n * n;
  const size_t wb = dtype == WOLF_C64 ? wolf::poly_work_bytes<float2>(n) : wolf::poly_work_bytes<double2>(n);
  const size_t s_bytes = nn * real_bytes(dtype), mu_bytes = nn * eb;
  wolf_status s;
  if ((s = check_buf(w_src, big, "w_src")) != WOLF_OK) return s;
  if ((s = check_buf(work, wb, "work")) != WOLF_OK) return s;
  if ((s = check_buf(s_out, s_bytes, "s_out")) != WOLF_OK) return s;
  if ((s = check_buf(mu_out, mu_bytes, "mu_out")) != WOLF_OK) return s;
  if (intervals_overlap(w_src, big, work, wb) || intervals_overlap(s_out, s_bytes, mu_out, mu_bytes) ||
      intervals_overlap(s_out, s_bytes, w_src, big) || intervals_overlap(s_out, s_bytes, work, wb) ||
      intervals_overlap(mu_out, mu_bytes, w_src, big) || intervals_overlap(mu_out, mu_bytes, work, wb))
    return fail(WOLF_EINVAL, "%s: buffers overlap", who);
  std::vector<double> alpha(n_pairs), beta(n_pairs), gamma(n_pairs), coef(n_pairs);
  for (int k = 0; k < n_pairs; ++k) {
    const double lz = wavelength_m[k] * z_m[k];
    alpha[k] = farfield ? 0.0 : pitch_m * pitch_m / lz;
    beta[k] = out_pitch_m * pitch_m / lz;
    gamma[k] = out_pitch_m * out_pitch_m / lz;
    const double c = kind == WOLF_PRIMARY ? 1.0 / ((4.0 * M_PI * z_m[k]) * (4.0 * M_PI * z_m[k])) : 1.0 / (lz * lz);
    coef[k] = weight[k] * c * pitch_m * pitch_m * pitch_m * pitch_m;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (dtype == WOLF_C64)
    e = wolf::launch_poly<float2>(n, (const float2*)w_src, n_pairs, alpha.data(), beta.data(), gamma.data(),
                                  coef.data(), ip, jp, s_floor_rel, work, (float*)s_out, (float2*)mu_out, st);
  else
    e = wolf::launch_poly<double2>(n, (const double2*)w_src, n_pairs, alpha.data(), beta.data(), gamma.data(),
                                   coef.data(), ip, jp, s_floor_rel, work, (double*)s_out, (double2*)mu_out, st);
  return launched(e, who);
}

WOLF_API int64_t wolf_polychromatic_work_bytes(int32_t n, int32_t dtype) {
  if (!supported_n(n) || (dtype != WOLF_C64 && dtype != WOLF_C128)) return -1;
  return (int64_t)(dtype == WOLF_C64 ? wolf::poly_work_bytes<float2>(n) : wolf::poly_work_bytes<double2>(n));
}

WOLF_API int64_t wolf_batch_work_bytes(int32_t n, int32_t dtype) {
  if (!supported_n(n) || (dtype != WOLF_C64 && dtype != WOLF_C128)) return -1;
  return (int64_t)batch_work_bytes(n, dtype);
}

WOLF_API wolf_status wolf_propagate_adjoint_diag(const void* g_diag, void* g_in, int32_t n, double pitch_m,
                                                 double wavelength_m, double z_m, int32_t farfield, int32_t kind,
                                                 int32_t dtype, void* stream) {
  const char* who = "wolf_propagate_adjoint_diag";
  if (!supported_n(n)) return fail(WOLF_EUNSUPPORTED, "%s: N=%d unsupported", who, n);
  if (dtype != WOLF_C64 && dtype != WOLF_C128) return fail(WOLF_EINVAL, "%s: bad dtype", who);
  if (!pos_finite(pitch_m) || !pos_finite(wavelength_m) || !pos_finite(z_m))
    return fail(WOLF_EINVAL, "%s: pitch, wavelength and z must be finite and > 0", who);
  if (farfield != 0 && farfield != 1) return fail(WOLF_EINVAL, "%s: farfield must be 0 or 1", who);
  if (kind != WOLF_SECONDARY && kind != WOLF_PRIMARY) return fail(WOLF_EINVAL, "%s: bad kind", who);
  wolf_status s;
  if ((s = check_buf(g_diag, (size_t)n * n * real_bytes(dtype), "g_diag")) != WOLF_OK) return s;
  if ((s = check_buf(g_in, n4(n) * elem_bytes(dtype), "g_in")) != WOLF_OK) return s;
  if (intervals_overlap(g_diag, (size_t)n * n * real_bytes(dtype), g_in, n4(n) * elem_bytes(dtype)))
    return fail(WOLF_EINVAL, "%s: g_in overlaps g_diag", who);
  const wolf::OperatorTables op = make_op(n, pitch_m, wavelength_m, z_m, farfield == 1, kind, true);
  const wolf::Plan plan = plan_for(n, dtype);
  void* scratch = nullptr;
  if (plan.coop && (s = stream_scratch(stream, &scratch)) != WOLF_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = dtype == WOLF_C64
                     ? wolf::launch_operator_diag<float2>(n, (const float*)g_diag, (float2*)g_in, op, plan, scratch, st)
                     : wolf::launch_operator_diag<double2>(n, (const double*)g_diag, (double2*)g_in, op, plan, scratch,
                                                           st);
  return launched(e, who);
}

WOLF_API wolf_status wolf_diag_embed(const void* g, int32_t n, int32_t dtype, void* out, void* stream) {
  if (!supported_n(n)) return fail(WOLF_EUNSUPPORTED, "wolf_diag_embed: N=%d unsupported", n);
  if (dtype != WOLF_C64 && dtype != WOLF_C128) return fail(WOLF_EINVAL, "wolf_diag_embed: bad dtype");
  wolf_status s;
  if ((s = check_buf(g, (size_t)n * n * real_bytes(dtype), "g")) != WOLF_OK) return s;
  if ((s = check_buf(out, n4(n) * elem_bytes(dtype), "out")) != WOLF_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = dtype == WOLF_C64 ? wolf::launch_diag_embed<float2>(n, (const float*)g, (float2*)out, st)
                                   : wolf::launch_diag_embed<double2>(n, (const double*)g, (double2*)out, st);
  return launched(e, "wolf_diag_embed");
}

WOLF_API int64_t wolf_fit_work_bytes(int32_t n, int32_t dtype) {
  if (!supported_n(n) || n > 128 || (dtype != WOLF_C64 && dtype != WOLF_C128)) return -1;
  return (int64_t)wolf::fit_work_bytes(n, (int)real_bytes(dtype));
}

WOLF_API wolf_status wolf_fit_gradient(const void* ga, const float* imap, int32_t n, double pitch_m, double sigma_g_m,
                                       int32_t dtype, void* work, float* d_imap, double* d_sigma, void* stream) {
  const char* who = "wolf_fit_gradient";
  if (!supported_n(n) || n > 128) return fail(WOLF_EUNSUPPORTED, "%s: N=%d unsupported (N <= 128)", who, n);
  if (dtype != WOLF_C64 && dtype != WOLF_C128) return fail(WOLF_EINVAL, "%s: bad dtype", who);
  if (!pos_finite(pitch_m) || !pos_finite(sigma_g_m)) return fail(WOLF_EINVAL, "%s: pitch and sigma_g must be > 0", who);
  wolf_status s;
  if ((s = check_buf(ga, n4(n) * elem_bytes(dtype), "ga")) != WOLF_OK) return s;
  if ((s = check_buf(imap, (size_t)n * n * 4, "imap")) != WOLF_OK) return s;
  if ((s = check_buf(work, wolf::fit_work_bytes(n, (int)real_bytes(dtype)), "work")) != WOLF_OK) return s;
  if ((s = check_buf(d_imap, (size_t)n * n * 4, "d_imap")) != WOLF_OK) return s;
  if ((s = check_buf(d_sigma, 8, "d_sigma")) != WOLF_OK) return s;
  const double inv2g2_px = pitch_m * pitch_m / (2.0 * sigma_g_m * sigma_g_m);
  const double sg_scale = pitch_m * pitch_m / (sigma_g_m * sigma_g_m * sigma_g_m);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = dtype == WOLF_C64
                     ? wolf::launch_fit_gradient<float2>(n, (const float2*)ga, imap, inv2g2_px, sg_scale, work, d_imap,
                                                         d_sigma, st)
                     : wolf::launch_fit_gradient<double2>(n, (const double2*)ga, imap, inv2g2_px, sg_scale, work,
                                                          d_imap, d_sigma, st);
  return launched(e, who);
}

WOLF_API wolf_status wolf_set_plan(int32_t n, int32_t dtype, int32_t fused_slab, int64_t slab_chunk,
                                   int64_t col_chunk, int32_t coop_cols, int32_t coop_lookahead) {
  if (!supported_n(n)) return fail(WOLF_EUNSUPPORTED, "wolf_set_plan: N=%d unsupported", n);
  if (dtype != WOLF_C64 && dtype != WOLF_C128) return fail(WOLF_EINVAL, "wolf_set_plan: bad dtype");
  std::lock_guard<std::mutex> lk(g_plan_mu);
  if (fused_slab == -1 && slab_chunk == -1 && col_chunk == -1) {
    g_plans.erase({n, dtype});
    return WOLF_OK;
  }
  if (fused_slab < 0 || fused_slab > 3) return fail(WOLF_EINVAL, "wolf_set_plan: fused_slab must be 0..3");
  const wolf::Plan p{fused_slab, (long long)slab_chunk, (long long)col_chunk, coop_cols > 0 ? 1 : 0,
                     coop_cols > 0 ? coop_cols : 0, coop_cols > 0 ? coop_lookahead : 1};
  if (!plan_valid(n, dtype, p)) return fail(WOLF_EINVAL, "wolf_set_plan: plan not valid for N=%d", n);
  g_plans[{n, dtype}] = p;
  return WOLF_OK;
}

WOLF_API wolf_status wolf_get_plan(int32_t n, int32_t dtype, int32_t* fused_slab, int64_t* slab_chunk,
                                   int64_t* col_chunk, int32_t* coop_cols, int32_t* coop_lookahead) {
  if (!supported_n(n)) return fail(WOLF_EUNSUPPORTED, "wolf_get_plan: N=%d unsupported", n);
  if (dtype != WOLF_C64 && dtype != WOLF_C128) return fail(WOLF_EINVAL, "wolf_get_plan: bad dtype");
  if (!fused_slab || !slab_chunk || !col_chunk || !coop_cols || !coop_lookahead)
    return fail(WOLF_EINVAL, "wolf_get_plan: null output");
  const wolf::Plan p = plan_for(n, dtype);
  *fused_slab = p.fused_slab;
  *slab_chunk = p.slab_chunk;
  *col_chunk = p.col_chunk;
  *coop_cols = p.coop ? p.coop_cols : 0;
  *coop_lookahead = p.coop_lookahead;
  return WOLF_OK;
}

WOLF_API wolf_status wolf_coop_error_flag(void* stream, int32_t* flag) {
  if (!flag) return fail(WOLF_EINVAL, "wolf_coop_error_flag: null output");
  void* scratch = nullptr;
  wolf_status s = stream_scratch(stream, &scratch);
  if (s != WOLF_OK) return s;
  unsigned v = 0;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (hipStreamSynchronize(st) != hipSuccess || hipMemcpy(&v, scratch, sizeof v, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(WOLF_EDEVICE, "wolf_coop_error_flag: cannot read the flag");
  *flag = (int32_t)v;
  return WOLF_OK;
}

WOLF_API wolf_status wolf_memory_ceiling(void* buf, int64_t bytes, int32_t mode, void* stream) {
  const char* who = "wolf_memory_ceiling";
  if (mode < 0 || mode > 5) return fail(WOLF_EINVAL, "%s: mode must be 0..5", who);
  if (bytes <= 0 || bytes % (256 * 64) != 0) return fail(WOLF_EINVAL, "%s: bytes must be a positive multiple of 16384", who);
  wolf_status s;
  if ((s = check_buf(buf, (size_t)bytes, "buf")) != WOLF_OK) return s;
  return launched(wolf::launch_ceiling(buf, bytes, mode, static_cast<hipStream_t>(stream)), who);
}

WOLF_API wolf_status wolf_autotune(int32_t n, int32_t dtype, void* work, int32_t reps, double* best_ms,
                                   void* stream) {
  if (!supported_n(n)) return fail(WOLF_EUNSUPPORTED, "wolf_autotune: N=%d unsupported", n);
  if (dtype != WOLF_C64 && dtype != WOLF_C128) return fail(WOLF_EINVAL, "wolf_autotune: bad dtype");
  if (reps < 1 || reps > 1000) return fail(WOLF_EINVAL, "wolf_autotune: reps must be in [1, 1000]");
  wolf_status s;
  if ((s = check_buf(work, n4(n) * elem_bytes(dtype), "work")) != WOLF_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const long long nn = (long long)n * n;
  const int c = wolf::axis_tile_cols(n, (int)elem_bytes(dtype));
  std::vector<wolf::Plan> cands;
  const wolf::Plan def = default_plan(n, dtype);
  // Row-pass chunks of the fused_slab = 0 candidates: the built-in one where the built-in plan is a row pass.
  const long long rows_chunk = def.fused_slab == 0 ? def.slab_chunk : row_chunk_slabs(n, dtype);
  for (int fused = 3; fused >= 0; --fused) {
    const int c0 = 64 / (int)elem_bytes(dtype);
    for (int cols : {c0, 2 * c0, 4 * c0}) {
      for (int la : {1, 2}) {
        wolf::Plan p{fused, fused ? 0 : rows_chunk, nn, 1, cols, la};
        if (plan_valid(n, dtype, p)) cands.push_back(p);
      }
    }
    for (long long cols = nn; cols >= c; cols >>= 1) {
      // Chunks below 4 MB only add launches.
      if (cols < nn && cols * nn * (long long)elem_bytes(dtype) < (4ll << 20)) break;
      wolf::Plan p{fused, fused ? 0 : rows_chunk, cols, 0, 0, 1};
      if (plan_valid(n, dtype, p)) cands.push_back(p);
      if (fused && cols == c_best_paired(n, dtype)) {
        // The grouped schedule (in place): slab pass and j1 pass over groups of 4 and 16 i1 planes.
        for (long long planes : {4ll, 16ll}) {
          wolf::Plan q{fused, planes * n, cols, 0, 0, 1};
          if (planes * n < nn && plan_valid(n, dtype, q)) cands.push_back(q);
        }
      }
      if (!fused && cols == nn) {
        wolf::Plan q{0, 0, cols, 0, 0, 1};
        if (plan_valid(n, dtype, q)) cands.push_back(q);
      }
    }
  }
  void* scratch = nullptr;
  if ((s = stream_scratch(stream, &scratch)) != WOLF_OK) return s;
  if (hipMemsetAsync(work, 0, n4(n) * elem_bytes(dtype), st) != hipSuccess)
    return fail(WOLF_EDEVICE, "wolf_autotune: memset failed");
  const wolf::OperatorTables op = make_op(n, 20e-6, 632.8e-9, 0.5, false, WOLF_SECONDARY, false);
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
    return fail(WOLF_EDEVICE, "wolf_autotune: event creation failed");
  double best = 1e300;
  wolf::Plan best_plan = def;
  hipError_t e = hipSuccess;
  for (const auto& p : cands) {
    for (int r = 0; r < reps + 1 && e == hipSuccess; ++r) {
      if (r == 1) e = hipEventRecord(a, st);
      if (e == hipSuccess) {
        e = dtype == WOLF_C64 ? wolf::launch_operator<float2>(n, (float2*)work, (float2*)work, op, p, scratch, st)
                              : wolf::launch_operator<double2>(n, (double2*)work, (double2*)work, op, p, scratch, st);
      }
    }
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (e != hipSuccess) break;
    const double per = ms / reps;
    if (per < best) {
      best = per;
      best_plan = p;
    }
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  if (e != hipSuccess) return fail(WOLF_EDEVICE, "wolf_autotune: %s", hipGetErrorString(e));
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    g_plans[{n, dtype}] = best_plan;
  }
  if (best_ms) *best_ms = best;
  g_last_error.clear();
  return WOLF_OK;
}

}  // extern "C"
