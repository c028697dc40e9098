// Driver of the sanitizer build of libwolf's host code (test infrastructure): every entry point of
// include/wolf.h with valid arguments (each must return WOLF_OK and record sane launches) and with
// invalid ones (each must fail with the documented status and launch nothing). Built with
// AddressSanitizer and UndefinedBehaviorSanitizer against the HIP stand-in of hip_stub.cpp.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "hip_stub.h"
#include "wolf.h"

static int g_fail = 0;
static int g_checks = 0;

#define EXPECT(cond, ...)                                   \
  do {                                                      \
    ++g_checks;                                             \
    if (!(cond)) {                                          \
      ++g_fail;                                             \
      std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      std::fprintf(stderr, __VA_ARGS__);                    \
      std::fprintf(stderr, "\n");                           \
    }                                                       \
  } while (0)

static const double kNaN = std::numeric_limits<double>::quiet_NaN();
static const double kInf = std::numeric_limits<double>::infinity();
static void* S0 = nullptr;  // default stream

static size_t eb(int dtype) { return dtype == WOLF_C64 ? 8 : 16; }
static size_t n4(int n) { return (size_t)n * n * n * n; }

// A valid call: WOLF_OK, at least one launch, every launch within the limits of a gfx950 dispatch.
static void ok_call(wolf_status s, const char* what) {
  const auto l = stub::launches();
  EXPECT(s == WOLF_OK, "%s returned %d (%s)", what, s, wolf_last_error_message());
  EXPECT(std::strlen(wolf_last_error_message()) == 0, "%s: error message left after success", what);
  EXPECT(!l.empty(), "%s launched nothing", what);
  for (const auto& k : l) {
    const unsigned long long threads = (unsigned long long)k.bx * k.by * k.bz;
    EXPECT(k.gx >= 1 && k.gy >= 1 && k.gz >= 1, "%s: empty grid", what);
    EXPECT(threads >= 1 && threads <= 1024, "%s: block of %llu threads", what, threads);
    EXPECT(k.shm <= 160 * 1024, "%s: %zu bytes of dynamic LDS", what, k.shm);
  }
  stub::clear_launches();
}

// An invalid call: the expected status, a message, and nothing launched.
static void bad_call(wolf_status s, wolf_status want, const char* what) {
  EXPECT(s == want, "%s returned %d, expected %d", what, s, want);
  EXPECT(std::strlen(wolf_last_error_message()) > 0 || s == WOLF_OK, "%s: no error message", what);
  EXPECT(stub::launches().empty(), "%s launched %zu kernels after failing", what, stub::launches().size());
  stub::clear_launches();
}

static wolf_source gsm() {
  wolf_source s{};
  s.model = WOLF_MODEL_GSM;
  s.geometry = WOLF_GEO_NONE;
  s.amplitude = 1.0;
  s.sigma_s_m = 0.1e-3;
  s.sigma_g_m = 0.05e-3;
  return s;
}

static void sources(int n, int dtype) {
  void* w = stub::device_alloc(n4(n) * eb(dtype));
  float* imap = static_cast<float*>(stub::device_alloc((size_t)n * n * 4));
  uint8_t* mask = static_cast<uint8_t*>(stub::device_alloc((size_t)n * n));
  const double p = 20e-6;
  for (int model = 0; model < 4; ++model) {
    for (int geo = 0; geo < 5; ++geo) {
      wolf_source s = gsm();
      s.model = model;
      s.geometry = geo;
      s.geo_r0_m = 4 * p;
      s.geo_r1_m = 2 * p;
      s.intensity_map = imap;
      s.mask = mask;
      if (geo == 1) {
        s.lens_focal_m = 0.2;
        s.wavelength_m = 632.8e-9;
      }
      ok_call(wolf_build_source(&s, n, p, dtype, w, S0), "wolf_build_source");
      if ((n & (n - 1)) == 0) ok_call(wolf_propagate_source(&s, n, p, 632.8e-9, 0.3, geo & 1, WOLF_SECONDARY, dtype, w, nullptr, S0),
                                      "wolf_propagate_source");
    }
  }
  wolf_source s = gsm();
  bad_call(wolf_build_source(nullptr, n, p, dtype, w, S0), WOLF_EINVAL, "null source");
  bad_call(wolf_build_source(&s, n + 1, p, dtype, w, S0), WOLF_EUNSUPPORTED, "odd N");
  bad_call(wolf_build_source(&s, n, -p, dtype, w, S0), WOLF_EINVAL, "negative pitch");
  bad_call(wolf_build_source(&s, n, kNaN, dtype, w, S0), WOLF_EINVAL, "NaN pitch");
  bad_call(wolf_build_source(&s, n, p, 7, w, S0), WOLF_EINVAL, "bad dtype");
  bad_call(wolf_build_source(&s, n, p, dtype, nullptr, S0), WOLF_EINVAL, "null output");
  int host_buffer[4];
  bad_call(wolf_build_source(&s, n, p, dtype, host_buffer, S0), WOLF_EINVAL, "host output");
  void* small = stub::device_alloc(n4(n) * eb(dtype) - 1);
  bad_call(wolf_build_source(&s, n, p, dtype, small, S0), WOLF_EINVAL, "output one byte short");
  s.amplitude = -1;
  bad_call(wolf_build_source(&s, n, p, dtype, w, S0), WOLF_EINVAL, "negative amplitude");
  s = gsm();
  s.sigma_s_m = kNaN;
  bad_call(wolf_build_source(&s, n, p, dtype, w, S0), WOLF_EINVAL, "NaN sigma_s");
  s = gsm();
  s.sigma_g_m = 0;
  bad_call(wolf_build_source(&s, n, p, dtype, w, S0), WOLF_EINVAL, "zero sigma_g");
  s = gsm();
  s.model = 9;
  bad_call(wolf_build_source(&s, n, p, dtype, w, S0), WOLF_EINVAL, "bad model");
  s = gsm();
  s.geometry = WOLF_GEO_ANNULUS;
  s.geo_r0_m = 2 * p;
  s.geo_r1_m = 3 * p;
  bad_call(wolf_build_source(&s, n, p, dtype, w, S0), WOLF_EINVAL, "annulus r1 > r0");
  s = gsm();
  s.geometry = WOLF_GEO_CIRCLE;
  s.geo_r0_m = kInf;
  bad_call(wolf_build_source(&s, n, p, dtype, w, S0), WOLF_EINVAL, "infinite radius");
  s = gsm();
  s.geometry = WOLF_GEO_MASK;
  s.mask = nullptr;
  bad_call(wolf_build_source(&s, n, p, dtype, w, S0), WOLF_EINVAL, "mask geometry without a mask");
  s = gsm();
  s.model = WOLF_MODEL_MAP;
  s.intensity_map = static_cast<const float*>(stub::device_alloc((size_t)n * n * 4 - 1));  // one byte short
  bad_call(wolf_build_source(&s, n, p, dtype, w, S0), WOLF_EINVAL, "map one byte short");
  s = gsm();
  s.lens_focal_m = 0.2;
  s.wavelength_m = 0;
  bad_call(wolf_build_source(&s, n, p, dtype, w, S0), WOLF_EINVAL, "lens without a wavelength");
}

static void propagation(int n, int dtype) {
  const size_t bytes = n4(n) * eb(dtype);
  void* a = stub::device_alloc(bytes);
  void* b = stub::device_alloc(bytes);
  char* two = static_cast<char*>(stub::device_alloc(2 * bytes));
  const double p = 20e-6, lam = 632.8e-9, z = 0.1;
  double dx = 0;
  ok_call(wolf_propagate_fresnel(a, b, n, p, lam, z, WOLF_SECONDARY, dtype, &dx, S0), "fresnel");
  EXPECT(std::fabs(dx - lam * z / (n * p)) <= 1e-18, "output pitch");
  ok_call(wolf_propagate_fresnel(a, a, n, p, lam, z, WOLF_PRIMARY, dtype, nullptr, S0), "fresnel in place");
  ok_call(wolf_propagate_farfield(a, b, n, p, lam, z, WOLF_SECONDARY, dtype, nullptr, S0), "far field");
  for (int far = 0; far < 2; ++far)
    ok_call(wolf_propagate_adjoint(a, b, n, p, lam, z, far, WOLF_SECONDARY, dtype, S0), "adjoint");
  void* g = stub::device_alloc((size_t)n * n * (dtype == WOLF_C64 ? 4 : 8));
  ok_call(wolf_propagate_adjoint_diag(g, b, n, p, lam, z, 0, WOLF_SECONDARY, dtype, S0), "adjoint diag");
  ok_call(wolf_diag_embed(g, n, dtype, b, S0), "diag embed");
  for (int geo = 0; geo < 3; ++geo)
    ok_call(wolf_propagate_lens(a, b, n, p, lam, 0.2, geo, 5 * p, z, WOLF_SECONDARY, dtype, nullptr, S0), "lens");
  bad_call(wolf_propagate_lens(a, b, n, p, lam, 0.2, 3, 5 * p, z, WOLF_SECONDARY, dtype, nullptr, S0), WOLF_EINVAL,
           "lens with an annulus pupil");
  bad_call(wolf_propagate_lens(a, b, n, p, lam, kNaN, 0, 0, z, WOLF_SECONDARY, dtype, nullptr, S0), WOLF_EINVAL,
           "NaN focal length");
  bad_call(wolf_propagate_fresnel(two, two + 8, n, p, lam, z, 0, dtype, nullptr, S0), WOLF_EINVAL, "partial overlap 2");
  bad_call(wolf_propagate_fresnel(a, b, n, p, lam, -z, 0, dtype, nullptr, S0), WOLF_EINVAL, "negative z");
  bad_call(wolf_propagate_fresnel(a, b, n, p, kInf, z, 0, dtype, nullptr, S0), WOLF_EINVAL, "infinite wavelength");
  bad_call(wolf_propagate_fresnel(a, b, n, p, lam, z, 2, dtype, nullptr, S0), WOLF_EINVAL, "bad kind");
  bad_call(wolf_propagate_fresnel(a, b, 12, p, lam, z, 0, dtype, nullptr, S0), WOLF_EUNSUPPORTED, "N not a power of 2");
  bad_call(wolf_propagate_fresnel(a, b, 512, p, lam, z, 0, dtype, nullptr, S0), WOLF_EUNSUPPORTED, "N too large");
  bad_call(wolf_propagate_fresnel(a, b, 0, p, lam, z, 0, dtype, nullptr, S0), WOLF_EUNSUPPORTED, "N = 0");
  bad_call(wolf_propagate_fresnel(a, b, -8, p, lam, z, 0, dtype, nullptr, S0), WOLF_EUNSUPPORTED, "negative N");
  bad_call(wolf_propagate_adjoint(a, b, n, p, lam, z, 2, 0, dtype, S0), WOLF_EINVAL, "adjoint farfield = 2");
  // Observables.
  void* s = stub::device_alloc((size_t)n * n * (dtype == WOLF_C64 ? 4 : 8));
  void* mu = stub::device_alloc((size_t)n * n * eb(dtype));
  ok_call(wolf_spectral_density(a, n, dtype, s, S0), "S");
  ok_call(wolf_degree_of_coherence(a, n, dtype, n / 2, n / 2, 1e-12, mu, S0), "mu slice");
  ok_call(wolf_degree_of_coherence(a, n, dtype, -1, -1, 1e-12, b, S0), "mu full");
  ok_call(wolf_degree_of_coherence_noalloc(a, n, dtype, n / 2, n / 2, 1e-12, mu, S0), "mu slice, no allocation");
  ok_call(wolf_degree_of_coherence_noalloc(a, n, dtype, -1, -1, 1e-12, b, S0), "mu full, no allocation");
  bad_call(wolf_degree_of_coherence_noalloc(a, n, dtype, -1, 0, 1e-12, mu, S0), WOLF_EINVAL, "noalloc mu half -1");
  bad_call(wolf_degree_of_coherence_noalloc(a, n, dtype, -1, -1, 1e-12, a, S0), WOLF_EINVAL, "noalloc mu in place");
  bad_call(wolf_degree_of_coherence(a, n, dtype, n, 0, 1e-12, mu, S0), WOLF_EINVAL, "mu P1 out of range");
  bad_call(wolf_degree_of_coherence(a, n, dtype, -1, 0, 1e-12, mu, S0), WOLF_EINVAL, "mu half -1");
  bad_call(wolf_degree_of_coherence(a, n, dtype, 0, 0, -1.0, mu, S0), WOLF_EINVAL, "negative floor");
  bad_call(wolf_degree_of_coherence(a, n, dtype, 0, 0, kNaN, mu, S0), WOLF_EINVAL, "NaN floor");
  bad_call(wolf_degree_of_coherence(a, n, dtype, -1, -1, 1e-12, mu, S0), WOLF_EINVAL, "full mu into a slice buffer");
  bad_call(wolf_degree_of_coherence(a, n, dtype, -1, -1, 1e-12, a, S0), WOLF_EINVAL, "mu in place");
  ok_call(wolf_chirp_table(n, p, lam, z, dtype, mu, S0), "chirp table");
  bad_call(wolf_chirp_table(n, p, lam, 0.0, dtype, mu, S0), WOLF_EINVAL, "chirp table z = 0");
  // Padded operator, any even N.
  if (n >= 8) {
    const int m = n - 2;
    void* wa = stub::device_alloc(n4(m) * eb(dtype));
    void* wk = stub::device_alloc(n4(m) * eb(dtype));
    for (int nz : {m, 2 * m, 2 * n, 4 * n, m + 4})
      ok_call(wolf_propagate_padded(wa, wa, m, nz, p, lam, z, 0, 0, dtype, wk, nullptr, S0), "padded");
    bad_call(wolf_propagate_padded(wa, wa, m, m - 2, p, lam, z, 0, 0, dtype, wk, nullptr, S0), WOLF_EUNSUPPORTED,
             "n_fft < N");
    bad_call(wolf_propagate_padded(wa, wa, m, m, p, lam, z, 0, 0, dtype, wa, nullptr, S0), WOLF_EINVAL,
             "padded work = input");
  }
  // Direct sum.
  if (n <= 16) {
    const int64_t wb = wolf_direct_work_bytes(n, dtype);
    EXPECT(wb > 0, "direct work bytes");
    void* wk = stub::device_alloc((size_t)wb);
    ok_call(wolf_propagate_direct(a, b, n, p, lam, z, WOLF_SECONDARY, dtype, wk, nullptr, S0), "direct");
    bad_call(wolf_propagate_direct(a, b, n, p, lam, z, WOLF_SECONDARY, dtype, a, nullptr, S0), WOLF_EINVAL,
             "direct work = input");
  }
  EXPECT(wolf_direct_work_bytes(256, dtype) == -1, "direct at N = 256 unsupported");
  // Fit gradient.
  {
    const int64_t fb = wolf_fit_work_bytes(n, dtype);
    EXPECT(fb > 0, "fit work bytes");
    void* wk = stub::device_alloc((size_t)fb);
    float* imap = static_cast<float*>(stub::device_alloc((size_t)n * n * 4));
    float* dimap = static_cast<float*>(stub::device_alloc((size_t)n * n * 4));
    double* dsig = static_cast<double*>(stub::device_alloc(8));
    ok_call(wolf_fit_gradient(a, imap, n, p, 0.1e-3, dtype, wk, dimap, dsig, S0), "fit gradient");
    bad_call(wolf_fit_gradient(a, imap, n, p, -1.0, dtype, wk, dimap, dsig, S0), WOLF_EINVAL, "fit sigma < 0");
  }
  // Batch and polychromatic sums.
  {
    const int k = 3;
    double lams[k] = {500e-9, 600e-9, 700e-9}, zs[k] = {0.1, 0.2, 0.3}, ws[k] = {1.0, 0.5, 0.0};
    const int64_t wb = wolf_batch_work_bytes(n, dtype);
    void* wk = stub::device_alloc((size_t)wb);
    void* ss = stub::device_alloc((size_t)k * n * n * (dtype == WOLF_C64 ? 4 : 8));
    void* mm = stub::device_alloc((size_t)k * n * n * eb(dtype));
    for (int far = 0; far < 2; ++far) {
      ok_call(wolf_propagate_batch(a, n, p, k, lams, zs, ws, far, 0, dtype, n / 2, n - 1, 1e-12, wk, ss, mm, S0), "batch");
      // The same shape again replays the recorded graph: no kernel launch of its own.
      EXPECT(wolf_propagate_batch(a, n, p, k, lams, zs, ws, far, 0, dtype, n / 2, n - 1, 1e-12, wk, ss, mm, S0) == WOLF_OK,
             "batch replay");
      EXPECT(stub::launches().empty(), "batch replay launched kernels outside its graph");
    }
    double bad_w[k] = {1.0, -1.0, 1.0};
    bad_call(wolf_propagate_batch(a, n, p, k, lams, zs, bad_w, 0, 0, dtype, n / 2, n - 1, 1e-12, wk, ss, mm, S0), WOLF_EINVAL,
             "negative weight");
    bad_call(wolf_propagate_batch(a, n, p, 0, lams, zs, ws, 0, 0, dtype, n / 2, n - 1, 1e-12, wk, ss, mm, S0), WOLF_EINVAL,
             "no pairs");
    bad_call(wolf_propagate_batch(a, n, p, k, nullptr, zs, ws, 0, 0, dtype, n / 2, n - 1, 1e-12, wk, ss, mm, S0), WOLF_EINVAL,
             "null wavelengths");
    bad_call(wolf_propagate_batch(a, n, p, k, lams, zs, ws, 0, 0, dtype, n / 2, n - 1, 1e-12, wk, ss, ss, S0), WOLF_EINVAL,
             "S and mu overlap");
    const int64_t pb = wolf_polychromatic_work_bytes(n, dtype);
    void* pw = stub::device_alloc((size_t)pb);
    for (int far = 0; far < 2; ++far)
      ok_call(wolf_propagate_polychromatic(a, n, p, k, lams, zs, ws, 1e-4, far, 0, dtype, n / 2, n - 1, 1e-12, pw, ss, mm, S0),
              "polychromatic");
    bad_call(wolf_propagate_polychromatic(a, n, p, k, lams, zs, ws, -1e-4, 0, 0, dtype, n / 2, n - 1, 1e-12, pw, ss, mm, S0),
             WOLF_EINVAL, "negative output pitch");
  }
  // Memory ceilings.
  void* big = stub::device_alloc(64 * 1024);
  for (int mode = 0; mode < 6; ++mode) ok_call(wolf_memory_ceiling(big, 64 * 1024, mode, S0), "memory ceiling");
  bad_call(wolf_memory_ceiling(big, 1000, 0, S0), WOLF_EINVAL, "ceiling size not a multiple of 16 KB");
  bad_call(wolf_memory_ceiling(big, 128 * 1024, 0, S0), WOLF_EINVAL, "ceiling beyond the allocation");
  bad_call(wolf_memory_ceiling(big, 64 * 1024, 6, S0), WOLF_EINVAL, "ceiling mode 6");
}

static void plans() {
  for (int dtype = 0; dtype < 2; ++dtype) {
    for (int n = 2; n <= 256; n *= 2) {
      int32_t f = -9, w = -9, la = -9;
      int64_t sc = -9, cc = -9;
      EXPECT(wolf_get_plan(n, dtype, &f, &sc, &cc, &w, &la) == WOLF_OK, "get_plan %d", n);
      EXPECT(wolf_set_plan(n, dtype, f, sc, cc, w, la) == WOLF_OK, "default plan of N=%d dtype %d rejected: %s", n, dtype,
             wolf_last_error_message());
      // Every combination in a small range: valid ones are kept, invalid ones rejected, none crashes.
      for (int ff = -1; ff <= 4; ++ff)
        for (long long s : {-1ll, 0ll, 1ll, 3ll, 64ll, (long long)n * n, (long long)n * n * 2})
          for (long long c : {-1ll, 0ll, 8ll, 16ll, 1000ll, (long long)n * n})
            for (int cw : {0, 8, 1024}) {
              const wolf_status r = wolf_set_plan(n, dtype, ff, s, c, cw, 1);
              EXPECT(r == WOLF_OK || r == WOLF_EINVAL || r == WOLF_EUNSUPPORTED, "set_plan status %d", r);
              if (r == WOLF_OK) {
                int32_t f2, w2, la2;
                int64_t s2, c2;
                wolf_get_plan(n, dtype, &f2, &s2, &c2, &w2, &la2);
                if (!(ff == -1 && s == -1 && c == -1))
                  EXPECT(f2 == ff && s2 == s && c2 == c, "plan not kept for N=%d", n);
              }
            }
      EXPECT(wolf_set_plan(n, dtype, -1, -1, -1, 0, 1) == WOLF_OK, "restore default");
      EXPECT(wolf_set_plan(n, dtype, 1, 0, 0, 1024, 1) != WOLF_OK, "cooperative tile of 1024 columns accepted");
      EXPECT(wolf_set_plan(n, dtype, 1, 0, 0, 12, 1) != WOLF_OK, "cooperative tile of 12 columns accepted");
    }
  }
  EXPECT(wolf_get_plan(12, 0, nullptr, nullptr, nullptr, nullptr, nullptr) == WOLF_EUNSUPPORTED, "get_plan N=12");
  EXPECT(wolf_get_plan(16, 0, nullptr, nullptr, nullptr, nullptr, nullptr) == WOLF_EINVAL, "get_plan null outputs");
  stub::clear_launches();
  // The autotuner times every candidate (events of the stand-in report 1 ms each) and keeps one.
  for (int dtype = 0; dtype < 2; ++dtype) {
    const int n = 16;
    void* wk = stub::device_alloc(n4(n) * eb(dtype));
    double best = 0;
    EXPECT(wolf_autotune(n, dtype, wk, 2, &best, S0) == WOLF_OK, "autotune: %s", wolf_last_error_message());
    EXPECT(best == 0.5, "autotune best %g (1 ms for 2 runs per candidate)", best);
    EXPECT(wolf_autotune(n, dtype, wk, 0, &best, S0) == WOLF_EINVAL, "autotune reps = 0");
    int32_t f, w, la;
    int64_t sc, cc;
    wolf_get_plan(n, dtype, &f, &sc, &cc, &w, &la);
    EXPECT(wolf_set_plan(n, dtype, f, sc, cc, w, la) == WOLF_OK, "autotuned plan not valid");
    wolf_set_plan(n, dtype, -1, -1, -1, 0, 1);
  }
  stub::clear_launches();
}

int main() {
  EXPECT(wolf_version() >= 1, "version");
  for (int s = -5; s <= 1; ++s) EXPECT(wolf_status_string(s) != nullptr, "status string");
  EXPECT(std::fabs(wolf_output_pitch(128, 20e-6, 632.8e-9, 0.5) - 632.8e-9 * 0.5 / (128 * 20e-6)) < 1e-20, "pitch");
  for (int dtype = 0; dtype < 2; ++dtype) {
    for (int n : {2, 4, 8, 16, 32}) {
      sources(n, dtype);
      propagation(n, dtype);
    }
    sources(10, dtype);  // any even N for the builder
  }
  plans();
  std::printf("%d checks, %d failures\n", g_checks, g_fail);
  if (g_fail == 0) std::printf("ALL OK\n");
  return g_fail == 0 ? 0 : 1;
}
