// Device building blocks for the CSD propagation kernels (gfx950, wave64).
//
// The propagation operator of the paper's Sec. 2.1, eqs. (W_general), (W_fresnel) and
// (W_farfield), sampled on the grid of Sec. 3.1, eqs. (point)/(n12), factorises over the four
// array axes (i1, j1, i2, j2). Along each axis it is a diagonal multiply, a centred length-N
// DFT and another diagonal multiply:
//   axis of the second point: pre = q(z, xi) (-1)^n, forward DFT,  post = q(z, x) (-1)^k
//   axis of the first point:  pre = q*(z, xi) (-1)^n, inverse DFT, post = q*(z, x) (-1)^k
// q is the quadratic-phase propagator of eq. (q_factor). The factors (-1)^n and (-1)^k turn
// the plain DFT into the DFT on centred indices n - N/2, k - N/2. Each axis also carries a
// (-1)^(N/2), which cancels over the four axes.
//
// The pre/post tables and the twiddles are computed in FP64, with exact integer-index argument
// reduction, and rounded once to the working precision. They are the only FP64 steps.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

namespace wolf {

// LDS of one gfx950 compute unit, shared by the workgroups resident on it.
constexpr size_t kMaxLds = 160 * 1024;

// ---------------------------------------------------------------------------------------------
// Complex helpers on float2 / double2 (interleaved re, im: the layout of torch complex64/128).
// ---------------------------------------------------------------------------------------------
template <class T> struct real_of;
template <> struct real_of<float2> { using type = float; };
template <> struct real_of<double2> { using type = double; };

template <class T> __device__ __forceinline__ T cadd(T a, T b) { return T{a.x + b.x, a.y + b.y}; }
template <class T> __device__ __forceinline__ T csub(T a, T b) { return T{a.x - b.x, a.y - b.y}; }
template <class T> __device__ __forceinline__ T cmul(T a, T b) {
  return T{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class T> __device__ __forceinline__ T cconj(T a) { return T{a.x, -a.y}; }
// a b with each real product rounded before its sum (no fused multiply-add). A pass that either loads
// its input or forms it (the source) applies its first factor with this, so that both forms give the
// same bits: a contraction may fuse either product of a sum, and the compiler chooses per call site.
template <class T> __device__ __forceinline__ T cmul_exact(T a, T b) {
#pragma clang fp contract(off)
  return T{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class T, class R> __device__ __forceinline__ T cscale(T a, R s) { return T{a.x * s, a.y * s}; }

// Multiply by SIGN * i (SIGN = -1: forward DFT kernel e^{-2 pi i/4}; +1: inverse).
template <int SIGN, class T> __device__ __forceinline__ T rot90(T a) {
  if constexpr (SIGN < 0) return T{a.y, -a.x};
  else return T{-a.y, a.x};
}

// cos and sin of 2 pi j / 16, j = 0..15, to 20 digits (the in-register radix <= 16 twiddles).
__device__ constexpr double kCos16[16] = {
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
__device__ constexpr double kSin16[16] = {
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173};

__host__ __device__ constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x >> 1); }
__host__ __device__ constexpr int bitrev(int x, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r = (r << 1) | ((x >> i) & 1);
  return r;
}

// b * e^{SIGN 2 pi i j16 / 16}; j16 is a compile-time constant once the callers are unrolled.
template <int SIGN, class T> __device__ __forceinline__ T twiddle16(T b, int j16) {
  using R = typename real_of<T>::type;
  if (j16 == 0) return b;
  if (j16 == 4) return rot90<SIGN>(b);
  const R c = (R)kCos16[j16];
  const R s = (R)(SIGN * kSin16[j16]);
  return T{b.x * c - b.y * s, b.x * s + b.y * c};
}

// cos and sin of 2 pi j / 32, j = 0..15, to 21 digits (the odd twiddles of the 32-point DFT).
__device__ constexpr double kCos32[16] = {
    1.0, 0.980785280403230449126, 0.923879532511286756128, 0.831469612302545237079,
    0.707106781186547524401, 0.555570233019602224743, 0.382683432365089771728, 0.195090322016128267848,
    0.0, -0.195090322016128267848, -0.382683432365089771728, -0.555570233019602224743,
    -0.707106781186547524401, -0.831469612302545237079, -0.923879532511286756128, -0.980785280403230449126};
__device__ constexpr double kSin32[16] = {
    0.0, 0.195090322016128267848, 0.382683432365089771728, 0.555570233019602224743,
    0.707106781186547524401, 0.831469612302545237079, 0.923879532511286756128, 0.980785280403230449126,
    1.0, 0.980785280403230449126, 0.923879532511286756128, 0.831469612302545237079,
    0.707106781186547524401, 0.555570233019602224743, 0.382683432365089771728, 0.195090322016128267848};

template <int R, int SIGN, class T> __device__ __forceinline__ void dft_reg(T* v);

// 32-point DFT from two 16-point DFTs of the even and odd samples (one radix-2 step).
template <int SIGN, class T> __device__ __forceinline__ void dft_reg32(T* v) {
  using R = typename real_of<T>::type;
  T e[16], o[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    e[i] = v[2 * i];
    o[i] = v[2 * i + 1];
  }
  dft_reg<16, SIGN>(e);
  dft_reg<16, SIGN>(o);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const R c = (R)kCos32[k];
    const R s = (R)(SIGN * kSin32[k]);
    const T b = T{o[k].x * c - o[k].y * s, o[k].x * s + o[k].y * c};
    v[k] = cadd(e[k], b);
    v[k + 16] = csub(e[k], b);
  }
}

// In-register DFT of length R <= 32: X[k] = sum_n v[n] e^{SIGN 2 pi i n k / R}, natural order in
// and out. Iterative radix-2 decimation in time on bit-reversed input (R <= 16), fully unrolled;
// R = 32 takes one more radix-2 step over two 16-point DFTs.
template <int R, int SIGN, class T> __device__ __forceinline__ void dft_reg(T* v) {
  static_assert(R >= 1 && R <= 32 && (R & (R - 1)) == 0, "radix");
  if constexpr (R == 32) {
    dft_reg32<SIGN>(v);
  } else if constexpr (R > 1) {
    constexpr int L = ilog2(R);
    T w[R];
#pragma unroll
    for (int i = 0; i < R; ++i) w[i] = v[bitrev(i, L)];
#pragma unroll
    for (int s = 1; s <= L; ++s) {
      const int m = 1 << s, h = m >> 1;
#pragma unroll
      for (int k = 0; k < R; k += m) {
#pragma unroll
        for (int j = 0; j < h; ++j) {
          const T a = w[k + j];
          const T b = twiddle16<SIGN>(w[k + j + h], j * (16 / m));
          w[k + j] = cadd(a, b);
          w[k + j + h] = csub(a, b);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = w[i];
  }
}

// ---------------------------------------------------------------------------------------------
// Mixed-radix register DFTs (lengths whose odd factors are 3, 5 and 7).
// Their twiddles are compile-time constants: cos and sin of 2 pi j / R, with the angle reduced
// exactly in integers to [0, pi/4] (quadrant, then the complement within it) and the Taylor series
// of sin and cos summed there in double (12 terms at |x| <= pi/4 are below the rounding level).
// ---------------------------------------------------------------------------------------------
constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double ct_sin_series(double x) {
  double term = x, sum = x;
  for (int k = 1; k <= 12; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}

constexpr double ct_cos_series(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k <= 12; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}

// cos (want_sin false) or sin of 2 pi j / R. With 4j = qR + r, 0 <= r < R, the angle is
// q pi/2 + (pi/2) r/R; for 2r > R the within-quadrant angle is taken as the complement.
constexpr double ct_trig(long long j, long long r_len, bool want_sin) {
  j %= r_len;
  if (j < 0) j += r_len;
  const long long q = (4 * j) / r_len;
  long long r = 4 * j - q * r_len;
  bool swap = false;
  if (2 * r > r_len) {
    r = r_len - r;
    swap = true;
  }
  const double x = (kPi / 2.0) * (double)r / (double)r_len;
  double c = ct_cos_series(x), s = ct_sin_series(x);
  if (swap) {
    const double t = c;
    c = s;
    s = t;
  }
  for (long long k = 0; k < q; ++k) {  // a quarter turn maps (c, s) to (-s, c)
    const double t = c;
    c = -s;
    s = t;
  }
  return want_sin ? s : c;
}

template <int R> struct RootTable {
  double c[R], s[R];
  constexpr RootTable() : c{}, s{} {
    for (int j = 0; j < R; ++j) {
      c[j] = ct_trig(j, R, false);
      s[j] = ct_trig(j, R, true);
    }
  }
};
template <int R> __device__ constexpr RootTable<R> kRoots{};

__host__ __device__ constexpr bool is_pow2(int r) { return r >= 1 && (r & (r - 1)) == 0; }
__host__ __device__ constexpr int smallest_odd_factor(int r) {
  for (int p = 3; p <= r; p += 2)
    if (r % p == 0) return p;
  return 1;
}

// b * e^{SIGN 2 pi i e / R} for a compile-time e once the callers are unrolled.
template <int R, int SIGN, class T> __device__ __forceinline__ T twiddle_ct(T b, int e) {
  using Rt = typename real_of<T>::type;
  if (e % R == 0) return b;
  const Rt c = (Rt)kRoots<R>.c[e % R];
  const Rt s = (Rt)(SIGN * kRoots<R>.s[e % R]);
  return T{b.x * c - b.y * s, b.x * s + b.y * c};
}

// P-point DFT, P odd, from the (P-1)/2 sums and differences of mirrored samples:
//   X[k]     = x0 + sum_j (x_j + x_{P-j}) cos(2 pi jk/P) + SIGN i sum_j (x_j - x_{P-j}) sin(2 pi jk/P),
//   X[P - k] = the same with -SIGN,   j, k = 1 .. (P-1)/2.
template <int P, int SIGN, class T> __device__ __forceinline__ void dft_odd(T* v) {
  using Rt = typename real_of<T>::type;
  constexpr int H = (P - 1) / 2;
  T sm[H], df[H];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    sm[j] = cadd(v[j + 1], v[P - 1 - j]);
    df[j] = csub(v[j + 1], v[P - 1 - j]);
  }
  T y[P];
  y[0] = v[0];
#pragma unroll
  for (int j = 0; j < H; ++j) y[0] = cadd(y[0], sm[j]);
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    T a = v[0], b{(Rt)0, (Rt)0};
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      const Rt c = (Rt)kRoots<P>.c[(j * k) % P];
      const Rt s = (Rt)kRoots<P>.s[(j * k) % P];
      a = T{a.x + sm[j - 1].x * c, a.y + sm[j - 1].y * c};
      b = T{b.x + df[j - 1].x * s, b.y + df[j - 1].y * s};
    }
    // SIGN i b = SIGN (-b.y, b.x)
    y[k] = T{a.x - (Rt)SIGN * b.y, a.y + (Rt)SIGN * b.x};
    y[P - k] = T{a.x + (Rt)SIGN * b.y, a.y - (Rt)SIGN * b.x};
  }
#pragma unroll
  for (int k = 0; k < P; ++k) v[k] = y[k];
}

// In-register DFT of length R (odd factors 3, 5, 7; power-of-two part <= 32), natural order in and
// out. R = P M with P the smallest odd factor: the M-point DFTs of the P decimated sequences
// x[P m + r], the twiddles e^{SIGN 2 pi i r k'/R}, then P-point DFTs across r:
//   X[k' + M k''] = sum_r e^{SIGN 2 pi i r k''/P} (e^{SIGN 2 pi i r k'/R} Y_r[k']).
template <int R, int SIGN, class T> __device__ __forceinline__ void dft_any(T* v) {
  if constexpr (is_pow2(R)) {
    dft_reg<R, SIGN>(v);
  } else if constexpr (smallest_odd_factor(R) == R) {
    dft_odd<R, SIGN>(v);
  } else {
    constexpr int P = smallest_odd_factor(R), M = R / P;
    T sub[P][M];
#pragma unroll
    for (int r = 0; r < P; ++r) {
#pragma unroll
      for (int m = 0; m < M; ++m) sub[r][m] = v[P * m + r];
      dft_any<M, SIGN>(sub[r]);
    }
#pragma unroll
    for (int k1 = 0; k1 < M; ++k1) {
      T t[P];
#pragma unroll
      for (int r = 0; r < P; ++r) t[r] = twiddle_ct<R, SIGN>(sub[r][k1], r * k1);
      dft_odd<P, SIGN>(t);
#pragma unroll
      for (int k2 = 0; k2 < P; ++k2) v[k1 + M * k2] = t[k2];
    }
  }
}

// Split of a length-N DFT across N2 threads holding N1 elements each (N = N1 N2, N1 >= N2).
template <int N> struct Split {
  static constexpr int L = ilog2(N);
  static constexpr int N1 = 1 << ((L + 1) / 2);
  static constexpr int N2 = N / N1;
  static constexpr int Q = N1 / N2;  // second-stage DFTs per thread
  static_assert(N1 * N2 == N && N1 >= N2, "split");
};

// ---------------------------------------------------------------------------------------------
// FP64 tables.
// ---------------------------------------------------------------------------------------------
// Phase description of one diagonal factor along an axis: the entry at index n is
//   scale * exp(i pi [sign * (n - N/2)^2 * alpha + (n mod 2)])
// = scale * (-1)^n * q(z, d (n - N/2))^{sign}, with alpha = d^2 / (lambda z).
// alpha = 0 gives the bare checkerboard (the far-field source side, where q is set to 1).
struct Chirp {
  double alpha;
  double scale;
  int sign;        // +1: q, -1: q*
  int checker;     // 1: fold (-1)^n in
};

// Aperture at the input plane of an operator (the pupil of a thin lens there, Sec. 2.2).
// geo: 0 none, 1 circle (di^2 + dj^2 <= thr), 2 square (di^2 <= thr and dj^2 <= thr), with
// di = i - N/2, dj = j - N/2 in pixels and thr = floor((r / pitch)^2 (1 + 1e-9)): the same integer
// decision as the source geometry.
struct Pupil {
  int geo;
  long long thr;
};

__host__ __device__ __forceinline__ bool pupil_pass(const Pupil& pu, int i, int j, int N) {
  const long long di = (long long)i - N / 2, dj = (long long)j - N / 2;
  if (pu.geo == 1) return di * di + dj * dj <= pu.thr;
  if (pu.geo == 2) return di * di <= pu.thr && dj * dj <= pu.thr;
  return true;
}

// pi * r (r already reduced to [-1, 1]) -> (cos, sin) in FP64.
__device__ __forceinline__ void sincospi_reduced(double r, double* s, double* c) { sincospi(r, s, c); }

// Reduce x (= phase / pi) modulo 2 into [-1, 1]. x - 2 rint(x / 2) is exact for |x| < 2^52.
__device__ __forceinline__ double reduce_mod2(double x) { return x - 2.0 * rint(0.5 * x); }

template <class T> __device__ __forceinline__ T chirp_entry(const Chirp& ch, int n, int N) {
  using R = typename real_of<T>::type;
  const long long d = (long long)n - (long long)(N / 2);
  double ph = (double)(d * d) * ch.alpha;           // (n - N/2)^2 alpha, one FP64 rounding
  ph = reduce_mod2((double)ch.sign * ph);
  if (ch.checker && (n & 1)) ph = reduce_mod2(ph + 1.0);
  double s, c;
  sincospi_reduced(ph, &s, &c);
  return T{(R)(c * ch.scale), (R)(s * ch.scale)};
}

// Host copy of chirp_entry in FP64 (std math, not rounded to the working precision), for
// scalars set up at launch time.
inline double2 chirp_entry_host(const Chirp& ch, int n, int N) {
  const long long d = (long long)n - (long long)(N / 2);
  auto red = [](double x) { return x - 2.0 * std::rint(0.5 * x); };
  double ph = (double)(d * d) * ch.alpha;
  ph = red((double)ch.sign * ph);
  if (ch.checker && (n & 1)) ph = red(ph + 1.0);
  const double c = std::cos(M_PI * ph), s = std::sin(M_PI * ph);
  return double2{c * ch.scale, s * ch.scale};
}

// Twiddle e^{SIGN 2 pi i j / N}, j in [0, N): the argument 2 j / N is exact for N a power of two.
template <class T, int SIGN> __device__ __forceinline__ T twiddle_entry(int j, int N) {
  using R = typename real_of<T>::type;
  double s, c;
  sincospi((double)(SIGN * 2) * (double)j / (double)N, &s, &c);
  return T{(R)c, (R)s};
}

// ok ? a : 0, component by component (a select of whole structs can be lowered through scratch memory).
template <class T> __device__ __forceinline__ T keep_or_zero(bool ok, T a) {
  using R = typename real_of<T>::type;
  return T{ok ? a.x : (R)0, ok ? a.y : (R)0};
}

// p[ok ? i : 0]: every lane loads, lanes outside the data read element 0 (a valid address) and are
// zeroed by the caller. Without a branch around each load the compiler issues all of a thread's
// loads before it waits on the first; a conditional load whose value is used in its own branch is
// waited on at once.
template <class T> __device__ __forceinline__ T load_or_first(const T* p, bool ok, long long i) {
  return p[ok ? i : 0];
}

// Monotone map of a double to an unsigned 64-bit key (for atomicMax over reals) and back.
__device__ __forceinline__ unsigned long long order_key(double v) {
  const unsigned long long b = __double_as_longlong(v);
  return (b >> 63) ? ~b : (b | (1ull << 63));
}
__device__ __forceinline__ double key_value(unsigned long long k) {
  const unsigned long long b = (k >> 63) ? (k & ~(1ull << 63)) : ~k;
  return __longlong_as_double((long long)b);
}

// One output point m of the observables: S[m] = c s0[m]; mu(P, m) = post1[P_i] post1[P_j] post2[m_i]
// post2[m_j] b0[m] / sqrt(s0[P] s0[m]) where both s0 exceed floor * max s0 (key: order key of the
// maximum) and c > 0, else 0. The factor c cancels in mu. Phases in FP64.
template <class T, class R>
__device__ __forceinline__ void emit_observables(const R* s0, const T* b0, unsigned long long key, int n, int pi, int pj,
                                                 long long m, double c, const Chirp& post1, const Chirp& post2,
                                                 double floor_rel, R* s_out, T* mu_out) {
  const int mi = (int)(m / n), mj = (int)(m - (long long)mi * n);
  const R sm = s0[m];
  s_out[m] = (R)(c * (double)sm);
  const R tau = (R)(floor_rel * key_value(key));
  const R sp = s0[(long long)pi * n + pj];
  T out{(R)0, (R)0};
  if (c > 0.0 && sp > tau && sm > tau) {
    const double2 ph = cmul(cmul(chirp_entry<double2>(post1, pi, n), chirp_entry<double2>(post1, pj, n)),
                            cmul(chirp_entry<double2>(post2, mi, n), chirp_entry<double2>(post2, mj, n)));
    const T f{(R)ph.x, (R)ph.y};
    const R d = sqrt(sp) * sqrt(sm);
    const T v = cmul(f, b0[m]);
    out = T{v.x / d, v.y / d};
  }
  mu_out[m] = out;
}

}  // namespace wolf
