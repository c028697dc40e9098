// Per-element source CSD (Sec. 3.2, eq. GSM_source; Algorithms 6-7; eq. W_def; Sec. 2.2 thin lens),
// shared by the source builder and by the slab pass that generates its input instead of loading it.
//
// In pixel units (d = pitch), every model factorises as
//   W0[p1; p2] = A * fx(i1, i2) * fy(j1, j2) * m(p1) * m(p2)
//   f(a, b)    = exp(-(a'^2 + b'^2) pitch^2 / (4 sS^2) - (a - b)^2 pitch^2 / (2 sg^2))
//              * exp(i pi (a'^2 - b'^2) pitch^2 / (lambda f_lens)),   a' = a - N/2, b' = b - N/2
//   m(p)       = Y(p) * sqrt(I(p)) for the MAP model, Y(p) otherwise,
// and the incoherent model is A m(p1) delta(p1, p2). The y flip of eq. (n12) drops out: only squares
// and squared differences of the coordinates appear. A slab p1 = (i1, j1) needs the two axis rows
// fx(i1, .) and fy(j1, .), built in FP64 and rounded once, and the scalar A m(p1); each element is
// then one complex multiply and one scale, in this order on every path, so the values are the same
// bits wherever they are formed.
#pragma once
#include "wolf_device.hpp"
#include "wolf_internal.hpp"

namespace wolf {

// Y at centred pixel offsets (di, dj) for the geometries decided by the coordinates (none, circle,
// square, annulus). |di|, |dj| <= 128, so the squares and their sum (<= 32768) are exact in 32-bit
// integers, and a threshold above 2^30 decides like one of 2^30.
__device__ __forceinline__ int clamp_thr(long long t) { return t > (1ll << 30) ? (1 << 30) : (int)t; }
__device__ __forceinline__ bool inside_coords(const SourceParams& sp, int di, int dj) {
  const int a = di * di, b = dj * dj;
  const int t0 = clamp_thr(sp.t0);
  switch (sp.geometry) {
    case 1: return a + b <= t0;
    case 2: return a <= t0 && b <= t0;
    case 3: return a + b <= t0 && a + b > clamp_thr(sp.t1);
    default: return true;
  }
}

__device__ __forceinline__ bool inside(const SourceParams& sp, int di, int dj, int n, int i, int j) {
  return sp.geometry == 4 ? sp.mask[(long long)i * n + j] != 0 : inside_coords(sp, di, dj);
}

// FP64 with no fused multiply-add (as source_value): the lens phase p alpha - 2 rint(p alpha / 2)
// would otherwise be fused or not per call site, and the rows of the builder and of the passes that
// form the source must be the same bits.
template <class T>
__device__ __forceinline__ T axis_factor(const SourceParams& sp, int a, int b, int n) {
#pragma clang fp contract(off)
  using R = typename real_of<T>::type;
  const long long da = a - n / 2, db = b - n / 2;
  const double e = -(double)(da * da + db * db) * sp.inv4s2_px - (double)((da - db) * (da - db)) * sp.inv2g2_px;
  const double mag = exp(e);
  if (sp.lens_alpha == 0.0) return T{(R)mag, (R)0};
  const double x = (double)(da * da - db * db) * sp.lens_alpha;
  const double ph = x - 2.0 * rint(0.5 * x);  // x reduced to [-1, 1] (half turns)
  double s, c;
  sincospi(ph, &s, &c);
  return T{(R)(mag * c), (R)(mag * s)};
}

// W0 = m (fx fy): each real product rounded, then each sum, with no fused multiply-add, so the
// value is the same bits in every kernel that forms it (a contraction may fuse either product of a
// complex multiply, and compilers choose per call site).
template <class T>
__device__ __forceinline__ T source_value(T fx, T fy, typename real_of<T>::type m) {
#pragma clang fp contract(off)
  const T c{fx.x * fy.x - fx.y * fy.y, fx.x * fy.y + fx.y * fy.x};
  return T{c.x * m, c.y * m};
}

// A m(p1) of slab p1 = (i1, j1).
template <class R>
__device__ __forceinline__ R slab_scale(const SourceParams& sp, int i1, int j1, int n) {
  R m1 = inside(sp, i1 - n / 2, j1 - n / 2, n, i1, j1) ? (R)1 : (R)0;
  if (sp.model == 1) m1 *= sqrt((R)sp.imap[(long long)i1 * n + j1]);
  return m1 * (R)sp.amplitude;
}

// W0[p1; (i2, j2)] of the non-incoherent models from the slab's rows fx, fy and am1 = A m(p1).
template <class T>
__device__ __forceinline__ T source_entry(const SourceParams& sp, const T* fx, const T* fy,
                                          typename real_of<T>::type am1, int i2, int j2, int n) {
  using R = typename real_of<T>::type;
  R m = inside(sp, i2 - n / 2, j2 - n / 2, n, i2, j2) ? am1 : (R)0;
  if (sp.model == 1) m *= sqrt((R)sp.imap[(long long)i2 * n + j2]);
  return source_value(fx[i2], fy[j2], m);
}

// The same value for the models without a per-point map (GSM, coherent) and the geometries of
// inside_coords: no loads besides the rows.
template <class T>
__device__ __forceinline__ T source_entry_coords(const SourceParams& sp, const T* fx, const T* fy,
                                                 typename real_of<T>::type am1, int i2, int j2, int n) {
  using R = typename real_of<T>::type;
  const R m = inside_coords(sp, i2 - n / 2, j2 - n / 2) ? am1 : (R)0;
  return source_value(fx[i2], fy[j2], m);
}

}  // namespace wolf
