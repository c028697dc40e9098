// Matrix-core building blocks shared by the contraction kernels: 16 x 16 x 4 MFMA products of each
// precision, complex tiles in the 3M form and their LDS-staged inner step.
#pragma once
#include "wolf_device.hpp"

namespace wolf {

// ---------------------------------------------------------------------------------------------
// Complex contractions on the matrix cores: v_mfma_f32_16x16x4f32 for complex64 (2x the FP32 vector
// rate without packed math), v_mfma_f64_16x16x4f64 for complex128. A workgroup's TM x TN complex tile (TM
// pairs: 64 x 64, or 32 x 128 for a complex64 group of at most 32 pairs) is four 32 x 32 wavefront blocks
// of 2 x 2 MFMA tiles. A complex product takes three real ones (the 3M form): T1 = Ar Br, T2 = Ai Bi and
// T3 = (Ar + Ai)(Br + Bi) are accumulated apart, then re = T1 - T2 and im = T3 - T1 - T2. Operands are
// staged in LDS as separate re / im planes [16][width + 16]: lane l of a 16 x 16 x 4 step reads
// A[k 4 + l / 16][row l % 16] and B[k 4 + l / 16][col l % 16] (output layout: Mfma<T>::row); with a row
// stride of 16 mod 64 words (or 48) the four k rows of a step fall on distinct banks.
// ---------------------------------------------------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

// The 16 x 16 x 4 matrix-core product of each precision (FP32 for complex64, FP64 for complex128), and
// the row within its 16 x 16 tile of output i of a lane (the two layouts differ; both were checked with
// a probe): column lane % 16 in both.
template <class T> struct Mfma;
template <> struct Mfma<float2> {
  using V = v4f;
  __device__ __forceinline__ static V mac(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int i) { return 4 * (lane / 16) + i; }
};
template <> struct Mfma<double2> {
  using V = v4d;
  __device__ __forceinline__ static V mac(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int i) { return lane / 16 + 4 * i; }
};

template <int TM> struct MTile {
  static_assert(TM == 64 || TM == 32, "tile height");
  static constexpr int TN = 4096 / TM;                 // columns of the workgroup tile
  static constexpr int WC = TN / 32;                   // wavefront blocks along the columns
  static constexpr int LDA = TM + 16, LDB = TN + 16;   // LDS row strides of the A and B planes
  static constexpr int QA = TM * 16 / 256, QB = TN * 16 / 256;  // staged elements per thread and step
};

template <class T> struct CTile {
  using R = typename real_of<T>::type;
  using V = typename Mfma<T>::V;
  V t1[2][2], t2[2][2], t3[2][2];
  __device__ __forceinline__ R re(int r, int q, int i) const { return t1[r][q][i] - t2[r][q][i]; }
  __device__ __forceinline__ R im(int r, int q, int i) const { return t3[r][q][i] - t1[r][q][i] - t2[r][q][i]; }
};

template <class T> __device__ __forceinline__ void ctile_zero(CTile<T>& c) {
  using V = typename Mfma<T>::V;
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int q = 0; q < 2; ++q) c.t1[r][q] = c.t2[r][q] = c.t3[r][q] = V{0, 0, 0, 0};
}

// c += A B over the 16 staged values of the contraction index, for the wavefront block at (row0, col0).
// Bit q of `cols` (wavefront-uniform) enables the 16 columns col0 + 16 q; a disabled block is left as is.
template <class T, int LDA, int LDB>
__device__ __forceinline__ void ctile_mfma16(CTile<T>& c, const typename real_of<T>::type (*ar)[LDA],
                                             const typename real_of<T>::type (*ai)[LDA],
                                             const typename real_of<T>::type (*br)[LDB],
                                             const typename real_of<T>::type (*bi)[LDB], int row0, int col0,
                                             int lane, int cols = 3) {
  using R = typename real_of<T>::type;
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    const int kk = ks * 4 + lane / 16, l16 = lane % 16;
    R xr[2], xi[2], xs[2], yr[2], yi[2], ys[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      xr[r] = ar[kk][row0 + 16 * r + l16];
      xi[r] = ai[kk][row0 + 16 * r + l16];
      xs[r] = xr[r] + xi[r];
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      yr[q] = br[kk][col0 + 16 * q + l16];
      yi[q] = bi[kk][col0 + 16 * q + l16];
      ys[q] = yr[q] + yi[q];
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (!((cols >> q) & 1)) continue;
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        c.t1[r][q] = Mfma<T>::mac(xr[r], yr[q], c.t1[r][q]);
        c.t2[r][q] = Mfma<T>::mac(xi[r], yi[q], c.t2[r][q]);
        c.t3[r][q] = Mfma<T>::mac(xs[r], ys[q], c.t3[r][q]);
      }
    }
  }
}

}  // namespace wolf
