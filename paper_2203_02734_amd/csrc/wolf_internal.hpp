// Internal declarations shared by the kernel translation units and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wolf_device.hpp"

namespace wolf {

// One pass of the propagation operator: the 1D DFT along `axis` of the N^4 array
// (0 = i1, 1 = j1, 2 = i2, 3 = j2), with the diagonal factors `pre` (input index) and `post`
// (output index). sign -1 = direct DFT, +1 = inverse (unnormalised).
template <class T>
hipError_t launch_axis_pass(int n, const T* src, T* dst, int axis, int sign, const Chirp& pre, const Chirp& post,
                            hipStream_t st);

// Fused pass over the two fastest axes (i2, j2) of each contiguous N x N slab.
// `slab_scale` multiplies slab (i1, j1) by pre1[i1] * pre1[j1], the first-point pre-factor.
template <class T>
hipError_t launch_slab_pass(int n, const T* src, T* dst, int sign, const Chirp& pre, const Chirp& post,
                            const Chirp& slab_pre, hipStream_t st);
template <class T> bool slab_pass_supported(int n);

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

template <class T>
hipError_t launch_spectral_density(int n, const T* w, typename real_of<T>::type* s, hipStream_t st);

// mu slice (ip >= 0) or full mu (ip < 0). scratch: at least 16 + N*N*sizeof(real) bytes.
template <class T>
hipError_t launch_coherence(int n, const T* w, int ip, int jp, double floor_rel, T* mu, void* scratch,
                            hipStream_t st);

template <class T>
hipError_t launch_chirp_table(int n, const Chirp& ch, T* out, hipStream_t st);

}  // namespace wolf
