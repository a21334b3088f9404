// stencil.h -- the LDS stencil shared by the PSF convolution (Sec. 3.1, Eq. 15)
// and its transpose in the adjoint.
//
// A thread owns R vertically adjacent outputs of one column. For each of the K
// stencil columns it reads the R + K - 1 LDS values of that input column once
// and applies the column's K taps to all R outputs. Taps come from a
// column-major table (the K taps of a column are contiguous), read through the
// constant address space with a wave-uniform address, so they arrive by scalar
// loads into SGPRs and feed v_fmac directly. With the LDS row stride a
// compile-time constant, every LDS read uses an immediate offset.
#pragma once

#include <stdint.h>

#include "internal.h"

namespace lensed {

typedef const float __attribute__((address_space(4))) cfloat;

// The same address as a constant-address-space pointer held in SGPRs.
__device__ __forceinline__ cfloat* uniform_const(const float* p) {
  const uint64_t v = (uint64_t)(uintptr_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (cfloat*)((((uint64_t)hi) << 32) | lo);
}

// acc[r] += sum_{l < K} sum_{k < K} Fc[l K + k] Sb[(r + k) SW + l].
template <int K, int SW, int R>
__device__ __forceinline__ void stencil_columns(const float* __restrict__ Sb, cfloat* Fc, float (&acc)[R]) {
  for (int l = 0; l < K; ++l) {
    float v[R + K - 1];
#pragma unroll
    for (int m = 0; m < R + K - 1; ++m) v[m] = Sb[m * SW + l];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const float f = Fc[l * K + k];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = fmaf(f, v[r + k], acc[r]);
    }
  }
}

// Wide tiles of the 21 x 21 stencil: the tile spans up to WIDE_MAX_TW columns
// (a whole row of a 200-pixel image) and its LDS rows are WIDE_STRIDE floats
// apart, a multiple of 64 dwords, so the R + 20 rows a thread reads in one
// stencil column pair up as ds_read2st64 off a single base address.
constexpr int WIDE_STRIDE = 256;
constexpr int WIDE_MAX_TW = WIDE_STRIDE - 20;
constexpr int WIDE_MAX_THREADS = 1024;
inline bool psf_wide(int square_psf, int TW) { return square_psf == 21 && TW > 64 && TW <= WIDE_MAX_TW; }

// Outputs per thread of the PSF and adjoint stencil kernels for a launch; the
// launchers, the plans and the tile model all take it from here.
inline int psf_rows(int square_psf, int TW, int TH) {
  return (square_psf == 21 && (TW == 32 || TW == 64 || psf_wide(square_psf, TW)) && TH % 8 == 0) ? 8 : 4;
}
// Whether the launch uses a specialised stencil (compile-time K and LDS stride).
inline bool psf_specialised(int square_psf, int TW) {
  return ((square_psf == 21 || square_psf == 7 || square_psf == 1) && (TW == 32 || TW == 64)) ||
         (psf_wide(square_psf, TW));
}
// LDS bytes of a PSF or adjoint stencil block.
inline size_t psf_lds_bytes(int square_psf, int TW, int TH, int ph, int pw) {
  const size_t stride = psf_wide(square_psf, TW) ? WIDE_STRIDE : (size_t)(TW + pw - 1);
  return sizeof(float) * stride * (size_t)(TH + ph - 1);
}

}  // namespace lensed
