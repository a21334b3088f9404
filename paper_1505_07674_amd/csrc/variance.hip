// variance.hip -- per-pixel weights estimated from the data (Sec. 3.3, Eqs. 18-21).
//
// When an observation comes without a variance map, the photon counts
// k = g (d + b) (effective gain g, subtracted offset b) are taken as Poisson, so
// s^2 = (d + b) / g and the weight is w = e g / (d + b), e being the optional
// multiplicative extra weight factor. Pixels whose counts are not positive get
// w = 0. An elementwise, bandwidth-bound grid-stride pass; float64 arithmetic
// rounded once to float32.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace lensed {
namespace {

__device__ __forceinline__ float pixel_weight(float d, double g, double b, float e) {
  const double db = (double)d + b;
  const double k = g * db;                         // Eq. 18
  if (!(k > 0.0)) return 0.0f;
  return (float)((double)e * g / db);              // e / s^2 with s^2 = (d + b) / g (Eq. 21)
}

constexpr int VAR_BLOCK = 256;

__global__ __launch_bounds__(VAR_BLOCK) void weights_kernel(const float* __restrict__ data, int64_t n, double gain,
                                                            const float* __restrict__ gain_map, double offset,
                                                            const float* __restrict__ offset_map,
                                                            const float* __restrict__ extra,
                                                            float* __restrict__ weight) {
  const int64_t stride = (int64_t)gridDim.x * VAR_BLOCK;
  for (int64_t i = (int64_t)blockIdx.x * VAR_BLOCK + threadIdx.x; i < n; i += stride) {
    const double g = gain_map ? (double)gain_map[i] : gain;
    const double b = offset_map ? (double)offset_map[i] : offset;
    const float e = extra ? extra[i] : 1.0f;
    weight[i] = pixel_weight(data[i], g, b, e);
  }
}

}  // namespace

hipError_t launch_weights_from_data(const float* data, int64_t n, double gain, const float* gain_map, double offset,
                                    const float* offset_map, const float* extra, float* weight, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  // enough workgroups to cover every XCD several times, grid-stride beyond that
  int64_t blocks = (n + VAR_BLOCK - 1) / VAR_BLOCK;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(weights_kernel, dim3((unsigned)blocks), dim3(VAR_BLOCK), 0, stream, data, n, gain, gain_map,
                     offset, offset_map, extra, weight);
  return hipGetLastError();
}

}  // namespace lensed
