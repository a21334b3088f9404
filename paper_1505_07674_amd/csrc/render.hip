// render.hip -- pixel luminosities by N x N midpoint subsampling.
//
// L_i = integral of I over pixel i (Sec. 2.1 Eq. 3) approximated by the
// weighted sum of Eq. 14 with the "subN" midpoint rule (Sec. 4.5). One thread
// per pixel sums its N^2 subsamples in registers; a block covers 256
// consecutive pixels of one image in row-major order, so stores are coalesced
// and only the last block of an image is ragged. The per-point constants are
// read through wave-uniform addresses (scalar loads), and the integration rule
// and the SIE branch are resolved once per block.
#include "internal.h"
#include "kernels.h"
#include "sb_device.h"

namespace lensed {
namespace {

template <int MODE>
__device__ float pixel_sum_dispatch(const PointConst& c, int N, float ux, float uy, float d, float cx, float cy) {
  switch (N) {
    case 1: return pixel_sum<1, MODE>(c, ux, uy, d, cx, cy);
    case 2: return pixel_sum<2, MODE>(c, ux, uy, d, cx, cy);
    case 3: return pixel_sum<3, MODE>(c, ux, uy, d, cx, cy);
    case 4: return pixel_sum<4, MODE>(c, ux, uy, d, cx, cy);
    case 5: return pixel_sum<5, MODE>(c, ux, uy, d, cx, cy);
    case 6: return pixel_sum<6, MODE>(c, ux, uy, d, cx, cy);
    case 7: return pixel_sum<7, MODE>(c, ux, uy, d, cx, cy);
    case 8: return pixel_sum<8, MODE>(c, ux, uy, d, cx, cy);
    default: return pixel_sum_rt<MODE>(c, N, ux, uy, d, cx, cy);
  }
}

__global__ __launch_bounds__(RENDER_BLOCK) void render_kernel(WorkArgs w, const PointConst* __restrict__ pcs,
                                                               float* __restrict__ L) {
  int point, tile;
  if (w.items) {
    const int2 it = w.items[blockIdx.x];
    point = it.x;
    tile = it.y;
  } else {
    point = w.point0;
    tile = blockIdx.x;
  }
  const SysDesc sd = w.sys_table ? w.sys_table[w.point_sys ? w.point_sys[point] : 0] : w.single;
  const int64_t loff = w.point_loff ? w.point_loff[point] : 0;
  const int pix = tile * RENDER_BLOCK + (int)threadIdx.x;
  if (pix >= sd.H * sd.W) return;
  const int r = pix / sd.W;
  const int col = pix - r * sd.W;
  const float ux = (float)col - 0.5f * (float)(sd.W - 1);
  const float uy = (float)r - 0.5f * (float)(sd.H - 1);
  const PointConst& c = pcs[point];
  float acc;
  switch (c.sie_mode) {
    case 0: acc = pixel_sum_dispatch<0>(c, sd.N, ux, uy, sd.d, sd.cx, sd.cy); break;
    case 1: acc = pixel_sum_dispatch<1>(c, sd.N, ux, uy, sd.d, sd.cx, sd.cy); break;
    default: acc = pixel_sum_dispatch<2>(c, sd.N, ux, uy, sd.d, sd.cx, sd.cy); break;
  }
  const float wgt = sd.d * sd.d / (float)(sd.N * sd.N);
  L[loff + pix] = acc * wgt;
}

}  // namespace

hipError_t launch_render(const WorkArgs& w, const PointConst* pcs, float* L, int n_blocks, hipStream_t stream) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(render_kernel, dim3(n_blocks), dim3(RENDER_BLOCK), 0, stream, w, pcs, L);
  return hipGetLastError();
}

}  // namespace lensed
