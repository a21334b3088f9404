// render.hip -- pixel luminosities by N x N midpoint subsampling.
//
// L_i = integral of I over pixel i (Sec. 2.1 Eq. 3) approximated by the
// weighted sum of Eq. 14 with the "subN" midpoint rule or the Cartesian square
// of a Gauss-Kronrod rule (g3k7, g5k11, g7k15; Sec. 4.5). One thread
// per pixel sums its N^2 subsamples in registers; a block covers 256
// consecutive pixels of one image in row-major order, so stores are coalesced
// and only the last block of an image is ragged. The per-point constants are
// read through wave-uniform addresses (scalar loads), and the integration rule
// and the SIE branch are resolved once per block. The lens light and the
// source light are summed separately and signed once per pixel.
#include "internal.h"
#include "kernels.h"
#include "sb_device.h"

namespace lensed {
namespace {

template <int MODE>
__device__ float pixel_sum_dispatch(const PointConst& c, int rule, int N, const PixelGeom& g, bool& cusp) {
  switch (rule) {
    case 1: return pixel_sum_gk<7, MODE>(c, g, cusp);
    case 2: return pixel_sum_gk<11, MODE>(c, g, cusp);
    case 3: return pixel_sum_gk<15, MODE>(c, g, cusp);
    default: break;
  }
  switch (N) {
    case 1: return pixel_sum<1, MODE>(c, g, cusp);
    case 2: return pixel_sum<2, MODE>(c, g, cusp);
    case 3: return pixel_sum<3, MODE>(c, g, cusp);
    case 4: return pixel_sum<4, MODE>(c, g, cusp);
    case 5: return pixel_sum<5, MODE>(c, g, cusp);
    case 6: return pixel_sum<6, MODE>(c, g, cusp);
    case 7: return pixel_sum<7, MODE>(c, g, cusp);
    case 8: return pixel_sum<8, MODE>(c, g, cusp);
    default: return pixel_sum_rt<MODE>(c, N, g, cusp);
  }
}

__device__ __forceinline__ void resolve_item(const WorkArgs& w, int& point, int& tile) {
  if (w.items) {
    const int2 it = w.items[blockIdx.x];
    point = it.x;
    tile = it.y;
  } else {
    point = w.point0;
    tile = blockIdx.x;
  }
}

__device__ __forceinline__ PixelGeom pixel_geom(const SysDesc& sd, int pix) {
  const int r = pix / sd.W;
  const int col = pix - r * sd.W;
  PixelGeom g;
  g.ux = (float)col - 0.5f * (float)(sd.W - 1);
  g.uy = (float)r - 0.5f * (float)(sd.H - 1);
  g.d = sd.d;
  g.cx = sd.cx;
  g.cy = sd.cy;
  return g;
}

__global__ __launch_bounds__(RENDER_BLOCK) void render_kernel(WorkArgs w, const PointConst* __restrict__ pcs,
                                                               float* __restrict__ L, CuspList cl) {
  int point, tile;
  resolve_item(w, point, tile);
  const SysDesc sd = w.sys_table ? w.sys_table[w.point_sys ? w.point_sys[point] : 0] : w.single;
  const int64_t loff = w.point_loff ? w.point_loff[point] : 0;
  const int pix = tile * RENDER_BLOCK + (int)threadIdx.x;
  const bool active = pix < sd.H * sd.W;
  bool cusp = false;
  if (active) {
    const PixelGeom g = pixel_geom(sd, pix);
    const PointConst& c = pcs[point];
    float acc;
    switch (c.rmode) {
      case 0: acc = pixel_sum_dispatch<0>(c, sd.rule, sd.N, g, cusp); break;
      case 1: acc = pixel_sum_dispatch<1>(c, sd.rule, sd.N, g, cusp); break;
      case 2: acc = pixel_sum_dispatch<2>(c, sd.rule, sd.N, g, cusp); break;
      default: acc = pixel_sum_dispatch<3>(c, sd.rule, sd.N, g, cusp); break;
    }
    L[loff + pix] = (float)((double)acc * sd.wgt);
  }
  // one list entry per wave that has pixels next to a cuspy source centre
  const unsigned long long mask = __ballot(cusp);
  if (mask != 0ull && (threadIdx.x & 63) == 0) {
    const int slot = atomicAdd(cl.count, 1);
    CuspEntry e;
    e.point = point;
    e.pix0 = pix;
    e.mask = mask;
    cl.entries[slot] = e;
  }
}

// Adds the float64 cusp corrections to the flagged pixels; a fixed grid of
// waves walks the list written by render_kernel (each pixel appears at most
// once), one entry per wave at a time. Only a few pixels of a flagged wave, and
// a part of their subsamples, lie inside the re-tracing radius, so the wave
// first finds those subsamples (float32, as the render saw them) and queues
// them in LDS, then re-traces the queue in float64 64 at a time with every lane
// busy. Each pixel then adds its subsamples' corrections in the rule's order
// (zero outside the radius), as a serial loop over its subsamples would.
constexpr int CUSP_WAVES = 4;
constexpr int CUSP_BLOCKS = 2048;
constexpr int CUSP_CHUNK = 16;   // subsamples per pass

// LDS written by some lanes of a wave and read by others: order the accesses
// and wait for the writes.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ void subsample_xy(const GkRule* R, int N, int kx, int ky, const PixelGeom& g, float& x,
                                             float& y) {
  y = R ? fmaf(g.uy + R->x[ky], g.d, g.cy) : fmaf(g.uy + sub_offset_rt(ky, N), g.d, g.cy);
  x = R ? fmaf(g.ux + R->x[kx], g.d, g.cx) : fmaf(g.ux + sub_offset_rt(kx, N), g.d, g.cx);
}

__global__ __launch_bounds__(64 * CUSP_WAVES) void cusp_kernel(WorkArgs w, const PointConst* __restrict__ pcs,
                                                               const PointConst64* __restrict__ p64s,
                                                               float* __restrict__ L, CuspList cl) {
  __shared__ float dval[CUSP_WAVES][CUSP_CHUNK * 64];             // [subsample][lane]
  __shared__ unsigned short queue[CUSP_WAVES][CUSP_CHUNK * 64];   // lane | subsample << 6
  const int n = *cl.count;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wave = blockIdx.x * CUSP_WAVES + wv;
  float* __restrict__ dv = dval[wv];
  unsigned short* __restrict__ qu = queue[wv];
  for (int i = wave; i < n; i += gridDim.x * CUSP_WAVES) {
    const CuspEntry e = cl.entries[i];
    const bool mine = (e.mask >> lane) & 1ull;
    const SysDesc sd = w.sys_table ? w.sys_table[w.point_sys ? w.point_sys[e.point] : 0] : w.single;
    const int64_t loff = w.point_loff ? w.point_loff[e.point] : 0;
    const int pix = e.pix0 + lane;
    const PixelGeom g = pixel_geom(sd, pix);
    const PointConst& c = pcs[e.point];
    const PointConst64& c64 = p64s[e.point];
    const GkRule* R = sd.rule > 0 ? &kGkRules[sd.rule - 1] : nullptr;
    const int N = sd.N, NN = N * N;
    float acc = 0.0f;
    for (int s0 = 0; s0 < NN; s0 += CUSP_CHUNK) {
      const int ns = min(CUSP_CHUNK, NN - s0);
      // the chunk's subsamples inside the radius, queued in (subsample, lane) order
      int qn = 0;
      for (int j = 0; j < ns; ++j) {
        const int ky = (s0 + j) / N, kx = s0 + j - ky * N;
        float x, y;
        subsample_xy(R, N, kx, ky, g, x, y);
        const bool within = mine && render_source_R2(c, x, y) < c.cusp_r2;
        dv[j * 64 + lane] = 0.0f;
        const unsigned long long b = __ballot(within);
        if (within) qu[qn + __popcll(b & ((1ull << lane) - 1ull))] = (unsigned short)(lane | (j << 6));
        qn += __popcll(b);
      }
      wave_lds_sync();
      // float64 re-tracing of the queue, 64 subsamples at a time
      for (int q0 = 0; q0 < qn; q0 += 64) {
        if (q0 + lane < qn) {
          const int item = qu[q0 + lane];
          const int pl = item & 63, j = item >> 6;
          const int ky = (s0 + j) / N, kx = s0 + j - ky * N;
          const PixelGeom gq = pixel_geom(sd, e.pix0 + pl);
          float x, y;
          subsample_xy(R, N, kx, ky, gq, x, y);
          const float sR2 = render_source_R2(c, x, y);
          const double ox = R ? R->xd[kx] : ((double)kx + 0.5) / N - 0.5;
          const double oy = R ? R->xd[ky] : ((double)ky + 0.5) / N - 0.5;
          float dx, dy;
          source_offset_f64(c64, gq, ox, oy, dx, dy);
          const float exact = sersic_shape(source_R2(c, dx, dy), c.se, c.sB);
          const float d = exact - sersic_shape(sR2, c.se, c.sB);
          dv[j * 64 + pl] = R ? R->w[kx] * R->w[ky] * d : d;
        }
      }
      wave_lds_sync();
      for (int j = 0; j < ns; ++j) acc += dv[j * 64 + lane];
      wave_lds_sync();
    }
    if (mine) L[loff + pix] = (float)((double)L[loff + pix] + (double)(c.sI * acc) * sd.wgt);
  }
}

// |Kronrod - embedded Gauss| x pixel weight for every pixel of one point (the
// per-pixel integration error estimate of a Gauss-Kronrod rule), float32
// subsample values without the cusp re-tracing.
template <int K>
__device__ float rule_error_pixel(const PointConst& c, const PixelGeom& g) {
  bool cusp = false;
  float gauss = 0.0f, k = 0.0f;
  switch (c.rmode) {
    case 0: k = pixel_sum_gk<K, 0, true>(c, g, cusp, &gauss); break;
    case 1: k = pixel_sum_gk<K, 1, true>(c, g, cusp, &gauss); break;
    case 2: k = pixel_sum_gk<K, 2, true>(c, g, cusp, &gauss); break;
    default: k = pixel_sum_gk<K, 3, true>(c, g, cusp, &gauss); break;
  }
  return fabsf(k - gauss);
}

__global__ __launch_bounds__(RENDER_BLOCK) void rule_error_kernel(WorkArgs w, const PointConst* __restrict__ pcs,
                                                                   float* __restrict__ E) {
  const SysDesc sd = w.single;
  const int pix = blockIdx.x * RENDER_BLOCK + (int)threadIdx.x;
  if (pix >= sd.H * sd.W) return;
  const PixelGeom g = pixel_geom(sd, pix);
  const PointConst& c = pcs[w.point0];
  float e;
  switch (sd.rule) {
    case 1: e = rule_error_pixel<7>(c, g); break;
    case 2: e = rule_error_pixel<11>(c, g); break;
    default: e = rule_error_pixel<15>(c, g); break;
  }
  E[pix] = (float)((double)e * sd.wgt);
}

}  // namespace

hipError_t launch_rule_error(const WorkArgs& w, const PointConst* pcs, float* E, int n_blocks, hipStream_t stream) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(rule_error_kernel, dim3(n_blocks), dim3(RENDER_BLOCK), 0, stream, w, pcs, E);
  return hipGetLastError();
}

// Composite models (Sec. 5: extra Sersic components and a flat sky): the first
// image of each model becomes the sum of the model's K images plus the sky's
// pixel luminosity sky[m] pixscale^2, summed in float64. Block b walks the
// (model, tile) items b, b + gridDim.x, ...
__global__ __launch_bounds__(RENDER_BLOCK) void compose_kernel(float* __restrict__ L, const int64_t* __restrict__ loff,
                                                                const int* __restrict__ point_sys,
                                                                const SysDesc* __restrict__ sys, int K, int n_models,
                                                                const float* __restrict__ sky, int tiles_per_model) {
  const int64_t n_items = (int64_t)n_models * tiles_per_model;
  for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
    const int m = (int)(item / tiles_per_model);
    const int tile = (int)(item - (int64_t)m * tiles_per_model);
    const int64_t p0 = (int64_t)m * K;
    const SysDesc& sd = sys[point_sys ? point_sys[p0] : 0];
    const int pix = tile * RENDER_BLOCK + (int)threadIdx.x;
    if (pix >= sd.H * sd.W) continue;
    double v = sky ? (double)sky[m] * (double)sd.d * (double)sd.d : 0.0;
    for (int j = 0; j < K; ++j) v += (double)L[loff[p0 + j] + pix];
    L[loff[p0] + pix] = (float)v;
  }
}

// One composite model of a plain call: out = sum over j < K of L[j npix + pix],
// plus sky_px (the sky's pixel luminosity), in float64; out may be L itself.
__global__ __launch_bounds__(RENDER_BLOCK) void sum_images_kernel(const float* L, int64_t npix, int K, double sky_px,
                                                                   float* out) {
  const int64_t pix = (int64_t)blockIdx.x * RENDER_BLOCK + threadIdx.x;
  if (pix >= npix) return;
  double v = sky_px;
  for (int j = 0; j < K; ++j) v += (double)L[(int64_t)j * npix + pix];
  out[pix] = (float)v;
}

__global__ void zero_count_kernel(int* count) { *count = 0; }

hipError_t launch_sum_images(const float* L, int64_t npix, int K, double sky_px, float* out, hipStream_t stream) {
  if (npix <= 0) return hipSuccess;
  hipLaunchKernelGGL(sum_images_kernel, dim3((unsigned)((npix + RENDER_BLOCK - 1) / RENDER_BLOCK)), dim3(RENDER_BLOCK),
                     0, stream, L, npix, K, sky_px, out);
  return hipGetLastError();
}

hipError_t launch_zero_count(int* count, hipStream_t stream) {
  hipLaunchKernelGGL(zero_count_kernel, dim3(1), dim3(1), 0, stream, count);
  return hipGetLastError();
}

hipError_t launch_compose(float* L, const int64_t* loff, const int* point_sys, const SysDesc* sys, int K, int n_models,
                          const float* sky, int tiles_per_model, hipStream_t stream) {
  const int64_t n_items = (int64_t)n_models * tiles_per_model;
  if (n_items <= 0) return hipSuccess;
  const int grid = (int)(n_items < 65536 ? n_items : 65536);
  hipLaunchKernelGGL(compose_kernel, dim3(grid), dim3(RENDER_BLOCK), 0, stream, L, loff, point_sys, sys, K, n_models,
                     sky, tiles_per_model);
  return hipGetLastError();
}

hipError_t launch_render(const WorkArgs& w, const PointConst* pcs, const PointConst64* p64s, float* L, int n_blocks,
                         const CuspList& cl, hipStream_t stream, hipEvent_t between) {
  if (n_blocks <= 0) return hipSuccess;
  hipError_t e = for_item_parts(w, n_blocks, [&](const WorkArgs& part, int n) {
    hipLaunchKernelGGL(render_kernel, dim3(n), dim3(RENDER_BLOCK), 0, stream, part, pcs, L, cl);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  if (between && (e = hipEventRecord(between, stream)) != hipSuccess) return e;
  const int waves = n_blocks * (RENDER_BLOCK / 64);   // list capacity
  int grid = (waves + CUSP_WAVES - 1) / CUSP_WAVES;
  if (grid > CUSP_BLOCKS) grid = CUSP_BLOCKS;
  hipLaunchKernelGGL(cusp_kernel, dim3(grid), dim3(64 * CUSP_WAVES), 0, stream, w, pcs, p64s, L, cl);
  return hipGetLastError();
}

}  // namespace lensed
