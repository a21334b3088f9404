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

// Pixel sum of schedule class NC: the N x N midpoint rule with N = NC (1..8)
// unrolled at compile time, or (NC = 0) a Gauss-Kronrod rule or a larger N.
template <int NC, int MODE>
__device__ __forceinline__ float pixel_sum_class(const PointConst& c, const RenderVariant& k, int rule, int N,
                                                 const PixelGeom& g, bool& cusp) {
  if (NC > 0) return pixel_sum<(NC > 0 ? NC : 1), MODE>(c, k, g, cusp);
  switch (rule) {
    case 1: return pixel_sum_gk<7, MODE>(c, k, g, cusp);
    case 2: return pixel_sum_gk<11, MODE>(c, k, g, cusp);
    case 3: return pixel_sum_gk<15, MODE>(c, k, g, cusp);
    default: return pixel_sum_rt<MODE>(c, k, N, g, cusp);
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

// Geometry of pixel pix of an image, and the variant of the render constants
// its subsamples use.
__device__ __forceinline__ PixelGeom pixel_geom(const SysDesc& sd, int pix, int* variant = nullptr) {
  const int r = pix / sd.W;
  const int col = pix - r * sd.W;
  if (variant) *variant = render_variant(r, col);
  PixelGeom g;
  g.ux = (float)col - 0.5f * (float)(sd.W - 1);
  g.uy = (float)r - 0.5f * (float)(sd.H - 1);
  g.d = sd.d;
  g.cx = sd.cx;
  g.cy = sd.cy;
  return g;
}

// Appends a cusp-list entry for a wave with flagged lanes (lane l renders unit
// unit0 + l; the entry covers pixel `half` of each unit).
__device__ __forceinline__ void push_cusp(const CuspList& cl, bool flag, int point, int unit0, int ppt, int half) {
  const unsigned long long mask = __ballot(flag);
  if (mask != 0ull && (threadIdx.x & 63) == 0) {
    const int slot = atomicAdd(cl.count, 1);
    CuspEntry e;
    e.point = point;
    e.unit0 = unit0;
    e.mask = mask;
    e.ppt = ppt;
    e.half = half;
    cl.entries[slot] = e;
  }
}

// One kernel per schedule class, so that the registers of the large rules do
// not set the occupancy of the small ones. A thread renders one unit: PPT = 1
// pixel, or PPT = 2 horizontally adjacent pixels (2j, 2j+1) of a row, which
// share the row terms and the constants (only for midpoint classes and images
// of even width, so that a pair never straddles two rows). Item (point, tile)
// covers units tile * B .. + B - 1 (B = blockDim.x, up to RENDER_BLOCK_MAX):
// consecutive pixels, or, in a masked plan, consecutive entries of the
// system's unit list.
template <int NC, int PPT>
__global__ __launch_bounds__(RENDER_BLOCK_MAX, NC > 0 && NC <= 4 ? 8 : 1) void render_kernel(
    WorkArgs w, const PointConst* __restrict__ pcs, float* __restrict__ L, CuspList cl) {
  int point, tile;
  resolve_item(w, point, tile);
  const SysDesc sd = w.sys_table ? w.sys_table[w.point_sys ? w.point_sys[point] : 0] : w.single;
  const int64_t loff = w.point_loff ? w.point_loff[point] : 0;
  const int unit = tile * (int)blockDim.x + (int)threadIdx.x;
  const bool active = unit < unit_count(sd, PPT);
  bool cusp = false, cusp1 = false;
  if (active) {
    const int pix = unit_pixel(sd, unit, PPT);
    int v;
    const PixelGeom g = pixel_geom(sd, pix, &v);
    const PointConst& c = pcs[point];
    const RenderVariant& k = c.rv[v];
    if (PPT == 2 && NC > 0) {
      constexpr int N = NC > 0 ? NC : 1;
      float a0, a1;
      switch (c.rmode) {
        case 0: pixel_sum_pair<N, 0>(c, k, g, a0, a1, cusp, cusp1); break;
        case 1: pixel_sum_pair<N, 1>(c, k, g, a0, a1, cusp, cusp1); break;
        case 2: pixel_sum_pair<N, 2>(c, k, g, a0, a1, cusp, cusp1); break;
        default: pixel_sum_pair<N, 3>(c, k, g, a0, a1, cusp, cusp1); break;
      }
      L[loff + pix] = (float)((double)a0 * sd.wgt);
      L[loff + pix + 1] = (float)((double)a1 * sd.wgt);
    } else {
      float acc;
      switch (c.rmode) {
        case 0: acc = pixel_sum_class<NC, 0>(c, k, sd.rule, sd.N, g, cusp); break;
        case 1: acc = pixel_sum_class<NC, 1>(c, k, sd.rule, sd.N, g, cusp); break;
        case 2: acc = pixel_sum_class<NC, 2>(c, k, sd.rule, sd.N, g, cusp); break;
        default: acc = pixel_sum_class<NC, 3>(c, k, sd.rule, sd.N, g, cusp); break;
      }
      L[loff + pix] = (float)((double)acc * sd.wgt);
    }
  }
  // one list entry per wave (and pixel of a pair) that has pixels next to a cuspy source centre
  const int unit0 = tile * (int)blockDim.x + (int)(threadIdx.x & ~63u);
  push_cusp(cl, cusp, point, unit0, PPT, 0);
  if (PPT == 2) push_cusp(cl, cusp1, point, unit0, PPT, 1);
}

// Adds the float64 cusp corrections to the flagged pixels; a fixed grid of
// waves walks the list written by render_kernel (each pixel appears at most
// once), one entry per wave at a time. Only a few pixels of a flagged wave, and
// a part of their subsamples, lie inside the re-tracing radius. The wave lists
// the entry's F flagged pixels in LDS and tests the F x (subsamples) pairs 64
// at a time (float32, as the render saw them), queueing those inside the
// radius; then it re-traces the queue in float64 64 at a time with every lane
// busy. Lane f < F then adds its pixel's corrections in the rule's order (zero
// outside the radius), as a serial loop over its subsamples would.
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
  __shared__ float dval[CUSP_WAVES][CUSP_CHUNK * 64];             // [subsample][flagged pixel]
  __shared__ unsigned short queue[CUSP_WAVES][CUSP_CHUNK * 64];   // flagged pixel | subsample << 6
  __shared__ int fpix[CUSP_WAVES][64];                            // the entry's flagged pixels
  const int n = *cl.count;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wave = blockIdx.x * CUSP_WAVES + wv;
  float* __restrict__ dv = dval[wv];
  unsigned short* __restrict__ qu = queue[wv];
  int* __restrict__ fp = fpix[wv];
  for (int i = wave; i < n; i += gridDim.x * CUSP_WAVES) {
    const CuspEntry e = cl.entries[i];
    const bool mine = (e.mask >> lane) & 1ull;
    const int F = __popcll(e.mask);
    const SysDesc sd = w.sys_table ? w.sys_table[w.point_sys ? w.point_sys[e.point] : 0] : w.single;
    const int64_t loff = w.point_loff ? w.point_loff[e.point] : 0;
    if (mine) fp[__popcll(e.mask & ((1ull << lane) - 1ull))] = unit_pixel(sd, e.unit0 + lane, e.ppt) + e.half;
    wave_lds_sync();
    const PointConst& c = pcs[e.point];
    const PointConst64& c64 = p64s[e.point];
    const GkRule* R = sd.rule > 0 ? &kGkRules[sd.rule - 1] : nullptr;
    const int N = sd.N, NN = N * N;
    const int pix = lane < F ? fp[lane] : 0;   // the flagged pixel whose sum this lane keeps
    float acc = 0.0f;
    for (int s0 = 0; s0 < NN; s0 += CUSP_CHUNK) {
      const int ns = min(CUSP_CHUNK, NN - s0);
      for (int j = 0; j < ns; ++j) dv[j * 64 + lane] = 0.0f;
      // the (flagged pixel, subsample) pairs of the chunk inside the radius, queued in pair order
      int qn = 0;
      for (int b = 0; b < F * ns; b += 64) {
        const int item = b + lane;
        bool within = false;
        int f = 0, j = 0;
        if (item < F * ns) {
          f = item / ns;
          j = item - f * ns;
          const int ky = (s0 + j) / N, kx = s0 + j - ky * N;
          int v;
          const PixelGeom g = pixel_geom(sd, fp[f], &v);
          float x, y;
          subsample_xy(R, N, kx, ky, g, x, y);
          within = render_source_R2(c, c.rv[v], x, y) < c.cusp_r2;
        }
        const unsigned long long bal = __ballot(within);
        if (within) qu[qn + __popcll(bal & ((1ull << lane) - 1ull))] = (unsigned short)(f | (j << 6));
        qn += __popcll(bal);
      }
      wave_lds_sync();
      // float64 re-tracing of the queue, 64 subsamples at a time
      for (int q0 = 0; q0 < qn; q0 += 64) {
        if (q0 + lane < qn) {
          const int it = qu[q0 + lane];
          const int f = it & 63, j = it >> 6;
          const int ky = (s0 + j) / N, kx = s0 + j - ky * N;
          int vq;
          const PixelGeom gq = pixel_geom(sd, fp[f], &vq);
          const RenderVariant& kq = c.rv[vq];
          float x, y;
          subsample_xy(R, N, kx, ky, gq, x, y);
          const float sR2 = render_source_R2(c, kq, x, y);
          const double ox = R ? R->xd[kx] : ((double)kx + 0.5) / N - 0.5;
          const double oy = R ? R->xd[ky] : ((double)ky + 0.5) / N - 0.5;
          float dx, dy;
          source_offset_f64(c64, gq, ox, oy, dx, dy);
          const float exact = sersic_shape(source_R2(kq, dx, dy), kq.se, kq.sB);
          const float d = exact - sersic_shape(sR2, kq.se, kq.sB);
          dv[j * 64 + f] = R ? R->w[kx] * R->w[ky] * d : d;
        }
      }
      wave_lds_sync();
      if (lane < F)
        for (int j = 0; j < ns; ++j) acc += dv[j * 64 + lane];
      wave_lds_sync();
    }
    if (lane < F) L[loff + pix] = (float)((double)L[loff + pix] + (double)(c.sI * acc) * sd.wgt);
  }
}

// |Kronrod - embedded Gauss| x pixel weight for every pixel of one point (the
// per-pixel integration error estimate of a Gauss-Kronrod rule), float32
// subsample values without the cusp re-tracing.
template <int K>
__device__ float rule_error_pixel(const PointConst& c, const RenderVariant& kv, const PixelGeom& g) {
  bool cusp = false;
  float gauss = 0.0f, k = 0.0f;
  switch (c.rmode) {
    case 0: k = pixel_sum_gk<K, 0, true>(c, kv, g, cusp, &gauss); break;
    case 1: k = pixel_sum_gk<K, 1, true>(c, kv, g, cusp, &gauss); break;
    case 2: k = pixel_sum_gk<K, 2, true>(c, kv, g, cusp, &gauss); break;
    default: k = pixel_sum_gk<K, 3, true>(c, kv, g, cusp, &gauss); break;
  }
  return fabsf(k - gauss);
}

__global__ __launch_bounds__(RENDER_BLOCK) void rule_error_kernel(WorkArgs w, const PointConst* __restrict__ pcs,
                                                                   float* __restrict__ E) {
  const SysDesc sd = w.single;
  const int pix = blockIdx.x * RENDER_BLOCK + (int)threadIdx.x;
  if (pix >= sd.H * sd.W) return;
  int v;
  const PixelGeom g = pixel_geom(sd, pix, &v);
  const PointConst& c = pcs[w.point0];
  const RenderVariant& k = c.rv[v];
  float e;
  switch (sd.rule) {
    case 1: e = rule_error_pixel<7>(c, k, g); break;
    case 2: e = rule_error_pixel<11>(c, k, g); break;
    default: e = rule_error_pixel<15>(c, k, g); break;
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

int render_class(const SysDesc& sd) { return sd.rule == 0 && sd.N <= RENDER_MAX_CLASS ? sd.N : 0; }

hipError_t launch_render(const WorkArgs& w, const PointConst* pcs, const PointConst64* p64s, float* L,
                         const RenderSpan* spans, int n_spans, const CuspList& cl, hipStream_t stream,
                         hipEvent_t between) {
  int n_waves = 0;   // cusp-list capacity: one entry per wave and pixel of a thread
  for (int i = 0; i < n_spans; ++i) n_waves += spans[i].count * (spans[i].block / 64) * (spans[i].ppt == 2 ? 2 : 1);
  if (n_waves <= 0) return hipSuccess;
  for (int i = 0; i < n_spans; ++i) {
    if (spans[i].count <= 0) continue;
    WorkArgs ws = w;
    if (ws.items) ws.items += spans[i].offset;
    const bool pair = spans[i].ppt == 2 && spans[i].klass > 0;
    const int bs = spans[i].block;
    if (bs < 64 || bs > RENDER_BLOCK_MAX || bs % 64 != 0) return hipErrorInvalidValue;
    hipError_t e = for_item_parts(ws, spans[i].count, [&](const WorkArgs& part, int n) {
      switch (spans[i].klass) {
#define LENSED_RENDER_CLASS(NC)                                                                                     \
  case NC:                                                                                                          \
    if (pair)                                                                                                       \
      hipLaunchKernelGGL((render_kernel<NC, 2>), dim3(n), dim3(bs), 0, stream, part, pcs, L, cl);                   \
    else                                                                                                            \
      hipLaunchKernelGGL((render_kernel<NC, 1>), dim3(n), dim3(bs), 0, stream, part, pcs, L, cl);                   \
    break;
        LENSED_RENDER_CLASS(1)
        LENSED_RENDER_CLASS(2)
        LENSED_RENDER_CLASS(3)
        LENSED_RENDER_CLASS(4)
        LENSED_RENDER_CLASS(5)
        LENSED_RENDER_CLASS(6)
        LENSED_RENDER_CLASS(7)
        LENSED_RENDER_CLASS(8)
#undef LENSED_RENDER_CLASS
        default:
          hipLaunchKernelGGL((render_kernel<0, 1>), dim3(n), dim3(bs), 0, stream, part, pcs, L, cl);
          break;
      }
      return hipGetLastError();
    });
    if (e != hipSuccess) return e;
  }
  hipError_t e;
  if (between && (e = hipEventRecord(between, stream)) != hipSuccess) return e;
  int grid = (n_waves + CUSP_WAVES - 1) / CUSP_WAVES;
  if (grid > CUSP_BLOCKS) grid = CUSP_BLOCKS;
  hipLaunchKernelGGL(cusp_kernel, dim3(grid), dim3(64 * CUSP_WAVES), 0, stream, w, pcs, p64s, L, cl);
  return hipGetLastError();
}

hipError_t launch_render(const WorkArgs& w, const PointConst* pcs, const PointConst64* p64s, float* L, int n_blocks,
                         const CuspList& cl, hipStream_t stream, hipEvent_t between) {
  const RenderSpan span{render_class(w.single), 1, 0, n_blocks, RENDER_BLOCK};
  return launch_render(w, pcs, p64s, L, &span, 1, cl, stream, between);
}

}  // namespace lensed
