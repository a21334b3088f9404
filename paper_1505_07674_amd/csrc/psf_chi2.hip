// psf_chi2.hip -- PSF convolution (Sec. 3.1, Eq. 15) fused with the weighted
// chi^2 of the log-likelihood (Sec. 3.2, Eq. 17).
//
// Each block owns a TW x TH tile of output pixels of one image. It stages the
// tile plus a halo of p rows and q columns in LDS, reading the unconvolved
// image with clamped indices (the replicate padding of Eq. 15), then every
// thread computes R vertically adjacent outputs: for each stencil column it
// keeps R + 2p LDS values in registers and applies the 2p + 1 kernel taps of
// that column to all R outputs. Kernel taps are wave-uniform scalar loads from
// a column-major copy of the flipped kernel written by the prologue.
// The chi^2 contribution w (d - L*)^2 is accumulated with Kahan summation per
// thread, combined across the block with error-free TwoSum steps, and written
// as one (hi, lo) float pair per tile; the final sum over tiles is float64.
#include "internal.h"
#include "kernels.h"
#include "stencil.h"

namespace lensed {
namespace {

__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// P >= 0: square (2P+1)^2 PSF, tile width TWc, ROWS outputs per thread; with
// TWc = 0 a wide tile: runtime width sd.TW <= WIDE_MAX_TW, LDS stride WIDE_STRIDE.
// P = -1: any PSF and tile width, ROWS = 4.
template <int P, int TWc, int ROWS>
__global__ __launch_bounds__(P >= 0 && TWc == 0 ? WIDE_MAX_THREADS : 512) void psf_kernel(
    WorkArgs w, const float* __restrict__ L, float* __restrict__ out, float2* __restrict__ partials, int mode) {
  constexpr bool WIDE = P >= 0 && TWc == 0;
  extern __shared__ float S[];
  __shared__ float red_hi[16], red_lo[16];
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
  const int p = P >= 0 ? P : sd.ph / 2;
  const int q = P >= 0 ? P : sd.pw / 2;
  const int TW = (P >= 0 && !WIDE) ? TWc : sd.TW, TH = sd.TH;
  const int SW = TW + 2 * q, SH = TH + 2 * p;     // staged columns and rows
  const int LS = WIDE ? WIDE_STRIDE : SW;         // LDS row stride
  const int ty = tile / sd.tiles_x, tx = tile - ty * sd.tiles_x;
  const int x0 = tx * TW, y0 = ty * TH;
  const float* __restrict__ Lp = L + loff;
  const int tid = threadIdx.x;
  const int jx = tid % TW, jy = tid / TW;
  const int rows_per_pass = blockDim.x / TW;
  if (sd.ptile_w && !sd.ptile_w[tile]) {   // no pixel with w > 0 (gradient plans): zero chi^2, zero rho
    if (mode == 2)
      for (int k = tid; k < TW * TH; k += blockDim.x) {
        const int gi = y0 + k / TW, gj = x0 + k % TW;
        if (gi < sd.H && gj < sd.W) out[loff + (size_t)gi * sd.W + gj] = 0.0f;
      }
    if (tid == 0) partials[(w.point_pbase ? w.point_pbase[point] : 0) + tile] = make_float2(0.0f, 0.0f);
    return;
  }

  // Stage the tile and its halo, four rows per pass so that four loads are in
  // flight before their LDS stores.
  for (int col = jx; col < SW; col += TW) {
    const int gj = min(max(x0 + col - q, 0), sd.W - 1);
    for (int row0 = jy; row0 < SH; row0 += 4 * rows_per_pass) {
      float v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int row = row0 + u * rows_per_pass;
        const int gi = min(max(y0 + row - p, 0), sd.H - 1);
        v[u] = row < SH ? Lp[(size_t)gi * sd.W + gj] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int row = row0 + u * rows_per_pass;
        if (row < SH) S[row * LS + col] = v[u];
      }
    }
  }
  __syncthreads();

  const int i0 = jy * ROWS;
  float acc[ROWS];
#pragma unroll
  for (int r = 0; r < ROWS; ++r) acc[r] = 0.0f;
  if (P >= 0) {
    constexpr int K = 2 * (P > 0 ? P : 0) + 1;
    constexpr int SWc = WIDE ? WIDE_STRIDE : (TWc > 0 ? TWc : 1) + K - 1;
    // taps F[K-1-k][K-1-l] of stencil column l, contiguous in k
    stencil_columns<K, SWc, ROWS>(S + i0 * SWc + jx, uniform_const(sd.psfn + K * K), acc);
  } else {
    const int KH = 2 * p + 1, KW = 2 * q + 1;
    const float* __restrict__ F = sd.psfn;
    for (int l = 0; l < KW; ++l) {
      for (int k = 0; k < KH; ++k) {
        const float f = F[(KH - 1 - k) * KW + (KW - 1 - l)];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) acc[r] = fmaf(f, S[(i0 + r + k) * SW + jx + l], acc[r]);
      }
    }
  }

  const int gj = x0 + jx;
  if (mode == 0) {
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      const int gi = y0 + i0 + r;
      if (gi < sd.H && gj < sd.W && i0 + r < TH) out[loff + (size_t)gi * sd.W + gj] = acc[r];
    }
    return;
  }

  // Kahan accumulation of w (d - L*)^2 over this thread's outputs.
  float sum = 0.0f, comp = 0.0f;
#pragma unroll
  for (int r = 0; r < ROWS; ++r) {
    const int gi = y0 + i0 + r;
    if (gi < sd.H && gj < sd.W && i0 + r < TH) {
      const size_t idx = (size_t)gi * sd.W + gj;
      const float res = sd.data[idx] - acc[r];
      const float wres = sd.weight[idx] * res;
      if (mode == 2) out[loff + idx] = wres;
      const float term = wres * res;
      const float yk = term - comp;
      const float t = sum + yk;
      comp = (t - sum) - yk;
      sum = t;
    }
  }
  float hi = sum, lo = -comp;
  // wave reduction with error-free transformations; the last wave of a block
  // whose size is not a multiple of 64 adds only the lanes it has
  const int lane = tid & 63, wid = tid >> 6;
  const int nact = min(64, (int)blockDim.x - (tid & ~63));
  for (int off = 32; off > 0; off >>= 1) {
    const float h2 = __shfl_down(hi, off, 64);
    const float l2 = __shfl_down(lo, off, 64);
    if (lane + off < nact) {
      float s, e;
      two_sum(hi, h2, s, e);
      hi = s;
      lo = lo + l2 + e;
    }
  }
  if (lane == 0) {
    red_hi[wid] = hi;
    red_lo[wid] = lo;
  }
  __syncthreads();
  if (tid == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    float h = red_hi[0], lsum = red_lo[0];
    for (int i = 1; i < nw; ++i) {
      float s, e;
      two_sum(h, red_hi[i], s, e);
      h = s;
      lsum = lsum + red_lo[i] + e;
    }
    const int base = w.point_pbase ? w.point_pbase[point] : 0;
    partials[base + tile] = make_float2(h, lsum);
  }
}

__global__ void finalize_kernel(const float2* __restrict__ partials, const int* __restrict__ pbase,
                                const int* __restrict__ ntiles, int n_points, int single_ntiles,
                                double* __restrict__ logl) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_points) return;
  const int base = pbase ? pbase[p] : 0;
  const int nt = ntiles ? ntiles[p] : single_ntiles;
  double s = 0.0;
  for (int t = 0; t < nt; ++t) {
    const float2 v = partials[base + t];
    s += (double)v.x + (double)v.y;
  }
  logl[p] = -0.5 * s;
}

template <int P, int TWc, int R>
hipError_t launch_psf_t(const WorkArgs& w, const float* L, float* out, float2* partials, int mode, int n_blocks,
                        int threads, size_t lds, hipStream_t stream) {
  return for_item_parts(w, n_blocks, [&](const WorkArgs& part, int n) {
    hipLaunchKernelGGL((psf_kernel<P, TWc, R>), dim3(n), dim3(threads), lds, stream, part, L, out, partials, mode);
    return hipGetLastError();
  });
}

template <int P, int R>
hipError_t launch_psf_w(int TW, const WorkArgs& w, const float* L, float* out, float2* partials, int mode,
                        int n_blocks, int threads, size_t lds, hipStream_t stream) {
  if (TW == 64) return launch_psf_t<P, 64, R>(w, L, out, partials, mode, n_blocks, threads, lds, stream);
  return launch_psf_t<P, 32, R>(w, L, out, partials, mode, n_blocks, threads, lds, stream);
}

}  // namespace

hipError_t launch_psf(const WorkArgs& w, const float* L, float* out, float2* partials, int mode, int n_blocks,
                      int square_psf, int TW, int TH, int max_ph, int max_pw, hipStream_t stream) {
  if (n_blocks <= 0) return hipSuccess;
  const int R = psf_rows(square_psf, TW, TH);
  const int threads = TW * (TH / R);
  const size_t lds = psf_lds_bytes(square_psf, TW, TH, max_ph, max_pw);
  // Specialised stencils for the square PSFs of the standard workloads.
  if (psf_specialised(square_psf, TW)) {
    if (psf_wide(square_psf, TW))
      return launch_psf_t<10, 0, 8>(w, L, out, partials, mode, n_blocks, threads, lds, stream);
    if (square_psf == 21) {
      if (R == 8) return launch_psf_w<10, 8>(TW, w, L, out, partials, mode, n_blocks, threads, lds, stream);
      return launch_psf_w<10, 4>(TW, w, L, out, partials, mode, n_blocks, threads, lds, stream);
    }
    if (square_psf == 7) return launch_psf_w<3, 4>(TW, w, L, out, partials, mode, n_blocks, threads, lds, stream);
    return launch_psf_w<0, 4>(TW, w, L, out, partials, mode, n_blocks, threads, lds, stream);
  }
  return launch_psf_t<-1, 0, 4>(w, L, out, partials, mode, n_blocks, threads, lds, stream);
}

hipError_t launch_finalize(const float2* partials, const int* point_pbase, const int* point_ntiles, int n_points,
                           int single_ntiles, double* logl, hipStream_t stream) {
  if (n_points <= 0) return hipSuccess;
  const int threads = 64;
  hipLaunchKernelGGL(finalize_kernel, dim3((n_points + threads - 1) / threads), dim3(threads), 0, stream, partials,
                     point_pbase, point_ntiles, n_points, single_ntiles, logl);
  return hipGetLastError();
}

}  // namespace lensed
