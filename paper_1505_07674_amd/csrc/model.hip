// model.hip -- general models: several SIEs with free centres, an external
// shear, several Sersic components in the image or the source plane, a flat
// sky (the models of the paper's fits of real lenses, Sec. 5), and lenses on
// several planes (the multi-plane extension named in Sec. 6).
//
// Evaluated in float64 throughout (the float32 folding of the 17-parameter
// render does not carry over to an arbitrary number of components), then
// rounded once per pixel; the PSF and chi^2 stages are the common ones. On
// gfx950 the float64 vector rate equals the unpacked float32 one; the cost is
// the float64 transcendentals.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "sb_device.h"

namespace lensed {
namespace {

// Deflection of SIE k at (x, y), added to (ax, ay) (Eq. 1's alpha about the
// lens centre, in the lens frame rotated by phi).
__device__ inline void add_sie(const ModelConst& m, int k, double x, double y, double& ax, double& ay) {
  const double* s = m.sie[k];
  const double dx = x - s[0], dy = y - s[1];
  const double xp = s[2] * dx + s[3] * dy, yp = s[2] * dy - s[3] * dx;
  const double psi = sqrt(s[4] * xp * xp + yp * yp);
  if (psi > 0.0) {
    double a1, a2;
    if (m.sie_sphere[k]) {
      a1 = s[6] * xp / psi;
      a2 = s[6] * yp / psi;
    } else {
      a1 = s[6] * atan(s[5] * xp / psi);
      a2 = s[6] * atanh(s[5] * yp / psi);
    }
    ax += s[2] * a1 - s[3] * a2;
    ay += s[3] * a1 + s[2] * a2;
  }
}

// Sersic component j (Eq. 22) at (px, py).
__device__ inline double sersic_at(const ModelConst& m, int j, double px, double py) {
  const double* s = m.ser[j];
  const double dx = px - s[0], dy = py - s[1];
  const double xp = s[2] * dx + s[3] * dy, yp = s[2] * dy - s[3] * dx;
  const double R2 = s[4] * xp * xp + s[5] * yp * yp;
  // (R/R_e)^{1/n} = exp(ln(R^2 / R_e^2) / (2n))
  const double t = R2 > 0.0 ? exp(0.5 * s[7] * log(R2 * s[6] * s[6])) : 0.0;
  return s[9] * exp(-s[8] * (t - 1.0));
}

// Surface brightness of a general model with one lens plane at (x, y) (Eqs.
// 1-2 with several deflectors in one plane, Eq. 22 for every Sersic, plus the
// sky).
__device__ double model_sb(const ModelConst& m, double x, double y) {
  double ax = 0.0, ay = 0.0;
  for (int k = 0; k < m.n_sie; ++k) add_sie(m, k, x, y, ax, ay);
  ax += m.g1 * x + m.g2 * y;
  ay += m.g2 * x - m.g1 * y;
  const double bx = x - ax, by = y - ay;
  double I = m.sky;
  for (int j = 0; j < m.n_sersic; ++j) I += m.plane[j] ? sersic_at(m, j, bx, by) : sersic_at(m, j, x, y);
  return I;
}

// The same with P = spec.n_planes lens planes: the ray's position on plane j
// is x_j = x - sum_{i<j} beta_ij alpha_i(x_i) (beta_iP = 1 for the source
// plane P), taken plane by plane in order of distance; alpha_i sums the SIEs
// of plane i (and the shear on plane 0); each Sersic is evaluated at the
// position on its own plane.
__device__ double model_sb_planes(const ModelConst& m, const ModelSpec& spec, double x, double y) {
  const int P = spec.n_planes;
  double ax[MAX_PLANES], ay[MAX_PLANES];
  double I = m.sky;
  for (int j = 0; j <= P; ++j) {
    double px = x, py = y;
    for (int i = 0; i < j; ++i) {
      const double b = j == P ? 1.0 : spec.beta[i][j];
      px -= b * ax[i];
      py -= b * ay[i];
    }
    for (int k = 0; k < m.n_sersic; ++k)
      if (m.plane[k] == j) I += sersic_at(m, k, px, py);
    if (j < P) {
      double dx = 0.0, dy = 0.0;
      for (int k = 0; k < m.n_sie; ++k)
        if (spec.sie_plane[k] == j) add_sie(m, k, px, py, dx, dy);
      if (j == 0) {
        dx += m.g1 * px + m.g2 * py;
        dy += m.g2 * px - m.g1 * py;
      }
      ax[j] = dx;
      ay[j] = dy;
    }
  }
  return I;
}

// One thread per pixel, one block per (point, render tile): the pixel's
// quadrature (N x N midpoint or Gauss-Kronrod), times the pixel weight.
__global__ __launch_bounds__(RENDER_BLOCK) void model_render_kernel(WorkArgs w, ModelSpec spec,
                                                                     const ModelConst* __restrict__ mcs,
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
  const ModelConst& m = mcs[point];
  const int r = pix / sd.W, c = pix - r * sd.W;
  const double ux = (double)c - 0.5 * (double)(sd.W - 1), uy = (double)r - 0.5 * (double)(sd.H - 1);
  const double d = sd.d, cx = sd.cx, cy = sd.cy;
  const int N = sd.N;
  const GkRule* R = sd.rule > 0 ? &kGkRules[sd.rule - 1] : nullptr;
  double acc = 0.0;
  for (int ky = 0; ky < N; ++ky) {
    const double oy = R ? R->xd[ky] : ((double)ky + 0.5) / N - 0.5;
    const double y = cy + (uy + oy) * d;
    for (int kx = 0; kx < N; ++kx) {
      const double ox = R ? R->xd[kx] : ((double)kx + 0.5) / N - 0.5;
      const double wgt = R ? (double)R->w[kx] * (double)R->w[ky] : 1.0;
      const double x = cx + (ux + ox) * d;
      acc += wgt * (spec.n_planes > 1 ? model_sb_planes(m, spec, x, y) : model_sb(m, x, y));
    }
  }
  L[loff + pix] = (float)(acc * sd.wgt);
}

}  // namespace

hipError_t launch_model_render(const WorkArgs& w, const ModelSpec& spec, const ModelConst* mcs, float* L, int n_blocks,
                               hipStream_t stream) {
  if (n_blocks <= 0) return hipSuccess;
  return for_item_parts(w, n_blocks, [&](const WorkArgs& part, int n) {
    hipLaunchKernelGGL(model_render_kernel, dim3(n), dim3(RENDER_BLOCK), 0, stream, part, spec, mcs, L);
    return hipGetLastError();
  });
}

}  // namespace lensed
