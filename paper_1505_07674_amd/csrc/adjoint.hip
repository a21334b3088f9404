// adjoint.hip -- gradient of the log-likelihood with respect to the 17 parameters.
//
// log L = -1/2 sum_i w_i (d_i - L*_i)^2 (Sec. 3.2, Eq. 17), L* = A L with A the
// replicate-padded PSF convolution (Sec. 3.1, Eq. 15) and L_j the midpoint sum
// of Eq. 14. With rho = w (d - L*) (written by the PSF kernel in mode 2):
//   d log L / d theta = sum_j g_j (d^2/N^2) sum_k dI(x_jk)/d theta,  g = A^T rho.
// A^T rho is a zero-padded correlation of rho with the kernel for interior
// pixels; pixels on the first/last row or column use kernel tables folded by
// the padding (computed by the prologue). The per-subsample partial derivatives
// of I(x) = I_lens(x) + I_source(beta(x)) are written out in closed form:
// through the Sersic profiles (Eqs. 22-23, with db_n/dn), and for the lens
// parameters through beta = x - alpha(x) (Eq. 1) using the SIE Jacobian
//   d alpha'/d x' = theta_E sqrt(q)/(psi r^2) [[y'^2, -x'y'], [-x'y', x'^2]].
// Sums are float32 per thread, combined across the block with TwoSum and
// across tiles in float64.
#include <math.h>

#include "internal.h"
#include "kernels.h"
#include "sb_device.h"
#include "stencil.h"

namespace lensed {
namespace {

__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void resolve(const WorkArgs& w, int& point, int& tile) {
  if (w.items) {
    const int2 it = w.items[blockIdx.x];
    point = it.x;
    tile = it.y;
  } else {
    point = w.point0;
    tile = blockIdx.x;
  }
}

// ---------------------------------------------------------------------------
// g = A^T rho, interior pixels: g[u][v] = sum_{a,b} rho0[u+a][v+b] F[a][b].
// ---------------------------------------------------------------------------
// TWc = 0 with P >= 0: a wide tile (runtime width, LDS stride WIDE_STRIDE), as
// in the forward stencil.
template <int P, int TWc, int ROWS>
__global__ __launch_bounds__(P >= 0 && TWc == 0 ? WIDE_MAX_THREADS : 512) void adj_psf_kernel(
    WorkArgs w, const float* __restrict__ R, float* __restrict__ G) {
  constexpr bool WIDE = P >= 0 && TWc == 0;
  extern __shared__ float S[];
  int point, tile;
  resolve(w, point, tile);
  const SysDesc sd = w.sys_table ? w.sys_table[w.point_sys ? w.point_sys[point] : 0] : w.single;
  const int64_t loff = w.point_loff ? w.point_loff[point] : 0;
  const int p = P >= 0 ? P : sd.ph / 2;
  const int q = P >= 0 ? P : sd.pw / 2;
  const int TW = (P >= 0 && !WIDE) ? TWc : sd.TW, TH = sd.TH;
  const int SW = TW + 2 * q, SH = TH + 2 * p;     // staged columns and rows
  const int LS = WIDE ? WIDE_STRIDE : SW;         // LDS row stride
  const int ty = tile / sd.tiles_x, tx = tile - ty * sd.tiles_x;
  const int x0 = tx * TW, y0 = ty * TH;
  const float* __restrict__ Rp = R + loff;
  const int tid = threadIdx.x;
  const int jx = tid % TW, jy = tid / TW;
  const int rows_per_pass = blockDim.x / TW;
  for (int row = jy; row < SH; row += rows_per_pass) {
    const int gi = y0 + row - p;
    for (int col = jx; col < SW; col += TW) {
      const int gj = x0 + col - q;
      S[row * LS + col] = (gi >= 0 && gi < sd.H && gj >= 0 && gj < sd.W) ? Rp[(size_t)gi * sd.W + gj] : 0.0f;
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
    // taps F[k][l] of stencil column l, contiguous in k
    stencil_columns<K, SWc, ROWS>(S + i0 * SWc + jx, uniform_const(sd.psfn + 2 * K * K), acc);
  } else {
    const float* __restrict__ F = sd.psfn;
    const int KH = 2 * p + 1, KW = 2 * q + 1;
    for (int l = 0; l < KW; ++l)
      for (int k = 0; k < KH; ++k) {
        const float f = F[k * KW + l];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) acc[r] = fmaf(f, S[(i0 + r + k) * SW + jx + l], acc[r]);
      }
  }
  const int gj = x0 + jx;
#pragma unroll
  for (int r = 0; r < ROWS; ++r) {
    const int gi = y0 + i0 + r;
    const bool border = gi == 0 || gi == sd.H - 1 || gj == 0 || gj == sd.W - 1;
    if (gi < sd.H && gj < sd.W && i0 + r < TH && !border) G[loff + (size_t)gi * sd.W + gj] = acc[r];
  }
}

// Border pixels of g with the folded tables; blockIdx.y is the point. Eight
// lanes share a pixel: lane `sub` takes the table rows a = -p + sub, -p + sub + 8,
// ..., and the eight partial sums are added in a fixed order by shuffles.
constexpr int BORDER_LANES = 8;

__global__ __launch_bounds__(64) void adj_border_kernel(WorkArgs w, const float* __restrict__ R, float* __restrict__ G,
                                                         int n_border, int point_base) {
  const int point = point_base + (int)blockIdx.y;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int t = (int)(gid / BORDER_LANES), sub = (int)(gid % BORDER_LANES);
  if (t >= n_border) return;   // the eight lanes of a pixel leave together
  const SysDesc sd = w.sys_table ? w.sys_table[w.point_sys ? w.point_sys[point] : 0] : w.single;
  const int64_t loff = w.point_loff ? w.point_loff[point] : 0;
  const int H = sd.H, W = sd.W;
  int u, v;
  if (H <= 2 || W <= 2) {   // every pixel touches a border
    u = t / W;
    v = t - u * W;
  } else if (t < W) {
    u = 0;
    v = t;
  } else if (t < 2 * W) {
    u = H - 1;
    v = t - W;
  } else {
    const int k = t - 2 * W;
    u = 1 + (k >> 1);
    v = (k & 1) ? W - 1 : 0;
  }
  const int cr = (H == 1) ? 3 : (u == 0 ? 1 : (u == H - 1 ? 2 : 0));
  const int cc = (W == 1) ? 3 : (v == 0 ? 1 : (v == W - 1 ? 2 : 0));
  const int p = sd.ph / 2, q = sd.pw / 2;
  const float* __restrict__ K = sd.adjk + (size_t)(cr * 4 + cc) * sd.ph * sd.pw;
  const float* __restrict__ Rp = R + loff;
  float acc = 0.0f;
  for (int a = -p + sub; a <= p; a += BORDER_LANES) {
    const int i = u + a;
    if (i < 0 || i >= H) continue;
    for (int b = -q; b <= q; ++b) {
      const int j = v + b;
      if (j < 0 || j >= W) continue;
      acc = fmaf(K[(a + p) * sd.pw + (b + q)], Rp[(size_t)i * W + j], acc);
    }
  }
  acc += __shfl_xor(acc, 4, BORDER_LANES);
  acc += __shfl_xor(acc, 2, BORDER_LANES);
  acc += __shfl_xor(acc, 1, BORDER_LANES);
  if (sub == 0) G[loff + (size_t)u * W + v] = acc;
}

// ---------------------------------------------------------------------------
// Per-subsample partial derivatives.
// ---------------------------------------------------------------------------

// Uniform per-point values used by the gradient kernel.
struct GradUniform {
  float te, sq, q, s, iqp;   // theta_E, sqrt(q), q, s = 1 - q^2, 1/q' (0 when q = 1)
  float c2, s2, gam;         // shear: cos 2phi, sin 2phi, gamma
  float RH, RS;              // half-light radii
  float qH, qS;              // Sersic axis ratios
  float bH, bS;              // natural-log Sersic constants b = B ln 2
  float dbH, dbS;            // db/dn
};

// Sersic value and derivatives at scaled squared radius rho2.
struct SersicD {
  float I, E, D;     // value, I/I_e, dI/drho2
  float dn;          // dI/dn
};

__device__ __forceinline__ SersicD sersic_d(float rho2, float e, float B, float Ie, float b, float db) {
  SersicD r;
  const float L2 = hw_log2(rho2);
  const float t = hw_exp2(e * L2);
  r.E = hw_exp2(fmaf(-B, t, B));
  r.I = Ie * r.E;
  const bool pos = rho2 > 0.0f;
  r.D = pos ? -r.I * b * t * e / rho2 : 0.0f;
  // dI/dn = I [b'(1 - t) + b t ln(rho2) / (2 n^2)],  1/(2n^2) = 2 e^2
  const float tl = pos ? t * (L2 * LN2F) : 0.0f;
  r.dn = r.I * fmaf(db, 1.0f - t, b * tl * 2.0f * e * e);
  return r;
}

// Series of d/ds [atan(sqrt(s) u)/sqrt(s)] and d/ds [atanh(sqrt(s) v)/sqrt(s)] for small s.
__device__ __forceinline__ float datan_ds_series(float s, float u) {
  const float u2 = u * u, z = s * u2;
  // sum_{k>=1} (-1)^k k s^{k-1} u^{2k+1}/(2k+1)
  const float poly = fmaf(z, fmaf(z, fmaf(z, fmaf(z, fmaf(z, -6.0f / 13.0f, 5.0f / 11.0f), -4.0f / 9.0f), 3.0f / 7.0f),
                              -2.0f / 5.0f),
                         1.0f / 3.0f);
  return -u * u2 * poly;
}
__device__ __forceinline__ float datanh_ds_series(float s, float v) {
  const float v2 = v * v, z = s * v2;
  const float poly = fmaf(z, fmaf(z, fmaf(z, fmaf(z, fmaf(z, 6.0f / 13.0f, 5.0f / 11.0f), 4.0f / 9.0f), 3.0f / 7.0f),
                              2.0f / 5.0f),
                         1.0f / 3.0f);
  return v * v2 * poly;
}

constexpr float S_SERIES = 0.0625f;   // use the series for 1 - q^2 below this

// Adds the 17 partial derivatives of I at subsample (x, y) to acc, times the
// quadrature weight sw when WT (a Gauss-Kronrod node). With `override`, the
// offset of beta from the source centre is (odx, ody) instead of the float32
// lens equation (the float64 re-traced value near a cuspy source).
template <int MODE, bool WT = false>
__device__ __forceinline__ void subsample_grad(const PointConst& c, const GradUniform& U, float x, float y,
                                               float (&acc)[NPAR], bool override = false, float odx = 0.0f,
                                               float ody = 0.0f, float sw = 1.0f) {
  // ---- SIE in its own frame
  const float xp = fmaf(c.cL, x, c.sL * y);
  const float yp = fmaf(c.cL, y, -c.sL * x);
  const float yp2 = yp * yp;
  const float psi2 = fmaf(c.q2 * xp, xp, yp2);
  const float r2 = fmaf(xp, xp, yp2);
  const bool live = psi2 > 0.0f;
  const float ip = live ? hw_rsq(psi2) : 0.0f;
  const float u0 = xp * ip, v0 = yp * ip;   // x'/psi, y'/psi
  float a, b;                                // atan(q'u0)/q', atanh(q'v0)/q'
  if (MODE == 0) {
    a = u0;
    b = v0;
  } else if (MODE == 1) {
    a = atan_small(c.qp * u0) * U.iqp;
    b = atanh_poly(c.qp * v0) * U.iqp;
  } else {
    const float ir = live ? hw_rsq(r2) : 0.0f;
    const float psi = psi2 * ip;
    const float r = r2 * ir;
    a = live ? 2.0f * atan_unit(c.qp * xp * hw_rcp(psi + r)) * U.iqp : 0.0f;
    const float num = fmaf(c.qp, fabsf(yp), psi);
    b = live ? copysignf(LN2F * hw_log2(num * ir * c.iq), yp) * U.iqp : 0.0f;
  }
  const float apx = U.te * U.sq * a, apy = U.te * U.sq * b;   // alpha' in the frame
  // d/ds of a and b
  float da, db;
  if (U.s < S_SERIES) {
    da = datan_ds_series(U.s, u0);
    db = datanh_ds_series(U.s, v0);
  } else {
    const float pr = live ? psi2 * hw_rcp(r2) : 0.0f;   // psi^2 / r^2
    da = (u0 * pr - a) * (0.5f / U.s);
    db = (v0 * pr * (1.0f / (U.q * U.q)) - b) * (0.5f / U.s);
  }
  const float pr2 = live ? psi2 * hw_rcp(r2) : 0.0f;
  // frame derivatives
  const float dte_x = U.sq * a, dte_y = U.sq * b;
  const float dphi_x = U.te * U.sq * (v0 - b), dphi_y = U.te * U.sq * (a - u0);
  const float dq_x = U.te * (a * (0.5f / U.sq) + U.sq * (-2.0f * U.q * da - U.q * u0 * u0 * u0 * pr2));
  const float dq_y = U.te * (b * (0.5f / U.sq) + U.sq * (-2.0f * U.q * db - v0 * u0 * u0 * pr2 / U.q));
  // back to the image frame
  auto rot_x = [&](float fx, float fy) { return fmaf(c.cL, fx, -c.sL * fy); };
  auto rot_y = [&](float fx, float fy) { return fmaf(c.sL, fx, c.cL * fy); };
  const float ax = rot_x(apx, apy), ay = rot_y(apx, apy);
  // ---- lens equation and source
  const float bx = fmaf(c.m11, x, fmaf(c.m12, y, -ax));
  const float by = fmaf(c.m12, x, fmaf(c.m22, y, -ay));
  const float dx = override ? odx : bx - c.sx0, dy = override ? ody : by - c.sy0;
  const float sxp = fmaf(c.sc, dx, c.ss * dy);
  const float syp = fmaf(c.sc, dy, -c.ss * dx);
  const float srho2 = fmaf(c.sqa * sxp, sxp, c.sqb * syp * syp);
  SersicD Sd = sersic_d(srho2, c.se, c.sB, c.sI, U.bS, U.dbS);
  if (WT) {
    Sd.E *= sw;
    Sd.D *= sw;
    Sd.dn *= sw;
  }
  const float gxp = 2.0f * c.sqa * sxp, gyp = 2.0f * c.sqb * syp;   // d rho2 / d(x', y') of the source frame
  const float Gx = Sd.D * fmaf(gxp, c.sc, -gyp * c.ss);
  const float Gy = Sd.D * fmaf(gxp, c.ss, gyp * c.sc);
  // ---- lens light
  const float hxp = fmaf(c.hc, x, c.hs * y);
  const float hyp = fmaf(c.hc, y, -c.hs * x);
  const float hrho2 = fmaf(c.hqa * hxp, hxp, c.hqb * hyp * hyp);
  SersicD Hd = sersic_d(hrho2, c.he, c.hB, c.hI, U.bH, U.dbH);
  if (WT) {
    Hd.E *= sw;
    Hd.D *= sw;
    Hd.dn *= sw;
  }
  // ---- accumulate
  acc[0] -= Gx * rot_x(dte_x, dte_y) + Gy * rot_y(dte_x, dte_y);
  acc[1] -= Gx * rot_x(dq_x, dq_y) + Gy * rot_y(dq_x, dq_y);
  acc[2] -= Gx * rot_x(dphi_x, dphi_y) + Gy * rot_y(dphi_x, dphi_y);
  acc[3] -= Gx * fmaf(U.c2, x, U.s2 * y) + Gy * fmaf(U.s2, x, -U.c2 * y);
  acc[4] -= 2.0f * U.gam * (Gx * fmaf(-U.s2, x, U.c2 * y) + Gy * fmaf(U.c2, x, U.s2 * y));
  acc[5] += Hd.E;
  acc[6] += -2.0f * hrho2 * Hd.D / U.RH;
  acc[7] += Hd.dn;
  acc[8] += Hd.D * (c.hqa * hxp * hxp - c.hqb * hyp * hyp) / U.qH;
  acc[9] += Hd.D * 2.0f * hxp * hyp * (c.hqa - c.hqb);
  acc[10] -= Gx;
  acc[11] -= Gy;
  acc[12] += Sd.E;
  acc[13] += -2.0f * srho2 * Sd.D / U.RS;
  acc[14] += Sd.dn;
  acc[15] += Sd.D * (c.sqa * sxp * sxp - c.sqb * syp * syp) / U.qS;
  acc[16] += Sd.D * 2.0f * sxp * syp * (c.sqa - c.sqb);
}

template <int MODE>
__device__ __forceinline__ void pixel_grad(const PointConst& c, const GradUniform& U, int N, const PixelGeom& g,
                                           float (&acc)[NPAR]) {
  for (int ky = 0; ky < N; ++ky) {
    const float y = fmaf(g.uy + sub_offset_rt(ky, N), g.d, g.cy);
    for (int kx = 0; kx < N; ++kx) {
      const float x = fmaf(g.ux + sub_offset_rt(kx, N), g.d, g.cx);
      subsample_grad<MODE>(c, U, x, y, acc);
    }
  }
}

// The same over the Cartesian square of a Gauss-Kronrod rule (K nodes), each
// subsample weighted by w_i w_j (the pixel weight d^2 multiplies later).
template <int MODE>
__device__ __forceinline__ void pixel_grad_gk(const PointConst& c, const GradUniform& U, int rule, int K,
                                              const PixelGeom& g, float (&acc)[NPAR]) {
  const GkRule& R = kGkRules[rule - 1];
  for (int ky = 0; ky < K; ++ky) {
    const float y = fmaf(g.uy + R.x[ky], g.d, g.cy);
    for (int kx = 0; kx < K; ++kx) {
      const float x = fmaf(g.ux + R.x[kx], g.d, g.cx);
      subsample_grad<MODE, true>(c, U, x, y, acc, false, 0.0f, 0.0f, R.w[kx] * R.w[ky]);
    }
  }
}

// One thread per pixel, one block per (point, render tile): sums
// g_pix * d^2/N^2 * dI/dtheta over the pixel's subsamples, then over the block.
__global__ __launch_bounds__(RENDER_BLOCK) void grad_kernel(WorkArgs w, const PointConst* __restrict__ pcs,
                                                             const GradConst* __restrict__ gcs,
                                                             const float* __restrict__ G,
                                                             const int* __restrict__ gpbase,
                                                             float2* __restrict__ gpart) {
  __shared__ float red_hi[RENDER_BLOCK / 64][NPAR], red_lo[RENDER_BLOCK / 64][NPAR];
  int point, tile;
  resolve(w, point, tile);
  const SysDesc sd = w.sys_table ? w.sys_table[w.point_sys ? w.point_sys[point] : 0] : w.single;
  const int64_t loff = w.point_loff ? w.point_loff[point] : 0;
  const PointConst& c = pcs[point];
  const GradConst& gc = gcs[point];
  GradUniform U;
  U.te = gc.theta[0];
  U.q = gc.theta[1];
  U.sq = sqrtf(U.q);
  U.s = (1.0f - U.q) * (1.0f + U.q);
  U.iqp = c.sie_mode == 0 ? 0.0f : 1.0f / c.qp;
  float s2, c2;
  sincosf(2.0f * gc.theta[4], &s2, &c2);
  U.c2 = c2;
  U.s2 = s2;
  U.gam = gc.theta[3];
  U.RH = gc.theta[6];
  U.RS = gc.theta[13];
  U.qH = gc.theta[8];
  U.qS = gc.theta[15];
  U.bH = c.hB * LN2F;
  U.bS = c.sB * LN2F;
  U.dbH = gc.dB_dn_h * LN2F;
  U.dbS = gc.dB_dn_s * LN2F;

  float acc[NPAR];
#pragma unroll
  for (int k = 0; k < NPAR; ++k) acc[k] = 0.0f;
  const int pix = tile * RENDER_BLOCK + (int)threadIdx.x;
  if (pix < sd.H * sd.W) {
    const float gp = G[loff + pix];
    if (gp != 0.0f) {   // pixels outside the reach of any weighted residual add nothing
      const int r = pix / sd.W;
      const int col = pix - r * sd.W;
      PixelGeom geo;
      geo.ux = (float)col - 0.5f * (float)(sd.W - 1);
      geo.uy = (float)r - 0.5f * (float)(sd.H - 1);
      geo.d = sd.d;
      geo.cx = sd.cx;
      geo.cy = sd.cy;
      if (sd.rule == 0) {
        switch (c.sie_mode) {
          case 0: pixel_grad<0>(c, U, sd.N, geo, acc); break;
          case 1: pixel_grad<1>(c, U, sd.N, geo, acc); break;
          default: pixel_grad<2>(c, U, sd.N, geo, acc); break;
        }
      } else {
        switch (c.sie_mode) {
          case 0: pixel_grad_gk<0>(c, U, sd.rule, sd.N, geo, acc); break;
          case 1: pixel_grad_gk<1>(c, U, sd.rule, sd.N, geo, acc); break;
          default: pixel_grad_gk<2>(c, U, sd.rule, sd.N, geo, acc); break;
        }
      }
      const float wgt = (float)sd.wgt * gp;
#pragma unroll
      for (int k = 0; k < NPAR; ++k) acc[k] *= wgt;
    }
  }
  // block reduction of the 17 sums with error-free transformations
  float lo[NPAR];
#pragma unroll
  for (int k = 0; k < NPAR; ++k) lo[k] = 0.0f;
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int k = 0; k < NPAR; ++k) {
      const float h2 = __shfl_down(acc[k], off, 64);
      const float l2 = __shfl_down(lo[k], off, 64);
      float s, e;
      two_sum(acc[k], h2, s, e);
      acc[k] = s;
      lo[k] = lo[k] + l2 + e;
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NPAR; ++k) {
      red_hi[wid][k] = acc[k];
      red_lo[wid][k] = lo[k];
    }
  }
  __syncthreads();
  if (threadIdx.x < NPAR) {
    const int k = threadIdx.x;
    float h = red_hi[0][k], l = red_lo[0][k];
    for (int i = 1; i < RENDER_BLOCK / 64; ++i) {
      float s, e;
      two_sum(h, red_hi[i][k], s, e);
      h = s;
      l = l + red_lo[i][k] + e;
    }
    const int base = gpbase ? gpbase[point] : 0;
    gpart[(size_t)(base + tile) * NPAR + k] = make_float2(h, l);
  }
}

// Cusp correction of the gradient: the waves the forward render flagged (same
// pixels, same float32 test) get, for each subsample in the cusp zone, the
// partials at the float64 re-traced source offset minus the float32 ones,
// weighted by g d^2/N^2 (midpoint rule) or g d^2 w_i w_j (Gauss-Kronrod) and
// added to corr[point][k] in float64.
constexpr int GCUSP_WAVES = 4;
constexpr int GCUSP_BLOCKS = 1024;

// The subsamples inside the radius are first found in float32 and queued per
// wave in LDS, then each lane takes one queued subsample at a time, so the
// float64 re-tracing and the two sets of partials run with every lane busy.
constexpr int GCUSP_CHUNK = 16;   // subsamples per pass

__device__ __forceinline__ void gcusp_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ PixelGeom gcusp_geom(const SysDesc& sd, int pix) {
  const int r = pix / sd.W;
  const int col = pix - r * sd.W;
  PixelGeom geo;
  geo.ux = (float)col - 0.5f * (float)(sd.W - 1);
  geo.uy = (float)r - 0.5f * (float)(sd.H - 1);
  geo.d = sd.d;
  geo.cx = sd.cx;
  geo.cy = sd.cy;
  return geo;
}

__global__ __launch_bounds__(64 * GCUSP_WAVES) void grad_cusp_kernel(WorkArgs w, const PointConst* __restrict__ pcs,
                                                                     const PointConst64* __restrict__ p64s,
                                                                     const GradConst* __restrict__ gcs,
                                                                     const float* __restrict__ G, CuspList cl,
                                                                     double* __restrict__ corr) {
  __shared__ unsigned short queue[GCUSP_WAVES][GCUSP_CHUNK * 64];   // lane | subsample << 6
  const int n = *cl.count;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wave = blockIdx.x * GCUSP_WAVES + wv;
  unsigned short* __restrict__ qu = queue[wv];
  for (int i = wave; i < n; i += gridDim.x * GCUSP_WAVES) {
    const CuspEntry e = cl.entries[i];
    const bool mine = (e.mask >> lane) & 1ull;
    const SysDesc sd = w.sys_table ? w.sys_table[w.point_sys ? w.point_sys[e.point] : 0] : w.single;
    const int64_t loff = w.point_loff ? w.point_loff[e.point] : 0;
    const PointConst& c = pcs[e.point];
    const GradConst& gc = gcs[e.point];
    GradUniform U;
    U.te = gc.theta[0];
    U.q = gc.theta[1];
    U.sq = sqrtf(U.q);
    U.s = (1.0f - U.q) * (1.0f + U.q);
    U.iqp = c.sie_mode == 0 ? 0.0f : 1.0f / c.qp;
    float s2, c2;
    sincosf(2.0f * gc.theta[4], &s2, &c2);
    U.c2 = c2;
    U.s2 = s2;
    U.gam = gc.theta[3];
    U.RH = gc.theta[6];
    U.RS = gc.theta[13];
    U.qH = gc.theta[8];
    U.qS = gc.theta[15];
    U.bH = c.hB * LN2F;
    U.bS = c.sB * LN2F;
    U.dbH = gc.dB_dn_h * LN2F;
    U.dbS = gc.dB_dn_s * LN2F;
    const int lpix = mine ? unit_pixel(sd, e.unit0 + lane, e.ppt) + e.half : 0;   // this lane's pixel
    const PixelGeom geo = gcusp_geom(sd, lpix);
    // the render constants the forward render used for this lane's pixel
    const int prow = lpix / sd.W;
    const RenderVariant& kv = c.rv[render_variant(prow, lpix - prow * sd.W)];
    const int N = sd.N, NN = N * N;
    const GkRule* Rg = sd.rule > 0 ? &kGkRules[sd.rule - 1] : nullptr;
    float acc[NPAR];
#pragma unroll
    for (int k = 0; k < NPAR; ++k) acc[k] = 0.0f;
    for (int s0 = 0; s0 < NN; s0 += GCUSP_CHUNK) {
      const int ns = min(GCUSP_CHUNK, NN - s0);
      int qn = 0;
      for (int j = 0; j < ns; ++j) {
        const int ky = (s0 + j) / N, kx = s0 + j - ky * N;
        const float y = fmaf(geo.uy + (Rg ? Rg->x[ky] : sub_offset_rt(ky, N)), geo.d, geo.cy);
        const float x = fmaf(geo.ux + (Rg ? Rg->x[kx] : sub_offset_rt(kx, N)), geo.d, geo.cx);
        const bool within = mine && render_source_R2(c, kv, x, y) < c.cusp_r2;
        const unsigned long long b = __ballot(within);
        if (within) qu[qn + __popcll(b & ((1ull << lane) - 1ull))] = (unsigned short)(lane | (j << 6));
        qn += __popcll(b);
      }
      gcusp_lds_sync();
      for (int q0 = 0; q0 < qn; q0 += 64) {
        if (q0 + lane < qn) {
          const int item = qu[q0 + lane];
          const int pl = item & 63, j = item >> 6;
          const int ky = (s0 + j) / N, kx = s0 + j - ky * N;
          const int qpix = unit_pixel(sd, e.unit0 + pl, e.ppt) + e.half;
          const PixelGeom gq = gcusp_geom(sd, qpix);
          const float y = fmaf(gq.uy + (Rg ? Rg->x[ky] : sub_offset_rt(ky, N)), gq.d, gq.cy);
          const float x = fmaf(gq.ux + (Rg ? Rg->x[kx] : sub_offset_rt(kx, N)), gq.d, gq.cx);
          const double oy = Rg ? Rg->xd[ky] : ((double)ky + 0.5) / N - 0.5;
          const double ox = Rg ? Rg->xd[kx] : ((double)kx + 0.5) / N - 0.5;
          const float sw = Rg ? Rg->w[kx] * Rg->w[ky] : 1.0f;
          float dx, dy;
          source_offset_f64(p64s[e.point], gq, ox, oy, dx, dy);
          float a64[NPAR], a32[NPAR];
#pragma unroll
          for (int k = 0; k < NPAR; ++k) a64[k] = a32[k] = 0.0f;
          switch (c.sie_mode) {
            case 0:
              subsample_grad<0, true>(c, U, x, y, a32, false, 0.0f, 0.0f, sw);
              subsample_grad<0, true>(c, U, x, y, a64, true, dx, dy, sw);
              break;
            case 1:
              subsample_grad<1, true>(c, U, x, y, a32, false, 0.0f, 0.0f, sw);
              subsample_grad<1, true>(c, U, x, y, a64, true, dx, dy, sw);
              break;
            default:
              subsample_grad<2, true>(c, U, x, y, a32, false, 0.0f, 0.0f, sw);
              subsample_grad<2, true>(c, U, x, y, a64, true, dx, dy, sw);
              break;
          }
          const float wg = (float)sd.wgt * G[loff + qpix];
#pragma unroll
          for (int k = 0; k < NPAR; ++k) acc[k] = fmaf(a64[k] - a32[k], wg, acc[k]);
        }
      }
      gcusp_lds_sync();
    }
    // every lane of an entry belongs to the same point
#pragma unroll
    for (int k = 0; k < NPAR; ++k) {
      float v = acc[k];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if (lane == 0 && v != 0.0f) atomicAdd(&corr[(size_t)e.point * NPAR + k], (double)v);
    }
  }
}

// grad[p][k] = sum over the point's render tiles of (hi + lo) plus the cusp
// correction, in float64.
// Sum of one gradient entry k of point p over its tiles (and its cusp term).
__device__ double grad_entry(const float2* __restrict__ gpart, int base, int ntiles, const double* __restrict__ corr,
                             int p, int k) {
  double s = corr ? corr[(size_t)p * NPAR + k] : 0.0;
  for (int i = 0; i < ntiles; ++i) {
    const float2 v = gpart[(size_t)(base + i) * NPAR + k];
    s += (double)v.x + (double)v.y;
  }
  return s;
}

// With magnitudes, slots 5 and 12 of the sums hold d log L / d I_e and slots
// 6, 7 and 13, 14 the derivatives at fixed I_e; the chain rule through
// I_e(m, R_e, n) gives d/dm = g_I I_e dlnI/dm and adds g_I I_e dlnI/dR_e and
// g_I I_e dlnI/dn to the radius and index entries. With an image-plane source
// position, slots 10 and 11 hold d log L / d beta; the chain rule through
// beta(x_I, y_I, theta_E, q_L, phi_L, gamma, phi_gamma) gives d/dx_I, d/dy_I and
// adds g_beta . d beta / d theta_k to the five lens entries.
__global__ void finalize_grad_kernel(const float2* __restrict__ gpart, const int* __restrict__ gpbase, int ntiles,
                                     int n_points, const double* __restrict__ corr,
                                     const GradConst* __restrict__ gcs, float* __restrict__ grad) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_points * NPAR) return;
  const int p = t / NPAR, k = t - p * NPAR;
  const int base = gpbase ? gpbase[p] : 0;
  double s = grad_entry(gpart, base, ntiles, corr, p, k);
  if (gcs && gcs[p].srcpos && (k <= 4 || k == 10 || k == 11)) {
    const float* J = gcs[p].src_jac;
    const double gx = k == 10 ? s : grad_entry(gpart, base, ntiles, corr, p, 10);
    const double gy = k == 11 ? s : grad_entry(gpart, base, ntiles, corr, p, 11);
    const int col = k <= 4 ? k + 2 : k - 10;
    const double chain = gx * (double)J[col] + gy * (double)J[7 + col];
    s = k <= 4 ? s + chain : chain;
  }
  if (gcs && gcs[p].amp) {
    const GradConst& gc = gcs[p];
    if (k >= 5 && k <= 7) {
      const double gI = k == 5 ? s : grad_entry(gpart, base, ntiles, corr, p, 5);
      s = k == 5 ? gI * (double)gc.amp_chain[0] : s + gI * (double)gc.amp_chain[k - 5];
    } else if (k >= 12 && k <= 14) {
      const double gI = k == 12 ? s : grad_entry(gpart, base, ntiles, corr, p, 12);
      s = k == 12 ? gI * (double)gc.amp_chain[3] : s + gI * (double)gc.amp_chain[k - 9];
    }
  }
  grad[t] = (float)s;
}

template <int P, int TWc, int R>
hipError_t launch_adj_t(const WorkArgs& w, const float* R_, float* G, int n_blocks, int threads, size_t lds,
                        hipStream_t st) {
  return for_item_parts(w, n_blocks, [&](const WorkArgs& part, int n) {
    hipLaunchKernelGGL((adj_psf_kernel<P, TWc, R>), dim3(n), dim3(threads), lds, st, part, R_, G);
    return hipGetLastError();
  });
}

template <int P, int R>
hipError_t launch_adj_w(int TW, const WorkArgs& w, const float* R_, float* G, int n_blocks, int threads, size_t lds,
                        hipStream_t st) {
  if (TW == 64) return launch_adj_t<P, 64, R>(w, R_, G, n_blocks, threads, lds, st);
  return launch_adj_t<P, 32, R>(w, R_, G, n_blocks, threads, lds, st);
}

}  // namespace

hipError_t launch_adjoint_psf(const WorkArgs& w, const float* R, float* G, int n_blocks, int square_psf, int TW,
                              int TH, int ph, int pw, int n_points, int H, int W, hipStream_t st) {
  if (n_blocks <= 0) return hipSuccess;
  const int Rr = psf_rows(square_psf, TW, TH);
  const int threads = TW * (TH / Rr);
  const size_t lds = psf_lds_bytes(square_psf, TW, TH, ph, pw);
  hipError_t e;
  if (psf_wide(square_psf, TW)) {
    e = launch_adj_t<10, 0, 8>(w, R, G, n_blocks, threads, lds, st);
  } else if (psf_specialised(square_psf, TW)) {
    if (square_psf == 21) e = Rr == 8 ? launch_adj_w<10, 8>(TW, w, R, G, n_blocks, threads, lds, st)
                                      : launch_adj_w<10, 4>(TW, w, R, G, n_blocks, threads, lds, st);
    else if (square_psf == 7) e = launch_adj_w<3, 4>(TW, w, R, G, n_blocks, threads, lds, st);
    else e = launch_adj_w<0, 4>(TW, w, R, G, n_blocks, threads, lds, st);
  } else {
    e = launch_adj_t<-1, 0, 4>(w, R, G, n_blocks, threads, lds, st);
  }
  if (e != hipSuccess) return e;
  const int nb = (H <= 2 || W <= 2) ? H * W : 2 * W + 2 * (H - 2);
  // one grid row per point, at most 65535 rows per launch
  for (int p0 = 0; p0 < n_points; p0 += 65535) {
    const int np = n_points - p0 < 65535 ? n_points - p0 : 65535;
    hipLaunchKernelGGL(adj_border_kernel, dim3((unsigned)(((int64_t)nb * BORDER_LANES + 63) / 64), np), dim3(64), 0, st, w, R, G, nb, p0);
    const hipError_t le = hipGetLastError();
    if (le != hipSuccess) return le;
  }
  return hipSuccess;
}

hipError_t launch_grad(const WorkArgs& w, const PointConst* pcs, const PointConst64* p64s, const GradConst* gcs,
                       const float* G, const int* gpbase, float2* gpart, int n_blocks, const CuspList& cl,
                       double* corr, hipStream_t st, hipEvent_t between) {
  if (n_blocks <= 0) return between ? hipEventRecord(between, st) : hipSuccess;
  hipError_t e = for_item_parts(w, n_blocks, [&](const WorkArgs& part, int n) {
    hipLaunchKernelGGL(grad_kernel, dim3(n), dim3(RENDER_BLOCK), 0, st, part, pcs, gcs, G, gpbase, gpart);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  if (between && (e = hipEventRecord(between, st)) != hipSuccess) return e;
  const int waves = n_blocks * (RENDER_BLOCK / 64);
  int grid = (waves + GCUSP_WAVES - 1) / GCUSP_WAVES;
  if (grid > GCUSP_BLOCKS) grid = GCUSP_BLOCKS;
  hipLaunchKernelGGL(grad_cusp_kernel, dim3(grid), dim3(64 * GCUSP_WAVES), 0, st, w, pcs, p64s, gcs, G, cl, corr);
  return hipGetLastError();
}

hipError_t launch_finalize_grad(const float2* gpart, const int* gpbase, int ntiles, int n_points, const double* corr,
                                const GradConst* gcs, float* grad, hipStream_t st) {
  if (n_points <= 0) return hipSuccess;
  const int n = n_points * NPAR;
  hipLaunchKernelGGL(finalize_grad_kernel, dim3((n + 127) / 128), dim3(128), 0, st, gpart, gpbase, ntiles, n_points,
                     corr, gcs, grad);
  return hipGetLastError();
}

}  // namespace lensed
