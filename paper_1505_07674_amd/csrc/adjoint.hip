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
// Each partial is a fixed per-point linear combination of 17 moments (sums
// over subsamples of products that vary per subsample, e.g. sum D h'_x^2),
// so the kernels accumulate the moments and the final pass maps them to the
// 17 partials in float64 (grad_from_moments). Sums are float32 per thread,
// combined across the block and across tiles in float64.
#include <math.h>

#include "internal.h"
#include "kernels.h"
#include "sb_device.h"
#include "stencil.h"

namespace lensed {
namespace {

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

// Border pixels of g with the folded tables. A block takes a segment of up to
// BORDER_SEG consecutive pixels on one side of the image (top row, bottom row,
// then the left and right columns without their corners; blockIdx.y is the
// point) and stages the window of rho they read in LDS, zero outside the image,
// so every table row is a full PW-tap dot product (a zero tap adds exactly
// nothing). Each pixel has BORDER_SUB lanes: lane `sub` takes the table rows
// a = a_lo + sub, a_lo + sub + BORDER_SUB, ... of the rows that fall inside the
// image, and the partial sums are added in a fixed order by shuffles. PW = 0:
// the table width is a runtime value.
constexpr int BORDER_SEG = 64;
constexpr int BORDER_SUB = 4;

__host__ __device__ inline int border_row_segments(int W) { return (W + BORDER_SEG - 1) / BORDER_SEG; }
__host__ __device__ inline int border_side_segments(int H) { return H > 2 ? (H - 2 + BORDER_SEG - 1) / BORDER_SEG : 0; }
// Segments of an H x W image: every pixel on the first or last row or column
// lies in exactly one (the bottom row is absent when H = 1, the right column
// when W = 1).
__host__ __device__ inline int border_segments(int H, int W) {
  return border_row_segments(W) * (H > 1 ? 2 : 1) + border_side_segments(H) * (W > 1 ? 2 : 1);
}
// LDS floats of the largest window for a PSF of ph x pw.
__host__ __device__ inline int border_lds_floats(int ph, int pw) {
  const int row = ph * (BORDER_SEG + pw - 1), col = (BORDER_SEG + ph - 1) * pw;
  return row > col ? row : col;
}

template <int PW>
__global__ __launch_bounds__(BORDER_SEG* BORDER_SUB) void adj_border_kernel(WorkArgs w, const float* __restrict__ R,
                                                                             float* __restrict__ G, int point_base) {
  extern __shared__ float S[];
  const int point = point_base + (int)blockIdx.y;
  const SysDesc sd = w.sys_table ? w.sys_table[w.point_sys ? w.point_sys[point] : 0] : w.single;
  const int64_t loff = w.point_loff ? w.point_loff[point] : 0;
  if (w.point_goff && w.point_goff[point] != loff) return;   // a composite model's later component: no rho of its own
  const int H = sd.H, W = sd.W, p = sd.ph / 2, q = sd.pw / 2;
  const int pw = PW > 0 ? PW : sd.pw;
  const int nrow = border_row_segments(W), nbot = H > 1 ? nrow : 0;
  const int nside = border_side_segments(H), nright = W > 1 ? nside : 0;
  int seg = (int)blockIdx.x;
  bool is_row;
  int u0, v0;
  if (seg < nrow) {
    is_row = true, u0 = 0, v0 = seg * BORDER_SEG;
  } else if ((seg -= nrow) < nbot) {
    is_row = true, u0 = H - 1, v0 = seg * BORDER_SEG;
  } else if ((seg -= nbot) < nside) {
    is_row = false, u0 = 1 + seg * BORDER_SEG, v0 = 0;
  } else if ((seg -= nside) < nright) {
    is_row = false, u0 = 1 + seg * BORDER_SEG, v0 = W - 1;
  } else {
    return;   // uniform over the block, before any barrier
  }
  const int len = is_row ? min(BORDER_SEG, W - v0) : min(BORDER_SEG, H - 1 - u0);
  const int u1 = is_row ? u0 : u0 + len - 1, v1 = is_row ? v0 + len - 1 : v0;
  // window of rho: rows u0 - p .. u1 + p, columns v0 - q .. v1 + q
  const int wr0 = u0 - p, wc0 = v0 - q;
  const int WC = v1 - v0 + 1 + 2 * q, n_win = (u1 - u0 + 1 + 2 * p) * WC;
  const float* __restrict__ Rp = R + loff;
  for (int i = (int)threadIdx.x; i < n_win; i += (int)blockDim.x) {
    const int r = i / WC, gi = wr0 + r, gj = wc0 + (i - r * WC);
    S[i] = (gi >= 0 && gi < H && gj >= 0 && gj < W) ? Rp[(size_t)gi * W + gj] : 0.0f;
  }
  // PW > 0: the four folded tables the segment's pixels use (one row class,
  // every column class; the side columns are all of row class 0) go to LDS too
  const int ntab = sd.ph * pw;
  float* __restrict__ SK = S + border_lds_floats(sd.ph, pw);
  const int t0 = is_row ? 4 * ((H == 1) ? 3 : (u0 == 0 ? 1 : 2)) : 0;
  if (PW > 0)
    for (int i = (int)threadIdx.x; i < 4 * ntab; i += (int)blockDim.x) SK[i] = sd.adjk[(size_t)t0 * ntab + i];
  __syncthreads();
  const int j = (int)threadIdx.x / BORDER_SUB, sub = (int)threadIdx.x % BORDER_SUB;
  float acc = 0.0f;
  const int u = is_row ? u0 : u0 + j, v = is_row ? v0 + j : v0;
  if (j < len) {
    const int cr = (H == 1) ? 3 : (u == 0 ? 1 : (u == H - 1 ? 2 : 0));
    const int cc = (W == 1) ? 3 : (v == 0 ? 1 : (v == W - 1 ? 2 : 0));
    const float* __restrict__ K =
        PW > 0 ? SK + (size_t)(cr * 4 + cc - t0) * ntab : sd.adjk + (size_t)(cr * 4 + cc) * ntab;
    const int a_lo = max(-p, -u), a_hi = min(p, H - 1 - u);
    for (int a = a_lo + sub; a <= a_hi; a += BORDER_SUB) {
      const float* __restrict__ Kr = K + (a + p) * pw;
      const float* __restrict__ Sr = S + (u + a - wr0) * WC + (v - q - wc0);
      if (PW > 0) {
#pragma unroll
        for (int b = 0; b < PW; ++b) acc = fmaf(Kr[b], Sr[b], acc);
      } else {
        for (int b = 0; b < pw; ++b) acc = fmaf(Kr[b], Sr[b], acc);
      }
    }
  }
  acc += __shfl_xor(acc, 2, BORDER_SUB);
  acc += __shfl_xor(acc, 1, BORDER_SUB);
  if (j < len && sub == 0) G[loff + (size_t)u * W + v] = acc;
}

// ---------------------------------------------------------------------------
// Per-subsample partial derivatives.
// ---------------------------------------------------------------------------

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
  r.D = pos ? -r.I * b * t * e * hw_rcp(rho2) : 0.0f;
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
// SER: 1 the series in s, 0 the closed form, -1 chosen here by s (a per-point
// choice that a caller may take once outside its subsample loop).
template <int MODE, bool WT = false, int SER = -1>
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
  const float apx = U.tesq * a, apy = U.tesq * b;   // alpha' in the frame
  // d/ds of a and b
  float da, db;
  if (SER == 1 || (SER < 0 && U.s < S_SERIES)) {
    da = datan_ds_series(U.s, u0);
    db = datanh_ds_series(U.s, v0);
  } else {
    const float pr = live ? psi2 * hw_rcp(r2) : 0.0f;   // psi^2 / r^2
    da = (u0 * pr - a) * U.hs;
    db = (v0 * pr * U.iq2 - b) * U.hs;
  }
  const float pr2 = live ? psi2 * hw_rcp(r2) : 0.0f;
  // back to the image frame
  const float ax = fmaf(c.cL, apx, -c.sL * apy), ay = fmaf(c.sL, apx, c.cL * apy);
  // ---- lens equation and source
  const float bx = fmaf(c.m11, x, fmaf(c.m12, y, -ax));
  const float by = fmaf(c.m12, x, fmaf(c.m22, y, -ay));
  const float dx = override ? odx : bx - c.sx0, dy = override ? ody : by - c.sy0;
  const float sxp = fmaf(c.sc, dx, c.ss * dy);
  const float syp = fmaf(c.sc, dy, -c.ss * dx);
  const float sx2 = sxp * sxp, sy2 = syp * syp;
  const float srho2 = fmaf(c.sqa, sx2, c.sqb * sy2);
  SersicD Sd = sersic_d(srho2, c.se, c.sB, c.sI, U.bS, U.dbS);
  if (WT) {
    Sd.E *= sw;
    Sd.D *= sw;
    Sd.dn *= sw;
  }
  // dI/dbeta in the SIE frame: D times the source-frame gradient of rho^2,
  // rotated by phi_S - phi_L
  const float gxp = 2.0f * c.sqa * sxp, gyp = 2.0f * c.sqb * syp;
  const float Gx = Sd.D * fmaf(gxp, U.kS1, -gyp * U.kS2);
  const float Gy = Sd.D * fmaf(gxp, U.kS2, gyp * U.kS1);
  // ---- lens light
  const float hxp = fmaf(c.hc, x, c.hs * y);
  const float hyp = fmaf(c.hc, y, -c.hs * x);
  const float hx2 = hxp * hxp, hy2 = hyp * hyp;
  const float hrho2 = fmaf(c.hqa, hx2, c.hqb * hy2);
  SersicD Hd = sersic_d(hrho2, c.he, c.hB, c.hI, U.bH, U.dbH);
  if (WT) {
    Hd.E *= sw;
    Hd.D *= sw;
    Hd.dn *= sw;
  }
  // ---- accumulate the moments (grad_from_moments maps them to the partials)
  const float u2pr = u0 * u0 * pr2;
  acc[0] += fmaf(a, Gx, b * Gy);
  acc[1] += fmaf(Gx, fmaf(2.0f, da, u0 * u2pr), Gy * fmaf(2.0f, db, v0 * u2pr * U.iq2));
  acc[2] += fmaf(v0 - b, Gx, (a - u0) * Gy);
  acc[3] += fmaf(Gx, xp, -Gy * yp);
  acc[4] += fmaf(Gx, yp, Gy * xp);
  acc[5] += Hd.E;
  acc[6] += Hd.D * hx2;
  acc[7] += Hd.dn;
  acc[8] += Hd.D * hy2;
  acc[9] += Hd.D * (hxp * hyp);
  acc[10] += Gx;
  acc[11] += Gy;
  acc[12] += Sd.E;
  acc[13] += Sd.D * sx2;
  acc[14] += Sd.dn;
  acc[15] += Sd.D * sy2;
  acc[16] += Sd.D * (sxp * syp);
}

// The 17 partials from the moments, for one point, in float64:
//   M0 = sum a G'x + b G'y,  M1 = sum G'x (2 da + u0^3 pr) + G'y (2 db + v0 u0^2 pr / q^2),
//   M2 = sum (v0 - b) G'x + (a - u0) G'y,  M3 = sum G'x x' - G'y y',  M4 = sum G'x y' + G'y x'
// (G' = dI/dbeta in the SIE frame, x' the SIE frame), M10, M11 = sum G', and
// per Sersic the value, dI/dn and D times x'^2, y'^2, x'y' in its own frame.
__device__ void grad_from_moments(const double (&M)[NPAR], const PointConst& c, const GradConst& gc, double (&g)[NPAR]) {
  const double te = gc.theta[0], q = gc.theta[1], sq = sqrt(q), gam = gc.theta[3];
  const double cL = c.cL, sL = c.sL;
  // the shear angle relative to the SIE frame
  const double ph = 2.0 * ((double)gc.theta[4] - (double)gc.theta[2]);
  const double c2 = cos(ph), s2 = sin(ph);
  g[0] = -sq * M[0];
  g[1] = -te * (0.5 / sq * M[0] - sq * q * M[1]);
  g[2] = -te * sq * M[2];
  g[3] = -(c2 * M[3] + s2 * M[4]);
  g[4] = -2.0 * gam * (c2 * M[4] - s2 * M[3]);
  const double hqa = c.hqa, hqb = c.hqb, sqa = c.sqa, sqb = c.sqb;
  g[5] = M[5];
  g[6] = -2.0 / gc.theta[6] * (hqa * M[6] + hqb * M[8]);
  g[7] = M[7];
  g[8] = (hqa * M[6] - hqb * M[8]) / gc.theta[8];
  g[9] = 2.0 * (hqa - hqb) * M[9];
  g[10] = -(cL * M[10] - sL * M[11]);
  g[11] = -(sL * M[10] + cL * M[11]);
  g[12] = M[12];
  g[13] = -2.0 / gc.theta[13] * (sqa * M[13] + sqb * M[15]);
  g[14] = M[14];
  g[15] = (sqa * M[13] - sqb * M[15]) / gc.theta[15];
  g[16] = 2.0 * (sqa - sqb) * M[16];
}

// The subsample offsets (k + 1/2)/N - 1/2 by a multiply with 1/N (to a float32
// rounding of the quotient: the gradient needs the abscissae to float32
// accuracy, not bit for bit those of the render).
template <int MODE, int SER>
__device__ __forceinline__ void pixel_grad(const PointConst& c, const GradUniform& U, int N, const PixelGeom& g,
                                           float (&acc)[NPAR]) {
  const float iN = 1.0f / (float)N;
  for (int ky = 0; ky < N; ++ky) {
    const float y = fmaf(g.uy + fmaf((float)ky + 0.5f, iN, -0.5f), g.d, g.cy);
    for (int kx = 0; kx < N; ++kx) {
      const float x = fmaf(g.ux + fmaf((float)kx + 0.5f, iN, -0.5f), g.d, g.cx);
      subsample_grad<MODE, false, SER>(c, U, x, y, acc);
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
// The series-or-closed-form choice of the SIE's d/ds is per point, taken once
// outside the subsample loops. Six waves per SIMD (at most 80 VGPRs, no
// spills) hide the latency of the transcendental chains better than five.
// (A kernel per N with the midpoint loops unrolled issued 7 % fewer
// instructions but needed 96 VGPRs, and five waves ran 6 % slower.)
__global__ __launch_bounds__(RENDER_BLOCK, 6) void grad_kernel(WorkArgs w, const PointConst* __restrict__ pcs,
                                                             const GradConst* __restrict__ gcs,
                                                             const float* __restrict__ G,
                                                             const int* __restrict__ gpbase,
                                                             float2* __restrict__ gpart) {
  static_assert(RENDER_BLOCK == 256, "the block sums read four entries per lane");
  __shared__ float part[NPAR][RENDER_BLOCK];
  int point, tile;
  resolve(w, point, tile);
  const SysDesc sd = w.sys_table ? w.sys_table[w.point_sys ? w.point_sys[point] : 0] : w.single;
  const int64_t loff = w.point_loff ? w.point_loff[point] : 0;
  const PointConst& c = pcs[point];
  const GradConst& gc = gcs[point];
  const GradUniform& U = gc.u;

  const int base = gpbase ? gpbase[point] : 0;
  const int n_sup = grad_support_count(sd);
  if (tile * RENDER_BLOCK >= n_sup) {   // past the support's last pixel: zero sums
    if ((int)threadIdx.x < NPAR) gpart[(size_t)(base + tile) * NPAR + threadIdx.x] = make_float2(0.0f, 0.0f);
    return;
  }
  float acc[NPAR];
#pragma unroll
  for (int k = 0; k < NPAR; ++k) acc[k] = 0.0f;
  const int unit = tile * RENDER_BLOCK + (int)threadIdx.x;
  const int64_t goff = w.point_goff ? w.point_goff[point] : loff;   // the composite model's g
  if (unit < n_sup) {
    const int pix = grad_support_pixel(sd, unit);
    const float gp = G[goff + pix];
    if (gp != 0.0f) {   // pixels outside the reach of any weighted residual add nothing
      const int r = row_of(sd, pix);
      const int col = pix - r * sd.W;
      PixelGeom geo;
      geo.ux = (float)col - 0.5f * (float)(sd.W - 1);
      geo.uy = (float)r - 0.5f * (float)(sd.H - 1);
      geo.d = sd.d;
      geo.cx = sd.cx;
      geo.cy = sd.cy;
      if (sd.rule == 0) {
        const bool ser = U.s < S_SERIES;
        switch (c.sie_mode) {
          case 0: pixel_grad<0, 1>(c, U, sd.N, geo, acc); break;   // q = 1: s = 0
          case 1:
            if (ser) pixel_grad<1, 1>(c, U, sd.N, geo, acc);
            else pixel_grad<1, 0>(c, U, sd.N, geo, acc);
            break;
          default:
            if (ser) pixel_grad<2, 1>(c, U, sd.N, geo, acc);
            else pixel_grad<2, 0>(c, U, sd.N, geo, acc);
            break;
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
  // block sums of the 17 moments: the threads' float32 sums go to LDS, wave w
  // adds moments w, w + 4, ... in float64 (four entries per lane, then a fixed
  // shuffle tree; float64 holds the sum of 256 float32 values exactly enough
  // that no cancellation is lost), stored as a float32 pair hi + lo
#pragma unroll
  for (int k = 0; k < NPAR; ++k) part[k][threadIdx.x] = acc[k];
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int k = wid; k < NPAR; k += RENDER_BLOCK / 64) {
    double v = ((double)part[k][lane] + (double)part[k][lane + 64]) +
               ((double)part[k][lane + 128] + (double)part[k][lane + 192]);
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) {
      const float hi = (float)v;
      gpart[(size_t)(base + tile) * NPAR + k] = make_float2(hi, (float)(v - (double)hi));
    }
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
  const int r = row_of(sd, pix);
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
    const int64_t goff = w.point_goff ? w.point_goff[e.point] : loff;   // the composite model's g
    const PointConst& c = pcs[e.point];
    const GradConst& gc = gcs[e.point];
    const GradUniform& U = gc.u;
    const int lpix = mine ? unit_pixel(sd, e.unit0 + lane, e.ppt) + e.half : 0;   // this lane's pixel
    const PixelGeom geo = gcusp_geom(sd, lpix);
    // the render constants the forward render used for this lane's pixel
    const int prow = row_of(sd, lpix);
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
          const float wg = (float)sd.wgt * G[goff + qpix];
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

// One block per point: wave w sums the moments k = w, w + 4, ... over the
// point's render tiles (hi + lo, float64, lanes striding over the tiles, then
// a fixed shuffle tree) and adds the cusp correction.
constexpr int FGRAD_THREADS = 256;

// With magnitudes, slots 5 and 12 of the sums hold d log L / d I_e and slots
// 6, 7 and 13, 14 the derivatives at fixed I_e; the chain rule through
// I_e(m, R_e, n) gives d/dm = g_I I_e dlnI/dm and adds g_I I_e dlnI/dR_e and
// g_I I_e dlnI/dn to the radius and index entries. With an image-plane source
// position, slots 10 and 11 hold d log L / d beta; the chain rule through
// beta(x_I, y_I, theta_E, q_L, phi_L, gamma, phi_gamma) gives d/dx_I, d/dy_I and
// adds g_beta . d beta / d theta_k to the five lens entries.
__global__ __launch_bounds__(FGRAD_THREADS) void finalize_grad_kernel(
    const float2* __restrict__ gpart, const int* __restrict__ gpbase, int ntiles, const double* __restrict__ corr,
    const PointConst* __restrict__ pcs, const GradConst* __restrict__ gcs, float* __restrict__ grad, int point_base) {
  __shared__ double M[NPAR];
  const int p = point_base + (int)blockIdx.x;
  const int base = gpbase ? gpbase[p] : 0;
  const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
  for (int k = wv; k < NPAR; k += FGRAD_THREADS / 64) {
    double s = 0.0;
    for (int i = lane; i < ntiles; i += 64) {
      const float2 v = gpart[(size_t)(base + i) * NPAR + k];
      s += (double)v.x + (double)v.y;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) M[k] = s + (corr ? corr[(size_t)p * NPAR + k] : 0.0);
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double g[NPAR];
  const GradConst& gc = gcs[p];
  grad_from_moments(M, pcs[p], gc, g);
  if (gc.srcpos) {
    const float* J = gc.src_jac;
    const double gx = g[10], gy = g[11];
    for (int k = 0; k <= 4; ++k) g[k] += gx * (double)J[k + 2] + gy * (double)J[7 + k + 2];
    g[10] = gx * (double)J[0] + gy * (double)J[7];
    g[11] = gx * (double)J[1] + gy * (double)J[8];
  }
  if (gc.amp) {
    const double gIh = g[5], gIs = g[12];
    g[5] = gIh * (double)gc.amp_chain[0];
    g[6] += gIh * (double)gc.amp_chain[1];
    g[7] += gIh * (double)gc.amp_chain[2];
    g[12] = gIs * (double)gc.amp_chain[3];
    g[13] += gIs * (double)gc.amp_chain[4];
    g[14] += gIs * (double)gc.amp_chain[5];
  }
  for (int k = 0; k < NPAR; ++k) grad[(size_t)p * NPAR + k] = (float)g[k];
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
  const int nseg = border_segments(H, W);
  // the window, and with 21-wide tables also the four tables of a segment
  const size_t blds = (size_t)(border_lds_floats(ph, pw) + (pw == 21 ? 4 * ph * pw : 0)) * sizeof(float);
  // one grid row per point, at most 65535 rows per launch
  for (int p0 = 0; p0 < n_points; p0 += 65535) {
    const int np = n_points - p0 < 65535 ? n_points - p0 : 65535;
    if (pw == 21)
      hipLaunchKernelGGL(adj_border_kernel<21>, dim3((unsigned)nseg, np), dim3(BORDER_SEG * BORDER_SUB), blds, st, w,
                         R, G, p0);
    else
      hipLaunchKernelGGL(adj_border_kernel<0>, dim3((unsigned)nseg, np), dim3(BORDER_SEG * BORDER_SUB), blds, st, w,
                         R, G, p0);
    const hipError_t le = hipGetLastError();
    if (le != hipSuccess) return le;
  }
  return hipSuccess;
}

// The adjoint's support, rebuilt from the weights on every launch so that a
// plan stays right when the caller changes the weights in place. Row pass:
// any w > 0 within q = pw/2 columns (clamped to the row); it also marks the
// PSF tiles that hold a pixel with w > 0.
__global__ __launch_bounds__(256) void grad_support_rows_kernel(const SysDesc* __restrict__ sys) {
  const SysDesc& sd = sys[blockIdx.y];
  const int pix = (int)blockIdx.x * 256 + (int)threadIdx.x;
  if (!sd.gsup || pix >= sd.H * sd.W) return;
  const int r = row_of(sd, pix), c = pix - r * sd.W, q = sd.pw / 2;
  const float* wr = sd.weight + (size_t)r * sd.W;
  const int c1 = min(c + q, sd.W - 1);
  bool any = false;
  for (int cc = max(c - q, 0); cc <= c1; ++cc) any = any || wr[cc] > 0.0f;
  sd.gflags[pix] = any ? 1 : 0;
  if (sd.ptile_w && wr[c] > 0.0f) sd.ptile_w[(r / sd.TH) * sd.tiles_x + c / sd.TW] = 1;
}

// Column pass: any row-pass flag within p = ph/2 rows (clamped to the column).
__global__ __launch_bounds__(256) void grad_support_cols_kernel(const SysDesc* __restrict__ sys) {
  const SysDesc& sd = sys[blockIdx.y];
  const int npix = sd.H * sd.W;
  const int pix = (int)blockIdx.x * 256 + (int)threadIdx.x;
  if (!sd.gsup || pix >= npix) return;
  const int r = row_of(sd, pix), c = pix - r * sd.W, p = sd.ph / 2;
  const int r1 = min(r + p, sd.H - 1);
  bool any = false;
  for (int rr = max(r - p, 0); rr <= r1; ++rr) any = any || sd.gflags[(size_t)rr * sd.W + c] != 0;
  sd.gflags[npix + pix] = any ? 1 : 0;
}

// Compaction of the flags f[0 .. n) of units of `ppt` pixels (a unit is
// flagged if any of its pixels is) into out[], the first pixel of each flagged
// unit in order; returns their number to every thread. Each thread counts a
// chunk of consecutive units; the chunks' first slots come from a wave-level
// prefix sum (shuffles) and a scan of the 16 wave totals in LDS.
constexpr int GSUP_THREADS = 1024;
__device__ int compact_units(const unsigned char* f, int npix, int ppt, int* out, int* wsum) {
  const int n = npix / ppt;
  const int chunk = (n + GSUP_THREADS - 1) / GSUP_THREADS;
  const int t = (int)threadIdx.x, lane = t & 63, wv = t >> 6;
  const int b = min(t * chunk, n), e = min(b + chunk, n);
  auto flag = [&](int u) { return ppt == 1 ? f[u] != 0 : (f[2 * u] | f[2 * u + 1]) != 0; };
  int cnt = 0;
#pragma unroll 4
  for (int u = b; u < e; ++u) cnt += flag(u);
  int incl = cnt;   // inclusive prefix over the wave
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  if (t == 0) {   // exclusive prefix of the wave totals, and the total in wsum[16]
    int acc = 0;
    for (int k = 0; k < GSUP_THREADS / 64; ++k) {
      const int v = wsum[k];
      wsum[k] = acc;
      acc += v;
    }
    wsum[GSUP_THREADS / 64] = acc;
  }
  __syncthreads();
  int pos = wsum[wv] + incl - cnt;
  for (int u = b; u < e; ++u)
    if (flag(u)) out[pos++] = u * ppt;
  const int total = wsum[GSUP_THREADS / 64];
  __syncthreads();   // wsum[] is reused by the next call
  return total;
}

// One block per system: the support's pixels, and with uact its render units.
__global__ __launch_bounds__(GSUP_THREADS) void grad_support_compact_kernel(SysDesc* __restrict__ sys) {
  __shared__ int scan[GSUP_THREADS / 64 + 1];
  SysDesc& sd = sys[blockIdx.x];
  if (!sd.gsup) return;   // uniform over the block
  const int npix = sd.H * sd.W;
  const unsigned char* f = sd.gflags + npix;
  const int n = compact_units(f, npix, 1, sd.gsup, scan);
  if (threadIdx.x == 0) *sd.gsup_n = n;
  if (!sd.uact) return;
  const int nu = compact_units(f, npix, sd.uppt == 2 ? 2 : 1, sd.uact, scan);
  if (threadIdx.x == 0) sd.n_active = nu;
}

// Zeroes the unconvolved image of every point outside its system's support
// (one block per point): a gradient plan renders only the support, and the
// PSF stage, which multiplies w = 0 by its outputs there, must read finite
// values, not what an earlier launch left (a NaN point's image, or g).
__global__ __launch_bounds__(256) void grad_support_clear_kernel(WorkArgs w, float* __restrict__ L, int point_base) {
  const int point = point_base + (int)blockIdx.x;
  const SysDesc& sd = w.sys_table[w.point_sys ? w.point_sys[point] : 0];
  if (!sd.uact) return;
  const int npix = sd.H * sd.W;
  const unsigned char* need = sd.gflags + npix;
  float* img = L + w.point_loff[point];
  for (int pix = (int)threadIdx.x; pix < npix; pix += 256)
    if (!need[pix]) img[pix] = 0.0f;
}

hipError_t launch_grad_clear(const WorkArgs& w, float* L, int n_points, hipStream_t st) {
  for (int p0 = 0; p0 < n_points; p0 += 1 << 20) {   // at most 2^20 blocks per launch
    const int np = n_points - p0 < (1 << 20) ? n_points - p0 : (1 << 20);
    hipLaunchKernelGGL(grad_support_clear_kernel, dim3((unsigned)np), dim3(256), 0, st, w, L, p0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

__global__ __launch_bounds__(256) void grad_sky_kernel(const float* __restrict__ R, const int64_t* __restrict__ loff,
                                                        const int* __restrict__ point_sys,
                                                        const SysDesc* __restrict__ sys, int K,
                                                        float* __restrict__ grad_sky, int model_base) {
  __shared__ double part[256];
  const int m = model_base + (int)blockIdx.x;
  const int64_t p0 = (int64_t)m * K;
  const SysDesc& sd = sys[point_sys ? point_sys[p0] : 0];
  const int npix = sd.H * sd.W;
  const float* rho = R + loff[p0];
  double acc = 0.0;
  for (int i = (int)threadIdx.x; i < npix; i += 256) acc += (double)rho[i];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) grad_sky[m] = (float)(part[0] * (double)sd.d * (double)sd.d);
}

hipError_t launch_grad_sky(const float* R, const int64_t* loff, const int* point_sys, const SysDesc* sys, int K,
                           int n_models, float* grad_sky, hipStream_t st) {
  for (int m0 = 0; m0 < n_models; m0 += 1 << 20) {   // at most 2^20 blocks per launch
    const int nm = n_models - m0 < (1 << 20) ? n_models - m0 : (1 << 20);
    hipLaunchKernelGGL(grad_sky_kernel, dim3((unsigned)nm), dim3(256), 0, st, R, loff, point_sys, sys, K, grad_sky,
                       m0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_grad_support(SysDesc* sys, int n_sys, int max_pixels, hipStream_t st) {
  if (n_sys <= 0 || max_pixels <= 0) return hipSuccess;
  const dim3 grid((unsigned)((max_pixels + 255) / 256), (unsigned)n_sys);
  hipLaunchKernelGGL(grad_support_rows_kernel, grid, dim3(256), 0, st, sys);
  hipLaunchKernelGGL(grad_support_cols_kernel, grid, dim3(256), 0, st, sys);
  hipLaunchKernelGGL(grad_support_compact_kernel, dim3((unsigned)n_sys), dim3(GSUP_THREADS), 0, st, sys);
  return hipGetLastError();
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
                                const PointConst* pcs, const GradConst* gcs, float* grad, hipStream_t st) {
  if (n_points <= 0) return hipSuccess;
  // at most 2^20 blocks per launch (the grid stays far below 2^32 work-items)
  for (int p0 = 0; p0 < n_points; p0 += 1 << 20) {
    const int np = n_points - p0 < (1 << 20) ? n_points - p0 : (1 << 20);
    hipLaunchKernelGGL(finalize_grad_kernel, dim3((unsigned)np), dim3(FGRAD_THREADS), 0, st, gpart, gpbase, ntiles,
                       corr, pcs, gcs, grad, p0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace lensed
