// model.hip -- general models: several SIEs with free centres, an external
// shear, several Sersic components in the image or the source plane, a flat
// sky (the models of the paper's fits of real lenses, Sec. 5), and lenses on
// several planes (the multi-plane extension named in Sec. 6).
//
// Coordinates, deflections and radii are float64 (the float32 folding of the
// 17-parameter render does not carry over to an arbitrary number of
// components), and so are the SIE's atan and atanh, whose errors would move
// rays near a cuspy source centre. The Sersic profiles take their powers of
// two as an exact integer part and a float32 fraction (exp2_split,
// log2_split): errors of a few 1e-7 of each subsample's light that vary with
// the argument, at a fraction of the float64 library functions' cost. Each
// pixel is rounded once; the PSF and chi^2 stages are the common ones.
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

constexpr double LN2 = 0.693147180559945309417;

// 2^a for float64 a: the integer part exact (ldexp), the fraction in [0, 1)
// by the float32 hardware exp2 (relative error about 1e-7).
__device__ inline double exp2_split(double a) {
  a = fmax(a, -1100.0);
  const double k = floor(a);
  return ldexp((double)__builtin_amdgcn_exp2f((float)(a - k)), (int)k);
}

// log2 u for finite u > 0: the binary exponent exact, the mantissa in [1/2, 1)
// by the float32 hardware log2 (absolute error about 1e-7).
__device__ inline double log2_split(double u) {
  int k;
  const double f = frexp(u, &k);
  return (double)k + (double)__builtin_amdgcn_logf((float)f);
}

// Sersic component j (Eq. 22) at (px, py): the offset, rotation and radius in
// float64; the profile exp(-b ((R/R_e)^{1/n} - 1)) as powers of two, whose
// exponents are float64 and whose fractional parts go through the hardware
// float32 exp2 / log2 (per-subsample relative errors of a few 1e-7 that
// vary with the argument, against the float64 library functions' many
// instructions each).
__device__ inline double sersic_at(const ModelConst& m, int j, double px, double py) {
  const double* s = m.ser[j];
  const double dx = px - s[0], dy = py - s[1];
  const double xp = s[2] * dx + s[3] * dy, yp = s[2] * dy - s[3] * dx;
  const double R2 = s[4] * xp * xp + s[5] * yp * yp;
  // (R/R_e)^{1/n} = 2^(log2(R^2 / R_e^2) / (2n))
  const double t = R2 > 0.0 ? exp2_split(0.5 * s[7] * log2_split(R2 * s[6] * s[6])) : 0.0;
  return s[9] * exp2_split(s[8] * LOG2E * (1.0 - t));
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
  // render units are single pixels: the whole image, or in a gradient plan the
  // support of g (the only pixels the PSF outputs with w > 0 read)
  const int unit = tile * RENDER_BLOCK + (int)threadIdx.x;
  if (unit >= unit_count(sd, 1)) return;
  const int pix = unit_pixel(sd, unit, 1);
  const ModelConst& m = mcs[point];
  const int r = row_of(sd, pix), c = pix - r * sd.W;
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

// ---------------------------------------------------------------------------
// Adjoint of general models with one lens plane: d log L / d theta =
// sum_j g_j wgt sum_k w_k dI(x_jk)/d theta, g = A^T rho (the common adjoint PSF
// stage), the derivative of Eq. 17 through Eqs. 15, 14, 2, 1 and 22. The
// partials of I at a subsample come from forward-mode dual numbers in float64,
// one component per pass (an SIE, a Sersic, or the shear and the sky
// together; blockIdx.y is the pass), so that a thread keeps at most 7 sums:
//   SIE k        dI/dtheta_k = -G . d alpha_k/d theta_k  (x_c, y_c, theta_E, q, phi)
//   Sersic j     dS_j/d(x, y, I_e, R_e, n, q, phi) at x (foreground) or beta
//   shear, sky   G . d beta/d(gamma, phi_gamma), 1
// with G = sum over the lensed Sersics of grad S_j(beta).
// ---------------------------------------------------------------------------

// Value and M partial derivatives.
template <int M>
struct Dl {
  double v;
  double d[M];
};

template <int M>
__device__ inline Dl<M> dconst(double v) {
  Dl<M> r;
  r.v = v;
#pragma unroll
  for (int i = 0; i < M; ++i) r.d[i] = 0.0;
  return r;
}
template <int M>
__device__ inline Dl<M> dvar(double v, int k) {
  Dl<M> r = dconst<M>(v);
  r.d[k] = 1.0;
  return r;
}
// f(a) with f'(a) = fp
template <int M>
__device__ inline Dl<M> dchain(const Dl<M>& a, double f, double fp) {
  Dl<M> r;
  r.v = f;
#pragma unroll
  for (int i = 0; i < M; ++i) r.d[i] = fp * a.d[i];
  return r;
}
template <int M>
__device__ inline Dl<M> operator+(const Dl<M>& a, const Dl<M>& b) {
  Dl<M> r;
  r.v = a.v + b.v;
#pragma unroll
  for (int i = 0; i < M; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <int M>
__device__ inline Dl<M> operator-(const Dl<M>& a, const Dl<M>& b) {
  Dl<M> r;
  r.v = a.v - b.v;
#pragma unroll
  for (int i = 0; i < M; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <int M>
__device__ inline Dl<M> operator-(const Dl<M>& a) {
  return dchain(a, -a.v, -1.0);
}
template <int M>
__device__ inline Dl<M> operator*(const Dl<M>& a, const Dl<M>& b) {
  Dl<M> r;
  r.v = a.v * b.v;
#pragma unroll
  for (int i = 0; i < M; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <int M>
__device__ inline Dl<M> operator*(const Dl<M>& a, double b) {
  return dchain(a, a.v * b, b);
}
template <int M>
__device__ inline Dl<M> operator+(const Dl<M>& a, double b) {
  return dchain(a, a.v + b, 1.0);
}
template <int M>
__device__ inline Dl<M> operator/(const Dl<M>& a, const Dl<M>& b) {
  Dl<M> r;
  r.v = a.v / b.v;
  const double ib = 1.0 / b.v;
#pragma unroll
  for (int i = 0; i < M; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib;
  return r;
}
template <int M>
__device__ inline Dl<M> dsqrt(const Dl<M>& a) {
  const double s = sqrt(a.v);
  return dchain(a, s, 0.5 / s);
}
// exp and log of a Sersic argument, as in sersic_at (relative errors of a few
// 1e-7 in the value and the derivatives).
template <int M>
__device__ inline Dl<M> dexp(const Dl<M>& a) {
  const double e = exp2_split(a.v * LOG2E);
  return dchain(a, e, e);
}
template <int M>
__device__ inline Dl<M> dlog(const Dl<M>& a) {
  return dchain(a, log2_split(a.v) * LN2, 1.0 / a.v);
}
template <int M>
__device__ inline Dl<M> datan(const Dl<M>& a) {
  return dchain(a, atan(a.v), 1.0 / (1.0 + a.v * a.v));
}
template <int M>
__device__ inline Dl<M> datanh(const Dl<M>& a) {
  return dchain(a, atanh(a.v), 1.0 / (1.0 - a.v * a.v));
}

// atan(sqrt(s) u) / sqrt(s) (HYP false) or atanh(sqrt(s) u) / sqrt(s) (HYP
// true), s = 1 - q^2 >= 0: below SIE_SERIES_S by the series
// u sum_k (-+1)^k (s u^2)^k / (2k + 1), which also gives the round limit s = 0
// and its derivative in s. The SIE keeps |u| <= 1/q for the atan and |u| <= 1
// for the atanh, so s u^2 < 0.053 there and 15 terms reach 1e-19.
constexpr double SIE_SERIES_S = 0.05;

template <bool HYP, int M>
__device__ inline Dl<M> atan_over_root(const Dl<M>& s, const Dl<M>& u) {
  if (s.v < SIE_SERIES_S) {
    const Dl<M> z = s * u * u;
    constexpr int K = 14;
    Dl<M> p = dconst<M>((HYP || K % 2 == 0 ? 1.0 : -1.0) / (2 * K + 1));
    for (int k = K - 1; k >= 0; --k) p = p * z + (HYP || k % 2 == 0 ? 1.0 : -1.0) / (2 * k + 1);
    return u * p;
  }
  const Dl<M> r = dsqrt(s);
  return (HYP ? datanh(r * u) : datan(r * u)) / r;
}

// Deflection of SIE k at (x, y) with its derivatives in (x_c, y_c, theta_E, q,
// phi): alpha' = theta_E sqrt(q) (atan(q' u)/q', atanh(q' v)/q'), u = x'/psi,
// v = y'/psi, rotated back by phi (the same deflection as add_sie).
__device__ inline void sie_deflection_d(const ModelConst& m, int k, double x, double y, Dl<5>& ax, Dl<5>& ay) {
  const double* s = m.sie[k];
  Dl<5> dx = dconst<5>(x - s[0]), dy = dconst<5>(y - s[1]);
  dx.d[0] = -1.0;
  dy.d[1] = -1.0;
  Dl<5> c = dconst<5>(s[2]), sn = dconst<5>(s[3]);
  c.d[4] = -s[3];
  sn.d[4] = s[2];
  const Dl<5> te = dvar<5>(s[7], 2), q = dvar<5>(s[8], 3);
  const Dl<5> xp = c * dx + sn * dy, yp = c * dy - sn * dx;
  const Dl<5> psi2 = q * q * xp * xp + yp * yp;
  if (!(psi2.v > 0.0)) {   // the centre itself: no deflection
    ax = ay = dconst<5>(0.0);
    return;
  }
  const Dl<5> psi = dsqrt(psi2);
  const Dl<5> ss = -(q * q) + 1.0;
  const Dl<5> f = te * dsqrt(q);
  const Dl<5> a1 = f * atan_over_root<false>(ss, xp / psi), a2 = f * atan_over_root<true>(ss, yp / psi);
  ax = c * a1 - sn * a2;
  ay = sn * a1 + c * a2;
}

// Sersic j at (px, py) and its gradient in (px, py).
__device__ inline double sersic_and_grad(const ModelConst& m, int j, double px, double py, double& gx, double& gy) {
  const double* s = m.ser[j];
  const double dx = px - s[0], dy = py - s[1];
  const double xp = s[2] * dx + s[3] * dy, yp = s[2] * dy - s[3] * dx;
  const double R2 = s[4] * xp * xp + s[5] * yp * yp;
  if (!(R2 > 0.0)) {
    gx = gy = 0.0;
    return s[9] * exp2_split(s[8] * LOG2E);
  }
  const double t = exp2_split(0.5 * s[7] * log2_split(R2 * s[6] * s[6]));
  const double S = s[9] * exp2_split(s[8] * LOG2E * (1.0 - t));
  const double D = -s[8] * S * t * 0.5 * s[7] / R2;   // dS/dR^2
  const double ex = 2.0 * s[4] * xp, ey = 2.0 * s[5] * yp;   // dR^2/dx', dR^2/dy'
  gx = D * (ex * s[2] - ey * s[3]);
  gy = D * (ex * s[3] + ey * s[2]);
  return S;
}

// Sersic j at (px, py) with its derivatives in (x, y, I_e, R_e, n, q, phi).
__device__ inline Dl<7> sersic_d(const ModelConst& m, int j, double px, double py) {
  const double* s = m.ser[j];
  Dl<7> dx = dconst<7>(px - s[0]), dy = dconst<7>(py - s[1]);
  dx.d[0] = -1.0;
  dy.d[1] = -1.0;
  const Dl<7> Ie = dvar<7>(s[9], 2), Re = dvar<7>(1.0 / s[6], 3), n = dvar<7>(1.0 / s[7], 4), q = dvar<7>(s[4], 5);
  Dl<7> c = dconst<7>(s[2]), sn = dconst<7>(s[3]), b = dconst<7>(s[8]);
  c.d[6] = -s[3];
  sn.d[6] = s[2];
  b.d[4] = s[10];
  const Dl<7> xp = c * dx + sn * dy, yp = c * dy - sn * dx;
  const Dl<7> R2 = q * xp * xp + yp * yp / q;
  const Dl<7> t = R2.v > 0.0 ? dexp(dlog(R2 / (Re * Re)) * (dconst<7>(0.5) / n)) : dconst<7>(0.0);
  return Ie * dexp(-(b * (t + -1.0)));
}

// ---- Several lens planes: the ray's positions in dual numbers --------------
// With lenses on several planes a deflector's parameters move the rays of every
// later plane, so the pass carries derivatives through the whole chain: the
// position on plane j is x - sum_{i<j} beta_ij alpha_i(x_i) in dual numbers
// whose variables are the pass's own parameters (those of SIE comp, of Sersic
// comp, or the shear), and every deflector and Sersic is evaluated at dual
// positions.

// SIE k at the dual position (x, y); own: its (x_c, y_c, theta_E, q, phi) are
// the variables 0..4.
__device__ inline void sie_alpha_dual(const ModelConst& m, int k, const Dl<7>& x, const Dl<7>& y, bool own,
                                      Dl<7>& ax, Dl<7>& ay) {
  const double* s = m.sie[k];
  Dl<7> xc = dconst<7>(s[0]), yc = dconst<7>(s[1]), c = dconst<7>(s[2]), sn = dconst<7>(s[3]);
  Dl<7> te = dconst<7>(s[7]), q = dconst<7>(s[8]);
  if (own) {
    xc.d[0] = 1.0;
    yc.d[1] = 1.0;
    te.d[2] = 1.0;
    q.d[3] = 1.0;
    c.d[4] = -s[3];
    sn.d[4] = s[2];
  }
  const Dl<7> dx = x - xc, dy = y - yc;
  const Dl<7> xp = c * dx + sn * dy, yp = c * dy - sn * dx;
  const Dl<7> psi2 = q * q * xp * xp + yp * yp;
  if (!(psi2.v > 0.0)) {   // the centre itself: no deflection
    ax = ay = dconst<7>(0.0);
    return;
  }
  const Dl<7> psi = dsqrt(psi2);
  const Dl<7> ss = -(q * q) + 1.0;
  const Dl<7> f = te * dsqrt(q);
  const Dl<7> a1 = f * atan_over_root<false>(ss, xp / psi), a2 = f * atan_over_root<true>(ss, yp / psi);
  ax = c * a1 - sn * a2;
  ay = sn * a1 + c * a2;
}

// The external shear's deflection at (x, y) added to (ax, ay); own: (gamma,
// phi_gamma) are the variables 0, 1.
__device__ inline void shear_alpha_dual(const ModelConst& m, const Dl<7>& x, const Dl<7>& y, bool own, Dl<7>& ax,
                                        Dl<7>& ay) {
  Dl<7> gam = dconst<7>(m.gam), c2 = dconst<7>(m.c2g), s2 = dconst<7>(m.s2g);
  if (own) {
    gam.d[0] = 1.0;
    c2.d[1] = -2.0 * m.s2g;
    s2.d[1] = 2.0 * m.c2g;
  }
  const Dl<7> g1 = gam * c2, g2 = gam * s2;
  ax = ax + g1 * x + g2 * y;
  ay = ay + g2 * x - g1 * y;
}

// Sersic j at the dual position (px, py); own: its (x, y, I_e, R_e, n, q, phi)
// are the variables 0..6.
__device__ inline Dl<7> sersic_at_dual(const ModelConst& m, int j, const Dl<7>& px, const Dl<7>& py,
                                               bool own) {
  const double* s = m.ser[j];
  Dl<7> x0 = dconst<7>(s[0]), y0 = dconst<7>(s[1]), Ie = dconst<7>(s[9]), Re = dconst<7>(1.0 / s[6]);
  Dl<7> n = dconst<7>(1.0 / s[7]), q = dconst<7>(s[4]), c = dconst<7>(s[2]), sn = dconst<7>(s[3]);
  Dl<7> b = dconst<7>(s[8]);
  if (own) {
    x0.d[0] = 1.0;
    y0.d[1] = 1.0;
    Ie.d[2] = 1.0;
    Re.d[3] = 1.0;
    n.d[4] = 1.0;
    b.d[4] = s[10];
    q.d[5] = 1.0;
    c.d[6] = -s[3];
    sn.d[6] = s[2];
  }
  const Dl<7> dx = px - x0, dy = py - y0;
  const Dl<7> xp = c * dx + sn * dy, yp = c * dy - sn * dx;
  const Dl<7> R2 = q * xp * xp + yp * yp / q;
  const Dl<7> t = R2.v > 0.0 ? dexp(dlog(R2 / (Re * Re)) * (dconst<7>(0.5) / n)) : dconst<7>(0.0);
  return Ie * dexp(-(b * (t + -1.0)));
}

// I at the subsample (x, y) of a model with spec.n_planes > 1 (the sky left
// out), with its derivatives in the pass's parameters (kind 0: SIE comp, 1:
// Sersic comp, 2: the shear).
__device__ Dl<7> planes_dual(const ModelConst& m, const ModelSpec& spec, double x, double y, int kind, int comp) {
  const int P = spec.n_planes;
  Dl<7> ax[MAX_PLANES], ay[MAX_PLANES];
  Dl<7> I = dconst<7>(0.0);
  for (int j = 0; j <= P; ++j) {
    Dl<7> px = dconst<7>(x), py = dconst<7>(y);
    for (int i = 0; i < j; ++i) {
      const double b = j == P ? 1.0 : spec.beta[i][j];
      px = px - ax[i] * b;
      py = py - ay[i] * b;
    }
    for (int k = 0; k < m.n_sersic; ++k)
      if (m.plane[k] == j) I = I + sersic_at_dual(m, k, px, py, kind == 1 && comp == k);
    if (j < P) {
      Dl<7> dx = dconst<7>(0.0), dy = dconst<7>(0.0);
      for (int k = 0; k < m.n_sie; ++k)
        if (spec.sie_plane[k] == j) {
          Dl<7> a, b;
          sie_alpha_dual(m, k, px, py, kind == 0 && comp == k, a, b);
          dx = dx + a;
          dy = dy + b;
        }
      if (j == 0 && spec.shear) shear_alpha_dual(m, px, py, kind == 2, dx, dy);
      ax[j] = dx;
      ay[j] = dy;
    }
  }
  return I;
}

// beta at (x, y) (every SIE, the shear), with SIE `skip` left out, and G.
__device__ inline void source_side(const ModelConst& m, double x, double y, int skip, double& ax, double& ay) {
  ax = m.g1 * x + m.g2 * y;
  ay = m.g2 * x - m.g1 * y;
  for (int k = 0; k < m.n_sie; ++k)
    if (k != skip) add_sie(m, k, x, y, ax, ay);
}
__device__ inline void lensed_gradient(const ModelConst& m, double bx, double by, double& Gx, double& Gy) {
  Gx = Gy = 0.0;
  for (int j = 0; j < m.n_sersic; ++j)
    if (m.plane[j]) {
      double gx, gy;
      sersic_and_grad(m, j, bx, by, gx, gy);
      Gx += gx;
      Gy += gy;
    }
}

// PLANES: the model has several lens planes (planes_dual per subsample).
template <bool PLANES>
__global__ __launch_bounds__(RENDER_BLOCK) void model_grad_kernel(WorkArgs w, ModelSpec spec,
                                                                   const ModelConst* __restrict__ mcs,
                                                                   const float* __restrict__ G,
                                                                   const int* __restrict__ gpbase,
                                                                   double* __restrict__ gpart, int P) {
  __shared__ double red[RENDER_BLOCK / 64][7];
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
  const ModelConst& m = mcs[point];
  // the pass: SIE k, Sersic j, or the shear and the sky
  const int pass = (int)blockIdx.y;
  const int kind = pass < spec.n_sie ? 0 : (pass < spec.n_sie + spec.n_sersic ? 1 : 2);
  const int comp = kind == 0 ? pass : pass - spec.n_sie;
  const int off = kind == 0 ? 5 * comp : (kind == 1 ? 5 * spec.n_sie + (spec.shear ? 2 : 0) + 7 * comp : 5 * spec.n_sie);
  const int npar = kind == 0 ? 5 : (kind == 1 ? 7 : (spec.shear ? 2 : 0) + (spec.sky ? 1 : 0));
  const int n_sup = grad_support_count(sd);
  if (tile * RENDER_BLOCK >= n_sup) {   // past the support's last pixel: zero sums
    if ((int)threadIdx.x < npar) {
      const int i = threadIdx.x;
      const int slot = kind == 2 && spec.sky && i == npar - 1 ? P - 1 : off + i;
      gpart[(size_t)(gpbase[point] + tile) * P + slot] = 0.0;
    }
    return;
  }
  double acc[7];
#pragma unroll
  for (int i = 0; i < 7; ++i) acc[i] = 0.0;
  const int unit = tile * RENDER_BLOCK + (int)threadIdx.x;
  const int pix = unit < n_sup ? grad_support_pixel(sd, unit) : 0;
  const float gp = unit < n_sup ? G[loff + pix] : 0.0f;
  if (gp != 0.0f) {   // pixels outside the reach of any weighted residual add nothing
    const int r = row_of(sd, pix), c = pix - r * sd.W;
    const double ux = (double)c - 0.5 * (double)(sd.W - 1), uy = (double)r - 0.5 * (double)(sd.H - 1);
    const double d = sd.d, cx = sd.cx, cy = sd.cy;
    const int N = sd.N;
    const GkRule* R = sd.rule > 0 ? &kGkRules[sd.rule - 1] : nullptr;
    for (int ky = 0; ky < N; ++ky) {
      const double oy = R ? R->xd[ky] : ((double)ky + 0.5) / N - 0.5;
      const double y = cy + (uy + oy) * d;
      for (int kx = 0; kx < N; ++kx) {
        const double ox = R ? R->xd[kx] : ((double)kx + 0.5) / N - 0.5;
        const double wq = R ? (double)R->w[kx] * (double)R->w[ky] : 1.0;
        const double x = cx + (ux + ox) * d;
        if (PLANES) {
          if (kind < 2 || spec.shear) {
            const Dl<7> I = planes_dual(m, spec, x, y, kind, comp);
            const int nd = kind == 0 ? 5 : (kind == 1 ? 7 : 2);
            for (int i = 0; i < nd; ++i) acc[i] += wq * I.d[i];
          }
          if (kind == 2 && spec.sky) acc[spec.shear ? 2 : 0] += wq;
        } else if (kind == 0) {
          double ax, ay, Gx, Gy;
          source_side(m, x, y, comp, ax, ay);
          Dl<5> akx, aky;
          sie_deflection_d(m, comp, x, y, akx, aky);
          lensed_gradient(m, x - ax - akx.v, y - ay - aky.v, Gx, Gy);
#pragma unroll
          for (int i = 0; i < 5; ++i) acc[i] -= wq * (Gx * akx.d[i] + Gy * aky.d[i]);
        } else if (kind == 1) {
          double px = x, py = y;
          if (m.plane[comp]) {
            double ax, ay;
            source_side(m, x, y, -1, ax, ay);
            px = x - ax;
            py = y - ay;
          }
          const Dl<7> S = sersic_d(m, comp, px, py);
#pragma unroll
          for (int i = 0; i < 7; ++i) acc[i] += wq * S.d[i];
        } else {
          int i = 0;
          if (spec.shear) {
            double ax, ay, Gx, Gy;
            source_side(m, x, y, -1, ax, ay);
            lensed_gradient(m, x - ax, y - ay, Gx, Gy);
            const double c2 = m.c2g, s2 = m.s2g;
            // beta = x - alpha_SIE - Gamma x, Gamma = gamma [[c2, s2], [s2, -c2]]
            acc[0] -= wq * (Gx * (c2 * x + s2 * y) + Gy * (s2 * x - c2 * y));
            acc[1] -= wq * 2.0 * m.gam * (Gx * (c2 * y - s2 * x) + Gy * (c2 * x + s2 * y));
            i = 2;
          }
          if (spec.sky) acc[i] += wq;
        }
      }
    }
    const double scale = (double)gp * sd.wgt;
#pragma unroll
    for (int i = 0; i < 7; ++i) acc[i] *= scale;
  }
  // block sums in float64, in a fixed order
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    double v = acc[i];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane == 0) red[wid][i] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < npar) {
    const int i = threadIdx.x;
    double v = red[0][i];
    for (int k = 1; k < RENDER_BLOCK / 64; ++k) v += red[k][i];
    // the sky is the model's last parameter; the other slots of a pass are consecutive
    const int slot = kind == 2 && spec.sky && i == npar - 1 ? P - 1 : off + i;
    gpart[(size_t)(gpbase[point] + tile) * P + slot] = v;
  }
}

// grad[p][k] = sum over the point's render tiles, float64, rounded once.
__global__ __launch_bounds__(64) void model_finalize_grad_kernel(const double* __restrict__ gpart,
                                                                  const int* __restrict__ gpbase, int ntiles, int P,
                                                                  float* __restrict__ grad, int point_base) {
  const int p = point_base + (int)blockIdx.x;
  const int base = gpbase[p];
  for (int k = threadIdx.x; k < P; k += blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < ntiles; ++i) s += gpart[(size_t)(base + i) * P + k];
    grad[(size_t)p * P + k] = (float)s;
  }
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

hipError_t launch_model_grad(const WorkArgs& w, const ModelSpec& spec, const ModelConst* mcs, const float* G,
                            const int* gpbase, double* gpart, int P, int n_blocks, hipStream_t stream) {
  if (n_blocks <= 0) return hipSuccess;
  const int passes = spec.n_sie + spec.n_sersic + ((spec.shear || spec.sky) ? 1 : 0);
  return for_item_parts(w, n_blocks, [&](const WorkArgs& part, int n) {
    if (spec.n_planes > 1)
      hipLaunchKernelGGL(model_grad_kernel<true>, dim3(n, passes), dim3(RENDER_BLOCK), 0, stream, part, spec, mcs, G,
                         gpbase, gpart, P);
    else
      hipLaunchKernelGGL(model_grad_kernel<false>, dim3(n, passes), dim3(RENDER_BLOCK), 0, stream, part, spec, mcs, G,
                         gpbase, gpart, P);
    return hipGetLastError();
  });
}

hipError_t launch_model_finalize_grad(const double* gpart, const int* gpbase, int ntiles, int P, int n_points,
                                      float* grad, hipStream_t stream) {
  for (int p0 = 0; p0 < n_points; p0 += 1 << 20) {
    const int np = n_points - p0 < (1 << 20) ? n_points - p0 : (1 << 20);
    hipLaunchKernelGGL(model_finalize_grad_kernel, dim3((unsigned)np), dim3(64), 0, stream, gpart, gpbase, ntiles, P,
                       grad, p0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace lensed
