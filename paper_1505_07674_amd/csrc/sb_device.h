// sb_device.h -- surface brightness of the image plane at one subsample, float32.
//
// Lens equation beta = x - alpha(x) (Sec. 2.1, Eq. 1) through a singular
// isothermal ellipsoid (Kormann et al. 1994, as used in Sec. 4) and an external
// shear; I(x) = I_lens(x) + I_source(beta) (Eq. 2) with elliptical Sersic
// profiles (Sec. 4.1, Eqs. 22-23).
//
// Everything is written in base 2 for the hardware v_exp_f32 / v_log_f32:
//   Sersic   I = I_e exp(-b [(R/R_e)^{1/n} - 1]) = I_e 2^{B (1 - t)},
//            t = 2^{log2(R^2/R_e^2) / (2n)},  B = b log2(e)
//   SIE      alpha'_x = k atan(u),  alpha'_y = k atanh(v),  u = q' x'/psi,  v = q' y'/psi,
//            k = theta_E sqrt(q)/q',  psi = sqrt(q^2 x'^2 + y'^2),  r = sqrt(x'^2 + y'^2)
// Bounds: |u| <= q'/q and |v| <= q'. For q' <= 1/2 both are evaluated by minimax
// polynomials fitted on those ranges. Otherwise |u| may exceed 1, and
//   atan(u)  = 2 atan(q' x' / (psi + r))          (|argument| <= sqrt((1-q)/(1+q)) <= 1)
//   atanh(v) = sign(y') ln((psi + q'|y'|) / (q r))   (no cancellation for any q)
// are used instead. At psi = 0 the deflection is zero.
#pragma once

#include "internal.h"
#include "sie_poly.h"

namespace lensed {

__device__ __forceinline__ float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float hw_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

template <int DEG>
__device__ __forceinline__ float horner(const float (&c)[DEG + 1], float s) {
  float p = c[DEG];
#pragma unroll
  for (int k = DEG - 1; k >= 0; --k) p = fmaf(p, s, c[k]);
  return p;
}

__device__ __forceinline__ float atan_small(float u) {
  return u * horner<ATAN_SMALL_POLY_DEGREE>(ATAN_SMALL_POLY, u * u);
}
__device__ __forceinline__ float atan_unit(float u) { return u * horner<ATAN_UNIT_POLY_DEGREE>(ATAN_UNIT_POLY, u * u); }
__device__ __forceinline__ float atanh_poly(float v) { return v * horner<ATANH_POLY_DEGREE>(ATANH_POLY, v * v); }

// Source-plane position of image-plane point (x, y).
template <int MODE>
__device__ __forceinline__ void lens_map(const PointConst& c, float x, float y, float& bx, float& by) {
  if (MODE == 0) {
    const float r2 = fmaf(x, x, y * y);
    const float ir = r2 > 0.0f ? hw_rsq(r2) : 0.0f;
    const float s = c.kc * ir;
    bx = fmaf(c.m11, x, fmaf(c.m12, y, -s * x));
    by = fmaf(c.m12, x, fmaf(c.m22, y, -s * y));
  } else {
    const float xp = fmaf(c.cL, x, c.sL * y);
    const float yp = fmaf(c.cL, y, -c.sL * x);
    const float yp2 = yp * yp;
    const float psi2 = fmaf(c.q2 * xp, xp, yp2);
    const float ip = psi2 > 0.0f ? hw_rsq(psi2) : 0.0f;
    float At, Ah;
    if (MODE == 1) {
      const float tq = c.qp * ip;
      At = atan_small(tq * xp);
      Ah = atanh_poly(tq * yp);
    } else {
      const float r2 = fmaf(xp, xp, yp2);
      const float ir = hw_rsq(r2);
      const float psi = psi2 * ip;
      const float r = r2 * ir;
      At = 2.0f * atan_unit(c.qp * xp * hw_rcp(psi + r));
      const float num = fmaf(c.qp, fabsf(yp), psi);
      const float l = LN2F * hw_log2(num * ir * c.iq);
      At = psi2 > 0.0f ? At : 0.0f;
      Ah = psi2 > 0.0f ? copysignf(l, yp) : 0.0f;
    }
    const float ax = fmaf(c.kc, At, -c.ks * Ah);
    const float ay = fmaf(c.ks, At, c.kc * Ah);
    bx = fmaf(c.m11, x, fmaf(c.m12, y, -ax));
    by = fmaf(c.m12, x, fmaf(c.m22, y, -ay));
  }
}

// Elliptical Sersic profile in two steps: the scaled squared radius
// R^2/R_e^2 = qa x'^2 + qb y'^2 (rotation (cs, sn), qa = q/R_e^2, qb = 1/(q R_e^2)),
// then I = I_e 2^{B (1 - t)} with t = (R^2/R_e^2)^{e}, e = 1/(2n), B = b_n log2(e).
__device__ __forceinline__ float sersic_r2(float dx, float dy, float cs, float sn, float qa, float qb) {
  const float xp = fmaf(cs, dx, sn * dy);
  const float yp = fmaf(cs, dy, -sn * dx);
  return fmaf(qa * xp, xp, qb * yp * yp);
}
__device__ __forceinline__ float sersic_from_r2(float R2, float e, float B, float Ie) {
  const float t = hw_exp2(e * hw_log2(R2));
  return Ie * hw_exp2(fmaf(-B, t, B));
}

// Midpoint offset of subsample k of N, in pixel units: (k + 1/2)/N - 1/2.
template <int N>
__device__ __forceinline__ constexpr float sub_offset(int k) {
  return (float(k) + 0.5f) / float(N) - 0.5f;
}
__device__ __forceinline__ float sub_offset_rt(int k, int N) { return (float(k) + 0.5f) / float(N) - 0.5f; }

// Where the pixel's subsamples sit: centre (ux, uy) in pixels from the grid
// centre (exact half-integers), pixel scale d, grid centre (cx, cy).
struct PixelGeom {
  float ux, uy, d, cx, cy;
};

// Float64 re-tracing of one subsample: exact abscissa (as the rule defines it),
// SIE + shear lens equation in float64, offset from the source centre.
__device__ __forceinline__ void source_offset_f64(const PointConst64& e, const PixelGeom& g, int kx, int ky, int N,
                                                  float& dx, float& dy) {
  const double x = (double)g.cx + ((double)g.ux + (((double)kx + 0.5) / N - 0.5)) * (double)g.d;
  const double y = (double)g.cy + ((double)g.uy + (((double)ky + 0.5) / N - 0.5)) * (double)g.d;
  double ax = 0.0, ay = 0.0;
  if (e.mode == 0) {
    const double r = sqrt(x * x + y * y);
    if (r > 0.0) {
      ax = e.te * x / r;
      ay = e.te * y / r;
    }
  } else {
    const double xp = e.cL * x + e.sL * y, yp = -e.sL * x + e.cL * y;
    const double psi = sqrt(e.q2 * xp * xp + yp * yp);
    if (psi > 0.0) {
      const double a1 = e.k * atan(e.qp * xp / psi), a2 = e.k * atanh(e.qp * yp / psi);
      ax = e.cL * a1 - e.sL * a2;
      ay = e.sL * a1 + e.cL * a2;
    }
  }
  dx = (float)(e.m11 * x + e.m12 * y - ax - e.sx0);
  dy = (float)(e.m12 * x + e.m22 * y - ay - e.sy0);
}

// Scaled squared source radius of subsample (x, y), float32 path.
template <int MODE>
__device__ __forceinline__ float source_r2(const PointConst& c, float x, float y) {
  float bx, by;
  lens_map<MODE>(c, x, y, bx, by);
  return sersic_r2(bx - c.sx0, by - c.sy0, c.sc, c.ss, c.sqa, c.sqb);
}

// Surface brightness at one subsample; `cusp` is raised when the float32 source
// radius falls inside the cusp zone, where a correction kernel later replaces
// this subsample's source light by its float64 re-traced value.
template <int MODE>
__device__ __forceinline__ float surface_brightness(const PointConst& c, float x, float y, bool& cusp) {
  const float Ih = sersic_from_r2(sersic_r2(x, y, c.hc, c.hs, c.hqa, c.hqb), c.he, c.hB, c.hI);
  const float sR2 = source_r2<MODE>(c, x, y);
  cusp = cusp || (sR2 < c.cusp_r2);
  return Ih + sersic_from_r2(sR2, c.se, c.sB, c.sI);
}

// Sum of the surface brightness over the N x N midpoint abscissae of a pixel.
template <int N, int MODE>
__device__ __forceinline__ float pixel_sum(const PointConst& c, const PixelGeom& g, bool& cusp) {
  float acc = 0.0f;
#pragma unroll
  for (int ky = 0; ky < N; ++ky) {
    const float y = fmaf(g.uy + sub_offset<N>(ky), g.d, g.cy);
#pragma unroll
    for (int kx = 0; kx < N; ++kx) {
      const float x = fmaf(g.ux + sub_offset<N>(kx), g.d, g.cx);
      acc += surface_brightness<MODE>(c, x, y, cusp);
    }
  }
  return acc;
}

template <int MODE>
__device__ __forceinline__ float pixel_sum_rt(const PointConst& c, int N, const PixelGeom& g, bool& cusp) {
  float acc = 0.0f;
  for (int ky = 0; ky < N; ++ky) {
    const float y = fmaf(g.uy + sub_offset_rt(ky, N), g.d, g.cy);
    for (int kx = 0; kx < N; ++kx) {
      const float x = fmaf(g.ux + sub_offset_rt(kx, N), g.d, g.cx);
      acc += surface_brightness<MODE>(c, x, y, cusp);
    }
  }
  return acc;
}

// Correction for one flagged pixel: for every subsample in the cusp zone, the
// source light at the float64 re-traced offset minus its float32 value.
template <int MODE>
__device__ __forceinline__ float cusp_correction(const PointConst& c, const PointConst64& c64, int N,
                                                 const PixelGeom& g) {
  float acc = 0.0f;
  for (int ky = 0; ky < N; ++ky) {
    const float y = fmaf(g.uy + sub_offset_rt(ky, N), g.d, g.cy);
    for (int kx = 0; kx < N; ++kx) {
      const float x = fmaf(g.ux + sub_offset_rt(kx, N), g.d, g.cx);
      const float sR2 = source_r2<MODE>(c, x, y);
      if (sR2 < c.cusp_r2) {
        float dx, dy;
        source_offset_f64(c64, g, kx, ky, N, dx, dy);
        const float exact = sersic_from_r2(sersic_r2(dx, dy, c.sc, c.ss, c.sqa, c.sqb), c.se, c.sB, c.sI);
        acc += exact - sersic_from_r2(sR2, c.se, c.sB, c.sI);
      }
    }
  }
  return acc;
}

}  // namespace lensed
