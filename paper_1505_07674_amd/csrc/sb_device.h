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

#include <utility>

#include "gk_rules.h"
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

// Float64 re-tracing of one subsample: exact abscissa (as the rule defines it:
// offsets ox, oy in pixel units), SIE + shear lens equation in float64, offset
// from the source centre.
__device__ __forceinline__ void source_offset_f64(const PointConst64& e, const PixelGeom& g, double ox, double oy,
                                                  float& dx, float& dy) {
  const double x = (double)g.cx + ((double)g.ux + ox) * (double)g.d;
  const double y = (double)g.cy + ((double)g.uy + oy) * (double)g.d;
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

// ---------------------------------------------------------------------------
// Forward render, float32, with the folded constants: the uniform part of
// PointConst (mode, polynomial coefficients, amplitudes, cusp radius) and the
// pixel's RenderVariant k. Every product and sum is written out with explicit
// fmaf so that the render kernel and the cusp correction, which must reproduce
// the render's float32 value of a subsample, round identically.
// ---------------------------------------------------------------------------

// Terms of the subsample grid that depend on the row (y) only.
constexpr float SIE_TINY = 1e-30f;

struct RowTerms {
  float y2t;          // sphere: y^2 + SIE_TINY
  float sLy, cLy;     // SIE frame: x' = cL x + sL y, y' = cL y - sL x
  float rX, rY;       // B1 y + C1, B2 y + C2: row part of the source frame of beta
  float s12y, s22y;   // sphere: s12 y, s22 y
  float hby, hcy2;    // lens light: hb y, hc y^2
};

__device__ __forceinline__ RowTerms row_terms(const RenderVariant& k, float y) {
  RowTerms r;
  r.y2t = fmaf(y, y, SIE_TINY);
  r.sLy = k.sL * y;
  r.cLy = k.cL * y;
  r.rX = fmaf(k.B1, y, k.C1);
  r.rY = fmaf(k.B2, y, k.C2);
  r.s12y = k.s12 * y;
  r.s22y = k.s22 * y;
  r.hby = k.hb * y;
  r.hcy2 = k.hc * y * y;
  return r;
}

// p0 + s (c[1] + s (c[2] + ... + s c[D])): a deflection polynomial with q'
// folded into its coefficients (uniform c[1..D], per-variant leading p0 = q').
template <int D>
__device__ __forceinline__ float folded_poly(const float* c, float p0, float s) {
  float p = c[D];
#pragma unroll
  for (int j = D - 1; j >= 1; --j) p = fmaf(p, s, c[j]);
  return fmaf(p, s, p0);
}

// Source-frame coordinates (X, Y) of beta - (x_S, y_S), (R/R_e)^2 = X^2 + Y^2,
// for the image-plane subsample (x, row y): Eq. 1 with the SIE + external shear,
// the shear matrix, the source centre and the source ellipse folded into
// per-point constants. The polynomials take w = x'/psi (mode 1) or
// w = x'/(psi + r) (modes 2, 3) and return the folded atan (and atanh)
// directly: atan(q' w) = w P(w^2) with P's coefficients c_k q'^(2k+1).
//
// The lens centre needs no branch: x'^2 carries SIE_TINY (arcsec^2), so that at
// x' = y' = 0 exactly psi = q sqrt(SIE_TINY), r = sqrt(SIE_TINY), the atan argument
// is 0 and the atanh log argument is psi/(q r) = 1: the deflection there is 0
// (to rounding), the value the method takes at its singular point. Elsewhere
// the offset changes x'^2 by a relative 1e-30 / x'^2, below float32 resolution
// for any |x'| above 1e-11 arcsec.
template <int RM>
__device__ __forceinline__ void source_frame(const PointConst& c, const RenderVariant& k, const RowTerms& r, float x,
                                             float& X, float& Y) {
  const float lX = fmaf(k.A1, x, r.rX);
  const float lY = fmaf(k.A2, x, r.rY);
  if (RM == 0) {
    const float s = k.tac * hw_rsq(fmaf(x, x, r.y2t));   // alpha = s (x, y)
    X = fmaf(-s, fmaf(k.s11, x, r.s12y), lX);
    Y = fmaf(-s, fmaf(k.s21, x, r.s22y), lY);
    return;
  }
  const float xp = fmaf(k.cL, x, r.sLy);
  const float yp = fmaf(-k.sL, x, r.cLy);
  const float yp2 = yp * yp;
  const float x2t = fmaf(xp, xp, SIE_TINY);
  const float psi2 = fmaf(k.q2, x2t, yp2);
  float At, Ah;
  if (RM == 1) {
    const float ip = hw_rsq(psi2);
    const float w1 = ip * xp, w2 = ip * yp;
    At = w1 * folded_poly<ATAN_SMALL_POLY_DEGREE>(c.poly, k.qp, w1 * w1);
    Ah = w2 * folded_poly<ATANH_POLY_DEGREE>(c.poly + ATAN_SMALL_POLY_DEGREE, k.qp, w2 * w2);
  } else {
    const float r2 = x2t + yp2;
    const float psi = __builtin_amdgcn_sqrtf(psi2);
    const float ir = hw_rsq(r2);
    const float w = xp * hw_rcp(fmaf(r2, ir, psi));
    At = RM == 2 ? w * folded_poly<ATAN_SMALL_POLY_DEGREE>(c.poly, k.qp, w * w)
                 : w * folded_poly<ATAN_UNIT_POLY_DEGREE>(c.poly, k.qp, w * w);
    Ah = copysignf(hw_log2(fmaf(k.qp, fabsf(yp), psi) * ir * k.iq), yp);
  }
  X = fmaf(k.cXt, At, fmaf(k.cXh, Ah, lX));
  Y = fmaf(k.cYt, At, fmaf(k.cYh, Ah, lY));
}

// (R/R_e)^2 of the source at offset (dx, dy) from its centre.
__device__ __forceinline__ float source_R2(const RenderVariant& k, float dx, float dy) {
  const float X = fmaf(k.s11, dx, k.s12 * dy);
  const float Y = fmaf(k.s21, dx, k.s22 * dy);
  return fmaf(X, X, Y * Y);
}

// Sersic shape I / I_e = exp2(B (1 - t)), t = (R^2/R_e^2)^e; the amplitude I_e is
// a per-point factor and multiplies the pixel sums instead of every subsample.
__device__ __forceinline__ float sersic_shape(float R2, float e, float B) {
  return hw_exp2(fmaf(-B, hw_exp2(e * hw_log2(R2)), B));
}

// Lens-light and source shapes at one subsample, and the cusp flag.
template <int RM>
__device__ __forceinline__ void subsample_light(const PointConst& c, const RenderVariant& k, const RowTerms& r,
                                                float x, float& h, float& s, bool& cusp) {
  h = sersic_shape(fmaf(fmaf(k.ha, x, r.hby), x, r.hcy2), k.he, k.hB);
  float sX, sY;
  source_frame<RM>(c, k, r, x, sX, sY);
  const float sR2 = fmaf(sX, sX, sY * sY);
  cusp = cusp || (sR2 < c.cusp_r2);
  s = sersic_shape(sR2, k.se, k.sB);
}

// Lens-light and source sums times their amplitudes, the low parts first (they
// are zero unless an amplitude was derived from a magnitude).
__device__ __forceinline__ float amplitudes(const PointConst& c, float sh, float ss) {
  const float lo = fmaf(c.hIlo, sh, c.sIlo * ss);
  return fmaf(c.hI, sh, fmaf(c.sI, ss, lo));
}

// Sum of the surface brightness over the N x N midpoint abscissae of a pixel.
template <int N, int RM>
__device__ __forceinline__ float pixel_sum(const PointConst& c, const RenderVariant& k, const PixelGeom& g,
                                           bool& cusp) {
  float sh = 0.0f, ss = 0.0f;
  float xs[N];
#pragma unroll
  for (int kx = 0; kx < N; ++kx) xs[kx] = fmaf(g.ux + sub_offset<N>(kx), g.d, g.cx);
#pragma unroll
  for (int ky = 0; ky < N; ++ky) {
    const RowTerms r = row_terms(k, fmaf(g.uy + sub_offset<N>(ky), g.d, g.cy));
#pragma unroll
    for (int kx = 0; kx < N; ++kx) {
      float h, s;
      subsample_light<RM>(c, k, r, xs[kx], h, s, cusp);
      if (ky == 0 && kx == 0) {
        sh = h;
        ss = s;
      } else {
        sh += h;
        ss += s;
      }
    }
  }
  return amplitudes(c, sh, ss);
}

// The same for two horizontally adjacent pixels of one row (the second one
// pixel to the right): the row terms are computed once for both.
template <int N, int RM>
__device__ __forceinline__ void pixel_sum_pair(const PointConst& c, const RenderVariant& k, const PixelGeom& g,
                                               float& acc0, float& acc1, bool& cusp0, bool& cusp1) {
  float sh0 = 0.0f, ss0 = 0.0f, sh1 = 0.0f, ss1 = 0.0f;
  float xs0[N], xs1[N];
#pragma unroll
  for (int kx = 0; kx < N; ++kx) {
    xs0[kx] = fmaf(g.ux + sub_offset<N>(kx), g.d, g.cx);
    xs1[kx] = fmaf((g.ux + 1.0f) + sub_offset<N>(kx), g.d, g.cx);
  }
#pragma unroll
  for (int ky = 0; ky < N; ++ky) {
    const RowTerms r = row_terms(k, fmaf(g.uy + sub_offset<N>(ky), g.d, g.cy));
#pragma unroll
    for (int kx = 0; kx < N; ++kx) {
      float h0, s0, h1, s1;
      subsample_light<RM>(c, k, r, xs0[kx], h0, s0, cusp0);
      subsample_light<RM>(c, k, r, xs1[kx], h1, s1, cusp1);
      if (ky == 0 && kx == 0) {
        sh0 = h0;
        ss0 = s0;
        sh1 = h1;
        ss1 = s1;
      } else {
        sh0 += h0;
        ss0 += s0;
        sh1 += h1;
        ss1 += s1;
      }
    }
  }
  acc0 = amplitudes(c, sh0, ss0);
  acc1 = amplitudes(c, sh1, ss1);
}

template <int RM>
__device__ __forceinline__ float pixel_sum_rt(const PointConst& c, const RenderVariant& k, int N, const PixelGeom& g,
                                              bool& cusp) {
  float sh = 0.0f, ss = 0.0f;
  for (int ky = 0; ky < N; ++ky) {
    const RowTerms r = row_terms(k, fmaf(g.uy + sub_offset_rt(ky, N), g.d, g.cy));
    for (int kx = 0; kx < N; ++kx) {
      float h, s;
      subsample_light<RM>(c, k, r, fmaf(g.ux + sub_offset_rt(kx, N), g.d, g.cx), h, s, cusp);
      sh += h;
      ss += s;
    }
  }
  return amplitudes(c, sh, ss);
}

// (R/R_e)^2 of the source seen by the float32 render at subsample (x, y).
__device__ __forceinline__ float render_source_R2(const PointConst& c, const RenderVariant& k, float x, float y) {
  const RowTerms r = row_terms(k, y);
  float X, Y;
  switch (c.rmode) {
    case 0: source_frame<0>(c, k, r, x, X, Y); break;
    case 1: source_frame<1>(c, k, r, x, X, Y); break;
    case 2: source_frame<2>(c, k, r, x, X, Y); break;
    default: source_frame<3>(c, k, r, x, X, Y); break;
  }
  return fmaf(X, X, Y * Y);
}

// ---------------------------------------------------------------------------
// Gauss-Kronrod product rules (Sec. 3.1 Eq. 14, Sec. 4.5: g3k7, g5k11, g7k15):
// offsets on [-1/2, 1/2] pixel, Kronrod weights and embedded Gauss weights (0 at
// the Kronrod-only nodes), each summing to 1, from gk_rules.h.
// ---------------------------------------------------------------------------
struct GkRule {
  float x[15], w[15], g[15];
  double xd[15];
};

template <size_t K, size_t... I>
constexpr GkRule make_gk_rule(const double (&x)[K], const double (&w)[K], const double (&g)[K],
                              std::index_sequence<I...>) {
  return GkRule{{float(x[I])...}, {float(w[I])...}, {float(g[I])...}, {x[I]...}};
}

static __constant__ GkRule kGkRules[3] = {
    make_gk_rule(GK7_X, GK7_W, GK7_G, std::make_index_sequence<7>{}),
    make_gk_rule(GK11_X, GK11_W, GK11_G, std::make_index_sequence<11>{}),
    make_gk_rule(GK15_X, GK15_W, GK15_G, std::make_index_sequence<15>{}),
};

// Kronrod-weighted sum over the K x K nodes of a pixel (rows rolled, columns
// unrolled); with ERR also the embedded Gauss sum, returned in gauss.
template <int K, int RM, bool ERR = false>
__device__ __forceinline__ float pixel_sum_gk(const PointConst& c, const RenderVariant& kv, const PixelGeom& g,
                                              bool& cusp, float* gauss = nullptr) {
  const GkRule& R = kGkRules[(K - 7) / 4];
  float xs[K];
#pragma unroll
  for (int kx = 0; kx < K; ++kx) xs[kx] = fmaf(g.ux + R.x[kx], g.d, g.cx);
  float sh = 0.0f, ss = 0.0f, gh = 0.0f, gs = 0.0f;
#pragma unroll 1
  for (int ky = 0; ky < K; ++ky) {
    const RowTerms r = row_terms(kv, fmaf(g.uy + R.x[ky], g.d, g.cy));
    float rh = 0.0f, rs = 0.0f, qh = 0.0f, qs = 0.0f;
#pragma unroll
    for (int kx = 0; kx < K; ++kx) {
      float h, s;
      subsample_light<RM>(c, kv, r, xs[kx], h, s, cusp);
      rh = fmaf(R.w[kx], h, rh);
      rs = fmaf(R.w[kx], s, rs);
      if (ERR) {
        qh = fmaf(R.g[kx], h, qh);
        qs = fmaf(R.g[kx], s, qs);
      }
    }
    sh = fmaf(R.w[ky], rh, sh);
    ss = fmaf(R.w[ky], rs, ss);
    if (ERR) {
      gh = fmaf(R.g[ky], qh, gh);
      gs = fmaf(R.g[ky], qs, gs);
    }
  }
  if (ERR) *gauss = amplitudes(c, gh, gs);
  return amplitudes(c, sh, ss);
}

}  // namespace lensed
