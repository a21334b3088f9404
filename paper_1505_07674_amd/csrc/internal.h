// internal.h -- device-side data layout shared by the kernels of liblensed_hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lensed {

constexpr int NPAR = 17;
constexpr float LN2F = 0.693147180559945309f;
constexpr double LOG2E = 1.44269504088896340736;
// Source-plane radius around a cuspy source centre inside which subsamples are
// re-traced in float64 (the float32 ray position carries ~1e-7 arcsec of rounding).
// With an image-plane source position every point puts the source centre on one
// of its images, where the lens magnifies that rounding; the radius doubles.
constexpr double CUSP_RADIUS_ARCSEC = 0.03;
constexpr double CUSP_RADIUS_IMAGE_PLANE_ARCSEC = 0.06;

// Float32 constants of the forward render, folded in float64 from the
// parameters (prologue kernel) and rounded to float32. Each point carries
// RENDER_VARIANTS roundings of them: variant v rounds every constant c to the
// float32 neighbour below or above it, upward in a share of the variants equal
// to c's position between its two neighbours (to 1/32 of their gap). Pixel
// (row, col) uses the variant of its cell in an ordered-dither pattern
// (render_variant). Every pixel thus sees each constant within one float32
// spacing, while the mean over any 4 x 8 block of pixels is the float64
// constant (to 1/32 of a spacing): the rounding
// of the constants stops acting as a coherent perturbation of the model,
// which a chi^2 far from its minimum would otherwise amplify (a relative
// model bias eps moves log L by about 2 eps relative).
//
//   lens light  R^2/R_e^2 = (ha x + hb y) x + hc y^2,  I = I_e exp2(hB (1 - t)), t = exp2(he log2(R^2/R_e^2))
//   source      the same with (se, sB) at the source frame of beta - x_S:
//               X = A1 x + (B1 y + C1) + cXt At + cXh Ah,  Y = A2 x + (B2 y + C2) + cYt At + cYh Ah
//   SIE frame   x' = cL x + sL y, y' = cL y - sL x, psi^2 = q2 x'^2 + y'^2; At, Ah the folded deflection terms
//   sphere      alpha = tac (x, y)/r, X = A1 x + (B1 y + C1) - (tac/r)(s11 x + s12 y) (Y: s21, s22)
struct RenderVariant {
  float cL, sL, q2, iq;
  float qp;                      // q' = sqrt(1 - q^2), the leading coefficient of the folded polynomials
  float A1, A2, B1, B2, C1, C2;
  float cXt, cXh, cYt, cYh;
  float ha, hb, hc, he, hB;
  float se, sB;
  float tac;
  float s11, s12, s21, s22;
  float pad[5];
};
static_assert(sizeof(RenderVariant) == 32 * 4, "RenderVariant layout");
constexpr int RENDER_VARIANTS = 16;

// Variant of pixel (row, col): a 4 x 4 Bayer ordered dither over cells of two
// horizontally adjacent pixels (so a thread that renders a pixel pair (2j, 2j+1)
// needs one set), repeating every 4 rows and 8 columns.
__device__ __forceinline__ int render_variant(int row, int col) {
  return (int)((0x5D7F91B36E4CA280ull >> (4 * (((row & 3) << 2) | ((col >> 1) & 3)))) & 15ull);
}

// Per-point constants derived once from the 17 parameters (prologue kernel).
// The uniform part (PointHead) is read with wave-uniform addresses, so it lives
// in scalar registers; each render thread reads its pixel's variant of the
// folded constants from rv. Invalid points carry NaN in the amplitudes and in
// the lens matrix, which turns every result of that point into NaN.
struct PointHead {
  int sie_mode;        // 0: isothermal sphere (q = 1); 1: atanh by polynomial (q' <= 1/2); 2: atanh by log
  float cL, sL;        // frame rotation of the SIE
  float q2;            // q_L^2
  float qp;            // q' = sqrt(1 - q_L^2)
  float kc, ks;        // k cos(phi_L), k sin(phi_L), k = theta_E sqrt(q)/q' (mode 0: kc = theta_E)
  float iq;            // 1/q_L
  float m11, m12, m22; // beta = M x - alpha_SIE(x), M = 1 - shear matrix
  // lens light: I = hI * exp2(hB (1 - t)), t = exp2(he * log2(hqa x'^2 + hqb y'^2))
  float hc, hs, hqa, hqb, he, hB, hI;
  // source: same, about (sx0, sy0)
  float sx0, sy0, sc, ss, sqa, sqb, se, sB, sI;
  // source subsamples with R^2/R_e^2 below this are re-traced in float64 (0 = never)
  float cusp_r2;
  // rmode: 0 sphere, 1 polynomials (q' <= 1/2), 2 log + half-angle atan with
  // argument <= 1/sqrt(3) (q >= 1/2), 3 log + half-angle atan on [0, 1] (q < 1/2).
  int rmode;
  // Higher coefficients of the deflection polynomials with q' folded in, so that
  // they take x'/psi (mode 1) or x'/(psi + r) (modes 2, 3) directly: atan
  // (mode 1: poly[1..5]; mode 2: poly[1..5]; mode 3: poly[1..8]) and, in mode 1,
  // atanh (poly[6..10]); coefficient k is c_k q'^(2k+1). The leading q' is per
  // variant.
  float poly[11];
  // low parts of the two amplitudes (I_e - float(I_e)), non-zero only when I_e
  // is derived in float64 from a magnitude: they keep the float32 rounding of
  // the amplitude from scaling every pixel of a component the same way
  float hIlo, sIlo;
  float pad[22];
};
static_assert(sizeof(PointHead) == 64 * 4, "PointHead layout");

struct PointConst : PointHead {
  RenderVariant rv[RENDER_VARIANTS];
};
static_assert(sizeof(PointConst) == sizeof(PointHead) + RENDER_VARIANTS * sizeof(RenderVariant), "PointConst layout");

// Float64 lens constants for the rare re-tracing of subsamples that land next
// to the centre of a cuspy (n > 1) source, where the float32 rounding of the
// ray position (~1e-7 arcsec) is amplified by the steep profile.
struct PointConst64 {
  double cL, sL, q2, qp, k, te;   // SIE frame, k = theta_E sqrt(q)/q'
  double m11, m12, m22;           // 1 - shear matrix
  double sx0, sy0;                // source centre
  int mode;                       // 0: isothermal sphere
  int pad0;
  double pad[4];
};
static_assert(sizeof(PointConst64) == 16 * 8, "PointConst64 layout");

// Per-point values of the gradient's per-subsample arithmetic, derived in
// float64 by the prologue and read with uniform addresses (scalar registers).
struct GradUniform {
  float tesq;          // theta_E sqrt(q)
  float iqp;           // 1/q' (0 when q = 1)
  float s;             // 1 - q^2
  float hs;            // 1/(2 s) (0 when s = 0)
  float iq2;           // 1/q^2
  float bH, bS;        // natural-log Sersic constants b_n of the lens light and the source
  float dbH, dbS;      // db_n/dn
  float kS1, kS2;      // cos, sin (phi_S - phi_L): source-frame gradient into the SIE frame
};

// Extra per-point values needed by the adjoint.
struct GradConst {
  float theta[NPAR];   // raw parameters
  float dB_dn_h;       // d(b_n log2 e)/dn for the lens light
  float dB_dn_s;       // same for the source
  float bh, bs;        // b_n of lens light and source
  // Magnitude parametrisation (amp != 0): theta[5] and theta[12] are total
  // magnitudes; I_e * d ln I_e / d(m, R_e, n) of the lens light [0..2] and of
  // the source [3..5], which carry d log L / d I_e over to the parameters.
  float amp_chain[6];
  int amp;
  // Image-plane source position (srcpos != 0): theta[10], theta[11] are an
  // image-plane point x_I and the source centre is beta(x_I). Jacobian of beta
  // (row 0: x, row 1: y) with respect to (x_I, y_I, theta_E, q_L, phi_L, gamma,
  // phi_gamma), row-major.
  float src_jac[14];
  int srcpos;
  GradUniform u;
  float pad[10];
};
static_assert(sizeof(GradConst) == 64 * 4, "GradConst layout");

// Geometry and schedule of one system (one observation).
struct SysDesc {
  int H, W, N;            // image size and subsampling
  int ph, pw;             // PSF dimensions (odd)
  float d, cx, cy;        // pixel scale and grid centre
  const float* psf;       // caller's PSF (unnormalised)
  float* psfn;            // library copies normalised to unit sum: row-major, column-major flipped,
                          // column-major (3 ph pw floats)
  const float* data;
  const float* weight;
  int TW, TH;             // PSF/chi^2 output tile
  int tiles_x, n_ptiles;  // PSF tiles per row, per image
  int n_rtiles;           // render tiles (RENDER_BLOCK pixels each) per image
  int rule;               // 0 N x N midpoint; 1, 2, 3: Gauss-Kronrod g3k7, g5k11, g7k15 (N = 7, 11, 15)
  int amp;                // 0: theta[5], theta[12] are I_e; 1: total magnitudes with zero point zp
  float zp;
  int srcpos;             // 0: theta[10], theta[11] are the source centre; 1: an image-plane point
  double wgt;             // quadrature weight pixscale^2 / N^2, in float64
  float* adjk;            // 16 folded PSF tables of the adjoint (or nullptr)
  float* adjk_pad;
  // Render units of a masked plan (built on the host) or of a gradient plan
  // (uact below, rebuilt on the device): the first pixel of each unit (a
  // pixel, or a pair of adjacent pixels) that the chi^2 can see, row-major;
  // nullptr: every pixel, unit u starting at pixel u * ppt.
  const int* active;
  int n_active;           // units in `active`
  int pad_active;
  unsigned int wdiv_m;    // row of pixel n: (n wdiv_m) >> wdiv_s (row_of)
  int wdiv_s;
  // Support of the adjoint's g = A^T rho in a gradient plan: every pixel within
  // the PSF box of a pixel with w > 0 (replicate padding only moves a tap
  // towards the image, so the clamped border taps stay inside that box).
  // Rebuilt from the weights by every gradient launch (grad_support_*
  // kernels): gsup[0 .. *gsup_n) its pixels in row-major order, gflags 2 H W
  // bytes of scratch. nullptr: every pixel.
  int* gsup;
  int* gsup_n;
  unsigned char* gflags;
  // Render units over the same support (a 17-parameter gradient plan renders
  // only these): the support kernels write the first pixel of each unit of
  // uppt pixels to uact, which `active` also points to, and their number to
  // n_active of the device copy of this descriptor. nullptr: not rebuilt.
  int* uact;
  int uppt;
  // Per PSF output tile of a gradient plan: 1 if it holds a pixel with w > 0
  // (set by the support kernels each launch, cleared by the PSF preparation);
  // the PSF stage skips the others, whose chi^2 terms and rho are all zero.
  // nullptr: every tile is convolved.
  unsigned char* ptile_w;
};

// floor(n / W) for 0 <= n < 2^28 (every pixel index: H W <= 2^28) by one
// 32 x 32 -> 64-bit product and a shift instead of an integer division
// (Granlund & Montgomery 1994, Thm. 4.2): with 2^(l-1) < W <= 2^l the
// multiplier m = floor(2^(28+l) / W) + 1 satisfies 2^(28+l) < m W <= 2^(28+l) + 2^l.
__host__ __device__ __forceinline__ int row_of(const SysDesc& sd, int n) {
  return (int)(((unsigned long long)(unsigned)n * sd.wdiv_m) >> sd.wdiv_s);
}
inline void set_row_divisor(SysDesc& d) {
  int l = 0;
  while ((1ll << l) < (long long)d.W) ++l;
  d.wdiv_s = 28 + l;
  d.wdiv_m = (unsigned int)((1ull << (28 + l)) / (unsigned long long)d.W + 1ull);
}

// First pixel of render unit u of an image rendered with ppt pixels per unit.
__device__ __forceinline__ int unit_pixel(const SysDesc& sd, int u, int ppt) {
  return sd.active ? sd.active[u] : u * ppt;
}
// Render units of an image.
__host__ __device__ __forceinline__ int unit_count(const SysDesc& sd, int ppt) {
  return sd.active ? sd.n_active : (sd.H * sd.W + ppt - 1) / ppt;
}
// Pixels of the adjoint's support, and pixel u of it.
__device__ __forceinline__ int grad_support_count(const SysDesc& sd) { return sd.gsup ? *sd.gsup_n : sd.H * sd.W; }
__device__ __forceinline__ int grad_support_pixel(const SysDesc& sd, int u) { return sd.gsup ? sd.gsup[u] : u; }

constexpr int RENDER_BLOCK = 256;

// A wave of the render kernel with pixels next to a cuspy source centre: the
// point, the lane mask of flagged pixels, and where the lanes' pixels are:
// lane l rendered render unit unit0 + l of the point's image (unit_pixel), and
// the entry covers pixel `half` of each unit (0, or 1 for the second pixel of
// a pair when a thread renders ppt = 2 adjacent pixels).
struct CuspEntry {
  int point;
  int unit0;
  unsigned long long mask;
  int ppt;
  int half;
};

// Correction work list filled by the render kernel (count reset by the prologue).
struct CuspList {
  CuspEntry* entries;   // capacity: one entry per render wave of the launch
  int* count;
};   // pixels per render tile / threads per render block

}  // namespace lensed
