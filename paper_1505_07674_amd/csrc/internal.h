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

// Per-point constants derived once from the 17 parameters (prologue kernel).
// Read with wave-uniform addresses, so they live in scalar registers in the
// render kernels. Invalid points carry NaN in the amplitudes and in the lens
// matrix, which turns every result of that point into NaN.
struct PointConst {
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
  float pad[4];
  // ---- folded forms used by the forward render (the adjoint uses the fields above)
  // rmode: 0 sphere, 1 polynomials (q' <= 1/2), 2 log + half-angle atan with
  // argument <= 1/sqrt(3) (q >= 1/2), 3 log + half-angle atan on [0, 1] (q < 1/2).
  int rmode;
  // alpha_x = tac At - ths Ah, alpha_y = tas At + thc Ah, with the factors 2
  // (half angle) and ln 2 (log2) of modes 2 and 3 folded in; mode 0: tac = theta_E.
  float tac, tas, thc, ths;
  // scaled frame of the Sersic profiles: (R/R_e)^2 = X^2 + Y^2,
  // X = a11 dx + a12 dy, Y = a21 dx + a22 dy (sqrt(q)/R_e and 1/(sqrt(q) R_e) folded in)
  float h11, h12, h21, h22;
  float s11, s12, s21, s22;
  // the source frame of beta - (x_S, y_S) in one step: with S = (s11 s12; s21 s22),
  // X = A1 x + (B1 y + C1) + cXt At + cXh Ah, Y = A2 x + (B2 y + C2) + cYt At + cYh Ah,
  // (A1 A2) = S (m11 m12), (B1 B2) = S (m12 m22), (C1 C2) = -S (x_S y_S),
  // cXt = -(s11 tac + s12 tas), cXh = s11 ths - s12 thc, and the same with s21, s22.
  float A1, A2, B1, B2, C1, C2, cXt, cXh, cYt, cYh;
  // low parts of the two amplitudes (I_e - float(I_e)), non-zero only when I_e
  // is derived in float64 from a magnitude: they keep the float32 rounding of
  // the amplitude from scaling every pixel of a component the same way
  float hIlo, sIlo;
  float pad2[7];
};
static_assert(sizeof(PointConst) == 64 * 4, "PointConst layout");

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
  float pad[5];
};
static_assert(sizeof(GradConst) == 48 * 4, "GradConst layout");

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
};

constexpr int RENDER_BLOCK = 256;

// A wave of the render kernel with pixels next to a cuspy source centre: the
// point, the first pixel of the wave and the lane mask of flagged pixels.
struct CuspEntry {
  int point;
  int pix0;
  unsigned long long mask;
};

// Correction work list filled by the render kernel (count reset by the prologue).
struct CuspList {
  CuspEntry* entries;   // capacity: one entry per render wave of the launch
  int* count;
};   // pixels per render tile / threads per render block

}  // namespace lensed
