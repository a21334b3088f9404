// prologue.hip -- per-point derived constants and PSF normalisation.
//
// One thread per parameter point turns the 17 float32 parameters into the
// wave-uniform constants the render kernels consume (trigonometry, the shear
// matrix, reciprocal radii and the Sersic b_n). b_n is the root of
// P(2n, b) = 1/2 (R_e is the half-light radius, Sec. 4.1 Eq. 22), solved here in
// float64 by a bracketed Halley iteration on the power series of the
// regularised incomplete gamma function. Extra blocks normalise each system's
// PSF to unit sum (Sec. 3.1).
#include <math.h>

#include "internal.h"
#include "kernels.h"
#include "sie_poly.h"

namespace lensed {
namespace {

// Root of P(a, b) = 1/2 by Halley's method, safeguarded by bisection, from the
// start b0. P(a, x) = x^a e^{-x} / Gamma(a+1) * (1 + x/(a+1) + x^2/((a+1)(a+2)) + ...),
// dP/dx = x^{a-1} e^{-x} / Gamma(a) = (x^a e^{-x} / Gamma(a+1)) a / x and
// d2P/dx2 = dP/dx ((a - 1)/x - 1). Stopping: once a step is below 1e-4 of b,
// one more step brings the error, cubically, below rounding, and the loop ends
// there. (Waiting for
// a step below 4e-16 of b instead lets rounding noise in f keep the iteration
// going, and an f that rounds to exactly 0 made the bracket send b off by a
// bisection step: dozens of extra iterations for some n, and a wave waits for
// its slowest lane.)
__device__ double gamma_median(double a, double b0) {
  const double lga1 = lgamma(a + 1.0);
  double lo = 0.0, hi = a + 40.0;
  double b = (b0 > lo && b0 < hi) ? b0 : 0.5 * a + 1e-3;
  bool last = false;
  for (int it = 0; it < 100; ++it) {
    const double pref = exp(a * log(b) - b - lga1);
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 600; ++k) {
      term *= b / (a + (double)k);
      sum += term;
      if (term <= 1e-17 * sum) break;
    }
    const double f = pref * sum - 0.5;
    if (f == 0.0) break;
    if (f > 0.0) hi = b; else lo = b;
    const double d1 = pref * a / b, d2 = d1 * ((a - 1.0) / b - 1.0);
    double nb = b - 2.0 * f * d1 / (2.0 * d1 * d1 - f * d2);
    const bool inside = nb >= lo && nb <= hi;
    if (!inside) nb = 0.5 * (lo + hi);
    const double step = fabs(nb - b);
    b = nb;
    if (last || step <= 4e-16 * b) break;
    if (inside && step <= 1e-4 * b) last = true;
  }
  return b;
}

// b_n (R_e is the half-light radius, Sec. 4.1 Eq. 22), started from the
// asymptotic expansion of Ciotti & Bertin (1999): within 4e-4 for n >= 0.5 and
// within 2e-3 at n = 0.3, so Halley needs two or three steps.
__device__ double sersic_bn(double n) {
  const double in = 1.0 / n;
  const double b0 = 2.0 * n - 1.0 / 3.0 +
                    in * (4.0 / 405.0 + in * (46.0 / 25515.0 + in * (131.0 / 1148175.0 - in * (2194697.0 / 30690717750.0))));
  return gamma_median(2.0 * n, b0);
}

// Digamma psi(z), z > 0: psi(z) = psi(z + 1) - 1/z up to z >= 8, then the
// asymptotic expansion psi(z) ~ ln z - 1/(2z) - sum_k B_2k / (2k z^2k)
// (Abramowitz & Stegun 6.3.18) to z^-12, below 1e-15 relative there.
__device__ double digamma_d(double z) {
  double shift = 0.0;
  while (z < 8.0) {
    shift += 1.0 / z;
    z += 1.0;
  }
  const double w = 1.0 / (z * z);
  const double tail =
      w * (1.0 / 12.0 + w * (-1.0 / 120.0 + w * (1.0 / 252.0 + w * (-1.0 / 240.0 + w * (1.0 / 132.0 + w * (-691.0 / 32760.0))))));
  return log(z) - 0.5 / z - tail - shift;
}

// Sersic amplitude from a total magnitude (Sec. 4.1: the amplitude is set by
// the total magnitude). The elliptical profile with the geometric-mean radius
// has the circular profile's flux F = 2 pi n R_e^2 I_e e^{b} Gamma(2n) / b^{2n},
// and F = 10^{-0.4 (m - zp)}, so
//   ln I_e = -0.4 ln 10 (m - zp) + 2n ln b - ln(2 pi n R_e^2) - b - ln Gamma(2n),
// and with b = b_n(n):
//   d ln I_e/dm = -0.4 ln 10,  d ln I_e/dR_e = -2/R_e,
//   d ln I_e/dn = 2 ln b + (2n/b - 1) db/dn - 1/n - 2 psi(2n).
struct AmpFromMag {
  double I;          // I_e
  double dm, dR, dn; // I_e times the three logarithmic derivatives
};
__device__ AmpFromMag amplitude_from_magnitude(double m, double Re, double n, double b, double db_dn, double zp) {
  const double ln10 = 2.302585092994045684;
  const double two_pi = 6.283185307179586477;
  const double lnI = -0.4 * ln10 * (m - zp) + 2.0 * n * log(b) - log(two_pi * n * Re * Re) - b - lgamma(2.0 * n);
  AmpFromMag a;
  a.I = exp(lnI);
  a.dm = a.I * (-0.4 * ln10);
  a.dR = a.I * (-2.0 / Re);
  a.dn = a.I * (2.0 * log(b) + (2.0 * n / b - 1.0) * db_dn - 1.0 / n - 2.0 * digamma_d(2.0 * n));
  return a;
}

// Lens equation in float64 (Eq. 1): beta = x - alpha_SIE(x) - alpha_shear(x),
// SIE in the area-preserving convention about the origin (alpha = 0 at its
// centre), external shear about the same centre.
__device__ void lens_map_f64(const double (&v)[7], double& bx, double& by) {
  const double x = v[0], y = v[1], te = v[2], q = v[3], ph = v[4], g = v[5], phg = v[6];
  const double c = cos(ph), s = sin(ph);
  const double xp = c * x + s * y, yp = c * y - s * x;
  const double psi = sqrt(q * q * xp * xp + yp * yp);
  double axp = 0.0, ayp = 0.0;
  if (psi > 0.0) {
    const double s2 = (1.0 - q) * (1.0 + q);
    if (s2 > 0.0) {
      const double qp = sqrt(s2), k = te * sqrt(q) / qp;
      axp = k * atan(qp * xp / psi);
      ayp = k * atanh(qp * yp / psi);
    } else {
      axp = te * xp / psi;
      ayp = te * yp / psi;
    }
  }
  const double g1 = g * cos(2.0 * phg), g2 = g * sin(2.0 * phg);
  bx = x - (c * axp - s * ayp) - (g1 * x + g2 * y);
  by = y - (s * axp + c * ayp) - (g2 * x - g1 * y);
}

// d beta / d v by central differences in float64 (step 1e-6 of the scale: error
// ~1e-10 relative); q_L steps backwards with a second-order stencil where a
// forward step would leave q <= 1.
__device__ void lens_map_jacobian(const double (&v)[7], float (&jac)[14]) {
  for (int j = 0; j < 7; ++j) {
    const double h = 1e-6 * fmax(fabs(v[j]), 1.0) * (j == 3 ? 0.25 : 1.0);
    double a[7], b[7], bxa, bya, bxb, byb;
    for (int i = 0; i < 7; ++i) a[i] = b[i] = v[i];
    double dx, dy;
    if (j == 3 && v[3] + h > 1.0) {
      double c2[7];
      for (int i = 0; i < 7; ++i) c2[i] = v[i];
      a[3] = v[3] - h;
      c2[3] = v[3] - 2.0 * h;
      double bx0, by0, bx2, by2;
      lens_map_f64(v, bx0, by0);
      lens_map_f64(a, bxa, bya);
      lens_map_f64(c2, bx2, by2);
      dx = (3.0 * bx0 - 4.0 * bxa + bx2) / (2.0 * h);
      dy = (3.0 * by0 - 4.0 * bya + by2) / (2.0 * h);
    } else {
      a[j] = v[j] + h;
      b[j] = v[j] - h;
      lens_map_f64(a, bxa, bya);
      lens_map_f64(b, bxb, byb);
      dx = (bxa - bxb) / (2.0 * h);
      dy = (bya - byb) / (2.0 * h);
    }
    jac[j] = (float)dx;
    jac[7 + j] = (float)dy;
  }
}

__device__ bool ok_q(float q) { return q > 0.0f && q <= 1.0f; }
__device__ bool ok_n(float n) { return n >= 0.2f && n <= 10.0f; }

// Float32 rounding of c for render variant v: the float32 neighbour below or
// above c, upward for a share of the RENDER_VARIANTS variants equal to c's
// position between the two (so the mean over the variants is c to within 1/32
// of their gap). Exactly representable and non-finite values are returned as
// they are.
__device__ float dither_round(double c, int v) {
  const float f = (float)c;
  if (!isfinite(f) || (double)f == c) return f;
  float lo, hi;
  if ((double)f < c) {
    lo = f;
    hi = nextafterf(f, __builtin_inff());
  } else {
    hi = f;
    lo = nextafterf(f, -__builtin_inff());
  }
  // hi - lo is a power of two, so the quotient is an exact scaling
  const double frac = ldexp(c - (double)lo, -ilogb((double)hi - (double)lo));
  return frac + ((v + 0.5) / RENDER_VARIANTS - 0.5) >= 0.5 ? hi : lo;
}

// Per system (one block each): the PSF normalised to unit sum in float64 and
// stored three ways (row-major; column-major flipped, the convolution's taps;
// column-major, the transpose's taps), and for the adjoint the 16 folded
// tables of the transposed convolution. For border class (cr, cc) (0 interior,
// 1 first, 2 last, 3 both, per axis) the entry at offset (a, b) sums the
// kernel over the offsets the replicate padding maps there: first -> offsets
// a..p, last -> -p..a, both -> all (only a = 0). Each such sum is a rectangle
// of a float64 summed-area table of the PSF.
// The normalisation by a block of T threads (part: T doubles of LDS); returns
// 1 / sum.
template <int T>
__device__ double psf_normalise(const SysDesc& sd, double* part) {
  const int n = sd.ph * sd.pw, t = (int)threadIdx.x;
  double acc = 0.0;
  for (int i = t; i < n; i += T) acc += (double)sd.psf[i];
  part[t] = acc;
  __syncthreads();
  for (int w = T / 2; w > 0; w >>= 1) {
    if (t < w) part[t] += part[t + w];
    __syncthreads();
  }
  const double inv = 1.0 / part[0];
  for (int i = t; i < n; i += T) {
    sd.psfn[i] = (float)((double)sd.psf[i] * inv);
    const int l = i / sd.ph, k = i - l * sd.ph;
    sd.psfn[n + i] = (float)((double)sd.psf[(sd.ph - 1 - k) * sd.pw + (sd.pw - 1 - l)] * inv);
    sd.psfn[2 * n + i] = (float)((double)sd.psf[k * sd.pw + l] * inv);
  }
  return inv;
}

// Launched before the prologue when the plan has the adjoint (the forward
// plans normalise in extra blocks of the prologue kernel instead, one launch
// fewer per call).
constexpr int PSF_PREP_THREADS = 256;
__global__ __launch_bounds__(PSF_PREP_THREADS) void psf_prepare_kernel(SysDesc single, SysDesc* __restrict__ table) {
  __shared__ double part[PSF_PREP_THREADS];
  __shared__ double sat[(MAX_PSF + 1) * (MAX_PSF + 1)];
  const SysDesc sd = table ? table[blockIdx.x] : single;
  const int n = sd.ph * sd.pw, t = (int)threadIdx.x;
  if (sd.ptile_w)   // the support kernels, which run next, mark the tiles with w > 0
    for (int i = t; i < sd.n_ptiles; i += PSF_PREP_THREADS) sd.ptile_w[i] = 0;
  const double inv = psf_normalise<PSF_PREP_THREADS>(sd, part);
  if (!sd.adjk) return;   // uniform over the block
  // summed-area table S[i][j] = sum of psf[a][b] over a < i, b < j: row sums, then column sums
  const int SW = sd.pw + 1;
  for (int i = t; i <= sd.ph; i += PSF_PREP_THREADS) {
    double r = 0.0;
    sat[i * SW] = 0.0;
    for (int j = 0; j < sd.pw; ++j) {
      if (i > 0) r += (double)sd.psf[(i - 1) * sd.pw + j];
      sat[i * SW + j + 1] = r;
    }
  }
  __syncthreads();
  for (int j = t; j <= sd.pw; j += PSF_PREP_THREADS) {
    double c = 0.0;
    for (int i = 0; i <= sd.ph; ++i) {
      c += sat[i * SW + j];
      sat[i * SW + j] = c;
    }
  }
  __syncthreads();
  const int p = sd.ph / 2, q = sd.pw / 2;
  for (int i = t; i < 16 * n; i += PSF_PREP_THREADS) {
    const int cls = i / n, e = i - cls * n;
    const int cr = cls >> 2, cc = cls & 3;
    const int a = e / sd.pw - p, b = e % sd.pw - q;
    int a0, a1, b0, b1;
    switch (cr) {
      case 0: a0 = a; a1 = a; break;
      case 1: a0 = a; a1 = a >= 0 ? p : a - 1; break;
      case 2: a0 = -p; a1 = a <= 0 ? a : -p - 1; break;
      default: a0 = -p; a1 = a == 0 ? p : -p - 1; break;
    }
    switch (cc) {
      case 0: b0 = b; b1 = b; break;
      case 1: b0 = b; b1 = b >= 0 ? q : b - 1; break;
      case 2: b0 = -q; b1 = b <= 0 ? b : -q - 1; break;
      default: b0 = -q; b1 = b == 0 ? q : -q - 1; break;
    }
    double sum = 0.0;
    if (a1 >= a0 && b1 >= b0) {
      if (a0 == a1 && b0 == b1) {
        sum = (double)sd.psf[(a0 + p) * sd.pw + (b0 + q)];   // a single tap, exactly
      } else {
        const int r0 = a0 + p, r1 = a1 + p + 1, c0 = b0 + q, c1 = b1 + q + 1;
        sum = (sat[r1 * SW + c1] - sat[r0 * SW + c1]) - (sat[r1 * SW + c0] - sat[r0 * SW + c0]);
      }
    }
    sd.adjk[i] = (float)(sum * inv);
  }
}

// One block of 64 threads covers PROLOGUE_POINTS points, PROLOGUE_LANES lanes
// each: first `solves` lanes of a point each find one root of P(2n, b) = 1/2
// (b_n of the lens and the source light; with the adjoint also b at n +- h for
// db_n/dn), then one lane derives the rest, and all the point's lanes share the
// 16 x 32 dithered roundings of the render variants. Extra blocks normalise
// the systems' PSFs.
constexpr int PROLOGUE_LANES = 16;
constexpr int PROLOGUE_POINTS = 64 / PROLOGUE_LANES;
__global__ __launch_bounds__(64) void prologue_kernel(const float* __restrict__ theta, int n_points,
                                                      PointConst* __restrict__ pcs, PointConst64* __restrict__ p64s,
                                                      GradConst* __restrict__ gcs, const SysDesc* __restrict__ table,
                                                      const int* __restrict__ point_sys, int* __restrict__ cusp_count,
                                                      double* __restrict__ grad_corr, SysDesc single, int solves,
                                                      int point_blocks) {
  if (cusp_count && blockIdx.x == 0 && threadIdx.x == 0) *cusp_count = 0;
  if ((int)blockIdx.x >= point_blocks) {   // PSF normalisation, one block per system
    __shared__ double part[64];
    const int s = blockIdx.x - point_blocks;
    psf_normalise<64>(table ? table[s] : single, part);
    return;
  }
  __shared__ double roots[64];
  __shared__ double folded[PROLOGUE_POINTS][32];
  const int pl = threadIdx.x / PROLOGUE_LANES, j = threadIdx.x % PROLOGUE_LANES;
  const int p = blockIdx.x * PROLOGUE_POINTS + pl;
  if (p >= n_points) return;   // no barrier below waits for these lanes' points
  float t[NPAR];
  bool valid = true;
  for (int k = 0; k < NPAR; ++k) {
    t[k] = theta[(size_t)p * NPAR + k];
    valid = valid && isfinite(t[k]);
  }
  valid = valid && ok_q(t[1]) && ok_q(t[8]) && ok_q(t[15]) && t[6] > 0.0f && t[13] > 0.0f && ok_n(t[7]) &&
          ok_n(t[14]);
  // roots: j = 0, 1: b_n of lens and source light; j = 2, 3 (4, 5): the same at n + h (n - h), h = 1e-5 n
  {
    double r = 0.0;
    if (valid && j < solves) {
      const double n = (j & 1) ? t[14] : t[7];
      r = j < 2 ? sersic_bn(n) : sersic_bn(j < 4 ? n + 1e-5 * n : n - 1e-5 * n);
    }
    roots[threadIdx.x] = r;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  const double* rt = roots + pl * PROLOGUE_LANES;
  if (j == 0) {   // the point's head, its float64 folded constants (to LDS) and the adjoint's constants
    PointHead c;
    const double te = t[0], q = t[1], phL = t[2], g = t[3], phg = t[4];
    c.cL = (float)cos(phL);
    c.sL = (float)sin(phL);
    const double s2 = (1.0 - q) * (1.0 + q);
    const double qp = sqrt(s2);
    c.q2 = (float)(q * q);
    c.qp = (float)qp;
    c.iq = (float)(1.0 / q);
    if (s2 == 0.0) {
      c.sie_mode = 0;
      c.kc = (float)te;
      c.ks = 0.0f;
    } else {
      c.sie_mode = qp <= 0.5 ? 1 : 2;
      const double k = te * sqrt(q) / qp;
      c.kc = (float)(k * cos(phL));
      c.ks = (float)(k * sin(phL));
    }
    const double g1 = g * cos(2.0 * phg), g2 = g * sin(2.0 * phg);
    c.m11 = (float)(1.0 - g1);
    c.m12 = (float)(-g2);
    c.m22 = (float)(1.0 + g1);

    const double bh = rt[0], bs = rt[1];
    // amplitudes: I_e given, or from total magnitudes (the point's system decides)
    const SysDesc* own = table ? &table[point_sys ? point_sys[p] : 0] : &single;
    const int amp = own->amp;
    double Ih = t[5], Is = t[12];
    AmpFromMag ah = {0.0, 0.0, 0.0, 0.0}, as = {0.0, 0.0, 0.0, 0.0};
    double dbh = 0.0, dbs = 0.0;
    if (valid && gcs) {
      // central differences of the root, truncation of order 1e-10 relative
      dbh = (rt[2] - rt[4]) / (2e-5 * (double)t[7]);
      dbs = (rt[3] - rt[5]) / (2e-5 * (double)t[14]);
    }
    if (valid && amp) {
      ah = amplitude_from_magnitude(t[5], t[6], t[7], bh, dbh, own->zp);
      as = amplitude_from_magnitude(t[12], t[13], t[14], bs, dbs, own->zp);
      Ih = ah.I;
      Is = as.I;
    }
    // source centre: given, or the image of an image-plane point (Sec. 5)
    const int srcpos = own->srcpos;
    double xs = t[10], ys = t[11];
    float jac[14] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    if (valid && srcpos) {
      const double v[7] = {t[10], t[11], t[0], t[1], t[2], t[3], t[4]};
      lens_map_f64(v, xs, ys);
      if (gcs) lens_map_jacobian(v, jac);
    }
    {
      const double Re = t[6], qh = t[8], ph = t[9];
      c.hc = (float)cos(ph);
      c.hs = (float)sin(ph);
      c.hqa = (float)(qh / (Re * Re));
      c.hqb = (float)(1.0 / (qh * Re * Re));
      c.he = (float)(0.5 / (double)t[7]);
      c.hB = (float)(bh * LOG2E);
      c.hI = (float)Ih;
    }
    {
      const double Re = t[13], qs = t[15], ph = t[16];
      c.sx0 = (float)xs;
      c.sy0 = (float)ys;
      c.sc = (float)cos(ph);
      c.ss = (float)sin(ph);
      c.sqa = (float)(qs / (Re * Re));
      c.sqb = (float)(1.0 / (qs * Re * Re));
      c.se = (float)(0.5 / (double)t[14]);
      c.sB = (float)(bs * LOG2E);
      c.sI = (float)Is;
    }
    // re-trace in float64 near a cuspy (n > 1) source centre (source-plane radius)
    {
      const double Re = t[13], rc = (srcpos ? CUSP_RADIUS_IMAGE_PLANE_ARCSEC : CUSP_RADIUS_ARCSEC) / Re;
      c.cusp_r2 = t[14] > 1.0f ? (float)(rc * rc) : 0.0f;
    }
    // folded constants of the forward render (float64), then their dithered
    // float32 roundings, one set per variant
    double tac = te, tas = 0.0, thc = 0.0, ths = 0.0;
    c.rmode = 0;
    for (int k = 0; k < 11; ++k) c.poly[k] = 0.0f;
    if (s2 != 0.0) {
      const double k = te * sqrt(q) / qp;
      const double fa = qp <= 0.5 ? 1.0 : 2.0, fh = qp <= 0.5 ? 1.0 : 0.693147180559945309417;
      c.rmode = qp <= 0.5 ? 1 : (q >= 0.5 ? 2 : 3);
      tac = fa * k * cos(phL);
      tas = fa * k * sin(phL);
      thc = fh * k * cos(phL);
      ths = fh * k * sin(phL);
      // deflection polynomials with q' folded in: coefficient j is c_j q'^(2j+1)
      const double qp2 = qp * qp;
      double pw = qp * qp2;
      if (c.rmode == 3) {
        for (int j = 1; j <= ATAN_UNIT_POLY_DEGREE; ++j, pw *= qp2) c.poly[j] = (float)(ATAN_UNIT_POLY_D[j] * pw);
      } else {
        for (int j = 1; j <= ATAN_SMALL_POLY_DEGREE; ++j, pw *= qp2) c.poly[j] = (float)(ATAN_SMALL_POLY_D[j] * pw);
      }
      if (c.rmode == 1) {
        pw = qp * qp2;
        for (int j = 1; j <= ATANH_POLY_DEGREE; ++j, pw *= qp2)
          c.poly[ATAN_SMALL_POLY_DEGREE + j] = (float)(ATANH_POLY_D[j] * pw);
      }
    }
    double f[32];
    for (int k = 0; k < 32; ++k) f[k] = 0.0;
    f[0] = cos(phL);
    f[1] = sin(phL);
    f[2] = q * q;
    f[3] = 1.0 / q;
    f[4] = qp;
    {
      const double Re = t[13], qs = t[15], ph = t[16];
      const double a = sqrt(qs) / Re, b = 1.0 / (sqrt(qs) * Re), cs = cos(ph), sn = sin(ph);
      const double s11 = a * cs, s12 = a * sn, s21 = -b * sn, s22 = b * cs;
      // the source frame of the lens equation in one step (float64 products, one rounding each)
      const double m11 = 1.0 - g1, m12 = -g2, m22 = 1.0 + g1;
      f[5] = s11 * m11 + s12 * m12;            // A1
      f[6] = s21 * m11 + s22 * m12;            // A2
      f[7] = s11 * m12 + s12 * m22;            // B1
      f[8] = s21 * m12 + s22 * m22;            // B2
      f[9] = -(s11 * xs + s12 * ys);           // C1
      f[10] = -(s21 * xs + s22 * ys);          // C2
      f[11] = -(s11 * tac + s12 * tas);        // cXt
      f[12] = s11 * ths - s12 * thc;           // cXh
      f[13] = -(s21 * tac + s22 * tas);        // cYt
      f[14] = s21 * ths - s22 * thc;           // cYh
      f[23] = s11;
      f[24] = s12;
      f[25] = s21;
      f[26] = s22;
    }
    {
      // lens light about the origin: R^2/R_e^2 = X^2 + Y^2 = (ha x + hb y) x + hc y^2
      const double Re = t[6], qh = t[8], ph = t[9];
      const double a = sqrt(qh) / Re, b = 1.0 / (sqrt(qh) * Re), cs = cos(ph), sn = sin(ph);
      const double h11 = a * cs, h12 = a * sn, h21 = -b * sn, h22 = b * cs;
      f[15] = h11 * h11 + h21 * h21;           // ha
      f[16] = 2.0 * (h11 * h12 + h21 * h22);   // hb
      f[17] = h12 * h12 + h22 * h22;           // hc
    }
    f[18] = 0.5 / (double)t[7];                // he
    f[19] = bh * LOG2E;                        // hB
    f[20] = 0.5 / (double)t[14];               // se
    f[21] = bs * LOG2E;                        // sB
    f[22] = tac;
    if (!valid) f[5] = f[6] = __builtin_nan("");
    for (int k = 0; k < 32; ++k) folded[pl][k] = f[k];
    c.hIlo = (float)(Ih - (double)c.hI);
    c.sIlo = (float)(Is - (double)c.sI);
    for (int k = 0; k < 22; ++k) c.pad[k] = 0.0f;
    if (!valid) {
      const float nan = __builtin_nanf("");
      c.m11 = c.m12 = c.m22 = nan;
      c.hI = c.sI = nan;
    }
    static_cast<PointHead&>(pcs[p]) = c;   // the variants are already in place
    if (p64s) {
      PointConst64 e;
      e.cL = cos(phL);
      e.sL = sin(phL);
      e.q2 = q * q;
      e.qp = qp;
      e.te = te;
      e.k = s2 == 0.0 ? te : te * sqrt(q) / qp;
      e.mode = s2 == 0.0 ? 0 : 1;
      e.pad0 = 0;
      e.m11 = 1.0 - g1;
      e.m12 = -g2;
      e.m22 = 1.0 + g1;
      e.sx0 = xs;
      e.sy0 = ys;
      for (int k = 0; k < 4; ++k) e.pad[k] = 0.0;
      if (!valid) e.m11 = e.m12 = e.m22 = __builtin_nan("");
      p64s[p] = e;
    }

    if (grad_corr)
      for (int k = 0; k < NPAR; ++k) grad_corr[(size_t)p * NPAR + k] = 0.0;
    if (gcs) {
      GradConst gc;
      for (int k = 0; k < NPAR; ++k) gc.theta[k] = t[k];
      gc.bh = (float)bh;
      gc.bs = (float)bs;
      gc.dB_dn_h = valid ? (float)(dbh * LOG2E) : __builtin_nanf("");
      gc.dB_dn_s = valid ? (float)(dbs * LOG2E) : __builtin_nanf("");
      gc.amp_chain[0] = (float)ah.dm;
      gc.amp_chain[1] = (float)ah.dR;
      gc.amp_chain[2] = (float)ah.dn;
      gc.amp_chain[3] = (float)as.dm;
      gc.amp_chain[4] = (float)as.dR;
      gc.amp_chain[5] = (float)as.dn;
      gc.amp = amp;
      for (int k = 0; k < 14; ++k) gc.src_jac[k] = jac[k];
      gc.srcpos = srcpos;
      GradUniform& u = gc.u;
      u.tesq = (float)(te * sqrt(q));
      u.iqp = s2 == 0.0 ? 0.0f : (float)(1.0 / qp);
      u.s = (float)s2;
      u.hs = s2 == 0.0 ? 0.0f : (float)(0.5 / s2);
      u.iq2 = (float)(1.0 / (q * q));
      u.bH = (float)bh;
      u.bS = (float)bs;
      u.dbH = (float)dbh;
      u.dbS = (float)dbs;
      u.kS1 = (float)cos((double)t[16] - phL);
      u.kS2 = (float)sin((double)t[16] - phL);
      for (int k = 0; k < 10; ++k) gc.pad[k] = 0.0f;
      gcs[p] = gc;
    }
  }
  // the dithered float32 roundings of the folded constants, one set per render
  // variant: lane j of the point rounds constants j and j + 16
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  for (int k = j; k < 32; k += PROLOGUE_LANES) {
    const double fk = folded[pl][k];
    for (int v = 0; v < RENDER_VARIANTS; ++v) reinterpret_cast<float*>(&pcs[p].rv[v])[k] = dither_round(fk, v);
  }
}

}  // namespace

// General models: one thread per point turns its parameters (layout of
// lensed_model: per SIE x_c, y_c, theta_E, q, phi; shear gamma, phi_gamma; per
// Sersic x, y, I_e, R_e, n, q, phi; sky) into ModelConst; model_bn_kernel
// then adds the b_n roots. An invalid point gets sky = NaN, which makes its
// image NaN.
__global__ __launch_bounds__(64) void model_prologue_kernel(const float* __restrict__ theta, int n_points, int n_params, ModelSpec spec,
                                      ModelConst* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_points) return;
  const float* t = theta + (size_t)p * n_params;
  bool valid = true;
  for (int i = 0; i < n_params; ++i) valid = valid && isfinite(t[i]);
  ModelConst& m = out[p];   // written in place (a local copy would live in scratch)
  m.n_sie = spec.n_sie;
  m.n_sersic = spec.n_sersic;
  int o = 0;
  for (int k = 0; k < MAX_SIE; ++k) {
    for (int i = 0; i < 9; ++i) m.sie[k][i] = 0.0;
    m.sie_sphere[k] = 0;
    if (k >= spec.n_sie) continue;
    const double te = t[o + 2], q = t[o + 3], ph = t[o + 4];
    valid = valid && q > 0.0 && q <= 1.0;
    const double s2 = (1.0 - q) * (1.0 + q), qp = sqrt(fmax(s2, 0.0));
    m.sie[k][0] = t[o];
    m.sie[k][1] = t[o + 1];
    m.sie[k][2] = cos(ph);
    m.sie[k][3] = sin(ph);
    m.sie[k][4] = q * q;
    m.sie[k][5] = qp;
    m.sie_sphere[k] = s2 == 0.0;
    m.sie[k][6] = s2 == 0.0 ? te : te * sqrt(q) / qp;
    m.sie[k][7] = te;
    m.sie[k][8] = q;
    o += 5;
  }
  m.g1 = m.g2 = m.gam = m.c2g = m.s2g = 0.0;
  if (spec.shear) {
    m.gam = t[o];
    m.c2g = cos(2.0 * (double)t[o + 1]);
    m.s2g = sin(2.0 * (double)t[o + 1]);
    m.g1 = m.gam * m.c2g;
    m.g2 = m.gam * m.s2g;
    o += 2;
  }
  for (int j = 0; j < MAX_SERSIC; ++j) {
    for (int i = 0; i < 11; ++i) m.ser[j][i] = 0.0;
    m.plane[j] = 0;
    if (j >= spec.n_sersic) continue;
    const double Re = t[o + 3], n = t[o + 4], q = t[o + 5], ph = t[o + 6];
    valid = valid && Re > 0.0 && n >= 0.2 && n <= 10.0 && q > 0.0 && q <= 1.0;
    m.plane[j] = spec.plane[j];
    m.ser[j][0] = t[o];
    m.ser[j][1] = t[o + 1];
    m.ser[j][2] = cos(ph);
    m.ser[j][3] = sin(ph);
    m.ser[j][4] = q;
    m.ser[j][5] = 1.0 / q;
    m.ser[j][6] = 1.0 / Re;
    m.ser[j][7] = 1.0 / n;
    m.ser[j][9] = t[o + 2];   // b_n (slot 8) and db_n/dn (slot 10): model_bn_kernel
    o += 7;
  }
  m.sky = spec.sky ? (double)t[o] : 0.0;
  if (!valid) m.sky = __builtin_nan("");
}

// b_n of every Sersic of every valid point, one root solve per thread: lane
// c of a block is a (point, component) pair, and with with_db the block's
// second and third waves solve at n (1 +- 1e-5) for db_n/dn by central
// differences (truncation of order 1e-10 relative). Runs after
// model_prologue_kernel, whose NaN sky marks the invalid points.
constexpr int MODEL_BN_PAIRS = 64;
__global__ __launch_bounds__(3 * MODEL_BN_PAIRS) void model_bn_kernel(const float* __restrict__ theta, int n_points,
                                                                     int n_params, ModelSpec spec,
                                                                     ModelConst* __restrict__ out) {
  __shared__ double root[3][MODEL_BN_PAIRS];
  const int c = (int)(threadIdx.x % MODEL_BN_PAIRS), v = (int)(threadIdx.x / MODEL_BN_PAIRS);
  const int64_t pair = (int64_t)blockIdx.x * MODEL_BN_PAIRS + c;
  const bool live = pair < (int64_t)n_points * spec.n_sersic;
  const int p = live ? (int)(pair / spec.n_sersic) : 0, j = live ? (int)(pair % spec.n_sersic) : 0;
  const bool valid = live && !isnan(out[p].sky);
  const int o = 5 * spec.n_sie + (spec.shear ? 2 : 0) + 7 * j;
  const double n = valid ? (double)theta[(size_t)p * n_params + o + 4] : 1.0;
  if (valid) root[v][c] = sersic_bn(v == 0 ? n : (v == 1 ? n + 1e-5 * n : n - 1e-5 * n));
  __syncthreads();
  if (!valid || v != 0) return;
  out[p].ser[j][8] = root[0][c];
  if (blockDim.x == 3 * MODEL_BN_PAIRS) out[p].ser[j][10] = (root[1][c] - root[2][c]) / (2e-5 * n);
}

hipError_t launch_model_prologue(const float* theta, int n_points, int n_params, const ModelSpec& spec,
                                 ModelConst* out, hipStream_t stream, bool with_db) {
  if (n_points <= 0) return hipSuccess;
  hipLaunchKernelGGL(model_prologue_kernel, dim3((n_points + 63) / 64), dim3(64), 0, stream, theta, n_points, n_params,
                     spec, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || spec.n_sersic <= 0) return e;
  const int64_t pairs = (int64_t)n_points * spec.n_sersic;
  hipLaunchKernelGGL(model_bn_kernel, dim3((unsigned)((pairs + MODEL_BN_PAIRS - 1) / MODEL_BN_PAIRS)),
                     dim3(with_db ? 3 * MODEL_BN_PAIRS : MODEL_BN_PAIRS), 0, stream, theta, n_points, n_params, spec, out);
  return hipGetLastError();
}

hipError_t launch_prologue(const float* theta, int n_points, PointConst* pcs, PointConst64* p64s, GradConst* gcs,
                           const SysDesc& single, SysDesc* table, int n_sys, int* cusp_count, hipStream_t stream,
                           double* grad_corr, const int* point_sys, bool adjoint_tables) {
  const int threads = 64;
  const int solves = gcs ? 6 : 2;
  const int ppb = PROLOGUE_POINTS;
  const int point_blocks = (n_points + ppb - 1) / ppb;
  // with the adjoint the PSF also gets its folded tables, in a kernel of its own
  const bool prep = adjoint_tables && n_sys > 0;
  if (prep) {
    hipLaunchKernelGGL(psf_prepare_kernel, dim3(n_sys), dim3(PSF_PREP_THREADS), 0, stream, single, table);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int blocks = point_blocks + (prep ? 0 : n_sys);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(prologue_kernel, dim3(blocks), dim3(threads), 0, stream, theta, n_points, pcs,
                     p64s, gcs, table, point_sys, cusp_count, grad_corr, single, solves, point_blocks);
  return hipGetLastError();
}

}  // namespace lensed
