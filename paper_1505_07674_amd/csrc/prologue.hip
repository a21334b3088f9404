// prologue.hip -- per-point derived constants and PSF normalisation.
//
// One thread per parameter point turns the 17 float32 parameters into the
// wave-uniform constants the render kernels consume (trigonometry, the shear
// matrix, reciprocal radii and the Sersic b_n). b_n is the root of
// P(2n, b) = 1/2 (R_e is the half-light radius, Sec. 4.1 Eq. 22), solved here in
// float64 by a bracketed Newton iteration on the power series of the
// regularised incomplete gamma function. Extra blocks normalise each system's
// PSF to unit sum (Sec. 3.1).
#include <math.h>

#include "internal.h"
#include "kernels.h"

namespace lensed {
namespace {

// Root of P(a, b) = 1/2 by Newton's method, safeguarded by bisection, from the
// start b0. P(a, x) = x^a e^{-x} / Gamma(a+1) * (1 + x/(a+1) + x^2/((a+1)(a+2)) + ...)
// and dP/dx = x^{a-1} e^{-x} / Gamma(a) = (x^a e^{-x} / Gamma(a+1)) a / x.
__device__ double gamma_median(double a, double b0) {
  const double lga1 = lgamma(a + 1.0);
  double lo = 0.0, hi = a + 40.0;
  double b = (b0 > lo && b0 < hi) ? b0 : 0.5 * a + 1e-3;
  for (int it = 0; it < 100; ++it) {
    const double pref = exp(a * log(b) - b - lga1);
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 600; ++k) {
      term *= b / (a + (double)k);
      sum += term;
      if (term <= 1e-17 * sum) break;
    }
    const double f = pref * sum - 0.5;
    if (f > 0.0) hi = b; else lo = b;
    double nb = b - f * b / (pref * a);
    if (!(nb > lo && nb < hi)) nb = 0.5 * (lo + hi);
    const double step = fabs(nb - b);
    b = nb;
    if (step <= 4e-16 * b) break;
  }
  return b;
}

// b_n (R_e is the half-light radius, Sec. 4.1 Eq. 22), started from the
// asymptotic expansion of Ciotti & Bertin (1999): within 4e-4 for n >= 0.5 and
// within 2e-3 at n = 0.3, so Newton needs two or three steps.
__device__ double sersic_bn(double n) {
  const double in = 1.0 / n;
  const double b0 = 2.0 * n - 1.0 / 3.0 +
                    in * (4.0 / 405.0 + in * (46.0 / 25515.0 + in * (131.0 / 1148175.0 - in * (2194697.0 / 30690717750.0))));
  return gamma_median(2.0 * n, b0);
}

// d b_n / dn by a central difference of the root with h = 1e-5 n (truncation
// of order 1e-10 times the third derivative, rounding of order 1e-11), each
// side started from the converged b_n.
__device__ double sersic_bn_deriv(double n, double b) {
  const double h = 1e-5 * n;
  return (gamma_median(2.0 * (n + h), b + 2.0 * h) - gamma_median(2.0 * (n - h), b - 2.0 * h)) / (2.0 * h);
}

__device__ bool ok_q(float q) { return q > 0.0f && q <= 1.0f; }
__device__ bool ok_n(float n) { return n >= 0.2f && n <= 10.0f; }

__global__ void prologue_kernel(const float* __restrict__ theta, int n_points, PointConst* __restrict__ pcs,
                                PointConst64* __restrict__ p64s, GradConst* __restrict__ gcs, SysDesc single,
                                SysDesc* __restrict__ table, int n_sys, int point_blocks, int* __restrict__ cusp_count,
                                double* __restrict__ grad_corr) {
  if (cusp_count && blockIdx.x == 0 && threadIdx.x == 0) *cusp_count = 0;
  if ((int)blockIdx.x >= point_blocks) {
    // PSF normalisation: one block per system, float64 sum over the array.
    const int s = blockIdx.x - point_blocks;
    const SysDesc sd = table ? table[s] : single;
    const int n = sd.ph * sd.pw;
    __shared__ double part[64];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += (double)sd.psf[i];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
      __syncthreads();
    }
    const double inv = 1.0 / part[0];
    // three copies: row-major; column-major flipped (the convolution's taps, column
    // l = KW-1-b, row k = KH-1-a for entry (a, b)); column-major (the transpose's taps)
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      sd.psfn[i] = (float)((double)sd.psf[i] * inv);
      const int l = i / sd.ph, k = i - l * sd.ph;
      sd.psfn[n + i] = (float)((double)sd.psf[(sd.ph - 1 - k) * sd.pw + (sd.pw - 1 - l)] * inv);
      sd.psfn[2 * n + i] = (float)((double)sd.psf[k * sd.pw + l] * inv);
    }
    if (sd.adjk) {
      // Folded tables of the transposed convolution: for border class (cr, cc)
      // (0 interior, 1 first, 2 last, 3 both, per axis) the entry at offset (a, b)
      // sums the normalised kernel over the offsets the replicate padding maps
      // there: first -> offsets a..p, last -> -p..a, both -> all (only a = 0).
      const int p = sd.ph / 2, q = sd.pw / 2;
      for (int i = threadIdx.x; i < 16 * n; i += blockDim.x) {
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
        double acc = 0.0;
        for (int aa = a0; aa <= a1; ++aa)
          for (int bb = b0; bb <= b1; ++bb) acc += (double)sd.psf[(aa + p) * sd.pw + (bb + q)];
        sd.adjk[i] = (float)(acc * inv);
      }
    }
    return;
  }
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_points) return;
  float t[NPAR];
  bool valid = true;
  for (int k = 0; k < NPAR; ++k) {
    t[k] = theta[(size_t)p * NPAR + k];
    valid = valid && isfinite(t[k]);
  }
  valid = valid && ok_q(t[1]) && ok_q(t[8]) && ok_q(t[15]) && t[6] > 0.0f && t[13] > 0.0f && ok_n(t[7]) &&
          ok_n(t[14]);

  PointConst c;
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

  double bh = 0.0, bs = 0.0;
  if (valid) {
    bh = sersic_bn(t[7]);
    bs = sersic_bn(t[14]);
  }
  {
    const double Re = t[6], qh = t[8], ph = t[9];
    c.hc = (float)cos(ph);
    c.hs = (float)sin(ph);
    c.hqa = (float)(qh / (Re * Re));
    c.hqb = (float)(1.0 / (qh * Re * Re));
    c.he = (float)(0.5 / (double)t[7]);
    c.hB = (float)(bh * LOG2E);
    c.hI = t[5];
  }
  {
    const double Re = t[13], qs = t[15], ph = t[16];
    c.sx0 = t[10];
    c.sy0 = t[11];
    c.sc = (float)cos(ph);
    c.ss = (float)sin(ph);
    c.sqa = (float)(qs / (Re * Re));
    c.sqb = (float)(1.0 / (qs * Re * Re));
    c.se = (float)(0.5 / (double)t[14]);
    c.sB = (float)(bs * LOG2E);
    c.sI = t[12];
  }
  // re-trace in float64 within 0.03 arcsec (source plane) of a cuspy (n > 1) source centre
  {
    const double Re = t[13], rc = CUSP_RADIUS_ARCSEC / Re;
    c.cusp_r2 = t[14] > 1.0f ? (float)(rc * rc) : 0.0f;
  }
  for (int k = 0; k < 4; ++k) c.pad[k] = 0.0f;
  // folded constants of the forward render
  double tac = te, tas = 0.0, thc = 0.0, ths = 0.0;
  c.rmode = 0;
  if (s2 != 0.0) {
    const double k = te * sqrt(q) / qp;
    const double fa = qp <= 0.5 ? 1.0 : 2.0, fh = qp <= 0.5 ? 1.0 : 0.693147180559945309417;
    c.rmode = qp <= 0.5 ? 1 : (q >= 0.5 ? 2 : 3);
    tac = fa * k * cos(phL);
    tas = fa * k * sin(phL);
    thc = fh * k * cos(phL);
    ths = fh * k * sin(phL);
  }
  c.tac = (float)tac;
  c.tas = (float)tas;
  c.thc = (float)thc;
  c.ths = (float)ths;
  {
    const double Re = t[6], qh = t[8], ph = t[9];
    const double a = sqrt(qh) / Re, b = 1.0 / (sqrt(qh) * Re), cs = cos(ph), sn = sin(ph);
    c.h11 = (float)(a * cs);
    c.h12 = (float)(a * sn);
    c.h21 = (float)(-b * sn);
    c.h22 = (float)(b * cs);
  }
  {
    const double Re = t[13], qs = t[15], ph = t[16];
    const double a = sqrt(qs) / Re, b = 1.0 / (sqrt(qs) * Re), cs = cos(ph), sn = sin(ph);
    const double s11 = a * cs, s12 = a * sn, s21 = -b * sn, s22 = b * cs;
    c.s11 = (float)s11;
    c.s12 = (float)s12;
    c.s21 = (float)s21;
    c.s22 = (float)s22;
    // the source frame of the lens equation in one step (float64 products, one rounding each)
    const double m11 = 1.0 - g1, m12 = -g2, m22 = 1.0 + g1, xs = t[10], ys = t[11];
    c.A1 = (float)(s11 * m11 + s12 * m12);
    c.A2 = (float)(s21 * m11 + s22 * m12);
    c.B1 = (float)(s11 * m12 + s12 * m22);
    c.B2 = (float)(s21 * m12 + s22 * m22);
    c.C1 = (float)(-(s11 * xs + s12 * ys));
    c.C2 = (float)(-(s21 * xs + s22 * ys));
    c.cXt = (float)(-(s11 * tac + s12 * tas));
    c.cXh = (float)(s11 * ths - s12 * thc);
    c.cYt = (float)(-(s21 * tac + s22 * tas));
    c.cYh = (float)(s21 * ths - s22 * thc);
  }
  for (int k = 0; k < 9; ++k) c.pad2[k] = 0.0f;
  if (!valid) {
    const float nan = __builtin_nanf("");
    c.m11 = c.m12 = c.m22 = nan;
    c.hI = c.sI = nan;
    c.A1 = c.A2 = nan;
  }
  pcs[p] = c;
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
    e.sx0 = t[10];
    e.sy0 = t[11];
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
    gc.dB_dn_h = valid ? (float)(sersic_bn_deriv(t[7], bh) * LOG2E) : __builtin_nanf("");
    gc.dB_dn_s = valid ? (float)(sersic_bn_deriv(t[14], bs) * LOG2E) : __builtin_nanf("");
    for (int k = 0; k < 11; ++k) gc.pad[k] = 0.0f;
    gcs[p] = gc;
  }
}

}  // namespace

hipError_t launch_prologue(const float* theta, int n_points, PointConst* pcs, PointConst64* p64s, GradConst* gcs,
                           const SysDesc& single, SysDesc* table, int n_sys, int* cusp_count, hipStream_t stream,
                           double* grad_corr) {
  const int threads = 64;
  const int point_blocks = (n_points + threads - 1) / threads;
  const int blocks = point_blocks + n_sys;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(prologue_kernel, dim3(blocks), dim3(threads), 0, stream, theta, n_points, pcs, p64s, gcs,
                     single, table, n_sys, point_blocks, cusp_count, grad_corr);
  return hipGetLastError();
}

}  // namespace lensed
