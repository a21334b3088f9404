// lensed_oracle.cpp -- TEST INFRASTRUCTURE, not part of the product.
//
// A plain, serial, double-precision CPU implementation of the forward model and
// likelihood of Tessore, Bellagamba & Metcalf, "LENSED: a code for the forward
// reconstruction of lenses and sources from strong lensing observations"
// (MNRAS 2016). It exists only to check the GPU library: the test-suite, the
// smoke check and the CPU-baseline leg of the benchmark may load it; nothing in
// the product path may. It shares no code with the GPU library.
//
// Every step is written as its definition, with no blocking, fusion or reordering:
//   lens equation                      Sec. 2.1, Eq. (1)
//   image-plane surface brightness     Sec. 2.1, Eq. (2)
//   pixel luminosity and quadrature    Sec. 2.1 Eq. (3), Sec. 3.1 Eq. (14); N x N
//                                      midpoint subsampling (the "subN" rules, Sec. 4.5)
//   PSF convolution, replicate padding Sec. 3.1, Eq. (15)
//   log-likelihood with weights        Sec. 3.2, Eq. (17)
//   Sersic profile, geometric radius   Sec. 4.1, Eqs. (22)-(23)
//   singular isothermal ellipsoid      Sec. 4 (Kormann et al. 1994; formula not printed
//                                      in the paper, area-preserving convention)
//   external shear                     Sec. 5 / Table 4 (formula not printed)
//   amplitude from a total magnitude   Sec. 4.1 (I_0 set by the total magnitude)
//   image-plane source position        Sec. 5 (a position on the image plane mapped
//                                      to the source plane by the lens equation)
//
// The gradient of the log-likelihood is obtained by running the very same
// templated code on forward-mode dual numbers carrying 17 partial derivatives.
//
// Parameter vector (17 values), lens centred on the coordinate origin:
//   0 theta_E  1 q_L  2 phi_L  3 gamma  4 phi_gamma
//   5 I_H  6 R_H  7 n_H  8 q_H  9 phi_H                       (lens light at the origin)
//  10 x_S 11 y_S 12 I_S 13 R_S 14 n_S 15 q_S 16 phi_S          (source)
// Angles are counter-clockwise from +x to the major axis (Sec. 4).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

namespace {

constexpr int NPAR = 17;

// ---------------------------------------------------------------------------
// Forward-mode dual number: value and the 17 partial derivatives.
// ---------------------------------------------------------------------------
struct Dual {
  double v;
  double d[NPAR];
  Dual() : v(0) { for (int i = 0; i < NPAR; ++i) d[i] = 0; }
  Dual(double x) : v(x) { for (int i = 0; i < NPAR; ++i) d[i] = 0; }
  static Dual var(double x, int k) { Dual r(x); r.d[k] = 1; return r; }
};

inline double value(double x) { return x; }
inline double value(const Dual& x) { return x.v; }

// chain rule helper: f(a) with f'(a) = fp
inline Dual chain(const Dual& a, double f, double fp) {
  Dual r(f);
  for (int i = 0; i < NPAR; ++i) r.d[i] = fp * a.d[i];
  return r;
}

inline Dual operator+(const Dual& a, const Dual& b) {
  Dual r(a.v + b.v); for (int i = 0; i < NPAR; ++i) r.d[i] = a.d[i] + b.d[i]; return r;
}
inline Dual operator-(const Dual& a, const Dual& b) {
  Dual r(a.v - b.v); for (int i = 0; i < NPAR; ++i) r.d[i] = a.d[i] - b.d[i]; return r;
}
inline Dual operator-(const Dual& a) {
  Dual r(-a.v); for (int i = 0; i < NPAR; ++i) r.d[i] = -a.d[i]; return r;
}
inline Dual operator*(const Dual& a, const Dual& b) {
  Dual r(a.v * b.v); for (int i = 0; i < NPAR; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r;
}
inline Dual operator/(const Dual& a, const Dual& b) {
  Dual r(a.v / b.v);
  for (int i = 0; i < NPAR; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
  return r;
}
inline Dual operator+(const Dual& a, double b) { return a + Dual(b); }
inline Dual operator+(double a, const Dual& b) { return Dual(a) + b; }
inline Dual operator-(const Dual& a, double b) { return a - Dual(b); }
inline Dual operator-(double a, const Dual& b) { return Dual(a) - b; }
inline Dual operator*(const Dual& a, double b) { return a * Dual(b); }
inline Dual operator*(double a, const Dual& b) { return Dual(a) * b; }
inline Dual operator/(const Dual& a, double b) { return a / Dual(b); }
inline Dual operator/(double a, const Dual& b) { return Dual(a) / b; }

inline Dual sqrt(const Dual& a) { double s = std::sqrt(a.v); return chain(a, s, 0.5 / s); }
inline Dual exp(const Dual& a) { double e = std::exp(a.v); return chain(a, e, e); }
inline Dual log(const Dual& a) { return chain(a, std::log(a.v), 1.0 / a.v); }
inline Dual sin(const Dual& a) { return chain(a, std::sin(a.v), std::cos(a.v)); }
inline Dual cos(const Dual& a) { return chain(a, std::cos(a.v), -std::sin(a.v)); }
inline Dual atan(const Dual& a) { return chain(a, std::atan(a.v), 1.0 / (1.0 + a.v * a.v)); }
inline Dual atanh(const Dual& a) { return chain(a, std::atanh(a.v), 1.0 / (1.0 - a.v * a.v)); }
double digamma(double z);
inline double lgamma_of(double a) { return std::lgamma(a); }
inline Dual lgamma_of(const Dual& a) { return chain(a, std::lgamma(a.v), digamma(a.v)); }

// ---------------------------------------------------------------------------
// Special functions used by the Sersic normalisation b_n.
// ---------------------------------------------------------------------------

// Digamma psi(z), z > 0: upward recurrence psi(z) = psi(z+1) - 1/z until z >= 10,
// then the asymptotic series of Abramowitz & Stegun 6.3.18.
double digamma(double z) {
  double acc = 0.0;
  while (z < 10.0) { acc -= 1.0 / z; z += 1.0; }
  const double z2 = 1.0 / (z * z);
  // B2/2 = 1/12, B4/4 = -1/120, B6/6 = 1/252, B8/8 = -1/240, B10/10 = 1/132, B12/12 = -691/32760
  const double series = z2 * (1.0 / 12 - z2 * (1.0 / 120 - z2 * (1.0 / 252 - z2 * (1.0 / 240 - z2 * (1.0 / 132 - z2 * (691.0 / 32760))))));
  return acc + std::log(z) - 0.5 / z - series;
}

// Regularised lower incomplete gamma function P(a, x) by its power series
//   P(a,x) = e^{-x} x^a / Gamma(a+1) * sum_{k>=0} x^k / ((a+1)(a+2)...(a+k)).
// Also returns dP/da through the term-wise derivative
//   d/da log(term_k) = log x - psi(a+1) - sum_{j=1..k} 1/(a+j).
double gamma_p_series(double a, double x, double* dP_da) {
  if (x <= 0.0) { if (dP_da) *dP_da = 0.0; return 0.0; }
  const double pref = std::exp(-x + a * std::log(x) - std::lgamma(a + 1.0));
  const double lx = std::log(x), psi1 = digamma(a + 1.0);
  double term = 1.0, sum = 1.0;          // term_k / pref
  double hsum = 0.0;                     // sum_{j=1..k} 1/(a+j)
  double dsum = (lx - psi1);             // sum_k term_k * dlog(term_k)/da
  for (int k = 1; k < 100000; ++k) {
    term *= x / (a + k);
    hsum += 1.0 / (a + k);
    sum += term;
    dsum += term * (lx - psi1 - hsum);
    if (term < 1e-18 * sum) break;
  }
  if (dP_da) *dP_da = pref * dsum;
  return pref * sum;
}

// b_n: the root of P(2n, b) = 1/2, i.e. the constant that makes R_e the
// half-light radius of the Sersic profile (Sec. 4.1, Eq. 22). Newton's method on
// the series above, safeguarded by bisection, started from the leading terms of
// the Ciotti & Bertin (1999) asymptotic expansion.
double bn_exact(double n) {
  const double a = 2.0 * n;
  double lo = 0.0, hi = a + 20.0 + 10.0 * std::sqrt(a);
  double b = 2.0 * n - 1.0 / 3.0 + 4.0 / (405.0 * n) + 46.0 / (25515.0 * n * n);
  if (!(b > lo && b < hi)) b = 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    const double f = gamma_p_series(a, b, nullptr) - 0.5;
    if (f < 0) lo = b; else hi = b;
    const double fp = std::exp((a - 1.0) * std::log(b) - b - std::lgamma(a));
    double bn = b - f / fp;
    if (!(bn > lo && bn < hi)) bn = 0.5 * (lo + hi);
    const double step = std::fabs(bn - b);
    b = bn;
    if (step <= 1e-15 * b) break;
  }
  return b;
}

// db_n/dn by implicit differentiation of P(2n, b_n) = 1/2:
//   2 dP/da + dP/dx * db/dn = 0,  dP/dx = x^{a-1} e^{-x} / Gamma(a).
double bn_derivative(double n, double b) {
  const double a = 2.0 * n;
  double dPda = 0.0;
  gamma_p_series(a, b, &dPda);
  const double dPdx = std::exp((a - 1.0) * std::log(b) - b - std::lgamma(a));
  return -2.0 * dPda / dPdx;
}

inline double bn_of(double n) { return bn_exact(n); }
inline Dual bn_of(const Dual& n) {
  const double b = bn_exact(n.v);
  return chain(n, b, bn_derivative(n.v, b));
}

// ---------------------------------------------------------------------------
// Model components.
// ---------------------------------------------------------------------------

// atan(sqrt(s) u)/sqrt(s) and atanh(sqrt(s) v)/sqrt(s) with s = q'^2 = 1 - q^2.
// For small s the Taylor series in s is used, which is smooth through s = 0 (the
// singular isothermal sphere); the two forms agree to rounding at the switch.
template <class T> T atan_over(T s, T u) {
  using std::atan; using std::sqrt;
  if (value(s) >= 1e-4) { T r = sqrt(s); return atan(r * u) / r; }
  T z = s * u * u, acc = T(0.0), pw = T(1.0);
  for (int k = 0; k < 12; ++k) { acc = acc + pw / double(2 * k + 1); pw = pw * (-1.0) * z; }
  return u * acc;
}
template <class T> T atanh_over(T s, T v) {
  using std::atanh; using std::sqrt;
  if (value(s) >= 1e-4) { T r = sqrt(s); return atanh(r * v) / r; }
  T z = s * v * v, acc = T(0.0), pw = T(1.0);
  for (int k = 0; k < 12; ++k) { acc = acc + pw / double(2 * k + 1); pw = pw * z; }
  return v * acc;
}

// Deflection of a singular isothermal ellipsoid centred on the origin, with
// convergence kappa = theta_E / (2 sqrt(q x'^2 + y'^2/q)) in the frame rotated by
// phi (counter-clockwise from +x to the major axis):
//   psi = sqrt(q^2 x'^2 + y'^2),  q' = sqrt(1 - q^2)
//   alpha'_x = theta_E sqrt(q)/q' atan(q' x'/psi),  alpha'_y = theta_E sqrt(q)/q' atanh(q' y'/psi)
// rotated back to the image frame. At psi = 0 the deflection is set to zero.
template <class T> void sie_deflection(T te, T q, T phi, T x, T y, T& ax, T& ay) {
  using std::cos; using std::sin; using std::sqrt;
  const T c = cos(phi), s = sin(phi);
  const T xp = c * x + s * y, yp = -s * x + c * y;
  const T psi = sqrt(q * q * xp * xp + yp * yp);
  if (value(psi) == 0.0) { ax = T(0.0); ay = T(0.0); return; }
  const T s2 = 1.0 - q * q;
  const T k = te * sqrt(q);
  const T axp = k * atan_over(s2, xp / psi);
  const T ayp = k * atanh_over(s2, yp / psi);
  ax = c * axp - s * ayp;
  ay = s * axp + c * ayp;
}

// External shear about the lens centre: gamma_1 = gamma cos(2 phi), gamma_2 = gamma sin(2 phi),
// alpha = (gamma_1 x + gamma_2 y, gamma_2 x - gamma_1 y).
template <class T> void shear_deflection(T g, T phi, T x, T y, T& ax, T& ay) {
  using std::cos; using std::sin;
  const T g1 = g * cos(2.0 * phi), g2 = g * sin(2.0 * phi);
  ax = g1 * x + g2 * y;
  ay = g2 * x - g1 * y;
}

// Elliptical Sersic profile (Sec. 4.1, Eqs. 22-23), amplitude I_e at the
// half-light "radius" R_e, centred on (x0, y0) and rotated by phi:
//   R = sqrt(q x'^2 + y'^2/q),  I = I_e exp(-b_n [(R/R_e)^{1/n} - 1]),
// with b = b_n passed in (it depends on n only, so it is solved once per point).
template <class T> T sersic(T x, T y, T x0, T y0, T Ie, T Re, T n, T q, T phi, T b) {
  using std::cos; using std::sin; using std::sqrt; using std::exp; using std::log;
  const T dx = x - x0, dy = y - y0;
  const T c = cos(phi), s = sin(phi);
  const T xp = c * dx + s * dy, yp = -s * dx + c * dy;
  const T R2 = q * xp * xp + yp * yp / q;
  if (value(R2) == 0.0) return Ie * exp(b);
  const T R = sqrt(R2);
  const T t = exp(log(R / Re) / n);   // (R/R_e)^{1/n}
  return Ie * exp(-b * (t - 1.0));
}

template <class T> struct Params {
  T p[NPAR];
  T b_lens, b_src;   // b_n of the lens light and of the source
};

// Amplitude I_e of a Sersic component of total magnitude m (zero point zp: a
// component of magnitude zp has unit total flux). The map (x', y') ->
// (sqrt(q) x', y'/sqrt(q)) has unit Jacobian, so the elliptical profile has the
// flux of the circular one: F = int_0^inf I(R) 2 pi R dR
//   = 2 pi n R_e^2 I_e e^{b_n} Gamma(2n) / b_n^{2n}   (Sec. 4.1, Eq. 22),
// and F = 10^{-0.4 (m - zp)}. Written as one exponential of the logarithms.
template <class T> T intensity_from_magnitude(T m, T Re, T n, T b, double zp) {
  using std::exp; using std::log;
  const double pi = 3.14159265358979323846;
  const T lnF = (m - zp) * (-0.4 * std::log(10.0));
  return exp(lnF + 2.0 * n * log(b) - std::log(2.0 * pi) - log(n) - 2.0 * log(Re) - b - lgamma_of(2.0 * n));
}

// Parameters of a point; with magnitudes (amplitude != 0) the two amplitude
// slots 5 and 12 hold total magnitudes and are replaced by I_e; with an
// image-plane source position (srcpos != 0) slots 10 and 11 hold a point x_I of
// the image plane, and the source centre is its image under the lens equation,
// beta = x_I - alpha_SIE(x_I) - alpha_shear(x_I) (Eq. 1).
template <class T> Params<T> make_params(const T* th, int amplitude = 0, double zp = 0.0, int srcpos = 0) {
  Params<T> P;
  for (int i = 0; i < NPAR; ++i) P.p[i] = th[i];
  P.b_lens = bn_of(P.p[7]);
  P.b_src = bn_of(P.p[14]);
  if (amplitude) {
    P.p[5] = intensity_from_magnitude(th[5], th[6], th[7], P.b_lens, zp);
    P.p[12] = intensity_from_magnitude(th[12], th[13], th[14], P.b_src, zp);
  }
  if (srcpos) {
    T ax, ay, gx, gy;
    sie_deflection(th[0], th[1], th[2], th[10], th[11], ax, ay);
    shear_deflection(th[3], th[4], th[10], th[11], gx, gy);
    P.p[10] = th[10] - ax - gx;
    P.p[11] = th[11] - ay - gy;
  }
  return P;
}

// Surface brightness of the image plane at x (Eq. 2): lens light at x plus the
// source at the position given by the lens equation (Eq. 1).
template <class T> T surface_brightness(const Params<T>& P, T x, T y) {
  const T* p = P.p;
  T ax, ay, gx, gy;
  sie_deflection(p[0], p[1], p[2], x, y, ax, ay);
  shear_deflection(p[3], p[4], x, y, gx, gy);
  const T bx = x - ax - gx, by = y - ay - gy;
  const T zero(0.0);
  const T lens = sersic(x, y, zero, zero, p[5], p[6], p[7], p[8], p[9], P.b_lens);
  const T src = sersic(bx, by, p[10], p[11], p[12], p[13], p[14], p[15], p[16], P.b_src);
  return lens + src;
}

// ---------------------------------------------------------------------------
// General models (Sec. 5: several lenses and light components, a flat sky, free
// centres). Parameters, in this order:
//   per SIE        x_c, y_c, theta_E, q, phi            (deflection about its centre)
//   shear, if any  gamma, phi_gamma                     (about the origin)
//   per Sersic     x, y, I_e, R_e, n, q, phi            (evaluated at the position of
//                                                        the ray on the Sersic's plane)
//   sky, if any    surface brightness
// One lens plane (Eq. 1): beta = x - sum_k alpha_SIE_k(x - c_k) - alpha_shear(x);
// the deflectors of one plane add.
//
// Several lens planes (the extension named in Sec. 6, in the standard form of
// the multi-plane lens equation): lens planes 0..P-1 ordered by distance, the
// source plane P. The ray through the image-plane point x sits at
//   x_0 = x,   x_j = x - sum_{i<j} beta_ij alpha_i(x_i)   (j = 1..P),
// where alpha_i is the summed deflection of the plane-i deflectors (scaled, as
// theta_E is, to the source plane) and beta_ij = D_ij D_s / (D_j D_is) is the
// distance ratio of planes i < j, given with the model; beta_iP = 1. The shear
// belongs to plane 0. A light component on plane j is evaluated at x_j: plane 0
// is light seen unlensed, plane P the source.
// ---------------------------------------------------------------------------
}  // namespace
extern "C" {
typedef struct {
  int32_t n_sie;        // 0..8
  int32_t shear;        // 0 or 1
  int32_t n_sersic;     // 1..8
  int32_t sky;          // 0 or 1
  int32_t plane[8];     // per Sersic: its plane, 0..n_planes (n_planes = the source plane)
  int32_t n_planes;     // lens planes P, 1..8 (0 reads as 1)
  int32_t sie_plane[8]; // per SIE: its lens plane, 0..P-1
  int32_t reserved;     // 0
  double beta[8][8];    // beta[i][j], 0 <= i < j < P: distance ratio, in [0, 1]
} lo_model;
}
namespace {

int lens_planes(const lo_model& M) { return M.n_planes < 1 ? 1 : M.n_planes; }

int model_nparams(const lo_model& M) { return 5 * M.n_sie + (M.shear ? 2 : 0) + 7 * M.n_sersic + (M.sky ? 1 : 0); }

template <class T> struct GenericParams {
  const lo_model* M;
  std::vector<T> p;   // model_nparams values
  std::vector<T> b;   // b_n of every Sersic
};

template <class T> GenericParams<T> make_generic(const lo_model& M, const T* th) {
  GenericParams<T> G;
  G.M = &M;
  G.p.assign(th, th + model_nparams(M));
  const int o = 5 * M.n_sie + (M.shear ? 2 : 0);
  for (int j = 0; j < M.n_sersic; ++j) G.b.push_back(bn_of(G.p[o + 7 * j + 4]));
  return G;
}

// Summed deflection of the deflectors of lens plane `plane` at (x, y).
template <class T> void plane_deflection(const GenericParams<T>& G, int plane, T x, T y, T& ax, T& ay) {
  const lo_model& M = *G.M;
  const T* p = G.p.data();
  ax = T(0.0);
  ay = T(0.0);
  for (int k = 0; k < M.n_sie; ++k) {
    if ((lens_planes(M) > 1 ? M.sie_plane[k] : 0) != plane) continue;
    const T* s = p + 5 * k;
    T sx, sy;
    sie_deflection(s[2], s[3], s[4], x - s[0], y - s[1], sx, sy);
    ax = ax + sx;
    ay = ay + sy;
  }
  if (M.shear && plane == 0) {
    T gx, gy;
    shear_deflection(p[5 * M.n_sie], p[5 * M.n_sie + 1], x, y, gx, gy);
    ax = ax + gx;
    ay = ay + gy;
  }
}

// Position of the ray through the image-plane point (x, y) on every plane,
// lens planes 0..P-1 and the source plane P (the multi-plane lens equation;
// with one plane, Eq. 1).
template <class T> void plane_positions(const GenericParams<T>& G, T x, T y, std::vector<T>& px, std::vector<T>& py) {
  const lo_model& M = *G.M;
  const int P = lens_planes(M);
  std::vector<T> ax(P), ay(P);
  px.assign(P + 1, x);
  py.assign(P + 1, y);
  for (int j = 0; j <= P; ++j) {
    T sx = x, sy = y;
    for (int i = 0; i < j; ++i) {
      const double b = j == P ? 1.0 : M.beta[i][j];
      sx = sx - b * ax[i];
      sy = sy - b * ay[i];
    }
    px[j] = sx;
    py[j] = sy;
    if (j < P) plane_deflection(G, j, sx, sy, ax[j], ay[j]);
  }
}

template <class T> T surface_brightness(const GenericParams<T>& G, T x, T y) {
  const lo_model& M = *G.M;
  const T* p = G.p.data();
  std::vector<T> px, py;
  plane_positions(G, x, y, px, py);
  int o = 5 * M.n_sie + (M.shear ? 2 : 0);
  T I(0.0);
  for (int j = 0; j < M.n_sersic; ++j, o += 7) {
    const T* s = p + o;
    const int k = M.plane[j];
    I = I + sersic(px[k], py[k], s[0], s[1], s[2], s[3], s[4], s[5], s[6], G.b[j]);
  }
  if (M.sky) I = I + p[o];
  return I;
}

// The lens planes of a model: P in 1..8, every SIE on a lens plane, distance
// ratios in [0, 1] (D_ij <= D_is for planes i < j before the source).
bool model_shape_valid(const lo_model& M) {
  if (M.n_planes < 0 || M.n_planes > 8) return false;
  const int P = lens_planes(M);
  if (P == 1) return true;
  for (int k = 0; k < M.n_sie; ++k) if (M.sie_plane[k] < 0 || M.sie_plane[k] >= P) return false;
  for (int i = 0; i < P; ++i)
    for (int j = i + 1; j < P; ++j) if (!(M.beta[i][j] >= 0.0 && M.beta[i][j] <= 1.0)) return false;
  return true;
}

bool model_valid(const lo_model* M, const double* th) {
  if (!M || M->n_sie < 0 || M->n_sie > 8 || M->n_sersic < 1 || M->n_sersic > 8) return false;
  if ((M->shear != 0 && M->shear != 1) || (M->sky != 0 && M->sky != 1)) return false;
  if (!model_shape_valid(*M)) return false;
  for (int i = 0; i < model_nparams(*M); ++i) if (!std::isfinite(th[i])) return false;
  for (int k = 0; k < M->n_sie; ++k) if (!(th[5 * k + 3] > 0.0 && th[5 * k + 3] <= 1.0)) return false;
  const int o = 5 * M->n_sie + (M->shear ? 2 : 0);
  for (int j = 0; j < M->n_sersic; ++j) {
    const double* s = th + o + 7 * j;
    if (M->plane[j] < 0 || M->plane[j] > lens_planes(*M)) return false;
    if (!(s[3] > 0.0) || !(s[4] >= 0.2 && s[4] <= 10.0) || !(s[5] > 0.0 && s[5] <= 1.0)) return false;
  }
  return true;
}

bool params_valid(const double* th) {
  for (int i = 0; i < NPAR; ++i) if (!std::isfinite(th[i])) return false;
  const double qs[3] = {th[1], th[8], th[15]};
  for (double q : qs) if (!(q > 0.0 && q <= 1.0)) return false;
  if (!(th[6] > 0.0) || !(th[13] > 0.0)) return false;
  if (!(th[7] >= 0.2 && th[7] <= 10.0) || !(th[14] >= 0.2 && th[14] <= 10.0)) return false;
  return true;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI for the Python tests.
// ---------------------------------------------------------------------------
extern "C" {

typedef struct {
  int32_t height, width;     // pixels; row-major [height][width], row 0 = smallest y
  double pixscale;           // arcsec per pixel
  double center_x, center_y; // image-plane coordinates of the grid centre
  int32_t nsub;              // N of the N x N midpoint rule
  int32_t psf_h, psf_w;      // odd PSF dimensions
  const double* psf;         // [psf_h * psf_w], normalised here to unit sum
  const double* data;        // [height * width]
  const double* weight;      // [height * width], 1/s^2, 0 = masked
  // Optional explicit 1-D rule (Eq. 14, Sec. 4.5): when rule_n > 0 the pixel is
  // integrated by the Cartesian square of rule_n offsets rule_x (pixel units,
  // in [-1/2, 1/2]) with weights rule_w (summing to 1), replacing the N x N
  // midpoint rule.
  int32_t rule_n;
  const double* rule_x;
  const double* rule_w;
  // Amplitude parametrisation: 0 = theta[5], theta[12] are I_e; 1 = they are
  // total magnitudes with zero point zero_point (Sec. 4.1).
  int32_t amplitude;
  double zero_point;
  // Source position: 0 = theta[10], theta[11] are the source centre; 1 = they
  // are a point of the image plane that the source centre is mapped from.
  int32_t source_position;
} lo_system;

int lo_param_count(void) { return NPAR; }
double lo_digamma(double z) { return digamma(z); }
double lo_gamma_p(double a, double x) { return gamma_p_series(a, x, nullptr); }
double lo_bn(double n) { return bn_exact(n); }
double lo_bn_deriv(double n) { return bn_derivative(n, bn_exact(n)); }
double lo_intensity_from_magnitude(double m, double Re, double n, double zp) {
  return intensity_from_magnitude(m, Re, n, bn_exact(n), zp);
}

void lo_sie_deflection(double te, double q, double phi, double x, double y, double* ax, double* ay) {
  sie_deflection<double>(te, q, phi, x, y, *ax, *ay);
}
void lo_shear_deflection(double g, double phi, double x, double y, double* ax, double* ay) {
  shear_deflection<double>(g, phi, x, y, *ax, *ay);
}
double lo_sersic(double x, double y, double x0, double y0, double Ie, double Re, double n, double q, double phi) {
  return sersic<double>(x, y, x0, y0, Ie, Re, n, q, phi, bn_exact(n));
}
double lo_surface_brightness(const double* theta, double x, double y) {
  if (!params_valid(theta)) return std::numeric_limits<double>::quiet_NaN();
  const Params<double> P = make_params(theta);
  return surface_brightness(P, x, y);
}

// Neumaier's compensated summation.
double lo_sum_compensated(const double* x, int64_t n) {
  double s = 0.0, c = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double t = s + x[i];
    if (std::fabs(s) >= std::fabs(x[i])) c += (s - t) + x[i]; else c += (x[i] - t) + s;
    s = t;
  }
  return s + c;
}

}  // extern "C"

namespace {

// Pixel luminosities (Eq. 3) by the N x N midpoint product rule (Eq. 14): the
// abscissae of pixel (r, c) are
//   x = center_x + (c - (W-1)/2 + (kx + 1/2)/N - 1/2) * pixscale,
//   y = center_y + (r - (H-1)/2 + (ky + 1/2)/N - 1/2) * pixscale,
// each with weight pixscale^2 / N^2.
// The same with the Cartesian square of an explicit 1-D rule (offsets ux,
// weights wx): L = pixscale^2 sum_{i,j} wx_i wx_j I(x_i, y_j).
template <class T, class Model>
void render_rule(const lo_system& S, const Model& P, int n, const double* ux, const double* wx, std::vector<T>& L) {
  const int H = S.height, W = S.width;
  const double d = S.pixscale;
  L.assign(size_t(H) * W, T(0.0));
  for (int r = 0; r < H; ++r)
    for (int c = 0; c < W; ++c) {
      T acc(0.0);
      for (int ky = 0; ky < n; ++ky)
        for (int kx = 0; kx < n; ++kx) {
          const double x = S.center_x + (c - 0.5 * (W - 1) + ux[kx]) * d;
          const double y = S.center_y + (r - 0.5 * (H - 1) + ux[ky]) * d;
          acc = acc + (wx[kx] * wx[ky]) * surface_brightness(P, T(x), T(y));
        }
      L[size_t(r) * W + c] = acc * (d * d);
    }
}

template <class T, class Model> void render_unconvolved(const lo_system& S, const Model& P, std::vector<T>& L) {
  if (S.rule_n > 0) {
    render_rule(S, P, S.rule_n, S.rule_x, S.rule_w, L);
    return;
  }
  const int H = S.height, W = S.width, N = S.nsub;
  const double d = S.pixscale, wk = d * d / double(N * N);
  L.assign(size_t(H) * W, T(0.0));
  for (int r = 0; r < H; ++r)
    for (int c = 0; c < W; ++c) {
      T acc(0.0);
      for (int ky = 0; ky < N; ++ky)
        for (int kx = 0; kx < N; ++kx) {
          const double x = S.center_x + (c - 0.5 * (W - 1) + (kx + 0.5) / N - 0.5) * d;
          const double y = S.center_y + (r - 0.5 * (H - 1) + (ky + 0.5) / N - 0.5) * d;
          acc = acc + surface_brightness(P, T(x), T(y));
        }
      L[size_t(r) * W + c] = acc * wk;
    }
}

// Discrete PSF convolution (Eq. 15) with the kernel normalised to unit sum and
// the image padded by repeating the closest pixel:
//   L*_ij = sum_{k=-p..p} sum_{l=-q..q} F_{-k,-l} L_{clamp(i+k), clamp(j+l)},
// F_{a,b} being the element at row offset a and column offset b from the centre.
template <class T> void psf_convolve(int H, int W, const std::vector<T>& L, int ph, int pw, const double* psf,
                                     std::vector<T>& out) {
  const int p = ph / 2, q = pw / 2;
  double tot = 0.0;
  for (int i = 0; i < ph * pw; ++i) tot += psf[i];
  out.assign(size_t(H) * W, T(0.0));
  for (int i = 0; i < H; ++i)
    for (int j = 0; j < W; ++j) {
      T acc(0.0);
      for (int k = -p; k <= p; ++k)
        for (int l = -q; l <= q; ++l) {
          const double F = psf[size_t(-k + p) * pw + (-l + q)] / tot;
          const int ii = std::min(std::max(i + k, 0), H - 1);
          const int jj = std::min(std::max(j + l, 0), W - 1);
          acc = acc + F * L[size_t(ii) * W + jj];
        }
      out[size_t(i) * W + j] = acc;
    }
}

bool system_valid(const lo_system* S) {
  if (!S || S->height <= 0 || S->width <= 0 || S->nsub < 1) return false;
  if (S->amplitude < 0 || S->amplitude > 1 || !std::isfinite(S->zero_point)) return false;
  if (S->source_position < 0 || S->source_position > 1) return false;
  if (S->rule_n < 0 || (S->rule_n > 0 && (!S->rule_x || !S->rule_w))) return false;
  if (S->psf_h < 1 || S->psf_w < 1 || S->psf_h % 2 == 0 || S->psf_w % 2 == 0) return false;
  return true;
}

template <class T, class Model>
void model_image(const lo_system& S, const Model& P, int apply_psf, std::vector<T>& out) {
  std::vector<T> L;
  render_unconvolved(S, P, L);
  if (apply_psf && S.psf) psf_convolve(S.height, S.width, L, S.psf_h, S.psf_w, S.psf, out);
  else out.swap(L);
}

}  // namespace

extern "C" {

// Model image: unconvolved pixel luminosities (apply_psf = 0) or their PSF
// convolution (apply_psf != 0). Returns 0, or 1 for an invalid system; invalid
// parameters fill the image with NaN.
int lo_render(const lo_system* S, const double* theta, int apply_psf, double* out) {
  if (!system_valid(S) || !theta || !out) return 1;
  const size_t n = size_t(S->height) * S->width;
  if (!params_valid(theta)) {
    for (size_t i = 0; i < n; ++i) out[i] = std::numeric_limits<double>::quiet_NaN();
    return 0;
  }
  const Params<double> P = make_params(theta, S->amplitude, S->zero_point, S->source_position);
  std::vector<double> img;
  model_image(*S, P, apply_psf, img);
  std::memcpy(out, img.data(), n * sizeof(double));
  return 0;
}

// Per-pixel integration error estimate of a Gauss-Kronrod rule (Sec. 3.1): the
// system's rule (Kronrod weights) minus the same abscissae with the embedded
// Gauss weights gw (zero at the Kronrod-only nodes), in absolute value, before
// the PSF. Returns 0, or 1 without a rule.
int lo_render_error(const lo_system* S, const double* theta, const double* gw, double* out) {
  if (!system_valid(S) || S->rule_n <= 0 || !gw || !theta || !out) return 1;
  const size_t n = size_t(S->height) * S->width;
  if (!params_valid(theta)) {
    for (size_t i = 0; i < n; ++i) out[i] = std::numeric_limits<double>::quiet_NaN();
    return 0;
  }
  const Params<double> P = make_params(theta, S->amplitude, S->zero_point, S->source_position);
  std::vector<double> K, G;
  render_rule(*S, P, S->rule_n, S->rule_x, S->rule_w, K);
  render_rule(*S, P, S->rule_n, S->rule_x, gw, G);
  for (size_t i = 0; i < n; ++i) out[i] = std::fabs(K[i] - G[i]);
  return 0;
}

// PSF convolution alone (Eq. 15), for pins of the stencil.
int lo_psf_convolve(int H, int W, const double* L, int ph, int pw, const double* psf, double* out) {
  if (H <= 0 || W <= 0 || ph % 2 == 0 || pw % 2 == 0 || ph < 1 || pw < 1) return 1;
  std::vector<double> in(L, L + size_t(H) * W), res;
  psf_convolve(H, W, in, ph, pw, psf, res);
  std::memcpy(out, res.data(), res.size() * sizeof(double));
  return 0;
}

// chi^2 = sum_i w_i (d_i - L*_i)^2 summed with compensation; log L = -chi^2 / 2 (Eq. 17).
double lo_loglike(const lo_system* S, const double* theta) {
  if (!system_valid(S) || !theta || !S->data || !S->weight) return std::numeric_limits<double>::quiet_NaN();
  if (!params_valid(theta)) return std::numeric_limits<double>::quiet_NaN();
  const Params<double> P = make_params(theta, S->amplitude, S->zero_point, S->source_position);
  std::vector<double> img;
  model_image(*S, P, 1, img);
  std::vector<double> terms(img.size());
  for (size_t i = 0; i < img.size(); ++i) {
    const double r = S->data[i] - img[i];
    terms[i] = S->weight[i] * r * r;
  }
  return -0.5 * lo_sum_compensated(terms.data(), int64_t(terms.size()));
}

// log L and its gradient with respect to the 17 parameters, by forward-mode
// differentiation of the same computation.
double lo_loglike_grad(const lo_system* S, const double* theta, double* grad) {
  const double nan = std::numeric_limits<double>::quiet_NaN();
  if (!system_valid(S) || !theta || !grad || !S->data || !S->weight) return nan;
  if (!params_valid(theta)) { for (int i = 0; i < NPAR; ++i) grad[i] = nan; return nan; }
  Dual th[NPAR];
  for (int i = 0; i < NPAR; ++i) th[i] = Dual::var(theta[i], i);
  const Params<Dual> P = make_params(th, S->amplitude, S->zero_point, S->source_position);
  std::vector<Dual> img;
  model_image(*S, P, 1, img);
  std::vector<double> terms(img.size());
  double g[NPAR] = {0};
  for (size_t i = 0; i < img.size(); ++i) {
    const double r = S->data[i] - img[i].v;
    terms[i] = S->weight[i] * r * r;
    for (int k = 0; k < NPAR; ++k) g[k] += S->weight[i] * r * img[i].d[k];
  }
  for (int k = 0; k < NPAR; ++k) grad[k] = g[k];
  return -0.5 * lo_sum_compensated(terms.data(), int64_t(terms.size()));
}

// Model image and log L of a general model (see lo_model).
int lo_model_nparams(const lo_model* M) { return M ? model_nparams(*M) : -1; }

// Position of the ray through the image-plane point (x, y) on the lens planes
// 0..P-1 and the source plane P: px, py [P + 1], written. Returns 1 for an
// invalid model or point.
int lo_model_positions(const lo_model* M, const double* theta, double x, double y, double* px, double* py) {
  if (!M || !theta || !px || !py || !model_valid(M, theta)) return 1;
  const GenericParams<double> G = make_generic(*M, theta);
  std::vector<double> vx, vy;
  plane_positions(G, x, y, vx, vy);
  for (size_t j = 0; j < vx.size(); ++j) {
    px[j] = vx[j];
    py[j] = vy[j];
  }
  return 0;
}

int lo_render_model(const lo_system* S, const lo_model* M, const double* theta, int apply_psf, double* out) {
  if (!system_valid(S) || !M || !theta || !out) return 1;
  const size_t n = size_t(S->height) * S->width;
  if (!model_valid(M, theta)) {
    for (size_t i = 0; i < n; ++i) out[i] = std::numeric_limits<double>::quiet_NaN();
    return 0;
  }
  const GenericParams<double> G = make_generic(*M, theta);
  std::vector<double> img;
  model_image(*S, G, apply_psf, img);
  std::memcpy(out, img.data(), n * sizeof(double));
  return 0;
}

double lo_loglike_model(const lo_system* S, const lo_model* M, const double* theta) {
  if (!system_valid(S) || !M || !theta || !S->data || !S->weight) return std::numeric_limits<double>::quiet_NaN();
  if (!model_valid(M, theta)) return std::numeric_limits<double>::quiet_NaN();
  const GenericParams<double> G = make_generic(*M, theta);
  std::vector<double> img;
  model_image(*S, G, 1, img);
  std::vector<double> terms(img.size());
  for (size_t i = 0; i < img.size(); ++i) {
    const double r = S->data[i] - img[i];
    terms[i] = S->weight[i] * r * r;
  }
  return -0.5 * lo_sum_compensated(terms.data(), int64_t(terms.size()));
}

// Surface brightness and its 17 partial derivatives at one image-plane point.
double lo_surface_brightness_grad(const double* theta, double x, double y, double* grad) {
  const double nan = std::numeric_limits<double>::quiet_NaN();
  if (!params_valid(theta)) { for (int i = 0; i < NPAR; ++i) grad[i] = nan; return nan; }
  Dual th[NPAR];
  for (int i = 0; i < NPAR; ++i) th[i] = Dual::var(theta[i], i);
  const Params<Dual> P = make_params(th);
  const Dual I = surface_brightness(P, Dual(x), Dual(y));
  for (int i = 0; i < NPAR; ++i) grad[i] = I.d[i];
  return I.v;
}

}  // extern "C"
