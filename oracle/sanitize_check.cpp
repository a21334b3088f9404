// sanitize_check.cpp -- TEST INFRASTRUCTURE: a host-only driver that runs every
// entry point of the FP64 oracle once on small inputs, built with the address
// and undefined-behaviour sanitizers by tests/test_oracle_sanitize.py. It
// includes the oracle's single source file, so the sanitizers see every line
// of it; it checks only that each call returns and gives finite values where
// the inputs are valid (the numerical pins live in the Python tests).
#include "lensed_oracle.cpp"

#include <cstdio>
#include <cstdlib>

namespace {

int failures = 0;

void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "sanitize_check: %s\n", what);
    ++failures;
  }
}

bool all_finite(const std::vector<double>& v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

lo_system small_system(int H, int W, int N, int ph, int pw, const std::vector<double>& psf, const double* data,
                       const double* weight) {
  lo_system S{};
  S.height = H;
  S.width = W;
  S.pixscale = 0.08;
  S.center_x = 0.05;
  S.center_y = -0.03;
  S.nsub = N;
  S.psf_h = ph;
  S.psf_w = pw;
  S.psf = psf.data();
  S.data = data;
  S.weight = weight;
  return S;
}

}  // namespace

int main() {
  const double theta[NPAR] = {1.1, 0.7, 0.6, 0.04, 0.5, 0.1, 1.2, 3.5, 0.8, 0.9,
                              0.1, -0.05, 1.0, 0.15, 2.5, 0.7, 1.0};
  const int H = 23, W = 19, ph = 5, pw = 7;
  std::vector<double> psf(ph * pw);
  for (int i = 0; i < ph * pw; ++i) psf[i] = 1.0 + 0.1 * (i % 5);
  std::vector<double> data(H * W), weight(H * W);
  for (int i = 0; i < H * W; ++i) {
    data[i] = 0.01 * (i % 7);
    weight[i] = (i % 5) ? 1e4 : 0.0;
  }
  lo_system S = small_system(H, W, 3, ph, pw, psf, data.data(), weight.data());

  for (double n : {0.2, 0.5, 1.0, 4.0, 10.0}) {
    expect(std::isfinite(lo_bn(n)) && std::isfinite(lo_bn_deriv(n)), "b_n");
    expect(std::isfinite(lo_intensity_from_magnitude(20.0, 0.3, n, 25.0)), "magnitude");
  }
  expect(std::isfinite(lo_digamma(2.5)) && std::isfinite(lo_gamma_p(3.0, 2.0)), "special functions");
  double ax, ay;
  lo_sie_deflection(1.0, 0.6, 0.3, 0.4, -0.2, &ax, &ay);
  expect(std::isfinite(ax) && std::isfinite(ay), "SIE");
  lo_shear_deflection(0.05, 0.4, 0.4, -0.2, &ax, &ay);
  expect(std::isfinite(ax) && std::isfinite(ay), "shear");

  std::vector<double> img(H * W), img2(H * W), g(NPAR);
  expect(lo_render(&S, theta, 0, img.data()) == 0 && all_finite(img), "render");
  expect(lo_render(&S, theta, 1, img2.data()) == 0 && all_finite(img2), "render with PSF");
  expect(lo_psf_convolve(H, W, img.data(), ph, pw, psf.data(), img2.data()) == 0 && all_finite(img2), "PSF");
  expect(std::isfinite(lo_loglike(&S, theta)), "log L");
  expect(std::isfinite(lo_loglike_grad(&S, theta, g.data())) && all_finite(g), "gradient");
  expect(std::isfinite(lo_surface_brightness_grad(theta, 0.3, 0.2, g.data())) && all_finite(g), "SB gradient");
  double th_bad[NPAR];
  std::memcpy(th_bad, theta, sizeof th_bad);
  th_bad[1] = 1.5;
  expect(lo_render(&S, th_bad, 1, img.data()) == 0 && std::isnan(img[0]), "invalid point gives NaN");

  // Gauss-Kronrod style explicit rule with an error map (3 nodes, embedded 1-node rule)
  const double rx[3] = {-0.3, 0.0, 0.3}, rw[3] = {0.3, 0.4, 0.3}, gw[3] = {0.0, 1.0, 0.0};
  lo_system R = S;
  R.rule_n = 3;
  R.rule_x = rx;
  R.rule_w = rw;
  expect(lo_render_error(&R, theta, gw, img.data()) == 0 && all_finite(img), "error map");
  R.amplitude = 1;
  R.zero_point = 25.0;
  R.source_position = 1;
  double th_mag[NPAR];
  std::memcpy(th_mag, theta, sizeof th_mag);
  th_mag[5] = 21.0;
  th_mag[12] = 22.0;
  th_mag[10] = 1.0;
  th_mag[11] = 0.3;
  expect(std::isfinite(lo_loglike_grad(&R, th_mag, g.data())) && all_finite(g), "magnitudes, image-plane source");

  // one pixel, no PSF
  const double one = 1.0;
  lo_system P1 = small_system(1, 1, 2, 1, 1, std::vector<double>{1.0}, data.data(), weight.data());
  P1.psf = &one;
  expect(lo_render(&P1, theta, 1, img.data()) == 0 && std::isfinite(img[0]), "single pixel");

  // general model: two SIEs on two planes, shear, three Sersics (one per plane), sky
  lo_model M{};
  M.n_sie = 2;
  M.shear = 1;
  M.n_sersic = 3;
  M.sky = 1;
  M.plane[0] = 0;
  M.plane[1] = 1;
  M.plane[2] = 2;
  M.n_planes = 2;
  M.sie_plane[0] = 0;
  M.sie_plane[1] = 1;
  M.beta[0][1] = 0.6;
  const int np = lo_model_nparams(&M);
  expect(np == 2 * 5 + 2 + 3 * 7 + 1, "model parameter count");
  std::vector<double> mp = {0.0, 0.0, 1.0, 0.8, 0.3,   0.4, -0.2, 0.3, 0.9, 1.0,   0.05, 0.4,
                            0.0, 0.0, 0.1, 1.0, 4.0, 0.8, 0.9,   0.4, -0.2, 0.2, 0.3, 1.0, 0.9, 0.2,
                            0.1, 0.05, 1.0, 0.15, 1.5, 0.7, 1.0,   0.01};
  expect((int)mp.size() == np, "model parameter vector");
  expect(lo_render_model(&S, &M, mp.data(), 1, img.data()) == 0 && all_finite(img), "model render");
  expect(std::isfinite(lo_loglike_model(&S, &M, mp.data())), "model log L");
  double px[3], py[3];
  expect(lo_model_positions(&M, mp.data(), 0.3, 0.2, px, py) == 0, "plane positions");

  std::vector<double> terms = {1.0, 1e-16, -1.0, 3.0};
  expect(lo_sum_compensated(terms.data(), (int64_t)terms.size()) == 3.0 + 1e-16, "compensated sum");

  if (failures) return 1;
  std::printf("sanitize_check ok\n");
  return 0;
}
