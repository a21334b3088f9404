// model.h -- shape and per-point constants of general models (several lenses
// and light components, a flat sky, free centres), evaluated in float64.
#pragma once

namespace lensed {

// General models (several lenses and light components, a flat sky, free
// centres): the model's shape (a copy of lensed_model) and per-point constants
// in float64, derived by the model prologue.
constexpr int MAX_SIE = 8, MAX_SERSIC = 8, MAX_PLANES = 8;
struct ModelSpec {
  int n_sie, shear, n_sersic, sky;
  int plane[MAX_SERSIC];          // per Sersic: its plane, 0..n_planes (n_planes: the source)
  int n_planes;                   // lens planes, 1..8
  int sie_plane[MAX_SIE];         // per SIE: its lens plane (0 with one plane)
  double beta[MAX_PLANES][MAX_PLANES];  // distance ratios beta_ij, i < j < n_planes (0 with one plane)
};
struct ModelConst {
  double sie[MAX_SIE][9];      // x_c, y_c, cos, sin, q^2, q', k = theta_E sqrt(q)/q' (theta_E when q = 1),
                               // theta_E, q
  double g1, g2;               // external shear (zero without one)
  double gam, c2g, s2g;        // gamma, cos 2 phi_gamma, sin 2 phi_gamma
  double ser[MAX_SERSIC][11];  // x0, y0, cos, sin, q, 1/q, 1/R_e, 1/n, b_n, I_e, db_n/dn (0 unless asked for)
  double sky;                  // flat sky surface brightness (NaN marks an invalid point)
  int n_sie, n_sersic;
  int sie_sphere[MAX_SIE];     // 1 where q = 1
  int plane[MAX_SERSIC];       // the Sersic's plane: 0 light at x, n_planes light at the source
};

}  // namespace lensed
