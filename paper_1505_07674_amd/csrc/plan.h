// plan.h -- tile-shape selection and batched execution plans.
#pragma once

#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"
#include "kernels.h"
#include "lensed.h"

struct lensed_ctx;

namespace lensed {


struct TileShape {
  int TW, TH;
};

// Chooses the TW x TH output tile of the PSF/chi^2 kernel for a launch. The
// model counts lane slots of the stencil (ragged tiles and partly idle waves
// included) plus the LDS staging of the halo and ranks the candidates; the
// autotuner times the best-ranked few on the real launch and records the
// fastest per set of system shapes, which then overrides the model.
class TileCache {
 public:
  // The tile for one image (the single-point entry points): the specialised
  // 32- or 64-wide tiles, ranked by latency, not by throughput.
  static TileShape latency_best(const lensed_system& s);
  TileShape choose(const lensed_system& s);
  TileShape choose_common(const lensed_system* s, int n);
  std::vector<TileShape> ranked(const lensed_system* s, int n, int k) const;
  bool has_measured(const lensed_system* s, int n) const { return measured_.count(key(s, n)) != 0; }
  void set_measured(const lensed_system* s, int n, TileShape t) { measured_[key(s, n)] = t; }
  // Render schedule (pixels per thread of the midpoint classes, threads per
  // block): the measured choice for this set of image sizes and rules, else one
  // pixel per thread in RENDER_BLOCK-thread blocks.
  RenderSchedule render_schedule(const lensed_system* s, int n) const {
    auto it = render_measured_.find(render_key(s, n));
    return it == render_measured_.end() ? RenderSchedule{1, RENDER_BLOCK} : it->second;
  }
  bool has_render_measured(const lensed_system* s, int n) const { return render_measured_.count(render_key(s, n)) != 0; }
  void set_render_measured(const lensed_system* s, int n, RenderSchedule r) { render_measured_[render_key(s, n)] = r; }
  static double model_cost(int H, int W, int ph, int pw, TileShape t, int sq);
  static std::vector<TileShape> candidates(int sq, const lensed_system* s = nullptr, int n = 0);
  // The cost model's best tile for one system (no cache, no allocation).
  static TileShape model_best(const lensed_system& s);

 private:
  static std::string key(const lensed_system* s, int n);
  static std::string render_key(const lensed_system* s, int n);
  static int launch_square(const lensed_system* s, int n);
  std::map<std::tuple<int, int, int, int>, TileShape> cache_;
  std::map<std::string, TileShape> measured_;
  std::map<std::string, RenderSchedule> render_measured_;
};

int validate_system(lensed_ctx* c, const lensed_system* s, bool need_data, int index);
SysDesc make_desc(const lensed_system& s, const TileShape& t);
int square_psf_code(int ph, int pw);

// One batched evaluation: n_points parameter points over n_systems systems.
// Work lists are (point, tile) items ordered by decreasing cost (longest first);
// the unconvolved images of all points live in one scratch buffer.
class BatchPlan {
 public:
  ~BatchPlan();
  // grad == nullptr: log L only; otherwise also d log L / d theta (single system;
  // with a general model, one lens plane).
  // K > 1 or sky: every image is the sum of K consecutive points plus sky[i]
  // pixscale^2 (sky per image); G > 1: every log L is the sum over G consecutive
  // images (the bands of a model). map has one entry per point.
  // model: a general model (ModelSpec, params_per_point values per point) instead
  // of the 17-parameter one.
  bool matches(const lensed_system* systems, int n_systems, const float* theta, const int32_t* map, int n_points,
               const double* logl, const float* grad = nullptr, int K = 1, const float* sky = nullptr,
               int G = 1, const ModelSpec* model = nullptr, bool masked = false,
               const float* grad_sky = nullptr) const;
  // force: use this tile shape instead of the cache's choice (autotuning);
  // force_render: use this render schedule (pixels per thread where the class
  // allows it, threads per block) instead of the cache's.
  // masked: render only the pixels the chi^2 can see (the support of w > 0
  // dilated by the PSF, clamped at the borders) and convolve only the PSF tiles
  // that hold a pixel with w > 0; the other pixels and tile sums stay zero.
  hipError_t build(const lensed_system* systems, int n_systems, const float* theta, const int32_t* map,
                   int n_points, double* logl, TileCache& tiles, std::string& msg, float* grad = nullptr,
                   const TileShape* force = nullptr, int K = 1, const float* sky = nullptr, int G = 1,
                   const ModelSpec* model = nullptr, int params_per_point = NPAR,
                   const RenderSchedule* force_render = nullptr, bool masked = false,
                   float* grad_sky = nullptr);
  // Runs the plan stage by stage (a warm-up, then three timed runs) and returns
  // the fastest PSF + chi^2 stage, or the fastest render kernels, in milliseconds.
  hipError_t psf_ms(hipStream_t s, float* ms) const { return stage_ms(s, 3, ms); }
  hipError_t render_ms(hipStream_t s, float* ms) const { return stage_ms(s, 1, ms); }
  // The most pixels per thread a render class of this plan could take (1 or 2).
  int max_ppt() const { return max_ppt_; }
  // The schedule in use: PSF tile, pixels per thread of the midpoint classes and
  // threads per render block.
  TileShape psf_tile() const { return {TW_, TH_}; }
  int render_ppt() const { return ppt_; }
  int render_block() const { return rbs_; }
  int64_t rendered_pixels() const { return rendered_pixels_; }
  int64_t rendered_subsamples() const { return rendered_subsamples_; }
  hipError_t capture(hipStream_t cap);
  // events, when given, are LENSED_NSTAGES + 1 events recorded around the stages
  // (prologue, render kernel, cusp corrections and composition, PSF + chi^2,
  // finalize; with a gradient A^T rho, gradient kernel, its cusp corrections and sums)
  hipError_t enqueue(hipStream_t s, hipEvent_t* events = nullptr) const;
  hipError_t run(hipStream_t s) const;

 private:
  std::vector<lensed_system> systems_;
  std::vector<int32_t> map_;
  const float* theta_ = nullptr;
  double* logl_ = nullptr;
  float* grad_ = nullptr;
  int n_points_ = 0;
  int K_ = 1;                     // points per image
  int G_ = 1;                     // images per log L (bands)
  const float* sky_ = nullptr;    // [n_images] flat sky surface brightness, or nullptr
  float* grad_sky_ = nullptr;     // gradient plans with a sky: d log L / d sky per model, or nullptr
  int64_t* d_goff_ = nullptr;     // gradient plans with K > 1: offset of each point's model image (g)
  int n_images_ = 0, n_models_ = 0;
  int* d_mpbase_ = nullptr;       // first partial-sum slot of each log L
  int* d_mntiles_ = nullptr;      // PSF tiles summed into each log L
  int compose_tiles_ = 0;         // render tiles of the largest image
  bool has_model_ = false;        // general model: model prologue and float64 render
  ModelSpec spec_{};
  int params_per_point_ = NPAR;
  ModelConst* d_mc_ = nullptr;

  char* mem_ = nullptr;
  SysDesc* d_sys_ = nullptr;
  int* d_point_sys_ = nullptr;
  int64_t* d_loff_ = nullptr;
  int* d_pbase_ = nullptr;
  int* d_ntiles_ = nullptr;
  int2* d_ritems_ = nullptr;
  int2* d_gitems_ = nullptr;      // gradient plans: (point, 256-pixel tile of the support of g) items
  int n_gitems_ = 0;
  int2* d_pitems_ = nullptr;
  PointConst* d_pc_ = nullptr;
  PointConst64* d_p64_ = nullptr;
  CuspList cusp_{nullptr, nullptr};
  GradConst* d_gc_ = nullptr;
  float* d_R_ = nullptr;          // weighted residuals (gradient plans)
  int* d_gpbase_ = nullptr;       // first gradient-partial tile of each point
  float2* d_gpart_ = nullptr;     // [tiles][17] (hi, lo)
  double* d_gcorr_ = nullptr;     // [points][17] float64 cusp corrections
  double* d_mgpart_ = nullptr;    // general-model gradients: [tiles][params per point]
  int grad_ntiles_ = 0;
  float* d_L_ = nullptr;
  float2* d_part_ = nullptr;
  int n_ritems_ = 0, n_pitems_ = 0;
  std::vector<RenderSpan> rspans_;   // render items by schedule class
  int square_psf_ = -1, TW_ = 32, TH_ = 32, max_ph_ = 1, max_pw_ = 1;
  hipGraph_t graph_ = nullptr;
  hipGraphExec_t exec_ = nullptr;
  int ppt_ = 1;
  int rbs_ = RENDER_BLOCK;        // threads (render units) per render block
  int64_t max_pixels_ = 0;        // largest image of the plan (pixels)
  int max_ppt_ = 1;
  bool masked_ = false;
  int64_t rendered_pixels_ = 0;   // pixels the render stage computes per launch
  int64_t rendered_subsamples_ = 0;
  hipError_t stage_ms(hipStream_t s, int stage, float* ms) const;
};

}  // namespace lensed
