// plan.hip -- tile-shape model and batched plans with captured hipGraphs.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "plan.h"
#include "stencil.h"

namespace lensed {

namespace {
// Calls f(t) for every candidate PSF output tile of a launch over systems s
// (sq: the launch's square-PSF code); a shape may come more than once.
template <class F>
void each_candidate(int sq, const lensed_system* s, int n, F f) {
  const int tws[] = {16, 32, 40, 48, 64};
  const int ths[] = {16, 20, 24, 32, 40, 48, 64};
  for (int tw : tws)
    for (int th : ths) {
      const int threads = tw * th / psf_rows(sq, tw, th);
      if (threads >= 64 && threads <= 512) f(TileShape{tw, th});
    }
  // Wide tiles of the 21 x 21 stencil: a whole image row, or a half or a third
  // of it, so that the tiles cover the image without ragged columns; heights
  // whose LDS block stays within 64 KiB.
  for (int i = 0; s && i < n; ++i)
    for (int parts = 1; parts <= 3; ++parts) {
      const int tw = (s[i].width + parts - 1) / parts;
      if (!psf_wide(sq, tw)) continue;
      for (int th : {16, 24, 32, 40}) {
        const int threads = tw * th / psf_rows(sq, tw, th);
        if (threads < 64 || threads > WIDE_MAX_THREADS || psf_lds_bytes(sq, tw, th, 21, 21) > 65536) continue;
        f(TileShape{tw, th});
      }
    }
}
}  // namespace

std::vector<TileShape> TileCache::candidates(int sq, const lensed_system* s, int n) {
  std::vector<TileShape> out;
  each_candidate(sq, s, n, [&](TileShape t) {
    if (std::none_of(out.begin(), out.end(), [&](const TileShape& o) { return o.TW == t.TW && o.TH == t.TH; }))
      out.push_back(t);
  });
  return out;
}

TileShape TileCache::model_best(const lensed_system& s) {
  TileShape best{32, 32};
  double bc = 1e300;
  const int sq = square_psf_code(s.psf_h, s.psf_w);
  each_candidate(sq, &s, 1, [&](TileShape t) {
    const double cst = model_cost(s.height, s.width, s.psf_h, s.psf_w, t, sq);
    if (cst < bc) {
      bc = cst;
      best = t;
    }
  });
  return best;
}

// Lane slots of one launch: per tile, the block's lanes (whole waves) times the
// per-thread work of R outputs (R ph pw FMAs and pw (R + ph - 1) LDS reads),
// plus the LDS staging of the tile and its halo and a fixed block cost. The
// generic stencil (runtime sizes, taps by vector loads) costs twice as much
// per tap as the specialised ones. sq is the square-PSF code of the launch
// (-1 when its systems differ), which decides the kernel and R.
double TileCache::model_cost(int H, int W, int ph, int pw, TileShape t, int sq) {
  const int R = psf_rows(sq, t.TW, t.TH);
  const double ntiles = (double)((W + t.TW - 1) / t.TW) * (double)((H + t.TH - 1) / t.TH);
  const int threads = t.TW * t.TH / R;
  const double lanes = 64.0 * ((threads + 63) / 64);
  const double tap = psf_specialised(sq, t.TW) ? 1.0 : 2.0;
  const double per_lane = tap * (double)R * ph * pw + 0.5 * (double)pw * (R + ph - 1);
  const double staging = 6.0 * (double)(t.TW + pw - 1) * (double)(t.TH + ph - 1);
  return ntiles * (lanes * per_lane + staging + 2000.0);
}

// One image runs on a few blocks, so what counts is how long a block takes:
// its waves share the CU's four SIMDs, and each thread applies R ph pw taps.
// Cost: (waves per SIMD, from the block's own waves or from the whole launch
// spread over 1024 SIMDs, whichever is larger) x the taps per thread, plus
// the block's LDS staging per thread.
TileShape TileCache::latency_best(const lensed_system& s) {
  const int sq = square_psf_code(s.psf_h, s.psf_w);
  TileShape best{32, 32};
  double bc = 1e300;
  each_candidate(sq, &s, 1, [&](TileShape t) {
    if (t.TW != 32 && t.TW != 64) return;
    const int R = psf_rows(sq, t.TW, t.TH);
    const int threads = t.TW * t.TH / R;
    const double waves = (double)((threads + 63) / 64);
    const double ntiles = (double)((s.width + t.TW - 1) / t.TW) * (double)((s.height + t.TH - 1) / t.TH);
    const double per_simd = std::max(std::ceil(waves / 4.0), std::ceil(ntiles * waves / 1024.0));
    const double tap = psf_specialised(sq, t.TW) ? 1.0 : 2.0;
    const double cst = per_simd * tap * R * s.psf_h * s.psf_w +
                       6.0 * (double)(t.TW + s.psf_w - 1) * (double)(t.TH + s.psf_h - 1) / threads;
    if (cst < bc) {
      bc = cst;
      best = t;
    }
  });
  return best;
}

std::string TileCache::key(const lensed_system* s, int n) {
  std::vector<std::string> parts;
  for (int i = 0; i < n; ++i)
    parts.push_back(std::to_string(s[i].height) + "x" + std::to_string(s[i].width) + "p" +
                    std::to_string(s[i].psf_h) + "x" + std::to_string(s[i].psf_w));
  std::sort(parts.begin(), parts.end());
  parts.erase(std::unique(parts.begin(), parts.end()), parts.end());
  std::string k;
  for (const auto& p : parts) k += p + ";";
  return k;
}

std::string TileCache::render_key(const lensed_system* s, int n) {
  std::vector<std::string> parts;
  for (int i = 0; i < n; ++i)
    parts.push_back(std::to_string(s[i].height) + "x" + std::to_string(s[i].width) + "n" + std::to_string(s[i].nsub) +
                    "r" + std::to_string(s[i].rule));
  std::sort(parts.begin(), parts.end());
  parts.erase(std::unique(parts.begin(), parts.end()), parts.end());
  std::string k;
  for (const auto& p : parts) k += p + ";";
  return k;
}

int TileCache::launch_square(const lensed_system* s, int n) {
  int sq = square_psf_code(s[0].psf_h, s[0].psf_w);
  for (int i = 1; i < n; ++i)
    if (square_psf_code(s[i].psf_h, s[i].psf_w) != sq) sq = -1;
  return sq;
}

std::vector<TileShape> TileCache::ranked(const lensed_system* s, int n, int k) const {
  const int sq = launch_square(s, n);
  std::vector<std::pair<double, TileShape>> all;
  for (const TileShape& t : candidates(sq, s, n)) {
    double cst = 0.0;
    for (int i = 0; i < n; ++i) cst += model_cost(s[i].height, s[i].width, s[i].psf_h, s[i].psf_w, t, sq);
    all.push_back({cst, t});
  }
  std::stable_sort(all.begin(), all.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
  std::vector<TileShape> out;
  for (int i = 0; i < (int)all.size() && i < k; ++i) out.push_back(all[i].second);
  return out;
}

TileShape TileCache::choose(const lensed_system& s) {
  auto m = measured_.find(key(&s, 1));
  if (m != measured_.end()) return m->second;
  const auto shape = std::make_tuple(s.height, s.width, s.psf_h, s.psf_w);
  auto it = cache_.find(shape);
  if (it != cache_.end()) return it->second;
  const TileShape best = model_best(s);
  cache_[shape] = best;
  return best;
}

TileShape TileCache::choose_common(const lensed_system* s, int n) {
  if (n == 1) return choose(s[0]);
  auto m = measured_.find(key(s, n));
  if (m != measured_.end()) return m->second;
  const std::vector<TileShape> r = ranked(s, n, 1);
  return r.empty() ? TileShape{32, 32} : r[0];
}

namespace {
bool same_system(const lensed_system& a, const lensed_system& b) {
  return a.height == b.height && a.width == b.width && a.pixscale == b.pixscale && a.center_x == b.center_x &&
         a.center_y == b.center_y && a.nsub == b.nsub && a.psf_h == b.psf_h && a.psf_w == b.psf_w &&
         a.psf == b.psf && a.data == b.data && a.weight == b.weight && a.rule == b.rule &&
         a.amplitude == b.amplitude && a.zero_point == b.zero_point && a.source_position == b.source_position;
}
size_t align256(size_t x) { return (x + 255) / 256 * 256; }
}  // namespace

BatchPlan::~BatchPlan() {
  if (exec_) (void)hipGraphExecDestroy(exec_);
  if (graph_) (void)hipGraphDestroy(graph_);
  if (mem_) (void)hipFree(mem_);
}

bool BatchPlan::matches(const lensed_system* systems, int n_systems, const float* theta, const int32_t* map,
                        int n_points, const double* logl, const float* grad, int K, const float* sky, int G,
                        const ModelSpec* model, bool masked, const float* grad_sky) const {
  if (masked != masked_ || grad_sky != grad_sky_) return false;
  if (theta != theta_ || logl != logl_ || grad != grad_ || n_points != n_points_ || K != K_ || sky != sky_ ||
      G != G_ || (model != nullptr) != has_model_ ||
      (model && std::memcmp(model, &spec_, sizeof(ModelSpec)) != 0) ||
      (size_t)n_systems != systems_.size())
    return false;
  for (int s = 0; s < n_systems; ++s)
    if (!same_system(systems[s], systems_[s])) return false;
  return std::equal(map_.begin(), map_.end(), map);
}

hipError_t BatchPlan::build(const lensed_system* systems, int n_systems, const float* theta, const int32_t* map,
                            int n_points, double* logl, TileCache& tiles, std::string& msg, float* grad,
                            const TileShape* force, int K, const float* sky, int G, const ModelSpec* model,
                            int params_per_point, const RenderSchedule* force_render, bool masked, float* grad_sky) {
  systems_.assign(systems, systems + n_systems);
  map_.assign(map, map + n_points);
  theta_ = theta;
  logl_ = logl;
  grad_ = grad;
  n_points_ = n_points;
  K_ = K;
  G_ = G;
  has_model_ = model != nullptr;
  if (model) spec_ = *model;
  params_per_point_ = params_per_point;
  sky_ = sky;
  grad_sky_ = grad && sky ? grad_sky : nullptr;
  n_images_ = n_points / K;
  n_models_ = n_images_ / G;

  const TileShape ts = force ? *force : tiles.choose_common(systems, n_systems);
  TW_ = ts.TW;
  TH_ = ts.TH;
  std::vector<SysDesc> desc(n_systems);
  std::vector<size_t> psf_off(n_systems);
  size_t psf_total = 0;
  square_psf_ = square_psf_code(systems[0].psf_h, systems[0].psf_w);
  max_ph_ = max_pw_ = 1;
  for (int s = 0; s < n_systems; ++s) {
    desc[s] = make_desc(systems[s], ts);
    psf_off[s] = psf_total;
    psf_total += (size_t)systems[s].psf_h * systems[s].psf_w;
    max_ph_ = std::max(max_ph_, systems[s].psf_h);
    max_pw_ = std::max(max_pw_, systems[s].psf_w);
    if (square_psf_code(systems[s].psf_h, systems[s].psf_w) != square_psf_) square_psf_ = -1;
  }

  // Pixels per render thread: two for a midpoint class whose images all have
  // an even width (a pair never straddles two rows), if the schedule says so;
  // general-model plans keep one (their kernel walks one pixel per thread). The
  // gradient kernels have item lists of their own.
  const RenderSchedule rs = force_render ? *force_render : tiles.render_schedule(systems, n_systems);
  ppt_ = rs.ppt == 2 ? 2 : 1;
  rbs_ = rs.block >= 64 && rs.block <= RENDER_BLOCK_MAX && rs.block % 64 == 0 ? rs.block : RENDER_BLOCK;
  if (model) ppt_ = 1, rbs_ = RENDER_BLOCK;   // the general-model render walks 256-pixel tiles
  std::vector<int> class_div(RENDER_MAX_CLASS + 1, 2);   // pixels per thread each class allows
  class_div[0] = 1;
  for (int s = 0; s < n_systems; ++s)
    if (desc[s].W % 2 != 0) class_div[render_class(desc[s])] = 1;
  max_ppt_ = 1;
  if (!model)
    for (int s = 0; s < n_systems; ++s) max_ppt_ = std::max(max_ppt_, class_div[render_class(desc[s])]);
  auto class_ppt = [&](int klass) { return std::min(ppt_, class_div[klass]); };

  // Masked plans: per system, the render units the chi^2 can see and the PSF
  // tiles that hold a pixel with w > 0 (from the weights, read back once here).
  // An output pixel reads L within its (2p+1) x (2q+1) stencil, clamped at the
  // borders, so the pixels needed are the w > 0 support dilated by that box.
  masked_ = masked && !grad && !model;
  std::vector<std::vector<int>> units(n_systems);
  std::vector<std::vector<char>> ptile_on(n_systems);
  if (masked_) {
    for (int s = 0; s < n_systems; ++s) {
      const SysDesc& d = desc[s];
      const size_t npx = (size_t)d.H * d.W;
      std::vector<float> w(npx);
      hipError_t e = hipMemcpy(w.data(), d.weight, sizeof(float) * npx, hipMemcpyDeviceToHost);
      if (e != hipSuccess) {
        msg = "reading weights";
        return e;
      }
      const int p = d.ph / 2, q = d.pw / 2;
      // separable box dilation: distance to the nearest marked pixel along rows, then along columns
      std::vector<char> rowd(npx, 0), need(npx, 0);
      std::vector<int> nxt(std::max(d.H, d.W) + 1);
      for (int r = 0; r < d.H; ++r) {
        const float* wr = &w[(size_t)r * d.W];
        nxt[d.W] = 1 << 29;
        for (int c = d.W - 1; c >= 0; --c) nxt[c] = wr[c] > 0.0f ? c : nxt[c + 1];
        int last = -(1 << 29);
        for (int c = 0; c < d.W; ++c) {
          if (wr[c] > 0.0f) last = c;
          rowd[(size_t)r * d.W + c] = (c - last <= q) || (nxt[c] - c <= q);
        }
      }
      for (int c = 0; c < d.W; ++c) {
        nxt[d.H] = 1 << 29;
        for (int r = d.H - 1; r >= 0; --r) nxt[r] = rowd[(size_t)r * d.W + c] ? r : nxt[r + 1];
        int last = -(1 << 29);
        for (int r = 0; r < d.H; ++r) {
          if (rowd[(size_t)r * d.W + c]) last = r;
          need[(size_t)r * d.W + c] = (r - last <= p) || (nxt[r] - r <= p);
        }
      }
      const int pp = class_ppt(render_class(d));
      for (size_t pix = 0; pix < npx; pix += pp)
        if (need[pix] || (pp == 2 && need[pix + 1])) units[s].push_back((int)pix);
      ptile_on[s].assign(d.n_ptiles, 0);
      for (int r = 0; r < d.H; ++r)
        for (int c = 0; c < d.W; ++c)
          if (w[(size_t)r * d.W + c] > 0.0f) ptile_on[s][(r / d.TH) * d.tiles_x + c / d.TW] = 1;
      desc[s].n_active = (int)units[s].size();
    }
  }
  rendered_pixels_ = rendered_subsamples_ = 0;

  std::vector<int64_t> loff(n_points);
  std::vector<int> pbase(n_points), ntiles(n_points), gpbase(n_points);
  int gtot = 0;
  int64_t Ltot = 0;
  int ptot = 0;
  struct Item {
    int64_t cost;
    int point, tile, klass;
  };
  std::vector<Item> ritems, pitems;
  for (int p = 0; p < n_points; ++p) {
    const SysDesc& d = desc[map[p]];
    loff[p] = Ltot;
    Ltot += (int64_t)d.H * d.W;
    pbase[p] = ptot;
    ntiles[p] = p % K == 0 ? d.n_ptiles : 0;
    ptot += ntiles[p];
    gpbase[p] = gtot;
    gtot += d.n_rtiles;
    const int klass = render_class(d), pp = class_ppt(klass);
    const int64_t nunits = masked_ ? (int64_t)units[map[p]].size() : ((int64_t)d.H * d.W + pp - 1) / pp;
    const int64_t npix = masked_ ? nunits * pp : (int64_t)d.H * d.W;
    rendered_pixels_ += npix;
    rendered_subsamples_ += npix * d.N * d.N;
    const int nrt = (int)((nunits + rbs_ - 1) / rbs_);
    for (int t = 0; t < nrt; ++t) {
      const int64_t px = std::min<int64_t>(rbs_, nunits - (int64_t)t * rbs_) * pp;
      ritems.push_back({px * d.N * d.N, p, t, klass});
    }
    compose_tiles_ = std::max(compose_tiles_, d.n_rtiles);
    if (p % K != 0) continue;   // a composite model is blurred and compared once, on its first image
    for (int t = 0; t < d.n_ptiles; ++t)
      if (!masked_ || ptile_on[map[p]][t]) pitems.push_back({(int64_t)d.ph * d.pw, p, t, 0});
  }
  // render items: grouped by schedule class (one kernel each), longest first within a class
  auto by_class_cost = [](const Item& a, const Item& b) {
    return a.klass != b.klass ? a.klass < b.klass : a.cost > b.cost;
  };
  auto by_cost = [](const Item& a, const Item& b) { return a.cost > b.cost; };
  std::stable_sort(ritems.begin(), ritems.end(), by_class_cost);
  std::stable_sort(pitems.begin(), pitems.end(), by_cost);
  rspans_.clear();
  int cusp_slots = 0;
  for (int i = 0; i < (int)ritems.size(); ++i) {
    const int klass = ritems[i].klass;
    if (rspans_.empty() || rspans_.back().klass != klass) rspans_.push_back({klass, class_ppt(klass), i, 0, rbs_});
    ++rspans_.back().count;
    cusp_slots += (rbs_ / 64) * class_ppt(klass);
  }
  n_ritems_ = (int)ritems.size();
  n_pitems_ = (int)pitems.size();
  std::vector<int2> ri(n_ritems_), pi(n_pitems_);
  for (int i = 0; i < n_ritems_; ++i) ri[i] = make_int2(ritems[i].point, ritems[i].tile);
  // the gradient kernels take one pixel per thread: (point, tile) items, tile t
  // covering pixels 256 t .. 256 t + 255 of the support of g (tiles past the
  // support's end write zero sums)
  std::vector<int2> gi;
  if (grad)
    for (int p = 0; p < n_points; ++p)
      for (int t = 0; t < desc[map[p]].n_rtiles; ++t) gi.push_back(make_int2(p, t));
  n_gitems_ = (int)gi.size();
  for (int i = 0; i < n_pitems_; ++i) pi[i] = make_int2(pitems[i].point, pitems[i].tile);

  // one device allocation for every table and scratch buffer of the plan
  size_t off = 0;
  const size_t o_sys = off; off = align256(off + sizeof(SysDesc) * n_systems);
  const size_t o_ps = off; off = align256(off + sizeof(int) * n_points);
  const size_t o_loff = off; off = align256(off + sizeof(int64_t) * n_points);
  const size_t o_pb = off; off = align256(off + sizeof(int) * n_points);
  const size_t o_nt = off; off = align256(off + sizeof(int) * n_points);
  const size_t o_mpb = off; off = align256(off + sizeof(int) * n_models_);
  const size_t o_mnt = off; off = align256(off + sizeof(int) * n_models_);
  const size_t o_ri = off; off = align256(off + sizeof(int2) * n_ritems_);
  const size_t o_gi = off; off = align256(off + sizeof(int2) * n_gitems_);
  const size_t o_pi = off; off = align256(off + sizeof(int2) * n_pitems_);
  const size_t o_pc = off; off = align256(off + sizeof(PointConst) * n_points);
  const size_t o_mc = off; off = align256(off + (has_model_ ? sizeof(ModelConst) * n_points : 0));
  const size_t o_p64 = off; off = align256(off + sizeof(PointConst64) * n_points);
  const size_t o_psf = off; off = align256(off + 3 * sizeof(float) * psf_total);
  const size_t o_cc = off; off = align256(off + sizeof(int));
  const size_t o_ce = off; off = align256(off + sizeof(CuspEntry) * (size_t)cusp_slots);
  const size_t o_L = off; off = align256(off + sizeof(float) * (size_t)Ltot);
  const size_t o_part = off; off = align256(off + sizeof(float2) * (size_t)ptot);
  const bool g = grad != nullptr;
  const bool g17 = g && !has_model_;   // the 17-parameter adjoint (else the general-model one)
  const size_t o_gc = off; off = align256(off + (g17 ? sizeof(GradConst) * n_points : 0));
  const size_t o_R = off; off = align256(off + (g ? sizeof(float) * (size_t)Ltot : 0));
  const size_t o_gpb = off; off = align256(off + (g ? sizeof(int) * n_points : 0));
  const size_t o_gpart = off; off = align256(off + (g17 ? sizeof(float2) * (size_t)gtot * NPAR : 0));
  const size_t o_mgpart = off;
  off = align256(off + (g && has_model_ ? sizeof(double) * (size_t)gtot * params_per_point : 0));
  const size_t o_adjk = off; off = align256(off + (g ? sizeof(float) * 16 * psf_total : 0));
  const size_t o_gcorr = off; off = align256(off + (g17 ? sizeof(double) * (size_t)n_points * NPAR : 0));
  const bool composite_grad = g && K > 1;   // a component's gradient reads its model's g
  const size_t o_goff = off; off = align256(off + (composite_grad ? sizeof(int64_t) * n_points : 0));
  std::vector<size_t> o_units(n_systems), o_gsup(n_systems);
  for (int s = 0; s < n_systems; ++s) {
    o_units[s] = off;
    off = align256(off + sizeof(int) * units[s].size());
  }
  // the adjoint's support per system: its count (a 256-byte slot), pixel list
  // and two flag planes, then the render units over it (aligned)
  auto gsup_units_offset = [](size_t npix) { return align256(256 + sizeof(int) * npix + 2 * npix); };
  max_pixels_ = 0;
  for (int s = 0; s < n_systems; ++s) {
    const size_t npix = (size_t)desc[s].H * desc[s].W;
    max_pixels_ = std::max<int64_t>(max_pixels_, (int64_t)npix);
    o_gsup[s] = off;
    if (g) off = align256(align256(off + gsup_units_offset(npix) + sizeof(int) * npix) + desc[s].n_ptiles);
  }
  hipError_t e = hipMalloc((void**)&mem_, off);
  if (e != hipSuccess) {
    msg = "scratch of " + std::to_string(off) + " bytes";
    mem_ = nullptr;
    return e;
  }
  d_sys_ = (SysDesc*)(mem_ + o_sys);
  d_point_sys_ = (int*)(mem_ + o_ps);
  d_loff_ = (int64_t*)(mem_ + o_loff);
  d_pbase_ = (int*)(mem_ + o_pb);
  d_ntiles_ = (int*)(mem_ + o_nt);
  d_mpbase_ = (int*)(mem_ + o_mpb);
  d_mntiles_ = (int*)(mem_ + o_mnt);
  d_ritems_ = (int2*)(mem_ + o_ri);
  d_gitems_ = n_gitems_ ? (int2*)(mem_ + o_gi) : nullptr;
  d_pitems_ = (int2*)(mem_ + o_pi);
  d_pc_ = (PointConst*)(mem_ + o_pc);
  d_mc_ = has_model_ ? (ModelConst*)(mem_ + o_mc) : nullptr;
  d_p64_ = (PointConst64*)(mem_ + o_p64);
  cusp_.count = (int*)(mem_ + o_cc);
  cusp_.entries = (CuspEntry*)(mem_ + o_ce);
  d_L_ = (float*)(mem_ + o_L);
  d_part_ = (float2*)(mem_ + o_part);
  for (int s = 0; s < n_systems; ++s) desc[s].psfn = (float*)(mem_ + o_psf) + 3 * psf_off[s];
  if (masked_)
    for (int s = 0; s < n_systems; ++s) desc[s].active = (const int*)(mem_ + o_units[s]);
  if (g) {
    d_gc_ = g17 ? (GradConst*)(mem_ + o_gc) : nullptr;
    d_R_ = (float*)(mem_ + o_R);
    d_gpbase_ = (int*)(mem_ + o_gpb);
    d_gpart_ = g17 ? (float2*)(mem_ + o_gpart) : nullptr;
    d_mgpart_ = g17 ? nullptr : (double*)(mem_ + o_mgpart);
    d_gcorr_ = g17 ? (double*)(mem_ + o_gcorr) : nullptr;
    d_goff_ = composite_grad ? (int64_t*)(mem_ + o_goff) : nullptr;
    grad_ntiles_ = desc[0].n_rtiles;
    for (int s = 0; s < n_systems; ++s) {
      desc[s].adjk = (float*)(mem_ + o_adjk) + 16 * psf_off[s];
      const size_t npix = (size_t)desc[s].H * desc[s].W;
      desc[s].gsup_n = (int*)(mem_ + o_gsup[s]);
      desc[s].gsup = (int*)(mem_ + o_gsup[s] + 256);
      desc[s].gflags = (unsigned char*)(mem_ + o_gsup[s] + 256 + sizeof(int) * npix);
      // the forward render covers only the support too, in units rebuilt with it
      desc[s].uact = (int*)(mem_ + o_gsup[s] + gsup_units_offset(npix));
      desc[s].active = desc[s].uact;
      desc[s].uppt = has_model_ ? 1 : class_ppt(render_class(desc[s]));
      desc[s].n_active = 0;   // written by the support kernels before each render
      desc[s].ptile_w = (unsigned char*)(mem_ + align256(o_gsup[s] + gsup_units_offset(npix) + sizeof(int) * npix));
    }
  }

  std::vector<int> ps(map, map + n_points);
  std::vector<int> mpbase(n_models_), mntiles(n_models_);
  for (int m = 0; m < n_models_; ++m) {   // a model's images have consecutive partial-sum slots
    mpbase[m] = pbase[(size_t)m * G * K];
    mntiles[m] = 0;
    for (int b = 0; b < G; ++b) mntiles[m] += ntiles[((size_t)m * G + b) * K];
  }
  if ((e = hipMemcpy(d_sys_, desc.data(), sizeof(SysDesc) * n_systems, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(d_point_sys_, ps.data(), sizeof(int) * n_points, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(d_loff_, loff.data(), sizeof(int64_t) * n_points, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(d_pbase_, pbase.data(), sizeof(int) * n_points, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(d_ntiles_, ntiles.data(), sizeof(int) * n_points, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(d_mpbase_, mpbase.data(), sizeof(int) * n_models_, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(d_mntiles_, mntiles.data(), sizeof(int) * n_models_, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(d_ritems_, ri.data(), sizeof(int2) * n_ritems_, hipMemcpyHostToDevice)) != hipSuccess ||
      (n_gitems_ &&
       (e = hipMemcpy(d_gitems_, gi.data(), sizeof(int2) * n_gitems_, hipMemcpyHostToDevice)) != hipSuccess) ||
      (e = hipMemcpy(d_pitems_, pi.data(), sizeof(int2) * n_pitems_, hipMemcpyHostToDevice)) != hipSuccess ||
      (g && (e = hipMemcpy(d_gpbase_, gpbase.data(), sizeof(int) * n_points, hipMemcpyHostToDevice)) != hipSuccess)) {
    msg = "uploading work lists";
    return e;
  }
  if (d_goff_) {
    std::vector<int64_t> goff(n_points);
    for (int p = 0; p < n_points; ++p) goff[p] = loff[p - p % K];
    if ((e = hipMemcpy(d_goff_, goff.data(), sizeof(int64_t) * n_points, hipMemcpyHostToDevice)) != hipSuccess) {
      msg = "uploading the model image offsets";
      return e;
    }
  }
  if (masked_) {
    // pixels and tile sums a masked plan never computes stay zero for every run
    for (int s = 0; s < n_systems; ++s)
      if (!units[s].empty() &&
          (e = hipMemcpy((void*)desc[s].active, units[s].data(), sizeof(int) * units[s].size(),
                         hipMemcpyHostToDevice)) != hipSuccess) {
        msg = "uploading render units";
        return e;
      }
    if ((e = hipMemset(d_L_, 0, sizeof(float) * (size_t)Ltot)) != hipSuccess ||
        (e = hipMemset(d_part_, 0, sizeof(float2) * (size_t)ptot)) != hipSuccess ||
        (e = hipDeviceSynchronize()) != hipSuccess) {
      msg = "clearing the masked scratch";
      return e;
    }
  }
  return hipSuccess;
}

hipError_t BatchPlan::enqueue(hipStream_t st, hipEvent_t* ev) const {
  WorkArgs w;
  std::memset(&w, 0, sizeof(w));
  w.sys_table = d_sys_;
  w.point_sys = d_point_sys_;
  w.point_loff = d_loff_;
  w.point_pbase = d_pbase_;
  SysDesc none;
  std::memset(&none, 0, sizeof(none));
  hipError_t e;
  if (ev && (e = hipEventRecord(ev[0], st)) != hipSuccess) return e;
  // the 17-parameter prologue also normalises the PSFs; with a general model it does only that
  if ((e = launch_prologue(theta_, has_model_ ? 0 : n_points_, d_pc_, d_p64_, d_gc_, none, d_sys_,
                           (int)systems_.size(), cusp_.count, st, d_gcorr_, d_point_sys_, grad_ != nullptr)) !=
      hipSuccess)
    return e;
  if (has_model_ && (e = launch_model_prologue(theta_, n_points_, params_per_point_, spec_, d_mc_, st,
                                                grad_ != nullptr)) != hipSuccess)
    return e;
  // a gradient plan's support (the pixels g can reach, which are also the only
  // pixels its forward render needs), from the weights as they are now
  if (grad_ && (e = launch_grad_support(d_sys_, (int)systems_.size(), (int)max_pixels_, st)) != hipSuccess) return e;
  if (grad_ && (e = launch_grad_clear(w, d_L_, n_points_, st)) != hipSuccess) return e;
  if (ev && (e = hipEventRecord(ev[1], st)) != hipSuccess) return e;
  WorkArgs wr = w;
  wr.items = d_ritems_;
  wr.n_items = n_ritems_;
  if (has_model_) {
    if ((e = launch_model_render(wr, spec_, d_mc_, d_L_, n_ritems_, st)) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[2], st)) != hipSuccess) return e;
  } else {
    if ((e = launch_render(wr, d_pc_, d_p64_, d_L_, rspans_.data(), (int)rspans_.size(), cusp_, st,
                           ev ? ev[2] : nullptr)) != hipSuccess)
      return e;
    if (ev && n_ritems_ <= 0 && (e = hipEventRecord(ev[2], st)) != hipSuccess) return e;
  }
  if ((K_ > 1 || sky_) &&
      (e = launch_compose(d_L_, d_loff_, d_point_sys_, d_sys_, K_, n_images_, sky_, compose_tiles_, st)) != hipSuccess)
    return e;
  if (ev && (e = hipEventRecord(ev[3], st)) != hipSuccess) return e;
  WorkArgs wp = w;
  wp.items = d_pitems_;
  wp.n_items = n_pitems_;
  const int mode = grad_ ? 2 : 1;
  if ((e = launch_psf(wp, d_L_, d_R_, d_part_, mode, n_pitems_, square_psf_, TW_, TH_, max_ph_, max_pw_, st)) !=
      hipSuccess)
    return e;
  if (ev && (e = hipEventRecord(ev[4], st)) != hipSuccess) return e;
  if ((e = launch_finalize(d_part_, d_mpbase_, d_mntiles_, n_models_, 0, logl_, st)) != hipSuccess) return e;
  if (ev && (e = hipEventRecord(ev[5], st)) != hipSuccess) return e;
  if (grad_) {
    WorkArgs wg = w;
    wg.items = d_gitems_;
    wg.n_items = n_gitems_;
    wg.point_goff = d_goff_;
    WorkArgs wa = wp;   // the adjoint PSF: the border pass skips a model's later components
    wa.point_goff = d_goff_;
    if (grad_sky_ && (e = launch_grad_sky(d_R_, d_loff_, d_point_sys_, d_sys_, K_, n_models_, grad_sky_, st)) !=
        hipSuccess)
      return e;
    // g = A^T rho overwrites the unconvolved images, which are no longer needed
    const lensed_system& s0 = systems_[0];
    if ((e = launch_adjoint_psf(wa, d_R_, d_L_, n_pitems_, square_psf_, TW_, TH_, max_ph_, max_pw_, n_points_,
                                s0.height, s0.width, st)) != hipSuccess)
      return e;
    if (ev && (e = hipEventRecord(ev[6], st)) != hipSuccess) return e;
    if (has_model_) {
      if ((e = launch_model_grad(wg, spec_, d_mc_, d_L_, d_gpbase_, d_mgpart_, params_per_point_, n_gitems_, st)) !=
          hipSuccess)
        return e;
      if (ev && (e = hipEventRecord(ev[7], st)) != hipSuccess) return e;
      if ((e = launch_model_finalize_grad(d_mgpart_, d_gpbase_, grad_ntiles_, params_per_point_, n_points_, grad_,
                                          st)) != hipSuccess)
        return e;
    } else {
      if ((e = launch_grad(wg, d_pc_, d_p64_, d_gc_, d_L_, d_gpbase_, d_gpart_, n_gitems_, cusp_, d_gcorr_, st,
                           ev ? ev[7] : nullptr)) != hipSuccess)
        return e;
      if ((e = launch_finalize_grad(d_gpart_, d_gpbase_, grad_ntiles_, n_points_, d_gcorr_, d_pc_, d_gc_, grad_,
                                    st)) != hipSuccess)
        return e;
    }
    if (ev && (e = hipEventRecord(ev[8], st)) != hipSuccess) return e;
  } else if (ev) {
    for (int k = 6; k <= LENSED_NSTAGES; ++k)
      if ((e = hipEventRecord(ev[k], st)) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t BatchPlan::capture(hipStream_t cap) {
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t le = enqueue(cap);
  e = hipStreamEndCapture(cap, &graph_);
  if (le != hipSuccess) return le;
  if (e != hipSuccess) return e;
  return hipGraphInstantiate(&exec_, graph_, nullptr, nullptr, 0);
}

hipError_t BatchPlan::stage_ms(hipStream_t s, int stage, float* ms) const {
  hipEvent_t ev[LENSED_NSTAGES + 1] = {};
  hipError_t e = hipSuccess;
  for (auto& x : ev)
    if (e == hipSuccess) e = hipEventCreate(&x);
  // one warm-up run, then the fastest of three timed ones (the minimum is the
  // measurement least disturbed by clock changes and other work)
  if (e == hipSuccess) e = enqueue(s, ev);
  *ms = 1e30f;
  for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
    e = enqueue(s, ev);
    if (e == hipSuccess) e = hipEventSynchronize(ev[LENSED_NSTAGES]);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, ev[stage], ev[stage + 1]);
    if (e == hipSuccess && t < *ms) *ms = t;
  }
  for (auto& x : ev)
    if (x) (void)hipEventDestroy(x);
  return e;
}

hipError_t BatchPlan::run(hipStream_t s) const {
  if (exec_) return hipGraphLaunch(exec_, s);
  return enqueue(s);
}

}  // namespace lensed
