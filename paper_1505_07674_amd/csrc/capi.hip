// capi.hip -- the extern "C" boundary of liblensed_hip: contexts, validation,
// workspace, the plain launch sequences and the batched plans (work lists,
// scratch layout, captured hipGraphs).
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"
#include "lensed.h"
#include "mlp.h"
#include "plan.h"

using namespace lensed;

// The layout the Python binding mirrors (LensedSystemC).
static_assert(offsetof(lensed_system, psf) == 32 && offsetof(lensed_system, rule) == 56 &&
                  offsetof(lensed_system, amplitude) == 60 && offsetof(lensed_system, zero_point) == 64 &&
                  offsetof(lensed_system, source_position) == 68 && sizeof(lensed_system) == 72,
              "lensed_system layout");
static_assert(offsetof(lensed_model, n_planes) == 48 && offsetof(lensed_model, beta) == 88 &&
                  sizeof(lensed_model) == 600,
              "lensed_model layout");

struct lensed_ctx {
  int device = 0;
  hipStream_t cap = nullptr;        // private stream used only for graph capture
  std::string err;
  char* arena = nullptr;            // workspace of the plain calls
  size_t arena_bytes = 0;
  bool use_graphs = true;
  bool autotune = true;             // time the best-ranked tile shapes on the first batch of a shape set
  int force_ppt = 0;                // 1 or 2: render pixels per thread fixed (not timed)
  int force_block = 0;              // 128, 256 or 512: render threads per block fixed (not timed)
  std::vector<std::unique_ptr<BatchPlan>> plans;   // most recently used last
  TileCache tiles;
  bool profiling = false;                          // per-stage hipEvents, no graphs
  std::vector<std::vector<hipEvent_t>> pending;    // event sets of profiled calls
  double stage_ms[LENSED_NSTAGES] = {0};
  int schedule[4] = {0, 0, 0, 0};   // of the last batched plan run: PSF tile width, height; render pixels per
                                    // thread, threads per render block
  int64_t rendered[2] = {0, 0};  // of the last batched plan run: pixels and subsamples rendered per launch
  int stage_calls = 0;
  char* mlp_mem = nullptr;                          // surrogate scratch
  MlpScratch mlp;
  std::vector<int32_t> composite_map;               // system of every point of a composite launch
};

namespace {

int set_err(lensed_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(lensed_ctx* c, hipError_t e, const char* what) {
  const int code = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? LENSED_OUT_OF_MEMORY
                                                                                : LENSED_HIP_ERROR;
  return set_err(c, code, std::string(what) + ": " + hipGetErrorString(e));
}

#define LENSED_HIP(ctx, call)                          \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
  } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int ensure_arena(lensed_ctx* c, size_t bytes) {
  if (c->arena_bytes >= bytes) return LENSED_OK;
  if (c->arena) {
    // earlier calls may still use the old workspace
    LENSED_HIP(c, hipDeviceSynchronize());
    LENSED_HIP(c, hipFree(c->arena));
    c->arena = nullptr;
    c->arena_bytes = 0;
  }
  const size_t n = align_up(std::max(bytes, (size_t)1 << 20), (size_t)1 << 20);
  LENSED_HIP(c, hipMalloc((void**)&c->arena, n));
  c->arena_bytes = n;
  return LENSED_OK;
}

int ensure_mlp(lensed_ctx* c, int rows) {
  if (c->mlp.cap >= rows) return LENSED_OK;
  if (c->mlp_mem) {
    LENSED_HIP(c, hipDeviceSynchronize());
    LENSED_HIP(c, hipFree(c->mlp_mem));
    c->mlp_mem = nullptr;
    c->mlp = MlpScratch();
  }
  const size_t R = (size_t)std::max(rows, 256);
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off = align_up(off + bytes, 256); return o; };
  const size_t o_wb = take(sizeof(uint16_t) * MLP_WB_SIZE);
  const size_t o_x0 = take(sizeof(uint16_t) * R * MLP_KPAD);
  size_t o_z[3], o_h[3];
  for (int l = 0; l < 3; ++l) {
    o_z[l] = take(sizeof(float) * R * MLP_H);
    o_h[l] = take(sizeof(uint16_t) * R * MLP_H);
  }
  const size_t o_d = take(sizeof(float) * R), o_sq = take(sizeof(float) * R);
  const size_t o_dz = take(sizeof(float) * R * MLP_H), o_dz2 = take(sizeof(float) * R * MLP_H);
  const size_t o_dzb = take(sizeof(uint16_t) * R * MLP_H), o_dzb2 = take(sizeof(uint16_t) * R * MLP_H);
  const size_t o_g = take(sizeof(float) * MLP_NPARAM);
  LENSED_HIP(c, hipMalloc((void**)&c->mlp_mem, off));
  char* b = c->mlp_mem;
  c->mlp.cap = (int)R;
  c->mlp.wb = (uint16_t*)(b + o_wb);
  c->mlp.X0 = (uint16_t*)(b + o_x0);
  for (int l = 0; l < 3; ++l) {
    c->mlp.Z[l] = (float*)(b + o_z[l]);
    c->mlp.H[l] = (uint16_t*)(b + o_h[l]);
  }
  c->mlp.d = (float*)(b + o_d);
  c->mlp.sq = (float*)(b + o_sq);
  c->mlp.dZ = (float*)(b + o_dz);
  c->mlp.dZ2 = (float*)(b + o_dz2);
  c->mlp.dZb = (uint16_t*)(b + o_dzb);
  c->mlp.dZb2 = (uint16_t*)(b + o_dzb2);
  c->mlp.grad = (float*)(b + o_g);
  return LENSED_OK;
}

constexpr int MLP_MAX_BATCH = 1 << 16;

int check_mlp_batch(lensed_ctx* c, int batch) {
  if (batch < 0 || batch > MLP_MAX_BATCH)
    return set_err(c, LENSED_INVALID_ARGUMENT, "batch must be in 0.." + std::to_string(MLP_MAX_BATCH));
  return LENSED_OK;
}

}  // namespace

namespace lensed {

int validate_system(lensed_ctx* c, const lensed_system* s, bool need_data, int index) {
  const std::string where = index >= 0 ? "system " + std::to_string(index) + ": " : "";
  if (!s) return set_err(c, LENSED_INVALID_ARGUMENT, where + "system is NULL");
  if (s->height <= 0 || s->width <= 0) return set_err(c, LENSED_INVALID_ARGUMENT, where + "height and width must be > 0");
  if ((int64_t)s->height * s->width > ((int64_t)1 << 28))
    return set_err(c, LENSED_INVALID_ARGUMENT, where + "image larger than 2^28 pixels");
  if (!(s->pixscale > 0.0f) || !std::isfinite(s->pixscale))
    return set_err(c, LENSED_INVALID_ARGUMENT, where + "pixscale must be finite and > 0");
  if (!std::isfinite(s->center_x) || !std::isfinite(s->center_y))
    return set_err(c, LENSED_INVALID_ARGUMENT, where + "grid centre must be finite");
  if (s->rule < LENSED_RULE_MIDPOINT || s->rule > LENSED_RULE_G7K15)
    return set_err(c, LENSED_INVALID_ARGUMENT, where + "rule must be one of the LENSED_RULE_* values");
  if (s->rule == LENSED_RULE_MIDPOINT && (s->nsub < 1 || s->nsub > 16))
    return set_err(c, LENSED_INVALID_ARGUMENT, where + "nsub must be in 1..16");
  if (s->psf_h < 1 || s->psf_w < 1 || s->psf_h % 2 == 0 || s->psf_w % 2 == 0)
    return set_err(c, LENSED_INVALID_ARGUMENT, where + "PSF dimensions must be odd and >= 1");
  if (s->psf_h > MAX_PSF || s->psf_w > MAX_PSF)
    return set_err(c, LENSED_INVALID_ARGUMENT, where + "PSF side larger than " + std::to_string(MAX_PSF));
  if (!s->psf) return set_err(c, LENSED_INVALID_ARGUMENT, where + "psf is NULL");
  if (s->amplitude != LENSED_AMP_INTENSITY && s->amplitude != LENSED_AMP_MAGNITUDE)
    return set_err(c, LENSED_INVALID_ARGUMENT, where + "amplitude must be LENSED_AMP_INTENSITY or LENSED_AMP_MAGNITUDE");
  if (!std::isfinite(s->zero_point)) return set_err(c, LENSED_INVALID_ARGUMENT, where + "zero_point must be finite");
  if (s->source_position != LENSED_SOURCE_PLANE && s->source_position != LENSED_IMAGE_PLANE)
    return set_err(c, LENSED_INVALID_ARGUMENT,
                   where + "source_position must be LENSED_SOURCE_PLANE or LENSED_IMAGE_PLANE");
  if (need_data && (!s->data || !s->weight))
    return set_err(c, LENSED_INVALID_ARGUMENT, where + "data and weight are required");
  return LENSED_OK;
}

SysDesc make_desc(const lensed_system& s, const TileShape& t) {
  SysDesc d;
  std::memset(&d, 0, sizeof(d));
  d.H = s.height;
  d.W = s.width;
  d.rule = s.rule;
  d.amp = s.amplitude;
  d.zp = s.zero_point;
  d.srcpos = s.source_position;
  d.N = s.rule == LENSED_RULE_MIDPOINT ? s.nsub : 2 * (2 * s.rule + 1) + 1;   // g3k7, g5k11, g7k15: 7, 11, 15 nodes
  d.ph = s.psf_h;
  d.pw = s.psf_w;
  d.d = s.pixscale;
  d.cx = s.center_x;
  d.cy = s.center_y;
  d.psf = s.psf;
  d.psfn = nullptr;
  d.data = s.data;
  d.weight = s.weight;
  d.TW = t.TW;
  d.TH = t.TH;
  d.tiles_x = (s.width + t.TW - 1) / t.TW;
  d.n_ptiles = d.tiles_x * ((s.height + t.TH - 1) / t.TH);
  d.n_rtiles = (int)(((int64_t)s.height * s.width + RENDER_BLOCK - 1) / RENDER_BLOCK);
  // the midpoint weights 1/N^2 are folded here; the Gauss-Kronrod weights (summing to 1) multiply in the kernel
  d.wgt = (double)s.pixscale * (double)s.pixscale /
          (s.rule == LENSED_RULE_MIDPOINT ? (double)s.nsub * (double)s.nsub : 1.0);
  set_row_divisor(d);
  return d;
}

int square_psf_code(int ph, int pw) {
  if (ph != pw) return -1;
  return (ph == 21 || ph == 7 || ph == 1) ? ph : -1;
}

}  // namespace lensed

extern "C" {

int lensed_param_count(void) { return LENSED_NPARAM; }

const char* lensed_status_string(int status) {
  switch (status) {
    case LENSED_OK: return "ok";
    case LENSED_INVALID_ARGUMENT: return "invalid argument";
    case LENSED_HIP_ERROR: return "HIP runtime error";
    case LENSED_OUT_OF_MEMORY: return "out of device memory";
    case LENSED_NOT_SUPPORTED: return "not supported";
    case LENSED_TOO_LARGE: return "input exceeds the static workspace";
    default: return "unknown status";
  }
}

const char* lensed_last_error(const lensed_ctx* ctx) { return ctx ? ctx->err.c_str() : "no context"; }

int lensed_create(lensed_ctx** out, int device) {
  if (!out) return LENSED_INVALID_ARGUMENT;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return LENSED_NOT_SUPPORTED;
  if (device < 0 || device >= count) return LENSED_INVALID_ARGUMENT;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return LENSED_HIP_ERROR;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return LENSED_NOT_SUPPORTED;
  if (hipSetDevice(device) != hipSuccess) return LENSED_HIP_ERROR;
  auto* c = new lensed_ctx();
  c->device = device;
  if (hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return LENSED_HIP_ERROR;
  }
  const char* g = std::getenv("LENSED_NO_GRAPHS");
  c->use_graphs = !(g && g[0] == '1');
  const char* t = std::getenv("LENSED_NO_AUTOTUNE");
  c->autotune = !(t && t[0] == '1');
  const char* r = std::getenv("LENSED_RENDER_PPT");
  c->force_ppt = (r && (r[0] == '1' || r[0] == '2') && r[1] == 0) ? r[0] - '0' : 0;
  const char* rb = std::getenv("LENSED_RENDER_BLOCK");
  const int fb = rb ? std::atoi(rb) : 0;
  c->force_block = (fb == 128 || fb == 256 || fb == 512) ? fb : 0;
  *out = c;
  return LENSED_OK;
}

void lensed_destroy(lensed_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  c->plans.clear();
  for (auto& ev : c->pending)
    for (auto& e : ev) (void)hipEventDestroy(e);
  if (c->arena) (void)hipFree(c->arena);
  if (c->mlp_mem) (void)hipFree(c->mlp_mem);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  delete c;
}

int lensed_render(lensed_ctx* c, const lensed_system* sys, const float* theta, float* image, int apply_psf,
                  void* stream) {
  if (!c) return LENSED_INVALID_ARGUMENT;
  int rc = validate_system(c, sys, false, -1);
  if (rc) return rc;
  if (!theta || !image) return set_err(c, LENSED_INVALID_ARGUMENT, "theta and image are required");
  LENSED_HIP(c, hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  const TileShape ts = TileCache::latency_best(*sys);   // one image: a latency-ranked tile
  SysDesc sd = make_desc(*sys, ts);
  const size_t npix = (size_t)sd.H * sd.W;
  const size_t off_pc = 0;
  const size_t off_p64 = align_up(off_pc + sizeof(PointConst), 256);
  const size_t off_psf = align_up(off_p64 + sizeof(PointConst64), 256);
  const size_t off_cc = align_up(off_psf + 3 * sizeof(float) * sd.ph * sd.pw, 256);
  const size_t off_ce = align_up(off_cc + sizeof(int), 256);
  const size_t off_L = align_up(off_ce + sizeof(CuspEntry) * (size_t)sd.n_rtiles * (RENDER_BLOCK / 64), 256);
  const size_t total = align_up(off_L + sizeof(float) * npix, 256);
  if ((rc = ensure_arena(c, total))) return rc;
  PointConst* pc = (PointConst*)(c->arena + off_pc);
  PointConst64* p64 = (PointConst64*)(c->arena + off_p64);
  CuspList cl{(CuspEntry*)(c->arena + off_ce), (int*)(c->arena + off_cc)};
  sd.psfn = (float*)(c->arena + off_psf);
  float* L = apply_psf ? (float*)(c->arena + off_L) : image;
  WorkArgs w;
  std::memset(&w, 0, sizeof(w));
  w.single = sd;
  LENSED_HIP(c, launch_prologue(theta, 1, pc, p64, nullptr, sd, nullptr, 1, cl.count, st));
  LENSED_HIP(c, launch_render(w, pc, p64, L, sd.n_rtiles, cl, st));
  if (apply_psf)
    LENSED_HIP(c, launch_psf(w, L, image, nullptr, 0, sd.n_ptiles, square_psf_code(sd.ph, sd.pw), sd.TW, sd.TH,
                             sd.ph, sd.pw, st));
  return LENSED_OK;
}

int lensed_render_composite(lensed_ctx* c, const lensed_system* sys, const float* theta, int n_components, float sky,
                            float* image, int apply_psf, void* stream) {
  if (!c) return LENSED_INVALID_ARGUMENT;
  int rc = validate_system(c, sys, false, -1);
  if (rc) return rc;
  if (n_components < 1 || n_components > 64)
    return set_err(c, LENSED_INVALID_ARGUMENT, "n_components must be in 1..64");
  if (!std::isfinite(sky)) return set_err(c, LENSED_INVALID_ARGUMENT, "sky must be finite");
  if (!theta || !image) return set_err(c, LENSED_INVALID_ARGUMENT, "theta and image are required");
  LENSED_HIP(c, hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  const int K = n_components;
  const TileShape ts = TileCache::latency_best(*sys);   // one image: a latency-ranked tile
  SysDesc sd = make_desc(*sys, ts);
  const size_t npix = (size_t)sd.H * sd.W;
  const size_t off_pc = 0;
  const size_t off_p64 = align_up(off_pc + sizeof(PointConst) * K, 256);
  const size_t off_psf = align_up(off_p64 + sizeof(PointConst64) * K, 256);
  const size_t off_cc = align_up(off_psf + 3 * sizeof(float) * sd.ph * sd.pw, 256);
  const size_t off_ce = align_up(off_cc + sizeof(int), 256);
  const size_t off_L = align_up(off_ce + sizeof(CuspEntry) * (size_t)sd.n_rtiles * (RENDER_BLOCK / 64), 256);
  const size_t total = align_up(off_L + sizeof(float) * npix * K, 256);
  if ((rc = ensure_arena(c, total))) return rc;
  PointConst* pc = (PointConst*)(c->arena + off_pc);
  PointConst64* p64 = (PointConst64*)(c->arena + off_p64);
  CuspList cl{(CuspEntry*)(c->arena + off_ce), (int*)(c->arena + off_cc)};
  sd.psfn = (float*)(c->arena + off_psf);
  float* L = (float*)(c->arena + off_L);
  WorkArgs w;
  std::memset(&w, 0, sizeof(w));
  w.single = sd;
  LENSED_HIP(c, launch_prologue(theta, K, pc, p64, nullptr, sd, nullptr, 1, cl.count, st));
  for (int j = 0; j < K; ++j) {       // one component at a time: its cusp list starts empty
    if (j > 0) LENSED_HIP(c, launch_zero_count(cl.count, st));
    w.point0 = j;
    LENSED_HIP(c, launch_render(w, pc, p64, L + (size_t)j * npix, sd.n_rtiles, cl, st));
  }
  const double sky_px = (double)sky * (double)sd.d * (double)sd.d;
  LENSED_HIP(c, launch_sum_images(L, (int64_t)npix, K, sky_px, apply_psf ? L : image, st));
  w.point0 = 0;
  if (apply_psf)
    LENSED_HIP(c, launch_psf(w, L, image, nullptr, 0, sd.n_ptiles, square_psf_code(sd.ph, sd.pw), sd.TW, sd.TH,
                             sd.ph, sd.pw, st));
  return LENSED_OK;
}

int lensed_render_error(lensed_ctx* c, const lensed_system* sys, const float* theta, float* error, void* stream) {
  if (!c) return LENSED_INVALID_ARGUMENT;
  int rc = validate_system(c, sys, false, -1);
  if (rc) return rc;
  if (sys->rule == LENSED_RULE_MIDPOINT)
    return set_err(c, LENSED_INVALID_ARGUMENT, "the error estimate needs a Gauss-Kronrod rule");
  if (!theta || !error) return set_err(c, LENSED_INVALID_ARGUMENT, "theta and error are required");
  LENSED_HIP(c, hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  const TileShape ts = TileCache::latency_best(*sys);   // one image: a latency-ranked tile
  SysDesc sd = make_desc(*sys, ts);
  const size_t off_pc = 0;
  const size_t off_p64 = align_up(off_pc + sizeof(PointConst), 256);
  const size_t off_psf = align_up(off_p64 + sizeof(PointConst64), 256);
  const size_t off_cc = align_up(off_psf + 3 * sizeof(float) * sd.ph * sd.pw, 256);
  const size_t total = align_up(off_cc + sizeof(int), 256);
  if ((rc = ensure_arena(c, total))) return rc;
  PointConst* pc = (PointConst*)(c->arena + off_pc);
  PointConst64* p64 = (PointConst64*)(c->arena + off_p64);
  sd.psfn = (float*)(c->arena + off_psf);
  WorkArgs w;
  std::memset(&w, 0, sizeof(w));
  w.single = sd;
  LENSED_HIP(c, launch_prologue(theta, 1, pc, p64, nullptr, sd, nullptr, 1, (int*)(c->arena + off_cc), st));
  LENSED_HIP(c, launch_rule_error(w, pc, error, sd.n_rtiles, st));
  return LENSED_OK;
}

int lensed_weights_from_data(lensed_ctx* c, const float* data, int64_t n, double gain, const float* gain_map,
                             double offset, const float* offset_map, const float* extra, float* weight,
                             void* stream) {
  if (!c) return LENSED_INVALID_ARGUMENT;
  if (n < 0) return set_err(c, LENSED_INVALID_ARGUMENT, "n must be >= 0");
  if (n > 0 && (!data || !weight)) return set_err(c, LENSED_INVALID_ARGUMENT, "data and weight are required");
  if (!gain_map && !(std::isfinite(gain) && gain > 0.0))
    return set_err(c, LENSED_INVALID_ARGUMENT, "gain must be finite and > 0");
  if (!offset_map && !std::isfinite(offset)) return set_err(c, LENSED_INVALID_ARGUMENT, "offset must be finite");
  LENSED_HIP(c, hipSetDevice(c->device));
  LENSED_HIP(c, launch_weights_from_data(data, n, gain, gain_map, offset, offset_map, extra, weight,
                                         (hipStream_t)stream));
  return LENSED_OK;
}

int lensed_loglike(lensed_ctx* c, const lensed_system* sys, const float* theta, double* logl, void* stream) {
  if (!c) return LENSED_INVALID_ARGUMENT;
  int rc = validate_system(c, sys, true, -1);
  if (rc) return rc;
  if (!theta || !logl) return set_err(c, LENSED_INVALID_ARGUMENT, "theta and logl are required");
  LENSED_HIP(c, hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  const TileShape ts = TileCache::latency_best(*sys);   // one image: a latency-ranked tile
  SysDesc sd = make_desc(*sys, ts);
  const size_t npix = (size_t)sd.H * sd.W;
  const size_t off_pc = 0;
  const size_t off_p64 = align_up(off_pc + sizeof(PointConst), 256);
  const size_t off_psf = align_up(off_p64 + sizeof(PointConst64), 256);
  const size_t off_cc = align_up(off_psf + 3 * sizeof(float) * sd.ph * sd.pw, 256);
  const size_t off_ce = align_up(off_cc + sizeof(int), 256);
  const size_t off_L = align_up(off_ce + sizeof(CuspEntry) * (size_t)sd.n_rtiles * (RENDER_BLOCK / 64), 256);
  const size_t off_part = align_up(off_L + sizeof(float) * npix, 256);
  const size_t total = align_up(off_part + sizeof(float2) * sd.n_ptiles, 256);
  if ((rc = ensure_arena(c, total))) return rc;
  PointConst* pc = (PointConst*)(c->arena + off_pc);
  PointConst64* p64 = (PointConst64*)(c->arena + off_p64);
  CuspList cl{(CuspEntry*)(c->arena + off_ce), (int*)(c->arena + off_cc)};
  sd.psfn = (float*)(c->arena + off_psf);
  float* L = (float*)(c->arena + off_L);
  float2* part = (float2*)(c->arena + off_part);
  WorkArgs w;
  std::memset(&w, 0, sizeof(w));
  w.single = sd;
  LENSED_HIP(c, launch_prologue(theta, 1, pc, p64, nullptr, sd, nullptr, 1, cl.count, st));
  LENSED_HIP(c, launch_render(w, pc, p64, L, sd.n_rtiles, cl, st));
  LENSED_HIP(c, launch_psf(w, L, nullptr, part, 1, sd.n_ptiles, square_psf_code(sd.ph, sd.pw), sd.TW, sd.TH, sd.ph,
                           sd.pw, st));
  LENSED_HIP(c, launch_finalize(part, nullptr, nullptr, 1, sd.n_ptiles, logl, st));
  return LENSED_OK;
}

namespace {

// The batched log L of lensed_loglike_batch (K = 1, no sky) and of
// lensed_loglike_composite: find or build the plan for these arguments (with
// the autotuner on a new set of shapes), then replay its graph.
int run_batch(lensed_ctx* c, const lensed_system* systems, int n_systems, const float* theta,
              const int32_t* system_of_point, int n_points, double* logl, void* stream, int K, const float* sky,
              int G = 1, const ModelSpec* model = nullptr, int params_per_point = NPAR, bool masked = false) {
  BatchPlan* plan = nullptr;
  for (size_t i = 0; i < c->plans.size(); ++i) {
    if (c->plans[i]->matches(systems, n_systems, theta, system_of_point, n_points, logl, nullptr, K, sky, G,
                             model, masked)) {
      std::unique_ptr<BatchPlan> keep = std::move(c->plans[i]);
      c->plans.erase(c->plans.begin() + i);
      c->plans.push_back(std::move(keep));
      plan = c->plans.back().get();
      break;
    }
  }
  if (!plan) {
    if (c->plans.size() >= 8) {
      LENSED_HIP(c, hipDeviceSynchronize());
      c->plans.erase(c->plans.begin());
    }
    if (c->autotune && !c->tiles.has_measured(systems, n_systems)) {
      // Autotuner: time the PSF + chi^2 stage of the model's best-ranked tile
      // shapes on this very launch (stage by stage, fastest of three runs after a
      // warm-up) and keep
      // the fastest for every later plan over the same set of system shapes.
      const std::vector<TileShape> cand = c->tiles.ranked(systems, n_systems, 6);
      TileShape best = cand.empty() ? TileShape{32, 32} : cand[0];
      float best_ms = 1e30f;
      for (const TileShape& t : cand) {
        BatchPlan trial;
        std::string msg;
        if (trial.build(systems, n_systems, theta, system_of_point, n_points, logl, c->tiles, msg, nullptr, &t, K,
                        sky, G, model, params_per_point, 0, masked) != hipSuccess) {
          (void)hipGetLastError();
          continue;
        }
        float ms = 0.0f;
        LENSED_HIP(c, trial.psf_ms((hipStream_t)stream, &ms));
        if (ms < best_ms) {
          best_ms = ms;
          best = t;
        }
      }
      c->tiles.set_measured(systems, n_systems, best);
    }
    if (model) {
      // the general-model render takes one pixel per thread in 256-thread blocks
      c->tiles.set_render_measured(systems, n_systems, RenderSchedule{1, RENDER_BLOCK});
    } else if (c->force_ppt || c->force_block) {
      c->tiles.set_render_measured(systems, n_systems,
                                   RenderSchedule{c->force_ppt ? c->force_ppt : 1,
                                                  c->force_block ? c->force_block : RENDER_BLOCK});
    } else if (c->autotune && !c->tiles.has_render_measured(systems, n_systems)) {
      // Render schedule: one or two pixels per thread (two share the row terms
      // of the subsample grid) in blocks of 128, 256 or 512 threads, timed the
      // same way on this launch's render kernels.
      RenderSchedule best{1, RENDER_BLOCK};
      float best_ms = 1e30f;
      bool pairs = true;
      for (int ppt = 1; ppt <= 2 && pairs; ++ppt) {
        for (const int bs : {128, 256, 512}) {
          const RenderSchedule cand{ppt, bs};
          BatchPlan trial;
          std::string msg;
          if (trial.build(systems, n_systems, theta, system_of_point, n_points, logl, c->tiles, msg, nullptr, nullptr,
                          K, sky, G, model, params_per_point, &cand, masked) != hipSuccess) {
            (void)hipGetLastError();
            continue;
          }
          if (ppt == 2 && trial.max_ppt() < 2) {   // no class of this launch takes two pixels
            pairs = false;
            break;
          }
          float ms = 0.0f;
          LENSED_HIP(c, trial.render_ms((hipStream_t)stream, &ms));
          if (ms < best_ms) {
            best_ms = ms;
            best = cand;
          }
        }
      }
      c->tiles.set_render_measured(systems, n_systems, best);
    }
    std::unique_ptr<BatchPlan> np(new BatchPlan());
    std::string msg;
    hipError_t e = np->build(systems, n_systems, theta, system_of_point, n_points, logl, c->tiles, msg, nullptr,
                             nullptr, K, sky, G, model, params_per_point, nullptr, masked);
    if (e != hipSuccess) return hip_fail(c, e, ("batch plan: " + msg).c_str());
    if (c->use_graphs) {
      e = np->capture(c->cap);
      if (e != hipSuccess) return hip_fail(c, e, "batch plan graph capture");
    }
    c->plans.push_back(std::move(np));
    plan = c->plans.back().get();
  }
  c->schedule[0] = plan->psf_tile().TW;
  c->schedule[1] = plan->psf_tile().TH;
  c->schedule[2] = plan->render_ppt();
  c->schedule[3] = plan->render_block();
  c->rendered[0] = plan->rendered_pixels();
  c->rendered[1] = plan->rendered_subsamples();
  if (c->profiling) {
    std::vector<hipEvent_t> ev(LENSED_NSTAGES + 1);
    for (auto& e : ev) LENSED_HIP(c, hipEventCreate(&e));
    LENSED_HIP(c, plan->enqueue((hipStream_t)stream, ev.data()));
    c->pending.push_back(std::move(ev));
    return LENSED_OK;
  }
  LENSED_HIP(c, plan->run((hipStream_t)stream));
  return LENSED_OK;
}

}  // namespace

int lensed_loglike_batch(lensed_ctx* c, const lensed_system* systems, int n_systems, const float* theta,
                         const int32_t* system_of_point, int n_points, double* logl, void* stream) {
  if (!c) return LENSED_INVALID_ARGUMENT;
  if (n_points < 0) return set_err(c, LENSED_INVALID_ARGUMENT, "n_points must be >= 0");
  if (n_points == 0) return LENSED_OK;
  if (!systems || n_systems <= 0) return set_err(c, LENSED_INVALID_ARGUMENT, "at least one system is required");
  if (!theta || !logl || !system_of_point)
    return set_err(c, LENSED_INVALID_ARGUMENT, "theta, system_of_point and logl are required");
  for (int s = 0; s < n_systems; ++s) {
    const int rc = validate_system(c, &systems[s], true, s);
    if (rc) return rc;
  }
  for (int p = 0; p < n_points; ++p)
    if (system_of_point[p] < 0 || system_of_point[p] >= n_systems)
      return set_err(c, LENSED_INVALID_ARGUMENT, "system_of_point[" + std::to_string(p) + "] out of range");
  LENSED_HIP(c, hipSetDevice(c->device));
  return run_batch(c, systems, n_systems, theta, system_of_point, n_points, logl, stream, 1, nullptr);
}

int lensed_loglike_batch_masked(lensed_ctx* c, const lensed_system* systems, int n_systems, const float* theta,
                                const int32_t* system_of_point, int n_points, double* logl, void* stream) {
  if (!c) return LENSED_INVALID_ARGUMENT;
  if (n_points < 0) return set_err(c, LENSED_INVALID_ARGUMENT, "n_points must be >= 0");
  if (n_points == 0) return LENSED_OK;
  if (!systems || n_systems <= 0) return set_err(c, LENSED_INVALID_ARGUMENT, "at least one system is required");
  if (!theta || !logl || !system_of_point)
    return set_err(c, LENSED_INVALID_ARGUMENT, "theta, system_of_point and logl are required");
  for (int s = 0; s < n_systems; ++s) {
    const int rc = validate_system(c, &systems[s], true, s);
    if (rc) return rc;
  }
  for (int p = 0; p < n_points; ++p)
    if (system_of_point[p] < 0 || system_of_point[p] >= n_systems)
      return set_err(c, LENSED_INVALID_ARGUMENT, "system_of_point[" + std::to_string(p) + "] out of range");
  LENSED_HIP(c, hipSetDevice(c->device));
  return run_batch(c, systems, n_systems, theta, system_of_point, n_points, logl, stream, 1, nullptr, 1, nullptr,
                   NPAR, true);
}

int lensed_loglike_composite(lensed_ctx* c, const lensed_system* systems, int n_systems, const float* theta,
                             int n_components, const float* sky, const int32_t* system_of_model, int n_models,
                             double* logl, void* stream) {
  if (!c) return LENSED_INVALID_ARGUMENT;
  if (n_models < 0) return set_err(c, LENSED_INVALID_ARGUMENT, "n_models must be >= 0");
  if (n_components < 1) return set_err(c, LENSED_INVALID_ARGUMENT, "n_components must be >= 1");
  if (n_models == 0) return LENSED_OK;
  if ((int64_t)n_models * n_components > INT32_MAX / NPAR)
    return set_err(c, LENSED_INVALID_ARGUMENT, "n_models x n_components too large");
  if (!systems || n_systems <= 0) return set_err(c, LENSED_INVALID_ARGUMENT, "at least one system is required");
  if (!theta || !logl || !system_of_model)
    return set_err(c, LENSED_INVALID_ARGUMENT, "theta, system_of_model and logl are required");
  for (int s = 0; s < n_systems; ++s) {
    const int rc = validate_system(c, &systems[s], true, s);
    if (rc) return rc;
  }
  for (int m = 0; m < n_models; ++m)
    if (system_of_model[m] < 0 || system_of_model[m] >= n_systems)
      return set_err(c, LENSED_INVALID_ARGUMENT, "system_of_model[" + std::to_string(m) + "] out of range");
  LENSED_HIP(c, hipSetDevice(c->device));
  const int n_points = n_models * n_components;
  c->composite_map.resize(n_points);
  for (int p = 0; p < n_points; ++p) c->composite_map[p] = system_of_model[p / n_components];
  return run_batch(c, systems, n_systems, theta, c->composite_map.data(), n_points, logl, stream, n_components, sky);
}

namespace {

// The device copy of a validated lensed_model.
int model_spec(lensed_ctx* c, const lensed_model* m, ModelSpec& spec) {
  if (!m) return set_err(c, LENSED_INVALID_ARGUMENT, "model is NULL");
  if (m->n_sie < 0 || m->n_sie > MAX_SIE) return set_err(c, LENSED_INVALID_ARGUMENT, "n_sie must be in 0..8");
  if (m->n_sersic < 1 || m->n_sersic > MAX_SERSIC)
    return set_err(c, LENSED_INVALID_ARGUMENT, "n_sersic must be in 1..8");
  if ((m->shear != 0 && m->shear != 1) || (m->sky != 0 && m->sky != 1))
    return set_err(c, LENSED_INVALID_ARGUMENT, "shear and sky must be 0 or 1");
  if (m->n_planes < 0 || m->n_planes > MAX_PLANES)
    return set_err(c, LENSED_INVALID_ARGUMENT, "n_planes must be in 0..8");
  const int P = m->n_planes < 1 ? 1 : m->n_planes;
  std::memset(&spec, 0, sizeof(spec));
  spec.n_sie = m->n_sie;
  spec.shear = m->shear;
  spec.n_sersic = m->n_sersic;
  spec.sky = m->sky;
  spec.n_planes = P;
  for (int j = 0; j < m->n_sersic; ++j) {
    if (m->plane[j] < 0 || m->plane[j] > P)
      return set_err(c, LENSED_INVALID_ARGUMENT,
                     "plane[" + std::to_string(j) + "] must be a plane index in 0..n_planes");
    spec.plane[j] = m->plane[j];
  }
  if (P > 1) {
    for (int k = 0; k < m->n_sie; ++k) {
      if (m->sie_plane[k] < 0 || m->sie_plane[k] >= P)
        return set_err(c, LENSED_INVALID_ARGUMENT,
                       "sie_plane[" + std::to_string(k) + "] must be a lens plane in 0..n_planes-1");
      spec.sie_plane[k] = m->sie_plane[k];
    }
    for (int i = 0; i < P; ++i)
      for (int j = i + 1; j < P; ++j) {
        if (!(m->beta[i][j] >= 0.0 && m->beta[i][j] <= 1.0))
          return set_err(c, LENSED_INVALID_ARGUMENT,
                         "beta[" + std::to_string(i) + "][" + std::to_string(j) + "] must be in [0, 1]");
        spec.beta[i][j] = m->beta[i][j];
      }
  }
  return LENSED_OK;
}

int spec_params(const ModelSpec& s) { return 5 * s.n_sie + (s.shear ? 2 : 0) + 7 * s.n_sersic + (s.sky ? 1 : 0); }

}  // namespace

int lensed_model_nparams(const lensed_model* model) {
  ModelSpec spec;
  if (model_spec(nullptr, model, spec) != LENSED_OK) return -1;
  return spec_params(spec);
}

int lensed_render_model(lensed_ctx* c, const lensed_system* sys, const lensed_model* model, const float* theta,
                        float* image, int apply_psf, void* stream) {
  if (!c) return LENSED_INVALID_ARGUMENT;
  int rc = validate_system(c, sys, false, -1);
  if (rc) return rc;
  ModelSpec spec;
  if ((rc = model_spec(c, model, spec))) return rc;
  if (!theta || !image) return set_err(c, LENSED_INVALID_ARGUMENT, "theta and image are required");
  LENSED_HIP(c, hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  const TileShape ts = TileCache::latency_best(*sys);   // one image: a latency-ranked tile
  SysDesc sd = make_desc(*sys, ts);
  const size_t npix = (size_t)sd.H * sd.W;
  const size_t off_mc = 0;
  const size_t off_psf = align_up(off_mc + sizeof(ModelConst), 256);
  const size_t off_cc = align_up(off_psf + 3 * sizeof(float) * sd.ph * sd.pw, 256);
  const size_t off_L = align_up(off_cc + sizeof(int), 256);
  const size_t total = align_up(off_L + sizeof(float) * npix, 256);
  if ((rc = ensure_arena(c, total))) return rc;
  ModelConst* mc = (ModelConst*)(c->arena + off_mc);
  sd.psfn = (float*)(c->arena + off_psf);
  float* L = apply_psf ? (float*)(c->arena + off_L) : image;
  WorkArgs w;
  std::memset(&w, 0, sizeof(w));
  w.single = sd;
  // the 17-parameter prologue with no points normalises the PSF
  LENSED_HIP(c, launch_prologue(theta, 0, nullptr, nullptr, nullptr, sd, nullptr, 1, (int*)(c->arena + off_cc), st));
  LENSED_HIP(c, launch_model_prologue(theta, 1, spec_params(spec), spec, mc, st));
  LENSED_HIP(c, launch_model_render(w, spec, mc, L, sd.n_rtiles, st));
  if (apply_psf)
    LENSED_HIP(c, launch_psf(w, L, image, nullptr, 0, sd.n_ptiles, square_psf_code(sd.ph, sd.pw), sd.TW, sd.TH,
                             sd.ph, sd.pw, st));
  return LENSED_OK;
}

int lensed_loglike_model_batch(lensed_ctx* c, const lensed_system* systems, int n_systems, const lensed_model* model,
                               const float* theta, const int32_t* system_of_point, int n_points, double* logl,
                               void* stream) {
  if (!c) return LENSED_INVALID_ARGUMENT;
  ModelSpec spec;
  int rc = model_spec(c, model, spec);
  if (rc) return rc;
  if (n_points < 0) return set_err(c, LENSED_INVALID_ARGUMENT, "n_points must be >= 0");
  if (n_points == 0) return LENSED_OK;
  if (!systems || n_systems <= 0) return set_err(c, LENSED_INVALID_ARGUMENT, "at least one system is required");
  if (!theta || !logl || !system_of_point)
    return set_err(c, LENSED_INVALID_ARGUMENT, "theta, system_of_point and logl are required");
  for (int s = 0; s < n_systems; ++s)
    if ((rc = validate_system(c, &systems[s], true, s))) return rc;
  for (int p = 0; p < n_points; ++p)
    if (system_of_point[p] < 0 || system_of_point[p] >= n_systems)
      return set_err(c, LENSED_INVALID_ARGUMENT, "system_of_point[" + std::to_string(p) + "] out of range");
  LENSED_HIP(c, hipSetDevice(c->device));
  return run_batch(c, systems, n_systems, theta, system_of_point, n_points, logl, stream, 1, nullptr, 1, &spec,
                   spec_params(spec));
}

int lensed_loglike_multiband(lensed_ctx* c, const lensed_system* systems, int n_systems, const float* theta,
                             int n_bands, const int32_t* band_system, int n_components, const float* sky,
                             int n_models, double* logl, void* stream) {
  if (!c) return LENSED_INVALID_ARGUMENT;
  if (n_models < 0) return set_err(c, LENSED_INVALID_ARGUMENT, "n_models must be >= 0");
  if (n_bands < 1) return set_err(c, LENSED_INVALID_ARGUMENT, "n_bands must be >= 1");
  if (n_components < 1) return set_err(c, LENSED_INVALID_ARGUMENT, "n_components must be >= 1");
  if (n_models == 0) return LENSED_OK;
  if ((int64_t)n_models * n_bands * n_components > INT32_MAX / NPAR)
    return set_err(c, LENSED_INVALID_ARGUMENT, "n_models x n_bands x n_components too large");
  if (!systems || n_systems <= 0) return set_err(c, LENSED_INVALID_ARGUMENT, "at least one system is required");
  if (!theta || !logl || !band_system)
    return set_err(c, LENSED_INVALID_ARGUMENT, "theta, band_system and logl are required");
  for (int s = 0; s < n_systems; ++s) {
    const int rc = validate_system(c, &systems[s], true, s);
    if (rc) return rc;
  }
  for (int b = 0; b < n_bands; ++b)
    if (band_system[b] < 0 || band_system[b] >= n_systems)
      return set_err(c, LENSED_INVALID_ARGUMENT, "band_system[" + std::to_string(b) + "] out of range");
  LENSED_HIP(c, hipSetDevice(c->device));
  const int n_points = n_models * n_bands * n_components;
  c->composite_map.resize(n_points);
  for (int p = 0; p < n_points; ++p) c->composite_map[p] = band_system[(p / n_components) % n_bands];
  return run_batch(c, systems, n_systems, theta, c->composite_map.data(), n_points, logl, stream, n_components, sky,
                   n_bands);
}

int lensed_batch_schedule(lensed_ctx* c, int* out) {
  if (!c) return LENSED_INVALID_ARGUMENT;
  if (!out) return set_err(c, LENSED_INVALID_ARGUMENT, "out is NULL");
  for (int k = 0; k < 3; ++k) out[k] = c->schedule[k];
  return LENSED_OK;
}

int lensed_batch_render_block(lensed_ctx* c, int* out) {
  if (!c) return LENSED_INVALID_ARGUMENT;
  if (!out) return set_err(c, LENSED_INVALID_ARGUMENT, "out is NULL");
  out[0] = c->schedule[3];
  return LENSED_OK;
}

int lensed_batch_rendered(lensed_ctx* c, int64_t* out) {
  if (!c) return LENSED_INVALID_ARGUMENT;
  if (!out) return set_err(c, LENSED_INVALID_ARGUMENT, "out is NULL");
  out[0] = c->rendered[0];
  out[1] = c->rendered[1];
  return LENSED_OK;
}

int lensed_set_profiling(lensed_ctx* c, int enable) {
  if (!c) return LENSED_INVALID_ARGUMENT;
  c->profiling = enable != 0;
  return LENSED_OK;
}

int lensed_stage_times(lensed_ctx* c, double* ms, int n, int* calls) {
  if (!c || !ms || n < LENSED_NSTAGES) return set_err(c, LENSED_INVALID_ARGUMENT, "ms needs LENSED_NSTAGES slots");
  LENSED_HIP(c, hipSetDevice(c->device));
  for (auto& ev : c->pending) {
    LENSED_HIP(c, hipEventSynchronize(ev.back()));
    for (int k = 0; k < LENSED_NSTAGES; ++k) {
      float t = 0.0f;
      LENSED_HIP(c, hipEventElapsedTime(&t, ev[k], ev[k + 1]));
      c->stage_ms[k] += t;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    c->stage_calls += 1;
  }
  c->pending.clear();
  for (int k = 0; k < LENSED_NSTAGES; ++k) ms[k] = c->stage_ms[k];
  if (calls) *calls = c->stage_calls;
  for (int k = 0; k < LENSED_NSTAGES; ++k) c->stage_ms[k] = 0.0;
  c->stage_calls = 0;
  return LENSED_OK;
}

}  // extern "C"

// The gradient plans of one system (17-parameter model, or a general model).
static int run_grad(lensed_ctx* c, const lensed_system* sys, const float* theta, int n_points, double* logl,
                    float* grad, void* stream, const ModelSpec* spec, int params_per_point, int K = 1,
                    const float* sky = nullptr, float* grad_sky = nullptr) {
  LENSED_HIP(c, hipSetDevice(c->device));
  std::vector<int32_t> map(n_points, 0);
  BatchPlan* plan = nullptr;
  for (size_t i = 0; i < c->plans.size(); ++i) {
    if (c->plans[i]->matches(sys, 1, theta, map.data(), n_points, logl, grad, K, sky, 1, spec, false, grad_sky)) {
      std::unique_ptr<BatchPlan> keep = std::move(c->plans[i]);
      c->plans.erase(c->plans.begin() + i);
      c->plans.push_back(std::move(keep));
      plan = c->plans.back().get();
      break;
    }
  }
  if (!plan) {
    if (c->plans.size() >= 8) {
      LENSED_HIP(c, hipDeviceSynchronize());
      c->plans.erase(c->plans.begin());
    }
    // the render schedule: as fixed by LENSED_RENDER_PPT, else as measured for
    // these shapes by a batched call (one pixel per thread when none was)
    if (c->force_ppt || c->force_block)
      c->tiles.set_render_measured(sys, 1, RenderSchedule{c->force_ppt ? c->force_ppt : 1,
                                                         c->force_block ? c->force_block : RENDER_BLOCK});
    std::unique_ptr<BatchPlan> np(new BatchPlan());
    std::string msg;
    hipError_t e = np->build(sys, 1, theta, map.data(), n_points, logl, c->tiles, msg, grad, nullptr, K, sky, 1,
                             spec, params_per_point, nullptr, false, grad_sky);
    if (e != hipSuccess) return hip_fail(c, e, ("gradient plan: " + msg).c_str());
    if (c->use_graphs) {
      e = np->capture(c->cap);
      if (e != hipSuccess) return hip_fail(c, e, "gradient plan graph capture");
    }
    c->plans.push_back(std::move(np));
    plan = c->plans.back().get();
  }
  if (c->profiling) {
    std::vector<hipEvent_t> ev(LENSED_NSTAGES + 1);
    for (auto& e : ev) LENSED_HIP(c, hipEventCreate(&e));
    LENSED_HIP(c, plan->enqueue((hipStream_t)stream, ev.data()));
    c->pending.push_back(std::move(ev));
    return LENSED_OK;
  }
  LENSED_HIP(c, plan->run((hipStream_t)stream));
  return LENSED_OK;
}

extern "C" int lensed_loglike_grad(lensed_ctx* c, const lensed_system* sys, const float* theta, int n_points,
                                   double* logl, float* grad, void* stream) {
  if (!c) return LENSED_INVALID_ARGUMENT;
  if (n_points < 0) return set_err(c, LENSED_INVALID_ARGUMENT, "n_points must be >= 0");
  if (n_points == 0) return LENSED_OK;
  int rc = validate_system(c, sys, true, -1);
  if (rc) return rc;
  if (!theta || !logl || !grad) return set_err(c, LENSED_INVALID_ARGUMENT, "theta, logl and grad are required");
  return run_grad(c, sys, theta, n_points, logl, grad, stream, nullptr, NPAR);
}

extern "C" int lensed_loglike_composite_grad(lensed_ctx* c, const lensed_system* sys, const float* theta,
                                             int n_components, const float* sky, int n_models, double* logl,
                                             float* grad, float* grad_sky, void* stream) {
  if (!c) return LENSED_INVALID_ARGUMENT;
  if (n_models < 0) return set_err(c, LENSED_INVALID_ARGUMENT, "n_models must be >= 0");
  if (n_components < 1) return set_err(c, LENSED_INVALID_ARGUMENT, "n_components must be >= 1");
  if (n_models == 0) return LENSED_OK;
  if ((int64_t)n_models * n_components > INT32_MAX / NPAR)
    return set_err(c, LENSED_INVALID_ARGUMENT, "n_models x n_components too large");
  int rc = validate_system(c, sys, true, -1);
  if (rc) return rc;
  if (!theta || !logl || !grad) return set_err(c, LENSED_INVALID_ARGUMENT, "theta, logl and grad are required");
  if ((sky == nullptr) != (grad_sky == nullptr))
    return set_err(c, LENSED_INVALID_ARGUMENT, "sky and grad_sky are given together or not at all");
  return run_grad(c, sys, theta, n_models * n_components, logl, grad, stream, nullptr, NPAR, n_components, sky,
                  grad_sky);
}

extern "C" int lensed_loglike_model_grad(lensed_ctx* c, const lensed_system* sys, const lensed_model* model,
                                         const float* theta, int n_points, double* logl, float* grad, void* stream) {
  if (!c) return LENSED_INVALID_ARGUMENT;
  ModelSpec spec;
  int rc = model_spec(c, model, spec);
  if (rc) return rc;
  if (n_points < 0) return set_err(c, LENSED_INVALID_ARGUMENT, "n_points must be >= 0");
  if (n_points == 0) return LENSED_OK;
  if ((int64_t)n_points * spec_params(spec) > INT32_MAX)
    return set_err(c, LENSED_INVALID_ARGUMENT, "n_points x parameters too large");
  if ((rc = validate_system(c, sys, true, -1))) return rc;
  if (!theta || !logl || !grad) return set_err(c, LENSED_INVALID_ARGUMENT, "theta, logl and grad are required");
  return run_grad(c, sys, theta, n_points, logl, grad, stream, &spec, spec_params(spec));
}

extern "C" {

int lensed_mlp_param_count(void) { return MLP_NPARAM; }

int lensed_mlp_forward(lensed_ctx* c, const float* params, const float* norm, const float* x, float* y, int batch,
                       void* stream) {
  if (!c) return LENSED_INVALID_ARGUMENT;
  int rc = check_mlp_batch(c, batch);
  if (rc) return rc;
  if (batch == 0) return LENSED_OK;
  if (!params || !norm || !x || !y) return set_err(c, LENSED_INVALID_ARGUMENT, "params, norm, x and y are required");
  LENSED_HIP(c, hipSetDevice(c->device));
  if ((rc = ensure_mlp(c, batch))) return rc;
  LENSED_HIP(c, mlp_forward(params, norm, x, y, batch, c->mlp, (hipStream_t)stream));
  return LENSED_OK;
}

int lensed_mlp_grad(lensed_ctx* c, const float* params, const float* norm, const float* x, const float* y, int batch,
                    float* grad, float* loss, void* stream) {
  if (!c) return LENSED_INVALID_ARGUMENT;
  int rc = check_mlp_batch(c, batch);
  if (rc) return rc;
  if (batch == 0) return set_err(c, LENSED_INVALID_ARGUMENT, "the loss needs at least one row");
  if (!params || !norm || !x || !y || !grad || !loss)
    return set_err(c, LENSED_INVALID_ARGUMENT, "params, norm, x, y, grad and loss are required");
  LENSED_HIP(c, hipSetDevice(c->device));
  if ((rc = ensure_mlp(c, batch))) return rc;
  LENSED_HIP(c, mlp_grad(params, norm, x, y, batch, grad, loss, c->mlp, (hipStream_t)stream));
  return LENSED_OK;
}

int lensed_mlp_adam(lensed_ctx* c, float* params, const float* grad, float* m, float* v, int step, double lr,
                    double beta1, double beta2, double eps, void* stream) {
  if (!c) return LENSED_INVALID_ARGUMENT;
  if (!params || !grad || !m || !v) return set_err(c, LENSED_INVALID_ARGUMENT, "params, grad, m and v are required");
  if (step < 1 || !std::isfinite(lr) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) ||
      !(eps > 0.0))
    return set_err(c, LENSED_INVALID_ARGUMENT, "step >= 1, finite lr, betas in [0,1) and eps > 0 are required");
  LENSED_HIP(c, hipSetDevice(c->device));
  LENSED_HIP(c, mlp_adam(params, grad, m, v, MLP_NPARAM, step, lr, beta1, beta2, eps, (hipStream_t)stream));
  return LENSED_OK;
}

int lensed_mlp_train_step(lensed_ctx* c, float* params, float* m, float* v, int step, const float* norm,
                          const float* x, const float* y, int batch, double lr, float* loss, void* stream) {
  if (!c) return LENSED_INVALID_ARGUMENT;
  int rc = check_mlp_batch(c, batch);
  if (rc) return rc;
  if (batch == 0) return set_err(c, LENSED_INVALID_ARGUMENT, "the loss needs at least one row");
  if (!params || !m || !v || !norm || !x || !y || !loss)
    return set_err(c, LENSED_INVALID_ARGUMENT, "params, m, v, norm, x, y and loss are required");
  if (step < 1 || !std::isfinite(lr)) return set_err(c, LENSED_INVALID_ARGUMENT, "step >= 1 and finite lr required");
  LENSED_HIP(c, hipSetDevice(c->device));
  if ((rc = ensure_mlp(c, batch))) return rc;
  hipStream_t st = (hipStream_t)stream;
  LENSED_HIP(c, mlp_grad(params, norm, x, y, batch, c->mlp.grad, loss, c->mlp, st));
  LENSED_HIP(c, mlp_adam(params, c->mlp.grad, m, v, MLP_NPARAM, step, lr, 0.9, 0.999, 1e-8, st));
  return LENSED_OK;
}

}  // extern "C"
