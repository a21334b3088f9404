// kernels.h -- host-side launch wrappers of the liblensed_hip kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"
#include "model.h"

namespace lensed {

constexpr int MAX_PSF = 63;   // largest PSF side accepted (LDS staging bound)

// Work description shared by the render, PSF/chi^2 and adjoint kernels.
// Plain calls use `single` and `point0` with implicit item = (point0, blockIdx.x);
// batched calls pass device tables and an explicit (point, tile) item list.
struct WorkArgs {
  SysDesc single;               // used when sys_table == nullptr
  const SysDesc* sys_table;     // [n_systems] or nullptr
  const int* point_sys;         // [n_points] system of each point, or nullptr (system 0)
  const int64_t* point_loff;    // [n_points] offset of the point's image in the scratch, or nullptr (0)
  const int64_t* point_goff;    // [n_points] offset of the image whose g = A^T rho the point's gradient
                                // reads (the first image of its composite model), or nullptr (point_loff)
  const int* point_pbase;       // [n_points] first partial-sum slot of the point, or nullptr (0)
  const int2* items;            // [n_items] (point, tile), or nullptr
  int n_items;                  // grid size when items is given
  int point0;                   // point of a plain call
};

// Item lists longer than this are launched in several parts: every grid
// dimension must stay below 2^32 work-items (2^22 blocks of at most 512).
constexpr int MAX_ITEM_BLOCKS = 1 << 22;

// Calls launch(part, n) for consecutive parts of w's item list (w.items advanced,
// n <= MAX_ITEM_BLOCKS blocks each); a plain call (no item list) goes out whole.
template <class F>
hipError_t for_item_parts(const WorkArgs& w, int n_blocks, F launch) {
  if (!w.items) return launch(w, n_blocks);
  for (int off = 0; off < n_blocks; off += MAX_ITEM_BLOCKS) {
    WorkArgs part = w;
    part.items = w.items + off;
    part.n_items = n_blocks - off < MAX_ITEM_BLOCKS ? n_blocks - off : MAX_ITEM_BLOCKS;
    const hipError_t e = launch(part, part.n_items);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Also clears *cusp_count (may be nullptr) and, when gcs is given, the 17
// cusp-correction accumulators of every point in grad_corr. The system of
// point p is table[point_sys[p]] (table[0] without point_sys; single without
// table); its amplitude mode decides whether theta[5] and theta[12] are I_e or
// total magnitudes. adjoint_tables: the systems' adjk tables (set in their
// descriptors) are filled too, as every gradient plan needs.
hipError_t launch_prologue(const float* theta, int n_points, PointConst* pcs, PointConst64* p64s, GradConst* gcs,
                           const SysDesc& single, SysDesc* table, int n_sys, int* cusp_count, hipStream_t stream,
                           double* grad_corr = nullptr, const int* point_sys = nullptr, bool adjoint_tables = false);

// Unconvolved pixel luminosities into L (scratch or the caller's image): the
// float32 render kernel, then the float64 cusp corrections of the pixels it
// flagged. cl.entries needs one slot per render wave (n_blocks * 4); cl.count
// must be zero when the render kernel starts (the prologue clears it). A
// non-null `between` is recorded on the stream after the render kernel.
hipError_t launch_render(const WorkArgs& w, const PointConst* pcs, const PointConst64* p64s, float* L, int n_blocks,
                         const CuspList& cl, hipStream_t stream, hipEvent_t between = nullptr);

// Schedule class of a system's render: N (1..RENDER_MAX_CLASS) for the N x N
// midpoint rule, each its own kernel with the rule unrolled; 0 for the
// Gauss-Kronrod rules and larger N.
constexpr int RENDER_MAX_CLASS = 8;
int render_class(const SysDesc& sd);

// A run of render items of one class: items [offset, offset + count) of w.items
// (or, for a plain call, blocks 0..count-1 of w.single), with ppt pixels per
// thread (2 only for classes 1..RENDER_MAX_CLASS and images of even width) and
// block threads per block (64 <= block <= RENDER_BLOCK_MAX, a multiple of 64):
// an item covers block render units of ppt pixels.
struct RenderSpan {
  int klass, ppt, offset, count, block;
};
constexpr int RENDER_BLOCK_MAX = 512;
// A render schedule: pixels per thread and threads per block.
struct RenderSchedule {
  int ppt, block;
};
// Batched form: one launch per span, then one cusp-correction pass over all of
// them. cl.entries needs one slot per render wave and pixel of a thread.
hipError_t launch_render(const WorkArgs& w, const PointConst* pcs, const PointConst64* p64s, float* L,
                         const RenderSpan* spans, int n_spans, const CuspList& cl, hipStream_t stream,
                         hipEvent_t between = nullptr);

// General models: per-point float64 constants from the parameters (n_params
// per point, the layout of lensed_model), and the float64 render into L.
// with_db: also db_n/dn of every Sersic (the adjoint needs it).
hipError_t launch_model_prologue(const float* theta, int n_points, int n_params, const ModelSpec& spec,
                                 ModelConst* out, hipStream_t stream, bool with_db = false);
hipError_t launch_model_render(const WorkArgs& w, const ModelSpec& spec, const ModelConst* mcs, float* L, int n_blocks,
                               hipStream_t stream);
// Adjoint of a general model with one lens plane: per (point, render tile) and
// model parameter, g d^2 w dI/dtheta summed over the tile's pixels and
// subsamples in float64 (gpart[(gpbase[point] + tile) P + k], P parameters per
// point; g = A^T rho in G), then their sums over the tiles into grad (float32,
// [n_points][P]).
hipError_t launch_model_grad(const WorkArgs& w, const ModelSpec& spec, const ModelConst* mcs, const float* G,
                             const int* gpbase, double* gpart, int P, int n_blocks, hipStream_t stream);
hipError_t launch_model_finalize_grad(const double* gpart, const int* gpbase, int ntiles, int P, int n_points,
                                      float* grad, hipStream_t stream);

// Composite models (K consecutive points each): L[first image of model m] =
// sum of its K unconvolved images + sky[m] pixscale^2 (sky may be nullptr), in
// float64 per pixel, before the PSF stage. tiles_per_model: RENDER_BLOCK-pixel
// tiles of the largest image.
hipError_t launch_compose(float* L, const int64_t* loff, const int* point_sys, const SysDesc* sys, int K, int n_models,
                          const float* sky, int tiles_per_model, hipStream_t stream);

// One composite model of a plain call: out = sum of the K consecutive images of
// npix pixels in L + sky_px, in float64 (out may be L).
hipError_t launch_sum_images(const float* L, int64_t npix, int K, double sky_px, float* out, hipStream_t stream);
// *count = 0 by a kernel (capturable, unlike a memset node).
hipError_t launch_zero_count(int* count, hipStream_t stream);

// Weights from the data (Sec. 3.3): w = extra * g / (d + b) where g (d + b) > 0, else 0.
// gain_map / offset_map / extra may be nullptr (scalar gain, scalar offset, 1).
hipError_t launch_weights_from_data(const float* data, int64_t n, double gain, const float* gain_map, double offset,
                                    const float* offset_map, const float* extra, float* weight, hipStream_t stream);

// Per-pixel integration error estimate of a Gauss-Kronrod rule for the single
// point w.point0 of w.single (rule > 0): |Kronrod - embedded Gauss| x pixel weight.
hipError_t launch_rule_error(const WorkArgs& w, const PointConst* pcs, float* E, int n_blocks, hipStream_t stream);

// mode 0: PSF convolution of L into out (L* images, same offsets as L).
// mode 1: PSF convolution fused with the weighted chi^2; one compensated
//         (hi, lo) float pair per tile is written to partials.
// mode 2: as mode 1, and the weighted residual w (d - L*) is written to out.
// Every system of one launch uses the same TW x TH output tile (the block is
// TW x TH/R threads, R = psf_rows()). square_psf = 21, 7 or 1 with TW = 32 or 64
// selects a specialised stencil when every PSF of the launch has that square
// size; anything else runs the generic one.
hipError_t launch_psf(const WorkArgs& w, const float* L, float* out, float2* partials, int mode, int n_blocks,
                      int square_psf, int TW, int TH, int max_ph, int max_pw, hipStream_t stream);


// log L = -1/2 * sum over the point's tiles of (hi + lo), in float64.
hipError_t launch_finalize(const float2* partials, const int* point_pbase, const int* point_ntiles, int n_points,
                           int single_ntiles, double* logl, hipStream_t stream);

// g = A^T rho for every point of a single-system launch (same tiles as the PSF
// kernel, border pixels by the folded tables); R and G use the image offsets.
hipError_t launch_adjoint_psf(const WorkArgs& w, const float* R, float* G, int n_blocks, int square_psf, int TW,
                              int TH, int ph, int pw, int n_points, int H, int W, hipStream_t st);

// d log L / d sky of every composite model m (its points m K .. m K + K - 1,
// its rho in R at the offset of its first image): the sky adds sky d^2 to
// every pixel of L, the PSF keeps a constant image constant, so the
// derivative is d^2 times the sum of rho over the image. One block per model.
hipError_t launch_grad_sky(const float* R, const int64_t* loff, const int* point_sys, const SysDesc* sys, int K,
                           int n_models, float* grad_sky, hipStream_t st);

// Rebuilds the adjoint's support (SysDesc::gsup) of every system in the device
// table sys[0 .. n_sys) whose gsup is set, from its weights: a row pass and a
// column pass of the PSF-box dilation of w > 0 into gflags, then one block per
// system compacts the flags into the pixel list and, where uact is set, into
// the render units (writing n_active of the table entry). max_pixels bounds H W.
hipError_t launch_grad_support(SysDesc* sys, int n_sys, int max_pixels, hipStream_t st);

// Zeroes each point's unconvolved image L outside its system's support, for the
// systems whose render units are rebuilt with it (uact set); w carries the
// device system table, the point-to-system map and the image offsets.
hipError_t launch_grad_clear(const WorkArgs& w, float* L, int n_points, hipStream_t st);

// Per-(point, render tile) sums of g d^2/N^2 times the 17 gradient moments of
// the subsamples (each partial dI/dtheta is a fixed per-point combination of
// them): gpart[(gpbase[p] + tile) * 17 + k], tile t covering pixels
// 256 t .. 256 t + 255 of the support (zero past its end),
// then the float64 cusp corrections of the waves in cl (the list the forward
// render filled) added to corr[p * 17 + k], which must start at zero.
hipError_t launch_grad(const WorkArgs& w, const PointConst* pcs, const PointConst64* p64s, const GradConst* gcs,
                       const float* G, const int* gpbase, float2* gpart, int n_blocks, const CuspList& cl,
                       double* corr, hipStream_t st, hipEvent_t between = nullptr);

// Sums the gradient moments of every point (tiles and cusp corrections), maps
// them to the 17 partials, and for points of a system with magnitudes carries
// d log L / d I_e over to d/dm, d/dR_e and d/dn, with an image-plane source
// position d/dbeta over to the image-plane point and the lens (gcs).
hipError_t launch_finalize_grad(const float2* gpart, const int* gpbase, int ntiles, int n_points, const double* corr,
                                const PointConst* pcs, const GradConst* gcs, float* grad, hipStream_t st);

}  // namespace lensed
