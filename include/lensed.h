/* lensed.h -- C ABI of the MI355X forward strong-lensing likelihood library.
 *
 * Implements the forward model and likelihood of Tessore, Bellagamba & Metcalf,
 * "LENSED: a code for the forward reconstruction of lenses and sources from
 * strong lensing observations" (MNRAS 2016) as hand-written HIP kernels for
 * gfx950 (liblensed_hip.so).
 *
 * Model (17 float32 parameters per point, lens centred on the coordinate origin):
 *   index  0 theta_E    SIE equivalent-circular Einstein radius (arcsec), >= 0
 *          1 q_L        SIE axis ratio, (0, 1]
 *          2 phi_L      SIE position angle (rad, counter-clockwise from +x to the major axis)
 *          3 gamma      external shear magnitude
 *          4 phi_gamma  external shear angle (rad): gamma_1 = gamma cos 2phi, gamma_2 = gamma sin 2phi
 *          5 I_H        lens-light Sersic surface brightness at R_H (or its total
 *                       magnitude, when the system's amplitude is LENSED_AMP_MAGNITUDE)
 *          6 R_H        lens-light half-light radius (geometric mean of the semi-axes), > 0
 *          7 n_H        lens-light Sersic index, [0.2, 10]
 *          8 q_H        lens-light axis ratio, (0, 1]
 *          9 phi_H      lens-light position angle
 *         10 x_S, 11 y_S  source centre (arcsec)
 *         12 I_S, 13 R_S, 14 n_S, 15 q_S, 16 phi_S   source Sersic, as for the lens light
 *                       (I_S likewise a total magnitude in magnitude mode)
 *   Lens equation beta = x - alpha_SIE(x) - alpha_shear(x)        (Sec. 2.1, Eq. 1)
 *   I(x) = I_lens(x) + I_source(beta)                             (Sec. 2.1, Eq. 2)
 *   Sersic I = I_e exp(-b_n [(R/R_e)^{1/n} - 1]), R = sqrt(q x'^2 + y'^2/q)
 *   with b_n the exact root of P(2n, b_n) = 1/2                   (Sec. 4.1, Eqs. 22-23)
 *   SIE: kappa = theta_E / (2 sqrt(q x'^2 + y'^2/q))              (Sec. 4, Kormann et al. 1994)
 *
 * Conventions shared by every call
 *   - Images are row-major float32 [height][width]; row 0 is the smallest y.
 *     Pixel (r, c) is centred on x = center_x + (c - (W-1)/2) pixscale,
 *     y = center_y + (r - (H-1)/2) pixscale.
 *   - Pixel luminosity (Sec. 2.1 Eq. 3) uses the N x N midpoint rule
 *     (Sec. 3.1 Eq. 14, the "subN" rules of Sec. 4.5): abscissae at
 *     ((k + 1/2)/N - 1/2) pixscale from the pixel centre, weights pixscale^2/N^2.
 *   - The PSF is an odd (2p+1) x (2q+1) float32 array centred on its middle
 *     element; the library normalises a private copy to unit sum and convolves
 *     with replicate padding (Sec. 3.1, Eq. 15).
 *   - Every data pointer (images, weights, PSF, theta, outputs) is a DEVICE
 *     pointer owned by the caller, except where a comment says HOST. The caller
 *     keeps buffers alive until the stream has completed the call.
 *   - All calls are asynchronous on `stream` (a hipStream_t; NULL = null stream)
 *     and return once the work is enqueued.
 *   - Parameter values live on the device, so they are not validated on the
 *     host: a point with q outside (0,1], R_e <= 0, n outside [0.2, 10] or a
 *     non-finite value yields NaN for that point only.
 *   - One context per host thread; calls on one context must not overlap.
 *
 * Return codes: LENSED_OK, or one of the errors below; nothing is enqueued when
 * an error is returned for invalid arguments.
 */
#ifndef LENSED_H
#define LENSED_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LENSED_NPARAM 17

enum {
  LENSED_OK = 0,
  LENSED_INVALID_ARGUMENT = 1, /* null pointer, non-positive size, even PSF side,
                                  nsub outside 1..16, bad system index, ...     */
  LENSED_HIP_ERROR = 2,        /* a HIP runtime call failed; see lensed_last_error */
  LENSED_OUT_OF_MEMORY = 3,    /* workspace allocation failed                   */
  LENSED_NOT_SUPPORTED = 4,    /* no usable gfx950 device                       */
  LENSED_TOO_LARGE = 5         /* input exceeds the static workspace of lensed_loglike_noalloc */
};

/* Bytes of the static device workspace of lensed_loglike_noalloc (per device). */
#define LENSED_NOALLOC_SCRATCH_BYTES (6u << 20)

typedef struct lensed_ctx lensed_ctx;

/* One observation (Sec. 3, step i): data d_i, weights w_i = 1/s_i^2 (0 = masked,
 * Sec. 3.2), PSF array, grid geometry, integration rule and the meaning of the
 * two Sersic amplitude parameters and of the source position. */
typedef struct {
  int32_t height, width;      /* pixels, > 0                                    */
  float pixscale;             /* arcsec per pixel, > 0                          */
  float center_x, center_y;   /* image-plane coordinates of the grid centre     */
  int32_t nsub;               /* N of the N x N midpoint rule, 1..16            */
  int32_t psf_h, psf_w;       /* odd, >= 1 (1 x 1 = no blurring)                */
  const float* psf;           /* device [psf_h * psf_w], any positive scale     */
  const float* data;          /* device [height * width]; may be NULL for render */
  const float* weight;        /* device [height * width]; may be NULL for render */
  int32_t rule;               /* pixel integration rule (Eq. 14, Sec. 4.5):
                                 LENSED_RULE_MIDPOINT (nsub x nsub "subN"), or the
                                 Cartesian square of a Gauss-Kronrod rule
                                 LENSED_RULE_G3K7 / _G5K11 / _G7K15 (nsub ignored) */
  int32_t amplitude;          /* theta[5] and theta[12] (Sec. 4.1):
                                 LENSED_AMP_INTENSITY: I_e, the surface brightness
                                 at R_e; LENSED_AMP_MAGNITUDE: the component's total
                                 magnitude m, with I_e set so that its total flux is
                                 10^(-0.4 (m - zero_point)) in data units x arcsec^2 */
  float zero_point;           /* magnitude of unit total flux (finite)          */
  int32_t source_position;    /* theta[10], theta[11] (Sec. 5):
                                 LENSED_SOURCE_PLANE: the source centre;
                                 LENSED_IMAGE_PLANE: a point x_I of the image plane,
                                 the source centre being its image under the lens
                                 equation, beta = x_I - alpha(x_I) (Eq. 1, float64);
                                 the gradient is then with respect to x_I        */
} lensed_system;

#define LENSED_RULE_MIDPOINT 0
#define LENSED_RULE_G3K7 1
#define LENSED_RULE_G5K11 2
#define LENSED_RULE_G7K15 3

#define LENSED_AMP_INTENSITY 0
#define LENSED_AMP_MAGNITUDE 1

#define LENSED_SOURCE_PLANE 0
#define LENSED_IMAGE_PLANE 1

/* Creates a context bound to HIP device `device` (its workspace arena, cached
 * batch plans and graphs). Returns LENSED_NOT_SUPPORTED if the device is not
 * gfx950. The context owns only its own allocations; lensed_destroy frees them. */
int lensed_create(lensed_ctx** out, int device);
void lensed_destroy(lensed_ctx* ctx);

/* Number of model parameters per point (17). */
int lensed_param_count(void);

/* Static description of a status code. */
const char* lensed_status_string(int status);

/* Text of the last HIP or validation error recorded on the context. */
const char* lensed_last_error(const lensed_ctx* ctx);

/* Model image of one parameter point (Sec. 3, step iv): the pixel luminosities
 * of Eq. 3 by the N x N midpoint rule, then, if apply_psf != 0, the PSF
 * convolution of Eq. 15.
 *   theta  device float32 [17]
 *   image  device float32 [height * width], written
 * data and weight of the system are not read. */
int lensed_render(lensed_ctx* ctx, const lensed_system* sys, const float* theta,
                  float* image, int apply_psf, void* stream);

/* Log-likelihood of one point (Sec. 3.2, Eq. 17): log L = -chi^2/2 with
 * chi^2 = sum_i w_i (d_i - L*_i)^2, the constant term dropped.
 * chi^2 is accumulated in float32 with compensated summation and the final sum
 * over tiles is taken in float64.
 *   theta  device float32 [17]
 *   logl   device float64 [1], written
 * This is the plain form: one launch sequence per call. */
int lensed_loglike(lensed_ctx* ctx, const lensed_system* sys, const float* theta,
                   double* logl, void* stream);

/* lensed_loglike without a context and without any allocation, for callers
 * that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc. Every intermediate (per-point
 * constants, normalised PSF copies, the unconvolved image, cusp work list,
 * per-tile chi^2 sums) lives in one static device array of
 * LENSED_NOALLOC_SCRATCH_BYTES per device, which the library holds until the
 * process ends; its device address is looked up once per device. The call
 * runs on the calling thread's current HIP device, asynchronously on `stream`
 * (a stream of that device), and gives the same log L as lensed_loglike, bit
 * for bit.
 *   sys    as for lensed_loglike (data and weight required)
 *   theta  device float32 [17]
 *   logl   device float64 [1], written
 * Returns LENSED_TOO_LARGE, before any launch, when the image and PSF need
 * more than the workspace (about 4.4 bytes per pixel plus 52 KB: images up to
 * about 1.4 million pixels, 1180 x 1180), INVALID_ARGUMENT as lensed_loglike,
 * HIP_ERROR if a launch fails. Every call on a device shares its workspace, and
 * each call leaves its contents behind: calls that may overlap on one device
 * (on different streams, or from several threads) race and must be ordered by
 * the caller. Nothing here needs zeroed memory: the prologue kernel clears the
 * one counter it uses. */
int lensed_loglike_noalloc(const lensed_system* sys, const float* theta, double* logl, void* stream);

/* Log-likelihoods of many points over many systems in one graph launch
 * (Eq. 17 for every point). Work is split into (point, tile) items, ordered
 * longest first, and the schedule is chosen per system shape by the autotuner.
 *   systems          HOST array [n_systems] (their data pointers are device pointers)
 *   theta            device float32 [n_points * 17], point-major
 *   system_of_point  HOST int32 [n_points], values in [0, n_systems)
 *   logl             device float64 [n_points], written
 * The plan (work lists, scratch layout, captured graph) is cached on the context
 * keyed by the systems, the mapping and the theta/logl pointers. The first call
 * for a new set of system shapes also autotunes the schedule: it times the PSF +
 * chi^2 stage of the cost model's six best-ranked tile shapes, then the render
 * kernels with one and with two pixels per thread in blocks of 128, 256 and
 * 512 threads, on this launch (synchronising `stream`), and keeps the fastest
 * for every later plan over the same shapes; LENSED_NO_AUTOTUNE=1 in the
 * environment keeps the model's tile and one pixel per thread in 256-thread
 * blocks, LENSED_RENDER_PPT=1 or 2 and LENSED_RENDER_BLOCK=128, 256 or 512
 * (read by lensed_create) fix the render schedule. Every schedule gives the
 * same results bit for bit. */
int lensed_loglike_batch(lensed_ctx* ctx, const lensed_system* systems, int n_systems,
                         const float* theta, const int32_t* system_of_point, int n_points,
                         double* logl, void* stream);

/* lensed_loglike_batch restricted to the pixels that Eq. 17 can see. A pixel
 * with w = 0 is masked (Sec. 3.2), so log L needs L* only where w > 0, and by
 * Eq. 15 (replicate padding) L* there reads L only within the PSF's
 * (2p+1) x (2q+1) box around it, clamped to the image. The plan renders only
 * the pixels of that dilated support and convolves only the PSF output tiles
 * that hold a pixel with w > 0; everything else stays zero. The result equals
 * lensed_loglike_batch bit for bit whenever the data are finite where w = 0
 * (a non-finite datum at a masked pixel makes the unmasked sum NaN, 0 x inf).
 * Arguments, ownership and errors as lensed_loglike_batch; the plan reads the
 * weights back to the host once when it is built, so the weights must not
 * change between calls that reuse the plan (same pointers: same plan). */
int lensed_loglike_batch_masked(lensed_ctx* ctx, const lensed_system* systems, int n_systems,
                                const float* theta, const int32_t* system_of_point, int n_points,
                                double* logl, void* stream);

/* Per-pixel integration error estimate of a Gauss-Kronrod rule (Sec. 3.1: the
 * embedded Gauss rule estimates the error of each pixel and is saved with the
 * output): error[i] = |L_i(Kronrod) - L_i(embedded Gauss)| before the PSF, for
 * one parameter point.
 *   sys     its rule must be a LENSED_RULE_G*K* value (INVALID_ARGUMENT otherwise);
 *           data and weight are not used
 *   theta   device float32 [17]
 *   error   device float32 [height * width], written
 * The subsample values are the float32 render's, without the float64 re-tracing
 * near a cuspy source centre that lensed_render applies. */
int lensed_render_error(lensed_ctx* ctx, const lensed_system* sys, const float* theta, float* error, void* stream);

/* ---- General models -------------------------------------------------------
 * The paper's fits of real lenses (Sec. 5) use several lenses (two SIEs for a
 * lens with a companion), several Sersic components, a flat sky and, in its
 * tests, free centres. A general model lists them; its parameters per point,
 * in this order (float32):
 *   per SIE          x_c, y_c, theta_E, q, phi        deflection about (x_c, y_c)
 *   shear, if any    gamma, phi_gamma                 about the origin
 *   per Sersic       x, y, I_e, R_e, n, q, phi        Eqs. 22-23 centred on (x, y)
 *   sky, if any      surface brightness
 * beta = x - sum_k alpha_SIE_k(x - c_k) - alpha_shear(x) (Eq. 1: the deflectors
 * of one lens plane add); a Sersic with plane LENSED_LIGHT_FOREGROUND is light
 * at x (unlensed: lens galaxies), LENSED_LIGHT_LENSED light at beta (sources).
 *
 * Several lens planes (the extension named in Sec. 6, in the standard form of
 * the multi-plane lens equation): n_planes = P lens planes, ordered by
 * distance, and the source plane P. The ray through the image-plane point x
 * sits at x_0 = x and x_j = x - sum_{i<j} beta_ij alpha_i(x_i) (j = 1..P), with
 * alpha_i the summed deflection of the SIEs of plane i (theta_E scaled to the
 * source plane, as for one plane) and beta_iP = 1; the shear belongs to plane 0.
 * A Sersic on plane j is evaluated at x_j. With P = 1 this is the one-plane
 * model above, and sie_plane and beta are not read.
 *
 * These models trace rays in float64 (the Sersic profiles take the fractional
 * parts of their powers of two in float32) and round once per pixel (the PSF
 * and chi^2 stages are the common ones); lensed_loglike_model_grad gives their
 * adjoint, with one or several lens planes. */
#define LENSED_LIGHT_FOREGROUND 0
#define LENSED_LIGHT_LENSED 1
typedef struct {
  int32_t n_sie;        /* 0..8 */
  int32_t shear;        /* 0 or 1 */
  int32_t n_sersic;     /* 1..8 */
  int32_t sky;          /* 0 or 1 */
  int32_t plane[8];     /* per Sersic: its plane, 0..n_planes (with one lens plane:
                           LENSED_LIGHT_FOREGROUND or LENSED_LIGHT_LENSED) */
  int32_t n_planes;     /* lens planes P, 1..8 (0 reads as 1) */
  int32_t sie_plane[8]; /* per SIE: its lens plane, 0..P-1 */
  int32_t reserved;     /* 0 */
  double beta[8][8];    /* beta[i][j], 0 <= i < j < P: distance ratio
                           D_ij D_s / (D_j D_is), in [0, 1]; other entries unused */
} lensed_model;

/* Parameters per point of a model (-1 for an invalid model). */
int lensed_model_nparams(const lensed_model* model);

/* Model image of one point of a general model.
 *   theta  device float32 [lensed_model_nparams(model)]
 *   image  device float32 [height * width], written
 * Out-of-domain parameters (q outside (0, 1], R_e <= 0, n outside [0.2, 10],
 * non-finite values) give a NaN image. */
int lensed_render_model(lensed_ctx* ctx, const lensed_system* sys, const lensed_model* model, const float* theta,
                        float* image, int apply_psf, void* stream);

/* log L (Eq. 17) of n_points points of a general model over several systems,
 * in one graph launch like lensed_loglike_batch.
 *   theta  device float32 [n_points * lensed_model_nparams(model)] */
int lensed_loglike_model_batch(lensed_ctx* ctx, const lensed_system* systems, int n_systems,
                               const lensed_model* model, const float* theta, const int32_t* system_of_point,
                               int n_points, double* logl, void* stream);

/* log L and its gradient with respect to every parameter of a general model
 * (the paper's real-lens models, Sec. 5: several SIEs with free centres, the
 * shear, several Sersic components, the sky; lenses on several planes, Sec. 6),
 * for n_points points of one system: the derivative of Eq. 17 through Eqs. 15,
 * 14, 2, 1 and 22, by the transposed PSF of lensed_loglike_grad and float64
 * partial derivatives per subsample (forward-mode dual numbers, one component
 * at a time; with several planes the duals follow the ray plane by plane).
 *   theta  device float32 [n_points * P], P = lensed_model_nparams(model)
 *   logl   device float64 [n_points], written
 *   grad   device float32 [n_points * P], written (d log L / d theta, in the
 *          parameter order of the model)
 * Like lensed_loglike_grad, each call renders and differentiates only the
 * pixels within the PSF box of a weighted pixel, from the weights as they are. */
int lensed_loglike_model_grad(lensed_ctx* ctx, const lensed_system* sys, const lensed_model* model,
                              const float* theta, int n_points, double* logl, float* grad, void* stream);

/* ---- Composite models ---------------------------------------------------
 * The paper's fits of real lenses (Sec. 5) add further Sersic components and a
 * flat sky to the base model. A composite model here is K parameter points
 * (each a full 17-parameter point: give the components the same lens
 * parameters to describe one lens with several light components) whose pixel
 * luminosities are summed, plus a flat sky of surface brightness `sky` (pixel
 * luminosity sky * pixscale^2); the PSF (Eq. 15) applies to the sum. */

/* Model image of one composite model.
 *   theta         device float32 [n_components * 17], component j at theta + 17 j
 *   n_components  1..64
 *   sky           flat sky surface brightness (finite)
 *   image         device float32 [height * width], written
 * Components are summed in float64 per pixel. */
int lensed_render_composite(lensed_ctx* ctx, const lensed_system* sys, const float* theta, int n_components,
                            float sky, float* image, int apply_psf, void* stream);

/* log L (Eq. 17) of n_models composite models of n_components points each, in
 * one graph launch like lensed_loglike_batch.
 *   theta            device float32 [n_models * n_components * 17]; model m is the
 *                    n_components consecutive points starting at point m * n_components
 *   sky              device float32 [n_models], or NULL for no sky
 *   system_of_model  HOST int32 [n_models], indices into systems
 *   logl             device float64 [n_models], written
 * n_components = 1 with sky = NULL is lensed_loglike_batch. Errors as there;
 * LENSED_INVALID_ARGUMENT for n_components < 1. */
int lensed_loglike_composite(lensed_ctx* ctx, const lensed_system* systems, int n_systems, const float* theta,
                             int n_components, const float* sky, const int32_t* system_of_model, int n_models,
                             double* logl, void* stream);

/* log L of composite models (as lensed_loglike_composite, one system) and its
 * gradient with respect to every component's 17 parameters and the sky: the
 * components share the model's residual, so component k's gradient is that of
 * Eq. 17 through Eqs. 15, 14, 2 and 1 with g = A^T rho of the model, and the
 * sky, which adds sky x pixscale^2 to every pixel, has d log L / d sky =
 * pixscale^2 x sum of rho (the PSF keeps a constant image constant).
 *   theta     device float32 [n_models * n_components * 17], as in
 *             lensed_loglike_composite
 *   sky       device float32 [n_models], or NULL for no sky
 *   logl      device float64 [n_models], written
 *   grad      device float32 [n_models * n_components * 17], written
 *   grad_sky  device float32 [n_models], written; NULL exactly when sky is NULL
 * n_components = 1 without a sky is lensed_loglike_grad. A multi-band fit
 * (lensed_loglike_multiband) sums the bands' log L, so its gradient is the
 * sum over its bands of this one, band by band. Errors as
 * lensed_loglike_composite; LENSED_INVALID_ARGUMENT when only one of sky and
 * grad_sky is given. */
int lensed_loglike_composite_grad(lensed_ctx* ctx, const lensed_system* sys, const float* theta, int n_components,
                                  const float* sky, int n_models, double* logl, float* grad, float* grad_sky,
                                  void* stream);

/* Simultaneous fits of several bands (Sec. 6 names the joint reconstruction of
 * multiple bands as an extension): the bands' noise is independent, so a
 * model's log L is the sum over its bands of Eq. 17, each band being its own
 * system (data, weights, PSF, grid) and its own composite image.
 *   theta        device float32 [n_models * n_bands * n_components * 17]; band b of
 *                model m is the n_components points from point (m n_bands + b) n_components
 *                (tie the geometry across bands by giving it the same values)
 *   band_system  HOST int32 [n_bands], the system of each band
 *   sky          device float32 [n_models * n_bands] (per model and band), or NULL
 *   logl         device float64 [n_models], written: sum over the bands
 * One graph launch, like lensed_loglike_batch. */
int lensed_loglike_multiband(lensed_ctx* ctx, const lensed_system* systems, int n_systems, const float* theta,
                             int n_bands, const int32_t* band_system, int n_components, const float* sky,
                             int n_models, double* logl, void* stream);

/* Weights of an observation that comes without a variance map (Sec. 3.3,
 * Eqs. 18-21). The photon counts k_i = g_i (d_i + b_i) (effective gain g_i =
 * electronic gain x exposure time; offset b_i = whatever was subtracted from
 * the data, e.g. the sky) are taken as Poisson, Var k_i = k_i, so the data
 * variance is s_i^2 = (d_i + b_i) / g_i and the weight is
 *   w_i = e_i / s_i^2 = e_i g_i / (d_i + b_i),
 * with e_i the optional multiplicative extra weight factor (e_i = 0 masks the
 * pixel). Pixels with k_i <= 0 get w_i = 0.
 *   data        device float32 [n]
 *   gain_map    device float32 [n], or NULL: `gain` for every pixel (finite, > 0)
 *   offset_map  device float32 [n], or NULL: `offset` for every pixel (finite)
 *   extra       device float32 [n], or NULL: 1
 *   weight      device float32 [n], written (usable as lensed_system.weight)
 * Arithmetic in float64, rounded once. n == 0 does nothing. Errors:
 * LENSED_INVALID_ARGUMENT for n < 0, NULL data or weight with n > 0, or a bad
 * scalar gain or offset. */
int lensed_weights_from_data(lensed_ctx* ctx, const float* data, int64_t n, double gain, const float* gain_map,
                             double offset, const float* offset_map, const float* extra, float* weight,
                             void* stream);

/* Log-likelihood and its gradient with respect to the 17 parameters for
 * n_points points of one system: the derivative of Eq. 17 through Eqs. 15, 14,
 * 2 and 1, computed by a hand-written adjoint (transposed PSF with the
 * replicate-padding fold, then per-subsample partial derivatives).
 *   theta  device float32 [n_points * 17]
 *   logl   device float64 [n_points], written
 *   grad   device float32 [n_points * 17], written (d log L / d theta)
 * Any integration rule of the system (midpoint or Gauss-Kronrod) and either
 * amplitude parametrisation (the entries 5 and 12 are then d/dm). Each call
 * derives from the weights as they are then the pixels within the PSF box of
 * a pixel with w > 0 (the only pixels log L and g = A^T rho depend on) and
 * renders and differentiates only those; PSF output tiles without a weighted
 * pixel are skipped, so non-finite data there does not reach log L (the
 * weights may change between calls that reuse the cached plan). */
int lensed_loglike_grad(lensed_ctx* ctx, const lensed_system* sys, const float* theta,
                        int n_points, double* logl, float* grad, void* stream);

/* ---- Surrogate network of log L ------------------------------------------
 * A multilayer perceptron 17 -> 256 -> 256 -> 256 -> 1 with SiLU activations,
 * run on the matrix cores with bfloat16 operands and float32 accumulation. It
 * is trained on (theta, log L) pairs that the exact likelihood produces during
 * a nested-sampling run and used to screen constrained draws; every accepted
 * point is still evaluated exactly (not part of the paper's method: a training
 * pattern added to its sampling loop, Sec. 3.2).
 *   params  device float32 [LENSED_MLP_NPARAM], caller-owned master weights,
 *           layout W1 [256][17], b1 [256], W2 [256][256], b2, W3 [256][256], b3,
 *           W4 [1][256], b4 [1]; converted to bfloat16 on every call
 *   norm    device float32 [36]: x_shift [17], x_scale [17], y_shift, y_scale;
 *           the network sees (x - x_shift) * x_scale and outputs
 *           y_shift + y_scale * net(...)
 *   x       device float32 [batch][17]; y device float32 [batch]
 *   batch   0..65536 rows
 * The context owns the scratch (grown on demand); calls on one context must not
 * overlap. */
#define LENSED_MLP_NPARAM 136449
int lensed_mlp_param_count(void);

/* y = network(x). */
int lensed_mlp_forward(lensed_ctx* ctx, const float* params, const float* norm, const float* x, float* y,
                       int batch, void* stream);

/* Mean squared error in normalised target units, loss = mean((out - (y - y_shift)/y_scale)^2)
 * (device float32 [1]), and its gradient with respect to params (device float32 [LENSED_MLP_NPARAM]). */
int lensed_mlp_grad(lensed_ctx* ctx, const float* params, const float* norm, const float* x, const float* y,
                    int batch, float* grad, float* loss, void* stream);

/* One Adam update (Kingma & Ba 2015) with bias correction for step >= 1:
 * m, v device float32 [LENSED_MLP_NPARAM] moments (start at zero). The
 * hyperparameters are float64 so that 1 - beta and the bias corrections
 * 1 - beta^step are formed exactly before rounding to float32. Invalid
 * arguments: step < 1, non-finite lr, beta outside [0, 1), eps <= 0. */
int lensed_mlp_adam(lensed_ctx* ctx, float* params, const float* grad, float* m, float* v, int step, double lr,
                    double beta1, double beta2, double eps, void* stream);

/* lensed_mlp_grad then lensed_mlp_adam with beta1 = 0.9, beta2 = 0.999, eps = 1e-8. */
int lensed_mlp_train_step(lensed_ctx* ctx, float* params, float* m, float* v, int step, const float* norm,
                          const float* x, const float* y, int batch, double lr, float* loss, void* stream);

/* Instrumentation. With profiling enabled, lensed_loglike_batch runs its stages
 * without the captured graph and records a hipEvent between consecutive stages
 * on `stream`. lensed_stage_times waits for the recorded events and returns,
 * summed over the profiled calls since the previous query, the milliseconds of
 *   ms[0] prologue, ms[1] render kernel, ms[2] float64 cusp corrections,
 *   ms[3] PSF + chi^2, ms[4] finalize,
 * and for lensed_loglike_grad (also profiled) ms[5] A^T rho (the transposed
 * PSF), ms[6] the per-subsample gradient kernel, ms[7] its float64 cusp
 * corrections and the final sums (zero for calls without a gradient)
 * (ms is a HOST array of at least LENSED_NSTAGES doubles; *calls, if not NULL,
 * receives the number of calls summed), then resets the sums. */
#define LENSED_NSTAGES 8
int lensed_set_profiling(lensed_ctx* ctx, int enable);
int lensed_stage_times(lensed_ctx* ctx, double* ms, int n, int* calls);

/* The schedule of the most recent batched call (the batching of Eq. 17 over
 * points and systems): out[0], out[1] the PSF + chi^2 output tile width and
 * height, out[2] the pixels per render thread of the midpoint rules (1, or 2
 * horizontally adjacent pixels sharing the row terms of the subsample grid).
 * On the first batch over a new set of image shapes the library times the
 * best-ranked tiles and both render schedules on that launch and keeps the
 * fastest (unless LENSED_NO_AUTOTUNE is set). out is a HOST array of 3 ints;
 * all zero before any batched call. INVALID_ARGUMENT if out is NULL. */
int lensed_batch_schedule(lensed_ctx* ctx, int* out);

/* Threads per block of the render kernels in the most recent batched call
 * (128, 256 or 512; chosen with the pixels per thread, as above). out is a
 * HOST int, zero before any batched call. INVALID_ARGUMENT if out is NULL. */
int lensed_batch_render_block(lensed_ctx* ctx, int* out);

/* Work of the most recent batched call: out[0] pixels and out[1] subsamples
 * (integration points) its render stage evaluates per launch (all pixels of
 * every point, or only the visible ones of a masked call). out is a HOST array
 * of 2 int64. INVALID_ARGUMENT if out is NULL. */
int lensed_batch_rendered(lensed_ctx* ctx, int64_t* out);

#ifdef __cplusplus
}
#endif

#endif /* LENSED_H */
