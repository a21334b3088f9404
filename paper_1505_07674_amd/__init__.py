"""MI355X-native forward strong-lensing likelihood.

Hot path of the forward reconstruction method of Tessore, Bellagamba & Metcalf
(LENSED, MNRAS 2016): ray-trace every pixel subsample through an SIE plus
external shear (Eq. 1), add the lensed Sersic source to the Sersic lens light
(Eq. 2), integrate over the pixel (Eqs. 3, 14), convolve with the PSF (Eq. 15)
and reduce the weighted chi^2 / log-likelihood (Eq. 17) -- all in hand-written
HIP kernels for gfx950 behind the C ABI of include/lensed.h.
"""
from .binding import (MLP_NPARAM, NPARAM, Context, Model, loglike_model_batch, loglike_model_grad, loglike_composite_grad, render_model, LensedError, LogLikeFn, LogLikeModelFn, System, default_context, loglike,
                      loglike_batch, loglike_grad, mlp_adam, mlp_forward, mlp_grad, mlp_train_step, render,
                      loglike_composite, loglike_multiband, render_composite, render_error, weights_from_data)

__all__ = ["MLP_NPARAM", "NPARAM", "Context", "Model", "loglike_model_batch", "loglike_model_grad", "loglike_composite_grad", "render_model", "LensedError", "LogLikeFn", "LogLikeModelFn", "System", "default_context", "loglike",
           "loglike_batch", "loglike_grad", "mlp_adam", "mlp_forward", "mlp_grad", "mlp_train_step", "render",
           "render_error", "weights_from_data", "loglike_composite", "loglike_multiband", "render_composite"]
