"""ctypes binding of liblensed_hip.so: argument marshalling only.

Every step of the forward model and likelihood runs in the library's HIP
kernels; torch supplies device memory and the current stream. The binding
raises if the library has not been built -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblensed_hip.so")
NPARAM = 17

LENSED_OK = 0
_STATUS = {0: "ok", 1: "invalid argument", 2: "HIP runtime error", 3: "out of device memory", 4: "not supported"}


class LensedError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, 'error')} ({status}): {message}")
        self.status = status


class LensedSystemC(ctypes.Structure):
    """Mirror of lensed_system in include/lensed.h."""
    _fields_ = [
        ("height", ctypes.c_int32), ("width", ctypes.c_int32),
        ("pixscale", ctypes.c_float),
        ("center_x", ctypes.c_float), ("center_y", ctypes.c_float),
        ("nsub", ctypes.c_int32),
        ("psf_h", ctypes.c_int32), ("psf_w", ctypes.c_int32),
        ("psf", ctypes.c_void_p), ("data", ctypes.c_void_p), ("weight", ctypes.c_void_p),
        ("rule", ctypes.c_int32),
        ("amplitude", ctypes.c_int32),
        ("zero_point", ctypes.c_float),
        ("source_position", ctypes.c_int32),
    ]


class LensedModelC(ctypes.Structure):
    """Mirror of lensed_model in include/lensed.h."""
    _fields_ = [("n_sie", ctypes.c_int32), ("shear", ctypes.c_int32), ("n_sersic", ctypes.c_int32),
                ("sky", ctypes.c_int32), ("plane", ctypes.c_int32 * 8), ("n_planes", ctypes.c_int32),
                ("sie_plane", ctypes.c_int32 * 8), ("reserved", ctypes.c_int32),
                ("beta", (ctypes.c_double * 8) * 8)]


class Model:
    """A general model (several SIEs with free centres, an optional shear, several
    Sersic components, an optional flat sky; Sec. 5). planes: one entry per
    Sersic, "foreground" (light at x: lens galaxies), "lensed" (light at the
    source plane) or the index of the plane the light sits on.
    Parameters per point: per SIE (x_c, y_c, theta_E, q, phi); shear (gamma,
    phi_gamma); per Sersic (x, y, I_e, R_e, n, q, phi); sky.

    Lenses on several planes: beta, a P x P array of the distance ratios
    beta[i][j] (i < j) of the multi-plane lens equation, and sie_planes, the
    lens plane of every SIE (default: all on plane 0); "lensed" is then plane P."""

    def __init__(self, n_sie: int, planes: Sequence, shear: bool = True, sky: bool = False,
                 sie_planes: Optional[Sequence[int]] = None, beta=None):
        planes = list(planes)
        n_planes = 1 if beta is None else len(beta)
        codes = []
        for p in planes:
            if p == "foreground":
                codes.append(0)
            elif p == "lensed":
                codes.append(n_planes)
            elif isinstance(p, (int, np.integer)):
                codes.append(int(p))
            else:
                raise ValueError("planes must be 'foreground', 'lensed' or a plane index")
        codes += [0] * max(0, 8 - len(codes))
        sp = [0] * int(n_sie) if sie_planes is None else [int(k) for k in sie_planes]
        if len(sp) != n_sie:
            raise ValueError("sie_planes needs one lens plane per SIE")
        b = ((ctypes.c_double * 8) * 8)()
        if beta is not None:
            beta = np.asarray(beta, np.float64)
            if beta.shape != (n_planes, n_planes) or n_planes > 8:
                raise ValueError("beta must be a square array of at most 8 x 8")
            for i in range(n_planes):
                for j in range(n_planes):
                    b[i][j] = beta[i, j]
        self.n_planes = n_planes
        self.c_struct = LensedModelC(int(n_sie), int(bool(shear)), len(planes), int(bool(sky)),
                                     (ctypes.c_int32 * 8)(*codes[:8]), n_planes,
                                     (ctypes.c_int32 * 8)(*(sp + [0] * (8 - len(sp)))[:8]), 0, b)
        self.n_params = lib().lensed_model_nparams(ctypes.byref(self.c_struct))
        if self.n_params < 0 or len(planes) > 8:
            raise ValueError("invalid model: 0..8 SIEs, 1..8 Sersic components, planes and ratios in range")


RULES = {"sub": 0, "g3k7": 1, "g5k11": 2, "g7k15": 3}
AMPLITUDES = {"intensity": 0, "magnitude": 1}
SOURCE_POSITIONS = {"source": 0, "image": 1}


_lib = None
_lib_lock = threading.Lock()


def lib():
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1505_07674_amd.build` "
                                   "(or __graft_entry__.build()) first")
            L = ctypes.CDLL(LIB_PATH)
            i, vp, cp = ctypes.c_int, ctypes.c_void_p, ctypes.c_char_p
            sp = ctypes.POINTER(LensedSystemC)
            sig = {
                "lensed_create": (i, [ctypes.POINTER(vp), i]),
                "lensed_destroy": (None, [vp]),
                "lensed_param_count": (i, []),
                "lensed_status_string": (cp, [i]),
                "lensed_last_error": (cp, [vp]),
                "lensed_render": (i, [vp, sp, vp, vp, i, vp]),
                "lensed_render_error": (i, [vp, sp, vp, vp, vp]),
                "lensed_model_nparams": (i, [vp]),
                "lensed_render_model": (i, [vp, sp, vp, vp, vp, i, vp]),
                "lensed_loglike_model_batch": (i, [vp, sp, i, vp, vp, ctypes.POINTER(ctypes.c_int32), i, vp, vp]),
                "lensed_render_composite": (i, [vp, sp, vp, i, ctypes.c_float, vp, i, vp]),
                "lensed_loglike_composite": (i, [vp, sp, i, vp, i, vp, ctypes.POINTER(ctypes.c_int32), i, vp, vp]),
                "lensed_loglike_multiband": (i, [vp, sp, i, vp, i, ctypes.POINTER(ctypes.c_int32), i, vp, i, vp,
                                                 vp]),
                "lensed_weights_from_data": (i, [vp, vp, ctypes.c_int64, ctypes.c_double, vp, ctypes.c_double, vp, vp,
                                                 vp, vp]),
                "lensed_loglike": (i, [vp, sp, vp, vp, vp]),
                "lensed_loglike_batch": (i, [vp, sp, i, vp, ctypes.POINTER(ctypes.c_int32), i, vp, vp]),
                "lensed_loglike_grad": (i, [vp, sp, vp, i, vp, vp, vp]),
                "lensed_loglike_model_grad": (i, [vp, sp, vp, vp, i, vp, vp, vp]),
                "lensed_loglike_composite_grad": (i, [vp, sp, vp, i, vp, i, vp, vp, vp, vp]),
                "lensed_set_profiling": (i, [vp, i]),
                "lensed_mlp_param_count": (i, []),
                "lensed_mlp_forward": (i, [vp, vp, vp, vp, vp, i, vp]),
                "lensed_mlp_grad": (i, [vp, vp, vp, vp, vp, i, vp, vp, vp]),
                "lensed_mlp_adam": (i, [vp, vp, vp, vp, vp, i, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, vp]),
                "lensed_mlp_train_step": (i, [vp, vp, vp, vp, i, vp, vp, vp, i, ctypes.c_double, vp, vp]),
                "lensed_stage_times": (i, [vp, ctypes.POINTER(ctypes.c_double), i, ctypes.POINTER(ctypes.c_int)]),
                "lensed_batch_schedule": (i, [vp, ctypes.POINTER(ctypes.c_int)]),
                "lensed_batch_render_block": (i, [vp, ctypes.POINTER(ctypes.c_int)]),
                "lensed_batch_rendered": (i, [vp, ctypes.POINTER(ctypes.c_int64)]),
                "lensed_loglike_batch_masked": (i, [vp, sp, i, vp, ctypes.POINTER(ctypes.c_int32), i, vp, vp]),
            }
            for name, (res, args) in sig.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            _lib = L
        return _lib


class Context:
    """Owns a lensed_ctx (workspace, cached batch plans and graphs) on one device."""

    def __init__(self, device: int = 0):
        self.device = int(device)
        h = ctypes.c_void_p()
        rc = lib().lensed_create(ctypes.byref(h), self.device)
        if rc != LENSED_OK:
            raise LensedError(rc, f"lensed_create(device={device})")
        self._h = h

    @property
    def handle(self):
        return self._h

    def check(self, rc: int, what: str):
        if rc != LENSED_OK:
            msg = lib().lensed_last_error(self._h)
            raise LensedError(rc, f"{what}: {msg.decode() if msg else ''}")

    STAGES = ("prologue", "render", "cusp", "psf_chi2", "finalize", "adjoint_psf", "grad", "grad_cusp")

    def set_profiling(self, enable: bool):
        """Run batched and gradient calls stage by stage with hipEvents between the stages (no graph)."""
        self.check(lib().lensed_set_profiling(self._h, int(bool(enable))), "lensed_set_profiling")

    def stage_times(self):
        """Summed per-stage milliseconds of the profiled calls since the last query, and their count."""
        ms = (ctypes.c_double * len(self.STAGES))()
        calls = ctypes.c_int()
        self.check(lib().lensed_stage_times(self._h, ms, len(self.STAGES), ctypes.byref(calls)),
                   "lensed_stage_times")
        return dict(zip(self.STAGES, list(ms))), calls.value

    def batch_schedule(self):
        """Schedule of the most recent batched call: PSF + chi^2 tile (width, height), render pixels per thread
        and render threads per block."""
        out = (ctypes.c_int * 3)()
        self.check(lib().lensed_batch_schedule(self._h, out), "lensed_batch_schedule")
        block = ctypes.c_int()
        self.check(lib().lensed_batch_render_block(self._h, ctypes.byref(block)), "lensed_batch_render_block")
        return {"psf_tile": [out[0], out[1]], "render_pixels_per_thread": out[2], "render_block": block.value}

    def batch_rendered(self):
        """Pixels and subsamples the render stage of the most recent batched call evaluates per launch."""
        out = (ctypes.c_int64 * 2)()
        self.check(lib().lensed_batch_rendered(self._h, out), "lensed_batch_rendered")
        return {"pixels": int(out[0]), "subsamples": int(out[1])}

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().lensed_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_contexts = {}


def default_context(device: Optional[int] = None) -> Context:
    dev = torch.cuda.current_device() if device is None else int(device)
    ctx = _contexts.get(dev)
    if ctx is None:
        ctx = Context(dev)
        _contexts[dev] = ctx
    return ctx


def _stream_handle(stream: Optional[torch.cuda.Stream]) -> ctypes.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_tensor(t: torch.Tensor, dtype: torch.dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    return t.contiguous()


class System:
    """One observation resident on the GPU (Sec. 3, step i).

    data, weight: float32 [H, W] (weight = 1/s^2, 0 = masked); psf: float32
    odd [ph, pw] (normalised by the library). data/weight may be None for
    render-only use.
    """

    def __init__(self, psf: torch.Tensor, data: Optional[torch.Tensor] = None,
                 weight: Optional[torch.Tensor] = None, *, pixscale: float, nsub: int = 1,
                 height: Optional[int] = None, width: Optional[int] = None,
                 center: Tuple[float, float] = (0.0, 0.0), rule: str = "sub", amplitude: str = "intensity",
                 zero_point: float = 0.0, source_position: str = "source"):
        """rule: "sub" (nsub x nsub midpoint) or a Gauss-Kronrod product rule
        "g3k7", "g5k11", "g7k15" (Sec. 4.5; nsub is then ignored).
        amplitude: "intensity" (theta[5], theta[12] are I_e) or "magnitude"
        (they are total magnitudes with the given zero point, Sec. 4.1).
        source_position: "source" (theta[10], theta[11] are the source centre)
        or "image" (an image-plane point mapped to the source centre by the lens
        equation, Sec. 5)."""
        if rule not in RULES:
            raise ValueError(f"rule must be one of {sorted(RULES)}")
        if amplitude not in AMPLITUDES:
            raise ValueError(f"amplitude must be one of {sorted(AMPLITUDES)}")
        if source_position not in SOURCE_POSITIONS:
            raise ValueError(f"source_position must be one of {sorted(SOURCE_POSITIONS)}")
        self.source_position = source_position
        self.rule, self.amplitude, self.zero_point = rule, amplitude, float(zero_point)
        self.psf = _dev_tensor(psf, torch.float32, "psf")
        if self.psf.dim() != 2:
            raise ValueError("psf must be 2-D")
        self.data = None if data is None else _dev_tensor(data, torch.float32, "data")
        self.weight = None if weight is None else _dev_tensor(weight, torch.float32, "weight")
        ref = self.data if self.data is not None else self.weight
        if ref is not None:
            if ref.dim() != 2:
                raise ValueError("data and weight must be 2-D [H, W]")
            height, width = ref.shape
        if height is None or width is None:
            raise ValueError("height and width are required without data")
        for t in (self.data, self.weight):
            if t is not None and tuple(t.shape) != (height, width):
                raise ValueError("data and weight must have the same [H, W] shape")
        self.height, self.width = int(height), int(width)
        self.pixscale, self.nsub = float(pixscale), int(nsub)
        self.center = (float(center[0]), float(center[1]))
        self._c = LensedSystemC(
            self.height, self.width, self.pixscale, self.center[0], self.center[1], self.nsub,
            int(self.psf.shape[0]), int(self.psf.shape[1]), self.psf.data_ptr(),
            None if self.data is None else self.data.data_ptr(),
            None if self.weight is None else self.weight.data_ptr(), RULES[rule], AMPLITUDES[amplitude],
            self.zero_point, SOURCE_POSITIONS[source_position])

    @property
    def c_struct(self) -> LensedSystemC:
        return self._c

    @property
    def device(self) -> torch.device:
        return self.psf.device


def _theta2d(theta: torch.Tensor) -> torch.Tensor:
    t = _dev_tensor(theta, torch.float32, "theta")
    if t.dim() == 1:
        t = t.view(1, -1)
    if t.dim() != 2 or t.shape[1] != NPARAM:
        raise ValueError(f"theta must be [{NPARAM}] or [P, {NPARAM}]")
    return t


def render(theta: torch.Tensor, system: System, apply_psf: bool = True, *, ctx: Optional[Context] = None,
           stream=None) -> torch.Tensor:
    """Model image [H, W] of one point: Eq. 3 by N x N midpoint subsampling, then Eq. 15."""
    t = _theta2d(theta)
    if t.shape[0] != 1:
        raise ValueError("render takes a single parameter point")
    ctx = ctx or default_context(t.device.index)
    out = torch.empty((system.height, system.width), dtype=torch.float32, device=t.device)
    rc = lib().lensed_render(ctx.handle, ctypes.byref(system.c_struct), ctypes.c_void_p(t.data_ptr()),
                             ctypes.c_void_p(out.data_ptr()), int(bool(apply_psf)), _stream_handle(stream))
    ctx.check(rc, "lensed_render")
    return out


def _model_theta(theta: torch.Tensor, model: Model) -> torch.Tensor:
    t = _dev_tensor(theta, torch.float32, "theta")
    if t.dim() == 1:
        t = t.view(1, -1)
    if t.dim() != 2 or t.shape[1] != model.n_params:
        raise ValueError(f"theta must be [{model.n_params}] or [P, {model.n_params}] for this model")
    return t


def render_model(theta: torch.Tensor, system: System, model: Model, apply_psf: bool = True, *,
                 ctx: Optional[Context] = None, stream=None) -> torch.Tensor:
    """Model image [H, W] of one point of a general model."""
    t = _model_theta(theta, model)
    if t.shape[0] != 1:
        raise ValueError("render_model takes a single parameter point")
    ctx = ctx or default_context(t.device.index)
    out = torch.empty((system.height, system.width), dtype=torch.float32, device=t.device)
    rc = lib().lensed_render_model(ctx.handle, ctypes.byref(system.c_struct), ctypes.byref(model.c_struct),
                                   ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                   int(bool(apply_psf)), _stream_handle(stream))
    ctx.check(rc, "lensed_render_model")
    return out


def loglike_model_batch(theta: torch.Tensor, system_of_point, systems: Sequence[System], model: Model, *,
                        out: Optional[torch.Tensor] = None, ctx: Optional[Context] = None,
                        stream=None) -> torch.Tensor:
    """log L of P points of a general model over several systems -> float64 [P]."""
    t = _model_theta(theta, model)
    P = t.shape[0]
    sop = np.ascontiguousarray(np.asarray(system_of_point, dtype=np.int32).reshape(-1))
    if sop.size != P:
        raise ValueError("system_of_point must have one entry per point")
    ctx = ctx or default_context(t.device.index)
    if out is None:
        out = torch.empty(P, dtype=torch.float64, device=t.device)
    sa = _SystemArray(systems)
    rc = lib().lensed_loglike_model_batch(ctx.handle, sa.arr, len(sa.systems), ctypes.byref(model.c_struct),
                                          ctypes.c_void_p(t.data_ptr()),
                                          sop.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), P,
                                          ctypes.c_void_p(out.data_ptr()), _stream_handle(stream))
    ctx.check(rc, "lensed_loglike_model_batch")
    return out


def render_composite(theta: torch.Tensor, system: System, sky: float = 0.0, apply_psf: bool = True, *,
                     ctx: Optional[Context] = None, stream=None) -> torch.Tensor:
    """Model image [H, W] of one composite model: the summed pixel luminosities of
    the K points theta [K, 17] plus a flat sky (sky x pixscale^2 per pixel), then
    the PSF (Sec. 5)."""
    t = _theta2d(theta)
    ctx = ctx or default_context(t.device.index)
    out = torch.empty((system.height, system.width), dtype=torch.float32, device=t.device)
    rc = lib().lensed_render_composite(ctx.handle, ctypes.byref(system.c_struct), ctypes.c_void_p(t.data_ptr()),
                                       t.shape[0], float(sky), ctypes.c_void_p(out.data_ptr()), int(bool(apply_psf)),
                                       _stream_handle(stream))
    ctx.check(rc, "lensed_render_composite")
    return out


def render_error(theta: torch.Tensor, system: System, *, ctx: Optional[Context] = None,
                 stream=None) -> torch.Tensor:
    """Per-pixel |Kronrod - embedded Gauss| estimate [H, W] of a Gauss-Kronrod system (before the PSF)."""
    t = _theta2d(theta)
    if t.shape[0] != 1:
        raise ValueError("render_error takes a single parameter point")
    ctx = ctx or default_context(t.device.index)
    out = torch.empty((system.height, system.width), dtype=torch.float32, device=t.device)
    rc = lib().lensed_render_error(ctx.handle, ctypes.byref(system.c_struct), ctypes.c_void_p(t.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()), _stream_handle(stream))
    ctx.check(rc, "lensed_render_error")
    return out


def weights_from_data(data: torch.Tensor, gain, offset=0.0, extra: Optional[torch.Tensor] = None, *,
                      out: Optional[torch.Tensor] = None, ctx: Optional[Context] = None,
                      stream=None) -> torch.Tensor:
    """Weights w = extra * g / (d + b) of an observation without a variance map
    (Sec. 3.3, Eqs. 18-21); 0 where the counts g (d + b) are not positive. gain
    and offset are numbers or float32 device tensors of the data's shape."""
    if data.dtype != torch.float32 or not data.is_cuda:
        raise ValueError("data must be a float32 device tensor")
    d = data.contiguous()
    ctx = ctx or default_context(d.device.index)

    def as_map(v, what):
        if isinstance(v, torch.Tensor):
            if v.dtype != torch.float32 or v.device != d.device or v.shape != d.shape:
                raise ValueError(f"{what} map must be float32 on the data's device with the data's shape")
            return 0.0, v.contiguous()
        return float(v), None
    g, gmap = as_map(gain, "gain")
    b, bmap = as_map(offset, "offset")
    e = None
    if extra is not None:
        _, e = as_map(extra, "extra")
    if out is None:
        out = torch.empty_like(d)
    elif out.dtype != torch.float32 or out.device != d.device or out.shape != d.shape or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 tensor of the data's shape on its device")
    ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    rc = lib().lensed_weights_from_data(ctx.handle, ptr(d), d.numel(), g, ptr(gmap), b, ptr(bmap), ptr(e), ptr(out),
                                        _stream_handle(stream))
    ctx.check(rc, "lensed_weights_from_data")
    return out


def loglike(theta: torch.Tensor, system: System, *, out: Optional[torch.Tensor] = None,
            ctx: Optional[Context] = None, stream=None) -> torch.Tensor:
    """log L = -chi^2/2 of one point (Eq. 17) as a float64 [1] device tensor (plain form)."""
    t = _theta2d(theta)
    if t.shape[0] != 1:
        raise ValueError("loglike takes a single parameter point; use loglike_batch")
    ctx = ctx or default_context(t.device.index)
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=t.device)
    rc = lib().lensed_loglike(ctx.handle, ctypes.byref(system.c_struct), ctypes.c_void_p(t.data_ptr()),
                              ctypes.c_void_p(out.data_ptr()), _stream_handle(stream))
    ctx.check(rc, "lensed_loglike")
    return out


class _SystemArray:
    def __init__(self, systems: Sequence[System]):
        self.systems = list(systems)
        self.arr = (LensedSystemC * len(self.systems))(*[s.c_struct for s in self.systems])


def loglike_batch(theta: torch.Tensor, system_of_point, systems: Sequence[System], *,
                  out: Optional[torch.Tensor] = None, ctx: Optional[Context] = None, stream=None,
                  masked: bool = False) -> torch.Tensor:
    """log L of P points over several systems in one graph launch -> float64 [P].
    masked: render only the pixels the chi^2 can see (lensed_loglike_batch_masked);
    the same result, bit for bit, for finite data."""
    t = _theta2d(theta)
    P = t.shape[0]
    sop = np.ascontiguousarray(np.asarray(system_of_point, dtype=np.int32).reshape(-1))
    if sop.size != P:
        raise ValueError("system_of_point must have one entry per point")
    ctx = ctx or default_context(t.device.index)
    if out is None:
        out = torch.empty(P, dtype=torch.float64, device=t.device)
    sa = _SystemArray(systems)
    fn = lib().lensed_loglike_batch_masked if masked else lib().lensed_loglike_batch
    rc = fn(ctx.handle, sa.arr, len(sa.systems), ctypes.c_void_p(t.data_ptr()),
            sop.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), P, ctypes.c_void_p(out.data_ptr()),
            _stream_handle(stream))
    ctx.check(rc, "lensed_loglike_batch_masked" if masked else "lensed_loglike_batch")
    return out


def loglike_composite(theta: torch.Tensor, n_components: int, system_of_model, systems: Sequence[System],
                      sky: Optional[torch.Tensor] = None, *, out: Optional[torch.Tensor] = None,
                      ctx: Optional[Context] = None, stream=None) -> torch.Tensor:
    """log L of M composite models of K = n_components points each (theta [M K, 17],
    model m = rows m K .. m K + K - 1; sky: float32 [M] device tensor or None) ->
    float64 [M] (Sec. 5, Eq. 17)."""
    t = _theta2d(theta)
    K = int(n_components)
    if K < 1 or t.shape[0] % K:
        raise ValueError("theta must hold n_components rows per model")
    M = t.shape[0] // K
    som = np.ascontiguousarray(np.asarray(system_of_model, dtype=np.int32).reshape(-1))
    if som.size != M:
        raise ValueError("system_of_model must have one entry per model")
    if sky is not None and (sky.dtype != torch.float32 or sky.device != t.device or sky.numel() != M or
                            not sky.is_contiguous()):
        raise ValueError("sky must be a contiguous float32 tensor of one value per model on theta's device")
    ctx = ctx or default_context(t.device.index)
    if out is None:
        out = torch.empty(M, dtype=torch.float64, device=t.device)
    sa = _SystemArray(systems)
    sky_p = None if sky is None else ctypes.c_void_p(sky.data_ptr())
    rc = lib().lensed_loglike_composite(ctx.handle, sa.arr, len(sa.systems), ctypes.c_void_p(t.data_ptr()), K, sky_p,
                                        som.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), M,
                                        ctypes.c_void_p(out.data_ptr()), _stream_handle(stream))
    ctx.check(rc, "lensed_loglike_composite")
    return out


def loglike_multiband(theta: torch.Tensor, band_systems: Sequence[System], n_components: int = 1,
                      sky: Optional[torch.Tensor] = None, *, out: Optional[torch.Tensor] = None,
                      ctx: Optional[Context] = None, stream=None) -> torch.Tensor:
    """Sum over bands of log L for M models (theta [M B K, 17]: model m, band b is
    the K = n_components rows from (m B + b) K; band b uses band_systems[b]; sky
    float32 [M B] or None) -> float64 [M] (independent bands, Eq. 17 each)."""
    t = _theta2d(theta)
    B, K = len(band_systems), int(n_components)
    if B < 1 or K < 1 or t.shape[0] % (B * K):
        raise ValueError("theta must hold n_bands x n_components rows per model")
    M = t.shape[0] // (B * K)
    if sky is not None and (sky.dtype != torch.float32 or sky.device != t.device or sky.numel() != M * B or
                            not sky.is_contiguous()):
        raise ValueError("sky must be a contiguous float32 tensor of one value per model and band")
    ctx = ctx or default_context(t.device.index)
    if out is None:
        out = torch.empty(M, dtype=torch.float64, device=t.device)
    sa = _SystemArray(band_systems)
    bands = np.arange(B, dtype=np.int32)
    sky_p = None if sky is None else ctypes.c_void_p(sky.data_ptr())
    rc = lib().lensed_loglike_multiband(ctx.handle, sa.arr, B, ctypes.c_void_p(t.data_ptr()), B,
                                        bands.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), K, sky_p, M,
                                        ctypes.c_void_p(out.data_ptr()), _stream_handle(stream))
    ctx.check(rc, "lensed_loglike_multiband")
    return out


def loglike_grad(theta: torch.Tensor, system: System, *, ctx: Optional[Context] = None,
                 stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """log L and d log L / d theta for P points of one system -> (float64 [P], float32 [P, 17])."""
    t = _theta2d(theta)
    P = t.shape[0]
    ctx = ctx or default_context(t.device.index)
    ll = torch.empty(P, dtype=torch.float64, device=t.device)
    g = torch.empty((P, NPARAM), dtype=torch.float32, device=t.device)
    rc = lib().lensed_loglike_grad(ctx.handle, ctypes.byref(system.c_struct), ctypes.c_void_p(t.data_ptr()), P,
                                   ctypes.c_void_p(ll.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                                   _stream_handle(stream))
    ctx.check(rc, "lensed_loglike_grad")
    return ll, g


def loglike_composite_grad(theta: torch.Tensor, n_components: int, system: System, *,
                           sky: Optional[torch.Tensor] = None, ctx: Optional[Context] = None,
                           stream=None):
    """log L and its gradient for composite models of n_components points on one
    system -> (float64 [n_models], float32 [n_models * n_components, 17],
    float32 [n_models] d log L / d sky or None without a sky)."""
    t = _theta2d(theta)
    n_points = t.shape[0]
    if n_components < 1 or n_points % n_components:
        raise ValueError("theta must hold n_models x n_components points")
    n_models = n_points // n_components
    ctx = ctx or default_context(t.device.index)
    ll = torch.empty(n_models, dtype=torch.float64, device=t.device)
    g = torch.empty((n_points, NPARAM), dtype=torch.float32, device=t.device)
    sk = gs = None
    if sky is not None:
        sk = sky.to(device=t.device, dtype=torch.float32).contiguous()
        if sk.numel() != n_models:
            raise ValueError("sky must hold one value per model")
        gs = torch.empty(n_models, dtype=torch.float32, device=t.device)
    rc = lib().lensed_loglike_composite_grad(ctx.handle, ctypes.byref(system.c_struct), ctypes.c_void_p(t.data_ptr()),
                                             int(n_components), ctypes.c_void_p(sk.data_ptr() if sk is not None else None),
                                             n_models, ctypes.c_void_p(ll.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                                             ctypes.c_void_p(gs.data_ptr() if gs is not None else None),
                                             _stream_handle(stream))
    ctx.check(rc, "lensed_loglike_composite_grad")
    return ll, g, gs


def loglike_model_grad(theta: torch.Tensor, system: System, model: Model, *, ctx: Optional[Context] = None,
                       stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """log L and d log L / d theta for P points of a general model (one lens
    plane) on one system -> (float64 [P], float32 [P, model.n_params])."""
    t = _model_theta(theta, model)
    P = t.shape[0]
    ctx = ctx or default_context(t.device.index)
    ll = torch.empty(P, dtype=torch.float64, device=t.device)
    g = torch.empty((P, model.n_params), dtype=torch.float32, device=t.device)
    rc = lib().lensed_loglike_model_grad(ctx.handle, ctypes.byref(system.c_struct), ctypes.byref(model.c_struct),
                                         ctypes.c_void_p(t.data_ptr()), P, ctypes.c_void_p(ll.data_ptr()),
                                         ctypes.c_void_p(g.data_ptr()), _stream_handle(stream))
    ctx.check(rc, "lensed_loglike_model_grad")
    return ll, g


MLP_NPARAM = 136449


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def mlp_forward(params: torch.Tensor, norm: torch.Tensor, x: torch.Tensor, *, out: Optional[torch.Tensor] = None,
                ctx: Optional[Context] = None, stream=None) -> torch.Tensor:
    """Surrogate prediction y [B] for inputs x [B, 17] (bfloat16 MFMA kernels)."""
    params = _dev_tensor(params, torch.float32, "params")
    norm = _dev_tensor(norm, torch.float32, "norm")
    x = _dev_tensor(x, torch.float32, "x")
    if params.numel() != MLP_NPARAM or norm.numel() != 36 or x.dim() != 2 or x.shape[1] != NPARAM:
        raise ValueError("params [136449], norm [36] and x [B, 17] expected")
    ctx = ctx or default_context(x.device.index)
    B = x.shape[0]
    if out is None:
        out = torch.empty(B, dtype=torch.float32, device=x.device)
    rc = lib().lensed_mlp_forward(ctx.handle, _ptr(params), _ptr(norm), _ptr(x), _ptr(out), B,
                                  _stream_handle(stream))
    ctx.check(rc, "lensed_mlp_forward")
    return out


def mlp_grad(params: torch.Tensor, norm: torch.Tensor, x: torch.Tensor, y: torch.Tensor, *,
             ctx: Optional[Context] = None, stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """(loss [1], gradient [136449]) of the mean squared error in normalised target units."""
    params = _dev_tensor(params, torch.float32, "params")
    norm = _dev_tensor(norm, torch.float32, "norm")
    x = _dev_tensor(x, torch.float32, "x")
    y = _dev_tensor(y, torch.float32, "y")
    ctx = ctx or default_context(x.device.index)
    g = torch.empty(MLP_NPARAM, dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    rc = lib().lensed_mlp_grad(ctx.handle, _ptr(params), _ptr(norm), _ptr(x), _ptr(y), x.shape[0], _ptr(g),
                               _ptr(loss), _stream_handle(stream))
    ctx.check(rc, "lensed_mlp_grad")
    return loss, g


def mlp_adam(params: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int, lr: float,
             beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, *, ctx: Optional[Context] = None,
             stream=None) -> None:
    """In-place Adam update of params, m, v."""
    ctx = ctx or default_context(params.device.index)
    rc = lib().lensed_mlp_adam(ctx.handle, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr),
                               float(beta1), float(beta2), float(eps), _stream_handle(stream))
    ctx.check(rc, "lensed_mlp_adam")


def mlp_train_step(params: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int, norm: torch.Tensor,
                   x: torch.Tensor, y: torch.Tensor, lr: float, *, loss: Optional[torch.Tensor] = None,
                   ctx: Optional[Context] = None, stream=None) -> torch.Tensor:
    """Gradient and Adam step in one call; returns the loss tensor [1] (before the step)."""
    ctx = ctx or default_context(params.device.index)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=params.device)
    rc = lib().lensed_mlp_train_step(ctx.handle, _ptr(params), _ptr(m), _ptr(v), int(step), _ptr(norm), _ptr(x),
                                     _ptr(y), x.shape[0], float(lr), _ptr(loss), _stream_handle(stream))
    ctx.check(rc, "lensed_mlp_train_step")
    return loss


class LogLikeFn(torch.autograd.Function):
    """log L(theta) for [P, 17] points of one system with the hand-written adjoint as backward."""

    @staticmethod
    def forward(ctx_, theta: torch.Tensor, system: System):
        ll, g = loglike_grad(theta.detach(), system)
        ctx_.save_for_backward(g)
        return ll

    @staticmethod
    def backward(ctx_, grad_out: torch.Tensor):
        (g,) = ctx_.saved_tensors
        return (grad_out.to(g.dtype)[:, None] * g), None


class LogLikeModelFn(torch.autograd.Function):
    """log L(theta) for [P, n_params] points of a general model on one system,
    with the library's adjoint (lensed_loglike_model_grad) as backward."""

    @staticmethod
    def forward(ctx_, theta: torch.Tensor, system: System, model: Model):
        ll, g = loglike_model_grad(theta.detach(), system, model)
        ctx_.save_for_backward(g)
        return ll

    @staticmethod
    def backward(ctx_, grad_out: torch.Tensor):
        (g,) = ctx_.saved_tensors
        return (grad_out.to(g.dtype)[:, None] * g), None, None
