"""Python binding of libecc: spatially adaptive correlation/convolution on MI355X.

Thin wrappers with the C ABI's names (include/ecc.h). Tensors are torch tensors on a
HIP device (float32, contiguous rows); every call passes raw device pointers and the
current HIP stream. No computation happens here: if the library is missing the import
of `lib()` raises.
"""
from __future__ import annotations

import atexit
import ctypes as C
import sys
import weakref
from typing import Optional

from . import _lib
from ._lib import (BATCH_AUTOTUNE, BATCH_PERSISTENT, CONVOLUTION, CORRELATION, GROUP_ROTATION,
                   GROUP_SCALE, PREC_FP32, PREC_MFMA_BF16_HILO, PREC_MFMA_FP16_HILO, STRATEGY_AUTO,
                   STRATEGY_TILED, STRATEGY_TWO_PASS, STRATEGY_DIRECT, WS_BACKWARD_CONVOLUTION,
                   WS_BACKWARD_CORRELATION, WS_EXTENDED_CONVOLUTION, WS_EXTENDED_CORRELATION,
                   WS_MATCH_ROTATIONS, WS_NORMALIZED_CONVOLUTION, WS_SCALE_SMOOTH, WS_JOINT_CONVOLUTION,
                   GROUP_ROTATION_SCALE, EccError,
                   GroupParams, Instance)

__all__ = [
    "lib", "Context", "FilterPlan", "ecc_extended", "ecc_scale_smooth", "ecc_match_rotations",
    "ecc_normalized_convolution", "WS_NORMALIZED_CONVOLUTION",
    "ecc_gradient_field", "ecc_voting_filter", "ecc_find_peaks", "detect_pattern",
    "ecc_joint_convolution", "GROUP_ROTATION_SCALE", "WS_JOINT_CONVOLUTION",
    "ecc_match_rotations_noalloc", "VolumePlan", "ecc_extended_3d",
    "ecc_extended_backward", "ecc_extended_save", "ecc_backward_saved_size", "ExtConv", "ExtCorr",
    "CORRELATION", "CONVOLUTION", "GROUP_ROTATION", "GROUP_SCALE", "PREC_FP32", "EccError",
    "STRATEGY_AUTO", "STRATEGY_TWO_PASS", "STRATEGY_TILED", "STRATEGY_DIRECT", "BatchPlan", "BATCH_AUTOTUNE",
    "PREC_MFMA_FP16_HILO", "PREC_MFMA_BF16_HILO",
    "BATCH_PERSISTENT",
    "GroupParams",
    "WS_EXTENDED_CORRELATION", "WS_EXTENDED_CONVOLUTION", "WS_SCALE_SMOOTH", "WS_MATCH_ROTATIONS",
    "WS_BACKWARD_CONVOLUTION", "WS_BACKWARD_CORRELATION",
]

_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = _lib.load()
    return _LIB


def _check(status):
    if status != _lib.ECC_OK:
        raise EccError(status, lib().ecc_last_error(None).decode())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _img(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32):
        raise TypeError(f"{name} must be a float32 tensor on a HIP device")
    if t.stride(-1) != 1:
        raise ValueError(f"{name} must have unit column stride")
    return t


def _ld(t):
    return t.stride(-2) if t.dim() >= 2 else t.shape[-1]


# Contexts and batch plans still open when the interpreter exits are destroyed by an exit
# hook, while the HIP runtime is fully alive; finalizers that run later, during interpreter
# teardown, do not call into the library (a runtime call at that point can block forever).
_open_contexts = weakref.WeakSet()
_open_batches = weakref.WeakSet()
_exit_hook = []


def _close_all_at_exit():
    for b in list(_open_batches):
        try:
            b.close()
        except Exception:
            pass
    for c in list(_open_contexts):
        try:
            c.close()
        except Exception:
            pass


def _track(registry, obj):
    # registered on first use, i.e. after torch (imported by the caller to make device
    # tensors) has registered its own exit handlers, so that this one runs before them
    if not _exit_hook:
        atexit.register(_close_all_at_exit)
        _exit_hook.append(True)
    registry.add(obj)


class Context:
    """Owns a libecc context on one HIP device."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        _check(lib().ecc_create(device, C.byref(h)))
        self.h = h
        self.device = device
        self._plans = weakref.WeakSet()
        _track(_open_contexts, self)

    def close(self):
        """Destroys the context; plans made from it are closed first."""
        if self.h:
            for p in list(self._plans):
                p.close()
            lib().ecc_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # (bound at definition: module globals are gone when the interpreter tears down)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def fft_size(self, n: int, R: int) -> int:
        P = C.c_int()
        _check(lib().ecc_fft_size(self.h, n, R, C.byref(P)))
        return P.value

    def set_strategy(self, strategy: int):
        _check(lib().ecc_set_strategy(self.h, strategy))

    def set_autotune(self, enable: bool = True):
        """Block shapes chosen from on-device measurements (taken once per context, at the
        next forward call or describe) instead of an operation count."""
        _check(lib().ecc_set_autotune(self.h, 1 if enable else 0))

    def autotune_export(self) -> str:
        """The autotuner's measurements as JSON text (see ecc_autotune_export)."""
        n = C.c_size_t()
        _check(lib().ecc_autotune_export(self.h, None, 0, C.byref(n)))
        buf = C.create_string_buffer(n.value + 1)
        _check(lib().ecc_autotune_export(self.h, buf, n.value + 1, C.byref(n)))
        return buf.value.decode()

    def autotune_import(self, text: str):
        """Takes measurements exported on the same kind of device; no calibration runs."""
        _check(lib().ecc_autotune_import(self.h, text.encode()))

    def workspace_size(self, call: int, plan: "FilterPlan", ny: int, nx: int, batch: int = 1) -> int:
        """Bytes of context workspace that `call` (an ecc_ws_call value, WS_*) needs."""
        n = C.c_size_t()
        _check(lib().ecc_workspace_size(self.h, call, plan.h, batch, ny, nx, C.byref(n)))
        return n.value

    def workspace_reserve(self, nbytes: int):
        _check(lib().ecc_workspace_reserve(self.h, nbytes))

    def workspace_allocated(self) -> int:
        n = C.c_size_t()
        _check(lib().ecc_workspace_allocated(self.h, C.byref(n)))
        return n.value

    def volume_workspace_size(self, plan: "VolumePlan", nz: int, ny: int, nx: int) -> int:
        """Bytes of context workspace ecc_extended_3d needs for this volume size."""
        n = C.c_size_t()
        _check(lib().ecc_volume_workspace_size(self.h, plan.h, nz, ny, nx, C.byref(n)))
        return n.value

    def describe(self, op: int, plan: "FilterPlan", ny: int, nx: int):
        """(strategy, transform length, block side) that ecc_extended would use."""
        s, n, b = C.c_int(), C.c_int(), C.c_int()
        _check(lib().ecc_describe(self.h, op, plan.h, ny, nx, C.byref(s), C.byref(n), C.byref(b)))
        return s.value, n.value, b.value


class FilterPlan:
    """A filter decomposed into components F_k, k = 0..K (see ecc_filter_plan_create)."""

    def __init__(self, ctx: Context, h):
        self.ctx = ctx
        self.h = h
        ctx._plans.add(self)
        S, K, M = C.c_int(), C.c_int(), C.c_int()
        _check(lib().ecc_filter_plan_info(h, C.byref(S), C.byref(K), C.byref(M)))
        self.S, self.K, self.M = S.value, K.value, M.value

    @classmethod
    def rotation(cls, ctx: Context, filt, K: int, angular_samples: int = 0, stream=None):
        filt = _img(filt, "filter").contiguous()
        gp = GroupParams(angular_samples=angular_samples)
        h = C.c_void_p()
        _check(lib().ecc_filter_plan_create(ctx.h, GROUP_ROTATION, _ptr(filt), filt.shape[-1], K,
                                            C.byref(gp), _stream(stream), C.byref(h)))
        return cls(ctx, h)

    @classmethod
    def joint(cls, ctx: Context, filt, K: int, n_log: int = 9, scale_min: float = 1.0, scale_max: float = 2.0,
              period_factor: float = 1.5, angular_samples: int = 0, stream=None):
        """Rotation-and-scale plan of an S x S float32 device filter: modes (k, l), k = -K..K,
        n_log (odd) log-radial modes over the scale range [scale_min, scale_max]."""
        filt = _img(filt, "filter").contiguous()
        gp = GroupParams(angular_samples=angular_samples, sigma0=0.0, scale_min=scale_min, scale_max=scale_max,
                         scale_components=n_log, scale_period_factor=period_factor)
        h = C.c_void_p()
        _check(lib().ecc_filter_plan_create(ctx.h, GROUP_ROTATION_SCALE, _ptr(filt), filt.shape[-1], K,
                                            C.byref(gp), _stream(stream), C.byref(h)))
        return cls(ctx, h)

    @classmethod
    def scale(cls, ctx: Context, sigma0=1.0, scale_min=1.0, scale_max=8.0, components=24,
              period_factor=1.5, stream=None):
        gp = GroupParams(0, sigma0, scale_min, scale_max, components, period_factor)
        h = C.c_void_p()
        _check(lib().ecc_filter_plan_create(ctx.h, GROUP_SCALE, None, 0, 0, C.byref(gp),
                                            _stream(stream), C.byref(h)))
        return cls(ctx, h)

    @classmethod
    def from_components(cls, ctx: Context, comps, group=GROUP_ROTATION, gp: Optional[GroupParams] = None,
                        stream=None):
        """comps: complex64 tensor (K+1, S, S) on the device."""
        import torch
        if not (comps.is_cuda and comps.dtype == torch.complex64 and comps.dim() == 3):
            raise TypeError("comps must be a (K+1, S, S) complex64 device tensor")
        comps = comps.contiguous()
        h = C.c_void_p()
        _check(lib().ecc_filter_plan_from_components(ctx.h, group, _ptr(comps), comps.shape[-1],
                                                     comps.shape[0] - 1,
                                                     C.byref(gp) if gp is not None else None,
                                                     _stream(stream), C.byref(h)))
        return cls(ctx, h)

    def components(self, stream=None):
        import torch
        U = C.c_int()
        _check(lib().ecc_filter_plan_component_count(self.h, C.byref(U)))
        out = torch.empty((U.value, self.S, self.S), dtype=torch.complex64, device=f"cuda:{self.ctx.device}")
        _check(lib().ecc_filter_plan_get_components(self.h, _ptr(out), _stream(stream)))
        return out

    def close(self):
        if self.h:
            lib().ecc_filter_plan_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # (bound at definition: module globals are gone when the interpreter tears down)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class VolumePlan:
    """Spherical-harmonic components of an S x S x S filter up to band limit K (steering
    in 3D; see ecc_volume_plan_create)."""

    def __init__(self, ctx: Context, filt, K: int, stream=None):
        import torch
        if not (isinstance(filt, torch.Tensor) and filt.is_cuda and filt.dtype == torch.float32 and filt.dim() == 3):
            raise TypeError("filter must be an (S, S, S) float32 tensor on a HIP device")
        filt = filt.contiguous()
        h = C.c_void_p()
        _check(lib().ecc_volume_plan_create(ctx.h, _ptr(filt), filt.shape[-1], K, _stream(stream), C.byref(h)))
        self.ctx, self.h, self.S, self.K = ctx, h, filt.shape[-1], K
        ctx._plans.add(self)
        U, M = C.c_int(), C.c_int()
        _check(lib().ecc_volume_plan_info(h, C.byref(U), C.byref(M)))
        self.U, self.M = U.value, M.value

    def components(self, stream=None):
        """(comps complex64 (U, S, S, S) on the device, table int32 (U, 3) of (l, m', m),
        weights float32 (U,))."""
        import numpy as np
        import torch
        comps = torch.empty((self.U, self.S, self.S, self.S), dtype=torch.complex64,
                            device=f"cuda:{self.ctx.device}")
        table = np.zeros((self.U, 3), dtype=np.int32)
        w = np.zeros(self.U, dtype=np.float32)
        _check(lib().ecc_volume_plan_components(self.h, _ptr(comps), table.ctypes.data_as(C.c_void_p),
                                                w.ctypes.data_as(C.c_void_p), _stream(stream)))
        return comps, table, w

    def close(self):
        if self.h:
            lib().ecc_volume_plan_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # (bound at definition: module globals are gone when the interpreter tears down)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def ecc_extended_3d(ctx: Context, op: int, plan: VolumePlan, signal, alpha, beta, gamma, out=None, stream=None):
    """Extended correlation / convolution of an (nz, ny, nx) float32 device volume with the
    rotation field given by ZYZ Euler angles alpha, beta, gamma (same shape)."""
    import torch
    vols = (signal, alpha, beta, gamma)
    for t, n in zip(vols, ("signal", "alpha", "beta", "gamma")):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.dim() == 3
                and t.is_contiguous()):
            raise TypeError(f"{n} must be a contiguous (nz, ny, nx) float32 tensor on a HIP device")
        if t.shape != signal.shape:
            raise ValueError("signal and angle volumes differ in shape")
    if out is None:
        out = torch.empty(signal.shape, dtype=torch.float32, device=signal.device)
    if not (out.is_contiguous() and out.shape == signal.shape and out.dtype == torch.float32):
        raise ValueError("out must be a contiguous float32 volume of the signal's shape")
    nz, ny, nx = signal.shape
    _check(lib().ecc_extended_3d(ctx.h, op, plan.h, nz, ny, nx, _ptr(signal), _ptr(alpha), _ptr(beta), _ptr(gamma),
                                 _ptr(out), _stream(stream)))
    return out


def ecc_extended(ctx: Context, op: int, plan: FilterPlan, signal, field, out=None, stream=None):
    """Extended correlation (op=CORRELATION) or convolution (op=CONVOLUTION).
    signal, field: (ny, nx) or (batch, ny, nx) float32 device tensors."""
    import torch
    _img(signal, "signal")
    _img(field, "field")
    if out is None:
        out = torch.empty(signal.shape, dtype=torch.float32, device=signal.device)
    _img(out, "out")
    ny, nx = signal.shape[-2], signal.shape[-1]
    batch = signal.shape[0] if signal.dim() == 3 else 1
    for t in (signal, field, out):
        if t.dim() == 3 and t.stride(0) != t.shape[-2] * t.stride(-2):
            raise ValueError("batched images must be stacked with image stride ny * ld")
    _check(lib().ecc_extended(ctx.h, op, plan.h, batch, ny, nx, _ptr(signal), _ld(signal),
                              _ptr(field), _ld(field), _ptr(out), _ld(out), PREC_FP32,
                              _stream(stream)))
    return out


def ecc_normalized_convolution(ctx: Context, plan: FilterPlan, signal, field, out=None, stream=None,
                               precision=PREC_FP32):
    """Extended convolution of the signal over that of the constant 1 (rotation plans:
    line-integral convolution with an anisotropic filter; scale plans: the smoothing of
    ecc_scale_smooth). signal, field: (ny, nx) or (batch, ny, nx) float32 device tensors."""
    import torch
    _img(signal, "signal")
    _img(field, "field")
    if out is None:
        out = torch.empty(signal.shape, dtype=torch.float32, device=signal.device)
    _img(out, "out")
    ny, nx = signal.shape[-2], signal.shape[-1]
    batch = signal.shape[0] if signal.dim() == 3 else 1
    for t in (signal, field, out):
        if t.dim() == 3 and t.stride(0) != t.shape[-2] * t.stride(-2):
            raise ValueError("batched images must be stacked with image stride ny * ld")
    _check(lib().ecc_normalized_convolution(ctx.h, plan.h, batch, ny, nx, _ptr(signal), _ld(signal),
                                            _ptr(field), _ld(field), _ptr(out), _ld(out), precision,
                                            _stream(stream)))
    return out


def ecc_joint_convolution(ctx: Context, plan: FilterPlan, signal, angle, scale, normalized=False, out=None,
                          stream=None):
    """Extended convolution with joint rotation (angle) and scale fields, or the normalised
    smoothing (normalized=True); (ny, nx) or (batch, ny, nx) float32 device tensors."""
    import torch
    for t, n in ((signal, "signal"), (angle, "angle"), (scale, "scale")):
        _img(t, n)
    if out is None:
        out = torch.empty(signal.shape, dtype=torch.float32, device=signal.device)
    _img(out, "out")
    ny, nx = signal.shape[-2], signal.shape[-1]
    batch = signal.shape[0] if signal.dim() == 3 else 1
    for t in (signal, angle, scale, out):
        if t.dim() == 3 and t.stride(0) != t.shape[-2] * t.stride(-2):
            raise ValueError("batched images must be stacked with image stride ny * ld")
    _check(lib().ecc_joint_convolution(ctx.h, plan.h, batch, ny, nx, _ptr(signal), _ld(signal), _ptr(angle),
                                       _ld(angle), _ptr(scale), _ld(scale), _ptr(out), _ld(out),
                                       1 if normalized else 0, _stream(stream)))
    return out


def ecc_scale_smooth(ctx: Context, plan: FilterPlan, signal, scale, out=None, stream=None, precision=PREC_FP32):
    import torch
    _img(signal, "signal")
    _img(scale, "scale")
    if out is None:
        out = torch.empty(signal.shape, dtype=torch.float32, device=signal.device)
    ny, nx = signal.shape
    _check(lib().ecc_scale_smooth(ctx.h, plan.h, ny, nx, _ptr(signal), _ld(signal), _ptr(scale),
                                  _ld(scale), _ptr(out), _ld(out), precision, _stream(stream)))
    return out


def ecc_match_rotations(ctx: Context, plan: FilterPlan, signal, n_angles=64, precision=PREC_FP32,
                        stream=None):
    """Best angle score and index per pixel (precision: PREC_FP32, PREC_MFMA_FP16_HILO or
    PREC_MFMA_BF16_HILO for the angle search)."""
    import torch
    _img(signal, "signal")
    ny, nx = signal.shape
    score = torch.empty((ny, nx), dtype=torch.float32, device=signal.device)
    index = torch.empty((ny, nx), dtype=torch.int32, device=signal.device)
    _check(lib().ecc_match_rotations(ctx.h, plan.h, ny, nx, _ptr(signal), _ld(signal), n_angles,
                                     _ptr(score), _ptr(index), nx, precision, _stream(stream)))
    return score, index


def ecc_match_rotations_noalloc(ctx: Context, plan: FilterPlan, signal, score, index, n_angles=64,
                                precision=PREC_FP32, stream=None):
    """ecc_match_rotations into the caller's score (float32) and index (int32) tensors,
    with the library allocating nothing (the plan must have run ecc_match_rotations with
    the same size and n_angles once)."""
    import torch
    _img(signal, "signal")
    ny, nx = signal.shape
    if score.shape != (ny, nx) or index.shape != (ny, nx) or score.dtype != torch.float32 \
            or index.dtype != torch.int32 or not score.is_contiguous() or not index.is_contiguous():
        raise ValueError("score / index must be contiguous float32 / int32 tensors of the signal's shape")
    _check(lib().ecc_match_rotations_noalloc(ctx.h, plan.h, ny, nx, _ptr(signal), _ld(signal), n_angles,
                                             _ptr(score), _ptr(index), nx, precision, _stream(stream)))
    return score, index


def ecc_gradient_field(ctx: Context, image, magnitude=None, angle=None, stream=None):
    """(|grad I|, atan2(I_y, I_x)) of (ny, nx) or (batch, ny, nx) float32 device images."""
    import torch
    _img(image, "image")
    if magnitude is None:
        magnitude = torch.empty(image.shape, dtype=torch.float32, device=image.device)
    if angle is None:
        angle = torch.empty(image.shape, dtype=torch.float32, device=image.device)
    _img(magnitude, "magnitude")
    _img(angle, "angle")
    if _ld(magnitude) != _ld(angle):
        raise ValueError("magnitude and angle must share their row stride")
    ny, nx = image.shape[-2], image.shape[-1]
    batch = image.shape[0] if image.dim() == 3 else 1
    for t in (image, magnitude, angle):
        if t.dim() == 3 and t.stride(0) != t.shape[-2] * t.stride(-2):
            raise ValueError("batched images must be stacked with image stride ny * ld")
    _check(lib().ecc_gradient_field(ctx.h, batch, ny, nx, _ptr(image), _ld(image), _ptr(magnitude), _ptr(angle),
                                    _ld(magnitude), _stream(stream)))
    return magnitude, angle


def ecc_voting_filter(ctx: Context, pattern, stream=None):
    """Consensus filter (S x S float32) of an S x S float32 device pattern, S odd."""
    import torch
    _img(pattern, "pattern")
    if pattern.dim() != 2 or pattern.shape[0] != pattern.shape[1] or not pattern.is_contiguous():
        raise ValueError("pattern must be a contiguous S x S tensor")
    F = torch.empty_like(pattern)
    _check(lib().ecc_voting_filter(ctx.h, pattern.shape[0], _ptr(pattern), _ptr(F), _stream(stream)))
    return F


def ecc_find_peaks(ctx: Context, response, radius, threshold, relative=False, max_peaks=64, stream=None):
    """Peaks of a (ny, nx) float32 device response: (rows, cols, values) device tensors of the
    strongest ones, by decreasing value (waits for the stream to read their number)."""
    import torch
    _img(response, "response")
    ny, nx = response.shape
    dev = response.device
    rows = torch.empty(max_peaks, dtype=torch.int32, device=dev)
    cols = torch.empty(max_peaks, dtype=torch.int32, device=dev)
    vals = torch.empty(max_peaks, dtype=torch.float32, device=dev)
    count = torch.empty(1, dtype=torch.int32, device=dev)
    _check(lib().ecc_find_peaks(ctx.h, ny, nx, _ptr(response), _ld(response), radius, C.c_float(threshold),
                                1 if relative else 0, max_peaks, _ptr(rows), _ptr(cols), _ptr(vals), _ptr(count),
                                _stream(stream)))
    n = int(count.item())
    return rows[:n], cols[:n], vals[:n]


def detect_pattern(ctx: Context, image, pattern, K, radius=8, threshold=0.3, relative=True, max_peaks=64,
                   stream=None):
    """Pattern detection by extended convolution (Sec. 5), as a sequence of library calls:
    signal and field of the image, the pattern's consensus filter, its plan (band limit K),
    the extended convolution, the peaks. Returns (rows, cols, values, response)."""
    H, theta = ecc_gradient_field(ctx, image, stream=stream)
    F = ecc_voting_filter(ctx, pattern, stream=stream)
    plan = FilterPlan.rotation(ctx, F, K, stream=stream)
    try:
        D = ecc_extended(ctx, CONVOLUTION, plan, H, theta, stream=stream)
    finally:
        plan.close()
    rows, cols, vals = ecc_find_peaks(ctx, D, radius, threshold, relative, max_peaks, stream=stream)
    return rows, cols, vals, D


def ecc_backward_saved_size(ctx: Context, plan: FilterPlan, batch, ny, nx) -> int:
    n = C.c_size_t()
    _check(lib().ecc_backward_saved_size(ctx.h, plan.h, batch, ny, nx, C.byref(n)))
    return n.value


def ecc_extended_save(ctx: Context, plan: FilterPlan, signal, field, saved, out=None, stream=None):
    import torch
    signal = signal.contiguous()
    field = field.contiguous()
    if out is None:
        out = torch.empty(signal.shape, dtype=torch.float32, device=signal.device)
    batch = signal.shape[0] if signal.dim() == 3 else 1
    ny, nx = signal.shape[-2:]
    _check(lib().ecc_extended_save(ctx.h, plan.h, batch, ny, nx, _ptr(signal), _ptr(field),
                                   _ptr(out), _ptr(saved), _stream(stream)))
    return out


def ecc_extended_backward(ctx: Context, plan: FilterPlan, signal, field, grad_out, need_signal=True,
                          need_comps=True, need_field=True, saved=None, stream=None, op=CONVOLUTION):
    """Adjoint of the extended convolution (op=CONVOLUTION) or correlation
    (op=CORRELATION, saved must be None): returns (grad_signal, grad_comps, grad_field)."""
    import torch
    signal = signal.contiguous()
    field = field.contiguous()
    grad_out = grad_out.contiguous()
    batch = signal.shape[0] if signal.dim() == 3 else 1
    ny, nx = signal.shape[-2:]
    dev = signal.device
    gs = torch.empty(signal.shape, dtype=torch.float32, device=dev) if need_signal else None
    gf = torch.empty(signal.shape, dtype=torch.float32, device=dev) if need_field else None
    gc = torch.empty((plan.K + 1, plan.S, plan.S), dtype=torch.complex64, device=dev) if need_comps else None
    _check(lib().ecc_extended_backward(ctx.h, op, plan.h, batch, ny, nx, _ptr(signal),
                                       _ptr(field), _ptr(grad_out), _ptr(gs), _ptr(gc), _ptr(gf),
                                       _ptr(saved), _stream(stream)))
    return gs, gc, gf


def _ext_conv_function():
    import torch

    class ExtConv(torch.autograd.Function):
        """y = extended convolution of `signal` with components `comps` ((K+1, S, S)
        complex64) steered by the angle field `theta`; backward uses the hand-written
        adjoint. The modulated-signal stack is kept from the forward pass only when the
        backward reads it (ecc_backward_saved_size > 0: the two-pass filter gradient) and
        checkpoint is False; checkpoint=True always recomputes it in backward."""

        @staticmethod
        def forward(ctx_, signal, theta, comps, ectx, checkpoint=False):
            plan = FilterPlan.from_components(ectx, comps.detach())
            sig = signal.detach().contiguous()
            th = theta.detach().contiguous()
            batch = sig.shape[0] if sig.dim() == 3 else 1
            nbytes = 0 if checkpoint else ecc_backward_saved_size(ectx, plan, batch, sig.shape[-2],
                                                                  sig.shape[-1])
            if nbytes == 0:
                y = ecc_extended(ectx, CONVOLUTION, plan, sig, th)
                saved = None
            else:
                saved = torch.empty(nbytes // 4, dtype=torch.float32, device=sig.device)
                y = ecc_extended_save(ectx, plan, sig, th, saved)
            ctx_.plan, ctx_.ectx, ctx_.saved_stack = plan, ectx, saved
            ctx_.save_for_backward(sig, th)
            return y

        @staticmethod
        def backward(ctx_, gy):
            sig, th = ctx_.saved_tensors
            gs, gc, gf = ecc_extended_backward(
                ctx_.ectx, ctx_.plan, sig, th, gy, need_signal=ctx_.needs_input_grad[0],
                need_comps=ctx_.needs_input_grad[2], need_field=ctx_.needs_input_grad[1],
                saved=ctx_.saved_stack)
            return gs, gf, gc, None, None

    return ExtConv


def _ext_corr_function():
    import torch

    class ExtCorr(torch.autograd.Function):
        """y = extended correlation of `signal` with components `comps` ((K+1, S, S)
        complex64) steered by the angle field `theta`; backward uses the hand-written
        adjoint (recomputing what it needs)."""

        @staticmethod
        def forward(ctx_, signal, theta, comps, ectx):
            plan = FilterPlan.from_components(ectx, comps.detach())
            sig = signal.detach().contiguous()
            th = theta.detach().contiguous()
            y = ecc_extended(ectx, CORRELATION, plan, sig, th)
            ctx_.plan, ctx_.ectx = plan, ectx
            ctx_.save_for_backward(sig, th)
            return y

        @staticmethod
        def backward(ctx_, gy):
            sig, th = ctx_.saved_tensors
            gs, gc, gf = ecc_extended_backward(
                ctx_.ectx, ctx_.plan, sig, th, gy, need_signal=ctx_.needs_input_grad[0],
                need_comps=ctx_.needs_input_grad[2], need_field=ctx_.needs_input_grad[1],
                op=CORRELATION)
            return gs, gf, gc, None

    return ExtCorr


class _Lazy:
    def __init__(self, make):
        self._make = make
        self._f = None

    def apply(self, *args, **kw):
        if self._f is None:
            self._f = self._make()
        return self._f.apply(*args, **kw)


ExtConv = _Lazy(_ext_conv_function)
ExtCorr = _Lazy(_ext_corr_function)


class BatchPlan:
    """ecc_batch_plan: many independent correlations (each its own image, plan and sizes)
    run as a few kernel launches captured in one HIP graph.

    instances: list of (op, FilterPlan, signal, field, out) with 2D float32 device tensors.
    The tensors and plans must stay alive while the batch plan is used."""

    def __init__(self, ctx: Context, instances, flags: int = 0):
        self.ctx = ctx
        self._keep = list(instances)
        arr = self._array(instances)
        h = C.c_void_p()
        _check(lib().ecc_batch_plan_create(ctx.h, arr, len(instances), flags, C.byref(h)))
        self.h = h
        _track(_open_batches, self)

    @staticmethod
    def _array(instances):
        arr = (Instance * max(1, len(instances)))()
        for i, (op, plan, sig, fld, out) in enumerate(instances):
            for t, name in ((sig, "signal"), (fld, "field"), (out, "out")):
                _img(t, name)
                if t.dim() != 2:
                    raise ValueError(f"{name} must be a 2D tensor")
            arr[i] = Instance(op, plan.h, sig.shape[0], sig.shape[1], sig.data_ptr(), _ld(sig),
                              fld.data_ptr(), _ld(fld), out.data_ptr(), _ld(out))
        return arr

    def update(self, instances):
        arr = self._array(instances)
        _check(lib().ecc_batch_update(self.h, arr, len(instances)))
        self._keep = list(instances)

    def execute(self, stream=None):
        _check(lib().ecc_batch_execute(self.h, _stream(stream)))

    def info(self):
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        _check(lib().ecc_batch_info(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return {"graph_instances": a.value, "launches": b.value, "blocks": c.value}

    def close(self):
        if getattr(self, "h", None):
            lib().ecc_batch_plan_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # (bound at definition: module globals are gone when the interpreter tears down)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
