"""APSM partially linear multiuser detection on MI355X (gfx950).

A thin Python binding over libapsm.so (the C ABI declared in include/apsm.h):
argument marshalling only.  Every step of training and detection runs in the
library's HIP kernels; PyTorch provides device memory and the stream.  There
is no CPU fallback: if the library is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

__all__ = ["Params", "Model", "train", "train_noalloc", "train_batched", "detect", "Batch", "BatchItem", "APSMError",
           "unrolled_loss", "APSMUnrolled", "library", "shutdown", "tune_save", "tune_load", "linear_mmse", "track", "LIB_PATH", "MOD_NONE", "MOD_QPSK",
           "MOD_QAM16", "ERR_WORKSPACE", "ERR_NONFINITE", "FLAG_TRAIN_NONFINITE", "FLAG_DETECT_NONFINITE"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libapsm.so")

MOD_NONE, MOD_QPSK, MOD_QAM16 = 0, 2, 4
ERR_INVALID_ARG, ERR_SHAPE, ERR_UNSUPPORTED, ERR_HIP, ERR_WORKSPACE, ERR_NONFINITE = 1, 2, 3, 4, 5, 6
FLAG_TRAIN_NONFINITE, FLAG_DETECT_NONFINITE = 1, 2
_MODS = {None: MOD_NONE, "none": MOD_NONE, "qpsk": MOD_QPSK, "qam16": MOD_QAM16,
         MOD_NONE: MOD_NONE, MOD_QPSK: MOD_QPSK, MOD_QAM16: MOD_QAM16}


class APSMError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = f"{where}: {library().apsm_strerror(code).decode()} (code {code})"
        if code == 4:
            msg += f": {library().apsm_last_hip_error().decode()}"
        super().__init__(msg)
        self.code = code


class _CParams(ctypes.Structure):
    _fields_ = [("sigma2", ctypes.c_float), ("eps", ctypes.c_float), ("mu", ctypes.c_float),
                ("w_lin", ctypes.c_float), ("w_gauss", ctypes.c_float),
                ("window", ctypes.c_int32), ("dict_cap", ctypes.c_int32),
                ("init", ctypes.c_int32), ("pos_weights", ctypes.POINTER(ctypes.c_float)),
                ("weights", ctypes.c_int32), ("extrapolate", ctypes.c_int32),
                ("set_types", ctypes.c_void_p)]


INIT = {"zero": 0, "linear": 1, "continue": 2}
WEIGHTS = {"position": 0, "violation": 1, "active": 2}
# Set kinds of the training samples (APSM_SET_*), as uint8 codes in a
# [P][K][2] device tensor laid out as the pilot symbols.
SET_SLAB, SET_PLANE, SET_UPPER, SET_LOWER = 0, 1, 2, 3


class _CModel(ctypes.Structure):
    _fields_ = [("M2", ctypes.c_int32), ("K", ctypes.c_int32), ("dict_cap", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("dict", ctypes.c_void_p),
                ("alpha", ctypes.c_void_p), ("w", ctypes.c_void_p), ("state", ctypes.c_void_p),
                ("packed", ctypes.c_void_p)]


class _CBatchItem(ctypes.Structure):
    _fields_ = [("model", _CModel), ("sigma2", ctypes.c_float), ("P", ctypes.c_int32),
                ("rx_pilot", ctypes.c_void_p), ("sym_pilot", ctypes.c_void_p),
                ("S", ctypes.c_int32), ("modulation", ctypes.c_int32), ("rx", ctypes.c_void_p),
                ("soft", ctypes.c_void_p), ("hard", ctypes.c_void_p), ("truth", ctypes.c_void_p),
                ("err_count", ctypes.c_void_p)]


class _CUnrolled(ctypes.Structure):
    _fields_ = [("n_inst", ctypes.c_int32), ("P", ctypes.c_int32), ("M2", ctypes.c_int32),
                ("K", ctypes.c_int32), ("S", ctypes.c_int32), ("passes", ctypes.c_int32),
                ("ckpt_every", ctypes.c_int32), ("window", ctypes.c_int32),
                ("w_lin", ctypes.c_float), ("w_gauss", ctypes.c_float)]


_lib = None


def library() -> ctypes.CDLL:
    """Load libapsm.so once (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2201_05024_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, f32 = ctypes.c_void_p, ctypes.c_int, ctypes.c_float
        L.apsm_train.argtypes = [ctypes.POINTER(_CParams), i32, i32, i32, vp, vp,
                                 ctypes.POINTER(_CModel), vp]
        L.apsm_train.restype = i32
        L.apsm_train_batched.argtypes = [ctypes.POINTER(_CParams), i32, i32, i32, i32, vp, vp,
                                         ctypes.POINTER(_CModel), vp]
        L.apsm_train_batched.restype = i32
        L.apsm_detect.argtypes = [ctypes.POINTER(_CModel), f32, i32, vp, vp, vp, i32, vp, vp, vp]
        L.apsm_detect.restype = i32
        L.apsm_get_status.argtypes = [ctypes.POINTER(_CModel), ctypes.POINTER(ctypes.c_int32)]
        L.apsm_get_status.restype = i32
        L.apsm_model_packed_bytes.argtypes = [i32, i32, i32]
        L.apsm_model_packed_bytes.restype = ctypes.c_size_t
        L.apsm_model_pack.argtypes = [ctypes.POINTER(_CModel), vp]
        L.apsm_model_pack.restype = i32
        L.apsm_batch_create.argtypes = [ctypes.POINTER(_CParams), ctypes.POINTER(_CBatchItem), i32,
                                        ctypes.POINTER(vp)]
        L.apsm_batch_create.restype = i32
        L.apsm_batch_workspace_bytes.argtypes = [vp]
        L.apsm_batch_workspace_bytes.restype = ctypes.c_size_t
        L.apsm_batch_bind.argtypes = [vp, vp, ctypes.c_size_t, vp]
        L.apsm_batch_bind.restype = i32
        L.apsm_batch_tune.argtypes = [vp, vp]
        L.apsm_batch_tune.restype = i32
        L.apsm_batch_train.argtypes = [vp, vp]
        L.apsm_batch_train.restype = i32
        L.apsm_batch_kernel_rows.argtypes = [vp, vp]
        L.apsm_batch_kernel_rows.restype = i32
        L.apsm_batch_train_prepared.argtypes = [vp, vp]
        L.apsm_batch_train_prepared.restype = i32
        L.apsm_batch_detect.argtypes = [vp, vp]
        L.apsm_batch_detect.restype = i32
        L.apsm_batch_set_form.argtypes = [vp, i32, i32]
        L.apsm_batch_set_form.restype = i32
        L.apsm_batch_destroy.argtypes = [vp]
        L.apsm_batch_destroy.restype = None
        L.apsm_unrolled_workspace_bytes.argtypes = [ctypes.POINTER(_CUnrolled)]
        L.apsm_unrolled_workspace_bytes.restype = ctypes.c_size_t
        L.apsm_unrolled_forward.argtypes = [ctypes.POINTER(_CUnrolled), vp, vp, vp, vp, vp, vp,
                                            ctypes.c_size_t, vp, vp]
        L.apsm_unrolled_forward.restype = i32
        L.apsm_unrolled_backward.argtypes = [ctypes.POINTER(_CUnrolled), vp, vp, vp, vp, vp, vp,
                                             ctypes.c_size_t, vp, vp, vp]
        L.apsm_unrolled_backward.restype = i32
        L.apsm_strerror.argtypes = [i32]
        L.apsm_strerror.restype = ctypes.c_char_p
        L.apsm_last_hip_error.argtypes = []
        L.apsm_last_hip_error.restype = ctypes.c_char_p
        L.apsm_version.argtypes = []
        L.apsm_version.restype = ctypes.c_char_p
        L.apsm_train_noalloc.argtypes = [ctypes.POINTER(_CParams), i32, i32, i32, vp, vp,
                                         ctypes.POINTER(_CModel), vp]
        L.apsm_train_noalloc.restype = i32
        L.apsm_tune_save.argtypes = [ctypes.c_char_p]
        L.apsm_tune_save.restype = i32
        L.apsm_tune_load.argtypes = [ctypes.c_char_p]
        L.apsm_tune_load.restype = i32
        L.apsm_linear_mmse.argtypes = [vp, f32, i32, i32, i32, vp, vp]
        L.apsm_linear_mmse.restype = i32
        L.apsm_track.argtypes = [ctypes.POINTER(_CParams), ctypes.POINTER(_CModel), i32, vp, i32, vp, vp, vp,
                                 vp, vp]
        L.apsm_track.restype = i32
        L.apsm_shutdown.argtypes = []
        L.apsm_shutdown.restype = None
        L.apsm_ball_workspace_bytes.argtypes = [i32, i32, i32]
        L.apsm_ball_workspace_bytes.restype = ctypes.c_size_t
        L.apsm_project_ball.argtypes = [ctypes.POINTER(_CModel), f32, f32, f32, f32, vp, ctypes.c_size_t, vp, vp]
        L.apsm_project_ball.restype = i32
        L.apsm_pocs.argtypes = [ctypes.POINTER(_CParams), i32, i32, i32, vp, vp, ctypes.POINTER(_CModel), f32,
                                i32, vp, ctypes.c_size_t, vp]
        L.apsm_pocs.restype = i32
        _lib = L
    return _lib


@dataclass
class Params:
    """Design parameters (see apsm_params_t): sigma^2, eps, relaxation mu,
    window W, sum-space weights, dictionary capacity, optional position
    weights omega (omega[0] for the newest set)."""

    sigma2: float = 0.5
    eps: float = 0.05
    mu: float = 1.0
    window: int = 16
    w_lin: float = 0.5
    w_gauss: float = 0.5
    dict_cap: int = 256
    pos_weights: Optional[Sequence[float]] = None
    init: str = "zero"               # "zero" | "linear" (f_0 = the model's w) | "continue"
    weights: str = "position"        # "position" | "violation" | "active"
    extrapolate: bool = False        # extrapolated relaxation mu * M_n
    set_types: object = None         # uint8 device tensor [P][K][2] of SET_* codes, None: hyperslabs

    def _c(self):
        pw = None
        keep = None
        if self.pos_weights is not None:
            keep = (ctypes.c_float * len(self.pos_weights))(*[float(x) for x in self.pos_weights])
            pw = ctypes.cast(keep, ctypes.POINTER(ctypes.c_float))
        st = None
        if self.set_types is not None:
            t = self.set_types
            if not (t.is_cuda and t.dtype == _torch().uint8 and t.is_contiguous() and t.shape[-1] == 2):
                raise TypeError("set_types must be a contiguous uint8 device tensor [..][P][K][2]")
            st = t.data_ptr()
        p = _CParams(self.sigma2, self.eps, self.mu, self.w_lin, self.w_gauss,
                     int(self.window), int(self.dict_cap), INIT[self.init], pw, WEIGHTS[self.weights],
                     int(bool(self.extrapolate)), st)
        return p, keep


def _torch():
    import torch
    return torch


def _stream_handle(stream) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _check(t, dtype, shape, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Model:
    """A trained detector (the whole filter state) in caller-owned tensors."""

    def __init__(self, M2: int, K: int, dict_cap: int, device=None, sigma2: float = 0.5):
        torch = _torch()
        dev = device if device is not None else torch.device("cuda")
        self.M2, self.K, self.dict_cap, self.sigma2 = int(M2), int(K), int(dict_cap), float(sigma2)
        self.dict = torch.zeros((M2, dict_cap), dtype=torch.float32, device=dev)   # component-major
        self.alpha = torch.zeros((dict_cap, K), dtype=torch.float32, device=dev)
        self.w = torch.zeros((K, M2), dtype=torch.float32, device=dev)
        self.state = torch.zeros(4, dtype=torch.int32, device=dev)
        nbytes = library().apsm_model_packed_bytes(self.M2, self.K, self.dict_cap)
        self.packed = torch.zeros(nbytes, dtype=torch.uint8, device=dev) if nbytes else None

    def _c(self) -> _CModel:
        return _CModel(self.M2, self.K, self.dict_cap, 0, self.dict.data_ptr(),
                       self.alpha.data_ptr(), self.w.data_ptr(), self.state.data_ptr(),
                       self.packed.data_ptr() if self.packed is not None else None)

    def pack(self, stream=None) -> "Model":
        """Rebuild the packed form after writing dict/alpha/w/state directly."""
        m = self._c()
        rc = library().apsm_model_pack(ctypes.byref(m), _stream_handle(stream))
        if rc:
            raise APSMError(rc, "apsm_model_pack")
        return self

    def status(self):
        """The model's state words (synchronises the device).  'flags' holds
        FLAG_TRAIN_NONFINITE / FLAG_DETECT_NONFINITE bits; their presence is
        reported here, not raised."""
        out = (ctypes.c_int32 * 4)()
        m = self._c()
        rc = library().apsm_get_status(ctypes.byref(m), out)
        if rc and rc != ERR_NONFINITE:
            raise APSMError(rc, "apsm_get_status")
        return {"size": out[0], "head": out[1], "steps": out[2], "flags": out[3]}


def tune_save(path: str) -> None:
    """Write the tuning cache (apsm_tune_save) as JSON."""
    rc = library().apsm_tune_save(os.fsencode(path))
    if rc:
        raise APSMError(rc, "apsm_tune_save")


def tune_load(path: str) -> None:
    """Merge a saved tuning cache (apsm_tune_load)."""
    rc = library().apsm_tune_load(os.fsencode(path))
    if rc:
        raise APSMError(rc, "apsm_tune_load")


def linear_mmse(h, n0: float, w=None, stream=None):
    """Linear MMSE filters from channel estimates (apsm_linear_mmse):
    h [n][K][2M] or [K][2M] float32 device tensor (column k of H as
    [Re h_k; Im h_k]) -> w of the same shape, w_k = [Re u_k; Im u_k]."""
    torch = _torch()
    squeeze = h.dim() == 2
    hh = h.unsqueeze(0) if squeeze else h
    n, K, M2 = hh.shape
    _check(hh, torch.float32, (n, K, M2), "h")
    if w is None:
        w = torch.empty_like(hh)
    else:
        w = w.view(n, K, M2)
    rc = library().apsm_linear_mmse(hh.data_ptr(), float(n0), M2, K, n, w.data_ptr(), _stream_handle(stream))
    if rc:
        raise APSMError(rc, "apsm_linear_mmse")
    return w[0] if squeeze else w


def ball_workspace(model: "Model"):
    """A device workspace for project_ball / pocs with this model's shape."""
    torch = _torch()
    n = library().apsm_ball_workspace_bytes(model.M2, model.K, model.dict_cap)
    if n == 0:
        raise APSMError(ERR_UNSUPPORTED, "apsm_ball_workspace_bytes")
    return torch.empty(n, dtype=torch.uint8, device=model.dict.device)


def project_ball(model: "Model", radius: float, params: Params, workspace=None, norms=None, stream=None):
    """Project every user's filter onto {f : ||f_k||_H <= radius}
    (apsm_project_ball, with params' sigma2, w_lin and w_gauss).  Returns the
    norms before the projection, a [K] float32 device tensor."""
    torch = _torch()
    if workspace is None:
        workspace = ball_workspace(model)
    if norms is None:
        norms = torch.empty(model.K, dtype=torch.float32, device=model.dict.device)
    _check(norms, torch.float32, (model.K,), "norms")
    m = model._c()
    rc = library().apsm_project_ball(ctypes.byref(m), float(params.sigma2), float(params.w_lin),
                                     float(params.w_gauss), float(radius), workspace.data_ptr(),
                                     workspace.numel(), norms.data_ptr(), _stream_handle(stream))
    if rc:
        raise APSMError(rc, "apsm_project_ball")
    return norms


def pocs(rx_pilot, sym_pilot, params: Params, radius: float, cycles: int, model: Optional["Model"] = None,
         workspace=None, stream=None) -> "Model":
    """Cyclic projections (apsm_pocs): `cycles` times the windowed parallel
    projections over the pilots' sets, then the projection onto the ball."""
    torch = _torch()
    P, M2 = rx_pilot.shape
    K = sym_pilot.shape[1]
    _check(rx_pilot, torch.float32, (P, M2), "rx_pilot")
    _check(sym_pilot, torch.float32, (P, K, 2), "sym_pilot")
    if params.set_types is not None:
        _check(params.set_types, torch.uint8, (P, K, 2), "set_types")
    if model is None:
        model = Model(M2, K, params.dict_cap, rx_pilot.device, params.sigma2)
    if workspace is None:
        workspace = ball_workspace(model)
    cp, keep = params._c()
    m = model._c()
    rc = library().apsm_pocs(ctypes.byref(cp), M2, K, P, rx_pilot.data_ptr(), sym_pilot.data_ptr(),
                             ctypes.byref(m), float(radius), int(cycles), workspace.data_ptr(), workspace.numel(),
                             _stream_handle(stream))
    del keep
    if rc:
        raise APSMError(rc, "apsm_pocs")
    return model


def track(model: "Model", rx, params: Params, modulation="qpsk", truth=None, decided=None, hard=None,
          errors=None, stream=None):
    """Decision-directed tracking of one block (apsm_track): detect rx
    [S][2M] with the frozen model, continue its training on the decided
    symbols.  Returns {'decided', 'hard', 'errors'} (decisions of the frozen
    model)."""
    torch = _torch()
    S = rx.shape[0]
    _check(rx, torch.float32, (S, model.M2), "rx")
    mod = _MODS[modulation]
    dev = rx.device
    if decided is None:
        decided = torch.empty((S, model.K, 2), dtype=torch.float32, device=dev)
    if truth is not None and errors is None:
        errors = torch.zeros(model.K, dtype=torch.int64, device=dev)
    p, keep = params._c()
    m = model._c()
    ptr = lambda t: t.data_ptr() if t is not None else None  # noqa: E731
    rc = library().apsm_track(ctypes.byref(p), ctypes.byref(m), S, rx.data_ptr(), mod, ptr(decided), ptr(hard),
                              ptr(truth), ptr(errors), _stream_handle(stream))
    del keep
    if rc:
        raise APSMError(rc, "apsm_track")
    return {"decided": decided, "hard": hard, "errors": errors}


def shutdown() -> None:
    """Release the library's host-side caches (apsm_shutdown)."""
    library().apsm_shutdown()


def train(rx_pilot, sym_pilot, params: Params, model: Optional[Model] = None, stream=None) -> Model:
    """rx_pilot [P][M2] float32, sym_pilot [P][K][2] float32 (device) -> Model."""
    torch = _torch()
    P, M2 = rx_pilot.shape
    K = sym_pilot.shape[1]
    _check(rx_pilot, torch.float32, (P, M2), "rx_pilot")
    _check(sym_pilot, torch.float32, (P, K, 2), "sym_pilot")
    if params.set_types is not None:
        _check(params.set_types, torch.uint8, (P, K, 2), "set_types")
    if model is None:
        model = Model(M2, K, params.dict_cap, rx_pilot.device, params.sigma2)
    model.sigma2 = float(params.sigma2)
    p, keep = params._c()
    m = model._c()
    rc = library().apsm_train(ctypes.byref(p), M2, K, P, rx_pilot.data_ptr(), sym_pilot.data_ptr(),
                              ctypes.byref(m), _stream_handle(stream))
    del keep
    if rc:
        raise APSMError(rc, "apsm_train")
    return model


def train_noalloc(rx_pilot, sym_pilot, params: Params, model: Model, stream=None) -> Model:
    """apsm_train_noalloc: training of one detector (dict_cap <= 4096) that
    allocates no device memory; `model` must be allocated by the caller."""
    torch = _torch()
    P, M2 = rx_pilot.shape
    K = sym_pilot.shape[1]
    _check(rx_pilot, torch.float32, (P, M2), "rx_pilot")
    _check(sym_pilot, torch.float32, (P, K, 2), "sym_pilot")
    model.sigma2 = float(params.sigma2)
    p, keep = params._c()
    m = model._c()
    rc = library().apsm_train_noalloc(ctypes.byref(p), M2, K, P, rx_pilot.data_ptr(), sym_pilot.data_ptr(),
                                      ctypes.byref(m), _stream_handle(stream))
    del keep
    if rc:
        raise APSMError(rc, "apsm_train_noalloc")
    return model


def train_batched(rx_pilot, sym_pilot, params: Params, models=None, stream=None):
    """rx_pilot [n][P][M2], sym_pilot [n][P][K][2] float32 (device) -> list of n
    Models, trained concurrently in one launch."""
    torch = _torch()
    n, P, M2 = rx_pilot.shape
    K = sym_pilot.shape[2]
    _check(rx_pilot, torch.float32, (n, P, M2), "rx_pilot")
    _check(sym_pilot, torch.float32, (n, P, K, 2), "sym_pilot")
    if params.set_types is not None:
        _check(params.set_types, torch.uint8, (n, P, K, 2), "set_types")
    if models is None:
        models = [Model(M2, K, params.dict_cap, rx_pilot.device, params.sigma2) for _ in range(n)]
    if len(models) != n:
        raise ValueError("need one model per instance")
    for m in models:
        m.sigma2 = float(params.sigma2)
    p, keep = params._c()
    arr = (_CModel * n)(*[m._c() for m in models]) if n else None
    rc = library().apsm_train_batched(ctypes.byref(p), M2, K, P, n, rx_pilot.data_ptr(),
                                      sym_pilot.data_ptr(), arr, _stream_handle(stream))
    del keep
    if rc:
        raise APSMError(rc, "apsm_train_batched")
    return models


def detect(model: Model, rx, modulation="qpsk", truth=None, want_soft: bool = True,
           want_hard: bool = True, sigma2: Optional[float] = None, soft=None, hard=None,
           errors=None, stream=None):
    """Evaluate the frozen filter on rx [S][M2] float32.  Returns a dict with
    'soft' [S][K][2] float32, 'hard' [S][K] uint8 and 'errors' [K] int64 (each
    present when requested).  Output tensors may be passed in to reuse them;
    `errors` is accumulated into, as the C ABI specifies."""
    torch = _torch()
    S = rx.shape[0]
    _check(rx, torch.float32, (S, model.M2), "rx")
    mod = _MODS[modulation]
    dev = rx.device
    if want_soft and soft is None:
        soft = torch.empty((S, model.K, 2), dtype=torch.float32, device=dev)
    if mod != MOD_NONE and want_hard and hard is None:
        hard = torch.empty((S, model.K), dtype=torch.uint8, device=dev)
    if truth is not None:
        _check(truth, torch.uint8, (S, model.K), "truth")
        if errors is None:
            errors = torch.zeros(model.K, dtype=torch.int64, device=dev)
    if soft is not None:
        _check(soft, torch.float32, (S, model.K, 2), "soft")
    if hard is not None:
        _check(hard, torch.uint8, (S, model.K), "hard")
    if errors is not None:
        _check(errors, torch.int64, (model.K,), "errors")
    m = model._c()
    ptr = lambda t: t.data_ptr() if t is not None else None  # noqa: E731
    rc = library().apsm_detect(ctypes.byref(m), float(sigma2 if sigma2 is not None else model.sigma2),
                               S, rx.data_ptr(), ptr(soft), ptr(hard), mod, ptr(truth),
                               ptr(errors), _stream_handle(stream))
    if rc:
        raise APSMError(rc, "apsm_detect")
    return {"soft": soft, "hard": hard, "errors": errors}


@dataclass
class BatchItem:
    """One detector of a Batch: its model, pilots, and (optionally) received
    vectors to detect with their outputs.  Tensors are device tensors as for
    train() and detect()."""

    model: Model
    rx_pilot: object
    sym_pilot: object
    rx: object = None
    modulation: object = "qpsk"
    soft: object = None
    hard: object = None
    truth: object = None
    errors: object = None
    sigma2: Optional[float] = None


class Batch:
    """Detectors of different shapes trained in one launch and detected in one
    launch (apsm_batch_* of the C ABI).  The workspace is a uint8 device tensor
    owned by this object; every tensor named by the items is kept alive."""

    def __init__(self, params: Params, items: Sequence[BatchItem], stream=None):
        torch = _torch()
        if not items:
            raise ValueError("a batch needs at least one item")
        self.items = list(items)
        arr = (_CBatchItem * len(items))()
        ptr = lambda t: t.data_ptr() if t is not None else None  # noqa: E731
        for c, it in zip(arr, self.items):
            m = it.model
            P = it.rx_pilot.shape[0]
            _check(it.rx_pilot, torch.float32, (P, m.M2), "rx_pilot")
            _check(it.sym_pilot, torch.float32, (P, m.K, 2), "sym_pilot")
            S = 0 if it.rx is None else it.rx.shape[0]
            if it.rx is not None:
                _check(it.rx, torch.float32, (S, m.M2), "rx")
            if it.soft is not None:
                _check(it.soft, torch.float32, (S, m.K, 2), "soft")
            if it.hard is not None:
                _check(it.hard, torch.uint8, (S, m.K), "hard")
            if it.truth is not None:
                _check(it.truth, torch.uint8, (S, m.K), "truth")
            if it.errors is not None:
                _check(it.errors, torch.int64, (m.K,), "errors")
            sig = float(it.sigma2 if it.sigma2 is not None else params.sigma2)
            m.sigma2 = sig
            c.model = m._c()
            c.sigma2 = sig
            c.P = P
            c.rx_pilot = ptr(it.rx_pilot)
            c.sym_pilot = ptr(it.sym_pilot)
            c.S = S
            c.modulation = _MODS[it.modulation]
            c.rx = ptr(it.rx)
            c.soft = ptr(it.soft)
            c.hard = ptr(it.hard)
            c.truth = ptr(it.truth)
            c.err_count = ptr(it.errors)
        p, keep = params._c()
        h = ctypes.c_void_p()
        rc = library().apsm_batch_create(ctypes.byref(p), arr, len(items), ctypes.byref(h))
        del keep
        if rc:
            raise APSMError(rc, "apsm_batch_create")
        self._h = h
        nbytes = library().apsm_batch_workspace_bytes(h)
        dev = self.items[0].rx_pilot.device
        # apsm_batch_bind writes the tables (counters included); the kernel
        # rows after them are computed on the device, so no clearing is needed
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        off = (-self.workspace.data_ptr()) % 256
        self._ws_ptr = self.workspace.data_ptr() + off
        rc = library().apsm_batch_bind(h, self._ws_ptr, nbytes, _stream_handle(stream))
        if rc:
            raise APSMError(rc, "apsm_batch_bind")

    def tune(self, stream=None) -> "Batch":
        rc = library().apsm_batch_tune(self._h, _stream_handle(stream))
        if rc:
            raise APSMError(rc, "apsm_batch_tune")
        return self

    def set_form(self, persistent: bool, cus: int = 0) -> "Batch":
        """Persistent (claiming, on `cus` CUs; 0 = all) or
        one-workgroup-per-item detection launches."""
        rc = library().apsm_batch_set_form(self._h, int(bool(persistent)), int(cus))
        if rc:
            raise APSMError(rc, "apsm_batch_set_form")
        return self

    def train(self, stream=None) -> "Batch":
        rc = library().apsm_batch_train(self._h, _stream_handle(stream))
        if rc:
            raise APSMError(rc, "apsm_batch_train")
        return self

    def kernel_rows(self, stream=None) -> "Batch":
        """First part of train(): the kernel rows of the pilots (whole GPU)."""
        rc = library().apsm_batch_kernel_rows(self._h, _stream_handle(stream))
        if rc:
            raise APSMError(rc, "apsm_batch_kernel_rows")
        return self

    def train_prepared(self, stream=None) -> "Batch":
        """Second part of train(), ordered after kernel_rows() by the caller."""
        rc = library().apsm_batch_train_prepared(self._h, _stream_handle(stream))
        if rc:
            raise APSMError(rc, "apsm_batch_train_prepared")
        return self

    def detect(self, stream=None) -> "Batch":
        rc = library().apsm_batch_detect(self._h, _stream_handle(stream))
        if rc:
            raise APSMError(rc, "apsm_batch_detect")
        return self

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            library().apsm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # pragma: no cover - interpreter shutdown
            pass


def _autograd_function():
    torch = _torch()

    class APSMUnrolledFn(torch.autograd.Function):
        """L(theta) of unrolled APSM training (apsm_unrolled_forward) with the
        library's hand-written adjoint as its backward (apsm_unrolled_backward)."""

        @staticmethod
        def forward(ctx, theta, rx_pilot, sym_pilot, rx_val, sym_val, passes, ckpt_every, w_lin, w_gauss):
            n, P, M2 = rx_pilot.shape
            K = sym_pilot.shape[2]
            S = rx_val.shape[1]
            W = theta.shape[0] - 3
            _check(theta, torch.float32, (3 + W,), "theta")
            _check(rx_pilot, torch.float32, (n, P, M2), "rx_pilot")
            _check(sym_pilot, torch.float32, (n, P, K, 2), "sym_pilot")
            _check(rx_val, torch.float32, (n, S, M2), "rx_val")
            _check(sym_val, torch.float32, (n, S, K, 2), "sym_val")
            u = _CUnrolled(n, P, M2, K, S, int(passes), int(ckpt_every), W, float(w_lin), float(w_gauss))
            nbytes = library().apsm_unrolled_workspace_bytes(ctypes.byref(u))
            if nbytes == 0:
                raise APSMError(1, "apsm_unrolled_workspace_bytes")
            ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=theta.device)
            ws_ptr = ws.data_ptr() + (-ws.data_ptr()) % 256
            loss = torch.empty(1, dtype=torch.float32, device=theta.device)
            args = (theta.data_ptr(), rx_pilot.data_ptr(), sym_pilot.data_ptr(), rx_val.data_ptr(),
                    sym_val.data_ptr(), ws_ptr, nbytes)
            rc = library().apsm_unrolled_forward(ctypes.byref(u), *args, loss.data_ptr(), _stream_handle(None))
            if rc:
                raise APSMError(rc, "apsm_unrolled_forward")
            ctx.keep = (u, args, ws, theta, rx_pilot, sym_pilot, rx_val, sym_val)
            return loss.reshape(())

        @staticmethod
        def backward(ctx, g_loss):
            u, args, ws, theta = ctx.keep[:4]
            up = g_loss.reshape(1).to(torch.float32).contiguous()
            grad = torch.empty_like(theta)
            rc = library().apsm_unrolled_backward(ctypes.byref(u), *args, up.data_ptr(), grad.data_ptr(),
                                                  _stream_handle(None))
            if rc:
                raise APSMError(rc, "apsm_unrolled_backward")
            return grad, None, None, None, None, None, None, None, None

    return APSMUnrolledFn


_APSM_UNROLLED = None


def APSMUnrolled():
    """The torch.autograd.Function class (created on first use)."""
    global _APSM_UNROLLED
    if _APSM_UNROLLED is None:
        _APSM_UNROLLED = _autograd_function()
    return _APSM_UNROLLED


def unrolled_loss(theta, rx_pilot, sym_pilot, rx_val, sym_val, passes: int, ckpt_every: int = 5,
                  w_lin: float = 0.5, w_gauss: float = 0.5):
    """Differentiable L(theta), theta = [sigma, eps, mu, omega_0..omega_{W-1}]
    (float32 device tensor); inputs [n][P][M2], [n][P][K][2], [n][S][M2],
    [n][S][K][2] float32 device tensors.  loss.backward() runs the library's
    adjoint."""
    return APSMUnrolled().apply(theta, rx_pilot, sym_pilot, rx_val, sym_val, passes, ckpt_every, w_lin,
                                w_gauss)
