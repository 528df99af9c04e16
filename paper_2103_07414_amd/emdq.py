"""Thin ctypes binding of libemdq.so (C-ABI in include/emdq.h).

Argument marshalling only: every step of the EMDQ path runs in the library's
HIP kernels.  Device buffers are torch CUDA tensors (PyTorch is used for
device memory and streams); their data pointers and the current stream are
handed to the C functions of the same names.  There is no CPU fallback: if
the library is missing, importing the functions fails loudly.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libemdq.so")

OK, WARN_NOT_CONVERGED, EINVAL, ETOOFEW, ENOINLIERS, ENONFINITE, EHIP, ENOMEM = \
    0, 1, -1, -2, -3, -4, -5, -6

# every function declared in include/emdq.h
EXPORTS = ("emdq_params_default", "emdq_alpha", "emdq_model_create", "emdq_model_free",
           "emdq_fit", "emdq_model_set_nodes", "emdq_field", "emdq_warp",
           "emdq_uncertainty", "emdq_track_nodes", "emdq_model_set_precision",
           "emdq_model_status", "emdq_model_results", "emdq_status_string",
           "emdq_batch_create", "emdq_batch_free", "emdq_batch_fit", "emdq_batch_field",
           "emdq_batch_warp", "emdq_fit_from", "emdq_learned_start",
           "emdq_batch_learned_start", "emdq_start_features", "emdq_start_train_work_floats",
           "emdq_start_train_step", "emdq_batch_autotune", "emdq_batch_set_variant",
           "emdq_batch_prepare", "emdq_batch_launch", "emdq_batch_prepare_step",
           "emdq_batch_launch_step", "emdq_fit_warp_static")

STATIC_MAX_N = 8192   # EMDQ_STATIC_MAX_N

START_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "start_mlp.npy")
N_START_WEIGHTS = 24961

PREC_F32, PREC_F16, PREC_BF16 = 0, 1, 2
PRECISIONS = {"f32": PREC_F32, "f16": PREC_F16, "bf16": PREC_BF16}


class Params(C.Structure):
    """emdq_params."""
    _fields_ = [("alpha0", C.c_float), ("ref_w", C.c_int), ("ref_h", C.c_int),
                ("max_iter", C.c_int), ("p_thresh", C.c_float), ("gamma_min", C.c_float),
                ("gamma_max", C.c_float), ("sigma2_min", C.c_float), ("flags", C.c_uint)]


class Region(C.Structure):
    """emdq_region."""
    _fields_ = [("zx0", C.c_int), ("zy0", C.c_int), ("w", C.c_int), ("h", C.c_int),
                ("out_xy", C.c_void_p), ("frame_rgb", C.c_void_p), ("fw", C.c_int),
                ("fh", C.c_int), ("frame_pitch_bytes", C.c_int), ("canvas", C.c_void_p),
                ("cw", C.c_int), ("ch", C.c_int), ("canvas_pitch_px", C.c_int),
                ("ox", C.c_int), ("oy", C.c_int)]


class EmdqError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {status_string(status)} ({status})")
        self.status = status


_lib = None

# Models and batches still open.  They are released by an exit handler,
# which runs before the interpreter (and torch, and the HIP runtime after it)
# starts tearing down; a release that would only happen during that teardown
# is skipped instead (the process is ending and the driver reclaims the
# memory), so no HIP call runs after the runtime has begun to shut down.
_open = weakref.WeakSet()


def _close_open():
    for obj in list(_open):
        try:
            obj.close()
        except Exception:
            pass


def _release(obj, _finalizing=sys.is_finalizing):
    """__del__ of Model and Batch: release unless the interpreter is
    already finalising.  (What it needs is bound when it is defined: during
    the interpreter's teardown this module's globals may already be None.)"""
    if _finalizing():
        return
    try:
        obj.close()
    except Exception:
        pass


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libemdq.so not found at {LIB_PATH}; build it with "
                               "__graft_entry__.build() (there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        I, F, P, U8P = C.c_int, C.c_float, C.c_void_p, C.c_void_p
        L.emdq_params_default.argtypes = [C.POINTER(Params)]
        L.emdq_params_default.restype = None
        L.emdq_alpha.argtypes = [C.POINTER(Params), I, I]
        L.emdq_alpha.restype = F
        L.emdq_model_create.argtypes = [I, C.POINTER(P)]
        L.emdq_model_create.restype = I
        L.emdq_model_free.argtypes = [P]
        L.emdq_model_free.restype = None
        L.emdq_fit.argtypes = [P, P, P, I, I, I, C.POINTER(Params), P]
        L.emdq_fit.restype = I
        L.emdq_fit_from.argtypes = [P, P, P, I, I, I, C.POINTER(Params), P, P]
        L.emdq_fit_from.restype = I
        L.emdq_learned_start.argtypes = [P, P, I, I, I, C.POINTER(Params), P, P, P]
        L.emdq_learned_start.restype = I
        L.emdq_start_features.argtypes = [P, P, I, I, I, C.POINTER(Params), P, P]
        L.emdq_start_features.restype = I
        L.emdq_start_train_work_floats.argtypes = [I]
        L.emdq_start_train_work_floats.restype = C.c_size_t
        L.emdq_start_train_step.argtypes = [P, P, P, I, P, P, I, P, I, F, I, P, P]
        L.emdq_start_train_step.restype = I
        L.emdq_model_set_nodes.argtypes = [P, P, P, P, P, I, F, P]
        L.emdq_model_set_nodes.restype = I
        L.emdq_field.argtypes = [P, I, I, I, I, P, P]
        L.emdq_field.restype = I
        L.emdq_warp.argtypes = [P, U8P, I, I, I, P, I, I, I, I, I, I, I, I, I, P]
        L.emdq_warp.restype = I
        L.emdq_uncertainty.argtypes = [P, F, I, I, I, I, P, P]
        L.emdq_uncertainty.restype = I
        L.emdq_track_nodes.argtypes = [P, F, I, P, P, P, P, P]
        L.emdq_track_nodes.restype = I
        L.emdq_model_set_precision.argtypes = [P, I]
        L.emdq_model_set_precision.restype = I
        L.emdq_model_status.argtypes = [P, P]
        L.emdq_model_status.restype = I
        L.emdq_model_results.argtypes = [P, P, P, P, P, C.POINTER(I), C.POINTER(I),
                                         C.POINTER(F), C.POINTER(F), P]
        L.emdq_model_results.restype = I
        L.emdq_batch_create.argtypes = [I, C.POINTER(P)]
        L.emdq_batch_create.restype = I
        L.emdq_batch_free.argtypes = [P]
        L.emdq_batch_free.restype = None
        PP = C.POINTER(C.c_void_p)
        IP = C.POINTER(C.c_int)
        L.emdq_batch_fit.argtypes = [P, I, PP, PP, PP, IP, IP, IP, PP, C.POINTER(Params), P]
        L.emdq_batch_learned_start.argtypes = [P, I, PP, PP, IP, IP, IP, C.POINTER(Params), P,
                                               PP, P]
        L.emdq_batch_learned_start.restype = I
        L.emdq_batch_fit.restype = I
        L.emdq_batch_field.argtypes = [P, I, PP, C.POINTER(Region), P]
        L.emdq_batch_field.restype = I
        L.emdq_batch_warp.argtypes = [P, I, PP, C.POINTER(Region), P]
        L.emdq_batch_warp.restype = I
        L.emdq_batch_autotune.argtypes = [P, I, PP, C.POINTER(Region), C.c_char_p,
                                          C.POINTER(I), P]
        L.emdq_batch_autotune.restype = I
        L.emdq_batch_set_variant.argtypes = [P, I]
        L.emdq_batch_set_variant.restype = I
        L.emdq_batch_prepare.argtypes = [P, I, I, PP, C.POINTER(Region)]
        L.emdq_batch_prepare.restype = I
        L.emdq_batch_launch.argtypes = [P, P]
        L.emdq_batch_launch.restype = I
        L.emdq_batch_prepare_step.argtypes = [P, I, PP, PP, PP, IP, IP, IP, C.POINTER(Params),
                                              P, PP, C.POINTER(Region)]
        L.emdq_batch_prepare_step.restype = I
        L.emdq_batch_launch_step.argtypes = [P, P]
        L.emdq_batch_launch_step.restype = I
        L.emdq_fit_warp_static.argtypes = [P, P, I, C.POINTER(Params), U8P, I, I, I, P, I, I,
                                           I, I, I, I, I, I, I, P, P]
        L.emdq_fit_warp_static.restype = I
        L.emdq_status_string.argtypes = [I]
        L.emdq_status_string.restype = C.c_char_p
        _lib = L
        atexit.register(_close_open)
    return _lib


def status_string(status: int) -> str:
    return lib().emdq_status_string(int(status)).decode()


def _check(status: int, where: str, allow_warn: bool = True) -> int:
    if status < 0 or (status > 0 and not allow_warn):
        raise EmdqError(status, where)
    return status


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dev(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def emdq_params_default() -> Params:
    p = Params()
    lib().emdq_params_default(C.byref(p))
    return p


def emdq_alpha(params: Params | None, frame_w: int, frame_h: int) -> float:
    return lib().emdq_alpha(C.byref(params) if params is not None else None, frame_w, frame_h)


def emdq_model_create(n_max: int) -> int:
    h = C.c_void_p()
    _check(lib().emdq_model_create(int(n_max), C.byref(h)), "emdq_model_create")
    return h.value


def emdq_model_free(model: int) -> None:
    lib().emdq_model_free(model)


def emdq_fit(model: int, src, dst, frame_w: int, frame_h: int, params: Params | None = None,
             stream=None) -> int:
    """src, dst: CUDA float32 [N, 2].  Returns the enqueue status."""
    import torch
    if src.shape != dst.shape or src.dim() != 2 or src.shape[1] != 2:
        raise ValueError("src and dst must both be [N, 2]")
    ps = _dev(src, torch.float32, "src")
    pd = _dev(dst, torch.float32, "dst")
    return _check(lib().emdq_fit(model, ps, pd, int(src.shape[0]), int(frame_w), int(frame_h),
                                 C.byref(params) if params is not None else None,
                                 _stream(stream)), "emdq_fit")


def emdq_fit_from(model: int, src, dst, frame_w: int, frame_h: int, init_p,
                  params: Params | None = None, stream=None) -> int:
    """As emdq_fit, starting from init_p (CUDA float32 [N])."""
    import torch
    if src.shape != dst.shape or src.dim() != 2 or src.shape[1] != 2:
        raise ValueError("src and dst must both be [N, 2]")
    if tuple(init_p.shape) != (src.shape[0],):
        raise ValueError("init_p must be [N]")
    ps = _dev(src, torch.float32, "src")
    pd = _dev(dst, torch.float32, "dst")
    pp = _dev(init_p, torch.float32, "init_p")
    return _check(lib().emdq_fit_from(model, ps, pd, int(src.shape[0]), int(frame_w),
                                      int(frame_h), C.byref(params) if params is not None
                                      else None, pp, _stream(stream)), "emdq_fit_from")


def load_start_weights(device="cuda", path=None):
    """The trained weights of the learned EM start as a CUDA float32 tensor."""
    import numpy as np
    import torch
    w = np.load(path or START_WEIGHTS, allow_pickle=False).astype(np.float32)
    if w.shape != (N_START_WEIGHTS,):
        raise ValueError(f"expected {N_START_WEIGHTS} weights, got {w.shape}")
    return torch.from_numpy(w).to(device)


def emdq_learned_start(src, dst, frame_w: int, frame_h: int, weights, out,
                       params: Params | None = None, stream=None) -> int:
    """Learned starting posteriors: src, dst CUDA float32 [N, 2]; weights
    CUDA float32 [24961]; out CUDA float32 [N]."""
    import torch
    if src.shape != dst.shape or src.dim() != 2 or src.shape[1] != 2:
        raise ValueError("src and dst must both be [N, 2]")
    if tuple(out.shape) != (src.shape[0],) or tuple(weights.shape) != (N_START_WEIGHTS,):
        raise ValueError("out must be [N] and weights [24961]")
    return _check(lib().emdq_learned_start(
        _dev(src, torch.float32, "src"), _dev(dst, torch.float32, "dst"), int(src.shape[0]),
        int(frame_w), int(frame_h), C.byref(params) if params is not None else None,
        _dev(weights, torch.float32, "weights"), _dev(out, torch.float32, "out"),
        _stream(stream)), "emdq_learned_start")


def emdq_start_features(src, dst, frame_w: int, frame_h: int, out, params: Params | None = None,
                        stream=None) -> int:
    """The learned start's features: src, dst CUDA float32 [N, 2]; out
    CUDA float32 [N, 64]."""
    import torch
    if src.shape != dst.shape or src.dim() != 2 or src.shape[1] != 2:
        raise ValueError("src and dst must both be [N, 2]")
    if tuple(out.shape) != (src.shape[0], 64):
        raise ValueError("out must be [N, 64]")
    return _check(lib().emdq_start_features(
        _dev(src, torch.float32, "src"), _dev(dst, torch.float32, "dst"), int(src.shape[0]),
        int(frame_w), int(frame_h), C.byref(params) if params is not None else None,
        _dev(out, torch.float32, "out"), _stream(stream)), "emdq_start_features")


def emdq_start_train_work_floats(groups: int) -> int:
    return int(lib().emdq_start_train_work_floats(int(groups)))


def emdq_start_train_step(weights, adam_m, adam_v, step: int, feat, label, idx, lr: float,
                          groups: int, work, stream=None) -> int:
    """One Adam step on the learned start (all CUDA tensors): weights, adam_m,
    adam_v float32 [24961]; feat float32 [M, 64]; label float32 [M]; idx int32
    [B]; work float32 [emdq_start_train_work_floats(groups)]."""
    import torch
    for t, name in ((weights, "weights"), (adam_m, "adam_m"), (adam_v, "adam_v")):
        if tuple(t.shape) != (N_START_WEIGHTS,):
            raise ValueError(f"{name} must be [24961]")
    m = int(feat.shape[0])
    if tuple(feat.shape) != (m, 64) or tuple(label.shape) != (m,):
        raise ValueError("feat must be [M, 64] and label [M]")
    if work.numel() < emdq_start_train_work_floats(min(groups, int(idx.shape[0]))):
        raise ValueError("work is too small")
    return _check(lib().emdq_start_train_step(
        _dev(weights, torch.float32, "weights"), _dev(adam_m, torch.float32, "adam_m"),
        _dev(adam_v, torch.float32, "adam_v"), int(step), _dev(feat, torch.float32, "feat"),
        _dev(label, torch.float32, "label"), m, _dev(idx, torch.int32, "idx"),
        int(idx.shape[0]), float(lr), int(groups), _dev(work, torch.float32, "work"),
        _stream(stream)), "emdq_start_train_step")


def emdq_model_set_nodes(model: int, x_xy, scale, q, mask, alpha: float, stream=None) -> int:
    """Host (numpy) arrays: x_xy [N, 2], scale [N], q [N, 4] float32, mask [N] uint8."""
    import numpy as np
    x = np.ascontiguousarray(x_xy, dtype=np.float32)
    s = np.ascontiguousarray(scale, dtype=np.float32)
    qq = np.ascontiguousarray(q, dtype=np.float32)
    n = x.shape[0]
    if x.shape != (n, 2) or s.shape != (n,) or qq.shape != (n, 4):
        raise ValueError("shapes must be x [N,2], scale [N], q [N,4]")
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    if m is not None and m.shape != (n,):
        raise ValueError("mask must be [N]")
    return _check(lib().emdq_model_set_nodes(
        model, x.ctypes.data, s.ctypes.data, qq.ctypes.data,
        None if m is None else m.ctypes.data, n, float(alpha), _stream(stream)),
        "emdq_model_set_nodes")


def emdq_field(model: int, zx0: int, zy0: int, w: int, h: int, out, stream=None) -> int:
    """out: CUDA float32 [h, w, 2]."""
    import torch
    if tuple(out.shape) != (h, w, 2):
        raise ValueError("out must be [h, w, 2]")
    po = _dev(out, torch.float32, "out")
    return _check(lib().emdq_field(model, zx0, zy0, w, h, po, _stream(stream)), "emdq_field")


def emdq_warp(model: int, frame, canvas, ox: int, oy: int, zx0: int, zy0: int, w: int, h: int,
              stream=None) -> int:
    """frame: CUDA uint8 [fh, fw, 3]; canvas: CUDA float32 [ch, cw, 4] (updated)."""
    import torch
    if frame.dim() != 3 or frame.shape[2] != 3:
        raise ValueError("frame must be [fh, fw, 3]")
    if canvas.dim() != 3 or canvas.shape[2] != 4:
        raise ValueError("canvas must be [ch, cw, 4]")
    pf = _dev(frame, torch.uint8, "frame")
    pc = _dev(canvas, torch.float32, "canvas")
    fh, fw = int(frame.shape[0]), int(frame.shape[1])
    ch, cw = int(canvas.shape[0]), int(canvas.shape[1])
    return _check(lib().emdq_warp(model, pf, fw, fh, 3 * fw, pc, cw, ch, cw, ox, oy, zx0, zy0,
                                  w, h, _stream(stream)), "emdq_warp")


def emdq_fit_warp_static(src, dst, frame, canvas, ox: int, oy: int, zx0: int, zy0: int, w: int,
                         h: int, info, params: Params | None = None, stream=None) -> int:
    """Allocation-free fit + warp: src, dst CUDA float32 [N, 2]; frame CUDA
    uint8 [fh, fw, 3]; canvas CUDA float32 [ch, cw, 4] (updated); info CUDA
    int32 [3] (status, EM iterations, inliers, written on the stream)."""
    import torch
    if src.shape != dst.shape or src.dim() != 2 or src.shape[1] != 2:
        raise ValueError("src and dst must both be [N, 2]")
    if frame.dim() != 3 or frame.shape[2] != 3:
        raise ValueError("frame must be [fh, fw, 3]")
    if canvas.dim() != 3 or canvas.shape[2] != 4:
        raise ValueError("canvas must be [ch, cw, 4]")
    if tuple(info.shape) != (3,):
        raise ValueError("info must be [3]")
    fh, fw = int(frame.shape[0]), int(frame.shape[1])
    ch, cw = int(canvas.shape[0]), int(canvas.shape[1])
    return _check(lib().emdq_fit_warp_static(
        _dev(src, torch.float32, "src"), _dev(dst, torch.float32, "dst"), int(src.shape[0]),
        C.byref(params) if params is not None else None, _dev(frame, torch.uint8, "frame"),
        fw, fh, 3 * fw, _dev(canvas, torch.float32, "canvas"), cw, ch, cw, int(ox), int(oy),
        int(zx0), int(zy0), int(w), int(h), _dev(info, torch.int32, "info"), _stream(stream)),
        "emdq_fit_warp_static")


def emdq_uncertainty(model: int, beta: float, zx0: int, zy0: int, w: int, h: int, out,
                     stream=None) -> int:
    """out: CUDA float32 [h, w]."""
    import torch
    if tuple(out.shape) != (h, w):
        raise ValueError("out must be [h, w]")
    po = _dev(out, torch.float32, "out")
    return _check(lib().emdq_uncertainty(model, float(beta), zx0, zy0, w, h, po,
                                         _stream(stream)), "emdq_uncertainty")


def emdq_track_nodes(model: int, beta: float, pos, scale, q, sigma2, stream=None) -> int:
    """CUDA float32 tensors, updated in place: pos [n, 2], scale [n], q [n, 4],
    sigma2 [n]."""
    import torch
    n = int(scale.shape[0]) if scale.dim() == 1 else -1
    if n < 0 or tuple(pos.shape) != (n, 2) or tuple(q.shape) != (n, 4) or \
            tuple(sigma2.shape) != (n,):
        raise ValueError("shapes must be pos [n,2], scale [n], q [n,4], sigma2 [n]")
    args = [_dev(t, torch.float32, name) for t, name in
            ((pos, "pos"), (scale, "scale"), (q, "q"), (sigma2, "sigma2"))]
    return _check(lib().emdq_track_nodes(model, float(beta), n, *args, _stream(stream)),
                  "emdq_track_nodes")


def emdq_model_set_precision(model: int, precision) -> int:
    """precision: PREC_F32 / PREC_F16 / PREC_BF16 or "f32" / "f16" / "bf16"."""
    if isinstance(precision, str):
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        precision = PRECISIONS[precision]
    return _check(lib().emdq_model_set_precision(model, int(precision)),
                  "emdq_model_set_precision")


def emdq_model_status(model: int, stream=None) -> int:
    return lib().emdq_model_status(model, _stream(stream))


def emdq_model_results(model: int, n: int, stream=None) -> dict:
    """Copies the fit to numpy arrays (waits for the stream)."""
    import numpy as np
    scale = np.zeros(n, np.float32)
    q = np.zeros((n, 4), np.float32)
    p = np.zeros(n, np.float32)
    mask = np.zeros(n, np.uint8)
    n_in, iters = C.c_int(), C.c_int()
    s2, g = C.c_float(), C.c_float()
    st = lib().emdq_model_results(model, scale.ctypes.data, q.ctypes.data, p.ctypes.data,
                                  mask.ctypes.data, C.byref(n_in), C.byref(iters), C.byref(s2),
                                  C.byref(g), _stream(stream))
    return dict(status=st, scale=scale, q=q, p=p, mask=mask, n_in=n_in.value,
                iters=iters.value, sigma2=s2.value, gamma=g.value)


class Model:
    """Owns an emdq_model handle."""

    def __init__(self, n_max: int):
        self.handle = emdq_model_create(n_max)
        self.n = 0
        _open.add(self)

    def fit(self, src, dst, frame_w, frame_h, params=None, stream=None):
        self.n = int(src.shape[0])
        return emdq_fit(self.handle, src, dst, frame_w, frame_h, params, stream)

    def fit_from(self, src, dst, frame_w, frame_h, init_p, params=None, stream=None):
        self.n = int(src.shape[0])
        return emdq_fit_from(self.handle, src, dst, frame_w, frame_h, init_p, params, stream)

    def set_nodes(self, x_xy, scale, q, mask, alpha, stream=None):
        self.n = int(len(scale))
        return emdq_model_set_nodes(self.handle, x_xy, scale, q, mask, alpha, stream)

    def field(self, zx0, zy0, w, h, out, stream=None):
        return emdq_field(self.handle, zx0, zy0, w, h, out, stream)

    def warp(self, frame, canvas, ox, oy, zx0, zy0, w, h, stream=None):
        return emdq_warp(self.handle, frame, canvas, ox, oy, zx0, zy0, w, h, stream)

    def uncertainty(self, beta, zx0, zy0, w, h, out, stream=None):
        return emdq_uncertainty(self.handle, beta, zx0, zy0, w, h, out, stream)

    def track_nodes(self, beta, pos, scale, q, sigma2, stream=None):
        return emdq_track_nodes(self.handle, beta, pos, scale, q, sigma2, stream)

    def set_precision(self, precision):
        return emdq_model_set_precision(self.handle, precision)

    def status(self, stream=None):
        return emdq_model_status(self.handle, stream)

    def results(self, stream=None):
        return emdq_model_results(self.handle, self.n, stream)

    def close(self):
        if self.handle:
            emdq_model_free(self.handle)
            self.handle = None
        _open.discard(self)

    def __del__(self, _rel=_release):
        _rel(self)


class Batch:
    """Owns an emdq_batch handle: many pairs, one launch per phase."""

    def __init__(self, max_pairs: int):
        h = C.c_void_p()
        _check(lib().emdq_batch_create(int(max_pairs), C.byref(h)), "emdq_batch_create")
        self.handle = h.value
        self.max_pairs = int(max_pairs)
        _open.add(self)

    @staticmethod
    def _handles(models):
        return (C.c_void_p * len(models))(*[m.handle for m in models])

    @staticmethod
    def _pairs(models, srcs, dsts, sizes):
        """The per-pair match arrays and frame sizes of fit / prepare_step as
        C arrays: src, dst pointers, n, frame_w, frame_h."""
        import torch
        k = len(models)
        if not (len(srcs) == len(dsts) == len(sizes) == k):
            raise ValueError("models, srcs, dsts and sizes must have the same length")
        ps, pd, ns = [], [], []
        for m, a, b in zip(models, srcs, dsts):
            if a.shape != b.shape or a.dim() != 2 or a.shape[1] != 2:
                raise ValueError("src and dst must both be [N, 2]")
            ps.append(_dev(a, torch.float32, "src"))
            pd.append(_dev(b, torch.float32, "dst"))
            ns.append(int(a.shape[0]))
            m.n = int(a.shape[0])
        arr = lambda v, t: (t * k)(*v)
        return (arr(ps, C.c_void_p), arr(pd, C.c_void_p), arr(ns, C.c_int),
                arr([w for w, _ in sizes], C.c_int), arr([h for _, h in sizes], C.c_int))

    def learned_start(self, srcs, dsts, sizes, weights, outs, params=None, stream=None):
        """Learned starting posteriors of every pair in one launch: outs are
        CUDA float32 [N_i]; weights as load_start_weights()."""
        import torch
        k = len(srcs)
        if not (len(dsts) == len(sizes) == len(outs) == k):
            raise ValueError("srcs, dsts, sizes and outs must have the same length")
        if tuple(weights.shape) != (N_START_WEIGHTS,):
            raise ValueError("weights must be [24961]")
        arr = lambda v, t: (t * k)(*v)
        ps = [_dev(a, torch.float32, "src") for a in srcs]
        pd = [_dev(a, torch.float32, "dst") for a in dsts]
        po = []
        for a, o in zip(srcs, outs):
            if tuple(o.shape) != (a.shape[0],):
                raise ValueError("out must be [N]")
            po.append(_dev(o, torch.float32, "out"))
        return _check(lib().emdq_batch_learned_start(
            self.handle, k, arr(ps, C.c_void_p), arr(pd, C.c_void_p),
            arr([int(a.shape[0]) for a in srcs], C.c_int), arr([w for w, _ in sizes], C.c_int),
            arr([h for _, h in sizes], C.c_int),
            C.byref(params) if params is not None else None,
            _dev(weights, torch.float32, "weights"), arr(po, C.c_void_p), _stream(stream)),
            "emdq_batch_learned_start")

    def fit(self, models, srcs, dsts, sizes, params=None, stream=None, init_ps=None):
        """models: list of Model; srcs, dsts: CUDA float32 [N_i, 2];
        sizes: list of (frame_w, frame_h); init_ps: None (plain start) or
        CUDA float32 [N_i] starting posteriors per pair."""
        import torch
        k = len(models)
        cs = self._pairs(models, srcs, dsts, sizes)
        pi = None
        if init_ps is not None:
            if len(init_ps) != k:
                raise ValueError("init_ps must have one entry per pair")
            pi = (C.c_void_p * k)(*[_dev(t, torch.float32, "init_p") for t in init_ps])
        return _check(lib().emdq_batch_fit(
            self.handle, k, self._handles(models), *cs, pi,
            C.byref(params) if params is not None else None, _stream(stream)),
            "emdq_batch_fit")

    def field(self, models, rects, outs, stream=None):
        """rects: list of (zx0, zy0, w, h); outs: CUDA float32 [h, w, 2]."""
        regs = self._field_regions(models, rects, outs)
        return _check(lib().emdq_batch_field(self.handle, len(models), self._handles(models),
                                             regs, _stream(stream)), "emdq_batch_field")

    @staticmethod
    def _field_regions(models, rects, outs):
        import torch
        regs = (Region * len(models))()
        for r, (zx0, zy0, w, h), o in zip(regs, rects, outs):
            if tuple(o.shape) != (h, w, 2):
                raise ValueError("out must be [h, w, 2]")
            r.zx0, r.zy0, r.w, r.h = zx0, zy0, w, h
            r.out_xy = _dev(o, torch.float32, "out")
        return regs

    @staticmethod
    def _warp_regions(models, frames, canvases, offsets, rects):
        import torch
        regs = (Region * len(models))()
        for r, f, c, (ox, oy), (zx0, zy0, w, h) in zip(regs, frames, canvases, offsets, rects):
            if f.dim() != 3 or f.shape[2] != 3 or c.dim() != 3 or c.shape[2] != 4:
                raise ValueError("frame must be [fh, fw, 3] and canvas [ch, cw, 4]")
            r.zx0, r.zy0, r.w, r.h = zx0, zy0, w, h
            r.frame_rgb = _dev(f, torch.uint8, "frame")
            r.fh, r.fw = int(f.shape[0]), int(f.shape[1])
            r.frame_pitch_bytes = 3 * r.fw
            r.canvas = _dev(c, torch.float32, "canvas")
            r.ch, r.cw = int(c.shape[0]), int(c.shape[1])
            r.canvas_pitch_px = r.cw
            r.ox, r.oy = ox, oy
        return regs

    def autotune(self, models, rects, outs, cache_path=None, stream=None) -> int:
        """Times the field-kernel shapes on batch_field(models, rects, outs)
        and keeps the fastest; returns its index."""
        regs = self._field_regions(models, rects, outs)
        v = C.c_int(-1)
        _check(lib().emdq_batch_autotune(self.handle, len(models), self._handles(models), regs,
                                         None if cache_path is None else
                                         os.fsencode(cache_path), C.byref(v),
                                         _stream(stream)), "emdq_batch_autotune")
        return v.value

    def set_variant(self, variant: int):
        return _check(lib().emdq_batch_set_variant(self.handle, int(variant)),
                      "emdq_batch_set_variant")

    def prepare_field(self, models, rects, outs):
        """Job table of a batched field launch for launch() (host-blocking)."""
        self._keep = (models, outs)
        return _check(lib().emdq_batch_prepare(self.handle, 0, len(models),
                                               self._handles(models),
                                               self._field_regions(models, rects, outs)),
                      "emdq_batch_prepare")

    def prepare_warp(self, models, frames, canvases, offsets, rects):
        self._keep = (models, frames, canvases)
        return _check(lib().emdq_batch_prepare(self.handle, 1, len(models),
                                               self._handles(models),
                                               self._warp_regions(models, frames, canvases,
                                                                  offsets, rects)),
                      "emdq_batch_prepare")

    def launch(self, stream=None):
        """The prepared launch: one kernel, capturable in a graph."""
        return _check(lib().emdq_batch_launch(self.handle, _stream(stream)),
                      "emdq_batch_launch")

    def prepare_step(self, models, srcs, dsts, sizes, frames, canvases, offsets, rects,
                     weights=None, starts=None, params=None):
        """Job tables of a whole step for launch_step() (host-blocking): the
        learned start into `starts` (if `weights` is given), the batched fit
        from it (else from p = 1), and the batched warp."""
        import torch
        k = len(models)
        if (weights is None) != (starts is None):
            raise ValueError("weights and starts go together")
        cs = self._pairs(models, srcs, dsts, sizes)
        arr = lambda v, t: (t * k)(*v)
        pw, pst = None, None
        if weights is not None:
            if tuple(weights.shape) != (N_START_WEIGHTS,):
                raise ValueError("weights must be [24961]")
            pw = _dev(weights, torch.float32, "weights")
            for a, o in zip(srcs, starts):
                if tuple(o.shape) != (a.shape[0],):
                    raise ValueError("start must be [N]")
            pst = arr([_dev(o, torch.float32, "start") for o in starts], C.c_void_p)
        regs = self._warp_regions(models, frames, canvases, offsets, rects)
        self._keep_step = (models, srcs, dsts, frames, canvases, weights, starts)
        return _check(lib().emdq_batch_prepare_step(
            self.handle, k, self._handles(models), *cs,
            C.byref(params) if params is not None else None, pw, pst, regs),
            "emdq_batch_prepare_step")

    def launch_step(self, stream=None):
        """The prepared step: no copy, no host synchronisation, capturable in
        one graph."""
        return _check(lib().emdq_batch_launch_step(self.handle, _stream(stream)),
                      "emdq_batch_launch_step")

    def warp(self, models, frames, canvases, offsets, rects, stream=None):
        """frames: CUDA uint8 [fh, fw, 3]; canvases: CUDA float32 [ch, cw, 4];
        offsets: (ox, oy); rects: (zx0, zy0, w, h)."""
        regs = self._warp_regions(models, frames, canvases, offsets, rects)
        return _check(lib().emdq_batch_warp(self.handle, len(models), self._handles(models),
                                            regs, _stream(stream)), "emdq_batch_warp")

    def close(self):
        if self.handle:
            lib().emdq_batch_free(self.handle)
            self.handle = None
        _open.discard(self)

    def __del__(self, _rel=_release):
        _rel(self)
