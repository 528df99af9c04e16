"""ctypes loader for the FP64 EMDQ oracle (oracle/emdq_oracle.c).

TEST INFRASTRUCTURE.  Only tests/, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares nothing with the GPU
library and never calls it; see emdq_oracle.c for the paper passages each
function follows.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

OK, WARN_NOT_CONVERGED, EINVAL, ETOOFEW, ENOINLIERS, ENONFINITE = 0, 1, -1, -2, -3, -4

_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_U8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


class Params(C.Structure):
    _fields_ = [("alpha0", C.c_double), ("ref_w", C.c_int), ("ref_h", C.c_int),
                ("max_iter", C.c_int), ("p_thresh", C.c_double),
                ("gamma_min", C.c_double), ("gamma_max", C.c_double),
                ("sigma2_min", C.c_double)]


def lib():
    """Load the oracle library, building it first if it is missing.
    ORACLE_LIB may name another build of emdq_oracle.c (the mutation test
    uses it to load copies with planted mistakes)."""
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIB", _build.LIB)
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        I, Dd = C.c_int, C.c_double
        L.oracle_params_default.argtypes = [C.POINTER(Params)]
        L.oracle_alpha.restype = Dd
        L.oracle_alpha.argtypes = [Dd, I, I, I, I]
        L.oracle_dq_from_rt.argtypes = [Dd, Dd, Dd, _D]
        L.oracle_dq_decode.restype = I
        L.oracle_dq_decode.argtypes = [_D] + [C.POINTER(Dd)] * 4
        L.oracle_warp_point.restype = I
        L.oracle_warp_point.argtypes = [Dd, _D, Dd, Dd, C.POINTER(Dd), C.POINTER(Dd)]
        L.oracle_weighted_fit.restype = I
        L.oracle_weighted_fit.argtypes = [I, _D, _D, _D, C.POINTER(Dd), _D]
        L.oracle_mstep.argtypes = [I, _D, _D, _D, Dd, _D, _D]
        L.oracle_blend_at.restype = I
        L.oracle_blend_at.argtypes = [I, _D, _D, _D, _D, Dd, Dd, Dd,
                                      C.POINTER(Dd), C.POINTER(Dd)]
        L.oracle_estep.argtypes = [I, _D, _D, _D, _D, _D, Dd, _D]
        L.oracle_posterior.argtypes = [I, _D, _D, Dd, C.POINTER(Params), _D,
                                       C.POINTER(Dd), C.POINTER(Dd)]
        L.oracle_fit.restype = I
        L.oracle_fit.argtypes = [I, _D, _D, I, I, C.POINTER(Params), _D, _D, _D, _U8,
                                 C.POINTER(I), C.POINTER(Dd), C.POINTER(Dd)]
        L.oracle_fit_init.restype = I
        L.oracle_fit_init.argtypes = [I, _D, _D, I, I, C.POINTER(Params), C.c_void_p, _D, _D,
                                      _D, _U8, C.POINTER(I), C.POINTER(Dd), C.POINTER(Dd)]
        L.oracle_init_features.argtypes = [I, _D, _D, Dd, _D]
        L.oracle_init_mlp.argtypes = [I, _D, _D, _D]
        L.oracle_init_mlp_bf16.argtypes = [I, _D, _D, _D]
        L.oracle_bf16.restype = Dd
        L.oracle_bf16.argtypes = [Dd]
        L.oracle_start_grad.restype = Dd
        L.oracle_start_grad.argtypes = [I, _D, _D, _D, _D]
        L.oracle_field.restype = I
        L.oracle_field.argtypes = [I, _D, _D, _D, _U8, Dd, I, I, I, I, _D]
        L.oracle_field_points.restype = I
        L.oracle_field_points.argtypes = [I, _D, _D, _D, _U8, Dd, I, _D, _D]
        L.oracle_bilinear.restype = I
        L.oracle_bilinear.argtypes = [_U8, I, I, I, Dd, Dd, _D]
        L.oracle_merge.argtypes = [_D, _D]
        L.oracle_dq_then.argtypes = [_D, _D, _D]
        L.oracle_update.argtypes = [Dd, _D, Dd, _D, C.POINTER(Dd), _D]
        L.oracle_uncertainty.argtypes = [I, _D, _U8, Dd, I, I, I, I, _D]
        L.oracle_blend_dq.restype = I
        L.oracle_blend_dq.argtypes = [I, _D, _D, _D, _U8, Dd, Dd, Dd, C.POINTER(Dd), _D]
        L.oracle_track_nodes.restype = I
        L.oracle_track_nodes.argtypes = [I, _D, _D, _D, _U8, Dd, Dd, I, _D, _D, _D, _D]
        L.oracle_warp.restype = I
        L.oracle_warp.argtypes = [I, _D, _D, _D, _U8, Dd, _U8, I, I, I, _D, I, I, I,
                                  I, I, I, I, I, I, C.c_void_p]
        _lib = L
    return _lib


def _d(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def params(**kw) -> Params:
    p = Params()
    lib().oracle_params_default(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def alpha(w: int, h: int, alpha0: float = 2e-4, ref_w: int = 480, ref_h: int = 270) -> float:
    return lib().oracle_alpha(alpha0, ref_w, ref_h, w, h)


def dq_from_rt(theta: float, tx: float, ty: float) -> np.ndarray:
    q = np.zeros(4)
    lib().oracle_dq_from_rt(theta, tx, ty, q)
    return q


def dq_decode(q):
    out = [C.c_double() for _ in range(4)]
    rc = lib().oracle_dq_decode(_d(q, (4,)), *[C.byref(o) for o in out])
    if rc != 0:
        raise ValueError("DQ with zero real part")
    return tuple(o.value for o in out)


def warp_point(scale: float, q, x: float, y: float):
    ox, oy = C.c_double(), C.c_double()
    if lib().oracle_warp_point(scale, _d(q, (4,)), x, y, C.byref(ox), C.byref(oy)) != 0:
        raise ValueError("DQ with zero real part")
    return ox.value, oy.value


def weighted_fit(x, y, w):
    x, y, w = _d(x), _d(y), _d(w)
    n = w.shape[0]
    s = C.c_double()
    q = np.zeros(4)
    degenerate = lib().oracle_weighted_fit(n, x, y, w, C.byref(s), q)
    return s.value, q, bool(degenerate)


def mstep(x, y, p, alpha_):
    x, y, p = _d(x), _d(y), _d(p)
    n = p.shape[0]
    s, q = np.zeros(n), np.zeros((n, 4))
    lib().oracle_mstep(n, x, y, p, alpha_, s, q)
    return s, q


def estep(x, y, p, s, q, alpha_):
    x, y, p, s, q = _d(x), _d(y), _d(p), _d(s), _d(q)
    n = p.shape[0]
    e2 = np.zeros(n)
    lib().oracle_estep(n, x, y, p, s, q, alpha_, e2)
    return e2


def blend_at(x, s, q, wt, alpha_, zx, zy):
    x, s, q, wt = _d(x), _d(s), _d(q), _d(wt)
    fx, fy = C.c_double(), C.c_double()
    rc = lib().oracle_blend_at(wt.shape[0], x, s, q, wt, alpha_, zx, zy,
                               C.byref(fx), C.byref(fy))
    if rc != 0:
        raise ValueError("no weight at point")
    return fx.value, fy.value


def posterior(e2, p, u, prm=None):
    e2, p = _d(e2), _d(p)
    prm = prm or params()
    out = np.zeros_like(p)
    s2, g = C.c_double(), C.c_double()
    lib().oracle_posterior(p.shape[0], e2, p, u, C.byref(prm), out, C.byref(s2), C.byref(g))
    return out, s2.value, g.value


class Fit:
    """Result of the oracle EM fit."""

    def __init__(self, status, scale, q, p, mask, iters, sigma2, gamma, alpha_):
        self.status, self.scale, self.q, self.p = status, scale, q, p
        self.mask, self.iters, self.sigma2, self.gamma = mask, iters, sigma2, gamma
        self.alpha = alpha_

    @property
    def n_in(self) -> int:
        return int(self.mask.sum())


def fit(src, dst, frame_w: int, frame_h: int, prm: Params | None = None,
        init_p=None) -> Fit:
    """EM fit; src, dst: [N, 2] (float32 inputs are widened exactly).
    init_p: starting posteriors (None: the plain start p = 1)."""
    x, y = _d(src), _d(dst)
    n = x.shape[0]
    prm = prm or params()
    s, q, p = np.zeros(n), np.zeros((n, 4)), np.zeros(n)
    mask = np.zeros(n, dtype=np.uint8)
    it, s2, g = C.c_int(), C.c_double(), C.c_double()
    ip = None if init_p is None else _d(init_p, (n,))
    rc = lib().oracle_fit_init(n, x, y, frame_w, frame_h, C.byref(prm),
                               None if ip is None else ip.ctypes.data_as(C.c_void_p), s, q, p,
                               mask, C.byref(it), C.byref(s2), C.byref(g))
    a = lib().oracle_alpha(prm.alpha0, prm.ref_w, prm.ref_h, frame_w, frame_h)
    return Fit(rc, s, q, p, mask, it.value, s2.value, g.value, a)


def field(x, s, q, mask, alpha_, zx0: int, zy0: int, w: int, h: int):
    x, s, q = _d(x), _d(s), _d(q)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    out = np.zeros((h, w, 2))
    rc = lib().oracle_field(s.shape[0], x, s, q, mask, alpha_, zx0, zy0, w, h, out)
    return rc, out


def field_points(x, s, q, mask, alpha_, pts):
    x, s, q, pts = _d(x), _d(s), _d(q), _d(pts)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    m = pts.shape[0]
    out = np.zeros((m, 2))
    rc = lib().oracle_field_points(s.shape[0], x, s, q, mask, alpha_, m, pts, out)
    return rc, out


def bilinear(frame, ux: float, uy: float):
    frame = np.ascontiguousarray(frame, dtype=np.uint8)
    fh, fw = frame.shape[:2]
    rgb = np.zeros(3)
    rc = lib().oracle_bilinear(frame, fw, fh, fw * 3, ux, uy, rgb)
    return None if rc != 0 else rgb


def merge(px, v):
    px, v = _d(px).copy(), _d(v)
    lib().oracle_merge(px, v)
    return px


def warp(x, s, q, mask, alpha_, frame, canvas, ox: int, oy: int, zx0: int, zy0: int,
         w: int, h: int):
    """Returns (status, new canvas [ch, cw, 4] float64, valid [h, w] uint8)."""
    x, s, q = _d(x), _d(s), _d(q)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    frame = np.ascontiguousarray(frame, dtype=np.uint8)
    fh, fw = frame.shape[:2]
    cv = _d(canvas).copy()
    ch, cw = cv.shape[:2]
    valid = np.zeros((h, w), dtype=np.uint8)
    rc = lib().oracle_warp(s.shape[0], x, s, q, mask, alpha_, frame, fw, fh, fw * 3, cv,
                           cw, ch, cw, ox, oy, zx0, zy0, w, h,
                           valid.ctypes.data_as(C.c_void_p))
    return rc, cv, valid


def dq_then(a, b):
    """The motion applying a first, then b (the "*" of App. A)."""
    out = np.zeros(4)
    lib().oracle_dq_then(_d(a, (4,)), _d(b, (4,)), out)
    return out


def update(s_old, q_old, ds, dq):
    """App. A warp-function update -> (s_new, q_new)."""
    s_new = C.c_double()
    q_new = np.zeros(4)
    lib().oracle_update(s_old, _d(q_old, (4,)), ds, _d(dq, (4,)), C.byref(s_new), q_new)
    return s_new.value, q_new


def uncertainty(x, mask, beta, zx0, zy0, w, h):
    """Eq. (8) at the grid points -> [h, w]."""
    x = _d(x)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    out = np.zeros((h, w))
    lib().oracle_uncertainty(mask.shape[0], x, mask, beta, zx0, zy0, w, h, out)
    return out


def blend_dq(x, s, q, mask, alpha_, zx, zy):
    """Eqs. (2)-(3) at (zx, zy) over the inliers, DQ normalised -> (s, q)."""
    x, s, q = _d(x), _d(s), _d(q)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    so = C.c_double()
    qo = np.zeros(4)
    if lib().oracle_blend_dq(s.shape[0], x, s, q, mask, alpha_, zx, zy, C.byref(so), qo) != 0:
        raise ValueError("no weight at point")
    return so.value, qo


def track_nodes(x, s, q, mask, alpha_, beta, pos, s_node, q_node, sig2):
    """One node tracking step (Sec. III-C/E, Eqs. (8)-(9), App. A) on copies
    of the node arrays -> (status, pos, s_node, q_node, sig2)."""
    x, s, q = _d(x), _d(s), _d(q)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    pos = np.array(pos, dtype=np.float64, order="C")
    s_node = np.array(s_node, dtype=np.float64, order="C")
    q_node = np.array(q_node, dtype=np.float64, order="C")
    sig2 = np.array(sig2, dtype=np.float64, order="C")
    rc = lib().oracle_track_nodes(s.shape[0], x, s, q, mask, alpha_, beta, s_node.shape[0],
                                  pos, s_node, q_node, sig2)
    return rc, pos, s_node, q_node, sig2


KNN, N_FEAT, N_HIDDEN = 16, 64, 128
N_WEIGHTS = N_HIDDEN * N_FEAT + N_HIDDEN + N_HIDDEN * N_HIDDEN + N_HIDDEN + N_HIDDEN + 1


def init_features(src, dst, alpha_):
    """kNN features of the learned EM start -> [N, 64]."""
    x, y = _d(src), _d(dst)
    out = np.zeros((x.shape[0], N_FEAT))
    lib().oracle_init_features(x.shape[0], x, y, alpha_, out)
    return out


def init_mlp(feat, weights, bf16=False):
    """The learned start's network on features [N, 64] -> p [N]; bf16: its
    two matrix products with BF16 operands (oracle_init_mlp_bf16)."""
    feat = _d(feat)
    w = _d(weights, (N_WEIGHTS,))
    out = np.zeros(feat.shape[0])
    (lib().oracle_init_mlp_bf16 if bf16 else lib().oracle_init_mlp)(feat.shape[0], feat, w, out)
    return out


def bf16(v) -> np.ndarray:
    """Each value rounded to bfloat16 (nearest, ties to even), as float64."""
    a = np.asarray(v, dtype=np.float64)
    return np.array([lib().oracle_bf16(float(x)) for x in a.ravel()]).reshape(a.shape)


def start_grad(feat, label, weights):
    """Mean BCE of the learned start and its gradient -> (loss, grad [24961])."""
    feat, label = _d(feat), _d(label)
    w = _d(weights, (N_WEIGHTS,))
    g = np.zeros(N_WEIGHTS)
    loss = lib().oracle_start_grad(feat.shape[0], feat, label, w, g)
    return loss, g
