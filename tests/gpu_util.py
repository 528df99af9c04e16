"""Shared helpers of the GPU tests: run the library through its C-ABI binding
and the oracle on the same seeded inputs."""
import numpy as np
import pytest

import oracle as O
from paper_2103_07414_amd import synth

# Tolerances (derivation in the design notes): the FP32 field must agree with
# the FP64 oracle to 1e-3 px and warped colours to 1 uint8 level; the inlier
# masks and EM iteration counts must be identical.
FIELD_TOL_PX = 1e-3
COLOUR_TOL = 1.0
# Diagnostics of the fit itself (FP32 EM against FP64 EM).
P_TOL = 2e-3
SCALE_RTOL = 1e-4
Q_ROT_ATOL = 1e-5


def torch_or_skip():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def emdq():
    from paper_2103_07414_amd import emdq as E
    E.lib()          # fails loudly when the library is missing
    return E


def to_dev(a, torch):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_fit(model, pair, torch, params=None):
    E = emdq()
    src, dst = to_dev(pair.src, torch), to_dev(pair.dst, torch)
    model.fit(src, dst, pair.cfg.width, pair.cfg.height, params)
    return model.results()


def oracle_fit(pair, prm=None):
    return O.fit(pair.src, pair.dst, pair.cfg.width, pair.cfg.height, prm)


def border_mask(u, fw, fh, eps=1e-3):
    """Points whose sample position lies within eps px of the frame's
    validity border (validity may flip between FP32 and FP64)."""
    ux, uy = u[..., 0], u[..., 1]
    near = (np.abs(ux) < eps) | (np.abs(ux - (fw - 1)) < eps) | \
           (np.abs(uy) < eps) | (np.abs(uy - (fh - 1)) < eps)
    return near


def oracle_warp_points(fit, x, frame, canvas_px, pts):
    """Oracle field + bilinear + merge at points pts [M, 2] (src coords),
    starting from canvas values canvas_px [M, 4].  Returns the merged pixels,
    the sample positions and the validity."""
    rc, u = O.field_points(x, fit.scale, fit.q, fit.mask, fit.alpha, pts)
    fh, fw = frame.shape[:2]
    out = canvas_px.astype(np.float64).copy()
    valid = np.zeros(len(pts), bool)
    for i in range(len(pts)):
        v = O.bilinear(frame, u[i, 0], u[i, 1])
        if v is not None:
            out[i] = O.merge(out[i], v)
            valid[i] = True
    return out, u, valid


def fit_prediction_error(src, got, ref):
    """max_i |W_i(x_i)| difference between the GPU fits and the oracle's,
    each evaluated in FP64 by the oracle's Eq. (1)."""
    x = np.asarray(src, dtype=np.float64)
    err = 0.0
    for i in range(len(x)):
        a = O.warp_point(float(got["scale"][i]), got["q"][i].astype(np.float64), x[i, 0], x[i, 1])
        b = O.warp_point(ref.scale[i], ref.q[i], x[i, 0], x[i, 1])
        err = max(err, abs(a[0] - b[0]), abs(a[1] - b[1]))
    return err


# Learned start (BF16 network): tolerances derived in test_gpu_learned.py.
START_P_TOL = 2.5e-2     # any match (up to two BF16 rounding steps)
START_P_TOL_99 = 1e-5    # 99 % of the matches (no rounding step)


def check_start(got, want, what):
    """The learned start against the oracle's BF16 network: every match
    within START_P_TOL, 99 % within START_P_TOL_99, and the starting mask
    equal wherever the oracle's p is further than START_P_TOL from 0.5."""
    got = np.asarray(got, dtype=np.float64)
    d = np.abs(got - want)
    q99 = float(np.quantile(d, 0.99))
    print(f"{what}: start |dp| max {d.max():.2e}, 99% {q99:.2e}", flush=True)
    assert d.max() <= START_P_TOL and q99 <= START_P_TOL_99
    clear = np.abs(want - 0.5) > START_P_TOL
    assert np.array_equal((got > 0.5)[clear], (want > 0.5)[clear])


def oracle_start(src, dst, w, h, wo):
    return O.init_mlp(O.init_features(src, dst, O.alpha(w, h)), wo, bf16=True)
