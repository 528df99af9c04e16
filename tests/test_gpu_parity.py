"""GPU parity: the HIP path, called through the C-ABI, against the FP64 oracle
on the same seeded inputs.

Every pair is compared element by element over its whole output: the small
pairs, the production-size pair (1280 x 1024, N = 2000, 4096^2 canvas, the
launch configuration the benchmark times) and a 1920 x 1080, N = 4000 pair."""
import numpy as np
import pytest

import oracle as O
from paper_2103_07414_amd import synth

from gpu_util import (COLOUR_TOL, FIELD_TOL_PX, P_TOL, Q_ROT_ATOL, SCALE_RTOL, border_mask,
                      emdq, fit_prediction_error, gpu_fit, oracle_fit, oracle_warp_points,
                      to_dev, torch_or_skip)

pytestmark = pytest.mark.gpu


def _fit_parity(cfg, pair_id, torch):
    E = emdq()
    P = synth.gen_config(cfg, pair_id, with_frame=False)
    ref = oracle_fit(P)
    m = E.Model(P.cfg.n_matches)
    got = gpu_fit(m, P, torch)
    margin = float(np.abs(ref.p - 0.5).min())
    print(f"config {cfg} pair {pair_id}: iters {ref.iters}/{got['iters']} n_in "
          f"{ref.n_in}/{got['n_in']} min|p-0.5| {margin:.3e} "
          f"max|dp| {np.abs(got['p'] - ref.p).max():.2e}", flush=True)
    assert got["status"] == ref.status
    assert got["iters"] == ref.iters
    assert np.array_equal(got["mask"], ref.mask)
    assert got["n_in"] == ref.n_in
    assert np.abs(got["p"] - ref.p).max() <= P_TOL
    assert np.allclose(got["scale"], ref.scale, rtol=SCALE_RTOL, atol=0)
    # rotation halves of the DQs; the translation halves are checked through
    # each fit's prediction at its own match (what the field depends on)
    assert np.abs(got["q"][:, :2] - ref.q[:, :2]).max() <= Q_ROT_ATOL
    pred_err = fit_prediction_error(P.src, got, ref)
    print(f"  max fit prediction err {pred_err:.2e} px", flush=True)
    assert pred_err <= FIELD_TOL_PX
    assert got["sigma2"] == pytest.approx(ref.sigma2, rel=1e-3)
    assert got["gamma"] == pytest.approx(ref.gamma, rel=1e-4)
    return P, ref, m, got


@pytest.mark.parametrize("pair_id", [1, 2, 3])
def test_fit_parity_small(pair_id):
    torch = torch_or_skip()
    _fit_parity(1, pair_id, torch)


@pytest.mark.parametrize("pair_id", [1, 2, 3])
def test_fit_parity_production(pair_id):
    torch = torch_or_skip()
    _fit_parity(2, pair_id, torch)


@pytest.mark.parametrize("cfg", [4, 5])
def test_fit_parity_1920x1080(cfg):
    """N = 4000 and 5000 (multi-chunk M-step sweeps, config 5 with 40 %
    outliers): the same bar as at production size; the per-fit prediction
    is where a loss of precision in the M-step's moments shows first."""
    torch = torch_or_skip()
    _fit_parity(cfg, 1, torch)


@pytest.mark.parametrize("pair_id", [1, 2])
def test_field_parity_small_whole_roi(pair_id):
    """Fit + field on the GPU vs fit + field in the oracle, every pixel,
    over a ROI that also extends past the frame."""
    torch = torch_or_skip()
    P, ref, m, got = _fit_parity(1, pair_id, torch)
    zx0, zy0, w, h = -20, -13, 363, 270          # ragged: not multiples of 32
    out = torch.empty((h, w, 2), dtype=torch.float32, device="cuda")
    m.field(zx0, zy0, w, h, out)
    rc, want = O.field(P.src, ref.scale, ref.q, ref.mask, ref.alpha, zx0, zy0, w, h)
    err = np.abs(out.cpu().numpy() - want).max()
    print(f"field max err {err:.2e} px", flush=True)
    assert rc == 0 and err <= FIELD_TOL_PX


def test_field_kernel_alone_from_oracle_nodes():
    """The field kernel fed the oracle's own fits (set_nodes): isolates the
    blend from the EM."""
    torch = torch_or_skip()
    E = emdq()
    P = synth.gen_config(1, 3, with_frame=False)
    ref = oracle_fit(P)
    m = E.Model(P.cfg.n_matches)
    m.set_nodes(P.src, ref.scale.astype(np.float32), ref.q.astype(np.float32), ref.mask,
                ref.alpha)
    assert m.status() == 0
    w, h = 320, 240
    out = torch.empty((h, w, 2), dtype=torch.float32, device="cuda")
    m.field(0, 0, w, h, out)
    s32 = ref.scale.astype(np.float32).astype(np.float64)
    q32 = ref.q.astype(np.float32).astype(np.float64)
    rc, want = O.field(P.src, s32, q32, ref.mask, float(np.float32(ref.alpha)), 0, 0, w, h)
    err = np.abs(out.cpu().numpy() - want).max()
    print(f"field (oracle nodes) max err {err:.2e} px", flush=True)
    assert err <= FIELD_TOL_PX


@pytest.mark.parametrize("pair_id", [1, 2, 3])
def test_field_parity_production_whole_roi(pair_id):
    """Every one of the 1,310,720 field points of the production pair."""
    torch = torch_or_skip()
    P, ref, m, got = _fit_parity(2, pair_id, torch)
    W, H = P.cfg.width, P.cfg.height
    out = torch.empty((H, W, 2), dtype=torch.float32, device="cuda")
    m.field(0, 0, W, H, out)
    rc, want = O.field(P.src, ref.scale, ref.q, ref.mask, ref.alpha, 0, 0, W, H)
    err = np.abs(out.cpu().numpy() - want).max()
    print(f"production field max err {err:.2e} px over {W * H} points", flush=True)
    assert rc == 0 and err <= FIELD_TOL_PX


def test_warp_parity_small_whole_canvas():
    """Warp + merge of one frame into an empty canvas, then a second merge
    of another frame on top (TSDF running average), every canvas pixel."""
    torch = torch_or_skip()
    E = emdq()
    P = synth.gen_config(1, 1)
    P2 = synth.gen_config(1, 2)
    ref = oracle_fit(P)
    ref2 = oracle_fit(P2)
    cw, ch, ox, oy = synth.canvas_layout(P.cfg)
    W, H = P.cfg.width, P.cfg.height
    canvas = torch.zeros((ch, cw, 4), dtype=torch.float32, device="cuda")
    m = E.Model(P.cfg.n_matches)
    gpu_fit(m, P, torch)
    m.warp(to_dev(P.frame, torch), canvas, ox, oy, 0, 0, W, H)
    m2 = E.Model(P2.cfg.n_matches)
    gpu_fit(m2, P2, torch)
    m2.warp(to_dev(P2.frame, torch), canvas, ox, oy, 0, 0, W, H)
    got = canvas.cpu().numpy()

    cv0 = np.zeros((ch, cw, 4))
    rc, cv1, v1 = O.warp(P.src, ref.scale, ref.q, ref.mask, ref.alpha, P.frame, cv0,
                         ox, oy, 0, 0, W, H)
    rc2, cv2, v2 = O.warp(P2.src, ref2.scale, ref2.q, ref2.mask, ref2.alpha, P2.frame, cv1,
                          ox, oy, 0, 0, W, H)
    _, u1 = O.field(P.src, ref.scale, ref.q, ref.mask, ref.alpha, 0, 0, W, H)
    _, u2 = O.field(P2.src, ref2.scale, ref2.q, ref2.mask, ref2.alpha, 0, 0, W, H)
    near = border_mask(u1, W, H) | border_mask(u2, W, H)
    keep = np.ones((ch, cw), bool)
    keep[oy:oy + H, ox:ox + W] = ~near
    d = np.abs(got - cv2)[keep]
    print(f"warp max colour err {d[:, :3].max():.3e}, alpha err {d[:, 3].max()}, "
          f"border-excluded {near.sum()}", flush=True)
    assert d[:, 3].max() == 0.0
    assert d[:, :3].max() <= COLOUR_TOL
    # outside the target rectangle nothing is touched
    outside = np.ones((ch, cw), bool)
    outside[oy:oy + H, ox:ox + W] = False
    assert not got[outside].any()


def _warp_parity_whole_roi(P, ref, m, canvas_layout, seed, torch):
    """Warp into a canvas of random colours and weights at the layout's
    offset; every ROI pixel against the oracle's warp of the same ROI, except
    those whose sample point lies within 1e-3 px of the frame border; the
    rest of the canvas must keep its bits."""
    cw, ch, ox, oy = canvas_layout
    W, H = P.cfg.width, P.cfg.height
    rng = np.random.default_rng(seed)
    init = rng.uniform(0, 255, (ch, cw, 4)).astype(np.float32)
    init[..., 3] = rng.integers(0, 31, (ch, cw)).astype(np.float32)
    canvas = to_dev(init, torch)
    m.warp(to_dev(P.frame, torch), canvas, ox, oy, 0, 0, W, H)
    got = canvas.cpu().numpy()
    roi0 = init[oy:oy + H, ox:ox + W].astype(np.float64)
    rc, want, valid = O.warp(P.src, ref.scale, ref.q, ref.mask, ref.alpha, P.frame, roi0,
                             0, 0, 0, 0, W, H)
    _, u = O.field(P.src, ref.scale, ref.q, ref.mask, ref.alpha, 0, 0, W, H)
    keep = ~border_mask(u, W, H)
    d = np.abs(got[oy:oy + H, ox:ox + W] - want)[keep]
    print(f"warp {W}x{H}: max colour err {d[:, :3].max():.3e}, alpha err {d[:, 3].max()}, "
          f"merged {int(valid.sum())}, border-excluded {int((~keep).sum())}", flush=True)
    assert rc == 0
    assert d[:, 3].max() == 0.0 and d[:, :3].max() <= COLOUR_TOL
    outside = np.ones((ch, cw), bool)
    outside[oy:oy + H, ox:ox + W] = False
    assert np.array_equal(got[outside], init[outside])


@pytest.mark.parametrize("pair_id", [1, 2])
def test_warp_parity_production_whole_roi(pair_id):
    """1280 x 1024 frame into the 4096^2 RGBA FP32 canvas (the benchmark's
    launch), every ROI pixel against the oracle."""
    torch = torch_or_skip()
    E = emdq()
    P = synth.gen_config(2, pair_id)
    ref = oracle_fit(P)
    m = E.Model(P.cfg.n_matches)
    got_fit = gpu_fit(m, P, torch)
    assert np.array_equal(got_fit["mask"], ref.mask)
    _warp_parity_whole_roi(P, ref, m, synth.canvas_layout(P.cfg), 10 + pair_id, torch)


def test_field_and_warp_parity_fhd_whole_frame():
    """1920 x 1080, N = 4000 in FP32: launches of 1020 32 x 64 tiles, which
    take two 32-row blocks per wavefront.  Fit, every field point and every
    warped pixel against the oracle."""
    torch = torch_or_skip()
    P, ref, m, got = _fit_parity(4, 1, torch)
    W, H = P.cfg.width, P.cfg.height
    out = torch.empty((H, W, 2), dtype=torch.float32, device="cuda")
    m.field(0, 0, W, H, out)
    rc, want = O.field(P.src, ref.scale, ref.q, ref.mask, ref.alpha, 0, 0, W, H)
    err = np.abs(out.cpu().numpy() - want).max()
    print(f"1920x1080 field max err {err:.2e} px over {W * H} points", flush=True)
    assert rc == 0 and err <= FIELD_TOL_PX
    P = synth.gen_config(4, 1)
    _warp_parity_whole_roi(P, ref, m, (W + 40, H + 24, 17, 9), 41, torch)


def test_identity_and_similarity_invariants():
    torch = torch_or_skip()
    E = emdq()
    rng = np.random.default_rng(21)
    src = rng.uniform(0, 319, (200, 2)).astype(np.float32)
    m = E.Model(200)
    m.fit(to_dev(src, torch), to_dev(src, torch), 320, 240)
    r = m.results()
    assert r["status"] == 0 and r["n_in"] == 200 and r["iters"] == 2
    out = torch.empty((240, 320, 2), dtype=torch.float32, device="cuda")
    m.field(0, 0, 320, 240, out)
    gy, gx = np.mgrid[0:240, 0:320]
    assert np.abs(out.cpu().numpy() - np.stack([gx, gy], -1)).max() <= FIELD_TOL_PX
    # one exact similarity is reproduced everywhere
    src, dst = synth.similarity_matches(200, 320, 240, 0.06, 1.04, (5.0, -3.0), seed=22)
    m.fit(to_dev(src, torch), to_dev(dst, torch), 320, 240)
    r = m.results()
    assert r["n_in"] == 200
    m.field(0, 0, 320, 240, out)
    c = np.array([159.5, 119.5])
    pts = np.stack([gx, gy], -1).astype(np.float64)
    R = np.array([[np.cos(0.06), -np.sin(0.06)], [np.sin(0.06), np.cos(0.06)]])
    want = c + 1.04 * (pts - c) @ R.T + np.array([5.0, -3.0])
    # inputs are FP32-rounded, so the fit sees the similarity to ~1e-5 px
    assert np.abs(out.cpu().numpy() - want).max() <= FIELD_TOL_PX


def test_not_converged_status_matches_oracle():
    torch = torch_or_skip()
    E = emdq()
    P = synth.gen_config(2, 3, with_frame=False)
    prm = E.emdq_params_default()
    prm.max_iter = 3
    ref = oracle_fit(P, O.params(max_iter=3))
    m = E.Model(P.cfg.n_matches)
    r = gpu_fit(m, P, torch, prm)
    assert ref.status == O.WARN_NOT_CONVERGED
    assert r["status"] == E.WARN_NOT_CONVERGED and r["iters"] == 3
    assert np.array_equal(r["mask"], ref.mask)


def test_determinism_bit_identical():
    torch = torch_or_skip()
    E = emdq()
    P = synth.gen_config(2, 1)
    cw, ch, ox, oy = synth.canvas_layout(P.cfg)
    W, H = P.cfg.width, P.cfg.height
    outs = []
    for _ in range(2):
        m = E.Model(P.cfg.n_matches)
        r = gpu_fit(m, P, torch)
        f = torch.empty((H, W, 2), dtype=torch.float32, device="cuda")
        m.field(0, 0, W, H, f)
        cv = torch.zeros((H + 64, W + 64, 4), dtype=torch.float32, device="cuda")
        m.warp(to_dev(P.frame, torch), cv, 32, 32, 0, 0, W, H)
        outs.append((r["p"], r["q"], r["scale"], f.cpu().numpy(), cv.cpu().numpy()))
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
