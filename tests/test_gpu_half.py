"""GPU parity of the half-precision blend (FP16 / BF16 MFMA operands, FP32
accumulation and epilogue) against the FP64 oracle.

Tolerances.  The half-precision error is dominated by the FP16 rounding of
two coded columns: the translation deviation q'_x (up to ~26 px for nodes far
from the tile centre that still carry weight) and the scale deviation
s_j - s0, whose error is multiplied by the absolute coordinate (~2000 px) in
Eq. (1).  An emulation of the kernel's rounding points on the 1920 x 1080,
N = 5000 pair gives up to 6e-4 px from each and 7e-4 px together; the GPU
measured 1.0e-3 px there.  FP16 is held to twice that, 2e-3 px.  BF16
operands carry a unit roundoff 8x larger (2^-8 against 2^-11): 1.6e-2 px.
The EM fit is FP32 in every mode, so masks and iteration counts are still
those of the oracle."""
import numpy as np
import pytest

import oracle as O
from paper_2103_07414_amd import synth

from gpu_util import (COLOUR_TOL, border_mask, emdq, gpu_fit, oracle_fit, oracle_warp_points,
                      to_dev, torch_or_skip)

pytestmark = pytest.mark.gpu

HALF_TOL_PX = {"f16": 2e-3, "bf16": 1.6e-2}


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_half_field_from_oracle_nodes_whole_roi(prec):
    """The oracle's fits loaded as nodes; every pixel of a ragged ROI that
    extends past the frame on all sides (partial 64 x 128 tiles)."""
    torch = torch_or_skip()
    E = emdq()
    P = synth.gen_config(1, 3, with_frame=False)
    ref = oracle_fit(P)
    m = E.Model(P.cfg.n_matches)
    m.set_precision(prec)
    m.set_nodes(P.src, ref.scale.astype(np.float32), ref.q.astype(np.float32), ref.mask,
                ref.alpha)
    zx0, zy0, w, h = -21, -9, 363, 271
    out = torch.empty((h, w, 2), dtype=torch.float32, device="cuda")
    m.field(zx0, zy0, w, h, out)
    s32 = ref.scale.astype(np.float32).astype(np.float64)
    q32 = ref.q.astype(np.float32).astype(np.float64)
    rc, want = O.field(P.src, s32, q32, ref.mask, float(np.float32(ref.alpha)), zx0, zy0, w, h)
    err = np.abs(out.cpu().numpy() - want).max()
    print(f"{prec} field (oracle nodes) max err {err:.2e} px", flush=True)
    assert rc == 0 and err <= HALF_TOL_PX[prec]


@pytest.mark.parametrize("cfg,pair_id,prec", [(2, 1, "f16"), (4, 1, "f16"), (4, 2, "f16"),
                                              (4, 1, "bf16"), (5, 1, "f16")])
def test_half_field_sampled(cfg, pair_id, prec):
    """GPU fit (FP32) + half-precision field at full frame size, sampled
    pixels against the oracle's field of the oracle's fit."""
    torch = torch_or_skip()
    E = emdq()
    P = synth.gen_config(cfg, pair_id, with_frame=False)
    ref = oracle_fit(P)
    m = E.Model(P.cfg.n_matches)
    got = gpu_fit(m, P, torch)
    assert np.array_equal(got["mask"], ref.mask) and got["iters"] == ref.iters
    m.set_precision(prec)
    W, H = P.cfg.width, P.cfg.height
    out = torch.empty((H, W, 2), dtype=torch.float32, device="cuda")
    m.field(0, 0, W, H, out)
    rng = np.random.default_rng(100 + pair_id)
    pts = np.concatenate([rng.integers(0, [W, H], (4000, 2)),
                          [[0, 0], [W - 1, 0], [0, H - 1], [W - 1, H - 1]]]).astype(np.float64)
    rc, want = O.field_points(P.src, ref.scale, ref.q, ref.mask, ref.alpha, pts)
    g = out.cpu().numpy()[pts[:, 1].astype(int), pts[:, 0].astype(int)]
    err = np.abs(g - want).max()
    print(f"config {cfg} pair {pair_id} {prec}: n_in {got['n_in']} field max err {err:.2e} px",
          flush=True)
    assert rc == 0 and err <= HALF_TOL_PX[prec]


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_half_warp_small_whole_canvas(prec):
    torch = torch_or_skip()
    E = emdq()
    P = synth.gen_config(1, 1)
    ref = oracle_fit(P)
    cw, ch, ox, oy = synth.canvas_layout(P.cfg)
    W, H = P.cfg.width, P.cfg.height
    canvas = torch.zeros((ch, cw, 4), dtype=torch.float32, device="cuda")
    m = E.Model(P.cfg.n_matches)
    gpu_fit(m, P, torch)
    m.set_precision(prec)
    m.warp(to_dev(P.frame, torch), canvas, ox, oy, 0, 0, W, H)
    got = canvas.cpu().numpy()
    rc, cv, valid = O.warp(P.src, ref.scale, ref.q, ref.mask, ref.alpha, P.frame,
                           np.zeros((ch, cw, 4)), ox, oy, 0, 0, W, H)
    _, u = O.field(P.src, ref.scale, ref.q, ref.mask, ref.alpha, 0, 0, W, H)
    keep = np.ones((ch, cw), bool)
    keep[oy:oy + H, ox:ox + W] = ~border_mask(u, W, H, eps=HALF_TOL_PX[prec])
    d = np.abs(got - cv)[keep]
    print(f"{prec} warp max colour err {d[:, :3].max():.3e}", flush=True)
    assert d[:, 3].max() == 0.0 and d[:, :3].max() <= COLOUR_TOL


def test_half_warp_production_sampled():
    """FP16 warp of the 1280 x 1024 frame into the 4096^2 canvas."""
    torch = torch_or_skip()
    E = emdq()
    P = synth.gen_config(2, 1)
    ref = oracle_fit(P)
    cw, ch, ox, oy = synth.canvas_layout(P.cfg)
    W, H = P.cfg.width, P.cfg.height
    rng = np.random.default_rng(31)
    init = rng.uniform(0, 255, (ch, cw, 4)).astype(np.float32)
    init[..., 3] = rng.integers(0, 31, (ch, cw)).astype(np.float32)
    canvas = to_dev(init, torch)
    m = E.Model(P.cfg.n_matches)
    gpu_fit(m, P, torch)
    m.set_precision("f16")
    m.warp(to_dev(P.frame, torch), canvas, ox, oy, 0, 0, W, H)
    got = canvas.cpu().numpy()
    pts = rng.integers(0, [W, H], (3000, 2)).astype(np.float64)
    px, py = pts[:, 0].astype(int), pts[:, 1].astype(int)
    want, u, valid = oracle_warp_points(ref, P.src, P.frame, init[py + oy, px + ox], pts)
    keep = ~border_mask(u, W, H, eps=HALF_TOL_PX["f16"])
    d = np.abs(got[py + oy, px + ox] - want)[keep]
    print(f"f16 production warp max colour err {d[:, :3].max():.3e}", flush=True)
    assert d[:, 3].max() == 0.0 and d[:, :3].max() <= COLOUR_TOL
    assert np.array_equal(got[:oy], init[:oy])


def test_half_deterministic_and_f32_restored():
    """Two FP16 evaluations are bit-identical; switching back to FP32 gives
    the FP32 kernel's bits again."""
    torch = torch_or_skip()
    E = emdq()
    P = synth.gen_config(1, 2, with_frame=False)
    m = E.Model(P.cfg.n_matches)
    gpu_fit(m, P, torch)
    W, H = P.cfg.width, P.cfg.height
    outs = {}
    for tag, prec in [("a", "f32"), ("b", "f16"), ("c", "f16"), ("d", "f32")]:
        m.set_precision(prec)
        o = torch.empty((H, W, 2), dtype=torch.float32, device="cuda")
        m.field(0, 0, W, H, o)
        outs[tag] = o.cpu().numpy()
    assert np.array_equal(outs["b"], outs["c"])
    assert np.array_equal(outs["a"], outs["d"])
    assert not np.array_equal(outs["a"], outs["b"])


def test_half_field_in_slabs_matches_oracle():
    """A region wider than the factor tables (4096 columns) is processed in
    slabs; every column, across the slab seam, against the oracle."""
    torch = torch_or_skip()
    E = emdq()
    P = synth.gen_config(1, 2, with_frame=False)
    ref = oracle_fit(P)
    m = E.Model(P.cfg.n_matches)
    m.set_precision("f16")
    m.set_nodes(P.src, ref.scale.astype(np.float32), ref.q.astype(np.float32), ref.mask,
                ref.alpha)
    zx0, zy0, w, h = -3900, 100, 4200, 5
    out = torch.empty((h, w, 2), dtype=torch.float32, device="cuda")
    m.field(zx0, zy0, w, h, out)
    s32 = ref.scale.astype(np.float32).astype(np.float64)
    q32 = ref.q.astype(np.float32).astype(np.float64)
    # far left the weights vanish (NaN on both sides); compare where the
    # oracle is finite and the blend is well conditioned
    rc, want = O.field(P.src, s32, q32, ref.mask, float(np.float32(ref.alpha)), zx0, zy0, w, h)
    got = out.cpu().numpy()
    near = np.arange(w) + zx0 >= -40
    err = np.abs(got[:, near] - want[:, near]).max()
    print(f"slab field max err {err:.2e} px over {near.sum()} columns", flush=True)
    assert err <= HALF_TOL_PX["f16"]


@pytest.mark.parametrize("prec", ["f32", "f16", "bf16"])
def test_field_small_inlier_counts(prec):
    """Inlier counts around the blend's chunk of 64 (one to four chunks,
    ragged and exact): the oracle's nodes of a production pair with the mask
    cut to the n_keep inliers nearest the region, every pixel of a ragged
    300 x 201 region at the frame centre.  (The kept nodes lie within a few
    hundred px of every pixel, where the FP16 per-axis factors do not
    underflow.)"""
    torch = torch_or_skip()
    E = emdq()
    P = synth.gen_config(2, 1, with_frame=False)
    ref = oracle_fit(P)
    W, H = P.cfg.width, P.cfg.height
    zx0, zy0, w, h = W // 2 - 150, H // 2 - 100, 300, 201
    centre = np.array([zx0 + w / 2, zy0 + h / 2])
    inl = np.flatnonzero(ref.mask)
    order = inl[np.argsort(np.linalg.norm(P.src[inl] - centre, axis=1), kind="stable")]
    s32 = ref.scale.astype(np.float32)
    q32 = ref.q.astype(np.float32)
    tol = 1e-3 if prec == "f32" else HALF_TOL_PX[prec]
    m = E.Model(P.cfg.n_matches)
    if prec != "f32":
        m.set_precision(prec)
    out = torch.empty((h, w, 2), dtype=torch.float32, device="cuda")
    for n_keep in (1, 37, 64, 65, 128, 129, 192, 193, 255):
        mask = np.zeros_like(ref.mask)
        mask[order[:n_keep]] = 1
        m.set_nodes(P.src, s32, q32, mask, ref.alpha)
        m.field(zx0, zy0, w, h, out)
        rc, want = O.field(P.src, s32.astype(np.float64), q32.astype(np.float64), mask,
                           float(np.float32(ref.alpha)), zx0, zy0, w, h)
        err = np.abs(out.cpu().numpy() - want).max()
        print(f"{prec} n_in {n_keep}: field max err {err:.2e} px", flush=True)
        assert m.results()["n_in"] == n_keep
        assert rc == 0 and err <= tol, (prec, n_keep, err)
    m.close()


def _corner_nodes(n, seed):
    """Node fits only in the top-left 250 x 250 px of a 1920 x 1080 region:
    one similarity (rotation 0.03 rad, scale 1.01, shift (4, -3) px) with
    small per-node departures (1e-4 rad, 0.2 px, 1e-4), so that the FP16
    deviation coding stays accurate across the region (its coded
    translations grow with the rotation departure times the coordinate) and
    the test isolates the FP16 range."""
    rng = np.random.default_rng(seed)
    x = rng.uniform([0, 0], [250, 250], (n, 2)).astype(np.float32)
    th = 0.03 + rng.uniform(-1e-4, 1e-4, n)
    tx, ty = 4.0 + rng.uniform(-0.2, 0.2, n), -3.0 + rng.uniform(-0.2, 0.2, n)
    c, s = np.cos(th / 2), np.sin(th / 2)
    q = np.stack([c, s, (c * tx + s * ty) / 2, (c * ty - s * tx) / 2], 1).astype(np.float32)
    scale = (1.01 + rng.uniform(-1e-4, 1e-4, n)).astype(np.float32)
    return x, scale, q


def test_f16_far_from_every_inlier_uses_the_f32_blend():
    """FP16 range: pixels more than ~1150 px from every node along an axis
    get no FP16 weight (and pixels a little closer only subnormal weights).
    Such tiles are blended in FP32 instead: no NaN, the whole field within
    the FP16 bar of the oracle, and the far tiles bit-identical to the FP32
    mode (the same kernel and bits there)."""
    torch = torch_or_skip()
    E = emdq()
    W, H, n = 1920, 1080, 300
    x, scale, q = _corner_nodes(n, 5)
    alpha = float(np.float32(O.alpha(W, H)))
    outs = {}
    for prec in ("f16", "f32"):
        m = E.Model(n)
        m.set_precision(prec)
        m.set_nodes(x, scale, q, None, alpha)
        outs[prec] = torch.empty((H, W, 2), dtype=torch.float32, device="cuda")
        m.field(0, 0, W, H, outs[prec])
    f16, f32 = outs["f16"].cpu().numpy(), outs["f32"].cpu().numpy()
    assert np.isfinite(f16).all()
    rc, want = O.field(x, scale.astype(np.float64), q.astype(np.float64), np.ones(n, np.uint8),
                       alpha, 0, 0, W, H)
    err = float(np.abs(f16 - want).max())
    far = np.array_equal(f16[:, 1536:], f32[:, 1536:])
    print(f"f16 corner nodes: max err {err:.2e} px, far tiles equal to f32: {far}", flush=True)
    assert rc == 0 and err <= HALF_TOL_PX["f16"]
    assert far


def test_f16_warp_far_from_every_inlier_uses_the_f32_blend():
    """The same in warp mode: the far tiles merge exactly what the FP32 mode
    merges, and the FP16 canvas stays within one level of the FP32 one."""
    torch = torch_or_skip()
    E = emdq()
    W, H, n = 1920, 1080, 300
    x, scale, q = _corner_nodes(n, 6)
    alpha = float(np.float32(O.alpha(W, H)))
    rng = np.random.default_rng(9)
    frame = to_dev(rng.integers(0, 256, (H, W, 3)).astype(np.uint8), torch)
    canv = {}
    for prec in ("f16", "f32"):
        m = E.Model(n)
        m.set_precision(prec)
        m.set_nodes(x, scale, q, None, alpha)
        canv[prec] = torch.zeros((H, W, 4), dtype=torch.float32, device="cuda")
        m.warp(frame, canv[prec], 0, 0, 0, 0, W, H)
    a, b = canv["f16"].cpu().numpy(), canv["f32"].cpu().numpy()
    assert np.array_equal(a[:, 1536:], b[:, 1536:])
    assert np.abs(a[..., :3] - b[..., :3]).max() <= COLOUR_TOL + 1e-3
    assert (a[..., 3] > 0).sum() > 0.9 * W * H
