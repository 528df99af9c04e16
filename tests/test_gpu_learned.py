"""GPU parity of the learned EM start (kNN features + MLP) and of the EM
started from it, against the FP64 oracle with the same trained weights.

Tolerance of the start: the logit is an FP32 sum of ~200 products of size
<= ~10 (relative error ~1e-6, so |dz| <~ 1e-4 with erf's own few ulps), and
|dp| <= |dz| / 4: 1e-4 on p.  The neighbour order is decided in FP64 on both
sides, so the features are the same up to FP32 rounding.  The EM from the
start is then held to the plain fit's bar: identical masks and iteration
counts, field within 1e-3 px."""
import numpy as np
import pytest

import oracle as O
from paper_2103_07414_amd import synth

from gpu_util import FIELD_TOL_PX, emdq, to_dev, torch_or_skip

pytestmark = pytest.mark.gpu
START_P_TOL = 1e-4


def _start(E, torch, P):
    w = E.load_start_weights()
    src, dst = to_dev(P.src, torch), to_dev(P.dst, torch)
    out = torch.empty(P.cfg.n_matches, dtype=torch.float32, device="cuda")
    E.emdq_learned_start(src, dst, P.cfg.width, P.cfg.height, w, out)
    wo = np.load(E.START_WEIGHTS, allow_pickle=False).astype(np.float64)
    a = O.alpha(P.cfg.width, P.cfg.height)
    want = O.init_mlp(O.init_features(P.src, P.dst, a), wo)
    return src, dst, out, want


@pytest.mark.parametrize("cfg,pair_id", [(1, 1), (2, 1), (5, 1)])
def test_learned_start_parity(cfg, pair_id):
    torch = torch_or_skip()
    E = emdq()
    P = synth.gen_config(cfg, pair_id, with_frame=False)
    _, _, out, want = _start(E, torch, P)
    got = out.cpu().numpy().astype(np.float64)
    err = np.abs(got - want).max()
    print(f"config {cfg}: start max |dp| {err:.2e}, accuracy vs labels "
          f"{np.mean((got > 0.5) == P.inlier):.4f}", flush=True)
    assert err <= START_P_TOL


@pytest.mark.parametrize("cfg,pair_id", [(2, 1), (2, 2), (5, 1)])
def test_em_from_learned_start_parity(cfg, pair_id):
    torch = torch_or_skip()
    E = emdq()
    P = synth.gen_config(cfg, pair_id, with_frame=False)
    src, dst, out, want = _start(E, torch, P)
    W, H = P.cfg.width, P.cfg.height
    m = E.Model(P.cfg.n_matches)
    m.fit_from(src, dst, W, H, out)
    got = m.results()
    ref = O.fit(P.src, P.dst, W, H, init_p=want)
    plain = O.fit(P.src, P.dst, W, H)
    print(f"config {cfg} pair {pair_id}: iters learned {got['iters']}/{ref.iters} "
          f"plain {plain.iters}", flush=True)
    assert got["status"] == ref.status and got["iters"] == ref.iters
    assert np.array_equal(got["mask"], ref.mask)
    fld = torch.empty((H, W, 2), dtype=torch.float32, device="cuda")
    m.field(0, 0, W, H, fld)
    rng = np.random.default_rng(pair_id)
    pts = rng.integers(0, [W, H], (2000, 2)).astype(np.float64)
    _, wf = O.field_points(P.src, ref.scale, ref.q, ref.mask, ref.alpha, pts)
    g = fld.cpu().numpy()[pts[:, 1].astype(int), pts[:, 0].astype(int)]
    assert np.abs(g - wf).max() <= FIELD_TOL_PX


def test_fit_from_ones_is_the_plain_fit():
    torch = torch_or_skip()
    E = emdq()
    P = synth.gen_config(2, 3, with_frame=False)
    src, dst = to_dev(P.src, torch), to_dev(P.dst, torch)
    a, b = E.Model(2000), E.Model(2000)
    a.fit(src, dst, 1280, 1024)
    b.fit_from(src, dst, 1280, 1024, torch.ones(2000, dtype=torch.float32, device="cuda"))
    ra, rb = a.results(), b.results()
    assert ra["iters"] == rb["iters"]
    for k in ("p", "q", "scale", "mask"):
        assert np.array_equal(ra[k], rb[k]), k


def test_fit_from_nonfinite_start_reported():
    torch = torch_or_skip()
    E = emdq()
    P = synth.gen_config(1, 1, with_frame=False)
    init = torch.full((200,), 0.9, dtype=torch.float32, device="cuda")
    init[5] = float("nan")
    m = E.Model(200)
    m.fit_from(to_dev(P.src, torch), to_dev(P.dst, torch), 320, 240, init)
    assert m.status() == E.ENONFINITE
