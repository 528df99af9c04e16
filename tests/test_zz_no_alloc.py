"""The allocation-free fit + warp (emdq_fit_warp_static) against the entry
points it stands for, emdq_fit followed by emdq_warp on a model: the same
canvas bits, the same status, EM iterations and inlier count.  Two calls in
a row on the one static array, the second with fewer matches and a smaller
frame, region and canvas; the first goes through the three-launch EM (more
than 2048 matches), the second through the fused two-launch EM."""
import numpy as np
import pytest

from paper_2103_07414_amd import synth
from gpu_util import emdq, to_dev, torch_or_skip

pytestmark = pytest.mark.gpu


def _canvas(torch, ch, cw, seed):
    # a canvas already holding merged colour, so the merge arithmetic counts
    rng = np.random.default_rng(seed)
    c = np.zeros((ch, cw, 4), np.float32)
    c[..., :3] = rng.uniform(0, 255, (ch, cw, 3))
    c[..., 3] = rng.integers(0, 31, (ch, cw))
    return to_dev(c, torch)


def _reference(E, torch, pair, canvas, ox, oy, rect):
    m = E.Model(pair.cfg.n_matches)
    try:
        m.fit(to_dev(pair.src, torch), to_dev(pair.dst, torch), pair.cfg.width, pair.cfg.height)
        m.warp(to_dev(pair.frame, torch), canvas, ox, oy, *rect)
        r = m.results()
    finally:
        m.close()
    return r


@pytest.mark.parametrize("case", [(4, 1, 2), (1, 1, 1)])
def test_static_step_equals_fit_then_warp(case):
    torch = torch_or_skip()
    E = emdq()
    # config 4 (1920x1080, N = 4000), then config 1 (320x240, N = 200), or
    # twice the small pair
    big_cfg, small_cfg, seed = case
    info = torch.full((3,), -99, dtype=torch.int32, device="cuda")
    for k, (config, ch, cw, ox, oy, rect) in enumerate([
            (big_cfg, 1200, 2048, 40, 60, None), (small_cfg, 300, 400, 20, 30, None)]):
        pair = synth.gen_config(config, seed + k)
        W, H = pair.cfg.width, pair.cfg.height
        if rect is None:
            rect = (0, 0, W, H)
        ref_canvas = _canvas(torch, ch, cw, 10 + k)
        got_canvas = ref_canvas.clone()
        ref = _reference(E, torch, pair, ref_canvas, ox, oy, rect)
        print(f"static step call {k}: config {config} seed {seed + k} N={pair.cfg.n_matches} "
              f"frame {W}x{H}", flush=True)
        E.emdq_fit_warp_static(to_dev(pair.src, torch), to_dev(pair.dst, torch),
                               to_dev(pair.frame, torch), got_canvas, ox, oy, *rect, info)
        torch.cuda.synchronize()
        st, iters, n_in = (int(v) for v in info.cpu().numpy())
        assert (st, iters, n_in) == (ref["status"], ref["iters"], ref["n_in"])
        assert st >= 0 and n_in > 0
        a, b = got_canvas.cpu().numpy(), ref_canvas.cpu().numpy()
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), \
            f"canvas differs at {int((a != b).any(-1).sum())} pixels"


def test_static_step_rejects_oversize_and_bad_args():
    torch = torch_or_skip()
    E = emdq()
    L = E.lib()
    n = E.STATIC_MAX_N + 1
    src = torch.zeros((n, 2), dtype=torch.float32, device="cuda")
    frame = torch.zeros((8, 8, 3), dtype=torch.uint8, device="cuda")
    canvas = torch.zeros((8, 8, 4), dtype=torch.float32, device="cuda")
    info = torch.zeros(3, dtype=torch.int32, device="cuda")
    with pytest.raises(E.EmdqError) as e:
        E.emdq_fit_warp_static(src, src, frame, canvas, 0, 0, 0, 0, 8, 8, info)
    assert e.value.status == E.EINVAL
    with pytest.raises(E.EmdqError) as e:
        E.emdq_fit_warp_static(src[:1], src[:1], frame, canvas, 0, 0, 0, 0, 8, 8, info)
    assert e.value.status == E.ETOOFEW
    # the target rectangle leaves the canvas
    with pytest.raises(E.EmdqError) as e:
        E.emdq_fit_warp_static(src[:4], src[:4], frame, canvas, 1, 0, 0, 0, 8, 8, info)
    assert e.value.status == E.EINVAL
    assert L.emdq_fit_warp_static(None, None, 4, None, None, 8, 8, 24, None, 8, 8, 8, 0, 0, 0, 0,
                                  8, 8, None, None) == E.EINVAL
