"""Generator determinism and the binding's host-side argument checks (CPU)."""
import numpy as np
import pytest

from paper_2103_07414_amd import synth


def test_generator_is_deterministic():
    a = synth.gen_config(1, 2)
    b = synth.gen_config(1, 2)
    for x, y in [(a.src, b.src), (a.dst, b.dst), (a.inlier, b.inlier), (a.frame, b.frame)]:
        assert x.tobytes() == y.tobytes()
    c = synth.gen_config(1, 3)
    assert a.src.tobytes() != c.src.tobytes()


@pytest.mark.parametrize("config", [1, 2])
def test_generator_shapes_and_statistics(config):
    P = synth.gen_config(config, 1)
    cfg = P.cfg
    assert P.src.shape == (cfg.n_matches, 2) and P.src.dtype == np.float32
    assert P.dst.shape == (cfg.n_matches, 2) and P.dst.dtype == np.float32
    assert P.frame.shape == (cfg.height, cfg.width, 3) and P.frame.dtype == np.uint8
    assert P.frame.min() == 0 and P.frame.max() == 255          # min-max stretched
    assert (~P.inlier).sum() == round(cfg.outlier_rate * cfg.n_matches)
    assert (P.src[:, 0] >= 0).all() and (P.src[:, 0] <= cfg.width - 1).all()
    # inliers follow the truth motion up to the N(0, 1 px) noise per axis
    r = P.dst[P.inlier].astype(np.float64) - P.truth_map(P.src[P.inlier].astype(np.float64))
    n = r.shape[0]
    assert abs(r.std() - cfg.noise_px) < 0.1
    assert (np.abs(r.mean(0)) < 4.0 * cfg.noise_px / np.sqrt(n)).all()   # 4 standard errors
    # the texture is smooth: neighbouring pixels differ much less than random
    d = np.abs(np.diff(P.frame.astype(float), axis=1)).mean()
    assert d < 20


def test_canvas_layout_centres_the_roi():
    cw, ch, ox, oy = synth.canvas_layout(synth.CONFIGS[2])
    assert (cw, ch, ox, oy) == (4096, 4096, 1408, 1536)
    cw, ch, ox, oy = synth.canvas_layout(synth.CONFIGS[1])
    assert (cw, ch, ox, oy) == (640, 480, 160, 120)


def test_similarity_matches_are_exact_in_fp64():
    src, dst = synth.similarity_matches(50, 320, 240, 0.1, 1.02, (3.0, -4.0), seed=7)
    c = np.array([159.5, 119.5])
    R = np.array([[np.cos(0.1), -np.sin(0.1)], [np.sin(0.1), np.cos(0.1)]])
    want = c + 1.02 * (src.astype(np.float64) - c) @ R.T + [3.0, -4.0]
    assert np.abs(dst - want).max() < 1e-3      # FP32 rounding only


def test_binding_rejects_host_tensors_and_bad_shapes():
    torch = pytest.importorskip("torch")
    from paper_2103_07414_amd import emdq as E
    x = torch.zeros((4, 2), dtype=torch.float32)          # host tensor
    with pytest.raises(TypeError):
        E.emdq_fit(0, x, x, 10, 10)
    with pytest.raises(ValueError):
        E.emdq_fit(0, torch.zeros((4, 3)), torch.zeros((4, 3)), 10, 10)
    with pytest.raises(ValueError):
        E.emdq_model_set_nodes(0, np.zeros((3, 2)), np.ones(2), np.zeros((3, 4)), None, 1e-3)
