"""Error paths and edge cases of the C-ABI on the GPU."""
import ctypes as C

import numpy as np
import pytest

from paper_2103_07414_amd import synth

from gpu_util import emdq, to_dev, torch_or_skip

pytestmark = pytest.mark.gpu


def test_too_few_and_invalid_arguments():
    torch = torch_or_skip()
    E = emdq()
    L = E.lib()
    m = E.Model(16)
    x = torch.zeros((1, 2), dtype=torch.float32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    assert L.emdq_fit(m.handle, x.data_ptr(), x.data_ptr(), 1, 10, 10, None, s) == E.ETOOFEW
    x = torch.zeros((17, 2), dtype=torch.float32, device="cuda")
    assert L.emdq_fit(m.handle, x.data_ptr(), x.data_ptr(), 17, 10, 10, None, s) == E.EINVAL
    assert L.emdq_fit(m.handle, None, x.data_ptr(), 4, 10, 10, None, s) == E.EINVAL
    assert L.emdq_fit(m.handle, x.data_ptr(), x.data_ptr(), 4, 0, 10, None, s) == E.EINVAL
    prm = E.emdq_params_default()
    prm.max_iter = 0
    assert L.emdq_fit(m.handle, x.data_ptr(), x.data_ptr(), 4, 10, 10, C.byref(prm), s) \
        == E.EINVAL
    assert L.emdq_field(m.handle, 0, 0, -1, 4, x.data_ptr(), s) == E.EINVAL
    assert L.emdq_field(m.handle, 0, 0, 4, 4, None, s) == E.EINVAL


def test_nonfinite_coordinates_reported():
    torch = torch_or_skip()
    E = emdq()
    P = synth.gen_config(1, 1)
    dst = P.dst.copy()
    dst[17, 0] = np.inf
    m = E.Model(P.cfg.n_matches)
    m.fit(to_dev(P.src, torch), to_dev(dst, torch), 320, 240)
    assert m.status() == E.ENONFINITE
    # after the error the field is NaN and the canvas is left as is, in
    # every precision
    for prec in ("f32", "f16", "bf16"):
        m.set_precision(prec)
        out = torch.zeros((8, 8, 2), dtype=torch.float32, device="cuda")
        m.field(0, 0, 8, 8, out)
        assert torch.isnan(out).all(), prec
        cv = torch.full((16, 16, 4), 7.0, dtype=torch.float32, device="cuda")
        m.warp(to_dev(P.frame, torch), cv, 0, 0, 0, 0, 16, 16)
        assert (cv == 7.0).all(), prec
    m.set_precision("f32")
    # the model recovers with the next good fit
    m.fit(to_dev(P.src, torch), to_dev(P.dst, torch), 320, 240)
    assert m.status() == E.OK


def test_empty_model_has_no_inliers():
    torch = torch_or_skip()
    E = emdq()
    m = E.Model(8)
    assert m.status() == E.ENOINLIERS
    mask = np.zeros(4, np.uint8)
    m.set_nodes(np.zeros((4, 2)), np.ones(4), np.tile([1.0, 0, 0, 0], (4, 1)), mask, 1e-3)
    assert m.status() == E.ENOINLIERS


def test_warp_rejects_bad_rectangles_and_alignment():
    torch = torch_or_skip()
    E = emdq()
    P = synth.gen_config(1, 1)
    m = E.Model(P.cfg.n_matches)
    m.fit(to_dev(P.src, torch), to_dev(P.dst, torch), 320, 240)
    frame = to_dev(P.frame, torch)
    cv = torch.zeros((100, 100, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(E.EmdqError):
        m.warp(frame, cv, 0, 0, 0, 0, 101, 10)          # leaves the canvas
    with pytest.raises(E.EmdqError):
        m.warp(frame, cv, -1, 0, 0, 0, 10, 10)
    L = E.lib()
    s = torch.cuda.current_stream().cuda_stream
    big = torch.zeros(4 * 100 * 100 + 1, dtype=torch.float32, device="cuda")
    assert L.emdq_warp(m.handle, frame.data_ptr(), 320, 240, 960, big.data_ptr() + 4, 100, 100,
                       100, 0, 0, 0, 0, 10, 10, s) == E.EINVAL      # not 16-byte aligned
    assert L.emdq_warp(m.handle, frame.data_ptr(), 320, 240, 900, cv.data_ptr(), 100, 100,
                       100, 0, 0, 0, 0, 10, 10, s) == E.EINVAL      # pitch < 3 w
    # zero-size ROI is a no-op
    assert m.warp(frame, cv, 0, 0, 0, 0, 0, 10) == E.OK
    assert not cv.any()


def test_two_matches_minimum_and_max_n():
    torch = torch_or_skip()
    E = emdq()
    src = np.array([[10.0, 10.0], [50.0, 30.0]], np.float32)
    dst = src + np.float32(2.0)
    m = E.Model(2)
    m.fit(to_dev(src, torch), to_dev(dst, torch), 64, 48)
    r = m.results()
    assert r["status"] == E.OK and r["n_in"] == 2
    out = torch.empty((4, 4, 2), dtype=torch.float32, device="cuda")
    m.field(0, 0, 4, 4, out)
    gy, gx = np.mgrid[0:4, 0:4]
    assert np.abs(out.cpu().numpy() - (np.stack([gx, gy], -1) + 2.0)).max() < 1e-3


def test_fresh_models_after_freed_ones_stop_where_the_oracle_stops():
    """A model's stop-flag slots in pinned memory may be memory a freed model
    used; its fits must still run to the oracle's iteration count (both EM
    paths: 1504 and 2807 matches), however many models came and went."""
    import oracle as O
    torch = torch_or_skip()
    E = emdq()
    pairs = synth.gen_batch(2, seed=3007, with_frame=False)
    refs = [O.fit(p.src, p.dst, p.cfg.width, p.cfg.height) for p in pairs]
    dev = [(to_dev(p.src, torch), to_dev(p.dst, torch)) for p in pairs]
    for cycle in range(4):
        for p, (s, d), ref in zip(pairs, dev, refs):
            m = E.Model(p.cfg.n_matches)
            m.fit(s, d, p.cfg.width, p.cfg.height)
            r = m.results()
            m.close()
            assert (r["status"], r["iters"]) == (ref.status, ref.iters), (cycle, p.cfg.n_matches)
            assert np.array_equal(r["mask"], ref.mask)
