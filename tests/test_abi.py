"""The C-ABI library loads on the host and exports every function the header
declares; host-only calls (no device work) behave as documented."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "emdq.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(emdq_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    from paper_2103_07414_amd import emdq as E
    L = E.lib()
    names = header_functions()
    assert len(names) == 32
    assert sorted(E.EXPORTS) == names
    for name in names:
        assert hasattr(L, name), name


def test_host_only_calls():
    from paper_2103_07414_amd import emdq as E
    p = E.emdq_params_default()
    assert (p.alpha0, p.ref_w, p.ref_h, p.max_iter) == (np.float32(2e-4), 480, 270, 50)
    assert (p.gamma_min, p.gamma_max, p.flags) == (np.float32(0.05), np.float32(0.95), 0)
    for w, h in [(320, 240), (1280, 1024), (1920, 1080), (480, 270)]:
        assert E.emdq_alpha(p, w, h) == np.float32(O.alpha(w, h))
    assert E.emdq_alpha(None, 0, 5) == 0.0
    assert E.status_string(E.ENONFINITE) == "non-finite match coordinates"
    assert E.status_string(99) == "unknown status"
    L = E.lib()
    h = C.c_void_p()
    assert L.emdq_model_create(1, C.byref(h)) == E.EINVAL      # n_max < 2
    assert L.emdq_model_create(4, None) == E.EINVAL
    assert L.emdq_fit(None, None, None, 4, 10, 10, None, None) == E.EINVAL
    assert L.emdq_field(None, 0, 0, 1, 1, None, None) == E.EINVAL
    assert L.emdq_model_status(None, None) == E.EINVAL
    assert L.emdq_model_set_precision(None, E.PREC_F16) == E.EINVAL
    assert L.emdq_uncertainty(None, 1e-3, 0, 0, 4, 4, None, None) == E.EINVAL
    assert L.emdq_track_nodes(None, 1e-3, 4, None, None, None, None, None) == E.EINVAL
    assert L.emdq_batch_create(0, C.byref(h)) == E.EINVAL
    assert L.emdq_batch_fit(None, 1, None, None, None, None, None, None, None, None,
                            None) == E.EINVAL
    assert L.emdq_batch_learned_start(None, 1, None, None, None, None, None, None, None, None,
                                      None) == E.EINVAL
    assert L.emdq_batch_warp(None, 1, None, None, None) == E.EINVAL
    L.emdq_batch_free(None)
    assert L.emdq_batch_autotune(None, 1, None, None, None, None, None) == E.EINVAL
    assert L.emdq_batch_set_variant(None, 0) == E.EINVAL
    assert L.emdq_batch_prepare(None, 0, 1, None, None) == E.EINVAL
    assert L.emdq_batch_launch(None, None) == E.EINVAL
    assert L.emdq_batch_prepare_step(None, 1, None, None, None, None, None, None, None, None,
                                     None, None) == E.EINVAL
    assert L.emdq_batch_launch_step(None, None) == E.EINVAL
    assert L.emdq_start_features(None, None, 4, 10, 10, None, None, None) == E.EINVAL
    assert L.emdq_start_train_work_floats(0) == 0
    assert L.emdq_start_train_work_floats(3) == 4 * 24962
    assert L.emdq_start_train_step(None, None, None, 1, None, None, 4, None, 4, 1e-3, 1, None,
                                   None) == E.EINVAL
    assert L.emdq_fit_from(None, None, None, 4, 10, 10, None, None, None) == E.EINVAL
    assert L.emdq_learned_start(None, None, 4, 10, 10, None, None, None, None) == E.EINVAL
    L.emdq_model_free(None)
    with pytest.raises(ValueError):
        E.emdq_model_set_precision(None, "f8")


def test_binding_has_no_cpu_path():
    """The binding refuses to run without the built library."""
    from paper_2103_07414_amd import emdq as E
    src = open(E.__file__).read()
    assert "oracle" not in src.replace("there is no CPU fallback", "")


def test_start_weights_file():
    """The trained learned-start weights ship in-tree, load without pickle
    and have the size the header states."""
    from paper_2103_07414_amd import emdq as E
    w = np.load(E.START_WEIGHTS, allow_pickle=False)
    assert w.dtype == np.float32 and w.shape == (E.N_START_WEIGHTS,) == (O.N_WEIGHTS,)
    assert np.isfinite(w).all()


def test_objects_alive_at_interpreter_exit_tear_down_quietly():
    """A model and a batch still referenced when the interpreter exits (here
    by an object of the main script, with torch imported first, as a bench
    script does): their destructors run after this module's globals have been
    cleared and must neither call into HIP nor raise ("Exception ignored in
    ... __del__")."""
    import subprocess
    import sys
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import torch\n"
        "from paper_2103_07414_amd import emdq as E\n"
        "class Holder:\n"
        "    def __init__(self):\n"
        "        m = E.Model.__new__(E.Model); m.handle = None; m.n = 0\n"
        "        b = E.Batch.__new__(E.Batch); b.handle = None\n"
        "        self.objs = [m, b]\n"
        "h = Holder()\n" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr
    assert "Exception ignored" not in r.stderr, r.stderr
