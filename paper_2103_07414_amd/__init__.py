"""EMDQ dense deformation field + warp on the MI355X (gfx950).

The compute path lives in the HIP library ``libemdq.so`` (sources under
``csrc/``, C-ABI in ``include/emdq.h``); :mod:`.emdq` is its thin ctypes
binding and :mod:`.synth` draws seeded synthetic inputs.
"""
