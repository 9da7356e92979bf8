"""CPU-side checks of the C-ABI library: it loads and exports every function
include/hlbm.h declares; the Python binding refuses to run without a GPU."""
import os

import pytest

from paper_2401_10878_amd import hlbm


def test_library_exports_every_declared_function():
    if not os.path.exists(hlbm.LIBPATH):
        pytest.skip("libhlbm.so not built (run __graft_entry__.build())")
    L = hlbm.load()
    names = hlbm.header_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_params_struct_covers_header_fields():
    txt = open(hlbm.HEADER).read()
    body = txt[txt.index("typedef struct {"):txt.index("} hlbm_params;")]
    for f, _ in hlbm.Params._fields_:
        assert f in body, f


def test_binding_fails_loudly_without_gpu(W):
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    if not os.path.exists(hlbm.LIBPATH):
        pytest.skip("libhlbm.so not built")
    wl = W.c1_two_spheres()
    with pytest.raises(RuntimeError):
        hlbm.Simulation(wl.params, wl.scene)
