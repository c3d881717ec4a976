"""CPU checks of the boundary: the built library loads and exports every
function that include/pic.h declares; the binding refuses to run without a GPU."""
import ctypes
import os

import pytest

import paper_2609_17151_amd as P


def test_header_declares_the_boundary():
    names = P.declared_functions()
    for n in ("pic_init", "pic_load_xsec", "pic_step", "pic_poisson", "pic_diag",
              "pic_get_particles", "pic_set_particles", "pic_sync", "pic_strerror", "pic_free",
              "pic_mlp_create", "pic_mlp_forward", "pic_mlp_train_step", "pic_mlp_grad", "pic_mlp_free"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(P.LIB_PATH), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(P.LIB_PATH)
    for n in P.declared_functions():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(P.LIB_PATH), reason="library not built")
def test_strerror_without_gpu():
    lib = P.load_library()
    assert lib.pic_strerror(P.ECAPACITY) == b"particle capacity exceeded"
    assert lib.pic_strerror(P.OK) == b"ok"


def test_no_cpu_fallback():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    import workloads as W
    with pytest.raises(RuntimeError):
        P.Sim(W.langmuir(n_particles=1024))
    with pytest.raises(RuntimeError):
        P.MLP(W.WARM_WIDTHS, 16)
