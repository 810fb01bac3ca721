"""The C-ABI library loads on any host and exports every function the header declares
(no compute call: this file runs without a GPU)."""
import ctypes as C
import os

import pytest

import paper_1312_0193_amd as nm


def test_header_declares_the_boundary():
    names = set(nm.declared_functions())
    for want in ("nomad_init", "nomad_train_epochs", "nomad_eval_rmse", "nomad_get_factors",
                 "nomad_get_partition", "nomad_get_trace", "nomad_destroy", "nomad_last_error",
                 "nomad_config_default"):
        assert want in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(nm.library_path()):
        pytest.skip("libnomad.so not built (run __graft_entry__.build())")
    lib = nm.load()
    for name in nm.declared_functions():
        assert hasattr(lib, name), name


def test_config_struct_matches_header_defaults():
    if not os.path.exists(nm.library_path()):
        pytest.skip("libnomad.so not built")
    cfg = nm.NomadConfig()
    nm.load().nomad_config_default(C.byref(cfg))
    assert cfg.sched == 0 and cfg.dtype == 0 and cfg.workers == 0 and cfg.k == 0
    assert C.sizeof(nm.NomadConfig) == 56


def test_null_arguments_are_rejected_without_a_device():
    if not os.path.exists(nm.library_path()):
        pytest.skip("libnomad.so not built")
    lib = nm.load()
    assert lib.nomad_init(None, None, 1, 1, 0, None, None, None, None, None, None) == nm.NOMAD_EINVAL
    assert b"out is NULL" in lib.nomad_last_error(None)
    ctx = C.c_void_p()
    cfg = nm.NomadConfig()
    lib.nomad_config_default(C.byref(cfg))
    cfg.k = 0
    assert lib.nomad_init(C.byref(ctx), C.byref(cfg), 10, 10, 0, None, None, None, None, None, None) == nm.NOMAD_EINVAL
    assert b"k=0" in lib.nomad_last_error(None)
    assert lib.nomad_train_epochs(None, 1, None) == nm.NOMAD_ESTATE
    lib.nomad_destroy(None)
