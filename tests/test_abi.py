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
                 "nomad_config_default", "nomad_init_batched", "nomad_batch_problem"):
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
    assert cfg.collect_stats == 0 and cfg.record_trace == 0


def test_binding_structs_match_the_c_header(tmp_path):
    """Field offsets and sizes of the ctypes structs equal those a C compiler gives for
    include/nomad.h."""
    import shutil
    import subprocess

    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    fields = {"nomad_config": nm.NomadConfig, "nomad_stats": nm.NomadStats,
              "nomad_problem_desc": nm.NomadProblemDesc}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "nomad.h"', "int main(void) {"]
    for cname, cls in fields.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            cf = "lambda" if fname == "lambda_" else fname
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {cf}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call([gcc, "-I", os.path.dirname(nm.HEADER), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    seen = {}
    for line in filter(None, out):
        cname, what, val = line.split()
        seen[(cname, what)] = int(val)
    for cname, cls in fields.items():
        assert seen[(cname, "size")] == C.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert seen[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


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


def test_batch_entry_points_reject_bad_arguments_without_a_device():
    if not os.path.exists(nm.library_path()):
        pytest.skip("libnomad.so not built")
    lib = nm.load()
    assert lib.nomad_batch_graph(None, 2) == nm.NOMAD_ESTATE
    assert b"not a batch" in lib.nomad_last_error(None)
    best = nm.NomadConfig()
    assert lib.nomad_tune_batched(1, None, None, None, nm.TUNE_PROGRESS(0), None, C.byref(best), None) == \
        nm.NOMAD_EINVAL
    assert b"NULL config" in lib.nomad_last_error(None)
    sub = C.c_void_p()
    assert lib.nomad_batch_problem(None, 0, C.byref(sub)) == nm.NOMAD_ESTATE
    assert lib.nomad_init_batched(C.byref(sub), 0, None, None, None) != nm.NOMAD_OK
