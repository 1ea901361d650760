"""The C ABI library loads and exports every function include/abm.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "abm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(abm_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("abm_pop_create", "abm_pop_step", "abm_pop_query", "abm_batch_create", "abm_batch_step",
                     "abm_batch_hist", "abm_mlp_train_step", "abm_mlp_grads", "abm_mlp_infer", "abm_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2503_10796_amd import abm
    lib = abm.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_no_gpu_calls_needed_for_sizes():
    from paper_2503_10796_amd import abm
    lib = abm.lib()
    dims = (ctypes.c_int * 5)(35, 256, 256, 256, 32)
    assert lib.abm_mlp_workspace_bytes(dims, 5, 4096) > 0
    assert lib.abm_mlp_workspace_bytes(dims, 0, 4096) == 0
    cap = (ctypes.c_int64 * 1)(1000)
    bcap = (ctypes.c_int64 * 1)(4096)
    assert lib.abm_batch_workspace_bytes(1, cap, bcap) > 0
    assert lib.abm_last_error() == b""
