"""The C-ABI library loads and exports every function include/split.h declares; host-side
argument checks that need no GPU. CPU only (no kernels are launched)."""
import ctypes
import os
import re

import pytest

import paper_2511_18022_amd as sg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "split.h")
HEADERS = sorted(os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
                 if f.endswith(".h"))


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(split_[a-z_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(sg.LIB_PATH):
        from paper_2511_18022_amd import _build
        _build.build()
    return sg.load_library()


def test_header_declares_the_binding_surface():
    assert declared_functions() == sorted(sg.EXPORTED)


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_null_context_is_rejected_without_touching_the_gpu(lib):
    null = ctypes.c_void_p()
    assert lib.split_instance_set_coords(null, 5, None) == sg.SPLIT_E_INVAL
    assert lib.split_instance_set_dist(null, 5, None) == sg.SPLIT_E_INVAL
    assert lib.split_eval(null, None, 1, None, 1, 1, 1, None, None, None) == sg.SPLIT_E_INVAL
    assert lib.split_set_form(null, 1) == sg.SPLIT_E_INVAL
    assert lib.split_timing_enable(null, 1) == sg.SPLIT_E_INVAL
    assert lib.split_timing_samples(null, None, 0, None) == sg.SPLIT_E_INVAL
    assert lib.split_stats_get(null, None) == sg.SPLIT_E_INVAL
    assert lib.split_ctx_create(0, None) == sg.SPLIT_E_INVAL
    assert lib.split_last_error(null) == b"null context"
    lib.split_ctx_destroy(null)
    assert lib.split_tuning_set(null, None) == sg.SPLIT_E_INVAL
    assert lib.split_tuning_get(null, None) == sg.SPLIT_E_INVAL
    assert lib.split_autotune(null, None, None, 1, None, 1, 1, 1, None, 1, 1, None, None,
                              None) == sg.SPLIT_E_INVAL
    assert lib.split_graph_create(null, 1, 1, None, 1, 1, 1, None, 1, None) == sg.SPLIT_E_INVAL
    assert lib.split_graph_launch(null, None, None, 1, None) == sg.SPLIT_E_INVAL
    assert lib.split_graph_stats(null, None, None) == sg.SPLIT_E_INVAL
    lib.split_graph_destroy(null)


def test_tuning_struct_matches_header():
    text = open(HEADER).read()
    body = re.search(r"typedef struct \{([^}]*)\} split_tuning;", text).group(1)
    fields = re.findall(r"int32_t\s+(\w+);", body)
    assert fields == [f for f, _ in sg.SplitTuningC._fields_]


def test_status_codes_match_header():
    text = open(HEADER).read()
    for name, val in re.findall(r"(SPLIT_E_[A-Z]+|SPLIT_OK)\s*=\s*(-?\d+)", text):
        assert getattr(sg, name) == int(val), name


def test_nn_parameter_count_matches_header_and_oracle():
    from oracle import nn
    text = open(os.path.join(ROOT, "include", "split_nn.h")).read()
    count = int(re.search(r"#define SPLIT_NN_PARAMS (\d+)", text).group(1))
    assert count == sg.NN_PARAMS == nn.n_params()
    split_h = open(os.path.join(ROOT, "include", "split.h")).read()
    assert int(re.search(r"#define SPLIT_MAX_N (\d+)", split_h).group(1)) == sg.SPLIT_MAX_N


def test_nn_null_handles_are_rejected(lib):
    null = ctypes.c_void_p()
    assert lib.split_nn_create(null, 0, 1.0, None) == sg.SPLIT_E_INVAL
    assert lib.split_nn_predict(null, None, 1, 1, None, None) == sg.SPLIT_E_INVAL
    assert lib.split_nn_train(null, None, None, 1, 1, 1, 1, 1.0, 0, None, None) == sg.SPLIT_E_INVAL
    assert lib.split_topk_smallest(null, None, 1, 1, None, None) == sg.SPLIT_E_INVAL
    assert lib.split_nn_screen(null, None, 1, 1, 1, None, 1, 1, 1, None, None, None, None, None,
                               None) == sg.SPLIT_E_INVAL
    assert lib.split_nn_timing_enable(null, 1) == sg.SPLIT_E_INVAL
    assert lib.split_nn_timing_get(null, None, None) == sg.SPLIT_E_INVAL
    assert lib.split_nn_timing_reset(null) == sg.SPLIT_E_INVAL
    lib.split_nn_destroy(null)
    assert lib.split_search(null, None, None, 1, None, 1, 1, 1, 1, 1, 1.0, 1, 0, None, None, None,
                            0, None, None, None) == sg.SPLIT_E_INVAL
