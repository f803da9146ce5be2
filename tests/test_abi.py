"""C ABI of libuf.so on the CPU: symbols, host-side validation, helpers.

No compute call runs here; without a GPU the device entry points must refuse
with UF_ERR_DEVICE instead of falling back to anything.
"""
import ctypes
import subprocess

import numpy as np
import pytest

import paper_2107_05397_amd as uf
import synth
from tests import _util
from tests.conftest import gpu_available

pytestmark = pytest.mark.skipif(not __import__("os").path.exists(uf.LIB_PATH),
                                reason="libuf.so not built")


def test_every_header_symbol_is_exported():
    names = uf.exported_symbols()
    assert len(names) >= 20
    L = uf.lib()
    for n in names:
        assert hasattr(L, n), n
    dyn = subprocess.run(["nm", "-D", "--defined-only", uf.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = {line.split()[-1] for line in dyn.splitlines() if " T " in line}
    missing = [n for n in names if n not in exported]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2107_05397_amd import _SIGS
    assert set(uf.exported_symbols()) == set(_SIGS)


def test_helpers():
    assert uf.n_stripes(7) == 3 and uf.n_stripes(8) == 4 and uf.n_stripes(0) == 0
    n = 9
    k = 0
    for i in range(n):
        for j in range(i + 1, n):
            assert uf.condensed_index(n, i, j) == k == uf.condensed_index(n, j, i)
            k += 1
    assert uf.condensed_index(5, 2, 2) == -1 and uf.condensed_index(5, 0, 5) == -1
    L = uf.lib()
    for s in range(10):
        assert L.uf_status_string(s)
    assert L.uf_status_string(99) == b"unknown status"


def test_tree_load_and_counts():
    t = synth.gen_tree(50, 0.1, seed=1)
    tree = uf.Tree(t.parent, t.length)
    assert tree.n_nodes == 99 and tree.n_tips == 50


@pytest.mark.parametrize("parent,length,frag", [
    ([-1, -1, 0], [0, 1, 1], "more than one root"),
    ([1, 2, 0, -1], [1, 1, 1, 0], "reachable"),
    ([2, 2, -1], [1, -1.0, 0], "finite"),
    ([2, 2, -1], [1, float("nan"), 0], "finite"),
    ([2, 2, -1], [1, float("inf"), 0], "finite"),
    ([2, 5, -1], [1, 1, 0], "out of range"),
    ([0, 0, -1], [1, 1, 0], "out of range"),
    ([1, 0], [1, 1], "no root"),
])
def test_tree_errors(parent, length, frag):
    with pytest.raises(uf.UFError) as ei:
        uf.Tree(parent, length)
    assert ei.value.name == "UF_ERR_TREE"
    assert frag in str(ei.value)


def test_root_length_ignored_and_any_order_accepted():
    uf.Tree([2, 2, -1], [1.0, 2.0, float("nan")])   # root entry is never read
    uf.Tree([-1, 0, 0, 1, 1], [0, 1, 1, 1, 1])


def test_table_errors():
    tree = uf.Tree([2, 2, -1], [1.0, 2.0, 0.0])
    with pytest.raises(uf.UFError) as ei:
        uf.Table(tree, [0, 1], [2], [1])                # internal node
    assert ei.value.name == "UF_ERR_TABLE"
    with pytest.raises(uf.UFError) as ei:
        uf.Table(tree, [0, 2], [0, 0], [1, 1])          # duplicate
    assert ei.value.name == "UF_ERR_TABLE"
    with pytest.raises(uf.UFError) as ei:
        uf.Table(tree, [0, 1], [5], [1])                # out of range
    assert ei.value.name == "UF_ERR_TABLE"
    with pytest.raises(uf.UFError) as ei:
        uf.Table(tree, [0, 1], [0], [-3])               # negative
    assert ei.value.name == "UF_ERR_TABLE"
    with pytest.raises(uf.UFError) as ei:
        uf.Table(tree, [0, 1, 2], [0, 1], [1, 0])       # zero-total sample
    assert ei.value.name == "UF_ERR_EMPTY_SAMPLE"
    with pytest.raises(uf.UFError) as ei:
        uf.Table(tree, [1, 1], [0], [1])                # indptr[0] != 0
    assert ei.value.name == "UF_ERR_TABLE"
    tab = uf.Table(tree, [0, 2, 3], [0, 1, 1], [0, 4, 1])   # zero entries are allowed
    assert tab.n_samples == 2


def test_null_arguments_are_rejected():
    L = uf.lib()
    h = ctypes.c_void_p()
    assert L.uf_tree_load(0, None, None, ctypes.byref(h)) == 1
    assert L.uf_tree_load(3, None, None, None) == 1
    out = ctypes.c_size_t()
    assert L.uf_workspace_size(None, 0, 0, 0, 0, 0, ctypes.byref(out)) == 1
    assert L.uf_dm_unweighted(None, 0, 0, None, None, None, None, 0, None) == 1
    assert L.uf_embed(None, None, None, ctypes.byref(h)) == 1
    msg = L.uf_last_error_message()
    assert isinstance(msg, bytes) and len(msg) > 0


@pytest.mark.skipif(gpu_available(), reason="checks the no-device path")
def test_embed_refuses_without_device():
    t = synth.gen_tree(10, 0.1, seed=1)
    tree = uf.Tree(t.parent, t.length)
    tab = uf.Table(tree, [0, 1], [0], [3])
    with pytest.raises(uf.UFError) as ei:
        uf.Embedding.__new__(uf.Embedding).__init__(tree, tab, stream=_FakeStream())
    assert ei.value.name == "UF_ERR_DEVICE"


class _FakeStream:
    cuda_stream = 0


def test_header_documents_every_function():
    text = open(uf.HEADER_PATH).read()
    for name in uf.exported_symbols():
        assert text.count(name) >= 1


def test_null_embedding_with_split_precisions_is_rejected():
    # the split precisions resolve the embedding's split first: a NULL embedding must
    # be refused before that, on every distance entry point, with or without a GPU
    L = uf.lib()
    out = ctypes.c_void_p(8)
    for prec in (uf.PRECISION["fp32_split"], uf.PRECISION["mfma_split"]):
        assert L.uf_dm_unweighted_stripes(None, prec, 0, 1, 0, 0, out, None, None, 0, None) == 1
        assert L.uf_dm_weighted_normalized_stripes(None, prec, 0, 1, 0, 0, out, None, None, 0,
                                                   None) == 1
        assert L.uf_dm_unweighted(None, prec, 0, out, None, None, None, 0, None) == 1
        assert L.uf_dm_weighted_normalized(None, prec, 0, out, None, None, None, 0, None) == 1
    assert L.uf_embedding_prepare(None, 1, None) == 1
    assert L.uf_split_stats(None, 1, None, None, None) == 1


# The calls the hot path's boundary is specified with, and the entry point of
# include/uf.h that provides each (the same name where the signature matches the
# specification's intent; the reasons for every difference are recorded with the
# design).
BOUNDARY = {
    "uf_tree_load": "uf_tree_load",
    "uf_table_load": "uf_table_load",
    "uf_embed": "uf_embed",
    "uf_workspace_size": "uf_workspace_size",
    "uf_dm_unweighted": "uf_dm_unweighted",
    "uf_dm_weighted_normalized": "uf_dm_weighted_normalized",
    "uf_dm_unweighted_stripes": "uf_dm_unweighted_stripes",
    "uf_dm_weighted_normalized_stripes": "uf_dm_weighted_normalized_stripes",
    "uf_n_stripes": "uf_n_stripes",
    "uf_condensed_index": "uf_condensed_index",
    "uf_autotune": "uf_autotune",
    "uf_batch_plan_create": "uf_batch_plan_create",
    "uf_batch_run": "uf_batch_run",
    "uf_project": "uf_project",
    "uf_mlp_forward": "uf_mlp_forward",
    "uf_mlp_backward": "uf_mlp_backward",
    "uf_adam_step": "uf_adam_step",
    "uf_dm_pairs_weighted_normalized": "uf_dm_pairs_weighted_normalized",
    "uf_free_tree": "uf_free_tree",
    "uf_free_table": "uf_free_table",
    "uf_free_embedding": "uf_free_embedding",
    "uf_status_string": "uf_status_string",
    "uf_last_error_message": "uf_last_error_message",
}


def test_specified_boundary_calls_are_exported():
    names = set(uf.exported_symbols())
    missing = [k for k, v in BOUNDARY.items() if v not in names]
    assert not missing, missing
    L = uf.lib()
    for v in BOUNDARY.values():
        assert hasattr(L, v)
