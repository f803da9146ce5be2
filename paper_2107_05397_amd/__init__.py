"""Striped UniFrac on MI355X (gfx950): Python binding of ``libuf.so``.

Argument marshalling only: every step of the distance computation runs in the
HIP kernels behind the C ABI of ``include/uf.h``.  PyTorch supplies device
memory (outputs and workspace are CUDA tensors) and streams.  There is no CPU
fallback: if the library is missing or no gfx950 device is present the calls
raise.

Typical use::

    import paper_2107_05397_amd as uf
    tree = uf.Tree(parent, length)
    table = uf.Table(tree, indptr, tips, counts)
    emb = uf.Embedding(tree, table)
    d, row_means, grand_mean = uf.dm_weighted_normalized(emb, "fp32", row_means=True)
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Tuple

import numpy as np

__all__ = [
    "UFError", "lib", "Tree", "Table", "Embedding", "workspace_size", "dm", "dm_unweighted",
    "dm_weighted_normalized", "dm_stripes", "n_stripes", "condensed_index", "set_chunk_nodes",
    "exported_symbols", "LIB_PATH", "HEADER_PATH", "profile_enable", "profile_reset",
    "profile_read", "Batch", "set_split_threshold", "split_stats", "project", "MLP", "sqdist", "topk_rows", "condensed_block",
    "gather_pairs", "Sparse", "rerank", "dm_pairs", "pcoa", "mantel",
]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libuf.so")
HEADER_PATH = os.path.join(os.path.dirname(HERE), "include", "uf.h")

PRECISION = {"fp64": 0, "fp32": 1, "mfma": 2, "mfma_bf16x2": 2, "fp32_split": 3, "mfma_split": 4}
LAYOUT = {"condensed": 0, "stripes": 1}
STATUS = {0: "UF_OK", 1: "UF_ERR_ARG", 2: "UF_ERR_TREE", 3: "UF_ERR_TABLE",
          4: "UF_ERR_EMPTY_SAMPLE", 5: "UF_ERR_RANGE", 6: "UF_ERR_NOMEM", 7: "UF_ERR_DEVICE",
          8: "UF_ERR_UNSUPPORTED", 9: "UF_ERR_WORKSPACE"}


class UFError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__(f"{self.name}: {message}")


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)

_SIGS = {
    "uf_tree_load": (ctypes.c_int, [_i64, _i64p, _f64p, ctypes.POINTER(_vp)]),
    "uf_tree_n_nodes": (_i64, [_vp]),
    "uf_tree_n_tips": (_i64, [_vp]),
    "uf_table_load": (ctypes.c_int, [_vp, _i64, _i64p, _i64p, _i64p, ctypes.POINTER(_vp)]),
    "uf_table_n_samples": (_i64, [_vp]),
    "uf_embed": (ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(_vp)]),
    "uf_embedding_n_samples": (_i64, [_vp]),
    "uf_embedding_scalars": (ctypes.c_int, [_vp, _f64p, _f64p]),
    "uf_embedding_prepare": (ctypes.c_int, [_vp, ctypes.c_int, _vp]),
    "uf_workspace_size": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _i64, _i64, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_size_t)]),
    "uf_set_chunk_nodes": (None, [_i64]),
    "uf_set_split_threshold": (ctypes.c_int, [ctypes.c_int, ctypes.c_double]),
    "uf_split_stats": (ctypes.c_int, [_vp, ctypes.c_int, _i64p, _i64p, _i64p]),
    "uf_dm_unweighted": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp,
                                        ctypes.c_size_t, _vp]),
    "uf_dm_weighted_normalized": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp,
                                                 _vp, ctypes.c_size_t, _vp]),
    "uf_dm_unweighted_stripes": (ctypes.c_int, [_vp, ctypes.c_int, _i64, _i64, ctypes.c_int,
                                                ctypes.c_int, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "uf_dm_weighted_normalized_stripes": (ctypes.c_int, [_vp, ctypes.c_int, _i64, _i64,
                                                         ctypes.c_int, ctypes.c_int, _vp, _vp, _vp,
                                                         ctypes.c_size_t, _vp]),
    "uf_dm_weighted_normalized_noalloc": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp,
                                                         _vp, _vp, _vp]),
    "uf_n_stripes": (_i64, [_i64]),
    "uf_condensed_index": (_i64, [_i64, _i64, _i64]),
    "uf_free_tree": (None, [_vp]),
    "uf_free_table": (None, [_vp]),
    "uf_free_embedding": (None, [_vp]),
    "uf_batch_create": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), _i64, ctypes.c_char_p, _vp,
                                       ctypes.POINTER(_vp)]),
    "uf_batch_plan_create": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), _i64, ctypes.c_int,
                                            ctypes.c_char_p, _vp, ctypes.POINTER(_vp)]),
    "uf_batch_n_tables": (_i64, [_vp]),
    "uf_batch_workspace_size": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "uf_batch_config": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                       _i64p]),
    "uf_batch_set_config": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "uf_batch_set_precision": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp]),
    "uf_batch_run": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.c_int, _vp, ctypes.c_size_t,
                                    _vp]),
    "uf_autotune": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, ctypes.c_char_p, _vp, _f64p]),
    "uf_free_batch": (None, [_vp]),
    "uf_project": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, _i64, ctypes.c_double, _vp, _vp]),
    "uf_mlp_create": (ctypes.c_int, [_i64, _i64p, _i64, ctypes.c_int, ctypes.POINTER(_vp)]),
    "uf_mlp_set": (ctypes.c_int, [_vp, _i64, _vp, _vp, _vp]),
    "uf_mlp_get": (ctypes.c_int, [_vp, _i64, ctypes.c_int, _vp, _vp, _vp]),
    "uf_mlp_backward": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _vp, _vp]),
    "uf_adam_step": (ctypes.c_int, [_vp, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float, _i64, _vp]),
    "uf_mlp_forward": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _vp, _vp]),
    "uf_mlp_loss_grad": (ctypes.c_int, [_vp, _vp, _i64, _vp, _vp, _vp, _i64, ctypes.c_float, _vp,
                                        _vp]),
    "uf_mlp_triplet_loss_grad": (ctypes.c_int, [_vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _i64,
                                                ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                                _vp, _vp]),
    "uf_mlp_adam": (ctypes.c_int, [_vp, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                   ctypes.c_float, ctypes.c_float, _i64, _vp]),
    "uf_free_mlp": (None, [_vp]),
    "uf_sqdist": (ctypes.c_int, [_vp, _i64, _vp, _i64, _i64, _vp, _vp]),
    "uf_topk_rows": (ctypes.c_int, [_vp, _i64, _i64, _i64, _vp, _vp, _vp]),
    "uf_condensed_block": (ctypes.c_int, [_vp, ctypes.c_int, _i64, _i64, _i64, _i64, _i64, _vp, _vp]),
    "uf_gather_pairs": (ctypes.c_int, [_vp, ctypes.c_int, _i64, _vp, _vp, _i64, _vp, _vp]),
    "uf_sparse_build": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(_vp)]),
    "uf_sparse_nnz": (_i64, [_vp]),
    "uf_free_sparse": (None, [_vp]),
    "uf_rerank_workspace_size": (ctypes.c_int, [_vp, _i64, ctypes.POINTER(ctypes.c_size_t)]),
    "uf_dm_rerank_weighted_normalized": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, _i64, _vp, _vp,
                                                        ctypes.c_size_t, _vp]),
    "uf_dm_pairs_weighted_normalized": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _vp,
                                                       ctypes.c_size_t, _vp]),
    "uf_pcoa_workspace_size": (ctypes.c_int, [_i64, _i64, ctypes.POINTER(ctypes.c_size_t)]),
    "uf_pcoa": (ctypes.c_int, [_vp, _i64, _vp, _vp, _i64, _i64, ctypes.c_int, _vp, _vp, _vp, _vp,
                               _vp, ctypes.c_size_t, _vp]),
    "uf_pca_workspace_size": (ctypes.c_int, [_i64, _i64, _i64, ctypes.POINTER(ctypes.c_size_t)]),
    "uf_pca_basis": (ctypes.c_int, [_vp, _i64, _i64, _i64, _i64, _i64, ctypes.c_int, _vp, _vp,
                                    _f64p, _vp, ctypes.c_size_t, _vp]),
    "uf_mantel_workspace_size": (ctypes.c_int, [_i64, ctypes.c_int, _i64,
                                                ctypes.POINTER(ctypes.c_size_t)]),
    "uf_mantel": (ctypes.c_int, [_vp, _vp, _i64, ctypes.c_int, _vp, _i64, ctypes.c_int, _vp, _vp,
                                 _vp, _vp, ctypes.c_size_t, _vp]),
    "uf_profile_enable": (None, [ctypes.c_int]),
    "uf_profile_reset": (None, []),
    "uf_profile_read": (ctypes.c_int, [ctypes.c_char_p, _f64p, _i64p]),
    "uf_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "uf_last_error_message": (ctypes.c_char_p, []),
}


def lib() -> ctypes.CDLL:
    """Load libuf.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2107_05397_amd.build` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    """Function names declared in include/uf.h."""
    text = open(HEADER_PATH).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(uf_[a-z0-9_]+)\s*\(", text)))


def _check(status: int):
    if status != 0:
        msg = lib().uf_last_error_message().decode(errors="replace")
        raise UFError(status, msg)


def _as(a, dtype):
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def n_stripes(n: int) -> int:
    return int(lib().uf_n_stripes(int(n)))


def condensed_index(n: int, i: int, j: int) -> int:
    return int(lib().uf_condensed_index(int(n), int(i), int(j)))


def set_chunk_nodes(nodes: int) -> None:
    """Branches per streamed chunk (0 = automatic, 8 GiB of chunk buffer)."""
    lib().uf_set_chunk_nodes(int(nodes))


def set_split_threshold(fraction: Optional[float] = None, variant: Optional[str] = None) -> None:
    """Dense-set threshold of the sparse-aware split, as a fraction of the samples
    (None: automatic cost model), for one variant or (variant None) both."""
    f = -1.0 if fraction is None else float(fraction)
    for v in ((variant,) if variant else ("unweighted", "weighted_normalized")):
        _check(lib().uf_set_split_threshold(_variant(v), f))


def split_stats(emb, variant: str = "weighted_normalized") -> Tuple[int, int, int]:
    """(dense branches, shared non-dense branches, enumerated pairs) of the split."""
    a, b, c = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().uf_split_stats(emb.handle, _variant(variant), ctypes.byref(a), ctypes.byref(b),
                                ctypes.byref(c)))
    return int(a.value), int(b.value), int(c.value)


def profile_enable(on: bool = True) -> None:
    """Record HIP events around every kernel launch (on the call's stream)."""
    lib().uf_profile_enable(1 if on else 0)


def profile_reset() -> None:
    lib().uf_profile_reset()


def profile_read(kernel: str) -> Tuple[float, int]:
    """(total milliseconds, launches) of one kernel since the last reset."""
    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_int64(0)
    _check(lib().uf_profile_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(cnt)))
    return float(ms.value), int(cnt.value)


class _Handle:
    _free = None

    def __init__(self):
        self._h = _vp()

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h and self._h.value:
            getattr(lib(), self._free)(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tree(_Handle):
    """Validated rooted tree (host).  parent: -1 for the root; any id order."""
    _free = "uf_free_tree"

    def __init__(self, parent, length):
        super().__init__()
        p = _as(parent, np.int64)
        l = _as(length, np.float64)
        if p.shape != l.shape:
            raise UFError(1, "parent and length differ in size")
        _check(lib().uf_tree_load(p.shape[0], _ptr(p, ctypes.c_int64), _ptr(l, ctypes.c_double),
                                  ctypes.byref(self._h)))

    @property
    def n_nodes(self) -> int:
        return int(lib().uf_tree_n_nodes(self._h))

    @property
    def n_tips(self) -> int:
        return int(lib().uf_tree_n_tips(self._h))


class Table(_Handle):
    """Validated CSR sample x tip count table (host)."""
    _free = "uf_free_table"

    def __init__(self, tree: Tree, indptr, tips, counts):
        super().__init__()
        self.tree = tree
        ip = _as(indptr, np.int64)
        tp = _as(tips, np.int64)
        ct = _as(counts, np.int64)
        if ip.ndim != 1 or ip.shape[0] < 1 or tp.shape != ct.shape or tp.shape[0] < ip[-1]:
            raise UFError(1, "malformed CSR arrays")
        _check(lib().uf_table_load(tree.handle, ip.shape[0] - 1, _ptr(ip, ctypes.c_int64),
                                   _ptr(tp, ctypes.c_int64), _ptr(ct, ctypes.c_int64),
                                   ctypes.byref(self._h)))

    @property
    def n_samples(self) -> int:
        return int(lib().uf_table_n_samples(self._h))


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return _vp(int(stream.cuda_stream))


class Embedding(_Handle):
    """Tree + table uploaded to the current HIP device, per-sample scalars computed."""
    _free = "uf_free_embedding"

    def __init__(self, tree: Tree, table: Table, stream=None):
        super().__init__()
        self.tree, self.table = tree, table
        _check(lib().uf_embed(tree.handle, table.handle, _stream_ptr(stream), ctypes.byref(self._h)))

    @property
    def n_samples(self) -> int:
        return int(lib().uf_embedding_n_samples(self._h))

    def scalars(self) -> Tuple[np.ndarray, np.ndarray]:
        """(sw, wu): sum_v l_v u_sv and sum_v l_v a_sv per sample (FP64)."""
        n = self.n_samples
        sw = np.zeros(max(n, 1))
        wu = np.zeros(max(n, 1))
        _check(lib().uf_embedding_scalars(self._h, _ptr(sw, ctypes.c_double),
                                          _ptr(wu, ctypes.c_double)))
        return sw[:n], wu[:n]

    def prepare(self, scalars: bool = True, split_weighted: bool = False,
                split_unweighted: bool = False, stream=None) -> None:
        """Re-run the device-side preparation from the resident table and tree:
        per-sample scalars and/or a rebuild of each requested variant's split."""
        what = (1 if scalars else 0) | (2 if split_unweighted else 0) | (4 if split_weighted else 0)
        _check(lib().uf_embedding_prepare(self._h, what, _stream_ptr(stream)))


def _variant(v: str) -> int:
    if v in ("weighted_normalized", "weighted", "wn"):
        return 1
    if v in ("unweighted", "uw"):
        return 0
    raise UFError(1, f"unknown variant {v!r}")


def workspace_size(emb: Embedding, variant: str, precision: str, stripe_begin: int = 0,
                   stripe_end: Optional[int] = None, row_stats: bool = False) -> int:
    if stripe_end is None:
        stripe_end = emb.n_samples // 2
    out = ctypes.c_size_t(0)
    _check(lib().uf_workspace_size(emb.handle, _variant(variant), PRECISION[precision],
                                   int(stripe_begin), int(stripe_end), int(bool(row_stats)),
                                   ctypes.byref(out)))
    return int(out.value)


def _workspace(nbytes: int, workspace):
    import torch
    if workspace is not None:
        if workspace.numel() * workspace.element_size() < nbytes:
            raise UFError(9, "workspace tensor smaller than workspace_size()")
        return workspace
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda")


def _tptr(t):
    return _vp(int(t.data_ptr())) if t is not None else _vp()


def dm(emb: Embedding, variant: str, precision: str = "fp64", out_dtype=None, out=None,
       row_means: bool = False, stream=None, workspace=None):
    """Full condensed distance matrix on the device.

    Returns (d, row_means, grand_mean); the last two are None unless requested.
    """
    import torch
    out_dtype = out_dtype or torch.float64
    n = emb.n_samples
    npairs = n * (n - 1) // 2
    if out is None:
        out = torch.empty(max(npairs, 1), dtype=out_dtype, device="cuda")
    if out.dtype not in (torch.float64, torch.float32) or out.numel() < npairs or not out.is_contiguous():
        raise UFError(1, "out must be a contiguous float32/float64 CUDA tensor of N(N-1)/2 entries")
    rm = gm = None
    if row_means:
        rm = torch.empty(max(n, 1), dtype=torch.float64, device="cuda")
        gm = torch.empty(1, dtype=torch.float64, device="cuda")
    ws = _workspace(workspace_size(emb, variant, precision, 0, n // 2, row_means), workspace)
    fn = lib().uf_dm_weighted_normalized if _variant(variant) else lib().uf_dm_unweighted
    _check(fn(emb.handle, PRECISION[precision], 1 if out.dtype == torch.float32 else 0,
              _tptr(out), _tptr(rm), _tptr(gm), _tptr(ws), ws.numel() * ws.element_size(),
              _stream_ptr(stream)))
    return out[:npairs], (rm[:n] if rm is not None else None), gm


def dm_weighted_normalized_noalloc(emb: Embedding, precision: str = "fp64", out=None,
                                   row_means=None, grand_mean=None, stream=None):
    """The weighted-normalized matrix into caller-provided tensors, with the
    library's fixed device scratch as workspace: the C call allocates nothing.
    out: contiguous float64/float32 CUDA tensor of >= N(N-1)/2 entries;
    row_means (>= N float64) and grand_mean (>= 1 float64) are optional."""
    import torch
    n = emb.n_samples
    npairs = n * (n - 1) // 2
    if out is None or out.dtype not in (torch.float64, torch.float32) or \
            out.numel() < npairs or not out.is_contiguous():
        raise UFError(1, "out must be a contiguous float32/float64 CUDA tensor of N(N-1)/2 entries")
    for t, k in ((row_means, n), (grand_mean, 1)):
        if t is not None and (t.dtype != torch.float64 or t.numel() < k or not t.is_contiguous()):
            raise UFError(1, "row_means / grand_mean must be contiguous float64 CUDA tensors")
    _check(lib().uf_dm_weighted_normalized_noalloc(
        emb.handle, PRECISION[precision], 1 if out.dtype == torch.float32 else 0, _tptr(out),
        _tptr(row_means), _tptr(grand_mean), _stream_ptr(stream)))
    return out


def dm_unweighted(emb, precision="mfma", **kw):
    return dm(emb, "unweighted", precision, **kw)


def dm_weighted_normalized(emb, precision="fp64", **kw):
    return dm(emb, "weighted_normalized", precision, **kw)


def dm_stripes(emb: Embedding, variant: str, precision: str, stripe_begin: int, stripe_end: int,
               layout: str = "stripes", out_dtype=None, out=None, row_sums: bool = False,
               stream=None, workspace=None):
    """Stripes [begin, end) of the matrix; returns (out, row_sums or None)."""
    import torch
    out_dtype = out_dtype or torch.float64
    n = emb.n_samples
    if layout == "stripes":
        need = max(stripe_end - stripe_begin, 0) * n
        shape = (max(stripe_end - stripe_begin, 0), n)
    else:
        need = n * (n - 1) // 2
        shape = (need,)
    if out is None:
        out = torch.zeros(max(need, 1), dtype=out_dtype, device="cuda")
    if out.numel() < need or not out.is_contiguous():
        raise UFError(1, "out too small or not contiguous")
    rs = torch.empty(max(n, 1), dtype=torch.float64, device="cuda") if row_sums else None
    ws = _workspace(workspace_size(emb, variant, precision, stripe_begin, stripe_end, row_sums),
                    workspace)
    fn = (lib().uf_dm_weighted_normalized_stripes if _variant(variant)
          else lib().uf_dm_unweighted_stripes)
    _check(fn(emb.handle, PRECISION[precision], int(stripe_begin), int(stripe_end),
              LAYOUT[layout], 1 if out.dtype == torch.float32 else 0, _tptr(out), _tptr(rs),
              _tptr(ws), ws.numel() * ws.element_size(), _stream_ptr(stream)))
    return out[:need].view(shape), (rs[:n] if rs is not None else None)


class Batch(_Handle):
    """Many tables on one tree: weighted normalized FP32, one graph replay per run."""
    _free = "uf_free_batch"

    def __init__(self, tree: Tree, tables, tune_cache: Optional[str] = None, stream=None):
        super().__init__()
        self.tree = tree
        self.tables = list(tables)
        arr = (_vp * len(self.tables))(*[t.handle.value for t in self.tables])
        _check(lib().uf_batch_create(tree.handle, arr, len(self.tables),
                                     tune_cache.encode() if tune_cache else None,
                                     _stream_ptr(stream), ctypes.byref(self._h)))
        self._ws = None
        self._outs = None

    @property
    def n_tables(self) -> int:
        return int(lib().uf_batch_n_tables(self._h))

    def workspace_size(self) -> int:
        out = ctypes.c_size_t(0)
        _check(lib().uf_batch_workspace_size(self._h, ctypes.byref(out)))
        return int(out.value)

    def config(self):
        """(stage_branches, wgs_per_cu, chunk_nodes, tile_stripes)."""
        ks, w, ts, kc = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int64(0)
        _check(lib().uf_batch_config(self._h, ctypes.byref(ks), ctypes.byref(w), ctypes.byref(ts),
                                     ctypes.byref(kc)))
        return int(ks.value), int(w.value), int(kc.value), int(ts.value)

    def set_config(self, stage_branches: int, wgs_per_cu: int, tile_stripes: int = 128) -> None:
        _check(lib().uf_batch_set_config(self._h, int(stage_branches), int(wgs_per_cu),
                                         int(tile_stripes)))

    def set_precision(self, precision: str = "fp32", stream=None) -> None:
        """"fp32" (persistent stripe kernel) or "fp32_split" (per-table sparse split on
        forked streams); the workspace is re-sized on the next run."""
        arr = (_vp * len(self.tables))(*[t.handle.value for t in self.tables])
        _check(lib().uf_batch_set_precision(self._h, PRECISION[precision], arr, _stream_ptr(stream)))
        self._ws = None

    def _workspace(self, workspace):
        if workspace is not None:
            return _workspace(self.workspace_size(), workspace)
        if self._ws is None:
            self._ws = _workspace(self.workspace_size(), None)
        return self._ws

    def outputs(self):
        """Per-table condensed FP32 output tensors (allocated once, reused)."""
        import torch
        if self._outs is None:
            self._outs = [torch.empty(max(t.n_samples * (t.n_samples - 1) // 2, 1),
                                      dtype=torch.float32, device="cuda") for t in self.tables]
        return self._outs

    def run(self, use_graph: bool = True, outs=None, workspace=None, stream=None):
        outs = outs if outs is not None else self.outputs()
        ws = self._workspace(workspace)
        arr = (_vp * len(outs))(*[o.data_ptr() for o in outs])
        _check(lib().uf_batch_run(self._h, arr, 1 if use_graph else 0, _tptr(ws),
                                  ws.numel() * ws.element_size(), _stream_ptr(stream)))
        return [o[: t.n_samples * (t.n_samples - 1) // 2] for o, t in zip(outs, self.tables)]

    def autotune(self, tune_cache: Optional[str] = None, workspace=None, stream=None) -> float:
        ws = self._workspace(workspace)
        ms = ctypes.c_double(0.0)
        _check(lib().uf_autotune(self._h, _tptr(ws), ws.numel() * ws.element_size(),
                                 tune_cache.encode() if tune_cache else None,
                                 _stream_ptr(stream), ctypes.byref(ms)))
        return float(ms.value)


# ---------------------------------------------------------------------------
# learned placement
# ---------------------------------------------------------------------------
def project(tree: Tree, emb: Embedding, dims, signs, out_dim: int = 4096, scale: float = 1.0,
            out=None, stream=None):
    """Sparse random projection of l*u: device bfloat16 [N][out_dim]."""
    import torch
    d = _as(dims, np.int32)
    sg = _as(signs, np.int8)
    if d.ndim != 2 or d.shape != sg.shape or d.shape[0] != tree.n_nodes:
        raise UFError(1, "dims/signs must be [n_nodes, per_node]")
    n = emb.n_samples
    if out is None:
        out = torch.empty((max(n, 1), out_dim), dtype=torch.bfloat16, device="cuda")
    _check(lib().uf_project(tree.handle, emb.handle, d.ctypes.data_as(_vp), sg.ctypes.data_as(_vp),
                            d.shape[1], out_dim, float(scale), _tptr(out), _stream_ptr(stream)))
    return out[:n]


class MLP(_Handle):
    """d0 -> ... -> dL perceptron trained by the library's BF16 MFMA kernels."""
    _free = "uf_free_mlp"

    def __init__(self, dims, max_rows: int, params=None, skip=None):
        """params: [(W, b)] per layer; skip: None, or the initial S [dL][d0] of a
        trainable linear path z = MLP(x) + S x."""
        super().__init__()
        self.dims = [int(x) for x in dims]
        self.max_rows = int(max_rows)
        self.has_skip = skip is not None
        arr = np.asarray(self.dims, dtype=np.int64)
        _check(lib().uf_mlp_create(len(self.dims) - 1, _ptr(arr, ctypes.c_int64), self.max_rows,
                                   1 if self.has_skip else 0, ctypes.byref(self._h)))
        if params is not None:
            for l, (w, b) in enumerate(params):
                self.set(l, w, b)
        if self.has_skip:
            self.set(self.n_layers, skip)

    @property
    def n_layers(self) -> int:
        return len(self.dims) - 1

    def set(self, layer: int, w=None, b=None, stream=None):
        wa = _as(w, np.float32) if w is not None else None
        ba = _as(b, np.float32) if b is not None else None
        _check(lib().uf_mlp_set(self._h, layer, wa.ctypes.data_as(_vp) if wa is not None else None,
                                ba.ctypes.data_as(_vp) if ba is not None else None,
                                _stream_ptr(stream)))

    def get(self, layer: int, what: str = "params", stream=None):
        """(w, b) of a layer; layer == n_layers is the linear path (b is None)."""
        sel = {"params": 0, "grads": 1, "adam_m": 2, "adam_v": 3}[what]
        if layer == self.n_layers:
            w = np.zeros((self.dims[-1], self.dims[0]), dtype=np.float32)
            _check(lib().uf_mlp_get(self._h, layer, sel, w.ctypes.data_as(_vp), None,
                                    _stream_ptr(stream)))
            return w, None
        w = np.zeros((self.dims[layer + 1], self.dims[layer]), dtype=np.float32)
        b = np.zeros(self.dims[layer + 1], dtype=np.float32)
        _check(lib().uf_mlp_get(self._h, layer, sel, w.ctypes.data_as(_vp), b.ctypes.data_as(_vp),
                                _stream_ptr(stream)))
        return w, b

    def forward(self, x, rows=None, out=None, stream=None):
        import torch
        n = int(rows.numel()) if rows is not None else int(x.shape[0])
        if out is None:
            out = torch.empty((max(n, 1), self.dims[-1]), dtype=torch.float32, device="cuda")
        _check(lib().uf_mlp_forward(self._h, _tptr(x), x.stride(0), _tptr(rows), n, _tptr(out),
                                    _stream_ptr(stream)))
        return out[:n]

    def loss_grad(self, x, pair_a, pair_b, target, loss=None, rel_floor: float = 0.0, stream=None):
        import torch
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device="cuda")
        _check(lib().uf_mlp_loss_grad(self._h, _tptr(x), x.stride(0), _tptr(pair_a), _tptr(pair_b),
                                      _tptr(target), int(pair_a.numel()), float(rel_floor),
                                      _tptr(loss), _stream_ptr(stream)))
        return loss

    def triplet_loss_grad(self, x, anchor, near, far, d_near, d_far, rank_weight: float = 1.0,
                          tau: float = 0.01, dist_weight: float = 1.0, loss=None, stream=None):
        """Ranking loss over (anchor, near, far) triples (device int32 index tensors
        into x, device FP32 exact distances d(a, near), d(a, far)); gradients stay in
        the MLP."""
        import torch
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device="cuda")
        _check(lib().uf_mlp_triplet_loss_grad(self._h, _tptr(x), x.stride(0), _tptr(anchor),
                                              _tptr(near), _tptr(far), _tptr(d_near), _tptr(d_far),
                                              int(anchor.numel()), float(dist_weight),
                                              float(rank_weight), float(tau), _tptr(loss),
                                              _stream_ptr(stream)))
        return loss

    def backward(self, x, dz, rows=None, stream=None):
        """Parameter gradients for the rows of the preceding forward(x, rows), given
        dz (device BF16 [n][dL])."""
        n = int(rows.numel()) if rows is not None else int(x.shape[0])
        _check(lib().uf_mlp_backward(self._h, _tptr(x), x.stride(0), _tptr(rows), n, _tptr(dz),
                                     _stream_ptr(stream)))

    def adam(self, lr: float, step: int, beta1: float = 0.9, beta2: float = 0.999,
             eps: float = 1e-8, weight_decay: float = 0.0, stream=None):
        if weight_decay == 0.0:
            _check(lib().uf_adam_step(self._h, lr, beta1, beta2, eps, int(step), _stream_ptr(stream)))
            return
        _check(lib().uf_mlp_adam(self._h, lr, beta1, beta2, eps, weight_decay, int(step),
                                 _stream_ptr(stream)))


def sqdist(a, b, out=None, stream=None):
    import torch
    if out is None:
        out = torch.empty((a.shape[0], b.shape[0]), dtype=torch.float32, device="cuda")
    _check(lib().uf_sqdist(_tptr(a), a.shape[0], _tptr(b), b.shape[0], a.shape[1], _tptr(out),
                           _stream_ptr(stream)))
    return out


def topk_rows(values, k: int, stream=None):
    """(idx int32 [rows][k], vals FP32 [rows][k]): the k smallest per row, sorted."""
    import torch
    rows, cols = values.shape
    idx = torch.empty((max(rows, 1), k), dtype=torch.int32, device="cuda")
    vals = torch.empty((max(rows, 1), k), dtype=torch.float32, device="cuda")
    _check(lib().uf_topk_rows(_tptr(values), rows, cols, k, _tptr(idx), _tptr(vals),
                              _stream_ptr(stream)))
    return idx[:rows], vals[:rows]


def _cond_dtype(cond):
    import torch
    if cond.dtype == torch.float64:
        return 0
    if cond.dtype == torch.float32:
        return 1
    raise UFError(1, "condensed matrix must be float32 or float64")


def condensed_block(cond, n: int, row_off: int, n_rows: int, col_off: int, n_cols: int,
                    stream=None):
    import torch
    out = torch.empty((max(n_rows, 1), max(n_cols, 1)), dtype=torch.float32, device="cuda")
    _check(lib().uf_condensed_block(_tptr(cond), _cond_dtype(cond), n, row_off, n_rows, col_off,
                                    n_cols, _tptr(out), _stream_ptr(stream)))
    return out[:n_rows, :n_cols]


def gather_pairs(cond, n: int, a, b, stream=None):
    import torch
    out = torch.empty(max(int(a.numel()), 1), dtype=torch.float32, device="cuda")
    _check(lib().uf_gather_pairs(_tptr(cond), _cond_dtype(cond), n, _tptr(a), _tptr(b),
                                 int(a.numel()), _tptr(out), _stream_ptr(stream)))
    return out[: int(a.numel())]


class Sparse(_Handle):
    """Per-sample lists of touched branches (l*u in FP64), for exact re-ranking."""
    _free = "uf_free_sparse"

    def __init__(self, emb: Embedding, stream=None):
        super().__init__()
        self.emb = emb
        _check(lib().uf_sparse_build(emb.handle, _stream_ptr(stream), ctypes.byref(self._h)))

    @property
    def nnz(self) -> int:
        return int(lib().uf_sparse_nnz(self._h))


def rerank(queries: Sparse, refs: Sparse, query_ids, cand, out=None, workspace=None, stream=None):
    """Exact weighted-normalized d(queries[query_ids[i]], refs[cand[i][c]]): FP64 [nq][k]."""
    import torch
    nq, k = int(cand.shape[0]), int(cand.shape[1])
    if out is None:
        out = torch.empty((max(nq, 1), k), dtype=torch.float64, device="cuda")
    need = ctypes.c_size_t(0)
    _check(lib().uf_rerank_workspace_size(queries.handle, nq, ctypes.byref(need)))
    ws = _workspace(int(need.value), workspace)
    _check(lib().uf_dm_rerank_weighted_normalized(queries.handle, refs.handle, _tptr(query_ids),
                                                  _tptr(cand), nq, k, _tptr(out),
                                                  _tptr(ws), ws.numel() * ws.element_size(),
                                                  _stream_ptr(stream)))
    return out[:nq]


def dm_pairs(a: Sparse, b: Sparse, pairs, out=None, workspace=None, stream=None):
    """Exact weighted-normalized d(a[pairs[0][p]], b[pairs[1][p]]): FP64 [n_pairs]
    (pairs: device int32 [2][n_pairs])."""
    import torch
    n = int(pairs.shape[1])
    if out is None:
        out = torch.empty(max(n, 1), dtype=torch.float64, device="cuda")
    need = ctypes.c_size_t(0)
    _check(lib().uf_rerank_workspace_size(a.handle, n, ctypes.byref(need)))
    ws = _workspace(int(need.value), workspace)
    pairs = pairs.contiguous()
    _check(lib().uf_dm_pairs_weighted_normalized(a.handle, b.handle, _tptr(pairs), n, _tptr(out),
                                                 _tptr(ws), ws.numel() * ws.element_size(),
                                                 _stream_ptr(stream)))
    return out[:n]


def pcoa(dm, n: int, dims: int, omega, power_iters: int = 3, row_means=None, grand_mean=None,
         workspace=None, stream=None):
    """Principal coordinates of a condensed FP64 distance matrix (device tensor).

    omega: device FP64 [n][n_cols] standard-normal test matrix (n_cols >= dims).
    row_means / grand_mean: device FP64 tensors from ``dm(..., row_means=True)``, or
    None to have them computed.  Returns (coords [n][dims] device FP64,
    eigenvalues numpy [dims], trace of the centred matrix)."""
    import torch
    n_cols = int(omega.shape[1])
    need = ctypes.c_size_t(0)
    _check(lib().uf_pcoa_workspace_size(int(n), n_cols, ctypes.byref(need)))
    ws = _workspace(int(need.value), workspace)
    coords = torch.empty((int(n), int(dims)), dtype=torch.float64, device="cuda")
    vals = np.zeros(int(dims), dtype=np.float64)
    tr = ctypes.c_double(0.0)
    _check(lib().uf_pcoa(_tptr(dm), int(n), _tptr(row_means) if row_means is not None else None,
                         _tptr(grand_mean) if grand_mean is not None else None, int(dims), n_cols,
                         int(power_iters), _tptr(omega), _tptr(coords),
                         vals.ctypes.data_as(ctypes.c_void_p), ctypes.byref(tr), _tptr(ws),
                         ws.numel() * ws.element_size(), _stream_ptr(stream)))
    return coords, vals, float(tr.value)


MANTEL_METHOD = {"pearson": 0, "spearman": 1}
ALTERNATIVE = {"two-sided": 0, "greater": 1, "less": 2}


def pca_basis(x, k: int, omega, power_iters: int = 3, d: Optional[int] = None, workspace=None,
              stream=None):
    """Top-k principal directions of the rows of x (device BF16 [n][ldx], first d
    columns): (basis device FP32 [k][d], eigenvalues numpy [k]).  omega: device
    FP64 [d][n_cols] standard normal test matrix."""
    import torch
    n, ldx = int(x.shape[0]), int(x.stride(0))
    d = int(d if d is not None else x.shape[1])
    c = int(omega.shape[1])
    if omega.dtype != torch.float64 or not omega.is_contiguous() or int(omega.shape[0]) != d:
        raise UFError(1, "omega must be a contiguous float64 [d][n_cols] tensor")
    nb = ctypes.c_size_t(0)
    _check(lib().uf_pca_workspace_size(n, d, c, ctypes.byref(nb)))
    ws = _workspace(int(nb.value), workspace)
    basis = torch.empty((k, d), dtype=torch.float32, device="cuda")
    vals = np.zeros(k, dtype=np.float64)
    _check(lib().uf_pca_basis(_tptr(x), n, d, ldx, int(k), c, int(power_iters), _tptr(omega),
                              _tptr(basis), vals.ctypes.data_as(_f64p), _tptr(ws),
                              ws.numel() * ws.element_size(), _stream_ptr(stream)))
    return basis, vals


def mantel(x, y, n: int, method: str = "pearson", perms=None, alternative: str = "two-sided",
           workspace=None, stream=None):
    """Mantel test between condensed FP64 device matrices x and y.

    perms: device int32 [n_perm][n] permutations of the first matrix's samples, or
    None for none.  Returns (statistic, p-value, numpy [n_perm] permuted statistics)."""
    n_perm = 0 if perms is None else int(perms.shape[0])
    need = ctypes.c_size_t(0)
    _check(lib().uf_mantel_workspace_size(int(n), MANTEL_METHOD[method], n_perm, ctypes.byref(need)))
    ws = _workspace(int(need.value), workspace)
    stat, pv = ctypes.c_double(0.0), ctypes.c_double(0.0)
    ps = np.zeros(max(n_perm, 1), dtype=np.float64)
    _check(lib().uf_mantel(_tptr(x), _tptr(y), int(n), MANTEL_METHOD[method], _tptr(perms), n_perm,
                           ALTERNATIVE[alternative], ctypes.byref(stat), ctypes.byref(pv),
                           ps.ctypes.data_as(ctypes.c_void_p), _tptr(ws),
                           ws.numel() * ws.element_size(), _stream_ptr(stream)))
    return float(stat.value), float(pv.value), ps[:n_perm]
