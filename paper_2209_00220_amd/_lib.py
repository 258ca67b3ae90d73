"""ctypes binding of ``include/bytestore.h``: the same names, argument marshalling only.

Every ``bst_*`` function here forwards to the C symbol of the same name and
raises ``BstError`` on a negative status.  Pointers are passed as Python ints
(device pointers from ``tensor.data_ptr()``, host pointers from numpy), streams
as the raw ``hipStream_t`` integer.  Loading fails loudly when the HIP library
has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbytestore.so")

BST_OK = 0
BST_DEV_BAD_ROW = 1
BST_DEV_OVERFLOW = 2
BITPACKED, BYTESLICE, PPVBS, PPVBS_CATEGORICAL = 0, 1, 2, 3
LAYOUT_NAMES = {BITPACKED: "bitpacked", BYTESLICE: "byteslice", PPVBS: "ppvbs"}
LT, LE, GT, GE, EQ, NE, BETWEEN = range(7)
OP_CODES = {"lt": LT, "le": LE, "gt": GT, "ge": GE, "eq": EQ, "ne": NE, "between": BETWEEN}
KMAX = 6
TILE_ROWS = 2048
BATCH_ROUND_ROBIN = 0xFFFFFFFF   # tiles_per_grab: static round-robin tiles, no counter
NBUF = 19
BUF_BS1, BUF_BS2, BUF_M2, BUF_DIR2, BUF_PACKED, BUF_DICT, BUF_TRIE = 0, 1, 6, 11, 16, 17, 18
(TUNE_SCAN_GRID, TUNE_LOOKUP_GRID, TUNE_BATCH_GRID, TUNE_BATCH_GRAB, TUNE_GATHER_ROWS, TUNE_BATCH_STREAMS,
 TUNE_BATCH_SOLO_TILES) = range(7)


class BstError(RuntimeError):
    pass


class Pred(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("lo", ctypes.c_uint32), ("hi", ctypes.c_uint32)]


class ColumnInfo(ctypes.Structure):
    _fields_ = [
        ("layout", ctypes.c_uint32), ("width_bits", ctypes.c_uint32), ("k_max", ctypes.c_uint32),
        ("dir_stride", ctypes.c_uint32), ("domain_mode", ctypes.c_uint32), ("categorical", ctypes.c_uint32),
        ("n_rows", ctypes.c_uint64), ("n_distinct", ctypes.c_uint64),
        ("bytes", ctypes.c_uint64 * NBUF), ("total_bytes", ctypes.c_uint64),
        ("rows_by_len", ctypes.c_uint64 * (KMAX + 1)), ("layout_bytes", ctypes.c_uint64),
        ("rows_end_by_mask", ctypes.c_uint64 * (KMAX + 1)),
    ]


_P = ctypes.c_void_p
_U64 = ctypes.c_uint64
_U32 = ctypes.c_uint32
_I = ctypes.c_int

# name: (restype, argtypes)
_PROTOS = {
    "bst_last_error": (ctypes.c_char_p, []),
    "bst_version": (_I, []),
    "bst_device_count": (_I, []),
    "bst_dict_build": (_I, [_P, _U64, _U32, _P]),
    "bst_dict_free": (None, [_P]),
    "bst_dict_info": (_I, [_P, _P, _P]),
    "bst_dict_values": (_I, [_P, _P, _P]),
    "bst_encode": (_I, [_P, _I, _U32, _U32, _U32, _P]),
    "bst_encode_host": (_I, [_P, _U64, _I, _U32, _P]),
    "bst_encode_codes": (_I, [_P, _P, _U64, _U32, _P]),
    "bst_free_host": (None, [_P]),
    "bst_host_info": (_I, [_P, _P]),
    "bst_host_code_table": (_I, [_P, _P, _P]),
    "bst_host_paper_view": (_I, [_P, _I, _I, _P, _P]),
    "bst_upload": (_I, [_P, _P, _P, _P]),
    "bst_column_free": (None, [_P]),
    "bst_column_info_get": (_I, [_P, _P]),
    "bst_scan": (_I, [_P, Pred, _P, _P, _P, _P]),
    "bst_scan_codes": (_I, [_P, _I, _U64, _U32, _U64, _U32, _P, _P, _P]),
    "bst_scan_stats": (_I, [_P, Pred, _P, _P, _P, _P]),
    "bst_lookup": (_I, [_P, _P, _U64, _P, _P, _P]),
    "bst_compact_workspace_bytes": (_U64, [_U64]),
    "bst_bv_compact": (_I, [_P, _U64, _P, _U64, _P, _P, _P, _P]),
    "bst_lookup_bv": (_I, [_P, _P, _P, _U64, _P, _P, _P, _P, _P]),
    "bst_lookup_bv_static": (_I, [_P, _P, _P, _U64, _P, _P, _P]),
    "bst_lookup_counted": (_I, [_P, _P, _P, _U64, _P, _P, _P]),
    "bst_lookup_bv_static_max_rows": (_U64, []),
    "bst_lookup_bv_static_max_ids": (_U64, []),
    "bst_bv_and": (_I, [_P, _P, _P, _U64, _P]),
    "bst_bv_or": (_I, [_P, _P, _P, _U64, _P]),
    "bst_bv_andnot": (_I, [_P, _P, _P, _U64, _P]),
    "bst_bv_not": (_I, [_P, _P, _U64, _P]),
    "bst_bv_popcount": (_I, [_P, _U64, _P, _P]),
    "bst_profile_literals": (_I, [_P, _I, _I, _P, _P]),
    "bst_auc": (_I, [_P, _P, _I, _P]),
    "bst_choose": (_I, [_P, _P, _I, _P]),
    "bst_advise": (_I, [_P, _I, _I, _P, _P, _I, _I, _P, _P, _P, _P, _P]),
    "bst_stream_probe": (_I, [_P, _U64, _P, _P]),
    "bst_batch_workspace_bytes": (_U64, [_I]),
    "bst_batch_prepare": (_I, [_P, _P, _P, _P, _I, _P, _P]),
    "bst_batch_launch": (_I, [_P, _U32, _U32, _I, _P]),
    "bst_batch_free": (None, [_P]),
    "bst_tune_set": (_I, [_I, ctypes.c_int64]),
    "bst_tune_get": (ctypes.c_int64, [_I]),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise BstError(
                "libbytestore.so is not built (expected at %s); run __graft_entry__.build() "
                "or python -m paper_2209_00220_amd.build" % LIB_PATH
            )
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_names():
    return list(_PROTOS)


def _check(rc: int, name: str) -> int:
    if rc < 0:
        msg = lib().bst_last_error()
        raise BstError("%s failed (%d): %s" % (name, rc, msg.decode() if msg else ""))
    return rc


def _call(name, *args):
    return _check(getattr(lib(), name)(*args), name)


def _ptr(x) -> int:
    """Pointer of a torch tensor, numpy array, int or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return x.data_ptr()


# ---- thin wrappers with the ABI's names -------------------------------------
def bst_version() -> int:
    return lib().bst_version()


def bst_device_count() -> int:
    return lib().bst_device_count()


def bst_dict_build(values: np.ndarray, n_threads: int = 0) -> int:
    values = np.ascontiguousarray(values, dtype=np.uint32)
    out = _P()
    _call("bst_dict_build", values.ctypes.data, values.shape[0], n_threads, ctypes.byref(out))
    return out.value


def bst_dict_free(d):
    lib().bst_dict_free(d)


def bst_dict_info(d):
    n, nd = _U64(), _U64()
    _call("bst_dict_info", d, ctypes.byref(n), ctypes.byref(nd))
    return n.value, nd.value


def bst_dict_values(d):
    _, nd = bst_dict_info(d)
    A = np.empty(nd, dtype=np.uint32)
    Q = np.empty(nd, dtype=np.uint64)
    _call("bst_dict_values", d, A.ctypes.data, Q.ctypes.data)
    return A, Q


def bst_encode(d, layout: int, width: int = 0, dir_stride: int = 0, n_threads: int = 0) -> int:
    out = _P()
    _call("bst_encode", d, layout, width, dir_stride, n_threads, ctypes.byref(out))
    return out.value


def bst_encode_host(values, layout: int, width: int = 0) -> int:
    values = np.ascontiguousarray(values, dtype=np.uint32)
    out = _P()
    _call("bst_encode_host", values.ctypes.data, values.shape[0], layout, width, ctypes.byref(out))
    return out.value


def bst_encode_codes(codes, lengths, k_max: int) -> int:
    codes = np.ascontiguousarray(codes, dtype=np.uint64)
    lengths = np.ascontiguousarray(lengths, dtype=np.uint8)
    out = _P()
    _call("bst_encode_codes", codes.ctypes.data, lengths.ctypes.data, codes.shape[0], k_max, ctypes.byref(out))
    return out.value


def bst_free_host(c):
    lib().bst_free_host(c)


def bst_host_info(c) -> ColumnInfo:
    info = ColumnInfo()
    _call("bst_host_info", c, ctypes.byref(info))
    return info


def bst_host_code_table(c, n_distinct: int):
    codes = np.empty(n_distinct, dtype=np.uint64)
    lens = np.empty(n_distinct, dtype=np.uint8)
    _call("bst_host_code_table", c, codes.ctypes.data, lens.ctypes.data)
    return codes, lens


def bst_host_paper_view(c, part: int, j: int) -> np.ndarray:
    nbytes = _U64()
    _call("bst_host_paper_view", c, part, j, None, ctypes.byref(nbytes))
    out = np.zeros(nbytes.value, dtype=np.uint8)
    _call("bst_host_paper_view", c, part, j, out.ctypes.data if out.size else None, ctypes.byref(nbytes))
    return out


def bst_upload(c, dev_ptrs, stream: int) -> int:
    arr = (_P * NBUF)(*[p if p else None for p in dev_ptrs])
    out = _P()
    _call("bst_upload", c, arr, stream, ctypes.byref(out))
    return out.value


def bst_column_free(col):
    lib().bst_column_free(col)


def bst_scan(col, pred: Pred, in_mask, out_bv, dev_status, stream: int):
    _call("bst_scan", col, pred, _ptr(in_mask), _ptr(out_bv), _ptr(dev_status), stream)


def bst_scan_codes(col, op: int, code_lo: int, len_lo: int, code_hi: int, len_hi: int, in_mask, out_bv, stream: int):
    _call("bst_scan_codes", col, op, code_lo, len_lo, code_hi, len_hi, _ptr(in_mask), _ptr(out_bv), stream)


def bst_scan_stats(col, pred: Pred, in_mask, out_bv, dev_counters, stream: int):
    _call("bst_scan_stats", col, pred, _ptr(in_mask), _ptr(out_bv), _ptr(dev_counters), stream)


def bst_lookup(col, row_ids, m: int, out_values, dev_status, stream: int):
    _call("bst_lookup", col, _ptr(row_ids), m, _ptr(out_values), _ptr(dev_status), stream)


def bst_compact_workspace_bytes(n_rows: int) -> int:
    return lib().bst_compact_workspace_bytes(n_rows)


def bst_bv_compact(bv, n_rows, out_ids, cap, dev_count, workspace, dev_status, stream):
    _call("bst_bv_compact", _ptr(bv), n_rows, _ptr(out_ids), cap, _ptr(dev_count), _ptr(workspace),
          _ptr(dev_status), stream)


def bst_lookup_bv(col, bv, out_values, cap, dev_count, ids_tmp, workspace, dev_status, stream):
    _call("bst_lookup_bv", col, _ptr(bv), _ptr(out_values), cap, _ptr(dev_count), _ptr(ids_tmp),
          _ptr(workspace), _ptr(dev_status), stream)


def bst_lookup_counted(col, row_ids, dev_count, cap, out_values, dev_status, stream):
    _call("bst_lookup_counted", col, _ptr(row_ids), _ptr(dev_count), cap, _ptr(out_values), _ptr(dev_status), stream)


def bst_lookup_bv_static(col, bv, out_values, cap, dev_count, dev_status, stream):
    _call("bst_lookup_bv_static", col, _ptr(bv), _ptr(out_values), cap, _ptr(dev_count), _ptr(dev_status), stream)


def bst_lookup_bv_static_max_rows():
    return int(lib().bst_lookup_bv_static_max_rows())


def bst_lookup_bv_static_max_ids():
    return int(lib().bst_lookup_bv_static_max_ids())


def bst_bv_and(a, b, out, n_rows, stream):
    _call("bst_bv_and", _ptr(a), _ptr(b), _ptr(out), n_rows, stream)


def bst_bv_or(a, b, out, n_rows, stream):
    _call("bst_bv_or", _ptr(a), _ptr(b), _ptr(out), n_rows, stream)


def bst_bv_andnot(a, b, out, n_rows, stream):
    _call("bst_bv_andnot", _ptr(a), _ptr(b), _ptr(out), n_rows, stream)


def bst_bv_not(a, out, n_rows, stream):
    _call("bst_bv_not", _ptr(a), _ptr(out), n_rows, stream)


def bst_bv_popcount(bv, n_rows, dev_count, stream):
    _call("bst_bv_popcount", _ptr(bv), n_rows, _ptr(dev_count), stream)


def bst_profile_literals(d, op: int, count: int = 100):
    lits = np.empty(count, dtype=np.uint32)
    sels = np.empty(count, dtype=np.float64)
    _call("bst_profile_literals", d, op, count, lits.ctypes.data, sels.ctypes.data)
    return lits, sels


def bst_auc(sels, times) -> float:
    s = np.ascontiguousarray(sels, dtype=np.float64)
    t = np.ascontiguousarray(times, dtype=np.float64)
    out = ctypes.c_double()
    _call("bst_auc", s.ctypes.data if s.size else None, t.ctypes.data if t.size else None, s.shape[0],
          ctypes.byref(out))
    return out.value


def bst_choose(layouts, aucs) -> int:
    l = np.ascontiguousarray(layouts, dtype=np.int32)
    a = np.ascontiguousarray(aucs, dtype=np.float64)
    out = _I()
    _call("bst_choose", l.ctypes.data, a.ctypes.data, l.shape[0], ctypes.byref(out))
    return out.value


def bst_advise(cols, op, lits, sels, repeats, scratch_bv, stream):
    n = len(cols)
    arr = (_P * n)(*cols)
    lits = np.ascontiguousarray(lits, dtype=np.uint32)
    sels = np.ascontiguousarray(sels, dtype=np.float64)
    times = np.zeros(n * lits.shape[0], dtype=np.float64)
    aucs = np.zeros(n, dtype=np.float64)
    chosen = _I()
    _call("bst_advise", arr, n, op, lits.ctypes.data, sels.ctypes.data, lits.shape[0], repeats,
          _ptr(scratch_bv), times.ctypes.data, aucs.ctypes.data, ctypes.byref(chosen), stream)
    return chosen.value, aucs, times.reshape(n, -1)


def bst_batch_workspace_bytes(n_items: int) -> int:
    return lib().bst_batch_workspace_bytes(n_items)


def bst_batch_prepare(cols, preds, in_masks, outs, workspace) -> int:
    n = len(cols)
    c_arr = (_P * n)(*cols)
    p_arr = (Pred * n)(*preds)
    i_arr = (_P * n)(*[_ptr(m) for m in in_masks]) if in_masks is not None else None
    o_arr = (_P * n)(*[_ptr(o) for o in outs])
    out = _P()
    _call("bst_batch_prepare", c_arr, p_arr, i_arr, o_arr, n, _ptr(workspace), ctypes.byref(out))
    return out.value


def bst_batch_launch(b, grid: int, tiles_per_grab: int, use_graph: bool, stream: int):
    _call("bst_batch_launch", b, grid, tiles_per_grab, 1 if use_graph else 0, stream)


def bst_batch_free(b):
    lib().bst_batch_free(b)


def bst_stream_probe(src, nbytes: int, dst, stream: int):
    _call("bst_stream_probe", _ptr(src), nbytes, _ptr(dst), stream)


def bst_tune_set(key: int, value: int):
    _call("bst_tune_set", key, value)


def bst_tune_get(key: int) -> int:
    return lib().bst_tune_get(key)
