"""Torch plumbing around the C ABI: device buffers, streams and result tensors.

torch owns every device allocation (``torch.empty`` on the current device) and
supplies the stream (``torch.cuda.current_stream()``); the library only reads
and writes the buffers it is handed.  Bitvectors are int64 tensors holding the
uint64 words; row IDs and values are int32 tensors holding uint32 bit patterns.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L

LAYOUTS = {"bitpacked": L.BITPACKED, "byteslice": L.BYTESLICE, "ppvbs": L.PPVBS,
           "ppvbs_categorical": L.PPVBS_CATEGORICAL}


def layout_code(layout) -> int:
    if isinstance(layout, str):
        return LAYOUTS[layout]
    return int(layout)


def stream_handle(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def nwords(n_rows: int) -> int:
    return (n_rows + 63) // 64


def bv_to_numpy(bv: torch.Tensor) -> np.ndarray:
    return bv.detach().cpu().numpy().view(np.uint64)


def bv_from_numpy(words: np.ndarray, device="cuda") -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(words, dtype=np.uint64).view(np.int64)).to(device)


def u32_to_numpy(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)


def u32_from_numpy(a: np.ndarray, device="cuda") -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).to(device)


def make_pred(op, lo: int, hi: int | None = None) -> L.Pred:
    code = L.OP_CODES[op] if isinstance(op, str) else int(op)
    return L.Pred(code, int(lo) & 0xFFFFFFFF, int(hi if hi is not None else lo) & 0xFFFFFFFF)


class Dictionary:
    """Sorted distinct values, counts and per-row ranks of a column (host)."""

    def __init__(self, values: np.ndarray, n_threads: int = 0):
        self.h = L.bst_dict_build(values, n_threads)
        self.n_rows, self.n_distinct = L.bst_dict_info(self.h)

    def values_counts(self):
        return L.bst_dict_values(self.h)

    def profile_literals(self, op="lt", count: int = 100):
        return L.bst_profile_literals(self.h, L.OP_CODES[op] if isinstance(op, str) else op, count)

    def close(self):
        if self.h:
            L.bst_dict_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HostColumn:
    """One encoded layout of a column, in host memory."""

    def __init__(self, handle: int):
        self.h = handle
        self.info = L.bst_host_info(handle)

    @classmethod
    def encode(cls, d: Dictionary, layout, width: int = 0, dir_stride: int = 0, n_threads: int = 0):
        return cls(L.bst_encode(d.h, layout_code(layout), width, dir_stride, n_threads))

    @classmethod
    def from_values(cls, values, layout, width: int = 0):
        return cls(L.bst_encode_host(values, layout_code(layout), width))

    @classmethod
    def from_codes(cls, codes, lengths, k_max: int):
        return cls(L.bst_encode_codes(codes, lengths, k_max))

    @property
    def n_rows(self) -> int:
        return int(self.info.n_rows)

    @property
    def layout(self) -> int:
        return int(self.info.layout)

    def code_table(self):
        return L.bst_host_code_table(self.h, int(self.info.n_distinct))

    def paper_view(self, part: int, j: int) -> np.ndarray:
        return L.bst_host_paper_view(self.h, part, j)

    def close(self):
        if self.h:
            L.bst_free_host(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DeviceColumn:
    """A host column copied into torch-owned device buffers."""

    def __init__(self, host: HostColumn, device="cuda", stream=None):
        self.host = host
        self.device = torch.device(device)
        info = host.info
        self.bufs = []
        ptrs = []
        for s in range(L.NBUF):
            nb = int(info.bytes[s])
            if nb:
                t = torch.empty(nb, dtype=torch.uint8, device=self.device)
                self.bufs.append(t)
                ptrs.append(t.data_ptr())
            else:
                self.bufs.append(None)
                ptrs.append(0)
        self.h = L.bst_upload(host.h, ptrs, stream_handle(stream))
        self.n_rows = int(info.n_rows)
        self.layout = int(info.layout)
        self.device_bytes = int(info.total_bytes)

    # -- buffers -----------------------------------------------------------
    def new_bv(self) -> torch.Tensor:
        return torch.empty(nwords(self.n_rows), dtype=torch.int64, device=self.device)

    # -- operations --------------------------------------------------------
    def scan(self, op, lo, hi=None, in_mask=None, out=None, status=None, stream=None) -> torch.Tensor:
        out = self.new_bv() if out is None else out
        L.bst_scan(self.h, make_pred(op, lo, hi), in_mask, out, status, stream_handle(stream))
        return out

    def scan_codes(self, op, code_lo, len_lo, code_hi=0, len_hi=0, in_mask=None, out=None, stream=None):
        out = self.new_bv() if out is None else out
        opc = L.OP_CODES[op] if isinstance(op, str) else int(op)
        L.bst_scan_codes(self.h, opc, int(code_lo), int(len_lo), int(code_hi), int(len_hi), in_mask, out,
                         stream_handle(stream))
        return out

    def scan_stats(self, op, lo, hi=None, in_mask=None, out=None, stream=None):
        out = self.new_bv() if out is None else out
        counters = torch.zeros(5, dtype=torch.int64, device=self.device)
        L.bst_scan_stats(self.h, make_pred(op, lo, hi), in_mask, out, counters, stream_handle(stream))
        return out, counters

    def lookup(self, ids: torch.Tensor, out=None, status=None, stream=None) -> torch.Tensor:
        m = int(ids.numel())
        out = torch.empty(m, dtype=torch.int32, device=self.device) if out is None else out
        L.bst_lookup(self.h, ids, m, out, status, stream_handle(stream))
        return out

    def lookup_bv(self, bv: torch.Tensor, cap: int, status=None, stream=None):
        """Values of the set rows in ascending order; returns (values[cap], count tensor)."""
        vals = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
        ids = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
        ws = torch.empty(int(L.bst_compact_workspace_bytes(self.n_rows)), dtype=torch.uint8, device=self.device)
        count = torch.zeros(1, dtype=torch.int64, device=self.device)
        L.bst_lookup_bv(self.h, bv, vals, cap, count, ids, ws, status, stream_handle(stream))
        return vals, count

    def close(self):
        if self.h:
            L.bst_column_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bv_compact(bv: torch.Tensor, n_rows: int, cap: int, status=None, stream=None):
    """Ascending row IDs of the set bits: (ids[cap] int32, count int64[1])."""
    dev = bv.device
    ids = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    ws = torch.empty(int(L.bst_compact_workspace_bytes(n_rows)), dtype=torch.uint8, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    L.bst_bv_compact(bv, n_rows, ids, cap, count, ws, status, stream_handle(stream))
    return ids, count


def bv_and(a, b, n_rows, out=None, stream=None):
    out = torch.empty_like(a) if out is None else out
    L.bst_bv_and(a, b, out, n_rows, stream_handle(stream))
    return out


def bv_or(a, b, n_rows, out=None, stream=None):
    out = torch.empty_like(a) if out is None else out
    L.bst_bv_or(a, b, out, n_rows, stream_handle(stream))
    return out


def bv_andnot(a, b, n_rows, out=None, stream=None):
    out = torch.empty_like(a) if out is None else out
    L.bst_bv_andnot(a, b, out, n_rows, stream_handle(stream))
    return out


def bv_not(a, n_rows, out=None, stream=None):
    out = torch.empty_like(a) if out is None else out
    L.bst_bv_not(a, out, n_rows, stream_handle(stream))
    return out


def bv_popcount(bv, n_rows, stream=None) -> torch.Tensor:
    count = torch.zeros(1, dtype=torch.int64, device=bv.device)
    L.bst_bv_popcount(bv, n_rows, count, stream_handle(stream))
    return count
