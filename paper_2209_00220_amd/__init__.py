"""MI355X-native ByteStore: PP-VBS / ByteSlice / Bit-Packed scans and lookups on gfx950.

The compute path is the HIP library ``libbytestore.so`` (C ABI in
``include/bytestore.h``); this package holds its ctypes binding (``_lib``),
torch buffer plumbing (``column``) and the host drivers built on it: the
layout advisor, batched scans with an autotuner, and a serving loop.
"""
from . import _lib
from ._lib import BITPACKED, BYTESLICE, PPVBS, BstError
from .column import DeviceColumn, Dictionary, HostColumn, bv_and, bv_compact, bv_or, bv_popcount

__all__ = [
    "_lib", "BITPACKED", "BYTESLICE", "PPVBS", "BstError", "DeviceColumn", "Dictionary", "HostColumn",
    "bv_and", "bv_compact", "bv_or", "bv_popcount",
]
